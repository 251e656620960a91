"""Throughput of the particle loop on one MI355X.

Metric: particle-steps/s of the batched FP32 form (push + gather + deposit +
MCC, with the sort, FP64 Poisson solve and diagnostics of each step inside
the timed region), beside the plain FP64 GPU form on identical inputs and the
FP64 CPU oracle on a bounded sample.

Default workload (batch8): 8 coaxial-trap instances on 256x1024 meshes,
16M macro-electrons each (128M total), paraxial mirror field, pressures
cycling 1e-6 / 3e-6 / 1e-5 mbar.  Synthetic inputs (pic_inputs).

Timed region: W warm-up steps, then K steps bracketed by device
synchronisation; HIP events on the library's stream time every launch of
the particle kernel inside the same region (steps then run as plain
launches).  The graph-replay rate of the same workload is reported beside.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (push+gather+deposit+MCC), batched FP32 vs plain FP64, 1 GPU"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle-step of the fused FP32 kernel:
# read r, z, vr, vt, vz, w (6 x 4 B) + key (8 B), write r, z, vr, vt, vz (5 x 4 B)
BYTES_FP32 = 52
# plain FP64 push kernel: read r, z, vr, vt, vz (5 x 8 B) + w on absorption only, write 5 x 8 B
BYTES_FP64_PUSH = 80

WORKLOAD_TEXT = {
    "batch8": "8 instances x 256x1024 mesh x 16M electrons (128M), mirror B (k=0.3), p=1e-6/3e-6/1e-5 mbar",
    "scan32": "32 instances x 128x512 mesh, 0.5M-8M electrons each, p/V/B scan",
    "coax512": "1 instance x 512x2048 mesh x 64M electrons, mirror B, -30 kV",
    "coax256": "1 instance x 256x1024 mesh x 4M electrons, mirror B, 1e-5 mbar",
}


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2206_14662_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measure(B, torch, cfgs, mode, steps, warmup, graph_too):
    sim = B.Sim(cfgs, mode=mode)
    ctx = sim.ctx
    B.pic_step(ctx, warmup)
    torch.cuda.synchronize()
    before = sum(B.pic_diag(ctx, k)["particle_steps"] for k in range(len(cfgs)))
    B.pic_timing(ctx, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.pic_step(ctx, steps)
    B.pic_sync(ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kern_ms = B.pic_timing(ctx, 0)
    after = sum(B.pic_diag(ctx, k)["particle_steps"] for k in range(len(cfgs)))
    out = dict(ps=after - before, wall=t1 - t0, launches=launches, kern_ms=kern_ms)
    if graph_too:
        before = after
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.pic_step(ctx, steps)
        B.pic_sync(ctx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        after = sum(B.pic_diag(ctx, k)["particle_steps"] for k in range(len(cfgs)))
        out["graph_rate"] = (after - before) / (t1 - t0)
    out["tuning"] = B.pic_tuning(ctx)
    out["n_live"] = sum(B.pic_diag(ctx, k)["n_live"] for k in range(len(cfgs)))
    sim.close()
    torch.cuda.synchronize()
    return out


def cpu_baseline(cfg0, target_s=12.0):
    """The FP64 oracle on a bounded sample of the workload: instance 0's mesh
    and parameters with its electron count cut to fit ~10-30 s of CPU work."""
    import oracle
    n = min(int(cfg0["n_init"]), 1_000_000)
    c = dict(cfg0, n_init=n, weight=cfg0["weight"] * cfg0["n_init"] / n)
    s = oracle.Sim(c)
    s.load()
    t0 = time.perf_counter()
    s.step(1)
    one = time.perf_counter() - t0
    k = max(1, min(50, int(target_s / max(one, 1e-3))))
    d0 = s.diag()
    t0 = time.perf_counter()
    s.step(k)
    dt = time.perf_counter() - t0
    d1 = s.diag()
    ps = k * (d0["n_live"] + d1["n_live"]) / 2.0
    return {"value": ps / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"instance 0 mesh {c['nr']}x{c['nz']}, {n} electrons (weight scaled), {k + 1} steps "
                      f"incl. FP64 Poisson, {dt:.1f} s timed"}


def read_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current sources."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except Exception:
        return None
    if t.get("source_hash") != source_hash():
        return None
    return t.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batch8", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scale", type=float, default=1.0, help="particle-count scale (tests only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy three times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a "
              "design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import pic_inputs as pi
    from paper_2206_14662_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        n = (2 << 30) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)
        return
    if args.workload == "batch8":
        cfgs = pi.batch8(n_per=int(16_000_000 * args.scale))
    elif args.workload == "scan32":
        cfgs = pi.scan32(n_scale=args.scale)
    else:
        cfgs = [getattr(pi, args.workload)(n_init=int(getattr(pi, args.workload)()["n_init"] * args.scale))]
    print(f"# workload {args.workload}: {len(cfgs)} instances, "
          f"{sum(c['n_init'] for c in cfgs)} electrons", file=sys.stderr, flush=True)

    r32 = measure(B, torch, cfgs, B.PIC_MODE_FP32_BATCHED, args.steps, args.warmup, True)
    value = r32["ps"] / r32["wall"]
    print(f"# fp32: {value:.4g} particle-steps/s, graph {r32['graph_rate']:.4g}", file=sys.stderr, flush=True)
    kern_avg_ms = r32["kern_ms"] / max(1, r32["launches"])
    bytes_per_launch = BYTES_FP32 * r32["ps"] / max(1, r32["launches"])
    achieved = bytes_per_launch / (kern_avg_ms * 1e-3) / 1e9
    traffic = read_traffic("k_particles", args.workload)

    fp64 = None
    if not args.no_fp64:
        r64 = measure(B, torch, cfgs, B.PIC_MODE_FP64_PLAIN, max(4, args.steps // 4), max(2, args.warmup // 4),
                      False)
        v64 = r64["ps"] / r64["wall"]
        fp64 = {"value": v64, "unit": "particle-steps/s", "steps": max(4, args.steps // 4),
                "push_kernel_avg_ms": r64["kern_ms"] / max(1, r64["launches"])}
        print(f"# fp64 plain: {v64:.4g} particle-steps/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfgs[0])
        print(f"# cpu oracle: {cpu['value']:.4g} particle-steps/s on {cpu['cores']} threads", file=sys.stderr,
              flush=True)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}",
                   "instances": len(cfgs), "electrons": int(sum(c["n_init"] for c in cfgs)),
                   "form": "FP32 batched (tile-sorted, fused persistent particle kernel, FP64 Poisson)",
                   "tuning": r32["tuning"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_particles", "bytes_per_particle_step": BYTES_FP32,
                     "avg_launch_ms": kern_avg_ms, "launches": r32["launches"]},
        "cpu_baseline": cpu,
        "graph_replay_value": r32["graph_rate"],
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": (value / fp64["value"]) if fp64 else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
