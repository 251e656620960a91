"""Throughput of the particle loop on one MI355X.

Metric: particle-steps/s of the batched FP32 form (push + gather + deposit +
MCC, with the sort, FP64 Poisson solve and diagnostics of each step inside
the timed region), beside the plain FP64 GPU form on identical inputs and the
FP64 CPU oracle on a bounded sample.

Default workload (batch8): 8 coaxial-trap instances on 256x1024 meshes,
16M macro-electrons each (128M total), paraxial mirror field, pressures
cycling 1e-6 / 3e-6 / 1e-5 mbar.  Synthetic inputs (pic_inputs).

Timed regions (one context, after W warm-up steps): K steps as the library
runs them (captured HIP graphs), bracketed by device synchronisation, give
`value`; K further steps as plain launches with HIP events on the library's
stream around every particle-kernel launch give the kernel's average
duration for the roofline (their own rate is reported as
`event_timed_value`).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (push+gather+deposit+MCC), batched FP32 vs plain FP64, 1 GPU"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle-step of the fused FP32 kernel: read r, z, vr,
# vt, vz (5 x 4 B) + key (8 B), write r, z, vr, vt, vz (5 x 4 B); every electron
# of these workloads carries its instance's macro-weight, so the weight array
# is not read (a per-particle weight would add 4 B)
BYTES_FP32 = 48
# the same with a per-particle weight array read (4 B more): the accounting of
# a kernel that streams the whole 24-B state plus the key
BYTES_FP32_WEIGHTED = 52
# plain FP64 push kernel: read r, z, vr, vt, vz (5 x 8 B) + w on absorption only, write 5 x 8 B
BYTES_FP64_PUSH = 80

WORKLOAD_TEXT = {
    "batch8": "8 instances x 256x1024 mesh x 16M electrons (128M), mirror B (k=0.3), p=1e-6/3e-6/1e-5 mbar",
    "scan32": "32 instances x 128x512 mesh, 0.5M-8M electrons each, p/V/B scan",
    "coax512": "1 instance x 512x2048 mesh x 64M electrons, mirror B, -30 kV",
    "coax256": "1 instance x 256x1024 mesh x 4M electrons, mirror B, 1e-5 mbar",
    "gun8": "8 instances of the paper's gun geometry (coax with the elliptic insert, open ends) x 256x512 mesh "
            "x 16M electrons (128M), 20-40 kV, 2.5e-2..1e-1 mbar",
}


def autotune(B, torch, cfgs, cache):
    """Tile shape, halo and sort interval from the library's autotuner, run on
    a scratch context of the same workload (its trial steps are not part of
    the measured run, which starts again from the initial state)."""
    sim = B.Sim(cfgs, mode=B.PIC_MODE_FP32_BATCHED)
    t0 = time.perf_counter()
    t = sim.autotune(trial_steps=48, cache_path=cache)
    t["tune_s"] = time.perf_counter() - t0
    tun = B.pic_tuning(sim.ctx)
    t["lanes"], t["use_graph"] = tun["lanes"], tun["use_graph"]
    sim.close()
    torch.cuda.synchronize()
    return t


def measure(B, torch, cfgs, mode, steps, warmup, graph_region, tuning=None):
    """Warm-up, then (graph_region) `steps` steps as the library runs them
    (HIP-graph replay) timed by the wall clock between device synchronisations,
    then `steps` more steps with HIP events recorded around every particle
    kernel launch (plain launches) for the kernel's average duration."""
    kw = {}
    if tuning:
        kw = {k: tuning[k] for k in ("tile_r", "tile_z", "halo", "sort_interval", "lanes", "use_graph")
              if k in tuning}
    sim = B.Sim(cfgs, mode=mode, **kw)
    ctx = sim.ctx
    n = len(cfgs)

    def psteps():
        d = [B.pic_diag(ctx, k) for k in range(n)]
        return sum(x["particle_steps"] for x in d), sum(x["n_far_deposit"] for x in d)

    def region(timed):
        ps0, far0 = psteps()
        if timed:
            B.pic_timing(ctx, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.pic_step(ctx, steps)
        B.pic_sync(ctx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        launches, kern_ms = B.pic_timing(ctx, 0) if timed else (0, 0.0)
        ps1, far1 = psteps()
        return dict(ps=ps1 - ps0, wall=t1 - t0, launches=launches, kern_ms=kern_ms,
                    far_frac=(far1 - far0) / max(1, ps1 - ps0))

    B.pic_step(ctx, warmup)
    torch.cuda.synchronize()
    out = {}
    if graph_region:
        out["run"] = region(False)
    out["events"] = region(True)
    if not graph_region:
        out["run"] = out["events"]
    out["tuning"] = B.pic_tuning(ctx)
    out["n_live"] = sum(B.pic_diag(ctx, k)["n_live"] for k in range(n))
    sim.close()
    torch.cuda.synchronize()
    return out


def cpu_baseline(cfg0, target_s=15.0):
    """The FP64 oracle on a bounded sample of the workload: instance 0 at its
    full size (mesh, parameters, electron count), for as many steps as fill
    about target_s seconds on the host cores."""
    import oracle
    s = oracle.Sim(dict(cfg0))
    s.load()
    t0 = time.perf_counter()
    s.step(1)
    one = time.perf_counter() - t0
    k = max(1, min(200, int(target_s / max(one, 1e-3))))
    d0 = s.diag()
    t0 = time.perf_counter()
    s.step(k)
    dt = time.perf_counter() - t0
    d1 = s.diag()
    ps = k * (d0["n_live"] + d1["n_live"]) / 2.0
    return {"value": ps / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"instance 0 of the workload ({cfg0['nr']}x{cfg0['nz']} mesh, {int(cfg0['n_init'])} electrons, "
                      f"p={cfg0['p_mbar']:g} mbar), {k} steps after one warm step, incl. FP64 Poisson, "
                      f"{dt:.1f} s timed",
            "build": "gcc -O3 -ffp-contract=off -fopenmp (plain C11, FP64)",
            **host_cpu()}


def host_cpu():
    """The host's CPU model, its physical cores and hardware threads (from
    /proc/cpuinfo) and the CPUs this process may run on."""
    model, phys, logical = None, set(), 0
    pid, core = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    logical += 1
                elif k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    pid = v
                elif k == "core id":
                    core = v
                elif not k and pid is not None and core is not None:
                    phys.add((pid, core))
                    pid, core = None, None
        if pid is not None and core is not None:
            phys.add((pid, core))
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = None
    return {"cpu_model": model, "host_physical_cores": len(phys) or None, "host_hw_threads": logical or None,
            "cpus_allowed": allowed}


def accuracy(B, torch, workload, steps, p_mbar=None, ref="gpu64"):
    """FP32 batched against FP64 on the same seed: relative errors of the
    time-averaged density (L2 over nodes above 20% of its maximum), the peak
    density and the peak outer (radial) current.  ref = "oracle" runs the
    FP64 CPU oracle itself; "gpu64" the plain FP64 GPU form, which matches
    the oracle step by step (used where a CPU run is out of reach)."""
    import numpy as np

    import pic_inputs as pi
    over = {} if p_mbar is None else {"p_mbar": p_mbar}
    if workload == "coax64hot":
        cfg = pi.coax64hot(n_init=50000, diag_interval=10, **over)
    else:
        cfg = getattr(pi, workload)(**over)
    g = B.Sim([cfg], mode=B.PIC_MODE_FP32_BATCHED)
    t0 = time.perf_counter()
    g.step(steps)
    d32 = g.diag(want_density=True)
    d32["wall_s"] = time.perf_counter() - t0
    S = d32["S"]
    g.close()
    torch.cuda.synchronize()
    print(f"# accuracy {workload}: FP32 done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    if ref == "oracle":
        import oracle
        o = oracle.Sim(cfg, fx_shift=S)
        o.load()
        for done in range(0, steps, 50):
            o.step(min(50, steps - done))
            print(f"# accuracy {workload}: oracle step {done + min(50, steps - done)}", file=sys.stderr, flush=True)
        d64 = o.diag()
        d64["time_avg_density"] = o.time_avg_density()
        ref_name = "FP64 CPU oracle"
    else:
        h = B.Sim([cfg], mode=B.PIC_MODE_FP64_PLAIN)
        for done in range(0, steps, 500):
            B.pic_step(h.ctx, min(500, steps - done))
            B.pic_sync(h.ctx)
            print(f"# accuracy {workload}: FP64 step {done + min(500, steps - done)}", file=sys.stderr, flush=True)
        d64 = h.diag(want_density=True)
        h.close()
        torch.cuda.synchronize()
        ref_name = "plain FP64 GPU form"
    wall64 = time.perf_counter() - t0
    na = np.asarray(d64["time_avg_density"]).reshape(-1)
    nb = np.asarray(d32["time_avg_density"]).reshape(-1)
    mask = na > 0.2 * na.max()

    def rel(a, b):
        return float(abs(a - b) / abs(b)) if b != 0 else None
    return {
        "workload": workload, "p_mbar": cfg["p_mbar"], "steps": steps, "reference": ref_name,
        "time_avg_density_rel_l2": float(np.linalg.norm((nb - na)[mask]) / np.linalg.norm(na[mask])),
        "peak_density_rel": rel(d32["peak_density"], d64["peak_density"]),
        "peak_time_avg_density_rel": rel(float(nb.max()), float(na.max())),
        "peak_I_outer_A": [d32["peak_I_outer"], d64["peak_I_outer"]],
        "peak_I_outer_rel": rel(d32["peak_I_outer"], d64["peak_I_outer"]),
        "n_live": [int(d32["n_live"]), int(d64["n_live"])],
        "n_elastic": [int(d32["n_elastic"]), int(d64["n_elastic"])],
        "n_ioniz": [int(d32["n_ioniz"]), int(d64["n_ioniz"])],
        "n_absorbed_outer": [int(d32["n_absorbed"][1]), int(d64["n_absorbed"][1])],
        "wall_s": [d32["wall_s"], wall64],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="batch8", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scale", type=float, default=1.0, help="particle-count scale (tests only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy three times (reference for HBM byte counters)")
    ap.add_argument("--no-tune", action="store_true", help="default tiles instead of the autotuner's choice")
    ap.add_argument("--tiles", default=None, help="TR,TZ,HALO,K[,LANES] instead of the autotuner")
    ap.add_argument("--tune-cache", default=os.path.join(os.environ.get("TMPDIR", "/tmp"), "picmcc_tune.jsonl"))
    ap.add_argument("--accuracy", default=None, choices=("coax64hot", "coax256", "coax512"),
                    help="instead of timing, report FP32-vs-FP64 errors on this workload")
    ap.add_argument("--acc-steps", type=int, default=2000)
    ap.add_argument("--acc-p-mbar", type=float, default=None, help="pressure override of the accuracy workload")
    ap.add_argument("--acc-ref", default="gpu64", choices=("gpu64", "oracle"))
    ap.add_argument("--shapes", action="store_true",
                    help="cubic against bilinear shapes in both forms on the workload's instance 0")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no multi-GPU "
              "path (instances would shard across GPUs with no communication)", file=sys.stderr)
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
    if args.shapes:
        c0 = (pi.batch8(n_per=int(16_000_000 * args.scale)) if args.workload == "batch8"
              else [getattr(pi, args.workload)(n_init=int(getattr(pi, args.workload)()["n_init"] * args.scale))])[0]
        out = {}
        for form, mode, graph in (("fp64_plain", B.PIC_MODE_FP64_PLAIN, False),
                                  ("fp32_batched", B.PIC_MODE_FP32_BATCHED, True)):
            steps = max(4, args.steps // 4) if not graph else args.steps
            res = {}
            for order in (1, 3):
                c = dict(c0, spline_order=order)
                m = measure(B, torch, [c], mode, steps, max(2, args.warmup // 4) if not graph else args.warmup, graph)
                r, e = m["run"], m["events"]
                res["bilinear" if order == 1 else "cubic"] = {
                    "particle_steps_per_s": r["ps"] / r["wall"], "ms_per_step": 1e3 * r["wall"] / steps,
                    "push_kernel_avg_ms": e["kern_ms"] / max(1, e["launches"])}
            res["cubic_over_bilinear"] = res["cubic"]["particle_steps_per_s"] / res["bilinear"]["particle_steps_per_s"]
            out[form] = res
        print(json.dumps({"metric": "particle-steps/s with cubic against bilinear shapes, both forms",
                          "config": {"workload": args.workload, "instance": 0, "electrons": int(c0["n_init"]),
                                     "mesh": [c0["nr"], c0["nz"]], "fp32_tiles": "default (8x32, halo 8, sort 16)"},
                          **out}), flush=True)
        return
    if args.accuracy:
        print(json.dumps({"metric": "fp32_vs_fp64_error", **accuracy(B, torch, args.accuracy, args.acc_steps,
                                                                          args.acc_p_mbar, args.acc_ref)}),
              flush=True)
        return
    if args.workload == "batch8":
        cfgs = pi.batch8(n_per=int(16_000_000 * args.scale))
    elif args.workload == "scan32":
        cfgs = pi.scan32(n_scale=args.scale)
    elif args.workload == "gun8":
        cfgs = pi.gun8(n_per=int(16_000_000 * args.scale))
    else:
        cfgs = [getattr(pi, args.workload)(n_init=int(getattr(pi, args.workload)()["n_init"] * args.scale))]
    print(f"# workload {args.workload}: {len(cfgs)} instances, "
          f"{sum(c['n_init'] for c in cfgs)} electrons", file=sys.stderr, flush=True)

    tuned = None
    if args.tiles:
        v = [int(x) for x in args.tiles.split(",")]
        tuned = dict(zip(("tile_r", "tile_z", "halo", "sort_interval", "lanes"), v), trials=0, ms_per_step=0.0,
                     tune_s=0.0)
    elif not args.no_tune:
        tuned = autotune(B, torch, cfgs, args.tune_cache)
        print(f"# autotune: {tuned}", file=sys.stderr, flush=True)
    r32 = measure(B, torch, cfgs, B.PIC_MODE_FP32_BATCHED, args.steps, args.warmup, True, tuned)
    run, ev = r32["run"], r32["events"]
    value = run["ps"] / run["wall"]
    print(f"# fp32: {value:.4g} particle-steps/s (graph replay), {ev['ps'] / ev['wall']:.4g} with kernel events",
          file=sys.stderr, flush=True)
    kern_avg_ms = ev["kern_ms"] / max(1, ev["launches"])
    bytes_per_launch = BYTES_FP32 * ev["ps"] / max(1, ev["launches"])
    achieved = bytes_per_launch / (kern_avg_ms * 1e-3) / 1e9
    from paper_2206_14662_amd import profiling
    traffic = profiling.read_traffic(os.path.join(ROOT, "profiles", f"k_particles_{args.workload}_traffic.txt"))

    fp64 = None
    if not args.no_fp64:
        r64 = measure(B, torch, cfgs, B.PIC_MODE_FP64_PLAIN, max(4, args.steps // 4), max(2, args.warmup // 4),
                      False)["events"]
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
        "ms_per_step": 1e3 * run["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}",
                   "instances": len(cfgs), "electrons": int(sum(c["n_init"] for c in cfgs)),
                   "form": "FP32 batched (tile-sorted, fused persistent particle kernel, FP64 Poisson)",
                   "tuning": r32["tuning"],
                   "autotune": ({k: tuned[k] for k in ("trials", "ms_per_step", "tune_s")} if tuned else None)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_particles", "bytes_per_particle_step": BYTES_FP32,
                     "frac_52B": achieved * BYTES_FP32_WEIGHTED / BYTES_FP32 / HBM_PEAK_GBS,
                     "avg_launch_ms": kern_avg_ms, "launches": ev["launches"],
                     "far_deposit_fraction": ev["far_frac"],
                     "timed_with": "HIP events around each launch, plain launches, same workload and run"},
        "cpu_baseline": cpu,
        "event_timed_value": ev["ps"] / ev["wall"],
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": (value / fp64["value"]) if fp64 else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
