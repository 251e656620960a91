"""Runs in the paper's collisional regime (Sec. II.B raised pressure, Sec. III
time evolution and pressure scan) with the batched FP32 form: one context
holds a synthetic coaxial trap at several neutral pressures, seeded by a weak
homogeneous Maxwellian cloud and the volumetric source, and advances them
together for a number of momentum-exchange times tau_d of the lowest
pressure.  Traces of the instantaneous peak density and of the wall currents
are sampled every `every` steps.

  python -m paper_2206_14662_amd.regime [--pressures 0.025,0.05,0.1] [--taud 20] [--out FILE]

The summary checks the paper's scalings on this synthetic trap: peak density
independent of pressure, radial current proportional to pressure, and the
peak density against the Brillouin-type limit eps0 B^2 / (2 m_e)
(omega_pe^2 <= Omega^2 / 2).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

E = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12
KB = 1.380649e-23


def trap(p_mbar, nr=128, nz=256, n0=1.0e15, weight=2.0e4, src_per_step=2.0, E_ref_eV=200.0, **over):
    """The synthetic trap at pressure p: a 1 eV seed cloud of density n0 in
    the load box (Sec. III.A), a weak volumetric source, the mirror field."""
    import pic_inputs as pi
    box = pi.coax64()
    vol = math.pi * (box["r_hi"] ** 2 - box["r_lo"] ** 2) * (box["z_hi"] - box["z_lo"])
    c = pi.coax64(nr=nr, nz=nz, p_mbar=p_mbar, mirror_k=0.3, n_init=int(round(n0 * vol / weight)),
                  weight=weight, load_mode=0, src_rate=src_per_step, src_T_eV=1.0, diag_interval=100, **over)
    n_n = 100.0 * p_mbar / (KB * c["T_gas_K"])
    v_ref = math.sqrt(2.0 * E_ref_eV * E / ME)
    tau_d = 1.0 / (n_n * c["sigma_el"] * v_ref)
    return c, tau_d


def force_balance(g, k, cfg, samples=64, gap=16, omit=()):
    """Sec. IV force terms of the electron fluid from the moments, averaged
    over `samples` snapshots `gap` steps apart (several cyclotron periods),
    in the cloud (n > 0.2 n_max).  With T = m_e sum w v v / V the full second
    moment (inertia plus pressure), the momentum balance in (r, theta, z) reads
        r:     -(dT_rr/dr + (T_rr - T_tt)/r + dT_rz/dz) + q n E_r + q G_t B_z - m D_r = 0
        theta: -(dT_rt/dr + 2 T_rt/r + dT_tz/dz) + q (G_z B_r - G_r B_z) - m D_t = 0
    with G = n u and D = (sum w nu_m / V) u the collisional drag.  Returns the
    median over cloud nodes of |sum| / (sum of |terms|) for both equations,
    and the median of the azimuthal drag-to-Lorentz ratio m D_t / (q G_r B_z).
    `omit` leaves named terms out of both sums ("stress", "curvature",
    "electric", "magnetic", "drag"), to show what each one carries."""
    import numpy as np
    acc = None
    for _ in range(samples):
        g.step(gap)
        m = g.moments(k)
        acc = m if acc is None else acc + m
    m = acc / samples
    f = g.fields(k)
    n, Gr, Gt, Gz = m[0], m[1], m[2], m[3]
    Trr, Trt, Trz, Ttt, Ttz = (ME * m[i] for i in (4, 5, 6, 7, 8))
    nu = m[10]
    d = (cfg["b"] - cfg["a"]) / cfg["nr"], cfg["L"] / cfg["nz"]
    r = (cfg["a"] + d[0] * np.arange(cfg["nr"] + 1))[:, None]
    q = -E
    safe = np.where(n > 0, n, 1.0)
    Dr, Dt = nu * Gr / safe, nu * Gt / safe
    grad = lambda a, ax: np.gradient(a, d[ax], axis=ax)
    radial = [("stress", -grad(Trr, 0)), ("curvature", -(Trr - Ttt) / r), ("stress", -grad(Trz, 1)),
              ("electric", q * n * f["Er"]), ("magnetic", q * Gt * f["Bz"]), ("drag", -ME * Dr)]
    azim = [("stress", -grad(Trt, 0)), ("curvature", -2.0 * Trt / r), ("stress", -grad(Ttz, 1)),
            ("magnetic", q * Gz * f["Br"]), ("magnetic", -q * Gr * f["Bz"]), ("drag", -ME * Dt)]
    radial = [v for name, v in radial if name not in omit]
    azim = [v for name, v in azim if name not in omit]
    cloud = n > 0.2 * n.max()
    cloud[0, :] = cloud[-1, :] = cloud[:, 0] = cloud[:, -1] = False

    def resid(terms):
        tot = np.abs(sum(terms))[cloud]
        mag = sum(np.abs(t) for t in terms)[cloud]
        return float(np.median(tot / np.maximum(mag, 1e-300)))
    ratio = (ME * Dt) / np.where(np.abs(q * Gr * f["Bz"]) > 0, q * Gr * f["Bz"], 1.0)
    return {"radial_residual": resid(radial), "azimuthal_residual": resid(azim),
            "drag_over_radial_lorentz_theta": float(np.median(ratio[cloud])), "cloud_nodes": int(cloud.sum())}


def run(pressures, taud=20.0, every=100, out=None, log=sys.stderr, balance=True, **over):
    import numpy as np
    import torch

    from paper_2206_14662_amd import binding as B

    made = [trap(p, **over) for p in pressures]
    cfgs = [m[0] for m in made]
    taus = [m[1] for m in made]
    dt = cfgs[0]["dt"]
    steps = int(math.ceil(taud * max(taus) / dt / every)) * every
    g = B.Sim(cfgs, mode=B.PIC_MODE_FP32_BATCHED)
    traces = [dict(t=[], n_peak=[], I_outer=[], I_inner=[], I_left=[], I_right=[], n_live=[]) for _ in cfgs]
    t0 = time.perf_counter()
    for done in range(0, steps, every):
        g.step(every)
        for k in range(len(cfgs)):
            d = g.diag(k, want_density=True)
            tr = traces[k]
            tr["t"].append((done + every) * dt / taus[k])
            tr["n_peak"].append(float(np.max(d["density"])))
            for name, w in (("I_inner", 0), ("I_outer", 1), ("I_left", 2), ("I_right", 3)):
                tr[name].append(float(d["I_wall"][w]))
            tr["n_live"].append(int(d["n_live"]))
        if (done // every) % 50 == 0:
            print(f"# regime: step {done + every}/{steps}, n_live {[tr['n_live'][-1] for tr in traces]}", file=log,
                  flush=True)
    wall = time.perf_counter() - t0
    final = [g.diag(k) for k in range(len(cfgs))]
    forces = [force_balance(g, k, cfgs[k]) if balance else None for k in range(len(cfgs))]
    g.close()
    torch.cuda.synchronize()
    B0 = cfgs[0]["B0"]
    n_brillouin = EPS0 * (B0 * B0) / (2.0 * ME)
    summary = []
    for k, p in enumerate(pressures):
        tr = traces[k]
        half = len(tr["t"]) // 2
        summary.append({
            "p_mbar": p, "tau_d_s": taus[k], "steps": steps, "t_end_over_tau_d": tr["t"][-1],
            "n_peak_max": max(tr["n_peak"]),
            "n_peak_late_mean": float(np.mean(tr["n_peak"][half:])),
            "I_outer_max_A": max(tr["I_outer"]),
            "I_outer_late_mean_over_p": float(np.mean(tr["I_outer"][half:])) / p,
            "I_left_right_late_mean_A": float(np.mean(np.add(tr["I_left"][half:], tr["I_right"][half:]))),
            "n_live_end": tr["n_live"][-1],
            "n_ioniz": int(final[k]["n_ioniz"]), "n_source": int(final[k]["n_source"]),
            "peak_over_brillouin": max(tr["n_peak"]) / n_brillouin,
            "force_balance": forces[k],
        })
    res = {"pressures_mbar": pressures, "brillouin_density": n_brillouin, "wall_s": wall, "summary": summary,
           "traces": traces}
    if out:
        with open(out, "w") as f:
            json.dump(res, f)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pressures", default="0.025,0.05,0.1")
    ap.add_argument("--taud", type=float, default=20.0)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--out", default=None)
    ap.add_argument("--sigma-el", type=float, default=None, help="elastic cross section (m^2)")
    ap.add_argument("--V-inner", type=float, default=None)
    ap.add_argument("--V-end", type=float, default=None)
    ap.add_argument("--B0", type=float, default=None)
    ap.add_argument("--weight", type=float, default=None, help="electrons per macro-electron")
    a = ap.parse_args()
    over = {k: v for k, v in (("sigma_el", a.sigma_el), ("V_inner", a.V_inner), ("V_end", a.V_end), ("B0", a.B0),
                                            ("weight", a.weight))
            if v is not None}
    res = run([float(x) for x in a.pressures.split(",")], a.taud, a.every, a.out, **over)
    print(json.dumps({k: v for k, v in res.items() if k != "traces"}), flush=True)


if __name__ == "__main__":
    main()
