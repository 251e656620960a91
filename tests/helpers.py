"""Shared test helpers: pair a GPU context with an oracle instance on the same
inputs, and compare particle sets matched by key."""
import numpy as np

import oracle
from paper_2206_14662_amd import binding as B


def by_key(st):
    o = np.argsort(st["key"], kind="stable")
    return {k: np.asarray(v)[o] for k, v in st.items()}


def gpu_and_oracle(cfg, state, fields=None, frozen=1, mode=B.PIC_MODE_FP64_PLAIN, **run):
    """A one-instance GPU context and an oracle instance holding `state`,
    both with the fixed-point shift of the configured weight."""
    S = B.pic_auto_shift(cfg["weight"])
    n = len(state["r"])
    run.setdefault("capacity_min", max(4096, 4 * n + 1024))
    g = B.Sim([dict(cfg, n_init=0, fx_shift=S)], mode=mode, **run)
    o = oracle.Sim(dict(cfg), fx_shift=S, capacity=max(1024, 2 * n))
    if fields is not None:
        g.set_fields(frozen=frozen, **fields)
        o.set_fields(**fields, frozen=frozen)
    g.set_particles(state)
    o.set_particles(state)
    return g, o


def rel_vec_err(a, b):
    """Per-particle relative error of the velocity vector."""
    da = np.sqrt((a["vr"] - b["vr"]) ** 2 + (a["vt"] - b["vt"]) ** 2 + (a["vz"] - b["vz"]) ** 2)
    nb = np.sqrt(b["vr"] ** 2 + b["vt"] ** 2 + b["vz"] ** 2)
    return da / np.maximum(nb, 1e-300)


COUNTERS = ("n_live", "n_elastic", "n_ioniz", "n_null_cand", "n_cap_overflow", "n_absorbed",
            "absorbed_W", "total_Q", "n_samples")


def f32_values(st):
    """A state whose floating-point arrays hold FP32 values (so the FP32 form
    and the FP64 oracle start from identical numbers)."""
    return {k: (v.astype(np.float32).astype(np.float64) if v.dtype.kind == "f" else v) for k, v in st.items()}


# Element-wise bars of one FP32 step against the FP64 oracle from the same
# FP32-valued state and field: the velocity error relative to the magnitudes
# the step adds up, |v_before| + |v_after| + |v_after - v_before| (the
# rounding of an FP32 sum scales with its terms, not with its result, which
# can nearly cancel for a slow electron), for the push alone and for a
# particle the oracle scattered, whose FP32 scattering (uniforms of 23 instead
# of 52 bits, float sincos/tan/atan/log) is ill-conditioned near back-scatter.
# Worst cases measured over 62 sampled steps (up to 400k electrons each):
# push 1.6e-7, scattered 2.9e-5, position 1.8e-7, one decision flip.
TOL_PUSH32 = 1e-6
TOL_COLL32 = 1e-4
TOL_POS32 = 1e-6


def fp32_step_parity(after, ref, ref_nocoll, max_flips, before=None):
    """Compare particles `after` (FP32 form, one step) with the oracle's `ref`
    from the same state, and with `ref_nocoll` (the oracle without the
    collision stage, which tells which particles the oracle scattered).
    Every particle present on both sides is matched by key; a decision flip
    is a particle present on one side only (an absorption or an ionisation
    decided differently at FP32 rounding) or one beyond its bar.  `before`
    (the state the step started from) sets each particle's velocity scale.
    Asserts the bars on all others and at most max_flips flips; returns the
    counts."""
    a, o, z = by_key(after), by_key(ref), by_key(ref_nocoll)
    keys = np.intersect1d(a["key"], o["key"])
    only = len(a["key"]) + len(o["key"]) - 2 * len(keys)
    ai, oi = np.searchsorted(a["key"], keys), np.searchsorted(o["key"], keys)
    aq = {k: v[ai] for k, v in a.items()}
    oq = {k: v[oi] for k, v in o.items()}
    zi = np.searchsorted(z["key"], keys)
    zi = np.minimum(zi, len(z["key"]) - 1)
    inz = z["key"][zi] == keys
    scattered = ~inz | (z["vr"][zi] != oq["vr"]) | (z["vt"][zi] != oq["vt"]) | (z["vz"][zi] != oq["vz"])
    speed = lambda d: np.sqrt(d["vr"] ** 2 + d["vt"] ** 2 + d["vz"] ** 2)
    scale = speed(oq)
    if before is not None:
        b = by_key(before)
        bi = np.minimum(np.searchsorted(b["key"], keys), len(b["key"]) - 1)
        inb = b["key"][bi] == keys
        bq = {k: np.where(inb, b[k][bi], oq[k]) for k in ("vr", "vt", "vz")}
        dv = {k: oq[k] - bq[k] for k in ("vr", "vt", "vz")}
        scale = scale + speed(bq) + speed(dv)
    dva = np.sqrt((aq["vr"] - oq["vr"]) ** 2 + (aq["vt"] - oq["vt"]) ** 2 + (aq["vz"] - oq["vz"]) ** 2)
    err = dva / np.maximum(scale, 1e-300)
    pos = np.maximum(np.abs(aq["r"] / oq["r"] - 1.0), np.abs(aq["z"] / oq["z"] - 1.0))
    bar = np.where(scattered, TOL_COLL32, TOL_PUSH32)
    bad = (err > bar) | (pos > TOL_POS32) | (aq["w"] != oq["w"])
    flips = only + int(bad.sum())
    ok = ~bad
    res = dict(matched=len(keys), scattered=int(scattered.sum()), flips=flips,
               max_err_push=float(err[ok & ~scattered].max(initial=0.0)),
               max_err_scattered=float(err[ok & scattered].max(initial=0.0)),
               max_pos=float(pos[ok].max(initial=0.0)))
    print("fp32 step parity:", res, flush=True)
    a_only = np.setdiff1d(a["key"], keys)
    o_only = np.setdiff1d(o["key"], keys)
    for kk in a_only[:4]:
        print("  flip: only in the FP32 step, key", int(kk), flush=True)
    for kk in o_only[:4]:
        print("  flip: only in the oracle step, key", int(kk), flush=True)
    for t in np.nonzero(bad)[0][:6]:
        sp = float(np.sqrt(oq["vr"][t] ** 2 + oq["vt"][t] ** 2 + oq["vz"][t] ** 2))
        print(f"  flip: key {int(keys[t])} scattered {bool(scattered[t])} err {err[t]:.3g} pos {pos[t]:.3g} "
              f"speed {sp:.4g} r {oq['r'][t]:.6g} z {oq['z'][t]:.6g}", flush=True)
    assert flips <= max_flips, res
    return res
