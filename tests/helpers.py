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
