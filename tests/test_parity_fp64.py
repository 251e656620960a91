"""Parity of the plain FP64 GPU form against the FP64 CPU oracle.

Bars: the deposited fixed-point grid is bit-exact; particle positions are
bit-exact (push and remap use only +, *, / and sqrt, all correctly rounded on
both sides, with contraction off); velocities match within 1e-12 relative
(collisions call log/sin/cos/tan/atan, which may differ by an ulp between the
host and device math libraries); event counters are equal.
"""
import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import COUNTERS, by_key, gpu_and_oracle, rel_vec_err
from paper_2206_14662_amd import binding as B

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 1, 777, 20000, 100003])
def test_deposit_bit_exact(n):
    cfg = pi.coax64()
    st = pi.particle_state(cfg, n, seed=100 + n, margin_cells=0.01)
    g, o = gpu_and_oracle(cfg, st, pi.random_fields(cfg, 1))
    assert np.array_equal(g.charge(), o.charge())
    assert g.charge().sum() == n * round(cfg["weight"] * 2.0 ** o.S)


def test_deposit_bit_exact_fine_mesh_ragged():
    cfg = pi.coax256()
    st = pi.particle_state(cfg, 300001, seed=7, margin_cells=0.001)
    g, o = gpu_and_oracle(cfg, st, pi.random_fields(cfg, 2))
    assert np.array_equal(g.charge(), o.charge())


def test_one_step_with_collisions():
    cfg = pi.coax64(p_mbar=30.0, E_cap_eV=3000.0)
    st = pi.cloud_state(cfg, 20000, seed=3)
    g, o = gpu_and_oracle(cfg, st, pi.random_fields(cfg, 4))
    g.step(1)
    o.step(1)
    gd, od = g.diag(), o.diag()
    assert gd["n_elastic"] > 100 and gd["n_ioniz"] > 100
    for k in COUNTERS:
        assert gd[k] == od[k], k
    gp, op = by_key(g.get_particles()), by_key(o.get_particles())
    assert np.array_equal(gp["key"], op["key"])
    assert np.array_equal(gp["r"], op["r"]) and np.array_equal(gp["z"], op["z"])
    assert np.array_equal(gp["w"], op["w"])
    assert rel_vec_err(gp, op).max() <= 1e-12
    assert np.array_equal(g.charge(), o.charge())


def test_many_steps_frozen_no_collisions_bit_exact():
    cfg = pi.coax64(collisions=0, mirror_k=0.3)
    st = pi.cloud_state(cfg, 30000, seed=5)
    Br, Bz = oracle.bfield(cfg)
    f = pi.random_fields(cfg, 6, e_scale=5e5)
    f["Br"], f["Bz"] = Br, Bz
    g, o = gpu_and_oracle(cfg, st, f)
    g.step(200)
    o.step(200)
    gd, od = g.diag(), o.diag()
    for k in COUNTERS:
        assert gd[k] == od[k], k
    gp, op = by_key(g.get_particles()), by_key(o.get_particles())
    for k in ("key", "r", "z", "vr", "vt", "vz"):
        assert np.array_equal(gp[k], op[k]), k
    assert np.array_equal(g.charge(), o.charge())


def test_several_steps_with_collisions_frozen():
    cfg = pi.coax64(p_mbar=1.0, E_cap_eV=3000.0)
    st = pi.cloud_state(cfg, 20000, seed=8)
    g, o = gpu_and_oracle(cfg, st, pi.random_fields(cfg, 9))
    g.step(10)
    o.step(10)
    gd, od = g.diag(), o.diag()
    for k in ("n_live", "n_elastic", "n_ioniz", "n_null_cand", "n_absorbed"):
        assert gd[k] == od[k], k
    gp, op = by_key(g.get_particles()), by_key(o.get_particles())
    assert np.array_equal(gp["key"], op["key"])
    assert np.max(np.abs(gp["r"] - op["r"]) / op["r"]) < 1e-12
    assert rel_vec_err(gp, op).max() <= 1e-11


@pytest.mark.parametrize("end_mode", [0, 1, 2])
def test_vacuum_potential(end_mode):
    cfg = pi.coax64(mirror_k=0.3, end_mode=end_mode)
    g = B.Sim([dict(cfg, n_init=0)])
    ref = oracle.vacuum(cfg)
    assert np.max(np.abs(g.phi() - ref)) <= 1e-10 * np.max(np.abs(ref))
    f = g.fields()
    Er, Ez = oracle.efield(cfg, ref)
    Br, Bz = oracle.bfield(cfg)
    assert np.max(np.abs(f["Er"] - Er)) <= 1e-8 * np.max(np.abs(Er))
    assert np.max(np.abs(f["Ez"] - Ez)) <= 1e-8 * np.max(np.abs(Er))
    assert np.array_equal(f["Br"], Br) and np.array_equal(f["Bz"], Bz)


def tall(**kw):
    """A mesh taller than 257 cells in r (the tridiagonal solve then holds two
    row segments per wave)."""
    return pi.coax64(nr=400, nz=256, **kw)


@pytest.mark.parametrize("maker,end_mode", [(pi.coax64, 0), (pi.coax256, 0), (tall, 0), (pi.coax64, 2),
                                            (pi.coax256, 2), (tall, 2)])
def test_poisson_solve_matches_oracle(maker, end_mode):
    cfg = maker(end_mode=end_mode)
    st = pi.cloud_state(cfg, 50000, seed=11)
    g, o = gpu_and_oracle(cfg, st, fields=None)
    assert np.array_equal(g.charge(), o.charge())
    vac = oracle.vacuum(cfg)
    sc_g, sc_o = g.phi() - vac, o.phi() - vac
    assert np.max(np.abs(sc_g - sc_o)) <= 1e-9 * np.max(np.abs(sc_o))
    fg = g.fields()
    fo = o.get_fields()
    scale = np.max(np.abs(fo["Er"]))
    assert np.max(np.abs(fg["Er"] - fo["Er"])) <= 1e-8 * scale
    assert np.max(np.abs(fg["Ez"] - fo["Ez"])) <= 1e-8 * scale


@pytest.mark.parametrize("mode", [0, 1])
def test_initial_load_matches_oracle(mode):
    """Positions of the Philox-driven load use only +, *, sqrt: bit-exact
    device and host Philox streams give bit-exact positions."""
    cfg = pi.coax64(n_init=30011, load_mode=mode)
    g = B.Sim([cfg])
    o = oracle.Sim(cfg, fx_shift=B.pic_auto_shift(cfg["weight"]))
    o.load()
    gp, op = by_key(g.get_particles()), by_key(o.get_particles())
    assert np.array_equal(gp["key"], op["key"])
    assert np.array_equal(gp["r"], op["r"]) and np.array_equal(gp["z"], op["z"])
    sv = np.sqrt(cfg["T_init_eV"] * 1.602176634e-19 / 9.1093837015e-31)
    for k in ("vr", "vt", "vz"):
        assert np.max(np.abs(gp[k] - op[k])) <= 1e-12 * sv
    assert np.array_equal(g.charge(), o.charge())


def test_self_consistent_run_small_case():
    """The 64x128 trap from its Philox load for 500 steps (the small
    configuration), self-consistent field: diagnostics agree."""
    cfg = pi.coax64hot(diag_interval=10)
    S = B.pic_auto_shift(cfg["weight"])
    g = B.Sim([cfg])
    o = oracle.Sim(cfg, fx_shift=S)
    o.load()
    st = o.get_particles()
    g.set_particles(st)  # identical start (velocities from the host load)
    g.step(500)
    o.step(500)
    gd, od = g.diag(want_density=True), o.diag()
    assert gd["n_elastic"] > 1000 and gd["n_ioniz"] > 100
    for k in ("n_live", "n_elastic", "n_ioniz", "n_absorbed", "n_samples"):
        assert abs(np.sum(gd[k]) - np.sum(od[k])) <= 0.002 * max(1, np.sum(od[k])), k
    avg_o = o.time_avg_density()
    assert np.linalg.norm(gd["time_avg_density"] - avg_o) <= 1e-3 * np.linalg.norm(avg_o)


def test_full_size_sampled_one_step():
    """The 256x1024, 4M-electron case in the launch configuration: one step,
    then a sample of particles is replayed through the oracle with the same
    field and step counter."""
    cfg = pi.coax256()
    g = B.Sim([cfg])
    f0 = g.fields()
    before = g.get_particles()
    g.step(1)
    after = by_key(g.get_particles())
    d = g.diag()
    W = round(cfg["weight"] * 2.0 ** d["S"])
    assert d["total_Q"] == d["n_live"] * W
    rng = np.random.default_rng(0)
    idx = rng.choice(len(before["r"]), 4096, replace=False)
    sample = {k: v[idx] for k, v in before.items()}
    o = oracle.Sim(cfg, fx_shift=d["S"], capacity=8192)
    o.set_fields(**f0, frozen=1)
    o.set_particles(sample)
    o.step(1)
    op = by_key(o.get_particles())
    pos = np.searchsorted(after["key"], op["key"])
    ok = op["key"] < np.uint64(1 << 63)
    pos, opk = pos[ok], {k: v[ok] for k, v in op.items()}
    assert np.array_equal(after["key"][pos], opk["key"])
    for k in ("r", "z"):
        assert np.array_equal(after[k][pos], opk[k])
    assert rel_vec_err({k: after[k][pos] for k in ("vr", "vt", "vz")}, opk).max() <= 1e-12
