"""Tabulated cross sections (LXCat-style energy / cross-section pairs) for
the MCC stage: the oracle's interpolation and null-collision bound pinned by
brute force and by the collision rate they produce; the GPU forms against the
oracle with a table; the return to the constant / Lotz model."""
import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import by_key, gpu_and_oracle, rel_vec_err
from paper_2206_14662_amd import binding as B

F32 = B.PIC_MODE_FP32_BATCHED
F64 = B.PIC_MODE_FP64_PLAIN
QE, ME = 1.602176634e-19, 9.1093837015e-31


def test_interpolation_is_linear_and_held_at_the_ends():
    E = np.array([1.0, 2.0, 4.0, 10.0])
    s = np.array([5.0, 3.0, 3.5, 1.0])
    assert oracle.xs_at(E, s, 0.5) == 5.0 and oracle.xs_at(E, s, 20.0) == 1.0
    for x, want in ((1.0, 5.0), (1.5, 4.0), (3.0, 3.25), (7.0, 2.25), (10.0, 1.0), (4.0, 3.5)):
        assert oracle.xs_at(E, s, x) == pytest.approx(want, rel=1e-15)


def test_null_bound_is_the_maximum_of_sigma_v():
    c = pi.coax64hot()
    rng = np.random.default_rng(5)
    for trial in range(5):
        E = np.sort(rng.uniform(0.0, 2.0 * c["E_cap_eV"], 40))
        E[0] = 0.0
        el = rng.uniform(0.0, 3e-19, 40)
        iz = rng.uniform(0.0, 1e-20, 40)
        got = oracle.xs_sigv_max(c, E, el, iz)
        x = np.linspace(0.0, c["E_cap_eV"], 400001)
        sel = np.interp(x, E, el)
        siz = np.where(x > c["iz_I_eV"], np.interp(x, E, iz), 0.0)
        brute = ((sel + siz) * np.sqrt(2 * QE * x / ME)).max()
        assert brute <= got * (1 + 1e-12) and got <= brute * (1 + 1e-4), (trial, got, brute)
    # a constant elastic table without ionisation: n sigma v_cap
    E = np.array([0.0, 1e6])
    got = oracle.xs_sigv_max(c, E, np.full(2, 1e-19), np.zeros(2))
    assert got == pytest.approx(1e-19 * np.sqrt(2 * QE * c["E_cap_eV"] / ME), rel=1e-14)


def test_bound_in_use_is_widened_and_rounded_up_to_12_bits():
    """The bound a table installs is the maximum of sigma v times (1 + 2^-20),
    rounded up to 12 significant bits: never below the widened maximum, less
    than 2^-11 above it, and a multiple of 2^(e - 12) for its binade."""
    rng = np.random.default_rng(9)
    for x in np.concatenate([rng.uniform(1e-14, 1e-12, 200), [2.0**-40, 3.0 * 2.0**-41, 1.2345e-13]]):
        b = oracle.xs_bound(x)
        w = x * (1 + 2.0**-20)
        assert w <= b < w * (1 + 2.0**-11)
        m, e = np.frexp(b)
        assert m * 4096 == np.floor(m * 4096)
    # already on the grid after widening: unchanged
    assert oracle.xs_bound(0.75 / (1 + 2.0**-20)) in (0.75, 0.75 + 2.0**-13)


def test_oracle_collision_rate_follows_the_table():
    """A mono-energetic beam: the elastic events per step are binomial with
    p = P_null n_n sigma(E) v / nu' for the table's sigma(E)."""
    c = pi.coax64(p_mbar=30.0, n_init=0)
    E0 = 137.0
    E, el, iz = pi.synthetic_xs(c)
    iz = np.zeros_like(iz)
    n = 200000
    v = np.sqrt(2 * QE * E0 / ME)
    rng = np.random.default_rng(6)
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    st = dict(r=np.full(n, 5e-3), z=np.full(n, 30e-3), vr=v * u[0], vt=v * u[1], vz=v * u[2],
              w=np.full(n, c["weight"]), key=np.arange(n, dtype=np.uint64))
    o = oracle.Sim(c, capacity=n + 1000)
    o.set_fields(**pi.uniform_fields(c), frozen=1)
    o.set_particles(st)
    o.set_cross_sections(E, el, iz)
    d = o.derived()
    o.step(1)
    got = o.diag()["n_elastic"]
    Es = 0.5 * ME * v * v / QE
    p = d["P_null"] * (d["n_n"] * np.interp(Es, E, el) * v) / d["nu_prime"]
    assert abs(got - n * p) <= 5 * np.sqrt(n * p * (1 - p)), (got, n * p)
    assert o.diag()["n_ioniz"] == 0


def test_oracle_table_of_the_analytic_model_reproduces_its_rates():
    """The constant elastic and Lotz cross sections sampled finely: event
    counts agree with the analytic model's within statistics (at a pressure
    where nu' dt << 1, so the two null bounds give the same per-step event
    probability to first order)."""
    c = pi.coax64(p_mbar=0.3, E_cap_eV=3000.0, n_init=0)
    st = pi.cloud_state(c, 60000, seed=8)
    E = np.geomspace(1e-3, 1e4, 4000)
    iz = np.array([oracle.sigma_iz(c, e) for e in E])
    runs = []
    for table in (False, True):
        o = oracle.Sim(c, capacity=200000)
        o.set_fields(**pi.uniform_fields(c, Bz=0.28), frozen=1)
        o.set_particles(st)
        if table:
            o.set_cross_sections(E, np.full_like(E, c["sigma_el"]), iz)
        o.step(20)
        runs.append(o.diag())
    for k in ("n_elastic", "n_ioniz"):
        a, b = runs[0][k], runs[1][k]
        assert a > 200 and abs(a - b) <= 5 * np.sqrt(a), (k, a, b)


def test_refused_tables():
    c = pi.coax64(n_init=0)
    o = oracle.Sim(c)
    for E, el, iz in (([1.0], [1.0], [0.0]), ([1.0, 1.0], [1e-19] * 2, [0.0] * 2),
                      ([1.0, 2.0], [-1e-19, 1e-19], [0.0] * 2)):
        with pytest.raises(ValueError):
            o.set_cross_sections(np.array(E), np.array(el), np.array(iz))


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [F64, F32])
def test_gpu_with_a_table_matches_the_oracle(mode):
    cfg = pi.coax64(p_mbar=30.0, E_cap_eV=3000.0)
    st = pi.cloud_state(cfg, 20000, seed=21)
    st = {k: (v.astype(np.float32).astype(np.float64) if v.dtype == np.float64 else v) for k, v in st.items()}
    f = {k: v.astype(np.float32).astype(np.float64) for k, v in pi.random_fields(cfg, 22).items()}
    E, el, iz = pi.synthetic_xs(cfg)
    g, o = gpu_and_oracle(cfg, st, f, mode=mode)
    g.set_cross_sections(0, E, el, iz)
    o.set_cross_sections(E, el, iz)
    g.step(1)
    o.step(1)
    gd, od = g.diag(), o.diag()
    assert gd["n_null_cand"] == od["n_null_cand"] > 100
    if mode == F64:
        assert gd["n_elastic"] == od["n_elastic"] and gd["n_ioniz"] == od["n_ioniz"]
        gp, op = by_key(g.get_particles()), by_key(o.get_particles())
        assert np.array_equal(gp["key"], op["key"])
        assert rel_vec_err(gp, op).max() <= 1e-12
        assert np.array_equal(g.charge(), o.charge())
    else:
        assert abs(gd["n_elastic"] - od["n_elastic"]) <= 2 and abs(gd["n_ioniz"] - od["n_ioniz"]) <= 2
    g.close()


@pytest.mark.gpu
def test_fp32_table_then_back_to_the_analytic_model():
    cfg = pi.coax64(p_mbar=3.0, n_init=40000, E_cap_eV=3000.0)
    ref = B.Sim([cfg], mode=F32)
    ref.step(20)
    want = (by_key(ref.get_particles()), ref.diag())
    ref.close()
    g = B.Sim([cfg], mode=F32)
    E, el, iz = pi.synthetic_xs(cfg)
    g.set_cross_sections(0, E, el, iz)
    g.set_cross_sections(0)  # back to constant elastic + Lotz before any step
    g.step(20)
    got = (by_key(g.get_particles()), g.diag())
    for k in ("key", "r", "z", "vr", "vt", "vz"):
        assert np.array_equal(want[0][k], got[0][k]), k
    assert got[1]["n_elastic"] == want[1]["n_elastic"]
    # with the table the candidate rate follows the table's tighter bound
    h = B.Sim([cfg], mode=F32)
    h.set_cross_sections(0, E, el, iz)
    h.step(20)
    d = h.diag()
    assert d["n_null_cand"] != want[1]["n_null_cand"] and d["n_elastic"] > 0
    with pytest.raises(B.PicError):
        h.set_cross_sections(0, np.array([2.0, 1.0]), np.ones(2) * 1e-19, np.zeros(2))
    h.close()
    g.close()
