"""Energy-dependent anisotropy of the scattering law (Sec. II.A: the angle
of Okhrimovskyy's analytic differential cross section depends on the
incoming energy).  CPU: the oracle's sampling law pinned by the closed-form
momentum-transfer moment of that cross section, and the mean energy loss of
elastic events following a tabulated xi(E).  GPU: both forms against the
oracle with a table, and a constant table against the constant parameter."""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import by_key, gpu_and_oracle, rel_vec_err
from paper_2206_14662_amd import binding as B

F32 = B.PIC_MODE_FP32_BATCHED
F64 = B.PIC_MODE_FP64_PLAIN
QE, ME, AMU = 1.602176634e-19, 9.1093837015e-31, 1.66053906660e-27


def mt_ratio(xi):
    """1 - <cos chi> of the cross section (1 - xi^2) / (1 - xi cos chi)^2,
    normalised over the sphere: the momentum-transfer over the integral
    cross section."""
    if xi == 0.0:
        return 1.0
    return 1.0 - 1.0 / xi + (1.0 - xi * xi) / (2.0 * xi * xi) * math.log((1.0 + xi) / (1.0 - xi))


def xi_table():
    """A synthetic xi(E): isotropic at low energy, forward-peaked at keV."""
    E = np.array([0.0, 10.0, 50.0, 100.0, 300.0, 1000.0, 1e5])
    xi = np.array([0.0, 0.2, 0.6, 0.8, 0.9, 0.95, 0.99])
    return E, xi


def test_sampling_law_has_the_cross_section_momentum_transfer_moment():
    n = 400000
    u = (np.arange(n) + 0.5) / n
    for xi in (-0.5, 0.0, 0.3, 0.8, 0.95):
        mu = np.array([oracle.okh_cos(xi, x) for x in u])
        assert mu.min() >= -1.0 - 1e-12 and mu.max() <= 1.0 + 1e-12
        assert np.mean(1.0 - mu) == pytest.approx(mt_ratio(xi), abs=2e-5), xi


def test_oracle_elastic_loss_follows_the_table():
    """Mono-energetic electrons without fields, elastic events only: each
    event loses (2m/M)(1 - cos chi) of the energy, so the mean loss over the
    events gives 1 - <cos chi> at the table's xi(E0), not at okh_xi."""
    c = pi.coax64(p_mbar=30.0, n_init=0, E_cap_eV=3000.0, okh_xi=0.0)
    E0, n = 100.0, 120000
    v = math.sqrt(2 * QE * E0 / ME)
    rng = np.random.default_rng(31)
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    st = dict(r=np.full(n, 5e-3), z=np.full(n, 30e-3), vr=v * u[0], vt=v * u[1], vz=v * u[2],
              w=np.full(n, c["weight"]), key=np.arange(n, dtype=np.uint64))
    E, xi = xi_table()
    want_xi = float(np.interp(E0, E, xi))
    o = oracle.Sim(c, capacity=n + 1000)
    o.set_fields(**pi.uniform_fields(c, Bz=0.0), frozen=1)
    o.set_particles(st)
    o.set_cross_sections(np.array([0.0, 1e6]), np.full(2, c["sigma_el"]), np.zeros(2))
    o.set_anisotropy(E, xi)
    o.step(1)
    p = by_key(o.get_particles())
    d = o.diag()
    o.close()
    En = 0.5 * ME * (p["vr"] ** 2 + p["vt"] ** 2 + p["vz"] ** 2) / QE
    rel = 1.0 - En / E0
    hit = np.abs(rel) > 1e-9
    assert hit.sum() == d["n_elastic"] > 5000 and d["n_ioniz"] == 0
    m_ratio = 2.0 * ME / (c["M_gas_amu"] * AMU)
    got = rel[hit].mean() / m_ratio
    sd = rel[hit].std() / m_ratio / math.sqrt(hit.sum())
    assert abs(got - mt_ratio(want_xi)) <= 5 * sd, (got, mt_ratio(want_xi), sd)
    assert abs(got - mt_ratio(0.0)) > 20 * sd


E_HARTREE = 27.211386245988   # eV, the atomic unit of energy


def test_screened_coulomb_xi_hand_values():
    """xi(E) = 4 e / (1 + 4 e), e = E / E0: 0 at rest, 1/2 at E0/4, 3/4 at
    3E0/4, 4/5 at E0, rising to 1 at high energy."""
    E0 = E_HARTREE
    for E, want in ((0.0, 0.0), (0.25 * E0, 0.5), (0.75 * E0, 0.75), (E0, 0.8), (10.0 * E0, 40.0 / 41.0)):
        assert oracle.xi_sc(E0, E) == pytest.approx(want, rel=1e-15, abs=1e-300)
    assert oracle.xi_sc(E0, 1e6) > 0.9999


def test_oracle_elastic_loss_follows_the_screened_coulomb_xi():
    """Mono-energetic elastic events with okh_E0_eV set: the mean energy loss
    gives 1 - <cos chi> at xi(E0) of the closed form, not at okh_xi."""
    E0, n = 150.0, 120000
    c = pi.coax64(p_mbar=30.0, n_init=0, E_cap_eV=3000.0, okh_xi=0.0, okh_E0_eV=E_HARTREE, lotz_a=0.0)
    v = math.sqrt(2 * QE * E0 / ME)
    rng = np.random.default_rng(35)
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    st = dict(r=np.full(n, 5e-3), z=np.full(n, 30e-3), vr=v * u[0], vt=v * u[1], vz=v * u[2],
              w=np.full(n, c["weight"]), key=np.arange(n, dtype=np.uint64))
    o = oracle.Sim(c, capacity=n + 1000)
    o.set_fields(**pi.uniform_fields(c, Bz=0.0), frozen=1)
    o.set_particles(st)
    o.step(1)
    p = by_key(o.get_particles())
    d = o.diag()
    o.close()
    En = 0.5 * ME * (p["vr"] ** 2 + p["vt"] ** 2 + p["vz"] ** 2) / QE
    rel = 1.0 - En / E0
    hit = np.abs(rel) > 1e-14    # forward-peaked: some events lose < 1e-9
    assert hit.sum() == d["n_elastic"] > 5000
    m_ratio = 2.0 * ME / (c["M_gas_amu"] * AMU)
    got = rel[hit].mean() / m_ratio
    sd = rel[hit].std() / m_ratio / math.sqrt(hit.sum())
    xi = 4 * (E0 / E_HARTREE) / (1 + 4 * (E0 / E_HARTREE))
    assert abs(got - mt_ratio(xi)) <= 5 * sd, (got, mt_ratio(xi), sd)
    assert abs(got - mt_ratio(0.0)) > 20 * sd


def test_refused_anisotropy_tables():
    o = oracle.Sim(pi.coax64(n_init=0))
    for E, xi in (([1.0], [0.1]), ([1.0, 1.0], [0.1, 0.2]), ([1.0, 2.0], [0.1, 1.0]), ([1.0, 2.0], [-1.0, 0.0])):
        with pytest.raises(ValueError):
            o.set_anisotropy(np.array(E), np.array(xi))
    o.set_anisotropy(*xi_table())
    o.set_anisotropy()
    o.close()


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [F64, F32])
def test_gpu_with_anisotropy_matches_the_oracle(mode):
    cfg = pi.coax64(p_mbar=30.0, E_cap_eV=3000.0)
    st = pi.cloud_state(cfg, 20000, seed=33)
    st = {k: (v.astype(np.float32).astype(np.float64) if v.dtype == np.float64 else v) for k, v in st.items()}
    f = {k: v.astype(np.float32).astype(np.float64) for k, v in pi.random_fields(cfg, 34).items()}
    g, o = gpu_and_oracle(cfg, st, f, mode=mode)
    E, xi = xi_table()
    g.set_anisotropy(0, E, xi)
    o.set_anisotropy(E, xi)
    g.step(2)
    o.step(2)
    gd, od = g.diag(), o.diag()
    assert gd["n_null_cand"] == od["n_null_cand"] > 100
    if mode == F64:
        assert gd["n_elastic"] == od["n_elastic"] > 100 and gd["n_ioniz"] == od["n_ioniz"] > 10
        gp, op = by_key(g.get_particles()), by_key(o.get_particles())
        assert np.array_equal(gp["key"], op["key"])
        assert rel_vec_err(gp, op).max() <= 1e-12
        assert np.array_equal(g.charge(), o.charge())
    else:
        assert abs(gd["n_elastic"] - od["n_elastic"]) <= 2 and abs(gd["n_ioniz"] - od["n_ioniz"]) <= 2
    g.close()


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [F64, F32])
def test_gpu_screened_coulomb_xi_matches_the_oracle(mode):
    cfg = pi.coax64(p_mbar=30.0, E_cap_eV=3000.0, okh_E0_eV=E_HARTREE)
    st = pi.cloud_state(cfg, 20000, seed=36)
    st = {k: (v.astype(np.float32).astype(np.float64) if v.dtype == np.float64 else v) for k, v in st.items()}
    f = {k: v.astype(np.float32).astype(np.float64) for k, v in pi.random_fields(cfg, 37).items()}
    g, o = gpu_and_oracle(cfg, st, f, mode=mode)
    g.step(2)
    o.step(2)
    gd, od = g.diag(), o.diag()
    assert gd["n_null_cand"] == od["n_null_cand"] > 100
    if mode == F64:
        assert gd["n_elastic"] == od["n_elastic"] > 100 and gd["n_ioniz"] == od["n_ioniz"] > 10
        gp, op = by_key(g.get_particles()), by_key(o.get_particles())
        assert np.array_equal(gp["key"], op["key"])
        assert rel_vec_err(gp, op).max() <= 1e-12
        assert np.array_equal(g.charge(), o.charge())
    else:
        assert abs(gd["n_elastic"] - od["n_elastic"]) <= 2 and abs(gd["n_ioniz"] - od["n_ioniz"]) <= 2
    g.close()


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [F64, F32])
def test_constant_table_is_the_constant_parameter(mode):
    cfg = pi.coax64(p_mbar=3.0, n_init=30000, E_cap_eV=3000.0, okh_xi=0.4)
    runs = []
    for table in (False, True):
        g = B.Sim([cfg], mode=mode)
        if table:
            g.set_anisotropy(0, np.array([0.0, 1e6]), np.full(2, 0.4))
        g.step(10)
        runs.append((by_key(g.get_particles()), g.diag()))
        if table:
            g.set_anisotropy(0)
            with pytest.raises(B.PicError):
                g.set_anisotropy(0, np.array([2.0, 1.0]), np.zeros(2))
        g.close()
    for k in ("key", "r", "z", "vr", "vt", "vz"):
        assert np.array_equal(runs[0][0][k], runs[1][0][k]), k
    assert runs[0][1]["n_elastic"] == runs[1][1]["n_elastic"] > 0
