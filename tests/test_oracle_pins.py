"""Pins of the FP64 CPU oracle against closed forms, invariants, brute force
and the paper's printed time scales (no GPU).

Each test names the part of the oracle it pins and the fact it checks; a
dropped term, a flipped sign or a transposed index in the oracle fails at
least one of them.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
import pic_inputs as pi

E = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12
KB = 1.380649e-23
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def quiet(**over):
    """Small trap with collisions off, for single-particle orbit tests."""
    c = pi.coax64(collisions=0, p_mbar=1e-12, **over)
    return c


def one_particle(c, r, z, vr, vt, vz, key=7):
    return dict(r=np.array([r]), z=np.array([z]), vr=np.array([vr]), vt=np.array([vt]),
                vz=np.array([vz]), w=np.array([c["weight"]]), key=np.array([key], dtype=np.uint64))


def frozen_sim(c, fields, state):
    s = oracle.Sim(c)
    s.set_fields(**fields, frozen=1)
    s.set_particles(state)
    return s


# --------------------------------------------------------------------------
# Philox and uniforms: the generator against its published known-answer
# vectors, the uniforms by behaviour.
# --------------------------------------------------------------------------

def test_philox_known_answer_vectors():
    kat = json.load(open(os.path.join(GOLD, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert [int(x) for x in oracle.philox(ctr, key)] == [int(x, 16) for x in v["out"]]


def test_philox_uniform_and_bit_balance():
    n = 1 << 14
    words = np.array([oracle.philox([i, 0, 5, 0], [123, 456]) for i in range(n)], dtype=np.uint64)
    # every output bit is set half of the time
    bits = np.stack([(words >> np.uint64(b)) & np.uint64(1) for b in range(32)], axis=-1)
    frac = bits.mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 5.0 * 0.5 / math.sqrt(n))
    # u52 of (w0,w1) is uniform on (0,1)
    u = np.array([oracle.u52(int(a), int(b)) for a, b in words[:, :2]])
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    assert u.min() > 0.0 and u.max() < 1.0


def test_philox_avalanche_and_key_dependence():
    rng = np.random.default_rng(1)
    flips = []
    for _ in range(300):
        ctr = [int(x) for x in rng.integers(0, 2**32, 4)]
        key = [int(x) for x in rng.integers(0, 2**32, 2)]
        base = oracle.philox(ctr, key)
        bit = int(rng.integers(0, 128))
        c2 = list(ctr)
        c2[bit // 32] ^= 1 << (bit % 32)
        o2 = oracle.philox(c2, key)
        flips.append(sum(bin(a ^ b).count("1") for a, b in zip(base, o2)))
        k2 = list(key)
        k2[0] ^= 1
        assert oracle.philox(ctr, k2) != base
    # a 10-round bijective mixer flips about half of the 128 output bits
    assert abs(np.mean(flips) - 64.0) < 2.0


def test_u52_open_interval_and_monotone():
    assert oracle.u52(0, 0) == 0.5 * 2.0**-52
    assert oracle.u52(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 0.5 * 2.0**-52
    assert oracle.u52(0, 1 << 12) > oracle.u52(0, 0)


# --------------------------------------------------------------------------
# Derived constants
# --------------------------------------------------------------------------

def test_derived_constants_closed_forms():
    c = pi.coax64()
    d = oracle.derive(c)
    assert d["n_n"] == pytest.approx(100.0 * 1e-6 / (KB * 300.0), rel=1e-14)
    assert d["n_n"] == pytest.approx(2.414e16, rel=1e-3)
    nu = d["n_n"] * (c["sigma_el"] + d["sig_iz_max"]) * d["v_cap"]
    assert d["P_null"] == pytest.approx(1.0 - math.exp(-nu * c["dt"]), rel=1e-9)
    assert 0.5 * ME * d["v_cap"] ** 2 / E == pytest.approx(c["E_cap_eV"], rel=1e-14)
    # the Lotz maximum in closed form equals the numerical maximum
    Es = np.linspace(c["iz_I_eV"] * 1.01, 400.0, 200001)
    sig = np.array([oracle.sigma_iz(c, x) for x in Es[::50]])
    assert d["sig_iz_max"] == pytest.approx(sig.max(), rel=1e-5)
    assert oracle.sigma_iz(c, c["iz_I_eV"]) == 0.0
    assert oracle.sigma_iz(c, 0.5 * c["iz_I_eV"]) == 0.0


def test_fixed_point_shift_rule():
    for w in (1.0, 312.5, 1250.0, 1e5, 3.3e7):
        S = oracle.auto_shift(w)
        assert w * 2.0**S <= 2.0**31 < w * 2.0 ** (S + 1)


# --------------------------------------------------------------------------
# Push: Boris rotation, remap, leapfrog positions (closed forms)
# --------------------------------------------------------------------------

def gyration_closed_form(r0, v0r, v0t, B, dt, n):
    """Boris in a uniform Bz rotates v by alpha = 2 atan(Omega dt / 2) per
    step (counter-clockwise for an electron in +Bz); positions follow
    x^n = x^0 + dt V sum_{m=1..n} e^{i m alpha}."""
    Om = E * B / ME
    alpha = 2.0 * math.atan(0.5 * Om * dt)
    V = complex(v0r, v0t)
    q = cmath.exp(1j * alpha)
    xs, vs = [], []
    for k in range(1, n + 1):
        x = r0 + dt * V * q * (1 - q**k) / (1 - q)
        xs.append(x)
        vs.append(V * q**k * cmath.exp(-1j * cmath.phase(x)))
    return np.array(xs), np.array(vs), alpha


def test_gyration_matches_closed_form():
    c = quiet()
    B = 0.28
    st = one_particle(c, 5e-3, 30e-3, 4e5, -7e5, 0.0)
    s = frozen_sim(c, pi.uniform_fields(c, Bz=B), st)
    n = 1500
    rs, vrs, vts = [], [], []
    for _ in range(n):
        s.step(1)
        p = s.get_particles()
        rs.append(p["r"][0]); vrs.append(p["vr"][0]); vts.append(p["vt"][0])
    xs, vs, alpha = gyration_closed_form(5e-3, 4e5, -7e5, B, c["dt"], n)
    np.testing.assert_allclose(rs, np.abs(xs), rtol=1e-12, atol=0)
    np.testing.assert_allclose(vrs, vs.real, rtol=0, atol=1e-10 * abs(complex(4e5, -7e5)))
    np.testing.assert_allclose(vts, vs.imag, rtol=0, atol=1e-10 * abs(complex(4e5, -7e5)))
    assert alpha == pytest.approx(2 * math.atan(0.5 * E * B / ME * c["dt"]), rel=1e-15)


def test_speed_conserved_under_pure_B():
    c = quiet(mirror_k=0.3)
    st = pi.cloud_state(c, 200, seed=4)
    st["vz"] *= 0.0  # stay well inside in z
    Br, Bz = oracle.bfield(c)
    s = frozen_sim(c, dict(Er=np.zeros_like(Br), Ez=np.zeros_like(Br), Br=Br, Bz=Bz), st)
    v0 = np.sqrt(st["vr"] ** 2 + st["vt"] ** 2 + st["vz"] ** 2)
    s.step(3000)
    p = s.get_particles()
    order = np.argsort(p["key"])
    v1 = np.sqrt(p["vr"] ** 2 + p["vt"] ** 2 + p["vz"] ** 2)[order]
    alive = p["key"][order].astype(np.int64)
    assert len(alive) > 150
    np.testing.assert_allclose(v1, v0[alive], rtol=1e-12)


def test_mirror_field_reflects_at_the_adiabatic_turning_point():
    """The mirror field B_z = B0 (1 + k zeta^2), zeta = (z - L/2)/(L/2), with
    B_r = -(r/2) dB_z/dz (divergence-free): a 100 eV electron at the centre
    with sin^2 of its pitch angle 0.85 keeps its magnetic moment (Larmor
    radius 1e-3 of the field's scale), so it turns where B = B0 / 0.85,
    zeta = sqrt((1/0.85 - 1)/k), and its guiding centre stays on its field
    line, r^2 B_z constant.  A dropped or sign-flipped B_r removes the mirror
    force (the electron reaches the end plate); B_r off by a factor moves the
    guiding centre off the line; a wrong zeta moves the turning point."""
    k = 0.3
    c = quiet(mirror_k=k)
    Br, Bz = oracle.bfield(c)
    L, r0 = c["L"], 5.5e-3
    v = math.sqrt(2.0 * 100.0 * E / ME)
    s2 = 0.85
    # all the perpendicular speed radial: the gyration centre sits beside the
    # electron in theta, at radius sqrt(r0^2 + rL^2)
    st = one_particle(c, r0, L / 2, v * math.sqrt(s2), 0.0, v * math.sqrt(1.0 - s2))
    rL = ME * v * math.sqrt(s2) / (E * c["B0"])
    s = frozen_sim(c, dict(Er=np.zeros_like(Br), Ez=np.zeros_like(Br), Br=Br, Bz=Bz), st)
    zs, rs = [], []
    for _ in range(6000):
        s.step(5)
        p = s.get_particles()
        assert len(p["r"]) == 1, "the electron left the trap"
        zs.append(p["z"][0]); rs.append(p["r"][0])
    zs, rs = np.array(zs), np.array(rs)
    zeta_turn = math.sqrt((1.0 / s2 - 1.0) / k)
    top = int(np.argmax(zs))
    assert 0 < top < len(zs) - 100 and zs[-1] < zs[top] - 5e-3  # turned and came back
    assert (zs[top] - L / 2) / (L / 2) == pytest.approx(zeta_turn, rel=0.01)
    # guiding centre near the turning point: r averaged over the samples within
    # 0.5 mm of it (many gyrations, the electron is slow there)
    near = np.abs(zs - zs[top]) < 0.5e-3
    assert near.sum() > 100
    r_gc = math.hypot(r0, rL) * math.sqrt(1.0 / (1.0 + k * zeta_turn ** 2))
    assert rs[near].mean() == pytest.approx(r_gc, rel=0.005)


def test_free_streaming_straight_line_and_angular_momentum():
    c = quiet()
    r0, z0, vr, vt, vz = 4e-3, 25e-3, -3e5, 8e5, 2e5
    s = frozen_sim(c, pi.uniform_fields(c), one_particle(c, r0, z0, vr, vt, vz))
    dt = c["dt"]
    for n in range(1, 2001):
        s.step(1)
        if n % 250 == 0:
            p = s.get_particles()
            r_exact = math.hypot(r0 + vr * n * dt, vt * n * dt)
            assert p["r"][0] == pytest.approx(r_exact, rel=1e-12)
            assert p["z"][0] == pytest.approx(z0 + vz * n * dt, rel=1e-12)
            assert p["r"][0] * p["vt"][0] == pytest.approx(r0 * vt, rel=1e-12)
            assert math.hypot(p["vr"][0], p["vt"][0]) == pytest.approx(math.hypot(vr, vt), rel=1e-13)


def test_exb_rigid_rotor_orbit():
    """Circular orbit in uniform E_r, Bz: the slow root of
    m w^2 r0 = e (E_r + w r0 Bz) (electron, q = -e); its azimuthal speed
    approaches the E x B drift u_theta = -E_r / Bz (Sec. IV.A, eq. for u_theta)."""
    c = quiet()
    B, Er, r0 = 0.28, -2.0e5, 5e-3
    disc = (E * r0 * B) ** 2 + 4.0 * ME * r0 * E * Er
    w = (E * r0 * B - math.sqrt(disc)) / (2.0 * ME * r0)
    vt0 = w * r0
    vE, Om = -Er / B, E * B / ME
    assert vt0 == pytest.approx(vE, rel=2.0 * vE / (Om * r0))
    s = frozen_sim(c, pi.uniform_fields(c, Er=Er, Bz=B), one_particle(c, r0, 30e-3, 0.0, vt0, 0.0))
    rs, vts = [], []
    for _ in range(2000):
        s.step(1)
        p = s.get_particles()
        rs.append(p["r"][0]); vts.append(p["vt"][0])
    assert np.max(np.abs(np.array(rs) - r0)) / r0 < 1e-3
    assert np.mean(vts) == pytest.approx(vt0, rel=1e-3)


def test_cyclotron_period_vs_paper_and_limit():
    gold = json.load(open(os.path.join(GOLD, "paper_timescales.json")))
    B = gold["tau_ce_B_T"]
    for dt, rel in ((1e-12, 3e-4), (1e-14, 1e-7)):
        alpha = 2.0 * math.atan(0.5 * E * B / ME * dt)
        T = 2.0 * math.pi / alpha * dt
        assert T == pytest.approx(2.0 * math.pi * ME / (E * B), rel=rel)
    # the oracle's orbit rotates by alpha per step: measure it over one period
    c = quiet()
    s = frozen_sim(c, pi.uniform_fields(c, Bz=B), one_particle(c, 5e-3, 30e-3, 3e5, 0.0, 0.0))
    xs, vs, alpha = gyration_closed_form(5e-3, 3e5, 0.0, B, c["dt"], 1)
    T_orbit = 2.0 * math.pi / alpha * c["dt"]
    f = gold["tolerance_factor"]
    assert gold["tau_ce_s"] / f < T_orbit < gold["tau_ce_s"] * f
    # plasma period at the quoted density
    wp = math.sqrt(gold["tau_pe_density_m3"] * E * E / (EPS0 * ME))
    assert gold["tau_pe_s"] / f < 2 * math.pi / wp < gold["tau_pe_s"] * f


def test_gather_reproduces_bilinear_fields():
    """With B = 0 and v = 0 one step gives v_r = 2 h E_r(x) exactly (no
    rotation since y = 0), so the gathered field is observable; bilinear
    weights reproduce fields of the form alpha + beta r + gamma z + delta r z."""
    c = quiet()
    d = oracle.derive(c)
    nr, nz = c["nr"], c["nz"]
    r = c["a"] + d["dr"] * np.arange(nr + 1)[:, None]
    z = d["dz"] * np.arange(nz + 1)[None, :]
    Er = 3e5 + 2e7 * r - 5e6 * z + 4e9 * r * z
    Ez = -1e5 + 7e6 * z + 1e7 * r
    f = dict(Er=Er, Ez=Ez, Br=np.zeros_like(Er), Bz=np.zeros_like(Er))
    st = pi.particle_state(c, 400, seed=11, v_scale=0.0)
    s = frozen_sim(c, f, st)
    s.step(1)
    p = s.get_particles()
    k = p["key"].astype(np.int64)
    r0, z0 = st["r"][k], st["z"][k]
    np.testing.assert_allclose(p["vr"] / (2 * d["h"]), 3e5 + 2e7 * r0 - 5e6 * z0 + 4e9 * r0 * z0,
                               rtol=1e-11, atol=1e-9 * 3e5)
    np.testing.assert_allclose(p["vz"] / (2 * d["h"]), -1e5 + 7e6 * z0 + 1e7 * r0,
                               rtol=1e-11, atol=1e-9 * 1e5)


# --------------------------------------------------------------------------
# Deposit (brute force with hat functions, exact charge)
# --------------------------------------------------------------------------

def test_deposit_brute_force_hat_functions():
    c = pi.coax64(nr=8, nz=12)
    d = oracle.derive(c)
    S = oracle.auto_shift(c["weight"])
    W = round(c["weight"] * 2.0**S)
    rn = c["a"] + d["dr"] * np.arange(c["nr"] + 1)
    zn = d["dz"] * np.arange(c["nz"] + 1)
    rng = np.random.default_rng(5)
    for _ in range(200):
        r = rng.uniform(c["a"], c["b"])
        z = rng.uniform(0, c["L"])
        Q = oracle.deposit_one(c, r, z, c["weight"], fx_shift=S)
        hat_r = np.maximum(0.0, 1.0 - np.abs(r - rn) / d["dr"])
        hat_z = np.maximum(0.0, 1.0 - np.abs(z - zn) / d["dz"])
        N = np.outer(hat_r, hat_z)
        assert Q.sum() == W
        assert np.max(np.abs(Q - W * N)) <= 3.0  # rounding, plus the exact-sum remainder
        assert np.count_nonzero(Q) <= 4
        # first moments of the hat-function projection are preserved
        assert abs((Q.sum(axis=1) * rn).sum() - W * r) <= 4 * d["dr"]
        assert abs((Q.sum(axis=0) * zn).sum() - W * z) <= 4 * d["dz"]


# --------------------------------------------------------------------------
# Field solve (closed forms, convergence, symmetry)
# --------------------------------------------------------------------------

def coax_exact(c, r):
    return c["V_inner"] + (c["V_outer"] - c["V_inner"]) * np.log(r / c["a"]) / math.log(c["b"] / c["a"])


def test_vacuum_coax_second_order():
    """With end_mode 0 and V_end = 0 the electrode data are the coaxial
    profile V ln(r/a)/ln(b/a) everywhere; the discrete solution and the nodal
    E converge to it at second order (E is pre-asymptotic on coarse meshes
    because ln r curves strongly near r = a)."""
    errs, eerrs = [], []
    for nr in (32, 64, 128, 256):
        c = pi.coax64(nr=nr, nz=16, V_end=0.0)
        phi = oracle.vacuum(c)
        d = oracle.derive(c)
        r = c["a"] + d["dr"] * np.arange(nr + 1)
        exact = coax_exact(c, r)[:, None]
        errs.append(np.max(np.abs(phi - exact)) / abs(c["V_inner"]))
        Er, Ez = oracle.efield(c, phi)
        Er_exact = -(c["V_outer"] - c["V_inner"]) / (r * math.log(c["b"] / c["a"]))
        eerrs.append(np.max(np.abs(Er - Er_exact[:, None])) / np.max(np.abs(Er_exact)))
    assert errs[-1] < 2e-5
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(orders) > 1.95, (errs, orders)
    eorders = [math.log2(eerrs[i] / eerrs[i + 1]) for i in range(3)]
    assert eorders[0] < eorders[1] < eorders[2] and eorders[2] > 1.85, (eerrs, eorders)


def test_uniform_charge_column_closed_form():
    """Uniform electron density n0 filling a < r < b with phi = 0 on the
    electrodes: far from the ends phi = (e n0 / 4 eps0) r^2 + C1 ln r + C2."""
    n0 = 1e15
    errs = []
    for nr in (16, 32, 64):
        c = pi.coax64(nr=nr, nz=4 * nr)
        S = 10
        V = oracle.node_volume(c)
        Q = np.rint(n0 * V * 2.0**S).astype(np.int64)
        phi = oracle.poisson_charge(c, Q, fx_shift=S)
        d = oracle.derive(c)
        r = c["a"] + d["dr"] * np.arange(nr + 1)
        k = E * n0 / (4 * EPS0)
        a, b = c["a"], c["b"]
        C1 = -k * (b * b - a * a) / math.log(b / a)
        C2 = -k * a * a - C1 * math.log(a)
        exact = k * r * r + C1 * np.log(r) + C2
        mid = phi[:, c["nz"] // 2]
        errs.append(np.max(np.abs(mid - exact)) / np.max(np.abs(exact)))
    assert errs[-1] < 1e-3
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) > 1.7, (errs, orders)


def test_poisson_green_reciprocity():
    c = pi.coax64(nr=12, nz=20)
    rng = np.random.default_rng(2)
    for _ in range(6):
        p = (int(rng.integers(1, 12)), int(rng.integers(1, 20)))
        q = (int(rng.integers(1, 12)), int(rng.integers(1, 20)))
        rp = np.zeros((13, 21)); rp[p] = 1.0
        rq = np.zeros((13, 21)); rq[q] = 1.0
        gp, gq = oracle.solve(c, rp), oracle.solve(c, rq)
        assert gp[q] == pytest.approx(gq[p], rel=1e-12)
        assert gp[p] > 0 and gq[q] > 0  # the operator is positive definite


def test_node_volume_uniform_density():
    """A quasi-uniform volume load (midpoint rule in r^2 and z) deposits
    n0 V_i at every node, so the sampled density equals n0."""
    c = pi.coax64(nr=16, nz=32, collisions=0)
    K, M = 400, 320
    a, b, L = c["a"], c["b"], c["L"]
    r = np.sqrt(a * a + (np.arange(K) + 0.5) / K * (b * b - a * a))
    z = (np.arange(M) + 0.5) / M * L
    R, Z = np.meshgrid(r, z, indexing="ij")
    n = R.size
    n0 = 1e15
    w = n0 * math.pi * (b * b - a * a) * L / n
    c["weight"] = w
    st = dict(r=R.ravel(), z=Z.ravel(), vr=np.zeros(n), vt=np.zeros(n), vz=np.zeros(n),
              w=np.full(n, w), key=np.arange(n, dtype=np.uint64))
    s = oracle.Sim(c)
    s.set_particles(st)
    V = oracle.node_volume(c)
    dens = s.charge() * 2.0**-s.S / V
    assert np.allclose(dens[1:-1, 1:-1], n0, rtol=2e-3)
    assert np.allclose(dens, n0, rtol=3e-2)  # boundary rows: midpoint-rule error only
    assert V.sum() == pytest.approx(math.pi * (b * b - a * a) * L, rel=1e-12)


# --------------------------------------------------------------------------
# Collision sampling
# --------------------------------------------------------------------------

@pytest.mark.parametrize("xi", [0.0, 0.5, 0.9, -0.3])
def test_okhrimovskyy_cdf(xi):
    u = (np.arange(4000) + 0.5) / 4000
    rng = np.random.default_rng(3)
    u = rng.uniform(size=20000)
    mu = np.array([oracle.okh_cos(xi, x) for x in u])
    assert mu.min() >= -1.0 and mu.max() <= 1.0
    if xi == 0.0:
        cdf = lambda m: (m + 1.0) / 2.0
    else:
        cdf = lambda m: (1 - xi * xi) / (2 * xi) * (1.0 / (1.0 - xi * m) - 1.0 / (1.0 + xi))
    assert stats.kstest(mu, cdf).pvalue > 1e-4


def test_opal_cdf():
    Ebar, E_av = 10.0, 200.0
    rng = np.random.default_rng(4)
    Es = np.array([oracle.opal_split(Ebar, E_av, x) for x in rng.uniform(size=20000)])
    assert Es.min() >= 0.0 and Es.max() <= E_av / 2.0 * (1 + 1e-15)
    cdf = lambda e: np.arctan(e / Ebar) / math.atan(E_av / (2 * Ebar))
    assert stats.kstest(Es, cdf).pvalue > 1e-4


def test_scatter_geometry():
    rng = np.random.default_rng(6)
    for _ in range(500):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        if rng.uniform() < 0.2:
            u = np.array([0.05, 0.02, math.copysign(1.0, rng.normal())])
            u /= np.linalg.norm(u)
        cx = rng.uniform(-1, 1)
        ph = rng.uniform(0, 2 * math.pi)
        o = oracle.scatter(u, cx, ph)
        assert np.linalg.norm(o) == pytest.approx(1.0, abs=1e-15)
        assert float(o @ u) == pytest.approx(cx, abs=1e-14)
    # azimuth uniform: the mean over phi is cos(chi) u
    u = np.array([0.6, 0.0, 0.8])
    outs = np.array([oracle.scatter(u, 0.3, ph) for ph in np.linspace(0, 2 * math.pi, 4000, endpoint=False)])
    np.testing.assert_allclose(outs.mean(axis=0), 0.3 * u, atol=1e-12)


def rate_cfg(p_mbar):
    return pi.coax64(p_mbar=p_mbar, lotz_a=0.0, M_gas_amu=1e12, E_cap_eV=10.0,
                     collisions=1, diag_interval=1)


def test_null_collision_rate_constant_sigma():
    """Monoenergetic particles, constant sigma, no fields: candidate and real
    event counts are binomial with p = P_null and p = P_null v0 / v_cap, and the
    real rate approaches n sigma v0 dt."""
    c = rate_cfg(10.0)
    d = oracle.derive(c)
    n, K = 20000, 100
    v0 = 1.0e6
    rng = np.random.default_rng(8)
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    st = dict(r=np.full(n, 5e-3), z=np.full(n, 30e-3), vr=v0 * u[0], vt=v0 * u[1], vz=v0 * u[2],
              w=np.full(n, c["weight"]), key=np.arange(n, dtype=np.uint64))
    s = frozen_sim(c, pi.uniform_fields(c), st)
    s.step(K)
    dg = s.diag()
    trials = n * K
    p_cand = d["P_null"]
    assert abs(dg["n_null_cand"] - trials * p_cand) < 5 * math.sqrt(trials * p_cand * (1 - p_cand))
    p_el = d["P_null"] * v0 / d["v_cap"]
    assert abs(dg["n_elastic"] - trials * p_el) < 5 * math.sqrt(trials * p_el * (1 - p_el))
    nu_dt = d["n_n"] * c["sigma_el"] * v0 * c["dt"]
    assert dg["n_elastic"] / trials == pytest.approx(nu_dt, rel=d["nu_prime"] * c["dt"] + 5 / math.sqrt(trials * p_el))
    assert dg["n_ioniz"] == 0


def test_lotz_cross_section_hand_values():
    """The Lotz single-shell ionisation cross section a q ln(E/I)/(E I) at a few
    energies, each value worked out by hand for the workloads' parameters
    (a = 4.5e-18 m^2 eV^2, q = 2, I = 15.4 eV, so a q = 9e-18):
      E = 20 eV:    9e-18 * ln(1.298701)  / 308   = 9e-18 * 0.2613648 / 308
      E = 100 eV:   9e-18 * ln(6.493506)  / 1540  = 9e-18 * 1.8708025 / 1540
      E = 1000 eV:  9e-18 * ln(64.93506)  / 15400 = 9e-18 * 4.1733877 / 15400
    zero at and below the threshold, largest at E = e I = 41.8615 eV where it
    equals a q / (e I^2) = 9e-18 / 644.6677 = 1.396068e-20 m^2."""
    c = pi.coax64()
    for E0, sig in ((20.0, 7.637282e-21), (100.0, 1.093326e-20), (1000.0, 2.438993e-21),
                    (41.86154, 1.396068e-20)):
        assert oracle.sigma_iz(c, E0) == pytest.approx(sig, rel=2e-6)
    assert oracle.sigma_iz(c, 15.4) == 0.0 and oracle.sigma_iz(c, 10.0) == 0.0
    top = oracle.sigma_iz(c, 41.86154)
    assert all(oracle.sigma_iz(c, E0) < top for E0 in (38.0, 41.0, 42.7, 46.0))


def test_null_collision_decision_both_processes():
    """Elastic and ionising collisions both switched on (Sec. II.A, null-collision
    MCC): a mono-energetic isotropic 100 eV beam, no fields, one step at
    nu' dt ~ 0.02.  Each electron is a candidate with probability P_null and then
    undergoes an elastic event with probability nu_el / nu' and an ionisation with
    probability nu_iz / nu', nu = n_n sigma(E0) v0, sigma_iz(100 eV) the hand value
    of the Lotz formula.  The three counts must each lie within 5 sigma of their
    binomial means; swapping or truncating either branch of the decision (e.g.
    ionising for R < nu_iz instead of nu_el <= R < nu_el + nu_iz) fails."""
    E0 = 100.0
    c = pi.coax64(p_mbar=1.2, E_cap_eV=100.5, M_gas_amu=1e12, diag_interval=1)
    d = oracle.derive(c)
    v0 = math.sqrt(2.0 * E0 * E / ME)
    n = 400000
    rng = np.random.default_rng(21)
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    st = dict(r=np.full(n, 5e-3), z=np.full(n, 30e-3), vr=v0 * u[0], vt=v0 * u[1], vz=v0 * u[2],
              w=np.full(n, c["weight"]), key=np.arange(n, dtype=np.uint64))
    s = frozen_sim(c, pi.uniform_fields(c), st)
    s.step(1)
    dg = s.diag()
    sig_iz = 1.093326e-20                       # hand value at 100 eV (test above)
    nu_el = d["n_n"] * c["sigma_el"] * v0
    nu_iz = d["n_n"] * sig_iz * v0
    assert 0.01 < d["nu_prime"] * c["dt"] < 0.03 and nu_iz < nu_el < d["nu_prime"]

    def within(count, p):
        return abs(count - n * p) < 5.0 * math.sqrt(n * p * (1.0 - p))

    assert within(dg["n_null_cand"], d["P_null"])
    assert within(dg["n_elastic"], d["P_null"] * nu_el / d["nu_prime"])
    assert within(dg["n_ioniz"], d["P_null"] * nu_iz / d["nu_prime"])
    assert dg["n_ioniz"] > 500 and dg["n_elastic"] > 5000
    assert dg["n_live"] == n + dg["n_ioniz"]


def _step_pair(c, st):
    """Same particles stepped with and without collisions."""
    f = pi.uniform_fields(c)
    a = frozen_sim(dict(c, collisions=0), f, st)
    b = frozen_sim(c, f, st)
    a.step(1)
    b.step(1)
    return a.get_particles(), b.get_particles(), b.diag()


def test_null_candidate_mask_counts_the_candidates_of_a_step():
    """The candidate mask used to pick test samples marks exactly the electrons
    whose null-collision test succeeds in a step."""
    c = pi.coax64(p_mbar=30.0, E_cap_eV=3000.0)
    st = pi.cloud_state(c, 20000, seed=16)
    s = frozen_sim(c, pi.uniform_fields(c), st)
    s.set_step(11)
    s.step(1)
    m = oracle.null_candidates(c, 11, st["key"])
    assert s.diag()["n_null_cand"] == m.sum() > 100


def test_elastic_energy_loss_matches_angle():
    c = pi.coax64(p_mbar=300.0, lotz_a=0.0, M_gas_amu=4.0, E_cap_eV=2000.0)
    d = oracle.derive(c)
    st = pi.cloud_state(c, 4000, seed=9)
    pre, post, dg = _step_pair(c, st)
    assert dg["n_elastic"] > 50
    i0 = np.argsort(pre["key"]); i1 = np.argsort(post["key"])
    v0 = np.stack([pre[k][i0] for k in ("vr", "vt", "vz")])
    v1 = np.stack([post[k][i1] for k in ("vr", "vt", "vz")])
    s0, s1 = np.linalg.norm(v0, axis=0), np.linalg.norm(v1, axis=0)
    hit = np.abs(s1 / s0 - 1.0) > 1e-13
    assert hit.sum() == dg["n_elastic"]
    cosx = (v0 * v1).sum(axis=0)[hit] / (s0[hit] * s1[hit])
    np.testing.assert_allclose((s1[hit] / s0[hit]) ** 2, 1.0 - d["mass_ratio2"] * (1.0 - cosx), rtol=1e-12)


def test_ionisation_energy_balance_and_child():
    c = pi.coax64(p_mbar=300.0, sigma_el=0.0, lotz_a=4.5e-16, E_cap_eV=2000.0)
    st = pi.cloud_state(c, 4000, seed=10)
    pre, post, dg = _step_pair(c, st)
    assert dg["n_ioniz"] > 50 and dg["n_elastic"] == 0
    kids = post["key"] >= np.uint64(1 << 63)
    assert kids.sum() == dg["n_ioniz"]
    assert len(post["key"]) == len(pre["key"]) + dg["n_ioniz"]
    pre_by_pos = {(r, z): i for i, (r, z) in enumerate(zip(pre["r"], pre["z"]))}
    post_by_key = {int(k): i for i, k in enumerate(post["key"])}
    half_m_e = 0.5 * ME / E
    for j in np.nonzero(kids)[0]:
        i = pre_by_pos[(post["r"][j], post["z"][j])]
        par = post_by_key[int(pre["key"][i])]
        E0 = half_m_e * (pre["vr"][i] ** 2 + pre["vt"][i] ** 2 + pre["vz"][i] ** 2)
        Ep = half_m_e * (post["vr"][par] ** 2 + post["vt"][par] ** 2 + post["vz"][par] ** 2)
        Es = half_m_e * (post["vr"][j] ** 2 + post["vt"][j] ** 2 + post["vz"][j] ** 2)
        assert E0 > c["iz_I_eV"]
        assert Ep + Es == pytest.approx(E0 - c["iz_I_eV"], rel=1e-12, abs=1e-12)
        assert Es <= 0.5 * (E0 - c["iz_I_eV"]) * (1 + 1e-12)
        assert post["w"][j] == pre["w"][i]


# --------------------------------------------------------------------------
# Load and whole-run invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [0, 1])
def test_initial_load_distribution(mode):
    c = pi.coax64(n_init=40000, load_mode=mode, T_init_eV=2.0)
    s = oracle.Sim(c)
    s.load()
    p = s.get_particles()
    assert np.array_equal(np.sort(p["key"]), np.arange(40000, dtype=np.uint64))
    u = (p["z"] - c["z_lo"]) / (c["z_hi"] - c["z_lo"])
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    if mode == 1:
        ur = (p["r"] - c["r_lo"]) / (c["r_hi"] - c["r_lo"])
    else:
        ur = (p["r"] ** 2 - c["r_lo"] ** 2) / (c["r_hi"] ** 2 - c["r_lo"] ** 2)
    assert stats.kstest(ur, "uniform").pvalue > 1e-4
    sv = math.sqrt(c["T_init_eV"] * E / ME)
    for k in ("vr", "vt", "vz"):
        assert stats.kstest(p[k] / sv, "norm").pvalue > 1e-4


def test_charge_bookkeeping_with_collisions():
    c = pi.coax64hot(n_init=20000)
    s = oracle.Sim(c)
    s.load()
    W = round(c["weight"] * 2.0**s.S)
    q0 = s.diag()["total_Q"]
    assert q0 == 20000 * W
    s.step(200)
    dg = s.diag()
    p = s.get_particles()
    assert dg["n_ioniz"] > 0 and dg["n_elastic"] > 0
    assert dg["total_Q"] == len(p["r"]) * W == s.charge().sum()
    assert dg["n_live"] + sum(dg["n_absorbed"]) == 20000 + dg["n_ioniz"]
    assert dg["total_Q"] + sum(dg["absorbed_W"]) == q0 + dg["n_ioniz"] * W
    assert np.all((p["r"] > c["a"]) & (p["r"] < c["b"]) & (p["z"] > 0) & (p["z"] < c["L"]))


def _dyadic_cfg():
    """A trap whose a, dr, dz are powers of two, so that on positions of a
    2^-20 m grid every FP32 operation of the deposit is exact."""
    return pi.coax64(a=2.0**-10, b=2.0**-10 + 64 * 2.0**-12, L=128 * 2.0**-12, nr=64, nz=128,
                     r_lo=2.0**-9, r_hi=2.0**-8, z_lo=2.0**-6, z_hi=2.0**-5, weight=2.0**17)


def test_fp32_deposit_exact_where_single_precision_is_exact():
    """Dyadic mesh, positions on a 2^-20 grid (cell offsets multiples of 2^-8)
    and a power-of-two weight: the single-precision deposit rounds nothing, so
    it must equal the FP64 deposit (itself pinned by brute force) node by node.
    A swapped offset or a dropped node fails here."""
    c = _dyadic_cfg()
    S = oracle.auto_shift(c["weight"])
    assert c["weight"] * 2.0**S == 2.0**31
    rng = np.random.default_rng(14)
    n = 3000
    r = c["a"] + rng.integers(1, 64 * 256, n) * 2.0**-20
    z = rng.integers(1, 128 * 256, n) * 2.0**-20
    w = np.full(n, c["weight"])
    q32 = oracle.deposit_f32(c, r, z, w, fx_shift=S)
    q64 = np.zeros_like(q32)
    for x, y in zip(r, z):
        q64 += oracle.deposit_one(c, x, y, c["weight"], fx_shift=S)
    assert np.array_equal(q32, q64)
    assert q32.sum() == n * 2**31


def test_fp32_deposit_within_single_precision_rounding():
    """Arbitrary FP32 positions: every particle adds exactly W = rint(w 2^S) of
    its FP32 weight, and each node differs from the FP64 deposit by no more
    than the particles' single-precision rounding allows.  With s = (r - a)/dr
    the FP32 cell offset is off by at most (3 s + a/dr + 1) 2^-24 (a, 1/dr
    rounded, a difference and a product), the z offset by (2 t + 1) 2^-24; a
    node weight then by their sum plus two product roundings, the node charge
    by W times that plus 1/2 for each of the two rint; the remainder node takes
    the other three's errors as well."""
    c = pi.coax64()
    S = oracle.auto_shift(c["weight"])
    st = pi.particle_state(c, 4000, seed=15, margin_cells=0.01)
    r, z = (st[k].astype(np.float32).astype(np.float64) for k in ("r", "z"))
    w = np.full(len(r), float(np.float32(c["weight"])))
    q32 = oracle.deposit_f32(c, r, z, w, fx_shift=S)
    W = round(w[0] * 2.0**S)
    assert q32.sum() == len(r) * W
    d = oracle.derive(c, fx_shift=S)
    nodes = q32.shape
    bound = np.zeros(nodes)
    q64 = np.zeros(nodes, dtype=np.int64)
    eps = 2.0**-24
    for x, y in zip(r, z):
        qi = oracle.deposit_one(c, x, y, w[0], fx_shift=S)
        q64 += qi
        s, t = (x - c["a"]) * d["inv_dr"], y * d["inv_dz"]
        e_w = ((3 * s + c["a"] * d["inv_dr"] + 1) + (2 * t + 1) + 2) * eps
        e_q = W * e_w + 1.0
        i = min(int(s), c["nr"] - 1)
        j = min(int(t), c["nz"] - 1)
        # the cell may differ by one on either side: bound the 4x4 block around it
        blk = np.full((4, 4), 4 * e_q)
        i0, j0 = max(i - 1, 0), max(j - 1, 0)
        bound[i0:i0 + 4, j0:j0 + 4] += blk[:min(4, nodes[0] - i0), :min(4, nodes[1] - j0)]
    diff = np.abs(q32 - q64)
    assert np.all(diff <= bound)
    assert diff.max() > 0                  # the single-precision path really differs


def test_non_finite_particles_are_removed_and_counted():
    """A particle whose new position is not finite (here a NaN or infinite
    velocity component) is removed and counted apart: it is not absorbed
    charge, deposits nothing, and the other particles step exactly as in a run
    without it."""
    c = pi.coax64(collisions=0)
    st = pi.cloud_state(c, 2000, seed=12)
    bad = {k: v.copy() for k, v in st.items()}
    bad["vr"][5] = np.nan
    bad["vz"][17] = np.inf
    bad["vt"][40] = -np.inf
    f = pi.random_fields(c, 13)
    a, b = frozen_sim(c, f, st), frozen_sim(c, f, bad)
    a.step(3)
    b.step(3)
    da, db = a.diag(), b.diag()
    assert db["n_nonfinite"] == 3 and da["n_nonfinite"] == 0
    assert db["n_absorbed"] == da["n_absorbed"] and db["absorbed_W"] == da["absorbed_W"]
    W = round(c["weight"] * 2.0**a.S)
    assert db["n_live"] == da["n_live"] - 3 and db["total_Q"] == db["n_live"] * W
    pa, pb = a.get_particles(), b.get_particles()
    keep = ~np.isin(pa["key"], st["key"][[5, 17, 40]])
    for k in ("key", "r", "z", "vr", "vt", "vz"):
        assert np.array_equal(pa[k][keep], pb[k]), k


def test_absorbing_walls_and_current():
    """Particles launched straight at the outer electrode are all absorbed
    there and the windowed current equals their charge over the window."""
    c = pi.coax64(collisions=0, diag_interval=50)
    n = 500
    st = dict(r=np.full(n, 9.9e-3), z=np.linspace(10e-3, 50e-3, n), vr=np.full(n, 2e6),
              vt=np.zeros(n), vz=np.zeros(n), w=np.full(n, c["weight"]), key=np.arange(n, dtype=np.uint64))
    s = frozen_sim(c, pi.uniform_fields(c), st)
    s.step(50)
    dg = s.diag()
    assert dg["n_absorbed"] == [0, n, 0, 0] and dg["n_live"] == 0
    assert dg["I_wall"][1] == pytest.approx(n * c["weight"] * E / (50 * c["dt"]), rel=1e-12)
    assert dg["peak_I_outer"] == dg["I_wall"][1]


def test_windowed_wall_currents_and_their_peaks():
    """The sampled current of a wall is the charge it absorbed over the last
    window of D steps divided by D dt, and the peaks are the largest such
    window values so far (Sec. III.A's time traces).  Ballistic electrons
    cross the outer wall 5 in window 1, 20 in window 3 and 8 in window 4, the
    inner one 12 in window 2 and 3 in window 4."""
    D = 10
    c = pi.coax64(nr=16, nz=32, collisions=0, diag_interval=D)
    groups = [(1, 3, 5), (0, 12, 4), (0, 17, 8)] + [(1, s, 2) for s in range(21, 31)] + [(1, 35, 8), (0, 38, 3)]
    s = frozen_sim(c, pi.uniform_fields(c), pi.ballistic_state(c, groups, 1.0e7))
    unit = c["weight"] * E / (D * c["dt"])  # one electron per window, in A
    # (inner, outer) of the window just sampled, and the peaks so far
    want = [((0, 5), (0, 5)), ((12, 0), (12, 5)), ((0, 20), (12, 20)), ((3, 8), (12, 20))]
    for (cur_in, cur_out), (pk_in, pk_out) in want:
        s.step(D)
        dg = s.diag()
        assert dg["I_wall"][0] == pytest.approx(cur_in * unit, rel=1e-12, abs=0.0)
        assert dg["I_wall"][1] == pytest.approx(cur_out * unit, rel=1e-12, abs=0.0)
        assert dg["I_wall"][2] == 0.0 and dg["I_wall"][3] == 0.0
        assert dg["peak_I_inner"] == pytest.approx(pk_in * unit, rel=1e-12)
        assert dg["peak_I_outer"] == pytest.approx(pk_out * unit, rel=1e-12)
    assert dg["n_absorbed"] == [15, 33, 0, 0] and dg["n_live"] == 0


def test_sampled_density_time_average_and_peak():
    """Density samples every D steps: charge over the node's volume.  A cloud
    of n electrons at one point, drifting along z by one cell per window, sits
    at a cell centre at every sample, so each sample puts n w / 4 on the
    cell's four nodes; an interior node's volume is 2 pi r_i dr dz (the hat
    function's r-weighted integral).  The time average over four samples and
    the peak follow in closed form."""
    D = 10
    c = pi.coax64(nr=16, nz=32, collisions=0, diag_interval=D)
    a, b, L, nr, nz = c["a"], c["b"], c["L"], c["nr"], c["nz"]
    dr, dz = (b - a) / nr, L / nz
    n, i, j0 = 1000, 5, 9
    st = dict(r=np.full(n, a + (i + 0.5) * dr), z=np.full(n, (j0 + 0.5) * dz), vr=np.zeros(n), vt=np.zeros(n),
              vz=np.full(n, dz / (D * c["dt"])), w=np.full(n, c["weight"]), key=np.arange(n, dtype=np.uint64))
    s = frozen_sim(c, pi.uniform_fields(c), st)
    s.step(4 * D)
    dg = s.diag()
    assert dg["n_samples"] == 4 and dg["n_live"] == n
    vol = lambda ii: 2.0 * math.pi * (a + ii * dr) * dr * dz
    q = n * c["weight"] / 4.0  # electrons per node and sample
    want = np.zeros((nr + 1, nz + 1))
    for k in range(1, 5):  # the cloud sits in cell (i, j0 + k) at sample k
        for ii in (i, i + 1):
            for jj in (j0 + k, j0 + k + 1):
                want[ii, jj] += q / vol(ii) / 4.0
    got = s.time_avg_density()
    assert np.allclose(got, want, rtol=1e-12, atol=0.0)
    assert np.count_nonzero(got) == 10
    assert dg["peak_density"] == pytest.approx(q / vol(i), rel=1e-12)


# --------------------------------------------------------------------------
# Volumetric seed source (Sec. II.A): uniform in space, Maxwellian in velocity
# --------------------------------------------------------------------------

@pytest.mark.parametrize("rate", [0.3, 37.5, 1000.0])
def test_seed_source_count_and_keys(rate):
    c = pi.coax64(n_init=0, src_rate=rate, collisions=0, p_mbar=1e-12)
    s = oracle.Sim(c, capacity=4096)
    s.load()
    for n in (1, 7, 20):
        s.step(n - s.diag()["step"])
        d = s.diag()
        assert d["n_source"] == math.floor(n * rate)
    st = s.get_particles()
    d = s.diag()
    # survivors carry distinct keys 2^62 + i, i < floor(20 R); the rest reached a wall
    keys = np.sort(st["key"])
    want = np.uint64(1 << 62) + np.arange(math.floor(20 * rate), dtype=np.uint64)
    assert len(np.unique(keys)) == len(keys) and np.all(np.isin(keys, want))
    assert len(keys) + sum(d["n_absorbed"]) == len(want)
    W = round(c["weight"] * 2.0 ** s.S)
    assert d["total_Q"] == len(keys) * W


def test_seed_source_uniform_in_volume_and_maxwellian():
    T = 3.0
    c = pi.coax64(n_init=0, src_rate=40000.0, src_T_eV=T, collisions=0, p_mbar=1e-12)
    s = oracle.Sim(c, capacity=65536)
    s.load()
    s.step(1)  # created after the push of step 0: still at their drawn state
    st = s.get_particles()
    a, b, L = c["a"], c["b"], c["L"]
    assert len(st["r"]) == 40000
    assert np.all((st["r"] > a) & (st["r"] <= b) & (st["z"] > 0) & (st["z"] < L))
    u = (st["r"] ** 2 - a * a) / (b * b - a * a)
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    assert stats.kstest(st["z"] / L, "uniform").pvalue > 1e-4
    sv = math.sqrt(T * E / ME)
    for k in ("vr", "vt", "vz"):
        assert stats.kstest(st[k] / sv, "norm").pvalue > 1e-4, k
    # src_T_eV = 0 takes the load temperature
    c0 = dict(c, src_T_eV=0.0, T_init_eV=0.5)
    s0 = oracle.Sim(c0, capacity=65536)
    s0.load()
    s0.step(1)
    v = s0.get_particles()["vz"]
    assert np.std(v) == pytest.approx(math.sqrt(0.5 * E / ME), rel=0.02)


# --------------------------------------------------------------------------
# Open (Neumann) ends, end_mode 2 (Sec. II.A: d(phi)/dz = 0 on the open
# boundaries)
# --------------------------------------------------------------------------

def test_neumann_vacuum_is_the_coaxial_log_at_second_order():
    errs = []
    for nr in (16, 32, 64):
        c = pi.coax64(nr=nr, nz=32, end_mode=2)
        v = oracle.vacuum(c)
        # no axial structure at all with open ends
        assert np.max(np.abs(v - v[:, :1])) <= 1e-12 * abs(c["V_inner"])
        a, b = c["a"], c["b"]
        r = a + (b - a) / nr * np.arange(nr + 1)
        exact = c["V_inner"] + (c["V_outer"] - c["V_inner"]) * np.log(r / a) / math.log(b / a)
        errs.append(np.max(np.abs(v[:, 7] - exact)) / abs(c["V_inner"]))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 1.8, (errs, orders)


def test_neumann_uniform_column_is_z_independent_closed_form():
    """A uniform density filling a < r < b, 0 <= z <= L with phi = 0 on the
    electrodes and open ends: phi depends on r only and follows
    (e n0 / 4 eps0) r^2 + C1 ln r + C2 at second order, at every z."""
    n0 = 1e15
    errs = []
    for nr in (16, 32, 64):
        c = pi.coax64(nr=nr, nz=64, end_mode=2)
        S = 10
        V = oracle.node_volume(c)
        Q = np.rint(n0 * V * 2.0**S).astype(np.int64)
        phi = oracle.poisson_charge(c, Q, fx_shift=S)
        d = oracle.derive(c)
        r = c["a"] + d["dr"] * np.arange(nr + 1)
        k = E * n0 / (4 * EPS0)
        a, b = c["a"], c["b"]
        C1 = -k * (b * b - a * a) / math.log(b / a)
        C2 = -k * a * a - C1 * math.log(a)
        exact = (k * r * r + C1 * np.log(r) + C2)[:, None]
        # z independence up to the rounding of the fixed-point charges
        assert np.max(np.abs(phi - phi[:, 32:33])) <= 1e-6 * np.max(np.abs(exact))
        errs.append(np.max(np.abs(phi - exact)) / np.max(np.abs(exact)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-3 and min(orders) > 1.7, (errs, orders)


def test_neumann_green_reciprocity_and_end_nodes():
    c = pi.coax64(nr=12, nz=20, end_mode=2)
    rng = np.random.default_rng(3)
    for _ in range(6):
        # sources anywhere in z, the end columns included
        p = (int(rng.integers(1, 12)), int(rng.integers(0, 21)))
        q = (int(rng.integers(1, 12)), int(rng.integers(0, 21)))
        rp = np.zeros((13, 21)); rp[p] = 1.0
        rq = np.zeros((13, 21)); rq[q] = 1.0
        gp, gq = oracle.solve(c, rp), oracle.solve(c, rq)
        assert gp[q] == pytest.approx(gq[p], rel=1e-12)
        assert gp[p] > 0 and gq[q] > 0
        assert np.all(gp[0] == 0) and np.all(gp[-1] == 0)  # electrodes stay at 0
    # a cosine profile in z is an eigenvector of the open-ended z operators:
    # the response keeps exactly that profile
    jz = np.arange(21)
    rhs = np.zeros((13, 21))
    rhs[5] = np.cos(np.pi * 3 * jz / 20)
    rhs[5, 0] *= 0.5  # the natural boundary halves the end rows (load of a half element)
    rhs[5, -1] *= 0.5
    g = oracle.solve(c, rhs)
    prof = np.cos(np.pi * 3 * jz / 20)
    for i in (3, 5, 9):
        coef = g[i, 1] / prof[1]
        assert np.allclose(g[i], coef * prof, rtol=0, atol=1e-12 * abs(coef))


# --------------------------------------------------------------------------
# Fluid moments (Sec. IV: force terms from moments of the distribution)
# --------------------------------------------------------------------------

def test_moments_conserve_the_particle_sums():
    c = pi.coax64()
    st = pi.cloud_state(c, 3000, seed=4)
    o = oracle.Sim(c, capacity=4096)
    o.set_particles(st)
    m = o.moments()
    V = oracle.node_volume(c).reshape(m.shape[1:])
    w, vr, vt, vz = st["w"], st["vr"], st["vt"], st["vz"]
    want = [w.sum(), (w * vr).sum(), (w * vt).sum(), (w * vz).sum(), (w * vr * vr).sum(), (w * vr * vt).sum(),
            (w * vr * vz).sum(), (w * vt * vt).sum(), (w * vt * vz).sum(), (w * vz * vz).sum()]
    for ch, x in enumerate(want):
        assert (m[ch] * V).sum() == pytest.approx(x, rel=1e-12, abs=1e-9 * abs(want[ch] if ch else 1.0)), ch


def test_moments_single_particle_brute_force():
    c = pi.coax64(nr=8, nz=8, lotz_a=0.0)
    d = oracle.derive(c)
    r, z = c["a"] + 2.3 * d["dr"], 5.6 * d["dz"]
    st = dict(r=np.array([r]), z=np.array([z]), vr=np.array([3e5]), vt=np.array([-1e6]), vz=np.array([2e5]),
              w=np.array([7.0]), key=np.array([1], dtype=np.uint64))
    o = oracle.Sim(c, capacity=16)
    o.set_particles(st)
    m = o.moments()
    V = oracle.node_volume(c).reshape(m.shape[1:])
    fr, fz = 0.3, 0.6
    weights = {(2, 5): (1 - fr) * (1 - fz), (3, 5): fr * (1 - fz), (2, 6): (1 - fr) * fz, (3, 6): fr * fz}
    vr, vt, vz = 3e5, -1e6, 2e5
    v = math.sqrt(vr * vr + vt * vt + vz * vz)
    q = [1, vr, vt, vz, vr * vr, vr * vt, vr * vz, vt * vt, vt * vz, vz * vz, d["nsig_el"] * v]
    for ch in range(11):
        got = m[ch] * V
        for (i, j), wk in weights.items():
            assert got[i, j] == pytest.approx(7.0 * wk * q[ch], rel=1e-9), (ch, i, j)
        assert np.count_nonzero(got) <= 4


def test_moments_drifting_maxwellian_pressure_and_drag():
    """Particles with a drift u and temperature T in a box: n u / n = u and the
    pressure tensor m (M2 - n u u) = n k T (isotropic); monoenergetic
    particles with a constant sigma give nu_m = n_n sigma v0 times n."""
    rng = np.random.default_rng(9)
    c = pi.coax64(nr=4, nz=4, lotz_a=0.0)
    N = 200000
    u = np.array([2e5, -5e5, 1e5])
    T = 5.0
    sv = math.sqrt(T * E / ME)
    st = dict(r=rng.uniform(c["a"], c["b"], N), z=rng.uniform(0, c["L"], N),
              vr=u[0] + sv * rng.normal(size=N), vt=u[1] + sv * rng.normal(size=N), vz=u[2] + sv * rng.normal(size=N),
              w=np.full(N, 1.0), key=np.arange(N, dtype=np.uint64))
    o = oracle.Sim(c, capacity=N)
    o.set_particles(st)
    m = o.moments()
    n = m[0][2, 2]
    flux = m[1:4, 2, 2]
    np.testing.assert_allclose(flux / n, u, atol=0.02 * sv)
    M2 = np.array([[m[4], m[5], m[6]], [m[5], m[7], m[8]], [m[6], m[8], m[9]]])[:, :, 2, 2]
    P = ME * (M2 - np.outer(flux, flux) / n)
    np.testing.assert_allclose(np.diag(P) / (n * T * E), 1.0, atol=0.03)
    assert abs(P[0, 1]) < 0.03 * n * T * E
    # monoenergetic
    v0 = 3e6
    dirs = rng.normal(size=(N, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    st2 = dict(st, vr=v0 * dirs[:, 0], vt=v0 * dirs[:, 1], vz=v0 * dirs[:, 2])
    o2 = oracle.Sim(c, capacity=N)
    o2.set_particles(st2)
    m2 = o2.moments()
    d = oracle.derive(c)
    np.testing.assert_allclose(m2[10], d["nsig_el"] * v0 * m2[0], rtol=1e-12, atol=0)


# --------------------------------------------------------------------------
# Potential-well depth along field lines (Sec. II.B)
# --------------------------------------------------------------------------

def test_well_depth_of_the_relative_end_plates_is_the_end_bias():
    """Uniform B: field lines are r = const.  With end plates at the coaxial
    profile + V_end the vacuum well on every line is |V_end| deep (the trap is
    long compared with b - a, so the middle sits at the coaxial profile), its
    maximum at mid-length; open ends give no well."""
    c = pi.coax64(nr=64, nz=128, mirror_k=0.0)
    r = np.array([2e-3, 4e-3, 6e-3, 8e-3])
    dep, zm = oracle.well_depth(c, oracle.vacuum(c), r)
    np.testing.assert_allclose(dep, abs(c["V_end"]), rtol=5e-3)
    np.testing.assert_allclose(zm, c["L"] / 2)
    c2 = dict(c, end_mode=2)
    dep2, _ = oracle.well_depth(c2, oracle.vacuum(c2), r)
    assert np.max(np.abs(dep2)) <= 1e-9 * abs(c["V_inner"])


def test_well_depth_brute_force_on_a_given_profile():
    """On lines through node radii (uniform B) phi is sampled at the nodes
    exactly: the depth is the brute-force max minus the higher side minimum;
    lines leaving the domain at the midplane report none."""
    c = pi.coax64(nr=8, nz=16, mirror_k=0.0)
    d = oracle.derive(c)
    z = np.arange(17) * d["dz"]
    rng = np.random.default_rng(5)
    prof = rng.normal(size=17) * 100.0
    phi = np.tile(prof, (9, 1))
    r_nodes = c["a"] + d["dr"] * np.array([1.0, 3.0, 6.0])
    dep, zm = oracle.well_depth(c, phi, np.append(r_nodes, c["b"] + 1e-3))
    jx = int(np.argmax(prof))
    want = prof[jx] - max(prof[:jx + 1].min(), prof[jx:].min())
    np.testing.assert_allclose(dep[:3], want, rtol=1e-12)
    np.testing.assert_allclose(zm[:3], z[jx])
    assert dep[3] == 0.0 and zm[3] == -1.0
