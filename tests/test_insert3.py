"""Cubic web-splines with the elliptic insert (weighted extended B-splines of
degree 3, Sec. II.A, on the gun geometry of Sec. III).

CPU: the oracle's cubic web-spline solver pinned by the plain cubic solver
(an insert outside the domain), by a manufactured solution on a true ellipse
(error falling by more than 5x per halving of the mesh in the mean, more
than the bilinear web-splines' 2.8x), by the coaxial profile under a flat
insert whose wall lies off the mesh lines, by Green reciprocity of the
weighted deposit and the weighted read, and by the exact bookkeeping of the
band charge; the library's host set-up against the oracle's unknown classes.
GPU: the corrected cubic solve against the oracle's banded factorisation
(deposits bit for bit), FP64 steps, and the batched FP32 form at FP32
accuracy."""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import by_key, gpu_and_oracle, rel_vec_err
from paper_2206_14662_amd import binding as B
from test_insert import _manufactured, ellipse


def ellipse3(nr=32, nz=64, **over):
    return ellipse(nr, nz, spline_order=3, **over)


def _one(c, r, z, w=None):
    return dict(r=np.array([r]), z=np.array([z]), vr=np.zeros(1), vt=np.zeros(1), vz=np.zeros(1),
                w=np.array([c["weight"] if w is None else w]), key=np.zeros(1, dtype=np.uint64))


# ---------------------------------------------------------------------------
# oracle pins (CPU)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("end_mode", [0, 2])
def test_insert_outside_the_domain_is_the_plain_cubic_solver(end_mode):
    """No support cell meets the band: every basis function is an inner one
    with weight 1, so the web-spline system is the plain cubic Galerkin
    system and both give the same coefficients (manufactured source and a
    particle cloud)."""
    c = pi.coax64(nr=32, nz=64, end_mode=end_mode, n_init=0, spline_order=3, ins_r0=0.05, ins_z0=0.03,
                  ins_er=1e-3, ins_ez=5e-3)
    info = oracle.is3_info(c)
    assert info["counts"][2] == info["counts"][3] == 0
    plain = dict(c, ins_er=0.0, ins_ez=0.0)
    f = lambda r, z: math.sin(700.0 * r) * math.cos(90.0 * z) + 1.0
    a, b = oracle.s3_poisson_fn(plain, f), oracle.is3_poisson_fn(c, f)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    st = pi.particle_state(c, 3000, seed=4)
    oa, ob = oracle.Sim(plain), oracle.Sim(c)
    oa.set_particles(st)
    ob.set_particles(st)
    assert np.array_equal(oa.charge3(), ob.charge3())
    assert not ob.charge3w().any()
    ca, cb = oa.coef3(), ob.coef3()
    assert np.abs(ca - cb).max() <= 1e-11 * np.abs(ca).max()
    sa, sb = oa.phi() - oracle.vacuum(plain), ob.phi() - oracle.vacuum(c)
    assert np.abs(sa - sb).max() <= 1e-11 * np.abs(sa).max()


def _ellipse_errors(nr, nz, pts):
    c = ellipse3(nr, nz)
    phi, f = _manufactured(c)
    cx = oracle.is3_poisson_fn(c, f)
    got = np.array([oracle.is3_phi_at(c, cx, r, z) for r, z in pts])
    ex = phi(pts[:, 0], pts[:, 1])
    err = np.abs(got - ex) / np.abs(ex).max()
    return np.sqrt(np.mean(err ** 2)), err.max()


def test_manufactured_solution_on_the_ellipse_cubic():
    """phi* = g (r - a)(b - r) sin(pi z / L) vanishes on every wall and on the
    ellipse; read at 1500 random points of the vacuum region (the band
    included), the cubic web-spline solution's error falls by more than 5x
    per halving in the mean and by more than 3.5x at its worst (the
    electrode rows, where the odd reflection of the cubic basis also fixes
    the second radial derivative, limit the maximum to second order)."""
    c = ellipse3()
    rng = np.random.default_rng(5)
    pts = np.column_stack([rng.uniform(c["a"], c["b"], 4000), rng.uniform(0.0, c["L"], 4000)])
    g = ((pts[:, 0] - c["ins_r0"]) / c["ins_er"]) ** 2 + ((pts[:, 1] - c["ins_z0"]) / c["ins_ez"]) ** 2 - 1
    pts = pts[g > 0][:1500]
    # some of them inside the band of the finest mesh
    fine = ellipse3(64, 128)
    assert sum(oracle.ins_weight(fine, r, z)[0] < 1.0 for r, z in pts) >= 50
    res = [_ellipse_errors(nr, nz, pts) for nr, nz in ((16, 32), (32, 64), (64, 128))]
    rms, mx = [e[0] for e in res], [e[1] for e in res]
    assert rms[0] / rms[1] > 5.0 and rms[1] / rms[2] > 5.0, rms
    assert mx[0] / mx[1] > 3.5 and mx[1] / mx[2] > 3.5, mx
    assert mx[2] < 1e-3


def _flat3_error(nr, band):
    """Uniform source f under a flat insert (wall r_w = b - er, off the mesh
    lines), open ends: phi = -f r^2 / 4 + A ln r + B with phi(a) = phi(r_w) = 0."""
    a, b, L, er = 1e-3, 10e-3, 60e-3, 2.37e-3
    c = pi.coax64(nr=nr, nz=8, end_mode=2, V_end=0.0, n_init=0, spline_order=3, ins_r0=b, ins_z0=L / 2,
                  ins_er=er, ins_ez=200 * L, ins_band=band)
    cx = oracle.is3_poisson_fn(c, lambda r, z: 1.0)
    rw = b - er
    A = (rw ** 2 - a ** 2) / 4 / math.log(rw / a)
    B = a ** 2 / 4 - A * math.log(a)
    rs = np.linspace(a, rw, 201)[1:-1]
    ex = -rs * rs / 4 + A * np.log(rs) + B
    got = np.array([oracle.is3_phi_at(c, cx, r, L / 2 + 0.3e-3) for r in rs])
    return np.abs(got - ex).max() / np.abs(ex).max()


def test_flat_insert_space_charge_profile():
    for band in (lambda nr: 0.0, lambda nr: 3.0 * nr / 16):
        e = [_flat3_error(nr, band(nr)) for nr in (16, 32, 64)]
        assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, e
        assert e[2] < 2e-3


def test_green_reciprocity_with_the_weights():
    """A charge deposits W w(x) B_i(x) (the plain cubic deposit plus the band
    correction rint(W (w - 1)) B_i(x)) and the potential is read as
    w(x) sum c_i B_i(x): the pair is symmetric, so the potential of charge 1
    at x2 equals that of charge 2 at x1, both in the band, one in the band
    and one far from it.  The integer deposit rounds each node's share to
    1 / W of the charge, so the test charge is a million macro-weights:
    W ~ 2^50 and the pair agrees to 1e-12."""
    c = ellipse3(64, 128)
    gam = oracle.ins_gamma(c)
    r_band = lambda s: c["ins_r0"] - c["ins_er"] * math.sqrt(1 + s * gam)
    pairs = [((r_band(0.3), c["ins_z0"]), (r_band(0.6), c["ins_z0"] + 0.7e-3)),
             ((r_band(0.2), c["ins_z0"] - 0.4e-3), (3.3e-3, 9.1e-3))]
    for x1, x2 in pairs:
        vals = []
        for src, at in ((x1, x2), (x2, x1)):
            o = oracle.Sim(c, capacity=16)
            o.set_particles(_one(c, *src, w=1e6 * c["weight"]))
            vals.append(oracle.is3_phi_at(c, o.coef3(), *at))
            o.close()
        assert vals[0] == pytest.approx(vals[1], rel=1e-12) and vals[0] != 0.0


def test_band_charge_bookkeeping():
    """Every electron deposits W into the plain cubic grid (the weights sum
    to 1, the remainder rule makes it exact) and rint(W (w - 1)) into the
    band grid; electrons outside the band add nothing there."""
    c = ellipse3(64, 128)
    st = pi.particle_state(c, 20000, seed=9)
    g = ((st["r"] - c["ins_r0"]) / c["ins_er"]) ** 2 + ((st["z"] - c["ins_z0"]) / c["ins_ez"]) ** 2 - 1
    st = {k: v[g > 0] for k, v in st.items()}
    o = oracle.Sim(c, capacity=32768)
    o.set_particles(st)
    W = np.rint(st["w"] * o.derived()["two_S"]).astype(np.int64)
    assert o.charge3().sum() == W.sum()
    wx = np.array([oracle.ins_weight(c, r, z)[0] for r, z in zip(st["r"], st["z"])])
    inband = wx < 1.0
    assert inband.sum() > 100
    assert o.charge3w().sum() == np.sum(np.rint(W[inband] * (wx[inband] - 1.0)).astype(np.int64))
    o.close()


def test_library_setup_matches_the_oracle_classes():
    """The library's host set-up (written apart from the oracle) gives the
    same unknown classes (inner, outer, exterior) as the oracle's."""
    for c in (ellipse3(32, 64), ellipse3(64, 128), ellipse3(32, 64, end_mode=2), pi.gun(spline_order=3)):
        lib = B.pic_insert_layout(c)
        assert lib["counts"][1:] == oracle.is3_info(c)["counts"][1:], c["nr"]
        assert 0 < lib["m"] < 0.25 * (c["nr"] + 1) * (c["nz"] + 1)
        assert lib["entries"] > lib["m"]


# ---------------------------------------------------------------------------
# GPU parity
# ---------------------------------------------------------------------------

F32 = B.PIC_MODE_FP32_BATCHED
F64 = B.PIC_MODE_FP64_PLAIN


def _outside(c, st):
    g = ((st["r"] - c["ins_r0"]) / c["ins_er"]) ** 2 + ((st["z"] - c["ins_z0"]) / c["ins_ez"]) ** 2 - 1
    return {k: v[g > 0] for k, v in st.items()}


def _case(name, **over):
    if name == "gun":
        return pi.gun(spline_order=3, n_init=0, **over)
    return ellipse3(64, 128, end_mode={"ellipse0": 0, "ellipse2": 2}[name], **over)


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["ellipse0", "ellipse2", "gun"])
def test_gpu_cubic_insert_solve_matches_the_oracle(case):
    """The two fast cubic solves with the correction through H against the
    oracle's banded factorisation of the web-spline system: the cubic and
    band deposits bit for bit, the expanded coefficients and the potential
    to solver rounding."""
    c = _case(case)
    st = _outside(c, pi.particle_state(c, 40000, seed=12))
    g, o = gpu_and_oracle(c, st, frozen=0)
    Qx, cx = g.spline3()
    assert np.array_equal(Qx, o.charge3())
    assert np.array_equal(g.band_charge(), o.charge3w())
    assert (o.charge3w() != 0).sum() > 50
    ocx = o.coef3()
    vac = oracle.vacuum(c)
    sg, so = g.phi() - vac, o.phi() - vac
    # the field the particles see, read from both coefficient sets at points
    # over the domain and in the band
    rng = np.random.default_rng(3)
    pts = _outside(c, dict(r=rng.uniform(c["a"], c["b"], 3000), z=rng.uniform(0.0, c["L"], 3000)))
    Eg = np.array([oracle.is3_field(c, cx, r, z) for r, z in zip(pts["r"], pts["z"])])
    Eo = np.array([oracle.is3_field(c, ocx, r, z) for r, z in zip(pts["r"], pts["z"])])
    ecx = np.abs(cx - ocx).max() / np.abs(ocx).max()
    ephi = np.abs(sg - so).max() / np.abs(so).max()
    efld = np.abs(Eg - Eo).max() / np.abs(Eo).max()
    print(f"{case}: coefficients {ecx:.2e}, nodal potential {ephi:.2e}, field at particles {efld:.2e}", flush=True)
    # the outer B-splines' coefficients, rebuilt from their blocks, carry the
    # inner ones' rounding times the extension weights (sums up to ~10^3)
    assert ecx <= 1e-8 and ephi <= 1e-9 and efld <= 1e-10
    g.close()


@pytest.mark.gpu
@pytest.mark.parametrize("collisions,end_mode", [(0, 0), (1, 2)])
def test_gpu_cubic_insert_steps_match_the_oracle(collisions, end_mode):
    """Self-consistent steps with electrons crossing the band and absorbed on
    the insert: the same events and absorptions, states to FP64 rounding."""
    c = ellipse3(64, 128, end_mode=end_mode, p_mbar=30.0 if collisions else 1e-6, E_cap_eV=3000.0,
                 collisions=collisions)
    st = _outside(c, pi.particle_state(c, 30000, seed=13, v_scale=3e6))
    g, o = gpu_and_oracle(c, st, frozen=0)
    g.step(15)
    o.step(15)
    gd, od = g.diag(), o.diag()
    for k in ("n_live", "n_absorbed", "n_elastic", "n_ioniz"):
        assert gd[k] == od[k], k
    assert gd["n_absorbed"][1] > 0
    gp, op = by_key(g.get_particles()), by_key(o.get_particles())
    assert np.array_equal(gp["key"], op["key"])
    np.testing.assert_allclose(gp["r"], op["r"], rtol=1e-11)
    np.testing.assert_allclose(gp["z"], op["z"], rtol=1e-11)
    assert rel_vec_err(gp, op).max() <= 1e-9
    assert np.array_equal(g.band_charge(), o.charge3w())
    g.close()


def _fp32_exact(st):
    return {k: (v.astype(np.float32).astype(np.float64) if v.dtype == np.float64 else v) for k, v in st.items()}


@pytest.mark.gpu
@pytest.mark.parametrize("end_mode", [0, 2])
def test_fp32_cubic_insert_one_step_against_the_oracle(end_mode):
    """The batched FP32 form from an FP32-valued state over the whole domain
    (band included): deposits and coefficients at FP32 accuracy, one step
    element-wise against the oracle."""
    c = ellipse3(64, 128, end_mode=end_mode, p_mbar=30.0, E_cap_eV=3000.0)
    st = _fp32_exact(_outside(c, pi.particle_state(c, 20000, seed=41)))
    g, o = gpu_and_oracle(c, st, frozen=0, mode=F32)
    Qg, cg = g.spline3()
    Qo, co = o.charge3(), o.coef3()
    W = round(c["weight"] * 2.0 ** o.S)
    assert Qg.sum() == Qo.sum() == len(st["r"]) * W
    # single-precision node charges: W ~ 2^31 rounds at ~2^-24 per node
    assert np.linalg.norm(Qg - Qo) <= 3e-6 * np.linalg.norm(Qo)
    Bg, Bo = g.band_charge(), o.charge3w()
    assert abs(Bg.sum() - Bo.sum()) <= 1e-5 * abs(Bo.sum()) and Bo.sum() < 0
    # the solve itself is FP64: the field at points over the domain and in
    # the band carries the deposit's single-precision rounding
    rng = np.random.default_rng(4)
    pts = _outside(c, dict(r=rng.uniform(c["a"], c["b"], 3000), z=rng.uniform(0.0, c["L"], 3000)))
    Eg = np.array([oracle.is3_field(c, cg, r, z) for r, z in zip(pts["r"], pts["z"])])
    Eo = np.array([oracle.is3_field(c, co, r, z) for r, z in zip(pts["r"], pts["z"])])
    efld = np.abs(Eg - Eo).max() / np.abs(Eo).max()
    print(f"end_mode {end_mode}: field at particles {efld:.2e}", flush=True)
    assert efld <= 1e-5
    g.step(1)
    o.step(1)
    gd, od = g.diag(), o.diag()
    assert gd["n_null_cand"] == od["n_null_cand"]
    assert abs(gd["n_elastic"] - od["n_elastic"]) <= 2 and abs(gd["n_ioniz"] - od["n_ioniz"]) <= 2
    assert gd["n_absorbed"] == od["n_absorbed"]
    gp, op = by_key(g.get_particles()), by_key(o.get_particles())
    keep = np.intersect1d(gp["key"], op["key"])
    assert len(keep) >= len(op["key"]) - 4
    gq = {k: v[np.searchsorted(gp["key"], keep)] for k, v in gp.items()}
    oq = {k: v[np.searchsorted(op["key"], keep)] for k, v in op.items()}
    np.testing.assert_allclose(gq["r"], oq["r"], rtol=2e-6)
    np.testing.assert_allclose(gq["z"], oq["z"], rtol=2e-6)
    assert np.quantile(rel_vec_err(gq, oq), 0.999) < 1e-4
    g.close()


@pytest.mark.gpu
def test_fp32_cubic_gun_is_invariant_and_tracks_the_oracle():
    """The gun with cubic shapes in the batched FP32 form: bit-identical
    across tile shapes, sort intervals and graph or plain launches; live
    electrons and ionisations against the FP64 oracle within FP32 drift."""
    c = pi.gun(spline_order=3, E_cap_eV=33020.0)
    ref = None
    for kw in (dict(tile_r=8, tile_z=32, sort_interval=8, use_graph=1),
               dict(tile_r=4, tile_z=16, sort_interval=3, halo=1, use_graph=0)):
        g = B.Sim([c], mode=F32, **kw)
        g.step(40)
        out = (by_key(g.get_particles()), g.spline3()[0], g.band_charge(), g.diag())
        g.close()
        if ref is None:
            ref = out
            continue
        for k in ("key", "r", "z", "vr", "vt", "vz"):
            assert np.array_equal(ref[0][k], out[0][k]), k
        assert np.array_equal(ref[1], out[1]) and np.array_equal(ref[2], out[2])
    d = ref[3]
    assert d["n_ioniz"] > 0
    assert d["n_live"] + sum(d["n_absorbed"]) == c["n_init"] + d["n_ioniz"]
    o = oracle.Sim(c, fx_shift=d["S"])
    o.load()
    o.step(40)
    od = o.diag()
    assert abs(d["n_live"] - od["n_live"]) <= 0.01 * od["n_live"]
    assert abs(d["n_ioniz"] - od["n_ioniz"]) <= 0.1 * od["n_ioniz"] + 5
