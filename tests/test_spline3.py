"""Cubic B-spline particle shapes and space-charge FEM (the paper's spline FEM
of higher order, Sec. II.A).  CPU: the oracle's cubic weights, deposit and
Galerkin solve pinned by the B-spline identities, a manufactured solution at
fourth order (third for the field) and Green reciprocity of the deposit /
gather pair.  GPU: the FP64 form's transform-based cubic solve against the
oracle's assembled one, and steps against the oracle; the batched FP32 form
invariant to its tiles and launches, at FP32 accuracy against the oracle for
one step and within 2% of it over a run."""
import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import by_key, gpu_and_oracle, rel_vec_err
from paper_2206_14662_amd import binding as B

F32 = B.PIC_MODE_FP32_BATCHED
F64 = B.PIC_MODE_FP64_PLAIN


def cubic(**over):
    kw = dict(spline_order=3, n_init=0)
    kw.update(over)
    return pi.coax64(**kw)


def test_cubic_weights():
    for f in (0.0, 0.13, 0.5, 0.77, 0.999):
        w, dw = oracle.s3_weights(f)
        off = np.array([-1.0, 0.0, 1.0, 2.0])
        assert w.sum() == pytest.approx(1.0, abs=1e-15)
        assert (w * off).sum() == pytest.approx(f, abs=1e-15)          # reproduces linear functions
        assert (w * off ** 2).sum() == pytest.approx(f * f + 1.0 / 3.0, abs=1e-14)  # B-spline variance 1/3
        assert dw.sum() == pytest.approx(0.0, abs=1e-15)
        assert (dw * off).sum() == pytest.approx(1.0, abs=1e-14)
        h = 1e-6
        wp, _ = oracle.s3_weights(f + h) if f + h < 1 else oracle.s3_weights(f)
        wm, _ = oracle.s3_weights(f - h) if f - h >= 0 else oracle.s3_weights(f)
        if 0 < f - h and f + h < 1:
            np.testing.assert_allclose((wp - wm) / (2 * h), dw, atol=1e-8)
    w, _ = oracle.s3_weights(0.0)
    np.testing.assert_allclose(w, [1 / 6, 4 / 6, 1 / 6, 0.0], atol=1e-16)


def test_cubic_deposit_is_exact():
    c = cubic()
    S = oracle.auto_shift(c["weight"])
    W = round(c["weight"] * 2.0 ** S)
    rng = np.random.default_rng(2)
    for _ in range(20):
        r, z = rng.uniform(c["a"], c["b"]), rng.uniform(0, c["L"])
        Qx = oracle.s3_deposit(c, r, z, W)
        assert Qx.sum() == W and (Qx != 0).sum() <= 16
        # the node charges are W times the weight products but for the last (the remainder)
        dr, dz = (c["b"] - c["a"]) / c["nr"], c["L"] / c["nz"]
        i0, j0 = int((r - c["a"]) / dr), int(z / dz)
        wr, _ = oracle.s3_weights((r - c["a"]) / dr - i0)
        wz, _ = oracle.s3_weights(z / dz - j0)
        blk = Qx[i0:i0 + 4, j0:j0 + 4]
        want = np.rint(W * np.outer(wr, wz))
        assert np.array_equal(blk.ravel()[:15], want.ravel()[:15].astype(np.int64))


def _manufactured(c):
    a, b, L = c["a"], c["b"], c["L"]
    kr, kz = np.pi / (b - a), np.pi / L
    phi = lambda r, z: np.sin(kr * (r - a)) * np.sin(kz * z)
    f = lambda r, z: (kr ** 2 + kz ** 2) * phi(r, z) - kr * np.cos(kr * (r - a)) * np.sin(kz * z) / r
    return phi, f


def test_manufactured_solution_fourth_order():
    """phi* = sin(pi (r-a)/(b-a)) sin(pi z/L) is odd about every wall, so the
    reflected cubic space holds it to fourth order (its gradient to third)."""
    rng = np.random.default_rng(1)
    errs, ferrs = [], []
    for nr, nz in ((8, 16), (16, 32), (32, 64)):
        c = cubic(nr=nr, nz=nz)
        phi, f = _manufactured(c)
        cx = oracle.s3_poisson_fn(c, f)
        pts = [(rng.uniform(c["a"], c["b"]), rng.uniform(0, c["L"])) for _ in range(200)]
        errs.append(max(abs(oracle.s3_phi_at(c, cx, r, z) - phi(r, z)) for r, z in pts))
        e = 0.0
        for r, z in pts[:60]:
            er, ez = oracle.s3_field(c, cx, r, z)
            h = 1e-7
            e = max(e, abs(er + (phi(r + h, z) - phi(r - h, z)) / (2 * h)),
                    abs(ez + (phi(r, z + h) - phi(r, z - h)) / (2 * h)))
        ferrs.append(e)
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12, errs
    assert ferrs[0] / ferrs[1] > 6 and ferrs[1] / ferrs[2] > 6, ferrs
    assert errs[-1] < 2e-7


def _manufactured_open(c):
    a, b, L = c["a"], c["b"], c["L"]
    kr, kz = np.pi / (b - a), np.pi / L
    phi = lambda r, z: np.sin(kr * (r - a)) * np.cos(kz * z)
    f = lambda r, z: (kr ** 2 + kz ** 2) * phi(r, z) - kr * np.cos(kr * (r - a)) * np.cos(kz * z) / r
    return phi, f


def test_manufactured_solution_fourth_order_open_ends():
    """Open ends (zero z-derivative at z = 0, L, Sec. II.A): phi* = sin(pi
    (r-a)/(b-a)) cos(pi z/L) is odd about the electrodes and even about the
    ends, so the cubic space with odd reflection in r and even reflection in z
    holds it to fourth order (its gradient to third).  Dropping the even
    reflection (Dirichlet ends) cannot represent cos(pi z/L) at the ends and
    fails this."""
    rng = np.random.default_rng(4)
    errs, ferrs = [], []
    for nr, nz in ((8, 16), (16, 32), (32, 64)):
        c = cubic(nr=nr, nz=nz, end_mode=2, V_end=0.0)
        phi, f = _manufactured_open(c)
        cx = oracle.s3_poisson_fn(c, f)
        pts = [(rng.uniform(c["a"], c["b"]), rng.uniform(0, c["L"])) for _ in range(200)]
        pts += [(rng.uniform(c["a"], c["b"]), z) for z in (0.0, c["L"] * (1 - 1e-12))]
        errs.append(max(abs(oracle.s3_phi_at(c, cx, r, z) - phi(r, z)) for r, z in pts))
        e = 0.0
        for r, z in pts[:60]:
            er, ez = oracle.s3_field(c, cx, r, z)
            h = 1e-7
            e = max(e, abs(er + (phi(r + h, z) - phi(r - h, z)) / (2 * h)),
                    abs(ez + (phi(r, z + h) - phi(r, z - h)) / (2 * h)))
        ferrs.append(e)
        # the z-derivative vanishes on the ends
        for r in np.linspace(c["a"], c["b"], 7)[1:-1]:
            assert abs(oracle.s3_field(c, cx, r, 0.0)[1]) < 1e-12 * abs(ferrs[-1] + 1.0) * 1e6
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12, errs
    assert ferrs[0] / ferrs[1] > 6 and ferrs[1] / ferrs[2] > 6, ferrs
    assert errs[-1] < 2e-7


def test_open_ends_column_charge_gives_a_z_independent_potential():
    """A source that does not depend on z, with open ends: the solution is
    the radial one at every z (the z-constant function is in the evenly
    reflected space), so every column of coefficients is the same."""
    c = cubic(nr=16, nz=32, end_mode=2, V_end=0.0)
    cx = oracle.s3_poisson_fn(c, lambda r, z: np.sin(7.0e2 * (r - c["a"])) + 1.0).reshape(c["nr"] + 3, -1)
    inner = cx[1:-1, :]                       # ghosted rows 0 .. nr, every z column (ghosts included)
    spread = np.abs(inner - inner[:, [1]]).max()
    assert spread <= 1e-12 * np.abs(inner).max() and np.abs(inner).max() > 0.0


def test_green_reciprocity_of_deposit_and_gather():
    """The potential of charge 1 read with the cubic basis at x2 equals that
    of charge 2 at x1 (symmetric system, the same basis for load and read)."""
    c = cubic(nr=32, nz=64)
    x1, x2 = (3.3e-3, 17.2e-3), (7.9e-3, 41.7e-3)
    vals = []
    for src, at in ((x1, x2), (x2, x1)):
        o = oracle.Sim(c, capacity=16)
        st = dict(r=np.array([src[0]]), z=np.array([src[1]]), vr=np.zeros(1), vt=np.zeros(1), vz=np.zeros(1),
                  w=np.array([c["weight"]]), key=np.zeros(1, dtype=np.uint64))
        o.set_particles(st)
        vals.append(oracle.s3_phi_at(c, o.coef3(), *at))
        o.close()
    assert vals[0] == pytest.approx(vals[1], rel=1e-9) and vals[0] != 0.0


def test_cubic_and_bilinear_agree_on_a_smooth_cloud():
    """Both discretise the same continuum problem: on a smooth cloud their
    space-charge potentials agree to the discretisation error."""
    c1 = pi.coax64(nr=64, nz=128, n_init=0)
    c3 = dict(c1, spline_order=3)
    st = pi.cloud_state(c1, 200000, seed=3)
    phis = []
    for c in (c1, c3):
        o = oracle.Sim(c, capacity=250000)
        o.set_particles(st)
        phis.append(o.phi() - oracle.vacuum(c))
        o.close()
    d = np.abs(phis[0] - phis[1]).max() / np.abs(phis[0]).max()
    assert d < 0.05, d


@pytest.mark.gpu
@pytest.mark.parametrize("end_mode", [0, 2])
def test_gpu_cubic_solve_matches_the_oracle(end_mode):
    """The transform-based cubic solve (sine modes for electrode ends, cosine
    modes for open ends) against the oracle's assembled Galerkin system."""
    c = cubic(nr=64, nz=128, end_mode=end_mode)
    st = pi.particle_state(c, 40000, seed=12)
    g, o = gpu_and_oracle(c, st, frozen=0)
    Qx, cx = g.spline3()
    assert np.array_equal(Qx, o.charge3())
    assert np.array_equal(g.charge(), o.charge())
    ocx = o.coef3()
    assert np.abs(cx - ocx).max() <= 1e-11 * np.abs(ocx).max()
    vac = oracle.vacuum(c)
    sg, so = g.phi() - vac, o.phi() - vac
    assert np.abs(sg - so).max() <= 1e-11 * np.abs(so).max()
    g.close()


@pytest.mark.gpu
@pytest.mark.parametrize("collisions,end_mode", [(0, 0), (1, 0), (1, 2)])
def test_gpu_cubic_steps_match_the_oracle(collisions, end_mode):
    c = cubic(nr=64, nz=128, p_mbar=30.0 if collisions else 1e-6, E_cap_eV=3000.0, collisions=collisions,
              end_mode=end_mode)
    st = pi.cloud_state(c, 30000, seed=13)
    g, o = gpu_and_oracle(c, st, frozen=0)
    g.step(15)
    o.step(15)
    gd, od = g.diag(), o.diag()
    for k in ("n_live", "n_absorbed", "n_elastic", "n_ioniz"):
        assert gd[k] == od[k], k
    gp, op = by_key(g.get_particles()), by_key(o.get_particles())
    assert np.array_equal(gp["key"], op["key"])
    np.testing.assert_allclose(gp["r"], op["r"], rtol=1e-11)
    np.testing.assert_allclose(gp["z"], op["z"], rtol=1e-11)
    assert rel_vec_err(gp, op).max() <= 1e-9
    g.close()


@pytest.mark.gpu
def test_cubic_configurations_refused():
    for cfgs, mode in (([cubic(), pi.coax64(n_init=0)], F64), ([cubic(), pi.coax64(n_init=0)], F32)):
        with pytest.raises(B.PicError) as e:
            B.Sim(cfgs, mode=mode)
        assert e.value.status == B.PIC_EINVAL


def _fp32_exact(st):
    return {k: (v.astype(np.float32).astype(np.float64) if v.dtype == np.float64 else v) for k, v in st.items()}


def _run32(cfg, steps, **run):
    g = B.Sim([cfg], mode=F32, **run)
    g.step(steps)
    out = (by_key(g.get_particles()), g.charge(), g.spline3()[0], g.diag())
    g.close()
    return out


@pytest.mark.gpu
def test_fp32_cubic_is_invariant_to_tiles_and_launches():
    """LDS windows or device atomics, graph or plain launches: the same bits."""
    cfg = cubic(nr=64, nz=128, n_init=40000, p_mbar=3.0, E_cap_eV=3000.0)
    ref = _run32(cfg, 30, tile_r=16, tile_z=16, sort_interval=8, use_graph=1)
    assert ref[3]["n_elastic"] > 100
    for kw in (dict(tile_r=8, tile_z=8, sort_interval=1, use_graph=0),
               dict(tile_r=4, tile_z=32, sort_interval=3, halo=1, chunk=300)):
        got = _run32(cfg, 30, **kw)
        for k in ("key", "r", "z", "vr", "vt", "vz"):
            assert np.array_equal(ref[0][k], got[0][k]), (kw, k)
        assert np.array_equal(ref[1], got[1]) and np.array_equal(ref[2], got[2])
        for k in ("n_live", "n_elastic", "n_ioniz", "n_null_cand"):
            assert ref[3][k] == got[3][k], (kw, k)


@pytest.mark.gpu
@pytest.mark.parametrize("end_mode", [0, 2])
def test_fp32_cubic_one_step_against_the_oracle(end_mode):
    c = cubic(nr=64, nz=128, p_mbar=30.0, E_cap_eV=3000.0, end_mode=end_mode)
    st = _fp32_exact(pi.cloud_state(c, 20000, seed=41))
    g, o = gpu_and_oracle(c, st, frozen=0, mode=F32)
    Qg, cg = g.spline3()
    Qo, co = o.charge3(), o.coef3()
    W = round(c["weight"] * 2.0 ** o.S)
    assert Qg.sum() == Qo.sum() == len(st["r"]) * W
    assert np.linalg.norm(Qg - Qo) <= 1e-6 * np.linalg.norm(Qo)
    assert np.abs(cg - co).max() <= 1e-5 * np.abs(co).max()
    g.step(1)
    o.step(1)
    gd, od = g.diag(), o.diag()
    assert gd["n_null_cand"] == od["n_null_cand"]
    assert abs(gd["n_elastic"] - od["n_elastic"]) <= 2 and abs(gd["n_ioniz"] - od["n_ioniz"]) <= 2
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
@pytest.mark.parametrize("end_mode", [0, 2])
def test_fp32_cubic_tracks_the_oracle_over_a_run(end_mode):
    """The small trap at the raised pressure, 300 self-consistent steps with
    cubic shapes: FP32 density and counts within 2% of the FP64 oracle."""
    cfg = cubic(n_init=50000, p_mbar=1e-1, diag_interval=10, end_mode=end_mode)
    g = B.Sim([cfg], mode=F32)
    o = oracle.Sim(cfg, fx_shift=g.diag()["S"])
    o.load()
    g.step(300)
    o.step(300)
    gd, od = g.diag(want_density=True), o.diag()
    na = o.time_avg_density()
    mask = na > 0.2 * na.max()
    rel = np.linalg.norm((gd["time_avg_density"] - na)[mask]) / np.linalg.norm(na[mask])
    assert rel < 0.02, rel
    assert gd["peak_density"] == pytest.approx(od["peak_density"], rel=0.02)
    assert gd["n_live"] == pytest.approx(od["n_live"], rel=0.02)
    g.close()


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [F64, F32])
def test_cubic_charge_bookkeeping_with_source_and_ionisation(mode):
    """Every path that deposits (the window, device atomics, ionisation
    children, seed-source electrons): the cubic grid and the bilinear grid
    each hold exactly W per live electron after every step."""
    cfg = cubic(n_init=30000, p_mbar=30.0, E_cap_eV=3000.0, src_rate=40.0, src_T_eV=2.0)
    g = B.Sim([cfg], mode=mode)
    W = None
    for _ in range(6):
        g.step(3)
        d = g.diag()
        W = W or round(cfg["weight"] * 2.0 ** d["S"])
        Qx, _ = g.spline3()
        assert Qx.sum() == d["n_live"] * W
        assert g.charge().sum() == d["n_live"] * W
    assert d["n_ioniz"] > 0 and d["n_source"] > 0
    g.close()


@pytest.mark.gpu
def test_fp32_cubic_autotune_and_growth_keep_the_bits():
    """The autotuner's trial shapes (the cubic windows included in the LDS
    budget) and storage regrowth change no result of a cubic run."""
    cfg = cubic(n_init=40000, p_mbar=3.0, E_cap_eV=3000.0)
    g = B.Sim([cfg], mode=F32, capacity_factor=1.3)
    t = g.autotune(trial_steps=4)
    assert t["trials"] >= 10 and t["ms_per_step"] > 0
    g.step(150)
    got = (by_key(g.get_particles()), g.spline3()[0], g.diag())
    g.close()
    ref = B.Sim([cfg], mode=F32, capacity_factor=8.0)
    ref.step(got[2]["step"])
    want = (by_key(ref.get_particles()), ref.spline3()[0], ref.diag())
    ref.close()
    for k in ("key", "r", "z", "vr", "vt", "vz"):
        assert np.array_equal(want[0][k], got[0][k]), k
    assert np.array_equal(want[1], got[1])
    assert want[2]["n_ioniz"] == got[2]["n_ioniz"] > 0
