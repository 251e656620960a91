"""Meshes whose nz is not a power of two: the z transforms (sine modes
between electrode ends, cosine modes with open ends) run as mixed-radix
FFTs of 2 nz points (radix 8, 4, 2, 3 and 5 passes), so nz may be any
multiple of 4 up to 4096 without a prime factor above 5.  CPU: the host-only
validation.  GPU: vacuum and space-charge potentials, the cubic solve and
self-consistent steps against the oracle, a batch whose instances have
different nz, and the batched FP32 form's invariance on such a mesh."""
import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import by_key, gpu_and_oracle, rel_vec_err
from paper_2206_14662_amd import binding as B

F32 = B.PIC_MODE_FP32_BATCHED


def _with_insert(**over):
    kw = dict(a=1e-3, b=10e-3, L=30e-3, n_init=0, ins_r0=10e-3, ins_z0=15e-3, ins_er=3.1e-3, ins_ez=7.3e-3)
    kw.update(over)
    return pi.coax64(**kw)


def test_mesh_sizes_accepted_and_refused():
    """Host-only validation (through the insert layout call)."""
    for nz in (96, 120, 160, 240, 1500):
        B.pic_insert_layout(_with_insert(nr=32, nz=nz))
    for nz in (28, 42, 98, 4100, 6):
        with pytest.raises(B.PicError) as e:
            B.pic_insert_layout(_with_insert(nr=32, nz=nz))
        assert e.value.status == B.PIC_EINVAL


@pytest.mark.gpu
@pytest.mark.parametrize("nr,nz", [(64, 96), (32, 12), (64, 160), (16, 1500), (40, 4000)])
@pytest.mark.parametrize("end_mode", [0, 2])
def test_field_solver_mixed_radix(nr, nz, end_mode):
    cfg = pi.coax64(nr=nr, nz=nz, n_init=0, end_mode=end_mode)
    g = B.Sim([cfg])
    ref = oracle.vacuum(cfg)
    assert np.max(np.abs(g.phi() - ref)) <= 1e-9 * np.max(np.abs(ref))
    g.close()
    st = pi.cloud_state(cfg, 5000, seed=nr + nz)
    g, o = gpu_and_oracle(cfg, st)
    assert np.array_equal(g.charge(), o.charge())
    sc_g, sc_o = g.phi() - ref, o.phi() - ref
    assert np.max(np.abs(sc_g - sc_o)) <= 1e-8 * np.max(np.abs(sc_o))
    g.close()


@pytest.mark.gpu
@pytest.mark.parametrize("end_mode", [0, 2])
def test_cubic_solve_mixed_radix(end_mode):
    c = pi.coax64(nr=64, nz=96, n_init=0, end_mode=end_mode, spline_order=3)
    st = pi.particle_state(c, 20000, seed=12)
    g, o = gpu_and_oracle(c, st, frozen=0)
    Qx, cx = g.spline3()
    assert np.array_equal(Qx, o.charge3())
    ocx = o.coef3()
    assert np.abs(cx - ocx).max() <= 1e-11 * np.abs(ocx).max()
    g.close()


@pytest.mark.gpu
def test_batch_of_different_nz():
    """One twiddle table serves every length: instances with nz = 128, 96 and
    160 in one context, each against the oracle."""
    cfgs = [pi.coax64(nz=nz, n_init=0, seed=5 + nz) for nz in (128, 96, 160)]
    S = B.pic_auto_shift(max(c["weight"] for c in cfgs))
    cfgs = [dict(c, fx_shift=S) for c in cfgs]
    g = B.Sim(cfgs, capacity_min=20000)
    for k, c in enumerate(cfgs):
        ref = oracle.vacuum(c)
        assert np.max(np.abs(g.phi(k) - ref)) <= 1e-9 * np.max(np.abs(ref)), k
        st = pi.cloud_state(c, 4000, seed=k)
        g.set_particles(st, k)
        o = oracle.Sim(c, fx_shift=S)
        o.set_particles(st)
        sc_g, sc_o = g.phi(k) - ref, o.phi() - ref
        assert np.max(np.abs(sc_g - sc_o)) <= 1e-8 * np.max(np.abs(sc_o)), k
    g.close()


@pytest.mark.gpu
def test_steps_on_a_mixed_radix_mesh():
    """FP64 steps with collisions match the oracle; the FP32 form is
    bit-identical across tile shapes on the same mesh."""
    c = pi.coax64(nr=48, nz=120, p_mbar=30.0, E_cap_eV=3000.0, n_init=0)
    st = pi.cloud_state(c, 20000, seed=3)
    g, o = gpu_and_oracle(c, st, frozen=0)
    g.step(10)
    o.step(10)
    gd, od = g.diag(), o.diag()
    for k in ("n_live", "n_elastic", "n_ioniz", "n_absorbed"):
        assert gd[k] == od[k], k
    gp, op = by_key(g.get_particles()), by_key(o.get_particles())
    assert np.array_equal(gp["key"], op["key"])
    np.testing.assert_allclose(gp["r"], op["r"], rtol=1e-11)
    assert rel_vec_err(gp, op).max() <= 1e-9
    g.close()
    c32 = dict(c, n_init=40000)
    out = []
    for kw in (dict(tile_r=8, tile_z=24, sort_interval=4), dict(tile_r=16, tile_z=40, sort_interval=7, halo=2)):
        h = B.Sim([c32], mode=F32, **kw)
        h.step(20)
        out.append((by_key(h.get_particles()), h.charge()))
        h.close()
    for k in ("key", "r", "z", "vr", "vt", "vz"):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    assert np.array_equal(out[0][1], out[1][1])
