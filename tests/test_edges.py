"""Edge cases: empty and one-particle instances inside a batch, particles on
mesh nodes and cell edges, the extreme mesh shapes the field solver accepts
(nz from 4 to 4096, tall and flat meshes), and invalid input refused."""
import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import by_key, gpu_and_oracle
from paper_2206_14662_amd import binding as B

pytestmark = pytest.mark.gpu
F32 = B.PIC_MODE_FP32_BATCHED
F64 = B.PIC_MODE_FP64_PLAIN


def test_batch_with_empty_and_single_particle_instances():
    cfgs = [pi.coax64(n_init=0, seed=1), pi.coax64(n_init=1, seed=2), pi.coax64(n_init=5000, seed=3, p_mbar=10.0,
                                                                            E_cap_eV=3000.0)]
    g = B.Sim(cfgs, mode=F32)
    g.step(50)
    d = [g.diag(k) for k in range(3)]
    assert d[0]["n_live"] == 0 and d[0]["total_Q"] == 0 and d[0]["particle_steps"] == 0
    assert d[1]["n_live"] + sum(d[1]["n_absorbed"]) == 1 + d[1]["n_ioniz"]
    assert d[2]["n_ioniz"] > 0
    batch = [(by_key(g.get_particles(k)), g.charge(k)) for k in range(3)]
    g.close()
    for k, c in enumerate(cfgs):
        h = B.Sim([c], mode=F32)
        h.step(50)
        p, q = by_key(h.get_particles()), h.charge()
        for a in ("key", "r", "z", "vr", "vt", "vz"):
            assert np.array_equal(p[a], batch[k][0][a]), (k, a)
        assert np.array_equal(q, batch[k][1])
        h.close()


@pytest.mark.parametrize("mode", [F64, F32])
def test_particles_on_nodes_and_cell_edges(mode):
    """Particles exactly on mesh nodes, on the last cell's outer edge in r and
    z, and next to the walls: deposits stay exact and land on the right
    nodes; a particle on an electrode is absorbed by the first push."""
    cfg = pi.coax64(collisions=0, p_mbar=1e-12)
    d = oracle.derive(cfg)
    a, b, L = cfg["a"], cfg["b"], cfg["L"]
    # 1 um from the walls: clear of them in FP32 as well (spacing ~1e-9 m there)
    r = np.array([a + 3 * d["dr"], a + 10 * d["dr"], b - 1e-6, a + 1e-6, a + 7.5 * d["dr"], b - d["dr"]])
    z = np.array([5 * d["dz"], 64 * d["dz"], L / 2, L / 3, L - 1e-6, 1e-6])
    n = len(r)
    st = dict(r=r, z=z, vr=np.zeros(n), vt=np.full(n, 1e5), vz=np.zeros(n), w=np.full(n, cfg["weight"]),
              key=np.arange(n, dtype=np.uint64))
    g, o = gpu_and_oracle(cfg, st, fields=pi.uniform_fields(cfg, Er=0.0, Bz=0.28), mode=mode)
    W = round(cfg["weight"] * 2.0 ** o.S)
    assert g.charge().sum() == n * W
    if mode == F64:
        assert np.array_equal(g.charge(), o.charge())
        # the node particles put their whole charge on their node
        q = g.charge()
        assert q[3, 5] == W and q[10, 64] == W
    g.step(1)
    o.step(1)
    assert g.diag()["n_live"] == o.diag()["n_live"]
    assert g.diag()["n_absorbed"] == o.diag()["n_absorbed"]
    g.close()


@pytest.mark.parametrize("nr,nz", [(4, 4), (6, 4096), (8, 2048), (300, 8), (512, 64)])
def test_field_solver_extreme_meshes(nr, nz):
    cfg = pi.coax64(nr=nr, nz=nz, n_init=0)
    g = B.Sim([cfg])
    ref = oracle.vacuum(cfg)
    assert np.max(np.abs(g.phi() - ref)) <= 1e-9 * np.max(np.abs(ref))
    st = pi.cloud_state(cfg, 2000, seed=nr + nz)
    g2, o = gpu_and_oracle(cfg, st)
    assert np.array_equal(g2.charge(), o.charge())
    vac = oracle.vacuum(cfg)
    sc_g, sc_o = g2.phi() - vac, o.phi() - vac
    assert np.max(np.abs(sc_g - sc_o)) <= 1e-8 * np.max(np.abs(sc_o))
    g.close()
    g2.close()


def test_invalid_input_is_refused_and_the_context_survives():
    cfg = pi.coax64(n_init=1000)
    g = B.Sim([cfg], mode=F32)
    bad = pi.cloud_state(cfg, 10, seed=1)
    bad["r"][3] = cfg["b"] + 1e-3  # outside the electrodes
    with pytest.raises(B.PicError) as e:
        g.set_particles(bad)
    assert e.value.status == B.PIC_EINVAL
    with pytest.raises(B.PicError):
        B.pic_step(g.ctx, -1)
    with pytest.raises(B.PicError) as e:
        B.pic_diag(g.ctx, 5)
    assert e.value.status == B.PIC_EINVAL
    g.step(3)
    assert g.diag()["step"] == 3
    g.close()
