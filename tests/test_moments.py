"""Fluid moments on the GPU (both forms) against the oracle's on the same
particles: equal up to the summation order of FP64 atomics."""
import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import gpu_and_oracle
from paper_2206_14662_amd import binding as B

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [B.PIC_MODE_FP64_PLAIN, B.PIC_MODE_FP32_BATCHED])
def test_moments_match_the_oracle(mode):
    cfg = pi.coax64(p_mbar=10.0, E_cap_eV=3000.0)
    st = pi.cloud_state(cfg, 30000, seed=8)
    # FP32-representable state: both forms then hold exactly the oracle's values
    st = {k: (v.astype(np.float32).astype(np.float64) if v.dtype == np.float64 else v) for k, v in st.items()}
    g, o = gpu_and_oracle(cfg, st, mode=mode)
    mg, mo = g.moments(), o.moments()
    assert mg.shape == mo.shape == (11, cfg["nr"] + 1, cfg["nz"] + 1)
    for ch in range(11):
        scale = np.max(np.abs(mo[ch]))
        assert np.max(np.abs(mg[ch] - mo[ch])) <= 1e-12 * scale, ch
    # after a self-consistent step with collisions the FP64 form still agrees
    if mode == B.PIC_MODE_FP64_PLAIN:
        g.step(3)
        o.step(3)
        mg, mo = g.moments(), o.moments()
        for ch in range(11):
            scale = np.max(np.abs(mo[ch]))
            assert np.max(np.abs(mg[ch] - mo[ch])) <= 1e-9 * scale, ch
    # the density channel integrates to the live electrons
    V = oracle.node_volume(cfg).reshape(mg.shape[1:])
    assert (mg[0] * V).sum() == pytest.approx(g.diag()["n_live"] * cfg["weight"], rel=1e-12)
    g.close()


@pytest.mark.parametrize("end_mode,mirror", [(0, 0.0), (0, 0.3), (2, 0.3)])
def test_well_depth_matches_the_oracle(end_mode, mirror):
    cfg = pi.coax64(end_mode=end_mode, mirror_k=mirror, p_mbar=10.0, E_cap_eV=3000.0)
    g = B.Sim([cfg], mode=B.PIC_MODE_FP64_PLAIN)
    r = np.linspace(1.5e-3, 9.5e-3, 17)
    # the library's depth on its own potential equals the oracle's on the same array
    for steps in (0, 20):
        g.step(steps)
        dep, zm = g.well_depth(r)
        dep_o, zm_o = oracle.well_depth(cfg, g.phi(), r)
        np.testing.assert_allclose(dep, dep_o, rtol=1e-12, atol=1e-9)
        np.testing.assert_array_equal(zm, zm_o)
    g.close()
