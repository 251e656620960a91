"""The allocation-free moments (pic_moments_noalloc) against pic_moments, the
entry point that allocates its accumulators: both forms, two calls in a row
on different contexts, the second on a smaller mesh with fewer electrons (the
scratch then still holds the first call's larger contents), and a mesh above
the scratch's limit refused."""
import numpy as np
import pytest
import torch

import pic_inputs as pi
from paper_2206_14662_amd import binding as B

pytestmark = pytest.mark.gpu
CHANNELS = 11


def _noalloc(g, k=0):
    n = g.nodes(k)
    out = torch.full((CHANNELS * n,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    B.pic_moments_noalloc(g.ctx, k, out.data_ptr())
    B.pic_sync(g.ctx)
    got = out.cpu().numpy().reshape((CHANNELS,) + g.shapes[k])
    del out
    return got


@pytest.mark.parametrize("mode", [B.PIC_MODE_FP64_PLAIN, B.PIC_MODE_FP32_BATCHED])
def test_noalloc_moments_match_the_allocating_entry_point(mode):
    big = pi.coax64(nr=128, nz=512, n_init=200000, p_mbar=3.0, E_cap_eV=3000.0)
    small = pi.coax64(n_init=20000, p_mbar=3.0, E_cap_eV=3000.0, seed=5)
    for cfg in (big, small):
        g = B.Sim([cfg], mode=mode)
        g.step(6)
        got = _noalloc(g)
        ref = g.moments()
        assert np.all(np.isfinite(got))
        for c in range(CHANNELS):
            scale = np.abs(ref[c]).max()
            assert scale > 0.0
            # the same sums; only the order of the floating-point atomics differs
            assert np.abs(got[c] - ref[c]).max() <= 1e-12 * scale, c
        g.close()


def test_noalloc_moments_refuse_a_mesh_above_the_scratch():
    g = B.Sim([pi.coax64(nr=512, nz=2048, n_init=0)])
    out = torch.zeros(CHANNELS * g.nodes(0), dtype=torch.float64, device="cuda")
    with pytest.raises(B.PicError) as e:
        B.pic_moments_noalloc(g.ctx, 0, out.data_ptr())
    assert e.value.status == B.PIC_EINVAL and "scratch" in str(e.value)
    g.close()
