"""The batched FP32 form at the benchmark's full sizes (8 x 256x1024 with 16M
electrons each; 32 x 128x512 with 0.5M-8M each), in the launch configuration
the benchmark runs: one step of the whole batch, then samples of particles
from several instances are replayed through the FP64 oracle with the same
(FP32-valued) fields and step counter, and the exact bookkeeping invariants
are checked for every instance."""
import numpy as np
import pytest

import oracle
import pic_inputs as pi
from helpers import by_key, rel_vec_err
from paper_2206_14662_amd import binding as B

pytestmark = pytest.mark.gpu
F32 = B.PIC_MODE_FP32_BATCHED


def sampled_step(cfgs, check, n_sample=4096):
    g = B.Sim(cfgs, mode=F32)
    fields = {k: g.fields(k) for k in check}
    before = {k: g.get_particles(k) for k in check}
    d0 = [g.diag(k) for k in range(len(cfgs))]
    g.step(1)
    d1 = [g.diag(k) for k in range(len(cfgs))]
    after = {k: by_key(g.get_particles(k)) for k in check}
    # exact bookkeeping on every instance of the batch
    for k, c in enumerate(cfgs):
        # the FP32 form carries FP32 weights: each electron deposits exactly
        # rint(float32(w) 2^S) (the FP64 weight itself may not be an FP32 value)
        W = round(float(np.float32(c["weight"])) * 2.0 ** d1[k]["S"])
        assert d1[k]["total_Q"] == d1[k]["n_live"] * W, k
        assert d1[k]["n_live"] + sum(d1[k]["n_absorbed"]) == c["n_init"] + d1[k]["n_ioniz"], k
        assert d1[k]["step"] == d0[k]["step"] + 1
        assert d1[k]["n_spawn_dropped"] == 0
    g.close()
    rng = np.random.default_rng(7)
    for k in check:
        b = before[k]
        idx = rng.choice(len(b["r"]), n_sample, replace=False)
        sample = {a: v[idx] for a, v in b.items()}
        o = oracle.Sim(cfgs[k], fx_shift=d1[k]["S"], capacity=4 * n_sample)
        o.set_fields(**{a: v.reshape(-1) for a, v in fields[k].items()}, frozen=1)
        o.set_particles(sample)
        o.step(1)
        op = by_key(o.get_particles())
        keep = op["key"] < np.uint64(1 << 63)
        opk = {a: v[keep] for a, v in op.items()}
        pos = np.searchsorted(after[k]["key"], opk["key"])
        pos = np.minimum(pos, len(after[k]["key"]) - 1)
        found = after[k]["key"][pos] == opk["key"]
        # survivors agree; an absorption decided differently at FP32 rounding is rare
        assert found.sum() >= len(opk["key"]) - 2, k
        pos = pos[found]
        ref = {a: v[found] for a, v in opk.items()}
        got = {a: after[k][a][pos] for a in ("r", "z", "vr", "vt", "vz", "w")}
        np.testing.assert_allclose(got["r"], ref["r"], rtol=2e-6)
        np.testing.assert_allclose(got["z"], ref["z"], rtol=2e-6)
        assert np.array_equal(got["w"], ref["w"])
        err = rel_vec_err(got, ref)
        assert np.quantile(err, 0.999) < 1e-4, (k, np.quantile(err, 0.999))


def test_batch8_full_size_sampled_one_step():
    sampled_step(pi.batch8(), check=(0, 5, 7))


def test_scan32_full_size_sampled_one_step():
    cfgs = pi.scan32()
    sizes = [c["n_init"] for c in cfgs]
    sampled_step(cfgs, check=(0, int(np.argmin(sizes)), int(np.argmax(sizes)), 31))
