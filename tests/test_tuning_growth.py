"""Re-tiling, the autotuner and device storage growth: none of them may
change any result (the FP32 form is bit-identical across tile shapes, halos
and sort intervals; both forms across storage layouts)."""
import json

import numpy as np
import pytest

import pic_inputs as pi
from helpers import by_key
from paper_2206_14662_amd import binding as B

pytestmark = pytest.mark.gpu
F32 = B.PIC_MODE_FP32_BATCHED
F64 = B.PIC_MODE_FP64_PLAIN


def hot(**over):
    kw = dict(p_mbar=3.0, n_init=40000, E_cap_eV=3000.0)
    kw.update(over)
    return pi.coax64(**kw)


def snapshot(g, k=0):
    return by_key(g.get_particles(k)), g.charge(k), g.diag(k)


def same(a, b, fields=("key", "r", "z", "vr", "vt", "vz", "w")):
    pa, qa, da = a
    pb, qb, db = b
    for k in fields:
        assert np.array_equal(pa[k], pb[k]), k
    assert np.array_equal(qa, qb)
    for k in ("step", "n_live", "n_elastic", "n_ioniz", "n_null_cand", "n_absorbed", "absorbed_W", "total_Q"):
        assert da[k] == db[k], k


def test_retune_mid_run_is_invisible():
    cfg = hot()
    ref = B.Sim([cfg], mode=F32)
    ref.step(45)
    want = snapshot(ref)
    ref.close()
    g = B.Sim([cfg], mode=F32)
    g.step(13)
    g.retune(tile_r=8, tile_z=32, halo=2, sort_interval=3)
    assert B.pic_tuning(g.ctx)["tile_z"] == 32
    g.step(20)
    g.retune(tile_r=32, tile_z=8, halo=0, sort_interval=16)
    g.step(12)
    same(want, snapshot(g))
    # out-of-range requests are refused and leave the context usable
    with pytest.raises(B.PicError):
        g.retune(tile_r=256, tile_z=256, halo=32)
    assert B.pic_tuning(g.ctx)["tile_r"] == 32
    g.step(1)
    g.close()


def test_autotune_picks_a_valid_choice_and_caches_it(tmp_path):
    cfgs = [hot(seed=5), hot(seed=6, nr=40, nz=64, n_init=15000)]
    cache = str(tmp_path / "tune.jsonl")
    g = B.Sim(cfgs, mode=F32)
    t = g.autotune(trial_steps=4, cache_path=cache)
    assert t["trials"] >= 10 and t["ms_per_step"] > 0
    cur = B.pic_tuning(g.ctx)
    for k in ("tile_r", "tile_z", "halo", "sort_interval"):
        assert cur[k] == t[k]
    steps = g.diag(0)["step"]
    got = [snapshot(g, k) for k in range(2)]
    g.close()
    lines = [json.loads(x) for x in open(cache)]
    assert len(lines) == 1 and lines[0]["tile_r"] == t["tile_r"]
    # the trial steps are ordinary steps: a default-tuned run of the same length matches
    ref = B.Sim(cfgs, mode=F32)
    ref.step(steps)
    for k in range(2):
        same(snapshot(ref, k), got[k])
    ref.close()
    # a second context with the same workload takes the cached choice
    h = B.Sim(cfgs, mode=F32)
    t2 = h.autotune(trial_steps=4, cache_path=cache)
    assert t2["trials"] == 0
    for k in ("tile_r", "tile_z", "halo", "sort_interval"):
        assert t2[k] == t[k]
    # the launch shape the trials chose is cached and restored with the tiles
    assert lines[0]["lanes"] in (1, 2) and B.pic_tuning(h.ctx)["lanes"] == lines[0]["lanes"] == cur["lanes"]
    # and so is the launch mode (graphs or plain launches), timed on that choice
    assert lines[0]["graphs"] in (0, 1) and B.pic_tuning(h.ctx)["use_graph"] == lines[0]["graphs"] == cur["use_graph"]
    h.close()
    # an explicit launch mode is kept: the cached choice does not override it
    h = B.Sim(cfgs, mode=F32, use_graph=1 - lines[0]["graphs"])
    h.autotune(trial_steps=4, cache_path=cache)
    assert B.pic_tuning(h.ctx)["use_graph"] == 1 - lines[0]["graphs"]
    h.close()
    # the last cached line of a signature wins: two particles per lane are restored as such
    with open(cache, "a") as f:
        f.write(json.dumps(dict(lines[0], tile_r=8, tile_z=16, lanes=2)) + "\n")
    h = B.Sim(cfgs, mode=F32)
    t3 = h.autotune(trial_steps=4, cache_path=cache)
    tun = B.pic_tuning(h.ctx)
    assert t3["trials"] == 0 and tun["lanes"] == 2 and (tun["tile_r"], tun["tile_z"]) == (8, 16)
    h.step(5)
    h.close()


@pytest.mark.parametrize("mode", [F32, F64])
def test_storage_grows_during_the_run(mode):
    # ionisation roughly doubles the population over the run; 1.3 x n_init
    # slots are more than 3/4 used from the start, so the store regrows at the
    # first capacity check and again later.  The run must match a roomy one.
    cfg = hot()
    roomy = B.Sim([cfg], mode=mode, capacity_factor=8.0)
    roomy.step(300)
    B.pic_sync(roomy.ctx)
    want = snapshot(roomy)
    assert want[2]["n_live"] > 1.5 * cfg["n_init"] and want[2]["n_spawn_dropped"] == 0
    assert roomy.capacity()[1] == 0
    roomy.close()
    g = B.Sim([cfg], mode=mode, capacity_factor=1.3)
    cap0, grows0 = g.capacity()
    assert cap0 == int(np.ceil(1.3 * cfg["n_init"])) and grows0 == 0
    g.step(300)
    B.pic_sync(g.ctx)
    cap1, grows1 = g.capacity()
    assert grows1 >= 2 and cap1 >= want[2]["n_live"]
    got = snapshot(g)
    assert got[2]["n_spawn_dropped"] == 0
    same(want, got)
    g.close()


def test_dropped_electrons_are_reported():
    # a population that outruns its store: the step call (or the next sync)
    # reports PIC_ECAPACITY instead of carrying on silently
    cfg = hot(p_mbar=100.0)
    g = B.Sim([cfg], mode=F32, capacity_factor=1.3)
    with pytest.raises(B.PicError) as e:
        g.step(400)
        B.pic_sync(g.ctx)
    assert e.value.status == B.PIC_ECAPACITY
    g.close()


@pytest.mark.parametrize("mode", [F32, F64])
def test_reserve_keeps_the_state(mode):
    cfg = hot()
    a = B.Sim([cfg], mode=mode)
    a.step(30)
    want = snapshot(a)
    a.close()
    g = B.Sim([cfg], mode=mode)
    g.step(10)
    g.reserve(5 * cfg["n_init"])
    assert g.capacity()[0] >= 5 * cfg["n_init"]
    g.step(20)
    same(want, snapshot(g))
    g.close()
