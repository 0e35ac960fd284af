"""Incremental mode on the GPU (af_incremental_*) against the oracle's
state machine (oracle/incremental.py) on the tiny scene: after every frame,
every point's label, stored score, its orientation and the confidence a are
bit-identical, and so are the counts of each trigger, the sample size, the
evaluations and the backlog.  The budget (700) is below the number of queued
points, so the backlog carries across frames; one frame moves the sensor by
5 cm (trigger iii must not fire) and the next by 15 cm (it must)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

STAT_KEYS = ("new_points", "trig_i", "trig_ii", "trig_iii", "sampled", "evaluated", "backlog")
ORC_KEYS = ("new", "trig_i", "trig_ii", "trig_iii", "sampled", "evaluated", "backlog")


def _origins(frames):
    out = []
    for j, f in enumerate(frames):
        o = np.asarray(f.origin, np.float32)
        if j == 4:
            o = (np.asarray(frames[3].origin, np.float64) + [0.05, 0, 0]).astype(np.float32)
        if j == 5:
            o = (np.asarray(frames[3].origin, np.float64) + [0.15, 0, 0]).astype(np.float32)
        out.append(o)
    return out


@pytest.mark.parametrize("budget", [700, 100000])
def test_incremental_against_oracle(synth_mod, oracle_mod, budget):
    import torch
    from oracle.incremental import IncrementalOracle
    from paper_2608_06412_amd import Context, default_config
    w = synth_mod.tiny()
    frames = w.frames(8)
    ctx = Context(default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 15,
                                 max_points=1 << 17))
    ctx.set_tool_kernels(0, w.tool, w.rot)
    ctx.incremental_enable(0, budget)
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    orc.set_tool(0, w.tool, w.rot)
    inc = IncrementalOracle(orc, 0, len(w.rot), budget=budget)
    for j, (f, o) in enumerate(zip(frames, _origins(frames))):
        ctx.incremental_frame(torch.from_numpy(f.xyz).cuda(), o, f.frame_id)
        ost = inc.frame(f.xyz, o, f.frame_id)
        gst = ctx.incremental_stats()
        print("frame", j, "gpu", gst, "oracle", ost, flush=True)
        for gk, ok in zip(STAT_KEYS, ORC_KEYS):
            assert gst[gk] == ost[ok], (j, gk)
        g = ctx.read_incremental()
        keys, lab, best, bdir, a = inc.labels()
        assert np.array_equal(g["key"], keys), j
        assert np.array_equal(g["label"], lab), (j, np.flatnonzero(g["label"] != lab)[:10])
        assert np.array_equal(g["best"].astype(np.int32), best), j
        assert np.array_equal(g["best_dir"].astype(np.int32), bdir), j
        assert np.array_equal(g["a"], a), j
    assert ost["backlog"] > 0 or budget > 10000
    if budget < 10000:
        assert (lab == 4).any() or (lab == 1).any()


def test_incremental_argument_errors(synth_mod):
    import torch
    from paper_2608_06412_amd import AFError, Context, default_config
    w = synth_mod.tiny()
    ctx = Context(default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 12,
                                 max_points=1 << 14))
    f = w.frames(1)[0]
    with pytest.raises(AFError):
        ctx.incremental_frame(torch.from_numpy(f.xyz).cuda(), f.origin, 0)   # not enabled
    with pytest.raises(AFError):
        ctx.incremental_enable(0, 100)                                        # no tool
    ctx.set_tool_kernels(0, w.tool, w.rot)
    with pytest.raises(AFError):
        ctx.incremental_enable(0, 0)
    ctx.integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, 0)
    with pytest.raises(AFError):
        ctx.incremental_enable(0, 100)                                        # map not empty


def test_incremental_moving_surface(synth_mod, oracle_mod):
    """Trigger (i): a plane moved 9 cm back (v = 2 cm, tau = 10 cm); GPU and
    oracle agree on every count and every point's state."""
    import torch
    from oracle.incremental import IncrementalOracle
    from paper_2608_06412_amd import Context, default_config
    from test_oracle_incremental import plane_frames
    w = synth_mod.tiny()
    ctx = Context(default_config(0.02, 0.10, r_c=0.01, max_blocks=1 << 12, max_points=1 << 14))
    ctx.set_tool_kernels(0, w.tool, w.rot)
    ctx.incremental_enable(0, 1000)
    orc = oracle_mod.Oracle(voxel=0.02, trunc=0.10, r_c=0.01)
    orc.set_tool(0, w.tool, w.rot)
    inc = IncrementalOracle(orc, 0, len(w.rot), budget=1000)
    fired = 0
    for xyz, o, fid in plane_frames():
        ctx.incremental_frame(torch.from_numpy(xyz).cuda(), o, fid)
        ost = inc.frame(xyz, o, fid)
        gst = ctx.incremental_stats()
        for gk, ok in zip(STAT_KEYS, ORC_KEYS):
            assert gst[gk] == ost[ok], (fid, gk)
        fired += gst["trig_i"]
        g = ctx.read_incremental()
        keys, lab, best, bdir, a = inc.labels()
        assert np.array_equal(g["key"], keys) and np.array_equal(g["label"], lab)
        assert np.array_equal(g["best"].astype(np.int32), best)
        assert np.array_equal(g["a"], a)
    assert fired > 0
