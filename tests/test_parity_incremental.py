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


def test_adaptive_cap_and_drains_against_oracle(synth_mod, oracle_mod):
    """The adaptive cap (lookup target 150,000, cap in [50, 3,000], first cap
    400) and drains of the backlog between frames (300 after even frames,
    everything after frame 5): after every frame and every drain, the cap,
    the counts and every point's state equal the oracle's."""
    import torch
    from oracle.incremental import IncrementalOracle
    from paper_2608_06412_amd import Context, default_config
    w = synth_mod.tiny()
    frames = w.frames(8)
    ctx = Context(default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 15,
                                 max_points=1 << 17))
    ctx.set_tool_kernels(0, w.tool, w.rot)
    ctx.incremental_enable(0, 400)
    ctx.incremental_budget(150000, 50, 3000)
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    orc.set_tool(0, w.tool, w.rot)
    inc = IncrementalOracle(orc, 0, len(w.rot), budget=400, lookup_target=150000, b_min=50,
                            b_max=3000)

    def same(where, gst, ost):
        for gk, ok in zip(STAT_KEYS + ("budget",), ORC_KEYS + ("budget",)):
            assert gst[gk] == ost[ok], (where, gk, gst, ost)
        g = ctx.read_incremental()
        keys, lab, best, bdir, a = inc.labels()
        assert np.array_equal(g["key"], keys), where
        assert np.array_equal(g["label"], lab), where
        assert np.array_equal(g["best"].astype(np.int32), best), where
        assert np.array_equal(g["best_dir"].astype(np.int32), bdir), where
        assert np.array_equal(g["a"], a), where

    caps = []
    for j, f in enumerate(frames):
        ctx.incremental_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
        ost = inc.frame(f.xyz, f.origin, f.frame_id)
        gst = ctx.incremental_stats()
        print("frame", j, gst, flush=True)
        same(("frame", j), gst, ost)
        caps.append(gst["budget"])
        if j % 2 == 0 or j == 5:
            m = 300 if j != 5 else 3000
            ctx.incremental_drain(m)
            same(("drain", j), ctx.incremental_stats(), inc.drain(m))
    assert len(set(caps)) > 2


def test_budget_and_drain_argument_errors(synth_mod):
    import torch
    from paper_2608_06412_amd import AFError, Context, default_config
    w = synth_mod.tiny()
    ctx = Context(default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 12,
                                 max_points=1 << 14))
    ctx.set_tool_kernels(0, w.tool, w.rot)
    with pytest.raises(AFError):
        ctx.incremental_budget(1000, 1, 10)          # not enabled
    ctx.incremental_enable(0, 100)
    for bad in ((-1, 1, 10), (1000, 0, 10), (1000, 20, 10), (1 << 41, 1, 10)):
        with pytest.raises(AFError):
            ctx.incremental_budget(*bad)
    ctx.incremental_budget(1000, 10, 500)
    with pytest.raises(AFError):
        ctx.incremental_drain(501)
    with pytest.raises(AFError):
        ctx.incremental_drain(-1)
    ctx.incremental_drain(0)
    f = w.frames(1)[0]
    ctx.incremental_frame(torch.from_numpy(f.xyz).cuda(), f.origin, 0)
    with pytest.raises(AFError):
        ctx.incremental_budget(1000, 10, 500)        # after the first frame


@pytest.mark.parametrize("dirs", ["yaw180", "fib256"])
def test_coarse_to_fine_against_oracle(synth_mod, oracle_mod, dirs):
    """The coarse-to-fine search (20 degree coarse pass, 25 degree fine window,
    0.3 m neighbour radius) on the paper's yaw set and on 256 Fibonacci
    directions, with a cap of 900 and a drain after frame 3: every frame's
    and the drain's counts, every point's state, the canonical test counts,
    and the canonical counts of the restricted evaluations equal the
    oracle's."""
    import torch
    from oracle.incremental import IncrementalOracle
    from paper_2608_06412_amd import Context, default_config
    w = synth_mod.tiny()
    d = synth_mod.yaw_directions(180) if dirs == "yaw180" else synth_mod.fibonacci_directions(256)
    rot = synth_mod.orientations(d, 1)
    frames = w.frames(7)
    ctx = Context(default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 15,
                                 max_points=1 << 17, max_orientations=256))
    ctx.set_tool_kernels(0, w.tool, rot)
    ctx.incremental_enable(0, 900)
    ctx.incremental_c2f(20.0, 25.0, 0.3)
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    orc.set_tool(0, w.tool, rot)
    inc = IncrementalOracle(orc, 0, len(rot), budget=900)
    inc.enable_c2f(rot, 20.0, 25.0, 0.3)
    with_neighbour = 0

    def same(where, gst, ost):
        for gk, ok in zip(STAT_KEYS, ORC_KEYS):
            assert gst[gk] == ost[ok], (where, gk, gst, ost)
        sg, so = ctx.score_stats(0), orc.score_stats()
        for k in ("candidate_tests", "canonical_tests", "canonical_lookups", "n_accessible",
                  "n_blocked", "n_no_candidate"):
            assert sg[k] == so[k], (where, k)
        g = ctx.read_incremental()
        keys, lab, best, bdir, a = inc.labels()
        assert np.array_equal(g["key"], keys), where
        assert np.array_equal(g["label"], lab), where
        assert np.array_equal(g["best"].astype(np.int32), best), where
        assert np.array_equal(g["best_dir"].astype(np.int32), bdir), where
        assert np.array_equal(g["a"], a), where

    for j, f in enumerate(frames):
        ctx.incremental_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
        ost = inc.frame(f.xyz, f.origin, f.frame_id)
        with_neighbour += len(inc.last_neighbour)
        gst = ctx.incremental_stats()
        print("frame", j, gst, "neighbours", len(inc.last_neighbour), flush=True)
        same(("frame", j), gst, ost)
        if j == 3:
            ctx.incremental_drain(900)
            same(("drain", j), ctx.incremental_stats(), inc.drain(900))
    assert with_neighbour > 500


def test_c2f_argument_errors(synth_mod):
    import torch
    from paper_2608_06412_amd import AFError, Context, default_config
    w = synth_mod.tiny()
    ctx = Context(default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 12,
                                 max_points=1 << 14))
    ctx.set_tool_kernels(0, w.tool, w.rot)
    with pytest.raises(AFError):
        ctx.incremental_c2f()                                  # not enabled
    ctx.incremental_enable(0, 100)
    for bad in ((0.0, 25.0, 0.3), (20.0, -1.0, 0.3), (20.0, 25.0, 0.0), (20.0, 25.0, 2.0)):
        with pytest.raises(AFError):
            ctx.incremental_c2f(*bad)                          # 2 m is 100 voxels
    ctx.incremental_c2f(20.0, 25.0, 0.3)
    f = w.frames(1)[0]
    ctx.incremental_frame(torch.from_numpy(f.xyz).cuda(), f.origin, 0)
    with pytest.raises(AFError):
        ctx.incremental_c2f(20.0, 25.0, 0.3)                   # after the first frame
