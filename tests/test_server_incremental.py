"""Serving streams in the incremental mode (Section 3.5) beside a stateless
stream (af_server): after every step, each incremental stream's labels,
stored scores and directions, a and trigger / backlog counts equal those of
its own eager incremental context fed the same frames; the first stream also
equals the oracle's state machine after every step.  Stream 0: the tiny scene
with a budget below its queue (the backlog carries across steps); stream 1:
the sliding-window walk with a window of 20^3 blocks and the coarse-to-fine
search; stream 2: the tiny scene without the incremental mode.  Both server
modes (batched and never batched)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

STAT_KEYS = ("new_points", "trig_i", "trig_ii", "trig_iii", "sampled", "evaluated", "backlog")
ORC_KEYS = ("new", "trig_i", "trig_ii", "trig_iii", "sampled", "evaluated", "backlog")


def _same_state(a, b, where):
    sa, sb = a.incremental_stats(), b.incremental_stats()
    for k in STAT_KEYS:
        assert sa[k] == sb[k], (where, k, sa, sb)
    ga, gb = a.read_incremental(), b.read_incremental()
    for k in ("key", "label", "best", "best_dir", "a"):
        assert np.array_equal(ga[k], gb[k]), (where, k)


@pytest.mark.parametrize("batch", [True, False])
def test_incremental_streams(synth_mod, oracle_mod, batch):
    import torch
    from oracle.incremental import IncrementalOracle
    from paper_2608_06412_amd import AFError, Context, Server, default_config
    tiny = synth_mod.tiny()
    walk = synth_mod.window_walk()
    feeds = [tiny.frames(12), walk.frames(12), tiny.frames(12)]
    GiB = 1 << 30
    srv = Server(4 * GiB, max_streams=3, batch=batch)

    def cfg(w, blocks):
        c = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=blocks, max_points=1 << 17,
                           max_orientations=64, max_tools=1)
        c.hbm_budget = GiB
        return c
    specs = [(tiny, 1 << 15, None, 700, False), (walk, 20 ** 3, [20] * 3, 900, True),
             (tiny, 1 << 15, None, 0, False)]
    sids, refs = [], []
    for w, blocks, win, budget, c2f in specs:
        sid = srv.admit(cfg(w, blocks))
        ctx = srv.context(sid)
        ref = Context(cfg(w, blocks)) if budget else None
        for c in (ctx, ref):
            if c is None:
                continue
            if win:
                c.set_window(win)
            c.set_tool_kernels(0, w.tool, w.rot)
            if budget:
                c.incremental_enable(0, budget)
                if c2f:
                    c.incremental_c2f()
        allx = np.concatenate([f.xyz for f in feeds[len(sids)]])
        srv.prepare(sid, allx.min(0) - 0.5, allx.max(0) + 0.5,
                    max(len(f.xyz) for f in feeds[len(sids)]), [0])
        sids.append(sid)
        refs.append(ref)
    # a recorded graph cannot take a context already in the incremental mode,
    # nor the incremental mode a context with a graph
    with pytest.raises(AFError):
        srv.context(sids[0]).graph_prepare([-1, -1, -1], [1, 1, 1], 100, [0])
    with pytest.raises(AFError):
        srv.context(sids[2]).incremental_enable(0, 100)
    orc = oracle_mod.Oracle(voxel=tiny.voxel, trunc=tiny.trunc, r_c=tiny.r_c)
    orc.set_tool(0, tiny.tool, tiny.rot)
    inc = IncrementalOracle(orc, 0, len(tiny.rot), budget=700)
    plain = Context(cfg(tiny, 1 << 15))
    plain.set_tool_kernels(0, tiny.tool, tiny.rot)
    for step in range(12):
        print("served incremental step", step, "batch", batch, flush=True)
        for s, sid in enumerate(sids):
            f = feeds[s][step]
            srv.submit(sid, f.xyz, f.origin, f.frame_id)
            x = torch.from_numpy(np.ascontiguousarray(f.xyz)).cuda()
            if refs[s] is not None:
                refs[s].incremental_frame(x, f.origin, f.frame_id)
            else:
                plain.integrate_frame(x, f.origin, f.frame_id)
                plain.score_points(0)
        ost = inc.frame(feeds[0][step].xyz, feeds[0][step].origin, feeds[0][step].frame_id)
        done = srv.step()
        assert sorted(d[0] for d in done) == sorted(sids) and all(d[2] == 0 for d in done), done
        for s in (0, 1):
            _same_state(srv.context(sids[s]), refs[s], (step, s))
        g = srv.context(sids[0]).read_incremental()
        keys, lab, best, bdir, a = inc.labels()
        assert np.array_equal(g["key"], keys) and np.array_equal(g["label"], lab), step
        assert np.array_equal(g["best"].astype(np.int32), best), step
        assert np.array_equal(g["best_dir"].astype(np.int32), bdir), step
        assert np.array_equal(g["a"], a), step
        gst = srv.context(sids[0]).incremental_stats()
        for gk, ok in zip(STAT_KEYS, ORC_KEYS):
            assert gst[gk] == ost[ok], (step, gk)
        la, lb = srv.context(sids[2]).read_labels(0), plain.read_labels(0)
        assert np.array_equal(la["label"], lb["label"]), step
        assert np.array_equal(la["first_free"], lb["first_free"]), step
    assert ost["backlog"] > 0
    assert srv.context(sids[1]).window_state()[2] >= 1
