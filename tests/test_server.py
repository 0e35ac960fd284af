"""Serving two concurrent sensor streams (af_server): each stream's labels,
first free orientations, statistics and TSDF after every frame equal those of
its own eager context fed the same frames (af_integrate_frame +
af_score_points), whatever the interleaving of submissions, and after frames
5, 12 and 20 of each stream its labels, first free orientations and
canonical counts equal the oracle's fed the same frames; admission
follows the device budget; a full frame queue is refused.  Stream 0: the tiny
scene with a cylinder; stream 1: a seeded box cluster with a box tool and
frames of 500-3,000 returns (v = 2 cm both).  Both modes: one scoring launch
per step across the streams (batched), and one per stream."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _streams(synth_mod):
    from paper_2608_06412_amd import default_config
    w = synth_mod.tiny()
    f0 = w.frames()
    scene = synth_mod.box_cluster_scene(seed=11, n_boxes=6, extent=1.5)
    counts = synth_mod.uneven_counts(20, lo=500, hi=3000, seed=4)
    f1 = synth_mod.make_frames(scene, synth_mod.circle_poses(20, radius=3.0, centre=(0.0, 0.0)),
                               counts, 0.01, 2, -52.0, 7.0)
    tools = [synth_mod.cylinder_tool(), synth_mod.batch_tools()[1]]
    rots = [synth_mod.orientations(synth_mod.fibonacci_directions(64), 1),
            synth_mod.orientations(synth_mod.fibonacci_directions(64), 2)]

    def cfg(budget):
        c = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 15, max_points=1 << 17,
                           max_orientations=128, max_tools=1)
        c.hbm_budget = int(budget)
        return c
    return [f0, f1], tools, rots, cfg


def _same(a, b, where):
    la, lb = a.read_labels(0), b.read_labels(0)
    assert np.array_equal(la["key"], lb["key"]), where
    assert np.array_equal(la["label"], lb["label"]), where
    assert np.array_equal(la["first_free"], lb["first_free"]), where
    sa, sb = a.score_stats(0), b.score_stats(0)
    for k in ("n_confident", "n_accessible", "n_blocked", "canonical_tests",
              "canonical_lookups"):
        assert sa[k] == sb[k], (where, k)


def _same_as_oracle(ctx, orc, K, where):
    orc.score(0)
    lab = ctx.read_labels(0)
    r = orc.read_results(K)
    assert np.array_equal(lab["key"], orc.read_points()["key"]), where
    assert np.array_equal(lab["label"], r["label"]), where
    assert np.array_equal(lab["first_free"].astype(np.int64), r["first_free"]), where
    sg, so = ctx.score_stats(0), orc.score_stats()
    for k in ("n_confident", "n_accessible", "n_blocked", "n_no_candidate", "canonical_tests",
              "canonical_lookups"):
        assert sg[k] == so[k], (where, k)


# True: one scoring launch for every step of two streams; 3: batched graphs
# with a threshold above two streams, so each is scored on its own stream
# after its unscored graph; None (the default) and False: each graph holds
# its own scoring launch
@pytest.mark.parametrize("batch", [True, 3, None, False])
def test_two_streams_equal_their_eager_contexts(synth_mod, oracle_mod, batch):
    import torch
    from paper_2608_06412_amd import AFError, Context, Server
    from paper_2608_06412_amd.af import AF_EBUSY, AF_ENOMEM
    frames, tools, rots, cfg = _streams(synth_mod)
    GiB = 1 << 30
    srv = Server(3 * GiB, max_streams=3, batch=batch)
    sids = [srv.admit(cfg(GiB)), srv.admit(cfg(GiB))]
    with pytest.raises(AFError) as e:
        srv.admit(cfg(2 * GiB))
    assert e.value.code == AF_ENOMEM
    refs = []
    for s, sid in enumerate(sids):
        srv.context(sid).set_tool_kernels(0, tools[s], rots[s])
        allx = np.concatenate([f.xyz for f in frames[s]])
        srv.prepare(sid, allx.min(0) - 0.5, allx.max(0) + 0.5,
                    max(len(f.xyz) for f in frames[s]), [0])
        r = Context(cfg(0))
        r.set_tool_kernels(0, tools[s], rots[s])
        refs.append(r)
    orcs = []
    w0 = synth_mod.tiny()     # both streams use its voxel, truncation and r_c
    for s in range(2):
        o = oracle_mod.Oracle(voxel=w0.voxel, trunc=w0.trunc, r_c=w0.r_c)
        o.set_tool(0, tools[s], rots[s])
        orcs.append(o)
    nxt = [0, 0]     # next frame to submit, per stream
    done = [0, 0]    # frames processed, per stream
    it = 0
    while min(done[s] - len(frames[s]) for s in range(2)) < 0 or any(
            srv.pending(sid) for sid in sids):
        # uneven arrivals: stream 0 every iteration (two frames every third),
        # stream 1 every other iteration
        plan = [2 if it % 3 == 0 else 1, 1 if it % 2 == 0 else 0]
        for s, sid in enumerate(sids):
            for _ in range(plan[s]):
                if nxt[s] < len(frames[s]) and srv.pending(sid) < 4:
                    f = frames[s][nxt[s]]
                    srv.submit(sid, f.xyz, f.origin, f.frame_id)
                    nxt[s] += 1
        out = srv.step()
        print("step", it, out, flush=True)
        for sid, fid, st in out:
            assert st == 0, (sid, fid, srv.last_error())
            s = sids.index(sid)
            f = frames[s][done[s]]
            assert fid == f.frame_id
            refs[s].integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
            refs[s].score_points(0)
            _same(srv.context(sid), refs[s], (s, fid))
            orcs[s].integrate_frame(f.xyz, f.origin, f.frame_id)
            if done[s] in (4, 11, len(frames[s]) - 1):
                _same_as_oracle(srv.context(sid), orcs[s], len(rots[s]), (s, fid))
            done[s] += 1
        it += 1
        assert it < 200
    for s, sid in enumerate(sids):
        for x, y in zip(srv.context(sid).read_tsdf(), refs[s].read_tsdf()):
            assert np.array_equal(x, y)
    # a full queue is refused; the queued frames still run in order
    sid = sids[0]
    extra = synth_mod.tiny(seed=3).frames()
    for j in range(4):
        srv.submit(sid, extra[j].xyz, extra[j].origin, 100 + j)
    with pytest.raises(AFError) as e:
        srv.submit(sid, extra[4].xyz, extra[4].origin, 104)
    assert e.value.code == AF_EBUSY
    got = []
    while srv.pending(sid):
        got += [fid for _, fid, st in srv.step() if st == 0]
    assert got == [100, 101, 102, 103]
    # releasing a stream returns its reservation
    srv.release(sids[1])
    assert srv.reserved() == GiB
    third = srv.admit(cfg(2 * GiB))
    assert srv.reserved() == 3 * GiB
    srv.release(third)
    srv.close()
