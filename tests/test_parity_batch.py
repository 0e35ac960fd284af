"""Batching: several tools scored in one persistent launch (af_score_tools)
give, per tool, exactly the labels, first free orientations and statistics
of separate per-tool launches (af_score_points); a 512-orientation table
(128 directions x 4 rolls) matches the oracle bit for bit.  Tiny scene
(v = 2 cm), four of the batching workload's tools."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

STAT_KEYS = ("n_points", "n_confident", "n_accessible", "n_blocked", "n_no_candidate",
             "candidate_tests", "canonical_tests", "canonical_lookups")


@pytest.fixture(scope="module")
def batch_run(synth_mod, oracle_mod):
    import torch
    assert torch.cuda.is_available()
    from paper_2608_06412_amd import Context, default_config
    w = synth_mod.tiny()
    frames = w.frames()
    tools = synth_mod.batch_tools()[:4]
    rots = [synth_mod.orientations(synth_mod.fibonacci_directions(128), 4),
            synth_mod.orientations(synth_mod.fibonacci_directions(64), 1),
            synth_mod.orientations(synth_mod.yaw_directions(70), 1),
            synth_mod.orientations(synth_mod.fibonacci_directions(32), 8)]
    cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 15, max_points=1 << 17,
                         max_orientations=512, max_tools=4)
    ctx = Context(cfg)
    for i, (tl, r) in enumerate(zip(tools, rots)):
        ctx.set_tool_kernels(i, tl, r)
    for f in frames:
        ctx.integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
    ctx.score_tools([0, 1, 2, 3])
    multi = [(ctx.read_labels(i), ctx.score_stats(i)) for i in range(4)]
    single = []
    for i in range(4):
        ctx.score_points(i)
        single.append((ctx.read_labels(i), ctx.score_stats(i)))
    print("points", ctx.num_points(), "K", [len(r) for r in rots], flush=True)
    return w, frames, ctx, tools, rots, multi, single


def test_multi_equals_single(batch_run):
    w, frames, ctx, tools, rots, multi, single = batch_run
    for i in range(4):
        (lm, sm), (ls, ss) = multi[i], single[i]
        assert np.array_equal(lm["key"], ls["key"])
        assert np.array_equal(lm["label"], ls["label"]), i
        assert np.array_equal(lm["first_free"], ls["first_free"]), i
        for k in STAT_KEYS + ("arm_lookups",):
            assert sm[k] == ss[k], (i, k)
        assert sm["canonical_tests"] > 0


def test_k512_against_oracle(batch_run, oracle_mod):
    w, frames, ctx, tools, rots, multi, single = batch_run
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    for f in frames:
        orc.integrate_frame(f.xyz, f.origin, f.frame_id)
    orc.set_tool(0, tools[0], rots[0])
    orc.score(0)
    keys, lbl, ff = orc.labels(len(rots[0]))
    lab = multi[0][0]
    assert np.array_equal(lab["key"], keys)
    assert np.array_equal(lab["label"], lbl)
    assert np.array_equal(lab["first_free"].astype(np.int64), ff.astype(np.int64))
    st = orc.score_stats()
    for k in ("n_confident", "n_accessible", "n_blocked", "canonical_tests",
              "canonical_lookups"):
        assert multi[0][1][k] == st[k], k


def test_subset_in_other_order(batch_run):
    w, frames, ctx, tools, rots, multi, single = batch_run
    ctx.score_tools([2, 0])
    for i in (2, 0):
        lab = ctx.read_labels(i)
        assert np.array_equal(lab["label"], single[i][0]["label"])
        assert np.array_equal(lab["first_free"], single[i][0]["first_free"])
        assert ctx.score_stats(i)["canonical_lookups"] == single[i][1]["canonical_lookups"]


def test_argument_errors(batch_run):
    from paper_2608_06412_amd import AFError
    w, frames, ctx, tools, rots, multi, single = batch_run
    for bad in ([], [0, 0], [0, 7], list(range(9))):
        with pytest.raises(AFError):
            ctx.score_tools(bad)
