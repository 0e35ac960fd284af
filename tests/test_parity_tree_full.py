"""GPU checks at the full size of the tree workload, in the configuration the
benchmark times: 600 frames of 20,000 returns, 1 cm voxels, 4 cm truncation,
saw box with a 1 m corridor at K = 256, the benchmark's capacities, the
library's default scoring configuration, scoring after every frame.

* Against the oracle, on sampled outputs it computes one region at a time:
  in four 17^3-voxel regions around seeded returns of the last frames, every
  voxel (S, W, cleared) and every point record (key, first frame, viewpoints,
  sensor sums) after frame 599, bit for bit.
* Properties that hold at any size, on the whole final map: weights within
  the cap, labels in range, first free orientation set exactly for accessible
  points and its candidate bit set; the normals and labels of the context
  that scored every frame (cached normal axes) equal those of a context that
  scored once at the end; the plainest scoring configuration gives the
  default configuration's labels, first free orientations and canonical
  counts."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_FRAMES = 600
REGION = 8          # half-width of each oracle region, voxels


@pytest.fixture(scope="module")
def full_run(synth_mod, oracle_mod):
    import torch
    assert torch.cuda.is_available()
    from paper_2608_06412_amd import Context, default_config
    w = synth_mod.tree(n_frames=N_FRAMES)
    frames = w.frames(N_FRAMES)
    print("generated %d frames" % N_FRAMES, flush=True)

    def make():
        cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 17,
                             max_points=1 << 22, max_orientations=len(w.rot), max_tools=1)
        c = Context(cfg)
        c.set_tool_kernels(0, w.tool, w.rot)
        return c

    ctx = make()
    assert ctx.score_variant() == ctx.score_variant_default()
    for f in frames:
        ctx.integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
        ctx.score_points(0)
        if f.frame_id % 100 == 99:
            print("scored frame %d, %d points" % (f.frame_id, ctx.num_points()), flush=True)
    once = make()
    for f in frames:
        once.integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
    once.score_points(0)
    print("second context scored once", flush=True)

    rng = np.random.default_rng(599)
    centres = [np.floor(frames[-1 - j].xyz[rng.integers(len(frames[-1 - j].xyz))]
                        .astype(np.float64) / w.voxel).astype(np.int64) for j in range(4)]
    orcs = []
    for c in centres:
        o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
        o.set_roi(c - REGION, c + REGION)
        orcs.append(o)
    for f in frames:
        for o in orcs:
            o.integrate_frame(f.xyz, f.origin, f.frame_id)
    print("oracle regions integrated", flush=True)
    return w, ctx, once, centres, orcs


def test_regions_bit_exact(full_run, oracle_mod):
    w, ctx, _, centres, orcs = full_run
    gk, gS, gW, gc = ctx.read_tsdf()
    gijk = oracle_mod.unpack_keys(gk)
    pts = ctx.read_points()
    pijk = oracle_mod.unpack_keys(pts["key"])
    wmax = 0
    for c, o in zip(centres, orcs):
        lo, hi = c - REGION, c + REGION
        inside = np.all((gijk >= lo) & (gijk <= hi), axis=1)
        ok, oS, oW, oc = o.read_tsdf()
        g = {int(k): (int(s), int(ww), int(cc)) for k, s, ww, cc in
             zip(gk[inside], gS[inside], gW[inside], gc[inside])}
        want = {int(k): (int(s), int(ww), int(cc)) for k, s, ww, cc in zip(ok, oS, oW, oc)}
        assert len(want) > 100 and g == want, c
        wmax = max(wmax, int(oW.max()))
        op = o.read_points()
        pin = np.all((pijk >= lo) & (pijk <= hi), axis=1)
        assert len(op["key"]) > 10 and np.array_equal(pts["key"][pin], op["key"])
        for name in ("first_frame", "n_vp", "vp", "sumq", "nq"):
            assert np.array_equal(pts[name][pin], op[name]), (c, name)
    print("largest weight in the regions", wmax, flush=True)


def test_whole_map_properties(full_run):
    w, ctx, _, _, _ = full_run
    gk, gS, gW, gc = ctx.read_tsdf()
    assert gW.max() <= 2000 and gS.min() >= 0
    lab = ctx.read_labels(0, with_w=True)
    assert set(np.unique(lab["label"])) <= {0, 1, 2, 3}
    acc = lab["label"] == 1
    assert acc.sum() > 100000
    assert np.all(lab["first_free"][acc] >= 0) and np.all(lab["first_free"][~acc] == -1)
    assert np.all((lab["w"] >= 2) == (lab["label"] != 0))
    dbg = ctx.read_point_debug(0)
    ff = lab["first_free"][acc].astype(np.int64)
    words = dbg["mask"][acc][np.arange(acc.sum()), ff // 64]
    assert np.all((words >> (ff % 64).astype(np.uint64)) & np.uint64(1) == 1)


def test_cached_normals_equal_fresh(full_run):
    _, ctx, once, _, _ = full_run
    ctx.score_points(0)
    a, b = ctx.read_point_debug(0), once.read_point_debug(0)
    assert np.array_equal(a["has_normal"], b["has_normal"])
    assert np.array_equal(a["normal"], b["normal"])
    la, lb = ctx.read_labels(0), once.read_labels(0)
    assert np.array_equal(la["key"], lb["key"])
    assert np.array_equal(la["label"], lb["label"])
    assert np.array_equal(la["first_free"], lb["first_free"])


def test_plain_configuration_agrees(full_run):
    _, ctx, _, _, _ = full_run
    keys = ("n_confident", "n_accessible", "n_blocked", "n_no_candidate", "candidate_tests",
            "canonical_tests", "canonical_lookups")
    ctx.score_points(0)
    ref = ctx.read_labels(0)
    st = ctx.score_stats(0)
    names = ctx.score_variants()
    default = ctx.score_variant()
    plain = names.index("plain wg256")
    try:
        ctx.set_score_variant(plain)
        ctx.score_points(0)
        got = ctx.read_labels(0)
        gst = ctx.score_stats(0)
    finally:
        ctx.set_score_variant(default)
    assert np.array_equal(got["label"], ref["label"])
    assert np.array_equal(got["first_free"], ref["first_free"])
    assert {k: gst[k] for k in keys} == {k: st[k] for k in keys}
