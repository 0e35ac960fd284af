"""GPU parity at the tree workload's full size (600 frames of 20,000 returns,
1 cm voxels, saw box with a 1 m corridor, K = 256), in the benchmark's launch
configuration (integrate + score every frame, default scoring kernel),
against the oracle's whole-map results stored in tests/golden/tree_full.json
(written by tests/golden/make_tree_golden.py, which calls only the oracle).

After 100, 300 and 600 frames: the whole TSDF (S, W, cleared of every voxel),
every point record, every point's label and first free orientation, every
confident point's normal and candidate mask, the label counts and the
canonical statistics equal the oracle's, compared through SHA-256 digests of
the full arrays, plus 400 seeded points element by element.  The same 600
frames through a recorded frame graph (af_graph_prepare with the scene's box,
af_graph_frame, every frame scored inside the graph) give the same digests
and statistics at each checkpoint."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "tree_full.json")
sys.path.insert(0, os.path.join(HERE, "golden"))


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/tree_full.json not written yet")
    return json.load(open(GOLDEN))


@pytest.fixture(scope="module")
def gpu_states(synth_mod, golden):
    """Run the 600 frames; at each checkpoint collect the library's state."""
    import torch
    from digest import labels_digest, masks_digest, normals_digest, points_digest, tsdf_digest
    from paper_2608_06412_amd import Context, default_config
    assert torch.cuda.is_available()
    w = synth_mod.tree()
    frames = w.frames(600)
    cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 17, max_points=1 << 22,
                         max_orientations=len(w.rot), max_tools=1)
    ctx = Context(cfg)
    ctx.set_tool_kernels(0, w.tool, w.rot)
    want = {cp["frames"]: cp for cp in golden["checkpoints"]}
    out = {}
    for i, f in enumerate(frames):
        ctx.integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
        ctx.score_points(0)
        if i + 1 not in want:
            continue
        print("checkpoint %d: %d points" % (i + 1, ctx.num_points()), flush=True)
        key, S, W, clr = ctx.read_tsdf()
        pts = ctx.read_points()
        lab = ctx.read_labels(0)
        dbg = ctx.read_point_debug(0)
        st = ctx.score_stats(0)
        out[i + 1] = {
            "n_voxels": int(len(key)), "n_points": int(len(pts["key"])),
            "tsdf_sha": tsdf_digest(key, S, W, clr),
            "points_sha": points_digest(pts),
            "labels_sha": labels_digest(lab["key"], lab["label"], lab["first_free"]),
            "normals_sha": normals_digest(lab["label"], dbg["has_normal"], dbg["normal"]),
            "masks_sha": masks_digest(lab["label"], dbg["mask"]),
            "label_counts": {str(k): int((lab["label"] == k).sum()) for k in range(4)},
            "score_stats": st,
            "lab": lab, "dbg": dbg,
        }
    return want, out


CHECKS = ["n_voxels", "n_points", "tsdf_sha", "points_sha", "label_counts", "labels_sha",
          "normals_sha", "masks_sha"]


@pytest.mark.parametrize("frames", [100, 300, 600])
def test_sample_points(gpu_states, frames):
    """The 400 seeded points, element by element (printed first on a digest
    mismatch, since they name the disagreeing points)."""
    want, out = gpu_states
    cp, g = want[frames], out[frames]
    lab, dbg = g["lab"], g["dbg"]
    for smp in cp["sample"]:
        j = smp["i"]
        assert lab["key"][j] == smp["key"], smp
        assert lab["label"][j] == smp["label"], smp
        assert lab["first_free"][j] == smp["first_free"], smp
        if smp["label"] != 0:
            assert dbg["has_normal"][j] == smp["has_normal"], smp
            assert [int(x) for x in dbg["normal"][j]] == smp["normal"], smp
            assert ["%016x" % int(x) for x in dbg["mask"][j]] == smp["mask"], smp


@pytest.mark.parametrize("frames", [100, 300, 600])
@pytest.mark.parametrize("what", CHECKS)
def test_whole_map(gpu_states, frames, what):
    want, out = gpu_states
    assert out[frames][what] == want[frames][what]


@pytest.mark.parametrize("frames", [100, 300, 600])
def test_score_stats(gpu_states, frames):
    want, out = gpu_states
    for k in ("n_points", "n_confident", "n_accessible", "n_blocked", "n_no_candidate",
              "candidate_tests", "canonical_tests", "canonical_lookups"):
        assert out[frames]["score_stats"][k] == want[frames]["score_stats"][k], k


@pytest.fixture(scope="module")
def gpu_states_recorded(synth_mod, golden):
    """The 600 frames as recorded frames; the state at each checkpoint."""
    import torch
    from digest import labels_digest, masks_digest, normals_digest, points_digest, tsdf_digest
    from paper_2608_06412_amd import Context, default_config
    w = synth_mod.tree()
    frames = w.frames(600)
    cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 17, max_points=1 << 22,
                         max_orientations=len(w.rot), max_tools=1)
    ctx = Context(cfg)
    ctx.set_tool_kernels(0, w.tool, w.rot)
    allx = np.concatenate([f.xyz for f in frames])
    ctx.graph_prepare(allx.min(0) - 0.5, allx.max(0) + 0.5, max(len(f.xyz) for f in frames), [0])
    want = {cp["frames"]: cp for cp in golden["checkpoints"]}
    out = {}
    for i, f in enumerate(frames):
        ctx.graph_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
        if i + 1 not in want:
            continue
        ctx.graph_sync()
        print("recorded checkpoint %d: %d points" % (i + 1, ctx.num_points()), flush=True)
        key, S, W, clr = ctx.read_tsdf()
        pts = ctx.read_points()
        lab = ctx.read_labels(0)
        dbg = ctx.read_point_debug(0)
        out[i + 1] = {
            "n_voxels": int(len(key)), "n_points": int(len(pts["key"])),
            "tsdf_sha": tsdf_digest(key, S, W, clr),
            "points_sha": points_digest(pts),
            "labels_sha": labels_digest(lab["key"], lab["label"], lab["first_free"]),
            "normals_sha": normals_digest(lab["label"], dbg["has_normal"], dbg["normal"]),
            "masks_sha": masks_digest(lab["label"], dbg["mask"]),
            "label_counts": {str(k): int((lab["label"] == k).sum()) for k in range(4)},
            "score_stats": ctx.score_stats(0),
        }
    return want, out


@pytest.mark.parametrize("frames", [100, 300, 600])
@pytest.mark.parametrize("what", CHECKS)
def test_recorded_whole_map(gpu_states_recorded, frames, what):
    want, out = gpu_states_recorded
    assert out[frames][what] == want[frames][what]


@pytest.mark.parametrize("frames", [100, 300, 600])
def test_recorded_score_stats(gpu_states_recorded, frames):
    want, out = gpu_states_recorded
    for k in ("n_points", "n_confident", "n_accessible", "n_blocked", "n_no_candidate",
              "candidate_tests", "canonical_tests", "canonical_lookups"):
        assert out[frames]["score_stats"][k] == want[frames]["score_stats"][k], k
