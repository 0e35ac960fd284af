"""GPU parity of the table form of a tool (af_set_tool_table, Section 3.4
"Tool kernel": the rotated tool as voxel offsets built by the caller, here a
pencil-shaped tool sampled as points and voxelised) against the oracle's
table form, on the tiny workload; the primitive builder's own table fed back
through the table form; and the argument checks."""
import numpy as np
import pytest

from tool_tables import table_from_points, table_of_tool

pytestmark = pytest.mark.gpu

SCORE_KEYS = ("n_points", "n_confident", "n_accessible", "n_blocked", "n_no_candidate",
              "candidate_tests", "canonical_tests", "canonical_lookups")


@pytest.fixture(scope="module")
def tiny_pair(synth_mod, oracle_mod):
    import torch
    assert torch.cuda.is_available()
    from paper_2608_06412_amd import Context, default_config
    w = synth_mod.tiny()
    cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 15, max_points=1 << 17,
                         max_orientations=256, max_tools=3)
    ctx = Context(cfg)
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    for f in w.frames():
        ctx.integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
        orc.integrate_frame(f.xyz, f.origin, f.frame_id)
    return w, ctx, orc


def test_primitive_table_through_table_form(tiny_pair):
    """The library's cylinder table read back and passed (shuffled, arm
    samples in their order) to af_set_tool_table: the stored tables are
    equal and scoring gives identical labels, first free orientations and
    statistics."""
    w, ctx, orc = tiny_pair
    K = len(w.rot)
    ctx.set_tool_kernels(0, w.tool, w.rot)
    begin, off, cls = table_of_tool(lambda k: ctx.read_tool_table(0, k), K)
    rng = np.random.default_rng(12)
    perm = []
    for k in range(K):
        seg = begin[k] + rng.permutation(int(begin[k + 1] - begin[k]))
        nm = cls[seg] == 1
        seg[nm] = np.sort(seg[nm])
        perm.append(seg)
    perm = np.concatenate(perm)
    dirs = np.asarray(w.rot).reshape(-1, 3, 3)[:, :, 0]
    ctx.set_tool_table(1, dirs, begin, off[perm], cls[perm])
    for k in range(K):
        a, b = ctx.read_tool_table(0, k), ctx.read_tool_table(1, k)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), k
    ctx.score_points(0)
    ctx.score_points(1)
    la, lb = ctx.read_labels(0), ctx.read_labels(1)
    assert np.array_equal(la["label"], lb["label"])
    assert np.array_equal(la["first_free"], lb["first_free"])
    sa, sb = ctx.score_stats(0), ctx.score_stats(1)
    for k in SCORE_KEYS:
        assert sa[k] == sb[k], k


def test_pencil_table_matches_oracle(tiny_pair, synth_mod):
    """A pencil tool (cone tip, shaft, 40 cm corridor) as a caller table:
    stored table, normals, candidate masks, labels, first free orientations
    and canonical counts equal the oracle's bit for bit."""
    w, ctx, orc = tiny_pair
    K = len(w.rot)
    body, far = synth_mod.pencil_points()
    dirs, begin, off, cls = table_from_points(body, far, w.rot, w.voxel, w.trunc, 0.03,
                                              shuffle_seed=5)
    ctx.set_tool_table(2, dirs, begin, off, cls)
    orc.set_tool_table(2, dirs, begin, off, cls)
    for k in range(0, K, 7):
        a, b = ctx.read_tool_table(2, k), orc.tool_table(2, k)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), k
    ctx.score_points(2)
    orc.score(2)
    lab = ctx.read_labels(2)
    keys, ol, off_ = orc.labels(K, lab["key"])
    assert np.array_equal(lab["label"], ol)
    assert np.array_equal(lab["first_free"], off_)
    dbg = ctx.read_point_debug(2)
    for i in range(0, len(keys), 5):
        r = orc.point_result(int(keys[i]), K)
        assert dbg["has_normal"][i] == (r["has_normal"] if r["label"] != 0 else -1)
        if r["label"] != 0:
            assert np.array_equal(dbg["normal"][i].astype(np.int64), r["normal"])
            assert np.array_equal(dbg["mask"][i], r["mask"])
    sg, so = ctx.score_stats(2), orc.score_stats()
    for k in SCORE_KEYS:
        assert sg[k] == so[k], k
    assert (ol == 1).sum() > 100 and (ol == 2).sum() > 10


@pytest.mark.parametrize("case", ["class", "near2", "near4", "dup", "range", "dir", "begin"])
def test_table_rejections(tiny_pair, case):
    """Invalid tables are refused with AF_EINVAL and leave the tool as it was."""
    from paper_2608_06412_amd.af import AF_EINVAL, AFError
    w, ctx, orc = tiny_pair
    dirs = np.array([[1.0, 0.0, 0.0]])
    off = np.array([[1, 0, 0], [2, 0, 0], [3, 0, 0], [2, 1, 0], [3, 1, 0]], np.int16)
    cls = np.array([1, 1, 1, 0, 2], np.uint8)
    begin = np.array([0, 5], np.uint32)
    ctx.set_tool_table(1, dirs, begin, off, cls)
    if case == "class":
        cls = cls.copy(); cls[3] = 3
    elif case == "near2":
        cls = cls.copy(); cls[2] = 0
    elif case == "near4":
        cls = cls.copy(); cls[3] = 1
    elif case == "dup":
        off = np.vstack([off, off[3:4]]); cls = np.append(cls, 0)
        begin = np.array([0, 6], np.uint32)
    elif case == "range":
        off = off.copy(); off[4, 2] = 512
    elif case == "dir":
        dirs = np.array([[1.0, 1e-4, 0.0]])
    elif case == "begin":
        begin = np.array([1, 5], np.uint32)
    with pytest.raises(AFError) as ei:
        ctx.set_tool_table(1, dirs, begin, off, cls)
    assert ei.value.code == AF_EINVAL
    o, c = ctx.read_tool_table(1, 0)
    assert len(o) == 5 and list(c) == [1, 1, 1, 0, 2]
