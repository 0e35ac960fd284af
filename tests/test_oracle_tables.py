"""The oracle's table form of a tool (Section 3.4 "Tool kernel": the tool as
voxel offsets, supplied by the caller) against its primitive builder, a
brute-force evaluation, and its argument checks."""
import math

import numpy as np
import pytest

from tool_tables import table_from_points, table_of_tool


def _tiny_oracle(oracle_mod, synth_mod, n_frames=8):
    w = synth_mod.tiny(n_frames=n_frames)
    o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    for f in w.frames():
        o.integrate_frame(f.xyz, f.origin, f.frame_id)
    return w, o


def _results(o, K):
    keys = o.read_points()["key"]
    out = [o.point_result(int(k), K) for k in keys]
    return (np.array([r["label"] for r in out]), np.array([r["first_free"] for r in out]),
            np.array([r["mask"] for r in out]), o.score_stats())


def test_primitive_table_round_trip(oracle_mod, synth_mod):
    """The primitive builder's own table, fed back as a caller table (entries
    shuffled), scores identically: labels, first free orientations, masks
    and every canonical count."""
    w, o = _tiny_oracle(oracle_mod, synth_mod)
    K = len(w.rot)
    o.set_tool(0, w.tool, w.rot)
    o.score(0)
    a = _results(o, K)
    begin, off, cls = table_of_tool(lambda k: o.tool_table(0, k), K)
    rng = np.random.default_rng(4)
    perm = np.concatenate([begin[k] + rng.permutation(begin[k + 1] - begin[k])
                           for k in range(K)]).astype(np.int64)
    # the NEAR entries keep their order (they are visited in the given order)
    near = cls == 1
    for k in range(K):
        seg = perm[begin[k]:begin[k + 1]]
        nidx = np.sort(seg[near[seg]])
        seg[near[seg]] = nidx
    dirs = np.asarray(w.rot).reshape(-1, 3, 3)[:, :, 0]
    o.set_tool_table(1, dirs, begin, off[perm], cls[perm])
    for k in range(K):
        ta, tb = o.tool_table(0, k), o.tool_table(1, k)
        assert np.array_equal(ta[0], tb[0]) and np.array_equal(ta[1], tb[1])
    o.score(1)
    b = _results(o, K)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert a[3] == b[3]
    assert (a[0] == 1).sum() > 100 and (a[0] == 2).sum() > 10


def _brute_free(o, key, s, off, cls, rc_u, n_c):
    body = 0
    for (dx, dy, dz), c in zip(off, cls):
        S, W, clr = o.voxel(key(s[0] + dx, s[1] + dy, s[2] + dz))
        occ = W > 0 and S < rc_u * W
        if c == 1 and (occ or (W == 0 and not clr)):
            return False
        if c == 0 and occ:
            body += 1
            if body >= n_c:
                return False
        if c == 2 and occ:
            return False
    return True


def test_pencil_table_brute_force(oracle_mod, synth_mod):
    """A pencil tool (cone tip, shaft, corridor) sampled as points and
    voxelised by the caller: for 60 points the oracle's label and first
    free orientation equal a direct evaluation of the table entries against
    the oracle's voxels (candidate masks taken from the oracle)."""
    w, o = _tiny_oracle(oracle_mod, synth_mod)
    K = len(w.rot)
    body, far = synth_mod.pencil_points()
    dirs, begin, off, cls = table_from_points(body, far, w.rot, w.voxel, w.trunc, 0.03,
                                              shuffle_seed=3)
    o.set_tool_table(0, dirs, begin, off, cls)
    o.score(0)
    prm = o.params()
    keys = o.read_points()["key"]
    rng = np.random.default_rng(9)
    seen = {1: 0, 2: 0}
    for k in rng.choice(keys, size=60, replace=False):
        r = o.point_result(int(k), K)
        if r["label"] in (0, 3):
            continue
        s = oracle_mod.unkey(int(k))
        ff = -1
        for j in range(K):
            if not (int(r["mask"][j // 64]) >> (j % 64)) & 1:
                continue
            if _brute_free(o, oracle_mod.key, s, off[begin[j]:begin[j + 1]],
                           cls[begin[j]:begin[j + 1]], prm["rc_u"], 5):
                ff = j
                break
        assert r["first_free"] == ff
        assert r["label"] == (1 if ff >= 0 else 2)
        seen[r["label"]] += 1
    assert seen[1] > 5


@pytest.mark.parametrize("case", ["class", "near2", "near4", "dup", "range", "dir", "begin"])
def test_table_rejections(oracle_mod, synth_mod, case):
    w = synth_mod.tiny(n_frames=1)
    o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    dirs = np.array([[1.0, 0.0, 0.0]])
    off = np.array([[1, 0, 0], [2, 0, 0], [3, 0, 0], [2, 1, 0], [3, 1, 0]], np.int16)
    cls = np.array([1, 1, 1, 0, 2], np.uint8)
    begin = np.array([0, 5], np.uint32)
    o.set_tool_table(0, dirs, begin, off, cls)          # valid
    if case == "class":
        cls = cls.copy(); cls[3] = 3
    elif case == "near2":
        cls = cls.copy(); cls[2] = 0
    elif case == "near4":
        cls = cls.copy(); cls[3] = 1
    elif case == "dup":
        off = np.vstack([off, off[3:4]]); cls = np.append(cls, 0); begin = np.array([0, 6], np.uint32)
    elif case == "range":
        off = off.copy(); off[4, 2] = 512
    elif case == "dir":
        dirs = np.array([[1.0, 1e-4, 0.0]])
    elif case == "begin":
        begin = np.array([1, 5], np.uint32)
    with pytest.raises(ValueError):
        o.set_tool_table(0, dirs, begin, off, cls)
    # the earlier valid table is still in place
    oo, cc = o.tool_table(0, 0)
    assert len(oo) == 5 and list(cc) == [1, 1, 1, 0, 2]
