"""Oracle sliding window (Section 3.3), pinned by other formulations:

* a window wider than the whole scene and sensor path never shifts and
  gives exactly the unbounded map, points, statistics and labels;
* the shift schedule on a straight sensor path, worked out by hand (the
  30 % rule, the re-centring, floor division on negative coordinates);
* every voxel of the windowed map equals a fresh, unbounded integration of
  the frames since that voxel was last outside the window, and nothing else
  is in the map;
* point records (first frame, frames seen, summed sensor position) equal a
  brute-force count of the returns that landed in their voxel while it was
  inside the window;
* in-window normals equal the PCA axis of the brute-force nearest points
  inside the window;
* points outside the window keep the label of their last scoring inside
  it, and read 255 if they never had one.
"""
import numpy as np
import pytest

BLOCKS = 20   # 3.2 m at v = 2 cm


@pytest.fixture(scope="module")
def walk(synth_mod):
    w = synth_mod.window_walk()
    return w, w.frames()


@pytest.fixture(scope="module")
def windowed(walk, oracle_mod):
    """The windowed oracle run, scored after every frame, with the window box
    of each frame and the labels of each scoring."""
    w, frames = walk
    o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    o.set_window([BLOCKS] * 3)
    o.set_tool(0, w.tool, w.rot)
    boxes, scored = [], []
    for f in frames:
        o.integrate_frame(f.xyz, f.origin, f.frame_id)
        lo, hi, _ = o.window()
        boxes.append((lo.copy(), hi.copy()))
        if f.frame_id % 3 == 2 or f.frame_id == len(frames) - 1:
            o.score(0)
            r = o.read_results(len(w.rot))
            scored.append((f.frame_id, o.read_points()["key"].copy(), r["label"].copy(),
                           r["first_free"].copy(), lo.copy(), hi.copy()))
    return o, boxes, scored


def _blocks_of(keys, oracle_mod):
    v = np.array([oracle_mod.unkey(int(k)) for k in keys], np.int64).reshape(-1, 3)
    return np.floor_divide(v, 8)


def _inside(blk, lo, hi):
    return np.all((blk >= lo) & (blk <= hi), axis=1)


def test_window_wider_than_everything_is_no_window(synth_mod, oracle_mod):
    w = synth_mod.tiny()
    frames = w.frames()
    a = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    b = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    b.set_window([4096, 4096, 4096])
    for o in (a, b):
        o.set_tool(0, w.tool, w.rot)
    for f in frames:
        a.integrate_frame(f.xyz, f.origin, f.frame_id)
        b.integrate_frame(f.xyz, f.origin, f.frame_id)
        assert a.frame_stats() == b.frame_stats()
    assert b.window()[2] == 0
    for x, y in zip(a.read_tsdf(), b.read_tsdf()):
        assert np.array_equal(x, y)
    pa, pb = a.read_points(), b.read_points()
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    a.score(0)
    b.score(0)
    ra, rb = a.read_results(len(w.rot)), b.read_results(len(w.rot))
    for k in ra:
        assert np.array_equal(ra[k], rb[k]), k
    assert a.score_stats() == b.score_stats()


def test_shift_schedule_on_a_straight_path(oracle_mod):
    # 10 blocks = 80 voxels: the window moves when the sensor is more than
    # 24 voxels from its centre.  The sensor walks +5 voxels per frame along
    # x and -5 along z (voxel centres, no returns), so the window re-centres
    # at frames 5, 10, 15 (offset 25 each time).
    v = 0.02
    o = oracle_mod.Oracle(voxel=v, trunc=0.06, r_c=0.01)
    o.set_window([10, 10, 10])
    assert o.window() is None
    empty = np.zeros((0, 3), np.float32)
    seen = []
    for j in range(16):
        q = np.array([(5 * j + 0.5) * v, 0.5 * v, (-5 * j + 0.5) * v], np.float32)
        o.integrate_frame(empty, q, j)
        lo, hi, shifts = o.window()
        seen.append((lo.tolist(), hi.tolist(), shifts))
    # centre c -> blocks floor(c / 8) - 5 .. + 9
    def box(cx, cz):
        return [cx // 8 - 5, -5, cz // 8 - 5], [cx // 8 + 4, 4, cz // 8 + 4]
    expect = []
    for j in range(16):
        k = j // 5
        lo, hi = box(25 * k, -25 * k)
        expect.append((lo, hi, k))
    assert seen == expect
    assert seen[5][0] == [-2, -5, -9]      # floor(-25 / 8) = -4


def test_set_window_rules(oracle_mod, synth_mod):
    o = oracle_mod.Oracle(voxel=0.02, trunc=0.06, r_c=0.01)
    with pytest.raises(ValueError):
        o.set_window([1, 4, 4])
    w = synth_mod.tiny()
    f = w.frames(1)[0]
    o.integrate_frame(f.xyz, f.origin, 0)
    with pytest.raises(ValueError):
        o.set_window([8, 8, 8])


def test_voxels_equal_fresh_integration_since_last_outside(walk, windowed, oracle_mod):
    w, frames = walk
    o, boxes, _ = windowed
    assert o.window()[2] >= 5                       # the walk shifts several times
    key, S, W, clr = o.read_tsdf()
    blk = _blocks_of(key, oracle_mod)
    lo_f, hi_f = boxes[-1]
    assert _inside(blk, lo_f, hi_f).all()           # nothing outside the final window
    # e(x): the last frame whose window did not hold x (-1: none)
    def last_outside(b):
        e = np.full(len(b), -1, np.int64)
        for j, (lo, hi) in enumerate(boxes):
            e[~_inside(b, lo, hi)] = j
        return e
    e = last_outside(blk)
    groups = sorted(set(e.tolist()))
    assert len(groups) >= 3                         # voxels of several epochs
    for g in groups:
        fresh = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
        for f in frames[g + 1:]:
            fresh.integrate_frame(f.xyz, f.origin, f.frame_id)
        fk, fS, fW, fc = fresh.read_tsdf()
        sel = last_outside(_blocks_of(fk, oracle_mod)) == g
        mine = e == g
        assert np.array_equal(fk[sel], key[mine]), g
        assert np.array_equal(fS[sel], S[mine]), g
        assert np.array_equal(fW[sel], W[mine]), g
        assert np.array_equal(fc[sel], clr[mine]), g


def test_point_records_by_brute_force(walk, windowed, oracle_mod):
    w, frames = walk
    o, boxes, _ = windowed
    scale = 256.0 / w.voxel
    first, nq, sumq = {}, {}, {}
    for j, f in enumerate(frames):
        P = np.rint(f.xyz.astype(np.float64) * scale).astype(np.int64)
        Q = np.rint(f.origin.astype(np.float64) * scale).astype(np.int64)
        ok = ~np.all(P == Q, axis=1)
        vox = np.floor_divide(P[ok], 256)
        vox = vox[_inside(np.floor_divide(vox, 8), *boxes[j])]
        for k in set(oracle_mod.pack_keys(vox).tolist()):
            first.setdefault(k, j)
            nq[k] = nq.get(k, 0) + 1
            sumq[k] = sumq.get(k, 0) + Q
    pts = o.read_points()
    assert len(pts["key"]) == len(first)
    for i, k in enumerate(pts["key"].tolist()):
        assert pts["first_frame"][i] == first[k]
        assert pts["nq"][i] == nq[k]
        assert np.array_equal(pts["sumq"][i], sumq[k])


def test_normals_use_points_inside_the_window(windowed, oracle_mod, walk):
    w, _ = walk
    o, boxes, _ = windowed
    lo, hi = boxes[-1]
    pts = o.read_points()
    r = o.read_results(len(w.rot))
    keys = pts["key"]
    vox = np.array([oracle_mod.unkey(int(k)) for k in keys], np.int64)
    inside = _inside(np.floor_divide(vox, 8), lo, hi)
    live = {tuple(v) for v in vox[inside].tolist()}
    offs = [(x, y, z) for z in range(-3, 4) for y in range(-3, 4) for x in range(-3, 4)]
    offs.sort(key=lambda d: (d[0] ** 2 + d[1] ** 2 + d[2] ** 2, d[2], d[1], d[0]))
    rows, idx = [], []
    for i in np.nonzero(inside & (r["has_normal"] >= 0) & (r["label"] != 0))[0][:3000]:
        s = vox[i]
        m = np.zeros(10, np.int64)
        for d in offs:
            if m[0] == 10:
                break
            if (s[0] + d[0], s[1] + d[1], s[2] + d[2]) in live:
                m[0] += 1
                m[1:4] += d
                m[4:] += (d[0] * d[0], d[0] * d[1], d[0] * d[2], d[1] * d[1], d[1] * d[2],
                          d[2] * d[2])
        rows.append(m)
        idx.append(i)
    assert len(idx) > 500
    axes, has = oracle_mod.pca_axes(np.array(rows))
    near_edge = 0
    for j, i in enumerate(idx):
        assert r["has_normal"][i] == has[j]
        if has[j]:
            a = axes[j]
            c = 256 * vox[i] + 128
            g = int(np.dot(a, pts["sumq"][i] - int(pts["nq"][i]) * c))
            if g < 0:
                a = -a
            assert np.array_equal(r["normal"][i], a), i
        b = np.floor_divide(vox[i], 8)
        near_edge += bool(np.any((8 * (b - lo) + vox[i] % 8 < 3) |
                                 (8 * (hi - b) + 7 - vox[i] % 8 < 3)))
    assert near_edge > 0   # some compared points have neighbours cut by the window


def test_labels_persist_outside_the_window(windowed, oracle_mod):
    o, _, scored = windowed
    last = {}
    for _, keys, label, ff, lo, hi in scored:
        ins = _inside(_blocks_of(keys, oracle_mod), lo, hi)
        for i in np.nonzero(ins)[0]:
            last[int(keys[i])] = (int(label[i]), int(ff[i]))
    _, keys, label, ff, lo, hi = scored[-1]
    outside = ~_inside(_blocks_of(keys, oracle_mod), lo, hi)
    for i, k in enumerate(keys.tolist()):
        assert (int(label[i]), int(ff[i])) == last.get(k, (255, -1)), k
    kept = [k for k in keys[outside].tolist() if k in last and last[k][0] != 0]
    never = [k for k in keys.tolist() if k not in last]
    assert len(kept) > 100 and len(never) > 0


def _incr_run(w, frames, oracle_mod, blocks, c2f=True, origins=None):
    from oracle.incremental import IncrementalOracle
    o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    if blocks is not None:
        o.set_window([blocks] * 3)
    o.set_tool(0, w.tool, w.rot)
    inc = IncrementalOracle(o, 0, len(w.rot), budget=900)
    if c2f:
        inc.enable_c2f(w.rot)
    per = []
    for j, f in enumerate(frames):
        before = inc.labels() if j else None
        st = inc.frame(f.xyz, f.origin if origins is None else origins[j], f.frame_id)
        per.append((before, dict(st), o.window(), inc.labels()))
    return per


def test_incremental_with_a_wide_window_is_without(synth_mod, oracle_mod):
    w = synth_mod.tiny()
    frames = w.frames(8)
    origins = [np.asarray(f.origin, np.float32) for f in frames]
    origins[5] = (np.asarray(frames[4].origin, np.float64) + [0.15, 0, 0]).astype(np.float32)
    a = _incr_run(w, frames, oracle_mod, None, origins=origins)
    b = _incr_run(w, frames, oracle_mod, 4096, origins=origins)
    for (_, sa, _, la), (_, sb, _, lb) in zip(a, b):
        assert sa == sb
        for x, y in zip(la, lb):
            assert np.array_equal(x, y)


def test_incremental_trigger_iii_only_inside_the_window(walk, oracle_mod):
    w, frames = walk
    per = _incr_run(w, frames[:20], oracle_mod, BLOCKS)
    cut = 0
    for j in range(1, len(per)):
        before, st, (lo, hi, _), _ = per[j]
        keys, lab = before[0], before[1]
        inacc = (lab == 2) | (lab == 3)
        ins = _inside(_blocks_of(keys, oracle_mod), lo, hi)
        # the walk moves 26 cm per frame: trigger (iii) fires every frame
        assert st["trig_iii"] == int(np.sum(inacc & ins)), j
        cut += int(np.sum(inacc & ~ins))
    assert cut > 0          # the window left some inaccessible points out
