"""Pins of the oracle's integration stage (CPU only).

Scan-centric TSDF integration, Section 3.2; ray-cleared band, Section 3.4
"Arm path checking"; weight cap with proportional rescaling, Section 3.6;
voxel-deduplicated points, Section 3.1.

Voxel size 2^-6 m is used wherever exact float32 <-> fixed-point round trips
are needed: positions are then integers in units of v/256 = 2^-14 m.
"""
import math

import numpy as np
import pytest

V = 2.0 ** -6          # voxel edge, metres
SC = 16384             # 256 / V, fixed-point units per metre


def f32(units):
    return (np.asarray(units, dtype=np.float64) / SC).astype(np.float32)


def dump(o):
    key, S, W, c = o.read_tsdf()
    import oracle
    ijk = oracle.unpack_keys(key)
    return {tuple(map(int, t)): (int(s), int(w), int(cc)) for t, s, w, cc in zip(ijk, S, W, c)}


def centre(i):
    return 256 * i + 128


def test_params(oracle_mod):
    o = oracle_mod.Oracle(voxel=0.02, trunc=0.06, r_c=0.01)
    p = o.params()
    assert (p["tau_u"], p["R"], p["rc_u"], p["dmin_u"]) == (768, 3, 128, 1280)
    o = oracle_mod.Oracle(voxel=0.01, trunc=0.04, r_c=0.01)
    p = o.params()
    assert (p["tau_u"], p["R"], p["rc_u"], p["dmin_u"]) == (1024, 4, 256, 2560)
    # default truncation min(4v, 0.1 m)
    o = oracle_mod.Oracle(voxel=0.01, trunc=0.0)
    assert o.params()["tau_u"] == 1024
    o = oracle_mod.Oracle(voxel=0.05, trunc=0.0)
    assert o.params()["tau_u"] == 512     # 0.1 m = 2 voxels


def test_isqrt_floor_div_keys(oracle_mod):
    rng = np.random.default_rng(0)
    vals = list(rng.integers(0, 2 ** 62, size=2000)) + list(range(0, 1000))
    for r in [1, 2, 3, 2 ** 20, 2 ** 26 + 1, 3037000499]:
        vals += [r * r - 1, r * r, r * r + 1]
    for n in vals:
        assert oracle_mod.isqrt(int(n)) == math.isqrt(int(n)), n
    for a, b in zip(rng.integers(-10 ** 12, 10 ** 12, 2000), rng.integers(1, 10 ** 6, 2000)):
        assert oracle_mod.floor_div(int(a), int(b)) == int(a) // int(b)
    pts = rng.integers(-2 ** 20, 2 ** 20, size=(500, 3))
    for p in pts:
        assert list(oracle_mod.unkey(oracle_mod.key(*p))) == list(p)
    k = oracle_mod.pack_keys(pts)
    assert [oracle_mod.key(*p) for p in pts] == list(k)
    assert np.array_equal(oracle_mod.unpack_keys(k), pts)


def test_single_return_closed_form(oracle_mod):
    """Sensor at the centre of voxel 0, return at the centre of voxel (10,0,0),
    tau = 3 voxels.  On the ray, voxel 10-k is exactly k voxels in front of the
    return: d = 256 k units.  The three voxels straight behind it are inside
    the 18 deg cone (cos = 1) and are skipped; no other voxel of the 7^3 cube
    is (for offset (k, m, n), k > 0, the cone needs 39 k^2 > 361 (m^2 + n^2)).
    Off-axis voxel (9,1,0): |C - Q| = 256 sqrt(82) = 2318.18 -> d = 2560 -
    2318 = 242.  Voxels beside or behind the return are farther from the
    sensor than the return and clamp to 0."""
    o = oracle_mod.Oracle(voxel=V, trunc=3 * V)
    Q = [centre(0)] * 3
    P = [centre(10), centre(0), centre(0)]
    o.integrate_frame(f32([P]), f32(Q), 0)
    t = dump(o)
    st = o.frame_stats()
    assert st["pairs_applied"] == 340 and st["pairs_excluded"] == 3
    for k in (1, 2, 3):
        assert (10 + k, 0, 0) not in t
    assert t[(9, 0, 0)][:2] == (256, 1)
    assert t[(8, 0, 0)][:2] == (512, 1)
    assert t[(7, 0, 0)][:2] == (768, 1)      # exactly tau
    assert t[(10, 0, 0)][:2] == (0, 1)
    assert t[(9, 1, 0)][:2] == (242, 1)
    assert t[(10, 1, 0)][:2] == (0, 1)
    assert t[(11, 1, 0)][:2] == (0, 1)       # behind, outside the cone
    assert t[(13, 1, 0)][:2] == (0, 1)       # cos = 768/sqrt(768^2+256^2) = 0.9487
    # band (tau, 2.25 tau] back along the ray in v/2 steps: lambda = 896..1664,
    # positions 2688 - lambda -> voxels 7, 6, 6, 5, 5, 4, 4
    cleared = {k for k, v in t.items() if v[2]}
    assert cleared == {(7, 0, 0), (6, 0, 0), (5, 0, 0), (4, 0, 0)}
    assert st["band_marks"] == 7
    assert t[(4, 0, 0)][:2] == (0, 0)
    # one surface point at the return's voxel
    pts = o.read_points()
    assert list(pts["key"]) == [oracle_mod.key(10, 0, 0)]


def test_negative_clamp_ablation(oracle_mod):
    """With the [-tau, tau] clamp a voxel beside the return keeps its negative
    distance: (10,1,0) has d = 2560 - isqrt(2560^2 + 256^2) = 2560 - 2572."""
    o = oracle_mod.Oracle(voxel=V, trunc=3 * V, clamp_negative=1)
    o.integrate_frame(f32([[centre(10), centre(0), centre(0)]]), f32([centre(0)] * 3), 0)
    t = dump(o)
    assert t[(10, 1, 0)][:2] == (-12, 1)
    assert t[(11, 1, 0)][0] < 0


def test_weight_cap_rescale(oracle_mod):
    """1500 returns at voxel 10 and 501 at voxel 11 (both on the x axis): voxel
    9 sees W = 2001 contributions, S = 1500*256 + 501*512 = 640512; the cap
    gives W = 2000, S = floor(640512*2000/2001) = 640191."""
    o = oracle_mod.Oracle(voxel=V, trunc=3 * V)
    P = [[centre(10), centre(0), centre(0)]] * 1500 + [[centre(11), centre(0), centre(0)]] * 501
    o.integrate_frame(f32(P), f32([centre(0)] * 3), 0)
    t = dump(o)
    assert t[(9, 0, 0)][:2] == (640191, 2000)
    # voxel 8: S = 1500*512 + 501*768 = 1152768 -> floor(1152768*2000/2001)
    assert t[(8, 0, 0)][:2] == (1152191, 2000)
    # a further frame adds one contribution and rescales again
    o.integrate_frame(f32([[centre(10), centre(0), centre(0)]]), f32([centre(0)] * 3), 1)
    t = dump(o)
    assert t[(9, 0, 0)][:2] == ((640191 + 256) * 2000 // 2001, 2000)


def test_dropped_returns(oracle_mod):
    o = oracle_mod.Oracle(voxel=V, trunc=3 * V)
    Q = [centre(0)] * 3
    good = [centre(5), centre(1), centre(2)]
    xyz = np.array([f32(good), [np.nan, 0, 0], [np.inf, 0, 0], f32(Q), [1e6, 0, 0]],
                   dtype=np.float32)
    o.integrate_frame(xyz, f32(Q), 0)
    st = o.frame_stats()
    assert (st["n_in"], st["n_valid"], st["n_dropped"]) == (5, 1, 4)
    with pytest.raises(ValueError):
        o.integrate_frame(xyz, f32(Q), 0)      # frame ids must increase
    with pytest.raises(ValueError):
        o.integrate_frame(xyz, np.array([np.nan, 0, 0], np.float32), 5)


def _brute_force_tsdf(frames, v, tau_u, R, cap=2000):
    """All voxels of the scene's bounding box x all returns: no cube
    enumeration, Python integers throughout."""
    scale = 256.0 / v
    S, W, clr = {}, {}, set()
    for fr in frames:
        Q = [int(np.rint(float(c) * scale)) for c in fr.origin]
        P = np.rint(fr.xyz.astype(np.float64) * scale).astype(np.int64)
        vox = P // 256
        lo = vox.min(0) - R
        hi = vox.max(0) + R
        dS, dW = {}, {}
        grid = np.stack(np.meshgrid(*[np.arange(lo[i], hi[i] + 1) for i in range(3)],
                                    indexing="ij"), -1).reshape(-1, 3)
        for r in range(len(P)):
            near = grid[np.abs(grid - vox[r]).max(1) <= R]
            p = [int(c) for c in P[r]]
            b = [p[i] - Q[i] for i in range(3)]
            bb = sum(c * c for c in b)
            for x in near:
                x = tuple(int(c) for c in x)
                c = [256 * x[i] + 128 for i in range(3)]
                a = [c[i] - p[i] for i in range(3)]
                ab = sum(a[i] * b[i] for i in range(3))
                aa = sum(t * t for t in a)
                if ab > 0 and 400 * ab * ab > 361 * aa * bb:
                    continue
                d = math.isqrt(bb) - math.isqrt(sum((c[i] - Q[i]) ** 2 for i in range(3)))
                d = max(0, min(tau_u, d))
                dS[x] = dS.get(x, 0) + d
                dW[x] = dW.get(x, 0) + 1
        for x in dW:
            s = S.get(x, 0) + dS[x]
            w = W.get(x, 0) + dW[x]
            if w > cap:
                s = s * cap // w
                w = cap
            S[x], W[x] = s, w
    return S, W


def test_brute_force_tiny(oracle_mod, synth_mod):
    """Per-voxel brute force over 3 frames x 60 returns of the tiny scene."""
    w = synth_mod.tiny(n_frames=3, n_hits=60)
    frames = w.frames()
    o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc)
    for f in frames:
        o.integrate_frame(f.xyz, f.origin, f.frame_id)
    p = o.params()
    S, W = _brute_force_tsdf(frames, w.voxel, p["tau_u"], p["R"])
    t = dump(o)
    got = {k: v[:2] for k, v in t.items() if v[1] > 0}
    assert got == {k: (S[k], W[k]) for k in W}


def _random_frames(rng, n_frames, n, scale_units=60000):
    """Returns/origins in exact 2^-14 m units, none on a voxel boundary."""
    frames = []
    for f in range(n_frames):
        Q = rng.integers(-scale_units, scale_units, 3)
        P = Q + rng.integers(-scale_units, scale_units, (n, 3))
        for arr in (P, Q):
            arr[arr % 256 == 0] += 1
        frames.append((P, Q))
    return frames


def _run(oracle_mod, frames, **kw):
    o = oracle_mod.Oracle(voxel=V, trunc=3 * V, **kw)
    for i, (P, Q) in enumerate(frames):
        o.integrate_frame(f32(P), f32(Q), i)
    return o


def test_order_independence(oracle_mod):
    rng = np.random.default_rng(1)
    frames = _random_frames(rng, 3, 400, 8000)
    a = dump(_run(oracle_mod, frames))
    shuffled = [(P[rng.permutation(len(P))], Q) for P, Q in frames]
    b = dump(_run(oracle_mod, shuffled))
    assert a == b


def test_translation_equivariance(oracle_mod):
    rng = np.random.default_rng(2)
    frames = _random_frames(rng, 3, 300, 8000)
    shift = np.array([256 * 7, -256 * 3, 256 * 11])
    a = dump(_run(oracle_mod, frames))
    b = dump(_run(oracle_mod, [(P + shift, Q + shift) for P, Q in frames]))
    sv = shift // 256
    assert {(k[0] + sv[0], k[1] + sv[1], k[2] + sv[2]): v for k, v in a.items()} == b


def test_rotation_equivariance(oracle_mod):
    """A 90 degree turn about z maps voxel centres onto voxel centres, so S and W
    map exactly: (x, y, z) -> (-y, x, z), voxel (i, j, k) -> (-j-1, i, k)."""
    rng = np.random.default_rng(3)
    frames = _random_frames(rng, 3, 300, 8000)

    def rot(A):
        return np.stack([-A[..., 1], A[..., 0], A[..., 2]], -1)

    a = dump(_run(oracle_mod, frames))
    b = dump(_run(oracle_mod, [(rot(P), rot(Q)) for P, Q in frames]))
    mapped = {(-k[1] - 1, k[0], k[2]): v[:2] for k, v in a.items() if v[1] > 0}
    assert mapped == {k: v[:2] for k, v in b.items() if v[1] > 0}


def test_points_and_viewpoints(oracle_mod):
    """New points are appended per frame in ascending key order; each (point,
    frame) adds the sensor position once to the running sum, and stores it as
    a viewpoint only if it moved more than 0.1 m from the last stored one, in a
    ring of 8."""
    o = oracle_mod.Oracle(voxel=V, trunc=3 * V, vp_min_dist=0.1)
    P = np.array([[centre(30), centre(2), centre(0)], [centre(31), centre(0), centre(0)],
                  [centre(30), centre(2), centre(0)], [centre(29), centre(5), centre(0)]])
    # 0.1 m = 1638.4 units -> novelty threshold rint = 1638
    origins = [[0, 0, 0], [1000, 0, 0], [1700, 0, 0], [1700, 1639, 0]]
    origins += [[1700 + 2000 * i, 1639, 0] for i in range(1, 9)]
    for f, q in enumerate(origins):
        Pf = P if f < 2 else P[:1]
        o.integrate_frame(f32(Pf), f32(q), f)
    pts = o.read_points()
    keys = [oracle_mod.key(29, 5, 0), oracle_mod.key(30, 2, 0), oracle_mod.key(31, 0, 0)]
    assert list(pts["key"]) == sorted(keys)
    assert list(pts["first_frame"]) == [0, 0, 0]
    i30 = list(pts["key"]).index(oracle_mod.key(30, 2, 0))
    i31 = list(pts["key"]).index(oracle_mod.key(31, 0, 0))
    # voxel (31,0,0) was seen in frames 0 and 1 only: origin 1000 units from the
    # first -> not novel
    assert pts["nq"][i31] == 2 and pts["n_vp"][i31] == 1
    assert list(pts["sumq"][i31]) == [1000, 0, 0]
    # voxel (30,2,0): frames 0..11; stored: 0, 1700 (>1638 from 0), (1700,1639)
    # (distance 1639 > 1638), then 8 more -> ring keeps the newest 8
    assert pts["nq"][i30] == len(origins)
    assert pts["n_vp"][i30] == 8
    stored = [[0, 0, 0], [1700, 0, 0], [1700, 1639, 0]] + origins[4:]
    assert pts["vp"][i30].tolist() == stored[-8:]
    assert list(pts["sumq"][i30]) == list(np.sum(origins, axis=0))


def test_region_of_interest_is_exact(oracle_mod, synth_mod):
    """With a region of interest (which also skips returns out of its reach),
    every voxel and point inside the region equals the unrestricted oracle's,
    on the tiny scene, for small regions placed around surface points."""
    w = synth_mod.tiny()
    frames = w.frames(8)
    full = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    for f in frames:
        full.integrate_frame(f.xyz, f.origin, f.frame_id)
    fk, fS, fW, fc = full.read_tsdf()
    fijk = oracle_mod.unpack_keys(fk)
    pts = full.read_points()
    rng = np.random.default_rng(5)
    for c in oracle_mod.unpack_keys(rng.choice(pts["key"], 4, replace=False)):
        lo, hi = c - 3, c + 3
        roi = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
        roi.set_roi(lo, hi)
        for f in frames:
            roi.integrate_frame(f.xyz, f.origin, f.frame_id)
        inside = np.all((fijk >= lo) & (fijk <= hi), axis=1)
        rk, rS, rW, rc = roi.read_tsdf()
        want = {int(k): (int(s), int(ww), int(cc)) for k, s, ww, cc in
                zip(fk[inside], fS[inside], fW[inside], fc[inside])}
        got = {int(k): (int(s), int(ww), int(cc)) for k, s, ww, cc in zip(rk, rS, rW, rc)}
        assert got == want and len(want) > 20
        rp = roi.read_points()
        pin = np.all((oracle_mod.unpack_keys(pts["key"]) >= lo) &
                     (oracle_mod.unpack_keys(pts["key"]) <= hi), axis=1)
        assert np.array_equal(rp["key"], pts["key"][pin])
        for name in ("n_vp", "vp", "sumq", "nq", "first_frame"):
            assert np.array_equal(rp[name], pts[name][pin]), name
