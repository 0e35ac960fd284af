"""Pins of the oracle's incremental mode (oracle/incremental.py and the C
helpers it uses), each against something other than the oracle itself:

* the sample hash is SplitMix64: its first outputs for seed 0 are the
  published ones;
* the confidence arithmetic is the paper's: a falls 1 -> 0.75 -> 0.5625 on
  conflicting evaluations, so for a well-observed point (c close to 1) one
  outlier keeps it accessible and two remove it; recovery adds 0.15 (1 - a);
  c = w / (w + 5) is 0.5 at w = 5 and first exceeds 0.7 at w = 12; the
  stored score never increases;
* the raw collision count of an orientation equals a table-free count of
  occupied voxels inside the analytic tool body;
* on the tiny scene: every evaluation equals the stateless per-point test at
  that frame; the budget takes queued points in canonical order and carries
  the rest; a sensor move of less than 0.1 m re-queues nothing, one of more
  re-queues exactly the points labelled inaccessible; the sample holds the
  256 changed voxels of smallest hash."""
import math

import numpy as np
import pytest

from test_oracle_scoring import _membership


def test_splitmix64_published_outputs(oracle_mod):
    from oracle.incremental import GOLDEN, mix64
    # SplitMix64 seeded with 0: state advances by the golden gamma, output = mix(state)
    assert [mix64(GOLDEN * i) for i in (1, 2, 3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_confidence_arithmetic(oracle_mod):
    from oracle.incremental import (LABEL_TENTATIVE, apply_evaluation, label_of)
    from oracle import LABEL_ACCESSIBLE, LABEL_BLOCKED, LABEL_UNSCORED
    n_c = 5
    st = dict(best=n_c, best_dir=-1, a=1.0, outcome=LABEL_UNSCORED)
    apply_evaluation(st, 2, 17, LABEL_ACCESSIBLE, n_c)        # first evaluation: a unchanged
    assert (st["best"], st["best_dir"], st["a"]) == (2, 17, 1.0)
    W = 2000                                                   # c = 2000/2005, close to 1
    assert label_of(st, W, n_c) == LABEL_ACCESSIBLE
    apply_evaluation(st, n_c, -1, LABEL_BLOCKED, n_c)         # one outlier
    assert st["a"] == 0.75 and st["best"] == 2                 # stored score kept
    assert label_of(st, W, n_c) == LABEL_ACCESSIBLE            # 0.748 > 0.7
    apply_evaluation(st, n_c, -1, LABEL_BLOCKED, n_c)         # two in a row
    assert st["a"] == 0.5625
    assert label_of(st, W, n_c) == LABEL_TENTATIVE             # 0.561 < 0.7
    apply_evaluation(st, 4, 3, LABEL_ACCESSIBLE, n_c)         # confirming, higher score
    assert st["a"] == 0.5625 + 0.15 * (1 - 0.5625) and st["best"] == 2
    apply_evaluation(st, 1, 9, LABEL_ACCESSIBLE, n_c)         # lower score is stored
    assert (st["best"], st["best_dir"]) == (1, 9)
    fresh = dict(best=1, best_dir=0, a=1.0, outcome=LABEL_ACCESSIBLE)
    assert label_of(fresh, 5, n_c) == LABEL_TENTATIVE          # c = 0.5 at w = k_c
    assert label_of(fresh, 11, n_c) == LABEL_TENTATIVE         # 11/16 = 0.6875
    assert label_of(fresh, 12, n_c) == LABEL_ACCESSIBLE        # 12/17 = 0.706
    blocked = dict(best=n_c, best_dir=-1, a=1.0, outcome=LABEL_UNSCORED)
    apply_evaluation(blocked, n_c, -1, LABEL_BLOCKED, n_c)
    apply_evaluation(blocked, n_c, -1, LABEL_BLOCKED, n_c)
    assert blocked["a"] == 1.0                                 # nothing stored to contradict
    assert label_of(blocked, W, n_c) == LABEL_BLOCKED


@pytest.fixture(scope="module")
def tiny_incr(oracle_mod, synth_mod):
    from oracle.incremental import IncrementalOracle
    w = synth_mod.tiny()
    frames = w.frames(8)
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    orc.set_tool(0, w.tool, w.rot)
    return w, frames, orc, IncrementalOracle(orc, 0, len(w.rot), budget=700)


def test_body_count_against_analytic_solid(tiny_incr, oracle_mod):
    w, frames, orc, inc = tiny_incr
    for f in frames[:4]:
        orc.integrate_frame(f.xyz, f.origin, f.frame_id)
    orc.score(0)
    p = orc.params()
    key, S, W, c = orc.read_tsdf()
    ijk = oracle_mod.unpack_keys(key)
    occ_ijk = ijk[(W > 0) & (S < p["rc_u"] * W.astype(np.int64))]
    checked = 0
    for k in orc.read_points()["key"][::7]:
        r = orc.point_result(k, len(w.rot))
        if r["label"] != 1:
            continue
        s = np.array(oracle_mod.unkey(k))
        rel = occ_ijk - s
        near = np.abs(rel).max(1) <= math.ceil((w.tool.length + w.tool.corridor) / w.voxel) + 2
        body, far, amb = _membership(w.tool, w.rot[r["first_free"]], w.voxel, rel[near])
        if amb.any():
            continue
        assert orc.body_hits(0, k, r["first_free"]) == int(body.sum())
        checked += 1
    assert checked >= 20


def test_sample_and_move_rule(oracle_mod, synth_mod):
    """The sample is the smallest hashes of the frame's changed voxels; a
    sensor move below 0.1 m re-queues nothing, one above re-queues exactly
    the points labelled inaccessible after the previous frame."""
    from oracle.incremental import IncrementalOracle, sample_hash
    w = synth_mod.tiny()
    frames = w.frames(6)
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    orc.set_tool(0, w.tool, w.rot)
    inc = IncrementalOracle(orc, 0, len(w.rot), budget=700)
    moves = []
    for j, f in enumerate(frames):
        origin = np.asarray(f.origin, np.float32)
        if j == 4:
            origin = (np.asarray(frames[3].origin, np.float64) + [0.05, 0, 0]).astype(np.float32)
        if j == 5:
            origin = (np.asarray(frames[3].origin, np.float64) + [0.15, 0, 0]).astype(np.float32)
        prev = inc.labels()[1] if inc.state else np.zeros(0, np.uint8)
        st = inc.frame(f.xyz, origin, f.frame_id)
        ch = orc.changed_voxels()
        assert st["sampled"] == min(256, len(ch))
        hs = [sample_hash(c, f.frame_id) for c in ch]
        assert len(set(hs)) == len(hs)                      # no ties to break
        moves.append((st["trig_iii"], int(np.isin(prev, (2, 3)).sum())))
    assert moves[4][0] == 0
    assert moves[5][0] == moves[5][1] > 0


def test_evaluations_equal_stateless_labels(oracle_mod, synth_mod):
    """Budget large enough for everything: after each frame, every point
    evaluated in that frame carries the stateless label and, if accessible,
    the body count of its first free orientation."""
    from oracle.incremental import IncrementalOracle
    w = synth_mod.tiny()
    frames = w.frames(4)
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    ref = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    orc.set_tool(0, w.tool, w.rot)
    ref.set_tool(0, w.tool, w.rot)
    inc = IncrementalOracle(orc, 0, len(w.rot), budget=10 ** 9)
    K = len(w.rot)
    for f in frames:
        inc.frame(f.xyz, f.origin, f.frame_id)
        ref.integrate_frame(f.xyz, f.origin, f.frame_id)
        ref.score(0)
        assert len(inc.last_evaluated) > 0
        for k in inc.last_evaluated:
            s2 = inc.state[k]
            r = ref.point_result(k, K)
            assert s2["outcome"] == r["label"] != 0
        # with an unlimited budget nothing confident stays queued
        for k in orc.read_points()["key"]:
            assert not inc.state[int(k)]["pending"] or ref.voxel(int(k))[1] < 2
    # the first frame evaluates every confident point: outcome == stateless label
    inc2 = IncrementalOracle(oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c), 0, K,
                             budget=10 ** 9)
    inc2.orc.set_tool(0, w.tool, w.rot)
    ref2 = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    ref2.set_tool(0, w.tool, w.rot)
    inc2.frame(frames[0].xyz, frames[0].origin, frames[0].frame_id)
    ref2.integrate_frame(frames[0].xyz, frames[0].origin, frames[0].frame_id)
    ref2.score(0)
    for k in inc2.orc.read_points()["key"]:
        s2 = inc2.state[int(k)]
        r = ref2.point_result(k, K)
        assert s2["outcome"] == r["label"]
        if r["label"] == 1:
            assert s2["best"] == ref2.body_hits(0, k, r["first_free"]) < 5
            assert s2["best_dir"] == r["first_free"]
        else:
            assert s2["best"] == 5


def test_budget_and_backlog(oracle_mod, synth_mod):
    from oracle.incremental import IncrementalOracle
    w = synth_mod.tiny()
    f = w.frames(1)[0]
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    orc.set_tool(0, w.tool, w.rot)
    inc = IncrementalOracle(orc, 0, len(w.rot), budget=100)
    st = inc.frame(f.xyz, f.origin, f.frame_id)
    keys = orc.read_points()["key"]
    conf = [int(k) for k in keys if orc.voxel(int(k))[1] >= 2]
    assert st["evaluated"] == min(100, len(conf)) == 100
    done = [k for k in keys if inc.state[int(k)]["outcome"] != 0]
    assert [int(k) for k in done] == conf[:100]                 # canonical order
    assert st["backlog"] == len(keys) - 100                     # the rest stay queued


def _plane(depth, n=60, seed=0):
    rng = np.random.default_rng(seed)
    yz = rng.uniform(-0.3, 0.3, size=(n, 2))
    return np.concatenate([np.full((n, 1), depth), yz], axis=1).astype(np.float32)


def plane_frames():
    """A 60 cm plane at 1 m seen head-on twice, then moved 9 cm back (v = 2 cm,
    tau = 10 cm): the TSDF at some old surface voxels jumps by more than 2v."""
    return [(_plane(d, seed=j), np.zeros(3, np.float32), j)
            for j, d in enumerate([1.0, 1.0, 1.09, 1.09])]


def test_trigger_i_on_a_moving_surface(oracle_mod, synth_mod):
    from oracle.incremental import IncrementalOracle
    w = synth_mod.tiny()
    orc = oracle_mod.Oracle(voxel=0.02, trunc=0.10, r_c=0.01)
    orc.set_tool(0, w.tool, w.rot)
    inc = IncrementalOracle(orc, 0, len(w.rot), budget=10 ** 6)
    par = orc.params()
    for xyz, o, fid in plane_frames():
        before = {int(k): orc.voxel(int(k))[:2] for k in orc.read_points()["key"]}
        st = inc.frame(xyz, o, fid)
        # the same test in metres, floating point: |T - T'| > 2v
        n_i = 0
        for k, (S0, W0) in before.items():
            S1, W1 = orc.voxel(k)[:2]
            if W0 > 0 and W1 > 0 and abs(S1 / W1 - S0 / W0) / par["scale"] > 2 * 0.02 + 1e-12:
                n_i += 1
        assert st["trig_i"] == n_i
        if fid == 2:
            assert n_i > 0


def _run(oracle_mod, synth_mod, n_frames, **kw):
    from oracle.incremental import IncrementalOracle
    w = synth_mod.tiny()
    frames = w.frames(n_frames)
    orc = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    orc.set_tool(0, w.tool, w.rot)
    return w, frames, IncrementalOracle(orc, 0, len(w.rot), **kw)


def test_drain_equals_a_larger_frame_budget(oracle_mod, synth_mod):
    """A frame with a small cap followed by a drain of everything queued
    leaves every point as a frame without a cap does (the drain evaluates the
    same points on the same map, in the same order), frame after frame."""
    w, frames, small = _run(oracle_mod, synth_mod, 6, budget=300)
    _, _, full = _run(oracle_mod, synth_mod, 6, budget=10 ** 9)
    for f in frames:
        st = small.frame(f.xyz, f.origin, f.frame_id)
        assert st["evaluated"] <= 300
        d = small.drain(10 ** 9)
        assert d["trig_i"] == 0
        ft = full.frame(f.xyz, f.origin, f.frame_id)
        # what stays queued is below the confidence gate, as after the full frame
        assert d["backlog"] == ft["backlog"]
        assert st["evaluated"] + d["evaluated"] == ft["evaluated"]
        for x, y in zip(small.labels(), full.labels()):
            assert np.array_equal(x, y)


def test_partial_drains_in_point_order(oracle_mod, synth_mod):
    """Drains of 150 take the queued points in point order: after a frame with
    cap 200 and two drains of 150, the evaluated points are the first 500
    queued ones, as with one frame of cap 500."""
    w, frames, a = _run(oracle_mod, synth_mod, 1, budget=200)
    _, _, b = _run(oracle_mod, synth_mod, 1, budget=500)
    f = frames[0]
    a.frame(f.xyz, f.origin, f.frame_id)
    first = list(a.last_evaluated)
    a.drain(150)
    first += a.last_evaluated
    a.drain(150)
    first += a.last_evaluated
    b.frame(f.xyz, f.origin, f.frame_id)
    assert first == list(b.last_evaluated) and len(first) == 500
    for x, y in zip(a.labels(), b.labels()):
        assert np.array_equal(x, y)


def test_adaptive_cap(oracle_mod, synth_mod):
    """The adaptive cap stays within [b_min, b_max], follows the previous
    frame's lookups per evaluation, and with a target no frame can reach it
    stays at b_max, which then matches a fixed cap of b_max exactly."""
    w, frames, ad = _run(oracle_mod, synth_mod, 8, budget=400, lookup_target=150000,
                         b_min=50, b_max=3000)
    caps = []
    prev = None
    for f in frames:
        st = ad.frame(f.xyz, f.origin, f.frame_id)
        assert 50 <= st["budget"] <= 3000
        if prev is not None and prev["evaluated"] and prev["lookups"]:
            want = 150000 * prev["evaluated"] // prev["lookups"]
            assert st["budget"] == min(3000, max(50, want))
        caps.append(st["budget"])
        prev = st
    assert caps[0] == 400 and len(set(caps)) > 2          # it adapts
    _, _, hi = _run(oracle_mod, synth_mod, 8, budget=900, lookup_target=10 ** 12, b_min=1,
                    b_max=900)
    _, _, fx = _run(oracle_mod, synth_mod, 8, budget=900)
    for j, f in enumerate(frames):
        a = hi.frame(f.xyz, f.origin, f.frame_id)
        b = fx.frame(f.xyz, f.origin, f.frame_id)
        assert a["budget"] == 900 and a["evaluated"] == b["evaluated"]
        for x, y in zip(hi.labels(), fx.labels()):
            assert np.array_equal(x, y)


def test_coarse_fine_sets_on_the_yaw_set(oracle_mod, synth_mod):
    """The paper's D = 180 yaw directions (2 degree steps): the coarse pass is
    every tenth direction (20 degrees apart, 18 of them) and the fine window
    of direction k is k-12 .. k+12 (within 24 degrees), 25 directions."""
    from oracle.incremental import coarse_fine_sets
    c, f = coarse_fine_sets(synth_mod.orientations(synth_mod.yaw_directions(180), 1))
    bits = lambda w: [k for k in range(180) if (int(w[k // 64]) >> (k % 64)) & 1]
    assert bits(c) == list(range(0, 180, 10))
    for k in (0, 7, 90, 179):
        assert bits(f[k]) == sorted((k + d) % 180 for d in range(-12, 13))
    # rolls share their direction's membership
    c4, f4 = coarse_fine_sets(synth_mod.orientations(synth_mod.yaw_directions(180), 4))
    assert bits(c4)[:8] == [0, 1, 2, 3, 40, 41, 42, 43]


def test_allow_restriction_by_single_orientations(oracle_mod, synth_mod):
    """Scoring with an allowed set gives, for each point, the first allowed
    orientation that is a free candidate: checked against scoring each
    allowed orientation on its own (one-orientation allow masks)."""
    w = synth_mod.tiny()
    rot = synth_mod.orientations(synth_mod.yaw_directions(180), 1)
    o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    for f in w.frames(6):
        o.integrate_frame(f.xyz, f.origin, f.frame_id)
    o.set_tool(0, w.tool, rot)
    keys = o.read_points()["key"]
    rng = np.random.default_rng(3)
    pick = keys[rng.choice(len(keys), 40, replace=False)]
    allow = np.zeros((len(pick), 3), np.uint64)
    for j in range(len(pick)):
        for k in rng.choice(180, 40, replace=False):
            allow[j, k // 64] |= np.uint64(1) << np.uint64(k % 64)
    o.score(0, pick, allow=allow)
    got = [o.point_result(int(k), 180) for k in pick]
    seen = 0
    for j, k in enumerate(pick):
        if got[j]["label"] == 0:
            continue
        first = -1
        for kk in range(180):
            if not (int(allow[j, kk // 64]) >> (kk % 64)) & 1:
                continue
            one = np.zeros((1, 3), np.uint64)
            one[0, kk // 64] = np.uint64(1) << np.uint64(kk % 64)
            o.score(0, [k], allow=one)
            if o.point_result(int(k), 180)["label"] == 1:
                first = kk
                break
        assert got[j]["first_free"] == first, (j, got[j], first)
        seen += first >= 0
    assert seen > 5


def test_nearest_resolved_neighbour_rule(oracle_mod, synth_mod):
    """The neighbour rule on hand-placed states: equal distances resolve by
    (dz, dy, dx); points farther than 0.3 m and unresolved points are not
    neighbours; the point itself is not its own neighbour."""
    from oracle.incremental import IncrementalOracle
    w = synth_mod.tiny()
    rot = synth_mod.orientations(synth_mod.yaw_directions(180), 1)
    o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    o.set_tool(0, w.tool, rot)
    inc = IncrementalOracle(o, 0, 180, budget=10)
    inc.enable_c2f(rot)
    key = oracle_mod.key
    st = lambda best, d: dict(best=best, best_dir=d, a=1.0, S=0, W=10, pending=False, outcome=1)
    inc.state = {key(0, 0, 0): st(2, 5), key(1, 0, 0): st(1, 30), key(0, 0, -1): st(0, 60),
                 key(0, -1, 0): st(5, 90),                  # not resolved (best = n_c)
                 key(20, 0, 0): st(0, 120)}                 # 0.4 m away at v = 2 cm
    allow = inc._allow([key(0, 0, 0), key(19, 0, 0), key(0, 0, 40)])
    assert inc.last_neighbour[key(0, 0, 0)] == (key(0, 0, -1), 60)   # dz = -1 first
    assert inc.last_neighbour[key(19, 0, 0)] == (key(20, 0, 0), 120)
    assert key(0, 0, 40) not in inc.last_neighbour                   # none within 0.3 m
    from oracle.incremental import coarse_fine_sets
    c, f = coarse_fine_sets(rot)
    assert np.array_equal(allow[0], c | f[60]) and np.array_equal(allow[2], c)


def test_c2f_searches_fewer_orientations(oracle_mod, synth_mod):
    """On the tiny scene with the yaw set, the coarse-to-fine search tests
    fewer candidates than the full search of the same evaluations, and every
    point it labels accessible is accessible under the full search too (its
    free orientation is one of the full set's)."""
    from oracle.incremental import IncrementalOracle
    w = synth_mod.tiny()
    rot = synth_mod.orientations(synth_mod.yaw_directions(180), 1)
    runs = []
    for c2f in (False, True):
        o = oracle_mod.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
        o.set_tool(0, w.tool, rot)
        inc = IncrementalOracle(o, 0, 180, budget=10 ** 9)
        if c2f:
            inc.enable_c2f(rot)
        tests = 0
        for f in w.frames(4):
            inc.frame(f.xyz, f.origin, f.frame_id)
            tests += o.score_stats()["candidate_tests"]
        runs.append((inc, tests))
    (full, t_full), (cf, t_cf) = runs
    assert t_cf < t_full
    kf, lf, _, _, _ = full.labels()
    kc, lc, _, _, _ = cf.labels()
    assert np.array_equal(kf, kc)
    acc_c = np.isin(lc, (1, 4))
    assert acc_c.sum() > 100
    assert np.all(np.isin(lf[acc_c], (1, 4)))
