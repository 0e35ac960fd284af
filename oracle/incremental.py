"""Incremental mode of the accessibility field -- CPU ORACLE, test
infrastructure only (only the tests, the smoke check and the benchmark's
CPU-baseline leg may use it).

Section 3.5 ("Incremental Updates and Confidence") keeps a state per surface
point and re-evaluates a point only when something near it changed.  This
module implements that state machine in plain Python on top of the C oracle
(integration and the per-point test of Section 3.4), in the paper's order:

1. integrate the frame;
2. queue points by the three triggers and on first observation:
   (i)   the TSDF at the point's voxel moved by more than 2v since the last
         frame;
   (ii)  a voxel within r_u = 3v of the point changed, judged from a sample of
         at most 256 of the frame's changed voxels;
   (iii) the sensor moved more than 0.1 m since the last time this trigger
         fired: every point currently classified inaccessible is queued;
3. evaluate queued points whose confidence c = w / (w + 5) is at least 0.2,
   at most `budget` of them per frame in canonical point order; the others
   stay queued (the backlog), and `drain` evaluates more of them between
   frames;
4. update each evaluated point's state: the best stored direction score
   never increases; the accessibility confidence a (initially 1) is
   multiplied by 0.75 when an evaluation finds blocked a point whose stored
   score says accessible, and recovers by 0.15 (1 - a) when an evaluation
   finds it accessible;
5. label every point: accessible iff the stored score is under n_c and
   c * a > 0.7 ("confident-accessible").

Readings where the paper leaves a choice (each matched by the GPU side):
an evaluation is the per-point test of Section 3.4 (first free orientation
in index order) and its score is the raw collision count, the number of body
voxels with TSDF < r_c, of that orientation; an evaluation that finds no free
orientation scores n_c.  A changed voxel is one that received a contribution
in the frame.  The sample of changed voxels is the 256 with the smallest
SplitMix64 hash of (voxel key XOR frame * 0x9E3779B97F4A7C15).  Trigger (i)
compares S/W exactly.  The budget is a fixed cap, or it adapts: the paper's
cap adapts to the frame time, which no test can reproduce, so the adaptive
cap follows a cost that both sides count exactly, the canonical lookups of
the frame's evaluations.  After a frame that evaluated n > 0 points for L > 0
lookups, the next frame's cap is lookup_target * n // L (integer division),
clamped to [b_min, b_max]; otherwise it stays.  The backlog is consumed
between frames by explicit drain calls (the caller knows when it is idle),
each evaluating up to a given number of queued points in point order; a drain
runs no trigger and does not change the cap.  Labels: UNSCORED (never
evaluated), ACCESSIBLE (confident-accessible), TENTATIVE (a free direction
is stored but c * a <= 0.7), BLOCKED / NO_CANDIDATE (no free direction ever
stored; the last evaluation found every candidate blocked / no candidate).
Trigger (iii) re-queues the points labelled BLOCKED or NO_CANDIDATE after the
previous frame.

With a sliding window (Section 3.3, set on the C oracle before the first
frame): trigger (iii) re-queues only the inaccessible points inside the
window (the paper's wording), and the nearest resolved neighbour of the
coarse-to-fine search is taken among points inside the window.  Nothing else
changes: points outside have no voxel (W = 0), so they are never selected,
trigger (i) needs W > 0 before and after, and their label follows from
c = 0.

Coarse-to-fine direction search (Section 3.6, optional): an evaluation tests
only the orientations of a coarse pass, plus those close to the direction
stored by the closest already-resolved neighbouring point.  Readings, for any orientation
set: the coarse pass holds the orientations whose approach direction was
taken by a greedy walk in index order that takes a direction when it is at
least 20 degrees from every direction taken before (dot product at most
cos 20 + 1e-12), together with every orientation sharing a taken direction;
the fine window of orientation k* holds the orientations whose direction is
within 25 degrees of k*'s (dot product at least cos 25 - 1e-12).  A resolved
point is one with a stored free direction (stored score below n_c) when the
evaluation step starts; the nearest resolved neighbour of a point is the
other resolved point of smallest (|d|^2, dz, dy, dx), d its voxel offset, with
|d| at most 0.3 m; without one, only the coarse pass is searched.  Among the
allowed orientations the evaluation is the usual one (candidate filters,
first free in index order).
"""
from __future__ import annotations

import math

import numpy as np

from . import LABEL_ACCESSIBLE, LABEL_BLOCKED, LABEL_NO_CANDIDATE, LABEL_UNSCORED, unpack_keys

LABEL_TENTATIVE = 4
MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    """The output function of Steele, Lea and Flood's SplitMix64."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def sample_hash(key: int, frame: int) -> int:
    return mix64((int(key) & MASK64) ^ ((int(frame) * GOLDEN) & MASK64))


def apply_evaluation(st, score: int, direction: int, outcome: int, n_c: int,
                     decay: float = 0.75, recover: float = 0.15):
    """State update of one evaluation (step 4): a recovers on an accessible
    finding, decays on a blocked finding that contradicts a stored free
    direction; the stored score only ever decreases."""
    if st["outcome"] != LABEL_UNSCORED:
        if score < n_c:
            st["a"] = st["a"] + recover * (1.0 - st["a"])
        elif st["best"] < n_c:
            st["a"] = decay * st["a"]
    if score < st["best"]:
        st["best"], st["best_dir"] = score, direction
    st["outcome"] = outcome


def label_of(st, W: int, n_c: int, k_c: int = 5, accept: float = 0.7) -> int:
    """Step 5, with c = W / (W + k_c) of the point's voxel."""
    if st["outcome"] == LABEL_UNSCORED:
        return LABEL_UNSCORED
    if st["best"] < n_c:
        c = W / (W + k_c)
        return LABEL_ACCESSIBLE if c * st["a"] > accept else LABEL_TENTATIVE
    return LABEL_NO_CANDIDATE if st["outcome"] == LABEL_NO_CANDIDATE else LABEL_BLOCKED


def _dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def coarse_fine_sets(rot, coarse_deg: float = 20.0, fine_deg: float = 25.0):
    """(coarse [mw] uint64, fine [K, mw] uint64) of an orientation set given
    as K row-major rotations whose column 0 is the approach direction."""
    R = np.asarray(rot, np.float64).reshape(-1, 9)
    d = [(float(r[0]), float(r[3]), float(r[6])) for r in R]
    K = len(d)
    mw = (K + 63) // 64
    cc = math.cos(coarse_deg * (math.pi / 180.0))
    cf = math.cos(fine_deg * (math.pi / 180.0))
    taken = []
    coarse = np.zeros(mw, np.uint64)
    for k in range(K):
        if d[k] in taken or all(_dot(d[k], c) <= cc + 1e-12 for c in taken):
            if d[k] not in taken:
                taken.append(d[k])
            coarse[k // 64] |= np.uint64(1) << np.uint64(k % 64)
    fine = np.zeros((K, mw), np.uint64)
    for a in range(K):
        for k in range(K):
            if _dot(d[k], d[a]) >= cf - 1e-12:
                fine[a, k // 64] |= np.uint64(1) << np.uint64(k % 64)
    return coarse, fine


def ball_offsets(r: int):
    """Integer offsets o with |o|^2 <= r^2."""
    return [(x, y, z) for z in range(-r, r + 1) for y in range(-r, r + 1)
            for x in range(-r, r + 1) if x * x + y * y + z * z <= r * r]


class IncrementalOracle:
    def __init__(self, orc, tool_id: int, K: int, budget: int, n_sample: int = 256,
                 r_u: int = 3, k_c: int = 5, decay: float = 0.75, recover: float = 0.15,
                 accept: float = 0.7, lookup_target: int = 0, b_min: int = 1,
                 b_max: int | None = None):
        self.orc, self.tool_id, self.K, self.budget = orc, tool_id, K, budget
        self.lookup_target, self.b_min = lookup_target, b_min
        self.b_max = budget if b_max is None else b_max
        self.c2f = None
        self.n_sample, self.k_c = n_sample, k_c
        self.decay, self.recover, self.accept = decay, recover, accept
        self.ball = ball_offsets(r_u)
        par = orc.params()
        self.scale = par["scale"]
        self.move_u2 = par["dmin_u"] ** 2          # 0.1 m, squared, fixed-point units
        self.n_c = orc.cfg.n_c
        self.conf_min_w = orc.cfg.conf_min_w
        self.state = {}       # key -> dict(best, best_dir, a, S, W, pending, outcome)
        self.q_last = None
        self.stats = {}

    def enable_c2f(self, rot, coarse_deg: float = 20.0, fine_deg: float = 25.0,
                   radius_m: float = 0.3):
        """Search only the coarse pass and the fine window (Section 3.6)."""
        coarse, fine = coarse_fine_sets(rot, coarse_deg, fine_deg)
        r = radius_m / self.orc.cfg.voxel
        self.c2f = dict(coarse=coarse, fine=fine, r2=int(math.floor(r * r + 1e-9)))

    def _allow(self, chosen):
        """Allowed orientations of each chosen point: the coarse pass, plus
        the fine window of its nearest resolved neighbour's stored direction."""
        c = self.c2f
        res = [(k, st["best_dir"]) for k, st in self.state.items() if st["best"] < self.n_c]
        if res:   # only points inside the sliding window
            ins = self._inside([k for k, _ in res])
            res = [r for r, i in zip(res, ins) if i]
        allow = np.tile(c["coarse"], (len(chosen), 1))
        self.last_neighbour = {}
        if not res or not chosen:
            return allow
        rk = unpack_keys(np.array([k for k, _ in res], np.int64))
        rdir = np.array([b for _, b in res], np.int64)
        pk = unpack_keys(np.array(chosen, np.int64))
        for j, s in enumerate(pk):
            d = rk - s
            d2 = (d * d).sum(1)
            code = (d2 << 30) | ((d[:, 2] + 512) << 20) | ((d[:, 1] + 512) << 10) | (d[:, 0] + 512)
            code = np.where((d2 == 0) | (d2 > c["r2"]), np.iinfo(np.int64).max, code)
            m = int(np.argmin(code))
            if code[m] == np.iinfo(np.int64).max:
                continue
            allow[j] |= c["fine"][rdir[m]]
            self.last_neighbour[chosen[j]] = (int(res[m][0]), int(rdir[m]))
        return allow

    def _label(self, st, W):
        return label_of(st, W, self.n_c, self.k_c, self.accept)

    def _inside(self, keys):
        """Whether each point key lies in the sliding window (all of them
        without one)."""
        keys = np.asarray(keys, np.int64)
        win = self.orc.window()
        if win is None or len(keys) == 0:
            return np.ones(len(keys), bool)
        blk = np.floor_divide(unpack_keys(keys), 8)
        return np.all((blk >= win[0]) & (blk <= win[1]), axis=1)

    def frame(self, xyz, origin, frame_id: int):
        orc = self.orc
        orc.integrate_frame(xyz, origin, frame_id)
        keys = orc.read_points()["key"]
        vox = {int(k): orc.voxel(int(k))[:2] for k in keys}
        # trigger (iii) needs the labels before this frame's evaluation
        Q = [int(np.rint(np.float64(np.float32(o)) * self.scale)) for o in origin]
        moved = False
        if self.q_last is None:
            self.q_last = Q
        elif sum((a - b) ** 2 for a, b in zip(Q, self.q_last)) > self.move_u2:
            moved = True
            self.q_last = Q
        n_new = n_i = n_ii = n_iii = 0
        inside = self._inside(keys)
        for j, k in enumerate(keys):
            k = int(k)
            S, W = vox[k]
            st = self.state.get(k)
            if st is None:
                st = dict(best=self.n_c, best_dir=-1, a=1.0, S=S, W=W, pending=True,
                          outcome=LABEL_UNSCORED)
                self.state[k] = st
                n_new += 1
                continue
            if st["W"] > 0 and W > 0 and abs(S * st["W"] - st["S"] * W) > 512 * W * st["W"]:
                st["pending"] = True
                n_i += 1
            if moved and inside[j] and self._label(st, st["W"]) in (LABEL_BLOCKED,
                                                                    LABEL_NO_CANDIDATE):
                st["pending"] = True
                n_iii += 1
            st["S"], st["W"] = S, W
        # trigger (ii): points within r_u of a sample of the changed voxels
        changed = orc.changed_voxels()
        order = sorted((sample_hash(c, frame_id), int(c)) for c in changed)
        sample = [c for _, c in order[:self.n_sample]]
        for c in sample:
            x, y, z = (int(v) for v in unpack_keys(np.array([c], np.int64))[0])
            for dx, dy, dz in self.ball:
                kk = _key(x + dx, y + dy, z + dz)
                st = self.state.get(kk)
                if st is not None and not st["pending"]:
                    st["pending"] = True
                    n_ii += 1
        # evaluate at most `budget` queued confident points, canonical order
        budget = self.budget
        chosen, lookups = self._evaluate(keys, vox, budget)
        if self.lookup_target > 0 and chosen and lookups > 0:
            self.budget = min(self.b_max, max(self.b_min,
                                              self.lookup_target * len(chosen) // lookups))
        self.stats = dict(new=n_new, trig_i=n_i, trig_ii=n_ii, trig_iii=n_iii,
                          sampled=len(sample), evaluated=len(chosen), budget=budget,
                          lookups=lookups,
                          backlog=sum(1 for s in self.state.values() if s["pending"]))
        return self.stats

    def drain(self, max_evals: int):
        """Between frames: evaluate up to max_evals queued confident points
        in point order (no trigger, the cap unchanged)."""
        keys = self.orc.read_points()["key"]
        vox = {int(k): self.orc.voxel(int(k))[:2] for k in keys}
        chosen, lookups = self._evaluate(keys, vox, max_evals)
        self.stats = dict(new=0, trig_i=0, trig_ii=0, trig_iii=0, sampled=0,
                          evaluated=len(chosen), budget=max_evals, lookups=lookups,
                          backlog=sum(1 for s in self.state.values() if s["pending"]))
        return self.stats

    def _evaluate(self, keys, vox, cap):
        """Steps 3-4 for the first `cap` queued confident points; returns
        them and their canonical lookups."""
        orc = self.orc
        chosen = [int(k) for k in keys
                  if self.state[int(k)]["pending"] and vox[int(k)][1] >= self.conf_min_w]
        chosen = chosen[:cap]
        lookups = 0
        if chosen:
            allow = self._allow(chosen) if self.c2f is not None else None
            orc.score(self.tool_id, np.array(chosen, np.int64), allow=allow)
            lookups = orc.score_stats()["canonical_lookups"]
        for k in chosen:
            st = self.state[k]
            st["pending"] = False
            r = orc.point_result(k, self.K)
            if r["label"] == LABEL_ACCESSIBLE:
                score, d = orc.body_hits(self.tool_id, k, r["first_free"]), r["first_free"]
            else:
                score, d = self.n_c, -1
            apply_evaluation(st, score, d, r["label"], self.n_c, self.decay, self.recover)
        self.last_evaluated = chosen
        return chosen, lookups

    def labels(self):
        """(keys, label, best, best_dir, a) in canonical point order."""
        keys = self.orc.read_points()["key"]
        lab, best, bdir, a = [], [], [], []
        for k in keys:
            st = self.state[int(k)]
            lab.append(self._label(st, st["W"]))
            best.append(st["best"])
            bdir.append(st["best_dir"])
            a.append(st["a"])
        return (np.asarray(keys), np.array(lab, np.uint8), np.array(best, np.int32),
                np.array(bdir, np.int32), np.array(a, np.float64))


def _key(x, y, z):
    m = (1 << 21) - 1
    return ((x + (1 << 20)) & m) | (((y + (1 << 20)) & m) << 21) | (((z + (1 << 20)) & m) << 42)
