"""ctypes front-end of the CPU oracle (test infrastructure only).

The oracle is a plain single-threaded C implementation of the accessibility
field hot path written from the paper; see ``oracle.c``.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package.  It
shares no code with the GPU library in ``paper_2608_06412_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")
_lib = None

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
          "-std=gnu11"]

LABEL_UNSCORED, LABEL_ACCESSIBLE, LABEL_BLOCKED, LABEL_NO_CANDIDATE = 0, 1, 2, 3
CLS_BODY, CLS_NEAR, CLS_FAR = 0, 1, 2


def build(force: bool = True) -> str:
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "smooth.c")]
    dep = max(os.path.getmtime(f) for f in srcs + [os.path.join(_HERE, "oracle.h")])
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < dep:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, *srcs, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class Config(ctypes.Structure):
    _fields_ = [("voxel", ctypes.c_double), ("trunc", ctypes.c_double),
                ("r_c", ctypes.c_double), ("n_c", ctypes.c_int32),
                ("weight_cap", ctypes.c_int32), ("conf_min_w", ctypes.c_int32),
                ("cos_normal", ctypes.c_double), ("obs_dot", ctypes.c_double),
                ("vp_min_dist", ctypes.c_double), ("n_vp", ctypes.c_int32),
                ("knn_k", ctypes.c_int32), ("clamp_negative", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class ToolDesc(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("length", ctypes.c_double), ("corridor", ctypes.c_double),
                ("r_s", ctypes.c_double), ("radius", ctypes.c_double),
                ("width", ctypes.c_double), ("height", ctypes.c_double)]


class FrameStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_in", "n_valid", "n_dropped", "pairs_applied", "pairs_excluded",
                 "band_marks", "new_points", "n_points", "voxels_folded")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ScoreStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_points", "n_confident", "n_accessible", "n_blocked",
                 "n_no_candidate", "candidate_tests", "canonical_tests",
                 "canonical_lookups")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=False)
    L = ctypes.CDLL(_SO)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.orc_create.restype = vp
    L.orc_create.argtypes = [ctypes.POINTER(Config)]
    L.orc_destroy.argtypes = [vp]
    L.orc_set_roi.argtypes = [vp, vp, vp]
    L.orc_integrate_frame.restype = ctypes.c_int
    L.orc_integrate_frame.argtypes = [vp, vp, i64, vp, i64]
    L.orc_frame_stats_get.argtypes = [vp, ctypes.POINTER(FrameStats)]
    L.orc_num_voxels.restype = i64
    L.orc_num_voxels.argtypes = [vp]
    L.orc_read_tsdf.restype = i64
    L.orc_read_tsdf.argtypes = [vp, vp, vp, vp, vp, i64]
    L.orc_voxel.restype = ctypes.c_int
    L.orc_voxel.argtypes = [vp, i64, vp, vp, vp]
    L.orc_num_points.restype = i64
    L.orc_num_points.argtypes = [vp]
    L.orc_read_points.restype = i64
    L.orc_read_points.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64]
    L.orc_set_tool.restype = ctypes.c_int
    L.orc_set_tool.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ToolDesc), i32, vp]
    L.orc_set_tool_table.restype = ctypes.c_int
    L.orc_set_tool_table.argtypes = [vp, ctypes.c_int, i32, vp, vp, vp, vp]
    L.orc_tool_table.restype = i64
    L.orc_tool_table.argtypes = [vp, ctypes.c_int, i32, vp, vp, i64]
    L.orc_score.restype = ctypes.c_int
    L.orc_score.argtypes = [vp, ctypes.c_int, vp, i64]
    L.orc_score_allow.restype = ctypes.c_int
    L.orc_score_allow.argtypes = [vp, ctypes.c_int, vp, i64, vp]
    L.orc_score_stats_get.argtypes = [vp, ctypes.POINTER(ScoreStats)]
    L.orc_read_results.restype = i64
    L.orc_read_results.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32]
    L.orc_point_result.restype = ctypes.c_int
    L.orc_point_result.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32]
    L.orc_pca_axis.restype = ctypes.c_int
    L.orc_pca_axis.argtypes = [i64, vp, vp, vp]
    L.orc_pca_axes.restype = None
    L.orc_pca_axes.argtypes = [vp, i64, vp, vp]
    L.orc_isqrt.restype = i64
    L.orc_isqrt.argtypes = [i64]
    L.orc_floor_div.restype = i64
    L.orc_floor_div.argtypes = [i64, i64]
    L.orc_key.restype = i64
    L.orc_key.argtypes = [i64, i64, i64]
    L.orc_unkey.argtypes = [i64, vp]
    L.orc_params.argtypes = [vp, vp, vp, vp, vp, vp]
    L.orc_set_window.restype = ctypes.c_int
    L.orc_set_window.argtypes = [vp, vp]
    L.orc_window.restype = ctypes.c_int
    L.orc_window.argtypes = [vp, vp, vp, vp]
    L.orc_changed_voxels.restype = i64
    L.orc_changed_voxels.argtypes = [vp, vp, i64]
    L.orc_body_hits.restype = ctypes.c_int
    L.orc_body_hits.argtypes = [vp, ctypes.c_int, i64, i32]
    L.orc_smooth.restype = ctypes.c_int
    L.orc_smooth.argtypes = [vp, vp, vp, i64, vp, i32, dbl, dbl, vp, vp, vp, vp]
    L.orc_smooth_dense.restype = ctypes.c_int
    L.orc_smooth_dense.argtypes = [vp, vp, vp, dbl, dbl, vp, vp, i64, vp, i32, dbl, dbl,
                                   vp, vp, vp, vp]
    L.orc_smooth_refine.restype = ctypes.c_int
    L.orc_smooth_refine.argtypes = [vp, vp, i64, vp, i32, vp, i32, dbl, dbl, i32, dbl, dbl,
                                    vp, vp, vp]
    _lib = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def isqrt(n: int) -> int:
    return _load().orc_isqrt(int(n))


def pca_axis(cnt: int, sx, sxx):
    """(has, axis) of the oracle's PCA step for neighbourhood moments: cnt,
    sum d (3) and sum dd^T (00 01 02 11 12 22); axis in fixed point 2^30."""
    a = np.ascontiguousarray(sx, dtype=np.int64).reshape(3)
    b = np.ascontiguousarray(sxx, dtype=np.int64).reshape(6)
    out = np.zeros(3, np.int64)
    has = _load().orc_pca_axis(int(cnt), _p(a), _p(b), _p(out))
    return has, out


def pca_axes(moments):
    """pca_axis over rows [n][10] of (cnt, sum d [3], sum dd^T [6]):
    (axes [n][3], has [n])."""
    m = np.ascontiguousarray(moments, dtype=np.int32).reshape(-1, 10)
    axes = np.zeros((len(m), 3), np.int64)
    has = np.zeros(len(m), np.int32)
    _load().orc_pca_axes(_p(m), len(m), _p(axes), _p(has))
    return axes, has


def floor_div(a: int, b: int) -> int:
    return _load().orc_floor_div(int(a), int(b))


def key(x, y, z) -> int:
    return _load().orc_key(int(x), int(y), int(z))


def unkey(k: int):
    out = np.zeros(3, dtype=np.int64)
    _load().orc_unkey(int(k), _p(out))
    return out


def pack_keys(ijk: np.ndarray) -> np.ndarray:
    """Vectorised voxel key packing (21 bits per axis, biased by 2^20)."""
    ijk = np.asarray(ijk, dtype=np.int64)
    m = (1 << 21) - 1
    b = 1 << 20
    return ((ijk[..., 0] + b) & m) | (((ijk[..., 1] + b) & m) << 21) | \
        (((ijk[..., 2] + b) & m) << 42)


def unpack_keys(k: np.ndarray) -> np.ndarray:
    k = np.asarray(k, dtype=np.int64)
    m = (1 << 21) - 1
    b = 1 << 20
    return np.stack([(k & m) - b, ((k >> 21) & m) - b, ((k >> 42) & m) - b], axis=-1)


def make_config(voxel, trunc, r_c=0.01, n_c=5, weight_cap=2000, conf_min_w=2,
                cos_normal=0.3420201433256687, obs_dot=0.25, vp_min_dist=0.1,
                n_vp=8, knn_k=10, clamp_negative=0) -> Config:
    return Config(voxel, trunc, r_c, n_c, weight_cap, conf_min_w, cos_normal, obs_dot,
                  vp_min_dist, n_vp, knn_k, clamp_negative, 0)


def tool_desc(tool) -> ToolDesc:
    return ToolDesc(int(tool.shape), 0, tool.length, tool.corridor, tool.r_s,
                    tool.radius, tool.width, tool.height)


class Oracle:
    def __init__(self, cfg: Config | None = None, **kw):
        self.L = _load()
        self.cfg = cfg if cfg is not None else make_config(**kw)
        self.h = self.L.orc_create(ctypes.byref(self.cfg))
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        self.K = {}

    def close(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    __del__ = close

    def params(self):
        t, r, rc, dm = (ctypes.c_int64() for _ in range(4))
        sc = ctypes.c_double()
        self.L.orc_params(self.h, ctypes.byref(t), ctypes.byref(r), ctypes.byref(rc),
                          ctypes.byref(dm), ctypes.byref(sc))
        return dict(tau_u=t.value, R=r.value, rc_u=rc.value, dmin_u=dm.value,
                    scale=sc.value)

    def set_window(self, blocks):
        L = np.ascontiguousarray(blocks, dtype=np.int64).reshape(3)
        if self.L.orc_set_window(self.h, _p(L)) != 0:
            raise ValueError("oracle rejected the window")

    def window(self):
        """(lo, hi, shifts) of the window in blocks, or None before it is set."""
        lo = np.zeros(3, np.int64)
        hi = np.zeros(3, np.int64)
        sh = ctypes.c_int64()
        on = self.L.orc_window(self.h, _p(lo), _p(hi), ctypes.byref(sh))
        return (lo, hi, sh.value) if on else None

    def set_roi(self, lo, hi):
        lo = np.ascontiguousarray(lo, dtype=np.int64)
        hi = np.ascontiguousarray(hi, dtype=np.int64)
        self.L.orc_set_roi(self.h, _p(lo), _p(hi))

    def integrate_frame(self, xyz, origin, frame_id):
        xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
        rc = self.L.orc_integrate_frame(self.h, _p(xyz), len(xyz), _p(o), int(frame_id))
        if rc != 0:
            raise ValueError("oracle integrate_frame failed (%d)" % rc)

    def frame_stats(self):
        st = FrameStats()
        self.L.orc_frame_stats_get(self.h, ctypes.byref(st))
        return st.as_dict()

    def read_tsdf(self):
        n = self.L.orc_num_voxels(self.h)
        key = np.zeros(n, np.int64)
        S = np.zeros(n, np.int64)
        W = np.zeros(n, np.int32)
        c = np.zeros(n, np.uint8)
        self.L.orc_read_tsdf(self.h, _p(key), _p(S), _p(W), _p(c), n)
        return key, S, W, c

    def voxel(self, k):
        S = ctypes.c_int64()
        W = ctypes.c_int32()
        c = ctypes.c_uint8()
        self.L.orc_voxel(self.h, int(k), ctypes.byref(S), ctypes.byref(W), ctypes.byref(c))
        return S.value, W.value, c.value

    def num_points(self):
        return self.L.orc_num_points(self.h)

    def read_points(self):
        n = self.num_points()
        key = np.zeros(n, np.int64)
        ff = np.zeros(n, np.int32)
        nvp = np.zeros(n, np.int32)
        vp = np.zeros((n, 8, 3), np.int32)
        sq = np.zeros((n, 3), np.int64)
        nq = np.zeros(n, np.int32)
        self.L.orc_read_points(self.h, _p(key), _p(ff), _p(nvp), _p(vp), _p(sq), _p(nq), n)
        return dict(key=key, first_frame=ff, n_vp=nvp, vp=vp, sumq=sq, nq=nq)

    def set_tool(self, tool_id, tool, rot):
        rot = np.ascontiguousarray(rot, dtype=np.float64).reshape(-1, 9)
        d = tool_desc(tool)
        rc = self.L.orc_set_tool(self.h, int(tool_id), ctypes.byref(d), len(rot), _p(rot))
        if rc != 0:
            raise ValueError("oracle set_tool failed (%d)" % rc)
        self.K[tool_id] = len(rot)

    def set_tool_table(self, tool_id, dirs, offset_begin, off, cls):
        d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        b = np.ascontiguousarray(offset_begin, dtype=np.uint32).reshape(-1)
        o = np.ascontiguousarray(off, dtype=np.int16).reshape(-1, 3)
        c = np.ascontiguousarray(cls, dtype=np.uint8).reshape(-1)
        assert len(b) == len(d) + 1
        o1 = o if len(o) else np.zeros((1, 3), np.int16)
        c1 = c if len(c) else np.zeros(1, np.uint8)
        rc = self.L.orc_set_tool_table(self.h, int(tool_id), len(d), _p(d), _p(b), _p(o1), _p(c1))
        if rc != 0:
            raise ValueError("oracle set_tool_table rejected the table")
        self.K[tool_id] = len(d)

    def tool_table(self, tool_id, k):
        cap = 1 << 17
        off = np.zeros((cap, 3), np.int32)
        cls = np.zeros(cap, np.uint8)
        m = self.L.orc_tool_table(self.h, int(tool_id), int(k), _p(off), _p(cls), cap)
        if m < 0:
            raise ValueError("no such tool/orientation")
        return off[:m].copy(), cls[:m].copy()

    def score(self, tool_id, keys=None, allow=None):
        """Score every point, or the listed keys; allow ([len(keys),
        ceil(K/64)] uint64) restricts each listed point's orientations."""
        if allow is not None:
            k = np.ascontiguousarray(keys, dtype=np.int64)
            al = np.ascontiguousarray(allow, dtype=np.uint64).reshape(len(k), -1)
            rc = self.L.orc_score_allow(self.h, int(tool_id), _p(k), len(k), _p(al))
        elif keys is None:
            rc = self.L.orc_score(self.h, int(tool_id), None, 0)
        else:
            k = np.ascontiguousarray(keys, dtype=np.int64)
            rc = self.L.orc_score(self.h, int(tool_id), _p(k), len(k))
        if rc != 0:
            raise ValueError("oracle score failed (%d)" % rc)

    def score_stats(self):
        st = ScoreStats()
        self.L.orc_score_stats_get(self.h, ctypes.byref(st))
        return st.as_dict()

    def read_results(self, K):
        """Every point's result of the last score() in canonical order:
        label (255 = not evaluated), first_free, has_normal, normal [n, 3],
        mask [n, ceil(K/64)]."""
        n = self.num_points()
        mw = (K + 63) // 64
        lbl = np.zeros(max(n, 1), np.uint8)
        ff = np.zeros(max(n, 1), np.int32)
        hn = np.zeros(max(n, 1), np.int32)
        nrm = np.zeros((max(n, 1), 3), np.int64)
        mask = np.zeros((max(n, 1), mw), np.uint64)
        m = self.L.orc_read_results(self.h, n, _p(lbl), _p(ff), _p(hn), _p(nrm), _p(mask), mw)
        return dict(label=lbl[:m], first_free=ff[:m], has_normal=hn[:m], normal=nrm[:m],
                    mask=mask[:m])

    def point_result(self, key, K):
        mw = (K + 63) // 64
        lbl = ctypes.c_uint8()
        ff = ctypes.c_int32()
        hn = ctypes.c_int32()
        n = np.zeros(3, np.int64)
        m = np.zeros(mw, np.uint64)
        rc = self.L.orc_point_result(self.h, int(key), ctypes.byref(lbl), ctypes.byref(ff),
                                     _p(n), ctypes.byref(hn), _p(m), mw)
        if rc != 0:
            raise KeyError(key)
        return dict(label=lbl.value, first_free=ff.value, normal=n, has_normal=hn.value,
                    mask=m)

    def smooth(self, p, q, samples, c=0.01, tau_s=0.005):
        """The smoothed score on this oracle's map (see smooth_dense)."""
        p, q, smp = _f32(p, 3), _f32(q, 4), _f32(samples, 3)
        assert len(p) == len(q)
        s, dq, dp, face = _smooth_out(len(p))
        rc = self.L.orc_smooth(self.h, _p(p), _p(q), len(p), _p(smp), len(smp), float(c),
                               float(tau_s), _p(s), _p(dq), _p(dp), _p(face))
        if rc != 0:
            raise ValueError("orc_smooth rejected its arguments")
        return s, dq, dp, face


    def smooth_refine(self, p, q0, samples, steps, eta, max_step, c=0.01, tau_s=0.005):
        """Gradient ascent of the orientation from len(q0) / len(p) starts per
        point; returns (q, s, face) per (point, start)."""
        p, q0, smp = _f32(p, 3), _f32(q0, 4), _f32(samples, 3)
        S = len(q0) // max(1, len(p))
        assert S * len(p) == len(q0)
        q = np.zeros((len(q0), 4))
        s = np.zeros(len(q0))
        face = np.zeros(len(q0))
        rc = self.L.orc_smooth_refine(self.h, _p(p), len(p), _p(q0), S, _p(smp), len(smp),
                                      float(c), float(tau_s), int(steps), float(eta),
                                      float(max_step), _p(q), _p(s), _p(face))
        if rc != 0:
            raise ValueError("orc_smooth_refine rejected its arguments")
        return q, s, face

    def changed_voxels(self):
        """Keys of the voxels that received a contribution in the last frame."""
        m = self.L.orc_changed_voxels(self.h, None, 0)
        k = np.zeros(max(1, m), np.int64)
        self.L.orc_changed_voxels(self.h, _p(k), m)
        return k[:m]

    def body_hits(self, tool_id, key, k):
        r = self.L.orc_body_hits(self.h, int(tool_id), int(key), int(k))
        if r < 0:
            raise ValueError("bad tool, key or orientation")
        return r

    def labels(self, K, keys=None):
        """(keys, label, first_free) for all points (canonical order) or the
        listed keys."""
        if keys is None:
            keys = self.read_points()["key"]
        lbl = np.zeros(len(keys), np.uint8)
        ff = np.zeros(len(keys), np.int32)
        for i, k in enumerate(keys):
            r = self.point_result(k, K)
            lbl[i] = r["label"]
            ff[i] = r["first_free"]
        return np.asarray(keys), lbl, ff


# ---- smoothed clearance score (smooth.c) ----
def _f32(a, cols):
    return np.ascontiguousarray(a, dtype=np.float32).reshape(-1, cols)


def _smooth_out(n):
    return (np.zeros(n), np.zeros((n, 4)), np.zeros((n, 3)), np.zeros(n))


def smooth_dense(val, origin, v, tau, p, q, samples, c=0.01, tau_s=0.005):
    """s, ds/dq, ds/dp and the smallest sample-to-face distance (voxels) of
    each (p, q) pair on a dense voxel block val[k, j, i] whose voxel
    (0, 0, 0) is `origin`; voxels outside read tau."""
    val = np.ascontiguousarray(val, dtype=np.float64)
    dims = np.array(val.shape[::-1], np.int64)
    org = np.ascontiguousarray(origin, dtype=np.int64)
    p, q, smp = _f32(p, 3), _f32(q, 4), _f32(samples, 3)
    assert len(p) == len(q)
    s, dq, dp, face = _smooth_out(len(p))
    rc = _load().orc_smooth_dense(_p(val), _p(dims), _p(org), float(v), float(tau), _p(p),
                                  _p(q), len(p), _p(smp), len(smp), float(c), float(tau_s),
                                  _p(s), _p(dq), _p(dp), _p(face))
    if rc != 0:
        raise ValueError("orc_smooth_dense rejected its arguments")
    return s, dq, dp, face
