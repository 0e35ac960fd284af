"""Thin ctypes binding of libaf.so (include/af.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch supplies device memory and streams: pass a CUDA float32
tensor of shape [n, 3] to ``integrate_frame``; the current torch stream is
used unless another is given.  There is no fallback: if libaf.so is missing
or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libaf.so")

AF_OK, AF_EINVAL, AF_ENOMEM, AF_EDEVICE, AF_ENOTOOL, AF_EOVERFLOW, AF_EBUSY = 0, -1, -2, -3, -4, -5, -6
UNSCORED, ACCESSIBLE, BLOCKED, NO_CANDIDATE, TENTATIVE = 0, 1, 2, 3, 4
NOT_EVALUATED = 255   # sliding window: never scored
CLS_BODY, CLS_NEAR, CLS_FAR = 0, 1, 2
TOOL_CYLINDER, TOOL_BOX = 0, 1

_ERRNAMES = {AF_EINVAL: "AF_EINVAL", AF_ENOMEM: "AF_ENOMEM", AF_EDEVICE: "AF_EDEVICE",
             AF_ENOTOOL: "AF_ENOTOOL", AF_EOVERFLOW: "AF_EOVERFLOW", AF_EBUSY: "AF_EBUSY"}


class AFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "error"), code, msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("voxel", ctypes.c_double), ("trunc", ctypes.c_double),
                ("r_c", ctypes.c_double), ("n_c", ctypes.c_int32),
                ("weight_cap", ctypes.c_int32), ("conf_min_w", ctypes.c_int32),
                ("cos_normal", ctypes.c_double), ("obs_dot", ctypes.c_double),
                ("vp_min_dist", ctypes.c_double), ("n_vp", ctypes.c_int32),
                ("knn_k", ctypes.c_int32), ("clamp_negative", ctypes.c_int32),
                ("max_tools", ctypes.c_int32), ("max_blocks", ctypes.c_int64),
                ("max_points", ctypes.c_int64), ("max_orientations", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("hbm_budget", ctypes.c_int64)]


class Tool(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("length", ctypes.c_double), ("corridor", ctypes.c_double),
                ("r_s", ctypes.c_double), ("radius", ctypes.c_double),
                ("width", ctypes.c_double), ("height", ctypes.c_double)]


class KernelTable(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("dir", ctypes.c_void_p), ("offset_begin", ctypes.c_void_p),
                ("off", ctypes.c_void_p), ("cls", ctypes.c_void_p)]


class FrameStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_in", "n_valid", "n_dropped", "pairs_applied", "pairs_excluded",
                 "band_marks", "new_points", "n_points", "voxels_folded", "n_blocks",
                 "new_blocks")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ScoreStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_points", "n_confident", "n_accessible", "n_blocked",
                 "n_no_candidate", "candidate_tests", "canonical_tests",
                 "canonical_lookups", "deep_tests", "deep_chunks_max",
                                   "coarse_checks", "coarse_clear", "chunks_body",
                                   "chunks_far", "arm_lookups")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class IncrStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("new_points", "trig_i", "trig_ii", "trig_iii", "changed", "sampled",
                 "queued", "evaluated", "backlog", "budget")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("integrate_ms", "k_integrate_ms", "score_ms", "k_normals_ms",
                 "k_mask_ms", "k_score_ms")] + \
               [("integrate_calls", ctypes.c_int64), ("score_calls", ctypes.c_int64),
                ("k_smooth_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


# name -> (restype, argtypes); also used by the export test
_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
SIGNATURES = {
    "af_config_default": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.c_double, ctypes.c_double]),
    "af_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(_vp)]),
    "af_destroy": (ctypes.c_int, [_vp]),
    "af_last_error": (ctypes.c_char_p, [_vp]),
    "af_set_tool_kernels": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(Tool), _i32, _vp, _vp]),
    "af_integrate_frame": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _vp]),
    "af_integrate_frame_host": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _vp]),
    "af_set_window": (ctypes.c_int, [_vp, _vp]),
    "af_window_state": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "af_score_points": (ctypes.c_int, [_vp, _i32, _vp]),
    "af_read_labels": (ctypes.c_int, [_vp, _i32, _i64, _i64, _vp, _vp, _vp, _vp, _vp]),
    "af_num_points": (_i64, [_vp]),
    "af_num_blocks": (_i64, [_vp]),
    "af_read_tsdf": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    "af_read_points": (ctypes.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "af_read_tool_table": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _i64, _vp]),
    "af_read_point_debug": (ctypes.c_int, [_vp, _i32, _i64, _i64, _vp, _vp, _vp, _vp]),
    "af_pca_axes": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
    "af_set_tool_table": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(KernelTable), _vp]),
    "af_frame_stats_get": (ctypes.c_int, [_vp, ctypes.POINTER(FrameStats)]),
    "af_score_stats_get": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ScoreStats)]),
    "af_device_bytes": (_i64, [_vp]),
    "af_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "af_timing_read": (ctypes.c_int, [_vp, ctypes.POINTER(Timing), ctypes.c_int]),
    "af_score_variant_count": (ctypes.c_int, []),
    "af_score_tools": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "af_score_variant_default": (ctypes.c_int, []),
    "af_graph_prepare": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p]),
    "af_graph_frame": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "af_graph_slot": (ctypes.c_void_p, [ctypes.c_void_p]),
    "af_graph_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "af_smooth_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "af_smooth_eval_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_float, ctypes.c_float, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "af_smooth_refine": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "af_incremental_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "af_incremental_budget": (ctypes.c_int, [_vp, _i64, _i32, _i32]),
    "af_incremental_drain": (ctypes.c_int, [_vp, _i32, _vp]),
    "af_incremental_c2f": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double]),
    "af_incremental_frame": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "af_incremental_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "af_read_incremental": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "af_server_create": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]),
    "af_server_batch": (ctypes.c_int, [_vp, _i32]),
    "af_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "af_server_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "af_server_reserved": (ctypes.c_int64, [ctypes.c_void_p]),
    "af_server_admit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "af_server_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "af_server_context": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.c_int32]),
    "af_server_hip_stream": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.c_int32]),
    "af_server_prepare": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_int32]),
    "af_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64]),
    "af_server_pending": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "af_server_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "af_score_variant_name": (ctypes.c_char_p, [_i32]),
    "af_set_score_variant": (ctypes.c_int, [_vp, _i32]),
    "af_get_score_variant": (_i32, [_vp]),
    "af_tune_score": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp]),
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError("libaf.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def default_config(voxel: float, trunc: float = 0.0, **overrides) -> Config:
    cfg = Config()
    rc = lib().af_config_default(ctypes.byref(cfg), float(voxel), float(trunc))
    if rc != AF_OK:
        raise AFError(rc, "bad voxel size")
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def tool_struct(tool) -> Tool:
    g = (lambda k, d=0.0: tool[k] if isinstance(tool, dict) and k in tool
         else getattr(tool, k, d))
    return Tool(int(g("shape", 0)), 0, float(g("length")), float(g("corridor")),
                float(g("r_s")), float(g("radius")), float(g("width")), float(g("height")))


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def unpack_keys(keys) -> np.ndarray:
    """Voxel indices [n, 3] of packed voxel keys (21 bits per axis holding
    index + 2^20, x lowest; the layout include/af.h states)."""
    k = np.asarray(keys, dtype=np.int64)
    m = (1 << 21) - 1
    return np.stack([(k & m), ((k >> 21) & m), ((k >> 42) & m)], axis=1) - (1 << 20)


def _check_f32(t, shape, name):
    if not (getattr(t, "is_cuda", False) and str(t.dtype) == "torch.float32"
            and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise TypeError("%s must be a contiguous CUDA float32 tensor of shape %s" % (name, shape))


def window_blocks(size_m, voxel: float):
    """Blocks per axis of a window of size_m[a] metres: ceil(size / 8 v), at
    least 2."""
    return np.array([max(2, int(math.ceil(float(L) / (8.0 * voxel) - 1e-9))) for L in size_m],
                    np.int32)


def pca_axes(moments) -> tuple:
    """af_pca_axes: (axes [n][3] int64, has [n] int32) for neighbourhood
    moments [n][10] (count, sum d [3], sum dd^T [6])."""
    m = np.ascontiguousarray(moments, dtype=np.int32).reshape(-1, 10)
    axes = np.zeros((len(m), 3), np.int64)
    has = np.zeros(len(m), np.int32)
    rc = lib().af_pca_axes(_p(m), len(m), _p(axes), _p(has))
    if rc != AF_OK:
        raise AFError(rc, "af_pca_axes failed")
    return axes, has


class Context:
    """One accessibility-field map on the current GPU (af_ctx)."""

    def __init__(self, cfg: Config | None = None, voxel: float | None = None,
                 trunc: float = 0.0, **overrides):
        self._lib = lib()
        if cfg is None:
            cfg = default_config(voxel, trunc, **overrides)
        self.cfg = cfg
        h = ctypes.c_void_p()
        rc = self._lib.af_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != AF_OK:
            raise AFError(rc, "af_create failed")
        self.h = h
        self.K = {}

    @classmethod
    def _borrow(cls, lib_, handle, cfg, owner):
        """A context owned by a Server (not destroyed by this object)."""
        self = cls.__new__(cls)
        self._lib, self.cfg, self.h, self.K, self._owner = lib_, cfg, handle, {}, owner
        return self

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self.h = None
            return
        if getattr(self, "h", None):
            self._lib.af_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != AF_OK:
            raise AFError(rc, self._lib.af_last_error(self.h).decode())

    # ---- the four calls of the hot path ----
    def set_tool_kernels(self, tool_id: int, tool, rot, stream=None):
        rot = np.ascontiguousarray(rot, dtype=np.float64).reshape(-1, 9)
        t = tool_struct(tool)
        self._check(self._lib.af_set_tool_kernels(self.h, int(tool_id), ctypes.byref(t),
                                                  len(rot), _p(rot), _stream_handle(stream)))
        self.K[tool_id] = len(rot)

    def set_tool_table(self, tool_id: int, dirs, offset_begin, off, cls, stream=None):
        """Caller-built kernel table (af_set_tool_table): dirs [K, 3] float64,
        offset_begin [K + 1] uint32, off [n, 3] int16, cls [n] uint8."""
        d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        b = np.ascontiguousarray(offset_begin, dtype=np.uint32).reshape(-1)
        o = np.ascontiguousarray(off, dtype=np.int16).reshape(-1, 3)
        c = np.ascontiguousarray(cls, dtype=np.uint8).reshape(-1)
        if len(b) != len(d) + 1:
            raise ValueError("offset_begin needs K + 1 entries")
        t = KernelTable(len(d), 0, d.ctypes.data, b.ctypes.data,
                        o.ctypes.data if len(o) else None, c.ctypes.data if len(c) else None)
        self._check(self._lib.af_set_tool_table(self.h, int(tool_id), ctypes.byref(t),
                                                _stream_handle(stream)))
        self.K[tool_id] = len(d)

    def integrate_frame(self, xyz, origin, frame_id: int, stream=None):
        """xyz: CUDA float32 tensor [n, 3] (contiguous), or a host array
        (numpy, [n, 3] float32) that af_integrate_frame_host copies; origin:
        3 floats."""
        if isinstance(xyz, np.ndarray):
            x = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
            o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
            self._check(self._lib.af_integrate_frame_host(
                self.h, _p(x) if len(x) else None, len(x), _p(o), int(frame_id),
                _stream_handle(stream)))
            return
        if not (getattr(xyz, "is_cuda", False) and str(xyz.dtype) == "torch.float32"
                and xyz.is_contiguous() and xyz.dim() == 2 and xyz.shape[1] == 3):
            raise TypeError("xyz must be a contiguous CUDA float32 tensor of shape [n, 3]")
        o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
        self._check(self._lib.af_integrate_frame(self.h, ctypes.c_void_p(xyz.data_ptr()),
                                                 int(xyz.shape[0]), _p(o), int(frame_id),
                                                 _stream_handle(stream)))

    def set_window(self, blocks):
        """Sliding window of blocks[a] voxel blocks per axis (af_set_window);
        before the first frame.  `blocks` may also be derived from a size in
        metres with window_blocks()."""
        b = np.ascontiguousarray(blocks, dtype=np.int32).reshape(3)
        self._check(self._lib.af_set_window(self.h, _p(b)))

    def window_state(self):
        """(lo, hi, shifts) of the window in blocks, or None before its first
        placement."""
        lo = np.zeros(3, np.int32)
        hi = np.zeros(3, np.int32)
        sh = ctypes.c_int64()
        rc = self._lib.af_window_state(self.h, _p(lo), _p(hi), ctypes.byref(sh))
        if rc < 0:
            self._check(rc)
        return (lo, hi, sh.value) if rc == 1 else None

    def score_points(self, tool_id: int, stream=None):
        self._check(self._lib.af_score_points(self.h, int(tool_id), _stream_handle(stream)))

    def read_labels(self, tool_id: int, first: int = 0, count: int | None = None,
                    with_w: bool = False, out: dict | None = None, keys: bool = True):
        """Labels of points [first, first + count) in canonical order.  `out`
        may hold preallocated host arrays ("key" int64, "label" uint8,
        "first_free" int16, at least count long; pinned memory makes the copy
        fast), which are filled and returned as views; keys=False skips the
        keys."""
        n = self.num_points()
        count = n - first if count is None else count
        count = max(0, min(count, n - first))

        def buf(name, dtype):
            a = None if out is None else out.get(name)
            if a is None:
                return np.zeros(count, dtype)
            if a.dtype != dtype or not a.flags["C_CONTIGUOUS"] or len(a) < count:
                raise ValueError("out[%r]: need a contiguous %s array of at least %d"
                                 % (name, np.dtype(dtype).name, count))
            return a
        key = buf("key", np.int64) if keys else None
        lbl = buf("label", np.uint8)
        ff = buf("first_free", np.int16)
        w = np.zeros(count, np.uint16) if with_w else None
        nw = ctypes.c_int64()
        self._check(self._lib.af_read_labels(self.h, int(tool_id), int(first), int(count),
                                             _p(key) if keys else None, _p(lbl), _p(ff),
                                             _p(w) if with_w else None, ctypes.byref(nw)))
        res = dict(label=lbl[:nw.value], first_free=ff[:nw.value])
        if keys:
            res["key"] = key[:nw.value]
        if with_w:
            res["w"] = w[:nw.value]
        return res

    # ---- inspection ----
    def num_points(self) -> int:
        n = self._lib.af_num_points(self.h)
        if n < 0:
            self._check(AF_EDEVICE)
        return n

    def num_blocks(self) -> int:
        return self._lib.af_num_blocks(self.h)

    def device_bytes(self) -> int:
        return self._lib.af_device_bytes(self.h)

    def read_tsdf(self):
        n = ctypes.c_int64()
        self._check(self._lib.af_read_tsdf(self.h, None, None, None, None, 0, ctypes.byref(n)))
        m = n.value
        key = np.zeros(m, np.int64)
        S = np.zeros(m, np.int64)
        W = np.zeros(m, np.int32)
        c = np.zeros(m, np.uint8)
        self._check(self._lib.af_read_tsdf(self.h, _p(key), _p(S), _p(W), _p(c), m,
                                           ctypes.byref(n)))
        o = np.argsort(key)
        return key[o], S[o], W[o], c[o]

    def read_points(self):
        n = self.num_points()
        key = np.zeros(n, np.int64)
        ff = np.zeros(n, np.int32)
        nvp = np.zeros(n, np.int32)
        vp = np.zeros((n, 8, 3), np.int32)
        sq = np.zeros((n, 3), np.int64)
        nq = np.zeros(n, np.int32)
        nw = ctypes.c_int64()
        self._check(self._lib.af_read_points(self.h, 0, n, _p(key), _p(ff), _p(nvp), _p(vp),
                                             _p(sq), _p(nq), ctypes.byref(nw)))
        return dict(key=key, first_frame=ff, n_vp=nvp, vp=vp, sumq=sq, nq=nq)

    def read_tool_table(self, tool_id: int, k: int):
        m = ctypes.c_int64()
        self._check(self._lib.af_read_tool_table(self.h, int(tool_id), int(k), None, None, 0,
                                                 ctypes.byref(m)))
        off = np.zeros((m.value, 3), np.int32)
        cls = np.zeros(m.value, np.uint8)
        self._check(self._lib.af_read_tool_table(self.h, int(tool_id), int(k), _p(off),
                                                 _p(cls), m.value, ctypes.byref(m)))
        return off, cls

    def read_point_debug(self, tool_id: int, first: int = 0, count: int | None = None):
        n = self.num_points()
        count = n - first if count is None else count
        count = max(0, min(count, n - first))
        mw = (self.K[tool_id] + 63) // 64
        nrm = np.zeros((count, 3), np.int32)
        hn = np.zeros(count, np.int32)
        mask = np.zeros((count, mw), np.uint64)
        nw = ctypes.c_int64()
        self._check(self._lib.af_read_point_debug(self.h, int(tool_id), int(first), int(count),
                                                  _p(nrm), _p(hn), _p(mask), ctypes.byref(nw)))
        return dict(normal=nrm, has_normal=hn, mask=mask)

    def frame_stats(self):
        st = FrameStats()
        self._check(self._lib.af_frame_stats_get(self.h, ctypes.byref(st)))
        return st.as_dict()

    def timing_enable(self, on: bool = True):
        self._check(self._lib.af_timing_enable(self.h, 1 if on else 0))

    def timing_read(self, reset: bool = False):
        t = Timing()
        self._check(self._lib.af_timing_read(self.h, ctypes.byref(t), 1 if reset else 0))
        return t.as_dict()

    def score_variants(self):
        n = self._lib.af_score_variant_count()
        return [self._lib.af_score_variant_name(i).decode() for i in range(n)]

    def set_score_variant(self, v: int):
        self._check(self._lib.af_set_score_variant(self.h, int(v)))

    def score_variant(self) -> int:
        return self._lib.af_get_score_variant(self.h)

    def score_tools(self, tool_ids, stream=None):
        """Score every point against several tools in one launch."""
        ids = (ctypes.c_int32 * len(tool_ids))(*[int(x) for x in tool_ids])
        self._check(self._lib.af_score_tools(self.h, ids, len(tool_ids), _stream_handle(stream)))

    def graph_prepare(self, lo, hi, max_returns: int, tool_ids, stream=None):
        """Record one frame (integration of up to max_returns returns, then
        scoring of tool_ids in one launch) as a HIP graph; the brick grid
        covers the scene box [lo, hi] (metres).  With a sliding window the
        grid is the window's (lo and hi are checked but not used) and a frame
        that moves the window runs eagerly and records the graph again."""
        lo = np.ascontiguousarray(lo, dtype=np.float32).reshape(3)
        hi = np.ascontiguousarray(hi, dtype=np.float32).reshape(3)
        ids = (ctypes.c_int32 * len(tool_ids))(*[int(x) for x in tool_ids])
        self._check(self._lib.af_graph_prepare(self.h, _p(lo), _p(hi), int(max_returns), ids,
                                               len(tool_ids), _stream_handle(stream)))

    def graph_frame(self, xyz, origin, frame_id: int, stream=None):
        """Replay the recorded frame on xyz (contiguous CUDA float32 [n, 3])."""
        if not (getattr(xyz, "is_cuda", False) and str(xyz.dtype) == "torch.float32"
                and xyz.is_contiguous() and xyz.dim() == 2 and xyz.shape[1] == 3):
            raise TypeError("xyz must be a contiguous CUDA float32 tensor of shape [n, 3]")
        o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
        self._check(self._lib.af_graph_frame(self.h, ctypes.c_void_p(xyz.data_ptr()),
                                             int(xyz.shape[0]), _p(o), int(frame_id),
                                             _stream_handle(stream)))

    def graph_slot(self) -> int:
        """Device address of the recorded frame's input slot (0 if none)."""
        return int(self._lib.af_graph_slot(self.h) or 0)

    def graph_sync(self):
        """Wait for replayed frames and raise on any overflow they reported."""
        self._check(self._lib.af_graph_sync(self.h))

    def smooth_eval(self, p, q, samples, c=0.01, tau_s=0.005, grad_s=None, s=None, dq=None,
                    dp=None, stream=None):
        """Smoothed clearance score of the pairs (p[n, 3], q[n, 4]) into the
        given CUDA float32 outputs (s[n]; dq[n, 4] and dp[n, 3] together)."""
        n = int(p.shape[0])
        _check_f32(p, (n, 3), "p")
        _check_f32(q, (n, 4), "q")
        _check_f32(samples, (samples.shape[0], 3), "samples")
        for t, shp, name in ((grad_s, (n,), "grad_s"), (s, (n,), "s"), (dq, (n, 4), "dq"),
                             (dp, (n, 3), "dp")):
            if t is not None:
                _check_f32(t, shp, name)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        self._check(self._lib.af_smooth_eval(self.h, ptr(p), ptr(q), n, ptr(samples),
                                             int(samples.shape[0]), float(c), float(tau_s),
                                             ptr(grad_s), ptr(s), ptr(dq), ptr(dp),
                                             _stream_handle(stream)))

    def smooth_eval_static(self, p, q, samples, c=0.01, tau_s=0.005, grad_s=None, s=None,
                           dq=None, dp=None, stream=None):
        """smooth_eval through af_smooth_eval_static: the library allocates
        nothing during the call (its scratch is a static device array)."""
        n = int(p.shape[0])
        _check_f32(p, (n, 3), "p")
        _check_f32(q, (n, 4), "q")
        _check_f32(samples, (samples.shape[0], 3), "samples")
        for t, shp, name in ((grad_s, (n,), "grad_s"), (s, (n,), "s"), (dq, (n, 4), "dq"),
                             (dp, (n, 3), "dp")):
            if t is not None:
                _check_f32(t, shp, name)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        self._check(self._lib.af_smooth_eval_static(self.h, ptr(p), ptr(q), n, ptr(samples),
                                                    int(samples.shape[0]), float(c),
                                                    float(tau_s), ptr(grad_s), ptr(s), ptr(dq),
                                                    ptr(dp), _stream_handle(stream)))

    def smooth_refine(self, p, q0, samples, steps=20, eta=1e-3, max_step=0.05, c=0.01,
                      tau_s=0.005, stream=None):
        """Orientation ascent from q0[n_points * n_starts, 4]; returns (q, s)
        as new CUDA tensors."""
        import torch
        n = int(p.shape[0])
        _check_f32(p, (n, 3), "p")
        if n == 0 or q0.shape[0] % n:
            raise ValueError("q0 must hold n_starts quaternions per point")
        _check_f32(q0, (q0.shape[0], 4), "q0")
        _check_f32(samples, (samples.shape[0], 3), "samples")
        q = torch.empty_like(q0)
        s = torch.empty(q0.shape[0], device=q0.device, dtype=torch.float32)
        self._check(self._lib.af_smooth_refine(
            self.h, ctypes.c_void_p(p.data_ptr()), n, ctypes.c_void_p(q0.data_ptr()),
            q0.shape[0] // n, ctypes.c_void_p(samples.data_ptr()), int(samples.shape[0]),
            float(c), float(tau_s), int(steps), float(eta), float(max_step),
            ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(s.data_ptr()),
            _stream_handle(stream)))
        return q, s

    def incremental_enable(self, tool_id: int, budget: int):
        """Switch this (still empty) map to the incremental mode for one tool."""
        self._check(self._lib.af_incremental_enable(self.h, int(tool_id), int(budget)))

    def incremental_budget(self, lookup_target: int, b_min: int, b_max: int):
        self._check(self._lib.af_incremental_budget(self.h, int(lookup_target), int(b_min),
                                                    int(b_max)))

    def incremental_c2f(self, coarse_deg: float = 20.0, fine_deg: float = 25.0,
                        radius_m: float = 0.3):
        self._check(self._lib.af_incremental_c2f(self.h, float(coarse_deg), float(fine_deg),
                                                 float(radius_m)))

    def incremental_drain(self, max_evals: int, stream=None):
        self._check(self._lib.af_incremental_drain(self.h, int(max_evals),
                                                   _stream_handle(stream)))

    def incremental_frame(self, xyz, origin, frame_id: int, stream=None):
        """Integrate a frame, then re-evaluate only the queued points."""
        if not (getattr(xyz, "is_cuda", False) and str(xyz.dtype) == "torch.float32"
                and xyz.is_contiguous() and xyz.dim() == 2 and xyz.shape[1] == 3):
            raise TypeError("xyz must be a contiguous CUDA float32 tensor of shape [n, 3]")
        o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
        self._check(self._lib.af_incremental_frame(self.h, ctypes.c_void_p(xyz.data_ptr()),
                                                   int(xyz.shape[0]), _p(o), int(frame_id),
                                                   _stream_handle(stream)))

    def incremental_stats(self):
        st = IncrStats()
        self._check(self._lib.af_incremental_stats(self.h, ctypes.byref(st)))
        return st.as_dict()

    def read_incremental(self, labels_only: bool = False, first: int = 0,
                         label_out: np.ndarray | None = None, keys: bool = True):
        """Incremental state in canonical point order from point `first`:
        key, label, best (stored collision count; n_c = none), best_dir, a
        (only key and label with labels_only).  label_out: a preallocated
        uint8 host array (pinned memory makes the copy fast) for the labels;
        keys=False skips the keys."""
        n = max(0, self.num_points() - first)
        key = np.zeros(n, np.int64) if keys else None
        if label_out is not None:
            if label_out.dtype != np.uint8 or not label_out.flags["C_CONTIGUOUS"] \
                    or len(label_out) < n:
                raise ValueError("label_out: need a contiguous uint8 array of at least %d" % n)
            lbl = label_out[:n]
        else:
            lbl = np.zeros(n, np.uint8)
        kp = _p(key) if keys else None
        nw = ctypes.c_int64()
        if labels_only:
            self._check(self._lib.af_read_incremental(self.h, int(first), n, kp, _p(lbl), None,
                                                      None, None, ctypes.byref(nw)))
            return dict(key=key, label=lbl) if keys else dict(label=lbl)
        best = np.zeros(n, np.uint8)
        bdir = np.zeros(n, np.int16)
        a = np.zeros(n, np.float64)
        self._check(self._lib.af_read_incremental(self.h, int(first), n, kp, _p(lbl), _p(best),
                                                  _p(bdir), _p(a), ctypes.byref(nw)))
        out = dict(label=lbl, best=best, best_dir=bdir, a=a)
        if keys:
            out["key"] = key
        return out

    def score_variant_default(self) -> int:
        return self._lib.af_score_variant_default()

    def tune_score(self, tool_id: int, reps: int = 3, stream=None):
        """Time every scoring configuration on the current map; keep the
        fastest.  Returns (best index, per-configuration ms)."""
        n = self._lib.af_score_variant_count()
        ms = (ctypes.c_float * n)()
        best = ctypes.c_int32()
        self._check(self._lib.af_tune_score(self.h, int(tool_id), int(reps),
                                            _stream_handle(stream), ctypes.byref(best), ms))
        return best.value, list(ms)

    def score_stats(self, tool_id: int):
        st = ScoreStats()
        self._check(self._lib.af_score_stats_get(self.h, int(tool_id), ctypes.byref(st)))
        return st.as_dict()


class Server:
    """Several sensor streams on one GPU (af_server): admission by device
    budget, one context, HIP stream, recorded frame graph and frame queue per
    stream, and a step that runs the oldest queued frame of every stream."""

    def __init__(self, hbm_budget: int, max_streams: int = 4, batch=None):
        """batch: None keeps the library's default (no cross-stream scoring
        launch), True batches every step of 2 or more streams, False never,
        an int sets the minimum number of streams (af_server_batch)."""
        self._lib = lib()
        h = ctypes.c_void_p()
        rc = self._lib.af_server_create(int(hbm_budget), int(max_streams), ctypes.byref(h))
        if rc != AF_OK:
            raise AFError(rc, "af_server_create failed")
        self.h = h
        self.max_streams = int(max_streams)
        self._ctx = {}
        if batch is not None:
            m = (2 if batch else 0) if isinstance(batch, bool) else int(batch)
            self._check(self._lib.af_server_batch(self.h, m))

    def close(self):
        if getattr(self, "h", None):
            for c in self._ctx.values():
                c.h = None
            self._ctx.clear()
            self._lib.af_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != AF_OK:
            raise AFError(rc, self._lib.af_server_last_error(self.h).decode())

    def reserved(self) -> int:
        return int(self._lib.af_server_reserved(self.h))

    def admit(self, cfg: Config) -> int:
        sid = ctypes.c_int32()
        self._check(self._lib.af_server_admit(self.h, ctypes.byref(cfg), ctypes.byref(sid)))
        handle = ctypes.c_void_p(self._lib.af_server_context(self.h, sid.value))
        self._ctx[sid.value] = Context._borrow(self._lib, handle, cfg, self)
        return sid.value

    def release(self, sid: int):
        self._check(self._lib.af_server_release(self.h, int(sid)))
        c = self._ctx.pop(int(sid), None)
        if c is not None:
            c.h = None

    def context(self, sid: int) -> Context:
        return self._ctx[int(sid)]

    def hip_stream(self, sid: int) -> int:
        return int(self._lib.af_server_hip_stream(self.h, int(sid)) or 0)

    def prepare(self, sid: int, lo, hi, max_returns: int, tool_ids):
        """Record the stream's frame graph (see Context.graph_prepare); a
        context in the incremental mode records none and takes a device slot
        of max_returns returns instead."""
        lo = np.ascontiguousarray(lo, dtype=np.float32).reshape(3)
        hi = np.ascontiguousarray(hi, dtype=np.float32).reshape(3)
        ids = (ctypes.c_int32 * len(tool_ids))(*[int(x) for x in tool_ids])
        self._check(self._lib.af_server_prepare(self.h, int(sid), _p(lo), _p(hi),
                                                int(max_returns), ids, len(tool_ids)))

    def submit(self, sid: int, xyz, origin, frame_id: int):
        """xyz: host float32 array [n, 3]; it is copied before the call returns."""
        x = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
        self._check(self._lib.af_server_submit(self.h, int(sid), _p(x), len(x), _p(o),
                                               int(frame_id)))

    def pending(self, sid: int) -> int:
        return int(self._lib.af_server_pending(self.h, int(sid)))

    def step(self):
        """Run the oldest queued frame of every stream; [(stream, frame id, status)]."""
        n = self.max_streams
        sids = (ctypes.c_int32 * n)()
        fids = (ctypes.c_int64 * n)()
        st = (ctypes.c_int32 * n)()
        nd = ctypes.c_int32()
        self._check(self._lib.af_server_step(self.h, sids, fids, st, n, ctypes.byref(nd)))
        return [(sids[i], fids[i], st[i]) for i in range(nd.value)]

    def last_error(self) -> str:
        return self._lib.af_server_last_error(self.h).decode()
