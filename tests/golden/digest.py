"""Digests of whole-map state for the full-size golden files: SHA-256 over
the arrays in a fixed order and dtype.  Holds no arithmetic of the method;
the golden writer (oracle side) and the GPU test (library side) both call
these on their own outputs."""
import hashlib

import numpy as np


def _sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def tsdf_digest(key, S, W, cleared):
    key = np.asarray(key, np.int64)
    o = np.argsort(key, kind="stable")
    return _sha(key[o], np.asarray(S, np.int64)[o], np.asarray(W, np.int64)[o],
                np.asarray(cleared, np.int64)[o])


def points_digest(p):
    return _sha(*(np.asarray(p[k], np.int64) for k in ("key", "first_frame", "n_vp", "vp",
                                                      "sumq", "nq")))


def labels_digest(key, label, first_free):
    return _sha(np.asarray(key, np.int64), np.asarray(label, np.int64),
                np.asarray(first_free, np.int64))


def normals_digest(label, has_normal, normal):
    """has_normal and normal of confident points (label != 0); unscored
    points enter as (-1, 0, 0, 0)."""
    label = np.asarray(label)
    hn = np.where(label == 0, -1, np.asarray(has_normal, np.int64))
    nrm = np.where((label == 0)[:, None], 0, np.asarray(normal, np.int64))
    return _sha(hn, nrm)


def masks_digest(label, mask):
    """Candidate masks of confident points; unscored points enter as 0."""
    label = np.asarray(label)
    m = np.where((np.asarray(label) == 0)[:, None], np.uint64(0), np.asarray(mask, np.uint64))
    return _sha(m)


def inside_window(keys, lo, hi):
    """Whether each point key's voxel lies in the block box [lo, hi] (key
    unpacking only: 21 bits per axis, biased by 2^20)."""
    k = np.asarray(keys, np.int64)
    m = (1 << 21) - 1
    v = np.stack([(k & m) - (1 << 20), ((k >> 21) & m) - (1 << 20),
                  ((k >> 42) & m) - (1 << 20)], axis=1)
    b = np.floor_divide(v, 8)
    return np.all((b >= np.asarray(lo)) & (b <= np.asarray(hi)), axis=1)
