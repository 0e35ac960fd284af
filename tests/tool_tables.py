"""Caller-side construction of kernel tables (Section 3.4 "Tool kernel"):
the tool's point samples rotated into each orientation and voxelised, plus
the three arm samples along the approach direction.  Used by the tests as
the "caller" of the table form of both the oracle and the library."""
import math

import numpy as np

ARM = (0.6, 1.25, 2.25)


def _round_away(x):
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def table_from_points(body, far, rot, voxel, tau, r_s, shuffle_seed=None):
    """(dirs [K, 3], offset_begin [K + 1], off [n, 3] int16, cls [n] uint8).
    A sample t of orientation R lands in voxel offset floor(R t / v + 1/2)
    (the voxel holding the sample when the point sits at its voxel centre);
    offsets closer than r_s to the tip are dropped; duplicates merge."""
    rot = np.asarray(rot, np.float64).reshape(-1, 3, 3)
    dirs = rot[:, :, 0].copy()
    begin = [0]
    offs, clss = [], []
    rng = np.random.default_rng(shuffle_seed) if shuffle_seed is not None else None
    for R in rot:
        d = R[:, 0]
        near = np.array([_round_away(f * tau / voxel * d) for f in ARM], np.int64)
        rows, cl = [near], [np.full(3, 1)]
        for pts, c in ((body, 0), (far, 2)):
            o = np.floor((np.asarray(pts) @ R.T) / voxel + 0.5).astype(np.int64)
            o = np.unique(o, axis=0)
            o = o[np.sqrt((o.astype(np.float64) ** 2).sum(1)) * voxel >= r_s]
            rows.append(o)
            cl.append(np.full(len(o), c))
        o = np.concatenate(rows)
        c = np.concatenate(cl)
        if rng is not None:
            perm = rng.permutation(len(o))
            o, c = o[perm], c[perm]
        offs.append(o)
        clss.append(c)
        begin.append(begin[-1] + len(o))
    return (dirs, np.array(begin, np.uint32), np.concatenate(offs).astype(np.int16),
            np.concatenate(clss).astype(np.uint8))


def table_of_tool(reader, K):
    """The stored table of a tool, orientation by orientation, as a caller
    table: reader(k) -> (off [m, 3], cls [m])."""
    begin = [0]
    offs, clss = [], []
    for k in range(K):
        o, c = reader(k)
        offs.append(np.asarray(o))
        clss.append(np.asarray(c))
        begin.append(begin[-1] + len(o))
    return (np.array(begin, np.uint32), np.concatenate(offs).astype(np.int16),
            np.concatenate(clss).astype(np.uint8))
