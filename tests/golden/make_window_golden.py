#!/usr/bin/env python3
"""Write tests/golden/window_full.json: the oracle's state for the tree
workload at its full size (600 frames of 20,000 returns, v = 1 cm,
tau = 4 cm, saw box with 1 m corridor, K = 256) with a sliding window of
125 blocks (10 m) per axis, after 100, 300 and all 600 frames, scoring at
those three frames only (so points outside the window keep the labels of an
earlier checkpoint, or 255).  Calls only the oracle (and synth for the seeded
inputs).

Each checkpoint records the window box and its shift count, digests of the
whole TSDF, every point record, every point's label and first free
orientation, and the normals and candidate masks of the confident points
inside the window, the label counts and canonical statistics, plus 400
seeded points in full.  About 30 minutes of single-threaded CPU.  Run from
the repository root:

    python3 tests/golden/make_window_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import synth  # noqa: E402
from digest import (inside_window, labels_digest, masks_digest, normals_digest,  # noqa: E402
                    points_digest, tsdf_digest)

CHECKPOINTS = (100, 300, 600)
N_SAMPLE = 400
BLOCKS = 125


def main():
    oracle.build(force=False)
    synth.build(force=False)
    w = synth.tree()
    t = time.time()
    frames = w.frames(600)
    print("frames generated in %.1f s" % (time.time() - t), flush=True)
    K = len(w.rot)
    o = oracle.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    o.set_window([BLOCKS] * 3)
    o.set_tool(0, w.tool, w.rot)
    out = {"workload": "tree: synth.tree() defaults, frames 0..599, window of %d blocks, "
                       "scored at the checkpoints only" % BLOCKS,
           "orientations": K, "blocks": BLOCKS, "checkpoints": []}
    t0 = time.time()
    for i, f in enumerate(frames):
        o.integrate_frame(f.xyz, f.origin, f.frame_id)
        if (i + 1) % 25 == 0:
            print("integrated %d frames, %d points, %.0f s" % (i + 1, o.num_points(),
                                                               time.time() - t0), flush=True)
        if i + 1 not in CHECKPOINTS:
            continue
        t = time.time()
        o.score(0)
        r = o.read_results(K)
        st = o.score_stats()
        pts = o.read_points()
        key, S, W, clr = o.read_tsdf()
        lo, hi, shifts = o.window()
        ins = inside_window(pts["key"], lo, hi)
        rng = np.random.default_rng(2000 + i)
        idx = np.sort(rng.choice(len(pts["key"]), size=N_SAMPLE, replace=False))
        sample = [{"i": int(j), "key": int(pts["key"][j]), "label": int(r["label"][j]),
                   "first_free": int(r["first_free"][j]), "inside": bool(ins[j])}
                  for j in idx]
        cp = {
            "frames": i + 1,
            "window": [[int(x) for x in lo], [int(x) for x in hi], int(shifts)],
            "n_voxels": int(len(key)), "n_points": int(len(pts["key"])),
            "n_inside": int(ins.sum()),
            "tsdf_sha": tsdf_digest(key, S, W, clr),
            "points_sha": points_digest(pts),
            "labels_sha": labels_digest(pts["key"], r["label"], r["first_free"]),
            "normals_sha": normals_digest(r["label"][ins], r["has_normal"][ins],
                                          r["normal"][ins]),
            "masks_sha": masks_digest(r["label"][ins], r["mask"][ins]),
            "label_counts": {str(k): int((r["label"] == k).sum()) for k in (0, 1, 2, 3, 255)},
            "score_stats": {k: int(v) for k, v in st.items()},
            "sample": sample,
        }
        out["checkpoints"].append(cp)
        print("checkpoint %d: %d points (%d inside), labels %s, scored in %.0f s" %
              (i + 1, cp["n_points"], cp["n_inside"], cp["label_counts"], time.time() - t),
              flush=True)
        with open(os.path.join(HERE, "window_full.json"), "w") as fh:
            json.dump(out, fh, indent=0)
    print("done in %.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
