#!/usr/bin/env python3
"""Write tests/golden/tree_full.json: the oracle's whole-map state for the
tree workload at its full size (600 frames of 20,000 returns, v = 1 cm,
tau = 4 cm, saw box with 1 m corridor, K = 256), after 100, 300 and all 600
frames.  Calls only the oracle (and synth for the seeded inputs).

At each checkpoint the oracle (no region restriction) scores every point,
and the file records digests of the whole TSDF, the point records, every
point's label and first free orientation, normals and candidate masks, the
label counts and canonical statistics, plus 400 seeded sample points in full.
About 30 minutes of single-threaded CPU.  Run from the repository root:

    python3 tests/golden/make_tree_golden.py
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
from digest import labels_digest, masks_digest, normals_digest, points_digest, tsdf_digest  # noqa: E402

CHECKPOINTS = (100, 300, 600)
N_SAMPLE = 400


def main():
    oracle.build(force=False)
    synth.build(force=False)
    w = synth.tree()
    t = time.time()
    frames = w.frames(600)
    print("frames generated in %.1f s" % (time.time() - t), flush=True)
    K = len(w.rot)
    o = oracle.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
    o.set_tool(0, w.tool, w.rot)
    out = {"workload": "tree: synth.tree() defaults, frames 0..599, oracle without region",
           "orientations": K, "checkpoints": []}
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
        assert np.all(r["label"] != 255)
        rng = np.random.default_rng(1000 + i)
        idx = np.sort(rng.choice(len(pts["key"]), size=N_SAMPLE, replace=False))
        sample = [{"i": int(j), "key": int(pts["key"][j]), "label": int(r["label"][j]),
                   "first_free": int(r["first_free"][j]),
                   "has_normal": int(r["has_normal"][j]) if r["label"][j] else -1,
                   "normal": [int(x) for x in r["normal"][j]],
                   "mask": ["%016x" % int(x) for x in r["mask"][j]]} for j in idx]
        cp = {
            "frames": i + 1,
            "n_voxels": int(len(key)), "n_points": int(len(pts["key"])),
            "tsdf_sha": tsdf_digest(key, S, W, clr),
            "points_sha": points_digest(pts),
            "labels_sha": labels_digest(pts["key"], r["label"], r["first_free"]),
            "normals_sha": normals_digest(r["label"], r["has_normal"], r["normal"]),
            "masks_sha": masks_digest(r["label"], r["mask"]),
            "label_counts": {str(k): int((r["label"] == k).sum()) for k in range(4)},
            "score_stats": {k: int(v) for k, v in st.items()},
            "sample": sample,
        }
        out["checkpoints"].append(cp)
        print("checkpoint %d: %d points, labels %s, scored in %.0f s" %
              (i + 1, cp["n_points"], cp["label_counts"], time.time() - t), flush=True)
        with open(os.path.join(HERE, "tree_full.json"), "w") as fh:
            json.dump(out, fh, indent=0)
    print("done in %.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
