#!/usr/bin/env python3
"""Benchmark of the accessibility-field hot path on one MI355X.

Workload (tree): a procedural 8 m tree (40 cm trunk, 5 branching levels,
branch radii 1-15 cm) scanned by a Mid-360-shaped sensor on a seeded orbiting,
climbing trajectory: 20,000 returns per frame at 10 Hz, range noise 2 cm;
1 cm voxels, 4 cm truncation; a 30 x 5 x 2 cm saw-box tool with a 1 m
corridor at 256 orientations (64 Fibonacci directions x 4 rolls).

One step = one frame through the whole hot path: integrate_frame (scan-centric
TSDF integration, ray-cleared band, surface points, fold) then score_points
(normals, candidate masks, collision-count search for every confident point).
The K timed frames are centred on frame 300 of the 600-frame sequence (never
before frame 100 or before --warmup): frames 0..F0-1 are an untimed pre-roll
(integrate + score), frames F0..F0+K-1 are timed back to back with their
returns already in HBM.  Frame latency (release -> labels on the host) is then
measured on a fresh map by replaying the sequence's first L frames (default:
all 600) at 10 Hz from pinned host memory.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("point×orientation tests/s + returns integrated/s; p99 frame latency @10 Hz")
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_score_tree.json")
SCORE_SRC = os.path.join(ROOT, "paper_2608_06412_amd", "csrc", "af_score.hip")
SMOOTH_SRC = os.path.join(ROOT, "paper_2608_06412_amd", "csrc", "af_smooth.hip")
SMOOTH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_smooth_refine.json")
# kernels whose per-launch device time the bench reports (symbol prefixes)
TRACE_KERNELS = ("k_score", "k_integrate_fold", "k_normals", "k_mask")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def score_bytes(lookups, confident, K):
    """Algorithmic bytes of the scoring step: an 8-byte voxel record per
    canonical lookup plus, per confident point, its key (8), candidate mask
    (K/8), weight (4) and outputs (3)."""
    return 8.0 * lookups + confident * (8 + K / 8 + 4 + 3)


def kscore_bytes(lookups, arm_lookups, confident, K):
    """The scoring kernel's own share: canonical lookups less the arm samples
    whose result the mask kernel precomputed, plus per confident point its
    key, mask and the two arm-sample planes (3 K/8), weight and outputs."""
    return 8.0 * (lookups - arm_lookups) + confident * (8 + 3 * K / 8 + 4 + 3)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _in_thread(fn, core):
    """Run fn() in a thread pinned to one host core (Linux affinity is per
    thread, so the process's other threads keep theirs); returns fn's value."""
    import threading
    box = {}

    def body():
        try:
            os.sched_setaffinity(0, {core})
        except (AttributeError, OSError):
            pass
        try:
            box["v"] = fn()
        except BaseException as e:   # re-raised in the caller
            box["e"] = e
    th = threading.Thread(target=body)
    th.start()
    th.join()
    if "e" in box:
        raise box["e"]
    return box["v"]


def cpu_baseline(w, frames, n_frames, n_points, seed=17, max_threads=16):
    """The oracle, unchanged: single-threaded on one pinned host core, then
    the same scoring loop on several cores over disjoint slices of the same
    seeded point sample (each thread with its own oracle holding the same
    map, since a scoring call owns its oracle's result arrays)."""
    import concurrent.futures as cf

    import oracle
    oracle.build(force=False)
    cores = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else [0]

    def make_map():
        orc = oracle.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
        t = time.perf_counter()
        nret = 0
        for f in frames[:n_frames]:
            orc.integrate_frame(f.xyz, f.origin, f.frame_id)
            nret += len(f.xyz)
        orc.set_tool(0, w.tool, w.rot)
        return orc, nret, time.perf_counter() - t

    def score(orc, keys):
        t = time.perf_counter()
        orc.score(0, keys=keys)
        return orc.score_stats()["canonical_tests"], time.perf_counter() - t

    orc, nret, t_int = _in_thread(make_map, cores[0])
    keys = orc.read_points()["key"]
    rng = np.random.default_rng(seed)
    sample = rng.choice(keys, size=min(n_points, len(keys)), replace=False)
    tests, t_score = _in_thread(lambda: score(orc, sample), cores[0])
    out = {
        "value": tests / t_score,
        "unit": "point-orientation tests/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("single-threaded C oracle pinned to host core %d: frames 0-%d of the tree "
                   "workload integrated (%d returns, %.1f s -> %.0f returns/s), then %d "
                   "seeded-random points of that map scored against all %d orientations "
                   "(%d canonical tests in %.1f s)"
                   % (cores[0], n_frames - 1, nret, t_int, nret / t_int, len(sample),
                      len(w.rot), tests, t_score)),
        "returns_per_s": nret / t_int,
        "cpu_model": _cpu_model(),
        "host_cpus_visible": len(cores),
    }
    # all cores of this process's share (at most max_threads): maps built in
    # parallel, then the timed scoring of disjoint slices
    P = max(1, min(max_threads, len(cores)))
    slices = np.array_split(sample, P)
    with cf.ThreadPoolExecutor(P) as ex:
        maps = list(ex.map(lambda c: _pinned_call(make_map, c), cores[:P]))
        t = time.perf_counter()
        res = list(ex.map(lambda a: _pinned_call(lambda: score(a[0][0], a[1]), a[2]),
                          zip(maps, slices, cores[:P])))
        wall = time.perf_counter() - t
    tests_all = sum(r[0] for r in res)
    out["all_cores"] = {
        "value": tests_all / wall, "unit": "point-orientation tests/s", "cores": P,
        "kind": "oracle", "same_tests": bool(tests_all == tests),
        "sample": ("the same %d points in %d disjoint slices, one oracle per thread, each "
                   "thread pinned to its own host core (%d canonical tests in %.1f s wall)"
                   % (len(sample), P, tests_all, wall)),
    }
    return out


def _pinned_call(fn, core):
    try:
        os.sched_setaffinity(0, {core})
    except (AttributeError, OSError):
        pass
    return fn()


def tree_window(warmup, steps):
    """First timed frame of the tree workload: the timed frames are centred on
    frame 300 of the 600-frame sequence, and start no earlier than frame 100
    or than `warmup`."""
    return max(warmup, 100, 300 - steps // 2)


def trace_summary(csv_path, warmup, steps):
    """Per-launch device time of the hot kernels from a rocprofv3 kernel-trace
    CSV of a tree bench run with the same --warmup/--steps: mean over all
    launches and over the timed frames' launches only (one launch per frame,
    frames F0..F0+steps-1 with F0 = tree_window(warmup, steps))."""
    first = tree_window(warmup, steps)
    import csv
    per = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            m = re.search(r"\b(k_[A-Za-z0-9_]+)\s*[<(]", name)
            if not m:
                continue
            base = m.group(1)
            for fam in ("k_score", "k_mask"):   # kernel variants reported under one name
                if base.startswith(fam):
                    base = fam
            if base not in TRACE_KERNELS:
                continue
            per.setdefault(base, []).append(
                (int(row["Start_Timestamp"]), int(row["End_Timestamp"]), name))
    out = {}
    for base, rows in per.items():
        rows.sort()
        d = np.array([(e - b) / 1e6 for b, e, _ in rows])
        timed = d[first:first + steps]
        out[base] = {"launches": int(len(d)), "avg_ms_all": float(d.mean()),
                     "timed_frames": [first, first + steps - 1],
                     "avg_ms_timed": float(timed.mean()) if len(timed) else None,
                     "timed_launches": int(len(timed)), "symbol": rows[0][2][:120]}
    return out


def _counter_rows(csv_path, counter):
    """(start time, kernel name, value) of every dispatch in a rocprofv3
    counter-collection CSV (values of one dispatch summed)."""
    import csv
    per = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            key = row["Dispatch_Id"]
            if key not in per:
                per[key] = [int(row["Start_Timestamp"]), row["Kernel_Name"], 0.0]
            per[key][2] += float(row["Counter_Value"])
    return sorted(per.values())


TRAFFIC_TARGETS = {
    # workload: (kernel name pattern, source file, traffic file, description)
    "tree": (r"\bk_score[A-Za-z0-9_]*\s*[<(]", "SCORE", "traffic_k_score_tree.json",
             "k_score (default scoring configuration)"),
    "smooth": (r"\bk_smooth_refine\s*[<(]", "SMOOTH", "traffic_k_smooth_refine.json",
               "k_smooth_refine"),
}


def traffic_summary(paths, warmup, steps, copy_bytes, workload="tree"):
    """The traffic file of a workload's dominant kernel from four rocprofv3
    --pmc CSVs: FETCH_SIZE and WRITE_SIZE of a bench run of that workload
    (the kernel's timed launches warmup..warmup+steps-1), and of the copy
    probe of copy_bytes, which fixes the KiB-per-byte scale of each counter."""
    fetch, write, cfetch, cwrite = paths
    pattern, src_key, fname, desc = TRAFFIC_TARGETS[workload]
    src = SCORE_SRC if src_key == "SCORE" else SMOOTH_SRC

    first = tree_window(warmup, steps) if workload == "tree" else warmup

    def score_mean(path, counter):
        rows = [v for _, name, v in _counter_rows(path, counter) if re.search(pattern, name)]
        timed = rows[first:first + steps]
        return float(np.mean(timed)), len(rows)

    def copy_kib(path, counter):
        rows = [v for _, name, v in _counter_rows(path, counter) if "copyBuffer" in name]
        return float(np.median(rows))
    f_kib, nf = score_mean(fetch, "FETCH_SIZE")
    w_kib, nw = score_mean(write, "WRITE_SIZE")
    # a copy of B bytes reads B and writes B: scale = B / (counter KiB * 1024)
    f_scale = copy_bytes / (copy_kib(cfetch, "FETCH_SIZE") * 1024.0)
    w_scale = copy_bytes / (copy_kib(cwrite, "WRITE_SIZE") * 1024.0)
    out = {
        "kernel": desc,
        "workload": "%s, launches %d-%d (timed launches of bench.py --warmup %d --steps %d)" % (
            workload, first, first + steps - 1, warmup, steps),
        "window": [first, first + steps - 1],
        "file": fname,
        "src_sha": src_sha(src),
        "fetch_kib_per_launch": f_kib, "write_kib_per_launch": w_kib,
        "fetch_scale": round(f_scale, 3), "write_scale": round(w_scale, 3),
        "bytes_per_launch": (f_kib * f_scale + w_kib * w_scale) * 1024.0,
        "launches_seen": [nf, nw],
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE -d <dir> -o p --output-format csv -- python3 bench.py "
            "--workload %s --warmup %d --steps %d --no-cpu-baseline --latency-frames 0" % (
                workload, warmup, steps),
            "rocprofv3 --pmc WRITE_SIZE -d <dir> -o p --output-format csv -- python3 bench.py "
            "--workload %s --warmup %d --steps %d --no-cpu-baseline --latency-frames 0" % (
                workload, warmup, steps),
            "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -d <dir> -o p --output-format csv -- "
            "python3 bench.py --copy-probe %d" % copy_bytes,
            "python3 bench.py --workload %s --warmup %d --steps %d --traffic-summary "
            "fetch.csv,write.csv,copy_fetch.csv,copy_write.csv" % (workload, warmup, steps)],
    }
    return out


def run_batch(args):
    """Batching workload: the tree scene with frames of 5,000-40,000 returns,
    eight seeded tools x 512 orientations scored in one persistent launch per
    frame.  Frames 0..W-1 warm up, W..W+K-1 are timed (integrate + score all
    tools).  Then, on the final map, one multi-tool launch is timed against
    eight per-tool launches and their labels are compared."""
    import torch
    import synth
    from paper_2608_06412_amd import Context, default_config

    W = args.warmup if args.warmup != 100 else 40
    K = args.steps if args.steps != 400 else 40
    w = synth.batch(n_frames=W + K)
    tools = synth.batch_tools()
    t = time.perf_counter()
    frames = w.frames(W + K)
    log("generated %d frames (%d-%d returns) in %.1f s" %
        (W + K, min(len(f.xyz) for f in frames), max(len(f.xyz) for f in frames),
         time.perf_counter() - t))
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    resident = [torch.from_numpy(f.xyz).to(dev) for f in frames]
    cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 17, max_points=1 << 22,
                         max_orientations=len(w.rot), max_tools=len(tools))
    ctx = Context(cfg)
    for i, tl in enumerate(tools):
        ctx.set_tool_kernels(i, tl, w.rot)
    ids = list(range(len(tools)))
    for i in range(W):
        ctx.integrate_frame(resident[i], frames[i].origin, frames[i].frame_id)
        ctx.score_tools(ids)
        if i % 10 == 0:
            log("warm-up frame %d, %d points" % (i, ctx.num_points()))
    ctx.timing_enable(True)
    ctx.timing_read(reset=True)
    tests = lookups = returns = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W, W + K):
        ctx.integrate_frame(resident[i], frames[i].origin, frames[i].frame_id)
        ctx.score_tools(ids)
        for j in ids:
            st = ctx.score_stats(j)
            tests += st["canonical_tests"]
            lookups += st["canonical_lookups"]
        returns += len(frames[i].xyz)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ctx.timing_read(reset=True)
    log("timed %d frames in %.2f s" % (K, wall))

    # one launch for all tools against one launch per tool, on the final map
    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / reps * 1e3
    ctx.timing_enable(False)
    ms_multi = timed(lambda: ctx.score_tools(ids))
    multi = [ctx.read_labels(j) for j in ids]
    ms_single = timed(lambda: [ctx.score_points(j) for j in ids])
    same = all(np.array_equal(multi[j]["label"], ctx.read_labels(j)["label"]) and
               np.array_equal(multi[j]["first_free"], ctx.read_labels(j)["first_free"])
               for j in ids)
    # the same frames through the recorded per-frame graph on a second context
    rec = Context(cfg)
    for i, tl in enumerate(tools):
        rec.set_tool_kernels(i, tl, w.rot)
    allx = np.concatenate([f.xyz for f in frames])
    rec.graph_prepare(allx.min(0) - 1.0, allx.max(0) + 1.0, max(len(f.xyz) for f in frames), ids)
    for i in range(W):
        rec.graph_frame(resident[i], frames[i].origin, frames[i].frame_id)
    rec.graph_sync()
    gtests = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W, W + K):
        rec.graph_frame(resident[i], frames[i].origin, frames[i].frame_id)
        rec.graph_sync()
        for j in ids:
            gtests += rec.score_stats(j)["canonical_tests"]
    torch.cuda.synchronize()
    gwall = time.perf_counter() - t0
    gsame = all(np.array_equal(ctx.read_labels(j)["label"], rec.read_labels(j)["label"]) and
                np.array_equal(ctx.read_labels(j)["first_free"], rec.read_labels(j)["first_free"])
                for j in ids)
    log("recorded frames: %.2f ms/frame (eager %.2f)" % (gwall / K * 1e3, wall / K * 1e3))
    out = {
        "metric": "point\u00d7orientation tests/s, 8 tools x 512 orientations",
        "value": tests / wall,
        "unit": "point-orientation tests/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "batch: the tree scene, frames of 5,000-40,000 returns (seeded "
                               "uniform), 8 seeded tools (cylinders and boxes, 2-8 cm "
                               "cross-sections, 0.3-1.5 m corridors) x 512 orientations "
                               "(128 directions x 4 rolls), all tools in one scoring launch",
                   "frames_timed": [W, W + K - 1], "tools": len(tools),
                   "orientations": len(w.rot), "map_points_end": int(ctx.num_points())},
        "returns_integrated_per_s": returns / (tm["integrate_ms"] / 1e3),
        "canonical_lookups_per_s": lookups / wall,
        "stage_ms_per_step": {"integrate": tm["integrate_ms"] / K, "score": tm["score_ms"] / K,
                              "k_normals": tm["k_normals_ms"] / K,
                              "k_mask_all_tools": tm["k_mask_ms"] / K,
                              "k_score_all_tools": tm["k_score_ms"] / K},
        "one_launch_vs_per_tool": {"ms_one_launch": ms_multi, "ms_per_tool_launches": ms_single,
                                   "speedup": ms_single / ms_multi,
                                   "labels_identical": bool(same)},
        "recorded_graph": {"ms_per_step": gwall / K * 1e3, "tests_per_s": gtests / gwall,
                           "eager_ms_per_step": wall / K * 1e3,
                           "same_tests": bool(gtests == tests),
                           "labels_identical": bool(gsame)},
    }
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Serving workload: four concurrent streams (trees and box clusters, own
    tools at 256 orientations, frames of 5,000-40,000 returns at 10 Hz, TSDF
    capacity 2e8 voxels each) admitted by a 24 GiB device budget (6 GiB per
    stream; a fifth stream is refused).  Frames 0..W-1 warm up; W..W+K-1 are
    run back to back, one frame of every stream per server step, against the
    plain sequential path (per frame: integrate, score, wait) on four other
    contexts, and against servers that batch every step's scoring into one
    launch and that never do; W+K..W+K+L-1 (default 150 per stream, 600
    frames) arrive at 10 Hz from each stream's phase, and the latency of each
    frame runs from its arrival to its labels on the host.  The main server
    keeps the library's default (each stream scored on its own stream, no
    cross-stream launch).  With --serve-incremental B every context (served and
    sequential) runs the incremental mode with a budget of B evaluations per
    frame, and labels are the incremental mode's."""
    import torch
    import synth
    from paper_2608_06412_amd import AFError, Context, Server, default_config

    W = args.warmup if args.warmup != 100 else 20
    K = args.steps if args.steps != 400 else 40
    L = args.latency_frames if args.latency_frames != 600 else 150
    n = W + K + L
    NS = args.serve_streams
    INC = args.serve_incremental

    def frame_on(c, x, f):
        if INC:
            c.incremental_frame(x, f.origin, f.frame_id)
        else:
            c.integrate_frame(x, f.origin, f.frame_id)
            c.score_points(0)

    def read_out(c):
        return c.read_incremental(labels_only=True) if INC else c.read_labels(0)
    specs = synth.serving(n_streams=NS, n_frames=n)
    t = time.perf_counter()
    frames = [sp.workload.frames(n) for sp in specs]
    log("generated %d x %d frames in %.1f s" % (NS, n, time.perf_counter() - t))
    torch.cuda.set_device(0)
    GiB = 1 << 30

    # four streams: 2e8 voxels and 4 M points each in 6 GiB; more streams
    # share the same 24 GiB with proportionally smaller maps
    per = 4.0 / NS

    def cfg(budget):
        w = specs[0].workload
        c = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=int(390625 * per),
                           max_points=int((1 << 22) * per), max_orientations=256, max_tools=1)
        c.hbm_budget = int(budget)
        return c
    stream_budget = int(6 * GiB * per)

    def make_server(batch):
        srv = Server(24 * GiB, max_streams=NS + 1, batch=batch)
        sids = [srv.admit(cfg(stream_budget)) for _ in specs]
        try:
            srv.admit(cfg(stream_budget))
            refused = False
        except AFError:
            refused = True
        for s, sp in enumerate(specs):
            w = sp.workload
            allx = np.concatenate([f.xyz for f in frames[s]])
            srv.context(sids[s]).set_tool_kernels(0, w.tool, w.rot)
            if INC:
                srv.context(sids[s]).incremental_enable(0, INC)
            srv.prepare(sids[s], allx.min(0) - 1.0, allx.max(0) + 1.0,
                        max(len(f.xyz) for f in frames[s]), [0])
        return srv, sids, refused

    # the server with the library's default (each stream scored on its own
    # stream), the server that batches every step, the one that never does
    # (explicitly), and the plain sequential path
    srv, sids, refused = make_server(None)
    srv_b, sids_b, _ = make_server(True)
    srv_o, sids_o, _ = make_server(False)
    seq = []
    for s, sp in enumerate(specs):
        w = sp.workload
        c = Context(cfg(0))
        c.set_tool_kernels(0, w.tool, w.rot)
        if INC:
            c.incremental_enable(0, INC)
        seq.append(c)
    resident = [[torch.from_numpy(f.xyz).cuda() for f in fr[:W + K]] for fr in frames]

    def serve_frames(lo, hi, srv=srv, sids=sids):
        tests = 0
        for k in range(lo, hi):
            for s, sid in enumerate(sids):
                f = frames[s][k]
                srv.submit(sid, f.xyz, f.origin, f.frame_id)
            for sid, fid, st in srv.step():
                if st != 0:
                    raise RuntimeError("stream %d frame %d: %s" % (sid, fid, srv.last_error()))
                tests += srv.context(sid).score_stats(0)["canonical_tests"]
        return tests

    def seq_frames(lo, hi):
        tests = 0
        for k in range(lo, hi):
            for s, c in enumerate(seq):
                f = frames[s][k]
                frame_on(c, resident[s][k], f)
                tests += c.score_stats(0)["canonical_tests"]
        return tests
    serve_frames(0, W)
    serve_frames(0, W, srv_b, sids_b)
    serve_frames(0, W, srv_o, sids_o)
    seq_frames(0, W)
    log("warm-up done; points per stream %s" % [srv.context(i).num_points() for i in sids])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tests_srv = serve_frames(W, W + K)
    wall_srv = time.perf_counter() - t0
    t0 = time.perf_counter()
    tests_b = serve_frames(W, W + K, srv_b, sids_b)
    wall_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    tests_o = serve_frames(W, W + K, srv_o, sids_o)
    wall_o = time.perf_counter() - t0
    t0 = time.perf_counter()
    tests_seq = seq_frames(W, W + K)
    torch.cuda.synchronize()
    wall_seq = time.perf_counter() - t0

    def same_as_seq(server, ids):
        if INC:
            return all(np.array_equal(server.context(sid).read_incremental()[k],
                                      seq[s].read_incremental()[k])
                       for s, sid in enumerate(ids) for k in ("label", "best", "best_dir", "a"))
        return all(np.array_equal(server.context(sid).read_labels(0)["label"],
                                  seq[s].read_labels(0)["label"]) and
                   np.array_equal(server.context(sid).read_labels(0)["first_free"],
                                  seq[s].read_labels(0)["first_free"])
                   for s, sid in enumerate(ids))
    same = same_as_seq(srv, sids) and same_as_seq(srv_b, sids_b) and same_as_seq(srv_o, sids_o)
    srv_b.close()
    srv_o.close()
    returns = sum(len(frames[s][k].xyz) for s in range(NS) for k in range(W, W + K))
    log("throughput: server %.1f ms per step, always batched %.1f, never batched %.1f, "
        "sequential %.1f" % (wall_srv / K * 1e3, wall_b / K * 1e3, wall_o / K * 1e3,
                             wall_seq / K * 1e3))

    # paced: every stream at 10 Hz from its phase
    def paced(run_one_step):
        arr = sorted((specs[s].phase + 0.1 * j, s, W + K + j) for s in range(NS) for j in range(L))
        lat = []
        i = 0
        t0 = time.perf_counter() + 0.05
        while i < len(arr) or run_one_step(None, peek=True):
            now = time.perf_counter() - t0
            while i < len(arr) and arr[i][0] <= now:
                run_one_step(arr[i])
                i += 1
            done = run_one_step(None)
            if done:
                end = time.perf_counter() - t0
                lat += [end - a for a in done]
            elif i < len(arr):
                time.sleep(max(0.0, min(0.002, arr[i][0] - (time.perf_counter() - t0))))
        return np.array(lat) * 1e3

    queue = []

    def srv_step(item, peek=False):
        if peek:
            return any(srv.pending(sid) for sid in sids)
        if item is not None:
            a, s, k = item
            f = frames[s][k]
            srv.submit(sids[s], f.xyz, f.origin, f.frame_id)
            queue.append((s, f.frame_id, a))
            return None
        if not any(srv.pending(sid) for sid in sids):
            return []
        done = []
        for sid, fid, st in srv.step():
            if st != 0:
                raise RuntimeError("stream %d frame %d: %s" % (sid, fid, srv.last_error()))
            s = sids.index(sid)
            read_out(srv.context(sid))
            j = next(j for j, q in enumerate(queue) if q[0] == s and q[1] == fid)
            done.append(queue.pop(j)[2])
        return done
    lat_srv = paced(srv_step)
    waiting = []
    pinned = {(s, k): torch.from_numpy(frames[s][k].xyz).pin_memory()
              for s in range(NS) for k in range(W + K, n)}

    def seq_step(item, peek=False):
        if peek:
            return bool(waiting)
        if item is not None:
            waiting.append(item)
            return None
        if not waiting:
            return []
        a, s, k = waiting.pop(0)
        f = frames[s][k]
        x = pinned[(s, k)].cuda(non_blocking=True)
        frame_on(seq[s], x, f)
        read_out(seq[s])
        return [a]
    lat_seq = paced(seq_step)
    same_end = same_as_seq(srv, sids)
    pct = lambda v, q: float(np.percentile(v, q))
    out = {
        "metric": "frame latency p50/p99 and throughput, %d concurrent streams at 10 Hz" % NS
                  + (", incremental mode" if INC else ""),
        "value": pct(lat_srv, 99),
        "unit": "ms (p99 frame latency, arrival to labels on the host)",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": wall_srv / K * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "serve: %d streams (trees and box clusters alternating), own "
                               "tool each at 256 orientations, frames of 5,000-40,000 returns at "
                               "10 Hz, TSDF capacity %.2g voxels per stream"
                               % (NS, 390625 * per * 512),
                   "frames_per_stream": {"warmup": W, "throughput": K, "paced": L},
                   "incremental_budget": INC,
                   "map_points_end": [int(srv.context(i).num_points()) for i in sids]},
        "admission": {"budget_bytes": 24 * GiB, "per_stream_bytes": stream_budget,
                      "admitted": len(sids),
                      "one_more_refused": refused,
                      "device_bytes": [int(srv.context(i).device_bytes()) for i in sids]},
        "latency_ms": {"p50": pct(lat_srv, 50), "p99": pct(lat_srv, 99), "max": float(lat_srv.max()),
                       "frames": int(len(lat_srv))},
        "sequential_latency_ms": {"p50": pct(lat_seq, 50), "p99": pct(lat_seq, 99),
                                  "max": float(lat_seq.max())},
        "throughput": {"frames_per_s": NS * K / wall_srv, "returns_per_s": returns / wall_srv,
                       "tests_per_s": tests_srv / wall_srv,
                       "mode": ("incremental frames, each on its own stream" if INC else
                                "the library default: each stream scored on its own stream"),
                       "always_batched_frames_per_s": NS * K / wall_b,
                       "never_batched_frames_per_s": NS * K / wall_o,
                       "sequential_frames_per_s": NS * K / wall_seq,
                       "sequential_tests_per_s": tests_seq / wall_seq,
                       "speedup": wall_seq / wall_srv,
                       "always_batched_over_never": wall_o / wall_b,
                       "same_tests": bool(tests_srv == tests_seq == tests_o == tests_b),
                       "labels_identical": bool(same), "labels_identical_after_paced": bool(same_end)},
    }
    print(json.dumps(out), flush=True)


def smooth_traffic():
    """HBM bytes per refinement launch from the committed counter summary,
    None once the kernel source has changed since it was measured."""
    if not os.path.exists(SMOOTH_TRAFFIC_FILE):
        return None
    tr = json.load(open(SMOOTH_TRAFFIC_FILE))
    return tr.get("bytes_per_launch") if tr.get("src_sha") == src_sha(SMOOTH_SRC) else None


def run_smooth(args):
    """Differentiation workload: the tree map after frames 0..F-1, 1,000,000
    of its surface points (voxel centres) x 64 starting directions (Fibonacci,
    tool axis turned onto each), the saw box as 64 samples (16 stations x 4
    corners over body and corridor), 20 ascent steps of the smoothed score
    (c = 1 cm, tau_s = 0.5 cm) in one kernel.  W untimed warm-up refinements
    on 1/16 of the pairs, then K timed full refinements."""
    import torch
    import synth
    from paper_2608_06412_amd import Context, default_config
    from paper_2608_06412_amd.af import unpack_keys

    F = 250
    W = args.warmup if args.warmup != 100 else 1
    K = args.steps if args.steps != 400 else 3
    w = synth.tree()
    frames = w.frames(F)
    torch.cuda.set_device(0)
    ctx = Context(default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 17,
                                 max_points=1 << 22))
    for f in frames:
        ctx.integrate_frame(torch.from_numpy(f.xyz).cuda(), f.origin, f.frame_id)
    n_map = ctx.num_points()
    allk = ctx.read_points()["key"]
    rng = np.random.default_rng(11)
    n_pts = args.smooth_points
    sel = allk[rng.choice(len(allk), n_pts, replace=len(allk) < n_pts)]
    ijk = unpack_keys(sel)

    def morton(b):
        # interleaved bits of the brick coordinates (16 bits per axis)
        b = (b - b.min(0)).astype(np.uint64)
        code = np.zeros(len(b), np.uint64)
        for bit in range(16):
            for a in range(3):
                code |= ((b[:, a] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + a)
        return code
    # the caller's pair order: points in Morton order of their bricks, so the
    # waves that share an L2 read neighbouring parts of the map
    order = np.lexsort((sel, morton(ijk >> 3)))
    p = ((ijk[order] + 0.5) * w.voxel).astype(np.float32)
    p_random = ((ijk + 0.5) * w.voxel).astype(np.float32)
    S = 64
    q0 = np.tile(synth.quaternion_towards(synth.fibonacci_directions(S)), (n_pts, 1))
    smp = synth.tool_samples(w.tool, 16)
    pd = torch.from_numpy(p).cuda()
    qd = torch.from_numpy(q0).cuda()
    sd = torch.from_numpy(smp).cuda()
    steps, eta, mx = 20, 1e-5, 0.05
    pairs = n_pts * S
    log("map %d points, %d blocks; %d pairs x %d steps, M = %d" %
        (n_map, ctx.num_blocks(), pairs, steps, len(smp)))
    sub = n_pts // 16
    for _ in range(W):
        ctx.smooth_refine(pd[:sub], qd[:sub * S], sd, steps=steps, eta=eta, max_step=mx)
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    ctx.timing_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(K):
        q, s = ctx.smooth_refine(pd, qd, sd, steps=steps, eta=eta, max_step=mx)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / K
    tm = ctx.timing_read(reset=True)
    k_ms = tm["k_smooth_ms"] / K
    # the same pairs in random point order, for comparison
    pr = torch.from_numpy(p_random).cuda()
    ctx.smooth_refine(pr, qd, sd, steps=steps, eta=eta, max_step=mx)
    torch.cuda.synchronize()
    k_ms_random = ctx.timing_read(reset=True)["k_smooth_ms"]
    del pr
    # the ascent's own check: s at the start against s at the end, per pair
    s_start = torch.empty(pairs, device="cuda")
    ctx.smooth_eval(pd.repeat_interleave(S, 0), qd, sd, s=s_start)
    torch.cuda.synchronize()
    gain = (s - s_start).cpu().numpy()
    taps = pairs * (steps + 1) * len(smp) * 8
    # per sample: the apron index of its cell's brick and the cell's 8 values
    bytes_alg = pairs * (steps + 1) * len(smp) * 36.0
    ach = bytes_alg / (k_ms / 1e3) / 1e9
    out = {
        "metric": "smoothed-score ascent: (point, start) pairs x steps per second",
        "value": pairs * steps / (k_ms / 1e3),
        "unit": "pair-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": k_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "smooth: tree map after %d frames, %d surface points x 64 "
                               "starts, saw box as 64 samples, 20 ascent steps, c = 1 cm, "
                               "tau_s = 0.5 cm" % (F, n_pts),
                   "map_points": int(n_map), "pairs": pairs, "ascent_steps": steps,
                   "samples": len(smp), "eta": eta, "max_step": mx},
        "wall_ms_per_refine": wall * 1e3,
        "random_point_order_ms": k_ms_random,
        "sample_evaluations_per_s": pairs * (steps + 1) * len(smp) / (k_ms / 1e3),
        "taps_per_s": taps / (k_ms / 1e3),
        "ascent": {"improved_frac": float((gain > 0).mean()),
                   "unchanged_frac": float((gain == 0).mean()),
                   "mean_gain": float(gain.mean())},
        "roofline": {"kernel": "k_smooth_refine", "bound": "hbm", "achieved": ach, "peak": 8000.0,
                     "unit": "GB/s", "frac": ach / 8000.0, "traffic": smooth_traffic(),
                     "bytes_model": "36 B per sample evaluation (apron index + 8 cell values "
                                    "of 4 B), 64 samples, 21 evaluations per pair; mostly "
                                    "L2 hits, so this is demand, not DRAM traffic"},
    }
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.Oracle(voxel=w.voxel, trunc=w.trunc, r_c=w.r_c)
        t0 = time.perf_counter()
        for f in frames[:args.cpu_frames]:
            orc.integrate_frame(f.xyz, f.origin, f.frame_id)
        okeys = orc.read_points()["key"]
        po = ((oracle.unpack_keys(okeys[rng.choice(len(okeys), 64)]) + 0.5) * w.voxel)
        po = po.astype(np.float32)
        qo = np.tile(synth.quaternion_towards(synth.fibonacci_directions(8)), (64, 1))
        t0 = time.perf_counter()
        orc.smooth_refine(po, qo, smp, steps=steps, eta=eta, max_step=mx)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 64 * 8 * steps / dt, "unit": "pair-steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "oracle fp64 ascent, 64 points x 8 starts x 20 steps "
                                         "on the map of the first %d frames" % args.cpu_frames}
    print(json.dumps(out), flush=True)


def run_incremental(args):
    """Incremental workload: the tree workload (frames 0..W-1 warm up,
    W..W+K-1 timed, then L frames paced at 10 Hz) with the incremental mode
    of Section 3.5: only queued points are re-evaluated, at most `budget` per
    frame.  Reports the frame time, evaluations per frame, the backlog and the
    paced latency beside the stateless path's frame time on the same frames
    (a second context), and how many points carry the same label under both."""
    import torch
    import synth
    from paper_2608_06412_amd import Context, default_config

    W = args.warmup
    K = args.steps
    L = args.latency_frames
    budget = args.incr_budget
    w = synth.tree(n_frames=W + K + L)
    frames = w.frames(W + K + L)
    torch.cuda.set_device(0)
    cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 17, max_points=1 << 22,
                         max_orientations=len(w.rot), max_tools=1)
    ctx = Context(cfg)
    ctx.set_tool_kernels(0, w.tool, w.rot)
    ctx.incremental_enable(0, budget)
    ref = Context(cfg)
    ref.set_tool_kernels(0, w.tool, w.rot)
    resident = [torch.from_numpy(f.xyz).cuda() for f in frames[:W + K]]
    for i in range(W):
        ctx.incremental_frame(resident[i], frames[i].origin, frames[i].frame_id)
        ref.integrate_frame(resident[i], frames[i].origin, frames[i].frame_id)
    torch.cuda.synchronize()
    evals, backlog, queued = [], [], []
    t0 = time.perf_counter()
    for i in range(W, W + K):
        ctx.incremental_frame(resident[i], frames[i].origin, frames[i].frame_id)
        st = ctx.incremental_stats()      # synchronises, as a consumer of the counts would
        evals.append(st["evaluated"])
        backlog.append(st["backlog"])
        queued.append(st["queued"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the stateless path on the same frames
    t0 = time.perf_counter()
    for i in range(W, W + K):
        ref.integrate_frame(resident[i], frames[i].origin, frames[i].frame_id)
        ref.score_points(0)
        ref.score_stats(0)
    torch.cuda.synchronize()
    wall_ref = time.perf_counter() - t0
    inc = ctx.read_incremental()
    lab_ref = ref.read_labels(0)["label"]
    same = float(np.mean(inc["label"] == lab_ref))
    # paced frames: arrival to incremental labels on the host
    lat = []
    pinned = [torch.from_numpy(f.xyz).pin_memory() for f in frames[W + K:]]
    staging = torch.empty((max(len(f.xyz) for f in frames), 3), device="cuda")
    # every label into a pinned array allocated once; keys of new points only
    # (points are only appended, so the host keeps the earlier ones)
    host_label = torch.empty(cfg.max_points, dtype=torch.uint8, pin_memory=True).numpy()
    keys = [ctx.read_incremental(labels_only=True)["key"]]
    known = len(keys[0])
    start = time.perf_counter() + 0.05
    for j, f in enumerate(frames[W + K:]):
        release = start + 0.1 * j
        while time.perf_counter() < release:
            time.sleep(0.0005)
        n = len(f.xyz)
        staging[:n].copy_(pinned[j], non_blocking=True)
        ctx.incremental_frame(staging[:n], f.origin, f.frame_id)
        m = len(ctx.read_incremental(labels_only=True, label_out=host_label, keys=False)["label"])
        if m > known:
            keys.append(ctx.read_incremental(labels_only=True, first=known)["key"])
            known = m
        lat.append((time.perf_counter() - release) * 1e3)
    lat = np.array(lat) if lat else np.zeros(1)
    out = {
        "metric": "incremental mode: frame time (integrate + triggers + budgeted re-evaluation)",
        "value": wall / K * 1e3,
        "unit": "ms per frame",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "incremental: tree workload (20,000 returns per frame, K = 256, "
                               "saw box), incremental mode with a budget of %d evaluations "
                               "per frame" % budget,
                   "frames_timed": [W, W + K - 1], "budget": budget,
                   "map_points_end": int(ctx.num_points())},
        "evaluated_per_frame": {"mean": float(np.mean(evals)), "max": int(np.max(evals))},
        "queued_per_frame_mean": float(np.mean(queued)),
        "backlog_end": int(backlog[-1]),
        "stateless_ms_per_frame": wall_ref / K * 1e3,
        "speedup_vs_stateless": wall_ref / wall,
        "labels_same_as_stateless_frac": same,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "frames": int(len(lat)), "rate_hz": 10,
                       "includes": "H2D of the frame, integrate, incremental update, D2H of "
                                   "every label (pinned host array) and of the new points' keys"},
    }
    print(json.dumps(out), flush=True)


def run_window(args):
    """Sliding-window workload: the tree sequence (600 frames, integrate and
    score every frame) with a window of --window-m metres per axis.  Reports
    the frame time (mean, p50, p99, and on the frames that shifted the
    window), the blocks the map holds at most beside the unbounded map's at
    the end, the shifts, and the points scored per frame."""
    import torch
    import synth
    from paper_2608_06412_amd import Context, default_config, window_blocks

    n = max(args.steps, 1) if args.steps != 400 else 600
    w = synth.tree(n_frames=max(600, n))
    frames = w.frames(n)
    torch.cuda.set_device(0)
    blocks = window_blocks([args.window_m] * 3, w.voxel)
    cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 17, max_points=1 << 22,
                         max_orientations=len(w.rot), max_tools=1)
    ctx = Context(cfg)
    ctx.set_window(blocks)
    ctx.set_tool_kernels(0, w.tool, w.rot)
    resident = [torch.from_numpy(f.xyz).cuda() for f in frames]
    if args.window_graph:
        # recorded frames: a shift runs eagerly and records again
        ctx.graph_prepare([-1.0] * 3, [1.0] * 3, max(len(f.xyz) for f in frames), [0])
    torch.cuda.synchronize()
    ms, shifted, held, scored = [], [], [], []
    last = 0
    for i, f in enumerate(frames):
        t0 = time.perf_counter()
        if args.window_graph:
            ctx.graph_frame(resident[i], f.origin, f.frame_id)
            ctx.graph_sync()
        else:
            ctx.integrate_frame(resident[i], f.origin, f.frame_id)
            ctx.score_points(0)
        st = ctx.score_stats(0)            # synchronises
        ms.append((time.perf_counter() - t0) * 1e3)
        sh = ctx.window_state()[2]
        shifted.append(sh != last)
        last = sh
        held.append(ctx.frame_stats()["n_blocks"])
        scored.append(st["n_confident"])
    ms = np.array(ms)
    shifted = np.array(shifted)
    out = {
        "metric": "sliding-window tree workload: frame time (integrate + in-window scoring)"
                  + (", recorded frames" if args.window_graph else ""),
        "value": float(ms.mean()),
        "unit": "ms per frame",
        "n_gpus": 1, "steps": len(frames), "warmup": 0,
        "ms_per_step": float(ms.mean()),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "window: tree workload (20,000 returns per frame, K = 256, saw "
                               "box), %.1f m window (%d blocks per axis)"
                               % (args.window_m, int(blocks[0])),
                   "frames": len(frames), "recorded_frames": bool(args.window_graph)},
        "ms_per_frame": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99)),
                         "shift_frames_mean": float(ms[shifted].mean()) if shifted.any() else None,
                         "other_frames_mean": float(ms[~shifted].mean())},
        "shifts": int(last),
        "blocks_held_max": int(max(held)),
        "points_end": int(ctx.num_points()),
        "confident_scored_per_frame_mean": float(np.mean(scored)),
        "device_bytes": int(ctx.device_bytes()),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--latency-frames", type=int, default=600,
                    help="frames of the tree sequence replayed at 10 Hz on a fresh map")
    ap.add_argument("--cpu-frames", type=int, default=6)
    ap.add_argument("--cpu-points", type=int, default=100000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the scoring kernel after the warm-up")
    ap.add_argument("--score-variant", default=None,
                    help="scoring configuration (index or name) when not tuning; default: "
                         "the library's default configuration")
    ap.add_argument("--serve-streams", type=int, default=4,
                    help="streams of the serve workload (the 24 GiB budget is shared)")
    ap.add_argument("--serve-incremental", type=int, default=0,
                    help="serve workload in the incremental mode with this budget (0: stateless)")
    ap.add_argument("--window-m", type=float, default=10.0,
                    help="window size per axis (metres) of the window workload")
    ap.add_argument("--window-graph", action="store_true",
                    help="window workload through recorded frames (af_graph_frame)")
    ap.add_argument("--workload", default="tree",
                    choices=["tree", "batch", "serve", "smooth", "incremental", "window"],
                    help="tree: the default single-tool workload; batch: 8 tools x 512 "
                         "orientations scored in one launch, frames of 5k-40k returns")
    ap.add_argument("--incr-budget", type=int, default=1 << 20,
                    help="evaluations per frame of the incremental workload")
    ap.add_argument("--smooth-points", type=int, default=1000000,
                    help="surface points of the smooth workload (64 starts each)")
    ap.add_argument("--trace-summary", default=None,
                    help="only summarise a rocprofv3 kernel_trace.csv of a bench run "
                         "with the same --warmup/--steps")
    ap.add_argument("--traffic-summary", default=None,
                    help="only write profiles/traffic_k_score_tree.json from four rocprofv3 "
                         "--pmc CSVs: FETCH_SIZE,WRITE_SIZE of a default run, then of the "
                         "copy probe (comma-separated)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes (3 times); "
                         "used to calibrate rocprofv3 FETCH_SIZE/WRITE_SIZE")
    args = ap.parse_args()
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary, args.warmup, args.steps), indent=1))
        return
    if args.traffic_summary:
        wl = "smooth" if args.workload == "smooth" else "tree"
        warm, steps = args.warmup, args.steps
        if wl == "smooth":   # the smooth workload's own defaults (see run_smooth)
            warm = warm if warm != 100 else 1
            steps = steps if steps != 400 else 3
        out = traffic_summary(args.traffic_summary.split(","), warm, steps,
                              args.copy_probe or (1 << 30), wl)
        with open(os.path.join(ROOT, "profiles", out["file"]), "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out, indent=1))
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a scene would "
              "shard by block-key owner, each GPU integrating and scoring its own blocks). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2608_06412_amd import Context, default_config

    synth.build(force=False)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "smooth":
        return run_smooth(args)
    if args.workload == "incremental":
        return run_incremental(args)
    if args.workload == "window":
        return run_window(args)
    if args.workload == "batch":
        run_batch(args)
        return
    W, K, L = args.warmup, args.steps, args.latency_frames
    F0 = tree_window(W, K)
    total = max(F0 + K, L)
    w = synth.tree(n_frames=max(600, total))
    t = time.perf_counter()
    frames = w.frames(total)
    log("generated %d frames in %.1f s" % (total, time.perf_counter() - t))

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    resident = [torch.from_numpy(f.xyz).to(dev) for f in frames[:F0 + K]]

    cfg = default_config(w.voxel, w.trunc, r_c=w.r_c, max_blocks=1 << 17,
                         max_points=1 << 22, max_orientations=len(w.rot), max_tools=1)
    ctx = Context(cfg)
    ctx.set_tool_kernels(0, w.tool, w.rot)
    Krot = len(w.rot)

    names = ctx.score_variants()
    if not args.tune and args.score_variant is not None:
        v = args.score_variant
        idx = int(v) if str(v).isdigit() else names.index(v)
        ctx.set_score_variant(idx)
    idx = ctx.score_variant()
    t = time.perf_counter()
    for i in range(F0):
        ctx.integrate_frame(resident[i], frames[i].origin, frames[i].frame_id)
        ctx.score_points(0)
        if i % 50 == 0:
            log("pre-roll frame %d, %d points" % (i, ctx.num_points()))
    torch.cuda.synchronize()
    log("pre-roll %d frames (warm-up %d) in %.1f s" % (F0, W, time.perf_counter() - t))
    if args.tune:
        best, ms = ctx.tune_score(0, reps=3)
        tuning = {"chosen": names[best], "ms": {n: round(m, 3) for n, m in zip(names, ms)},
                  "at_frame": F0}
        log("score tuning at frame %d: %s" % (F0, json.dumps(tuning)))
    else:
        tuning = {"chosen": names[ctx.score_variant()], "tuned": False}

    ctx.timing_enable(True)
    ctx.timing_read(reset=True)
    tests = lookups = conf = nominal = returns = accessible = deep = deep_chunks = cand = 0
    cchecks = cclear = cbody = cfar = 0
    byts = kbyts = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(F0, F0 + K):
        ctx.integrate_frame(resident[i], frames[i].origin, frames[i].frame_id)
        ctx.score_points(0)
        st = ctx.score_stats(0)
        tests += st["canonical_tests"]
        lookups += st["canonical_lookups"]
        conf += st["n_confident"]
        nominal += st["n_confident"] * Krot
        accessible += st["n_accessible"]
        deep += st["deep_tests"]
        deep_chunks += st["deep_chunks_max"]
        cchecks += st["coarse_checks"]
        cclear += st["coarse_clear"]
        cbody += st["chunks_body"]
        cfar += st["chunks_far"]
        cand += st["candidate_tests"]
        byts += score_bytes(st["canonical_lookups"], st["n_confident"], Krot)
        kbyts += kscore_bytes(st["canonical_lookups"], st["arm_lookups"], st["n_confident"], Krot)
        returns += len(frames[i].xyz)
        if (i - F0) % 50 == 0:
            log("timed frame %d: %d points, %d confident, %d canonical tests" %
                (i, st["n_points"], st["n_confident"], st["canonical_tests"]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.timing_read(reset=True)
    wall = t1 - t0
    log("timed frames %d-%d in %.2f s" % (F0, F0 + K - 1, wall))
    map_points = ctx.num_points()
    map_blocks = ctx.num_blocks()
    ctx.close()
    del resident

    # 10 Hz paced latency on a fresh map: release -> labels on the host, for
    # the sequence's first L frames.  The host keeps the keys in canonical
    # order (points are only appended), so each frame copies every point's
    # label and first free orientation and the new points' keys, into pinned
    # arrays allocated once.
    lat = np.zeros(0)
    if L > 0:
        pinned = [torch.from_numpy(f.xyz).pin_memory() for f in frames[:L]]
        nmax = max(len(f.xyz) for f in frames[:L])
        staging = torch.empty((nmax, 3), dtype=torch.float32, device=dev)
        lctx = Context(cfg)
        lctx.set_tool_kernels(0, w.tool, w.rot)
        if not args.tune and args.score_variant is not None:
            lctx.set_score_variant(idx)
        cap = cfg.max_points
        host = {"label": torch.empty(cap, dtype=torch.uint8, pin_memory=True).numpy(),
                "first_free": torch.empty(cap, dtype=torch.int16, pin_memory=True).numpy(),
                "key": torch.empty(cap, dtype=torch.int64, pin_memory=True).numpy()}
        known = 0
        lat_l = []
        torch.cuda.synchronize()
        tstart = time.perf_counter() + 0.05
        for j, f in enumerate(frames[:L]):
            release = tstart + 0.1 * j
            while time.perf_counter() < release:
                time.sleep(0.0005)
            n = len(f.xyz)
            staging[:n].copy_(pinned[j], non_blocking=True)
            lctx.integrate_frame(staging[:n], f.origin, f.frame_id)
            lctx.score_points(0)
            got = lctx.read_labels(0, out=host, keys=False)
            m = len(got["label"])
            if m > known:
                lctx.read_labels(0, first=known, count=m - known,
                                 out={"key": host["key"][known:], "label": host["label"][known:],
                                      "first_free": host["first_free"][known:]})
                known = m
            lat_l.append((time.perf_counter() - release) * 1e3)
            if j % 100 == 0:
                log("paced frame %d: %.1f ms, %d points" % (j, lat_l[-1], m))
        lat = np.array(lat_l)
        lctx.close()
        log("latency over %d paced frames: p50 %.1f ms, p99 %.1f ms" %
            (len(lat), np.percentile(lat, 50), np.percentile(lat, 99)))

    kernels = {"k_score": tm["k_score_ms"], "k_integrate_fold": tm["k_integrate_ms"],
               "k_normals": tm["k_normals_ms"], "k_mask": tm["k_mask_ms"]}
    dominant = max(kernels, key=kernels.get)
    score_s = tm["k_score_ms"] / 1e3
    achieved = kbyts / score_s / 1e9 if score_s > 0 else 0.0
    path_s = (tm["k_score_ms"] + tm["k_mask_ms"]) / 1e3
    path_achieved = byts / path_s / 1e9 if path_s > 0 else 0.0
    # measured HBM bytes per launch, only when the counters were taken on this
    # scoring source and on this frame window
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("src_sha") == src_sha(SCORE_SRC) and tr.get("window") == [F0, F0 + K - 1]:
            traffic = tr.get("bytes_per_launch")
    alg_launch = kbyts / max(K, 1)
    roofline = {"kernel": "k_score", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic,
                "limiter": "priced against HBM (algorithmic bytes); the measured limiter is "
                           "the latency of L2-resident gathers (DRAM traffic is a few percent "
                           "of the algorithmic bytes)",
                "dram_over_algorithmic": (traffic / alg_launch) if traffic and alg_launch else None,
                "algorithmic_bytes_per_launch": alg_launch,
                "bytes_model": "8 B per canonical lookup not answered by the mask kernel + "
                               "per confident point 8 B key + 3K/8 B mask and arm planes + "
                               "4 B weight + 3 B outputs",
                "score_path": {"kernels": "k_mask_walk + k_score",
                               "algorithmic_bytes_per_step": byts / max(K, 1),
                               "achieved": path_achieved, "frac": path_achieved / HBM_PEAK_GBS},
                "avg_launch_ms": tm["k_score_ms"] / max(tm["score_calls"], 1),
                "dominant_kernel": dominant}

    out = {
        "metric": METRIC,
        "value": tests / wall,
        "unit": "point-orientation tests/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": "tree: procedural 8 m tree, 20,000 returns/frame from an orbiting "
                        "Mid-360-shaped sensor, v=1 cm, tau=4 cm, saw box 30x5x2 cm + 1 m "
                        "corridor, K=256 (64 directions x 4 rolls)",
            "frames_timed": [F0, F0 + K - 1], "preroll_frames": F0,
            "returns_per_frame": int(np.mean([len(f.xyz) for f in frames])),
            "orientations": Krot, "voxel_m": w.voxel, "trunc_m": w.trunc,
            "map_points_end": int(map_points), "map_blocks_end": int(map_blocks),
        },
        "returns_integrated_per_s": returns / (tm["integrate_ms"] / 1e3),
        "nominal_tests_per_s": nominal / wall,
        "canonical_lookups_per_s": lookups / wall,
        "latency_ms": None if len(lat) == 0 else {
            "p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "max": float(lat.max()), "frames": int(len(lat)), "rate_hz": 10,
            "sequence_frames": [0, int(len(lat)) - 1],
            "includes": "H2D of the frame, integrate, score, D2H of every point's label and "
                        "first free orientation and of the new points' keys (pinned host "
                        "arrays); frames replayed on a fresh map"},
        "stage_ms_per_step": {k: v / max(K, 1) for k, v in
                              {"integrate": tm["integrate_ms"], "score": tm["score_ms"],
                               **kernels}.items()},
        "roofline": roofline,
        "score_tuning": tuning,
        "score_work_per_step": {"confident_points": conf / K, "accessible_points": accessible / K,
                                "candidate_tests": cand / K, "canonical_tests": tests / K,
                                "canonical_lookups": lookups / K, "deep_tests": deep / K,
                                "deep_tests_full_chunks": deep_chunks / K,
                                "coarse_checks": cchecks / K, "coarse_clear": cclear / K,
                                "deep_steps_body": cbody / K, "deep_steps_corridor": cfar / K},
    }
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(w, frames, args.cpu_frames, args.cpu_points)
        log("cpu baseline in %.1f s" % (time.perf_counter() - t))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
