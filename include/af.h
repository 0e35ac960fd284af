/*
 * af.h -- C ABI of the MI355X accessibility-field library (libaf.so).
 *
 * Implements the per-frame hot path of "Beyond Visibility: Real-Time Surface
 * Accessibility Fields from Sparse LiDAR" (Scott, Schofield, Green):
 *   integrate_frame  scan-centric TSDF integration of one LiDAR frame into a
 *                    hashed 8^3 voxel-block map (Section 3.2), the ray-cleared
 *                    band (Section 3.4, "Arm path checking") and the voxel-
 *                    deduplicated surface point set (Section 3.1);
 *   set_tool_kernels precomputed rotated tool kernels (Section 3.4, "Tool
 *                    kernel", "Self-exclusion"; Section 3.6);
 *   score_points     normal and observation filters, collision count and arm
 *                    samples for every confident point (Sections 3.4, 3.5);
 *   read_labels      the per-point accessibility field (Section 3.1).
 *
 * Conventions
 *   - All functions return AF_OK (0) or a negative AF_E* code; no exception or
 *     signal crosses the ABI.  af_last_error() gives a text for the last error.
 *   - A context is not thread-safe; use one context per host thread.
 *   - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *     default stream).  Work is enqueued asynchronously on that stream unless
 *     the function says it synchronises.
 *   - Device pointers must be device memory of the context's GPU; host
 *     pointers are ordinary host memory.  The library never keeps a caller's
 *     pointer after a call returns (device inputs must stay valid until the
 *     stream reaches the call).
 *   - Positions are world-frame metres (float32) and are quantised to
 *     integers in units of voxel/256 (round half to even of the fp64
 *     product); voxel i covers [i v, (i+1) v).  A voxel key packs the index
 *     (i + 2^20) in 21 bits per axis, x lowest.
 */
#ifndef AF_H
#define AF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  AF_OK = 0,
  AF_EINVAL = -1,    /* bad argument */
  AF_ENOMEM = -2,    /* device memory or HBM budget exhausted */
  AF_EDEVICE = -3,   /* HIP runtime error */
  AF_ENOTOOL = -4,   /* tool id never set */
  AF_EOVERFLOW = -5, /* block / point capacity exceeded (state is then incomplete) */
  AF_EBUSY = -6      /* a server's stream slots or a stream's frame queue are full */
};

/* point labels */
enum {
  AF_UNSCORED = 0,     /* TSDF confidence w/(w+5) < 0.2, i.e. W < 2 (Section 3.5) */
  AF_ACCESSIBLE = 1,   /* some candidate orientation is free */
  AF_BLOCKED = 2,      /* every candidate orientation collides */
  AF_NO_CANDIDATE = 3, /* no orientation passes the normal/observation filters */
  AF_TENTATIVE = 4,    /* incremental mode: a free direction is stored, but the
                          combined confidence c * a is not above 0.7 yet */
  AF_NOT_EVALUATED = 255 /* sliding window: never scored (outside the window at
                            every scoring call since the point was created) */
};

/* table entry classes */
enum { AF_CLS_BODY = 0, AF_CLS_NEAR = 1, AF_CLS_FAR = 2 };

/* tool shapes */
enum { AF_TOOL_CYLINDER = 0, AF_TOOL_BOX = 1 };

typedef struct af_ctx af_ctx;

typedef struct af_config {
  double voxel;           /* voxel edge v, metres (> 0) */
  double trunc;           /* truncation tau, metres; <= 0 selects min(4v, 0.1 m)
                             (Section 3.2; read as min, see the design notes) */
  double r_c;             /* collision threshold on the TSDF, metres */
  int32_t n_c;            /* body voxels below r_c that block an orientation (5) */
  int32_t weight_cap;     /* weight saturation with proportional rescale (2000) */
  int32_t conf_min_w;     /* minimum W of a scored point (2 <=> c >= 0.2) */
  double cos_normal;      /* cosine of the normal half-cone (cos 70 deg) */
  double obs_dot;         /* observation-side dot threshold (0.25) */
  double vp_min_dist;     /* novelty distance of stored viewpoints, metres (0.1) */
  int32_t n_vp;           /* stored viewpoints per point, 1..8 (8) */
  int32_t knn_k;          /* neighbours of the PCA normal (10) */
  int32_t clamp_negative; /* 0: clamp d to [0, tau] (paper); 1: [-tau, tau] */
  int32_t max_tools;      /* tool slots */
  int64_t max_blocks;     /* voxel-block capacity */
  int64_t max_points;     /* surface-point capacity */
  int32_t max_orientations; /* per tool */
  int32_t pad;
  int64_t hbm_budget;     /* bytes the context may allocate (0 = unlimited) */
} af_config;

typedef struct af_tool {
  int32_t shape;          /* AF_TOOL_CYLINDER or AF_TOOL_BOX */
  int32_t pad;
  double length;          /* body length along the approach axis (+x), m */
  double corridor;        /* approach corridor beyond the body, m */
  double r_s;             /* self-exclusion radius around the tip, m */
  double radius;          /* cylinder radius, m */
  double width, height;   /* box cross-section (local y, z), m */
} af_tool;

typedef struct af_frame_stats {
  int64_t n_in, n_valid, n_dropped;
  int64_t pairs_applied, pairs_excluded, band_marks;
  int64_t new_points, n_points, voxels_folded;
  int64_t n_blocks, new_blocks;
} af_frame_stats;

typedef struct af_score_stats {
  int64_t n_points, n_confident, n_accessible, n_blocked, n_no_candidate;
  int64_t candidate_tests, canonical_tests, canonical_lookups;
  /* diagnostics of the two-phase scoring configurations (0 for the others):
   * canonical tests not decided by the first table entries read per lane,
   * and the 64-entry chunks a full scan of those tests would take; coarse
   * corridor checks made and those that found every corridor brick clear;
   * 64-entry steps the deep scans took over body and over corridor entries;
   * the canonical lookups of arm samples whose result the mask pass
   * precomputed (configurations "near"; included in canonical_lookups) */
  int64_t deep_tests, deep_chunks_max;
  int64_t coarse_checks, coarse_clear;
  int64_t chunks_body, chunks_far;
  int64_t arm_lookups;
} af_score_stats;

/* Fill *cfg with the paper's constants for voxel size `voxel` and truncation
 * `trunc` (metres; <= 0 for the default) and capacities for a scene of about
 * a million surface points.  Returns AF_EINVAL for voxel <= 0. */
int af_config_default(af_config *cfg, double voxel, double trunc);

/* Create a context on the current HIP device: allocates the block pool, the
 * hash tables, the point arrays and the label arrays up front.  Returns
 * AF_EINVAL for an inconsistent configuration (truncation above 7 voxels,
 * n_vp outside 1..8, ...), AF_ENOMEM when the fixed allocations exceed
 * cfg->hbm_budget or the device, AF_EDEVICE on a HIP error.  *out receives
 * the context (NULL on error). */
int af_create(const af_config *cfg, af_ctx **out);

/* Release every device allocation of the context.  Synchronises the device. */
int af_destroy(af_ctx *ctx);

/* Text of the last error on this context (never NULL). */
const char *af_last_error(const af_ctx *ctx);

/* Section 3.4 "Tool kernel" / Section 3.6: precompute the rotated kernels of
 * tool `tool_id` (0 <= id < max_tools) for K orientations.  `rot` is a host
 * array of K row-major 3x3 rotation matrices (fp64) whose columns are the
 * tool's local axes in world coordinates: column 0 is the approach direction
 * (the tool extends along it from the tip at the surface point), columns 1-2
 * span the cross-section.  The table of orientation k lists, as voxel offsets
 * from the point's voxel: the three arm samples at 0.6, 1.25 and 2.25 times tau along
 * the approach direction (NEAR), the voxel centres inside the tool body
 * (BODY) and inside its corridor (FAR), minus the self-exclusion ball r_s;
 * BODY and FAR are each sorted by (|o|^2, z, y, x).  Built on the device; the
 * call synchronises `stream`.  Errors: AF_EINVAL (bad shape, K outside
 * 1..max_orientations, rotation column norms off by > 1e-9, an offset beyond
 * +-511 voxels or more than 16384 entries of one class), AF_ENOMEM. Replacing
 * a tool invalidates its labels. */
int af_set_tool_kernels(af_ctx *ctx, int32_t tool_id, const af_tool *tool,
                        int32_t K, const double *rot, void *stream);

/* Section 3.4 "Tool kernel": set tool `tool_id` from a caller-built table,
 * for tools that are not primitives (for instance points drawn on a mesh of
 * the tool, rotated and voxelised by the caller).  All arrays are
 * HOST memory owned by the caller; the library copies them.
 *   K             orientations, 1..max_orientations
 *   dir[K][3]     unit approach direction of each orientation (the normal
 *                 and observation filters use it; |norm - 1| <= 1e-9)
 *   offset_begin  [K + 1] entry ranges: orientation k owns entries
 *                 [offset_begin[k], offset_begin[k + 1]); offset_begin[0] = 0,
 *                 non-decreasing
 *   off[n][3]     voxel offsets (x, y, z) from the point's voxel, each
 *                 component within +-511
 *   cls[n]        AF_CLS_NEAR (exactly three per orientation: the arm samples
 *                 of Section 3.4 "Arm path checking"), AF_CLS_BODY (tool solid)
 *                 or AF_CLS_FAR (approach corridor)
 * The library stores each orientation's entries as its three NEAR entries in
 * the given order, then BODY and then FAR each sorted by (|o|^2, z, y, x); an
 * offset may appear once per class, and at most 16384 times per class and
 * orientation.  Labels do not depend on the entry order; canonical lookup
 * counts are counted in this stored order.  af_set_tool_kernels builds the
 * same form for its primitives, so af_read_tool_table of a primitive tool fed
 * back here gives identical results.  Synchronises `stream`.  Errors:
 * AF_EINVAL (bad id, K, direction, range, class, NEAR count, repeated offset;
 * the tool is then unchanged), AF_ENOMEM.  Replacing a tool invalidates its
 * labels. */
typedef struct af_kernel_table {
  int32_t K;
  int32_t pad;
  const double *dir;
  const uint32_t *offset_begin;
  const int16_t *off;
  const uint8_t *cls;
} af_kernel_table;
int af_set_tool_table(af_ctx *ctx, int32_t tool_id, const af_kernel_table *table, void *stream);

/* Section 3.2: integrate one frame.  `xyz` is a DEVICE array of n float32
 * triples (world frame), `origin` a HOST array of 3 floats (the sensor
 * position of the frame).  For every valid return the voxels of the index
 * cube of half-width ceil(tau/v) around it, except those inside the
 * cos > 0.95 cone behind it, receive d = |p - q| - |x - q| (voxel centre x,
 * clamped to [0, tau]) as integer sums S, W; the voxels between tau and 2.25 tau back
 * along the ray is marked ray-cleared; the return's voxel joins the surface
 * point set.  The frame is folded at the end (weights capped with
 * proportional rescaling of S).  Returns that are non-finite, out of range
 * (|x| >= 2^28 units) or at the sensor position are dropped and counted.
 * `frame_id` must increase strictly (AF_EINVAL otherwise).  The call
 * synchronises `stream` once, after block allocation.  AF_EOVERFLOW when the
 * block or point capacity is exceeded. */
int af_integrate_frame(af_ctx *ctx, const float *xyz, int64_t n,
                       const float origin[3], int64_t frame_id, void *stream);
/* af_integrate_frame for returns in HOST memory: `xyz` (n float32 triples)
 * is copied to a device buffer the context keeps (grown to the largest frame
 * seen, from the context's device budget: AF_ENOMEM if it does not fit) and
 * integrated from there.  The host array is no longer read when the call
 * returns.  Everything else as af_integrate_frame. */
int af_integrate_frame_host(af_ctx *ctx, const float *xyz, int64_t n,
                            const float origin[3], int64_t frame_id, void *stream);

/* Section 3.3 "Sliding-Window TSDF": bound the map to a box of blocks[a]
 * voxel blocks (8 voxels each) per axis that follows the sensor.  At the
 * first frame, and at every frame whose sensor voxel lies farther than 30 % of
 * the window's size (8 blocks[a] voxels) from the window's centre along some
 * axis, the window is re-centred on the sensor's voxel c: it then covers
 * blocks floor(c/8) - floor(blocks/2) .. + blocks - 1 on each axis, and
 * every block outside it is discarded before the frame (its voxels read
 * unknown again, W = 0; its memory is reused).  Frames write only voxels
 * inside the window and create surface points only there.  Points outside
 * keep their records and their last labels and are not scored; the normal's
 * neighbours are the points inside the window.  Memory then stays bounded
 * by the window (max_blocks of about blocks[0] blocks[1] blocks[2] suffice).
 * Call once, before the first frame; 2 <= blocks[a] <= 4096.  Allocates
 * 4 bytes per block and per point of capacity.  With the incremental mode
 * (Section 3.5), trigger (iii) re-queues only the inaccessible points inside
 * the window and the coarse-to-fine search takes its resolved neighbours
 * inside it; points outside have no voxel (W = 0: never selected, c = 0).
 * Frame graphs record the windowed frame (see af_graph_prepare);
 * af_score_tools lists the points and computes their normals once, then
 * scores the tools one after the other (their masks share one buffer).  Not
 * combinable with the smoothed score or variant tuning (those calls return
 * AF_EINVAL).  AF_EINVAL after a frame or once a frame graph is prepared. */
int af_set_window(af_ctx *ctx, const int32_t blocks[3]);
/* The window's current block box [lo, hi] (HOST arrays, either may be NULL)
 * and the number of shifts so far (the first placement is not a shift).
 * Returns 1 once placed, 0 before the first frame, AF_EINVAL without a
 * window. */
int af_window_state(af_ctx *ctx, int32_t lo[3], int32_t hi[3], int64_t *shifts);

/* Sections 3.4-3.5: label every surface point for tool `tool_id`: W < W_min
 * -> AF_UNSCORED; else candidates = orientations whose approach direction is
 * within the normal half-cone and seen from that side by a stored viewpoint;
 * the lowest-index candidate with no arm-sample hit (TSDF < r_c, or unknown
 * and not ray-cleared), fewer than n_c body voxels with TSDF < r_c and no
 * corridor voxel with TSDF < r_c is the point's first free orientation
 * (AF_ACCESSIBLE); none -> AF_BLOCKED; no candidate -> AF_NO_CANDIDATE.
 * Normal axes are kept between calls (this call and af_score_tools) and
 * recomputed only for points within 3 voxels of points added since; the
 * first call allocates that cache (32 bytes per point of capacity, 64 per
 * brick of the grid), AF_ENOMEM if the device budget cannot hold it.
 * Asynchronous on `stream`.  AF_ENOTOOL if the tool was never set.  With a
 * sliding window (af_set_window) only the points inside it are scored, with
 * normals computed afresh; the others keep their labels (AF_NOT_EVALUATED
 * if never scored); tools with K above 1024 or a reach above 255 voxels are
 * then refused (AF_EINVAL). */
int af_score_points(af_ctx *ctx, int32_t tool_id, void *stream);

/* Copy labels of points [first, first + count) in canonical order (by first
 * frame, then key) into HOST arrays (any may be NULL): voxel key, label,
 * first free orientation (-1 if none) and the point voxel's weight W.
 * Host arrays in pinned memory make the copies fast.  Synchronises the
 * context's last stream.  *n_written = number copied. */
int af_read_labels(af_ctx *ctx, int32_t tool_id, int64_t first, int64_t count,
                   int64_t *key, uint8_t *label, int16_t *first_free,
                   uint16_t *w, int64_t *n_written);

/* ---- inspection (tests and benchmarks); all synchronise ---- */
int64_t af_num_points(af_ctx *ctx);
int64_t af_num_blocks(af_ctx *ctx);
/* Every voxel with W > 0 or ray-cleared, unordered, into HOST arrays of
 * capacity cap; *n = number of such voxels (may exceed cap). */
int af_read_tsdf(af_ctx *ctx, int64_t *key, int64_t *S, int32_t *W,
                 uint8_t *cleared, int64_t cap, int64_t *n);
/* Point records in canonical order: key, first frame, stored viewpoints
 * (count and [8][3] fixed-point positions, oldest first), the running sum
 * of sensor positions ([3]) and its count. */
int af_read_points(af_ctx *ctx, int64_t first, int64_t count, int64_t *key,
                   int32_t *first_frame, int32_t *n_vp, int32_t *vp,
                   int64_t *sumq, int32_t *nq, int64_t *n_written);
/* Table of orientation k: offsets [m][3] and classes; *m = entry count. */
int af_read_tool_table(af_ctx *ctx, int32_t tool_id, int32_t k, int32_t *off,
                       uint8_t *cls, int64_t cap, int64_t *m);
/* Normals (int32 [3]: the oriented least principal axis in fixed point 2^30,
 * has_normal 1; 0 when the point has fewer than 3 neighbours, -1 when it is
 * not confident) and candidate masks ([ceil(K/64)] words) from the last
 * af_score_points of tool_id, for points [first, first+count). */
int af_read_point_debug(af_ctx *ctx, int32_t tool_id, int64_t first,
                        int64_t count, int32_t *normal, int32_t *has_normal,
                        uint64_t *mask, int64_t *n_written);
/* The PCA step of the normals (Section 3.4 "Approach directions") on
 * caller-given neighbourhoods, for tests: moments is a HOST array [n][10] of
 * (voxel count, sum of offsets [3], sum of offset products 00 01 02 11 12 22),
 * offsets in voxels; axes [n][3] receives the least principal axis of the
 * scatter count * sum(dd^T) - (sum d)(sum d)^T in fixed point 2^30 (unit
 * length, sign as the eigen-solver leaves it) and has[n] 1, or 0 and a zero
 * axis when the count is below 3.  No context; synchronous; uses its own
 * device buffers.  AF_EINVAL on n < 0 or NULL arrays, AF_EDEVICE on a HIP
 * error. */
int af_pca_axes(const int32_t *moments, int64_t n, int64_t *axes, int32_t *has);
int af_frame_stats_get(af_ctx *ctx, af_frame_stats *st);
int af_score_stats_get(af_ctx *ctx, int32_t tool_id, af_score_stats *st);
/* Bytes of device memory the context holds. */
int64_t af_device_bytes(af_ctx *ctx);

/* Per-stage device time, measured with hipEvents recorded on the call's own
 * stream around each stage (enabled by af_timing_enable; off by default).
 * Stages: whole integrate_frame work and its accumulation step (binning of
 * returns by block plus the per-block gather, fold and brick update); whole
 * score_points work and its normal, mask and score kernels.  Times in
 * milliseconds, summed over calls since the last reset. */
typedef struct af_timing {
  double integrate_ms, k_integrate_ms;
  double score_ms, k_normals_ms, k_mask_ms, k_score_ms;
  int64_t integrate_calls, score_calls;
  double k_smooth_ms;   /* af_smooth_refine kernels */
} af_timing;
int af_timing_enable(af_ctx *ctx, int on);
/* Synchronises the pending events, fills *out, and zeroes the sums if reset. */
int af_timing_read(af_ctx *ctx, af_timing *out, int reset);

/* Score every point against several tools (1..8, each with K <= 1024 and at
 * most 8200 orientations in total) in one persistent scoring launch: the
 * batching form of af_score_points (Section 3.4's tool kernels, one set per
 * tool).  Labels, first free orientations and statistics of each tool are
 * those af_score_points gives for it.  The first call for a tool gives it
 * its own candidate-mask buffers (3 K/8 bytes per point capacity), so the
 * tools' masks coexist.  Asynchronous on `stream`.  AF_EINVAL for a bad or
 * repeated id or too many orientations, AF_ENOTOOL for a tool without
 * kernels. */
int af_score_tools(af_ctx *ctx, const int32_t *tool_ids, int32_t n_tools, void *stream);

/* Scoring kernel configurations: "plain" (one orientation at a time, any K),
 * "swar" (candidate-parallel first entries, grid-relative lookups) and "near"
 * (arm samples taken from the mask pass), with unrolling, dynamic point
 * fetch, the 4^3-cell corridor skip ("coarse4") and the one-bit occupancy
 * plane ("bit") as options.  All give identical labels, first free
 * orientations and canonical counts; they differ in speed only.  A new
 * context uses af_score_variant_default(); configurations that need K <= 256
 * fall back to configuration 0 for larger K.  af_tune_score times every
 * configuration `reps` times on the
 * context's current map and tool (HIP events on `stream`), keeps the fastest
 * for later af_score_points calls, writes its index to *best and, if
 * ms_per_variant is not NULL, each configuration's mean time (host array of
 * af_score_variant_count() floats).  Synchronises `stream`. */
int af_score_variant_count(void);
int af_score_variant_default(void);
const char *af_score_variant_name(int32_t v);
int af_set_score_variant(af_ctx *ctx, int32_t v);
int32_t af_get_score_variant(af_ctx *ctx);
int af_tune_score(af_ctx *ctx, int32_t tool_id, int32_t reps, void *stream, int32_t *best,
                  float *ms_per_variant);

/* Recorded frame pipeline (the scan-centric update of Section 3.3 followed by
 * the per-point test of Section 3.5 for a set of tools, as one HIP graph).
 *
 * af_graph_prepare records, once, everything one frame does: integration of
 * up to `max_returns` returns, then normals, masks and the one-launch scoring
 * of tools `tool_ids[0..n_tools)` (as af_score_tools) over every point the
 * map then holds.  The brick grid is sized for the scene box [lo, hi]
 * (metres, merged with every block already mapped) and is not regrown while
 * the graph is in use, so no frame needs a host round trip.  Synchronises
 * `stream`.  AF_EINVAL for bad arguments or tools (as af_score_tools),
 * AF_ENOMEM, AF_EDEVICE if the capture fails; a failed call leaves no
 * recorded graph (af_graph_frame then returns AF_EINVAL).
 *
 * af_graph_frame replays the graph for one frame: `xyz` (device, n x 3 float,
 * n <= max_returns; may be af_graph_slot(), which skips a copy), sensor origin
 * and an increasing frame id as for af_integrate_frame.  Asynchronous on
 * `stream`; host-side counts and errors of replayed frames are settled by
 * af_graph_sync, which waits for them and reports AF_EOVERFLOW if any frame
 * since the last settlement overflowed the hash table, block or point
 * capacity, or mapped a block outside the recorded scene box (those frames'
 * results are then incomplete).  Every other call of this interface settles
 * first, so eager calls and replays may be mixed on one stream (a replay on
 * another stream than the previous one settles that one first).  A call that
 * reallocates a buffer the graph holds (a frame larger than the scratch
 * capacity, grid growth, af_set_tool_kernels) makes af_graph_frame return
 * AF_EINVAL until af_graph_prepare is called again.  Labels, first free
 * orientations, statistics and the map after each replay equal those of
 * af_integrate_frame followed by af_score_tools.
 *
 * With a sliding window (af_set_window, called first) the grid is the
 * window's and lo/hi are checked but not used; the recorded frame lists the
 * points inside the window and scores them tool by tool (as af_score_points
 * does with a window); tools must suit af_score_points with a window.  A
 * frame that places or moves the window (a host-side test on its origin)
 * runs eagerly instead -- af_integrate_frame, then af_score_tools over the
 * prepared tools -- and records the graph again for the new window (it
 * synchronises `stream`); a frame after a reallocation records the graph
 * again and replays it, instead of AF_EINVAL.
 * Labels, first free orientations, statistics and the map then equal those
 * of af_integrate_frame followed by af_score_points for each tool.  Before
 * the first frame the graph is recorded by that frame. */
int af_graph_prepare(af_ctx *ctx, const float lo[3], const float hi[3], int64_t max_returns,
                     const int32_t *tool_ids, int32_t n_tools, void *stream);
int af_graph_frame(af_ctx *ctx, const float *xyz, int64_t n, const float origin[3],
                   int64_t frame_id, void *stream);
float *af_graph_slot(af_ctx *ctx);
int af_graph_sync(af_ctx *ctx);

/* Smoothed clearance score (a differentiable form of the collision count of
 * Section 3.5, for refining approach directions between the K orientations):
 *
 *   s(p, q) = sum over samples o of log sigma((T(p + R(q/|q|) o) - c) / tau_s)
 *
 * T: the TSDF in metres, S/W of the map's voxels, read by trilinear
 * interpolation between voxel centres ((i, j, k) + 1/2) v; voxels without
 * weight, unallocated blocks and voxels outside the brick grid read the
 * truncation distance.  q = (w, x, y, z), any non-zero length; R(q/|q|) maps
 * the tool's local axes to world axes (its first column is the approach
 * direction).  samples: M x 3 points of the tool solid in its local frame
 * (metres, 1 <= M <= 1024).  Arithmetic is fp32 per sample; each pair's
 * position is split into voxel and fraction in double precision.
 *
 * af_smooth_eval: n pairs p[n x 3] (metres), q[n x 4]; writes s_out[n] (may
 * be NULL when gradients are asked for) and, if dq and dp are both given,
 * grad_s[i] * ds/dq (n x 4, through the normalisation) and grad_s[i] * ds/dp
 * (n x 3); grad_s NULL means 1.  All pointers are device memory; the map is
 * read as it stands after the calls before.  Asynchronous on `stream`.
 * AF_EINVAL for bad sizes or pointers.
 *
 * af_smooth_refine: for point i (p[n_points x 3]) and start j, the pair
 * i * n_starts + j starts from q0 (row-major, (n_points n_starts) x 4) and
 * takes `steps` ascent steps q <- (q + D) / |q + D| with D = eta ds/dq,
 * scaled down to length max_step if longer; q_out receives the final unit
 * quaternion and s_out its score.  Asynchronous on `stream`. */
int af_smooth_eval(af_ctx *ctx, const float *p, const float *q, int64_t n, const float *samples,
                   int32_t M, float c, float tau_s, const float *grad_s, float *s_out,
                   float *dq, float *dp, void *stream);
int af_smooth_refine(af_ctx *ctx, const float *p, int64_t n_points, const float *q0,
                     int32_t n_starts, const float *samples, int32_t M, float c, float tau_s,
                     int32_t steps, float eta, float max_step, float *q_out, float *s_out,
                     void *stream);

/* af_smooth_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, same kernels and bit-identical outputs, but its scratch
 * (the map's per-voxel values, brick tables, 9^3 apron bricks and work
 * counters) lives in a static 64 MiB device array that the library holds
 * on each GPU it runs on until the process ends; the call performs no
 * hipMalloc/hipFree.  The map must fit: about 2 KB per allocated block plus
 * 8 bytes per brick of the grid plus 2.9 KB per apron (at most 8 per block);
 * a larger map is refused with AF_ENOMEM and a message giving the need.
 * The grid must already cover the map (AF_EINVAL otherwise; every
 * af_integrate_frame keeps it so).  The array is shared by every call on one
 * GPU and keeps the last call's contents, so calls on one GPU must not
 * overlap in time (different streams or threads would race on it); each
 * call clears what it needs cleared.  The current device must be the
 * context's (AF_EINVAL).  Asynchronous on `stream`. */
int af_smooth_eval_static(af_ctx *ctx, const float *p, const float *q, int64_t n,
                          const float *samples, int32_t M, float c, float tau_s,
                          const float *grad_s, float *s_out, float *dq, float *dp, void *stream);

/* Incremental mode (Section 3.5, "Incremental Updates and Confidence"):
 * instead of re-testing every point each frame, a per-point state is kept
 * and a point is re-evaluated only when (i) the TSDF at its voxel moved by
 * more than 2v since the previous frame, (ii) a voxel within 3v of it
 * received a contribution -- judged from a sample of 256 of the frame's
 * changed voxels, those with the smallest SplitMix64 hash of
 * (voxel key XOR frame id * 0x9E3779B97F4A7C15) -- or (iii) the sensor moved
 * more than 0.1 m since the last time this fired and the point is labelled
 * AF_BLOCKED or AF_NO_CANDIDATE; new points are queued on first observation.
 * Queued points with W >= conf_min_w are evaluated, at most `budget` per
 * frame in point order; the rest stay queued.  An evaluation is the per-point
 * test of af_score_points; its score is the raw collision count (body voxels
 * with TSDF < r_c) of the first free orientation, n_c if none is free.  The
 * stored score only decreases (its orientation is kept with it); the
 * accessibility confidence a (1 at first) becomes 0.75 a when an evaluation
 * finds no free orientation while a free one is stored, and a + 0.15 (1 - a)
 * when it finds one.  Labels: AF_ACCESSIBLE iff the stored score is under
 * n_c and c a > 0.7 with c = W / (W + 5); AF_TENTATIVE when a score below
 * n_c is stored but c a <= 0.7; otherwise the last evaluation's AF_BLOCKED or
 * AF_NO_CANDIDATE; AF_UNSCORED before the first evaluation.
 *
 * af_incremental_enable: tool `tool_id` (K <= 1024, reach <= 255 voxels),
 * budget >= 1; before the context's first frame and before any frame graph
 * is prepared (AF_EINVAL otherwise).
 * Allocates the state (23 B per point of capacity) and a changed-voxel list
 * (4 B per voxel of block capacity).  af_incremental_frame integrates one
 * frame as af_integrate_frame does, then runs the steps above; it
 * synchronises `stream` once (inside the integration).  af_incremental_stats
 * synchronises and reports the counts of the last frame or drain.  af_read_incremental
 * copies state in canonical point order into host arrays (any may be NULL). */
typedef struct af_incr_stats {
  int64_t new_points, trig_i, trig_ii, trig_iii;   /* points queued by each cause */
  int64_t changed, sampled;                        /* changed voxels, sampled ones */
  int64_t queued, evaluated, backlog;              /* before selection, chosen, left */
  int64_t budget;                                  /* the cap the selection applied */
} af_incr_stats;
int af_incremental_enable(af_ctx *ctx, int32_t tool_id, int32_t budget);
int af_incremental_frame(af_ctx *ctx, const float *xyz, int64_t n, const float origin[3],
                         int64_t frame_id, void *stream);
/* Adaptive per-frame cap (Section 3.5's budget adapts to the frame; here to
 * a cost both the library and a checker count exactly): after a frame that
 * evaluated n > 0 points for L > 0 canonical lookups, the next frame's cap is
 * lookup_target * n / L (integer division) clamped to [b_min, b_max]; a frame
 * with no evaluation or no lookup keeps the cap.  lookup_target 0 keeps the
 * cap fixed.  The first frame's cap is the enable budget clamped to
 * [b_min, b_max].  Set after af_incremental_enable and before the first frame
 * (AF_EINVAL otherwise, or for b_min < 1, b_max < b_min, a negative or
 * > 2^40 target); grows the evaluation list to b_max entries (AF_ENOMEM). */
int af_incremental_budget(af_ctx *ctx, int64_t lookup_target, int32_t b_min, int32_t b_max);
/* Coarse-to-fine direction search (Section 3.6, "Accessibility scoring"):
 * each evaluation of the incremental mode tests only the orientations of a
 * coarse pass and of a fine window around the direction stored by the
 * closest resolved point.  Coarse pass: the orientations whose approach
 * direction a greedy walk in index order takes (a direction at least
 * coarse_deg from every direction taken before: dot <= cos + 1e-12), plus
 * the orientations sharing a taken direction.  Fine window of orientation
 * k*: the orientations within fine_deg of k*'s direction (dot >= cos -
 * 1e-12).  The nearest resolved neighbour of a point: the other point with a
 * stored free direction when the evaluation step starts, of smallest
 * (|d|^2, dz, dy, dx) with |d| <= radius_m (voxel offsets d); without one
 * only the coarse pass is searched.  The paper's setting is (20, 25, 0.3).
 * Set after af_incremental_enable and before the first frame; radius at most
 * 64 voxels (AF_EINVAL otherwise). */
int af_incremental_c2f(af_ctx *ctx, double coarse_deg, double fine_deg, double radius_m);
/* Consume the backlog between frames (Section 3.5: deferred evaluations are
 * done between LiDAR frames): evaluate up to max_evals queued points with
 * W >= conf_min_w in point order, update their state and every label, as a
 * frame's evaluation does, with no integration and no trigger; the frames'
 * cap is unchanged.  0 <= max_evals <= the largest cap (AF_EINVAL).
 * Asynchronous on `stream`.  af_incremental_stats then reports the drain
 * (zero trigger counts, budget = max_evals). */
int af_incremental_drain(af_ctx *ctx, int32_t max_evals, void *stream);
int af_incremental_stats(af_ctx *ctx, af_incr_stats *out);
int af_read_incremental(af_ctx *ctx, int64_t first, int64_t count, int64_t *key, uint8_t *label,
                        uint8_t *best, int16_t *best_dir, double *a, int64_t *n_written);

/* Serving several concurrent sensor streams (the real-time frame budget of
 * Section 3.6, for several sensors on one GPU).
 *
 * A server admits streams against a device budget: af_server_admit creates a
 * context from `cfg`, whose hbm_budget (> 0, bytes) is reserved against the
 * server's `hbm_budget`; AF_ENOMEM when it does not fit (nothing is
 * allocated then), AF_EBUSY when all `max_streams` (1..64) slots are taken.
 * Each stream keeps its map on the device until af_server_release, which also
 * returns its reservation.  af_server_context gives the stream's context (for
 * af_set_tool_kernels, af_read_labels and the other calls; the server owns
 * it) and af_server_hip_stream its HIP stream (non-blocking, default
 * priority), on which all of its frames run.
 *
 * af_server_prepare records the stream's frame graph (af_graph_prepare: scene
 * box lo/hi in metres, up to max_returns returns per frame, tools tool_ids)
 * and allocates four pinned host slots of max_returns returns; frames still
 * queued are dropped.  af_server_submit copies a frame (host xyz, n x 3
 * float) into a free slot and queues it: AF_EBUSY when four frames already
 * wait, AF_EINVAL for a stream without a recorded graph, n above max_returns
 * or a frame id that does not increase.  af_server_pending gives the queue
 * length (-1 for a bad id).  A stream whose context has a sliding window
 * (af_set_window on af_server_context, before af_server_prepare) records its
 * scoring in its own graph and is never batched; lo/hi are then unused.  A
 * stream whose context is in the incremental mode (af_incremental_enable,
 * before af_server_prepare) records no graph: af_server_prepare allocates a
 * device slot of max_returns returns (lo, hi and tool_ids unused), and each
 * step runs af_incremental_frame on the stream's HIP stream (it synchronises
 * that stream once, after block allocation, so such frames overlap the other
 * streams' work but not each other's first half).
 *
 * af_server_step takes the oldest queued frame of every stream (streams
 * visited round robin), launches each (host-to-device copy, then the recorded
 * frame) on its own HIP stream so that the GPU overlaps them, in batched mode
 * then the one scoring launch over all of them, then waits for all of them
 * and writes, for each frame processed, its stream id, frame id
 * and status (AF_OK, or the code af_graph_sync / af_graph_frame gave; a failed
 * frame is consumed) into the caller's arrays of `cap` >= max_streams
 * entries, and their number into *n_done.  Returns AF_EINVAL if the arrays
 * are too small, else AF_OK.  Not thread-safe: one host thread drives a
 * server. */
typedef struct af_server af_server;
int af_server_create(int64_t hbm_budget, int32_t max_streams, af_server **out);
/* Scoring the frames of all streams of a step in one launch: with
 * min_streams >= 2, each stream's recorded graph holds its integration,
 * normals and candidate masks, and a step in which at least min_streams
 * streams took a frame scores the points of all of them in ONE persistent
 * launch (each point against its own map and tools; at most 64 stream-tool
 * pairs per launch, further streams are scored on their own streams; more
 * than 64 KiB of table offsets fails the frames with AF_EDEVICE); a step
 * with fewer streams scores each on its own stream.  min_streams = 0: never
 * batch (each graph holds its own scoring launch, with the single-tool
 * kernel when the stream has one tool); 1 means 2.  Default 0: per-stream
 * launches run side by side on the runtime's hardware queues, and a stream
 * with one tool then scores with the single-tool kernel, which the
 * cross-stream launch cannot match; one launch also waits for the slowest
 * stream's masks.  Labels and counts are the same in every mode.  Set
 * before any stream is prepared (AF_EINVAL otherwise, or for
 * min_streams < 0). */
int af_server_batch(af_server *srv, int32_t min_streams);
int af_server_destroy(af_server *srv);
const char *af_server_last_error(af_server *srv);
int64_t af_server_reserved(af_server *srv);
int af_server_admit(af_server *srv, const af_config *cfg, int32_t *stream_id);
int af_server_release(af_server *srv, int32_t stream_id);
af_ctx *af_server_context(af_server *srv, int32_t stream_id);
void *af_server_hip_stream(af_server *srv, int32_t stream_id);
int af_server_prepare(af_server *srv, int32_t stream_id, const float lo[3], const float hi[3],
                      int64_t max_returns, const int32_t *tool_ids, int32_t n_tools);
int af_server_submit(af_server *srv, int32_t stream_id, const float *xyz, int64_t n,
                     const float origin[3], int64_t frame_id);
int32_t af_server_pending(af_server *srv, int32_t stream_id);
int af_server_step(af_server *srv, int32_t *stream_ids, int64_t *frame_ids, int32_t *status,
                   int32_t cap, int32_t *n_done);

#ifdef __cplusplus
}
#endif
#endif
