// Device-side data layout and kernel launchers of libaf (internal).
//
// Map: open-addressing hash of 8^3 voxel blocks (block key -> block id) over a
// block pool stored structure-of-arrays: S (int32) and W (uint16) per voxel,
// ray-cleared and surface bits (16 x uint32 per block).  A frame's
// contributions are summed per voxel in integers, so the result does not
// depend on the order in which returns are applied.
//
// Scoring reads a dense brick grid derived from the map after every fold: per
// 8^3 block position inside the bounding box of all blocks, 512 two-bit codes
// (bit 0: TSDF < r_c, bit 1: unknown and not ray-cleared) in 32 words, plus
// the 512 surface bits in 16 words, and one bit per brick telling whether any
// of its voxels has TSDF < r_c.  Positions outside the grid were never touched
// and read as unknown, not cleared.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "af.h"

namespace af {

constexpr int kBlockEdge = 8;
constexpr int kBlockVox = 512;
constexpr int64_t kKeyBias = 1LL << 20;
constexpr int64_t kKeyMask = (1LL << 21) - 1;
constexpr int64_t kCoordLim = (1LL << 28) - 4096;  // |P| bound, fixed-point units
constexpr int64_t kEmpty = -1;
constexpr int kMaxSpan = 27;      // blocks touched by one return's cube (R <= 7)
constexpr int kMaxBand = 18;      // band samples per return (1.25 tau / (v/2) for R <= 7)
constexpr int kMaxVp = 8;
constexpr int kTableMaxClass = 16384;
constexpr uint32_t kUnknownWord = 0xAAAAAAAAu;  // 16 voxels coded "unknown, not cleared"

// Status bits latched on the device.
constexpr int kStatusBlockOverflow = 1;
constexpr int kStatusPointOverflow = 2;
constexpr int kStatusHashFull = 4;
constexpr int kStatusOutsideGrid = 8;   // a block left the fixed grid's margin (recorded frames)

// Constants derived once from af_config (see af_context.hip).
struct Params {
  double scale;      // 256 / voxel: metres -> fixed-point units
  int32_t tau_u;     // truncation, units
  int32_t R;         // cube half-width, voxels
  int32_t rc_u;      // collision threshold, units
  int32_t n_c;
  int32_t cap;       // weight cap
  int32_t conf_min_w;
  int32_t n_vp;
  int32_t knn_k;
  int32_t clamp_neg;
  int32_t pad;
  int64_t dmin2;     // squared viewpoint novelty distance, units^2
  double cos2;       // cos_normal^2
  double obs2;       // obs_dot^2
};

// Per-frame device counters (zeroed at the start of each frame).
// Counters that many workgroups add to are spread over kStatSlots cache
// lines (slot = workgroup index mod kStatSlots): atomics on one address are
// serialised by the cache, so a single address would stall every workgroup.
constexpr int kStatSlots = 32;

struct FrameCounters {
  unsigned long long n_valid, n_dropped, pairs_applied, pairs_excluded;
  unsigned long long band_marks, voxels_folded;
  int32_t n_new_blocks, n_touched, n_new_points, status;
  int32_t n_changed;   // voxels that received a contribution (listed when fs.changed is set)
  int32_t bmin[3], bmax[3];
  int32_t blocks_before, points_before;
  int32_t free_before;   // evicted ids available when the frame started
  int32_t sticky;   // status bits of recorded frames since the host last looked (not reset per frame)
  int32_t sbmin[3], sbmax[3];   // block box of those frames (empty when sbmin > sbmax)
  int32_t snap_blocks, snap_points;   // block ids and points after the last recorded frame
  // per-slot fold statistics: [slot][0] applied pairs, [1] cone-excluded
  // pairs, [2] folded voxels (summed on the host; not part of the mid-frame
  // read of the fields above)
  unsigned long long fold[kStatSlots][16];
};

// One block of scoring counters; the device holds kStatSlots of them, one
// 128-byte line each (see kStatSlots), and the host sums them.
struct ScoreCounterBlock {
  unsigned long long n_confident, n_accessible, n_blocked, n_no_candidate;
  unsigned long long candidate_tests, canonical_tests, canonical_lookups;
  unsigned long long deep_tests, deep_chunks_max;  // diagnostics of the two-phase kernels
  unsigned long long coarse_checks, coarse_clear;   // corridor cell checks, and those clear
  unsigned long long chunks_body, chunks_far;       // 64-entry steps taken by deep scans
  unsigned long long arm_lookups;   // canonical arm-sample lookups answered by the mask kernel
  unsigned long long pad[2];
};

struct ScoreCounters {
  ScoreCounterBlock s[kStatSlots];
};

struct HashTable {
  int64_t *keys;   // kEmpty when free
  int32_t *vals;   // id, or -1 when the id could not be assigned
  uint32_t mask;   // capacity - 1 (power of two)
};

struct MapDev {
  HashTable h;
  int64_t *bkey;                 // [max_blocks]
  int32_t *S;                    // [max_blocks * 512]
  uint16_t *W;                   // [max_blocks * 512]
  uint32_t *clr;                 // [max_blocks * 16]
  uint32_t *surf;                // [max_blocks * 16]
  int32_t *touched;              // [max_blocks] last frame that touched the block
  int32_t *tpos;                 // [max_blocks] position in that frame's touched list
  int32_t *n_blocks;             // device counter (ids ever handed out)
  int64_t max_blocks;
  // sliding window only (null otherwise): ids of evicted blocks, reused
  // last-in first-out before n_blocks grows
  int32_t *free_ids;             // [max_blocks]
  int32_t *n_free;               // device counter
};

struct PointsDev {
  HashTable h;
  int64_t *key;       // [max_points]
  int32_t *first;     // first frame
  int32_t *addr;      // block id * 512 + voxel index of the point's voxel
  int32_t *last;      // last frame that updated the viewpoints
  int32_t *nvp;       // stored viewpoints
  int32_t *head;      // ring head
  int32_t *vp;        // [max_points * 8 * 3]
  int64_t *sumq;      // [max_points * 3]
  int32_t *nq;
  int32_t *normal;    // [max_points * 3]
  int32_t *has_normal;// 1 normal, 0 none, -1 not confident
  int32_t *n_points;  // device counter
  int64_t max_points;
  // optional point list: when sel is set, the normal, mask and default
  // scoring kernels visit points sel[0 .. *n_sel) instead of 0 .. n_points
  const int32_t *sel;
  const int32_t *n_sel;
};

// Per-frame scratch, sized for `cap` returns.
struct FrameScratch {
  int4 *P;            // fixed-point return + isqrt |P-Q| (0 when dropped)
  int32_t *span;      // [cap * kMaxSpan] block hash slots of the cube span
  int32_t *band;      // [cap * kMaxBand * 2] (hash slot, voxel index) pairs
  int32_t *pslot;     // [cap] point hash slot
  int32_t *new_blocks;// [cap * (kMaxSpan + kMaxBand)] hash slots of new blocks
  int64_t *new_keys;  // [cap] new point keys
  int64_t *new_sorted;  // [cap rounded up to 256] the new keys, sorted within each 256-key tile
  int32_t *new_kslot; // [cap] their hash slots
  int32_t *touched;   // [cap * (kMaxSpan + kMaxBand)] touched block ids
  int32_t *bin_cnt;   // [cap * (kMaxSpan + kMaxBand)] returns per touched block
  int32_t *bin_off;   // [cap * (kMaxSpan + kMaxBand) + 1] their prefix
  int32_t *bin_fill;  // [cap * (kMaxSpan + kMaxBand)] insertion cursors
  int32_t *bin_list;  // [cap * kMaxSpan] return ids grouped by block
  int64_t cap;
  int32_t *changed;   // null, or [max_blocks * 512]: voxel addresses (block * 512 + index)
                      // that received a contribution this frame (incremental mode)
};

struct GridDev {
  uint32_t *pred;     // [nbricks * 32]
  uint32_t *surf;     // [nbricks * 16]
  uint32_t *occ_any;  // [ceil(nbricks / 32)] brick holds a voxel with TSDF < r_c
  uint8_t *occ4;      // [nbricks] bit (x>>2) | (y>>2) << 1 | (z>>2) << 2: that 4^3 octant does
  uint32_t *occ1;     // [nbricks * 16] one bit per voxel (linear x | y << 3 | z << 6): TSDF < r_c
  int32_t g0[3];      // block coordinate of brick (0,0,0)
  int32_t gd[3];      // bricks per axis
  int32_t margin;     // bricks every block keeps from the grid's faces
};

struct ToolDev {
  int32_t K;
  uint32_t *entries;  // packed offsets + class
  uint32_t *begin;    // [K + 1]
  double *rot;        // [K * 9]
  uint8_t *label;     // [max_points]
  int16_t *first_free;// [max_points]
  uint64_t *mask;     // [max_points * ceil(K/64)]
  // arm-sample result per candidate orientation as two bit planes per mask
  // word: 0 no arm sample hits, 1..3 the first hit is arm sample 0..2
  uint64_t *nearp;    // [max_points * 2 * ceil(K/64)]
  ScoreCounters *counters;
  uint32_t *far_begin;  // [K] index of the first corridor entry
  // bit k set: orientation k has the same approach direction (first column
  // of its rotation) as orientation k - 1, so its candidate bit is the same
  uint64_t *same;       // [ceil(K / 64)]
  // coarse corridor lists over 4^3-voxel cells: for orientation k, the cell
  // offsets (relative to the point's cell) that its corridor entries can fall
  // in, for any position of the point inside its cell
  uint32_t *c4begin;    // [K + 1]
  uint32_t *c4entries;
  uint8_t *c4flag;      // [K] 1: list valid
  int64_t n_c4entries;
  // grid-relative form of the table for the current brick grid: per entry
  // {brick delta (ox>>3) + gx (oy>>3) + gx gy (oz>>3), in-brick offsets
  // (ox&7) | (oy&7) << 4 | (oz&7) << 8 | class << 30}.  Rebuilt whenever the
  // grid is reallocated.
  uint2 *xent;          // [entries]
  // grid-independent 4-byte form, when every offset component is within
  // +-255: (ox + 256) | (oy + 256) << 10 | (oz + 256) << 20 | class << 30
  uint32_t *rent;       // [entries] or null
  int64_t n_entries;
  int32_t reach;        // largest |offset| component over the table, voxels
};

// Table entry packing: 10-bit two's complement offsets, class in bits 30-31.
__host__ __device__ inline uint32_t pack_entry(int ox, int oy, int oz, int cls) {
  return (uint32_t)(ox & 1023) | ((uint32_t)(oy & 1023) << 10) |
         ((uint32_t)(oz & 1023) << 20) | ((uint32_t)cls << 30);
}
__host__ __device__ inline int entry_x(uint32_t e) { return (int)(e << 22) >> 22; }
__host__ __device__ inline int entry_y(uint32_t e) { return (int)(e << 12) >> 22; }
__host__ __device__ inline int entry_z(uint32_t e) { return (int)(e << 2) >> 22; }
__host__ __device__ inline int entry_cls(uint32_t e) { return (int)(e >> 30); }

// Open-addressing hash (linear probing) shared by the block and point maps.
__device__ inline uint32_t slot_of(int64_t key, uint32_t mask) {
  uint64_t h = (uint64_t)key * 0x9E3779B97F4A7C15ull;
  return (uint32_t)(h >> 29) & mask;
}

__device__ inline int32_t hash_find(HashTable t, int64_t key) {
  uint32_t s = slot_of(key, t.mask);
  for (uint32_t i = 0; i <= t.mask; ++i) {
    int64_t cur = t.keys[s];
    if (cur == key) return (int32_t)s;
    if (cur == kEmpty) return -1;
    s = (s + 1) & t.mask;
  }
  return -1;
}

__host__ __device__ inline int64_t pack_key(int64_t x, int64_t y, int64_t z) {
  return ((x + kKeyBias) & kKeyMask) | (((y + kKeyBias) & kKeyMask) << 21) |
         (((z + kKeyBias) & kKeyMask) << 42);
}
__host__ __device__ inline void unpack_key(int64_t k, int32_t &x, int32_t &y, int32_t &z) {
  x = (int32_t)((k & kKeyMask) - kKeyBias);
  y = (int32_t)(((k >> 21) & kKeyMask) - kKeyBias);
  z = (int32_t)(((k >> 42) & kKeyMask) - kKeyBias);
}

struct ToolGeom {     // tool constants in voxel units (host-derived, fp64)
  int32_t shape;
  int32_t pad;
  double Lv, Ev;      // body end, corridor end
  double a, b;        // half cross-section (cylinder: a = b = radius)
  double rv2;         // cylinder radius^2
  double rsv2;        // self-exclusion radius^2
  double lam[3];      // arm samples
};

// ---- launchers (stream-ordered) ----
// Per-frame parameters read by the integration kernels from device memory
// (so that a recorded frame graph can be replayed with new values).
struct FrameArgs {
  int64_t n;      // returns in the frame
  int3 Q;         // quantised sensor origin
  int32_t frame;  // frame id
  int3 wlo, whi;  // block box the frame may write (the sliding window; else unbounded)
};
// clear: when set, also resets the sticky status and block box of c (the
// first recorded frame after the host read them)
void launch_set_frame_args(FrameArgs *fa, int64_t n, int3 Q, int32_t frame, int3 wlo, int3 whi,
                           hipStream_t s, FrameCounters *clear = nullptr);

// Cached normal axes (state: -2 pending, 0 none, 1 axis valid).
struct NormalCache {
  int64_t *axis;      // [max_points * 3]
  int32_t *state;     // [max_points]
  int32_t *list;      // [max_points] points whose axis is recomputed
  int32_t *count;
  uint32_t *stale;    // [grid bricks * 16] voxels near new points; zero between calls
  int64_t stale_words;
};
// Normals of points [0, n) where only the axes of points within +-3 voxels of
// points [seen, n) are recomputed; `seen` is n of the previous call (0: all).
// nc.stale must cover the current grid.
void launch_normals_cached(const Params &p, MapDev m, PointsDev pts, GridDev g,
                           const NormalCache &nc, int64_t seen, int64_t n, hipStream_t s);

// Incremental mode: per-point state and per-frame scratch.
struct IncrCounters {
  int32_t new_points, trig_i, trig_ii, trig_iii;
  int32_t sampled, n_cand, queued, selectable;
  int32_t b1, b2, need, take_all;   // sample selection: top bin, second bin, count, all
};
struct IncrDev {
  uint8_t *best;          // [max_points] stored score; n_c = no free direction stored
  int16_t *best_dir;      // its orientation, -1 none
  double *a;              // accessibility confidence
  int32_t *S_prev;        // S, W of the point's voxel after the previous frame
  uint16_t *W_prev;
  uint32_t *pending;      // queued for evaluation
  uint8_t *outcome;       // label of the last evaluation (AF_UNSCORED: never)
  uint8_t *label;         // incremental label
  int32_t *sel;           // [budget] points evaluated this frame
  int32_t *n_sel;
  int32_t *bsum;          // [ceil(max_points / 1024)] selection block counts / offsets
  uint8_t *score_new;     // [budget] raw collision count of this frame's evaluation
  uint32_t *hist;         // [2 * 65536] sample histograms
  unsigned long long *cand_h;   // [1024] sample candidates: hash, key
  int64_t *cand_k;
  int64_t *sampled;       // [256] sampled changed voxels (keys)
  IncrCounters *ctr;
  int32_t *budget_dev;    // the cap the selection applies (this frame's, or a drain's)
  int32_t *frame_budget;  // the frames' cap (fixed, or adapted after every frame)
  int64_t max_points;
  int32_t budget;         // capacity of sel / score_new: the largest cap
  // adaptive cap: after a frame that evaluated n > 0 points for L > 0
  // canonical lookups, frame_budget = clamp(lookup_target * n / L, b_min,
  // b_max); lookup_target 0 keeps the cap fixed
  int64_t lookup_target;
  int32_t b_min, b_max;
  // coarse-to-fine direction search (Section 3.6), when c2f_on: the coarse
  // pass [mw] and the fine window of every orientation [K][mw] as allowed-
  // orientation masks; the neighbour offsets within the search radius
  // (x + 512 | (y + 512) << 10 | (z + 512) << 20), sorted by
  // (|d|^2, dz, dy, dx), zero excluded; a bit plane over the brick grid
  // (16 words per brick) of the resolved points' voxels, and their count
  int32_t c2f_on, c2f_mw, c2f_n_off;
  uint64_t *c2f_coarse, *c2f_fine;
  uint32_t *c2f_off;
  uint32_t *resolved;
  int32_t *n_resolved;
  // the sliding window's block box (unbounded without one): trigger (iii)
  // and the resolved neighbours only take points inside it
  int3 wlo, whi;
};
void launch_incr_init(const IncrDev &I, int32_t n_c, hipStream_t s);
void launch_incr_frame_front(PointsDev pts, MapDev m, const IncrDev &I, const int32_t *changed,
                             const FrameCounters *fc, int64_t n_points, int64_t seen, int32_t frame,
                             bool moved, int32_t min_w, hipStream_t s);
void launch_incr_frame_back(PointsDev pts, MapDev m, ToolDev t, GridDev g, const IncrDev &I,
                            int64_t n_points, int32_t n_c, hipStream_t s);
// Selection only (no trigger): a drain's list of up to max_evals queued points.
void launch_incr_drain_front(PointsDev pts, MapDev m, const IncrDev &I, int64_t n_points,
                             int32_t max_evals, int32_t min_w, hipStream_t s);
// Coarse-to-fine restriction of the listed points' candidate masks: mark the
// resolved points in the plane (cleared first, grid_bricks bricks), then
// AND each listed point's mask with the coarse pass and the fine window of
// its nearest resolved neighbour's stored direction.
void launch_incr_c2f(PointsDev pts, ToolDev t, GridDev g, const IncrDev &I, int64_t n_points,
                     int64_t grid_bricks, int32_t n_c, hipStream_t s);
// Set the frames' cap (and the selection's) to b.
void launch_incr_set_budget(const IncrDev &I, int32_t b, hipStream_t s);
// After a frame's evaluation: the next frame's cap from its cost.
void launch_incr_budget(const IncrDev &I, const ToolDev &t, hipStream_t s);

// Smoothed clearance score.  T9: apron bricks of 9^3 floats (a brick's 8^3
// voxels and the first layer of its +1 neighbours; tau where unmapped);
// bid9: apron index of every brick of the dense grid (-1: no mapped voxel
// within reach of a cell based in that brick).
struct SmoothField {
  const float *T9;
  const int32_t *bid9;
  int32_t g0[3], gd[3];
  float tau;            // metres
};
struct SmoothBuffers {
  float *T;             // [n_blocks * 512] per-voxel values (intermediate)
  int32_t *bid;         // [grid bricks] block id or -1 (intermediate)
  int32_t *bid9;        // [grid bricks]
  int32_t *brick_of;    // [apron_cap] grid brick of each apron
  float *T9;            // [apron_cap * 729]
  int32_t *count;       // aprons made
  unsigned long long *work;   // [8] pairs handed out from each XCD's range
  int64_t apron_cap;
};
void launch_smooth_prepare(const Params &p, MapDev m, int64_t n_blocks, GridDev g,
                           int64_t grid_bricks, float tau, const SmoothBuffers &b,
                           hipStream_t s);
void launch_smooth_eval(const SmoothField &f, double v, const float *p, const float *q, int64_t n,
                        const float *samples, int32_t M, float c, float tau_s,
                        const float *grad_s, float *s_out, float *dq, float *dp,
                        unsigned long long *work, hipStream_t s);
void launch_smooth_refine(const SmoothField &f, double v, const float *p, int64_t n_points,
                          const float *q0, int32_t n_starts, const float *samples, int32_t M,
                          float c, float tau_s, int32_t steps, float eta, float max_step,
                          float *q_out, float *s_out, unsigned long long *work, hipStream_t s);
// a recorded frame's end: status and block box into the sticky fields, and
// the block and point counts into the snapshot the host reads
void launch_stick_status(FrameCounters *c, const int32_t *n_blocks, const int32_t *n_points,
                         hipStream_t s);
void launch_zero_words(void *p, int64_t bytes, hipStream_t s);   // a fill kernel (graph-safe)
// nb: an upper bound of the frame's returns (sizes the launches)
void launch_frame_prep(const float *xyz, const FrameArgs *fa, int64_t nb, const Params &p,
                       MapDev m, PointsDev pts, FrameScratch fs, FrameCounters *c,
                       hipStream_t s);
void launch_assign_blocks(MapDev m, FrameScratch fs, FrameCounters *c, const FrameArgs *fa,
                          hipStream_t s);
void launch_commit_blocks(MapDev m, FrameCounters *c, hipStream_t s);
void launch_integrate(const FrameArgs *fa, int64_t nb, const Params &p, MapDev m,
                      FrameScratch fs, FrameCounters *c, GridDev g, int64_t max_touched,
                      hipStream_t s);
void launch_touch_band(const FrameArgs *fa, int64_t nb, const Params &p, MapDev m,
                       FrameScratch fs, FrameCounters *c, hipStream_t s);
void launch_points_append(int64_t n_new, MapDev m, PointsDev pts, FrameScratch fs,
                          FrameCounters *c, const FrameArgs *fa, hipStream_t s);
void launch_commit_points(PointsDev pts, FrameCounters *c, hipStream_t s);
void launch_points_view(const FrameArgs *fa, int64_t nb, const Params &p, PointsDev pts,
                        FrameScratch fs, hipStream_t s);
// Sliding window (Section 3.3).  On a shift, before the frame: blocks
// outside the new box [lo, hi] are cleared and their ids freed, the block
// hash is rebuilt from the live blocks, and points outside the box lose their
// voxel address.  In the shifting frame, between prep and block assignment,
// the blocks of points back inside the box are inserted (thaw); after
// assignment those points get their address and surface bit again (link).
void launch_window_evict(MapDev m, PointsDev pts, int64_t n_blocks, int64_t n_points, int3 lo,
                         int3 hi, hipStream_t s);
void launch_window_thaw(MapDev m, PointsDev pts, FrameScratch fs, FrameCounters *c,
                        int64_t n_points, int3 lo, int3 hi, hipStream_t s);
void launch_window_link(MapDev m, PointsDev pts, int64_t n_points, int3 lo, int3 hi,
                        hipStream_t s);
// Points of [0, n_points) inside the box, listed into sel (count in *n_sel).
// dev_n: n_points bounds the launch and the count is read on the device
void launch_window_list(PointsDev pts, int64_t n_points, int3 lo, int3 hi, int32_t *sel,
                        int32_t *n_sel, hipStream_t s, bool dev_n = false);
// label[i] = 255 (never evaluated), first_free[i] = -1 for i in [from, to).
void launch_label_fill(uint8_t *label, int16_t *first_free, int64_t from, int64_t to,
                       hipStream_t s);
void launch_grid_fill(GridDev g, hipStream_t s);
void launch_grid_rebuild(const Params &p, MapDev m, GridDev g, int64_t n_blocks,
                         hipStream_t s);

int launch_table_build(const ToolGeom &tg, int32_t K, const double *rot_dev,
                       uint32_t *counts_dev, uint32_t *begin_dev, int32_t *err_dev,
                       uint32_t *entries_dev, int pass, hipStream_t s);

int launch_table_grid(const ToolDev &t, const GridDev &g, hipStream_t s);
int launch_table_coarse(int32_t K, const uint32_t *begin, const uint32_t *counts,
                        const uint32_t *entries, uint32_t *far_begin, uint32_t *ccounts,
                        uint32_t *cbegin, uint32_t *centries, uint8_t *cflag, int pass, int sh,
                        hipStream_t s);

// dev_n: the kernels take the point count from the device counter; n_points
// is then only an upper bound that sizes the launch
void launch_normals(const Params &p, MapDev m, PointsDev pts, GridDev g,
                    int64_t n_points, hipStream_t s, bool dev_n = false);
void launch_pca_axes(const int32_t *mom, int64_t n, int64_t *axes, int32_t *has,
                     hipStream_t s);
void launch_mask(const Params &p, PointsDev pts, ToolDev t, GridDev g, int64_t n_points,
                 hipStream_t s, bool dev_n = false);
// Up to kMultiTools tools scored in one launch: their ids in the context's
// device mirror of the tool table and the offsets of their begin arrays in
// the launch's LDS copy (passed by value).
constexpr int kMultiTools = 8;
struct ToolSet {
  int32_t n;
  int32_t id[kMultiTools];
  int32_t base[kMultiTools];
};
int multi_begin_capacity();
void launch_score_multi(const Params &p, PointsDev pts, const ToolDev *tools_dev,
                        const ToolDev *host_tools, const ToolSet &set, GridDev g, int64_t n,
                        unsigned *work, hipStream_t s, bool dev_n = false);
void launch_score(const Params &p, PointsDev pts, ToolDev t, GridDev g, int64_t n_points,
                  int variant, unsigned *work, hipStream_t s, bool dev_n = false);
// One job of a cross-map scoring launch: every point of one context's map
// (its point count read on the device) against one of its tools.
struct ScoreJob {
  Params p;
  PointsDev pts;
  ToolDev t;
  GridDev g;
  int32_t base;        // offset of the tool's begin offsets in the launch's LDS
  int32_t pad;
  int64_t max_points;  // capacity of the map (sizes the launch)
};
constexpr int kMaxJobs = 64;
// One persistent launch over n_jobs jobs (jobs_dev: their device copy);
// -1 when a tool has more than kNearK orientations or the tables exceed LDS.
int launch_score_jobs(const ScoreJob *jobs_dev, const ScoreJob *jobs_host, int32_t n_jobs,
                      unsigned *work, hipStream_t s);
// For the server: record a context's frame graph without its scoring launch
// (integration, normals and masks of the tools), and describe its scoring
// jobs (one per tool) for a cross-map launch.
int ctx_graph_prepare_unscored(af_ctx *c, const float lo[3], const float hi[3],
                               int64_t max_returns, const int32_t *tool_ids, int32_t n_tools,
                               void *stream);
int ctx_score_jobs(af_ctx *c, const int32_t *tool_ids, int32_t n_tools, ScoreJob *out);
// Score such a frame on its own stream instead (what the scored graph does).
int ctx_score_stream(af_ctx *c, const int32_t *tool_ids, int32_t n_tools, void *stream);
// A context with a sliding window (its frames are scored inside its own graph,
// over the window's point list, so the server does not batch it).
bool ctx_windowed(const af_ctx *c);
// A context in the incremental mode (its frames run af_incremental_frame,
// eagerly, from a device slot of max_returns returns that ctx_frame_slot
// allocates; af_graph_slot returns it).
bool ctx_incremental(const af_ctx *c);
int ctx_frame_slot(af_ctx *c, int64_t max_returns);
int score_variants();
int score_variant_default();
// whether the configuration (after its fallbacks for this tool) honours PointsDev::sel
bool score_variant_takes_list(int variant, const ToolDev &t);
const char *score_variant_name(int v);

}  // namespace af
