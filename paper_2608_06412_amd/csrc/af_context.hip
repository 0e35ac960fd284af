// libaf host side: context and device memory, the C ABI of include/af.h and
// the stream-ordered sequence of kernels per call.
#include <math.h>
#include <stddef.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <cmath>
#include <string>
#include <vector>

#include "af_internal.h"

using namespace af;

struct af_ctx {
  af_config cfg;
  Params p;
  double tau;          // resolved truncation, metres
  int device;
  int64_t bytes;       // device bytes held
  std::vector<void *> allocs;
  MapDev map;
  PointsDev pts;
  FrameScratch fs;
  GridDev grid;
  int64_t grid_bricks;
  FrameCounters *counters;      // device
  FrameCounters *counters_host; // pinned
  std::vector<ToolDev> tools;
  std::vector<int64_t> tool_bytes;
  uint64_t *mask;               // shared candidate-mask scratch
  uint64_t *nearp;              // shared arm-sample planes
  ToolDev *tools_dev;           // device mirror of `tools` (for the multi-tool launch)
  FrameArgs *fargs;             // device: the current frame's n, origin, id
  // recorded frame pipeline (af_graph_prepare)
  hipGraph_t graph;
  hipGraphExec_t gexec;
  hipStream_t cap_stream;
  float *slot_xyz;              // device frame slot
  int64_t slot_cap;
  bool graph_dirty;             // recorded frames ran since the host mirrors were refreshed
  bool graph_stale;             // a buffer the graph holds was reallocated
  bool sticky_reset;            // the host has read the sticky status: the next frame clears it
  // what the graph was prepared with (a windowed context records it again
  // after every shift of the window)
  int32_t g_ids[kMultiTools];
  int32_t g_n;                  // tools of the prepared graph (0: none)
  bool g_score;
  // incremental mode
  bool incr_on;
  int32_t incr_tool;
  IncrDev incr;
  int32_t *incr_changed;        // [max_blocks * 512] changed voxel addresses of a frame
  int32_t q_last[3];            // sensor position when trigger (iii) last fired
  int64_t incr_seen;            // points that already have a state
  bool have_q;
  // smoothed score: apron bricks and their tables (SmoothBuffers), grown on demand
  SmoothBuffers sm;
  int64_t sm_T_cap;             // voxels of sm.T
  int64_t sm_bid_cap;           // bricks of sm.bid and sm.bid9
  // cached normal axes of the eager scoring calls (allocated on first use)
  NormalCache ncache;
  int64_t nc_seen;              // points whose neighbourhood the cache reflects
  std::vector<char> own_mask;   // tool has its own mask and plane buffers
  int32_t incr_budget0;         // the cap given to af_incremental_enable
  int64_t c2f_plane_bricks;     // bricks the coarse-to-fine resolved plane covers
  unsigned *work;               // point counter of the dynamic score variants
  // device copy of host-given returns (af_integrate_frame_host), grown on demand
  float *host_xyz;
  int64_t host_xyz_cap;         // returns it holds
  int score_variant;
  int64_t last_frame;
  int64_t n_points, n_blocks;   // host mirrors after the last frame
  int32_t bbox_lo[3], bbox_hi[3];
  bool have_bbox;
  // sliding window (af_set_window): L blocks per axis, centred (in voxels)
  // on the sensor of the frame that last shifted it; blocks [lo, hi]
  bool win_on, win_set;
  int32_t win_L[3], win_c[3], win_lo[3], win_hi[3];
  int64_t win_shifts;
  int32_t *win_sel, *win_nsel;  // device: points inside the window (scoring list)
  std::vector<int64_t> label_init;  // per tool: points whose label slot has been initialised
  hipStream_t last_stream;
  af_frame_stats fstats;
  std::string err;
  int status;
  // stage timing (hipEvents on the call's stream)
  bool timing;
  std::vector<hipEvent_t> ev_free, ev_inflight;
  struct Pending { int stage; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double stage_ms[6];
  int64_t integrate_calls, score_calls;
};

namespace {

const char *kNoError = "no error";

int fail(af_ctx *c, int code, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIP_TRY(ctx, expr)                                                             \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, AF_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                           \
  } while (0)

int dev_alloc(af_ctx *c, void **p, int64_t bytes) {
  if (bytes <= 0) bytes = 8;
  if (c->cfg.hbm_budget > 0 && c->bytes + bytes > c->cfg.hbm_budget)
    return fail(c, AF_ENOMEM, "HBM budget of %lld bytes exceeded (need %lld more)",
                (long long)c->cfg.hbm_budget, (long long)bytes);
  hipError_t e = hipMalloc(p, (size_t)bytes);
  if (e != hipSuccess) return fail(c, AF_ENOMEM, "hipMalloc(%lld): %s", (long long)bytes, hipGetErrorString(e));
  c->bytes += bytes;
  c->allocs.push_back(*p);
  return AF_OK;
}

void dev_free(af_ctx *c, void *p, int64_t bytes) {
  if (!p) return;
  hipFree(p);
  c->bytes -= bytes;
  c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), p), c->allocs.end());
}

uint32_t pow2_at_least(int64_t n) {
  uint64_t c = 1;
  while ((int64_t)c < n) c <<= 1;
  return (uint32_t)c;
}

#define ALLOC(ctx, ptr, count)                                                            \
  do {                                                                                    \
    int rc_ = dev_alloc(ctx, (void **)&(ptr), (int64_t)sizeof(*(ptr)) * (int64_t)(count)); \
    if (rc_ != AF_OK) return rc_;                                                         \
  } while (0)

int alloc_scratch(af_ctx *c, int64_t cap) {
  c->graph_stale = true;
  FrameScratch &f = c->fs;
  if (f.cap > 0) {
    dev_free(c, f.P, sizeof(int4) * f.cap);
    dev_free(c, f.span, sizeof(int32_t) * f.cap * kMaxSpan);
    dev_free(c, f.band, sizeof(int32_t) * f.cap * kMaxBand * 2);
    dev_free(c, f.pslot, sizeof(int32_t) * f.cap);
    dev_free(c, f.new_blocks, sizeof(int32_t) * f.cap * (kMaxSpan + kMaxBand));
    dev_free(c, f.new_keys, sizeof(int64_t) * f.cap);
    dev_free(c, f.new_sorted, sizeof(int64_t) * ((f.cap + 255) / 256 * 256));
    dev_free(c, f.new_kslot, sizeof(int32_t) * f.cap);
    dev_free(c, f.touched, sizeof(int32_t) * f.cap * (kMaxSpan + kMaxBand));
    dev_free(c, f.bin_cnt, sizeof(int32_t) * f.cap * (kMaxSpan + kMaxBand));
    dev_free(c, f.bin_off, sizeof(int32_t) * (f.cap * (kMaxSpan + kMaxBand) + 1));
    dev_free(c, f.bin_fill, sizeof(int32_t) * f.cap * (kMaxSpan + kMaxBand));
    dev_free(c, f.bin_list, sizeof(int32_t) * f.cap * kMaxSpan);
    memset(&f, 0, sizeof(f));
  }
  ALLOC(c, f.P, cap);
  ALLOC(c, f.span, cap * kMaxSpan);
  ALLOC(c, f.band, cap * kMaxBand * 2);
  ALLOC(c, f.pslot, cap);
  ALLOC(c, f.new_blocks, cap * (kMaxSpan + kMaxBand));
  ALLOC(c, f.new_keys, cap);
  ALLOC(c, f.new_sorted, (cap + 255) / 256 * 256);
  ALLOC(c, f.new_kslot, cap);
  ALLOC(c, f.touched, cap * (kMaxSpan + kMaxBand));
  ALLOC(c, f.bin_cnt, cap * (kMaxSpan + kMaxBand));
  ALLOC(c, f.bin_off, cap * (kMaxSpan + kMaxBand) + 1);
  ALLOC(c, f.bin_fill, cap * (kMaxSpan + kMaxBand));
  ALLOC(c, f.bin_list, cap * kMaxSpan);
  f.cap = cap;
  return AF_OK;
}

int hip_check(af_ctx *c, const char *where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, AF_EDEVICE, "%s: %s", where, hipGetErrorString(e));
  return AF_OK;
}

// Bricks of margin the grid keeps around every allocated block: every table
// lookup of a point (its brick plus any offset of any tool) stays inside the
// grid, so lookups need no bounds test.
int32_t grid_margin_need(const af_ctx *c) {
  int32_t need = 4;
  for (const ToolDev &t : c->tools)
    if (t.entries) need = std::max<int32_t>(need, (t.reach + 7) / 8 + 1);
  return need;
}

// Grow the brick grid so that it covers block box [lo, hi] with the margin
// above; new grids are filled with "unknown" (the caller rebuilds them from
// every block) and every tool's grid-relative table is recomputed.
// Whether the grid covers the block box with the margin every tool needs.
static bool grid_covers(const af_ctx *c) {
  if (!c->have_bbox) return true;
  const GridDev &g = c->grid;
  const int32_t need = grid_margin_need(c);
  bool inside = c->grid_bricks > 0;
  for (int a = 0; a < 3 && inside; ++a)
    inside = c->bbox_lo[a] - g.g0[a] >= need && g.g0[a] + g.gd[a] - 1 - c->bbox_hi[a] >= need;
  return inside;
}

int ensure_grid(af_ctx *c, hipStream_t s, bool &rebuilt, bool force = false) {
  rebuilt = false;
  if (!force && grid_covers(c)) return AF_OK;
  const int32_t need = grid_margin_need(c);
  GridDev &g = c->grid;
  GridDev ng;
  memset(&ng, 0, sizeof(ng));
  int64_t nb = 1;
  for (int a = 0; a < 3; ++a) {
    int32_t ext = c->bbox_hi[a] - c->bbox_lo[a] + 1;
    // a growing map gets a quarter of its extent as slack; a window's box
    // never grows, so its grid holds the tools' margin only
    int32_t margin = c->win_on ? need : std::max<int32_t>(need, ext / 4);
    ng.g0[a] = c->bbox_lo[a] - margin;
    ng.gd[a] = ext + 2 * margin;
    nb *= ng.gd[a];
  }
  ng.margin = need;
  if (nb * 128 >= (int64_t(1) << 32))
    return fail(c, AF_ENOMEM, "brick grid of %lld bricks exceeds 4 GiB", (long long)nb);
  // the lookups multiply brick strides in 24 bits (always true here: every
  // axis spans at least 2 * 4 + 1 bricks)
  if ((int64_t)ng.gd[0] * ng.gd[1] >= (int64_t(1) << 24))
    return fail(c, AF_ENOMEM, "brick grid of %d x %d bricks per layer", ng.gd[0], ng.gd[1]);
  c->graph_stale = true;
  if (c->grid_bricks == nb && g.gd[0] == ng.gd[0] && g.gd[1] == ng.gd[1] && g.gd[2] == ng.gd[2]) {
    // same extent at a new origin (a window shift): keep the buffers
    ng.pred = g.pred;
    ng.surf = g.surf;
    ng.occ_any = g.occ_any;
    ng.occ4 = g.occ4;
    ng.occ1 = g.occ1;
    c->grid = ng;
    launch_grid_fill(c->grid, s);
    for (const ToolDev &t : c->tools)
      if (t.entries && launch_table_grid(t, c->grid, s) != 0) return hip_check(c, "table grid");
    rebuilt = true;
    return hip_check(c, "grid fill");
  }
  if (c->grid_bricks > 0) {
    HIP_TRY(c, hipStreamSynchronize(s));
    dev_free(c, g.pred, sizeof(uint32_t) * 32 * c->grid_bricks);
    dev_free(c, g.surf, sizeof(uint32_t) * 16 * c->grid_bricks);
    dev_free(c, g.occ_any, sizeof(uint32_t) * ((c->grid_bricks + 31) / 32));
    dev_free(c, g.occ4, c->grid_bricks);
    dev_free(c, g.occ1, sizeof(uint32_t) * 16 * c->grid_bricks);
    c->grid_bricks = 0;
  }
  ALLOC(c, ng.pred, nb * 32);
  ALLOC(c, ng.surf, nb * 16);
  ALLOC(c, ng.occ_any, (nb + 31) / 32);
  ALLOC(c, ng.occ4, nb);
  ALLOC(c, ng.occ1, nb * 16);
  c->grid = ng;
  c->grid_bricks = nb;
  launch_grid_fill(c->grid, s);
  for (const ToolDev &t : c->tools)
    if (t.entries && launch_table_grid(t, c->grid, s) != 0) return hip_check(c, "table grid");
  rebuilt = true;
  return hip_check(c, "grid fill");
}

// ensure_grid outside a frame: a reallocated grid is refilled at once.
int regrid(af_ctx *c, hipStream_t s) {
  bool rebuilt = false;
  int rc = ensure_grid(c, s, rebuilt);
  if (rc != AF_OK) return rc;
  if (rebuilt) {
    launch_grid_rebuild(c->p, c->map, c->grid, c->n_blocks, s);
    return hip_check(c, "grid rebuild");
  }
  return AF_OK;
}

enum { ST_INTEGRATE, ST_K_INTEGRATE, ST_SCORE, ST_K_NORMALS, ST_K_MASK, ST_K_SCORE, ST_K_SMOOTH,
       ST_COUNT };

hipEvent_t timing_mark(af_ctx *c, hipStream_t s) {
  if (!c->timing) return nullptr;
  hipEvent_t e;
  if (!c->ev_free.empty()) {
    e = c->ev_free.back();
    c->ev_free.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  hipEventRecord(e, s);
  c->ev_inflight.push_back(e);
  return e;
}

int timing_flush(af_ctx *c) {
  for (auto &p : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess)
      return fail(c, AF_EDEVICE, "timing event failed");
    c->stage_ms[p.stage] += ms;
  }
  if (!c->ev_inflight.empty() && hipEventSynchronize(c->ev_inflight.back()) != hipSuccess)
    return fail(c, AF_EDEVICE, "timing event failed");
  c->ev_free.insert(c->ev_free.end(), c->ev_inflight.begin(), c->ev_inflight.end());
  c->ev_inflight.clear();
  c->pending.clear();
  return AF_OK;
}

void timing_pair(af_ctx *c, int stage, hipEvent_t a, hipEvent_t b) {
  if (!a || !b) return;
  c->pending.push_back({stage, a, b});
  if (c->ev_inflight.size() > 8192) timing_flush(c);
}

}  // namespace

extern "C" {

int af_timing_enable(af_ctx *c, int on) {
  if (!c) return AF_EINVAL;
  c->timing = on != 0;
  return AF_OK;
}

int af_timing_read(af_ctx *c, af_timing *out, int reset) {
  if (!c) return AF_EINVAL;
  int rc = timing_flush(c);
  if (rc != AF_OK) return rc;
  if (out) {
    out->integrate_ms = c->stage_ms[ST_INTEGRATE];
    out->k_integrate_ms = c->stage_ms[ST_K_INTEGRATE];
    out->score_ms = c->stage_ms[ST_SCORE];
    out->k_normals_ms = c->stage_ms[ST_K_NORMALS];
    out->k_mask_ms = c->stage_ms[ST_K_MASK];
    out->k_score_ms = c->stage_ms[ST_K_SCORE];
    out->integrate_calls = c->integrate_calls;
    out->score_calls = c->score_calls;
    out->k_smooth_ms = c->stage_ms[ST_K_SMOOTH];
  }
  if (reset) {
    for (double &x : c->stage_ms) x = 0;
    c->integrate_calls = c->score_calls = 0;
  }
  return AF_OK;
}

int af_config_default(af_config *cfg, double voxel, double trunc) {
  if (!cfg || !(voxel > 0)) return AF_EINVAL;
  memset(cfg, 0, sizeof(*cfg));
  cfg->voxel = voxel;
  cfg->trunc = trunc;
  cfg->r_c = 0.01;
  cfg->n_c = 5;
  cfg->weight_cap = 2000;
  cfg->conf_min_w = 2;
  cfg->cos_normal = 0.3420201433256687;  // cos 70 deg
  cfg->obs_dot = 0.25;
  cfg->vp_min_dist = 0.1;
  cfg->n_vp = 8;
  cfg->knn_k = 10;
  cfg->clamp_negative = 0;
  cfg->max_tools = 8;
  cfg->max_blocks = 1 << 18;
  cfg->max_points = 1 << 22;
  cfg->max_orientations = 1024;
  cfg->hbm_budget = 0;
  return AF_OK;
}

int af_create(const af_config *cfg, af_ctx **out) {
  if (!out) return AF_EINVAL;
  *out = nullptr;
  if (!cfg || !(cfg->voxel > 0) || cfg->n_vp < 1 || cfg->n_vp > kMaxVp || cfg->knn_k < 1 ||
      cfg->n_c < 1 || cfg->n_c > 64 || cfg->weight_cap < 1 || cfg->weight_cap > 60000 ||
      cfg->max_tools < 1 || cfg->max_blocks < 1 || cfg->max_blocks >= (1LL << 22) ||
      cfg->max_points < 1 || cfg->max_points >= (1LL << 30) || cfg->max_orientations < 1 ||
      cfg->max_orientations > 65536)
    return AF_EINVAL;
  af_ctx *c = new af_ctx();
  c->cfg = *cfg;
  c->err = kNoError;
  hipGetDevice(&c->device);
  // Section 3.2: tau = min(4v, 0.1 m) unless given (the text prints max; the
  // voxel-size study of Section 4.1 needs tau proportional to v).
  c->tau = cfg->trunc > 0 ? cfg->trunc : std::min(4.0 * cfg->voxel, 0.1);
  Params &p = c->p;
  memset(&p, 0, sizeof(p));
  p.scale = 256.0 / cfg->voxel;
  int64_t tau_u = llrint(c->tau * p.scale);
  int64_t R = (tau_u + 255) / 256;
  if (R < 1 || R > 7) {
    delete c;
    return AF_EINVAL;
  }
  p.tau_u = (int32_t)tau_u;
  p.R = (int32_t)R;
  p.rc_u = (int32_t)llrint(cfg->r_c * p.scale);
  p.n_c = cfg->n_c;
  p.cap = cfg->weight_cap;
  p.conf_min_w = cfg->conf_min_w;
  p.n_vp = cfg->n_vp;
  p.knn_k = cfg->knn_k;
  p.clamp_neg = cfg->clamp_negative ? 1 : 0;
  int64_t dmin = llrint(cfg->vp_min_dist * p.scale);
  p.dmin2 = dmin * dmin;
  p.cos2 = cfg->cos_normal * cfg->cos_normal;
  p.obs2 = cfg->obs_dot * cfg->obs_dot;
  c->last_frame = -1;
  c->last_stream = nullptr;

  auto bail = [&](int rc) {
    for (void *q : c->allocs) hipFree(q);
    if (c->counters_host) hipHostFree(c->counters_host);
    delete c;
    return rc;
  };
  int rc;
#define CREATE_ALLOC(ptr, count)                                                   \
  if ((rc = dev_alloc(c, (void **)&(ptr), (int64_t)sizeof(*(ptr)) * (int64_t)(count))) != AF_OK) \
    return bail(rc);
  const int64_t B = cfg->max_blocks, NP = cfg->max_points;
  MapDev &m = c->map;
  m.max_blocks = B;
  m.h.mask = pow2_at_least(2 * B) - 1;
  CREATE_ALLOC(m.h.keys, (int64_t)m.h.mask + 1);
  CREATE_ALLOC(m.h.vals, (int64_t)m.h.mask + 1);
  CREATE_ALLOC(m.bkey, B);
  CREATE_ALLOC(m.S, B * kBlockVox);
  CREATE_ALLOC(m.W, B * kBlockVox);
  CREATE_ALLOC(m.clr, B * 16);
  CREATE_ALLOC(m.surf, B * 16);
  CREATE_ALLOC(m.touched, B);
  CREATE_ALLOC(m.tpos, B);
  CREATE_ALLOC(m.n_blocks, 1);
  PointsDev &q = c->pts;
  q.max_points = NP;
  q.h.mask = pow2_at_least(2 * NP) - 1;
  CREATE_ALLOC(q.h.keys, (int64_t)q.h.mask + 1);
  CREATE_ALLOC(q.h.vals, (int64_t)q.h.mask + 1);
  CREATE_ALLOC(q.key, NP);
  CREATE_ALLOC(q.first, NP);
  CREATE_ALLOC(q.addr, NP);
  CREATE_ALLOC(q.last, NP);
  CREATE_ALLOC(q.nvp, NP);
  CREATE_ALLOC(q.head, NP);
  CREATE_ALLOC(q.vp, NP * kMaxVp * 3);
  CREATE_ALLOC(q.sumq, NP * 3);
  CREATE_ALLOC(q.nq, NP);
  CREATE_ALLOC(q.normal, NP * 3);
  CREATE_ALLOC(q.has_normal, NP);
  CREATE_ALLOC(q.n_points, 1);
  CREATE_ALLOC(c->counters, 1);
  CREATE_ALLOC(c->work, 1);
  c->score_variant = score_variant_default();
  CREATE_ALLOC(c->mask, NP * ((cfg->max_orientations + 63) / 64));
  CREATE_ALLOC(c->nearp, NP * 2 * ((cfg->max_orientations + 63) / 64));
  CREATE_ALLOC(c->tools_dev, cfg->max_tools);
  CREATE_ALLOC(c->fargs, 1);
  c->own_mask.assign(cfg->max_tools, 0);
  c->tools.assign(cfg->max_tools, ToolDev());
  c->tool_bytes.assign(cfg->max_tools, 0);
  c->label_init.assign(cfg->max_tools, 0);
  for (auto &t : c->tools) memset(&t, 0, sizeof(t));
  if (hipHostMalloc((void **)&c->counters_host, sizeof(FrameCounters)) != hipSuccess)
    return bail(AF_ENOMEM);
  memset(c->counters_host, 0, sizeof(FrameCounters));
  if (hipMemset(m.h.keys, 0xff, sizeof(int64_t) * ((int64_t)m.h.mask + 1)) != hipSuccess ||
      hipMemset(q.h.keys, 0xff, sizeof(int64_t) * ((int64_t)q.h.mask + 1)) != hipSuccess ||
      hipMemset(m.n_blocks, 0, sizeof(int32_t)) != hipSuccess ||
      hipMemset(q.n_points, 0, sizeof(int32_t)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return bail(AF_EDEVICE);
  if ((rc = alloc_scratch(c, 1 << 15)) != AF_OK) return bail(rc);
  *out = c;
  return AF_OK;
#undef CREATE_ALLOC
}

int af_destroy(af_ctx *c) {
  if (!c) return AF_EINVAL;
  hipDeviceSynchronize();
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  if (c->graph) hipGraphDestroy(c->graph);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  timing_flush(c);
  for (hipEvent_t e : c->ev_free) hipEventDestroy(e);
  for (void *q : c->allocs) hipFree(q);
  if (c->counters_host) hipHostFree(c->counters_host);
  delete c;
  return AF_OK;
}

const char *af_last_error(const af_ctx *c) { return c ? c->err.c_str() : "null context"; }

int64_t af_device_bytes(af_ctx *c) { return c ? c->bytes : 0; }

static int graph_settle(af_ctx *c);

// Release tool `tool_id`'s device buffers (after the stream has drained).
static int tool_release(af_ctx *c, int32_t tool_id, hipStream_t s) {
  ToolDev &t = c->tools[tool_id];
  if (!t.entries) return AF_OK;
  HIP_TRY(c, hipStreamSynchronize(s));
  dev_free(c, t.entries, c->tool_bytes[tool_id]);
  dev_free(c, t.begin, sizeof(uint32_t) * (t.K + 1));
  dev_free(c, t.rot, sizeof(double) * 9 * t.K);
  dev_free(c, t.label, c->cfg.max_points);
  dev_free(c, t.first_free, sizeof(int16_t) * c->cfg.max_points);
  dev_free(c, t.counters, sizeof(ScoreCounters));
  dev_free(c, t.far_begin, sizeof(uint32_t) * t.K);
  dev_free(c, t.same, sizeof(uint64_t) * ((t.K + 63) / 64));
  dev_free(c, t.xent, sizeof(uint2) * std::max<int64_t>(1, t.n_entries));
  if (t.rent) dev_free(c, t.rent, sizeof(uint32_t) * std::max<int64_t>(1, t.n_entries));
  if (c->own_mask[tool_id]) {
    const int64_t mw = (t.K + 63) / 64;
    dev_free(c, t.mask, sizeof(uint64_t) * c->cfg.max_points * mw);
    dev_free(c, t.nearp, sizeof(uint64_t) * c->cfg.max_points * 2 * mw);
    c->own_mask[tool_id] = 0;
  }
  dev_free(c, t.c4begin, sizeof(uint32_t) * (t.K + 1));
  dev_free(c, t.c4flag, t.K);
  dev_free(c, t.c4entries, sizeof(uint32_t) * std::max<int64_t>(1, t.n_c4entries));
  memset(&t, 0, sizeof(t));
  return AF_OK;
}

// Common tail of both table forms.  nt holds rot, begin, same and the
// packed entries (NEAR x3, BODY, FAR per orientation); counts[2k], counts[2k+1]
// are orientation k's BODY and FAR counts (device).  Builds the corridor
// lists, the grid-independent and grid-relative entry forms, the per-tool
// outputs, and installs the tool.
static int tool_finish(af_ctx *c, int32_t tool_id, ToolDev &nt, uint32_t *counts, uint32_t total,
                       hipStream_t s) {
  const int32_t K = nt.K;
  ALLOC(c, nt.label, c->cfg.max_points);
  ALLOC(c, nt.first_free, c->cfg.max_points);
  ALLOC(c, nt.counters, 1);
  HIP_TRY(c, hipMemsetAsync(nt.label, 0, c->cfg.max_points, s));
  HIP_TRY(c, hipMemsetAsync(nt.counters, 0, sizeof(ScoreCounters), s));
  uint32_t *ccounts = nullptr;
  ALLOC(c, nt.far_begin, K);
  ALLOC(c, ccounts, K);
  // coarse corridor lists over 4^3 cells
  ALLOC(c, nt.c4begin, K + 1);
  ALLOC(c, nt.c4flag, K);
  if (launch_table_coarse(K, nt.begin, counts, nt.entries, nt.far_begin, ccounts, nt.c4begin,
                          nullptr, nt.c4flag, 0, 2, s) != 0)
    return hip_check(c, "coarse4 count");
  uint32_t c4total = 0;
  HIP_TRY(c, hipMemcpyAsync(&c4total, nt.c4begin + K, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  ALLOC(c, nt.c4entries, std::max<uint32_t>(1u, c4total));
  if (launch_table_coarse(K, nt.begin, counts, nt.entries, nt.far_begin, ccounts, nt.c4begin,
                          nt.c4entries, nt.c4flag, 1, 2, s) != 0)
    return hip_check(c, "coarse4 fill");
  nt.n_c4entries = c4total;
  HIP_TRY(c, hipStreamSynchronize(s));
  dev_free(c, ccounts, sizeof(uint32_t) * K);
  {
    std::vector<uint32_t> he(total);
    HIP_TRY(c, hipMemcpy(he.data(), nt.entries, sizeof(uint32_t) * total, hipMemcpyDeviceToHost));
    int32_t reach = 0;
    for (uint32_t e : he)
      reach = std::max({reach, std::abs(entry_x(e)), std::abs(entry_y(e)), std::abs(entry_z(e))});
    nt.reach = reach;
    if (reach <= 255) {
      std::vector<uint32_t> rel(total);
      for (uint32_t j = 0; j < total; ++j) {
        const uint32_t e = he[j];
        rel[j] = (uint32_t)(entry_x(e) + 256) | ((uint32_t)(entry_y(e) + 256) << 10) |
                 ((uint32_t)(entry_z(e) + 256) << 20) | ((uint32_t)entry_cls(e) << 30);
      }
      ALLOC(c, nt.rent, std::max<int64_t>(1, total));
      HIP_TRY(c, hipMemcpy(nt.rent, rel.data(), sizeof(uint32_t) * total, hipMemcpyHostToDevice));
    }
  }
  nt.n_entries = total;
  ALLOC(c, nt.xent, std::max<int64_t>(1, total));
  nt.mask = c->mask;
  nt.nearp = c->nearp;
  ToolDev &t = c->tools[tool_id];
  t = nt;
  c->tool_bytes[tool_id] = sizeof(uint32_t) * (int64_t)total;
  c->label_init[tool_id] = 0;
  c->last_stream = s;
  if (c->grid_bricks > 0 && launch_table_grid(t, c->grid, s) != 0) return hip_check(c, "table grid");
  HIP_TRY(c, hipMemcpy(&c->tools_dev[tool_id], &t, sizeof(ToolDev), hipMemcpyHostToDevice));
  c->graph_stale = true;
  return regrid(c, s);
}

int af_set_tool_kernels(af_ctx *c, int32_t tool_id, const af_tool *tool, int32_t K,
                        const double *rot, void *stream) {
  if (!c) return AF_EINVAL;
  if (c->graph_dirty) {
    const int rc = graph_settle(c);
    if (rc != AF_OK) return rc;
  }
  if (tool_id < 0 || tool_id >= c->cfg.max_tools)
    return fail(c, AF_EINVAL, "tool id %d outside [0, %d)", tool_id, c->cfg.max_tools);
  if (!tool || !rot || K < 1 || K > c->cfg.max_orientations)
    return fail(c, AF_EINVAL, "bad tool, rotations or K=%d", K);
  if ((tool->shape != AF_TOOL_CYLINDER && tool->shape != AF_TOOL_BOX) || !(tool->length > 0) ||
      !(tool->corridor >= 0) || !(tool->r_s >= 0) ||
      (tool->shape == AF_TOOL_CYLINDER && !(tool->radius > 0)) ||
      (tool->shape == AF_TOOL_BOX && !(tool->width > 0 && tool->height > 0)))
    return fail(c, AF_EINVAL, "bad tool geometry");
  for (int32_t k = 0; k < K; ++k)
    for (int col = 0; col < 3; ++col) {
      double n2 = 0;
      for (int row = 0; row < 3; ++row) n2 += rot[9 * k + 3 * row + col] * rot[9 * k + 3 * row + col];
      if (!(fabs(sqrt(n2) - 1.0) <= 1e-9))
        return fail(c, AF_EINVAL, "orientation %d column %d is not a unit vector", k, col);
    }
  hipStream_t s = (hipStream_t)stream;
  const double v = c->cfg.voxel;
  ToolGeom tg;
  memset(&tg, 0, sizeof(tg));
  tg.shape = tool->shape;
  tg.Lv = tool->length / v;
  tg.Ev = (tool->length + tool->corridor) / v;
  if (tool->shape == AF_TOOL_CYLINDER) {
    tg.a = tool->radius / v;
    tg.b = tg.a;
  } else {
    tg.a = (0.5 * tool->width) / v;
    tg.b = (0.5 * tool->height) / v;
  }
  tg.rv2 = tg.a * tg.a;
  double rsv = tool->r_s / v;
  tg.rsv2 = rsv * rsv;
  const double fr[3] = {0.6, 1.25, 2.25};
  for (int j = 0; j < 3; ++j) tg.lam[j] = (fr[j] * c->tau) / v;

  int rc = tool_release(c, tool_id, s);
  if (rc != AF_OK) return rc;
  ToolDev nt;
  memset(&nt, 0, sizeof(nt));
  nt.K = K;
  uint32_t *counts = nullptr;
  int32_t *err = nullptr;
  ALLOC(c, nt.rot, 9 * (int64_t)K);
  ALLOC(c, nt.begin, K + 1);
  {
    std::vector<uint64_t> same((K + 63) / 64, 0ull);
    for (int32_t k = 1; k < K; ++k)
      if (rot[9 * k] == rot[9 * (k - 1)] && rot[9 * k + 3] == rot[9 * (k - 1) + 3] &&
          rot[9 * k + 6] == rot[9 * (k - 1) + 6])
        same[k >> 6] |= 1ull << (k & 63);
    ALLOC(c, nt.same, (K + 63) / 64);
    HIP_TRY(c, hipMemcpy(nt.same, same.data(), sizeof(uint64_t) * same.size(),
                         hipMemcpyHostToDevice));
  }
  ALLOC(c, counts, 2 * (int64_t)K);
  ALLOC(c, err, 1);
  HIP_TRY(c, hipMemcpyAsync(nt.rot, rot, sizeof(double) * 9 * K, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemsetAsync(err, 0, sizeof(int32_t), s));
  tg.pad = 0;
  if (launch_table_build(tg, K, nt.rot, counts, nt.begin, err, nullptr, 0, s) != 0)
    return hip_check(c, "table count");
  uint32_t total = 0;
  int32_t herr = 0;
  HIP_TRY(c, hipMemcpyAsync(&total, nt.begin + K, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (herr) {
    dev_free(c, counts, sizeof(uint32_t) * 2 * K);
    dev_free(c, err, sizeof(int32_t));
    dev_free(c, nt.rot, sizeof(double) * 9 * K);
    dev_free(c, nt.begin, sizeof(uint32_t) * (K + 1));
    dev_free(c, nt.same, sizeof(uint64_t) * ((K + 63) / 64));
    return fail(c, AF_EINVAL, "tool too large for the voxel size (%s)",
                herr & 2 ? "more than 16384 entries in one class" : "offset beyond 511 voxels");
  }
  ALLOC(c, nt.entries, total);
  if (launch_table_build(tg, K, nt.rot, counts, nt.begin, err, nt.entries, 1, s) != 0)
    return hip_check(c, "table fill");
  HIP_TRY(c, hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  dev_free(c, err, sizeof(int32_t));
  if (herr) return fail(c, AF_EINVAL, "tool table build failed (%d)", herr);
  rc = tool_finish(c, tool_id, nt, counts, total, s);
  dev_free(c, counts, sizeof(uint32_t) * 2 * K);
  return rc;
}

int af_set_tool_table(af_ctx *c, int32_t tool_id, const af_kernel_table *tab, void *stream) {
  if (!c) return AF_EINVAL;
  if (c->graph_dirty) {
    const int rc = graph_settle(c);
    if (rc != AF_OK) return rc;
  }
  if (tool_id < 0 || tool_id >= c->cfg.max_tools)
    return fail(c, AF_EINVAL, "tool id %d outside [0, %d)", tool_id, c->cfg.max_tools);
  if (!tab || !tab->dir || !tab->offset_begin || tab->K < 1 || tab->K > c->cfg.max_orientations)
    return fail(c, AF_EINVAL, "bad table or K");
  const int32_t K = tab->K;
  if (tab->offset_begin[0] != 0) return fail(c, AF_EINVAL, "offset_begin[0] must be 0");
  for (int32_t k = 0; k < K; ++k)
    if (tab->offset_begin[k + 1] < tab->offset_begin[k])
      return fail(c, AF_EINVAL, "offset_begin decreases at orientation %d", k);
  const uint32_t n_in = tab->offset_begin[K];
  if (n_in > 0 && (!tab->off || !tab->cls)) return fail(c, AF_EINVAL, "missing offsets or classes");
  for (int32_t k = 0; k < K; ++k) {
    const double *d = tab->dir + 3 * k;
    const double n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(fabs(sqrt(n2) - 1.0) <= 1e-9))
      return fail(c, AF_EINVAL, "direction %d is not a unit vector", k);
  }
  // canonical order per orientation: the three NEAR entries as given, then
  // BODY and FAR each sorted by (|o|^2, z, y, x)
  std::vector<uint32_t> entries;
  std::vector<uint32_t> begin(K + 1), counts(2 * (size_t)K);
  std::vector<std::array<int, 3>> near3((size_t)K * 3);
  entries.reserve(n_in);
  for (int32_t k = 0; k < K; ++k) {
    begin[k] = (uint32_t)entries.size();
    std::vector<std::array<int, 4>> body, far_;
    int nn = 0;
    for (uint32_t e = tab->offset_begin[k]; e < tab->offset_begin[k + 1]; ++e) {
      const int ox = tab->off[3 * (size_t)e], oy = tab->off[3 * (size_t)e + 1],
                oz = tab->off[3 * (size_t)e + 2];
      const int cl = tab->cls[e];
      if (cl != AF_CLS_BODY && cl != AF_CLS_NEAR && cl != AF_CLS_FAR)
        return fail(c, AF_EINVAL, "entry %u of orientation %d has class %d", e, k, cl);
      if (std::abs(ox) > 511 || std::abs(oy) > 511 || std::abs(oz) > 511)
        return fail(c, AF_EINVAL, "entry %u of orientation %d is beyond 511 voxels", e, k);
      if (cl == AF_CLS_NEAR) {
        if (nn >= 3) return fail(c, AF_EINVAL, "orientation %d has more than 3 NEAR entries", k);
        near3[3 * (size_t)k + nn] = {ox, oy, oz};
        entries.push_back(pack_entry(ox, oy, oz, AF_CLS_NEAR));
        ++nn;
      } else {
        (cl == AF_CLS_BODY ? body : far_).push_back({ox * ox + oy * oy + oz * oz, oz, oy, ox});
      }
    }
    if (nn != 3) return fail(c, AF_EINVAL, "orientation %d has %d NEAR entries (3 needed)", k, nn);
    for (auto *grp : {&body, &far_}) {
      std::sort(grp->begin(), grp->end());
      if (std::adjacent_find(grp->begin(), grp->end()) != grp->end())
        return fail(c, AF_EINVAL, "orientation %d lists an offset twice in one class", k);
      if ((int64_t)grp->size() > kTableMaxClass)
        return fail(c, AF_EINVAL, "orientation %d has more than %d entries in one class", k,
                    kTableMaxClass);
      const int cl = grp == &body ? AF_CLS_BODY : AF_CLS_FAR;
      for (const auto &q : *grp) entries.push_back(pack_entry(q[3], q[2], q[1], cl));
    }
    counts[2 * (size_t)k] = (uint32_t)body.size();
    counts[2 * (size_t)k + 1] = (uint32_t)far_.size();
  }
  begin[K] = (uint32_t)entries.size();
  // orientations sharing their predecessor's direction and arm samples
  std::vector<uint64_t> same((K + 63) / 64, 0ull);
  for (int32_t k = 1; k < K; ++k) {
    const double *d = tab->dir + 3 * k, *e = tab->dir + 3 * (k - 1);
    bool eq = d[0] == e[0] && d[1] == e[1] && d[2] == e[2];
    for (int j = 0; j < 3 && eq; ++j) eq = near3[3 * (size_t)k + j] == near3[3 * (size_t)(k - 1) + j];
    if (eq) same[k >> 6] |= 1ull << (k & 63);
  }
  // orientation frames for the candidate filters: column 0 is the direction
  std::vector<double> rot(9 * (size_t)K, 0.0);
  for (int32_t k = 0; k < K; ++k)
    for (int i = 0; i < 3; ++i) rot[9 * (size_t)k + 3 * i] = tab->dir[3 * k + i];

  hipStream_t s = (hipStream_t)stream;
  int rc = tool_release(c, tool_id, s);
  if (rc != AF_OK) return rc;
  ToolDev nt;
  memset(&nt, 0, sizeof(nt));
  nt.K = K;
  const uint32_t total = begin[K];
  uint32_t *dcounts = nullptr;
  ALLOC(c, nt.rot, 9 * (int64_t)K);
  ALLOC(c, nt.begin, K + 1);
  ALLOC(c, nt.same, (K + 63) / 64);
  ALLOC(c, nt.entries, std::max<uint32_t>(1u, total));
  ALLOC(c, dcounts, 2 * (int64_t)K);
  HIP_TRY(c, hipMemcpy(nt.rot, rot.data(), sizeof(double) * rot.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(nt.begin, begin.data(), sizeof(uint32_t) * begin.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(nt.same, same.data(), sizeof(uint64_t) * same.size(), hipMemcpyHostToDevice));
  if (total > 0)
    HIP_TRY(c, hipMemcpy(nt.entries, entries.data(), sizeof(uint32_t) * total, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(dcounts, counts.data(), sizeof(uint32_t) * counts.size(), hipMemcpyHostToDevice));
  rc = tool_finish(c, tool_id, nt, dcounts, total, s);
  dev_free(c, dcounts, sizeof(uint32_t) * 2 * K);
  return rc;
}

int af_set_window(af_ctx *c, const int32_t blocks[3]) {
  if (!c) return AF_EINVAL;
  if (!blocks) return fail(c, AF_EINVAL, "no window size");
  if (c->last_frame >= 0 || c->n_points > 0 || c->win_on)
    return fail(c, AF_EINVAL, "the window is set once, before the first frame");
  if (c->g_n) return fail(c, AF_EINVAL, "the window is set before the frame graph is prepared");
  for (int a = 0; a < 3; ++a)
    if (blocks[a] < 2 || blocks[a] > 4096)
      return fail(c, AF_EINVAL, "window of %d blocks on axis %d (2..4096)", blocks[a], a);
  ALLOC(c, c->map.free_ids, c->cfg.max_blocks);
  ALLOC(c, c->map.n_free, 1);
  ALLOC(c, c->win_sel, c->cfg.max_points);
  ALLOC(c, c->win_nsel, 1);
  HIP_TRY(c, hipMemset(c->map.n_free, 0, sizeof(int32_t)));
  HIP_TRY(c, hipDeviceSynchronize());
  for (int a = 0; a < 3; ++a) c->win_L[a] = blocks[a];
  c->win_on = true;
  c->win_set = false;
  c->win_shifts = 0;
  return AF_OK;
}

int af_window_state(af_ctx *c, int32_t lo[3], int32_t hi[3], int64_t *shifts) {
  if (!c) return AF_EINVAL;
  if (!c->win_on) return fail(c, AF_EINVAL, "no window");
  for (int a = 0; a < 3; ++a) {
    if (lo) lo[a] = c->win_lo[a];
    if (hi) hi[a] = c->win_hi[a];
  }
  if (shifts) *shifts = c->win_shifts;
  return c->win_set ? 1 : 0;
}

int af_integrate_frame_host(af_ctx *c, const float *xyz, int64_t n, const float origin[3],
                            int64_t frame_id, void *stream) {
  if (!c) return AF_EINVAL;
  if (n < 0 || (n > 0 && !xyz) || !origin) return fail(c, AF_EINVAL, "bad frame arguments");
  hipStream_t s = (hipStream_t)stream;
  if (n > c->host_xyz_cap) {
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->host_xyz) dev_free(c, c->host_xyz, sizeof(float) * 3 * c->host_xyz_cap);
    c->host_xyz = nullptr;
    c->host_xyz_cap = 0;
    const int64_t cap = std::max<int64_t>(n, 4096);
    ALLOC(c, c->host_xyz, 3 * cap);
    c->host_xyz_cap = cap;
  }
  if (n > 0)
    HIP_TRY(c, hipMemcpyAsync(c->host_xyz, xyz, sizeof(float) * 3 * n, hipMemcpyHostToDevice, s));
  // af_integrate_frame synchronises the stream after block allocation, so the
  // copy has completed when this call returns
  return af_integrate_frame(c, c->host_xyz, n, origin, frame_id, stream);
}

// Section 3.3: the window is placed at the first frame and moves (re-centred
// on the sensor voxel) once the sensor is more than 30 % of its size from
// the centre on any axis.  Q: the sensor origin in 1/256 voxel units.
static bool window_shift_due(const af_ctx *c, int3 Q) {
  if (!c->win_set) return true;
  const int32_t qv[3] = {Q.x >> 8, Q.y >> 8, Q.z >> 8};
  for (int a = 0; a < 3; ++a)
    if (10 * (int64_t)std::abs(qv[a] - c->win_c[a]) > 3 * 8 * (int64_t)c->win_L[a]) return true;
  return false;
}

int af_integrate_frame(af_ctx *c, const float *xyz, int64_t n, const float origin[3],
                       int64_t frame_id, void *stream) {
  if (!c) return AF_EINVAL;
  if (c->graph_dirty) {
    const int rc = graph_settle(c);
    if (rc != AF_OK) return rc;
  }
  if (n < 0 || (n > 0 && !xyz) || !origin)
    return fail(c, AF_EINVAL, "bad frame arguments");
  if (frame_id <= c->last_frame || frame_id > 0x7ffffffe)
    return fail(c, AF_EINVAL, "frame id %lld does not increase", (long long)frame_id);
  int3 Q;
  int *qq[3] = {&Q.x, &Q.y, &Q.z};
  for (int a = 0; a < 3; ++a) {
    double t = (double)origin[a] * c->p.scale;
    if (!(fabs(t) <= (double)kCoordLim)) return fail(c, AF_EINVAL, "sensor origin out of range");
    *qq[a] = (int)llrint(t);
  }
  hipStream_t s = (hipStream_t)stream;
  int rc;
  // Section 3.3: the window follows the sensor (see af_set_window)
  bool shift = false, thaw = false;
  int3 wlo = make_int3(-(1 << 30), -(1 << 30), -(1 << 30));
  int3 whi = make_int3(1 << 30, 1 << 30, 1 << 30);
  if (c->win_on) {
    const int32_t qv[3] = {Q.x >> 8, Q.y >> 8, Q.z >> 8};
    shift = window_shift_due(c, Q);
    if (shift) {
      for (int a = 0; a < 3; ++a) {
        c->win_c[a] = qv[a];
        c->win_lo[a] = (qv[a] >> 3) - c->win_L[a] / 2;
        c->win_hi[a] = c->win_lo[a] + c->win_L[a] - 1;
        c->bbox_lo[a] = c->win_lo[a];
        c->bbox_hi[a] = c->win_hi[a];
      }
      c->have_bbox = true;
      thaw = c->win_set;
      c->win_set = true;
    }
    wlo = make_int3(c->win_lo[0], c->win_lo[1], c->win_lo[2]);
    whi = make_int3(c->win_hi[0], c->win_hi[1], c->win_hi[2]);
  }
  // a shift may re-create one block per point besides the frame's own
  constexpr int64_t kPerReturn = kMaxSpan + kMaxBand;
  const int64_t need = n + (thaw ? (c->n_points + kPerReturn - 1) / kPerReturn : 0);
  if (need > c->fs.cap) {
    HIP_TRY(c, hipStreamSynchronize(s));
    if ((rc = alloc_scratch(c, std::max<int64_t>(need, 2 * c->fs.cap))) != AF_OK) return rc;
  }
  const int32_t frame = (int32_t)frame_id;
  hipEvent_t t0 = timing_mark(c, s);
  if (thaw) {
    launch_window_evict(c->map, c->pts, c->n_blocks, c->n_points, wlo, whi, s);
    c->win_shifts += 1;
  }
  launch_set_frame_args(c->fargs, n, Q, frame, wlo, whi, s);
  launch_frame_prep(xyz, c->fargs, n, c->p, c->map, c->pts, c->fs, c->counters, s);
  if (thaw) launch_window_thaw(c->map, c->pts, c->fs, c->counters, c->n_points, wlo, whi, s);
  launch_assign_blocks(c->map, c->fs, c->counters, c->fargs, s);
  launch_commit_blocks(c->map, c->counters, s);
  if (thaw) launch_window_link(c->map, c->pts, c->n_points, wlo, whi, s);
  HIP_TRY(c, hipMemcpyAsync(c->counters_host, c->counters, offsetof(FrameCounters, fold),
                            hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if ((rc = hip_check(c, "frame prep")) != AF_OK) return rc;
  FrameCounters h = *c->counters_host;
  if (h.n_new_blocks > 0 && !c->win_on) {   // (with a window the box is the window)
    for (int a = 0; a < 3; ++a) {
      if (!c->have_bbox || h.bmin[a] < c->bbox_lo[a]) c->bbox_lo[a] = h.bmin[a];
      if (!c->have_bbox || h.bmax[a] > c->bbox_hi[a]) c->bbox_hi[a] = h.bmax[a];
    }
    c->have_bbox = true;
  }
  bool rebuilt = false;
  if ((rc = ensure_grid(c, s, rebuilt, shift)) != AF_OK) return rc;
  launch_touch_band(c->fargs, n, c->p, c->map, c->fs, c->counters, s);
  launch_points_append(h.n_new_points, c->map, c->pts, c->fs, c->counters, c->fargs, s);
  launch_commit_points(c->pts, c->counters, s);
  launch_points_view(c->fargs, n, c->p, c->pts, c->fs, s);
  // new blocks take evicted ids first
  int64_t nb_after = std::min<int64_t>(
      (int64_t)h.blocks_before + std::max<int64_t>(0, (int64_t)h.n_new_blocks - h.free_before),
      c->cfg.max_blocks);
  hipEvent_t t1 = timing_mark(c, s);
  launch_integrate(c->fargs, n, c->p, c->map, c->fs, c->counters, c->grid,
                   std::max<int64_t>(1, std::min<int64_t>(nb_after, n * (kMaxSpan + kMaxBand))), s);
  hipEvent_t t2 = timing_mark(c, s);
  if (rebuilt) launch_grid_rebuild(c->p, c->map, c->grid, nb_after, s);
  hipEvent_t t5 = timing_mark(c, s);
  if (c->timing) {
    timing_pair(c, ST_INTEGRATE, t0, t5);
    timing_pair(c, ST_K_INTEGRATE, t1, t2);
    c->integrate_calls += 1;
  }
  if ((rc = hip_check(c, "integrate")) != AF_OK) return rc;
  c->last_frame = frame_id;
  c->last_stream = s;
  c->n_blocks = nb_after;
  c->n_points = std::min<int64_t>((int64_t)h.points_before + h.n_new_points, c->cfg.max_points);
  c->status = h.status;
  if (h.status & kStatusHashFull) return fail(c, AF_EOVERFLOW, "hash table full");
  if (h.status & kStatusBlockOverflow)
    return fail(c, AF_EOVERFLOW, "block capacity %lld exceeded", (long long)c->cfg.max_blocks);
  if (h.n_new_points + (int64_t)h.points_before > c->cfg.max_points)
    return fail(c, AF_EOVERFLOW, "point capacity %lld exceeded", (long long)c->cfg.max_points);
  return AF_OK;
}

static int cached_normals(af_ctx *c, hipStream_t s);

// Tools a windowed graph scores take the point list (reach of 255 voxels at most).
static int window_tools_ok(af_ctx *c, const int32_t *ids, int32_t n) {
  for (int32_t i = 0; i < n; ++i)
    if (!score_variant_takes_list(score_variant_default(), c->tools[ids[i]]))
      return fail(c, AF_EINVAL, "tool %d: reach above 255 voxels (not with a sliding window)",
                  ids[i]);
  return AF_OK;
}

// The score variant a listed (windowed) scoring of tool t runs.
static int window_variant(const af_ctx *c, const ToolDev &t) {
  return score_variant_takes_list(c->score_variant, t) ? c->score_variant
                                                         : score_variant_default();
}

// With a sliding window only the points inside it are scored (fresh normals
// over the window's point list, listed once for all the tools); the others
// keep their last labels, and a point never scored reads 255.
static int score_window(af_ctx *c, const int32_t *ids, int32_t n_tools, hipStream_t s) {
  int rc = window_tools_ok(c, ids, n_tools);
  if (rc != AF_OK) return rc;
  const int3 lo = make_int3(c->win_lo[0], c->win_lo[1], c->win_lo[2]);
  const int3 hi = make_int3(c->win_hi[0], c->win_hi[1], c->win_hi[2]);
  for (int32_t i = 0; i < n_tools; ++i) {
    ToolDev &t = c->tools[ids[i]];
    int64_t &init = c->label_init[ids[i]];
    if (init < c->n_points) {
      launch_label_fill(t.label, t.first_free, init, c->n_points, s);
      init = c->n_points;
    }
  }
  hipEvent_t t0 = timing_mark(c, s);
  for (int32_t i = 0; i < n_tools; ++i)
    HIP_TRY(c, hipMemsetAsync(c->tools[ids[i]].counters, 0, sizeof(ScoreCounters), s));
  launch_window_list(c->pts, c->n_points, lo, hi, c->win_sel, c->win_nsel, s);
  PointsDev ps = c->pts;
  ps.sel = c->win_sel;
  ps.n_sel = c->win_nsel;
  hipEvent_t t1 = timing_mark(c, s);
  launch_normals(c->p, c->map, ps, c->grid, c->n_points, s, true);
  hipEvent_t t2 = timing_mark(c, s);
  hipEvent_t t3 = t2;
  for (int32_t i = 0; i < n_tools; ++i) {
    const ToolDev &t = c->tools[ids[i]];
    launch_mask(c->p, ps, t, c->grid, c->n_points, s, true);
    if (i == 0) t3 = timing_mark(c, s);
    launch_score(c->p, ps, t, c->grid, c->n_points, window_variant(c, t), c->work, s, true);
  }
  hipEvent_t t4 = timing_mark(c, s);
  if (c->timing) {   // (the mask stage: the first tool's)
    timing_pair(c, ST_SCORE, t0, t4);
    timing_pair(c, ST_K_NORMALS, t1, t2);
    timing_pair(c, ST_K_MASK, t2, t3);
    timing_pair(c, ST_K_SCORE, t3, t4);
    c->score_calls += 1;
  }
  c->last_stream = s;
  return hip_check(c, "score (window)");
}

int af_score_points(af_ctx *c, int32_t tool_id, void *stream) {
  if (!c) return AF_EINVAL;
  if (c->graph_dirty) {
    const int rc = graph_settle(c);
    if (rc != AF_OK) return rc;
  }
  if (tool_id < 0 || tool_id >= c->cfg.max_tools) return fail(c, AF_EINVAL, "bad tool id");
  ToolDev &t = c->tools[tool_id];
  if (!t.entries) return fail(c, AF_ENOTOOL, "tool %d has no kernels", tool_id);
  hipStream_t s = (hipStream_t)stream;
  int rc = regrid(c, s);
  if (rc != AF_OK) return rc;
  if (c->win_on) return score_window(c, &tool_id, 1, s);
  hipEvent_t t0 = timing_mark(c, s);
  HIP_TRY(c, hipMemsetAsync(t.counters, 0, sizeof(ScoreCounters), s));
  hipEvent_t t1 = timing_mark(c, s);
  if ((rc = cached_normals(c, s)) != AF_OK) return rc;
  hipEvent_t t2 = timing_mark(c, s);
  launch_mask(c->p, c->pts, t, c->grid, c->n_points, s);
  hipEvent_t t3 = timing_mark(c, s);
  launch_score(c->p, c->pts, t, c->grid, c->n_points, c->score_variant, c->work, s);
  hipEvent_t t4 = timing_mark(c, s);
  if (c->timing) {
    timing_pair(c, ST_SCORE, t0, t4);
    timing_pair(c, ST_K_NORMALS, t1, t2);
    timing_pair(c, ST_K_MASK, t2, t3);
    timing_pair(c, ST_K_SCORE, t3, t4);
    c->score_calls += 1;
  }
  c->last_stream = s;
  return hip_check(c, "score");
}

// The tool set of one multi-tool launch: ids checked, LDS offsets, and each
// tool given its own mask buffers (masks of every tool must coexist).
static int make_toolset(af_ctx *c, const int32_t *tool_ids, int32_t n_tools, ToolSet &set,
                        ToolDev *host, bool own_buffers = true) {
  if (!tool_ids || n_tools < 1 || n_tools > kMultiTools)
    return fail(c, AF_EINVAL, "n_tools must be 1..%d", kMultiTools);
  memset(&set, 0, sizeof(set));
  set.n = n_tools;
  int32_t words = 0;
  for (int32_t i = 0; i < n_tools; ++i) {
    const int32_t id = tool_ids[i];
    if (id < 0 || id >= c->cfg.max_tools) return fail(c, AF_EINVAL, "bad tool id %d", id);
    if (!c->tools[id].entries) return fail(c, AF_ENOTOOL, "tool %d has no kernels", id);
    for (int32_t j = 0; j < i; ++j)
      if (tool_ids[j] == id) return fail(c, AF_EINVAL, "tool %d listed twice", id);
    if (c->tools[id].K > 1024) return fail(c, AF_EINVAL, "tool %d: K above 1024", id);
    set.id[i] = id;
    set.base[i] = words;
    words += c->tools[id].K + 1;
  }
  if (words > multi_begin_capacity())
    return fail(c, AF_EINVAL, "%d orientations exceed one launch", words - n_tools);
  for (int32_t i = 0; i < n_tools; ++i) {
    const int32_t id = set.id[i];
    ToolDev &t = c->tools[id];
    if (own_buffers && !c->own_mask[id]) {
      const int64_t mw = (t.K + 63) / 64;
      uint64_t *mk = nullptr, *np = nullptr;
      ALLOC(c, mk, c->cfg.max_points * mw);
      ALLOC(c, np, c->cfg.max_points * 2 * mw);
      t.mask = mk;
      t.nearp = np;
      c->own_mask[id] = 1;
      HIP_TRY(c, hipMemcpy(&c->tools_dev[id], &t, sizeof(ToolDev), hipMemcpyHostToDevice));
    }
    host[i] = t;
  }
  return AF_OK;
}

static int sync_last(af_ctx *c);

// Normals of every point, recomputing only the axes that points appended
// since the last call can have changed.
static int cached_normals(af_ctx *c, hipStream_t s) {
  NormalCache &nc = c->ncache;
  if (!nc.axis || !nc.state || !nc.list || !nc.count) {   // (a failed call may have left a part)
    c->nc_seen = 0;
    if (!nc.axis) ALLOC(c, nc.axis, 3 * c->cfg.max_points);
    if (!nc.state) ALLOC(c, nc.state, c->cfg.max_points);
    if (!nc.list) ALLOC(c, nc.list, c->cfg.max_points);
    if (!nc.count) ALLOC(c, nc.count, 1);
  }
  if (nc.stale_words < 16 * c->grid_bricks) {
    if (nc.stale) {
      HIP_TRY(c, hipStreamSynchronize(s));
      dev_free(c, nc.stale, sizeof(uint32_t) * nc.stale_words);
    }
    nc.stale = nullptr;
    nc.stale_words = 0;
    ALLOC(c, nc.stale, 16 * c->grid_bricks);
    nc.stale_words = 16 * c->grid_bricks;
    HIP_TRY(c, hipMemsetAsync(nc.stale, 0, sizeof(uint32_t) * nc.stale_words, s));
  }
  launch_normals_cached(c->p, c->map, c->pts, c->grid, nc, c->nc_seen, c->n_points, s);
  c->nc_seen = c->n_points;
  return AF_OK;
}

int af_score_tools(af_ctx *c, const int32_t *tool_ids, int32_t n_tools, void *stream) {
  if (!c) return AF_EINVAL;
  int rc;
  if (c->graph_dirty && (rc = graph_settle(c)) != AF_OK) return rc;
  ToolSet set;
  ToolDev host[kMultiTools];
  if ((rc = make_toolset(c, tool_ids, n_tools, set, host, !c->win_on)) != AF_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = regrid(c, s)) != AF_OK) return rc;
  if (c->win_on) return score_window(c, tool_ids, n_tools, s);
  hipEvent_t t0 = timing_mark(c, s);
  for (int32_t i = 0; i < n_tools; ++i)
    HIP_TRY(c, hipMemsetAsync(host[i].counters, 0, sizeof(ScoreCounters), s));
  hipEvent_t t1 = timing_mark(c, s);
  if ((rc = cached_normals(c, s)) != AF_OK) return rc;
  hipEvent_t t2 = timing_mark(c, s);
  for (int32_t i = 0; i < n_tools; ++i)
    launch_mask(c->p, c->pts, host[i], c->grid, c->n_points, s);
  hipEvent_t t3 = timing_mark(c, s);
  if (n_tools == 1)   // one tool: the single-tool kernel (same results)
    launch_score(c->p, c->pts, host[0], c->grid, c->n_points, c->score_variant, c->work, s);
  else
    launch_score_multi(c->p, c->pts, c->tools_dev, host, set, c->grid, c->n_points, c->work, s);
  hipEvent_t t4 = timing_mark(c, s);
  if (c->timing) {
    timing_pair(c, ST_SCORE, t0, t4);
    timing_pair(c, ST_K_NORMALS, t1, t2);
    timing_pair(c, ST_K_MASK, t2, t3);
    timing_pair(c, ST_K_SCORE, t3, t4);
    c->score_calls += 1;
  }
  c->last_stream = s;
  return hip_check(c, "score tools");
}

static_assert(offsetof(FrameCounters, sbmin) == offsetof(FrameCounters, sticky) + 4 &&
                  offsetof(FrameCounters, sbmax) == offsetof(FrameCounters, sticky) + 16,
              "sticky fields are cleared as one block");
static hipError_t clear_sticky(af_ctx *c) {
  int32_t v[7] = {0, 0x7fffffff, 0x7fffffff, 0x7fffffff, -0x7fffffff - 1, -0x7fffffff - 1,
                  -0x7fffffff - 1};
  return hipMemcpy(&c->counters->sticky, v, sizeof(v), hipMemcpyHostToDevice);
}

// Wait for recorded frames, refresh the host's point and block counts and
// report any status they raised (sticky across frames).
// One copy and one wait: the last frame left the counts in the counters'
// snapshot, and the sticky fields are reset by the next recorded frame.
static int graph_settle(af_ctx *c) {
  c->graph_dirty = false;
  HIP_TRY(c, hipMemcpyAsync(c->counters_host, c->counters, offsetof(FrameCounters, fold),
                            hipMemcpyDeviceToHost, c->last_stream));
  HIP_TRY(c, hipStreamSynchronize(c->last_stream));
  const FrameCounters h = *c->counters_host;
  c->n_blocks = std::min<int64_t>(h.snap_blocks, c->cfg.max_blocks);
  c->n_points = std::min<int64_t>(h.snap_points, c->cfg.max_points);
  if (h.sbmin[0] <= h.sbmax[0] && !c->win_on) {   // (with a window the box is the window)
    for (int a = 0; a < 3; ++a) {
      c->bbox_lo[a] = c->have_bbox ? std::min(c->bbox_lo[a], h.sbmin[a]) : h.sbmin[a];
      c->bbox_hi[a] = c->have_bbox ? std::max(c->bbox_hi[a], h.sbmax[a]) : h.sbmax[a];
    }
    c->have_bbox = true;
  }
  c->sticky_reset = true;
  c->status = h.sticky;
  // a windowed graph scores every point its frames create
  if (c->win_on && c->g_score)
    for (int32_t i = 0; i < c->g_n; ++i) c->label_init[c->g_ids[i]] = c->n_points;
  // a block beyond the recorded box: the grid must grow, so the graph is done
  if (h.sticky & kStatusOutsideGrid) c->graph_stale = true;
  if (h.sticky & kStatusHashFull) return fail(c, AF_EOVERFLOW, "hash table full");
  if (h.sticky & kStatusBlockOverflow)
    return fail(c, AF_EOVERFLOW, "block capacity %lld exceeded", (long long)c->cfg.max_blocks);
  if (h.sticky & kStatusPointOverflow)
    return fail(c, AF_EOVERFLOW, "point capacity %lld exceeded", (long long)c->cfg.max_points);
  if (h.sticky & kStatusOutsideGrid)
    return fail(c, AF_EOVERFLOW, "a block left the recorded scene box");
  return AF_OK;
}

static int graph_prepare(af_ctx *c, const float lo[3], const float hi[3], int64_t max_returns,
                         const int32_t *tool_ids, int32_t n_tools, void *stream, bool score);

int af_graph_prepare(af_ctx *c, const float lo[3], const float hi[3], int64_t max_returns,
                     const int32_t *tool_ids, int32_t n_tools, void *stream) {
  return graph_prepare(c, lo, hi, max_returns, tool_ids, n_tools, stream, true);
}

}  // extern "C"

namespace af {
int ctx_graph_prepare_unscored(af_ctx *c, const float lo[3], const float hi[3],
                               int64_t max_returns, const int32_t *tool_ids, int32_t n_tools,
                               void *stream) {
  return graph_prepare(c, lo, hi, max_returns, tool_ids, n_tools, stream, false);
}

int ctx_score_jobs(af_ctx *c, const int32_t *tool_ids, int32_t n_tools, ScoreJob *out) {
  if (!c || !out || n_tools < 1 || n_tools > kMultiTools) return AF_EINVAL;
  for (int32_t i = 0; i < n_tools; ++i) {
    const int32_t id = tool_ids[i];
    if (id < 0 || id >= c->cfg.max_tools || !c->tools[id].entries) return AF_ENOTOOL;
    ScoreJob &j = out[i];
    memset(&j, 0, sizeof(j));
    j.p = c->p;
    j.pts = c->pts;
    j.t = c->tools[id];
    j.g = c->grid;
    j.max_points = c->cfg.max_points;
  }
  return AF_OK;
}

bool ctx_windowed(const af_ctx *c) { return c && c->win_on; }

bool ctx_incremental(const af_ctx *c) { return c && c->incr_on; }

int ctx_frame_slot(af_ctx *c, int64_t max_returns) {
  if (!c || max_returns < 1) return AF_EINVAL;
  if (c->slot_xyz && c->slot_cap >= max_returns) return AF_OK;
  HIP_TRY(c, hipDeviceSynchronize());
  if (c->slot_xyz) dev_free(c, c->slot_xyz, sizeof(float) * 3 * c->slot_cap);
  c->slot_xyz = nullptr;
  c->slot_cap = 0;
  ALLOC(c, c->slot_xyz, 3 * max_returns);
  c->slot_cap = max_returns;
  return AF_OK;
}

// A recorded (unscored) frame scored on its own stream: the launch a scored
// graph ends with (a server step that batches fewer than two streams).
int ctx_score_stream(af_ctx *c, const int32_t *tool_ids, int32_t n_tools, void *stream) {
  if (!c) return AF_EINVAL;
  ToolSet set;
  ToolDev host[kMultiTools];
  const int rc = make_toolset(c, tool_ids, n_tools, set, host);
  if (rc != AF_OK) return rc;
  if (n_tools == 1)   // one tool: the single-tool kernel (same results)
    launch_score(c->p, c->pts, host[0], c->grid, c->cfg.max_points, c->score_variant, c->work,
                 (hipStream_t)stream, true);
  else
    launch_score_multi(c->p, c->pts, c->tools_dev, host, set, c->grid, c->cfg.max_points,
                       c->work, (hipStream_t)stream, true);
  return hip_check(c, "score on the stream");
}
}  // namespace af

extern "C" {

// Capture of one frame on the context's capture stream: integration of up to
// slot_cap returns (the frame's size, origin and id, and the window box, read
// from the device argument block), then normals, masks and scoring of the
// prepared tools.  Without a window the grid covers the scene box and every
// point is scored in one multi-tool launch; with one, the grid is the window's
// and the points inside it are listed and scored tool by tool, so a shift
// (which moves the grid) records the frame again.
static int graph_record(af_ctx *c, hipStream_t s) {
  ToolSet set;
  ToolDev host[kMultiTools];
  // (a windowed frame scores its tools one after the other: they share the
  // mask buffers)
  int rc = make_toolset(c, c->g_ids, c->g_n, set, host, !c->win_on);
  if (rc != AF_OK) return rc;
  if (c->win_on && (rc = window_tools_ok(c, c->g_ids, c->g_n)) != AF_OK) return rc;
  if (c->win_on)   // labels of points no graph scored yet read "never evaluated"
    for (int32_t i = 0; i < c->g_n; ++i) {
      int64_t &init = c->label_init[c->g_ids[i]];
      if (init < c->n_points) {
        launch_label_fill(c->tools[c->g_ids[i]].label, c->tools[c->g_ids[i]].first_free, init,
                          c->n_points, s);
        init = c->n_points;
      }
    }
  HIP_TRY(c, hipStreamSynchronize(s));
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  if (c->graph) hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = c->cap_stream;
  const int64_t cap = c->slot_cap, NP = c->cfg.max_points;
  const int32_t n_tools = c->g_n;
  HIP_TRY(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  launch_frame_prep(c->slot_xyz, c->fargs, cap, c->p, c->map, c->pts, c->fs, c->counters, cs);
  launch_assign_blocks(c->map, c->fs, c->counters, c->fargs, cs);
  launch_commit_blocks(c->map, c->counters, cs);
  launch_touch_band(c->fargs, cap, c->p, c->map, c->fs, c->counters, cs);
  launch_points_append(cap, c->map, c->pts, c->fs, c->counters, c->fargs, cs);
  launch_commit_points(c->pts, c->counters, cs);
  launch_points_view(c->fargs, cap, c->p, c->pts, c->fs, cs);
  launch_integrate(c->fargs, cap, c->p, c->map, c->fs, c->counters, c->grid,
                   std::min<int64_t>(c->cfg.max_blocks, cap * (kMaxSpan + kMaxBand)), cs);
  launch_stick_status(c->counters, c->map.n_blocks, c->pts.n_points, cs);
  for (int32_t i = 0; i < n_tools; ++i)
    launch_zero_words(host[i].counters, sizeof(ScoreCounters), cs);
  if (!c->win_on) {
    launch_normals(c->p, c->map, c->pts, c->grid, NP, cs, true);
    for (int32_t i = 0; i < n_tools; ++i)
      launch_mask(c->p, c->pts, host[i], c->grid, NP, cs, true);
    if (c->g_score) {
      if (n_tools == 1)   // one tool: the single-tool kernel (same results)
        launch_score(c->p, c->pts, host[0], c->grid, NP, c->score_variant, c->work, cs, true);
      else
        launch_score_multi(c->p, c->pts, c->tools_dev, host, set, c->grid, NP, c->work, cs, true);
    }
  } else {
    const int3 lo = make_int3(c->win_lo[0], c->win_lo[1], c->win_lo[2]);
    const int3 hi = make_int3(c->win_hi[0], c->win_hi[1], c->win_hi[2]);
    launch_window_list(c->pts, NP, lo, hi, c->win_sel, c->win_nsel, cs, true);
    PointsDev ps = c->pts;
    ps.sel = c->win_sel;
    ps.n_sel = c->win_nsel;
    launch_normals(c->p, c->map, ps, c->grid, NP, cs, true);
    for (int32_t i = 0; i < n_tools; ++i) {
      launch_mask(c->p, ps, host[i], c->grid, NP, cs, true);
      launch_score(c->p, ps, host[i], c->grid, NP, window_variant(c, host[i]), c->work, cs, true);
    }
  }
  hipGraph_t g = nullptr;
  const hipError_t e1 = hipStreamEndCapture(cs, &g);
  if (e1 != hipSuccess || !g)
    return fail(c, AF_EDEVICE, "frame graph capture: %s", hipGetErrorString(e1));
  c->graph = g;
  HIP_TRY(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  c->graph_stale = false;
  c->last_stream = s;
  return hip_check(c, "graph record");
}

static int graph_prepare(af_ctx *c, const float lo[3], const float hi[3], int64_t max_returns,
                         const int32_t *tool_ids, int32_t n_tools, void *stream, bool score) {
  if (!c) return AF_EINVAL;
  int rc;
  if (c->graph_dirty && (rc = graph_settle(c)) != AF_OK) return rc;
  c->g_n = 0;   // a prepare that fails leaves no graph to replay
  if (!lo || !hi || max_returns < 1) return fail(c, AF_EINVAL, "bad graph arguments");
  if (c->incr_on)
    return fail(c, AF_EINVAL, "a context in incremental mode runs its frames eagerly");
  if (c->win_on && !score)
    return fail(c, AF_EINVAL, "a windowed context scores inside its recorded frame");
  ToolSet set;
  ToolDev host[kMultiTools];
  if ((rc = make_toolset(c, tool_ids, n_tools, set, host, !c->win_on)) != AF_OK) return rc;
  if (c->win_on && (rc = window_tools_ok(c, tool_ids, n_tools)) != AF_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(c, hipStreamSynchronize(s));
  const double bs = 8.0 * c->cfg.voxel;
  int32_t blo[3], bhi[3];
  for (int a = 0; a < 3; ++a) {
    if (!(lo[a] < hi[a]) || !(fabs((double)lo[a]) < 1e4) || !(fabs((double)hi[a]) < 1e4))
      return fail(c, AF_EINVAL, "bad scene box");
    blo[a] = (int32_t)floor((double)lo[a] / bs);
    bhi[a] = (int32_t)floor((double)hi[a] / bs);
  }
  // the grid covers the scene box (and every block so far) and never grows;
  // with a window the box is the window's, wherever it is
  if (!c->win_on) {
    for (int a = 0; a < 3; ++a) {
      c->bbox_lo[a] = c->have_bbox ? std::min(c->bbox_lo[a], blo[a]) : blo[a];
      c->bbox_hi[a] = c->have_bbox ? std::max(c->bbox_hi[a], bhi[a]) : bhi[a];
    }
    c->have_bbox = true;
    if ((rc = regrid(c, s)) != AF_OK) return rc;
  }
  if (max_returns > c->fs.cap && (rc = alloc_scratch(c, max_returns)) != AF_OK) return rc;
  if (c->slot_xyz) dev_free(c, c->slot_xyz, sizeof(float) * 3 * c->slot_cap);
  c->slot_xyz = nullptr;
  ALLOC(c, c->slot_xyz, 3 * max_returns);
  c->slot_cap = max_returns;
  launch_normals(c->p, c->map, c->pts, c->grid, 0, s);   // uploads its constant table
  HIP_TRY(c, hipStreamSynchronize(s));
  HIP_TRY(c, clear_sticky(c));
  c->sticky_reset = false;
  for (int32_t i = 0; i < n_tools; ++i) c->g_ids[i] = tool_ids[i];
  c->g_score = score;
  if (c->win_on && !c->win_set) {
    // the window (and so the grid) is placed by the first frame, which runs
    // eagerly and records the graph
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_stale = false;
    c->g_n = n_tools;
    return AF_OK;
  }
  c->g_n = n_tools;
  if ((rc = graph_record(c, s)) != AF_OK) c->g_n = 0;
  return rc;
}

int af_graph_frame(af_ctx *c, const float *xyz, int64_t n, const float origin[3],
                   int64_t frame_id, void *stream) {
  if (!c) return AF_EINVAL;
  if (!c->g_n || (!c->gexec && !c->win_on)) return fail(c, AF_EINVAL, "no recorded frame graph");
  if (c->graph_stale && !c->win_on)
    return fail(c, AF_EINVAL, "buffers of the recorded frame graph were reallocated: prepare again");
  if (n < 0 || n > c->slot_cap || (n > 0 && !xyz) || !origin)
    return fail(c, AF_EINVAL, "bad frame arguments (n = %lld, slot %lld)", (long long)n,
                (long long)c->slot_cap);
  if (frame_id <= c->last_frame || frame_id > 0x7ffffffe)
    return fail(c, AF_EINVAL, "frame id %lld does not increase", (long long)frame_id);
  int3 Q;
  int *qq[3] = {&Q.x, &Q.y, &Q.z};
  for (int a = 0; a < 3; ++a) {
    double t = (double)origin[a] * c->p.scale;
    if (!(fabs(t) <= (double)kCoordLim)) return fail(c, AF_EINVAL, "sensor origin out of range");
    *qq[a] = (int)llrint(t);
  }
  hipStream_t s = (hipStream_t)stream;
  // a replay still running on another stream reads the slot: let it finish
  if (c->graph_dirty && s != c->last_stream) {
    const int rc = graph_settle(c);
    if (rc != AF_OK) return rc;
  }
  if (n > 0 && xyz != c->slot_xyz)
    HIP_TRY(c, hipMemcpyAsync(c->slot_xyz, xyz, sizeof(float) * 3 * n, hipMemcpyDefault, s));
  int3 wlo = make_int3(-(1 << 30), -(1 << 30), -(1 << 30));
  int3 whi = make_int3(1 << 30, 1 << 30, 1 << 30);
  if (c->win_on) {
    if (!c->gexec || window_shift_due(c, Q)) {
      // the frame that places or moves the window: evictions, block
      // re-creation and the grid's move run eagerly (as af_integrate_frame
      // and af_score_points would), then the frame is recorded again
      int rc;
      if (c->graph_dirty && (rc = graph_settle(c)) != AF_OK) return rc;
      if ((rc = af_integrate_frame(c, c->slot_xyz, n, origin, frame_id, stream)) != AF_OK)
        return rc;
      if ((rc = score_window(c, c->g_ids, c->g_n, s)) != AF_OK) return rc;
      return graph_record(c, s);
    }
    if (c->graph_stale) {   // (a windowed context records the frame again)
      int rc;
      if (c->graph_dirty && (rc = graph_settle(c)) != AF_OK) return rc;
      if ((rc = graph_record(c, s)) != AF_OK) return rc;
    }
    wlo = make_int3(c->win_lo[0], c->win_lo[1], c->win_lo[2]);
    whi = make_int3(c->win_hi[0], c->win_hi[1], c->win_hi[2]);
  }
  launch_set_frame_args(c->fargs, n, Q, (int32_t)frame_id, wlo, whi, s,
                        c->sticky_reset ? c->counters : nullptr);
  c->sticky_reset = false;
  HIP_TRY(c, hipGraphLaunch(c->gexec, s));
  c->last_frame = frame_id;
  c->last_stream = s;
  c->graph_dirty = true;
  return hip_check(c, "graph frame");
}

float *af_graph_slot(af_ctx *c) { return c ? c->slot_xyz : nullptr; }

int af_graph_sync(af_ctx *c) {
  if (!c) return AF_EINVAL;
  if (!c->graph_dirty) return sync_last(c);
  return graph_settle(c);
}

// Build the smoothed score's field in buffers b (enqueued on s).
static void smooth_build(af_ctx *c, const SmoothBuffers &b, hipStream_t s, SmoothField &f) {
  const float tau = (float)((double)c->p.tau_u / c->p.scale);
  launch_smooth_prepare(c->p, c->map, c->n_blocks, c->grid, c->grid_bricks, tau, b, s);
  f.T9 = b.T9;
  f.bid9 = b.bid9;
  for (int a = 0; a < 3; ++a) {
    f.g0[a] = c->grid.g0[a];
    f.gd[a] = c->grid_bricks > 0 ? c->grid.gd[a] : 0;
  }
  f.tau = tau;
}

// TSDF values and the brick table for the smoothed score, rebuilt from the
// current map (a few tens of microseconds; the map may change between calls).
static int smooth_prepare(af_ctx *c, hipStream_t s, SmoothField &f) {
  if (c->win_on) return fail(c, AF_EINVAL, "the smoothed score is not available with a window");
  int rc;
  if (c->graph_dirty && (rc = graph_settle(c)) != AF_OK) return rc;
  if ((rc = regrid(c, s)) != AF_OK) return rc;
  SmoothBuffers &b = c->sm;
  const int64_t nv = std::max<int64_t>(1, c->n_blocks * kBlockVox);
  const int64_t nb = std::max<int64_t>(1, c->grid_bricks);
  // every mapped block marks itself and its -1 neighbours: at most 8 aprons each
  const int64_t na = std::max<int64_t>(1, std::min<int64_t>(8 * c->n_blocks, c->grid_bricks));
  if (nv > c->sm_T_cap || nb > c->sm_bid_cap || na > b.apron_cap || !b.count || !b.work) {
    HIP_TRY(c, hipStreamSynchronize(s));
    if (nv > c->sm_T_cap) {
      if (b.T) dev_free(c, b.T, sizeof(float) * c->sm_T_cap);
      b.T = nullptr;
      c->sm_T_cap = 0;
      const int64_t cap = std::min<int64_t>(c->cfg.max_blocks * kBlockVox, nv + nv / 2 + kBlockVox);
      ALLOC(c, b.T, cap);
      c->sm_T_cap = cap;
    }
    if (nb > c->sm_bid_cap) {
      if (b.bid) dev_free(c, b.bid, sizeof(int32_t) * c->sm_bid_cap);
      if (b.bid9) dev_free(c, b.bid9, sizeof(int32_t) * c->sm_bid_cap);
      b.bid = b.bid9 = nullptr;
      c->sm_bid_cap = 0;
      ALLOC(c, b.bid, nb);
      ALLOC(c, b.bid9, nb);
      c->sm_bid_cap = nb;
    }
    if (na > b.apron_cap) {
      if (b.T9) dev_free(c, b.T9, sizeof(float) * 729 * b.apron_cap);
      if (b.brick_of) dev_free(c, b.brick_of, sizeof(int32_t) * b.apron_cap);
      b.T9 = nullptr;
      b.brick_of = nullptr;
      b.apron_cap = 0;
      const int64_t cap = std::min<int64_t>(std::max<int64_t>(1, c->grid_bricks), na + na / 2 + 64);
      ALLOC(c, b.T9, cap * 729);
      ALLOC(c, b.brick_of, cap);
      b.apron_cap = cap;
    }
    if (!b.count) ALLOC(c, b.count, 1);
    if (!b.work) ALLOC(c, b.work, 8);   // one counter per XCD
  }
  smooth_build(c, b, s, f);
  return hip_check(c, "smooth prepare");
}

static bool smooth_args_ok(int32_t M, float c_thr, float tau_s) {
  return M >= 1 && M <= 1024 && std::isfinite(c_thr) && tau_s > 0.f && std::isfinite(tau_s);
}

int af_smooth_eval(af_ctx *c, const float *p, const float *q, int64_t n, const float *samples,
                   int32_t M, float c_thr, float tau_s, const float *grad_s, float *s_out,
                   float *dq, float *dp, void *stream) {
  if (!c) return AF_EINVAL;
  if (n < 0 || (n > 0 && (!p || !q || !samples)) || !smooth_args_ok(M, c_thr, tau_s) ||
      (!dq) != (!dp) || (n > 0 && !s_out && !dq))
    return fail(c, AF_EINVAL, "bad smoothed-score arguments");
  hipStream_t s = (hipStream_t)stream;
  SmoothField f;
  int rc = smooth_prepare(c, s, f);
  if (rc != AF_OK) return rc;
  launch_smooth_eval(f, 256.0 / c->p.scale, p, q, n, samples, M, c_thr, tau_s, grad_s, s_out, dq,
                     dp, c->sm.work, s);
  c->last_stream = s;
  return hip_check(c, "smooth eval");
}

int af_smooth_refine(af_ctx *c, const float *p, int64_t n_points, const float *q0,
                     int32_t n_starts, const float *samples, int32_t M, float c_thr, float tau_s,
                     int32_t steps, float eta, float max_step, float *q_out, float *s_out,
                     void *stream) {
  if (!c) return AF_EINVAL;
  if (n_points < 0 || n_starts < 1 || steps < 0 || steps > 100000 ||
      (n_points > 0 && (!p || !q0 || !samples || !q_out || !s_out)) ||
      !smooth_args_ok(M, c_thr, tau_s) || !std::isfinite(eta) || !(max_step > 0.f) ||
      n_points > ((int64_t)1 << 40) / n_starts)
    return fail(c, AF_EINVAL, "bad refinement arguments");
  hipStream_t s = (hipStream_t)stream;
  SmoothField f;
  int rc = smooth_prepare(c, s, f);
  if (rc != AF_OK) return rc;
  hipEvent_t t0 = timing_mark(c, s);
  launch_smooth_refine(f, 256.0 / c->p.scale, p, n_points, q0, n_starts, samples, M, c_thr, tau_s,
                       steps, eta, max_step, q_out, s_out, c->sm.work, s);
  hipEvent_t t1 = timing_mark(c, s);
  if (c->timing) timing_pair(c, ST_K_SMOOTH, t0, t1);
  c->last_stream = s;
  return hip_check(c, "smooth refine");
}

// ---------------------------------------------------------------------------
// The no-allocation form of af_smooth_eval.  Its scratch (the per-voxel values,
// the brick tables, the apron bricks and the work counters that af_smooth_eval
// keeps in context buffers grown on demand) lives in this file-scope device
// array instead: each GPU the library runs on holds one copy, at its own
// address, until the process ends.  In host code `scratch` names a host-side
// stand-in, so the device address is looked up once per device with
// hipGetSymbolAddress and only that address is ever passed to kernels.
constexpr int64_t kStaticScratchBytes = int64_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];   // device address of `scratch`, per device id

// This GPU's scratch address (looked up on the first call on the device).
static int static_scratch(af_ctx *c, uint8_t **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(c, AF_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev != c->device)
    return fail(c, AF_EINVAL, "device %d is current, the context lives on device %d", dev,
                c->device);
  if (dev < 0 || dev >= kMaxDevices) return fail(c, AF_EDEVICE, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(c, AF_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = (uint8_t *)g_scratch_dev[dev];
  return AF_OK;
}

int af_smooth_eval_static(af_ctx *c, const float *p, const float *q, int64_t n,
                          const float *samples, int32_t M, float c_thr, float tau_s,
                          const float *grad_s, float *s_out, float *dq, float *dp, void *stream) {
  if (!c) return AF_EINVAL;
  if (n < 0 || (n > 0 && (!p || !q || !samples)) || !smooth_args_ok(M, c_thr, tau_s) ||
      (!dq) != (!dp) || (n > 0 && !s_out && !dq))
    return fail(c, AF_EINVAL, "bad smoothed-score arguments");
  hipStream_t s = (hipStream_t)stream;
  if (c->win_on) return fail(c, AF_EINVAL, "the smoothed score is not available with a window");
  uint8_t *base = nullptr;
  int rc = static_scratch(c, &base);
  if (rc != AF_OK) return rc;
  if (c->graph_dirty && (rc = graph_settle(c)) != AF_OK) return rc;
  if (!grid_covers(c))
    return fail(c, AF_EINVAL, "the brick grid must grow before this call (af_smooth_eval "
                              "or af_score_points grows it)");
  // carve the scratch: every part 256-byte aligned
  const int64_t nv = std::max<int64_t>(1, c->n_blocks * kBlockVox);
  const int64_t nb = std::max<int64_t>(1, c->grid_bricks);
  const int64_t na = std::max<int64_t>(1, std::min<int64_t>(8 * c->n_blocks, c->grid_bricks));
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = off;
    off += (bytes + 255) & ~int64_t(255);
    return at;
  };
  const int64_t oT = take(sizeof(float) * nv), oBid = take(sizeof(int32_t) * nb),
                oBid9 = take(sizeof(int32_t) * nb), oOf = take(sizeof(int32_t) * na),
                oT9 = take(sizeof(float) * 729 * na), oCount = take(sizeof(int32_t)),
                oWork = take(sizeof(unsigned long long) * 8);
  if (off > kStaticScratchBytes)
    return fail(c, AF_ENOMEM,
                "the map needs %lld bytes of scratch (%lld blocks, %lld grid bricks); the static "
                "scratch holds %lld (af_smooth_eval has no such limit)",
                (long long)off, (long long)c->n_blocks, (long long)c->grid_bricks,
                (long long)kStaticScratchBytes);
  SmoothBuffers b;
  memset(&b, 0, sizeof(b));
  b.T = (float *)(base + oT);
  b.bid = (int32_t *)(base + oBid);
  b.bid9 = (int32_t *)(base + oBid9);
  b.brick_of = (int32_t *)(base + oOf);
  b.T9 = (float *)(base + oT9);
  b.count = (int32_t *)(base + oCount);
  b.work = (unsigned long long *)(base + oWork);
  b.apron_cap = na;
  SmoothField f;
  smooth_build(c, b, s, f);   // clears the count, the brick tables and the work counters first
  launch_smooth_eval(f, 256.0 / c->p.scale, p, q, n, samples, M, c_thr, tau_s, grad_s, s_out, dq,
                     dp, b.work, s);
  c->last_stream = s;
  return hip_check(c, "smooth eval (static scratch)");
}

int af_incremental_enable(af_ctx *c, int32_t tool_id, int32_t budget) {
  if (!c) return AF_EINVAL;
  if (tool_id < 0 || tool_id >= c->cfg.max_tools) return fail(c, AF_EINVAL, "bad tool id");
  const ToolDev &t = c->tools[tool_id];
  if (!t.entries) return fail(c, AF_ENOTOOL, "tool %d has no kernels", tool_id);
  if (budget < 1) return fail(c, AF_EINVAL, "budget must be positive");
  if (c->p.n_c > 255) return fail(c, AF_EINVAL, "n_c above 255");
  if (c->last_frame >= 0 || c->n_points > 0)
    return fail(c, AF_EINVAL, "the incremental mode starts before the first frame");
  if (c->g_n) return fail(c, AF_EINVAL, "a context with a recorded frame graph runs stateless frames");
  if (!score_variant_takes_list(score_variant_default(), t))
    return fail(c, AF_EINVAL, "tool %d: K above 1024 or reach above 255 voxels", tool_id);
  budget = (int32_t)std::min<int64_t>(budget, c->cfg.max_points);
  IncrDev &I = c->incr;
  if (!c->incr_on) {
    const int64_t NP = c->cfg.max_points;
    memset(&I, 0, sizeof(I));
    ALLOC(c, I.best, NP);
    ALLOC(c, I.best_dir, NP);
    ALLOC(c, I.a, NP);
    ALLOC(c, I.S_prev, NP);
    ALLOC(c, I.W_prev, NP);
    ALLOC(c, I.pending, NP);
    ALLOC(c, I.outcome, NP);
    ALLOC(c, I.label, NP);
    ALLOC(c, I.n_sel, 1);
    ALLOC(c, I.bsum, (NP + 1023) / 1024);
    ALLOC(c, I.hist, 2 * 65536);
    ALLOC(c, I.cand_h, 1024);
    ALLOC(c, I.cand_k, 1024);
    ALLOC(c, I.sampled, 256);
    ALLOC(c, I.ctr, 1);
    ALLOC(c, I.budget_dev, 1);
    ALLOC(c, I.frame_budget, 1);
    ALLOC(c, c->incr_changed, c->cfg.max_blocks * kBlockVox);
    I.max_points = NP;
  }
  if (!c->incr_on || budget > I.budget) {
    if (I.sel) dev_free(c, I.sel, sizeof(int32_t) * I.budget);
    if (I.score_new) dev_free(c, I.score_new, I.budget);
    I.sel = nullptr;
    I.score_new = nullptr;
    ALLOC(c, I.sel, budget);
    ALLOC(c, I.score_new, budget);
  }
  I.budget = budget;
  I.lookup_target = 0;
  I.b_min = 1;
  I.b_max = budget;
  c->incr_budget0 = budget;
  c->incr_on = true;
  c->incr_tool = tool_id;
  c->have_q = false;
  c->incr_seen = 0;
  launch_incr_init(I, c->p.n_c, nullptr);
  launch_incr_set_budget(I, budget, nullptr);
  return hip_check(c, "incremental enable");
}

int af_incremental_c2f(af_ctx *c, double coarse_deg, double fine_deg, double radius_m) {
  if (!c) return AF_EINVAL;
  if (!c->incr_on) return fail(c, AF_EINVAL, "incremental mode not enabled");
  if (c->last_frame >= 0 || c->n_points > 0)
    return fail(c, AF_EINVAL, "the coarse-to-fine search is set before the first frame");
  const double r = radius_m / c->cfg.voxel;
  if (!(coarse_deg > 0 && coarse_deg <= 180) || !(fine_deg > 0 && fine_deg <= 180) ||
      !(radius_m > 0) || !(r <= 64.0))
    return fail(c, AF_EINVAL, "bad coarse-to-fine parameters (radius at most 64 voxels)");
  IncrDev &I = c->incr;
  const ToolDev &t = c->tools[c->incr_tool];
  const int32_t K = t.K, mw = (K + 63) / 64;
  std::vector<double> rot(9 * (size_t)K);
  HIP_TRY(c, hipMemcpy(rot.data(), t.rot, sizeof(double) * rot.size(), hipMemcpyDeviceToHost));
  auto dir = [&](int k, int i) { return rot[9 * (size_t)k + 3 * i]; };
  auto dot = [&](int a, int b) {
    return (dir(a, 0) * dir(b, 0) + dir(a, 1) * dir(b, 1)) + dir(a, 2) * dir(b, 2);
  };
  // coarse pass: greedy in index order, a direction at least coarse_deg from
  // every direction taken before is taken; orientations sharing a taken
  // direction belong to the pass as well
  const double cc = std::cos(coarse_deg * (M_PI / 180.0));
  const double cf = std::cos(fine_deg * (M_PI / 180.0));
  std::vector<int> taken;
  std::vector<uint64_t> coarse(mw, 0ull), fine((size_t)K * mw, 0ull);
  for (int k = 0; k < K; ++k) {
    bool same = false, far = true;
    for (int q : taken) {
      if (dir(k, 0) == dir(q, 0) && dir(k, 1) == dir(q, 1) && dir(k, 2) == dir(q, 2)) same = true;
      if (!(dot(k, q) <= cc + 1e-12)) far = false;
    }
    if (same || far) {
      if (!same) taken.push_back(k);
      coarse[k >> 6] |= 1ull << (k & 63);
    }
  }
  for (int a = 0; a < K; ++a)
    for (int k = 0; k < K; ++k)
      if (dot(k, a) >= cf - 1e-12) fine[(size_t)a * mw + (k >> 6)] |= 1ull << (k & 63);
  // neighbour offsets within the radius, nearest first, ties by (dz, dy, dx)
  const int64_t r2 = (int64_t)std::floor(r * r + 1e-9);
  const int rc = (int)std::floor(std::sqrt((double)r2));
  std::vector<std::array<int, 4>> offs;
  for (int z = -rc; z <= rc; ++z)
    for (int y = -rc; y <= rc; ++y)
      for (int x = -rc; x <= rc; ++x) {
        const int d2 = x * x + y * y + z * z;
        if (d2 > 0 && d2 <= r2) offs.push_back({d2, z, y, x});
      }
  std::sort(offs.begin(), offs.end());
  std::vector<uint32_t> packed(offs.size());
  for (size_t e = 0; e < offs.size(); ++e)
    packed[e] = (uint32_t)(offs[e][3] + 512) | ((uint32_t)(offs[e][2] + 512) << 10) |
                ((uint32_t)(offs[e][1] + 512) << 20);
  if (I.c2f_on) {
    dev_free(c, I.c2f_coarse, sizeof(uint64_t) * I.c2f_mw);
    dev_free(c, I.c2f_fine, sizeof(uint64_t) * (size_t)K * I.c2f_mw);
    dev_free(c, I.c2f_off, sizeof(uint32_t) * std::max(1, I.c2f_n_off));
    I.c2f_on = 0;
  }
  ALLOC(c, I.c2f_coarse, mw);
  ALLOC(c, I.c2f_fine, (int64_t)K * mw);
  ALLOC(c, I.c2f_off, std::max<int64_t>(1, (int64_t)packed.size()));
  if (!I.n_resolved) ALLOC(c, I.n_resolved, 1);
  HIP_TRY(c, hipMemcpy(I.c2f_coarse, coarse.data(), sizeof(uint64_t) * mw, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(I.c2f_fine, fine.data(), sizeof(uint64_t) * fine.size(),
                       hipMemcpyHostToDevice));
  if (!packed.empty())
    HIP_TRY(c, hipMemcpy(I.c2f_off, packed.data(), sizeof(uint32_t) * packed.size(),
                         hipMemcpyHostToDevice));
  I.c2f_mw = mw;
  I.c2f_n_off = (int32_t)packed.size();
  I.c2f_on = 1;
  return AF_OK;
}

// The resolved-voxel plane of the coarse-to-fine search, sized to the grid.
static int c2f_plane(af_ctx *c) {
  IncrDev &I = c->incr;
  if (!I.c2f_on || c->grid_bricks <= c->c2f_plane_bricks) return AF_OK;
  if (I.resolved) dev_free(c, I.resolved, sizeof(uint32_t) * 16 * c->c2f_plane_bricks);
  I.resolved = nullptr;
  c->c2f_plane_bricks = 0;
  ALLOC(c, I.resolved, 16 * c->grid_bricks);
  c->c2f_plane_bricks = c->grid_bricks;
  return AF_OK;
}

int af_incremental_budget(af_ctx *c, int64_t lookup_target, int32_t b_min, int32_t b_max) {
  if (!c) return AF_EINVAL;
  if (!c->incr_on) return fail(c, AF_EINVAL, "incremental mode not enabled");
  if (c->last_frame >= 0 || c->n_points > 0)
    return fail(c, AF_EINVAL, "the budget rule is set before the first frame");
  if (lookup_target < 0 || lookup_target > ((int64_t)1 << 40) || b_min < 1 || b_max < b_min)
    return fail(c, AF_EINVAL, "bad budget rule (target %lld, [%d, %d])",
                (long long)lookup_target, b_min, b_max);
  IncrDev &I = c->incr;
  b_max = (int32_t)std::min<int64_t>(b_max, c->cfg.max_points);
  b_min = std::min(b_min, b_max);
  if (b_max > I.budget) {
    HIP_TRY(c, hipDeviceSynchronize());
    dev_free(c, I.sel, sizeof(int32_t) * I.budget);
    dev_free(c, I.score_new, I.budget);
    I.sel = nullptr;
    I.score_new = nullptr;
    I.budget = 0;
    ALLOC(c, I.sel, b_max);
    ALLOC(c, I.score_new, b_max);
    I.budget = b_max;
  }
  I.lookup_target = lookup_target;
  I.b_min = b_min;
  I.b_max = b_max;
  const int32_t first = std::min(std::max(c->incr_budget0, b_min), b_max);
  launch_incr_set_budget(I, first, nullptr);
  return hip_check(c, "incremental budget");
}

// The sliding window's block box for the incremental kernels (unbounded
// without a window).
static void incr_window(af_ctx *c) {
  IncrDev &I = c->incr;
  if (c->win_on && c->win_set) {
    I.wlo = make_int3(c->win_lo[0], c->win_lo[1], c->win_lo[2]);
    I.whi = make_int3(c->win_hi[0], c->win_hi[1], c->win_hi[2]);
  } else {
    I.wlo = make_int3(-(1 << 30), -(1 << 30), -(1 << 30));
    I.whi = make_int3(1 << 30, 1 << 30, 1 << 30);
  }
}

int af_incremental_frame(af_ctx *c, const float *xyz, int64_t n, const float origin[3],
                         int64_t frame_id, void *stream) {
  if (!c) return AF_EINVAL;
  if (!c->incr_on) return fail(c, AF_EINVAL, "incremental mode not enabled");
  hipStream_t s = (hipStream_t)stream;
  c->fs.changed = c->incr_changed;
  int rc = af_integrate_frame(c, xyz, n, origin, frame_id, stream);
  c->fs.changed = nullptr;
  if (rc != AF_OK) return rc;
  // trigger (iii): the sensor position as integrated (fixed point), against
  // where the trigger last fired
  int32_t Q[3];
  for (int a = 0; a < 3; ++a) Q[a] = (int32_t)llrint((double)origin[a] * c->p.scale);
  bool moved = false;
  if (!c->have_q) {
    c->have_q = true;
    memcpy(c->q_last, Q, sizeof(Q));
  } else {
    int64_t d2 = 0;
    for (int a = 0; a < 3; ++a) d2 += (int64_t)(Q[a] - c->q_last[a]) * (Q[a] - c->q_last[a]);
    if (d2 > c->p.dmin2) {
      moved = true;
      memcpy(c->q_last, Q, sizeof(Q));
    }
  }
  IncrDev &I = c->incr;
  incr_window(c);
  if ((rc = c2f_plane(c)) != AF_OK) return rc;
  launch_incr_frame_front(c->pts, c->map, I, c->incr_changed, c->counters, c->n_points,
                          c->incr_seen, (int32_t)frame_id, moved, c->p.conf_min_w, s);
  c->incr_seen = c->n_points;
  PointsDev ps = c->pts;
  ps.sel = I.sel;
  ps.n_sel = I.n_sel;
  ToolDev &t = c->tools[c->incr_tool];
  HIP_TRY(c, hipMemsetAsync(t.counters, 0, sizeof(ScoreCounters), s));
  launch_normals(c->p, c->map, ps, c->grid, I.budget, s, true);
  launch_mask(c->p, ps, t, c->grid, I.budget, s, true);
  launch_incr_c2f(c->pts, t, c->grid, I, c->n_points, c->grid_bricks, c->p.n_c, s);
  launch_score(c->p, ps, t, c->grid, I.budget, score_variant_default(), c->work, s, true);
  launch_incr_frame_back(ps, c->map, t, c->grid, I, c->n_points, c->p.n_c, s);
  launch_incr_budget(I, t, s);
  c->last_stream = s;
  return hip_check(c, "incremental frame");
}

int af_incremental_drain(af_ctx *c, int32_t max_evals, void *stream) {
  if (!c) return AF_EINVAL;
  if (!c->incr_on) return fail(c, AF_EINVAL, "incremental mode not enabled");
  IncrDev &I = c->incr;
  if (max_evals < 0 || max_evals > I.budget)
    return fail(c, AF_EINVAL, "max_evals %d outside [0, %d]", max_evals, I.budget);
  if (c->graph_dirty) {
    const int rc = graph_settle(c);
    if (rc != AF_OK) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  incr_window(c);
  PointsDev ps = c->pts;
  ps.sel = I.sel;
  ps.n_sel = I.n_sel;
  ToolDev &t = c->tools[c->incr_tool];
  int rc = c2f_plane(c);
  if (rc != AF_OK) return rc;
  launch_incr_drain_front(c->pts, c->map, I, c->n_points, max_evals, c->p.conf_min_w, s);
  HIP_TRY(c, hipMemsetAsync(t.counters, 0, sizeof(ScoreCounters), s));
  launch_normals(c->p, c->map, ps, c->grid, I.budget, s, true);
  launch_mask(c->p, ps, t, c->grid, I.budget, s, true);
  launch_incr_c2f(c->pts, t, c->grid, I, c->n_points, c->grid_bricks, c->p.n_c, s);
  launch_score(c->p, ps, t, c->grid, I.budget, score_variant_default(), c->work, s, true);
  launch_incr_frame_back(ps, c->map, t, c->grid, I, c->n_points, c->p.n_c, s);
  c->last_stream = s;
  return hip_check(c, "incremental drain");
}

int af_incremental_stats(af_ctx *c, af_incr_stats *st) {
  if (!c || !st) return AF_EINVAL;
  if (!c->incr_on) return fail(c, AF_EINVAL, "incremental mode not enabled");
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  IncrCounters h;
  int32_t nsel = 0, nch = 0;
  HIP_TRY(c, hipMemcpy(&h, c->incr.ctr, sizeof(h), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(&nsel, c->incr.n_sel, sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(&nch, &c->counters->n_changed, sizeof(int32_t), hipMemcpyDeviceToHost));
  st->new_points = h.new_points;
  st->trig_i = h.trig_i;
  st->trig_ii = h.trig_ii;
  st->trig_iii = h.trig_iii;
  st->changed = nch;
  st->sampled = h.sampled;
  int32_t cap = 0;
  HIP_TRY(c, hipMemcpy(&cap, c->incr.budget_dev, sizeof(int32_t), hipMemcpyDeviceToHost));
  st->queued = h.queued;
  st->evaluated = nsel;
  st->backlog = (int64_t)h.queued - nsel;
  st->budget = cap;
  return AF_OK;
}

int af_read_incremental(af_ctx *c, int64_t first, int64_t count, int64_t *key, uint8_t *label,
                        uint8_t *best, int16_t *best_dir, double *a, int64_t *n_written) {
  if (!c) return AF_EINVAL;
  if (!c->incr_on) return fail(c, AF_EINVAL, "incremental mode not enabled");
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  const int64_t m = std::max<int64_t>(0, std::min<int64_t>(count, c->n_points - first));
  if (n_written) *n_written = m;
  if (m == 0 || first < 0) return first < 0 ? fail(c, AF_EINVAL, "bad range") : AF_OK;
  const IncrDev &I = c->incr;
  if (key) HIP_TRY(c, hipMemcpy(key, c->pts.key + first, sizeof(int64_t) * m, hipMemcpyDeviceToHost));
  if (label) HIP_TRY(c, hipMemcpy(label, I.label + first, m, hipMemcpyDeviceToHost));
  if (best) HIP_TRY(c, hipMemcpy(best, I.best + first, m, hipMemcpyDeviceToHost));
  if (best_dir)
    HIP_TRY(c, hipMemcpy(best_dir, I.best_dir + first, sizeof(int16_t) * m, hipMemcpyDeviceToHost));
  if (a) HIP_TRY(c, hipMemcpy(a, I.a + first, sizeof(double) * m, hipMemcpyDeviceToHost));
  return AF_OK;
}

int af_score_variant_count(void) { return score_variants(); }

const char *af_score_variant_name(int32_t v) { return score_variant_name(v); }

int af_set_score_variant(af_ctx *c, int32_t v) {
  if (!c) return AF_EINVAL;
  if (v < 0 || v >= score_variants()) return fail(c, AF_EINVAL, "score variant %d out of range", v);
  c->score_variant = v;
  return AF_OK;
}

int af_score_variant_default(void) { return af::score_variant_default(); }

int32_t af_get_score_variant(af_ctx *c) { return c ? c->score_variant : -1; }

int af_tune_score(af_ctx *c, int32_t tool_id, int32_t reps, void *stream, int32_t *best,
                  float *ms_per_variant) {
  if (!c) return AF_EINVAL;
  if (c->graph_dirty) {
    const int rc = graph_settle(c);
    if (rc != AF_OK) return rc;
  }
  if (tool_id < 0 || tool_id >= c->cfg.max_tools) return fail(c, AF_EINVAL, "bad tool id");
  if (c->win_on) return fail(c, AF_EINVAL, "variant tuning is not available with a window");
  ToolDev &t = c->tools[tool_id];
  if (!t.entries) return fail(c, AF_ENOTOOL, "tool %d has no kernels", tool_id);
  if (reps < 1) reps = 1;
  hipStream_t s = (hipStream_t)stream;
  launch_normals(c->p, c->map, c->pts, c->grid, c->n_points, s);
  launch_mask(c->p, c->pts, t, c->grid, c->n_points, s);
  hipEvent_t a, b;
  HIP_TRY(c, hipEventCreate(&a));
  HIP_TRY(c, hipEventCreate(&b));
  int nv = score_variants();
  float best_ms = 3.4e38f;
  int best_v = c->score_variant;
  for (int v = 0; v < nv; ++v) {
    launch_score(c->p, c->pts, t, c->grid, c->n_points, v, c->work, s);  // warm
    HIP_TRY(c, hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r)
      launch_score(c->p, c->pts, t, c->grid, c->n_points, v, c->work, s);
    HIP_TRY(c, hipEventRecord(b, s));
    HIP_TRY(c, hipEventSynchronize(b));
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, a, b));
    ms /= (float)reps;
    if (ms_per_variant) ms_per_variant[v] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best_v = v;
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  c->score_variant = best_v;
  if (best) *best = best_v;
  HIP_TRY(c, hipMemsetAsync(t.counters, 0, sizeof(ScoreCounters), s));
  c->last_stream = s;
  return hip_check(c, "tune");
}

static int sync_last(af_ctx *c) {
  if (c->graph_dirty) return graph_settle(c);
  HIP_TRY(c, hipStreamSynchronize(c->last_stream));
  return AF_OK;
}

int64_t af_num_points(af_ctx *c) {
  if (!c || sync_last(c) != AF_OK) return -1;
  return c->n_points;
}

int64_t af_num_blocks(af_ctx *c) {
  if (!c || sync_last(c) != AF_OK) return -1;
  return c->n_blocks;
}

int af_read_labels(af_ctx *c, int32_t tool_id, int64_t first, int64_t count, int64_t *key,
                   uint8_t *label, int16_t *first_free, uint16_t *w, int64_t *n_written) {
  if (!c) return AF_EINVAL;
  if (tool_id < 0 || tool_id >= c->cfg.max_tools) return fail(c, AF_EINVAL, "bad tool id");
  ToolDev &t = c->tools[tool_id];
  if (!t.entries) return fail(c, AF_ENOTOOL, "tool %d has no kernels", tool_id);
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  if (first < 0 || count < 0) return fail(c, AF_EINVAL, "bad range");
  int64_t m = std::max<int64_t>(0, std::min<int64_t>(count, c->n_points - first));
  if (n_written) *n_written = m;
  if (m == 0) return AF_OK;
  if (key) HIP_TRY(c, hipMemcpy(key, c->pts.key + first, sizeof(int64_t) * m, hipMemcpyDeviceToHost));
  if (label) HIP_TRY(c, hipMemcpy(label, t.label + first, m, hipMemcpyDeviceToHost));
  if (first_free)
    HIP_TRY(c, hipMemcpy(first_free, t.first_free + first, sizeof(int16_t) * m, hipMemcpyDeviceToHost));
  if (w) {
    std::vector<int32_t> addr(m);
    HIP_TRY(c, hipMemcpy(addr.data(), c->pts.addr + first, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    std::vector<uint16_t> Wall((size_t)c->n_blocks * kBlockVox);
    if (!Wall.empty())
      HIP_TRY(c, hipMemcpy(Wall.data(), c->map.W, sizeof(uint16_t) * Wall.size(), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) w[i] = addr[i] >= 0 ? Wall[addr[i]] : 0;
  }
  return AF_OK;
}

int af_read_tsdf(af_ctx *c, int64_t *key, int64_t *S, int32_t *W, uint8_t *cleared, int64_t cap,
                 int64_t *n) {
  if (!c) return AF_EINVAL;
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  const int64_t nb = c->n_blocks;
  std::vector<int64_t> bkey(nb);
  std::vector<int32_t> hS(nb * kBlockVox);
  std::vector<uint16_t> hW(nb * kBlockVox);
  std::vector<uint32_t> hc(nb * 16);
  if (nb > 0) {
    HIP_TRY(c, hipMemcpy(bkey.data(), c->map.bkey, sizeof(int64_t) * nb, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(hS.data(), c->map.S, sizeof(int32_t) * hS.size(), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(hW.data(), c->map.W, sizeof(uint16_t) * hW.size(), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(hc.data(), c->map.clr, sizeof(uint32_t) * hc.size(), hipMemcpyDeviceToHost));
  }
  int64_t cnt = 0;
  for (int64_t b = 0; b < nb; ++b) {
    int32_t bx, by, bz;
    unpack_key(bkey[b], bx, by, bz);
    for (int vi = 0; vi < kBlockVox; ++vi) {
      int64_t v = b * kBlockVox + vi;
      bool cl = (hc[b * 16 + (vi >> 5)] >> (vi & 31)) & 1u;
      if (hW[v] == 0 && !cl) continue;
      if (cnt < cap) {
        if (key) key[cnt] = pack_key(8 * bx + (vi & 7), 8 * by + ((vi >> 3) & 7), 8 * bz + (vi >> 6));
        if (S) S[cnt] = hS[v];
        if (W) W[cnt] = hW[v];
        if (cleared) cleared[cnt] = cl ? 1 : 0;
      }
      ++cnt;
    }
  }
  if (n) *n = cnt;
  return AF_OK;
}

int af_read_points(af_ctx *c, int64_t first, int64_t count, int64_t *key, int32_t *first_frame,
                   int32_t *n_vp, int32_t *vp, int64_t *sumq, int32_t *nq, int64_t *n_written) {
  if (!c) return AF_EINVAL;
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  if (first < 0 || count < 0) return fail(c, AF_EINVAL, "bad range");
  int64_t m = std::max<int64_t>(0, std::min<int64_t>(count, c->n_points - first));
  if (n_written) *n_written = m;
  if (m == 0) return AF_OK;
  const PointsDev &q = c->pts;
  if (key) HIP_TRY(c, hipMemcpy(key, q.key + first, sizeof(int64_t) * m, hipMemcpyDeviceToHost));
  if (first_frame)
    HIP_TRY(c, hipMemcpy(first_frame, q.first + first, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  if (nq) HIP_TRY(c, hipMemcpy(nq, q.nq + first, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  if (sumq) HIP_TRY(c, hipMemcpy(sumq, q.sumq + 3 * first, sizeof(int64_t) * 3 * m, hipMemcpyDeviceToHost));
  if (n_vp || vp) {
    std::vector<int32_t> cnt(m), head(m), ring(m * kMaxVp * 3);
    HIP_TRY(c, hipMemcpy(cnt.data(), q.nvp + first, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(head.data(), q.head + first, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(ring.data(), q.vp + first * kMaxVp * 3, sizeof(int32_t) * ring.size(),
                         hipMemcpyDeviceToHost));
    const int nv = c->cfg.n_vp;
    for (int64_t i = 0; i < m; ++i) {
      if (n_vp) n_vp[i] = cnt[i];
      if (!vp) continue;
      int start = (head[i] - cnt[i] + nv) % nv;  // oldest first
      for (int j = 0; j < kMaxVp; ++j)
        for (int a = 0; a < 3; ++a)
          vp[(i * kMaxVp + j) * 3 + a] =
              j < cnt[i] ? ring[(i * kMaxVp + (start + j) % nv) * 3 + a] : 0;
    }
  }
  return AF_OK;
}

int af_read_tool_table(af_ctx *c, int32_t tool_id, int32_t k, int32_t *off, uint8_t *cls,
                       int64_t cap, int64_t *m) {
  if (!c) return AF_EINVAL;
  if (tool_id < 0 || tool_id >= c->cfg.max_tools) return fail(c, AF_EINVAL, "bad tool id");
  ToolDev &t = c->tools[tool_id];
  if (!t.entries) return fail(c, AF_ENOTOOL, "tool %d has no kernels", tool_id);
  if (k < 0 || k >= t.K) return fail(c, AF_EINVAL, "orientation %d outside [0, %d)", k, t.K);
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  uint32_t be[2];
  HIP_TRY(c, hipMemcpy(be, t.begin + k, sizeof(be), hipMemcpyDeviceToHost));
  int64_t cnt = be[1] - be[0];
  if (m) *m = cnt;
  std::vector<uint32_t> e(cnt);
  if (cnt > 0) HIP_TRY(c, hipMemcpy(e.data(), t.entries + be[0], sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < cnt && i < cap; ++i) {
    if (off) {
      off[3 * i] = entry_x(e[i]);
      off[3 * i + 1] = entry_y(e[i]);
      off[3 * i + 2] = entry_z(e[i]);
    }
    if (cls) cls[i] = (uint8_t)entry_cls(e[i]);
  }
  return AF_OK;
}

int af_read_point_debug(af_ctx *c, int32_t tool_id, int64_t first, int64_t count, int32_t *normal,
                        int32_t *has_normal, uint64_t *mask, int64_t *n_written) {
  if (!c) return AF_EINVAL;
  if (tool_id < 0 || tool_id >= c->cfg.max_tools) return fail(c, AF_EINVAL, "bad tool id");
  ToolDev &t = c->tools[tool_id];
  if (!t.entries) return fail(c, AF_ENOTOOL, "tool %d has no kernels", tool_id);
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  int64_t m = std::max<int64_t>(0, std::min<int64_t>(count, c->n_points - first));
  if (n_written) *n_written = m;
  if (m == 0) return AF_OK;
  int32_t mw = (t.K + 63) / 64;
  if (normal)
    HIP_TRY(c, hipMemcpy(normal, c->pts.normal + 3 * first, sizeof(int32_t) * 3 * m, hipMemcpyDeviceToHost));
  if (has_normal)
    HIP_TRY(c, hipMemcpy(has_normal, c->pts.has_normal + first, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  if (mask)
    HIP_TRY(c, hipMemcpy(mask, t.mask + first * mw, sizeof(uint64_t) * mw * m, hipMemcpyDeviceToHost));
  return AF_OK;
}

int af_pca_axes(const int32_t *moments, int64_t n, int64_t *axes, int32_t *has) {
  if (n < 0 || (n > 0 && (!moments || !axes || !has))) return AF_EINVAL;
  if (n == 0) return AF_OK;
  int32_t *dm = nullptr, *dh = nullptr;
  int64_t *da = nullptr;
  hipError_t e = hipMalloc((void **)&dm, sizeof(int32_t) * 10 * n);
  if (e == hipSuccess) e = hipMalloc((void **)&da, sizeof(int64_t) * 3 * n);
  if (e == hipSuccess) e = hipMalloc((void **)&dh, sizeof(int32_t) * n);
  if (e == hipSuccess) e = hipMemcpy(dm, moments, sizeof(int32_t) * 10 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_pca_axes(dm, n, da, dh, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(axes, da, sizeof(int64_t) * 3 * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(has, dh, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
  hipFree(dm);
  hipFree(da);
  hipFree(dh);
  return e == hipSuccess ? AF_OK : AF_EDEVICE;
}

int af_frame_stats_get(af_ctx *c, af_frame_stats *st) {
  if (!c || !st) return AF_EINVAL;
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  FrameCounters h;
  HIP_TRY(c, hipMemcpy(&h, c->counters, sizeof(h), hipMemcpyDeviceToHost));
  st->n_valid = (int64_t)h.n_valid;
  st->n_dropped = (int64_t)h.n_dropped;
  st->n_in = st->n_valid + st->n_dropped;
  for (int i = 0; i < kStatSlots; ++i) {
    h.pairs_applied += h.fold[i][0];
    h.pairs_excluded += h.fold[i][1];
    h.voxels_folded += h.fold[i][2];
  }
  st->pairs_applied = (int64_t)h.pairs_applied;
  st->pairs_excluded = (int64_t)h.pairs_excluded;
  st->band_marks = (int64_t)h.band_marks;
  st->new_points = h.n_new_points;
  st->n_points = c->n_points;
  st->voxels_folded = (int64_t)h.voxels_folded;
  st->n_blocks = c->n_blocks;
  if (c->map.n_free) {   // sliding window: blocks held, not ids ever handed out
    int32_t nf = 0;
    HIP_TRY(c, hipMemcpy(&nf, c->map.n_free, sizeof(int32_t), hipMemcpyDeviceToHost));
    st->n_blocks -= nf;
  }
  st->new_blocks = h.n_new_blocks;
  return AF_OK;
}

int af_score_stats_get(af_ctx *c, int32_t tool_id, af_score_stats *st) {
  if (!c || !st) return AF_EINVAL;
  if (tool_id < 0 || tool_id >= c->cfg.max_tools) return fail(c, AF_EINVAL, "bad tool id");
  ToolDev &t = c->tools[tool_id];
  if (!t.entries) return fail(c, AF_ENOTOOL, "tool %d has no kernels", tool_id);
  int rc = sync_last(c);
  if (rc != AF_OK) return rc;
  std::vector<ScoreCounterBlock> blk(kStatSlots);
  HIP_TRY(c, hipMemcpy(blk.data(), t.counters, sizeof(ScoreCounters), hipMemcpyDeviceToHost));
  ScoreCounterBlock h;
  memset(&h, 0, sizeof(h));
  for (const ScoreCounterBlock &b : blk) {
    h.n_confident += b.n_confident;
    h.n_accessible += b.n_accessible;
    h.n_blocked += b.n_blocked;
    h.n_no_candidate += b.n_no_candidate;
    h.candidate_tests += b.candidate_tests;
    h.canonical_tests += b.canonical_tests;
    h.canonical_lookups += b.canonical_lookups;
    h.deep_tests += b.deep_tests;
    h.deep_chunks_max += b.deep_chunks_max;
    h.coarse_checks += b.coarse_checks;
    h.coarse_clear += b.coarse_clear;
    h.chunks_body += b.chunks_body;
    h.chunks_far += b.chunks_far;
    h.arm_lookups += b.arm_lookups;
  }
  st->n_points = c->n_points;
  st->n_confident = (int64_t)h.n_confident;
  st->n_accessible = (int64_t)h.n_accessible;
  st->n_blocked = (int64_t)h.n_blocked;
  st->n_no_candidate = (int64_t)h.n_no_candidate;
  st->candidate_tests = (int64_t)h.candidate_tests;
  st->canonical_tests = (int64_t)h.canonical_tests;
  st->canonical_lookups = (int64_t)h.canonical_lookups;
  st->deep_tests = (int64_t)h.deep_tests;
  st->deep_chunks_max = (int64_t)h.deep_chunks_max;
  st->coarse_checks = (int64_t)h.coarse_checks;
  st->coarse_clear = (int64_t)h.coarse_clear;
  st->chunks_body = (int64_t)h.chunks_body;
  st->chunks_far = (int64_t)h.chunks_far;
  st->arm_lookups = (int64_t)h.arm_lookups;
  return AF_OK;
}

}  // extern "C"
