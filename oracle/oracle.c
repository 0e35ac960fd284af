/*
 * Accessibility-field CPU ORACLE -- test infrastructure only (see oracle.h).
 *
 * Plain single-threaded C, fp64 where floating point is involved, built with
 * -O2 -fno-fast-math -ffp-contract=off.  Every voxel lives in one hash map
 * keyed by its packed index; nothing is blocked, tiled or reordered.
 *
 * Fixed point.  Positions are integers in units u = v/256 (P = rint(x*256/v),
 * round-half-even on the fp64 product).  Voxel i spans [256 i, 256 i + 256)
 * and its centre is C(i) = 256 i + 128.  Signed distances are integers in the
 * same unit, and a voxel keeps the integer sums S = sum of clamped distances
 * and W = number of contributions, so the TSDF value S/W of Section 3.2 is
 * exact and independent of the order in which returns are applied.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KEY_BIAS (1LL << 20)
#define KEY_MASK ((1LL << 21) - 1)
#define COORD_LIM ((1LL << 28) - 4096)
#define MAX_TOOLS 16
#define MAX_VP 8

enum { CLS_BODY = 0, CLS_NEAR = 1, CLS_FAR = 2 };
enum { LBL_UNSCORED = 0, LBL_ACCESSIBLE = 1, LBL_BLOCKED = 2, LBL_NOCAND = 3 };

/* ---------------------------------------------------------------- helpers */
int64_t orc_floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
  return q;
}

/* Exact floor square root. */
int64_t orc_isqrt(int64_t n) {
  if (n <= 0) return 0;
  int64_t r = (int64_t)sqrt((double)n);
  while (r > 0 && (__int128)r * r > n) r -= 1;
  while ((__int128)(r + 1) * (r + 1) <= n) r += 1;
  return r;
}

int64_t orc_key(int64_t x, int64_t y, int64_t z) {
  return ((x + KEY_BIAS) & KEY_MASK) | (((y + KEY_BIAS) & KEY_MASK) << 21) |
         (((z + KEY_BIAS) & KEY_MASK) << 42);
}

void orc_unkey(int64_t key, int64_t out[3]) {
  out[0] = (key & KEY_MASK) - KEY_BIAS;
  out[1] = ((key >> 21) & KEY_MASK) - KEY_BIAS;
  out[2] = ((key >> 42) & KEY_MASK) - KEY_BIAS;
}

/* ------------------------------------------------- int64 -> int64 hash map */
typedef struct {
  int64_t *keys, *vals;
  int64_t cap, n;
} hmap;

static uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

static void hm_init(hmap *h, int64_t cap) {
  h->cap = cap;
  h->n = 0;
  h->keys = (int64_t *)malloc(sizeof(int64_t) * cap);
  h->vals = (int64_t *)malloc(sizeof(int64_t) * cap);
  for (int64_t i = 0; i < cap; ++i) h->keys[i] = -1;
}

static void hm_free(hmap *h) {
  free(h->keys);
  free(h->vals);
}

static int64_t hm_get(const hmap *h, int64_t key) {
  int64_t i = (int64_t)(mix64((uint64_t)key) & (uint64_t)(h->cap - 1));
  for (;;) {
    if (h->keys[i] == key) return h->vals[i];
    if (h->keys[i] == -1) return -1;
    i = (i + 1) & (h->cap - 1);
  }
}

static void hm_put(hmap *h, int64_t key, int64_t val);

static void hm_grow(hmap *h) {
  hmap g;
  hm_init(&g, h->cap * 2);
  for (int64_t i = 0; i < h->cap; ++i)
    if (h->keys[i] != -1) hm_put(&g, h->keys[i], h->vals[i]);
  hm_free(h);
  *h = g;
}

static void hm_put(hmap *h, int64_t key, int64_t val) {
  if (2 * (h->n + 1) > h->cap) hm_grow(h);
  int64_t i = (int64_t)(mix64((uint64_t)key) & (uint64_t)(h->cap - 1));
  for (;;) {
    if (h->keys[i] == key) {
      h->vals[i] = val;
      return;
    }
    if (h->keys[i] == -1) {
      h->keys[i] = key;
      h->vals[i] = val;
      h->n += 1;
      return;
    }
    i = (i + 1) & (h->cap - 1);
  }
}

static void *grow_array(void *p, int64_t elem, int64_t *cap, int64_t need) {
  if (need <= *cap) return p;
  int64_t c = *cap ? *cap : 1024;
  while (c < need) c *= 2;
  p = realloc(p, (size_t)(elem * c));
  memset((char *)p + elem * (*cap), 0, (size_t)(elem * (c - *cap)));
  *cap = c;
  return p;
}

/* ------------------------------------------------------------ the oracle */
typedef struct {
  int32_t K;
  int64_t *begin;   /* K+1 prefix offsets into off/cls */
  int32_t *off;     /* [m][3] */
  uint8_t *cls;
  double *rot;      /* K x 9 */
} tool_tab;

struct orc {
  orc_config cfg;
  double scale, tau;
  int64_t tau_u, R, rc_u, dmin_u;
  int roi;
  int64_t roi_lo[3], roi_hi[3];
  /* sliding window (Section 3.3): L blocks per axis, centred (in voxels) on
   * the sensor of the frame that last shifted it; blocks [lo, hi] */
  int win_on, win_set;
  int64_t win_L[3], win_c[3], win_lo[3], win_hi[3], win_shifts;
  int64_t last_frame_id;
  /* voxels */
  hmap vmap;
  int64_t nv, vcap;
  int64_t *vkey, *S, *dS;
  int32_t *W, *dW;
  uint8_t *clr;
  int64_t *dirty, ndirty, dcap;
  int64_t *changed, nchanged, ccap;   /* keys of the voxels folded by the last frame */
  /* surface points, canonical order */
  hmap pmap;
  int64_t np, pcap;
  int64_t *pkey, *sumq;
  int32_t *first_frame, *nvp, *vphead, *vp, *nq, *last_frame;
  /* tools */
  tool_tab tools[MAX_TOOLS];
  /* last score results, by point index */
  int64_t rcap;
  uint8_t *label;
  int32_t *first_free, *has_normal;
  int64_t *normal;
  uint64_t *mask;
  int32_t mask_words;
  orc_frame_stats fst;
  orc_score_stats sst;
};

static int in_roi(const orc_t *o, int64_t x, int64_t y, int64_t z) {
  if (!o->roi) return 1;
  return x >= o->roi_lo[0] && x <= o->roi_hi[0] && y >= o->roi_lo[1] &&
         y <= o->roi_hi[1] && z >= o->roi_lo[2] && z <= o->roi_hi[2];
}

/* Whether voxel x lies in the sliding window (always, without a window or
 * before its first frame). */
static int in_window(const orc_t *o, int64_t x, int64_t y, int64_t z) {
  if (!o->win_on || !o->win_set) return 1;
  const int64_t v[3] = {x, y, z};
  for (int i = 0; i < 3; ++i) {
    int64_t b = orc_floor_div(v[i], 8);
    if (b < o->win_lo[i] || b > o->win_hi[i]) return 0;
  }
  return 1;
}

/* A voxel the integration may write: inside the region of interest and the
 * window. */
static int in_map(const orc_t *o, int64_t x, int64_t y, int64_t z) {
  return in_roi(o, x, y, z) && in_window(o, x, y, z);
}

orc_t *orc_create(const orc_config *cfg) {
  orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
  o->cfg = *cfg;
  if (o->cfg.n_vp > MAX_VP || o->cfg.n_vp < 1 || cfg->voxel <= 0) {
    free(o);
    return NULL;
  }
  /* Section 3.2: tau = min(4v, 0.1 m) when not given (the text prints max;
   * the voxel-size study of Section 4.1 needs tau to scale with v). */
  o->tau = cfg->trunc > 0 ? cfg->trunc : fmin(4.0 * cfg->voxel, 0.1);
  o->scale = 256.0 / cfg->voxel;
  o->tau_u = llrint(o->tau * o->scale);
  o->R = (o->tau_u + 255) / 256;          /* cube half-width ceil(tau/v) */
  o->rc_u = llrint(cfg->r_c * o->scale);
  o->dmin_u = llrint(cfg->vp_min_dist * o->scale);
  if (o->R < 1 || o->R > 7) {
    free(o);
    return NULL;
  }
  o->last_frame_id = -1;
  hm_init(&o->vmap, 1 << 16);
  hm_init(&o->pmap, 1 << 12);
  return o;
}

void orc_destroy(orc_t *o) {
  if (!o) return;
  hm_free(&o->vmap);
  hm_free(&o->pmap);
  free(o->vkey); free(o->S); free(o->dS); free(o->W); free(o->dW); free(o->clr);
  free(o->dirty);
  free(o->changed);
  free(o->pkey); free(o->sumq); free(o->first_frame); free(o->nvp);
  free(o->vphead); free(o->vp); free(o->nq); free(o->last_frame);
  for (int t = 0; t < MAX_TOOLS; ++t) {
    free(o->tools[t].begin); free(o->tools[t].off); free(o->tools[t].cls);
    free(o->tools[t].rot);
  }
  free(o->label); free(o->first_free); free(o->has_normal); free(o->normal);
  free(o->mask);
  free(o);
}

void orc_set_roi(orc_t *o, const int64_t lo[3], const int64_t hi[3]) {
  o->roi = 1;
  for (int i = 0; i < 3; ++i) {
    o->roi_lo[i] = lo[i];
    o->roi_hi[i] = hi[i];
  }
}

/* Section 3.3 "Sliding-Window TSDF": a box of L[i] blocks (8 voxels) per
 * axis.  At each frame, before integration: on the first frame, and whenever
 * the sensor's voxel is farther than 30 % of the window's size (8 L voxels)
 * from the window's centre along some axis, the window is re-centred on the
 * sensor's voxel c and covers blocks [floor(c/8) - floor(L/2), + L - 1];
 * every voxel outside it is discarded (it reads unknown again).  The frame
 * then writes only voxels inside the window and creates points only there.
 * Points outside keep their records and results and are not scored; the
 * normal's neighbours are the points inside the window.  Set before the
 * first frame (returns -1 otherwise, or for L < 2). */
int orc_set_window(orc_t *o, const int64_t L[3]) {
  if (o->last_frame_id >= 0) return -1;
  for (int i = 0; i < 3; ++i)
    if (L[i] < 2) return -1;
  o->win_on = 1;
  o->win_set = 0;
  o->win_shifts = 0;
  for (int i = 0; i < 3; ++i) o->win_L[i] = L[i];
  return 0;
}

/* Window box (blocks) and the number of shifts so far; returns 0 before the
 * first frame. */
int orc_window(const orc_t *o, int64_t lo[3], int64_t hi[3], int64_t *shifts) {
  for (int i = 0; i < 3; ++i) {
    lo[i] = o->win_lo[i];
    hi[i] = o->win_hi[i];
  }
  *shifts = o->win_shifts;
  return o->win_on && o->win_set;
}

/* Discard every voxel outside the window (arrays compacted, map rebuilt). */
static void evict_outside(orc_t *o) {
  int64_t m = 0;
  for (int64_t i = 0; i < o->nv; ++i) {
    int64_t v[3];
    orc_unkey(o->vkey[i], v);
    if (!in_window(o, v[0], v[1], v[2])) continue;
    o->vkey[m] = o->vkey[i];
    o->S[m] = o->S[i];
    o->dS[m] = o->dS[i];
    o->W[m] = o->W[i];
    o->dW[m] = o->dW[i];
    o->clr[m] = o->clr[i];
    ++m;
  }
  o->nv = m;
  hm_free(&o->vmap);
  hm_init(&o->vmap, 1 << 16);
  for (int64_t i = 0; i < m; ++i) hm_put(&o->vmap, o->vkey[i], i);
}

int orc_params(const orc_t *o, int64_t *tau_u, int64_t *R, int64_t *rc_u,
               int64_t *dmin_u, double *scale) {
  *tau_u = o->tau_u;
  *R = o->R;
  *rc_u = o->rc_u;
  *dmin_u = o->dmin_u;
  *scale = o->scale;
  return 0;
}

/* Voxel record, created on first touch. */
static int64_t voxel_slot(orc_t *o, int64_t key) {
  int64_t i = hm_get(&o->vmap, key);
  if (i >= 0) return i;
  i = o->nv;
  int64_t c = o->vcap;
  o->vkey = (int64_t *)grow_array(o->vkey, sizeof(int64_t), &c, i + 1);
  c = o->vcap;
  o->S = (int64_t *)grow_array(o->S, sizeof(int64_t), &c, i + 1);
  c = o->vcap;
  o->dS = (int64_t *)grow_array(o->dS, sizeof(int64_t), &c, i + 1);
  c = o->vcap;
  o->W = (int32_t *)grow_array(o->W, sizeof(int32_t), &c, i + 1);
  c = o->vcap;
  o->dW = (int32_t *)grow_array(o->dW, sizeof(int32_t), &c, i + 1);
  c = o->vcap;
  o->clr = (uint8_t *)grow_array(o->clr, sizeof(uint8_t), &c, i + 1);
  o->vcap = c;
  /* a slot freed by the window's eviction holds an old record */
  o->vkey[i] = key;
  o->S[i] = o->dS[i] = 0;
  o->W[i] = o->dW[i] = 0;
  o->clr[i] = 0;
  o->nv += 1;
  hm_put(&o->vmap, key, i);
  return i;
}

static void point_arrays(orc_t *o, int64_t need) {
  if (need <= o->pcap) return;
  int64_t c0 = o->pcap, c;
  c = c0; o->pkey = (int64_t *)grow_array(o->pkey, sizeof(int64_t), &c, need);
  c = c0; o->sumq = (int64_t *)grow_array(o->sumq, 3 * sizeof(int64_t), &c, need);
  c = c0; o->first_frame = (int32_t *)grow_array(o->first_frame, sizeof(int32_t), &c, need);
  c = c0; o->nvp = (int32_t *)grow_array(o->nvp, sizeof(int32_t), &c, need);
  c = c0; o->vphead = (int32_t *)grow_array(o->vphead, sizeof(int32_t), &c, need);
  c = c0; o->vp = (int32_t *)grow_array(o->vp, MAX_VP * 3 * sizeof(int32_t), &c, need);
  c = c0; o->nq = (int32_t *)grow_array(o->nq, sizeof(int32_t), &c, need);
  c = c0; o->last_frame = (int32_t *)grow_array(o->last_frame, sizeof(int32_t), &c, need);
  o->pcap = c;
}

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* Whether voxels within reach of return P (fixed point) can lie in the
 * region of interest: Chebyshev distance from P's voxel to the region at
 * most max(R, ceil(2.25 tau / v)) + 2 voxels. */
static int roi_reachable(const orc_t *o, const int64_t P[3]) {
  if (!o->roi) return 1;
  int64_t band = (9 * o->tau_u + 4 * 256 - 1) / (4 * 256);
  int64_t m = (o->R > band ? o->R : band) + 2;
  for (int i = 0; i < 3; ++i) {
    int64_t x = orc_floor_div(P[i], 256);
    if (x < o->roi_lo[i] - m || x > o->roi_hi[i] + m) return 0;
  }
  return 1;
}

/* Fixed-point quantisation: rint of the fp64 product (round half to even). */
static int quantize(double x, double scale, int64_t *out) {
  if (!isfinite(x)) return 0;
  double p = x * scale;
  if (!(fabs(p) <= (double)COORD_LIM)) return 0;
  *out = llrint(p);
  return 1;
}

/* Section 3.2 "Scan-centric integration": every voxel x of the index cube of
 * half-width R = ceil(tau/v) around the return's voxel, except those inside
 * the 18-degree cone behind the return (cos angle(x - p, p - q) > 0.95), gets
 * d = |p - q| - |x - q| clamped to [0, tau], at the voxel centre. */
static void accumulate_cube(orc_t *o, const int64_t P[3], const int64_t Q[3]) {
  int64_t ip[3], b[3];
  for (int i = 0; i < 3; ++i) {
    ip[i] = orc_floor_div(P[i], 256);
    b[i] = P[i] - Q[i];
  }
  int64_t bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  int64_t range_p = orc_isqrt(bb);
  for (int64_t dz = -o->R; dz <= o->R; ++dz)
    for (int64_t dy = -o->R; dy <= o->R; ++dy)
      for (int64_t dx = -o->R; dx <= o->R; ++dx) {
        int64_t x[3] = {ip[0] + dx, ip[1] + dy, ip[2] + dz};
        if (!in_map(o, x[0], x[1], x[2])) continue;
        int64_t c[3], a[3], cq[3];
        for (int i = 0; i < 3; ++i) {
          c[i] = 256 * x[i] + 128;
          a[i] = c[i] - P[i];
          cq[i] = c[i] - Q[i];
        }
        int64_t ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
        int64_t aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
        /* cos > 0.95  <=>  a.b > 0 and 400 (a.b)^2 > 361 |a|^2 |b|^2 */
        if (ab > 0 && (__int128)400 * ab * ab > (__int128)361 * aa * bb) {
          o->fst.pairs_excluded += 1;
          continue;
        }
        int64_t d = range_p - orc_isqrt(cq[0] * cq[0] + cq[1] * cq[1] + cq[2] * cq[2]);
        int64_t lo = o->cfg.clamp_negative ? -o->tau_u : 0;
        if (d < lo) d = lo;
        if (d > o->tau_u) d = o->tau_u;
        int64_t s = voxel_slot(o, orc_key(x[0], x[1], x[2]));
        if (o->dW[s] == 0) {
          int64_t c2 = o->dcap;
          o->dirty = (int64_t *)grow_array(o->dirty, sizeof(int64_t), &c2, o->ndirty + 1);
          o->dcap = c2;
          o->dirty[o->ndirty++] = s;
        }
        o->dS[s] += d;
        o->dW[s] += 1;
        o->fst.pairs_applied += 1;
      }
}

/* a / b rounded to nearest, halves away from zero (b > 0); odd in a, so the
 * band positions turn with the scene under axis flips and permutations. */
static int64_t round_div(int64_t a, int64_t b) {
  int64_t m = a < 0 ? -a : a;
  int64_t q = (2 * m + b) / (2 * b);
  return a < 0 ? -q : q;
}

/* Section 3.4 "Arm path checking": voxels between tau and 2.25 tau back from
 * the return, on its ray towards the sensor, are marked ray-cleared.
 * Samples every v/2 (at the nearest fixed-point position), never past the
 * sensor. */
static void mark_band(orc_t *o, const int64_t P[3], const int64_t Q[3]) {
  int64_t g[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
  int64_t L = orc_isqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  for (int64_t j = 1;; ++j) {
    int64_t lam = o->tau_u + 128 * j;
    if (4 * lam > 9 * o->tau_u || lam >= L) break;
    int64_t x[3];
    for (int i = 0; i < 3; ++i)
      x[i] = orc_floor_div(P[i] + round_div(lam * g[i], L), 256);
    if (!in_map(o, x[0], x[1], x[2])) continue;
    int64_t s = voxel_slot(o, orc_key(x[0], x[1], x[2]));
    o->clr[s] = 1;
    o->fst.band_marks += 1;
  }
}

int orc_integrate_frame(orc_t *o, const float *xyz, int64_t n,
                        const float origin[3], int64_t frame_id) {
  if (frame_id <= o->last_frame_id || n < 0) return -1;
  int64_t Q[3];
  for (int i = 0; i < 3; ++i)
    if (!quantize((double)origin[i], o->scale, &Q[i])) return -1;
  if (o->win_on) {
    int64_t qv[3];
    int shift = !o->win_set;
    for (int i = 0; i < 3; ++i) {
      qv[i] = orc_floor_div(Q[i], 256);
      int64_t d = qv[i] - o->win_c[i];
      if (o->win_set && 10 * (d < 0 ? -d : d) > 3 * 8 * o->win_L[i]) shift = 1;
    }
    if (shift) {
      for (int i = 0; i < 3; ++i) {
        o->win_c[i] = qv[i];
        o->win_lo[i] = orc_floor_div(qv[i], 8) - o->win_L[i] / 2;
        o->win_hi[i] = o->win_lo[i] + o->win_L[i] - 1;
      }
      if (o->win_set) {
        evict_outside(o);
        o->win_shifts += 1;
      }
      o->win_set = 1;
    }
  }
  memset(&o->fst, 0, sizeof(o->fst));
  o->fst.n_in = n;
  int64_t *P = (int64_t *)malloc(sizeof(int64_t) * 3 * (n > 0 ? n : 1));
  uint8_t *ok = (uint8_t *)malloc(n > 0 ? (size_t)n : 1);
  int64_t *fresh = NULL, nfresh = 0, fcap = 0;
  hmap seen;
  hm_init(&seen, 1024);

  for (int64_t r = 0; r < n; ++r) {
    int v = 1;
    for (int i = 0; i < 3; ++i) v &= quantize((double)xyz[3 * r + i], o->scale, &P[3 * r + i]);
    if (v && P[3 * r] == Q[0] && P[3 * r + 1] == Q[1] && P[3 * r + 2] == Q[2]) v = 0;
    ok[r] = (uint8_t)v;
    if (!v) {
      o->fst.n_dropped += 1;
      continue;
    }
    o->fst.n_valid += 1;
    /* With a region of interest, a return whose voxel lies farther from the
     * region than anything it touches (its cube reaches R voxels; its band
     * samples lie within 2.25 tau of it along the ray, plus rounding) cannot
     * change a voxel inside it, and is not expanded. */
    if (!roi_reachable(o, &P[3 * r])) continue;
    accumulate_cube(o, &P[3 * r], Q);
    mark_band(o, &P[3 * r], Q);
    /* Section 3.1: the voxel holding a return becomes a surface point. */
    int64_t ip[3];
    for (int i = 0; i < 3; ++i) ip[i] = orc_floor_div(P[3 * r + i], 256);
    if (!in_map(o, ip[0], ip[1], ip[2])) continue;
    int64_t k = orc_key(ip[0], ip[1], ip[2]);
    if (hm_get(&o->pmap, k) < 0 && hm_get(&seen, k) < 0) {
      hm_put(&seen, k, 1);
      fresh = (int64_t *)grow_array(fresh, sizeof(int64_t), &fcap, nfresh + 1);
      fresh[nfresh++] = k;
    }
  }

  /* Fold the frame: S += dS, W += dW; weights saturate at the cap with
   * proportional rescaling of S (Section 3.6, "TSDF integration"). */
  o->nchanged = 0;
  for (int64_t j = 0; j < o->ndirty; ++j) {
    int64_t s = o->dirty[j];
    o->changed = (int64_t *)grow_array(o->changed, sizeof(int64_t), &o->ccap, o->nchanged + 1);
    o->changed[o->nchanged++] = o->vkey[s];
    o->S[s] += o->dS[s];
    o->W[s] += o->dW[s];
    if (o->W[s] > o->cfg.weight_cap) {
      o->S[s] = orc_floor_div(o->S[s] * o->cfg.weight_cap, o->W[s]);
      o->W[s] = o->cfg.weight_cap;
    }
    o->dS[s] = 0;
    o->dW[s] = 0;
  }
  o->fst.voxels_folded = o->ndirty;
  o->ndirty = 0;

  /* New points of the frame are appended in ascending key order. */
  qsort(fresh, (size_t)nfresh, sizeof(int64_t), cmp_i64);
  point_arrays(o, o->np + nfresh);
  for (int64_t j = 0; j < nfresh; ++j) {
    int64_t p = o->np++;
    o->pkey[p] = fresh[j];
    o->first_frame[p] = (int32_t)frame_id;
    o->nvp[p] = 0;
    o->vphead[p] = 0;
    o->nq[p] = 0;
    o->last_frame[p] = -1;
    for (int i = 0; i < 3; ++i) o->sumq[3 * p + i] = 0;
    hm_put(&o->pmap, fresh[j], p);
  }
  o->fst.new_points = nfresh;
  o->fst.n_points = o->np;

  /* Once per (point, frame): accumulate the sensor position for the normal
   * orientation, and store it as a viewpoint if it moved more than the
   * novelty distance from the last stored one (ring of n_vp). */
  for (int64_t r = 0; r < n; ++r) {
    if (!ok[r]) continue;
    int64_t ip[3];
    for (int i = 0; i < 3; ++i) ip[i] = orc_floor_div(P[3 * r + i], 256);
    if (!in_map(o, ip[0], ip[1], ip[2])) continue;
    int64_t p = hm_get(&o->pmap, orc_key(ip[0], ip[1], ip[2]));
    if (o->last_frame[p] == (int32_t)frame_id) continue;
    o->last_frame[p] = (int32_t)frame_id;
    for (int i = 0; i < 3; ++i) o->sumq[3 * p + i] += Q[i];
    o->nq[p] += 1;
    int store = 1;
    if (o->nvp[p] > 0) {
      int last = (o->vphead[p] + o->cfg.n_vp - 1) % o->cfg.n_vp;
      int64_t d2 = 0;
      for (int i = 0; i < 3; ++i) {
        int64_t d = Q[i] - o->vp[(p * MAX_VP + last) * 3 + i];
        d2 += d * d;
      }
      store = d2 > o->dmin_u * o->dmin_u;
    }
    if (store) {
      for (int i = 0; i < 3; ++i) o->vp[(p * MAX_VP + o->vphead[p]) * 3 + i] = (int32_t)Q[i];
      o->vphead[p] = (o->vphead[p] + 1) % o->cfg.n_vp;
      if (o->nvp[p] < o->cfg.n_vp) o->nvp[p] += 1;
    }
  }
  hm_free(&seen);
  free(fresh);
  free(P);
  free(ok);
  o->last_frame_id = frame_id;
  return 0;
}

int orc_frame_stats_get(const orc_t *o, orc_frame_stats *st) {
  *st = o->fst;
  return 0;
}

int64_t orc_num_voxels(const orc_t *o) { return o->nv; }

int64_t orc_read_tsdf(const orc_t *o, int64_t *key, int64_t *S, int32_t *W,
                      uint8_t *cleared, int64_t cap) {
  int64_t *k = (int64_t *)malloc(sizeof(int64_t) * (o->nv > 0 ? o->nv : 1));
  for (int64_t i = 0; i < o->nv; ++i) k[i] = o->vkey[i];
  qsort(k, (size_t)o->nv, sizeof(int64_t), cmp_i64);
  int64_t m = o->nv < cap ? o->nv : cap;
  for (int64_t i = 0; i < m; ++i) {
    int64_t s = hm_get(&o->vmap, k[i]);
    key[i] = k[i];
    S[i] = o->S[s];
    W[i] = o->W[s];
    cleared[i] = o->clr[s];
  }
  free(k);
  return o->nv;
}

int orc_voxel(const orc_t *o, int64_t key, int64_t *S, int32_t *W,
              uint8_t *cleared) {
  int64_t s = hm_get(&o->vmap, key);
  if (s < 0) {
    *S = 0;
    *W = 0;
    *cleared = 0;
    return 0;
  }
  *S = o->S[s];
  *W = o->W[s];
  *cleared = o->clr[s];
  return 1;
}

int64_t orc_num_points(const orc_t *o) { return o->np; }

int64_t orc_read_points(const orc_t *o, int64_t *key, int32_t *first_frame,
                        int32_t *n_vp, int32_t *vp, int64_t *sumq, int32_t *nq,
                        int64_t cap) {
  int64_t m = o->np < cap ? o->np : cap;
  for (int64_t p = 0; p < m; ++p) {
    key[p] = o->pkey[p];
    first_frame[p] = o->first_frame[p];
    n_vp[p] = o->nvp[p];
    nq[p] = o->nq[p];
    /* viewpoints oldest first */
    int cnt = o->nvp[p];
    int start = (o->vphead[p] - cnt + o->cfg.n_vp) % o->cfg.n_vp;
    for (int j = 0; j < MAX_VP; ++j)
      for (int i = 0; i < 3; ++i)
        vp[(p * MAX_VP + j) * 3 + i] =
            j < cnt ? o->vp[(p * MAX_VP + (start + j) % o->cfg.n_vp) * 3 + i] : 0;
    for (int i = 0; i < 3; ++i) sumq[3 * p + i] = o->sumq[3 * p + i];
  }
  return o->np;
}

/* ------------------------------------------------------- tool kernel table */
typedef struct {
  int64_t n2;
  int32_t o[3];
} ent;

static int cmp_ent(const void *a, const void *b) {
  const ent *x = (const ent *)a, *y = (const ent *)b;
  if (x->n2 != y->n2) return x->n2 < y->n2 ? -1 : 1;
  for (int i = 2; i >= 0; --i)
    if (x->o[i] != y->o[i]) return x->o[i] < y->o[i] ? -1 : 1;
  return 0;
}

/* Section 3.4 "Tool kernel" / "Self-exclusion" / "Arm path checking": the
 * rotated tool is a set of voxel offsets from the point's voxel.  BODY holds
 * offsets whose centre lies in the rotated tool solid (0 <= x <= length),
 * FAR those in its corridor (length < x <= length + corridor), both minus the
 * self-exclusion ball of radius r_s around the tip; NEAR holds the three arm
 * samples at 0.6, 1.25 and 2.25 times tau along the approach axis.  Membership is
 * decided in fp64 in voxel units with a 1e-9 tolerance on the inclusive
 * bounds. */
static int build_orientation(const orc_tool *t, double v, double tau,
                             const double *R, ent **body, int64_t *nb,
                             ent **far_, int64_t *nf, int32_t near[3][3]) {
  const double eps = 1e-9;
  double Lv = t->length / v;
  double Ev = (t->length + t->corridor) / v;
  double a, b;
  if (t->shape == 0) {
    a = t->radius / v;
    b = a;
  } else {
    a = (0.5 * t->width) / v;
    b = (0.5 * t->height) / v;
  }
  double rv2 = a * a;
  double rsv = t->r_s / v;
  double rsv2 = rsv * rsv;
  double fr[3] = {0.6, 1.25, 2.25};
  for (int j = 0; j < 3; ++j) {
    double lam = (fr[j] * tau) / v;
    for (int i = 0; i < 3; ++i) near[j][i] = (int32_t)round(lam * R[3 * i]);
  }
  int64_t lo[3], hi[3];
  for (int i = 0; i < 3; ++i) {
    double mn = INFINITY, mx = -INFINITY;
    for (int cx = 0; cx < 2; ++cx)
      for (int cy = 0; cy < 2; ++cy)
        for (int cz = 0; cz < 2; ++cz) {
          double x = cx ? Ev : 0.0, y = cy ? a : -a, z = cz ? b : -b;
          double w = R[3 * i] * x + R[3 * i + 1] * y + R[3 * i + 2] * z;
          if (w < mn) mn = w;
          if (w > mx) mx = w;
        }
    lo[i] = (int64_t)floor(mn) - 1;
    hi[i] = (int64_t)ceil(mx) + 1;
  }
  int64_t cb = 0, cf = 0;
  *nb = 0;
  *nf = 0;
  *body = NULL;
  *far_ = NULL;
  for (int64_t oz = lo[2]; oz <= hi[2]; ++oz)
    for (int64_t oy = lo[1]; oy <= hi[1]; ++oy)
      for (int64_t ox = lo[0]; ox <= hi[0]; ++ox) {
        double fx = (double)ox, fy = (double)oy, fz = (double)oz;
        double x = (R[0] * fx + R[3] * fy) + R[6] * fz;
        double y = (R[1] * fx + R[4] * fy) + R[7] * fz;
        double z = (R[2] * fx + R[5] * fy) + R[8] * fz;
        int cross;
        if (t->shape == 0)
          cross = (y * y + z * z) <= rv2 + eps;
        else
          cross = fabs(y) <= a + eps && fabs(z) <= b + eps;
        if (!cross) continue;
        int64_t n2 = ox * ox + oy * oy + oz * oz;
        if ((double)n2 < rsv2) continue;
        if (x < -eps || x > Ev + eps) continue;
        if (ox < -511 || ox > 511 || oy < -511 || oy > 511 || oz < -511 || oz > 511)
          return -1;
        ent e = {n2, {(int32_t)ox, (int32_t)oy, (int32_t)oz}};
        if (x <= Lv + eps) {
          *body = (ent *)grow_array(*body, sizeof(ent), &cb, *nb + 1);
          (*body)[(*nb)++] = e;
        } else {
          *far_ = (ent *)grow_array(*far_, sizeof(ent), &cf, *nf + 1);
          (*far_)[(*nf)++] = e;
        }
      }
  qsort(*body, (size_t)*nb, sizeof(ent), cmp_ent);
  qsort(*far_, (size_t)*nf, sizeof(ent), cmp_ent);
  return 0;
}

int orc_set_tool(orc_t *o, int tool_id, const orc_tool *t, int32_t K,
                 const double *rot) {
  if (tool_id < 0 || tool_id >= MAX_TOOLS || K <= 0) return -1;
  tool_tab *tt = &o->tools[tool_id];
  free(tt->begin); free(tt->off); free(tt->cls); free(tt->rot);
  memset(tt, 0, sizeof(*tt));
  tt->K = K;
  tt->rot = (double *)malloc(sizeof(double) * 9 * K);
  memcpy(tt->rot, rot, sizeof(double) * 9 * K);
  tt->begin = (int64_t *)malloc(sizeof(int64_t) * (K + 1));
  int64_t cap = 0, m = 0;
  int64_t ccap = 0;
  tt->begin[0] = 0;
  for (int32_t k = 0; k < K; ++k) {
    ent *body, *far_;
    int64_t nb, nf;
    int32_t near[3][3];
    if (build_orientation(t, o->cfg.voxel, o->tau, rot + 9 * k, &body, &nb, &far_, &nf,
                          near) != 0)
      return -1;
    int64_t need = m + 3 + nb + nf;
    int64_t c0 = cap;
    tt->off = (int32_t *)grow_array(tt->off, 3 * sizeof(int32_t), &c0, need);
    tt->cls = (uint8_t *)grow_array(tt->cls, 1, &ccap, need);
    cap = c0;
    for (int j = 0; j < 3; ++j) {
      for (int i = 0; i < 3; ++i) tt->off[3 * m + i] = near[j][i];
      tt->cls[m++] = CLS_NEAR;
    }
    for (int64_t j = 0; j < nb; ++j) {
      for (int i = 0; i < 3; ++i) tt->off[3 * m + i] = body[j].o[i];
      tt->cls[m++] = CLS_BODY;
    }
    for (int64_t j = 0; j < nf; ++j) {
      for (int i = 0; i < 3; ++i) tt->off[3 * m + i] = far_[j].o[i];
      tt->cls[m++] = CLS_FAR;
    }
    tt->begin[k + 1] = m;
    free(body);
    free(far_);
  }
  return 0;
}

/* Section 3.4 "Tool kernel": a tool given as a caller-built table of voxel
 * offsets (for a tool that is not a primitive, e.g. a point cloud sampled
 * from its 3D model and voxelised under each orientation).  Orientation k
 * has approach direction dir[k] (used by the candidate filters) and the
 * entries [begin[k], begin[k+1]) of off/cls.  They are kept in the order the
 * scoring visits them: the three arm samples (NEAR) in the given order, then
 * the BODY offsets and then the FAR offsets, each sorted by
 * (|o|^2, z, y, x).  Returns -1 (tool unchanged) for K < 1, a direction whose
 * length is off 1 by more than 1e-9, a non-monotone begin, a class outside
 * 0..2, other than three NEAR entries, an offset component beyond 511 voxels
 * or an offset listed twice in one class. */
int orc_set_tool_table(orc_t *o, int tool_id, int32_t K, const double *dir,
                       const uint32_t *begin, const int16_t *off, const uint8_t *cls) {
  if (tool_id < 0 || tool_id >= MAX_TOOLS || K <= 0 || begin[0] != 0) return -1;
  for (int32_t k = 0; k < K; ++k) {
    const double *d = dir + 3 * k;
    if (!(fabs(sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - 1.0) <= 1e-9)) return -1;
    if (begin[k + 1] < begin[k]) return -1;
  }
  int64_t n = begin[K];
  int32_t *toff = (int32_t *)malloc(sizeof(int32_t) * 3 * (n > 0 ? n : 1));
  uint8_t *tcls = (uint8_t *)malloc(n > 0 ? n : 1);
  int64_t *tbeg = (int64_t *)malloc(sizeof(int64_t) * (K + 1));
  ent *grp = (ent *)malloc(sizeof(ent) * (n > 0 ? n : 1));
  int64_t m = 0;
  int ok = 1;
  tbeg[0] = 0;
  for (int32_t k = 0; k < K && ok; ++k) {
    int nnear = 0;
    for (uint32_t e = begin[k]; e < begin[k + 1] && ok; ++e) {
      if (cls[e] > CLS_FAR) ok = 0;
      for (int i = 0; i < 3; ++i)
        if (off[3 * e + i] < -511 || off[3 * e + i] > 511) ok = 0;
      if (ok && cls[e] == CLS_NEAR) {
        if (++nnear > 3) ok = 0;
        for (int i = 0; i < 3; ++i) toff[3 * m + i] = off[3 * e + i];
        tcls[m++] = CLS_NEAR;
      }
    }
    if (nnear != 3) ok = 0;
    const uint8_t order[2] = {CLS_BODY, CLS_FAR};
    for (int g = 0; g < 2 && ok; ++g) {
      int64_t ng = 0;
      for (uint32_t e = begin[k]; e < begin[k + 1]; ++e) {
        if (cls[e] != order[g]) continue;
        ent x;
        for (int i = 0; i < 3; ++i) x.o[i] = off[3 * e + i];
        x.n2 = (int64_t)x.o[0] * x.o[0] + (int64_t)x.o[1] * x.o[1] + (int64_t)x.o[2] * x.o[2];
        grp[ng++] = x;
      }
      qsort(grp, (size_t)ng, sizeof(ent), cmp_ent);
      for (int64_t j = 0; j < ng; ++j) {
        if (j > 0 && cmp_ent(&grp[j - 1], &grp[j]) == 0) ok = 0;
        for (int i = 0; i < 3; ++i) toff[3 * m + i] = grp[j].o[i];
        tcls[m++] = order[g];
      }
    }
    tbeg[k + 1] = m;
  }
  free(grp);
  if (!ok) {
    free(toff); free(tcls); free(tbeg);
    return -1;
  }
  tool_tab *tt = &o->tools[tool_id];
  free(tt->begin); free(tt->off); free(tt->cls); free(tt->rot);
  memset(tt, 0, sizeof(*tt));
  tt->K = K;
  tt->begin = tbeg;
  tt->off = toff;
  tt->cls = tcls;
  /* the candidate filters read the approach direction as column 0 */
  tt->rot = (double *)calloc(9 * (size_t)K, sizeof(double));
  for (int32_t k = 0; k < K; ++k)
    for (int i = 0; i < 3; ++i) tt->rot[9 * k + 3 * i] = dir[3 * k + i];
  return 0;
}

int64_t orc_tool_table(const orc_t *o, int tool_id, int32_t k, int32_t *off,
                       uint8_t *cls, int64_t cap) {
  if (tool_id < 0 || tool_id >= MAX_TOOLS) return -1;
  const tool_tab *tt = &o->tools[tool_id];
  if (tt->K <= 0 || k < 0 || k >= tt->K) return -1;
  int64_t b = tt->begin[k], m = tt->begin[k + 1] - b;
  for (int64_t j = 0; j < m && j < cap; ++j) {
    for (int i = 0; i < 3; ++i) off[3 * j + i] = tt->off[3 * (b + j) + i];
    cls[j] = tt->cls[b + j];
  }
  return m;
}

/* ---------------------------------------------------------------- scoring */
typedef struct {
  int64_t S;
  int32_t W;
  uint8_t clr;
} vrec;

static vrec lookup(const orc_t *o, int64_t x, int64_t y, int64_t z) {
  vrec r = {0, 0, 0};
  int64_t s = hm_get(&o->vmap, orc_key(x, y, z));
  if (s >= 0) {
    r.S = o->S[s];
    r.W = o->W[s];
    r.clr = o->clr[s];
  }
  return r;
}

static int nb_cmp(const void *a, const void *b) {
  const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
  int32_t nx = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  int32_t ny = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
  if (nx != ny) return nx < ny ? -1 : 1;
  for (int i = 2; i >= 0; --i)
    if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
  return 0;
}

/* Section 3.4 "Approach directions": the normal is the least principal axis
 * (PCA) of the k nearest surface voxels, oriented towards the mean of the
 * sensor positions recorded for the point.
 *
 * Neighbours: surface voxels within +-3 voxels of the point, the point itself
 * included, nearest first; voxels at equal distance are taken in ascending
 * (dz, dy, dx) order, and the walk stops at exactly k.  The scatter
 * M = n sum(dd^T) - (sum d)(sum d)^T (n^2 times the covariance) is exact in
 * int64 and converted exactly to double.
 *
 * Eigen-decomposition: cyclic Jacobi (Golub & Van Loan, "Matrix
 * Computations", the cyclic Jacobi method built on the 2x2 symmetric Schur
 * decomposition).  Eight sweeps over the pairs (0,1), (0,2), (1,2); a pair
 * whose off-diagonal entry is exactly zero is skipped.  For a pair (p, q):
 *   theta = (a_qq - a_pp) / (2 a_pq)
 *   t = sign(theta) / (|theta| + sqrt(theta^2 + 1)),  sign(0) = +1
 *   c = 1 / sqrt(t^2 + 1),  s = t c
 *   a_pp -= t a_pq,  a_qq += t a_pq,  a_pq = a_qp = 0
 *   for the third index r: a_rp <- c a_rp - s a_rq,  a_rq <- s a_rp + c a_rq
 *   for every row i of V:  v_ip <- c v_ip - s v_iq,  v_iq <- s v_ip + c v_iq
 * The axis is the column of V at the smallest diagonal entry (ties: lowest
 * index), stored in fixed point as llrint(2^30 v) per component.  Every
 * operation is an IEEE basic operation (+, -, *, /, sqrt) with contraction
 * off, written in this order.  Returns 0 with fewer than 3 neighbours. */
int orc_pca_axis(int64_t cnt, const int64_t sx[3], const int64_t sxx[6], int64_t out[3]) {
  out[0] = out[1] = out[2] = 0;
  if (cnt < 3) return 0;
  /* sxx: 00 01 02 11 12 22 */
  const int64_t m00 = cnt * sxx[0] - sx[0] * sx[0], m01 = cnt * sxx[1] - sx[0] * sx[1];
  const int64_t m02 = cnt * sxx[2] - sx[0] * sx[2], m11 = cnt * sxx[3] - sx[1] * sx[1];
  const int64_t m12 = cnt * sxx[4] - sx[1] * sx[2], m22 = cnt * sxx[5] - sx[2] * sx[2];
  double a[3][3] = {{(double)m00, (double)m01, (double)m02},
                    {(double)m01, (double)m11, (double)m12},
                    {(double)m02, (double)m12, (double)m22}};
  double v[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  static const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int sweep = 0; sweep < 8; ++sweep)
    for (int k = 0; k < 3; ++k) {
      const int p = pairs[k][0], q = pairs[k][1], r = 3 - p - q;
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
      double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
      if (theta < 0.0) t = -t;
      const double c = 1.0 / sqrt(t * t + 1.0);
      const double s = t * c;
      a[p][p] = a[p][p] - t * apq;
      a[q][q] = a[q][q] + t * apq;
      a[p][q] = a[q][p] = 0.0;
      const double arp = a[r][p], arq = a[r][q];
      a[r][p] = a[p][r] = c * arp - s * arq;
      a[r][q] = a[q][r] = s * arp + c * arq;
      for (int i = 0; i < 3; ++i) {
        const double vip = v[i][p], viq = v[i][q];
        v[i][p] = c * vip - s * viq;
        v[i][q] = s * vip + c * viq;
      }
    }
  int best = 0;
  for (int j = 1; j < 3; ++j)
    if (a[j][j] < a[best][best]) best = j;
  for (int i = 0; i < 3; ++i) out[i] = llrint(v[i][best] * 1073741824.0);
  return 1;
}

/* orc_pca_axis over n moment rows [n][10] (cnt, sum d [3], sum dd^T [6]). */
void orc_pca_axes(const int32_t *mom, int64_t n, int64_t *axes, int32_t *has) {
  for (int64_t i = 0; i < n; ++i) {
    const int32_t *m = mom + 10 * i;
    const int64_t sx[3] = {m[1], m[2], m[3]};
    const int64_t sxx[6] = {m[4], m[5], m[6], m[7], m[8], m[9]};
    has[i] = orc_pca_axis(m[0], sx, sxx, axes + 3 * i);
  }
}

static int point_normal(const orc_t *o, int64_t p, const int32_t *nbo, int nnb,
                        int64_t n_out[3]) {
  int64_t s[3];
  orc_unkey(o->pkey[p], s);
  int64_t sx[3] = {0, 0, 0}, sxx[6] = {0, 0, 0, 0, 0, 0};
  int64_t cnt = 0;
  for (int j = 0; j < nnb && cnt < o->cfg.knn_k; ++j) {
    const int32_t *d = nbo + 3 * j;
    if (hm_get(&o->pmap, orc_key(s[0] + d[0], s[1] + d[1], s[2] + d[2])) < 0) continue;
    if (!in_window(o, s[0] + d[0], s[1] + d[1], s[2] + d[2])) continue;
    cnt++;
    for (int a = 0; a < 3; ++a) sx[a] += d[a];
    sxx[0] += (int64_t)d[0] * d[0];
    sxx[1] += (int64_t)d[0] * d[1];
    sxx[2] += (int64_t)d[0] * d[2];
    sxx[3] += (int64_t)d[1] * d[1];
    sxx[4] += (int64_t)d[1] * d[2];
    sxx[5] += (int64_t)d[2] * d[2];
  }
  if (!orc_pca_axis(cnt, sx, sxx, n_out)) return 0;
  /* orientation: towards the mean sensor position, sum(q) / n_q, compared
   * exactly as n . (sum(q) - n_q c(s)) (a zero product keeps the sign) */
  __int128 g = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t ga = o->sumq[3 * p + a] - (int64_t)o->nq[p] * (256 * s[a] + 128);
    g += (__int128)n_out[a] * ga;
  }
  if (g < 0)
    for (int a = 0; a < 3; ++a) n_out[a] = -n_out[a];
  return 1;
}

/* Candidate filters of Section 3.4 for approach direction d (column 0 of the
 * orientation): inside the 70-degree cone around the outward normal (n.d >= cos70 |n|)
 * and seen from that side by at least one stored viewpoint V
 * ((V - s).d > 0.25 |V - s|).  Both tests are squared to avoid square roots. */
static int candidate(const orc_t *o, int64_t p, const int64_t s[3],
                     const int64_t n[3], int has_n, const double *R) {
  double d[3] = {R[0], R[3], R[6]};
  if (has_n) {
    double dot = ((double)n[0] * d[0] + (double)n[1] * d[1]) + (double)n[2] * d[2];
    double nn = (double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double c2 = o->cfg.cos_normal * o->cfg.cos_normal;
    if (!(dot >= 0.0 && dot * dot >= c2 * nn)) return 0;
  }
  int cnt = o->nvp[p];
  double o2 = o->cfg.obs_dot * o->cfg.obs_dot;
  for (int j = 0; j < cnt; ++j) {
    int64_t w[3];
    for (int i = 0; i < 3; ++i) w[i] = (int64_t)o->vp[(p * MAX_VP + j) * 3 + i] - (256 * s[i] + 128);
    double wd = ((double)w[0] * d[0] + (double)w[1] * d[1]) + (double)w[2] * d[2];
    double ww = (double)(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (wd > 0.0 && wd * wd > o2 * ww) return 1;
  }
  return 0;
}

/* Section 3.4: one orientation is free when none of its arm samples hits
 * (TSDF < r_c, or unknown and not ray-cleared), fewer than n_c body voxels
 * have TSDF < r_c, and no corridor voxel has TSDF < r_c.  Unknown voxels read
 * as free for the body and the corridor.  Entries are visited in table order
 * (arm samples, body, corridor) and the visit stops at the deciding hit; the
 * number of visited entries is the canonical lookup count. */
static int orientation_free(const orc_t *o, const tool_tab *tt, int32_t k,
                            const int64_t s[3], int64_t *lookups) {
  int body = 0;
  for (int64_t e = tt->begin[k]; e < tt->begin[k + 1]; ++e) {
    *lookups += 1;
    const int32_t *d = tt->off + 3 * e;
    vrec r = lookup(o, s[0] + d[0], s[1] + d[1], s[2] + d[2]);
    int occ = r.W > 0 && r.S < o->rc_u * (int64_t)r.W;
    if (tt->cls[e] == CLS_NEAR) {
      if (occ || (r.W == 0 && !r.clr)) return 0;
    } else if (tt->cls[e] == CLS_BODY) {
      if (occ && ++body >= o->cfg.n_c) return 0;
    } else {
      if (occ) return 0;
    }
  }
  return 1;
}

static int score_impl(orc_t *o, int tool_id, const int64_t *keys, int64_t n_keys,
                      const uint64_t *allow);

int orc_score(orc_t *o, int tool_id, const int64_t *keys, int64_t n_keys) {
  return score_impl(o, tool_id, keys, n_keys, NULL);
}

/* orc_score restricted to the allowed orientations of each listed point:
 * allow holds ceil(K/64) words per key; an orientation is a candidate only
 * when it passes the filters of Section 3.4 and its allow bit is set (the
 * coarse-to-fine direction search of Section 3.6 narrows the search this
 * way). */
int orc_score_allow(orc_t *o, int tool_id, const int64_t *keys, int64_t n_keys,
                    const uint64_t *allow) {
  if (!keys || !allow) return -1;
  return score_impl(o, tool_id, keys, n_keys, allow);
}

static int score_impl(orc_t *o, int tool_id, const int64_t *keys, int64_t n_keys,
                      const uint64_t *allow) {
  if (tool_id < 0 || tool_id >= MAX_TOOLS) return -1;
  const tool_tab *tt = &o->tools[tool_id];
  if (tt->K <= 0) return -4;
  int32_t K = tt->K;
  int32_t mw = (K + 63) / 64;
  if (o->mask_words != mw) {
    free(o->label); free(o->first_free); free(o->has_normal); free(o->normal);
    free(o->mask);
    o->label = NULL; o->first_free = NULL; o->has_normal = NULL; o->normal = NULL;
    o->mask = NULL;
    o->rcap = 0;
    o->mask_words = mw;
  }
  if (o->rcap < o->np) {
    /* grow, keeping earlier results (a window keeps those of points outside) */
    int64_t c0 = o->rcap, c;
    int64_t need = o->np > 0 ? o->np : 1;
    c = c0; o->label = (uint8_t *)grow_array(o->label, 1, &c, need);
    c = c0; o->first_free = (int32_t *)grow_array(o->first_free, sizeof(int32_t), &c, need);
    c = c0; o->has_normal = (int32_t *)grow_array(o->has_normal, sizeof(int32_t), &c, need);
    c = c0; o->normal = (int64_t *)grow_array(o->normal, 3 * sizeof(int64_t), &c, need);
    c = c0; o->mask = (uint64_t *)grow_array(o->mask, (int64_t)mw * sizeof(uint64_t), &c, need);
    for (int64_t p = c0; p < c; ++p) {
      o->label[p] = 255; /* not evaluated */
      o->first_free[p] = -1;
    }
    o->rcap = c;
  }
  if (!o->win_on)
    for (int64_t p = 0; p < o->np; ++p) {
      o->label[p] = 255; /* not evaluated */
      o->first_free[p] = -1;
    }
  memset(&o->sst, 0, sizeof(o->sst));
  o->sst.n_points = o->np;
  /* neighbour offsets, nearest first */
  int32_t nbo[343 * 3];
  int nnb = 0;
  for (int z = -3; z <= 3; ++z)
    for (int y = -3; y <= 3; ++y)
      for (int x = -3; x <= 3; ++x) {
        nbo[3 * nnb] = x;
        nbo[3 * nnb + 1] = y;
        nbo[3 * nnb + 2] = z;
        nnb++;
      }
  qsort(nbo, (size_t)nnb, 3 * sizeof(int32_t), nb_cmp);

  int64_t count = keys ? n_keys : o->np;
  for (int64_t j = 0; j < count; ++j) {
    int64_t p = keys ? hm_get(&o->pmap, keys[j]) : j;
    if (p < 0) continue;
    int64_t s[3];
    orc_unkey(o->pkey[p], s);
    /* with a window, every-point scoring skips the points outside it (their
     * results stay as they were) */
    if (!keys && !in_window(o, s[0], s[1], s[2])) continue;
    vrec self = lookup(o, s[0], s[1], s[2]);
    o->first_free[p] = -1;
    o->has_normal[p] = 0;
    for (int i = 0; i < 3; ++i) o->normal[3 * p + i] = 0;
    for (int w = 0; w < mw; ++w) o->mask[p * mw + w] = 0;
    /* Section 3.5: confidence c = w / (w + 5) < 0.2 (i.e. W < 2) is skipped */
    if (self.W < o->cfg.conf_min_w) {
      o->label[p] = LBL_UNSCORED;
      continue;
    }
    o->sst.n_confident++;
    int64_t n[3] = {0, 0, 0};
    int hn = point_normal(o, p, nbo, nnb, n);
    o->has_normal[p] = hn;
    for (int i = 0; i < 3; ++i) o->normal[3 * p + i] = n[i];
    int any = 0;
    for (int32_t k = 0; k < K; ++k)
      if ((!allow || ((allow[j * mw + k / 64] >> (k % 64)) & 1)) &&
          candidate(o, p, s, n, hn, tt->rot + 9 * k)) {
        o->mask[p * mw + k / 64] |= 1ULL << (k % 64);
        any = 1;
        o->sst.candidate_tests++;
      }
    if (!any) {
      o->label[p] = LBL_NOCAND;
      o->sst.n_no_candidate++;
      continue;
    }
    o->label[p] = LBL_BLOCKED;
    for (int32_t k = 0; k < K; ++k) {
      if (!((o->mask[p * mw + k / 64] >> (k % 64)) & 1)) continue;
      o->sst.canonical_tests++;
      if (orientation_free(o, tt, k, s, &o->sst.canonical_lookups)) {
        o->label[p] = LBL_ACCESSIBLE;
        o->first_free[p] = k;
        break;
      }
    }
    if (o->label[p] == LBL_ACCESSIBLE)
      o->sst.n_accessible++;
    else
      o->sst.n_blocked++;
  }
  return 0;
}

/* Keys of the voxels that received a contribution in the last frame (in
 * fold order); returns their number. */
int64_t orc_changed_voxels(const orc_t *o, int64_t *keys, int64_t cap) {
  int64_t m = o->nchanged < cap ? o->nchanged : cap;
  for (int64_t j = 0; j < m; ++j) keys[j] = o->changed[j];
  return o->nchanged;
}

/* Number of body voxels of orientation k with TSDF < r_c at point `key`
 * (the raw collision count of Section 3.5, all body entries visited). */
int orc_body_hits(const orc_t *o, int tool_id, int64_t key, int32_t k) {
  if (tool_id < 0 || tool_id >= MAX_TOOLS) return -1;
  const tool_tab *tt = &o->tools[tool_id];
  if (tt->K <= 0 || k < 0 || k >= tt->K) return -1;
  int64_t s[3];
  orc_unkey(key, s);
  int hits = 0;
  for (int64_t e = tt->begin[k]; e < tt->begin[k + 1]; ++e) {
    if (tt->cls[e] != CLS_BODY) continue;
    const int32_t *d = tt->off + 3 * e;
    vrec r = lookup(o, s[0] + d[0], s[1] + d[1], s[2] + d[2]);
    if (r.W > 0 && r.S < o->rc_u * (int64_t)r.W) ++hits;
  }
  return hits;
}

int orc_score_stats_get(const orc_t *o, orc_score_stats *st) {
  *st = o->sst;
  return 0;
}

/* Results of the last orc_score for points [0, count) in point order (the
 * canonical order): label (255 if not evaluated), first free orientation,
 * has_normal, normal [3] and mask words [mask_words]; returns the count. */
int64_t orc_read_results(const orc_t *o, int64_t count, uint8_t *label, int32_t *first_free,
                         int32_t *has_normal, int64_t *normal, uint64_t *mask,
                         int32_t mask_words) {
  int64_t m = count < o->np ? count : o->np;
  if (m > o->rcap) m = o->rcap;
  for (int64_t p = 0; p < m; ++p) {
    label[p] = o->label[p];
    first_free[p] = o->first_free[p];
    has_normal[p] = o->has_normal[p];
    for (int i = 0; i < 3; ++i) normal[3 * p + i] = o->normal[3 * p + i];
    for (int w = 0; w < mask_words; ++w)
      mask[p * mask_words + w] = w < o->mask_words ? o->mask[p * o->mask_words + w] : 0;
  }
  return m;
}

int orc_point_result(const orc_t *o, int64_t key, uint8_t *label,
                     int32_t *first_free, int64_t normal[3], int32_t *has_normal,
                     uint64_t *mask, int32_t mask_words) {
  int64_t p = hm_get(&o->pmap, key);
  if (p < 0 || p >= o->rcap) return -1;
  *label = o->label[p];
  *first_free = o->first_free[p];
  *has_normal = o->has_normal[p];
  for (int i = 0; i < 3; ++i) normal[i] = o->normal[3 * p + i];
  for (int w = 0; w < mask_words && w < o->mask_words; ++w)
    mask[w] = o->mask[p * o->mask_words + w];
  return 0;
}
