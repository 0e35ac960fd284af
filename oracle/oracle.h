/*
 * Accessibility-field CPU ORACLE -- test infrastructure only.
 *
 * A plain, single-threaded, slow and deliberately unoptimised implementation
 * of what the hot path computes, written from the paper (Scott, Schofield,
 * Green, "Beyond Visibility: Real-Time Surface Accessibility Fields from
 * Sparse LiDAR"): scan-centric TSDF integration (Section 3.2), the ray-cleared
 * band and arm-path samples (Section 3.4, "Arm path checking"), voxel
 * de-duplicated surface points (Section 3.1), PCA normals and the two
 * candidate-direction filters (Section 3.4, "Approach directions"), rotated
 * tool kernels with self-exclusion (Section 3.4, "Tool kernel",
 * "Self-exclusion") and the collision-count score with the confidence gate
 * (Section 3.5).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this code.  It shares no source with the GPU library.
 */
#ifndef AF_ORACLE_H
#define AF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc_t;

typedef struct orc_config {
  double voxel;          /* voxel edge v, metres */
  double trunc;          /* truncation tau, metres (<= 0: min(4v, 0.1 m)) */
  double r_c;            /* collision threshold on the TSDF, metres */
  int32_t n_c;           /* body hits that block an orientation */
  int32_t weight_cap;    /* weight saturation (2000) */
  int32_t conf_min_w;    /* W >= this <=> confidence w/(w+5) >= 0.2 */
  double cos_normal;     /* cos of the normal half-cone (70 deg) */
  double obs_dot;        /* observation-side dot threshold (0.25) */
  double vp_min_dist;    /* novelty distance for stored viewpoints, metres */
  int32_t n_vp;          /* stored viewpoints per point (<= 8) */
  int32_t knn_k;         /* neighbours for the PCA normal (10) */
  int32_t clamp_negative;/* 0: clamp d to [0,tau]; 1: [-tau,tau] (ablation) */
  int32_t pad;
} orc_config;

typedef struct orc_tool {
  int32_t shape;         /* 0 cylinder, 1 box */
  int32_t pad;
  double length, corridor, r_s, radius, width, height; /* metres */
} orc_tool;

typedef struct orc_frame_stats {
  int64_t n_in, n_valid, n_dropped;
  int64_t pairs_applied, pairs_excluded, band_marks;
  int64_t new_points, n_points, voxels_folded;
} orc_frame_stats;

typedef struct orc_score_stats {
  int64_t n_points, n_confident, n_accessible, n_blocked, n_no_candidate;
  int64_t candidate_tests, canonical_tests, canonical_lookups;
} orc_score_stats;

orc_t *orc_create(const orc_config *cfg);
void orc_destroy(orc_t *o);
/* Restrict every voxel update to index box [lo, hi] (inclusive); for checking
 * sampled outputs of workloads too large to integrate in full. */
void orc_set_roi(orc_t *o, const int64_t lo[3], const int64_t hi[3]);
int orc_integrate_frame(orc_t *o, const float *xyz, int64_t n,
                        const float origin[3], int64_t frame_id);
int orc_frame_stats_get(const orc_t *o, orc_frame_stats *st);
int64_t orc_num_voxels(const orc_t *o);
/* Every stored voxel (W > 0 or cleared), sorted by key. */
int64_t orc_read_tsdf(const orc_t *o, int64_t *key, int64_t *S, int32_t *W,
                      uint8_t *cleared, int64_t cap);
/* Per-voxel lookup; returns 1 if stored. */
int orc_voxel(const orc_t *o, int64_t key, int64_t *S, int32_t *W,
              uint8_t *cleared);
int64_t orc_num_points(const orc_t *o);
int64_t orc_read_points(const orc_t *o, int64_t *key, int32_t *first_frame,
                        int32_t *n_vp, int32_t *vp /* [n][8][3] */,
                        int64_t *sumq /* [n][3] */, int32_t *nq, int64_t cap);

/* Tool kernel table, Section 3.4 "Tool kernel": rot is K row-major 3x3
 * matrices whose columns are the tool's local axes in world coordinates. */
int orc_set_tool(orc_t *o, int tool_id, const orc_tool *t, int32_t K,
                 const double *rot);
/* Table of one orientation: offsets [m][3] and classes (0 body, 1 near arm
 * sample, 2 far corridor); returns m, or -1. */
/* A caller-built table: K directions [K][3], entry ranges begin[K + 1],
 * offsets off[n][3] and classes cls[n] (0 body, 1 arm sample, 2 corridor);
 * see oracle.c.  Returns 0, or -1 for an invalid table. */
int orc_set_tool_table(orc_t *o, int tool_id, int32_t K, const double *dir,
                       const uint32_t *begin, const int16_t *off, const uint8_t *cls);
int64_t orc_tool_table(const orc_t *o, int tool_id, int32_t k, int32_t *off,
                       uint8_t *cls, int64_t cap);

/* Score all points (keys == NULL) or only the listed point keys. */
int orc_score(orc_t *o, int tool_id, const int64_t *keys, int64_t n_keys);
/* orc_score of the listed keys with each point's orientations restricted to
 * the set bits of allow[key index][ceil(K/64)]. */
int orc_score_allow(orc_t *o, int tool_id, const int64_t *keys, int64_t n_keys,
                    const uint64_t *allow);
int orc_score_stats_get(const orc_t *o, orc_score_stats *st);
/* Results of the last orc_score for point `key`: label (0 unscored,
 * 1 accessible, 2 blocked, 3 no candidate), first free orientation, the
 * normal (int64 x3, has_normal), and the candidate mask words. */
/* The same for points [0, count) in canonical order; returns the count. */
int64_t orc_read_results(const orc_t *o, int64_t count, uint8_t *label, int32_t *first_free,
                         int32_t *has_normal, int64_t *normal, uint64_t *mask,
                         int32_t mask_words);
int orc_point_result(const orc_t *o, int64_t key, uint8_t *label,
                     int32_t *first_free, int64_t normal[3], int32_t *has_normal,
                     uint64_t *mask, int32_t mask_words);

/* Keys of the voxels that received a contribution in the last frame; returns
 * their number (keys: up to cap of them). */
int64_t orc_changed_voxels(const orc_t *o, int64_t *keys, int64_t cap);
/* Body voxels of orientation k with TSDF < r_c at point `key` (all visited). */
int orc_body_hits(const orc_t *o, int tool_id, int64_t key, int32_t k);

/* Smoothed clearance score (smooth.c): sum over tool samples o of
 * log sigma((T(p + R(q) o) - c) / tau_s) with trilinear T, and its gradients
 * with respect to the quaternion q (w, x, y, z) and the point p. */
int orc_smooth(const orc_t *o, const float *p, const float *q, int64_t n, const float *samples,
               int32_t M, double c, double tau_s, double *s, double *dq, double *dp,
               double *face);
int orc_smooth_dense(const double *val, const int64_t dims[3], const int64_t origin[3],
                     double v, double tau, const float *p, const float *q, int64_t n,
                     const float *samples, int32_t M, double c, double tau_s, double *s,
                     double *dq, double *dp, double *face);
int orc_smooth_refine(const orc_t *o, const float *p, int64_t n, const float *q0, int32_t S,
                      const float *samples, int32_t M, double c, double tau_s, int32_t steps,
                      double eta, double max_step, double *q_out, double *s_out, double *face);

/* Exposed for unit tests. */
/* Least principal axis of a neighbourhood from its moments (cnt, sum d,
 * sum dd^T as 00 01 02 11 12 22), in fixed point 2^30, unoriented; returns
 * 0 (axis zero) when cnt < 3. */
int orc_pca_axis(int64_t cnt, const int64_t sx[3], const int64_t sxx[6], int64_t out[3]);
void orc_pca_axes(const int32_t *mom, int64_t n, int64_t *axes, int32_t *has);
int64_t orc_isqrt(int64_t n);
int64_t orc_floor_div(int64_t a, int64_t b);
int64_t orc_key(int64_t x, int64_t y, int64_t z);
void orc_unkey(int64_t key, int64_t out[3]);
/* Sliding window of L[3] blocks (see oracle.c); before the first frame. */
int orc_set_window(orc_t *o, const int64_t L[3]);
int orc_window(const orc_t *o, int64_t lo[3], int64_t hi[3], int64_t *shifts);
int orc_params(const orc_t *o, int64_t *tau_u, int64_t *R, int64_t *rc_u,
               int64_t *dmin_u, double *scale);

#ifdef __cplusplus
}
#endif
#endif
