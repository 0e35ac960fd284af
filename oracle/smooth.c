/*
 * Smoothed clearance score -- CPU ORACLE, test infrastructure only.
 *
 * A differentiable companion of the collision-count score of Section 3.5:
 * instead of counting tool-kernel voxels whose TSDF is below the collision
 * threshold, every sample o of the tool (a point of the tool solid in its
 * local frame, approach axis +x, tip at the origin) contributes
 *
 *     log sigma((T(p + R(q) o) - c) / tau_s),
 *
 * where T is the TSDF (Section 3.2) read by trilinear interpolation between
 * voxel centres, so that the sum is differentiable in the point position p
 * and the tool orientation, given as a quaternion q (R maps the local axes to
 * world axes; its first column is the approach direction).  A voxel without
 * weight (never observed, or only ray-cleared) reads the truncation distance
 * tau, the value the map saturates to in free space.
 *
 * Everything here is plain double precision, one sample at a time, in the
 * order the definition reads.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares no source with
 * the GPU library.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "oracle.h"

typedef double (*field_fn)(const void *ctx, int64_t i, int64_t j, int64_t k);

typedef struct {
  const orc_t *o;
  double scale;   /* 256 / v: fixed-point units per metre */
  double tau;     /* metres */
} map_field;

/* T of voxel (i, j, k) of the oracle's map, metres. */
static double map_T(const void *ctx, int64_t i, int64_t j, int64_t k) {
  const map_field *m = (const map_field *)ctx;
  int64_t S;
  int32_t W;
  uint8_t cl;
  if (!orc_voxel(m->o, orc_key(i, j, k), &S, &W, &cl) || W <= 0) return m->tau;
  return ((double)S / (double)W) / m->scale;
}

typedef struct {
  const double *val;
  int64_t dims[3], origin[3];
  double tau;
} dense_field;

/* T of voxel (i, j, k) of a dense block of values (outside: tau). */
static double dense_T(const void *ctx, int64_t i, int64_t j, int64_t k) {
  const dense_field *d = (const dense_field *)ctx;
  int64_t a = i - d->origin[0], b = j - d->origin[1], c = k - d->origin[2];
  if (a < 0 || b < 0 || c < 0 || a >= d->dims[0] || b >= d->dims[1] || c >= d->dims[2])
    return d->tau;
  return d->val[(c * d->dims[1] + b) * d->dims[0] + a];
}

/* Rotation of the normalised quaternion qn = (w, x, y, z), row-major. */
static void quat_matrix(const double qn[4], double R[9]) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

/* J[a][b] = d (R(qn) o)_b / d qn_a of the matrix entries above. */
static void quat_jacobian(const double qn[4], const double o[3], double J[4][3]) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  const double ox = o[0], oy = o[1], oz = o[2];
  J[0][0] = -2 * z * oy + 2 * y * oz;
  J[0][1] = 2 * z * ox - 2 * x * oz;
  J[0][2] = -2 * y * ox + 2 * x * oy;
  J[1][0] = 2 * y * oy + 2 * z * oz;
  J[1][1] = 2 * y * ox - 4 * x * oy - 2 * w * oz;
  J[1][2] = 2 * z * ox + 2 * w * oy - 4 * x * oz;
  J[2][0] = -4 * y * ox + 2 * x * oy + 2 * w * oz;
  J[2][1] = 2 * x * ox + 2 * z * oz;
  J[2][2] = -2 * w * ox + 2 * z * oy - 4 * y * oz;
  J[3][0] = -4 * z * ox - 2 * w * oy + 2 * x * oz;
  J[3][1] = 2 * w * ox - 4 * z * oy + 2 * y * oz;
  J[3][2] = 2 * x * ox + 2 * y * oy;
}

/* log sigma(z) = -log(1 + exp(-z)), evaluated without overflow. */
static double log_sigmoid(double z) {
  return z >= 0 ? -log1p(exp(-z)) : z - log1p(exp(z));
}

/* sigma(-z) = 1 - sigma(z). */
static double sigmoid_neg(double z) {
  return z >= 0 ? exp(-z) / (1 + exp(-z)) : 1 / (1 + exp(z));
}

/* Trilinear T at world position x (metres) and its gradient (per metre).
 * Voxel (i, j, k) has its centre at ((i, j, k) + 1/2) v.  Also returns the
 * distance of x to the nearest cell face, in voxels. */
static double trilinear(field_fn T, const void *ctx, double v, const double x[3], double grad[3],
                        double *face) {
  int64_t i0[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    const double g = x[a] / v - 0.5;
    const double fl = floor(g);
    i0[a] = (int64_t)fl;
    f[a] = g - fl;
    const double d = f[a] < 1 - f[a] ? f[a] : 1 - f[a];
    if (d < *face) *face = d;
  }
  double val = 0, gx = 0, gy = 0, gz = 0;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        const double t = T(ctx, i0[0] + a, i0[1] + b, i0[2] + c);
        const double wx = a ? f[0] : 1 - f[0], wy = b ? f[1] : 1 - f[1],
                     wz = c ? f[2] : 1 - f[2];
        const double sx = a ? 1 : -1, sy = b ? 1 : -1, sz = c ? 1 : -1;
        val += wx * wy * wz * t;
        gx += sx * wy * wz * t;
        gy += wx * sy * wz * t;
        gz += wx * wy * sz * t;
      }
  grad[0] = gx / v;
  grad[1] = gy / v;
  grad[2] = gz / v;
  return val;
}

/* s(p, q) with its gradients: dq (4) with respect to the raw quaternion
 * (through q -> q / |q|), dp (3).  *face receives the smallest distance of a
 * sample to a cell face (voxels) if it is smaller than the value passed. */
static double smooth_one(field_fn T, const void *ctx, double v, const double p[3],
                         const double q[4], const double *samples, int32_t M, double c,
                         double tau_s, double dq[4], double dp[3], double *face) {
  const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double qn[4], R[9];
  for (int a = 0; a < 4; ++a) qn[a] = q[a] / nq;
  quat_matrix(qn, R);
  double s = 0, gqn[4] = {0, 0, 0, 0};
  for (int a = 0; a < 3; ++a) dp[a] = 0;
  for (int32_t m = 0; m < M; ++m) {
    const double *o = samples + 3 * m;
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = p[a] + (R[3 * a] * o[0] + R[3 * a + 1] * o[1] + R[3 * a + 2] * o[2]);
    double g[3];
    const double t = trilinear(T, ctx, v, x, g, face);
    const double z = (t - c) / tau_s;
    s += log_sigmoid(z);
    const double wgt = sigmoid_neg(z) / tau_s;   /* d log sigma(z) / dT */
    for (int a = 0; a < 3; ++a) dp[a] += wgt * g[a];
    double J[4][3];
    quat_jacobian(qn, o, J);
    for (int a = 0; a < 4; ++a) gqn[a] += wgt * (g[0] * J[a][0] + g[1] * J[a][1] + g[2] * J[a][2]);
  }
  /* d qn / d q = (I - qn qn^T) / |q| */
  const double r = qn[0] * gqn[0] + qn[1] * gqn[1] + qn[2] * gqn[2] + qn[3] * gqn[3];
  for (int a = 0; a < 4; ++a) dq[a] = (gqn[a] - qn[a] * r) / nq;
  return s;
}

static void smooth_many(field_fn T, const void *ctx, double v, const float *p, const float *q,
                        int64_t n, const float *samples_f, int32_t M, double c, double tau_s,
                        double *s, double *dq, double *dp, double *face) {
  double samples[3 * 1024];
  for (int32_t m = 0; m < 3 * M; ++m) samples[m] = samples_f[m];
  for (int64_t i = 0; i < n; ++i) {
    const double pp[3] = {p[3 * i], p[3 * i + 1], p[3 * i + 2]};
    const double qq[4] = {q[4 * i], q[4 * i + 1], q[4 * i + 2], q[4 * i + 3]};
    double g4[4], g3[3], fc = 1.0;
    s[i] = smooth_one(T, ctx, v, pp, qq, samples, M, c, tau_s, g4, g3, &fc);
    if (dq) memcpy(dq + 4 * i, g4, sizeof(g4));
    if (dp) memcpy(dp + 3 * i, g3, sizeof(g3));
    if (face) face[i] = fc;
  }
}

static int map_setup(const orc_t *o, map_field *m, double *v) {
  int64_t tau_u, R, rc_u, dmin_u;
  double scale;
  if (orc_params(o, &tau_u, &R, &rc_u, &dmin_u, &scale) != 0) return -1;
  m->o = o;
  m->scale = scale;
  m->tau = (double)tau_u / scale;
  *v = 256.0 / scale;
  return 0;
}

/* Score and gradients of n (point, quaternion) pairs on the oracle's map.
 * p: n x 3 metres; q: n x 4 (w, x, y, z), any non-zero length; samples:
 * M x 3 metres (M <= 1024).  dq, dp, face may be NULL. */
int orc_smooth(const orc_t *o, const float *p, const float *q, int64_t n, const float *samples,
               int32_t M, double c, double tau_s, double *s, double *dq, double *dp,
               double *face) {
  map_field m;
  double v;
  if (M < 1 || M > 1024 || map_setup(o, &m, &v) != 0) return -1;
  smooth_many(map_T, &m, v, p, q, n, samples, M, c, tau_s, s, dq, dp, face);
  return 0;
}

/* The same on a dense block of voxel values val[(k * ny + j) * nx + i] for
 * voxel (origin + (i, j, k)); voxels outside the block read tau. */
int orc_smooth_dense(const double *val, const int64_t dims[3], const int64_t origin[3],
                     double v, double tau, const float *p, const float *q, int64_t n,
                     const float *samples, int32_t M, double c, double tau_s, double *s,
                     double *dq, double *dp, double *face) {
  if (M < 1 || M > 1024 || !(v > 0)) return -1;
  dense_field d;
  d.val = val;
  for (int a = 0; a < 3; ++a) {
    d.dims[a] = dims[a];
    d.origin[a] = origin[a];
  }
  d.tau = tau;
  smooth_many(dense_T, &d, v, p, q, n, samples, M, c, tau_s, s, dq, dp, face);
  return 0;
}

/* Gradient ascent of the orientation: for point i and start j the quaternion
 * q0[i * S + j] is moved `steps` times by q <- (q + D) / |q + D| with
 * D = eta * ds/dq, D scaled down to length max_step when longer; then s is
 * evaluated once more.  q_out: (n * S) x 4, s_out: n * S; face (optional):
 * smallest sample-to-face distance over every evaluation. */
int orc_smooth_refine(const orc_t *o, const float *p, int64_t n, const float *q0, int32_t S,
                      const float *samples_f, int32_t M, double c, double tau_s, int32_t steps,
                      double eta, double max_step, double *q_out, double *s_out, double *face) {
  map_field m;
  double v;
  if (M < 1 || M > 1024 || S < 1 || steps < 0 || map_setup(o, &m, &v) != 0) return -1;
  double samples[3 * 1024];
  for (int32_t k = 0; k < 3 * M; ++k) samples[k] = samples_f[k];
  for (int64_t i = 0; i < n; ++i) {
    const double pp[3] = {p[3 * i], p[3 * i + 1], p[3 * i + 2]};
    for (int32_t j = 0; j < S; ++j) {
      const int64_t r = i * S + j;
      double q[4] = {q0[4 * r], q0[4 * r + 1], q0[4 * r + 2], q0[4 * r + 3]};
      double fc = 1.0, g4[4], g3[3];
      for (int32_t t = 0; t < steps; ++t) {
        smooth_one(map_T, &m, v, pp, q, samples, M, c, tau_s, g4, g3, &fc);
        double D[4], len = 0;
        for (int a = 0; a < 4; ++a) {
          D[a] = eta * g4[a];
          len += D[a] * D[a];
        }
        len = sqrt(len);
        if (len > max_step)
          for (int a = 0; a < 4; ++a) D[a] *= max_step / len;
        double nn = 0;
        for (int a = 0; a < 4; ++a) {
          q[a] += D[a];
          nn += q[a] * q[a];
        }
        nn = sqrt(nn);
        for (int a = 0; a < 4; ++a) q[a] /= nn;
      }
      s_out[r] = smooth_one(map_T, &m, v, pp, q, samples, M, c, tau_s, g4, g3, &fc);
      memcpy(q_out + 4 * r, q, sizeof(q));
      if (face) face[r] = fc;
    }
  }
  return 0;
}
