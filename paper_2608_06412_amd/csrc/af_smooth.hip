// Smoothed clearance score and its adjoint.
//
// A differentiable companion of the collision-count score of Section 3.5:
// each sample o of the tool solid (local frame, approach axis +x, tip at the
// origin) placed at p + R(q) o contributes log sigma((T - c) / tau_s), where
// T is the TSDF (Section 3.2) interpolated trilinearly between voxel centres
// and a voxel without weight reads the truncation distance.  Gradients with
// respect to the quaternion q (through q / |q|) and the point p come from the
// same pass: d log sigma(z) / dz = sigma(-z).
//
// Layout: one wave per (point, orientation) pair, one tool sample per lane,
// so the 64 lanes read neighbouring voxels along the tool and the sums are a
// wave reduction.  The TSDF is first expanded into "apron" bricks of 9^3
// floats: brick b holds voxels 8b .. 8b + 8 on each axis, i.e. its own 8^3
// voxels plus the first layer of its +x/+y/+z neighbours, so the 2^3 voxels
// of any interpolation cell whose lowest corner lies in b are all in b's
// apron brick.  Apron bricks exist for every mapped brick and every brick
// with a mapped +1 neighbour (the "halo"); a brick-to-apron table over the
// dense brick grid finds them, so a sample costs one table load and eight
// value loads, with no hashing and no per-tap bounds logic.
//
// Precision: the placement of a sample in its voxel cell (p + R o, divided by
// v) is computed in double precision, because an fp32 position is only good
// to ~1e-5 voxel at metre scale and the gradient's relative error follows the
// cell fractions; interpolation, score and adjoint are fp32.  The quaternion
// derivative comes from the torque: a small rotation dtheta applied after R
// moves sample u = R o by dtheta x u, so s changes by dtheta . sum(u x g) with
// g the weighted TSDF gradient; with dq = (0, dtheta) q / 2 this gives
// ds/dq = 2 (-tau.v, w tau + tau x v) / |q| for q / |q| = (w, v) and
// tau = sum(u x g) -- three sums per pair instead of four, no projection.
// This file lets the compiler fuse multiply-adds (unlike the table builder,
// nothing here needs to round like the oracle).

#include "af_internal.h"

#pragma clang fp contract(fast)

namespace af {
namespace {

constexpr int kSmoothThreads = 256;

__global__ void __launch_bounds__(kSmoothThreads)
k_smooth_values(MapDev m, int64_t n_vox, double scale, float tau, float *T) {
  const int64_t i = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
  if (i >= n_vox) return;
  const int32_t W = m.W[i];
  T[i] = W > 0 ? (float)(((double)m.S[i] / (double)W) / scale) : tau;
}

__global__ void __launch_bounds__(kSmoothThreads)
k_smooth_fill(int32_t *a, int64_t n, int32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kSmoothThreads)
    a[i] = value;
}

__global__ void __launch_bounds__(kSmoothThreads)
k_smooth_bid(MapDev m, int64_t n_blocks, GridDev g, int32_t *bid) {
  const int64_t id = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
  if (id >= n_blocks) return;
  int32_t b[3];
  unpack_key(m.bkey[id], b[0], b[1], b[2]);
  const int x = b[0] - g.g0[0], y = b[1] - g.g0[1], z = b[2] - g.g0[2];
  if ((unsigned)x < (unsigned)g.gd[0] && (unsigned)y < (unsigned)g.gd[1] &&
      (unsigned)z < (unsigned)g.gd[2])
    bid[((int64_t)z * g.gd[1] + y) * g.gd[0] + x] = (int32_t)id;
}

// Apron bricks: mark every brick whose cell may reach a mapped brick (the
// mapped brick itself and its -1 neighbours along any set of axes).
__global__ void __launch_bounds__(kSmoothThreads)
k_apron_mark(MapDev m, int64_t n_blocks, GridDev g, int32_t *bid9) {
  const int64_t id = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
  if (id >= n_blocks) return;
  int32_t b[3];
  unpack_key(m.bkey[id], b[0], b[1], b[2]);
  for (int k = 0; k < 8; ++k) {
    const int x = b[0] - g.g0[0] - (k & 1), y = b[1] - g.g0[1] - ((k >> 1) & 1),
              z = b[2] - g.g0[2] - (k >> 2);
    if ((unsigned)x < (unsigned)g.gd[0] && (unsigned)y < (unsigned)g.gd[1] &&
        (unsigned)z < (unsigned)g.gd[2])
      bid9[((int64_t)z * g.gd[1] + y) * g.gd[0] + x] = -2;
  }
}

// Number the marked bricks (any order) and record each apron's brick.
// (cap is at least the number of marked bricks, 8 per mapped block at most;
// an index past it would be left unmapped rather than read out of bounds.)
__global__ void __launch_bounds__(kSmoothThreads)
k_apron_assign(int32_t *bid9, int64_t n_bricks, int32_t *count, int32_t *brick_of, int64_t cap) {
  for (int64_t i = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x; i < n_bricks;
       i += (int64_t)gridDim.x * kSmoothThreads)
    if (bid9[i] == -2) {
      const int32_t e = atomicAdd(count, 1);
      if (e >= 0 && e < cap) {
        bid9[i] = e;
        brick_of[e] = (int32_t)i;
      } else {
        bid9[i] = -1;
      }
    }
}

// Fill apron e: voxel (lx, ly, lz) in [0, 9)^3 of brick brick_of[e].
__global__ void __launch_bounds__(kSmoothThreads)
k_apron_fill(const int32_t *count, const int32_t *brick_of, GridDev g, const int32_t *bid,
             const float *T, float tau, int64_t cap, float *T9) {
  const int64_t i = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
  const int64_t e = i / 729;
  if (e >= cap || e >= *count) return;
  const int v = (int)(i - e * 729);
  const int lx = v % 9, ly = (v / 9) % 9, lz = v / 81;
  const int64_t br = brick_of[e];
  const int bx = (int)(br % g.gd[0]), by = (int)((br / g.gd[0]) % g.gd[1]),
            bz = (int)(br / ((int64_t)g.gd[0] * g.gd[1]));
  const int x = bx + (lx >> 3), y = by + (ly >> 3), z = bz + (lz >> 3);
  float t = tau;
  if (x < g.gd[0] && y < g.gd[1] && z < g.gd[2]) {
    const int32_t id = bid[((int64_t)z * g.gd[1] + y) * g.gd[0] + x];
    if (id >= 0) t = T[(int64_t)id * 512 + ((lx & 7) | ((ly & 7) << 3) | ((lz & 7) << 6))];
  }
  T9[i] = t;
}

// x + the value DPP control `ctrl` routes to this lane (0 in rows outside
// row_mask).
template <int ctrl, int row_mask>
__device__ inline float dpp_add(float x) {
  const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, row_mask, 0xf, false);
  return x + __int_as_float(y);
}

// Sum over the wave, returned in every lane: swaps within quads, mirrors
// within half-rows and rows, then row broadcasts carry the row sums up to
// lane 63, which is read back.
__device__ inline float wave_sum(float x) {
  x = dpp_add<0xb1, 0xf>(x);    // quad_perm [1, 0, 3, 2]
  x = dpp_add<0x4e, 0xf>(x);    // quad_perm [2, 3, 0, 1]
  x = dpp_add<0x141, 0xf>(x);   // row_half_mirror
  x = dpp_add<0x140, 0xf>(x);   // row_mirror
  x = dpp_add<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// The 2^3 voxel values of the cell whose lowest corner is voxel (X, Y, Z),
// t[a | b << 1 | c << 2] for corner (X + a, Y + b, Z + c); tau where unmapped.
__device__ inline void cell_values(const SmoothField &f, int X, int Y, int Z, float t[8]) {
  const int bx = (X >> 3) - f.g0[0], by = (Y >> 3) - f.g0[1], bz = (Z >> 3) - f.g0[2];
  int32_t e = -1;
  if ((unsigned)bx < (unsigned)f.gd[0] && (unsigned)by < (unsigned)f.gd[1] &&
      (unsigned)bz < (unsigned)f.gd[2])
    e = f.bid9[((int64_t)bz * f.gd[1] + by) * f.gd[0] + bx];
  if (e < 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = f.tau;
    return;
  }
  const float *c = f.T9 + (int64_t)e * 729 + (Z & 7) * 81 + (Y & 7) * 9 + (X & 7);
#pragma unroll
  for (int k = 0; k < 8; ++k) t[k] = c[(k & 1) + ((k >> 1) & 1) * 9 + (k >> 2) * 81];
}

// A pair's point as integer voxel coordinate + fraction of p / v - 1/2.
struct PairBase {
  int ip[3];
  double rp[3];
};

__device__ inline PairBase pair_base(const float *p, double v) {
  PairBase b;
  for (int a = 0; a < 3; ++a) {
    const double g = (double)p[a] / v - 0.5;
    const double fl = floor(g);
    b.ip[a] = (int)fl;
    b.rp[a] = g - fl;
  }
  return b;
}

// Normalised quaternion, its norm, and the rotation (row-major, double for
// the placement of samples).
struct Rot {
  float qn[4];
  float nq;
  double R[9];
};

__device__ inline Rot make_rot(const float q[4]) {
  Rot r;
  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  const double n = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double in = 1.0 / n;
  const double w = q0 * in, x = q1 * in, y = q2 * in, z = q3 * in;
  r.nq = (float)n;
  r.qn[0] = (float)w;
  r.qn[1] = (float)x;
  r.qn[2] = (float)y;
  r.qn[3] = (float)z;
  r.R[0] = 1.0 - 2.0 * (y * y + z * z);
  r.R[1] = 2.0 * (x * y - w * z);
  r.R[2] = 2.0 * (x * z + w * y);
  r.R[3] = 2.0 * (x * y + w * z);
  r.R[4] = 1.0 - 2.0 * (x * x + z * z);
  r.R[5] = 2.0 * (y * z - w * x);
  r.R[6] = 2.0 * (x * z - w * y);
  r.R[7] = 2.0 * (y * z + w * x);
  r.R[8] = 1.0 - 2.0 * (x * x + y * y);
  return r;
}

__device__ inline float log_sigmoid(float z) {
  return z >= 0.f ? -log1pf(expf(-z)) : z - log1pf(expf(z));
}

// sigma(-z) = 1 / (1 + e^z) with the hardware exponential and reciprocal
// (about 1 ulp each; e^z = inf gives 0).
__device__ inline float sigmoid_neg(float z) {
  return __builtin_amdgcn_rcpf(1.f + __expf(z));
}

// One sample: returns its log sigma term (not with G == 2); with G > 0 adds
// the torque gs (u x dT/dx) into tq and, with G == 1, gs dT/dx into dp.
template <int G>
__device__ inline float smooth_sample(const SmoothField &f, const PairBase &pb, const Rot &r,
                                      double inv_v, const float o[3], float c, float inv_ts,
                                      float gs, float dp[3], float tq[3]) {
  int cell[3];
  float fr[3], u[3];
  for (int a = 0; a < 3; ++a) {
    const double ud = r.R[3 * a] * (double)o[0] + r.R[3 * a + 1] * (double)o[1] +
                      r.R[3 * a + 2] * (double)o[2];
    const double gl = pb.rp[a] + ud * inv_v;
    const double fl = floor(gl);
    cell[a] = pb.ip[a] + (int)fl;
    fr[a] = (float)(gl - fl);
    u[a] = (float)ud;
  }
  float t[8];
  cell_values(f, cell[0], cell[1], cell[2], t);
  const float fx = fr[0], fy = fr[1], fz = fr[2];
  // trilinear interpolation as lerps along x, then y, then z
  const float a00 = t[0] + fx * (t[1] - t[0]), a10 = t[2] + fx * (t[3] - t[2]);
  const float a01 = t[4] + fx * (t[5] - t[4]), a11 = t[6] + fx * (t[7] - t[6]);
  const float b0 = a00 + fy * (a10 - a00), b1 = a01 + fy * (a11 - a01);
  const float val = b0 + fz * (b1 - b0);
  const float z = (val - c) * inv_ts;
  if (G > 0) {
    // derivatives of the interpolant in cell units
    const float dx0 = (t[1] - t[0]) + fy * ((t[3] - t[2]) - (t[1] - t[0]));
    const float dx1 = (t[5] - t[4]) + fy * ((t[7] - t[6]) - (t[5] - t[4]));
    const float gx = dx0 + fz * (dx1 - dx0);
    const float gy = (a10 - a00) + fz * ((a11 - a01) - (a10 - a00));
    const float gz = b1 - b0;
    const float wgt = sigmoid_neg(z) * inv_ts * gs * (float)inv_v;
    const float g0 = wgt * gx, g1 = wgt * gy, g2 = wgt * gz;
    if (G == 1) {
      dp[0] += g0;
      dp[1] += g1;
      dp[2] += g2;
    }
    tq[0] += u[1] * g2 - u[2] * g1;
    tq[1] += u[2] * g0 - u[0] * g2;
    tq[2] += u[0] * g1 - u[1] * g0;
  }
  return G == 2 ? 0.f : log_sigmoid(z);
}

// s of one pair (wave-uniform result), gradients reduced over the wave.
// o0: the lane's sample of the first 64 (loaded once per kernel).
template <int G>
__device__ inline float smooth_pair(const SmoothField &f, const PairBase &pb, const Rot &r,
                                    double inv_v, const float *samples, int M, const float o0[3],
                                    float c, float inv_ts, float gs, float dp[3], float tq[3]) {
  const int lane = threadIdx.x & 63;
  float s = 0.f;
  for (int a = 0; a < 3; ++a) dp[a] = tq[a] = 0.f;
  if (lane < M) s += smooth_sample<G>(f, pb, r, inv_v, o0, c, inv_ts, gs, dp, tq);
  for (int m0 = 64; m0 < M; m0 += 64) {
    const int m = m0 + lane;
    if (m < M) {
      const float o[3] = {samples[3 * m], samples[3 * m + 1], samples[3 * m + 2]};
      s += smooth_sample<G>(f, pb, r, inv_v, o, c, inv_ts, gs, dp, tq);
    }
  }
  if (G != 2) s = wave_sum(s);
  if (G == 1)
    for (int a = 0; a < 3; ++a) dp[a] = wave_sum(dp[a]);
  if (G > 0)
    for (int a = 0; a < 3; ++a) tq[a] = wave_sum(tq[a]);
  return s;
}

// ds/dq from the torque tau: 2 (-tau.v, w tau + tau x v) / |q|.
__device__ inline void unnormalise(const Rot &r, const float tq[3], float dq[4]) {
  const float w = r.qn[0], x = r.qn[1], y = r.qn[2], z = r.qn[3];
  const float k = 2.f / r.nq;
  dq[0] = -k * (tq[0] * x + tq[1] * y + tq[2] * z);
  dq[1] = k * (w * tq[0] + tq[1] * z - tq[2] * y);
  dq[2] = k * (w * tq[1] + tq[2] * x - tq[0] * z);
  dq[3] = k * (w * tq[2] + tq[0] * y - tq[1] * x);
}

constexpr int kSmoothBatch = 16;   // pairs a wave takes from a work counter at once
constexpr int kXcds = 8;           // workgroup i runs on XCD i mod 8, each with its own L2

// Work distribution: the pairs are cut into kXcds contiguous ranges, one per
// XCD, so that (with pairs ordered in space) the waves sharing an L2 read the
// same part of the map; a wave whose range is exhausted helps the next ones.
// work[x] counts the pairs handed out from range x.
struct PairQueue {
  unsigned long long *work;
  int64_t n;
  int x;       // range being taken from
  int tried;   // ranges exhausted so far
};

__device__ inline PairQueue pair_queue(unsigned long long *work, int64_t n) {
  PairQueue pq;
  pq.work = work;
  pq.n = n;
  pq.x = blockIdx.x % kXcds;
  pq.tried = 0;
  return pq;
}

// First pair of the wave's next batch, -1 when every range is done
// (wave-uniform); the batch ends at the range's end.
__device__ inline int64_t take_batch(PairQueue &pq, int64_t &end) {
  while (pq.tried < kXcds) {
    const int64_t lo = pq.n * pq.x / kXcds, hi = pq.n * (pq.x + 1) / kXcds;
    unsigned long long b = 0;
    if ((threadIdx.x & 63) == 0) b = atomicAdd(&pq.work[pq.x], (unsigned long long)kSmoothBatch);
    const int64_t i = lo + (int64_t)__shfl(b, 0);
    if (i < hi) {
      end = i + kSmoothBatch < hi ? i + kSmoothBatch : hi;
      return i;
    }
    pq.x = (pq.x + 1) % kXcds;
    ++pq.tried;
  }
  return -1;
}

__device__ inline void lane_sample(const float *samples, int M, float o[3]) {
  const int lane = threadIdx.x & 63;
  const int m = lane < M ? lane : 0;
  o[0] = samples[3 * m];
  o[1] = samples[3 * m + 1];
  o[2] = samples[3 * m + 2];
}

template <int G>
__global__ void __launch_bounds__(kSmoothThreads)
k_smooth_eval(SmoothField f, double v, const float *p, const float *q, int64_t n,
              const float *samples, int M, float c, float tau_s, const float *grad_s,
              float *s_out, float *dq_out, float *dp_out, unsigned long long *work) {
  const int lane = threadIdx.x & 63;
  const double inv_v = 1.0 / v;
  const float inv_ts = 1.f / tau_s;
  float o0[3];
  lane_sample(samples, M, o0);
  PairQueue pq = pair_queue(work, n);
  int64_t end = 0;
  for (int64_t b0 = take_batch(pq, end); b0 >= 0; b0 = take_batch(pq, end))
  for (int64_t i = b0; i < end; ++i) {
    const PairBase pb = pair_base(p + 3 * i, v);
    const float q4[4] = {q[4 * i], q[4 * i + 1], q[4 * i + 2], q[4 * i + 3]};
    const Rot r = make_rot(q4);
    const float gs = grad_s ? grad_s[i] : 1.f;
    float dp[3], dqn[3];
    const float s = smooth_pair<G>(f, pb, r, inv_v, samples, M, o0, c, inv_ts, gs, dp, dqn);
    if (lane == 0) {
      if (s_out) s_out[i] = s;
      if (G == 1) {
        float dq[4];
        unnormalise(r, dqn, dq);
        for (int a = 0; a < 4; ++a) dq_out[4 * i + a] = dq[a];
        for (int a = 0; a < 3; ++a) dp_out[3 * i + a] = dp[a];
      }
    }
  }
}

// Orientation ascent: per (point, start) pair, `steps` updates
// q <- (q + D) / |q + D|, D = eta ds/dq clipped to length max_step, with q
// kept in registers; then s at the final q.
__global__ void __launch_bounds__(kSmoothThreads)
k_smooth_refine(SmoothField f, double v, const float *p, int64_t n_points, const float *q0,
                int n_starts, const float *samples, int M, float c, float tau_s, int steps,
                float eta, float max_step, float *q_out, float *s_out,
                unsigned long long *work) {
  const int lane = threadIdx.x & 63;
  const int64_t n = n_points * n_starts;
  const double inv_v = 1.0 / v;
  const float inv_ts = 1.f / tau_s;
  float o0[3];
  lane_sample(samples, M, o0);
  PairQueue pq = pair_queue(work, n);
  int64_t end = 0;
  for (int64_t b0 = take_batch(pq, end); b0 >= 0; b0 = take_batch(pq, end))
  for (int64_t i = b0; i < end; ++i) {
    const PairBase pb = pair_base(p + 3 * (i / n_starts), v);
    float q[4] = {q0[4 * i], q0[4 * i + 1], q0[4 * i + 2], q0[4 * i + 3]};
    float dp[3], dqn[3], dq[4];
    for (int t = 0; t < steps; ++t) {
      const Rot r = make_rot(q);
      smooth_pair<2>(f, pb, r, inv_v, samples, M, o0, c, inv_ts, 1.f, dp, dqn);
      unnormalise(r, dqn, dq);
      float D[4], len = 0.f;
      for (int a = 0; a < 4; ++a) {
        D[a] = eta * dq[a];
        len += D[a] * D[a];
      }
      len = sqrtf(len);
      const float sc = len > max_step ? max_step / len : 1.f;
      float nn = 0.f;
      for (int a = 0; a < 4; ++a) {
        q[a] += D[a] * sc;
        nn += q[a] * q[a];
      }
      nn = sqrtf(nn);
      for (int a = 0; a < 4; ++a) q[a] /= nn;
    }
    const Rot r = make_rot(q);
    const float s = smooth_pair<0>(f, pb, r, inv_v, samples, M, o0, c, inv_ts, 1.f, dp, dqn);
    if (lane == 0) {
      s_out[i] = s;
      for (int a = 0; a < 4; ++a) q_out[4 * i + a] = r.qn[a];
    }
  }
}

// Workgroups that fit on the chip at once (the pairs are handed out by the
// work counter, so a grid larger than that would only queue).
unsigned smooth_grid(const void *fn, int64_t pairs) {
  static int n_cu = 0;
  if (n_cu == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n_cu <= 0)
      n_cu = 1;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSmoothThreads, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const int64_t need = (pairs + 4 * kSmoothBatch - 1) / (4 * kSmoothBatch);
  const int64_t wg = std::min<int64_t>((int64_t)per_cu * n_cu, need);
  return (unsigned)std::max<int64_t>(1, wg);
}

}  // namespace

void launch_smooth_prepare(const Params &p, MapDev m, int64_t n_blocks, GridDev g,
                           int64_t grid_bricks, float tau, const SmoothBuffers &b,
                           hipStream_t s) {
  const int64_t nv = n_blocks * 512;
  auto blocks = [](int64_t n) { return dim3((unsigned)((n + kSmoothThreads - 1) / kSmoothThreads)); };
  const dim3 strided((unsigned)std::min<int64_t>(4096, (grid_bricks + kSmoothThreads - 1) / kSmoothThreads));
  hipLaunchKernelGGL(k_smooth_fill, dim3(1), dim3(kSmoothThreads), 0, s, b.count, 1, 0);
  if (grid_bricks <= 0) return;
  hipLaunchKernelGGL(k_smooth_fill, strided, dim3(kSmoothThreads), 0, s, b.bid, grid_bricks, -1);
  hipLaunchKernelGGL(k_smooth_fill, strided, dim3(kSmoothThreads), 0, s, b.bid9, grid_bricks, -1);
  if (n_blocks <= 0) return;
  hipLaunchKernelGGL(k_smooth_values, blocks(nv), dim3(kSmoothThreads), 0, s, m, nv, p.scale, tau,
                     b.T);
  hipLaunchKernelGGL(k_smooth_bid, blocks(n_blocks), dim3(kSmoothThreads), 0, s, m, n_blocks, g,
                     b.bid);
  hipLaunchKernelGGL(k_apron_mark, blocks(n_blocks), dim3(kSmoothThreads), 0, s, m, n_blocks, g,
                     b.bid9);
  hipLaunchKernelGGL(k_apron_assign, strided, dim3(kSmoothThreads), 0, s, b.bid9, grid_bricks,
                     b.count, b.brick_of, b.apron_cap);
  hipLaunchKernelGGL(k_apron_fill, blocks(b.apron_cap * 729), dim3(kSmoothThreads), 0, s, b.count,
                     b.brick_of, g, b.bid, b.T, tau, b.apron_cap, b.T9);
}

void launch_smooth_eval(const SmoothField &f, double v, const float *p, const float *q, int64_t n,
                        const float *samples, int32_t M, float c, float tau_s,
                        const float *grad_s, float *s_out, float *dq, float *dp,
                        unsigned long long *work, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_smooth_fill, dim3(1), dim3(kSmoothThreads), 0, s, (int32_t *)work,
                     2 * kXcds, 0);
  if (dq) {
    const void *fn = (const void *)k_smooth_eval<1>;
    hipLaunchKernelGGL(k_smooth_eval<1>, dim3(smooth_grid(fn, n)), dim3(kSmoothThreads), 0, s, f,
                       v, p, q, n, samples, M, c, tau_s, grad_s, s_out, dq, dp, work);
  } else {
    const void *fn = (const void *)k_smooth_eval<0>;
    hipLaunchKernelGGL(k_smooth_eval<0>, dim3(smooth_grid(fn, n)), dim3(kSmoothThreads), 0, s, f,
                       v, p, q, n, samples, M, c, tau_s, grad_s, s_out, dq, dp, work);
  }
}

void launch_smooth_refine(const SmoothField &f, double v, const float *p, int64_t n_points,
                          const float *q0, int32_t n_starts, const float *samples, int32_t M,
                          float c, float tau_s, int32_t steps, float eta, float max_step,
                          float *q_out, float *s_out, unsigned long long *work, hipStream_t s) {
  const int64_t n = n_points * n_starts;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_smooth_fill, dim3(1), dim3(kSmoothThreads), 0, s, (int32_t *)work,
                     2 * kXcds, 0);
  hipLaunchKernelGGL(k_smooth_refine, dim3(smooth_grid((const void *)k_smooth_refine, n)),
                     dim3(kSmoothThreads), 0, s, f, v, p, n_points, q0, n_starts, samples, M, c,
                     tau_s, steps, eta, max_step, q_out, s_out, work);
}

}  // namespace af
