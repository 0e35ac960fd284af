// Rotated tool kernels (Section 3.4, "Tool kernel", "Self-exclusion", "Arm
// path checking"; precomputed once, Section 3.6).  One workgroup per
// orientation enumerates the voxel offsets of the rotated tool's bounding
// box, keeps those whose centre lies in the body or in the corridor (minus the
// self-exclusion ball), sorts each class by (|o|^2, z, y, x) in LDS and
// writes packed entries: 3 arm samples, then body, then corridor.
#include "af_internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace af {
namespace {

constexpr int kTableThreads = 1024;

// 0 body, 2 corridor, -1 outside.  fp64 in voxel units with a 1e-9 slack on
// the inclusive bounds.
__device__ inline int classify(const ToolGeom &tg, const double *R, int ox, int oy, int oz) {
  const double eps = 1e-9;
  double fx = (double)ox, fy = (double)oy, fz = (double)oz;
  double x = (R[0] * fx + R[3] * fy) + R[6] * fz;
  double y = (R[1] * fx + R[4] * fy) + R[7] * fz;
  double z = (R[2] * fx + R[5] * fy) + R[8] * fz;
  bool cross = tg.shape == AF_TOOL_CYLINDER ? (y * y + z * z) <= tg.rv2 + eps
                                            : (fabs(y) <= tg.a + eps && fabs(z) <= tg.b + eps);
  if (!cross) return -1;
  int64_t n2 = (int64_t)ox * ox + (int64_t)oy * oy + (int64_t)oz * oz;
  if ((double)n2 < tg.rsv2) return -1;
  if (x < -eps || x > tg.Ev + eps) return -1;
  return x <= tg.Lv + eps ? AF_CLS_BODY : AF_CLS_FAR;
}

__device__ inline void bounds(const ToolGeom &tg, const double *R, int lo[3], int hi[3]) {
  for (int i = 0; i < 3; ++i) {
    double mn = 1e300, mx = -1e300;
    for (int c = 0; c < 8; ++c) {
      double x = (c & 1) ? tg.Ev : 0.0;
      double y = (c & 2) ? tg.a : -tg.a;
      double z = (c & 4) ? tg.b : -tg.b;
      double w = R[3 * i] * x + R[3 * i + 1] * y + R[3 * i + 2] * z;
      mn = w < mn ? w : mn;
      mx = w > mx ? w : mx;
    }
    lo[i] = (int)floor(mn) - 1;
    hi[i] = (int)ceil(mx) + 1;
  }
}

__global__ void __launch_bounds__(kTableThreads)
k_table(ToolGeom tg, int32_t K, const double *__restrict__ rot, uint32_t *counts,
        const uint32_t *begin, int32_t *err, uint32_t *entries, int pass) {
  __shared__ unsigned long long keys[kTableMaxClass];
  __shared__ int nkeys;
  __shared__ int lo[3], hi[3];
  const int k = blockIdx.x;
  if (k >= K) return;
  const double *R = rot + 9 * (int64_t)k;
  if (threadIdx.x == 0) bounds(tg, R, lo, hi);
  __syncthreads();
  const int64_t e0 = hi[0] - lo[0] + 1, e1 = hi[1] - lo[1] + 1, e2 = hi[2] - lo[2] + 1;
  const int64_t vol = e0 * e1 * e2;
  uint32_t out = pass ? begin[k] + 3 : 0;
  for (int cls = 0; cls <= 2; cls += 2) {
    if (threadIdx.x == 0) nkeys = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < vol; i += kTableThreads) {
      int ox = lo[0] + (int)(i % e0);
      int oy = lo[1] + (int)((i / e0) % e1);
      int oz = lo[2] + (int)(i / (e0 * e1));
      if (classify(tg, R, ox, oy, oz) != cls) continue;
      if (ox < -511 || ox > 511 || oy < -511 || oy > 511 || oz < -511 || oz > 511) {
        atomicOr(err, 1);
        continue;
      }
      int at = atomicAdd(&nkeys, 1);
      if (at >= kTableMaxClass) {
        atomicOr(err, 2);
        continue;
      }
      uint64_t n2 = (uint64_t)((int64_t)ox * ox + (int64_t)oy * oy + (int64_t)oz * oz);
      keys[at] = (n2 << 32) | ((uint64_t)(oz + 512) << 20) | ((uint64_t)(oy + 512) << 10) |
                 (uint64_t)(ox + 512);
    }
    __syncthreads();
    int n = nkeys < kTableMaxClass ? nkeys : kTableMaxClass;
    if (pass == 0) {
      if (threadIdx.x == 0) counts[2 * k + (cls == AF_CLS_FAR)] = (uint32_t)n;
      __syncthreads();
      continue;
    }
    // bitonic sort of keys[0, npow) with +inf padding
    int npow = 1;
    while (npow < n) npow <<= 1;
    for (int i = n + (int)threadIdx.x; i < npow; i += kTableThreads) keys[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= npow; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < npow; i += kTableThreads) {
          int j = i ^ stride;
          if (j > i) {
            bool up = (i & size) == 0;
            unsigned long long a = keys[i], b = keys[j];
            if ((a > b) == up) {
              keys[i] = b;
              keys[j] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < n; i += kTableThreads) {
      unsigned long long key = keys[i];
      int ox = (int)(key & 1023) - 512;
      int oy = (int)((key >> 10) & 1023) - 512;
      int oz = (int)((key >> 20) & 1023) - 512;
      entries[out + i] = pack_entry(ox, oy, oz, cls);
    }
    out += (uint32_t)n;
    __syncthreads();
  }
  if (pass == 1 && threadIdx.x < 3) {
    double lam = tg.lam[threadIdx.x];
    int o[3];
    for (int i = 0; i < 3; ++i) {
      double t = round(lam * R[3 * i]);
      o[i] = (int)t;
    }
    if (o[0] < -511 || o[0] > 511 || o[1] < -511 || o[1] > 511 || o[2] < -511 || o[2] > 511)
      atomicOr(err, 1);
    entries[begin[k] + threadIdx.x] = pack_entry(o[0], o[1], o[2], AF_CLS_NEAR);
  }
}

// Prefix of 3 + body + corridor entries over orientations (one thread).
__global__ void k_table_scan(int32_t K, const uint32_t *counts, uint32_t *begin) {
  uint32_t acc = 0;
  for (int k = 0; k < K; ++k) {
    begin[k] = acc;
    acc += 3 + counts[2 * k] + counts[2 * k + 1];
  }
  begin[K] = acc;
}

// Coarse corridor list of orientation k for cells of C = 2^SH voxels per
// axis: every cell offset floor((r + o)/C) (r in [0, C)^3 the point's
// position inside its cell, o a corridor entry), as a bitmap over the
// bounding box of those offsets, compacted in linear order.  A bounding box
// above kCoarseBits cells leaves the orientation without a list (cflag = 0).
constexpr int kCoarseBits = 1 << 18;

template <int SH>
__global__ void __launch_bounds__(256)
k_table_coarse(int32_t K, const uint32_t *begin, const uint32_t *counts, const uint32_t *entries,
               uint32_t *far_begin, uint32_t *ccounts, const uint32_t *cbegin,
               uint32_t *centries, uint8_t *cflag, int pass) {
  constexpr int CM = (1 << SH) - 1;
  __shared__ uint32_t bits[kCoarseBits / 32];
  __shared__ int lo[3], hi[3];
  __shared__ uint32_t part[256];
  const int k = blockIdx.x;
  if (k >= K) return;
  const uint32_t fb = begin[k] + 3 + counts[2 * k], e = begin[k + 1];
  if (threadIdx.x < 3) {
    lo[threadIdx.x] = 1 << 20;
    hi[threadIdx.x] = -(1 << 20);
  }
  __syncthreads();
  for (uint32_t j = fb + threadIdx.x; j < e; j += 256) {
    const uint32_t en = entries[j];
    const int o[3] = {entry_x(en), entry_y(en), entry_z(en)};
    for (int a = 0; a < 3; ++a) {
      atomicMin(&lo[a], o[a] >> SH);
      atomicMax(&hi[a], (o[a] + CM) >> SH);
    }
  }
  __syncthreads();
  const int dx = hi[0] - lo[0] + 1, dy = hi[1] - lo[1] + 1, dz = hi[2] - lo[2] + 1;
  const bool ok = fb >= e || (int64_t)dx * dy * dz <= kCoarseBits;
  if (pass == 0 && threadIdx.x == 0) {
    far_begin[k] = fb;
    cflag[k] = ok ? 1 : 0;
  }
  if (!ok || fb >= e) {
    if (pass == 0 && threadIdx.x == 0) ccounts[k] = 0;
    return;
  }
  const int nbits = dx * dy * dz, nwords = (nbits + 31) / 32;
  for (int w = threadIdx.x; w < nwords; w += 256) bits[w] = 0u;
  __syncthreads();
  for (uint32_t j = fb + threadIdx.x; j < e; j += 256) {
    const uint32_t en = entries[j];
    const int o[3] = {entry_x(en), entry_y(en), entry_z(en)};
    for (int c = 0; c < 8; ++c) {
      const int bx = ((o[0] + ((c & 1) ? CM : 0)) >> SH) - lo[0];
      const int by = ((o[1] + ((c & 2) ? CM : 0)) >> SH) - lo[1];
      const int bz = ((o[2] + ((c & 4) ? CM : 0)) >> SH) - lo[2];
      const int idx = (bz * dy + by) * dx + bx;
      atomicOr(&bits[idx >> 5], 1u << (idx & 31));
    }
  }
  __syncthreads();
  // per-thread contiguous word ranges, block prefix of their bit counts
  const int seg = (nwords + 255) / 256;
  const int w0 = threadIdx.x * seg < nwords ? threadIdx.x * seg : nwords;
  const int w1 = w0 + seg < nwords ? w0 + seg : nwords;
  uint32_t cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(bits[w]);
  part[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  if (pass == 0) {
    if (threadIdx.x == 255) ccounts[k] = part[255];
    return;
  }
  uint32_t at = cbegin[k] + part[threadIdx.x] - cnt;
  for (int w = w0; w < w1; ++w) {
    uint32_t m = bits[w];
    while (m) {
      const int b = __ffs(m) - 1;
      m &= m - 1;
      const int idx = 32 * w + b;
      const int bx = idx % dx, by = (idx / dx) % dy, bz = idx / (dx * dy);
      centries[at++] = pack_entry(bx + lo[0], by + lo[1], bz + lo[2], 0);
    }
  }
}

__global__ void k_coarse_scan(int32_t K, const uint32_t *ccounts, uint32_t *cbegin) {
  uint32_t acc = 0;
  for (int k = 0; k < K; ++k) {
    cbegin[k] = acc;
    acc += ccounts[k];
  }
  cbegin[K] = acc;
}

__global__ void k_table_grid(const uint32_t *entries, int64_t n, int32_t gx, int32_t gxy,
                             uint2 *xent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const uint32_t e = entries[i];
    const int ox = entry_x(e), oy = entry_y(e), oz = entry_z(e);
    const int32_t d = (ox >> 3) + gx * (oy >> 3) + gxy * (oz >> 3);
    const uint32_t o7 = (uint32_t)(ox & 7) | ((uint32_t)(oy & 7) << 4) |
                        ((uint32_t)(oz & 7) << 8) | ((uint32_t)entry_cls(e) << 30);
    xent[i] = make_uint2((uint32_t)d, o7);
  }
}

}  // namespace

int launch_table_grid(const ToolDev &t, const GridDev &g, hipStream_t s) {
  const int64_t n = t.n_entries;
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_table_grid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t.entries,
                     n, g.gd[0], g.gd[0] * g.gd[1], t.xent);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_table_coarse(int32_t K, const uint32_t *begin, const uint32_t *counts,
                        const uint32_t *entries, uint32_t *far_begin, uint32_t *ccounts,
                        uint32_t *cbegin, uint32_t *centries, uint8_t *cflag, int pass, int sh,
                        hipStream_t s) {
  if (sh != 2) return -1;
  hipLaunchKernelGGL(k_table_coarse<2>, dim3((unsigned)K), dim3(256), 0, s, K, begin, counts,
                     entries, far_begin, ccounts, cbegin, centries, cflag, pass);
  if (pass == 0) hipLaunchKernelGGL(k_coarse_scan, dim3(1), dim3(1), 0, s, K, ccounts, cbegin);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_table_build(const ToolGeom &tg, int32_t K, const double *rot_dev,
                       uint32_t *counts_dev, uint32_t *begin_dev, int32_t *err_dev,
                       uint32_t *entries_dev, int pass, hipStream_t s) {
  hipLaunchKernelGGL(k_table, dim3((unsigned)K), dim3(kTableThreads), 0, s, tg, K, rot_dev,
                     counts_dev, begin_dev, err_dev, entries_dev, pass);
  if (pass == 0) hipLaunchKernelGGL(k_table_scan, dim3(1), dim3(1), 0, s, K, counts_dev, begin_dev);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace af
