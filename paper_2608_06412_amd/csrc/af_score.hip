// Scoring kernels (Sections 3.4 and 3.5): PCA normals, candidate-direction
// masks and the per-point collision-count search over the rotated kernels.
#include "af_internal.h"

#include <algorithm>
#include <vector>

#pragma clang fp contract(off)

namespace af {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Neighbour window [-3, 3]^3 as (dx, dy, dz, |d|^2), sorted by |d|^2.
__constant__ int8_t c_nb[343 * 4];

__device__ inline int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ inline int64_t brick_index(const GridDev &g, int x, int y, int z) {
  int bx = (x >> 3) - g.g0[0], by = (y >> 3) - g.g0[1], bz = (z >> 3) - g.g0[2];
  if ((unsigned)bx >= (unsigned)g.gd[0] || (unsigned)by >= (unsigned)g.gd[1] ||
      (unsigned)bz >= (unsigned)g.gd[2])
    return -1;
  return ((int64_t)bz * g.gd[1] + by) * g.gd[0] + bx;
}

__device__ inline bool surf_bit(const GridDev &g, int x, int y, int z) {
  int64_t b = brick_index(g, x, y, z);
  if (b < 0) return false;
  int lin = (x & 7) | ((y & 7) << 3) | ((z & 7) << 6);
  return (g.surf[b * 16 + (lin >> 5)] >> (lin & 31)) & 1u;
}

// 2-bit code: bit 0 TSDF < r_c, bit 1 unknown and not ray-cleared.
__device__ inline uint32_t code_at(const GridDev &g, int x, int y, int z) {
  int64_t b = brick_index(g, x, y, z);
  if (b < 0) return 2u;
  int lin = (x & 7) | ((y & 7) << 3) | ((z & 7) << 6);
  return (g.pred[b * 32 + (lin >> 4)] >> (2 * (lin & 15))) & 3u;
}

__device__ inline int64_t round_shift(int64_t x, int sh) {
  if (sh <= 0) return x;
  int64_t m = x < 0 ? -x : x;
  int64_t q = (m + (1LL << (sh - 1))) >> sh;
  return x < 0 ? -q : q;
}

__device__ inline int bit_length(uint64_t m) { return m ? 64 - __clzll((long long)m) : 0; }

// Least principal axis of the k nearest surface voxels (ties at the k-th
// distance included), oriented towards the mean sensor position.  The
// scatter matrix M = n sum(dd^T) - (sum d)(sum d)^T is exact; the dominant
// eigenvector of B = tr(M) I - M is read from B^256 (eight squarings with
// 28-bit renormalisation by rounded shifts) as its largest-norm column.
__global__ void __launch_bounds__(kThreads)
k_normals(Params p, MapDev m, PointsDev pts, GridDev g, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  int32_t addr = pts.addr[i];
  int W = addr >= 0 ? (int)m.W[addr] : 0;
  if (W < p.conf_min_w) {
    pts.has_normal[i] = -1;
    return;
  }
  int32_t s[3];
  unpack_key(pts.key[i], s[0], s[1], s[2]);
  int cnt = 0, last = -1;
  int sx[3] = {0, 0, 0}, sxx[6] = {0, 0, 0, 0, 0, 0};
  for (int j = 0; j < 343; ++j) {
    int d2 = c_nb[4 * j + 3];
    if (cnt >= p.knn_k && d2 != last) break;
    int dx = c_nb[4 * j], dy = c_nb[4 * j + 1], dz = c_nb[4 * j + 2];
    if (!surf_bit(g, s[0] + dx, s[1] + dy, s[2] + dz)) continue;
    ++cnt;
    last = d2;
    sx[0] += dx; sx[1] += dy; sx[2] += dz;
    sxx[0] += dx * dx; sxx[1] += dx * dy; sxx[2] += dx * dz;
    sxx[3] += dy * dy; sxx[4] += dy * dz; sxx[5] += dz * dz;
  }
  int32_t *nout = pts.normal + 3 * i;
  if (cnt < 3) {
    pts.has_normal[i] = 0;
    nout[0] = nout[1] = nout[2] = 0;
    return;
  }
  const int sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  int64_t B[3][3];
  int64_t tr = 0;
  for (int a = 0; a < 3; ++a) tr += (int64_t)cnt * sxx[sym[a][a]] - (int64_t)sx[a] * sx[a];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      B[a][b] = (a == b ? tr : 0) - ((int64_t)cnt * sxx[sym[a][b]] - (int64_t)sx[a] * sx[b]);
  for (int it = 0; it < 8; ++it) {
    int64_t C[3][3];
    uint64_t mx = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        C[a][b] = B[a][0] * B[0][b] + B[a][1] * B[1][b] + B[a][2] * B[2][b];
        uint64_t mag = (uint64_t)(C[a][b] < 0 ? -C[a][b] : C[a][b]);
        mx = mag > mx ? mag : mx;
      }
    int sh = bit_length(mx) - 28;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) B[a][b] = round_shift(C[a][b], sh);
  }
  int best = 0;
  int64_t bn = -1;
  for (int c = 0; c < 3; ++c) {
    int64_t nrm = B[0][c] * B[0][c] + B[1][c] * B[1][c] + B[2][c] * B[2][c];
    if (nrm > bn) {
      bn = nrm;
      best = c;
    }
  }
  if (bn <= 0) {
    pts.has_normal[i] = 0;
    nout[0] = nout[1] = nout[2] = 0;
    return;
  }
  __int128 gdot = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t ga = pts.sumq[3 * i + a] - (int64_t)pts.nq[i] * (256 * (int64_t)s[a] + 128);
    gdot += (__int128)B[a][best] * ga;
  }
  int sgn = gdot < 0 ? -1 : 1;
  for (int a = 0; a < 3; ++a) nout[a] = (int32_t)(sgn * B[a][best]);
  pts.has_normal[i] = 1;
}

// One lane per point: the point's normal and viewpoint vectors stay in
// registers (fp64, exact conversions of integers) while every lane walks the
// same orientation list, so each direction is a wave-uniform load.
__global__ void __launch_bounds__(kThreads)
k_mask(Params p, PointsDev pts, ToolDev t, int64_t n, int32_t mw) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool act = i < n;
  const int hn = act ? pts.has_normal[i] : -1;
  double n0 = 0, n1 = 0, n2 = 0, nn = 0;
  double wx[kMaxVp], wy[kMaxVp], wz[kMaxVp], ww[kMaxVp];
  int nv = 0;
  if (hn >= 0) {
    if (hn > 0) {
      const int32_t *nvp = pts.normal + 3 * i;
      n0 = (double)nvp[0];
      n1 = (double)nvp[1];
      n2 = (double)nvp[2];
      nn = (double)((int64_t)nvp[0] * nvp[0] + (int64_t)nvp[1] * nvp[1] +
                    (int64_t)nvp[2] * nvp[2]);
    }
    int32_t s[3];
    unpack_key(pts.key[i], s[0], s[1], s[2]);
    nv = pts.nvp[i];
#pragma unroll
    for (int j = 0; j < kMaxVp; ++j) {
      if (j < nv) {
        const int32_t *V = pts.vp + (i * kMaxVp + j) * 3;
        int64_t a0 = (int64_t)V[0] - (256 * (int64_t)s[0] + 128);
        int64_t a1 = (int64_t)V[1] - (256 * (int64_t)s[1] + 128);
        int64_t a2 = (int64_t)V[2] - (256 * (int64_t)s[2] + 128);
        wx[j] = (double)a0;
        wy[j] = (double)a1;
        wz[j] = (double)a2;
        ww[j] = (double)(a0 * a0 + a1 * a1 + a2 * a2);
      } else {
        wx[j] = wy[j] = wz[j] = ww[j] = 0.0;
      }
    }
  }
  unsigned long long cand = 0;
  for (int w = 0; w < mw; ++w) {
    uint64_t word = 0;
    const int kend = t.K - 64 * w < 64 ? t.K - 64 * w : 64;
    for (int j = 0; j < kend; ++j) {
      const double *R = t.rot + 9 * (int64_t)(64 * w + j);
      const double d0 = R[0], d1 = R[3], d2 = R[6];
      bool ok = hn >= 0;
      if (hn > 0) {
        double dot = (n0 * d0 + n1 * d1) + n2 * d2;
        ok = dot >= 0.0 && dot * dot >= p.cos2 * nn;
      }
      if (ok) {
        bool seen = false;
#pragma unroll
        for (int v = 0; v < kMaxVp; ++v) {
          if (v < nv && !seen) {
            double wd = (wx[v] * d0 + wy[v] * d1) + wz[v] * d2;
            seen = wd > 0.0 && wd * wd > p.obs2 * ww[v];
          }
        }
        ok = seen;
      }
      word |= (uint64_t)ok << j;
    }
    if (act) t.mask[i * mw + w] = word;
    cand += (unsigned long long)__popcll(word);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    unsigned lo = __shfl_xor((unsigned)(cand & 0xffffffffu), off);
    unsigned hi = __shfl_xor((unsigned)(cand >> 32), off);
    cand += ((unsigned long long)hi << 32) | lo;
  }
  if (lane_id() == 0 && cand) atomicAdd(&t.counters->candidate_tests, cand);
}

// Position of the r-th (1-based) set bit of m, or 64.
__device__ inline int nth_bit(uint64_t m, int r) {
  if (__popcll(m) < r) return 64;
  for (int i = 1; i < r; ++i) m &= m - 1;
  return __ffsll((long long)m) - 1;
}

constexpr int kScoreThreads = 1024;
constexpr int kScoreWaves = kScoreThreads / 64;
constexpr int kLdsK = 256;   // orientations whose first table chunk lives in LDS

// One orientation of one point, lanes over table entries in order; returns
// true when free.  `lookups` counts entries up to the deciding one.  The first
// 64 entries of orientations below kLdsK come from LDS.
__device__ inline bool orientation_free(const Params &p, const ToolDev &t, const GridDev &g,
                                        const int32_t s[3], int k, const uint32_t *s_begin,
                                        const uint32_t *s_first, int kc, uint64_t &lookups) {
  const uint32_t b = k < kc ? s_begin[k] : t.begin[k];
  const uint32_t e = k < kc ? s_begin[k + 1] : t.begin[k + 1];
  const int lane = lane_id();
  int body = 0;
  for (uint32_t base = b; base < e; base += 64) {
    uint32_t idx = base + lane;
    bool hit = false;
    int cls = AF_CLS_BODY;
    if (idx < e) {
      uint32_t ent = (base == b && k < kc) ? s_first[64 * k + lane] : t.entries[idx];
      cls = entry_cls(ent);
      uint32_t code = code_at(g, s[0] + entry_x(ent), s[1] + entry_y(ent), s[2] + entry_z(ent));
      hit = cls == AF_CLS_NEAR ? code != 0u : (code & 1u) != 0u;
    }
    uint64_t nf = __ballot(hit && cls != AF_CLS_BODY);
    uint64_t bm = __ballot(hit && cls == AF_CLS_BODY);
    int stop = nf ? __ffsll((long long)nf) - 1 : 64;
    int sb = nth_bit(bm, p.n_c - body);
    stop = sb < stop ? sb : stop;
    if (stop < 64) {
      lookups += (uint64_t)stop + 1;
      return false;
    }
    body += __popcll(bm);
    lookups += (e - base) < 64u ? (e - base) : 64u;
  }
  return true;
}

// Persistent workgroups of 16 waves, one wave per point (grid-stride): the
// lowest-index candidate orientation that is free labels the point
// accessible.
__global__ void __launch_bounds__(kScoreThreads)
k_score(Params p, MapDev m, PointsDev pts, ToolDev t, GridDev g, int64_t n, int32_t mw) {
  __shared__ uint32_t s_begin[kLdsK + 1];
  __shared__ uint32_t s_first[kLdsK * 64];
  const int kc = t.K < kLdsK ? t.K : kLdsK;
  for (int j = threadIdx.x; j <= kc; j += kScoreThreads) s_begin[j] = t.begin[j];
  __syncthreads();
  for (int j = threadIdx.x; j < kc * 64; j += kScoreThreads) {
    uint32_t pos = s_begin[j >> 6] + (uint32_t)(j & 63);
    s_first[j] = pos < s_begin[(j >> 6) + 1] ? t.entries[pos] : 0u;
  }
  __syncthreads();
  const int lane = lane_id();
  const int64_t wave0 =
      (int64_t)blockIdx.x * kScoreWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kScoreWaves;
  uint64_t conf = 0, acc = 0, blk = 0, nocand = 0, tests = 0, lookups = 0;
  for (int64_t i = wave0; i < n; i += nwaves) {
    int hn = __builtin_amdgcn_readfirstlane(pts.has_normal[i]);
    uint8_t label;
    int16_t ff = -1;
    if (hn < 0) {
      label = AF_UNSCORED;
    } else {
      ++conf;
      int32_t s[3];
      unpack_key(pts.key[i], s[0], s[1], s[2]);
      label = AF_NO_CANDIDATE;
      for (int w = 0; w < mw && ff < 0; ++w) {
        uint64_t word = t.mask[i * mw + w];
        while (word) {
          int k = 64 * w + (__ffsll((long long)word) - 1);
          word &= word - 1;
          label = AF_BLOCKED;
          ++tests;
          if (orientation_free(p, t, g, s, k, s_begin, s_first, kc, lookups)) {
            label = AF_ACCESSIBLE;
            ff = (int16_t)k;
            break;
          }
        }
      }
      acc += label == AF_ACCESSIBLE;
      blk += label == AF_BLOCKED;
      nocand += label == AF_NO_CANDIDATE;
    }
    if (lane == 0) {
      t.label[i] = label;
      t.first_free[i] = ff;
    }
  }
  if (lane == 0) {
    if (conf) atomicAdd(&t.counters->n_confident, (unsigned long long)conf);
    if (acc) atomicAdd(&t.counters->n_accessible, (unsigned long long)acc);
    if (blk) atomicAdd(&t.counters->n_blocked, (unsigned long long)blk);
    if (nocand) atomicAdd(&t.counters->n_no_candidate, (unsigned long long)nocand);
    if (tests) atomicAdd(&t.counters->canonical_tests, (unsigned long long)tests);
    if (lookups) atomicAdd(&t.counters->canonical_lookups, (unsigned long long)lookups);
  }
}

bool g_tables_ready = false;

void init_tables() {
  if (g_tables_ready) return;
  std::vector<int> order;
  for (int z = -3; z <= 3; ++z)
    for (int y = -3; y <= 3; ++y)
      for (int x = -3; x <= 3; ++x) order.push_back(((x + 3) * 7 + (y + 3)) * 7 + (z + 3));
  auto d2 = [](int c) {
    int x = c / 49 - 3, y = (c / 7) % 7 - 3, z = c % 7 - 3;
    return x * x + y * y + z * z;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d2(a) < d2(b); });
  int8_t tab[343 * 4];
  for (int j = 0; j < 343; ++j) {
    int c = order[j];
    tab[4 * j] = (int8_t)(c / 49 - 3);
    tab[4 * j + 1] = (int8_t)((c / 7) % 7 - 3);
    tab[4 * j + 2] = (int8_t)(c % 7 - 3);
    tab[4 * j + 3] = (int8_t)d2(c);
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_nb), tab, sizeof(tab)) == hipSuccess) g_tables_ready = true;
}

}  // namespace

void launch_normals(const Params &p, MapDev m, PointsDev pts, GridDev g, int64_t n,
                    hipStream_t s) {
  init_tables();
  if (n <= 0) return;
  hipLaunchKernelGGL(k_normals, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, s, p, m, pts, g, n);
}

void launch_mask(const Params &p, PointsDev pts, ToolDev t, int64_t n, hipStream_t s) {
  int32_t mw = (t.K + 63) / 64;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mask, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     s, p, pts, t, n, mw);
}

void launch_score(const Params &p, MapDev m, PointsDev pts, ToolDev t, GridDev g, int64_t n,
                  hipStream_t s) {
  int32_t mw = (t.K + 63) / 64;
  if (n <= 0) return;
  int64_t wg = (n + kScoreWaves - 1) / kScoreWaves;
  if (wg > 512) wg = 512;   // two resident workgroups per CU
  hipLaunchKernelGGL(k_score, dim3((unsigned)wg), dim3(kScoreThreads), 0, s, p, m, pts, t, g, n,
                     mw);
}

}  // namespace af
