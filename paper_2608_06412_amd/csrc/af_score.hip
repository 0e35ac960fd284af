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

constexpr int kLdsK = 256;   // orientations whose table heads are staged in LDS

// Hit test of one table entry at point s: arm samples (NEAR) hit on TSDF < r_c
// or unknown-and-not-cleared; body and corridor entries hit on TSDF < r_c
// only.  With OCC, a brick without any voxel below r_c answers body and
// corridor entries from its occupancy bit.
template <int OCC>
__device__ inline bool entry_hits(const GridDev &g, const int32_t s[3], uint32_t ent) {
  const int cls = entry_cls(ent);
  const int x = s[0] + entry_x(ent), y = s[1] + entry_y(ent), z = s[2] + entry_z(ent);
  const int64_t b = brick_index(g, x, y, z);
  if (b < 0) return cls == AF_CLS_NEAR;
  const int lin = (x & 7) | ((y & 7) << 3) | ((z & 7) << 6);
  if (OCC && cls != AF_CLS_NEAR && !((g.occ_any[b >> 5] >> (b & 31)) & 1u)) return false;
  const uint32_t code = (g.pred[b * 32 + (lin >> 4)] >> (2 * (lin & 15))) & 3u;
  return cls == AF_CLS_NEAR ? code != 0u : (code & 1u) != 0u;
}

// Position of the deciding hit in a chunk (an arm/corridor hit, or the
// need-th body hit), or 64 if the chunk does not decide.
__device__ inline int chunk_stop(uint64_t nf, uint64_t bm, int need) {
  int stop = nf ? __ffsll((long long)nf) - 1 : 64;
  int sb = nth_bit(bm, need);
  return sb < stop ? sb : stop;
}

// Entries [b, e) of one orientation after its first chunk, UN chunks per
// step (several gathers per lane in flight); decisions are taken chunk by
// chunk in table order, so `lookups` stays the canonical count.
template <int UN, int OCC>
__device__ inline bool scan_rest(const Params &p, const ToolDev &t, const GridDev &g,
                                 const int32_t s[3], uint32_t b, uint32_t e, int body,
                                 uint64_t &lookups) {
  const int lane = lane_id();
  for (uint32_t base = b; base < e; base += 64 * UN) {
    bool hit[UN];
    uint32_t ent[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      uint32_t idx = base + 64 * u + lane;
      ent[u] = idx < e ? t.entries[idx] : 0u;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      uint32_t idx = base + 64 * u + lane;
      hit[u] = idx < e && entry_hits<OCC>(g, s, ent[u]);
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const uint32_t cb = base + 64 * u;
      uint64_t nf = __ballot(hit[u] && entry_cls(ent[u]) != AF_CLS_BODY);
      uint64_t bm = __ballot(hit[u] && entry_cls(ent[u]) == AF_CLS_BODY);
      if (cb >= e) break;
      int stop = chunk_stop(nf, bm, p.n_c - body);
      if (stop < 64) {
        lookups += (uint64_t)stop + 1;
        return false;
      }
      body += __popcll(bm);
      lookups += (e - cb) < 64u ? (e - cb) : 64u;
    }
  }
  return true;
}

// One wave per point: the lowest-index candidate orientation that is free
// labels the point accessible.  Persistent workgroups of NT threads take
// points by grid stride (FB = 0) or in batches of FB from a counter.  The first chunks of the next AH candidates are read together
// (they decide most blocked orientations); a candidate they leave undecided
// is finished before the next one is looked at.  With LK > 0 the table
// begin offsets and the first 64 entries of the first LK orientations are
// staged in LDS.
template <int NT, int LK, int AH, int UN, int OCC, int FB>
__global__ void __launch_bounds__(NT)
k_score(Params p, PointsDev pts, ToolDev t, GridDev g, int64_t n, int32_t mw,
        unsigned *work) {
  constexpr int NW = NT / 64;
  __shared__ uint32_t s_begin[LK > 0 ? LK + 1 : 1];
  __shared__ uint32_t s_first[LK > 0 ? LK * 64 : 1];
  const int kc = LK > 0 ? (t.K < LK ? t.K : LK) : 0;
  if (LK > 0) {
    for (int j = threadIdx.x; j <= kc; j += NT) s_begin[j] = t.begin[j];
    __syncthreads();
    for (int j = threadIdx.x; j < kc * 64; j += NT) {
      uint32_t pos = s_begin[j >> 6] + (uint32_t)(j & 63);
      s_first[j] = pos < s_begin[(j >> 6) + 1] ? t.entries[pos] : 0u;
    }
    __syncthreads();
  }
  const int lane = lane_id();
  const int64_t wave0 =
      (int64_t)blockIdx.x * NW + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * NW;
  uint64_t conf = 0, acc = 0, blk = 0, nocand = 0, tests = 0, lookups = 0;
  int64_t i = wave0, batch_end = wave0 + 1;
  if (FB > 0) {
    unsigned got = 0;
    if (lane == 0) got = atomicAdd(work, (unsigned)FB);
    i = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
    batch_end = i + FB;
  }
  while (i < n) {
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
      int w = 0;
      uint64_t word = mw > 0 ? t.mask[i * mw] : 0;
      while (ff < 0) {
        int ks[AH];
        int nk = 0;
        while (nk < AH) {
          while (!word && ++w < mw) word = t.mask[i * mw + w];
          if (!word) break;
          ks[nk++] = 64 * w + (__ffsll((long long)word) - 1);
          word &= word - 1;
        }
        if (nk == 0) break;
        label = AF_BLOCKED;
        uint32_t bs[AH], es[AH], ent[AH];
        bool hit[AH];
#pragma unroll
        for (int a = 0; a < AH; ++a) {
          const int k = a < nk ? ks[a] : ks[0];
          const bool cached = LK > 0 && k < kc;
          bs[a] = cached ? s_begin[k] : t.begin[k];
          es[a] = cached ? s_begin[k + 1] : t.begin[k + 1];
          const uint32_t idx = bs[a] + lane;
          ent[a] = idx < es[a] ? (cached ? s_first[64 * k + lane] : t.entries[idx]) : 0u;
        }
#pragma unroll
        for (int a = 0; a < AH; ++a)
          hit[a] = a < nk && bs[a] + lane < es[a] && entry_hits<OCC>(g, s, ent[a]);
#pragma unroll
        for (int a = 0; a < AH; ++a) {
          uint64_t nf = __ballot(hit[a] && entry_cls(ent[a]) != AF_CLS_BODY);
          uint64_t bm = __ballot(hit[a] && entry_cls(ent[a]) == AF_CLS_BODY);
          if (a >= nk || ff >= 0) continue;
          ++tests;
          int stop = chunk_stop(nf, bm, p.n_c);
          if (stop < 64) {
            lookups += (uint64_t)stop + 1;
            continue;
          }
          const uint32_t n0 = es[a] - bs[a] < 64u ? es[a] - bs[a] : 64u;
          lookups += n0;
          if (scan_rest<UN, OCC>(p, t, g, s, bs[a] + n0, es[a], __popcll(bm), lookups))
            ff = (int16_t)ks[a];
        }
      }
      if (ff >= 0) label = AF_ACCESSIBLE;
      acc += label == AF_ACCESSIBLE;
      blk += label == AF_BLOCKED;
      nocand += label == AF_NO_CANDIDATE;
    }
    if (lane == 0) {
      t.label[i] = label;
      t.first_free[i] = ff;
    }
    if (FB > 0) {
      if (++i >= batch_end) {
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(work, (unsigned)FB);
        i = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
        batch_end = i + FB;
      }
    } else {
      i += nwaves;
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

// Candidate-parallel variant.  The mask is taken one 64-orientation word at
// a time.  Phase 1: lane j examines the first E entries of orientation 64w+j
// (if it is a candidate), all gathers issued together; near the tip these
// decide most blocked orientations.  Phase 2: the word's candidates are taken
// in index order; decided ones only add their canonical counts, undecided
// ones are finished with lanes over entries.  The first E entries of the
// first kLdsK orientations are staged in LDS with an odd row stride.
template <int NT, int E, int UN, int OCC, int FB>
__global__ void __launch_bounds__(NT)
k_score_batch(Params p, PointsDev pts, ToolDev t, GridDev g, int64_t n, int32_t mw,
              unsigned *work) {
  constexpr int NW = NT / 64;
  constexpr int ST = E + 1;
  __shared__ uint32_t s_begin[kLdsK + 1];
  __shared__ uint32_t s_head[kLdsK * ST];
  const int kc = t.K < kLdsK ? t.K : kLdsK;
  for (int j = threadIdx.x; j <= kc; j += NT) s_begin[j] = t.begin[j];
  __syncthreads();
  for (int j = threadIdx.x; j < kc * E; j += NT) {
    const int k = j / E, q = j - k * E;
    const uint32_t pos = s_begin[k] + (uint32_t)q;
    s_head[k * ST + q] = pos < s_begin[k + 1] ? t.entries[pos] : 0u;
  }
  __syncthreads();
  const int lane = lane_id();
  const int64_t wave0 =
      (int64_t)blockIdx.x * NW + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * NW;
  uint64_t conf = 0, acc = 0, blk = 0, nocand = 0, tests = 0, lookups = 0;
  // points by grid stride (FB = 0) or in batches of FB from a shared counter
  int64_t i = wave0, batch_end = wave0 + 1;
  if (FB > 0) {
    unsigned got = 0;
    if (lane == 0) got = atomicAdd(work, (unsigned)FB);
    i = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
    batch_end = i + FB;
  }
  for (; i < n;) {
    const int hn = __builtin_amdgcn_readfirstlane(pts.has_normal[i]);
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
        const uint64_t word = t.mask[i * mw + w];
        if (!word) continue;
        label = AF_BLOCKED;
        // phase 1: lane j <-> orientation 64w + j
        const int k = 64 * w + lane;
        const bool cand = (word >> lane) & 1ull;
        int state = 0, pos = 0, body = 0;   // state 0 undecided, 1 blocked, 2 free
        if (cand) {
          const bool cached = k < kc;
          const uint32_t b = cached ? s_begin[k] : t.begin[k];
          const uint32_t e = cached ? s_begin[k + 1] : t.begin[k + 1];
          const uint32_t len = e - b;
          uint32_t ent[E];
#pragma unroll
          for (int q = 0; q < E; ++q)
            ent[q] = (uint32_t)q < len ? (cached ? s_head[k * ST + q] : t.entries[b + q]) : 0u;
          bool hit[E];
#pragma unroll
          for (int q = 0; q < E; ++q) hit[q] = (uint32_t)q < len && entry_hits<OCC>(g, s, ent[q]);
#pragma unroll
          for (int q = 0; q < E; ++q) {
            if (state == 0 && hit[q]) {
              if (entry_cls(ent[q]) != AF_CLS_BODY || ++body >= p.n_c) {
                state = 1;
                pos = q;
              }
            }
          }
          if (state == 0 && len <= (uint32_t)E) state = 2;
        }
        const int packed = state | (pos << 2) | (body << 10);
        // phase 2: candidates of this word in index order
        uint64_t rest = word;
        while (rest) {
          const int j = __ffsll((long long)rest) - 1;
          rest &= rest - 1;
          const int pk = __builtin_amdgcn_readfirstlane(__shfl(packed, j));
          const int kj = 64 * w + j;
          ++tests;
          const int st = pk & 3;
          if (st == 1) {
            lookups += (uint64_t)((pk >> 2) & 255) + 1;
            continue;
          }
          const bool cj = kj < kc;
          const uint32_t b = cj ? s_begin[kj] : t.begin[kj];
          const uint32_t e = cj ? s_begin[kj + 1] : t.begin[kj + 1];
          if (st == 2) {
            lookups += e - b;
            ff = (int16_t)kj;
            break;
          }
          lookups += E;
          if (scan_rest<UN, OCC>(p, t, g, s, b + E, e, pk >> 10, lookups)) {
            ff = (int16_t)kj;
            break;
          }
        }
      }
      if (ff >= 0) label = AF_ACCESSIBLE;
      acc += label == AF_ACCESSIBLE;
      blk += label == AF_BLOCKED;
      nocand += label == AF_NO_CANDIDATE;
    }
    if (lane == 0) {
      t.label[i] = label;
      t.first_free[i] = ff;
    }
    if (FB > 0) {
      if (++i >= batch_end) {
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(work, (unsigned)FB);
        i = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
        batch_end = i + FB;
      }
    } else {
      i += nwaves;
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

// Branch-free lookup: the point's brick (relative to the grid) and in-brick
// offset are hoisted; offsets outside the grid read "unknown, not cleared"
// from a clamped (valid) address, so every lane issues its load.
struct PointFrame {
  int rx, ry, rz;   // point voxel & 7
  int bx, by, bz;   // point brick - grid origin
};

__device__ inline PointFrame point_frame(const GridDev &g, const int32_t s[3]) {
  PointFrame f;
  f.rx = s[0] & 7;
  f.ry = s[1] & 7;
  f.rz = s[2] & 7;
  f.bx = (s[0] >> 3) - g.g0[0];
  f.by = (s[1] >> 3) - g.g0[1];
  f.bz = (s[2] >> 3) - g.g0[2];
  return f;
}

__device__ inline uint32_t code_fast(const GridDev &g, const PointFrame &f, uint32_t ent) {
  const int tx = f.rx + entry_x(ent), ty = f.ry + entry_y(ent), tz = f.rz + entry_z(ent);
  const int bx = f.bx + (tx >> 3), by = f.by + (ty >> 3), bz = f.bz + (tz >> 3);
  const bool in = (unsigned)bx < (unsigned)g.gd[0] && (unsigned)by < (unsigned)g.gd[1] &&
                  (unsigned)bz < (unsigned)g.gd[2];
  const unsigned brick = in ? (unsigned)((bz * g.gd[1] + by) * g.gd[0] + bx) : 0u;
  const unsigned lin = (unsigned)((tx & 7) | ((ty & 7) << 3) | ((tz & 7) << 6));
  const unsigned w = g.pred[(brick << 5) | (lin >> 4)];
  const unsigned code = (w >> ((lin & 15u) << 1)) & 3u;
  return in ? code : 2u;
}

__device__ inline bool code_hits(uint32_t ent, uint32_t code) {
  return entry_cls(ent) == AF_CLS_NEAR ? code != 0u : (code & 1u) != 0u;
}

template <int UN>
__device__ inline bool scan_fine(const Params &p, const ToolDev &t, const GridDev &g,
                                 const PointFrame &f, uint32_t b, uint32_t e, int &body,
                                 uint64_t &lookups) {
  const uint32_t lane = (uint32_t)lane_id();
  for (uint32_t base = b; base < e; base += 64 * UN) {
    uint32_t ent[UN], code[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const uint32_t idx = base + 64 * u + lane;
      ent[u] = t.entries[idx < e ? idx : e - 1];
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) code[u] = code_fast(g, f, ent[u]);
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const uint32_t cb = base + 64 * u;
      const bool hit = cb + lane < e && code_hits(ent[u], code[u]);
      uint64_t nf = __ballot(hit && entry_cls(ent[u]) != AF_CLS_BODY);
      uint64_t bm = __ballot(hit && entry_cls(ent[u]) == AF_CLS_BODY);
      if (cb >= e) break;
      int stop = chunk_stop(nf, bm, p.n_c - body);
      if (stop < 64) {
        lookups += (uint64_t)stop + 1;
        return false;
      }
      body += __popcll(bm);
      lookups += (e - cb) < 64u ? (e - cb) : 64u;
    }
  }
  return true;
}

// True if no brick of the coarse corridor list of orientation k (relative to
// the point's brick) holds a voxel with TSDF < r_c; then no corridor entry
// can hit (corridor hits need TSDF < r_c) and the fine scan can be skipped.
__device__ inline bool corridor_clear(const ToolDev &t, const GridDev &g, const PointFrame &f,
                                      int k) {
  const uint32_t cb = t.cbegin[k], ce = t.cbegin[k + 1];
  const uint32_t lane = (uint32_t)lane_id();
  for (uint32_t base = cb; base < ce; base += 64) {
    const uint32_t idx = base + lane;
    const uint32_t d = t.centries[idx < ce ? idx : ce - 1];
    const int bx = f.bx + entry_x(d), by = f.by + entry_y(d), bz = f.bz + entry_z(d);
    const bool in = (unsigned)bx < (unsigned)g.gd[0] && (unsigned)by < (unsigned)g.gd[1] &&
                    (unsigned)bz < (unsigned)g.gd[2];
    const unsigned brick = in ? (unsigned)((bz * g.gd[1] + by) * g.gd[0] + bx) : 0u;
    const bool occ = in && ((g.occ_any[brick >> 5] >> (brick & 31)) & 1u);
    if (__ballot(idx < ce && occ)) return false;
  }
  return true;
}

// Entries [b, e) of orientation k after its head: body entries finely, then
// the corridor -- skipped when its coarse bricks are clear (CO), finely
// otherwise.  Canonical lookups stay the table-order count.
template <int UN, int CO>
__device__ inline bool scan_rest_fast(const Params &p, const ToolDev &t, const GridDev &g,
                                      const PointFrame &f, int k, uint32_t b, uint32_t fb,
                                      uint32_t e, int body, uint64_t &lookups,
                                      uint64_t &cchecks, uint64_t &cclear) {
  if (!CO) return scan_fine<UN>(p, t, g, f, b, e, body, lookups);
  const uint32_t mid = fb > b ? fb : b;
  if (!scan_fine<UN>(p, t, g, f, b, mid, body, lookups)) return false;
  if (mid >= e) return true;
  if (t.cflag[k]) {
    ++cchecks;
    if (corridor_clear(t, g, f, k)) {
      ++cclear;
      lookups += e - mid;
      return true;
    }
  }
  return scan_fine<UN>(p, t, g, f, mid, e, body, lookups);
}

// Candidate-parallel scoring, branch-free.  Requires K <= kLdsK: every
// orientation's begin offset and first E entries are staged in LDS (rows
// padded to an odd stride); see k_score_batch for the two phases.
template <int NT, int E, int UN, int FB, int CO>
__global__ void __launch_bounds__(NT)
k_score_fast(Params p, PointsDev pts, ToolDev t, GridDev g, int64_t n, int32_t mw,
             unsigned *work) {
  constexpr int NW = NT / 64;
  constexpr int ST = E + 1;
  __shared__ uint32_t s_begin[kLdsK + 1];
  __shared__ uint32_t s_head[kLdsK * ST];
  const int K = t.K;
  for (int j = threadIdx.x; j <= K; j += NT) s_begin[j] = t.begin[j];
  __syncthreads();
  for (int j = threadIdx.x; j < K * E; j += NT) {
    const int k = j / E, q = j - k * E;
    const uint32_t pos = s_begin[k] + (uint32_t)q;
    s_head[k * ST + q] = pos < s_begin[k + 1] ? t.entries[pos] : 0u;
  }
  __syncthreads();
  const int lane = lane_id();
  const int64_t wave0 =
      (int64_t)blockIdx.x * NW + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * NW;
  uint64_t conf = 0, acc = 0, blk = 0, nocand = 0, tests = 0, lookups = 0, deep = 0, chunks = 0;
  uint64_t cchecks = 0, cclear = 0;
  int64_t i = wave0, batch_end = wave0 + 1;
  if (FB > 0) {
    unsigned got = 0;
    if (lane == 0) got = atomicAdd(work, (unsigned)FB);
    i = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
    batch_end = i + FB;
  }
  for (; i < n;) {
    const int hn = __builtin_amdgcn_readfirstlane(pts.has_normal[i]);
    uint8_t label;
    int16_t ff = -1;
    if (hn < 0) {
      label = AF_UNSCORED;
    } else {
      ++conf;
      int32_t s[3];
      unpack_key(pts.key[i], s[0], s[1], s[2]);
      const PointFrame f = point_frame(g, s);
      label = AF_NO_CANDIDATE;
      // all mask words of the point in one load (lane w holds word w)
      const uint64_t mine = lane < mw ? t.mask[i * mw + lane] : 0ull;
      for (int w = 0; w < mw && ff < 0; ++w) {
        const uint64_t word =
            ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(mine >> 32), w) << 32) |
            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mine, w);
        if (!word) continue;
        label = AF_BLOCKED;
        const int k = 64 * w + lane;
        const int kk = k < K ? k : K - 1;
        const bool cand = (word >> lane) & 1ull;
        const uint32_t len = s_begin[kk + 1] - s_begin[kk];
        uint32_t ent[E], code[E];
#pragma unroll
        for (int q = 0; q < E; ++q) ent[q] = s_head[kk * ST + q];
#pragma unroll
        for (int q = 0; q < E; ++q) code[q] = code_fast(g, f, ent[q]);
        int state = 0, pos = 0, body = 0;   // 0 undecided, 1 blocked, 2 free
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const bool hit = (uint32_t)q < len && code_hits(ent[q], code[q]);
          if (state == 0 && hit) {
            if (entry_cls(ent[q]) != AF_CLS_BODY || ++body >= p.n_c) {
              state = 1;
              pos = q;
            }
          }
        }
        if (state == 0 && len <= (uint32_t)E) state = 2;
        const int packed = cand ? (state | (pos << 2) | (body << 10)) : 0;
        uint64_t rest = word;
        while (rest) {
          const int j = __ffsll((long long)rest) - 1;
          rest &= rest - 1;
          const int pk = __builtin_amdgcn_readlane(packed, j);
          const int kj = 64 * w + j;
          ++tests;
          const int st = pk & 3;
          if (st == 1) {
            lookups += (uint64_t)((pk >> 2) & 255) + 1;
            continue;
          }
          const uint32_t b = s_begin[kj], e = s_begin[kj + 1];
          if (st == 2) {
            lookups += e - b;
            ff = (int16_t)kj;
            break;
          }
          lookups += E;
          ++deep;
          chunks += (e - b - E + 63) / 64;
          if (scan_rest_fast<UN, CO>(p, t, g, f, kj, b + E, CO ? t.far_begin[kj] : e, e, pk >> 10,
                                     lookups, cchecks, cclear)) {
            ff = (int16_t)kj;
            break;
          }
        }
      }
      if (ff >= 0) label = AF_ACCESSIBLE;
      acc += label == AF_ACCESSIBLE;
      blk += label == AF_BLOCKED;
      nocand += label == AF_NO_CANDIDATE;
    }
    if (lane == 0) {
      t.label[i] = label;
      t.first_free[i] = ff;
    }
    if (FB > 0) {
      if (++i >= batch_end) {
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(work, (unsigned)FB);
        i = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
        batch_end = i + FB;
      }
    } else {
      i += nwaves;
    }
  }
  if (lane == 0) {
    if (conf) atomicAdd(&t.counters->n_confident, (unsigned long long)conf);
    if (acc) atomicAdd(&t.counters->n_accessible, (unsigned long long)acc);
    if (blk) atomicAdd(&t.counters->n_blocked, (unsigned long long)blk);
    if (nocand) atomicAdd(&t.counters->n_no_candidate, (unsigned long long)nocand);
    if (tests) atomicAdd(&t.counters->canonical_tests, (unsigned long long)tests);
    if (lookups) atomicAdd(&t.counters->canonical_lookups, (unsigned long long)lookups);
    if (deep) atomicAdd(&t.counters->deep_tests, (unsigned long long)deep);
    if (chunks) atomicAdd(&t.counters->deep_chunks_max, (unsigned long long)chunks);
    if (cchecks) atomicAdd(&t.counters->coarse_checks, (unsigned long long)cchecks);
    if (cclear) atomicAdd(&t.counters->coarse_clear, (unsigned long long)cclear);
  }
}

using ScoreKernel = void (*)(Params, PointsDev, ToolDev, GridDev, int64_t, int32_t, unsigned *);

struct ScoreVariant {
  ScoreKernel fn;
  int threads;
  const char *name;
  int needs_lds_k;   // 1: only for K <= kLdsK
};

// The tunable score configurations (identical results; speed only).
const ScoreVariant kVariants[] = {
    {k_score<256, 0, 1, 1, 0, 0>, 256, "wg256 ahead1 unroll1"},
    {k_score<256, 0, 1, 1, 1, 0>, 256, "wg256 ahead1 unroll1 occ"},
    {k_score<256, 0, 2, 2, 1, 0>, 256, "wg256 ahead2 unroll2 occ"},
    {k_score<256, 0, 4, 4, 1, 0>, 256, "wg256 ahead4 unroll4 occ"},
    {k_score<256, 0, 2, 2, 1, 16>, 256, "wg256 ahead2 unroll2 occ dyn16"},
    {k_score<512, 128, 2, 2, 1, 0>, 512, "wg512 lds128 ahead2 unroll2 occ"},
    {k_score<1024, 256, 4, 4, 1, 0>, 1024, "wg1024 lds256 ahead4 unroll4 occ"},
    {k_score<1024, 256, 1, 1, 0, 0>, 1024, "wg1024 lds256 ahead1 unroll1"},
    {k_score<256, 0, 1, 4, 1, 0>, 256, "wg256 ahead1 unroll4 occ"},
    {k_score<256, 0, 4, 1, 0, 0>, 256, "wg256 ahead4 unroll1"},
    {k_score<256, 0, 2, 1, 0, 16>, 256, "wg256 ahead2 unroll1 dyn16"},
    {k_score<512, 0, 2, 2, 0, 0>, 512, "wg512 ahead2 unroll2"},
    {k_score<256, 0, 2, 1, 0, 4>, 256, "wg256 ahead2 unroll1 dyn4"},
    {k_score<256, 0, 1, 1, 0, 16>, 256, "wg256 ahead1 unroll1 dyn16"},
    {k_score<256, 0, 4, 1, 0, 16>, 256, "wg256 ahead4 unroll1 dyn16"},
    {k_score_batch<256, 16, 2, 1, 0>, 256, "batch wg256 head16 unroll2 occ"},
    {k_score_batch<256, 16, 1, 0, 16>, 256, "batch wg256 head16 unroll1 dyn16"},
    {k_score_batch<256, 16, 1, 0, 4>, 256, "batch wg256 head16 unroll1 dyn4"},
    {k_score_batch<256, 24, 1, 0, 16>, 256, "batch wg256 head24 unroll1 dyn16"},
    {k_score_batch<256, 32, 1, 0, 16>, 256, "batch wg256 head32 unroll1 dyn16"},
    {k_score_batch<256, 8, 1, 0, 16>, 256, "batch wg256 head8 unroll1 dyn16"},
    {k_score_batch<256, 16, 2, 0, 16>, 256, "batch wg256 head16 unroll2 dyn16"},
    {k_score_batch<512, 16, 1, 0, 16>, 512, "batch wg512 head16 unroll1 dyn16"},
    {k_score_fast<256, 8, 1, 16, 0>, 256, "fast wg256 head8 unroll1 dyn16", 1},
    {k_score_fast<256, 8, 2, 16, 0>, 256, "fast wg256 head8 unroll2 dyn16", 1},
    {k_score_fast<256, 4, 1, 16, 0>, 256, "fast wg256 head4 unroll1 dyn16", 1},
    {k_score_fast<256, 4, 2, 16, 0>, 256, "fast wg256 head4 unroll2 dyn16", 1},
    {k_score_fast<256, 8, 1, 4, 0>, 256, "fast wg256 head8 unroll1 dyn4", 1},
    {k_score_fast<512, 8, 2, 16, 0>, 512, "fast wg512 head8 unroll2 dyn16", 1},
    {k_score_fast<256, 4, 1, 16, 1>, 256, "fast wg256 head4 unroll1 dyn16 coarse", 1},
    {k_score_fast<256, 4, 2, 16, 1>, 256, "fast wg256 head4 unroll2 dyn16 coarse", 1},
    {k_score_fast<256, 8, 1, 16, 1>, 256, "fast wg256 head8 unroll1 dyn16 coarse", 1},
    {k_score_fast<256, 8, 2, 16, 1>, 256, "fast wg256 head8 unroll2 dyn16 coarse", 1},
    {k_score_fast<256, 6, 2, 16, 1>, 256, "fast wg256 head6 unroll2 dyn16 coarse", 1},
    {k_score_fast<512, 4, 2, 16, 1>, 512, "fast wg512 head4 unroll2 dyn16 coarse", 1},
};
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));
int g_resident[kNumVariants];   // workgroups per CU, from the occupancy query
int g_num_cu = 0;

__global__ void k_zero(unsigned *w) { *w = 0u; }

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

int score_variants() { return kNumVariants; }

const char *score_variant_name(int v) {
  return v >= 0 && v < kNumVariants ? kVariants[v].name : "";
}

void launch_score(const Params &p, PointsDev pts, ToolDev t, GridDev g, int64_t n, int variant,
                  unsigned *work, hipStream_t s) {
  int32_t mw = (t.K + 63) / 64;
  if (n <= 0) return;
  if (variant < 0 || variant >= kNumVariants) variant = 0;
  if (kVariants[variant].needs_lds_k && t.K > kLdsK) variant = 0;
  const ScoreVariant &v = kVariants[variant];
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess ||
        g_num_cu <= 0)
      g_num_cu = 256;
  }
  if (g_resident[variant] == 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, v.fn, v.threads, 0) != hipSuccess ||
        per_cu <= 0)
      per_cu = 1;
    g_resident[variant] = per_cu;
  }
  const int64_t nw = v.threads / 64;
  int64_t wg = (int64_t)g_resident[variant] * g_num_cu;
  int64_t need = (n + nw - 1) / nw;
  if (wg > need) wg = need;
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(1), 0, s, work);
  hipLaunchKernelGGL(v.fn, dim3((unsigned)wg), dim3(v.threads), 0, s, p, pts, t, g, n, mw, work);
}

}  // namespace af
