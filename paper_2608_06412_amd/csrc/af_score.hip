// Scoring kernels (Sections 3.4 and 3.5): PCA normals, candidate-direction
// masks and the per-point collision-count search over the rotated kernels.
#include "af_internal.h"

#include <algorithm>
#include <cstring>
#include <utility>
#include <vector>

#pragma clang fp contract(off)

namespace af {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Neighbour window [-3, 3]^3 as (dx, dy, dz, |d|^2), sorted by |d|^2.
__constant__ int8_t c_nb[343 * 4];

// The same window as a compile-time table, shell by shell, and inside a
// shell in ascending (dz, dy, dx) order: the order in which the kNN takes
// voxels tied at the same distance.
struct NbOrder {
  int8_t e[343][4];
};
constexpr NbOrder make_nb_order() {
  NbOrder o{};
  int n = 0;
  for (int d2 = 0; d2 <= 27; ++d2)
    for (int z = -3; z <= 3; ++z)
      for (int y = -3; y <= 3; ++y)
        for (int x = -3; x <= 3; ++x)
          if (x * x + y * y + z * z == d2) {
            o.e[n][0] = (int8_t)x;
            o.e[n][1] = (int8_t)y;
            o.e[n][2] = (int8_t)z;
            o.e[n][3] = (int8_t)d2;
            ++n;
          }
  return o;
}
constexpr NbOrder kNbOrder = make_nb_order();

// Shell boundaries of that table: shell s is entries [start[s], start[s + 1]).
struct NbShells {
  int n;
  int start[29];
};
constexpr NbShells make_nb_shells() {
  NbShells sh{};
  for (int j = 0; j < 343; ++j)
    if (j == 0 || kNbOrder.e[j][3] != kNbOrder.e[j - 1][3]) sh.start[sh.n++] = j;
  sh.start[sh.n] = 343;
  return sh;
}
constexpr NbShells kNbShells = make_nb_shells();

// Window accumulation from the 7 slices: one entry (compile-time offsets).
struct NbSums {
  int cnt;
  int sx[3], sxx[6];
};
template <int J>
__device__ inline void nb_entry(const uint64_t (&slice)[7], NbSums &a, int k) {
  constexpr int dx = kNbOrder.e[J][0], dy = kNbOrder.e[J][1], dz = kNbOrder.e[J][2];
  const int h = (int)((slice[dz + 3] >> (7 * (dy + 3) + dx + 3)) & 1u) & (a.cnt < k ? 1 : 0);
  a.cnt += h;
  a.sx[0] += dx * h; a.sx[1] += dy * h; a.sx[2] += dz * h;
  a.sxx[0] += dx * dx * h; a.sxx[1] += dx * dy * h; a.sxx[2] += dx * dz * h;
  a.sxx[3] += dy * dy * h; a.sxx[4] += dy * dz * h; a.sxx[5] += dz * dz * h;
}
template <int Lo, int... I>
__device__ inline void nb_range(std::integer_sequence<int, I...>, const uint64_t (&slice)[7],
                                NbSums &a, int k) {
  (nb_entry<Lo + I>(slice, a, k), ...);
}
// Shells S, S+1, ... until k voxels are taken (the last shell's voxels in
// table order, so ties at the k-th distance go to the lowest (dz, dy, dx)).
template <int S>
__device__ inline void nb_shells(const uint64_t (&slice)[7], NbSums &a, int k) {
  constexpr int lo = kNbShells.start[S], hi = kNbShells.start[S + 1];
  nb_range<lo>(std::make_integer_sequence<int, hi - lo>{}, slice, a, k);
  if constexpr (S + 1 < kNbShells.n) {
    if (a.cnt < k) nb_shells<S + 1>(slice, a, k);
  }
}

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

// Least principal axis of a neighbourhood from its moments: cnt voxels, sum
// d, sum dd^T (00 01 02 11 12 22).  The scatter M = cnt sum(dd^T) -
// (sum d)(sum d)^T is exact in integers; its eigenvectors come from cyclic
// Jacobi in fp64 (Golub & Van Loan's cyclic Jacobi method: eight sweeps over
// the pairs (0,1), (0,2), (1,2), a pair with a zero off-diagonal entry
// skipped, each rotation the 2x2 symmetric Schur decomposition with
// t = sign(theta) / (|theta| + sqrt(theta^2 + 1))), and the axis is the
// rotation product's column at the smallest diagonal entry (ties: lowest
// index), rounded to fixed point 2^30.  Only IEEE basic operations, with
// contraction off, in a fixed order, so the result is the same on any IEEE
// machine.  Returns 0 (no axis) with fewer than 3 voxels.
__device__ inline int pca_axis(int cnt, const int32_t sx[3], const int32_t sxx[6],
                               int64_t axis[3]) {
  axis[0] = axis[1] = axis[2] = 0;
  if (cnt < 3) return 0;
  const int64_t c = cnt;
  double a00 = (double)(c * sxx[0] - (int64_t)sx[0] * sx[0]);
  double a01 = (double)(c * sxx[1] - (int64_t)sx[0] * sx[1]);
  double a02 = (double)(c * sxx[2] - (int64_t)sx[0] * sx[2]);
  double a11 = (double)(c * sxx[3] - (int64_t)sx[1] * sx[1]);
  double a12 = (double)(c * sxx[4] - (int64_t)sx[1] * sx[2]);
  double a22 = (double)(c * sxx[5] - (int64_t)sx[2] * sx[2]);
  double v[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  // one plane rotation on (p, q) with r the third index; app, aqq, apq,
  // arp, arq name the entries of A it reads and writes
  auto rotate = [&](double &app, double &aqq, double &apq, double &arp, double &arq, int p,
                    int q) {
    const double b = apq;
    if (b == 0.0) return;
    const double theta = (aqq - app) / (2.0 * b);
    double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
    if (theta < 0.0) t = -t;
    const double cs = 1.0 / sqrt(t * t + 1.0);
    const double sn = t * cs;
    app = app - t * b;
    aqq = aqq + t * b;
    apq = 0.0;
    const double rp = arp, rq = arq;
    arp = cs * rp - sn * rq;
    arq = sn * rp + cs * rq;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double vip = v[i][p], viq = v[i][q];
      v[i][p] = cs * vip - sn * viq;
      v[i][q] = sn * vip + cs * viq;
    }
  };
  for (int sweep = 0; sweep < 8; ++sweep) {
    rotate(a00, a11, a01, a02, a12, 0, 1);   // r = 2: a_20 = a02, a_21 = a12
    rotate(a00, a22, a02, a01, a12, 0, 2);   // r = 1: a_10 = a01, a_12 = a12
    rotate(a11, a22, a12, a01, a02, 1, 2);   // r = 0: a_01 = a01, a_02 = a02
  }
  int best = 0;
  double dmin = a00;
  if (a11 < dmin) { best = 1; dmin = a11; }
  if (a22 < dmin) best = 2;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double e = best == 0 ? v[i][0] : (best == 1 ? v[i][1] : v[i][2]);
    axis[i] = (int64_t)__builtin_rint(e * 1073741824.0);
  }
  return 1;
}

// The least principal axis of point s's neighbourhood (before orientation):
// returns 1 and the axis, or 0 when there is none (fewer than 3 neighbours).
__device__ inline int normal_axis(const Params &p, const GridDev &g, const int32_t s[3],
                                  int64_t axis[3]) {
  // the point's brick and, when it is at least one brick inside the grid,
  // its neighbours' words by brick deltas (no per-voxel bounds test)
  const int bx = (s[0] >> 3) - g.g0[0], by = (s[1] >> 3) - g.g0[1], bz = (s[2] >> 3) - g.g0[2];
  const bool interior = bx >= 1 && by >= 1 && bz >= 1 && bx <= g.gd[0] - 2 &&
                        by <= g.gd[1] - 2 && bz <= g.gd[2] - 2;
  const int gx = g.gd[0], gxy = g.gd[0] * g.gd[1];
  const int b0 = (bz * g.gd[1] + by) * gx + bx;
  const int lx0 = s[0] & 7, ly0 = s[1] & 7, lz0 = s[2] & 7;
  int cnt = 0;
  int sx[3] = {0, 0, 0}, sxx[6] = {0, 0, 0, 0, 0, 0};
  if (interior) {
    // The window's surface bits as seven 49-bit slices (bit 7 (dy + 3) +
    // dx + 3 of slice dz + 3), read up front: per z, up to three 4-row y
    // groups in each of up to two x bricks, 42 independent word loads.
    const int dbxl = (lx0 - 3) >> 3, dbxr = (lx0 + 3) >> 3;
    const int glo = (ly0 - 3) >> 2;
    const int xsh = lx0 - 3 - 8 * dbxl;
    const __amdgpu_buffer_rsrc_t sr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)g.surf, (short)0, (int)((uint32_t)gxy * (uint32_t)g.gd[2] << 6), 0x00020000);
    uint64_t slice[7];
#pragma unroll
    for (int zz = 0; zz < 7; ++zz) {
      const int rz = lz0 + zz - 3;
      const int zb = b0 + ((rz >> 3) == 0 ? 0 : ((rz >> 3) > 0 ? gxy : -gxy));
      const int zw = (rz & 7) << 1;
      uint32_t wl[3], wr[3];
#pragma unroll
      for (int gi = 0; gi < 3; ++gi) {
        const int gg = glo + gi;
        const int yb = zb + ((gg >> 1) == 0 ? 0 : ((gg >> 1) > 0 ? gx : -gx));
        const int w = (gg & 1) | zw;
        wl[gi] = __builtin_amdgcn_raw_buffer_load_b32(sr, ((yb + dbxl) * 16 + w) << 2, 0, 0);
        wr[gi] = __builtin_amdgcn_raw_buffer_load_b32(sr, ((yb + dbxr) * 16 + w) << 2, 0, 0);
      }
      uint64_t sl = 0;
#pragma unroll
      for (int yy = 0; yy < 7; ++yy) {
        const int ry = ly0 + yy - 3;
        const int gi = (ry >> 2) - glo;
        const uint32_t l = gi == 0 ? wl[0] : (gi == 1 ? wl[1] : wl[2]);
        const uint32_t r = gi == 0 ? wr[0] : (gi == 1 ? wr[1] : wr[2]);
        const int yb8 = (ry & 3) << 3;
        const uint32_t v16 = ((l >> yb8) & 0xffu) | (((r >> yb8) & 0xffu) << 8);
        sl |= (uint64_t)((v16 >> xsh) & 0x7fu) << (7 * yy);
      }
      slice[zz] = sl;
    }
    // keep the window reads ahead of the shells (the compiler would sink
    // each slice into the first shell that uses it, serialising the reads)
#pragma unroll
    for (int zz = 0; zz < 7; ++zz) {
      uint32_t lo = (uint32_t)slice[zz], hi = (uint32_t)(slice[zz] >> 32);
      asm volatile("" : "+v"(lo), "+v"(hi));
      slice[zz] = ((uint64_t)hi << 32) | lo;
    }
    // whole shells in order until one ends with k found (ties included)
    NbSums a{};
    nb_shells<0>(slice, a, p.knn_k);
    cnt = a.cnt;
    for (int c = 0; c < 3; ++c) sx[c] = a.sx[c];
    for (int c = 0; c < 6; ++c) sxx[c] = a.sxx[c];
  } else {
    for (int j = 0; j < 343 && cnt < p.knn_k; ++j) {
      int dx = c_nb[4 * j], dy = c_nb[4 * j + 1], dz = c_nb[4 * j + 2];
      if (!surf_bit(g, s[0] + dx, s[1] + dy, s[2] + dz)) continue;
      ++cnt;
      sx[0] += dx; sx[1] += dy; sx[2] += dz;
      sxx[0] += dx * dx; sxx[1] += dx * dy; sxx[2] += dx * dz;
      sxx[3] += dy * dy; sxx[4] += dy * dz; sxx[5] += dz * dz;
    }
  }
  return pca_axis(cnt, sx, sxx, axis);
}

// Orient the axis towards the point's mean sensor position and store it.
__device__ inline void store_normal(const PointsDev &pts, int64_t i, const int32_t s[3],
                                    int has, const int64_t axis[3]) {
  int32_t *nout = pts.normal + 3 * i;
  if (!has) {
    pts.has_normal[i] = 0;
    nout[0] = nout[1] = nout[2] = 0;
    return;
  }
  __int128 gdot = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t ga = pts.sumq[3 * i + a] - (int64_t)pts.nq[i] * (256 * (int64_t)s[a] + 128);
    gdot += (__int128)axis[a] * ga;
  }
  int sgn = gdot < 0 ? -1 : 1;
  for (int a = 0; a < 3; ++a) nout[a] = (int32_t)(sgn * axis[a]);
  pts.has_normal[i] = 1;
}

// Least principal axis of the k nearest surface voxels (ties at the k-th
// distance taken in (dz, dy, dx) order), oriented towards the mean sensor
// position (Section 3.4 "Approach directions").
__global__ void __launch_bounds__(kThreads)
k_normals(Params p, MapDev m, PointsDev pts, GridDev g, int64_t n) {
  // n < 0: the point count on the device (recorded graphs, point lists)
  if (n < 0) n = pts.sel ? (int64_t)*pts.n_sel : (int64_t)*pts.n_points;
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= n) return;
  const int64_t i = pts.sel ? (int64_t)pts.sel[j] : j;
  int32_t addr = pts.addr[i];
  int W = addr >= 0 ? (int)m.W[addr] : 0;
  if (W < p.conf_min_w) {
    pts.has_normal[i] = -1;
    return;
  }
  int32_t s[3];
  unpack_key(pts.key[i], s[0], s[1], s[2]);
  int64_t axis[3];
  const int has = normal_axis(p, g, s, axis);
  store_normal(pts, i, s, has, axis);
}

// Cached normals.  A point's axis depends only on the surface voxels within
// +-3 of it, and surface voxels are only ever added (with new points), so an
// axis changes only for points within +-3 of a point appended since the last
// update.  Those voxels are marked in a bit plane over the brick grid (the
// surf plane's layout), the points on marked voxels are listed and their axes
// recomputed; every other point keeps its axis and is oriented anew (its
// mean sensor position moves whenever it is observed).

// One thread per (row of 7 voxels along x, brick it reaches): SET ors the
// row's bits into the plane, !SET clears the words again.
template <int SET>
__global__ void __launch_bounds__(128) k_normals_mark(PointsDev pts, GridDev g, NormalCache nc,
                                                      int64_t first) {
  const int t = threadIdx.x;
  if (t >= 98) return;
  int32_t s[3];
  unpack_key(pts.key[first + blockIdx.x], s[0], s[1], s[2]);
  const int r = t >> 1, y = s[1] + r % 7 - 3, z = s[2] + r / 7 - 3;
  const int xl = s[0] - 3, xh = s[0] + 3;
  int x0, x1;
  if ((t & 1) == 0) {
    x0 = xl;
    x1 = (xl | 7) < xh ? (xl | 7) : xh;
  } else {
    if ((xl >> 3) == (xh >> 3)) return;
    x0 = xh & ~7;
    x1 = xh;
  }
  const int64_t b = brick_index(g, x0, y, z);
  if (b < 0) return;
  const int row = ((y & 7) << 3) | ((z & 7) << 6);
  uint32_t *w = nc.stale + b * 16 + (row >> 5);
  if (SET)
    atomicOr(w, ((1u << (x1 - x0 + 1)) - 1u) << ((row & 31) + (x0 & 7)));
  else
    *w = 0u;
}

__global__ void __launch_bounds__(kThreads) k_normals_reset(NormalCache nc, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) nc.state[i] = -2;
}

// Every point: confidence gate; a confident point on a marked voxel, or one
// whose axis is pending, is listed (one list append per workgroup); any other
// confident point is oriented from its cached axis.
constexpr int kOrientThreads = 1024;
__global__ void __launch_bounds__(kOrientThreads)
k_normals_orient(Params p, MapDev m, PointsDev pts, GridDev g, NormalCache nc, int64_t n,
                 int marked) {
  __shared__ int part[kOrientThreads / 64 + 1];
  const int64_t i = (int64_t)blockIdx.x * kOrientThreads + threadIdx.x;
  bool take = false;
  if (i < n) {
    const int32_t addr = pts.addr[i];
    const bool conf = (addr >= 0 ? (int)m.W[addr] : 0) >= p.conf_min_w;
    int32_t s[3];
    unpack_key(pts.key[i], s[0], s[1], s[2]);
    bool stale = nc.state[i] == -2;
    if (marked && !stale) {
      const int64_t b = brick_index(g, s[0], s[1], s[2]);
      const int lin = (s[0] & 7) | ((s[1] & 7) << 3) | ((s[2] & 7) << 6);
      stale = b >= 0 && ((nc.stale[b * 16 + (lin >> 5)] >> (lin & 31)) & 1u);
    }
    if (!conf) {
      if (stale) nc.state[i] = -2;
      pts.has_normal[i] = -1;
    } else if (stale) {
      take = true;
    } else {
      const int64_t axis[3] = {nc.axis[3 * i], nc.axis[3 * i + 1], nc.axis[3 * i + 2]};
      store_normal(pts, i, s, nc.state[i] == 1, axis);
    }
  }
  const uint64_t bal = __ballot(take);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kOrientThreads / 64; ++w) {
      const int c = part[w];
      part[w] = t;
      t += c;
    }
    part[kOrientThreads / 64] = t ? atomicAdd(nc.count, t) : 0;
  }
  __syncthreads();
  if (take)
    nc.list[part[kOrientThreads / 64] + part[wave] + __popcll(bal & ((1ull << lane) - 1ull))] =
        (int32_t)i;
}

// Listed (confident) points: recompute, cache and orient the axis.
__global__ void __launch_bounds__(kThreads)
k_normals_axis(Params p, PointsDev pts, GridDev g, NormalCache nc) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= *nc.count) return;
  const int32_t i = nc.list[j];
  int32_t s[3];
  unpack_key(pts.key[i], s[0], s[1], s[2]);
  int64_t axis[3] = {0, 0, 0};
  const int has = normal_axis(p, g, s, axis);
  for (int a = 0; a < 3; ++a) nc.axis[3 * (int64_t)i + a] = axis[a];
  nc.state[i] = has;
  store_normal(pts, i, s, has, axis);
}

// ---------------------------------------------------------------------------
// Grid-relative lookups.  The grid keeps a margin of bricks around every
// allocated block that is wider than any table offset, so a lookup needs no
// bounds test.  A point is its linear brick index Bp plus its in-brick
// position rp = rx | ry << 4 | rz << 8; an entry is its brick delta plus its
// in-brick offset o7 in the same 4-bit fields.  One add gives rp + o7, whose
// bits 3, 7 and 11 are the per-axis brick carries and whose other bits are
// the target voxel's in-brick coordinates.  The word is read through a buffer
// resource over the grid (a stray offset reads 0 instead of faulting).
struct SwFrame {
  uint32_t Bp, rp;
};

struct SwGrid {
  __amdgpu_buffer_rsrc_t pred, occ1;
  uint32_t gx, gxy, nbricks;
  const uint32_t *occ_any;
};

__device__ inline SwGrid sw_grid(const GridDev &g) {
  SwGrid q;
  q.gx = (uint32_t)g.gd[0];
  q.gxy = (uint32_t)g.gd[0] * (uint32_t)g.gd[1];
  q.nbricks = q.gxy * (uint32_t)g.gd[2];
  q.pred = __builtin_amdgcn_make_buffer_rsrc((void *)g.pred, (short)0, (int)(q.nbricks << 7),
                                             0x00020000);
  q.occ1 = __builtin_amdgcn_make_buffer_rsrc((void *)g.occ1, (short)0, (int)(q.nbricks << 6),
                                             0x00020000);
  q.occ_any = g.occ_any;
  return q;
}

__device__ inline SwFrame sw_frame(const GridDev &g, const SwGrid &q, const int32_t s[3]) {
  const uint32_t bx = (uint32_t)((s[0] >> 3) - g.g0[0]);
  const uint32_t by = (uint32_t)((s[1] >> 3) - g.g0[1]);
  const uint32_t bz = (uint32_t)((s[2] >> 3) - g.g0[2]);
  SwFrame f;
  f.Bp = bx + q.gx * by + q.gxy * bz;
  f.rp = (uint32_t)(s[0] & 7) | ((uint32_t)(s[1] & 7) << 4) | ((uint32_t)(s[2] & 7) << 8);
  return f;
}

// The byte offset of an entry's 2-bit code word, and the code's bit position.
__device__ inline uint32_t code_sw_at(const SwGrid &q, const SwFrame &f, uint2 xe, uint32_t &bit) {
  const uint32_t tt = f.rp + xe.y;
  uint32_t brick = f.Bp + xe.x + ((tt >> 3) & 1u);
  brick += ((tt >> 7) & 1u) * q.gx;
  brick += ((tt >> 11) & 1u) * q.gxy;
  const uint32_t wib = ((tt >> 5) & 3u) | ((tt >> 6) & 0x1cu);   // (ly >> 1) | lz << 2
  bit = ((tt & 7u) << 1) | (tt & 0x10u);                          // 2 (lx + 8 (ly & 1))
  return ((brick << 5) | wib) << 2;
}

__device__ inline uint32_t code_sw(const SwGrid &q, const SwFrame &f, uint2 xe) {
  const uint32_t tt = f.rp + xe.y;
  uint32_t brick = f.Bp + xe.x + ((tt >> 3) & 1u);
  brick += ((tt >> 7) & 1u) * q.gx;
  brick += ((tt >> 11) & 1u) * q.gxy;
  const uint32_t wib = ((tt >> 5) & 3u) | ((tt >> 6) & 0x1cu);   // (ly >> 1) | lz << 2
  const uint32_t bit = ((tt & 7u) << 1) | (tt & 0x10u);          // 2 (lx + 8 (ly & 1))
  const uint32_t w =
      __builtin_amdgcn_raw_buffer_load_b32(q.pred, ((brick << 5) | wib) << 2, 0, 0);
  return (w >> bit) & 3u;
}

// Body and corridor entries only need "TSDF < r_c": one bit per voxel, so a
// whole brick is 64 bytes.
__device__ inline uint32_t occ_bit_sw(const SwGrid &q, const SwFrame &f, uint2 xe) {
  const uint32_t tt = f.rp + xe.y;
  uint32_t brick = f.Bp + xe.x + ((tt >> 3) & 1u);
  brick += ((tt >> 7) & 1u) * q.gx;
  brick += ((tt >> 11) & 1u) * q.gxy;
  const uint32_t wib = ((tt >> 6) & 1u) | ((tt >> 7) & 0xeu);   // (ly >> 2) | lz << 1
  const uint32_t bit = (tt & 7u) | ((tt >> 1) & 0x18u);          // lx | (ly & 3) << 3
  const uint32_t w =
      __builtin_amdgcn_raw_buffer_load_b32(q.occ1, ((brick << 4) | wib) << 2, 0, 0);
  return (w >> bit) & 1u;
}

__device__ inline uint32_t sw_cls(uint2 xe) { return xe.y >> 30; }

__device__ inline bool sw_hits(uint2 xe, uint32_t code) {
  return sw_cls(xe) == AF_CLS_NEAR ? code != 0u : (code & 1u) != 0u;
}

// The 4-byte grid-independent entry form: per axis a 10-bit field
// r + o + 256 (r the point's in-brick coordinate, |o| <= 255), so one add of
// the point's fields to the entry gives, per axis, the brick offset + 32 in
// bits 3-9 and the target's in-brick coordinate in bits 0-2 of each field.
// Bp carries the -32 bias of all three axes.
__device__ inline SwFrame rel_frame(const GridDev &g, const SwGrid &q, const int32_t s[3]) {
  const uint32_t bx = (uint32_t)((s[0] >> 3) - g.g0[0]);
  const uint32_t by = (uint32_t)((s[1] >> 3) - g.g0[1]);
  const uint32_t bz = (uint32_t)((s[2] >> 3) - g.g0[2]);
  SwFrame f;
  f.Bp = bx + q.gx * by + q.gxy * bz - 32u * (1u + q.gx + q.gxy);
  f.rp = (uint32_t)(s[0] & 7) | ((uint32_t)(s[1] & 7) << 10) | ((uint32_t)(s[2] & 7) << 20);
  return f;
}

__device__ inline uint32_t rel_brick(const SwGrid &q, const SwFrame &f, uint32_t tt) {
  // 24-bit multiplies: every grid axis spans at least 9 bricks and the grid
  // holds fewer than 2^25 bricks, so gx and gxy stay below 2^22
  return f.Bp + ((tt >> 3) & 127u) + __umul24(q.gx, (tt >> 13) & 127u) +
         __umul24(q.gxy, (tt >> 23) & 127u);
}

__device__ inline uint32_t code_rel(const SwGrid &q, const SwFrame &f, uint32_t e) {
  const uint32_t tt = f.rp + e;
  const uint32_t brick = rel_brick(q, f, tt);
  const uint32_t wib = ((tt >> 11) & 3u) | ((tt >> 18) & 0x1cu);   // (ly >> 1) | lz << 2
  const uint32_t bit = ((tt & 7u) << 1) | ((tt >> 6) & 0x10u);     // 2 (lx + 8 (ly & 1))
  const uint32_t w =
      __builtin_amdgcn_raw_buffer_load_b32(q.pred, ((brick << 5) | wib) << 2, 0, 0);
  return (w >> bit) & 3u;
}

// The plane's words hold bit lx + 8 (ly & 3) of word (ly >> 2) + 2 lz, so
// (little-endian) voxel (lx, ly, lz) is bit lx of byte ly + 8 lz of the
// brick's 64 bytes: one byte read, fewer address operations.
__device__ inline uint32_t occ_rel(const SwGrid &q, const SwFrame &f, uint32_t e) {
  const uint32_t tt = f.rp + e;
  const uint32_t brick = rel_brick(q, f, tt);
  const uint32_t byte = ((tt >> 10) & 7u) | ((tt >> 17) & 0x38u);  // ly + 8 lz
  const uint32_t w = __builtin_amdgcn_raw_buffer_load_b8(q.occ1, (brick << 6) | byte, 0, 0);
  return (w >> (tt & 7u)) & 1u;
}

// Uniform access to the two entry forms (RE: the 4-byte form).
template <int RE> struct EntryOf { using T = uint2; };
template <> struct EntryOf<1> { using T = uint32_t; };

template <int RE>
__device__ inline typename EntryOf<RE>::T load_entry(const ToolDev &t, uint32_t idx) {
  // a 32-bit byte offset from the table's base: one vector register per
  // address instead of a 64-bit pointer per lane
  if constexpr (RE)
    return *(const uint32_t *)((const char *)t.rent + (uint32_t)(idx << 2));
  else
    return t.xent[idx];
}
__device__ inline uint32_t ent_cls(uint2 xe) { return xe.y >> 30; }
__device__ inline uint32_t ent_cls(uint32_t e) { return e >> 30; }
template <int B1>
__device__ inline uint32_t ent_code(const SwGrid &q, const SwFrame &f, uint2 xe) {
  return B1 ? occ_bit_sw(q, f, xe) : code_sw(q, f, xe);
}
template <int B1>
__device__ inline uint32_t ent_code(const SwGrid &q, const SwFrame &f, uint32_t e) {
  return B1 ? occ_rel(q, f, e) : code_rel(q, f, e);
}

// Candidate masks (Section 3.4 "Approach directions"): one lane per point,
// its normal and viewpoint vectors in registers (fp64, exact conversions of
// integers).  For every candidate direction the lane also reads the
// direction's three arm samples (Section 3.4 "Arm path checking"; they depend
// on the approach direction only, so orientations that share it share the
// result) and records which one hits first, as two bit planes per mask word.
// An orientation that shares its predecessor's approach direction takes its
// candidate bit and arm-sample result, so only heads (orientations with a
// direction of their own) are evaluated, each head's result covering its run.
//
// MW mask words (from word w0 of mw) per launch, with the heads walked per
// lane: each lane first tests the normal cone of every head (wave-uniform
// directions), then visits only its own heads inside the cone, in any word,
// so the observation test and the arm samples run on as many heads as the
// wave's busiest lane has in its cone (consecutive heads of a direction set
// often share a band of the sphere, so one word can hold all of one lane's
// cone and none of its neighbour's).  The heads' directions, arm entries and
// runs are staged in LDS once per workgroup; each lane's words collect there,
// and the carries across words (orientations before a word's first head) are
// applied afterwards, in word order.  The rows of a workgroup's points are
// then written out together (a lane's own words are 8 bytes at a 96-byte
// stride, which the memory system would write back as partial lines).  A
// launch after the first takes its carry-in from the last orientation of word
// w0 - 1 as the previous launch wrote it: that orientation belongs to the run
// of the last head before word w0, so it holds that head's candidate bit and
// arm-sample result (every word but the last is full).
template <int MW>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_mask_walk(Params p, PointsDev pts, ToolDev t, GridDev g, int64_t n, int w0, int mw) {
  // n < 0: the point count on the device (recorded graphs, point lists)
  if (n < 0) n = pts.sel ? (int64_t)*pts.n_sel : (int64_t)*pts.n_points;
  if ((int64_t)blockIdx.x * kThreads >= n) return;   // whole workgroup past the end
  __shared__ double s_dir[3][64 * MW];
  __shared__ uint2 s_arm[3][64 * MW];
  __shared__ uint64_t s_run[64 * MW];
  __shared__ uint64_t s_word[3][MW][kThreads];   // candidate word, plane 0, plane 1
  for (int k = threadIdx.x; k < 64 * MW; k += kThreads) {
    const int w = w0 + (k >> 6), j = k & 63;
    const int kend = t.K - 64 * w < 64 ? t.K - 64 * w : 64;
    uint64_t run = 0ull;
    if (j < kend) {
      const uint64_t valid = kend == 64 ? ~0ull : ((1ull << kend) - 1ull);
      const uint64_t heads = ~t.same[w] & valid;
      const double *R = t.rot + 9 * (int64_t)(64 * w + j);
      s_dir[0][k] = R[0];
      s_dir[1][k] = R[3];
      s_dir[2][k] = R[6];
      const uint32_t b = t.begin[64 * w + j];
#pragma unroll
      for (int a = 0; a < 3; ++a) s_arm[a][k] = t.xent[b + a];
      if ((heads >> j) & 1ull) {
        const uint64_t above = j == 63 ? 0ull : heads & ~((2ull << j) - 1ull);
        run = (above ? (above & (~above + 1ull)) - 1ull : valid) & ~((1ull << j) - 1ull);
      }
    }
    s_run[k] = run;
  }
#pragma unroll
  for (int w = 0; w < MW; ++w)
#pragma unroll
    for (int c = 0; c < 3; ++c) s_word[c][w][threadIdx.x] = 0ull;
  const int64_t jj = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool act = jj < n;
  const int64_t i = pts.sel ? (act ? (int64_t)pts.sel[jj] : 0) : jj;
  const int hn = act ? pts.has_normal[i] : -1;
  double n0 = 0, n1 = 0, n2 = 0, nn = 0;
  double wx[kMaxVp], wy[kMaxVp], wz[kMaxVp], ww[kMaxVp];
  int nv = 0;
  SwFrame f;
  f.Bp = f.rp = 0u;
  const SwGrid q = sw_grid(g);
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
    f = sw_frame(g, q, s);
  } else {
#pragma unroll
    for (int j = 0; j < kMaxVp; ++j) wx[j] = wy[j] = wz[j] = ww[j] = 0.0;
  }
  // normal cone of every head
  uint64_t cone[MW];
#pragma unroll
  for (int w = 0; w < MW; ++w) {
    const int kend = t.K - 64 * (w0 + w) < 64 ? t.K - 64 * (w0 + w) : 64;
    const uint64_t valid = kend == 64 ? ~0ull : ((1ull << kend) - 1ull);
    const uint64_t heads = ~t.same[w0 + w] & valid;
    cone[w] = hn == 0 ? heads : 0ull;
    if (hn > 0) {
      for (uint64_t rem = heads; rem; rem &= rem - 1ull) {
        const int j = __ffsll((unsigned long long)rem) - 1;
        const double *R = t.rot + 9 * (int64_t)(64 * (w0 + w) + j);
        const double d0 = R[0], d1 = R[3], d2 = R[6];
        const double dot = (n0 * d0 + n1 * d1) + n2 * d2;
        if (dot >= 0.0 && dot * dot >= p.cos2 * nn) cone[w] |= 1ull << j;
      }
    }
  }
  __syncthreads();
  // A head's arm-sample words are requested in its iteration and decoded in
  // the next one, so their latency overlaps the next head's tests.
  uint32_t pw[3] = {0u, 0u, 0u}, pb[3] = {0u, 0u, 0u};
  uint64_t prun = 0ull;   // run of the head whose words are in flight (0: none)
  int pword = 0;          // its word
  auto settle = [&]() {
    if (!prun) return;
    const uint32_t r = ((pw[0] >> pb[0]) & 3u) ? 1u
                       : ((pw[1] >> pb[1]) & 3u) ? 2u
                       : ((pw[2] >> pb[2]) & 3u) ? 3u
                                                 : 0u;
    if (r & 1u) s_word[1][pword][threadIdx.x] |= prun;
    if (r >> 1) s_word[2][pword][threadIdx.x] |= prun;
  };
  int cw = 0;
  uint64_t rem = cone[0];
  for (;;) {
    // the lane's next head inside the cone, in word order
    while (!rem && cw < MW - 1) {
      ++cw;
#pragma unroll
      for (int u = 1; u < MW; ++u)
        if (u == cw) rem = cone[u];
    }
    if (!__any(rem != 0ull)) break;
    uint32_t cw3[3] = {0u, 0u, 0u}, cb[3] = {0u, 0u, 0u};
    uint64_t run = 0ull;
    if (rem) {
      const int k = 64 * cw + __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1ull;
      const double d0 = s_dir[0][k], d1 = s_dir[1][k], d2 = s_dir[2][k];
      bool seen = false;
#pragma unroll
      for (int v = 0; v < kMaxVp; ++v) {
        if (v < nv && !seen) {
          double wd = (wx[v] * d0 + wy[v] * d1) + wz[v] * d2;
          seen = wd > 0.0 && wd * wd > p.obs2 * ww[v];
        }
      }
      if (seen) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
          cw3[a] = __builtin_amdgcn_raw_buffer_load_b32(q.pred, code_sw_at(q, f, s_arm[a][k], cb[a]),
                                                        0, 0);
        run = s_run[k];
        s_word[0][cw][threadIdx.x] |= run;
      }
    }
    settle();   // the previous head's words, requested an iteration ago
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pw[a] = cw3[a];
      pb[a] = cb[a];
    }
    prun = run;
    pword = cw;
  }
  settle();
  // carries across words: orientations before a word's first head take the
  // candidate bit and arm-sample result of the last head before them
  unsigned long long cand = 0;
  bool ok = false;
  uint32_t nb = 0u;
  if (w0 > 0 && act) {
    ok = (t.mask[i * mw + w0 - 1] >> 63) != 0ull;
    nb = (uint32_t)(t.nearp[i * 2 * mw + w0 - 1] >> 63) |
         ((uint32_t)(t.nearp[i * 2 * mw + mw + w0 - 1] >> 63) << 1);
  }
#pragma unroll
  for (int w = 0; w < MW; ++w) {
    const int kend = t.K - 64 * (w0 + w) < 64 ? t.K - 64 * (w0 + w) : 64;
    const uint64_t valid = kend == 64 ? ~0ull : ((1ull << kend) - 1ull);
    const uint64_t heads = ~t.same[w0 + w] & valid;
    const uint64_t carry = heads ? ((heads & (~heads + 1ull)) - 1ull) : valid;
    uint64_t word = s_word[0][w][threadIdx.x] | (ok ? carry : 0ull);
    uint64_t pl0 = s_word[1][w][threadIdx.x] | ((nb & 1u) ? carry : 0ull);
    uint64_t pl1 = s_word[2][w][threadIdx.x] | ((nb >> 1) ? carry : 0ull);
    if (heads) {
      const int jl = 63 - __clzll((long long)heads);   // the word's last head
      ok = (word >> jl) & 1ull;
      nb = (uint32_t)((pl0 >> jl) & 1ull) | ((uint32_t)((pl1 >> jl) & 1ull) << 1);
    }
    if (pts.sel) {
      if (act) {
        t.mask[i * mw + w0 + w] = word;
        t.nearp[i * 2 * mw + w0 + w] = pl0;
        t.nearp[i * 2 * mw + mw + w0 + w] = pl1;
      }
    } else {
      s_word[0][w][threadIdx.x] = word;
      s_word[1][w][threadIdx.x] = pl0;
      s_word[2][w][threadIdx.x] = pl1;
    }
    cand += (unsigned long long)__popcll(word);
  }
  if (!pts.sel) {
    // rows of consecutive points are contiguous: written out together
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kThreads;
    const int np = n - i0 < kThreads ? (int)(n - i0) : kThreads;
    if (MW == mw) {
      for (int k = threadIdx.x; k < np * MW; k += kThreads)
        t.mask[i0 * MW + k] = s_word[0][k % MW][k / MW];
      for (int k = threadIdx.x; k < np * 2 * MW; k += kThreads) {
        const int r = k / (2 * MW), c = k % (2 * MW);
        t.nearp[i0 * 2 * MW + k] = c < MW ? s_word[1][c][r] : s_word[2][c - MW][r];
      }
    } else {   // this launch's words of each row
      for (int k = threadIdx.x; k < np * MW; k += kThreads) {
        const int r = k / MW, c = k % MW;
        t.mask[(i0 + r) * mw + w0 + c] = s_word[0][c][r];
        t.nearp[(i0 + r) * 2 * mw + w0 + c] = s_word[1][c][r];
        t.nearp[(i0 + r) * 2 * mw + mw + w0 + c] = s_word[2][c][r];
      }
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    unsigned lo = __shfl_xor((unsigned)(cand & 0xffffffffu), off);
    unsigned hi = __shfl_xor((unsigned)(cand >> 32), off);
    cand += ((unsigned long long)hi << 32) | lo;
  }
  if (lane_id() == 0 && cand)
    atomicAdd(&t.counters->s[(blockIdx.x * kWaves + (threadIdx.x >> 6)) % kStatSlots]
                   .candidate_tests,
              cand);
}

// Position of the r-th (1-based) set bit of m, or 64.
__device__ inline int nth_bit(uint64_t m, int r) {
  if (__popcll(m) < r) return 64;
  for (int i = 1; i < r; ++i) m &= m - 1;
  return __ffsll((long long)m) - 1;
}

constexpr int kLdsK = 256;    // orientations whose table heads the "swar" kernels stage in LDS
constexpr int kNearK = 1024;  // orientations whose table offsets the "near" kernels stage in LDS
constexpr int kLfK = 256;     // orientations whose first entries the "lds1" configurations stage

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
  if (n < 0) n = *pts.n_points;   // the point count on the device (recorded graphs)
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
  ScoreCounterBlock &sc = t.counters->s[(blockIdx.x * NW + (threadIdx.x >> 6)) % kStatSlots];
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
    if (conf) atomicAdd(&sc.n_confident, (unsigned long long)conf);
    if (acc) atomicAdd(&sc.n_accessible, (unsigned long long)acc);
    if (blk) atomicAdd(&sc.n_blocked, (unsigned long long)blk);
    if (nocand) atomicAdd(&sc.n_no_candidate, (unsigned long long)nocand);
    if (tests) atomicAdd(&sc.canonical_tests, (unsigned long long)tests);
    if (lookups) atomicAdd(&sc.canonical_lookups, (unsigned long long)lookups);
  }
}

// Sum over the lanes in m of a per-lane value below 16 held as four ballots
// of its bits.
__device__ inline uint32_t plane_sum(const uint64_t pl[4], uint64_t m) {
  return (uint32_t)__popcll(pl[0] & m) + 2u * (uint32_t)__popcll(pl[1] & m) +
         4u * (uint32_t)__popcll(pl[2] & m) + 8u * (uint32_t)__popcll(pl[3] & m);
}

// Lanes over entries [b, e) of one orientation, 64 per step, the next step's
// entries loaded while this step's voxel words are gathered.  B1: the
// entries are body or corridor entries only (no arm samples), read from the
// one-bit plane.  RE: the 4-byte entry form.
// With `first` (UN = 1), the first step's entries were already read by the
// caller (entry min(b + lane, any index of the orientation): lanes past e are
// masked out below).  CL: 0 entries of any class, 1 body entries only (a
// table lists body entries before corridor entries), 2 corridor entries only.
template <int UN, int B1, int RE, int CL = 0, int LZ = 0>
__device__ inline bool scan_fine_sw(const Params &p, const ToolDev &t, const SwGrid &q,
                                    const SwFrame &f, uint32_t b, uint32_t e, int &body,
                                    uint32_t &lookups, uint32_t &steps,
                                    const typename EntryOf<RE>::T *first = nullptr) {
  using Ent = typename EntryOf<RE>::T;
  if (b >= e) return true;
  const uint32_t lane = (uint32_t)lane_id();
  Ent ent[UN];
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    const uint32_t idx = b + 64 * u + lane;
    if (UN == 1 && first)
      ent[u] = *first;
    else
      ent[u] = load_entry<RE>(t, idx < e ? idx : e - 1);
  }
  // LZ: lookups and steps are added once, when the scan ends (a completed
  // range counts e - b lookups; a stop counts those before it plus stop + 1)
  for (uint32_t base = b; base < e; base += 64 * UN) {
    if (!LZ) ++steps;
    uint32_t code[UN];
    Ent nxt[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) code[u] = ent_code<B1>(q, f, ent[u]);
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const uint32_t idx = base + 64 * (UN + u) + lane;
      nxt[u] = load_entry<RE>(t, idx < e ? idx : e - 1);
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const uint32_t cb = base + 64 * u;
      uint64_t nf, bm;
      if (CL == 0) {
        const uint32_t cls = ent_cls(ent[u]);
        const bool hit = cb + lane < e &&
                         (B1 || cls != AF_CLS_NEAR ? (code[u] & 1u) != 0u : code[u] != 0u);
        nf = __ballot(hit && cls != AF_CLS_BODY);
        bm = __ballot(hit && cls == AF_CLS_BODY);
      } else {
        const uint64_t hm = __ballot(cb + lane < e && (code[u] & 1u) != 0u);
        nf = CL == 2 ? hm : 0ull;
        bm = CL == 1 ? hm : 0ull;
      }
      if (cb >= e) break;
      const int stop = CL == 1   ? nth_bit(bm, p.n_c - body)
                       : CL == 2 ? (nf ? __ffsll((long long)nf) - 1 : 64)
                                 : chunk_stop(nf, bm, p.n_c - body);
      if (stop < 64) {
        if (LZ) {
          lookups += (cb - b) + (uint32_t)stop + 1u;
          steps += (base - b) / (64u * UN) + 1u;
        } else {
          lookups += (uint32_t)stop + 1u;
        }
        return false;
      }
      body += __popcll(bm);
      if (!LZ) lookups += (e - cb) < 64u ? (e - cb) : 64u;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) ent[u] = nxt[u];
  }
  if (LZ) {
    lookups += e - b;
    steps += (e - b + 64u * UN - 1u) / (64u * UN);
  }
  return true;
}

// True if no 4^3 cell of the corridor list of orientation k holds a voxel
// with TSDF < r_c; corridor entries hit only such voxels, so the fine scan
// of the corridor can then be skipped.  c4 is the point's cell (voxel >> 2)
// relative to the grid; a cell's bit lives in its brick's octant byte.  The
// list holds every cell offset floor((r + o) / 4) over corridor entries o and
// positions r in [0, 4)^3 of the point inside its cell.
__device__ inline bool corridor_clear4_sw(const ToolDev &t, const SwGrid &q, const uint32_t c4[3],
                                          const uint8_t *occ4, int k) {
  const uint32_t cb = t.c4begin[k], ce = t.c4begin[k + 1];
  const uint32_t lane = (uint32_t)lane_id();
  for (uint32_t base = cb; base < ce; base += 64) {
    const uint32_t idx = base + lane;
    const uint32_t d = t.c4entries[idx < ce ? idx : ce - 1];
    const uint32_t X = c4[0] + (uint32_t)entry_x(d), Y = c4[1] + (uint32_t)entry_y(d),
                   Z = c4[2] + (uint32_t)entry_z(d);
    const uint32_t brick = (X >> 1) + q.gx * (Y >> 1) + q.gxy * (Z >> 1);
    const uint32_t bs = brick < q.nbricks ? brick : 0u;
    const uint32_t bit = (X & 1u) | ((Y & 1u) << 1) | ((Z & 1u) << 2);
    const bool occ = (occ4[bs] >> bit) & 1u;
    if (__ballot(idx < ce && occ)) return false;
  }
  return true;
}

// Entries [b, e) of orientation k after its first E: body entries finely,
// then the corridor -- skipped when its 4^3 cells are clear (CO), finely
// otherwise.  Canonical lookups stay the table-order count.
template <int UN, int CO, int B1, int RE = 0, int LZ = 0, int UC = 0, int UB = 0>
__device__ inline bool scan_rest_sw(const Params &p, const ToolDev &t, const SwGrid &q,
                                    const SwFrame &f, int k, uint32_t b, uint32_t e, int body,
                                    uint32_t &lookups, uint32_t &cchecks, uint32_t &cclear,
                                    uint32_t &sbody, uint32_t &sfar, const uint32_t c4[3],
                                    const uint8_t *occ4,
                                    const typename EntryOf<RE>::T *first = nullptr) {
  if (!CO) return scan_fine_sw<UN, B1, RE, 0, LZ>(p, t, q, f, b, e, body, lookups, sbody, first);
  const uint32_t fb = t.far_begin[k];
  const uint32_t mid = fb > b ? fb : b;
  if constexpr (UB > 0) {
    // the body's first chunk alone (most blocked candidates end there), the
    // rest UB chunks per step
    const uint32_t c1 = b + 64u < mid ? b + 64u : mid;
    if (!scan_fine_sw<UN, B1, RE, B1 ? 1 : 0, LZ>(p, t, q, f, b, c1, body, lookups, sbody, first))
      return false;
    if (!scan_fine_sw<UB, B1, RE, B1 ? 1 : 0, LZ>(p, t, q, f, c1, mid, body, lookups, sbody))
      return false;
  } else {
    if (!scan_fine_sw<UN, B1, RE, B1 ? 1 : 0, LZ>(p, t, q, f, b, mid, body, lookups, sbody, first))
      return false;
  }
  if (mid >= e) return true;
  if (t.c4flag[k] != 0) {
    ++cchecks;
    if (corridor_clear4_sw(t, q, c4, occ4, k)) {
      ++cclear;
      lookups += e - mid;
      return true;
    }
  }
  // the corridor: UC chunks per step (0: UN); a candidate that gets this far
  // is mostly free and reads its whole corridor, so two chunks in flight
  // hide one gather latency at little waste
  return scan_fine_sw<UC ? UC : UN, B1, RE, B1 ? 2 : 0, LZ>(p, t, q, f, mid, e, body, lookups,
                                                          sfar);
}

// Candidate-parallel scoring with grid-relative lookups (the configurations
// named "swar").  The mask is taken one 64-orientation word at a time.
// Phase 1: lane j reads the first E entries of orientation 64w + j (staged in
// LDS) and decides it if they block it, all gathers issued together.
// Phase 2, for the whole wave at once: candidates blocked within their first
// E entries (at entry pos) are summed from ballots -- tests by popcount,
// canonical lookups (pos + 1) from four bit-plane ballots -- so only the
// others are visited in index order, with lanes over their remaining
// entries.  Requires K <= kLdsK.
template <int NT, int E, int UN, int FB, int CO, int B1>
__global__ void __launch_bounds__(NT)
k_score_swar(Params p, PointsDev pts, ToolDev t, GridDev g, int64_t n, int32_t mw,
             unsigned *work) {
  if (n < 0) n = *pts.n_points;   // the point count on the device (recorded graphs)
  static_assert(E >= 1 && E <= 15, "head length must fit the 4-bit planes");
  static_assert(!B1 || E >= 3, "the one-bit plane serves only entries after the arm samples");
  constexpr int NW = NT / 64;
  constexpr int ST = E | 1;   // odd row stride of 8-byte entries: no bank conflicts
  __shared__ uint32_t s_begin[kLdsK + 1];
  __shared__ uint2 s_head[kLdsK * ST];
  const int K = t.K;
  for (int j = threadIdx.x; j <= K; j += NT) s_begin[j] = t.begin[j];
  __syncthreads();
  for (int j = threadIdx.x; j < K * E; j += NT) {
    const int k = j / E, qq = j - k * E;
    const uint32_t pos = s_begin[k] + (uint32_t)qq;
    s_head[k * ST + qq] = pos < s_begin[k + 1] ? t.xent[pos] : make_uint2(0u, 0u);
  }
  __syncthreads();
  const SwGrid q = sw_grid(g);
  const int lane = lane_id();
  const int64_t wave0 =
      (int64_t)blockIdx.x * NW + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * NW;
  ScoreCounterBlock &sc = t.counters->s[(blockIdx.x * NW + (threadIdx.x >> 6)) % kStatSlots];
  // per-wave counters in 32 bits (fewer scalar registers), flushed to the
  // 64-bit totals whenever the largest of them passes 2^30
  uint32_t conf = 0, acc = 0, blk = 0, nocand = 0, tests = 0, lookups = 0, deep = 0, chunks = 0;
  uint32_t cchecks = 0, cclear = 0, sbody = 0, sfar = 0;
  auto flush = [&]() {
    if (lane == 0) {
      if (conf) atomicAdd(&sc.n_confident, (unsigned long long)conf);
      if (acc) atomicAdd(&sc.n_accessible, (unsigned long long)acc);
      if (blk) atomicAdd(&sc.n_blocked, (unsigned long long)blk);
      if (nocand) atomicAdd(&sc.n_no_candidate, (unsigned long long)nocand);
      if (tests) atomicAdd(&sc.canonical_tests, (unsigned long long)tests);
      if (lookups) atomicAdd(&sc.canonical_lookups, (unsigned long long)lookups);
      if (deep) atomicAdd(&sc.deep_tests, (unsigned long long)deep);
      if (chunks) atomicAdd(&sc.deep_chunks_max, (unsigned long long)chunks);
      if (cchecks) atomicAdd(&sc.coarse_checks, (unsigned long long)cchecks);
      if (cclear) atomicAdd(&sc.coarse_clear, (unsigned long long)cclear);
      if (sbody) atomicAdd(&sc.chunks_body, (unsigned long long)sbody);
      if (sfar) atomicAdd(&sc.chunks_far, (unsigned long long)sfar);
    }
    conf = acc = blk = nocand = tests = lookups = deep = chunks = 0;
    cchecks = cclear = sbody = sfar = 0;
  };
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
      const SwFrame f = sw_frame(g, q, s);
      uint32_t c4[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) c4[a] = (uint32_t)((s[a] >> 2) - 2 * g.g0[a]);
      label = AF_NO_CANDIDATE;
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
        uint2 ent[E];
        uint32_t code[E];
#pragma unroll
        for (int qq = 0; qq < E; ++qq) ent[qq] = s_head[kk * ST + qq];
#pragma unroll
        for (int qq = 0; qq < E; ++qq) code[qq] = code_sw(q, f, ent[qq]);
        // branch-free head decision: hit bits of non-body and body entries,
        // then the first non-body hit and the n_c-th body hit
        uint32_t nbm = 0u, bhm = 0u;
#pragma unroll
        for (int qq = 0; qq < E; ++qq) {
          const uint32_t cls = sw_cls(ent[qq]);
          const uint32_t c = code[qq];
          const uint32_t hit =
              (cls == AF_CLS_NEAR ? (uint32_t)(c != 0u) : (c & 1u)) & (uint32_t)(qq < (int)len);
          nbm |= (hit & (uint32_t)(cls != AF_CLS_BODY)) << qq;
          bhm |= (hit & (uint32_t)(cls == AF_CLS_BODY)) << qq;
        }
        int pos = nbm ? __builtin_ctz(nbm) : 32;
        {
          int cnt = 0, p5 = 32;
#pragma unroll
          for (int qq = 0; qq < E; ++qq) {
            cnt += (int)((bhm >> qq) & 1u);
            p5 = (p5 == 32 && cnt >= p.n_c) ? qq : p5;
          }
          pos = p5 < pos ? p5 : pos;
        }
        const int body = __popc(bhm);
        const int state = pos < 32 ? 1 : (len <= (uint32_t)E ? 2 : 0);   // 1 blocked, 2 free
        const uint64_t fm = __ballot(cand && state == 2);
        uint64_t open = fm | __ballot(cand && state == 0);
        const uint32_t v = (cand && state == 1) ? (uint32_t)pos + 1u : 0u;
        const uint64_t pl[4] = {__ballot(v & 1u), __ballot(v & 2u), __ballot(v & 4u),
                                __ballot(v & 8u)};
        uint64_t left = word;
        for (;;) {
          if (!open) {
            tests += (uint32_t)__popcll(left);
            lookups += plane_sum(pl, left);
            break;
          }
          const int j = __ffsll((long long)open) - 1;
          open &= open - 1;
          const uint64_t below = left & ((1ull << j) - 1ull);
          tests += (uint32_t)__popcll(below) + 1u;
          lookups += plane_sum(pl, below);
          left &= ~((2ull << j) - 1ull);
          const int kj = 64 * w + j;
          const uint32_t b = s_begin[kj], e = s_begin[kj + 1];
          if ((fm >> j) & 1ull) {
            lookups += e - b;
            ff = (int16_t)kj;
            break;
          }
          lookups += E;
          ++deep;
          chunks += (e - b - E + 63) / 64;
          if (scan_rest_sw<UN, CO, B1>(p, t, q, f, kj, b + E, e,
                                       __builtin_amdgcn_readlane(body, j), lookups, cchecks,
                                       cclear, sbody, sfar, c4, g.occ4)) {
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
    if (lookups > (1u << 30) || chunks > (1u << 30)) flush();
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
  flush();
}

__device__ inline uint64_t readlane64(uint64_t v, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}

// Accumulated per-wave counts of the "near" kernels (flushed to a counter
// block; see near_flush).
struct NearAcc {
  uint32_t labv;   // per lane: lane 0 confident, 1 accessible, 2 blocked, 3 no candidate
  uint32_t tests, lookups, arm, deep, chunks, cchecks, cclear, sbody, sfar;
};

// A zeroed accumulator set held in vector registers: the counts are
// wave-uniform, but in scalar registers they cost this kernel occupancy.
__device__ inline NearAcc near_acc_zero() {
  NearAcc a;
  uint32_t *f = &a.labv;
  static_assert(sizeof(NearAcc) == 10 * sizeof(uint32_t), "ten counters");
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    uint32_t z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    f[k] = z;
  }
  return a;
}

template <int DIAG>
__device__ inline void near_flush(ScoreCounterBlock &sc, NearAcc &a, int lane) {
  if (lane < 4 && a.labv) {
    unsigned long long *dst = lane == 0   ? &sc.n_confident
                              : lane == 1 ? &sc.n_accessible
                              : lane == 2 ? &sc.n_blocked
                                          : &sc.n_no_candidate;
    atomicAdd(dst, (unsigned long long)a.labv);
  }
  if (lane == 0) {
    if (a.tests) atomicAdd(&sc.canonical_tests, (unsigned long long)a.tests);
    if (a.lookups) atomicAdd(&sc.canonical_lookups, (unsigned long long)a.lookups);
    if (a.arm) atomicAdd(&sc.arm_lookups, (unsigned long long)a.arm);
    if (DIAG) {
      if (a.deep) atomicAdd(&sc.deep_tests, (unsigned long long)a.deep);
      if (a.chunks) atomicAdd(&sc.deep_chunks_max, (unsigned long long)a.chunks);
      if (a.cchecks) atomicAdd(&sc.coarse_checks, (unsigned long long)a.cchecks);
      if (a.cclear) atomicAdd(&sc.coarse_clear, (unsigned long long)a.cclear);
      if (a.sbody) atomicAdd(&sc.chunks_body, (unsigned long long)a.sbody);
      if (a.sfar) atomicAdd(&sc.chunks_far, (unsigned long long)a.sfar);
    }
  }
  a = near_acc_zero();
}

// One point of the "near" scoring (see k_score_near): label and first free
// orientation of point i for tool t, whose begin offsets are s_begin.
// LF: s_first holds, for every orientation k, its 64 entries after the arm
// samples (lane l: entry min(begin[k] + 3 + l, begin[k + 1] - 1)), 4-byte
// form, so a candidate's first step reads its entries from LDS.
template <int UN, int CO, int B1, int PF, int RE, int LZ = 0, int UC = 0, int UB = 0, int LF = 0>
__device__ inline void near_point(const Params &p, const PointsDev &pts, const ToolDev &t,
                                  const GridDev &g, const SwGrid &q, const uint32_t *s_begin,
                                  int32_t mw, int64_t i, int lane, NearAcc &acc,
                                  const uint32_t *s_first = nullptr) {
  constexpr uint32_t E = 3;   // the arm samples
  constexpr int F = 64 / PF;  // prefix entries per candidate when PF > 1
  static_assert(PF == 1 || PF == 2 || PF == 4 || PF == 8, "PF divides the wave");
  const int hn = __builtin_amdgcn_readfirstlane(pts.has_normal[i]);
  uint8_t label;
  int16_t ff = -1;
  if (hn < 0) {
    label = AF_UNSCORED;
  } else {
    int32_t s[3];
    unpack_key(pts.key[i], s[0], s[1], s[2]);
    SwFrame f = RE ? rel_frame(g, q, s) : sw_frame(g, q, s);
    uint32_t c4[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c4[a] = (uint32_t)((s[a] >> 2) - 2 * g.g0[a]);
    // values every lane combines with its own entry: kept in vector
    // registers (scalar registers limit this kernel's occupancy)
    asm volatile("" : "+v"(f.Bp), "+v"(f.rp), "+v"(c4[0]), "+v"(c4[1]), "+v"(c4[2]));
    label = AF_NO_CANDIDATE;
    // lanes [0, mw): mask words; [mw, 3 mw): the two arm-sample planes
    const uint64_t mine = lane < mw       ? t.mask[i * mw + lane]
                          : lane < 3 * mw ? t.nearp[i * 2 * mw + (lane - mw)]
                                          : 0ull;
    for (int w = 0; w < mw && ff < 0; ++w) {
      const uint64_t word = readlane64(mine, w);
      if (!word) continue;
      label = AF_BLOCKED;
      const uint64_t pl[4] = {readlane64(mine, mw + w) & word,
                              readlane64(mine, 2 * mw + w) & word, 0ull, 0ull};
      uint64_t open = word & ~(pl[0] | pl[1]);
      uint64_t left = word;
      // PF = 1: the first step's entries of the next candidate are requested
      // before the current candidate is scanned
      using Ent = typename EntryOf<RE>::T;
      Ent pre{};
      auto first_step = [&](uint64_t o) {
        const int kn = 64 * w + (__ffsll((long long)o) - 1);
        if constexpr (LF != 0) {
          static_assert(RE == 1 && PF == 1 && UN == 1, "4-byte entries, one step");
          return (Ent)s_first[kn * 64 + lane];
        } else {
          const uint32_t bn = s_begin[kn] + E, en = s_begin[kn + 1];
          const uint32_t idx = bn + (uint32_t)lane;
          return load_entry<RE>(t, idx < en ? idx : en - 1);
        }
      };
      if (PF == 1 && open) pre = first_step(open);
      while (open && ff < 0) {
        // the next PF candidates that need their body and corridor
        int js[PF];
        int nb = 0;
#pragma unroll
        for (int c = 0; c < PF; ++c) {
          js[c] = open ? __ffsll((long long)open) - 1 : 0;
          nb += open != 0ull;
          open &= open - 1;
        }
        const Ent cur = pre;
        if (PF == 1 && open) pre = first_step(open);
        // their first F entries after the arm samples, F lanes each
        uint64_t nf = 0, bm = 0;
        if (PF > 1) {
          const int c = lane / F, off = lane % F;
          int jc = js[0];
#pragma unroll
          for (int cc = 1; cc < PF; ++cc) jc = c == cc ? js[cc] : jc;
          const int kc = 64 * w + jc;
          const uint32_t b = s_begin[kc] + E, e = s_begin[kc + 1];
          const uint32_t idx = b + (uint32_t)off;
          const bool valid = c < nb && idx < e;
          const auto ent = load_entry<RE>(t, valid ? idx : (e > 0 ? e - 1 : 0));
          const uint32_t code = ent_code<B1>(q, f, ent);
          const uint32_t cls = ent_cls(ent);
          const bool hit =
              valid && (B1 || cls != AF_CLS_NEAR ? (code & 1u) != 0u : code != 0u);
          nf = __ballot(hit && cls != AF_CLS_BODY);
          bm = __ballot(hit && cls == AF_CLS_BODY);
        }
#pragma unroll
        for (int c = 0; c < PF; ++c) {
          if (c >= nb) break;
          const int jj = js[c];
          const uint64_t below = left & ((1ull << jj) - 1ull);
          acc.tests += (uint32_t)__popcll(below) + 1u;
          const uint32_t a = plane_sum(pl, below);
          acc.lookups += a + E;
          acc.arm += a + E;
          left &= ~((2ull << jj) - 1ull);
          const int kj = 64 * w + jj;
          const uint32_t b = s_begin[kj] + E, e = s_begin[kj + 1];
          ++acc.deep;
          acc.chunks += (e - b + 63) / 64;
          uint32_t start = b;
          int body = 0;
          if (PF > 1) {
            const uint64_t fm = F >= 64 ? ~0ull : ((1ull << F) - 1ull);
            const uint64_t nf1 = (nf >> (F * c)) & fm, bm1 = (bm >> (F * c)) & fm;
            const int stop = chunk_stop(nf1, bm1, p.n_c);
            if (stop < F) {   // blocked within the prefix
              acc.lookups += (uint32_t)stop + 1u;
              continue;
            }
            const uint32_t nin = e - b < (uint32_t)F ? e - b : (uint32_t)F;
            acc.lookups += nin;
            body = __popcll(bm1);
            start = b + nin;
          }
          if (scan_rest_sw<UN, CO, B1, RE, LZ, UC, UB>(
                  p, t, q, f, kj, start, e, body, acc.lookups, acc.cchecks, acc.cclear, acc.sbody,
                  acc.sfar, c4, g.occ4, PF == 1 && UN == 1 ? &cur : nullptr)) {
            ff = (int16_t)kj;
            break;
          }
        }
      }
      if (ff < 0) {   // the rest are blocked by an arm sample
        acc.tests += (uint32_t)__popcll(left);
        const uint32_t a = plane_sum(pl, left);
        acc.lookups += a;
        acc.arm += a;
      }
    }
    if (ff >= 0) label = AF_ACCESSIBLE;
    acc.labv += (uint32_t)(lane == 0) | (uint32_t)(lane == 1 && label == AF_ACCESSIBLE) |
            (uint32_t)(lane == 2 && label == AF_BLOCKED) |
            (uint32_t)(lane == 3 && label == AF_NO_CANDIDATE);
  }
  if (lane == 0) {
    t.label[i] = label;
    t.first_free[i] = ff;
  }
}

// Scoring with the arm samples already evaluated by k_mask (the
// configurations named "near"): a candidate whose arm sample q hits first is
// blocked after q + 1 lookups, summed for the whole wave from the two planes;
// only the others are visited, scanning body and corridor from their fourth
// entry.  With PF > 1 the next PF such candidates first get their first
// 64/PF entries in one step (64/PF lanes each): most are blocked there, and
// only the undecided ones continue lane-parallel.  Requires K <= kNearK.
// Same labels, first free orientations and canonical counts as the plain
// scan.
template <int NT, int UN, int FB, int CO, int B1, int DIAG, int PF = 1, int RE = 0, int UC = 0,
          int UB = 0, int LF = 0>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8)))
k_score_near(Params p, PointsDev pts, ToolDev t, GridDev g, int64_t n, int32_t mw,
             unsigned *work) {
  // n < 0: the point count on the device (recorded graphs, point lists)
  if (n < 0) n = pts.sel ? (int64_t)*pts.n_sel : (int64_t)*pts.n_points;
  constexpr int NW = NT / 64;
  __shared__ uint32_t s_begin[kNearK + 1];
  // LF: the first 64 entries after the arm samples of every orientation
  // (K <= kLfK, 64 KiB), read from LDS instead of the table
  __shared__ uint32_t s_first[LF ? kLfK * 64 : 1];
  const int K = t.K;
  for (int j = threadIdx.x; j <= K; j += NT) s_begin[j] = t.begin[j];
  if constexpr (LF != 0) {
    static_assert(NT == 1024, "two workgroups of 68 KiB LDS fill a CU's 160 KiB at 8 waves/SIMD");
    for (int j = threadIdx.x; j < K * 64; j += NT) {
      const uint32_t b = t.begin[j >> 6] + 3u, e = t.begin[(j >> 6) + 1];
      const uint32_t idx = b + (uint32_t)(j & 63);
      s_first[j] = load_entry<1>(t, idx < e ? idx : e - 1);
    }
  }
  __syncthreads();
  const SwGrid q = sw_grid(g);
  const int lane = lane_id();
  const int64_t wave0 =
      (int64_t)blockIdx.x * NW + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * NW;
  ScoreCounterBlock &sc = t.counters->s[(blockIdx.x * NW + (threadIdx.x >> 6)) % kStatSlots];
  NearAcc a = near_acc_zero();
  int64_t i = wave0, batch_end = wave0 + 1;
  // with a point list, lane k holds the batch's k-th listed point (one read
  // per batch instead of one dependent read per point)
  int32_t selv = 0;
  auto fetch_list = [&]() {
    if (FB > 0 && pts.sel) {
      const int64_t idx = i + lane;
      selv = (lane < FB && idx < n) ? pts.sel[idx] : 0;
    }
  };
  if (FB > 0) {
    unsigned got = 0;
    if (lane == 0) got = atomicAdd(work, (unsigned)FB);
    i = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
    batch_end = i + FB;
    fetch_list();
  }
  for (; i < n;) {
    const int64_t pi =
        !pts.sel ? i
        : FB > 0 ? (int64_t)__builtin_amdgcn_readlane(selv, (int)(FB - (batch_end - i)))
                 : (int64_t)__builtin_amdgcn_readfirstlane(pts.sel[i]);
    near_point<UN, CO, B1, PF, RE, 1, UC, UB, LF>(p, pts, t, g, q, s_begin, mw, pi, lane, a,
                                                  s_first);
    if (a.lookups > (1u << 30)) near_flush<DIAG>(sc, a, lane);
    if (FB > 0) {
      if (++i >= batch_end) {
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(work, (unsigned)FB);
        i = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
        batch_end = i + FB;
        fetch_list();
      }
    } else {
      i += nwaves;
    }
  }
  near_flush<DIAG>(sc, a, lane);
}

// Several tools in one persistent launch: work item j is point j mod n of
// tool set.id[j / n] (tool-major, so a tool's table stays cached while the
// waves go through its points).  Every tool's begin offsets are staged in
// LDS (at set.base[ti]); each tool keeps its own masks, labels and counters.
// Same results as one k_score_near launch per tool.
constexpr int kMultiBegin = 8 * (kNearK + 1);

template <int NT, int UN, int FB, int CO, int B1, int PF, int RE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8)))
k_score_near_multi(Params p, PointsDev pts, const ToolDev *tools, ToolSet set, GridDev g,
                   int64_t n, unsigned *work) {
  if (n < 0) n = *pts.n_points;   // the point count on the device (recorded graphs)
  constexpr int NW = NT / 64;
  extern __shared__ uint32_t s_begin[];   // sized for the set at launch
  for (int ti = 0; ti < set.n; ++ti) {
    const uint32_t *bg = tools[set.id[ti]].begin;
    const int K = tools[set.id[ti]].K, o = set.base[ti];
    for (int j = threadIdx.x; j <= K; j += NT) s_begin[o + j] = bg[j];
  }
  __syncthreads();
  const SwGrid q = sw_grid(g);
  const int lane = lane_id();
  const int slot = (blockIdx.x * NW + (threadIdx.x >> 6)) % kStatSlots;
  NearAcc a = near_acc_zero();
  const int64_t total = n * set.n;
  int64_t j = 0, batch_end = 0;
  int cur = -1;
  ToolDev t;
  int32_t mw = 0;
  for (;;) {
    if (j >= batch_end) {
      unsigned got = 0;
      if (lane == 0) got = atomicAdd(work, (unsigned)FB);
      j = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
      batch_end = j + FB;
    }
    if (j >= total) break;
    const int ti = (int)(j / n);
    if (ti != cur) {
      if (cur >= 0) near_flush<0>(t.counters->s[slot], a, lane);
      cur = ti;
      t = tools[set.id[ti]];
      mw = (t.K + 63) / 64;
    }
    near_point<UN, CO, B1, PF, RE>(p, pts, t, g, q, s_begin + set.base[ti], mw,
                                   j - (int64_t)ti * n, lane, a);
    ++j;
  }
  if (cur >= 0) near_flush<0>(t.counters->s[slot], a, lane);
}

// Several maps in one persistent launch (a server step's streams): job j
// scores every point of one context's map for one of its tools, with that
// context's constants, points, grid and table.  Work item w is point
// w - start[j] of the job j whose range holds it (job-major); the jobs'
// point counts are read on the device (their frames were just integrated).
// Every job's begin offsets are staged in LDS at jobs[j].base.  Same results
// as one k_score_near launch per job.
template <int NT, int UN, int FB, int CO, int B1, int PF, int RE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8)))
k_score_near_jobs(const ScoreJob *jobs, int32_t n_jobs, unsigned *work) {
  constexpr int NW = NT / 64;
  extern __shared__ uint32_t s_begin[];   // sized for the jobs at launch
  for (int j = 0; j < n_jobs; ++j) {
    const uint32_t *bg = jobs[j].t.begin;
    const int K = jobs[j].t.K, o = jobs[j].base;
    for (int k = threadIdx.x; k <= K; k += NT) s_begin[o + k] = bg[k];
  }
  // s_start[j]: job j's first work item (prefix of the point counts, which
  // the device holds: the frames were just integrated)
  __shared__ int64_t s_start[kMaxJobs + 1];
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int j = 0; j < n_jobs; ++j) {
      s_start[j] = run;
      run += *jobs[j].pts.n_points;
    }
    s_start[n_jobs] = run;
  }
  __syncthreads();
  const int lane = lane_id();
  const int slot = (blockIdx.x * NW + (threadIdx.x >> 6)) % kStatSlots;
  const int64_t total = s_start[n_jobs];
  NearAcc a = near_acc_zero();
  int64_t w = 0, batch_end = 0;
  int cur = -1;
  const ScoreJob *jp = jobs;   // the current job (read in place: wave-uniform loads)
  SwGrid q;
  int32_t mw = 0;
  int64_t j0 = 0, j1 = 0;      // the current job's work items [j0, j1)
  for (;;) {
    if (w >= batch_end) {
      unsigned got = 0;
      if (lane == 0) got = atomicAdd(work, (unsigned)FB);
      w = (int64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
      batch_end = w + FB;
    }
    if (w >= total) break;
    if (w < j0 || w >= j1) {
      // the job whose range holds w (a scan of the LDS starts; jobs without
      // points have an empty range and are passed over)
      int ji = 0;
      while (s_start[ji + 1] <= w) ++ji;
      if (cur >= 0) near_flush<0>(jp->t.counters->s[slot], a, lane);
      cur = ji;
      jp = jobs + ji;
      q = sw_grid(jp->g);
      mw = (jp->t.K + 63) / 64;
      j0 = s_start[ji];
      j1 = s_start[ji + 1];
    }
    near_point<UN, CO, B1, PF, RE>(jp->p, jp->pts, jp->t, jp->g, q, s_begin + jp->base, mw,
                                   w - j0, lane, a);
    ++w;
  }
  if (cur >= 0) near_flush<0>(jp->t.counters->s[slot], a, lane);
}

using ScoreKernel = void (*)(Params, PointsDev, ToolDev, GridDev, int64_t, int32_t, unsigned *);

struct ScoreVariant {
  ScoreKernel fn;
  int threads;
  const char *name;
  int max_k;         // largest K the configuration handles (0: any)
  int needs_rel;     // 1: only with the 4-byte entry form (offsets within +-255)
  const char *above_k;   // the configuration that runs above max_k (null: the plain one)
};

// The tunable score configurations (identical results; speed only).
const ScoreVariant kVariants[] = {
    {k_score<256, 0, 1, 1, 0, 0>, 256, "plain wg256", 0},
    {k_score<256, 0, 2, 2, 1, 16>, 256, "plain wg256 ahead2 unroll2 occ dyn16", 0},
    {k_score_swar<256, 3, 1, 16, 2, 1>, 256, "swar wg256 head3 unroll1 dyn16 coarse4 bit", kLdsK},
    {k_score_swar<256, 4, 1, 16, 0, 0>, 256, "swar wg256 head4 unroll1 dyn16", kLdsK},
    {k_score_near<256, 1, 16, 2, 1, 0>, 256, "near wg256 unroll1 dyn16 coarse4 bit", kNearK},
    {k_score_near<256, 1, 16, 0, 1, 0>, 256, "near wg256 unroll1 dyn16 bit", kNearK},
    {k_score_near<256, 1, 8, 2, 1, 0, 1, 1>, 256, "near wg256 unroll1 dyn8 coarse4 bit rel", kNearK, 1},
    {k_score_near<256, 1, 8, 2, 1, 1, 1, 1>, 256, "near wg256 unroll1 dyn8 coarse4 bit rel diag", kNearK, 1},
    {k_score_near<256, 1, 16, 2, 1, 0, 1, 1>, 256, "near wg256 unroll1 dyn16 coarse4 bit rel", kNearK, 1},
    {k_score_near<256, 2, 8, 2, 1, 0, 1, 1>, 256, "near wg256 unroll2 dyn8 coarse4 bit rel", kNearK, 1},
    {k_score_near<512, 1, 8, 2, 1, 0, 1, 1>, 512, "near wg512 unroll1 dyn8 coarse4 bit rel", kNearK, 1},
    {k_score_near<256, 1, 8, 2, 1, 0, 2, 1>, 256, "near wg256 unroll1 dyn8 coarse4 bit prefix2 rel", kNearK, 1},
    {k_score_near<256, 1, 8, 2, 1, 0, 1, 1, 2>, 256, "near wg256 unroll1 dyn8 coarse4 bit rel corr2", kNearK, 1},
    {k_score_near<256, 1, 8, 2, 1, 1, 1, 1, 2>, 256, "near wg256 unroll1 dyn8 coarse4 bit rel corr2 diag", kNearK, 1},
    {k_score_near<256, 1, 8, 2, 1, 0, 1, 1, 0, 2>, 256, "near wg256 unroll1 dyn8 coarse4 bit rel body2", kNearK, 1},
    {k_score_near<1024, 1, 8, 2, 1, 0, 1, 1, 2, 0, 1>, 1024,
     "near wg1024 unroll1 dyn8 coarse4 bit rel corr2 lds1", kLfK, 1,
     "near wg256 unroll1 dyn8 coarse4 bit rel corr2"},
};
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

static int variant_index(const char *name) {
  for (int v = 0; v < kNumVariants; ++v)
    if (strcmp(kVariants[v].name, name) == 0) return v;
  return 0;
}
int g_resident[kNumVariants];   // workgroups per CU, from the occupancy query
int g_num_cu = 0;

// Test hook: the PCA step alone, on caller-given moments [n][10] (cnt, sum
// d [3], sum dd^T [6]).
__global__ void __launch_bounds__(kThreads)
k_pca_axes(const int32_t *mom, int64_t n, int64_t *axes, int32_t *has) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int32_t *m = mom + 10 * i;
  const int32_t sx[3] = {m[1], m[2], m[3]};
  const int32_t sxx[6] = {m[4], m[5], m[6], m[7], m[8], m[9]};
  int64_t ax[3];
  has[i] = pca_axis(m[0], sx, sxx, ax);
  for (int a = 0; a < 3; ++a) axes[3 * i + a] = ax[a];
}

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

void launch_normals_cached(const Params &p, MapDev m, PointsDev pts, GridDev g,
                           const NormalCache &nc, int64_t seen, int64_t n, hipStream_t s) {
  init_tables();
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(1), 0, s, (unsigned *)nc.count);
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  const bool all = seen <= 0 || (n - seen) * 8 > n;   // most of the map is new
  const bool marked = !all && n > seen;
  if (all)
    hipLaunchKernelGGL(k_normals_reset, dim3(blocks), dim3(kThreads), 0, s, nc, n);
  else if (marked)
    hipLaunchKernelGGL(k_normals_mark<1>, dim3((unsigned)(n - seen)), dim3(128), 0, s, pts, g, nc,
                       seen);
  hipLaunchKernelGGL(k_normals_orient, dim3((unsigned)((n + kOrientThreads - 1) / kOrientThreads)),
                     dim3(kOrientThreads), 0, s, p, m, pts, g, nc, n, marked ? 1 : 0);
  if (marked)
    hipLaunchKernelGGL(k_normals_mark<0>, dim3((unsigned)(n - seen)), dim3(128), 0, s, pts, g, nc,
                       seen);
  hipLaunchKernelGGL(k_normals_axis, dim3(blocks), dim3(kThreads), 0, s, p, pts, g, nc);
}

void launch_normals(const Params &p, MapDev m, PointsDev pts, GridDev g, int64_t n,
                    hipStream_t s, bool dev_n) {
  init_tables();
  if (n <= 0) return;
  hipLaunchKernelGGL(k_normals, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, s, p, m, pts, g, dev_n ? (int64_t)-1 : n);
}

void launch_pca_axes(const int32_t *mom, int64_t n, int64_t *axes, int32_t *has,
                     hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pca_axes, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, s, mom, n, axes, has);
}

void launch_mask(const Params &p, PointsDev pts, ToolDev t, GridDev g, int64_t n,
                 hipStream_t s, bool dev_n) {
  int32_t mw = (t.K + 63) / 64;
  if (n <= 0) return;
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
  const int64_t nn = dev_n ? (int64_t)-1 : n;
  // heads walked per lane, four mask words per launch (each launch after the
  // first reads the words the previous one wrote)
  for (int w0 = 0; w0 < mw; w0 += 4) {
    switch (mw - w0 < 4 ? mw - w0 : 4) {
      case 1: hipLaunchKernelGGL(k_mask_walk<1>, grid, dim3(kThreads), 0, s, p, pts, t, g, nn, w0, mw); break;
      case 2: hipLaunchKernelGGL(k_mask_walk<2>, grid, dim3(kThreads), 0, s, p, pts, t, g, nn, w0, mw); break;
      case 3: hipLaunchKernelGGL(k_mask_walk<3>, grid, dim3(kThreads), 0, s, p, pts, t, g, nn, w0, mw); break;
      default: hipLaunchKernelGGL(k_mask_walk<4>, grid, dim3(kThreads), 0, s, p, pts, t, g, nn, w0, mw); break;
    }
  }
}

int score_variants() { return kNumVariants; }


// The configuration a new context uses (the fastest on the tree workload).
int score_variant_default() {
  return variant_index("near wg1024 unroll1 dyn8 coarse4 bit rel corr2 lds1");
}

const char *score_variant_name(int v) {
  return v >= 0 && v < kNumVariants ? kVariants[v].name : "";
}

int multi_begin_capacity() { return kMultiBegin; }

// The tools of `set` (host copies of their tables in host_tools, indexed
// like set.id) in one persistent launch.
void launch_score_multi(const Params &p, PointsDev pts, const ToolDev *tools_dev,
                        const ToolDev *host_tools, const ToolSet &set, GridDev g, int64_t n,
                        unsigned *work, hipStream_t s, bool dev_n) {
  if (n <= 0 || set.n <= 0) return;
  bool rel = true;
  for (int i = 0; i < set.n; ++i) rel = rel && host_tools[i].rent != nullptr;
  using MultiKernel = void (*)(Params, PointsDev, const ToolDev *, ToolSet, GridDev, int64_t,
                               unsigned *);
  const MultiKernel fn = rel ? k_score_near_multi<256, 1, 8, 2, 1, 1, 1>
                             : k_score_near_multi<256, 1, 8, 2, 1, 1, 0>;
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess ||
        g_num_cu <= 0)
      g_num_cu = 256;
  }
  int32_t words = 0;
  for (int i = 0; i < set.n; ++i) words += host_tools[i].K + 1;
  const size_t lds = sizeof(uint32_t) * (size_t)words;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  int64_t wg = (int64_t)per_cu * g_num_cu;
  const int64_t need = (n * set.n + 3) / 4;
  if (wg > need) wg = need;
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(1), 0, s, work);
  hipLaunchKernelGGL(fn, dim3((unsigned)wg), dim3(256), lds, s, p, pts, tools_dev, set, g,
                     dev_n ? (int64_t)-1 : n, work);
}

int launch_score_jobs(const ScoreJob *jobs_dev, const ScoreJob *jobs_host, int32_t n_jobs,
                      unsigned *work, hipStream_t s) {
  if (n_jobs <= 0) return 0;
  if (n_jobs > kMaxJobs) return -1;
  bool rel = true;
  int64_t words = 0, np = 0;
  for (int j = 0; j < n_jobs; ++j) {
    rel = rel && jobs_host[j].t.rent != nullptr;
    words += jobs_host[j].t.K + 1;
    if (jobs_host[j].t.K > kNearK) return -1;
    np += jobs_host[j].max_points;
  }
  using JobKernel = void (*)(const ScoreJob *, int32_t, unsigned *);
  const JobKernel fn = rel ? k_score_near_jobs<256, 1, 8, 2, 1, 1, 1>
                           : k_score_near_jobs<256, 1, 8, 2, 1, 1, 0>;
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess ||
        g_num_cu <= 0)
      g_num_cu = 256;
  }
  const size_t lds = sizeof(uint32_t) * (size_t)words;
  if (lds > 64 * 1024) return -1;
  // occupancy of the last (kernel, LDS size) asked for (a server asks every step)
  static const void *last_fn = nullptr;
  static size_t last_lds = 0;
  static int last_per_cu = 0;
  int per_cu = 0;
  if ((const void *)fn == last_fn && lds == last_lds) {
    per_cu = last_per_cu;
  } else {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess ||
        per_cu <= 0)
      per_cu = 1;
    last_fn = (const void *)fn;
    last_lds = lds;
    last_per_cu = per_cu;
  }
  int64_t wg = (int64_t)per_cu * g_num_cu;
  const int64_t need = (np + 3) / 4;
  if (wg > need) wg = need;
  if (wg < 1) wg = 1;
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(1), 0, s, work);
  hipLaunchKernelGGL(fn, dim3((unsigned)wg), dim3(256), lds, s, jobs_dev, n_jobs, work);
  return 0;
}

static int effective_variant(int variant, const ToolDev &t) {
  if (variant < 0 || variant >= kNumVariants) variant = 0;
  if (kVariants[variant].max_k && t.K > kVariants[variant].max_k)
    variant = kVariants[variant].above_k ? variant_index(kVariants[variant].above_k) : 0;
  if (kVariants[variant].max_k && t.K > kVariants[variant].max_k) variant = 0;
  if (kVariants[variant].needs_rel && !t.rent) variant = 0;
  return variant;
}

bool score_variant_takes_list(int variant, const ToolDev &t) {
  return strncmp(kVariants[effective_variant(variant, t)].name, "near", 4) == 0;
}

void launch_score(const Params &p, PointsDev pts, ToolDev t, GridDev g, int64_t n, int variant,
                  unsigned *work, hipStream_t s, bool dev_n) {
  int32_t mw = (t.K + 63) / 64;
  if (n <= 0) return;
  variant = effective_variant(variant, t);
  if (pts.sel && !score_variant_takes_list(variant, t)) return;   // callers check first
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
  hipLaunchKernelGGL(v.fn, dim3((unsigned)wg), dim3(v.threads), 0, s, p, pts, t, g,
                     dev_n ? (int64_t)-1 : n, mw, work);
}

}  // namespace af
