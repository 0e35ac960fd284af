// Per-frame integration kernels: quantisation, block allocation in the hash
// map, scan-centric cube accumulation (Section 3.2), ray-cleared band
// (Section 3.4, "Arm path checking"), surface points (Section 3.1), the fold
// with the weight cap (Section 3.6) and the brick grid used by scoring.
#include "af_internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace af {
namespace {

constexpr int kThreads = 256;

__device__ inline int lane_id() { return (int)(threadIdx.x & 63u); }

// Insert `key`; returns its slot (fresh = newly inserted) or -1 if full.
__device__ int32_t hash_insert(HashTable t, int64_t key, bool &fresh) {
  uint32_t s = slot_of(key, t.mask);
  for (uint32_t i = 0; i <= t.mask; ++i) {
    int64_t cur = __hip_atomic_load(&t.keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == key) {
      fresh = false;
      return (int32_t)s;
    }
    if (cur == kEmpty) {
      unsigned long long prev = atomicCAS((unsigned long long *)&t.keys[s],
                                          (unsigned long long)kEmpty,
                                          (unsigned long long)key);
      if ((int64_t)prev == kEmpty) {
        fresh = true;
        return (int32_t)s;
      }
      if ((int64_t)prev == key) {
        fresh = false;
        return (int32_t)s;
      }
    }
    s = (s + 1) & t.mask;
  }
  fresh = false;
  return -1;
}

// Exact floor(sqrt(n)) for 0 <= n < 2^62.
__device__ inline int64_t isqrt64(int64_t n) {
  if (n <= 0) return 0;
  uint64_t u = (uint64_t)n;
  uint64_t r = (uint64_t)__builtin_sqrt((double)n);
  while (r * r > u) --r;
  while ((r + 1) * (r + 1) <= u) ++r;
  return (int64_t)r;
}

// a / b to nearest, halves away from zero (b > 0).
__device__ inline int64_t div_round(int64_t a, int64_t b) {
  int64_t m = a < 0 ? -a : a;
  int64_t q = (2 * m + b) / (2 * b);
  return a < 0 ? -q : q;
}

__device__ inline int64_t div_floor(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ inline void wave_count(unsigned long long *ctr, bool flag) {
  unsigned long long b = __ballot(flag);
  if (lane_id() == 0 && b) atomicAdd(ctr, (unsigned long long)__popcll(b));
}

struct Span {
  int lo[3], n[3];
};

__device__ inline Span cube_span(int4 P, int R) {
  Span s;
  int v[3] = {P.x >> 8, P.y >> 8, P.z >> 8};
  for (int i = 0; i < 3; ++i) {
    s.lo[i] = (v[i] - R) >> 3;
    s.n[i] = ((v[i] + R) >> 3) - s.lo[i] + 1;
  }
  return s;
}

__device__ inline bool in_box(int32_t bx, int32_t by, int32_t bz, int3 lo, int3 hi) {
  return bx >= lo.x && bx <= hi.x && by >= lo.y && by <= hi.y && bz >= lo.z && bz <= hi.z;
}

// --------------------------------------------------------------- prep
// Quantise each return, insert the blocks of its cube and of its band
// samples, and insert its voxel into the point set.
__global__ void __launch_bounds__(kThreads)
k_frame_prep(const float *__restrict__ xyz, const FrameArgs *fa, Params p, MapDev m,
             PointsDev pts, FrameScratch fs, FrameCounters *c) {
  const int64_t n = fa->n;
  const int3 Q = fa->Q;
  const int3 wlo = fa->wlo, whi = fa->whi;
  int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  bool in = r < n;
  bool ok = in;
  int P[3] = {0, 0, 0};
  if (in) {
    for (int i = 0; i < 3; ++i) {
      double t = (double)xyz[3 * r + i] * p.scale;
      if (!(fabs(t) <= (double)kCoordLim))
        ok = false;
      else
        P[i] = (int)__builtin_rint(t);
    }
    if (ok && P[0] == Q.x && P[1] == Q.y && P[2] == Q.z) ok = false;
  }
  wave_count(&c->n_valid, ok);
  wave_count(&c->n_dropped, in && !ok);
  if (!in) return;
  if (!ok) {
    fs.P[r] = make_int4(0, 0, 0, 0);
    return;
  }
  int64_t g[3] = {(int64_t)Q.x - P[0], (int64_t)Q.y - P[1], (int64_t)Q.z - P[2]};
  int64_t L = isqrt64(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  int4 P4 = make_int4(P[0], P[1], P[2], (int)L);
  fs.P[r] = P4;

  bool full = false;
  // blocks of the cube
  Span sp = cube_span(P4, p.R);
  int idx = 0;
  for (int bz = 0; bz < sp.n[2]; ++bz)
    for (int by = 0; by < sp.n[1]; ++by)
      for (int bx = 0; bx < sp.n[0]; ++bx) {
        if (!in_box(sp.lo[0] + bx, sp.lo[1] + by, sp.lo[2] + bz, wlo, whi)) {
          fs.span[r * kMaxSpan + idx++] = -1;   // outside the window: not written
          continue;
        }
        bool fresh;
        int32_t s = hash_insert(m.h, pack_key(sp.lo[0] + bx, sp.lo[1] + by, sp.lo[2] + bz), fresh);
        if (s < 0) full = true;
        if (fresh) fs.new_blocks[atomicAdd(&c->n_new_blocks, 1)] = s;
        fs.span[r * kMaxSpan + idx++] = s;
      }
  // band samples: (tau, 2.25 tau] back towards the sensor, every v/2
  int j = 0;
  for (; j < kMaxBand; ++j) {
    int64_t lam = (int64_t)p.tau_u + 128 * (j + 1);
    if (4 * lam > 9 * (int64_t)p.tau_u || lam >= L) break;
    int64_t vx = (P[0] + div_round(lam * g[0], L)) >> 8;
    int64_t vy = (P[1] + div_round(lam * g[1], L)) >> 8;
    int64_t vz = (P[2] + div_round(lam * g[2], L)) >> 8;
    if (!in_box((int32_t)(vx >> 3), (int32_t)(vy >> 3), (int32_t)(vz >> 3), wlo, whi)) {
      fs.band[2 * (r * kMaxBand + j)] = -3;   // outside the window: neither marked nor counted
      continue;
    }
    bool fresh;
    int32_t s = hash_insert(m.h, pack_key(vx >> 3, vy >> 3, vz >> 3), fresh);
    if (s < 0) full = true;
    if (fresh) fs.new_blocks[atomicAdd(&c->n_new_blocks, 1)] = s;
    fs.band[2 * (r * kMaxBand + j)] = s;
    fs.band[2 * (r * kMaxBand + j) + 1] = (int)((vx & 7) | ((vy & 7) << 3) | ((vz & 7) << 6));
  }
  if (j < kMaxBand) fs.band[2 * (r * kMaxBand + j)] = -2;  // end marker
  // the return's voxel is a surface point (inside the window)
  if (!in_box(P[0] >> 11, P[1] >> 11, P[2] >> 11, wlo, whi)) {
    fs.pslot[r] = -1;
    if (full) atomicOr(&c->status, kStatusHashFull);
    return;
  }
  bool fresh;
  int32_t ps = hash_insert(pts.h, pack_key(P[0] >> 8, P[1] >> 8, P[2] >> 8), fresh);
  if (ps < 0) full = true;
  if (fresh) {
    int at = atomicAdd(&c->n_new_points, 1);
    fs.new_keys[at] = pack_key(P[0] >> 8, P[1] >> 8, P[2] >> 8);
    fs.new_kslot[at] = ps;
  }
  fs.pslot[r] = ps;
  if (full) atomicOr(&c->status, kStatusHashFull);
}

__global__ void k_reset_counters(FrameCounters *c, MapDev m, PointsDev pts) {
  c->n_valid = c->n_dropped = c->pairs_applied = c->pairs_excluded = 0;
  c->band_marks = c->voxels_folded = 0;
  c->n_new_blocks = c->n_touched = c->n_new_points = c->status = 0;
  c->n_changed = 0;
  for (int i = 0; i < kStatSlots; ++i) c->fold[i][0] = c->fold[i][1] = c->fold[i][2] = 0ull;
  for (int i = 0; i < 3; ++i) {
    c->bmin[i] = 0x7fffffff;
    c->bmax[i] = -0x7fffffff - 1;
  }
  c->blocks_before = *m.n_blocks;
  c->points_before = *pts.n_points;
  c->free_before = m.n_free ? *m.n_free : 0;
}

// One workgroup per new block: assign its id and clear its voxels.
__global__ void __launch_bounds__(kThreads)
k_assign_blocks(MapDev m, FrameScratch fs, FrameCounters *c, const FrameArgs *fa) {
  const int32_t frame = fa->frame;
  int n_new = c->n_new_blocks;
  int64_t base = *m.n_blocks;
  const int nfree = c->free_before;   // evicted ids first (sliding window)
  for (int i = blockIdx.x; i < n_new; i += gridDim.x) {
    int32_t slot = fs.new_blocks[i];
    int64_t id = i < nfree ? (int64_t)m.free_ids[nfree - 1 - i] : base + (i - nfree);
    if (id >= m.max_blocks) {
      if (threadIdx.x == 0) {
        m.h.vals[slot] = -1;
        atomicOr(&c->status, kStatusBlockOverflow);
      }
      continue;
    }
    if (threadIdx.x == 0) {
      m.h.vals[slot] = (int32_t)id;
      int64_t k = m.h.keys[slot];
      m.bkey[id] = k;
      m.touched[id] = -1;
      int32_t b[3];
      unpack_key(k, b[0], b[1], b[2]);
      for (int a = 0; a < 3; ++a) {
        atomicMin(&c->bmin[a], b[a]);
        atomicMax(&c->bmax[a], b[a]);
      }
    }
    for (int t = threadIdx.x; t < kBlockVox; t += kThreads) {
      m.S[id * kBlockVox + t] = 0;
      m.W[id * kBlockVox + t] = 0;
    }
    if (threadIdx.x < 16) {
      m.clr[id * 16 + threadIdx.x] = 0;
      m.surf[id * 16 + threadIdx.x] = 0;
    }
  }
}

__global__ void k_commit_blocks(MapDev m, FrameCounters *c) {
  int64_t base = *m.n_blocks;
  int64_t add = c->n_new_blocks;
  const int64_t nfree = c->free_before;
  if (m.n_free) *m.n_free = (int32_t)(add < nfree ? nfree - add : 0);
  add = add > nfree ? add - nfree : 0;
  if (base + add > m.max_blocks) add = m.max_blocks - base;
  *m.n_blocks = (int32_t)(base + add);
}

// Mark every block of the frame touched (once) and set the band's cleared bits.
__global__ void __launch_bounds__(kThreads)
k_touch_band(const FrameArgs *fa, Params p, MapDev m, FrameScratch fs, FrameCounters *c) {
  const int64_t n = fa->n;
  const int32_t frame = fa->frame;
  int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int marks = 0;
  if (r < n) {
    int4 P = fs.P[r];
    if (P.w > 0) {
      Span sp = cube_span(P, p.R);
      int ns = sp.n[0] * sp.n[1] * sp.n[2];
      for (int i = 0; i < ns; ++i) {
        int32_t s = fs.span[r * kMaxSpan + i];
        int32_t id = s >= 0 ? m.h.vals[s] : -1;
        if (id >= 0 && atomicExch(&m.touched[id], frame) != frame) {
          int pos = atomicAdd(&c->n_touched, 1);
          fs.touched[pos] = id;
          m.tpos[id] = pos;
          fs.bin_cnt[pos] = 0;
        }
      }
      for (int j = 0; j < kMaxBand; ++j) {
        int32_t s = fs.band[2 * (r * kMaxBand + j)];
        if (s == -2) break;
        if (s == -3) continue;
        ++marks;
        int32_t id = s >= 0 ? m.h.vals[s] : -1;
        if (id < 0) continue;
        int vi = fs.band[2 * (r * kMaxBand + j) + 1];
        atomicOr(&m.clr[(int64_t)id * 16 + (vi >> 5)], 1u << (vi & 31));
        if (atomicExch(&m.touched[id], frame) != frame) {
          int pos = atomicAdd(&c->n_touched, 1);
          fs.touched[pos] = id;
          m.tpos[id] = pos;
          fs.bin_cnt[pos] = 0;
        }
      }
    }
  }
  unsigned long long s = marks;
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor((unsigned)s, off);
  if (lane_id() == 0 && s) atomicAdd(&c->band_marks, s);
}

// ---------------------------------------------------------------- points
// New point keys of the frame get ids in ascending key order (rank by
// counting smaller keys), are initialised and flagged in their block.
// New points are appended in key order.  Each workgroup first sorts its
// tile of (distinct) new keys in LDS with Batcher's bitonic network; a key's
// rank among all new keys is then the sum of its lower bounds in the tiles.
__global__ void __launch_bounds__(kThreads)
k_sort_new_tiles(FrameScratch fs, const FrameCounters *c) {
  static_assert((kThreads & (kThreads - 1)) == 0, "bitonic tile needs a power of two");
  __shared__ int64_t v[kThreads];
  const int m = c->n_new_points;
  const int base = blockIdx.x * kThreads;
  if (base >= m) return;
  const int t = threadIdx.x;
  v[t] = base + t < m ? fs.new_keys[base + t] : (int64_t)0x7fffffffffffffffLL;
  __syncthreads();
  for (int k = 2; k <= kThreads; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int q = t ^ j;
      if (q > t) {
        const int64_t a = v[t], b = v[q];
        if ((a > b) == ((t & k) == 0)) {
          v[t] = b;
          v[q] = a;
        }
      }
      __syncthreads();
    }
  fs.new_sorted[base + t] = v[t];
}

__global__ void __launch_bounds__(kThreads)
k_points_append(MapDev m, PointsDev pts, FrameScratch fs, FrameCounters *c, const FrameArgs *fa) {
  const int32_t frame = fa->frame;
  __shared__ int64_t tile[kThreads];
  int mcount = c->n_new_points;
  int i = blockIdx.x * kThreads + threadIdx.x;
  if ((int)(blockIdx.x * kThreads) >= mcount) return;
  int64_t key = i < mcount ? fs.new_keys[i] : 0;
  int rank = 0;
  for (int base = 0; base < mcount; base += kThreads) {
    __syncthreads();
    tile[threadIdx.x] = fs.new_sorted[base + threadIdx.x];
    __syncthreads();
    int lo = 0, hi = mcount - base < kThreads ? mcount - base : kThreads;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (tile[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    rank += lo;
  }
  if (i >= mcount) return;
  int64_t id = (int64_t)*pts.n_points + rank;
  int32_t slot = fs.new_kslot[i];
  if (id >= pts.max_points) {
    pts.h.vals[slot] = -1;
    atomicOr(&c->status, kStatusPointOverflow);
    return;
  }
  pts.h.vals[slot] = (int32_t)id;
  pts.key[id] = key;
  pts.first[id] = frame;
  pts.last[id] = -1;
  pts.nvp[id] = 0;
  pts.head[id] = 0;
  pts.nq[id] = 0;
  pts.sumq[3 * id] = pts.sumq[3 * id + 1] = pts.sumq[3 * id + 2] = 0;
  pts.has_normal[id] = -1;
  int32_t x, y, z;
  unpack_key(key, x, y, z);
  int32_t bs = hash_find(m.h, pack_key(x >> 3, y >> 3, z >> 3));
  int32_t bid = bs >= 0 ? m.h.vals[bs] : -1;
  int vi = (x & 7) | ((y & 7) << 3) | ((z & 7) << 6);
  pts.addr[id] = bid >= 0 ? bid * kBlockVox + vi : -1;
  if (bid >= 0) atomicOr(&m.surf[(int64_t)bid * 16 + (vi >> 5)], 1u << (vi & 31));
}

__global__ void k_commit_points(PointsDev pts, FrameCounters *c) {
  int64_t base = *pts.n_points;
  int64_t add = c->n_new_points;
  if (base + add > pts.max_points) add = pts.max_points - base;
  *pts.n_points = (int32_t)(base + add);
}

// Once per (point, frame): running sensor sum and the viewpoint ring.
__global__ void __launch_bounds__(kThreads)
k_points_view(const FrameArgs *fa, Params p, PointsDev pts, FrameScratch fs) {
  const int64_t n = fa->n;
  const int3 Q = fa->Q;
  const int32_t frame = fa->frame;
  int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n || fs.P[r].w == 0) return;
  int32_t s = fs.pslot[r];
  int32_t id = s >= 0 ? pts.h.vals[s] : -1;
  if (id < 0 || atomicExch(&pts.last[id], frame) == frame) return;
  pts.sumq[3 * (int64_t)id] += Q.x;
  pts.sumq[3 * (int64_t)id + 1] += Q.y;
  pts.sumq[3 * (int64_t)id + 2] += Q.z;
  pts.nq[id] += 1;
  int cnt = pts.nvp[id], head = pts.head[id];
  bool store = true;
  if (cnt > 0) {
    int last = (head + p.n_vp - 1) % p.n_vp;
    const int32_t *v = pts.vp + ((int64_t)id * kMaxVp + last) * 3;
    int64_t d0 = (int64_t)Q.x - v[0], d1 = (int64_t)Q.y - v[1], d2 = (int64_t)Q.z - v[2];
    store = d0 * d0 + d1 * d1 + d2 * d2 > p.dmin2;
  }
  if (store) {
    int32_t *v = pts.vp + ((int64_t)id * kMaxVp + head) * 3;
    v[0] = Q.x;
    v[1] = Q.y;
    v[2] = Q.z;
    pts.head[id] = (head + 1) % p.n_vp;
    pts.nvp[id] = cnt < p.n_vp ? cnt + 1 : cnt;
  }
}

// ------------------------------------------------------------ fold/bricks
// Two-bit code of one voxel: bit 0 TSDF < r_c, bit 1 unknown and not cleared.
__device__ inline uint32_t voxel_code(const Params &p, int32_t S, int32_t W, bool cleared) {
  bool occ = W > 0 && (int64_t)S < (int64_t)p.rc_u * W;
  bool unk = W == 0 && !cleared;
  return (occ ? 1u : 0u) | (unk ? 2u : 0u);
}

// Block `id` (512 threads, one voxel each; `code` is workgroup scratch)
// written to its brick of the grid.  clrw is the block's cleared-bit word of
// this thread's voxel, surfw its surface word t - 32 (threads 32..47), both
// loaded by the caller (early, so the loads overlap other work); bkey its key.
__device__ void write_brick(const Params &p, MapDev m, GridDev g, int64_t id, int32_t S,
                            int32_t W, uint8_t *code, uint32_t clrw, uint32_t surfw,
                            int64_t bkey) {
  int t = threadIdx.x;
  bool cl = (clrw >> (t & 31)) & 1u;
  uint32_t cd = voxel_code(p, S, W, cl);
  code[t] = (uint8_t)cd;
  int any_occ = __syncthreads_or((int)(cd & 1u));
  // occupancy of the brick's eight 4^3 octants: each wave holds one z slice
  // (64 voxels, lane = x | y << 3), so four masks of its ballot give the
  // slice's four (x, y) quadrants
  __shared__ uint32_t s_occ4;
  const uint64_t bal = __ballot(cd & 1u);
  {
    uint32_t nib = (uint32_t)((bal & 0x000000000F0F0F0Full) != 0) |
                   ((uint32_t)((bal & 0x00000000F0F0F0F0ull) != 0) << 1) |
                   ((uint32_t)((bal & 0x0F0F0F0F00000000ull) != 0) << 2) |
                   ((uint32_t)((bal & 0xF0F0F0F000000000ull) != 0) << 3);
    if (t == 0) s_occ4 = 0u;
    __syncthreads();
    if ((t & 63) == 0 && nib) atomicOr(&s_occ4, nib << (4 * ((t >> 8) & 1)));
    __syncthreads();
  }
  int32_t b[3];
  unpack_key(bkey, b[0], b[1], b[2]);
  int x = b[0] - g.g0[0], y = b[1] - g.g0[1], z = b[2] - g.g0[2];
  bool inside = (unsigned)x < (unsigned)g.gd[0] && (unsigned)y < (unsigned)g.gd[1] &&
                (unsigned)z < (unsigned)g.gd[2];
  if (inside) {
    int64_t brick = ((int64_t)z * g.gd[1] + y) * g.gd[0] + x;
    if (t < 32) {
      uint32_t w = 0;
      for (int j = 0; j < 16; ++j) w |= (uint32_t)code[t * 16 + j] << (2 * j);
      g.pred[brick * 32 + t] = w;
    } else if (t < 48) {
      g.surf[brick * 16 + (t - 32)] = surfw;
    } else if (t == 48) {
      uint32_t bit = 1u << (brick & 31);
      if (any_occ)
        atomicOr(&g.occ_any[brick >> 5], bit);
      else
        atomicAnd(&g.occ_any[brick >> 5], ~bit);
    } else if (t == 49) {
      g.occ4[brick] = (uint8_t)s_occ4;
    }
    if ((t & 63) == 0) {   // this wave's z slice: two words of the bit plane
      g.occ1[brick * 16 + 2 * (t >> 6)] = (uint32_t)bal;
      g.occ1[brick * 16 + 2 * (t >> 6) + 1] = (uint32_t)(bal >> 32);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------- binned integration
// Section 3.2 as a gather: every (return, block of its cube) pair is binned
// by block; one workgroup per touched block then gives each thread one voxel,
// which sums the clamped distances of the block's returns whose cube contains
// it (cone test, isqrt) in registers.  The fold with the weight cap
// (Section 3.6) and the block's brick follow in the same workgroup, so the
// map sees one plain store per voxel and no atomics.
__global__ void __launch_bounds__(kThreads)
k_bin_count(const FrameArgs *fa, Params p, MapDev m, FrameScratch fs) {
  const int64_t n = fa->n;
  int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n) return;
  int4 P = fs.P[r];
  if (P.w == 0) return;
  Span sp = cube_span(P, p.R);
  int ns = sp.n[0] * sp.n[1] * sp.n[2];
  for (int i = 0; i < ns; ++i) {
    int32_t s = fs.span[r * kMaxSpan + i];
    int32_t id = s >= 0 ? m.h.vals[s] : -1;
    if (id >= 0) atomicAdd(&fs.bin_cnt[m.tpos[id]], 1);
  }
}

// Exclusive prefix of the bin counts (one workgroup).
__global__ void __launch_bounds__(1024) k_bin_scan(FrameScratch fs, FrameCounters *c) {
  __shared__ int part[1024];
  const int nt = c->n_touched;
  const int t = threadIdx.x;
  const int seg = (nt + 1023) / 1024;
  const int lo = t * seg < nt ? t * seg : nt;
  const int hi = lo + seg < nt ? lo + seg : nt;
  int sum = 0;
  for (int j = lo; j < hi; ++j) sum += fs.bin_cnt[j];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;
  for (int j = lo; j < hi; ++j) {
    fs.bin_off[j] = run;
    fs.bin_fill[j] = run;
    run += fs.bin_cnt[j];
  }
  if (t == 1023) fs.bin_off[nt] = part[1023];
}

__global__ void __launch_bounds__(kThreads)
k_bin_fill(const FrameArgs *fa, Params p, MapDev m, FrameScratch fs) {
  const int64_t n = fa->n;
  int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n) return;
  int4 P = fs.P[r];
  if (P.w == 0) return;
  Span sp = cube_span(P, p.R);
  int ns = sp.n[0] * sp.n[1] * sp.n[2];
  for (int i = 0; i < ns; ++i) {
    int32_t s = fs.span[r * kMaxSpan + i];
    int32_t id = s >= 0 ? m.h.vals[s] : -1;
    if (id >= 0) fs.bin_list[atomicAdd(&fs.bin_fill[m.tpos[id]], 1)] = (int32_t)r;
  }
}

// LIST: also list every voxel that received a contribution (incremental
// mode); a separate instance, so the plain fold keeps its register budget.
template <int LIST>
__global__ void __launch_bounds__(kBlockVox)
k_integrate_fold(const FrameArgs *fa, Params p, MapDev m, FrameScratch fs, FrameCounters *c,
                 GridDev g) {
  const int3 Q = fa->Q;
  __shared__ int4 tile[kBlockVox];
  __shared__ int64_t tile_bb[kBlockVox];   // |P - Q|^2 of each return of the tile
  __shared__ int s_list[kBlockVox / 64 + 1]; // LIST: per-wave offsets, then the block's base
  __shared__ uint8_t code[kBlockVox];
  __shared__ unsigned long long s_stat[3];
  if (threadIdx.x < 3) s_stat[threadIdx.x] = 0ull;
  const int nt = c->n_touched;
  const int t = threadIdx.x;
  const int64_t lo_clamp = p.clamp_neg ? -(int64_t)p.tau_u : 0;
  unsigned applied = 0, excluded = 0, folded = 0;
  for (int i = blockIdx.x; i < nt; i += gridDim.x) {
    const int64_t id = fs.touched[i];
    // the block's own words first: their latency overlaps the gather below
    const int64_t v = id * kBlockVox + t;
    const int32_t S0 = m.S[v];
    const int32_t W0 = m.W[v];
    const uint32_t clrw = m.clr[id * 16 + (t >> 5)];
    const uint32_t surfw = (t >= 32 && t < 48) ? m.surf[id * 16 + (t - 32)] : 0u;
    const int64_t bkey = m.bkey[id];
    int32_t b[3];
    unpack_key(bkey, b[0], b[1], b[2]);
    if (t == 0) {
      bool in = true;
      for (int a = 0; a < 3; ++a)
        in = in && b[a] - g.g0[a] >= g.margin && b[a] - g.g0[a] < g.gd[a] - g.margin;
      if (!in) atomicOr(&c->status, kStatusOutsideGrid);
    }
    const int vx = 8 * b[0] + (t & 7), vy = 8 * b[1] + ((t >> 3) & 7), vz = 8 * b[2] + (t >> 6);
    const int64_t cq0 = 256 * (int64_t)vx + 128 - Q.x;  // voxel centre - sensor
    const int64_t cq1 = 256 * (int64_t)vy + 128 - Q.y;
    const int64_t cq2 = 256 * (int64_t)vz + 128 - Q.z;
    const int64_t dist_c = isqrt64(cq0 * cq0 + cq1 * cq1 + cq2 * cq2);
    const int beg = fs.bin_off[i], end = fs.bin_off[i + 1];
    int64_t dS = 0;
    int dW = 0;
    for (int tb = beg; tb < end; tb += kBlockVox) {
      __syncthreads();
      if (tb + t < end) {
        const int4 P = fs.P[fs.bin_list[tb + t]];
        tile[t] = P;
        const int64_t b0 = (int64_t)P.x - Q.x, b1 = (int64_t)P.y - Q.y, b2 = (int64_t)P.z - Q.z;
        tile_bb[t] = b0 * b0 + b1 * b1 + b2 * b2;
      }
      __syncthreads();
      const int cnt = end - tb < kBlockVox ? end - tb : kBlockVox;
      for (int j = 0; j < cnt; ++j) {
        const int4 P = tile[j];
        int ex = vx - (P.x >> 8), ey = vy - (P.y >> 8), ez = vz - (P.z >> 8);
        ex = ex < 0 ? -ex : ex;
        ey = ey < 0 ? -ey : ey;
        ez = ez < 0 ? -ez : ez;
        if (ex > p.R || ey > p.R || ez > p.R) continue;
        // 32-bit components: |a| <= 256 (R + 1) inside the cube, |b| < 2^29
        // (fixed-point coordinates are bounded by 2^28)
        const int32_t a0 = 256 * vx + 128 - P.x, a1 = 256 * vy + 128 - P.y,
                      a2 = 256 * vz + 128 - P.z;
        const int32_t b0 = P.x - Q.x, b1 = P.y - Q.y, b2 = P.z - Q.z;
        const int64_t ab = (int64_t)a0 * b0 + (int64_t)a1 * b1 + (int64_t)a2 * b2;
        // behind the return within the cos > 0.95 cone: 400 (a.b)^2 > 361 |a|^2 |b|^2.
        // Decided in double when the sides differ by more than 2^-40 relative
        // (each side is within 2^-50 of its exact value: |a.b| < 2^53 converts
        // exactly, |b|^2 rounds once, three roundings per product), otherwise
        // in 128-bit integers.
        if (ab > 0) {
          const int64_t aa = (int64_t)a0 * a0 + (int64_t)a1 * a1 + (int64_t)a2 * a2;
          const int64_t bb = tile_bb[j];
          const double x = 400.0 * (double)ab * (double)ab;
          const double y = 361.0 * (double)aa * (double)bb;
          bool behind;
          if (x > y * (1.0 + 0x1p-40))
            behind = true;
          else if (x < y * (1.0 - 0x1p-40))
            behind = false;
          else
            behind = (__int128)400 * ab * ab > (__int128)361 * aa * bb;
          if (behind) {
            ++excluded;
            continue;
          }
        }
        ++applied;
        int64_t d = (int64_t)P.w - dist_c;
        d = d < lo_clamp ? lo_clamp : (d > p.tau_u ? p.tau_u : d);
        dS += d;
        ++dW;
      }
    }
    int32_t S = S0;
    int32_t W = W0;
    if (dW > 0) {
      int64_t S2 = (int64_t)S + dS, W2 = (int64_t)W + dW;
      if (W2 > p.cap) {
        S2 = div_floor(S2 * p.cap, W2);
        W2 = p.cap;
      }
      S = (int32_t)S2;
      W = (int32_t)W2;
      m.S[v] = S;
      m.W[v] = (uint16_t)W;
      ++folded;
    }
    if (LIST) {   // list this voxel if it received a contribution (one atomic per block)
      const unsigned long long bal = __ballot(dW > 0);
      const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
      if (lane == 0) s_list[wave] = __popcll(bal);
      __syncthreads();
      if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < kBlockVox / 64; ++k) {
          const int n = s_list[k];
          s_list[k] = tot;
          tot += n;
        }
        s_list[kBlockVox / 64] = tot ? atomicAdd(&c->n_changed, tot) : 0;
      }
      __syncthreads();
      if (dW > 0)
        fs.changed[s_list[kBlockVox / 64] + s_list[wave] +
                   __popcll(bal & ((1ull << lane) - 1ull))] = (int32_t)v;
    }
    write_brick(p, m, g, id, S, W, code, clrw, surfw, bkey);
  }
  unsigned long long sa = applied, se = excluded, sf = folded;
  for (int off = 32; off >= 1; off >>= 1) {
    sa += __shfl_xor((unsigned)sa, off);
    se += __shfl_xor((unsigned)se, off);
    sf += __shfl_xor((unsigned)sf, off);
  }
  __syncthreads();
  if (lane_id() == 0) {
    if (sa) atomicAdd(&s_stat[0], sa);
    if (se) atomicAdd(&s_stat[1], se);
    if (sf) atomicAdd(&s_stat[2], sf);
  }
  __syncthreads();
  if (threadIdx.x < 3 && s_stat[threadIdx.x])
    atomicAdd(&c->fold[blockIdx.x % kStatSlots][threadIdx.x], s_stat[threadIdx.x]);
}

__global__ void __launch_bounds__(kBlockVox)
k_grid_rebuild(Params p, MapDev m, GridDev g, int64_t n_blocks) {
  __shared__ uint8_t code[kBlockVox];
  for (int64_t id = blockIdx.x; id < n_blocks; id += gridDim.x) {
    if (m.bkey[id] == kEmpty) continue;   // an evicted block's free id
    const int t = threadIdx.x;
    const int64_t v = id * kBlockVox + t;
    write_brick(p, m, g, id, m.S[v], m.W[v], code, m.clr[id * 16 + (t >> 5)],
                (t >= 32 && t < 48) ? m.surf[id * 16 + (t - 32)] : 0u, m.bkey[id]);
  }
}

__global__ void k_grid_fill(GridDev g, int64_t nbricks) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < nbricks * 32; j += stride) g.pred[j] = kUnknownWord;
  for (int64_t j = i; j < nbricks * 16; j += stride) g.surf[j] = 0u;
  for (int64_t j = i; j < (nbricks + 31) / 32; j += stride) g.occ_any[j] = 0u;
  for (int64_t j = i; j < nbricks; j += stride) g.occ4[j] = 0u;
  for (int64_t j = i; j < nbricks * 16; j += stride) g.occ1[j] = 0u;
}

__global__ void k_stick_status(FrameCounters *c, const int32_t *n_blocks,
                               const int32_t *n_points) {
  c->sticky |= c->status;
  if (c->n_new_blocks > 0)
    for (int a = 0; a < 3; ++a) {
      c->sbmin[a] = c->bmin[a] < c->sbmin[a] ? c->bmin[a] : c->sbmin[a];
      c->sbmax[a] = c->bmax[a] > c->sbmax[a] ? c->bmax[a] : c->sbmax[a];
    }
  c->snap_blocks = *n_blocks;
  c->snap_points = *n_points;
}

__global__ void k_zero_words(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void k_set_frame_args(FrameArgs *fa, int64_t n, int3 Q, int32_t frame, int3 wlo,
                                 int3 whi, FrameCounters *clear) {
  fa->n = n;
  fa->Q = Q;
  fa->frame = frame;
  fa->wlo = wlo;
  fa->whi = whi;
  if (clear) {
    clear->sticky = 0;
    for (int a = 0; a < 3; ++a) {
      clear->sbmin[a] = 0x7fffffff;
      clear->sbmax[a] = -0x7fffffff - 1;
    }
  }
}

// ------------------------------------------------------- sliding window
// One workgroup per block id: a live block outside [lo, hi] is cleared (its
// voxels read unknown again), its key removed and its id pushed on the free
// list.
__global__ void __launch_bounds__(kThreads)
k_window_evict(MapDev m, int64_t n_blocks, int3 lo, int3 hi) {
  for (int64_t id = blockIdx.x; id < n_blocks; id += gridDim.x) {
    const int64_t key = m.bkey[id];
    if (key == kEmpty) continue;
    int32_t b[3];
    unpack_key(key, b[0], b[1], b[2]);
    if (in_box(b[0], b[1], b[2], lo, hi)) continue;
    for (int t = threadIdx.x; t < kBlockVox; t += kThreads) {
      m.S[id * kBlockVox + t] = 0;
      m.W[id * kBlockVox + t] = 0;
    }
    if (threadIdx.x < 16) {
      m.clr[id * 16 + threadIdx.x] = 0;
      m.surf[id * 16 + threadIdx.x] = 0;
    }
    __syncthreads();   // every thread has read bkey[id] before it changes
    if (threadIdx.x == 0) {
      m.bkey[id] = kEmpty;
      m.touched[id] = -1;
      m.free_ids[atomicAdd(m.n_free, 1)] = (int32_t)id;
    }
  }
}

__global__ void k_hash_clear(HashTable h) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= (int64_t)h.mask;
       i += (int64_t)gridDim.x * blockDim.x) {
    h.keys[i] = kEmpty;
    h.vals[i] = -1;
  }
}

// Live blocks back into the cleared hash.
__global__ void __launch_bounds__(kThreads) k_window_rehash(MapDev m, int64_t n_blocks) {
  const int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (id >= n_blocks) return;
  const int64_t key = m.bkey[id];
  if (key == kEmpty) return;
  bool fresh;
  const int32_t s = hash_insert(m.h, key, fresh);
  if (s >= 0) m.h.vals[s] = (int32_t)id;   // the hash holds 2 max_blocks slots: never full
}

__device__ inline void point_block(const PointsDev &pts, int64_t i, int32_t v[3]) {
  unpack_key(pts.key[i], v[0], v[1], v[2]);
}

// Points outside [lo, hi] lose their voxel address (their block is gone).
__global__ void __launch_bounds__(kThreads)
k_window_points(PointsDev pts, int64_t n_points, int3 lo, int3 hi) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n_points) return;
  int32_t v[3];
  point_block(pts, i, v);
  if (!in_box(v[0] >> 3, v[1] >> 3, v[2] >> 3, lo, hi)) pts.addr[i] = -1;
}

// Points inside [lo, hi] without a block: their block joins the frame's new
// blocks (assigned and cleared with them).
__global__ void __launch_bounds__(kThreads)
k_window_thaw(MapDev m, PointsDev pts, FrameScratch fs, FrameCounters *c, int64_t n_points,
              int3 lo, int3 hi) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n_points || pts.addr[i] >= 0) return;
  int32_t v[3];
  point_block(pts, i, v);
  if (!in_box(v[0] >> 3, v[1] >> 3, v[2] >> 3, lo, hi)) return;
  bool fresh;
  const int32_t s = hash_insert(m.h, pack_key(v[0] >> 3, v[1] >> 3, v[2] >> 3), fresh);
  if (s < 0) atomicOr(&c->status, kStatusHashFull);
  if (fresh) fs.new_blocks[atomicAdd(&c->n_new_blocks, 1)] = s;
}

// After assignment: those points get their voxel address and surface bit.
__global__ void __launch_bounds__(kThreads)
k_window_link(MapDev m, PointsDev pts, int64_t n_points, int3 lo, int3 hi) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n_points || pts.addr[i] >= 0) return;
  int32_t v[3];
  point_block(pts, i, v);
  if (!in_box(v[0] >> 3, v[1] >> 3, v[2] >> 3, lo, hi)) return;
  const int32_t bs = hash_find(m.h, pack_key(v[0] >> 3, v[1] >> 3, v[2] >> 3));
  const int32_t bid = bs >= 0 ? m.h.vals[bs] : -1;
  if (bid < 0) return;   // block capacity exhausted (the frame reports it)
  const int vi = (v[0] & 7) | ((v[1] & 7) << 3) | ((v[2] & 7) << 6);
  pts.addr[i] = bid * kBlockVox + vi;
  atomicOr(&m.surf[(int64_t)bid * 16 + (vi >> 5)], 1u << (vi & 31));
}

// Points inside [lo, hi] listed: the waves' counts are combined in LDS, so
// a workgroup of 1024 points takes one atomic on the list's counter (one per
// wave serialised some 30,000 atomics on that address per call).  A negative
// n_points reads the count on the device (a recorded frame).
constexpr int kListThreads = 1024;
__global__ void __launch_bounds__(kListThreads)
k_window_list(PointsDev pts, int64_t n_points, int3 lo, int3 hi, int32_t *sel, int32_t *n_sel) {
  __shared__ int part[kListThreads / 64 + 1];
  const int64_t i = (int64_t)blockIdx.x * kListThreads + threadIdx.x;
  const int64_t n = n_points < 0 ? (int64_t)*pts.n_points : n_points;
  bool take = false;
  if (i < n) {
    int32_t v[3];
    point_block(pts, i, v);
    take = in_box(v[0] >> 3, v[1] >> 3, v[2] >> 3, lo, hi);
  }
  const unsigned long long bal = __ballot(take);
  const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
  if (lane == 0) part[wave] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int k = 0; k < kListThreads / 64; ++k) {
      const int c = part[k];
      part[k] = tot;
      tot += c;
    }
    part[kListThreads / 64] = tot ? atomicAdd(n_sel, tot) : 0;
  }
  __syncthreads();
  if (take)
    sel[part[kListThreads / 64] + part[wave] + __popcll(bal & ((1ull << lane) - 1ull))] =
        (int32_t)i;
}

__global__ void k_label_fill(uint8_t *label, int16_t *ff, int64_t from, int64_t to) {
  for (int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < to;
       i += (int64_t)gridDim.x * blockDim.x) {
    label[i] = 255;
    ff[i] = -1;
  }
}

inline unsigned grid_for(int64_t threads) {
  int64_t b = (threads + kThreads - 1) / kThreads;
  return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

void launch_zero_words(void *p, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 4;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256)),
                     dim3(256), 0, s, (uint32_t *)p, n);
}

void launch_stick_status(FrameCounters *c, const int32_t *n_blocks, const int32_t *n_points,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_stick_status, dim3(1), dim3(1), 0, s, c, n_blocks, n_points);
}

void launch_set_frame_args(FrameArgs *fa, int64_t n, int3 Q, int32_t frame, int3 wlo, int3 whi,
                           hipStream_t s, FrameCounters *clear) {
  hipLaunchKernelGGL(k_set_frame_args, dim3(1), dim3(1), 0, s, fa, n, Q, frame, wlo, whi, clear);
}

void launch_window_evict(MapDev m, PointsDev pts, int64_t n_blocks, int64_t n_points, int3 lo,
                         int3 hi, hipStream_t s) {
  if (n_blocks > 0)
    hipLaunchKernelGGL(k_window_evict, dim3((unsigned)std::min<int64_t>(n_blocks, 8192)),
                       dim3(kThreads), 0, s, m, n_blocks, lo, hi);
  const int64_t slots = (int64_t)m.h.mask + 1;
  hipLaunchKernelGGL(k_hash_clear, dim3((unsigned)std::min<int64_t>(4096, (slots + 255) / 256)),
                     dim3(256), 0, s, m.h);
  if (n_blocks > 0)
    hipLaunchKernelGGL(k_window_rehash, dim3(grid_for(n_blocks)), dim3(kThreads), 0, s, m,
                       n_blocks);
  if (n_points > 0)
    hipLaunchKernelGGL(k_window_points, dim3(grid_for(n_points)), dim3(kThreads), 0, s, pts,
                       n_points, lo, hi);
}

void launch_window_thaw(MapDev m, PointsDev pts, FrameScratch fs, FrameCounters *c,
                        int64_t n_points, int3 lo, int3 hi, hipStream_t s) {
  if (n_points > 0)
    hipLaunchKernelGGL(k_window_thaw, dim3(grid_for(n_points)), dim3(kThreads), 0, s, m, pts, fs,
                       c, n_points, lo, hi);
}

void launch_window_link(MapDev m, PointsDev pts, int64_t n_points, int3 lo, int3 hi,
                        hipStream_t s) {
  if (n_points > 0)
    hipLaunchKernelGGL(k_window_link, dim3(grid_for(n_points)), dim3(kThreads), 0, s, m, pts,
                       n_points, lo, hi);
}

void launch_window_list(PointsDev pts, int64_t n_points, int3 lo, int3 hi, int32_t *sel,
                        int32_t *n_sel, hipStream_t s, bool dev_n) {
  launch_zero_words(n_sel, sizeof(int32_t), s);
  if (n_points > 0)
    hipLaunchKernelGGL(k_window_list, dim3((unsigned)((n_points + kListThreads - 1) / kListThreads)),
                       dim3(kListThreads), 0, s, pts, dev_n ? (int64_t)-1 : n_points, lo, hi, sel,
                       n_sel);
}

void launch_label_fill(uint8_t *label, int16_t *first_free, int64_t from, int64_t to,
                       hipStream_t s) {
  if (to > from)
    hipLaunchKernelGGL(k_label_fill,
                       dim3((unsigned)std::min<int64_t>(1024, (to - from + 255) / 256)),
                       dim3(256), 0, s, label, first_free, from, to);
}

void launch_frame_prep(const float *xyz, const FrameArgs *fa, int64_t nb, const Params &p,
                       MapDev m, PointsDev pts, FrameScratch fs, FrameCounters *c,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(1), 0, s, c, m, pts);
  if (nb > 0)
    hipLaunchKernelGGL(k_frame_prep, dim3(grid_for(nb)), dim3(kThreads), 0, s, xyz, fa, p, m,
                       pts, fs, c);
}

void launch_assign_blocks(MapDev m, FrameScratch fs, FrameCounters *c, const FrameArgs *fa,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_assign_blocks, dim3(4096), dim3(kThreads), 0, s, m, fs, c, fa);
}

void launch_commit_blocks(MapDev m, FrameCounters *c, hipStream_t s) {
  hipLaunchKernelGGL(k_commit_blocks, dim3(1), dim3(1), 0, s, m, c);
}

void launch_integrate(const FrameArgs *fa, int64_t nb, const Params &p, MapDev m,
                      FrameScratch fs, FrameCounters *c, GridDev g, int64_t max_touched,
                      hipStream_t s) {
  if (nb > 0) {
    hipLaunchKernelGGL(k_bin_count, dim3(grid_for(nb)), dim3(kThreads), 0, s, fa, p, m, fs);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, fs, c);
    hipLaunchKernelGGL(k_bin_fill, dim3(grid_for(nb)), dim3(kThreads), 0, s, fa, p, m, fs);
  } else {
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, fs, c);
  }
  int64_t wg = max_touched < 8192 ? max_touched : 8192;
  if (wg > 0) {
    if (fs.changed)
      hipLaunchKernelGGL(k_integrate_fold<1>, dim3((unsigned)wg), dim3(kBlockVox), 0, s, fa, p,
                         m, fs, c, g);
    else
      hipLaunchKernelGGL(k_integrate_fold<0>, dim3((unsigned)wg), dim3(kBlockVox), 0, s, fa, p,
                         m, fs, c, g);
  }
}

void launch_touch_band(const FrameArgs *fa, int64_t nb, const Params &p, MapDev m,
                       FrameScratch fs, FrameCounters *c, hipStream_t s) {
  if (nb > 0)
    hipLaunchKernelGGL(k_touch_band, dim3(grid_for(nb)), dim3(kThreads), 0, s, fa, p, m, fs,
                       c);
}

void launch_points_append(int64_t n_new, MapDev m, PointsDev pts, FrameScratch fs,
                          FrameCounters *c, const FrameArgs *fa, hipStream_t s) {
  if (n_new > 0) {
    hipLaunchKernelGGL(k_sort_new_tiles, dim3(grid_for(n_new)), dim3(kThreads), 0, s, fs, c);
    hipLaunchKernelGGL(k_points_append, dim3(grid_for(n_new)), dim3(kThreads), 0, s, m, pts,
                       fs, c, fa);
  }
}

void launch_commit_points(PointsDev pts, FrameCounters *c, hipStream_t s) {
  hipLaunchKernelGGL(k_commit_points, dim3(1), dim3(1), 0, s, pts, c);
}

void launch_points_view(const FrameArgs *fa, int64_t nb, const Params &p, PointsDev pts,
                        FrameScratch fs, hipStream_t s) {
  if (nb > 0)
    hipLaunchKernelGGL(k_points_view, dim3(grid_for(nb)), dim3(kThreads), 0, s, fa, p, pts,
                       fs);
}

void launch_grid_fill(GridDev g, hipStream_t s) {
  int64_t nb = (int64_t)g.gd[0] * g.gd[1] * g.gd[2];
  int64_t blocks = (nb * 32 + kThreads - 1) / kThreads;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_grid_fill, dim3((unsigned)blocks), dim3(kThreads), 0, s, g, nb);
}

void launch_grid_rebuild(const Params &p, MapDev m, GridDev g, int64_t n_blocks,
                         hipStream_t s) {
  int64_t wg = n_blocks < 8192 ? n_blocks : 8192;
  if (wg > 0)
    hipLaunchKernelGGL(k_grid_rebuild, dim3((unsigned)wg), dim3(kBlockVox), 0, s, p, m, g,
                       n_blocks);
}

}  // namespace af
