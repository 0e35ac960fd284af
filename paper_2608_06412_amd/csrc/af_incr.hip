// Incremental mode (Section 3.5, "Incremental Updates and Confidence").
//
// A per-point state carries the best stored direction score (the raw
// collision count of a free orientation; n_c when none was ever free), that
// direction, the accessibility confidence a and a queued flag.  Each frame,
// after integration:
//   triggers  (i) the TSDF at the point's voxel moved by more than 2v (exact
//             in S/W), (iii) the sensor moved more than 0.1 m since the last
//             time this fired: points labelled inaccessible are queued; new
//             points are queued on first observation;
//   sample    the 256 changed voxels (voxels that received a contribution)
//             with the smallest SplitMix64 hash of key ^ frame * golden,
//             found by two 16-bit radix histograms and one small sort;
//             (ii) queues every point within 3v of a sampled voxel;
//   select    queued points with W >= the confidence minimum, the first
//             `budget` in point order (block counts, a scan, a ranked write);
//             the rest stay queued;
//   evaluate  normals, masks and the default scoring kernel on that list;
//             the raw collision count of each free orientation found;
//   update    a *= 0.75 when a blocked finding contradicts a stored free
//             direction, a += 0.15 (1 - a) on a free finding, stored score
//             only decreases; labels: accessible iff score < n_c and
//             c a > 0.7 with c = W / (W + 5).
// fp64 state arithmetic is written as plain operations (contraction is off
// for this file), so every replay rounds the same way.

#include "af_internal.h"

namespace af {
namespace {

constexpr int kT = 256;
constexpr int kSelT = 1024;         // points per selection block
constexpr int kSample = 256;        // changed voxels sampled per frame
constexpr int kCand = 1024;         // candidate capacity of the sample sort
constexpr unsigned long long kGolden = 0x9E3779B97F4A7C15ull;

// The output function of SplitMix64 (Steele, Lea and Flood).
__device__ inline unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Whether voxel (x, y, z) lies in the sliding window's block box.
__device__ inline bool in_window(const IncrDev &I, int32_t x, int32_t y, int32_t z) {
  return (x >> 3) >= I.wlo.x && (x >> 3) <= I.whi.x && (y >> 3) >= I.wlo.y &&
         (y >> 3) <= I.whi.y && (z >> 3) >= I.wlo.z && (z >> 3) <= I.whi.z;
}

__device__ inline int64_t voxel_key(const MapDev &m, int32_t addr) {
  int32_t b[3];
  unpack_key(m.bkey[addr >> 9], b[0], b[1], b[2]);
  const int lin = addr & 511;
  return pack_key(8 * (int64_t)b[0] + (lin & 7), 8 * (int64_t)b[1] + ((lin >> 3) & 7),
                  8 * (int64_t)b[2] + (lin >> 6));
}

__device__ inline unsigned long long sample_hash(int64_t key, int32_t frame) {
  return mix64((unsigned long long)key ^ ((unsigned long long)(int64_t)frame * kGolden));
}

// Workgroup counts of three per-thread flags (ballots, one exchange), added
// to d0, d1, d2 by thread 0.
template <int NT>
__device__ inline void wg_count3(bool f0, bool f1, bool f2, int *d0, int *d1, int *d2) {
  __shared__ int part[3][NT / 64];
  const uint64_t b0 = __ballot(f0), b1 = __ballot(f1), b2 = __ballot(f2);
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = __popcll(b0);
    part[1][threadIdx.x >> 6] = __popcll(b1);
    part[2][threadIdx.x >> 6] = __popcll(b2);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t0 = 0, t1 = 0, t2 = 0;
    for (int w = 0; w < NT / 64; ++w) {
      t0 += part[0][w];
      t1 += part[1][w];
      t2 += part[2][w];
    }
    if (t0) atomicAdd(d0, t0);
    if (t1) atomicAdd(d1, t1);
    if (t2) atomicAdd(d2, t2);
  }
}

// Workgroup sum of one value per thread, added to *dst by thread 0.
template <int NT>
__device__ inline void wg_add(int v, int *dst) {
  __shared__ int part[NT / 64];
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < NT / 64; ++w) t += part[w];
    if (t) atomicAdd(dst, t);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kT) k_incr_fill(uint32_t *a, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    a[i] = v;
}

// State of every point at enable time: nothing stored, not queued.
__global__ void __launch_bounds__(kT) k_incr_init(IncrDev I, int32_t n_c) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < I.max_points;
       i += (int64_t)gridDim.x * kT) {
    I.best[i] = (uint8_t)n_c;
    I.best_dir[i] = -1;
    I.a[i] = 1.0;
    I.S_prev[i] = 0;
    I.W_prev[i] = 0;
    I.pending[i] = 0u;
    I.outcome[i] = AF_UNSCORED;
    I.label[i] = AF_UNSCORED;
  }
}

// Triggers (i), (iii) and first observation; the point's S and W are kept
// for the next frame.
__global__ void __launch_bounds__(kT)
k_incr_triggers(PointsDev pts, MapDev m, IncrDev I, int64_t n, int64_t seen, int moved) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  int c_new = 0, c_i = 0, c_iii = 0;
  if (i < n) {
    const int32_t addr = pts.addr[i];
    const int64_t S = addr >= 0 ? (int64_t)m.S[addr] : 0;
    const int64_t W = addr >= 0 ? (int64_t)m.W[addr] : 0;
    if (i >= seen) {   // first observation (points are appended, never removed)
      I.pending[i] = 1u;
      c_new = 1;
    } else {
      const int64_t Sp = I.S_prev[i], Wp = I.W_prev[i];
      if (Wp > 0 && W > 0) {
        int64_t d = S * Wp - Sp * W;
        d = d < 0 ? -d : d;
        if (d > 512 * W * Wp) c_i = 1;   // |S/W - S'/W'| > 2v (2v = 512 units)
      }
      const uint8_t lb = I.label[i];
      if (moved && (lb == AF_BLOCKED || lb == AF_NO_CANDIDATE)) {
        int32_t x, y, z;   // (iii) takes the points inside the sliding window
        unpack_key(pts.key[i], x, y, z);
        c_iii = in_window(I, x, y, z);
      }
      if (c_i || c_iii) I.pending[i] = 1u;
    }
    I.S_prev[i] = (int32_t)S;
    I.W_prev[i] = (uint16_t)W;
  }
  wg_count3<kT>(c_new != 0, c_i != 0, c_iii != 0, &I.ctr->new_points, &I.ctr->trig_i,
                 &I.ctr->trig_iii);
}

// Histogram of the top 16 hash bits over the frame's changed voxels (level 0),
// or of bits 32..47 over those in the chosen top bin (level 1).
__global__ void __launch_bounds__(kT)
k_incr_hist(MapDev m, const int32_t *changed, const FrameCounters *fc, int32_t frame, IncrDev I,
            int level) {
  const int64_t nc = fc->n_changed;
  if (level == 1 && I.ctr->take_all) return;
  for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < nc; j += (int64_t)gridDim.x * kT) {
    const unsigned long long h = sample_hash(voxel_key(m, changed[j]), frame);
    if (level == 0)
      atomicAdd(&I.hist[h >> 48], 1u);
    else if ((int)(h >> 48) == I.ctr->b1)
      atomicAdd(&I.hist[65536 + ((h >> 32) & 0xffffu)], 1u);
  }
}

// One workgroup: the smallest bin at which the running count of `hist`
// reaches `need` (65536 bins, 64 per thread).
__device__ inline void find_bin(const uint32_t *hist, int need, int &bin, int &below) {
  __shared__ int sums[kSelT];
  const int t = threadIdx.x;
  int s = 0;
  for (int k = 0; k < 64; ++k) s += (int)hist[64 * t + k];
  sums[t] = s;
  __syncthreads();
  for (int off = 1; off < kSelT; off <<= 1) {
    const int v = t >= off ? sums[t - off] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  const int incl = sums[t], excl = incl - s;
  if (excl < need && incl >= need) {   // exactly one thread
    int run = excl;
    for (int k = 0; k < 64; ++k) {
      const int c = (int)hist[64 * t + k];
      if (run + c >= need) {
        bin = 64 * t + k;
        below = run;
        break;
      }
      run += c;
    }
  }
}

__global__ void __launch_bounds__(kSelT) k_incr_pick(const FrameCounters *fc, IncrDev I, int level) {
  IncrCounters *c = I.ctr;
  if (level == 0) {
    const int nc = fc->n_changed;
    if (nc <= kSample) {
      if (threadIdx.x == 0) c->take_all = 1;
      return;
    }
    int bin = -1, below = 0;
    find_bin(I.hist, kSample, bin, below);
    if (bin >= 0) {
      c->b1 = bin;
      c->need = kSample - below;
    }
  } else {
    if (c->take_all) return;
    int bin = -1, below = 0;
    find_bin(I.hist + 65536, c->need, bin, below);
    if (bin >= 0) c->b2 = bin;
  }
}

// Changed voxels whose hash is at most the selected prefix: the 256 smallest,
// plus any sharing the last 32-bit prefix.
__global__ void __launch_bounds__(kT)
k_incr_collect(MapDev m, const int32_t *changed, const FrameCounters *fc, int32_t frame,
               IncrDev I) {
  const int64_t nc = fc->n_changed;
  const IncrCounters *c = I.ctr;
  const int take_all = c->take_all, b1 = c->b1, b2 = c->b2;
  for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < nc; j += (int64_t)gridDim.x * kT) {
    const int64_t key = voxel_key(m, changed[j]);
    const unsigned long long h = sample_hash(key, frame);
    const int top = (int)(h >> 48), mid = (int)((h >> 32) & 0xffffu);
    if (take_all || top < b1 || (top == b1 && mid <= b2)) {
      const int slot = atomicAdd(&I.ctr->n_cand, 1);
      if (slot < kCand) {
        I.cand_h[slot] = h;
        I.cand_k[slot] = key;
      }
    }
  }
}

// Sort the candidates by hash (bitonic, one workgroup) and keep the first 256.
__global__ void __launch_bounds__(kSelT) k_incr_sort(IncrDev I) {
  __shared__ unsigned long long sh[kCand];
  __shared__ int64_t sk[kCand];
  const int t = threadIdx.x;
  const int n = I.ctr->n_cand < kCand ? I.ctr->n_cand : kCand;
  sh[t] = t < n ? I.cand_h[t] : ~0ull;
  sk[t] = t < n ? I.cand_k[t] : 0;
  __syncthreads();
  for (int k = 2; k <= kCand; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int q = t ^ j;
      if (q > t) {
        const unsigned long long a = sh[t], b = sh[q];
        if ((a > b) == ((t & k) == 0)) {
          sh[t] = b;
          sh[q] = a;
          const int64_t x = sk[t];
          sk[t] = sk[q];
          sk[q] = x;
        }
      }
      __syncthreads();
    }
  const int keep = n < kSample ? n : kSample;
  if (t < keep) I.sampled[t] = sk[t];
  if (t == 0) I.ctr->sampled = keep;
}

// Trigger (ii): every point within 3 voxels (|o|^2 <= 9) of a sampled voxel.
// One workgroup per sampled voxel, one thread per offset of the 7^3 cube.
__global__ void __launch_bounds__(384) k_incr_neigh(PointsDev pts, IncrDev I, int64_t n) {
  int hit = 0;
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  if (s < I.ctr->sampled && t < 343) {
    const int dx = t % 7 - 3, dy = (t / 7) % 7 - 3, dz = t / 49 - 3;
    if (dx * dx + dy * dy + dz * dz <= 9) {
      int32_t x, y, z;
      unpack_key(I.sampled[s], x, y, z);
      const int32_t slot = hash_find(pts.h, pack_key(x + dx, y + dy, z + dz));
      const int32_t pi = slot >= 0 ? pts.h.vals[slot] : -1;
      if (pi >= 0 && pi < n && atomicOr(&I.pending[pi], 1u) == 0u) hit = 1;
    }
  }
  wg_add<384>(hit, &I.ctr->trig_ii);
}

__device__ inline bool selectable(const PointsDev &pts, const MapDev &m, const IncrDev &I,
                                  int64_t i, int32_t min_w) {
  const int32_t addr = pts.addr[i];
  return I.pending[i] != 0u && addr >= 0 && (int32_t)m.W[addr] >= min_w;
}

// Selection, pass 1: selectable and queued points per block of 1024.
__global__ void __launch_bounds__(kSelT)
k_incr_sel_count(PointsDev pts, MapDev m, IncrDev I, int64_t n, int32_t min_w) {
  const int64_t i = (int64_t)blockIdx.x * kSelT + threadIdx.x;
  const int f = i < n && selectable(pts, m, I, i, min_w);
  const int q = i < n && I.pending[i] != 0u;
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const unsigned long long b = __ballot(f);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(&cnt, __popcll(b));
  __syncthreads();
  if (threadIdx.x == 0) I.bsum[blockIdx.x] = cnt;
  wg_add<kSelT>(q, &I.ctr->queued);
}

// Pass 2 (one workgroup): block offsets, the list length.
__global__ void __launch_bounds__(kSelT) k_incr_sel_scan(IncrDev I, int64_t nblk) {
  __shared__ int part[kSelT];
  const int t = threadIdx.x;
  const int64_t per = (nblk + kSelT - 1) / kSelT;
  const int64_t lo = t * per < nblk ? t * per : nblk, hi = lo + per < nblk ? lo + per : nblk;
  int s = 0;
  for (int64_t b = lo; b < hi; ++b) s += I.bsum[b];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < kSelT; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int64_t b = lo; b < hi; ++b) {
    const int c = I.bsum[b];
    I.bsum[b] = run;
    run += c;
  }
  if (t == kSelT - 1) {
    const int total = part[kSelT - 1];
    const int cap = *I.budget_dev;
    I.ctr->selectable = total;
    *I.n_sel = total < cap ? total : cap;
  }
}

// Pass 3: each selectable point's rank; the first `budget` are listed and
// leave the queue.
__global__ void __launch_bounds__(kSelT)
k_incr_sel_write(PointsDev pts, MapDev m, IncrDev I, int64_t n, int32_t min_w) {
  __shared__ int wave_base[kSelT / 64];
  const int64_t i = (int64_t)blockIdx.x * kSelT + threadIdx.x;
  const int f = i < n && selectable(pts, m, I, i, min_w);
  const unsigned long long b = __ballot(f);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wave_base[w] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int k = 0; k < kSelT / 64; ++k) {
      const int c = wave_base[k];
      wave_base[k] = run;
      run += c;
    }
  }
  __syncthreads();
  if (f) {
    const int rank = I.bsum[blockIdx.x] + wave_base[w] + __popcll(b & ((1ull << lane) - 1ull));
    if (rank < *I.budget_dev) {
      I.sel[rank] = (int32_t)i;
      I.pending[i] = 0u;
    }
  }
}

// Raw collision count (body voxels with TSDF < r_c) of each listed point's
// first free orientation; n_c for points without one.  Wave per point.
__global__ void __launch_bounds__(kT)
k_incr_count(PointsDev pts, ToolDev t, GridDev g, IncrDev I, int32_t n_c) {
  const int n = *I.n_sel;
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (kT / 64);
  for (int64_t j = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6; j < n; j += nw) {
    const int32_t pi = I.sel[j];
    int cnt = n_c;
    if (t.label[pi] == AF_ACCESSIBLE) {
      const int k = t.first_free[pi];
      int32_t s[3];
      unpack_key(pts.key[pi], s[0], s[1], s[2]);
      cnt = 0;
      // a table lists 3 arm samples, then the body entries, then the corridor
      // entries (from far_begin): only the body range is visited
      const uint32_t eb = t.far_begin[k];
      for (uint32_t e0 = t.begin[k] + 3; e0 < eb; e0 += 64) {
        const uint32_t e = e0 + lane;
        bool hit = false;
        if (e < eb) {
          const uint32_t ent = t.entries[e];
          if (entry_cls(ent) == AF_CLS_BODY) {
            const int x = s[0] + entry_x(ent), y = s[1] + entry_y(ent), z = s[2] + entry_z(ent);
            const int bx = (x >> 3) - g.g0[0], by = (y >> 3) - g.g0[1], bz = (z >> 3) - g.g0[2];
            if ((unsigned)bx < (unsigned)g.gd[0] && (unsigned)by < (unsigned)g.gd[1] &&
                (unsigned)bz < (unsigned)g.gd[2]) {
              const int64_t br = ((int64_t)bz * g.gd[1] + by) * g.gd[0] + bx;
              const int lin = (x & 7) | ((y & 7) << 3) | ((z & 7) << 6);
              hit = ((g.pred[br * 32 + (lin >> 4)] >> (2 * (lin & 15))) & 1u) != 0u;
            }
          }
        }
        cnt += __popcll(__ballot(hit));
      }
    }
    if (lane == 0) I.score_new[j] = (uint8_t)cnt;
  }
}

// State update of every listed point (one thread each).
__global__ void __launch_bounds__(kT) k_incr_update(ToolDev t, IncrDev I, int32_t n_c) {
  const int n = *I.n_sel;
  const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (j >= n) return;
  const int32_t pi = I.sel[j];
  const uint8_t outcome = t.label[pi];
  const int score = I.score_new[j];
  const int dir = outcome == AF_ACCESSIBLE ? t.first_free[pi] : -1;
  if (I.outcome[pi] != AF_UNSCORED) {
    const double a = I.a[pi];
    if (score < n_c)
      I.a[pi] = a + 0.15 * (1.0 - a);
    else if ((int)I.best[pi] < n_c)
      I.a[pi] = 0.75 * a;
  }
  if (score < (int)I.best[pi]) {
    I.best[pi] = (uint8_t)score;
    I.best_dir[pi] = (int16_t)dir;
  }
  I.outcome[pi] = outcome;
}

// Labels of every point from its state and the current weight.
__global__ void __launch_bounds__(kT)
k_incr_labels(PointsDev pts, MapDev m, IncrDev I, int64_t n, int32_t n_c) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  uint8_t lb = AF_UNSCORED;
  const uint8_t oc = I.outcome[i];
  if (oc != AF_UNSCORED) {
    if ((int)I.best[i] < n_c) {
      const int32_t addr = pts.addr[i];
      const double W = addr >= 0 ? (double)m.W[addr] : 0.0;
      const double c = W / (W + 5.0);
      lb = c * I.a[i] > 0.7 ? AF_ACCESSIBLE : AF_TENTATIVE;
    } else {
      lb = oc == AF_NO_CANDIDATE ? AF_NO_CANDIDATE : AF_BLOCKED;
    }
  }
  I.label[i] = lb;
}

// The next frame's cap from this frame's evaluation cost (one thread): n
// points evaluated for L canonical lookups give lookup_target * n / L,
// clamped; nothing evaluated, or no lookup, keeps the cap.
__global__ void k_incr_budget(IncrDev I, const ScoreCounters *sc) {
  const unsigned long long n = (unsigned long long)*I.n_sel;
  unsigned long long L = 0;
  for (int k = 0; k < kStatSlots; ++k) L += sc->s[k].canonical_lookups;
  if (n == 0 || L == 0) return;
  const unsigned long long want = (unsigned long long)I.lookup_target * n / L;
  const int32_t b = want < (unsigned long long)I.b_min   ? I.b_min
                    : want > (unsigned long long)I.b_max ? I.b_max
                                                         : (int32_t)want;
  *I.frame_budget = b;
}

// Coarse-to-fine search (Section 3.6).  The plane of resolved voxels: a
// point with a stored free direction (best < n_c) sets its voxel's bit.
__global__ void __launch_bounds__(kT) k_c2f_mark(PointsDev pts, GridDev g, IncrDev I, int64_t n,
                                                 int32_t n_c) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  int hit = 0;
  if (i < n && (int)I.best[i] < n_c) {
    int32_t x, y, z;
    unpack_key(pts.key[i], x, y, z);
    const int bx = (x >> 3) - g.g0[0], by = (y >> 3) - g.g0[1], bz = (z >> 3) - g.g0[2];
    if ((unsigned)bx < (unsigned)g.gd[0] && (unsigned)by < (unsigned)g.gd[1] &&
        (unsigned)bz < (unsigned)g.gd[2] && in_window(I, x, y, z)) {
      const int64_t b = ((int64_t)bz * g.gd[1] + by) * g.gd[0] + bx;
      const int lin = (x & 7) | ((y & 7) << 3) | ((z & 7) << 6);
      atomicOr(&I.resolved[b * 16 + (lin >> 5)], 1u << (lin & 31));
      hit = 1;
    }
  }
  wg_add<kT>(hit, I.n_resolved);
}

// One thread per listed point: the nearest resolved other point within the
// radius (offsets in (|d|^2, dz, dy, dx) order, the first set bit wins), its
// stored direction k*, and the mask restricted to the coarse pass and k*'s
// fine window.  The candidate count drops by the bits removed.
__global__ void __launch_bounds__(kT) k_c2f_restrict(PointsDev pts, ToolDev t, GridDev g,
                                                     IncrDev I) {
  const int n = *I.n_sel;
  const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
  int removed = 0;
  if (j < n) {
    const int32_t i = I.sel[j];
    int32_t x, y, z;
    unpack_key(pts.key[i], x, y, z);
    int kstar = -1;
    if (*I.n_resolved > 0) {
      for (int e = 0; e < I.c2f_n_off; ++e) {
        const uint32_t o = I.c2f_off[e];
        const int xx = x + (int)(o & 1023u) - 512, yy = y + (int)((o >> 10) & 1023u) - 512,
                  zz = z + (int)(o >> 20) - 512;
        const int bx = (xx >> 3) - g.g0[0], by = (yy >> 3) - g.g0[1], bz = (zz >> 3) - g.g0[2];
        if ((unsigned)bx >= (unsigned)g.gd[0] || (unsigned)by >= (unsigned)g.gd[1] ||
            (unsigned)bz >= (unsigned)g.gd[2])
          continue;
        const int64_t b = ((int64_t)bz * g.gd[1] + by) * g.gd[0] + bx;
        const int lin = (xx & 7) | ((yy & 7) << 3) | ((zz & 7) << 6);
        if (!((I.resolved[b * 16 + (lin >> 5)] >> (lin & 31)) & 1u)) continue;
        const int32_t slot = hash_find(pts.h, pack_key(xx, yy, zz));
        const int32_t pi = slot >= 0 ? pts.h.vals[slot] : -1;
        if (pi >= 0) kstar = I.best_dir[pi];
        break;
      }
    }
    const int mw = I.c2f_mw;
    for (int w = 0; w < mw; ++w) {
      uint64_t allow = I.c2f_coarse[w];
      if (kstar >= 0) allow |= I.c2f_fine[(int64_t)kstar * mw + w];
      const uint64_t m = t.mask[(int64_t)i * mw + w];
      removed += __popcll(m & ~allow);
      t.mask[(int64_t)i * mw + w] = m & allow;
    }
  }
  // the candidate tests the mask kernel counted for removed orientations
  for (int off = 32; off > 0; off >>= 1) removed += __shfl_xor(removed, off);
  if ((threadIdx.x & 63) == 0 && removed)
    atomicAdd(&t.counters->s[(blockIdx.x * (kT / 64) + (threadIdx.x >> 6)) % kStatSlots]
                   .candidate_tests,
              (unsigned long long)(-(long long)removed));
}

// Copy one device int to another (the cap for a frame's selection).
__global__ void k_incr_copy_int(const int32_t *src, int32_t *dst) { *dst = *src; }

unsigned grid_of(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

}  // namespace

void launch_incr_init(const IncrDev &I, int32_t n_c, hipStream_t s) {
  hipLaunchKernelGGL(k_incr_init, dim3(grid_of(std::min<int64_t>(I.max_points, 1 << 22), kT)),
                     dim3(kT), 0, s, I, n_c);
}

static void launch_select(PointsDev pts, MapDev m, const IncrDev &I, int64_t n_points,
                          int32_t min_w, hipStream_t s) {
  if (n_points > 0) {
    const int64_t nblk = (n_points + kSelT - 1) / kSelT;
    hipLaunchKernelGGL(k_incr_sel_count, dim3((unsigned)nblk), dim3(kSelT), 0, s, pts, m, I,
                       n_points, min_w);
    hipLaunchKernelGGL(k_incr_sel_scan, dim3(1), dim3(kSelT), 0, s, I, nblk);
    hipLaunchKernelGGL(k_incr_sel_write, dim3((unsigned)nblk), dim3(kSelT), 0, s, pts, m, I,
                       n_points, min_w);
  } else {
    hipLaunchKernelGGL(k_incr_fill, dim3(1), dim3(kT), 0, s, (uint32_t *)I.n_sel, (int64_t)1, 0u);
  }
}

void launch_incr_drain_front(PointsDev pts, MapDev m, const IncrDev &I, int64_t n_points,
                             int32_t max_evals, int32_t min_w, hipStream_t s) {
  hipLaunchKernelGGL(k_incr_fill, dim3(1), dim3(kT), 0, s, (uint32_t *)I.ctr,
                     (int64_t)(sizeof(IncrCounters) / 4), 0u);
  hipLaunchKernelGGL(k_incr_fill, dim3(1), dim3(kT), 0, s, (uint32_t *)I.budget_dev, (int64_t)1,
                     (uint32_t)max_evals);
  launch_select(pts, m, I, n_points, min_w, s);
}

void launch_incr_set_budget(const IncrDev &I, int32_t b, hipStream_t s) {
  hipLaunchKernelGGL(k_incr_fill, dim3(1), dim3(kT), 0, s, (uint32_t *)I.frame_budget, (int64_t)1,
                     (uint32_t)b);
  hipLaunchKernelGGL(k_incr_fill, dim3(1), dim3(kT), 0, s, (uint32_t *)I.budget_dev, (int64_t)1,
                     (uint32_t)b);
}

void launch_incr_c2f(PointsDev pts, ToolDev t, GridDev g, const IncrDev &I, int64_t n_points,
                     int64_t grid_bricks, int32_t n_c, hipStream_t s) {
  if (!I.c2f_on) return;
  hipLaunchKernelGGL(k_incr_fill, dim3(1), dim3(kT), 0, s, (uint32_t *)I.n_resolved, (int64_t)1,
                     0u);
  if (grid_bricks > 0) {
    hipLaunchKernelGGL(k_incr_fill, dim3(1024), dim3(kT), 0, s, I.resolved, grid_bricks * 16, 0u);
    if (n_points > 0)
      hipLaunchKernelGGL(k_c2f_mark, dim3(grid_of(n_points, kT)), dim3(kT), 0, s, pts, g, I,
                         n_points, n_c);
  }
  hipLaunchKernelGGL(k_c2f_restrict, dim3(grid_of(I.budget, kT)), dim3(kT), 0, s, pts, t, g, I);
}

void launch_incr_budget(const IncrDev &I, const ToolDev &t, hipStream_t s) {
  if (I.lookup_target > 0) hipLaunchKernelGGL(k_incr_budget, dim3(1), dim3(1), 0, s, I, t.counters);
}

void launch_incr_frame_front(PointsDev pts, MapDev m, const IncrDev &I, const int32_t *changed,
                             const FrameCounters *fc, int64_t n_points, int64_t seen, int32_t frame,
                             bool moved, int32_t min_w, hipStream_t s) {
  hipLaunchKernelGGL(k_incr_fill, dim3(1), dim3(kT), 0, s, (uint32_t *)I.ctr,
                     (int64_t)(sizeof(IncrCounters) / 4), 0u);
  hipLaunchKernelGGL(k_incr_copy_int, dim3(1), dim3(1), 0, s, I.frame_budget, I.budget_dev);
  hipLaunchKernelGGL(k_incr_fill, dim3(256), dim3(kT), 0, s, I.hist, (int64_t)2 * 65536, 0u);
  if (n_points > 0)
    hipLaunchKernelGGL(k_incr_triggers, dim3(grid_of(n_points, kT)), dim3(kT), 0, s, pts, m, I,
                       n_points, seen, moved ? 1 : 0);
  const dim3 wide(2048);
  hipLaunchKernelGGL(k_incr_hist, wide, dim3(kT), 0, s, m, changed, fc, frame, I, 0);
  hipLaunchKernelGGL(k_incr_pick, dim3(1), dim3(kSelT), 0, s, fc, I, 0);
  hipLaunchKernelGGL(k_incr_hist, wide, dim3(kT), 0, s, m, changed, fc, frame, I, 1);
  hipLaunchKernelGGL(k_incr_pick, dim3(1), dim3(kSelT), 0, s, fc, I, 1);
  hipLaunchKernelGGL(k_incr_collect, wide, dim3(kT), 0, s, m, changed, fc, frame, I);
  hipLaunchKernelGGL(k_incr_sort, dim3(1), dim3(kSelT), 0, s, I);
  hipLaunchKernelGGL(k_incr_neigh, dim3(kSample), dim3(384), 0, s, pts, I, n_points);
  launch_select(pts, m, I, n_points, min_w, s);
}

void launch_incr_frame_back(PointsDev pts, MapDev m, ToolDev t, GridDev g, const IncrDev &I,
                            int64_t n_points, int32_t n_c, hipStream_t s) {
  hipLaunchKernelGGL(k_incr_count, dim3(grid_of(I.budget, kT / 64)), dim3(kT), 0, s, pts, t, g,
                     I, n_c);
  hipLaunchKernelGGL(k_incr_update, dim3(grid_of(I.budget, kT)), dim3(kT), 0, s, t, I, n_c);
  if (n_points > 0)
    hipLaunchKernelGGL(k_incr_labels, dim3(grid_of(n_points, kT)), dim3(kT), 0, s, pts, m, I,
                       n_points, n_c);
}

}  // namespace af
