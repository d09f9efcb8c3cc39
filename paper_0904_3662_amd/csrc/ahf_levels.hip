// ahf_levels.hip -- the adaptive density hierarchy on the device.
//
// Method: Knollmann & Knebe, "AHF: AMIGA's Halo Finder", Sect. 2.1.  A domain
// grid covers the periodic box; every cell gets its triangular-shaped-cloud
// (TSC) particle density; a cell with more particles than the threshold is
// covered by 8 cells of half the size, where the density is computed again,
// and so on until no cell needs refinement.  The isolated refinements of each
// level, linked to the coarser volume that holds them, form the grid tree.
//
// Layout on the device (level L, b = g + L bits per axis):
//  * particles are sorted once by their Morton key at B = g + max_levels bits,
//    so every cell of every level owns one contiguous range of them;
//  * S_L (the cells of level L) are the 8 children of each refined cell of
//    level L-1, stored in key order: cell s is child s & 7 of parent s >> 3.
//    Level 0 is dense: cell s has key s;
//  * the mass field of level L is stored as 2x2x2 bricks; the bricks are the
//    children of every level-(L-1) cell within one cell of a refined cell, in
//    key order.  Level 0 bricks are all children of the (virtual) level -1;
//  * every brick slot (a level-L cell) knows the brick of level L+1 made of its
//    children (slot_child), so any cell of any level is found by descending
//    from the dense level 0 (tree_lookup), without hashing or searching.
//
// Deposit without float atomics: each thread owns one cell of S_L, sums the
// 27 TSC products of that cell's particles in registers (cells holding more
// than kHeavy particles are summed by whole blocks in fixed chunks and a fixed
// pairwise tree), the 8 cells of a refined parent are combined in LDS into
// the 4x4x4 patch they touch, and each brick cell gathers the at most 8 patches
// that cover it, in a fixed order.  Every float sum therefore has a fixed
// order and the result is bit-reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "ahf_block.h"
#include "ahf_internal.h"

namespace ahf {

constexpr int kT = 256;
// runs of consecutive tiles per XCD for kernels whose work varies by tile
// (16: measured against 1, 4 and 64, best by a small margin)
constexpr uint32_t kXcdRun = 16;
// the labels of the first levels start once a level has fewer cells
// (2^16: measured against never, 2^18 and 2^20 on the 16.8M workload)
constexpr uint64_t kLabEarlyCells = 1ull << 16;

static inline unsigned grid_for(uint64_t n, int t = kT) {
  uint64_t b = (n + t - 1) / t;
  if (b < 1) b = 1;
  if (b > (1u << 20)) b = 1u << 20;
  return (unsigned)b;
}

#define GRID_STRIDE(i, n)                                                       \
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (uint64_t)gridDim.x * blockDim.x)

// ------------------------------------------------------------ small kernels

__global__ void k_fill_i32(int32_t* a, uint64_t n, int32_t v) {
  GRID_STRIDE(i, n) a[i] = v;
}

// slot -> F index of the refined cell in it (-1 for other cells and ghost
// slots); the cell in slot i of brick i/8 is Bcell[i/8] + i%8 (level 0: i);
// also clears the dilation marks when given
__global__ void k_slots(Cnt nslot_c, const int32_t* __restrict__ Bcell,
                        const uint8_t* __restrict__ flag, const uint32_t* __restrict__ rankF,
                        int32_t* __restrict__ slot_f, uint8_t* __restrict__ mark) {
  const uint64_t nslot = cnt_of(nslot_c);
  GRID_STRIDE(i, nslot) {
    int64_t s = (int64_t)i;
    if (Bcell) {
      const int32_t c0 = Bcell[i >> 3];
      s = c0 >= 0 ? (int64_t)c0 + (int64_t)(i & 7) : -1;
    }
    slot_f[i] = (s >= 0 && flag[s]) ? (int32_t)rankF[s] : -1;
    if (mark) mark[i] = 0;
  }
}

// orders the LDS accesses of one wave: what a lane wrote before is seen by
// every lane of the wave after (the wave's LDS instructions run in order;
// this keeps the compiler from moving them across)
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Morton keys at B bits per axis, the identity permutation, the particle as
// one 32-byte record {X, Y, Z, mass | fx, fy, fz, 0} (input order), and the
// histograms of every 8-bit digit of the keys for the radix sort
__global__ __launch_bounds__(256) void k_keys(const uint32_t* __restrict__ X,
                                              const uint32_t* __restrict__ Y,
                                              const uint32_t* __restrict__ Z,
                                              const float* __restrict__ fx,
                                              const float* __restrict__ fy,
                                              const float* __restrict__ fz,
                                              const float* __restrict__ m, float mscalar,
                                              uint64_t n, int B, int npass, int word_ib,
                                              int kshift, uint64_t* __restrict__ keys,
                                              uint4* __restrict__ rec,
                                              uint32_t* __restrict__ ghist,
                                              uint32_t* __restrict__ err) {
  __shared__ uint32_t h[kRsMaxPass * 256];
  // each wave's 64 records (2 KB) pass through LDS, so that each of the two
  // 16-byte stores per lane writes one contiguous kilobyte (a lane storing
  // its own record's two halves at a 32-byte stride left half-written lines,
  // and 29% more bytes reached HBM than the records hold)
  __shared__ uint4 stage[256 / 64][128];
  for (int i = threadIdx.x; i < kRsMaxPass * 256; i += 256) h[i] = 0u;
  __syncthreads();
  const int s = kQBits - B;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint64_t base = (uint64_t)blockIdx.x * 256; base < n; base += (uint64_t)gridDim.x * 256) {
    const uint64_t i = base + threadIdx.x;
    const bool valid = i < n;
    uint64_t key = 0;
    if (valid) {
      const uint32_t x = X[i], y = Y[i], z = Z[i];
      if ((x | y | z) >= (1u << kQBits)) atomicOr(err, kErrCoord);
      const uint32_t xm = x & 0x1fffffu, ym = y & 0x1fffffu, zm = z & 0x1fffffu;
      // the sort orders by the key without its lowest kshift bits
      key = morton3(xm >> s, ym >> s, zm >> s) >> kshift;
      // word_ib >= 0: the sort starts on packed words (key << ib) | index
      keys[i] = (word_ib >= 0) ? ((key << word_ib) | i) : key;
      const float w = m ? m[i] : mscalar;
      stage[wv][2 * lane] = make_uint4(xm, ym, zm, __float_as_uint(w));
      stage[wv][2 * lane + 1] =
          make_uint4(fx ? __float_as_uint(fx[i]) : 0u, fy ? __float_as_uint(fy[i]) : 0u,
                     fz ? __float_as_uint(fz[i]) : 0u, 0u);
    }
    wave_lds_sync();
    // the wave's records start at uint4 2 * (wave base); lane l stores
    // uint4 l, then 64 + l of them (only those of valid elements)
    const uint64_t w0 = base + (uint64_t)(wv * 64);
    if (w0 < n) {
      const uint64_t nrec = 2 * ((n - w0) < 64 ? (n - w0) : 64);
      if ((uint64_t)lane < nrec) rec[2 * w0 + lane] = stage[wv][lane];
      if ((uint64_t)(64 + lane) < nrec) rec[2 * w0 + 64 + lane] = stage[wv][64 + lane];
    }
    wave_lds_sync();
    wave_digit_hist(key, valid, npass, h);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npass * 256; i += 256)
    if (h[i]) atomicAdd(&ghist[i], h[i]);
}

// records in sorted order: one random 32-byte read per particle.  Sorted
// position i: particle index from the packed word, its record, its full key
// rebuilt from the coordinates, and the level-0 cell starts: element i (and
// the terminal element n) starts every dense cell after the previous
// element's cell up to its own.  The previous element's key comes from the
// neighbouring lane, or for a wave's first lane from that element's record.
// Elements 0 .. n (n + 1 of them) in grid-stride rounds that every lane of
// the grid takes part in.
//
// When the sort left out the lowest `skip` key bits it ordered by key >>
// skip, ties by input index; a run of elements with equal key >> skip then
// still has to be put in full-key order (stable: equal keys keep the input
// order).  A run that lies within one wave is ranked there (its keys differ
// only in the low bits) and written in that order; a run that crosses into
// the next wave is written as it is and its start listed for k_fix_runs.
__device__ inline uint64_t key_of(const uint4& a, int s) {
  return morton3(a.x >> s, a.y >> s, a.z >> s);
}

__global__ __launch_bounds__(kT) void k_gather_rec(const uint64_t* __restrict__ words, int ib,
                                                   int s, uint64_t n,
                                                   const uint4* __restrict__ rec,
                                                   uint4* __restrict__ srec,
                                                   uint32_t* __restrict__ order,
                                                   uint64_t* __restrict__ skey, int sh0,
                                                   uint64_t ncell0, uint32_t* __restrict__ start0,
                                                   int skip, uint32_t* __restrict__ ncross,
                                                   uint32_t* __restrict__ cross) {
  const uint64_t im = (1ull << ib) - 1ull;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const int lane = (int)__lane_id();
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base <= n; base += stride) {
    const uint64_t i = base + threadIdx.x;
    const bool valid = i < n;
    uint32_t j = 0;
    uint4 a = make_uint4(0u, 0u, 0u, 0u), b = a;
    uint64_t key = 0;
    if (valid) {
      j = (uint32_t)(words[i] & im);
      a = rec[2 * (uint64_t)j];
      b = rec[2 * (uint64_t)j + 1];
      key = key_of(a, s);
    }
    uint64_t kprev = ((uint64_t)__shfl_up((uint32_t)(key >> 32), 1, 64) << 32) |
                     __shfl_up((uint32_t)key, 1, 64);
    if (lane == 0 && i > 0 && i <= n) kprev = key_of(rec[2 * (words[i - 1] & im)], s);
    uint64_t dst = i;
    if (skip) {
      uint64_t knext = ((uint64_t)__shfl_down((uint32_t)(key >> 32), 1, 64) << 32) |
                       __shfl_down((uint32_t)key, 1, 64);
      if (lane == 63 && i + 1 < n) knext = key_of(rec[2 * (words[i + 1] & im)], s);
      const bool sp = valid && i > 0 && ((kprev ^ key) >> skip) == 0;  // continues a run
      const bool sn = valid && i + 1 < n && ((knext ^ key) >> skip) == 0;
      if (__ballot(sp || sn) != 0ull) {
        const uint64_t heads = __ballot(!sp);  // lanes that do not continue the lane before
        const uint64_t conts = __ballot(sn);
        const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
        const uint64_t h_le = heads & le, h_gt = heads & ~le;
        const int st = h_le ? 63 - __builtin_clzll(h_le) : -1;  // the run's first lane
        const int en = h_gt ? __builtin_ctzll(h_gt) : 64;       // one past its last lane
        const bool longer = (sp || sn);
        // a run that began in an earlier wave, or goes on into the next one
        const bool crossing = st < 0 || (en == 64 && ((conts >> 63) & 1ull));
        const bool inside = longer && !crossing;
        if (longer && crossing && st == lane) cross[atomicAdd(ncross, 1u)] = (uint32_t)i;
        const uint64_t in_mask = __ballot(inside);
        if (in_mask) {
          const int r0 = __builtin_ctzll(in_mask), r1 = 63 - __builtin_clzll(in_mask);
          const uint32_t lmask = (skip >= 32) ? ~0u : ((1u << skip) - 1u);
          const uint32_t lo = (uint32_t)key & lmask;
          uint32_t rank = 0;
          for (int r = r0; r <= r1; ++r) {
            const uint32_t lr = (uint32_t)__builtin_amdgcn_readlane((int)lo, r);
            if (r >= st && r < en && (lr < lo || (lr == lo && r < lane))) ++rank;
          }
          if (inside) dst = i - (uint64_t)(lane - st) + rank;
        }
      }
    }
    if (valid) {
      order[dst] = j;
      srec[2 * dst] = a;
      srec[2 * dst + 1] = b;
      skey[dst] = key;
    }
    if (i > n) continue;
    const uint64_t ci = valid ? key >> sh0 : ncell0;
    const uint64_t cp = kprev >> sh0;
    for (uint64_t c = (i > 0) ? cp + 1 : 0; c <= ci; ++c) start0[c] = (uint32_t)i;
  }
}

// The runs the gather listed (those that cross from one wave into the next):
// the thread of each finds its end; up to kShortRun particles are sorted in
// place by that thread (insertion sort moving keys, records and indices),
// longer ones (dense cores) go to a list for k_fix_long_runs.
constexpr uint32_t kShortRun = 16;
__global__ void k_fix_runs(const uint32_t* __restrict__ ncross,
                           const uint32_t* __restrict__ cross, uint64_t* __restrict__ skey,
                           uint4* __restrict__ srec, uint32_t* __restrict__ order, uint64_t n,
                           int skip, uint32_t* __restrict__ nlong, uint32_t* __restrict__ long_a,
                           uint32_t* __restrict__ long_m) {
  const uint32_t nc = *ncross;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nc; t += gridDim.x * blockDim.x) {
    const uint64_t i = cross[t];
    const uint64_t k = skey[i];
    uint64_t j = i + 1;
    while (j < n && ((skey[j] ^ k) >> skip) == 0) ++j;
    const uint32_t m = (uint32_t)(j - i);
    if (m > kShortRun) {
      const uint32_t at = atomicAdd(nlong, 1u);
      long_a[at] = (uint32_t)i;
      long_m[at] = m;
      continue;
    }
    // stable insertion sort of the run by the full key
    for (uint32_t q = 1; q < m; ++q) {
      const uint64_t kq = skey[i + q];
      uint32_t r = q;
      while (r > 0 && skey[i + r - 1] > kq) --r;
      if (r == q) continue;
      const uint32_t oq = order[i + q];
      const uint4 a0 = srec[2 * (i + q)], a1 = srec[2 * (i + q) + 1];
      for (uint32_t u = q; u > r; --u) {
        skey[i + u] = skey[i + u - 1];
        order[i + u] = order[i + u - 1];
        srec[2 * (i + u)] = srec[2 * (i + u - 1)];
        srec[2 * (i + u) + 1] = srec[2 * (i + u - 1) + 1];
      }
      skey[i + r] = kq;
      order[i + r] = oq;
      srec[2 * (i + r)] = a0;
      srec[2 * (i + r) + 1] = a1;
    }
  }
}

// The long runs: one workgroup per run, a stable sort of (key, position in
// the run), then keys, indices and records written back permuted.  ka, kb,
// va, vb, rtmp are scratch at the particles' positions.
__global__ __launch_bounds__(kBT) void k_fix_long_runs(
    const uint32_t* __restrict__ nlong, const uint32_t* __restrict__ long_a,
    const uint32_t* __restrict__ long_m, uint64_t* __restrict__ skey, uint4* __restrict__ srec,
    uint32_t* __restrict__ order, uint64_t* __restrict__ ka, uint64_t* __restrict__ kb,
    uint32_t* __restrict__ va, uint32_t* __restrict__ vb, uint4* __restrict__ rtmp) {
  const uint32_t nr = *nlong;
  for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const uint64_t a = long_a[r];
    const uint32_t m = long_m[r];
    for (uint32_t k = threadIdx.x; k < m; k += kBT) {
      ka[a + k] = skey[a + k];
      va[a + k] = k;
    }
    __syncthreads();
    const bool fl = block_sort<uint64_t>(ka + a, va + a, kb + a, vb + a, m);
    const uint64_t* K = fl ? kb + a : ka + a;
    const uint32_t* V = fl ? vb + a : va + a;
    uint32_t* T = fl ? va + a : vb + a;  // the other index buffer
    for (uint32_t k = threadIdx.x; k < m; k += kBT) {
      const uint64_t j = a + V[k];
      T[k] = order[j];
      rtmp[2 * (a + k)] = srec[2 * j];
      rtmp[2 * (a + k) + 1] = srec[2 * j + 1];
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < m; k += kBT) {
      order[a + k] = T[k];
      skey[a + k] = K[k];
      srec[2 * (a + k)] = rtmp[2 * (a + k)];
      srec[2 * (a + k) + 1] = rtmp[2 * (a + k) + 1];
    }
    __syncthreads();
  }
}

__device__ inline uint32_t lower_bound_key(const uint64_t* __restrict__ a, uint32_t lo, uint32_t hi,
                                           uint64_t key) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// level L >= 1: the 8 children of every refined cell of level L-1 and their
// particle ranges (binary searches inside the parent's range)
__global__ void k_child_ranges(const uint64_t* __restrict__ skey, Cnt nS_c,
                               const uint32_t* __restrict__ pFs,
                               const uint32_t* __restrict__ pSstart,
                               const uint32_t* __restrict__ pScount,
                               const uint64_t* __restrict__ pSkey, int sh,
                               uint64_t* __restrict__ Skey, uint32_t* __restrict__ Sstart,
                               uint32_t* __restrict__ Scount) {
  const uint64_t nS = cnt_of(nS_c);
  GRID_STRIDE(s, nS) {
    const uint32_t ps = pFs[s >> 3];
    const uint32_t d = (uint32_t)(s & 7);
    const uint32_t a = pSstart[ps];
    const uint32_t e = a + pScount[ps];
    const uint64_t pk = pSkey ? pSkey[ps] : (uint64_t)ps;
    const uint64_t ck = (pk << 3) | d;
    // the 8 children of a parent sit on 8 consecutive lanes (nS is a multiple
    // of 8 and so is every lane group's first s): each finds where its child
    // starts, and ends where the next child starts.  A parent of at most 32
    // particles is read by its 8 lanes together (one load each per 8 keys),
    // which count the particles of every child digit; a larger one is
    // searched.
    uint32_t lo;
    if (e - a <= 32u) {
      uint64_t hist = 0;  // one byte per child digit
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t i = a + d + 8u * k;
        if (i < e) hist += 1ull << (8u * (uint32_t)((skey[i] >> sh) & 7u));
      }
#pragma unroll
      for (int m = 1; m < 8; m <<= 1) {
        const uint32_t l32 = __shfl_xor((uint32_t)hist, m, 8);
        const uint32_t h32 = __shfl_xor((uint32_t)(hist >> 32), m, 8);
        hist += ((uint64_t)h32 << 32) | l32;
      }
      const uint64_t below = d ? (hist & ((1ull << (8u * d)) - 1ull)) : 0ull;
      lo = a + (uint32_t)((below * 0x0101010101010101ull) >> 56);
    } else {
      lo = (d == 0) ? a : lower_bound_key(skey, a, e, ck << sh);
    }
    const uint32_t nxt = (uint32_t)__shfl_down((int)lo, 1, 8);
    const uint32_t hi = (d == 7) ? e : nxt;
    Skey[s] = ck;
    Sstart[s] = lo;
    Scount[s] = hi - lo;
  }
}

// refinement flags; cells too full for one thread are appended to Hs (in no
// particular order: the list only routes each such cell to its own sums)
// Heavy cells: every cell above kHeavy particles takes an index h (in no
// particular order: h only routes the cell to its own sums) and a contiguous
// run of chunk slots, whose chunks are later summed in the order of their
// index j inside that run.  The two counters start at zero.
struct HeavyList {
  uint32_t* nheavy;   // number of heavy cells
  uint32_t* nchunks;  // number of chunks
  uint32_t* Hs;       // cell of heavy index h
  int32_t* hidx;      // heavy index of a heavy cell
  uint32_t* nch;      // chunks of heavy cell h
  uint32_t* chofs;    // first chunk slot of heavy cell h
  uint32_t* ch_a;     // first particle of a chunk
  uint32_t* ch_n;     // particles in a chunk
};

__device__ inline uint32_t wave_excl_scan_u32(uint32_t v) {
  const uint32_t lane = __lane_id();
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += t;
  }
  return x - v;
}

// Refinement flags and the heavy-cell list (cells of more than `heavy`
// particles, summed by whole waves instead of one thread).  Each block takes one contiguous
// run of cells: a first pass counts its heavy cells and their chunks, one
// atomic per counter reserves the block's indices, a second pass writes them.
// On level 0 (count_out set) the counts come from the dense cell starts and
// are written here.
// (Atomics on one address from different blocks are served one after
// another far from the CU, so their number sets the cost: the grid is kept
// small.  Blocks of 512 threads fit into the wave slots that one block of
// the previous level's tile deposit, running beside on the other stream,
// frees; blocks of 1024 waited for that whole kernel.)
constexpr int kFlagT = 512;
constexpr unsigned kFlagBlocks = 512;

__global__ __launch_bounds__(kFlagT) void k_flags(const uint32_t* __restrict__ count,
                                                  const uint32_t* __restrict__ start, Cnt nS_c,
                                                  double thr, int can_refine, uint32_t heavy,
                                                  uint8_t* __restrict__ flag, HeavyList hl,
                                                  uint32_t* __restrict__ rank_unset,
                                                  uint32_t* __restrict__ count_out) {
  __shared__ uint32_t wh[kFlagT / 64], wc[kFlagT / 64];
  __shared__ uint32_t base_h, base_c;
  const uint64_t nS = cnt_of(nS_c);
  const int w = threadIdx.x >> 6;
  const int lane = (int)__lane_id();
  const uint64_t per = ((nS + gridDim.x - 1) / gridDim.x + kFlagT - 1) / kFlagT * kFlagT;
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint64_t hi = lo + per < nS ? lo + per : nS;
  // pass 1: flags, and the block's heavy cells and chunks per thread
  uint32_t my_h = 0, my_c = 0;
  for (uint64_t s0 = lo + threadIdx.x; s0 < hi; s0 += 8 * kFlagT) {
    uint32_t cs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t s = s0 + (uint64_t)k * kFlagT;
      cs[k] = s < hi ? (count_out ? start[s + 1] - start[s] : count[s]) : 0u;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t s = s0 + (uint64_t)k * kFlagT;
      if (s >= hi) break;
      const uint32_t c = cs[k];
      if (count_out) count_out[s] = c;
      const uint32_t f = (can_refine && (double)c > thr) ? 1u : 0u;
      flag[s] = (uint8_t)f;
      // the compaction fills in the rank of the refined cells
      if (rank_unset && !f) rank_unset[s] = 0xffffffffu;
      if (c > heavy) {
        my_h += 1;
        my_c += (c + kChunk - 1) / kChunk;
      }
    }
  }
  const uint32_t th = __syncthreads_count(my_h != 0);
  if (th == 0) return;  // uniform: no heavy cell in the block
  // block totals and one reservation
  const uint32_t ho = wave_excl_scan_u32(my_h), co = wave_excl_scan_u32(my_c);
  if (lane == 63) {
    wh[w] = ho + my_h;
    wc[w] = co + my_c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t sh = 0, sc = 0;
    for (int i = 0; i < kFlagT / 64; ++i) {
      const uint32_t a = wh[i], b = wc[i];
      wh[i] = sh;
      wc[i] = sc;
      sh += a;
      sc += b;
    }
    base_h = atomicAdd(hl.nheavy, sh);
    base_c = atomicAdd(hl.nchunks, sc);
  }
  __syncthreads();
  // pass 2: each thread's heavy cells in its own index range
  uint32_t h = base_h + wh[w] + ho;
  uint32_t o = base_c + wc[w] + co;
  if (my_h == 0) return;
  for (uint64_t s = lo + threadIdx.x; s < hi; s += kFlagT) {
    const uint32_t c = count_out ? start[s + 1] - start[s] : count[s];
    if (c <= heavy) continue;
    const uint32_t m = (c + kChunk - 1) / kChunk;
    const uint32_t a = start[s];
    hl.Hs[h] = (uint32_t)s;
    hl.hidx[s] = (int32_t)h;
    hl.nch[h] = m;
    hl.chofs[h] = o;
    for (uint32_t j = 0; j < m; ++j) {
      hl.ch_a[o + j] = a + j * kChunk;
      hl.ch_n[o + j] = min((uint32_t)kChunk, c - j * kChunk);
    }
    h += 1;
    o += m;
  }
}


// density criterion: a cell of S_L is refined where its TSC particle number
// (its deposited mass over the common particle mass) exceeds the threshold;
// the cell's field value sits in its own slot of the level's bricks
__global__ void k_flags_density(uint64_t nS, const float* __restrict__ mass,
                                const int32_t* __restrict__ Pbrick, double mscalar, double thr,
                                int can_refine, uint8_t* __restrict__ flag,
                                uint32_t* __restrict__ rank_unset) {
  GRID_STRIDE(s, nS) {
    const uint64_t slot = Pbrick ? (uint64_t)Pbrick[s >> 3] * 8 + (s & 7) : s;
    const uint32_t f = (can_refine && (double)mass[slot] / mscalar > thr) ? 1u : 0u;
    flag[s] = (uint8_t)f;
    if (rank_unset && !f) rank_unset[s] = 0xffffffffu;
  }
}

// ------------------------------------------------------------ TSC weights

// per-axis TSC weights of coordinate (X, f) on a grid with k = 21 - b sub-bits:
// u is the in-cell offset; 1-u is formed from the integer complement so that
// both tails keep full relative precision.
__device__ inline void tsc_axis(uint32_t X, float f, uint32_t mask, float scale, float w[3]) {
  const uint32_t lo = X & mask;
  const float u = ((float)lo + f) * scale;
  const float v = ((float)(mask - lo) + (1.0f - f)) * scale;
  const float c = u - 0.5f;
  w[0] = 0.5f * v * v;
  w[1] = 0.75f - c * c;
  w[2] = 0.5f * u * u;
}

struct Parts {
  const uint4* rec;  // 2 per particle, sorted order
};

__device__ inline void add_record(const uint4& r0, const uint4& r1, uint32_t mask, float scale,
                                  float T[27], double& msum) {
  float wx[3], wy[3], wz[3];
  tsc_axis(r0.x, __uint_as_float(r1.x), mask, scale, wx);
  tsc_axis(r0.y, __uint_as_float(r1.y), mask, scale, wy);
  tsc_axis(r0.z, __uint_as_float(r1.z), mask, scale, wz);
  const float m = __uint_as_float(r0.w);
  msum += (double)m;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float ma = m * wx[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const float mab = ma * wy[b];
#pragma unroll
      for (int c = 0; c < 3; ++c) T[a * 9 + b * 3 + c] = fmaf(mab, wz[c], T[a * 9 + b * 3 + c]);
    }
  }
}

__device__ inline void add_particle(const Parts& P, uint32_t p, uint32_t mask, float scale,
                                    float T[27], double& msum) {
  add_record(P.rec[2 * (uint64_t)p], P.rec[2 * (uint64_t)p + 1], mask, scale, T, msum);
}

// the particles [a, a+n) of one cell, in batches of K whose records are all
// loaded before the first is used: a cell of up to K particles waits for
// memory once
template <int K>
__device__ inline void add_range(const Parts& P, uint32_t a, uint32_t n, uint32_t mask, float scale,
                                 float T[27], double& msum) {
  for (uint32_t i = 0; i < n; i += K) {
    uint4 r[2 * K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (i + k < n) {
        r[2 * k] = P.rec[2 * (uint64_t)(a + i + k)];
        r[2 * k + 1] = P.rec[2 * (uint64_t)(a + i + k) + 1];
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (i + k < n) add_record(r[2 * k], r[2 * k + 1], mask, scale, T, msum);
  }
}

// ------------------------------------------------------------ heavy cells


// one wave per chunk of <= kChunk particles of one heavy cell (4 chunks per
// block of 256 threads); every lane sums at most kChunk/64 = 16 particles,
// then a fixed butterfly over the wave
__global__ __launch_bounds__(256) void k_heavy_chunk(
    const uint32_t* __restrict__ nchunks, const uint32_t* __restrict__ ch_a,
    const uint32_t* __restrict__ ch_n, Parts P, uint32_t mask, float scale,
    float* __restrict__ chT, double* __restrict__ chM) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t nc = *nchunks;
  for (uint32_t c = blockIdx.x * 4 + (threadIdx.x >> 6); c < nc; c += gridDim.x * 4) {
  const uint32_t a = ch_a[c];
  const uint32_t len = ch_n[c];
  float T[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) T[k] = 0.0f;
  double ms = 0.0;
  uint32_t i = lane;
  for (; i + 3 * 64 < len; i += 4 * 64) {
    uint4 r[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      r[2 * k] = P.rec[2 * (uint64_t)(a + i + k * 64)];
      r[2 * k + 1] = P.rec[2 * (uint64_t)(a + i + k * 64) + 1];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) add_record(r[2 * k], r[2 * k + 1], mask, scale, T, ms);
  }
  for (; i < len; i += 64) add_particle(P, a + i, mask, scale, T, ms);
#pragma unroll
  for (int k = 0; k < 27; ++k) {
    float v = T[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == (uint32_t)k) chT[(uint64_t)c * 27 + k] = v;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) ms += __shfl_xor(ms, d, 64);
  if (lane == 27) chM[c] = ms;
  }
}

// the chunks of each heavy cell summed by one wave: each run of 64 chunks
// (one per lane) as a pairwise tree (a butterfly, which leaves the same sum
// on every lane), the runs in chunk order; lane k keeps component k (the
// mass on lane 27).  A cell of one chunk is copied.
__global__ __launch_bounds__(256) void k_heavy_reduce(const uint32_t* __restrict__ nch,
                                                      const uint32_t* __restrict__ chofs,
                                                      const uint32_t* __restrict__ nHdev,
                                                      const float* __restrict__ chT,
                                                      const double* __restrict__ chM,
                                                      float* __restrict__ hT,
                                                      double* __restrict__ hM) {
  const uint64_t nH = *nHdev;
  const uint32_t lane = threadIdx.x & 63u;
  for (uint64_t h = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); h < nH;
       h += (uint64_t)gridDim.x * 4) {
    const uint32_t o = chofs[h], m = nch[h];
    if (m == 1) {  // most heavy cells: one chunk, copied
      if (lane < 27) hT[h * 27 + lane] = chT[(uint64_t)o * 27 + lane];
      if (lane == 27) hM[h] = chM[o];
      continue;
    }
    float acc = 0.0f;
    double accm = 0.0;
    for (uint32_t g = 0; g < m; g += 64) {
      const bool v = g + lane < m;
      const uint64_t c = (uint64_t)o + g + lane;
      float w[27];
#pragma unroll
      for (int k = 0; k < 27; ++k) w[k] = v ? chT[c * 27 + k] : 0.0f;
      double wm = v ? chM[c] : 0.0;
#pragma unroll
      for (int k = 0; k < 27; ++k)
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) w[k] += __shfl_xor(w[k], d, 64);
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) wm += __shfl_xor(wm, d, 64);
      float mine = 0.0f;
#pragma unroll
      for (int k = 0; k < 27; ++k)
        if (lane == (uint32_t)k) mine = w[k];
      acc += mine;
      accm += wm;
    }
    if (lane < 27) hT[h * 27 + lane] = acc;
    if (lane == 27) hM[h] = accm;
  }
}


// ------------------------------------------------------------ deposit

// Layout of the 4x4x4 patch of a parent: the cells are grouped by the brick
// they belong to (the parent's own brick first, then its 26 neighbours in
// offset order), so a brick reads each neighbour's share as one contiguous
// run.  layout[q] is the stored position of patch cell q = 16 px + 4 py + pz;
// inv is its inverse.
struct PatchLayout {
  uint8_t layout[64];
  uint8_t inv[64];
};

constexpr int patch_dir(int p) { return p == 0 ? -1 : (p == 3 ? 1 : 0); }

constexpr PatchLayout make_patch_layout() {
  PatchLayout t{};
  int n = 0;
  for (int k = 0; k < 27; ++k) {
    const int o = (k == 0) ? 13 : (k <= 13 ? k - 1 : k);
    const int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
    for (int q = 0; q < 64; ++q)
      if (patch_dir(q >> 4) == ox && patch_dir((q >> 2) & 3) == oy && patch_dir(q & 3) == oz) {
        t.layout[q] = (uint8_t)n;
        t.inv[n] = (uint8_t)q;
        ++n;
      }
  }
  return t;
}

// ------------------------------------------------------------ dense tiles
//
// Levels whose parents form a dense grid (level 0, whose parents are the
// virtual level -1, and level 1 over a well-refined level 0) deposit by
// tiles of 4x4x4 parents = 8x8x8 cells, one cell per thread.  Every wave
// holds 2x2x2 parents = 4x4x4 cells and adds their 27-tensors into a grid of
// its own (its cells plus a one-cell halo, in LDS) with no block barrier;
// after one barrier the eight wave grids are summed into the tile grid (the
// tile plus a one-cell halo).  The tile's inner cells go straight to their
// bricks and the rest (the tile's deposit into its faces and its neighbours'
// cells) to a buffer that k_tile_halo_add folds in afterwards.

constexpr int kTileT = 512;   // threads = cells per tile
constexpr int kTileMaxG = 8;  // largest domain grid (bits per axis) tiled: halo <= 1 GB
constexpr int kTileG = 10;    // cells per axis with the halo
constexpr int kTileH = kTileG * kTileG * kTileG;
constexpr int kTileBatch0 = 4;  // records in flight per cell: level 0 (about 6 particles per cell)
constexpr int kPatchBatch = 4;  // deeper levels
// level 1 (about one particle per cell): 2 or 4 records in flight, a tuning choice
constexpr int kWaveG = 6;     // a wave's 4x4x4 cells per axis with their halo
constexpr int kWaveH = kWaveG * kWaveG * kWaveG;

__device__ inline uint32_t tile_local_parent(uint32_t x, uint32_t y, uint32_t z) {
  // Morton index of a parent inside its 4x4x4 tile
  return (((x >> 1) & 1u) << 5) | (((y >> 1) & 1u) << 4) | (((z >> 1) & 1u) << 3) |
         ((x & 1u) << 2) | ((y & 1u) << 1) | (z & 1u);
}

// DENSE0: the tile's parents are virtual (every level-0 cell exists, cell =
// 8 * parent + digit, brick = parent); else parents are level-0 cells, a
// refined one (prank != ~0) holds 8 cells of S_1 at 8 * prank + digit, and
// bricks come from the level-0 slot -> level-1 brick map.  A cell's records
// are loaded in batches (kTileBatch0 on level 0, whose cells hold several
// particles each, kTileBatch1 on level 1), all of a batch before its first
// record is used.
template <bool DENSE0, int K1>
__global__ __launch_bounds__(kTileT) void k_tile_deposit(
    const uint32_t* __restrict__ prank,
    const uint32_t* __restrict__ Sstart, const uint32_t* __restrict__ Scount,
    const int32_t* __restrict__ hidx, const float* __restrict__ hT,
    const double* __restrict__ hM, Parts P, uint32_t mask, float scale, uint32_t heavy,
    const int32_t* __restrict__ pslot_child, float* __restrict__ mass,
    float* __restrict__ halo, double* __restrict__ Spmass, uint64_t nfp) {
  __shared__ float Wg[kTileT / 64][kWaveH];  // each wave's cells and their one-cell halo
  __shared__ int32_t sbr[64];  // brick of each parent's children (loaded with the first loads)
  const int t = threadIdx.x;
  float* wg = Wg[t >> 6];
  const uint64_t tile = xcd_tile_runs(blockIdx.x, gridDim.x, kXcdRun);
  for (int q = t & 63; q < kWaveH; q += 64) wg[q] = 0.0f;
  if (t < 64) sbr[t] = DENSE0 ? (int32_t)(tile * 64 + (uint64_t)t) : pslot_child[tile * 64 + (uint64_t)t];
  const uint32_t pm = (uint32_t)t >> 3, d = (uint32_t)t & 7u;
  const uint32_t px = (((pm >> 5) & 1u) << 1) | ((pm >> 2) & 1u);
  const uint32_t py = (((pm >> 4) & 1u) << 1) | ((pm >> 1) & 1u);
  const uint32_t pz = (((pm >> 3) & 1u) << 1) | (pm & 1u);
  const uint32_t cx = 2 * px + ((d >> 2) & 1u), cy = 2 * py + ((d >> 1) & 1u), cz = 2 * pz + (d & 1u);
  const uint64_t pg = tile * 64 + pm;
  float T[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) T[k] = 0.0f;
  // (a rank at or past nfp, which only a build that overflowed its plan can
  // hold, counts as unrefined)
  const uint32_t r = DENSE0 ? 0u : prank[pg];
  bool has = false;  // the cell holds particles (an empty cell adds only zeros)
  if (DENSE0 || (uint64_t)r < nfp) {
    const uint64_t s = DENSE0 ? pg * 8 + d : (uint64_t)r * 8 + d;
    const uint32_t n = Scount[s];
    const uint32_t a0 = Sstart[s];
    has = n > 0;
    double ms = 0.0;
    if (n > heavy) {
      const int32_t h = hidx[s];
#pragma unroll
      for (int k = 0; k < 27; ++k) T[k] = hT[(uint64_t)h * 27 + k];
      ms = hM[h];
    } else if (DENSE0) {
      add_range<kTileBatch0>(P, a0, n, mask, scale, T, ms);
    } else {
      add_range<K1>(P, a0, n, mask, scale, T, ms);  // about one particle per cell
    }
    if (Spmass) Spmass[s] = ms;
  }
  // 27 phases, one per neighbour offset in a fixed order: within a phase the
  // wave's cells add to distinct cells of its grid, so no two writes collide
  // and every grid cell sums its contributions in the same order on every run
  // (LDS float atomics instead of the read-add-write took twice as long).  A
  // wave without particles adds nothing.
  const int w0 = ((int)(cx & 3u) * kWaveG + (int)(cy & 3u)) * kWaveG + (int)(cz & 3u);
  if (__ballot(has) != 0ull) {
    wave_lds_sync();
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (has) wg[w0 + (a * kWaveG + b) * kWaveG + c] += T[a * 9 + b * 3 + c];
          wave_lds_sync();
        }
  }
  __syncthreads();
  for (int q = t; q < kTileH; q += kTileT) {
    const int gx = q / 100, gy = (q / 10) % 10, gz = q % 10;
    const int dx = gx - 1, dy = gy - 1, dz = gz - 1;
    // the wave grids covering this tile grid cell, in wave order (wave w
    // holds the cells 4 (w>>2 & 1, w>>1 & 1, w & 1) + [0, 4) per axis, so
    // per axis the low wave covers g < 6 and the high one g >= 4); the 8
    // reads are issued together from addresses clamped into the grid, and
    // only the covering ones are added
    const bool cov[2][3] = {{gx < kWaveG, gy < kWaveG, gz < kWaveG},
                            {gx >= 4, gy >= 4, gz >= 4}};
    const int ox[2] = {gx * kWaveG * kWaveG, (gx - 4) * kWaveG * kWaveG};
    const int oy[2] = {gy * kWaveG, (gy - 4) * kWaveG};
    const int oz[2] = {gz, gz - 4};
    float v[8];
#pragma unroll
    for (int w = 0; w < kTileT / 64; ++w) {
      const int i = (w >> 2) & 1, j = (w >> 1) & 1, k = w & 1;
      const bool c = cov[i][0] && cov[j][1] && cov[k][2];
      v[w] = Wg[w][c ? ox[i] + oy[j] + oz[k] : 0];
    }
    float sum = 0.0f;
#pragma unroll
    for (int w = 0; w < kTileT / 64; ++w) {
      const int i = (w >> 2) & 1, j = (w >> 1) & 1, k = w & 1;
      if (cov[i][0] && cov[j][1] && cov[k][2]) sum += v[w];
    }
    // cells off the tile's faces are final; face cells and the halo go to
    // the buffer, where k_tile_halo_add adds the neighbours' share
    if ((unsigned)(dx - 1) < 6u && (unsigned)(dy - 1) < 6u && (unsigned)(dz - 1) < 6u) {
      const int64_t br = sbr[tile_local_parent((uint32_t)dx >> 1, (uint32_t)dy >> 1, (uint32_t)dz >> 1)];
      const uint32_t dd = (((uint32_t)dx & 1u) << 2) | (((uint32_t)dy & 1u) << 1) | ((uint32_t)dz & 1u);
      if (br >= 0) mass[(uint64_t)br * 8 + dd] = sum;
    } else {
      halo[tile * kTileH + q] = sum;
    }
  }
}

// adds to the cells on a tile's faces what the neighbouring tiles deposited
// there (own tile first, then the neighbours in a fixed offset order); nb =
// tile bits per axis
__global__ __launch_bounds__(256) void k_tile_halo_add(int dense0, int nb,
                                                      const int32_t* __restrict__ pslot_child,
                                                      const float* __restrict__ halo,
                                                      float* __restrict__ mass) {
  const uint64_t tile = xcd_tile_runs(blockIdx.x, gridDim.x, kXcdRun);
  uint32_t tx, ty, tz;
  unmorton3(tile, tx, ty, tz);
  const uint32_t tm = (1u << nb) - 1u;
  for (int li = threadIdx.x; li < 512; li += 256) {
    const int cx = li >> 6, cy = (li >> 3) & 7, cz = li & 7;
    const bool fx = cx == 0 || cx == 7, fy = cy == 0 || cy == 7, fz = cz == 0 || cz == 7;
    if (!(fx || fy || fz)) continue;
    const uint64_t pp = tile * 64 + tile_local_parent((uint32_t)cx >> 1, (uint32_t)cy >> 1,
                                                      (uint32_t)cz >> 1);
    const int64_t br = dense0 ? (int64_t)pp : (int64_t)pslot_child[pp];
    const uint32_t dd = (((uint32_t)cx & 1u) << 2) | (((uint32_t)cy & 1u) << 1) | ((uint32_t)cz & 1u);
    const int sx = cx == 0 ? -1 : (cx == 7 ? 1 : 0);
    const int sy = cy == 0 ? -1 : (cy == 7 ? 1 : 0);
    const int sz = cz == 0 ? -1 : (cz == 7 ? 1 : 0);
    // the (up to 7) neighbour tiles whose halo covers this cell: loads first,
    // then the sum in a fixed order
    float hv[8];
#pragma unroll
    for (int m = 1; m < 8; ++m) {
      const int ax = (m & 4) ? sx : 0, ay = (m & 2) ? sy : 0, az = (m & 1) ? sz : 0;
      const bool ok = (!(m & 4) || sx) && (!(m & 2) || sy) && (!(m & 1) || sz);
      hv[m] = 0.0f;
      if (ok) {
        const uint64_t nt = morton3((tx + (uint32_t)ax) & tm, (ty + (uint32_t)ay) & tm,
                                    (tz + (uint32_t)az) & tm);
        const int q = ((cx - 8 * ax + 1) * kTileG + (cy - 8 * ay + 1)) * kTileG + (cz - 8 * az + 1);
        hv[m] = halo[nt * kTileH + q];
      }
    }
    float v = halo[tile * kTileH + ((cx + 1) * kTileG + (cy + 1)) * kTileG + (cz + 1)];
#pragma unroll
    for (int m = 1; m < 8; ++m) v += hv[m];
    if (br >= 0) mass[(uint64_t)br * 8 + dd] = v;
  }
}

__constant__ PatchLayout c_patch = make_patch_layout();

// one thread per cell of S_L (8 per refined parent); 32 parents per block.
// patch[f][px][py][pz] (4x4x4) holds what the particles of parent f give to
// the level-L cells 2P-1 .. 2P+2 per axis.
__global__ __launch_bounds__(256) void k_patches(Cnt nFp_c, const uint32_t* __restrict__ Sstart,
                                                 const uint32_t* __restrict__ Scount,
                                                 const int32_t* __restrict__ hidx,
                                                 const float* __restrict__ hT,
                                                 const double* __restrict__ hM, Parts P,
                                                 uint32_t mask, float scale, uint32_t heavy,
                                                 float* __restrict__ patch,
                                                 double* __restrict__ Spmass) {
  __shared__ float Ts[256][27];  // odd stride: the 64 lanes hit distinct banks
  __shared__ uint8_t inv[64];    // lane-dependent lookups: LDS, not the scalar cache
  const int t = threadIdx.x;
  const uint64_t nFp = cnt_of(nFp_c);
  if (t < 64) inv[t] = c_patch.inv[t];
  const uint64_t f = (uint64_t)xcd_tile_runs(blockIdx.x, gridDim.x, kXcdRun) * 32 + (t >> 3);
  const int d = t & 7;
  float T[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) T[k] = 0.0f;
  if (f < nFp) {
    const uint64_t s = f * 8 + d;
    const uint32_t n = Scount[s];
    double ms = 0.0;
    if (n > heavy) {
      const int32_t h = hidx[s];
#pragma unroll
      for (int k = 0; k < 27; ++k) T[k] = hT[(uint64_t)h * 27 + k];
      ms = hM[h];
    } else {
      const uint32_t a = Sstart[s];
      add_range<kPatchBatch>(P, a, n, mask, scale, T, ms);
    }
    if (Spmass) Spmass[s] = ms;
  }
#pragma unroll
  for (int k = 0; k < 27; ++k) Ts[t][k] = T[k];
  __syncthreads();
  if (f >= nFp) return;
  const int base = t & ~7;
  float out[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int q = inv[d * 8 + j];
    const int px = q >> 4, py = (q >> 2) & 3, pz = q & 3;
    float sum = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int a = px - ((c >> 2) & 1), b = py - ((c >> 1) & 1), e = pz - (c & 1);
      if (a >= 0 && a <= 2 && b >= 0 && b <= 2 && e >= 0 && e <= 2)
        sum += Ts[base + c][a * 9 + b * 3 + e];
    }
    out[j] = sum;
  }
  float4* dst = reinterpret_cast<float4*>(patch + f * 64 + d * 8);
  dst[0] = make_float4(out[0], out[1], out[2], out[3]);
  dst[1] = make_float4(out[4], out[5], out[6], out[7]);
}

// 8 lanes per brick (32 bricks per block): the lanes share the lookups of
// the refined parents among the 27 neighbours of the brick's parent through
// LDS; each lane then sums, for its cell, the (at most 8) patches covering it
// in a fixed order (own parent first)
// (nfp: the parents that have a patch; an F index at or past it, which only
// a build that overflowed its plan can hold, counts as no patch)
__global__ __launch_bounds__(256) void k_combine(int L, Cnt nB_c, const uint64_t* __restrict__ Bkey,
                                                 int pbits, Tree tree,
                                                 const int32_t* __restrict__ pslot_f,
                                                 const float* __restrict__ patch,
                                                 float* __restrict__ mass, uint64_t nfp) {
  __shared__ int32_t fn[32][28];
  __shared__ uint8_t lay[64];
  const uint64_t nB = cnt_of(nB_c);
  if (threadIdx.x < 64) lay[threadIdx.x] = c_patch.layout[threadIdx.x];
  const int lb = threadIdx.x >> 3;
  const int d = threadIdx.x & 7;
  const uint64_t bi = (uint64_t)xcd_tile_runs(blockIdx.x, gridDim.x, kXcdRun) * 32 + lb;
  if (bi < nB) {
    const uint64_t P = Bkey ? Bkey[bi] : bi;
    uint32_t qx, qy, qz;
    unmorton3(P, qx, qy, qz);
    const uint32_t msk = (1u << pbits) - 1u;
    // lane d looks up neighbours d, d+8, d+16 (and 24), together
    uint64_t k[4];
    int64_t slot[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = d + 8 * j;
      const int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
      k[j] = morton3((qx + dx) & msk, (qy + dy) & msk, (qz + dz) & msk);
      slot[j] = (o < 27) ? 0 : -1;
    }
    if (L == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) slot[j] = slot[j] < 0 ? -1 : (int64_t)k[j];
    } else {
      tree_lookup_k<4>(tree, L - 1, k, slot);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = d + 8 * j;
      if (o < 27) {
        int32_t f = slot[j] < 0 ? -1 : (L == 0 ? (int32_t)slot[j] : pslot_f[slot[j]]);
        if (f >= 0 && (uint64_t)f >= nfp) f = -1;
        fn[lb][o] = f;
      }
    }
  }
  __syncthreads();
  if (bi >= nB) return;
  const int ex = (d >> 2) & 1, ey = (d >> 1) & 1, ez = d & 1;
  float sum = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int sx = (c >> 2) & 1, sy = (c >> 1) & 1, sz = c & 1;
    const int ox = sx ? (ex ? 1 : -1) : 0, oy = sy ? (ey ? 1 : -1) : 0, oz = sz ? (ez ? 1 : -1) : 0;
    const int px = sx ? (ex ? 0 : 3) : ex + 1;
    const int py = sy ? (ey ? 0 : 3) : ey + 1;
    const int pz = sz ? (ez ? 0 : 3) : ez + 1;
    const int32_t f = fn[lb][(ox + 1) * 9 + (oy + 1) * 3 + (oz + 1)];
    if (f >= 0) sum += patch[(uint64_t)f * 64 + lay[px * 16 + py * 4 + pz]];
  }
  mass[bi * 8 + d] = sum;
}

// FP64 sums of a level: the field, the particle mass per cell, the counts
// FP64 sums of the brick masses, the per-cell particle masses and the cell
// counts: partial sums per block, then one block adds them in block order
__global__ __launch_bounds__(256) void k_level_sums(const float* __restrict__ a, Cnt na_c,
                                                    const double* __restrict__ b, Cnt nb_c,
                                                    const uint32_t* __restrict__ c, Cnt nc_c,
                                                    double* __restrict__ part) {
  __shared__ double lds[3][4];
  const uint64_t na = cnt_of(na_c), nb = cnt_of(nb_c), nc = cnt_of(nc_c);
  double s[3] = {0.0, 0.0, 0.0};
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint64_t i = i0; i < na; i += stride) s[0] += (double)a[i];
  if (b)
    for (uint64_t i = i0; i < nb; i += stride) s[1] += b[i];
  for (uint64_t i = i0; i < nc; i += stride) s[2] += (double)c[i];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double v = s[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) lds[k][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    part[(uint64_t)blockIdx.x * 3 + k] = (lds[k][0] + lds[k][1]) + (lds[k][2] + lds[k][3]);
  }
}

constexpr int kSumBlocks = 2048;
struct SumBlocks {
  int n[kMaxLevels];
};

// block L adds the partial sums of level L in block order
__global__ __launch_bounds__(256) void k_level_sums_final(const double* __restrict__ part_all,
                                                          SumBlocks nb, double* __restrict__ out_all) {
  __shared__ double lds[3][4];
  const int np = nb.n[blockIdx.x];
  const double* part = part_all + (uint64_t)blockIdx.x * 3 * kSumBlocks;
  double* out = out_all + 3 * blockIdx.x;
  double s[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < np; i += 256) {
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] += part[(uint64_t)i * 3 + k];
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double v = s[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) lds[k][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    out[k] = (lds[k][0] + lds[k][1]) + (lds[k][2] + lds[k][3]);
  }
}

// ------------------------------------------------------------ next level's bricks

__device__ inline uint64_t slot_of_s(uint64_t s, const int32_t* Pbrick) {
  return Pbrick ? (uint64_t)Pbrick[s >> 3] * 8 + (s & 7) : s;
}


// level 0 is dense: a cell is in the dilation when one of its 27 neighbours
// (itself included) is refined
__global__ void k_mark_dense0(int g, uint64_t ncell, const uint8_t* __restrict__ flag,
                              uint8_t* __restrict__ mark) {
  const uint32_t msk = (1u << g) - 1u;
  GRID_STRIDE(c, ncell) {
    uint32_t x, y, z;
    unmorton3(c, x, y, z);
    uint32_t any = 0;
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      const int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
      any |= flag[morton3((x + dx) & msk, (y + dy) & msk, (z + dz) & msk)];
    }
    mark[c] = any ? 1 : 0;
  }
}

// mark every level-L slot within one cell of a refined cell
// (the number of refined cells is read on the device: the grid is a bound)
__global__ void k_mark(int L, int bits, const uint32_t* __restrict__ nFdev,
                       const uint32_t* __restrict__ Fs, const uint64_t* __restrict__ Skey,
                       Tree tree, uint8_t* __restrict__ mark, uint32_t* __restrict__ err) {
  const uint64_t nF = *nFdev;
  GRID_STRIDE(i, nF * 27) {
    const uint64_t f = i / 27;
    const int o = (int)(i % 27);
    const uint32_t s = Fs[f];
    const uint64_t key = Skey ? Skey[s] : (uint64_t)s;
    const uint64_t nk = shift_key(key, bits, o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1);
    const int64_t slot = tree_lookup(tree, L, nk);
    if (slot < 0) atomicOr(err, kErrLookup);
    else mark[slot] = 1;
  }
}

// next level's bricks (one per marked slot, in key order by rank); a refined
// cell's slot is always marked, so its F entry is finished here too: its
// children's brick, and F_L moved to its final buffer.
// (capD, capF: the room of the next level's bricks and of F_L; a build
// whose levels are sized ahead writes nothing beyond them and is redone)
__global__ void k_build_bricks(Cnt nslot_c, const uint8_t* __restrict__ mark,
                               const uint32_t* __restrict__ rank,
                               const uint64_t* __restrict__ Bkey,
                               const int32_t* __restrict__ slot_f,
                               int32_t* __restrict__ slot_child, uint64_t* __restrict__ nBkey,
                               int32_t* __restrict__ nBcell, const uint32_t* __restrict__ Ftmp,
                               uint32_t* __restrict__ Fs, int32_t* __restrict__ nPbrick,
                               uint64_t capD, uint64_t capF, const uint32_t* __restrict__ nFraw) {
  const uint64_t nslot = cnt_of(nslot_c);
  GRID_STRIDE(i, nslot) {
    const uint32_t r = mark[i] ? rank[i] : 0xffffffffu;
    const bool has_brick = r < capD;
    const int32_t f = slot_f[i];
    const bool in_F = f >= 0 && (uint64_t)f < capF;
    if (in_F) nPbrick[f] = has_brick ? (int32_t)r : -1;
    slot_child[i] = has_brick ? (int32_t)r : -1;
    if (has_brick) {
      nBkey[r] = Bkey ? ((Bkey[i >> 3] << 3) | (i & 7)) : i;
      nBcell[r] = in_F ? f * 8 : -1;
    }
  }
  // F_L to its final buffer, every entry below the (clamped) count: a build
  // that overflowed its plan may hold refined cells without a slot, and its
  // later kernels still read every entry below that count
  const uint64_t nF = *nFraw < capF ? *nFraw : capF;
  GRID_STRIDE(f, nF) Fs[f] = Ftmp[f];
}

// the end of a level sized ahead: its refined cells and next-level bricks
// (raw[0], raw[1]) against their room; the counts the next levels read
// (cnt[0], cnt[1]) clamped to it, and an error flag when they did not fit,
// or when the last planned level still refines cells
__global__ void k_level_check(const uint32_t* __restrict__ raw, uint64_t capF, uint64_t capD,
                              int last, uint32_t* __restrict__ cnt, uint32_t* __restrict__ err) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t nF = raw[0], nD = raw[1];
  if ((uint64_t)nF > capF || (uint64_t)nD > capD || (last && nF > 0)) atomicOr(err, kErrCapacity);
  cnt[0] = (uint64_t)nF < capF ? nF : (uint32_t)capF;
  cnt[1] = (uint64_t)nD < capD ? nD : (uint32_t)capD;
}


// ------------------------------------------------------------ labels

// The forest keeps par[x] <= x, and a value stored in par[x] stays an
// ancestor of x for ever after.  Plain (cached) loads may return an older
// value, which is still an ancestor: a find then ends higher up the tree but
// at a node of the same component.  Only roots are changed by the atomic CAS,
// and a failed CAS returns the true parent, so every retry starts strictly
// lower than the last one and the loop ends.  Path-halving stores are
// device-scope atomics, so no cache line of par is ever dirty in an XCD's L2
// (a late write-back of such a line could otherwise undo a CAS).
__device__ inline int32_t uf_find(int32_t* par, int32_t x) {
  while (true) {
    const int32_t p = par[x];
    if (p == x) return x;
    const int32_t gp = par[p];
    if (gp == p) return p;
    __hip_atomic_store(&par[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = gp;
  }
}

// link the larger root under the smaller one
__device__ inline void uf_unite(int32_t* par, int32_t a, int32_t b) {
  a = uf_find(par, a);
  b = uf_find(par, b);
  while (a != b) {
    if (a > b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    const int32_t old = atomicCAS(&par[b], b, a);
    if (old == b) return;
    b = uf_find(par, old);
    a = uf_find(par, a);
  }
}


// half of the neighbour offsets of the connectivity (the other half is symmetric)
__constant__ int8_t c_half26[13][3] = {{1, -1, -1}, {1, -1, 0}, {1, -1, 1}, {1, 0, -1}, {1, 0, 0},
                                       {1, 0, 1},   {1, 1, -1}, {1, 1, 0},  {1, 1, 1},  {0, 1, -1},
                                       {0, 1, 0},   {0, 1, 1},  {0, 0, 1}};

__device__ inline bool conn_ok(int dx, int dy, int dz, int conn) {
  const int s = abs(dx) + abs(dy) + abs(dz);
  return conn == 6 ? s == 1 : (conn == 18 ? s <= 2 : true);
}

// the half-neighbourhood offsets that count as adjacent under conn
__device__ inline uint32_t conn_mask(int conn) {
  uint32_t m = 0;
#pragma unroll
  for (int o = 0; o < 13; ++o)
    if (conn_ok(c_half26[o][0], c_half26[o][1], c_half26[o][2], conn)) m |= 1u << o;
  return m;
}

constexpr int kUfTile = 256;

__device__ inline int32_t lds_find(volatile int32_t* lp, int32_t x) {
  while (true) {
    const int32_t p = lp[x];
    if (p == x) return x;
    const int32_t gp = lp[p];
    if (gp == p) return p;
    lp[x] = gp;
    x = gp;
  }
}

__device__ inline void lds_unite(int32_t* lp, int32_t a, int32_t b) {
  volatile int32_t* v = lp;
  a = lds_find(v, a);
  b = lds_find(v, b);
  while (a != b) {
    if (a > b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    const int32_t old = atomicCAS(&lp[b], b, a);
    if (old == b) return;
    b = lds_find(v, old);
    a = lds_find(v, a);
  }
}

// F indices of the 13 half-neighbourhood neighbours selected by `sel` (bit
// o = offset c_half26[o]); -1 where unselected or not refined.  nF: the
// level's refined cells in the pass; an index at or past it (which only a
// build that overflowed its plan can hold) counts as not refined.
__device__ inline void refined_neighbours(int Lp, int bits, const Tree& tree,
                                          const int32_t* __restrict__ slot_f, uint64_t key,
                                          uint32_t sel, int32_t (&g)[13], uint32_t* err,
                                          uint64_t nF) {
  uint64_t nk[13];
  int64_t slot[13];
#pragma unroll
  for (int o = 0; o < 13; ++o) {
    nk[o] = shift_key(key, bits, c_half26[o][0], c_half26[o][1], c_half26[o][2]);
    slot[o] = ((sel >> o) & 1u) ? 0 : -1;
  }
  tree_lookup_k<13>(tree, Lp, nk, slot);
#pragma unroll
  for (int o = 0; o < 13; ++o) {
    g[o] = -1;
    if ((sel >> o) & 1u) {
      if (slot[o] < 0) {
        atomicOr(err, kErrLookup);
      } else {
        const int32_t f = slot_f[slot[o]];
        g[o] = (f >= 0 && (uint64_t)f < nF) ? f : -1;
      }
    }
  }
}


// All levels are labelled in one pass per step.  Entry k of the set is the
// refined cells F_k of level k (key order), whose children make S_{k+1};
// element e of the concatenated range is the refined cell e - off[k] of the
// entry k holding e.  Neighbours are only looked up on the element's own
// level, so components never cross levels and one forest over all elements
// holds every level's components.  Indices and roots are global; a patch of
// level k+1 with id p (its rank among that level's roots) gets the slot
// off[k] + p in the per-patch arrays, which keeps the levels' slots apart.
struct LabLev {
  const uint32_t* Fs;      // S index of each refined cell of level k
  const uint64_t* Skey;    // keys of S_k (null on level 0, where index = key)
  const int32_t* slot_f;   // level-k slot -> index in F_k, or -1
  const uint32_t* Scount;  // particles per cell of S_k
  const double* Spmass;    // particle mass per cell of S_k, or null
  int32_t* Spatch;         // out: patch of each cell of S_{k+1}
  const int32_t* pSpatch;  // patch of each cell of S_k (null on level 0)
  uint32_t level;          // k
  uint32_t bits;           // bits per axis of level k
};
struct LabSet {
  uint32_t nlev;              // entries 0 .. nlev-1
  uint32_t total;             // off[nlev], for kernels that take a 32-bit count
  uint64_t off[kMaxLevels];   // first element of each entry; off[nlev] = total
  uint64_t toff[kMaxLevels];  // first tile (kUfTile elements) of each entry
  // first slot of each entry's patches in the per-patch arrays; pbase[nlev]
  // = slots in all (equal to off when the level sizes are known on the host;
  // laid out by the levels' capacities when they are known on the device only)
  uint64_t pbase[kMaxLevels];
  LabLev lv[kMaxLevels - 1];
};

// the element offsets of a set whose level sizes are on the device: entry j
// holds the refined cells of level k0 + j, counted at nF[2 (k0 + j)]
__global__ void k_labset_counts(LabSet* __restrict__ S, const uint32_t* __restrict__ nF, int k0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t tot = 0, nt = 0;
  for (uint32_t j = 0; j < S->nlev; ++j) {
    const uint64_t c = nF[2 * (k0 + (int)j)];
    S->off[j] = tot;
    S->toff[j] = nt;
    tot += c;
    nt += (c + kUfTile - 1) / kUfTile;
  }
  S->off[S->nlev] = tot;
  S->toff[S->nlev] = nt;
  S->total = (uint32_t)tot;
}

__device__ inline int lab_entry(const LabSet& S, uint64_t e) {
  int k = 0;
  while (k + 1 < (int)S.nlev && e >= S.off[k + 1]) ++k;
  return k;
}

// The tree lookups run on tiles of kUfTile elements that never straddle two
// entries, so the level of a lookup is uniform over the block; the element
// kernels without lookups find each element's entry per lane.  The set lives
// in device memory, so that it can be indexed per lane.
__device__ inline int lab_tile_entry(const LabSet& S, uint64_t tile) {
  int k = 0;
  while (k + 1 < (int)S.nlev && tile >= S.toff[k + 1]) ++k;
  return k;
}

// Each block unites the cells of kUfTile consecutive elements in LDS; edges
// that leave the tile are marked in xmask for the global pass.  par[e] leaves
// as the smallest index of e's component inside the tile.
__global__ __launch_bounds__(256) void k_uf_local(const LabSet* __restrict__ pS, Tree tree, int conn,
                                                  int32_t* __restrict__ par,
                                                  uint16_t* __restrict__ xmask,
                                                  uint32_t* __restrict__ err) {
  __shared__ int32_t lp[kUfTile];
  const LabSet& S = *pS;
  const uint32_t tile = xcd_tile_runs(blockIdx.x, gridDim.x, kXcdRun);
  if (tile >= S.toff[S.nlev]) return;  // past the true count (grid laid out for a bound)
  const int k = lab_tile_entry(S, tile);
  const LabLev& lv = S.lv[k];
  const uint64_t o = S.off[k];
  const uint64_t t0 = o + ((uint64_t)tile - S.toff[k]) * kUfTile;
  const uint64_t rest = S.off[k + 1] - t0;
  const uint32_t tn = (uint32_t)(rest < (uint64_t)kUfTile ? rest : (uint64_t)kUfTile);
  for (int i = threadIdx.x; i < kUfTile; i += 256) lp[i] = i;
  __syncthreads();
  const uint32_t cm = conn_mask(conn);
  for (uint32_t i = threadIdx.x; i < tn; i += 256) {
    const uint64_t e = t0 + i;
    const uint32_t s = lv.Fs[e - o];
    const uint64_t key = lv.Skey ? lv.Skey[s] : (uint64_t)s;
    uint32_t xm = 0;
    int32_t gs[13];
    refined_neighbours((int)lv.level, (int)lv.bits, tree, lv.slot_f, key, cm, gs, err,
                       S.off[k + 1] - o);
#pragma unroll
    for (int q = 0; q < 13; ++q) {
      if (gs[q] < 0) continue;
      const uint64_t g = o + (uint64_t)gs[q];
      if (g == e) continue;
      if (g >= t0 && g < t0 + tn) lds_unite(lp, (int32_t)i, (int32_t)(g - t0));
      else xm |= 1u << q;
    }
    xmask[e] = (uint16_t)xm;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < tn; i += 256)
    par[t0 + i] = (int32_t)(t0 + (uint64_t)lds_find(lp, (int32_t)i));
}

// The edges between tiles, on the global forest.  Most edges that leave a
// tile join the same two local roots (par[] holds each cell's tile-local
// root), so each block first collects the distinct (root, root) pairs of its
// cells in an LDS hash set and unites each pair once.
constexpr int kPairSlots = 2048;
static_assert(kUfTile % 256 == 0, "the union-find kernels loop over a tile in steps of 256");

__global__ __launch_bounds__(256) void k_uf_cross(const LabSet* __restrict__ pS, Tree tree,
                                                  const uint16_t* __restrict__ xmask,
                                                  int32_t* __restrict__ par,
                                                  uint32_t* __restrict__ err) {
  __shared__ unsigned long long set[kPairSlots];
  const LabSet& S = *pS;
  const uint32_t tile = xcd_tile_runs(blockIdx.x, gridDim.x, kXcdRun);
  if (tile >= S.toff[S.nlev]) return;  // past the true count (grid laid out for a bound)
  const int k = lab_tile_entry(S, tile);
  const LabLev& lv = S.lv[k];
  const uint64_t o = S.off[k];
  const uint64_t base = o + (tile - S.toff[k]) * kUfTile;
  for (int i = threadIdx.x; i < kPairSlots; i += 256) set[i] = ~0ull;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < (uint32_t)kUfTile; j += 256) {
    const uint64_t f = base + j;
    if (f >= S.off[k + 1]) break;
    uint32_t xm = xmask[f];
    if (xm) {
      const uint32_t s = lv.Fs[f - o];
      const uint64_t key = lv.Skey ? lv.Skey[s] : (uint64_t)s;
      const int32_t ra = par[f];  // tile-local root (written by k_uf_local)
      int32_t gs[13];
      refined_neighbours((int)lv.level, (int)lv.bits, tree, lv.slot_f, key, xm, gs, err,
                         S.off[k + 1] - o);
#pragma unroll
      for (int q = 0; q < 13; ++q) {
        if (gs[q] < 0) continue;
        const int32_t rb = par[o + (uint64_t)gs[q]];
        const int32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        if (lo == hi) continue;
        const unsigned long long pk = ((unsigned long long)(uint32_t)lo << 32) | (uint32_t)hi;
        uint32_t h = (uint32_t)((pk * 0x9E3779B97F4A7C15ull) >> 53) & (kPairSlots - 1);
        bool mine = false, full = true;
        for (int probe = 0; probe < kPairSlots; ++probe) {
          const unsigned long long old = atomicCAS(&set[h], ~0ull, pk);
          if (old == ~0ull) {
            mine = true;
            full = false;
            break;
          }
          if (old == pk) {
            full = false;
            break;
          }
          h = (h + 1) & (kPairSlots - 1);
        }
        if (mine || full) uf_unite(par, lo, hi);
      }
    }
  }
}

// roots go to a separate array: par itself may still receive path-halving
// stores from other threads, so it is never read back as the answer
// final roots; also clears the per-patch accumulators (nz >= n entries)
__global__ void k_uf_compress(int32_t* par, Cnt n_c, int32_t* __restrict__ root,
                              uint8_t* __restrict__ pred, uint64_t nz, uint32_t* __restrict__ z32,
                              unsigned long long* __restrict__ z64a,
                              unsigned long long* __restrict__ z64b) {
  const uint64_t n = cnt_of(n_c);
  GRID_STRIDE(i, nz) {
    z32[i] = 0u;
    z64a[i] = 0ull;
    if (z64b) z64b[i] = 0ull;
    if (i >= n) continue;
    const int32_t r = uf_find(par, (int32_t)i);
    root[i] = r;
    pred[i] = (r == (int32_t)i) ? 1 : 0;
  }
}

// patch id of every element (the rank of its root among its level's roots;
// the level's first element is always a root, so rank[off[k]] is the
// level's base) and of its 8 children, the cells of S_{k+1}; lab[e] is the
// patch's global slot.  The level's first element also writes the level's
// patch count.
__global__ void k_uf_label(const LabSet* __restrict__ pS, const int32_t* __restrict__ root,
                           const uint32_t* __restrict__ rank, const uint32_t* __restrict__ nroots,
                           int32_t* __restrict__ lab, uint32_t* __restrict__ npatch) {
  const LabSet& S = *pS;
  const uint64_t n = S.off[S.nlev];
  GRID_STRIDE(i, n) {
    const int k = lab_entry(S, i);
    const uint64_t o = S.off[k];
    const uint32_t r0 = rank[o];
    const int32_t l = (int32_t)(rank[root[i]] - r0);
    lab[i] = (int32_t)(S.pbase[k] + (uint64_t)l);
    int4* out = reinterpret_cast<int4*>(S.lv[k].Spatch + 8 * (i - o));
    out[0] = make_int4(l, l, l, l);
    out[1] = make_int4(l, l, l, l);
    if (i == o) {
      const uint64_t o1 = S.off[k + 1];
      npatch[S.lv[k].level + 1] = (o1 < n ? rank[o1] : *nroots) - r0;
    }
  }
}

// per patch: cells, particles (exact integer atomics); mass as fixed point.
// Refined cells are in key order and patches are compact, so neighbouring
// lanes mostly share a patch: each wave sums every run of equal patch ids
// (segmented scan) and adds it with one atomic per run.
__device__ inline uint64_t shfl_up_u64(uint64_t v, int d) {
  const uint32_t lo = __shfl_up((uint32_t)v, d, 64);
  const uint32_t hi = __shfl_up((uint32_t)(v >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

// every wave walks its own contiguous range of cells 64 at a time (the loads
// of four rows issued together) and keeps the run that reaches the end of a
// row as a carry, so a patch spread over many cells costs about one atomic
// per wave
__global__ __launch_bounds__(256) void k_patch_stats(const LabSet* __restrict__ pS,
                              const int32_t* __restrict__ lab,
                              double fscale,
                              uint32_t* __restrict__ ncells, unsigned long long* __restrict__ npart,
                              unsigned long long* __restrict__ mfix) {
  const LabSet& S = *pS;
  const uint64_t nF = S.off[S.nlev];
  const int lane = (int)__lane_id();
  const uint64_t le = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
  const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const uint64_t wid = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  uint64_t chunk = (nF + nw - 1) / nw;
  chunk = (chunk + 255) & ~255ull;
  const uint64_t r0 = wid * chunk;
  const uint64_t r1 = (r0 + chunk < nF) ? r0 + chunk : nF;
  int32_t cp = -1;  // carried run (wave-uniform)
  uint32_t cc = 0;
  uint64_t cn = 0, cm = 0;
  for (uint64_t base = r0; base < r1; base += 4 * 64) {
    // the loads of four rows of 64 first (indices clamped into the range),
    // then the rows in order
    int32_t pv[4];
    uint64_t npv[4], mfv[4];
    const int k0 = lab_entry(S, base);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint64_t fr = base + 64 * j + lane;
      const uint64_t f = fr < r1 ? fr : r1 - 1;
      int k = k0;
      while (k + 1 < (int)S.nlev && f >= S.off[k + 1]) ++k;
      const LabLev& lv = S.lv[k];
      const uint32_t s = lv.Fs[f - S.off[k]];
      pv[j] = lab[f];
      npv[j] = lv.Scount[s];
      mfv[j] = mfix ? (uint64_t)llrint(lv.Spmass[s] * fscale) : 0ull;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
    if (base + 64 * j >= r1) break;
    const bool valid = base + 64 * j + lane < r1;
    const int32_t p = valid ? pv[j] : -1;
    uint32_t c = valid ? 8u : 0u;
    uint64_t np = valid ? npv[j] : 0ull, mf = valid ? mfv[j] : 0ull;
    const int32_t pp = __shfl_up(p, 1, 64);
    const bool head = (lane == 0) || (pp != p);
    const uint64_t heads = __ballot(head);
    const int rstart = 63 - __clzll(heads & le);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t c2 = __shfl_up(c, d, 64);
      const uint64_t n2 = shfl_up_u64(np, d);
      const uint64_t m2 = shfl_up_u64(mf, d);
      if (lane - d >= rstart) {
        c += c2;
        np += n2;
        mf += m2;
      }
    }
    // the chunk's first run continues the carried run when the ids agree
    const int32_t p0 = __shfl(p, 0, 64);
    if (cp >= 0 && cp != p0) {
      if (lane == 0) {
        atomicAdd(&ncells[cp], cc);
        atomicAdd(&npart[cp], (unsigned long long)cn);
        if (mfix) atomicAdd(&mfix[cp], (unsigned long long)cm);
      }
      cp = -1;
    }
    if (cp >= 0 && rstart == 0) {
      c += cc;
      np += cn;
      mf += cm;
    }
    const uint64_t vmask = __ballot(valid);
    const int last = 63 - __clzll(vmask);
    const bool tail = valid && ((lane == last) || ((heads >> (lane + 1)) & 1ull));
    if (tail && lane != last) {
      atomicAdd(&ncells[p], c);
      atomicAdd(&npart[p], (unsigned long long)np);
      if (mfix) atomicAdd(&mfix[p], (unsigned long long)mf);
    }
    // the last run becomes the carry
    cp = __shfl(p, last, 64);
    cc = __shfl(c, last, 64);
    cn = ((uint64_t)(uint32_t)__shfl((uint32_t)(np >> 32), last, 64) << 32) |
         (uint32_t)__shfl((uint32_t)np, last, 64);
    cm = ((uint64_t)(uint32_t)__shfl((uint32_t)(mf >> 32), last, 64) << 32) |
         (uint32_t)__shfl((uint32_t)mf, last, 64);
    }
  }
  if (cp >= 0 && lane == 0) {
    atomicAdd(&ncells[cp], cc);
    atomicAdd(&npart[cp], (unsigned long long)cn);
    if (mfix) atomicAdd(&mfix[cp], (unsigned long long)cm);
  }
}

// per patch, from its root: the parent patch (the level-k patch of the
// root's cell, none on level 1) and the mass (fixed point back to FP64, or
// count x mass)
__global__ void k_patch_parent(const LabSet* __restrict__ pS, const int32_t* __restrict__ root,
                               const int32_t* __restrict__ lab, int32_t* __restrict__ parent,
                               const unsigned long long* __restrict__ npart,
                               const unsigned long long* __restrict__ mfix, double mscalar,
                               double inv_scale, double* __restrict__ pm) {
  const LabSet& S = *pS;
  const uint64_t nF = S.off[S.nlev];
  GRID_STRIDE(f, nF) {
    if (root[f] == (int32_t)f) {
      const int32_t p = lab[f];
      const int k = lab_entry(S, f);
      const int32_t* ps = S.lv[k].pSpatch;
      parent[p] = ps ? ps[S.lv[k].Fs[f - S.off[k]]] : -1;
      pm[p] = mfix ? (double)mfix[p] * inv_scale : (double)npart[p] * mscalar;
    }
  }
}

// The whole label pass in one block, for passes of few elements (the last
// levels, or a small hierarchy) with equal masses: union-find in LDS over
// every element (a block holds them all, so there are no tile edges), the
// roots' ranks by a block scan, then the patch ids of the elements and their
// children, the per-patch cells and particles (LDS sums), the parents and
// masses.  The results are those of the general pass, in one launch instead
// of eight.  Tree lookups go level by level, so their level is uniform over
// the block.
constexpr int kLabSmallT = 1024;
constexpr uint32_t kLabSmallMax = 4096;

__global__ __launch_bounds__(kLabSmallT) void k_label_small(
    const LabSet* __restrict__ pS, Tree tree, int conn, uint32_t* __restrict__ ncells,
    unsigned long long* __restrict__ npart, int32_t* __restrict__ parent,
    double* __restrict__ pm, double mscalar, uint32_t* __restrict__ npatch,
    uint32_t* __restrict__ err) {
  __shared__ int32_t lp[kLabSmallMax];
  __shared__ uint32_t rk[kLabSmallMax];
  __shared__ uint32_t sc[kLabSmallMax];
  __shared__ unsigned long long sp[kLabSmallMax];
  __shared__ uint32_t wsum[kLabSmallT / 64];
  const LabSet& S = *pS;
  const uint32_t n = (uint32_t)S.off[S.nlev];
  const uint32_t nslot = (uint32_t)S.pbase[S.nlev];  // >= n
  const uint32_t cm = conn_mask(conn);
  const uint32_t t = threadIdx.x;
  for (uint32_t e = t; e < nslot; e += kLabSmallT) {
    lp[e] = (int32_t)e;
    sc[e] = 0u;
    sp[e] = 0ull;
  }
  __syncthreads();
  for (int k = 0; k < (int)S.nlev; ++k) {
    const LabLev& lv = S.lv[k];
    const uint32_t o = (uint32_t)S.off[k], o1 = (uint32_t)S.off[k + 1];
    for (uint32_t e = o + t; e < o1; e += kLabSmallT) {
      const uint32_t s = lv.Fs[e - o];
      const uint64_t key = lv.Skey ? lv.Skey[s] : (uint64_t)s;
      int32_t gs[13];
      refined_neighbours((int)lv.level, (int)lv.bits, tree, lv.slot_f, key, cm, gs, err,
                         o1 - o);
#pragma unroll
      for (int q = 0; q < 13; ++q) {
        if (gs[q] < 0) continue;
        const uint32_t g = o + (uint32_t)gs[q];
        if (g != e) lds_unite(lp, (int32_t)e, (int32_t)g);
      }
    }
  }
  __syncthreads();
  // ranks of the roots (each component's smallest element) in element order
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < n; c0 += kLabSmallT) {
    const uint32_t e = c0 + t;
    const uint32_t isr = (e < n && lds_find(lp, (int32_t)e) == (int32_t)e) ? 1u : 0u;
    uint32_t inc = isr;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(inc, d, 64);
      if ((t & 63u) >= (uint32_t)d) inc += v;
    }
    if ((t & 63u) == 63u) wsum[t >> 6] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kLabSmallT / 64; ++w) {
      before += (w < (int)(t >> 6)) ? wsum[w] : 0u;
      tot += wsum[w];
    }
    if (isr) rk[e] = carry + before + inc - 1u;
    carry += tot;
    __syncthreads();
  }
  const uint32_t nroots = carry;
  for (int k = 0; k < (int)S.nlev; ++k) {
    const LabLev& lv = S.lv[k];
    const uint32_t o = (uint32_t)S.off[k], o1 = (uint32_t)S.off[k + 1];
    const uint32_t r0 = rk[o];  // a level's first element is a root
    for (uint32_t e = o + t; e < o1; e += kLabSmallT) {
      const int32_t r = lds_find(lp, (int32_t)e);
      const int32_t l = (int32_t)(rk[r] - r0);
      const uint32_t slot = (uint32_t)S.pbase[k] + (uint32_t)l;
      int4* out = reinterpret_cast<int4*>(lv.Spatch + 8 * (uint64_t)(e - o));
      out[0] = make_int4(l, l, l, l);
      out[1] = make_int4(l, l, l, l);
      const uint32_t s = lv.Fs[e - o];
      atomicAdd(&sc[slot], 8u);
      atomicAdd(&sp[slot], (unsigned long long)lv.Scount[s]);
      if (r == (int32_t)e) {
        // the patch of cell s of S_k: from this pass when it is a child of
        // the set's previous entry, else from an earlier pass (or none)
        int32_t pp = -1;
        if (k > 0) {
          const uint32_t op = (uint32_t)S.off[k - 1];
          const uint32_t ep = op + (s >> 3);
          pp = (int32_t)(rk[lds_find(lp, (int32_t)ep)] - rk[op]);
        } else if (lv.pSpatch) {
          pp = lv.pSpatch[s];
        }
        parent[slot] = pp;
      }
      if (e == o) npatch[lv.level + 1] = (o1 < n ? rk[o1] : nroots) - r0;
    }
  }
  __syncthreads();
  for (uint32_t e = t; e < nslot; e += kLabSmallT) {
    ncells[e] = sc[e];
    npart[e] = sp[e];
    pm[e] = (double)sp[e] * mscalar;
  }
}

// ------------------------------------------------------------ label queries

// patch id of each queried level-L cell (-1 if the cell is not in S_L)
__global__ void k_query_label(Tree tree, int L, const uint64_t* __restrict__ keys, uint64_t n,
                              const int32_t* __restrict__ Bcell,
                              const int32_t* __restrict__ Spatch, int32_t* __restrict__ out) {
  GRID_STRIDE(i, n) {
    const int64_t slot = tree_lookup(tree, L, keys[i]);
    int32_t r = -1;
    if (slot >= 0) {
      const int32_t bc = Bcell[slot >> 3];
      if (bc >= 0) r = Spatch[bc + (int32_t)(slot & 7)];
    }
    out[i] = r;
  }
}

// ------------------------------------------------------------ host orchestration

static double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

static Tree make_tree(const Hier* h) {
  Tree t;
  for (int l = 0; l < kMaxLevels; ++l) t.slot_child[l] = nullptr;
  for (size_t l = 0; l < h->lev.size() && l < (size_t)kMaxLevels; ++l)
    t.slot_child[l] = h->lev[l].slot_child;
  return t;
}

// Low 8-bit key digits the sort leaves out, as tuned or by depth: two when
// the keys have bits for 12 levels below the domain grid, one for 9, else
// none, so that the left-out bits lie 6 or more levels below the domain grid,
// where few particles share the remaining bits; never bits of the domain
// grid itself
static int sort_skip_bits(int B, int g, int want) {
  int k = want;
  if (k < 0) k = (B - g) >= 12 ? 2 : ((B - g) >= 9 ? 1 : 0);
  while (k > 0 && (8 * k + 2) / 3 > B - g) --k;
  return 8 * k;
}

// The build's zeroed block: 3 totals per level (FP64), then kDevU32 words of
// counters: [0] error flags, [1..7] per-level counters, [8 + 2L], [9 + 2L]
// heavy cells and chunks of level L; then, for a planned build, per level the
// raw and the clamped counts of refined cells and next-level bricks; then the
// sort's digit histograms.  The status block of a build is its first
// kZeroStatusWords words followed by the label counts.
constexpr int kDevU32 = 8 + 2 * kMaxLevels + 4 * kMaxLevels;
constexpr uint32_t kZeroStatusWords = 3 * kMaxLevels + (kDevU32 + 1) / 2;
static_assert(kZeroStatusWords + (4 + kMaxLevels + 1) / 2 <= kStatusWords, "status block size");

void build_hierarchy(Ctx* ctx, Ws& ws, Ws& wsd, const ahf_particles& p, const Params& prm,
                     hipStream_t st, Hier* h, bool finish, const Plan* plan) {
  const double t0 = now_ms();
  const bool graph = ctx->in_graph;  // no host involvement: see Ctx::in_graph
  h->prm = prm;
  h->n = p.n;
  const int g = prm.g;
  const int B = g + prm.Lmax;
  h->B = B;
  h->has_mass = p.mass != nullptr;
  h->mass_scalar = p.mass_scalar;
  const uint64_t n = p.n;

  if (!ctx->host_cnt) {
    void* hp = nullptr;
    HIP_CHECK(hipHostMalloc(&hp, 4096, hipHostMallocDefault));
    ctx->host_cnt = static_cast<uint32_t*>(hp);
    ctx->host_tot = reinterpret_cast<double*>(static_cast<char*>(hp) + 256);
    HIP_CHECK(hipEventCreateWithFlags(&ctx->cnt_ev, hipEventDisableTiming));
    for (auto& e : ctx->phase_ev) HIP_CHECK(hipEventCreateWithFlags(&e, kTimingEventFlags));
  }
  if (!graph) HIP_CHECK(hipEventRecord(ctx->phase_ev[0], st));
  // the zeroed block (cleared by a kernel, not a memset, so that a build can
  // be recorded into a graph)
  constexpr size_t kZeroWords = 3 * kMaxLevels + (kDevU32 + 1) / 2 + (kRsMaxPass * 256) / 2;
  uint64_t* zero = ws.get<uint64_t>(kZeroWords);
  k_fill_i32<<<grid_for(2 * kZeroWords), kT, 0, st>>>(reinterpret_cast<int32_t*>(zero),
                                                       2 * kZeroWords, 0);
  HIP_LAUNCH_CHECK();
  double* dev_tot = reinterpret_cast<double*>(zero);
  uint32_t* dev_u32 = reinterpret_cast<uint32_t*>(zero + 3 * kMaxLevels);
  uint32_t* lvraw = dev_u32 + 8 + 2 * kMaxLevels;
  uint32_t* lvcnt = lvraw + 2 * kMaxLevels;
  uint32_t* ghist0 = reinterpret_cast<uint32_t*>(zero + 3 * kMaxLevels + (kDevU32 + 1) / 2);
  h->planned = plan != nullptr;
  h->sizes_known = plan == nullptr;
  h->dev_lvcnt = plan ? lvcnt : nullptr;
  h->host_waits = 0;
  uint32_t* err = dev_u32;
  ctx->dev_err = err;

  // ---- keys and their stable sort
  // The radix sort may leave out the lowest `skip` key bits (fewer passes);
  // runs of particles that those bits alone would order are then sorted by
  // the gather (and k_fix_runs), so that everything after it sees the full
  // stable sort.
  const Tuning tune = ctx->tuning_for(n);
  const int skip = sort_skip_bits(B, g, tune.sort_skip);
  uint64_t* keys = ws.get<uint64_t>(n);
  uint4* rec = ws.get<uint4>(2 * n);
  const SortPlan sp = sort_plan(n, 3 * B - skip);
  h->sort_key_bits = (uint32_t)(3 * B - skip);
  h->sort_passes = n ? (uint32_t)sp.npass : 0u;
  h->order = h->mem.get<uint32_t>(n);
  uint4* srec = ws.get<uint4>(2 * n);
  uint64_t* skey = keys;
  // level 0 is dense: its cell starts come with the gather
  const uint64_t ncell0 = 1ull << (3 * g);
  uint32_t* start0 = h->mem.get<uint32_t>(ncell0 + 1);
  if (n > 0) {
    uint32_t* ghist = ghist0;
    unsigned kb = grid_for(n);
    if (kb > 2048) kb = 2048;
    AHF_TIMED(ctx, "keys", st,
              (k_keys<<<kb, 256, 0, st>>>(p.x, p.y, p.z, p.fx, p.fy, p.fz, p.mass,
                                          (float)p.mass_scalar, n, B, sp.npass,
                                          sp.q == 0 ? sp.ib : -1, skip, keys, rec, ghist,
                                          err)));
    uint64_t* spare = nullptr;
    const uint64_t* words = sort_keys(ctx, ws, keys, n, sp, ghist, st, &spare);
    skey = spare;  // the full sorted keys go to the sort's free buffer
    // with left-out key bits: the runs crossing wave boundaries, listed by
    // the gather (at most one per wave), then the long ones among them
    uint32_t* nfix = nullptr;
    uint32_t* cross = nullptr;
    Ws::Mark fm = ws.mark();
    if (skip) {
      nfix = ws.get<uint32_t>(2);
      cross = ws.get<uint32_t>((n + 1) / 64 + 2);
      k_fill_i32<<<1, 64, 0, st>>>(reinterpret_cast<int32_t*>(nfix), 2, 0);
      HIP_LAUNCH_CHECK();
    }
    AHF_TIMED(ctx, "gather", st,
              (k_gather_rec<<<grid_for(n + 1), kT, 0, st>>>(words, sp.ib, kQBits - B, n, rec,
                                                            srec, h->order, skey, 3 * (B - g),
                                                            ncell0, start0, skip, nfix, cross)));
    if (skip) {
      // scratch: the lists, and what the gather leaves behind
      const uint64_t lcap = n / (kShortRun + 1) + 1;
      uint32_t* long_a = ws.get<uint32_t>(lcap);
      uint32_t* long_m = ws.get<uint32_t>(lcap);
      uint64_t* kb2 = ws.get<uint64_t>(n);
      uint32_t* va2 = ws.get<uint32_t>(n);
      uint32_t* vb2 = ws.get<uint32_t>(n);
      AHF_TIMED(ctx, "fix_runs", st,
                (k_fix_runs<<<1024, 256, 0, st>>>(nfix, cross, skey, srec, h->order, n, skip,
                                                  nfix + 1, long_a, long_m)));
      AHF_TIMED(ctx, "fix_long_runs", st,
                (k_fix_long_runs<<<2048, kBT, 0, st>>>(nfix + 1, long_a, long_m, skey, srec,
                                                       h->order, const_cast<uint64_t*>(words),
                                                       kb2, va2, vb2, rec)));
    }
    ws.release(fm);
  }

  Parts P;
  P.rec = srec;
  if (!graph) HIP_CHECK(hipEventRecord(ctx->phase_ev[1], st));

  // ---- levels
  // With the count criterion a level's deposit needs only its cells and its
  // heavy-cell lists: it runs on the second stream while this one goes on
  // to the next level's cells.  (The density criterion needs the deposit
  // for the flags: one stream; so do the builds of a server's workers.)
  const bool density = (prm.flags & AHF_DENSITY_CRITERION) != 0;
  const bool overlap = !density && !ctx->one_stream;
  if (overlap && !ctx->dep_st) {
    HIP_CHECK(hipStreamCreateWithFlags(&ctx->dep_st, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&ctx->dep_ev, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming));
  }
  hipStream_t ds = overlap ? ctx->dep_st : st;
  Ws& wd = overlap ? wsd : ws;  // deposit scratch: kept to the end of the build when overlapped
  // Sizes of the level being built.  Synced (no plan): the host reads each
  // level's refined cells and next-level bricks once their kernels are done
  // (one wait per level) and sizes the next level exactly.  Planned: every
  // level is enqueued at once, sized by the plan's capacities; the kernels
  // read the true counts on the device (Cnt), clamped to the capacities, and
  // k_level_check flags a level that did not fit (the build is then redone
  // synced).
  const bool planned = plan != nullptr;
  const uint64_t nFp0 = 1ull << (3 * (g - 1));  // parents of level 0: the virtual level -1
  Cnt cFp = host_cnt(nFp0);                     // parents of the level (F_{L-1})
  Cnt cB = host_cnt(nFp0);                      // bricks of the level
  uint64_t* Bkey = nullptr;
  int32_t* Bcell = nullptr;
  int32_t* Pbrick = nullptr;
  h->lev.clear();
  h->lev.reserve(kMaxLevels);
  uint32_t* rank0 = nullptr;  // rank of each refined level-0 cell in F_0 (dense tiles)
  double* part_all = ws.get<double>((uint64_t)kMaxLevels * 3 * kSumBlocks);
  SumBlocks sum_blocks;
  // equal masses: the labels need only the cells, so those of the first
  // levels start, on a third stream, as soon as the levels get small (the
  // last levels leave most of the GPU idle); a planned build labels after it
  const bool early_labels = overlap && !(prm.flags & AHF_NO_LABELS) && !h->has_mass;
  const int last_level = planned ? plan->depth : prm.Lmax;
  for (int L = 0; L <= last_level; ++L) {
    h->lev.emplace_back();
    Level& lv = h->lev.back();
    const int b = g + L;
    lv.b = (uint32_t)b;
    const int sh = 3 * (B - b);
    if (L == 0 && g >= 2 && g <= kTileMaxG) rank0 = ws.get<uint32_t>(1ull << (3 * g));
    Ws::Mark lvl_mark = ws.mark();
    // the level's cells: all 8 children of every parent (level 0: dense)
    const Cnt cS = L == 0 ? host_cnt(ncell0) : Cnt{cFp.p, 8u, 8 * cFp.cap};
    const Cnt cSlot{cB.p, 8u, 8 * cB.cap};  // brick cells (slots) of the level
    uint32_t* rawF = planned ? lvraw + 2 * L : dev_u32 + 1;   // refined cells (raw count)
    uint32_t* rawD = planned ? lvraw + 2 * L + 1 : dev_u32 + 4;  // next-level bricks
    lv.nS = cS.cap;
    if (L == 0) {
      lv.Sstart = start0;
      lv.Scount = h->mem.get<uint32_t>(lv.nS);
      if (n == 0)  // no gather: every cell starts (and ends) at 0
        k_fill_i32<<<grid_for(lv.nS + 1), kT, 0, st>>>(reinterpret_cast<int32_t*>(lv.Sstart),
                                                       lv.nS + 1, 0);
    } else {
      const Level& pv = h->lev[L - 1];
      lv.Skey = h->mem.get<uint64_t>(lv.nS);
      lv.Sstart = h->mem.get<uint32_t>(lv.nS);
      lv.Scount = h->mem.get<uint32_t>(lv.nS);
      AHF_TIMED(ctx, "child_ranges", st,
                (k_child_ranges<<<grid_for(lv.nS), kT, 0, st>>>(skey, cS, pv.Fs, pv.Sstart,
                                                                pv.Scount, pv.Skey, sh, lv.Skey,
                                                                lv.Sstart, lv.Scount)));
    }
    lv.nB = cB.cap;
    lv.Bkey = Bkey;
    lv.Bcell = Bcell;
    lv.Pbrick = Pbrick;
    lv.Sflag = h->mem.get<uint8_t>(lv.nS);
    // particle mass per cell: only needed when masses differ (else count x m)
    lv.Spmass = p.mass ? h->mem.get<double>(lv.nS) : nullptr;

    // refinement flags and the cells too full for one thread
    const int can_refine = (L < prm.Lmax && b < kQBits) ? 1 : 0;
    const double thr = (L == 0) ? prm.dom_ref : prm.ref_ref;
    // heavy-cell lists, sized by bounds: cells above `heavy` particles (the
    // same threshold for the flag kernel's lists and the level's deposit) are
    // summed by waves; at most n/(heavy+1) of them, at most that many plus
    // n/kChunk chunks
    const uint32_t heavy = tune.heavy[L < 2 ? L : 2];
    const uint64_t maxH = std::min<uint64_t>(lv.nS, n / (heavy + 1) + 1);
    const uint64_t maxch = maxH + n / kChunk + 1;
    HeavyList hl;
    hl.nheavy = dev_u32 + 8 + 2 * L;   // the level's own counters, zero from the start
    hl.nchunks = dev_u32 + 9 + 2 * L;
    hl.Hs = wd.get<uint32_t>(maxH);
    hl.hidx = wd.get<int32_t>(lv.nS);  // read only for heavy cells
    hl.nch = wd.get<uint32_t>(maxH);
    hl.chofs = wd.get<uint32_t>(maxH);
    hl.ch_a = wd.get<uint32_t>(maxch);
    hl.ch_n = wd.get<uint32_t>(maxch);
    const int32_t* hidx = hl.hidx;
    // with the count criterion the flags come here; with the density
    // criterion they need the level's deposit and come after it
    k_flags<<<std::min(grid_for(lv.nS, kFlagT), kFlagBlocks), kFlagT, 0, st>>>(
        L == 0 ? nullptr : lv.Scount, lv.Sstart, cS, thr, density ? 0 : can_refine, heavy,
        lv.Sflag,
        hl, (L == 0 && !density) ? rank0 : nullptr, L == 0 ? lv.Scount : nullptr);
    HIP_LAUNCH_CHECK();
    if (overlap) {
      // the level's cells and heavy lists are complete: its deposit may start
      HIP_CHECK(hipEventRecord(ctx->dep_ev, st));
      HIP_CHECK(hipStreamWaitEvent(ds, ctx->dep_ev, 0));
    }
    uint32_t* Ftmp = ws.get<uint32_t>(lv.nS);
    uint32_t* rankF = (L == 0 && rank0) ? rank0 : ws.get<uint32_t>(lv.nS);
    const uint64_t nslot = cSlot.cap;
    uint8_t* mark = nullptr;
    uint32_t* rank = nullptr;
    auto flag_phase = [&]() {
    compact_flags(ws, lv.Sflag, cS, Ftmp, rankF, rawF, st);

    // the dilation of F_L: slots of level L that hold a brick on level L+1
    // (sized by the bound nF <= nS, so that one sync per level reads nF, the
    // heavy-cell count and the brick count together)
    if (can_refine) {
      lv.slot_f = h->mem.get<int32_t>(nslot);
      mark = ws.get<uint8_t>(nslot);
      rank = ws.get<uint32_t>(nslot);
      k_slots<<<grid_for(nslot), kT, 0, st>>>(cSlot, L == 0 ? nullptr : lv.Bcell, lv.Sflag, rankF,
                                              lv.slot_f, L == 0 ? nullptr : mark);
      HIP_LAUNCH_CHECK();
      if (L == 0) {
        AHF_TIMED(ctx, "mark", st,
                  (k_mark_dense0<<<grid_for(nslot), kT, 0, st>>>(g, nslot, lv.Sflag, mark)));
      } else {
        Tree tree = make_tree(h);
        unsigned mb = grid_for(lv.nS * 27);
        if (mb > 8192) mb = 8192;
        AHF_TIMED(ctx, "mark", st,
                  (k_mark<<<mb, kT, 0, st>>>(L, b, rawF, Ftmp, lv.Skey, tree, mark, err)));
      }
      compact_flags(ws, mark, cSlot, nullptr, rank, rawD, st);
    }
    if (planned) {
      // the counts stay on the device: clamped to the plan, checked
      k_level_check<<<1, 64, 0, st>>>(rawF, plan->capF[L], plan->capD[L], L == last_level ? 1 : 0,
                                      lvcnt + 2 * L, err);
      HIP_LAUNCH_CHECK();
    } else {
      // the counts travel to the host while the level's deposit runs
      HIP_CHECK(hipMemcpyAsync(ctx->host_cnt, dev_u32 + 1, 4 * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipEventRecord(ctx->cnt_ev, st));
    }
    };
    if (!density) flag_phase();

    const uint32_t mask = (1u << (kQBits - b)) - 1u;
    const float scale = std::ldexp(1.0f, -(kQBits - b));

    // heavy cells: chunked wave sums (sizes from the device counts; buffers
    // and grids from the bound maxH)
    float* hT = wd.get<float>(maxH * 27);
    double* hM = wd.get<double>(maxH);
    {
      float* chT = wd.get<float>(maxch * 27);
      double* chM = wd.get<double>(maxch);
      AHF_TIMED(ctx, "heavy_chunk", ds,
                (k_heavy_chunk<<<(unsigned)std::min<uint64_t>((maxch + 3) / 4, 2048), 256, 0, ds>>>(
                    hl.nchunks, hl.ch_a, hl.ch_n, P, mask, scale, chT, chM)));
      k_heavy_reduce<<<(unsigned)std::min<uint64_t>((maxH + 3) / 4, 2048), 256, 0, ds>>>(
          hl.nch, hl.chofs, hl.nheavy, chT, chM, hT, hM);
      HIP_LAUNCH_CHECK();
    }

    // TSC deposit: by dense tiles where the parents form a well-filled grid,
    // else parent patches, then brick cells
    lv.mass = h->mem.get<float>(8 * cB.cap);
    const bool tiles0 = L == 0 && g - 1 >= 2 && g <= kTileMaxG;
    const bool tiles1 = L == 1 && g >= 2 && g <= kTileMaxG && rank0 &&
                        8 * cFp.cap >= (1ull << (3 * g));
    if (tiles0 || tiles1) {
      const int pb = tiles0 ? g - 1 : g;  // bits per axis of the parent grid
      const uint64_t ntiles = 1ull << (3 * (pb - 2));
      float* halo = wd.get<float>(ntiles * kTileH);
      const Level& l0 = h->lev[0];
      if (tiles0)
        AHF_TIMED(ctx, "tile_deposit0", ds,
                  (k_tile_deposit<true, 2><<<(unsigned)ntiles, kTileT, 0, ds>>>(
                      nullptr, lv.Sstart, lv.Scount, hidx, hT, hM, P, mask, scale, heavy, nullptr,
                      lv.mass, halo, lv.Spmass, 0)));
      else if (tune.batch1 >= 4)
        AHF_TIMED(ctx, "tile_deposit1", ds,
                  (k_tile_deposit<false, 4><<<(unsigned)ntiles, kTileT, 0, ds>>>(
                      rank0, lv.Sstart, lv.Scount, hidx, hT, hM, P, mask, scale, heavy,
                      l0.slot_child, lv.mass, halo, lv.Spmass, cFp.cap)));
      else
        AHF_TIMED(ctx, "tile_deposit1", ds,
                  (k_tile_deposit<false, 2><<<(unsigned)ntiles, kTileT, 0, ds>>>(
                      rank0, lv.Sstart, lv.Scount, hidx, hT, hM, P, mask, scale, heavy,
                      l0.slot_child, lv.mass, halo, lv.Spmass, cFp.cap)));
      AHF_TIMED(ctx, "tile_halo", ds,
                (k_tile_halo_add<<<(unsigned)ntiles, 256, 0, ds>>>(
                    tiles0 ? 1 : 0, pb - 2, tiles0 ? nullptr : l0.slot_child, halo, lv.mass)));
    } else {
      float* patch = wd.get<float>(cFp.cap * 64);
      if (cFp.cap) {
        AHF_TIMED(ctx, "patches", ds,
                  (k_patches<<<(unsigned)((cFp.cap + 31) / 32), 256, 0, ds>>>(
                      cFp, lv.Sstart, lv.Scount, hidx, hT, hM, P, mask, scale, heavy, patch,
                      lv.Spmass)));
      }
      Tree tree = make_tree(h);
      const int32_t* pslot_f = (L > 0) ? h->lev[L - 1].slot_f : nullptr;
      AHF_TIMED(ctx, "combine", ds,
                (k_combine<<<(unsigned)((cB.cap + 31) / 32), 256, 0, ds>>>(
                    L, cB, Bkey, b - 1, tree, pslot_f, patch, lv.mass, cFp.cap)));
    }
    if (density) {
      k_flags_density<<<grid_for(lv.nS), kT, 0, st>>>(lv.nS, lv.mass, lv.Pbrick, p.mass_scalar,
                                                      thr, can_refine, lv.Sflag,
                                                      (L == 0) ? rank0 : nullptr);
      HIP_LAUNCH_CHECK();
      flag_phase();
    }
    {
      const uint64_t nmax = (8 * cB.cap > lv.nS) ? 8 * cB.cap : lv.nS;
      int nblk = (int)((nmax + 255) / 256);
      if (nblk > kSumBlocks) nblk = kSumBlocks;
      if (nblk < 1) nblk = 1;
      k_level_sums<<<nblk, 256, 0, ds>>>(lv.mass, cSlot, lv.Spmass, cS, lv.Scount, cS,
                                         part_all + (uint64_t)L * 3 * kSumBlocks);
      HIP_LAUNCH_CHECK();
      sum_blocks.n[L] = nblk;
    }

    uint64_t capF, capD;
    if (planned) {
      capF = plan->capF[L];
      capD = can_refine ? plan->capD[L] : 0;
      lv.capF = capF;
      // the early labels, once the levels get small (by their capacities)
      if (early_labels && L >= 2 && h->lab_done == 0 && 8 * cFp.cap < kLabEarlyCells)
        label_early(ctx, wsd, h, (uint32_t)L, st);
      if (L == last_level) {
        ws.release(lvl_mark);
        break;
      }
    } else {
      // the host enqueues the early labels while it would otherwise wait
      if (early_labels && L >= 2 && h->lab_done == 0 && 8 * cFp.cap < kLabEarlyCells)
        label_early(ctx, wsd, h, (uint32_t)L, st);
      HIP_CHECK(hipEventSynchronize(ctx->cnt_ev));
      h->host_waits += 1;
      capF = ctx->host_cnt[0];
      capD = can_refine ? ctx->host_cnt[3] : 0u;
      lv.nF = capF;
    }
    lv.capF = capF;
    lv.Fs = h->mem.get<uint32_t>(capF);  // filled from Ftmp by k_build_bricks below
    if (!planned && lv.nF == 0) {
      lv.slot_f = nullptr;  // no refined cell: nothing to look up
      ws.release(lvl_mark);
      break;
    }

    // bricks of level L+1: children of every level-L cell within one cell of F_L
    lv.slot_child = h->mem.get<int32_t>(nslot);
    uint64_t* nBkey = h->mem.get<uint64_t>(capD);
    int32_t* nBcell = h->mem.get<int32_t>(capD);
    int32_t* nPbrick = h->mem.get<int32_t>(capF);
    if (can_refine) {
      k_build_bricks<<<grid_for(std::max<uint64_t>(nslot, capF)), kT, 0, st>>>(
          cSlot, mark, rank, lv.Bkey, lv.slot_f, lv.slot_child, nBkey, nBcell, Ftmp, lv.Fs,
          nPbrick, capD, capF, rawF);
      HIP_LAUNCH_CHECK();
    } else {
      // the level cap: no brick of a next level (a planned build only gets
      // here with no refined cell, which the check kernel has verified)
      k_fill_i32<<<grid_for(nslot), kT, 0, st>>>(lv.slot_child, nslot, -1);
      HIP_LAUNCH_CHECK();
    }
    cFp = planned ? Cnt{lvcnt + 2 * L, 1u, capF} : host_cnt(capF);
    cB = planned ? Cnt{lvcnt + 2 * L + 1, 1u, capD} : host_cnt(capD);
    Bkey = nBkey;
    Bcell = nBcell;
    Pbrick = nPbrick;
    ws.release(lvl_mark);
  }

  // once labels have started early, the rest go to the label stream as well:
  // they need the cells only, not the deposits still running (a build with
  // no host involvement labels every level there)
  if (early_labels && (h->lab_done > 0 || graph) && h->lev.size() > 1)
    label_early(ctx, wsd, h, (uint32_t)(h->lev.size() - 1), st);
  if (overlap) {
    // the deposits back into the build stream
    HIP_CHECK(hipEventRecord(ctx->join_ev, ds));
    HIP_CHECK(hipStreamWaitEvent(st, ctx->join_ev, 0));
  }
  // every level's totals from its partial sums, one block per level
  k_level_sums_final<<<(unsigned)h->lev.size(), 256, 0, st>>>(part_all, sum_blocks, dev_tot);
  HIP_LAUNCH_CHECK();

  h->t_start = t0;
  if (graph) {
    // the host reads the block after the run (enqueue_status)
    h->dev_status = zero;
    return;
  }
  // totals and the device error flags, into pinned memory; read by
  // finish_build once the stream has passed this point
  HIP_CHECK(hipEventRecord(ctx->phase_ev[2], st));
  // (the error flags and the counters follow the totals in the zeroed
  // block: one copy)
  static_assert(sizeof(double) * 3 * kMaxLevels % 8 == 0, "flags right after the totals");
  static_assert(256 + sizeof(double) * 3 * kMaxLevels + sizeof(uint32_t) * kDevU32 <= 4096,
                "the pinned count area holds the copy");
  HIP_CHECK(hipMemcpyAsync(ctx->host_tot, dev_tot,
                           3 * kMaxLevels * sizeof(double) + kDevU32 * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, st));
  if (finish) {
    HIP_CHECK(hipStreamSynchronize(st));
    finish_build(ctx, h);
  }
}

static void label_finish(Hier* h, const uint32_t* hv);

// completes h from a host copy of its totals and device counters (the
// layout of the build's zeroed block); throws on device errors
static void finish_from(Hier* h, const double* tot) {
  uint32_t herr = 0;
  std::memcpy(&herr, tot + 3 * kMaxLevels, sizeof(uint32_t));
  if (h->planned) {
    // a level that outgrew its room: everything after it is clamped, so the
    // build is redone with a wait per level
    if (herr & kErrCapacity) throw Error{kStatusReplan, "a planned level outgrew its capacity"};
    // the true sizes from the device counts; levels past the last one that
    // has cells are dropped
    const uint32_t* u = reinterpret_cast<const uint32_t*>(tot + 3 * kMaxLevels);
    const uint32_t* cnt = u + 8 + 4 * kMaxLevels;
    size_t keep = h->lev.size();
    for (size_t L = 0; L < h->lev.size(); ++L) {
      Level& lv = h->lev[L];
      if (L > 0) {
        lv.nS = 8ull * cnt[2 * (L - 1)];
        lv.nB = cnt[2 * (L - 1) + 1];
        if (lv.nS == 0 && keep == h->lev.size()) keep = L;
      }
      lv.nF = cnt[2 * L];
    }
    h->lev.resize(keep);
    if (!h->lev.empty() && h->lev.back().nF == 0) h->lev.back().slot_f = nullptr;
    h->sizes_known = true;
    h->dev_lvcnt = nullptr;
  }
  for (size_t L = 0; L < h->lev.size(); ++L) {
    h->lev[L].tot_cell = tot[3 * L + 0];
    h->lev[L].nP = (uint64_t)tot[3 * L + 2];
    h->lev[L].tot_part = h->has_mass ? tot[3 * L + 1] : (double)h->lev[L].nP * h->mass_scalar;
  }
  h->ms[3] = now_ms() - h->t_start;
  if (herr & kErrCoord) throw Error{AHF_EINVAL, "a particle coordinate is >= 2^21"};
  if (herr) throw Error{AHF_EDEVICE, "internal consistency check failed on the device"};
}

void finish_build(Ctx* ctx, Hier* h) {
  finish_from(h, ctx->host_tot);
  float e01 = 0.0f, e12 = 0.0f;
  HIP_CHECK(hipEventElapsedTime(&e01, ctx->phase_ev[0], ctx->phase_ev[1]));
  HIP_CHECK(hipEventElapsedTime(&e12, ctx->phase_ev[1], ctx->phase_ev[2]));
  h->ms[0] = e01;
  h->ms[1] = e12;
}

// The status block: the build's zeroed block up to the end of its counters
// (level totals, error flags, counters, level counts), then the label counts.
__global__ void k_copy_status(uint64_t* __restrict__ dst, const uint64_t* __restrict__ blk,
                              const uint32_t* __restrict__ lab) {
  constexpr uint32_t kLabWords = (4 + kMaxLevels + 1) / 2;
  for (uint32_t i = threadIdx.x; i < kStatusWords; i += blockDim.x) {
    uint64_t v = 0;
    if (i < kZeroStatusWords) {
      v = blk[i];
    } else if (i < kZeroStatusWords + kLabWords && lab) {
      const uint32_t j = 2 * (i - kZeroStatusWords);
      const uint64_t lo = lab[j];
      const uint64_t hi = j + 1 < 4 + kMaxLevels ? lab[j + 1] : 0u;
      v = lo | (hi << 32);
    }
    dst[i] = v;
  }
}

void enqueue_status(Hier* h, uint64_t* dst, hipStream_t st) {
  k_copy_status<<<1, 64, 0, st>>>(dst, h->dev_status, h->lab_dev);
  HIP_LAUNCH_CHECK();
}

void finish_from_status(Hier* h, const uint64_t* status) {
  finish_from(h, reinterpret_cast<const double*>(status));
  if (h->lab_dev) label_finish(h, reinterpret_cast<const uint32_t*>(status + kZeroStatusWords));
}

void query_labels(Ws& ws, const Hier* h, int L, uint64_t n, const uint64_t* keys_host,
                  int32_t* out_host, hipStream_t st) {
  const Level& lv = h->lev[L];
  Ws::Mark m = ws.mark();
  uint64_t* dk = ws.get<uint64_t>(n);
  int32_t* dout = ws.get<int32_t>(n);
  HIP_CHECK(hipMemcpyAsync(dk, keys_host, n * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  k_query_label<<<grid_for(n), kT, 0, st>>>(make_tree(h), L, dk, n, lv.Bcell, lv.Spatch, dout);
  HIP_LAUNCH_CHECK();
  HIP_CHECK(hipMemcpyAsync(out_host, dout, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  ws.release(m);
}

// ------------------------------------------------------------ label queries without allocation
//
// For callers that cannot allocate device memory: the query keys and the
// results are staged in one file-scope device array instead of the context's
// workspace.  Each GPU holds its own copy of the array; its address on a
// device comes from hipGetSymbolAddress, taken once per device with that
// device current (the name itself is only a host-side stand-in).
constexpr uint64_t kStaticQueryMax = 1ull << 18;  // keys per call (3 MB of staging)
static __device__ __align__(256) uint64_t scratch[kStaticQueryMax + kStaticQueryMax / 2];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// the array's address on `device`, looked up on the first call for that
// device (the caller has made it current)
void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error{AHF_EINVAL, "device ordinal out of range"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

// patch ids of n level-L keys (host arrays) through the static staging area;
// level >= 1, labelled, n <= kStaticQueryMax
static void query_labels_static(const Hier* h, int L, uint64_t n, const uint64_t* keys_host,
                                int32_t* out_host, hipStream_t st) {
  const Level& lv = h->lev[L];
  uint64_t* dk = static_cast<uint64_t*>(static_scratch(h->ctx->device));
  int32_t* dout = reinterpret_cast<int32_t*>(dk + kStaticQueryMax);
  HIP_CHECK(hipMemcpyAsync(dk, keys_host, n * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  k_query_label<<<grid_for(n), kT, 0, st>>>(make_tree(h), L, dk, n, lv.Bcell, lv.Spatch, dout);
  HIP_LAUNCH_CHECK();
  HIP_CHECK(hipMemcpyAsync(out_host, dout, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
}

// the two pinned level sets of a context (the early and the final label pass)
// The level set of a label pass goes to the device as a kernel argument: the
// launch carries its own copy, so the host may reuse its memory at once and
// the hand-over is part of whatever records the launch into a graph.
static_assert(sizeof(LabSet) + sizeof(LabSet*) <= 4096, "kernel arguments are at most 4 KB");
__global__ void k_put_labset(LabSet* __restrict__ d, const LabSet s) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d = s;
}

// The label counts of a hierarchy: [0] error flags, [1] roots of the running
// batch, [4 + L] patches on level L.  Kept with the hierarchy.
static void label_counts(Ctx* ctx, Hier* h, hipStream_t st) {
  (void)ctx;
  if (h->lab_dev) return;
  h->lab_dev = h->mem.get<uint32_t>(4 + kMaxLevels);
  k_fill_i32<<<1, 64, 0, st>>>(reinterpret_cast<int32_t*>(h->lab_dev), 4 + kMaxLevels, 0);
  HIP_LAUNCH_CHECK();
}

// Labels the refined cells of levels k0 .. k1-1 (the patches of levels
// k0+1 .. k1) on st, all of them at once; level k0's patches (k0 > 0) must
// be labelled already.  With keep, the scratch stays allocated (ws may be
// handed to other work while these kernels run).
static void label_levels(Ctx* ctx, Ws& ws, Hier* h, uint32_t k0, uint32_t k1, bool keep,
                         hipStream_t st) {
  (void)ctx;
  uint32_t* dev = h->lab_dev;
  const Tree tree = make_tree(h);
  const double total_mass = h->lev.empty() ? 0.0 : h->lev[0].tot_part;
  double fscale = 1.0;
  if (h->has_mass) {
    int e = 0;
    std::frexp(total_mass > 0 ? total_mass : 1.0, &e);
    fscale = std::ldexp(1.0, 61 - e);
  }
  // entry j = the refined cells of level k0 + j, parents of the cells of
  // level k0 + j + 1
  // With the level sizes on the device only (a planned build labelling
  // during the build), the arrays and grids are laid out by the levels'
  // capacities and the element offsets come from the device counts.
  const bool dev_sizes = !h->sizes_known;
  LabSet S{};
  S.nlev = k1 > k0 ? k1 - k0 : 0u;
  uint64_t tot = 0, ntiles = 0;
  for (uint32_t j = 0; j < S.nlev; ++j) {
    const Level& pv = h->lev[k0 + j];
    const uint64_t c = dev_sizes ? pv.capF : pv.nF;
    S.off[j] = tot;
    S.toff[j] = ntiles;
    S.pbase[j] = tot;
    tot += c;
    ntiles += (c + kUfTile - 1) / kUfTile;
  }
  S.off[S.nlev] = tot;
  S.toff[S.nlev] = ntiles;
  S.pbase[S.nlev] = tot;
  S.total = (uint32_t)tot;
  if (tot >= (1ull << 31)) throw Error{AHF_ELIMIT, "too many refined cells to label"};
  const uint64_t tot1 = tot ? tot : 1;
  int32_t* Spatch = h->mem.get<int32_t>(8 * tot1);
  int32_t* pparent = h->mem.get<int32_t>(tot1);
  uint32_t* pncells = h->mem.get<uint32_t>(tot1);
  uint64_t* pnpart = h->mem.get<uint64_t>(tot1);
  double* pmass = h->mem.get<double>(tot1);
  for (uint32_t j = 0; j < S.nlev; ++j) {
    const uint32_t k = k0 + j;
    const Level& pv = h->lev[k];
    Level& lv = h->lev[k + 1];
    lv.Spatch = Spatch + 8 * S.pbase[j];
    lv.patch_parent = pparent + S.pbase[j];
    lv.patch_ncells = pncells + S.pbase[j];
    lv.patch_npart = pnpart + S.pbase[j];
    lv.patch_mass = pmass + S.pbase[j];
    S.lv[j] = LabLev{pv.Fs, pv.Skey, pv.slot_f, pv.Scount, pv.Spmass, lv.Spatch,
                     k > 0 ? pv.Spatch : nullptr, k, pv.b};
  }
  if (!tot) return;
  Ws::Mark m = ws.mark();
  if (tot <= kLabSmallMax && !h->has_mass) {
    // few elements: the whole pass in one block
    LabSet* dS = ws.get<LabSet>(1);
    k_put_labset<<<1, 64, 0, st>>>(dS, S);
    HIP_LAUNCH_CHECK();
    if (dev_sizes) {
      k_labset_counts<<<1, 64, 0, st>>>(dS, h->dev_lvcnt, (int)k0);
      HIP_LAUNCH_CHECK();
    }
    k_label_small<<<1, kLabSmallT, 0, st>>>(dS, tree, h->prm.conn, pncells,
                                            reinterpret_cast<unsigned long long*>(pnpart),
                                            pparent, pmass, h->mass_scalar, dev + 4, dev);
    HIP_LAUNCH_CHECK();
    if (!keep) ws.release(m);
    return;
  }
  int32_t* par = ws.get<int32_t>(tot);
  int32_t* root = ws.get<int32_t>(tot);
  uint8_t* pred = ws.get<uint8_t>(tot);
  uint32_t* rank = ws.get<uint32_t>(tot);
  int32_t* lab = ws.get<int32_t>(tot);
  uint16_t* xmask = ws.get<uint16_t>(tot);
  unsigned long long* mfix = h->has_mass ? ws.get<unsigned long long>(tot) : nullptr;
  LabSet* dS = ws.get<LabSet>(1);
  k_put_labset<<<1, 64, 0, st>>>(dS, S);
    HIP_LAUNCH_CHECK();
  if (dev_sizes) {
    k_labset_counts<<<1, 64, 0, st>>>(dS, h->dev_lvcnt, (int)k0);
    HIP_LAUNCH_CHECK();
  }
  const Cnt ctot{dev_sizes ? &dS->total : nullptr, 1u, tot};
  AHF_TIMED(ctx, "uf_hook", st,
            (k_uf_local<<<(unsigned)ntiles, 256, 0, st>>>(dS, tree, h->prm.conn, par, xmask, dev)));
  AHF_TIMED(ctx, "uf_cross", st,
            (k_uf_cross<<<(unsigned)ntiles, 256, 0, st>>>(dS, tree, xmask, par, dev)));
  k_uf_compress<<<grid_for(tot), kT, 0, st>>>(par, ctot, root, pred, tot, pncells,
                                              (unsigned long long*)pnpart, mfix);
  HIP_LAUNCH_CHECK();
  compact_flags(ws, pred, ctot, nullptr, rank, dev + 1, st);
  k_uf_label<<<grid_for(tot), kT, 0, st>>>(dS, root, rank, dev + 1, lab, dev + 4);
  HIP_LAUNCH_CHECK();
  k_patch_stats<<<(unsigned)std::min<uint64_t>(256, (tot + 4095) / 4096 + 1), 256, 0, st>>>(
      dS, lab, fscale, pncells, (unsigned long long*)pnpart, mfix);
  HIP_LAUNCH_CHECK();
  k_patch_parent<<<grid_for(tot), kT, 0, st>>>(dS, root, lab, pparent,
                                               (const unsigned long long*)pnpart, mfix,
                                               h->mass_scalar, 1.0 / fscale, pmass);
  HIP_LAUNCH_CHECK();
  // stream order keeps the released workspace from being reused early
  if (!keep) ws.release(m);
}

void label_early(Ctx* ctx, Ws& wsd, Hier* h, uint32_t k1, hipStream_t st) {
  if (!ctx->lab_st) {
    HIP_CHECK(hipStreamCreateWithFlags(&ctx->lab_st, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&ctx->lab_ev, hipEventDisableTiming));
  }
  if (k1 <= h->lab_done) return;
  label_counts(ctx, h, st);
  // the cells of levels lab_done .. k1 are complete on st
  HIP_CHECK(hipEventRecord(ctx->lab_ev, st));
  HIP_CHECK(hipStreamWaitEvent(ctx->lab_st, ctx->lab_ev, 0));
  label_levels(ctx, wsd, h, h->lab_done, k1, true, ctx->lab_st);
  h->lab_done = k1;
}

void label_enqueue(Ctx* ctx, Ws& ws, Hier* h, hipStream_t st) {
  const size_t nlev = h->lev.size();
  label_counts(ctx, h, st);
  ctx->dev_err = h->lab_dev;
  if (h->lab_done > 0) {
    // the levels labelled early, on their stream, come first
    HIP_CHECK(hipEventRecord(ctx->lab_ev, ctx->lab_st));
    HIP_CHECK(hipStreamWaitEvent(st, ctx->lab_ev, 0));
  }
  const uint32_t kend = nlev > 1 ? (uint32_t)(nlev - 1) : 0u;
  if (h->lab_done < kend) label_levels(ctx, ws, h, h->lab_done, kend, false, st);
  h->npatch_dev = h->lab_dev + 4;
}

// the label counts read back: [0] error flags, [4 + L] patches on level L
static void label_finish(Hier* h, const uint32_t* hv) {
  if (hv[0]) throw Error{AHF_EDEVICE, "internal consistency check failed while labelling"};
  for (size_t L = 1; L < h->lev.size(); ++L) h->lev[L].nPatch = hv[4 + L];
  h->npatch_dev = h->lab_dev + 4;
  h->labelled = true;
}

void label_hierarchy(Ctx* ctx, Ws& ws, Hier* h, hipStream_t st) {
  if (h->labelled) return;
  const double t0 = now_ms();
  const size_t nlev = h->lev.size();
  label_enqueue(ctx, ws, h, st);
  if (h->prm.flags & AHF_SUBSTRUCTURE) classify_levels(ctx, ws, h, st);
  std::vector<uint32_t> hv(4 + nlev);
  HIP_CHECK(hipMemcpyAsync(hv.data(), h->lab_dev, (4 + nlev) * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  label_finish(h, hv.data());
  if (h->prm.flags & AHF_SUBSTRUCTURE) finish_classify(ctx, h, st);
  h->ms[2] = now_ms() - t0;
  h->ms[3] += h->ms[2];
}


// ------------------------------------------------------------ substructure
//
// The grid tree walked from coarse to fine (Sect. 2.1, classification of the
// grid tree into substructure): every level-1 patch starts a host structure;
// where a patch has several children, the child with the most particles
// (ties: the lower patch id) continues the parent's structure and every
// other child starts a substructure of it.  Structures are numbered by
// (start level, start patch); base[L] = structures starting on levels <= L.

__global__ void k_struct_roots(const uint32_t* __restrict__ npdev, int32_t* __restrict__ pstruct,
                               int32_t* __restrict__ s_host, int32_t* __restrict__ s_level,
                               int32_t* __restrict__ s_patch, int32_t* __restrict__ s_depth,
                               uint32_t* __restrict__ base) {
  const uint32_t n = npdev[1];
  GRID_STRIDE(p, n) {
    pstruct[p] = (int32_t)p;
    s_host[p] = -1;
    s_level[p] = 1;
    s_patch[p] = (int32_t)p;
    s_depth[p] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) base[1] = n;
}

// the main branch of every parent: the largest (count, -id) among its children
__global__ void k_struct_best(int L, const uint32_t* __restrict__ npdev,
                              const int32_t* __restrict__ parent,
                              const uint64_t* __restrict__ npart,
                              unsigned long long* __restrict__ best) {
  const uint32_t n = npdev[L];
  GRID_STRIDE(p, n)
    atomicMax(&best[parent[p]], (unsigned long long)(npart[p] << 32) | (0xffffffffull - p));
}

// start flags over the bound nE (0 past the level's patch count)
__global__ void k_struct_split(int L, uint64_t nE, const uint32_t* __restrict__ npdev,
                               const int32_t* __restrict__ parent,
                               const unsigned long long* __restrict__ best,
                               uint8_t* __restrict__ start) {
  const uint32_t n = npdev[L];
  GRID_STRIDE(p, nE)
    start[p] = (p < n && (best[parent[p]] & 0xffffffffull) != 0xffffffffull - p) ? 1 : 0;
}

__global__ void k_struct_assign(int L, const uint32_t* __restrict__ npdev,
                                const int32_t* __restrict__ parent,
                                const uint8_t* __restrict__ start,
                                const uint32_t* __restrict__ rank,
                                const uint32_t* __restrict__ nstart,
                                const int32_t* __restrict__ ppstruct,
                                int32_t* __restrict__ pstruct, int32_t* __restrict__ s_host,
                                int32_t* __restrict__ s_level, int32_t* __restrict__ s_patch,
                                int32_t* __restrict__ s_depth, uint32_t* __restrict__ base) {
  const uint32_t n = npdev[L];
  const uint32_t b = base[L - 1];
  GRID_STRIDE(p, n) {
    const int32_t up = ppstruct[parent[p]];
    if (start[p]) {
      const uint32_t sid = b + rank[p];
      pstruct[p] = (int32_t)sid;
      s_host[sid] = up;
      s_level[sid] = L;
      s_patch[sid] = (int32_t)p;
      s_depth[sid] = s_depth[up] + 1;  // up < b: written on a coarser level
    } else {
      pstruct[p] = up;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) base[L] = b + *nstart;
}

// enqueues the classification of every level (counts stay on the device;
// arrays are sized by the label pass's bounds)
void classify_levels(Ctx* ctx, Ws& ws, Hier* h, hipStream_t st) {
  const size_t nlev = h->lev.size();
  if (nlev < 2) return;
  uint64_t bound = 0;
  for (size_t L = 1; L < nlev; ++L) bound += std::max<uint64_t>(h->lev[L - 1].nF, 1);
  h->s_host = h->mem.get<int32_t>(bound);
  h->s_level = h->mem.get<int32_t>(bound);
  h->s_patch = h->mem.get<int32_t>(bound);
  h->s_depth = h->mem.get<int32_t>(bound);
  h->cls_base = h->mem.get<uint32_t>(kMaxLevels + 1);
  HIP_CHECK(hipMemsetAsync(h->cls_base, 0, (kMaxLevels + 1) * sizeof(uint32_t), st));
  for (size_t L = 1; L < nlev; ++L) {
    const uint64_t nE = std::max<uint64_t>(h->lev[L - 1].nF, 1);  // bound on the patches of L
    h->lev[L].patch_struct = h->mem.get<int32_t>(nE);
  }
  k_struct_roots<<<grid_for(h->lev[0].nF), kT, 0, st>>>(
      h->npatch_dev, h->lev[1].patch_struct, h->s_host, h->s_level, h->s_patch, h->s_depth,
      h->cls_base);
  HIP_LAUNCH_CHECK();
  for (size_t L = 2; L < nlev; ++L) {
    const uint64_t nE = std::max<uint64_t>(h->lev[L - 1].nF, 1);
    const uint64_t nEp = std::max<uint64_t>(h->lev[L - 2].nF, 1);  // patches of level L-1
    Ws::Mark m = ws.mark();
    unsigned long long* best = ws.get<unsigned long long>(nEp);
    uint8_t* start = ws.get<uint8_t>(nE);
    uint32_t* rank = ws.get<uint32_t>(nE);
    uint32_t* nstart = ws.get<uint32_t>(1);
    HIP_CHECK(hipMemsetAsync(best, 0, nEp * sizeof(unsigned long long), st));
    k_struct_best<<<grid_for(nE), kT, 0, st>>>((int)L, h->npatch_dev, h->lev[L].patch_parent,
                                                h->lev[L].patch_npart, best);
    HIP_LAUNCH_CHECK();
    k_struct_split<<<grid_for(nE), kT, 0, st>>>((int)L, nE, h->npatch_dev,
                                                 h->lev[L].patch_parent, best, start);
    HIP_LAUNCH_CHECK();
    compact_flags(ws, start, nE, nullptr, rank, nstart, st);
    k_struct_assign<<<grid_for(nE), kT, 0, st>>>(
        (int)L, h->npatch_dev, h->lev[L].patch_parent, start, rank, nstart,
        h->lev[L - 1].patch_struct, h->lev[L].patch_struct, h->s_host, h->s_level, h->s_patch,
        h->s_depth, h->cls_base);
    HIP_LAUNCH_CHECK();
    ws.release(m);
  }
}

// after the stream has passed classify_levels: the number of structures
void finish_classify(Ctx* ctx, Hier* h, hipStream_t st) {
  (void)ctx;
  const size_t nlev = h->lev.size();
  uint32_t nst = 0;
  if (nlev >= 2) {
    HIP_CHECK(hipMemcpyAsync(&nst, h->cls_base + (nlev - 1), sizeof(uint32_t),
                             hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
  }
  h->nStruct = nst;
  h->classified = true;
}

void classify_hierarchy(Ctx* ctx, Ws& ws, Hier* h, hipStream_t st) {
  if (h->classified) return;
  if (!h->labelled) throw Error{AHF_EINVAL, "the hierarchy is not labelled"};
  classify_levels(ctx, ws, h, st);
  finish_classify(ctx, h, st);
}

}  // namespace ahf

extern "C" ahf_status ahf_hierarchy_query_label_static(const ahf_hierarchy* h, uint32_t level,
                                                       uint64_t n, const uint64_t* keys,
                                                       int32_t* out, void* stream) {
  using namespace ahf;
  auto fail = [](ahf_status c, const char* m) {
    set_last_error(m);
    return c;
  };
  if (!h || (n && (!keys || !out))) return fail(AHF_EINVAL, "bad arguments");
  if (level >= h->h.lev.size()) return fail(AHF_EINVAL, "level out of range");
  if (level >= 1 && !h->h.labelled) return fail(AHF_EINVAL, "the hierarchy is not labelled");
  if (n > kStaticQueryMax)
    return fail(AHF_ELIMIT, "more keys than the static staging area holds (262144 per call)");
  const uint32_t b = h->h.lev[level].b;
  for (uint64_t i = 0; i < n; ++i)
    if (3 * b < 64 && (keys[i] >> (3 * b)) != 0) return fail(AHF_EINVAL, "key beyond the level's bits");
  if (n == 0) return AHF_OK;
  if (level == 0) {
    for (uint64_t i = 0; i < n; ++i) out[i] = -1;
    return AHF_OK;
  }
  try {
    HIP_CHECK(hipSetDevice(h->h.ctx->device));
    query_labels_static(&h->h, (int)level, n, keys, out, (hipStream_t)stream);
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  }
  return AHF_OK;
}
