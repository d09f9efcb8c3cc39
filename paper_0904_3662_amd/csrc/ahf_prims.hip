// ahf_prims.hip -- device-wide primitives: exclusive scan, stable LSD radix
// sort of (uint64 key, uint32 value) pairs, deterministic FP64 reductions.
//
// All of them are deterministic: integer work is exact and every floating
// point sum is taken in a fixed order that depends only on the input size.
#include "ahf_internal.h"

namespace ahf {

// ------------------------------------------------------------------ block scan

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(v, d, 64);
    if (lane >= (uint32_t)d) v += t;
  }
  return v;
}

// exclusive scan across a block of NT threads; lds needs NT/64 + 1 words
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t& total, uint32_t* lds) {
  const uint32_t inc = wave_incl_scan(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) lds[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
      const uint32_t t = lds[i];
      lds[i] = s;
      s += t;
    }
    lds[NT / 64] = s;
  }
  __syncthreads();
  const uint32_t r = inc - v + lds[w];
  total = lds[NT / 64];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ compaction
//
// Positions of the nonzero bytes of a flag array, in index order, by
// reduce-then-scan over tiles of 8192 flags: count per tile, exclusive scan
// of the tile counts in one block, then each tile re-reads its flags and
// writes the index of every flagged element at its rank (list) and/or its
// rank at its index (rank).  One tile needs no count pass, and up to 8 tiles
// go through one block in one launch.

constexpr int kCfT = 256;
constexpr int kCfPer = 32;                 // flags per thread
constexpr int kCfTile = kCfT * kCfPer;     // 8192
constexpr int kCfMidT = 1024;
constexpr uint64_t kCfSumTiles = 2048;     // up to here a tile sums the counts before it

// the 32 flags of thread t of a tile, one bit each
__device__ inline uint32_t cf_bits(const uint8_t* __restrict__ flags, uint64_t n, uint64_t i0) {
  uint32_t m = 0;
  if (i0 + kCfPer <= n) {
    const uint4* p = reinterpret_cast<const uint4*>(flags + i0);
    const uint4 a = p[0], b = p[1];
    const uint32_t wds[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if ((wds[k] >> (8 * j)) & 255u) m |= 1u << (4 * k + j);
  } else {
    for (int k = 0; k < kCfPer; ++k)
      if (i0 + k < n && flags[i0 + k]) m |= 1u << k;
  }
  return m;
}

__global__ __launch_bounds__(kCfT) void k_cf_up(const uint8_t* __restrict__ flags, Cnt nc,
                                               uint32_t* __restrict__ tcnt) {
  __shared__ uint32_t lds[kCfT / 64 + 1];
  const uint64_t n = cnt_of(nc);
  const uint64_t i0 = (uint64_t)blockIdx.x * kCfTile + (uint64_t)threadIdx.x * kCfPer;
  const uint32_t c = (uint32_t)__popc(cf_bits(flags, n, i0));
  uint32_t tot;
  block_excl_scan<kCfT>(c, tot, lds);
  if (threadIdx.x == 0) tcnt[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kCfMidT) void k_cf_mid(const uint32_t* __restrict__ tcnt,
                                                    uint32_t ntiles, uint32_t* __restrict__ tofs) {
  __shared__ uint32_t lds[kCfMidT / 64 + 1];
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < ntiles; c0 += kCfMidT) {
    const uint32_t t = c0 + threadIdx.x;
    const uint32_t v = (t < ntiles) ? tcnt[t] : 0u;
    uint32_t tot;
    const uint32_t e = block_excl_scan<kCfMidT>(v, tot, lds);
    if (t < ntiles) tofs[t] = carry + e;
    carry += tot;
  }
}

// Writes one tile's part of the list and/or ranks, given the tile's flag bits
// per thread (m), its first flag t0 and its offset base; returns the tile's
// count.  The list goes out through LDS, one contiguous run per tile; a
// thread with any flag set writes the ranks of its 32 flags as one 128-byte
// run (all ones where the flag is clear).
__device__ inline uint32_t cf_tile(uint32_t m, uint64_t n, uint64_t t0, uint32_t base,
                                   uint32_t* __restrict__ list, uint32_t* __restrict__ rank,
                                   uint32_t* stage, uint32_t* lds) {
  const uint64_t i0 = t0 + (uint64_t)threadIdx.x * kCfPer;
  uint32_t tot;
  const uint32_t lpos = block_excl_scan<kCfT>((uint32_t)__popc(m), tot, lds);
  if (list) {
    uint32_t mm = m, p = lpos;
    while (mm) {
      const int k = __ffs(mm) - 1;
      mm &= mm - 1u;
      stage[p++] = (uint32_t)(i0 + k);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < tot; j += kCfT) list[base + j] = stage[j];
  }
  if (rank && m) {
    uint32_t r[kCfPer];
    uint32_t p = base + lpos;
#pragma unroll
    for (int k = 0; k < kCfPer; ++k) r[k] = ((m >> k) & 1u) ? p++ : 0xffffffffu;
    if (i0 + kCfPer <= n) {
      uint4* o = reinterpret_cast<uint4*>(rank + i0);
#pragma unroll
      for (int k = 0; k < kCfPer / 4; ++k)
        o[k] = make_uint4(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3]);
    } else {
#pragma unroll
      for (int k = 0; k < kCfPer; ++k)
        if (i0 + k < n) rank[i0 + k] = r[k];
    }
  }
  return tot;
}

// tile offset: from the scanned tile counts (tofs), or summed here from the
// tile counts of the tiles before this one (tcnt, few tiles), or 0 (one tile)
__global__ __launch_bounds__(kCfT) void k_cf_down(const uint8_t* __restrict__ flags, Cnt nc,
                                                 const uint32_t* __restrict__ tcnt,
                                                 const uint32_t* __restrict__ tofs,
                                                 uint32_t* __restrict__ list,
                                                 uint32_t* __restrict__ rank,
                                                 uint32_t* __restrict__ count) {
  __shared__ uint32_t lds[kCfT / 64 + 1];
  __shared__ uint32_t stage[kCfTile];
  const uint64_t n = cnt_of(nc);
  const uint64_t t0 = (uint64_t)blockIdx.x * kCfTile;
  uint32_t before = 0;
  if (!tofs && tcnt)
    for (uint32_t t = threadIdx.x; t < blockIdx.x; t += kCfT) before += tcnt[t];
  const uint32_t m = cf_bits(flags, n, t0 + (uint64_t)threadIdx.x * kCfPer);
  uint32_t tb = 0;
  if (!tofs && tcnt) block_excl_scan<kCfT>(before, tb, lds);
  const uint32_t base = tofs ? tofs[blockIdx.x] : (tcnt ? tb : 0u);
  const uint32_t tot = cf_tile(m, n, t0, base, list, rank, stage, lds);
  if (count && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *count = base + tot;
}

// a few tiles (2 .. kCfSmallTiles) in one block: every tile's flags are
// loaded first, then the tiles are written in order with a running offset
constexpr int kCfSmallTiles = 8;

__global__ __launch_bounds__(kCfT) void k_cf_small(const uint8_t* __restrict__ flags, Cnt nc,
                                                  uint32_t* __restrict__ list,
                                                  uint32_t* __restrict__ rank,
                                                  uint32_t* __restrict__ count) {
  __shared__ uint32_t lds[kCfT / 64 + 1];
  __shared__ uint32_t stage[kCfTile];
  const uint64_t n = cnt_of(nc);
  uint32_t m[kCfSmallTiles];
#pragma unroll
  for (int t = 0; t < kCfSmallTiles; ++t) {
    const uint64_t t0 = (uint64_t)t * kCfTile;
    m[t] = t0 < n ? cf_bits(flags, n, t0 + (uint64_t)threadIdx.x * kCfPer) : 0u;
  }
  uint32_t carry = 0;
#pragma unroll
  for (int t = 0; t < kCfSmallTiles; ++t) {
    const uint64_t t0 = (uint64_t)t * kCfTile;
    if (t0 >= n) break;  // uniform
    carry += cf_tile(m[t], n, t0, carry, list, rank, stage, lds);
  }
  if (count && threadIdx.x == 0) *count = carry;
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

void compact_flags(Ws& ws, const uint8_t* flags, uint64_t n, uint32_t* list, uint32_t* rank,
                   uint32_t* count, hipStream_t st) {
  compact_flags(ws, flags, host_cnt(n), list, rank, count, st);
}

// the number of flags may be known on the device only (nc.p): the tiles are
// laid out for the bound nc.cap, and tiles past the true count hold no flag
void compact_flags(Ws& ws, const uint8_t* flags, Cnt nc, uint32_t* list, uint32_t* rank,
                   uint32_t* count, hipStream_t st) {
  const uint64_t n = nc.cap;
  const uint64_t ntiles = (n + kCfTile - 1) / kCfTile;
  if (ntiles == 0) {
    // a kernel, not a memset: it may be recorded into a graph
    k_set_u32<<<1, 64, 0, st>>>(count, 0u);
    HIP_LAUNCH_CHECK();
    return;
  }
  if (ntiles > 1 && ntiles <= (uint64_t)kCfSmallTiles) {
    k_cf_small<<<1, kCfT, 0, st>>>(flags, nc, list, rank, count);
    HIP_LAUNCH_CHECK();
    return;
  }
  uint32_t* tcnt = nullptr;
  uint32_t* tofs = nullptr;
  if (ntiles > 1) {
    tcnt = ws.get<uint32_t>(ntiles);
    k_cf_up<<<(unsigned)ntiles, kCfT, 0, st>>>(flags, nc, tcnt);
    HIP_LAUNCH_CHECK();
    if (ntiles > kCfSumTiles) {
      // many tiles: scan the counts once instead of summing them per tile
      tofs = ws.get<uint32_t>(ntiles);
      k_cf_mid<<<1, kCfMidT, 0, st>>>(tcnt, (uint32_t)ntiles, tofs);
      HIP_LAUNCH_CHECK();
    }
  }
  k_cf_down<<<(unsigned)ntiles, kCfT, 0, st>>>(flags, nc, tcnt, tofs, list, rank, count);
  HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ radix sort
//
// Stable LSD sort of Morton keys with the particle index as tie-break, 8-bit
// digits.  Every pass is reduce-then-scan, with no waits between tiles:
//   k_rs_up    per tile of 4096 elements, the histogram of the pass digit;
//   k_rs_tscan per digit, the exclusive prefix over tiles plus the digit's
//              global offset (global digit histograms come from the kernel
//              that makes the keys);
//   k_rs_down  ranks the tile (4 waves of 1024 consecutive elements, 64 at a
//              time with ballot-based digit matching, so a rank counts only
//              elements before it: stable), stages it in LDS by digit and
//              writes each digit run to its place.
// The first passes move (key, index) pairs.  Once the key bits still to be
// sorted fit beside the index in 64 bits, a pass writes one packed word
// ((key >> 8q) << ib) | index and the remaining passes move 8 bytes per
// element instead of 12.  The sorted keys themselves are rebuilt from the
// particle coordinates by the consumer.

constexpr int kRsT = 256;
constexpr int kRsW = kRsT / 64;
constexpr int kRsR = 16;                 // rounds of 64 per wave
constexpr int kRsTile = kRsT * kRsR;     // 4096

SortPlan sort_plan(uint64_t n, int key_bits) {
  SortPlan sp;
  int ib = 1;
  while (ib < 32 && (1ull << ib) < n) ++ib;
  sp.ib = ib;
  sp.key_bits = key_bits;
  sp.npass = (key_bits + 7) / 8;
  int q = 0;
  while (key_bits - 8 * q > 64 - ib) ++q;
  sp.q = q;
  return sp;
}

__global__ void k_rs_offsets(const uint32_t* __restrict__ ghist, int npass,
                             uint32_t* __restrict__ gofs) {
  __shared__ uint32_t lds[kRsT / 64 + 1];
  for (int p = 0; p < npass; ++p) {
    uint32_t tot;
    const uint32_t v = ghist[p * 256 + threadIdx.x];
    gofs[p * 256 + threadIdx.x] = block_excl_scan<kRsT>(v, tot, lds);
  }
}

// digit histogram of every tile: th[d * ntiles + tile]
__global__ __launch_bounds__(kRsT) void k_rs_up(const uint64_t* __restrict__ in, uint64_t n,
                                               int shift, uint32_t ntiles,
                                               uint32_t* __restrict__ th) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t tile = xcd_tile(blockIdx.x, ntiles);
  const uint64_t tile0 = (uint64_t)tile * kRsTile;
  uint64_t key[kRsR];
#pragma unroll
  for (int r = 0; r < kRsR; ++r) {
    const uint64_t j = tile0 + (uint64_t)r * kRsT + threadIdx.x;
    key[r] = (j < n) ? __builtin_nontemporal_load(in + j) : 0ull;
  }
#pragma unroll
  for (int r = 0; r < kRsR; ++r) {
    const uint64_t j = tile0 + (uint64_t)r * kRsT + threadIdx.x;
    if (j < n) atomicAdd(&h[(uint32_t)(key[r] >> shift) & 255u], 1u);
  }
  __syncthreads();
  th[(uint64_t)threadIdx.x * ntiles + tile] = h[threadIdx.x];
}

constexpr int kTsT = 1024;

// one block per digit: tofs[d * ntiles + t] = gofs[d] + sum of th[d * ntiles + t'] over t' < t
__global__ __launch_bounds__(kTsT) void k_rs_tscan(const uint32_t* __restrict__ th,
                                                   uint32_t ntiles,
                                                   const uint32_t* __restrict__ gofs,
                                                   uint32_t* __restrict__ tofs) {
  __shared__ uint32_t lds[kTsT / 64 + 1];
  const uint32_t d = blockIdx.x;
  const uint32_t* row = th + (uint64_t)d * ntiles;
  uint32_t* orow = tofs + (uint64_t)d * ntiles;
  uint32_t carry = gofs[d];
  for (uint32_t c0 = 0; c0 < ntiles; c0 += kTsT * 4) {
    uint32_t v[4];
    const uint32_t a = c0 + threadIdx.x * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (a + k < ntiles) ? row[a + k] : 0u;
    const uint32_t s = (v[0] + v[1]) + (v[2] + v[3]);
    uint32_t tot;
    uint32_t e = block_excl_scan<kTsT>(s, tot, lds) + carry;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (a + k < ntiles) orow[a + k] = e;
      e += v[k];
    }
    carry += tot;
  }
}

enum RsIn { kInKeyIota = 0, kInKeyVal = 1, kInWord = 2 };
enum RsOut { kOutKeyVal = 0, kOutWord = 1 };

// One pass over one tile.  IN: (key, index) with the index implied by the
// position (first pass), (key, index) pairs, or packed words.  OUT: pairs, or
// packed words ((key >> pk_shift) << ib) | index.
template <int IN, int OUT>
__global__ __launch_bounds__(kRsT) void k_rs_down(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, uint64_t n, int shift,
    int pk_shift, int ib, uint32_t ntiles, const uint32_t* __restrict__ tofs) {
  constexpr bool kPack = OUT == kOutWord && IN != kInWord;
  __shared__ uint64_t sk[kRsTile];
  __shared__ uint8_t sdig[kPack ? kRsTile : 1];  // a packed word no longer holds this digit
  __shared__ uint32_t cnt[kRsW][256];
  __shared__ uint32_t doff[256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t lds[kRsT / 64 + 1];
  const int w = threadIdx.x >> 6;
  const uint32_t lane = __lane_id();
  const uint32_t tile = xcd_tile(blockIdx.x, ntiles);
  const uint32_t base_off = tofs[(uint64_t)threadIdx.x * ntiles + tile];
  for (int i = threadIdx.x; i < kRsW * 256; i += kRsT) (&cnt[0][0])[i] = 0u;
  __syncthreads();
  const uint64_t tile0 = (uint64_t)tile * kRsTile;
  const uint64_t wbase = tile0 + (uint64_t)w * (kRsR * 64);
  uint64_t key[kRsR];
  uint32_t val[kRsR];
  uint32_t rk[kRsR];
  // every load of the tile is issued before the first use
#pragma unroll
  for (int r = 0; r < kRsR; ++r) {
    const uint64_t j = wbase + (uint64_t)r * 64 + lane;
    key[r] = (j < n) ? __builtin_nontemporal_load(kin + j) : 0ull;
    if (IN == kInKeyVal) val[r] = (j < n) ? __builtin_nontemporal_load(vin + j) : 0u;
    if (IN == kInKeyIota) val[r] = (uint32_t)j;
  }
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < kRsR; ++r) {
    const uint64_t j = wbase + (uint64_t)r * 64 + lane;
    const bool valid = j < n;
    const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
    uint64_t peer = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bm = __ballot(on);
      peer &= on ? bm : ~bm;
    }
    const uint32_t before = cnt[w][d];
    const uint32_t mine = (uint32_t)__popcll(peer & lt);
    if (valid && (peer & lt) == 0ull) cnt[w][d] = before + (uint32_t)__popcll(peer);
    rk[r] = valid ? before + mine : 0xffffffffu;
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int ww = 0; ww < kRsW; ++ww) {
      const uint32_t t = cnt[ww][d];
      cnt[ww][d] = s;
      s += t;
    }
    uint32_t tot;
    doff[d] = block_excl_scan<kRsT>(s, tot, lds);
    gbase[d] = base_off;
  }
  __syncthreads();
  const uint32_t tn = (uint32_t)((n - tile0) < (uint64_t)kRsTile ? (n - tile0) : (uint64_t)kRsTile);
  // keys (or packed words) through LDS in digit order, then out
#pragma unroll
  for (int r = 0; r < kRsR; ++r) {
    if (rk[r] != 0xffffffffu) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
      const uint32_t pos = doff[d] + cnt[w][d] + rk[r];
      if (kPack) {
        sk[pos] = ((key[r] >> pk_shift) << ib) | (uint64_t)val[r];
        sdig[pos] = (uint8_t)d;
      } else {
        sk[pos] = key[r];
      }
      rk[r] = pos;
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < tn; i += kRsT) {
    const uint64_t k = sk[i];
    const uint32_t d = kPack ? (uint32_t)sdig[i] : (uint32_t)(k >> shift) & 255u;
    kout[(uint64_t)gbase[d] + (i - doff[d])] = k;
  }
  if (OUT == kOutKeyVal) {
    // the indices, through the same LDS with the digit beside each
    __syncthreads();
    uint32_t* sv = reinterpret_cast<uint32_t*>(sk);
    uint8_t* sd = reinterpret_cast<uint8_t*>(sk) + 4 * kRsTile;
#pragma unroll
    for (int r = 0; r < kRsR; ++r) {
      if (rk[r] != 0xffffffffu) {
        sv[rk[r]] = val[r];
        sd[rk[r]] = (uint8_t)((uint32_t)(key[r] >> shift) & 255u);
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < tn; i += kRsT) {
      const uint32_t d = sd[i];
      vout[(uint64_t)gbase[d] + (i - doff[d])] = sv[i];
    }
  }
}

uint64_t* sort_keys(Ctx* ctx, Ws& ws, uint64_t* keys, uint64_t n, const SortPlan& sp,
                    const uint32_t* ghist, hipStream_t st, uint64_t** spare) {
  if (spare) *spare = nullptr;
  if (n == 0) return keys;
  const uint32_t ntiles = (uint32_t)((n + kRsTile - 1) / kRsTile);
  uint32_t* gofs = ws.get<uint32_t>((uint64_t)sp.npass * 256);
  uint32_t* th = ws.get<uint32_t>((uint64_t)ntiles * 256);
  uint32_t* tofs = ws.get<uint32_t>((uint64_t)ntiles * 256);
  uint64_t* kt = ws.get<uint64_t>(n);
  uint32_t* va = (sp.q >= 2) ? ws.get<uint32_t>(n) : nullptr;
  uint32_t* vb = (sp.q >= 3) ? ws.get<uint32_t>(n) : nullptr;
  k_rs_offsets<<<1, kRsT, 0, st>>>(ghist, sp.npass, gofs);
  HIP_LAUNCH_CHECK();
  uint64_t* a = keys;
  uint64_t* b = kt;
  uint32_t* vin = nullptr;
  for (int p = 0; p < sp.npass; ++p) {
    // pass p sorts key bits [8p, 8p + 8): in a packed word they sit above the index
    const bool word_in = p >= sp.q;
    const int shift = word_in ? sp.ib + 8 * (p - sp.q) : 8 * p;
    AHF_TIMED(ctx, "rs_up", st, (k_rs_up<<<ntiles, kRsT, 0, st>>>(a, n, shift, ntiles, th)));
    AHF_TIMED(ctx, "rs_tscan", st,
              (k_rs_tscan<<<256, kTsT, 0, st>>>(th, ntiles, gofs + p * 256, tofs)));
    uint32_t* vout = (vin == va) ? vb : va;
    if (word_in) {
      AHF_TIMED(ctx, "rs_scatter", st,
                (k_rs_down<kInWord, kOutWord><<<ntiles, kRsT, 0, st>>>(
                    a, nullptr, b, nullptr, n, shift, 0, sp.ib, ntiles, tofs)));
    } else if (p == sp.q - 1) {
      if (p == 0)
        AHF_TIMED(ctx, "rs_scatter", st,
                  (k_rs_down<kInKeyIota, kOutWord><<<ntiles, kRsT, 0, st>>>(
                      a, nullptr, b, nullptr, n, shift, 8 * sp.q, sp.ib, ntiles, tofs)));
      else
        AHF_TIMED(ctx, "rs_scatter", st,
                  (k_rs_down<kInKeyVal, kOutWord><<<ntiles, kRsT, 0, st>>>(
                      a, vin, b, nullptr, n, shift, 8 * sp.q, sp.ib, ntiles, tofs)));
    } else {
      if (p == 0)
        AHF_TIMED(ctx, "rs_scatter", st,
                  (k_rs_down<kInKeyIota, kOutKeyVal><<<ntiles, kRsT, 0, st>>>(
                      a, nullptr, b, vout, n, shift, 0, sp.ib, ntiles, tofs)));
      else
        AHF_TIMED(ctx, "rs_scatter", st,
                  (k_rs_down<kInKeyVal, kOutKeyVal><<<ntiles, kRsT, 0, st>>>(
                      a, vin, b, vout, n, shift, 0, sp.ib, ntiles, tofs)));
      vin = vout;
    }
    std::swap(a, b);
  }
  if (spare) *spare = b;
  return a;
}

// ------------------------------------------------------------------ reductions

constexpr int kRedT = 256;
constexpr int kRedBlocks = 512;

__device__ inline double block_sum_f64(double v, double* lds) {
  // fixed butterfly inside each wave, then waves in index order
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
  }
  __syncthreads();
  return s;  // valid in thread 0
}

template <typename T>
__global__ __launch_bounds__(kRedT) void k_sum_partial(const T* __restrict__ a, uint64_t n,
                                                       double* __restrict__ part) {
  __shared__ double lds[kRedT / 64];
  double s = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * kRedT + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kRedT)
    s += (double)a[i];
  s = block_sum_f64(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedT) void k_sum_final(const double* __restrict__ part, int np,
                                                     double* __restrict__ out) {
  __shared__ double lds[kRedT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kRedT) s += part[i];
  s = block_sum_f64(s, lds);
  if (threadIdx.x == 0) *out = s;
}

template <typename T>
void sum_to_f64(Ws& ws, const T* a, uint64_t n, double* out, hipStream_t st) {
  int nb = (int)((n + kRedT - 1) / kRedT);
  if (nb > kRedBlocks) nb = kRedBlocks;
  if (nb < 1) nb = 1;
  double* part = ws.get<double>(nb);
  k_sum_partial<T><<<nb, kRedT, 0, st>>>(a, n, part);
  HIP_LAUNCH_CHECK();
  k_sum_final<<<1, kRedT, 0, st>>>(part, nb, out);
  HIP_LAUNCH_CHECK();
}

template void sum_to_f64<float>(Ws&, const float*, uint64_t, double*, hipStream_t);
template void sum_to_f64<double>(Ws&, const double*, uint64_t, double*, hipStream_t);
template void sum_to_f64<uint32_t>(Ws&, const uint32_t*, uint64_t, double*, hipStream_t);

}  // namespace ahf
