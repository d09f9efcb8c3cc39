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

// ------------------------------------------------------------------ scan

constexpr int kScanT = 256;
constexpr int kScanI = 8;
constexpr int kScanTile = kScanT * kScanI;

__global__ __launch_bounds__(kScanT) void k_scan_reduce(const uint32_t* __restrict__ in, uint64_t n,
                                                        uint32_t* __restrict__ bsum) {
  __shared__ uint32_t lds[kScanT / 64 + 1];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanI; ++i) {
    const uint64_t j = base + (uint64_t)i * kScanT + threadIdx.x;
    if (j < n) s += in[j];
  }
  uint32_t tot;
  block_excl_scan<kScanT>(s, tot, lds);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// blocked layout: thread t owns items [base + t*kScanI, base + t*kScanI + kScanI)
__global__ __launch_bounds__(kScanT) void k_scan_apply(const uint32_t* __restrict__ in,
                                                       uint32_t* __restrict__ out, uint64_t n,
                                                       const uint32_t* __restrict__ boff,
                                                       uint32_t* __restrict__ total_out) {
  __shared__ uint32_t lds[kScanT / 64 + 1];
  __shared__ uint32_t tile[kScanTile];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  // coalesced load into LDS
#pragma unroll
  for (int i = 0; i < kScanI; ++i) {
    const uint64_t j = base + (uint64_t)i * kScanT + threadIdx.x;
    tile[i * kScanT + threadIdx.x] = (j < n) ? in[j] : 0u;
  }
  __syncthreads();
  uint32_t v[kScanI];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanI; ++i) {
    v[i] = tile[threadIdx.x * kScanI + i];
    s += v[i];
  }
  uint32_t tot;
  uint32_t off = block_excl_scan<kScanT>(s, tot, lds);
  off += boff ? boff[blockIdx.x] : 0u;
#pragma unroll
  for (int i = 0; i < kScanI; ++i) {
    tile[threadIdx.x * kScanI + i] = off;
    off += v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanI; ++i) {
    const uint64_t j = base + (uint64_t)i * kScanT + threadIdx.x;
    if (j < n) out[j] = tile[i * kScanT + threadIdx.x];
  }
  if (total_out && boff == nullptr && threadIdx.x == 0) *total_out = tot;
}

void scan_u32(Ws& ws, const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total,
              hipStream_t st) {
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= 1) {
    k_scan_apply<<<1, kScanT, 0, st>>>(in, out, n, nullptr, total);
    HIP_LAUNCH_CHECK();
    return;
  }
  uint32_t* bsum = ws.get<uint32_t>(nb);
  k_scan_reduce<<<(unsigned)nb, kScanT, 0, st>>>(in, n, bsum);
  HIP_LAUNCH_CHECK();
  scan_u32(ws, bsum, bsum, nb, total, st);
  k_scan_apply<<<(unsigned)nb, kScanT, 0, st>>>(in, out, n, bsum, nullptr);
  HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ radix sort
//
// LSD, 8-bit digits, reduce-then-scan.  A tile of 4096 pairs is split over
// 4 waves of 1024 consecutive pairs; each wave ranks its pairs 64 at a time
// with ballot-based digit matching, so the rank of a pair counts only pairs
// before it in input order: the sort is stable.

constexpr int kRsT = 256;
constexpr int kRsW = kRsT / 64;
constexpr int kRsR = 16;                 // rounds of 64 per wave
constexpr int kRsTile = kRsT * kRsR;     // 4096

__global__ __launch_bounds__(kRsT) void k_rs_hist(const uint64_t* __restrict__ keys, uint64_t n,
                                                  int shift, uint32_t* __restrict__ ghist,
                                                  uint32_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
#pragma unroll 4
  for (int i = 0; i < kRsR; ++i) {
    const uint64_t j = base + (uint64_t)i * kRsT + threadIdx.x;
    if (j < n) atomicAdd(&h[(uint32_t)(keys[j] >> shift) & 255u], 1u);
  }
  __syncthreads();
  ghist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRsT) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                     const uint32_t* __restrict__ vin,
                                                     uint64_t* __restrict__ kout,
                                                     uint32_t* __restrict__ vout, uint64_t n,
                                                     int shift, const uint32_t* __restrict__ goff,
                                                     uint32_t ntiles) {
  __shared__ uint64_t sk[kRsTile];
  __shared__ uint32_t sv[kRsTile];
  __shared__ uint32_t cnt[kRsW][256];
  __shared__ uint32_t doff[256];
  __shared__ uint32_t lds[kRsT / 64 + 1];
  const int w = threadIdx.x >> 6;
  const uint32_t lane = __lane_id();
  for (int i = threadIdx.x; i < kRsW * 256; i += kRsT) (&cnt[0][0])[i] = 0u;
  __syncthreads();
  const uint64_t tile0 = (uint64_t)blockIdx.x * kRsTile;
  const uint64_t lt = lanemask_lt();
  uint64_t key[kRsR];
  uint32_t val[kRsR];
  uint32_t rk[kRsR];
#pragma unroll
  for (int r = 0; r < kRsR; ++r) {
    const uint64_t j = tile0 + (uint64_t)w * (kRsR * 64) + (uint64_t)r * 64 + lane;
    const bool valid = j < n;
    const uint64_t k = valid ? kin[j] : 0ull;
    const uint32_t v = valid ? vin[j] : 0u;
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
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
    key[r] = k;
    val[r] = v;
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
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRsR; ++r) {
    if (rk[r] != 0xffffffffu) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
      const uint32_t pos = doff[d] + cnt[w][d] + rk[r];
      sk[pos] = key[r];
      sv[pos] = val[r];
    }
  }
  __syncthreads();
  const uint32_t tn = (uint32_t)((n - tile0) < (uint64_t)kRsTile ? (n - tile0) : (uint64_t)kRsTile);
  for (uint32_t i = threadIdx.x; i < tn; i += kRsT) {
    const uint64_t k = sk[i];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    const uint64_t o = (uint64_t)goff[(uint64_t)d * ntiles + blockIdx.x] + (i - doff[d]);
    kout[o] = k;
    vout[o] = sv[i];
  }
}

// sorts by the low `bits` key bits; returns the buffers that hold the result
void sort_pairs(Ws& ws, uint64_t*& keys, uint32_t*& vals, uint64_t*& ktmp, uint32_t*& vtmp,
                uint64_t n, int bits, hipStream_t st) {
  if (n <= 1 || bits <= 0) return;
  const uint32_t ntiles = (uint32_t)((n + kRsTile - 1) / kRsTile);
  const uint64_t nh = (uint64_t)ntiles * 256;
  uint32_t* hist = ws.get<uint32_t>(nh);
  for (int shift = 0; shift < bits; shift += 8) {
    AHF_TIMED(ws.ctx(), "rs_hist", st,
              (k_rs_hist<<<ntiles, kRsT, 0, st>>>(keys, n, shift, hist, ntiles)));
    Ws::Mark m = ws.mark();
    scan_u32(ws, hist, hist, nh, nullptr, st);
    ws.release(m);
    AHF_TIMED(ws.ctx(), "rs_scatter", st,
              (k_rs_scatter<<<ntiles, kRsT, 0, st>>>(keys, vals, ktmp, vtmp, n, shift, hist, ntiles)));
    std::swap(keys, ktmp);
    std::swap(vals, vtmp);
  }
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
