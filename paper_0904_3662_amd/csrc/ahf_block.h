// ahf_block.h -- workgroup-wide primitives for workgroups of BT threads
// (BT a multiple of 256, 256 by default): fixed-order sums, scans and
// extrema, and a stable LSD radix sort of a segment held in global memory.
// Every thread of the workgroup calls them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ahf {

constexpr int kBT = 256;        // default threads of the workgroups that use these
constexpr int kBW = kBT / 64;   // their waves

__device__ inline uint64_t lanes_below() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// sum over the workgroup in a fixed order (wave butterflies, then waves in order)
template <int BT = kBT>
__device__ inline double block_sum(double x, double* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < BT / 64; ++i) t += red[i];
  return t;
}

template <int BT = kBT>
__device__ inline uint64_t block_or(uint64_t x, uint64_t* red) {
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = x;
  __syncthreads();
  uint64_t t = 0;
  for (int i = 0; i < BT / 64; ++i) t |= red[i];
  return t;
}

template <int BT = kBT>
__device__ inline uint64_t block_and(uint64_t x, uint64_t* red) {
  for (int o = 32; o > 0; o >>= 1) x &= __shfl_xor(x, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = x;
  __syncthreads();
  uint64_t t = ~0ull;
  for (int i = 0; i < BT / 64; ++i) t &= red[i];
  return t;
}

template <int BT = kBT>
__device__ inline int64_t block_max_i64(int64_t x, int64_t* red) {
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t y = __shfl_xor(x, o);
    x = y > x ? y : x;
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = x;
  __syncthreads();
  int64_t t = red[0];
  for (int i = 1; i < BT / 64; ++i) t = red[i] > t ? red[i] : t;
  return t;
}

// inclusive scan of one value per thread over the workgroup, in thread
// order; returns the thread's prefix and sets *total
template <int BT = kBT>
__device__ inline double block_scan(double x, double* red, double* total) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) red[w] = x;
  __syncthreads();
  double before = 0.0, all = 0.0;
  for (int i = 0; i < BT / 64; ++i) {
    if (i < w) before += red[i];
    all += red[i];
  }
  *total = all;
  return before + x;
}

// Stable LSD radix sort of n (key, val) pairs of a segment: the pairs are in
// (ka, va); kb, vb are as large.  Digits of 8 bits (the first 256 threads
// hold one digit's count each); a digit that every key shares is skipped.
// Returns true when the result is in (kb, vb).
template <class K, int BT = kBT>
__device__ bool block_sort(K* ka, uint32_t* va, K* kb, uint32_t* vb, uint32_t n) {
  static_assert(BT % 256 == 0, "a digit per thread of the first 256");
  constexpr int BW = BT / 64;
  __shared__ uint32_t hist[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[BW][256];
  __shared__ uint64_t red[BW];
  __shared__ uint32_t wt[4];
  uint64_t o = 0, a = ~0ull;
  for (uint32_t i = threadIdx.x; i < n; i += BT) {
    o |= (uint64_t)ka[i];
    a &= (uint64_t)ka[i];
  }
  const uint64_t any = block_or<BT>(o, red);
  const uint64_t all = block_and<BT>(a, red);
  const uint64_t vary = any ^ all;
  bool flipped = false;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const bool digit_thread = threadIdx.x < 256;
  for (int p = 0; p < (int)sizeof(K); ++p) {
    if (((vary >> (8 * p)) & 255u) == 0) continue;  // same digit everywhere
    K* src = flipped ? kb : ka;
    uint32_t* sv = flipped ? vb : va;
    K* dst = flipped ? ka : kb;
    uint32_t* dv = flipped ? va : vb;
    // digit counts, then each digit's first slot
    if (digit_thread) hist[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += 4 * BT) {
      K kk[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) kk[j] = (i0 + j * BT < n) ? src[i0 + j * BT] : K(0);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i0 + j * BT < n) atomicAdd(&hist[((uint64_t)kk[j] >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    {
      const uint32_t c = digit_thread ? hist[threadIdx.x] : 0u;
      uint32_t x = c;
      for (int s = 1; s < 64; s <<= 1) {
        const uint32_t y = __shfl_up(x, s);
        if (lane >= s) x += y;
      }
      if (digit_thread && lane == 63) wt[w] = x;
      __syncthreads();
      if (digit_thread) {
        uint32_t before = 0;
        for (int i = 0; i < w; ++i) before += wt[i];
        run[threadIdx.x] = before + x - c;  // exclusive: the digit's first slot
      }
    }
    __syncthreads();
    // chunks of BT in order; within a chunk, ranks by thread order (the
    // loads of four chunks go out together)
    for (uint32_t c4 = 0; c4 < n; c4 += 4 * BT) {
      K keyr[4];
      uint32_t valr[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t i = c4 + j * BT + threadIdx.x;
        keyr[j] = i < n ? src[i] : K(0);
        valr[j] = i < n ? sv[i] : 0u;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
      const uint32_t c0 = c4 + j * BT;
      if (c0 >= n) break;
      const uint32_t i = c0 + threadIdx.x;
      const bool valid = i < n;
      K key = keyr[j];
      const uint32_t val = valr[j];
      const uint32_t d = (uint32_t)(((uint64_t)key >> (8 * p)) & 255u);
      // lanes of this wave with the same digit
      uint64_t peer = __ballot(valid);
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = (d >> bit) & 1u;
        const uint64_t bm = __ballot(on);
        peer &= on ? bm : ~bm;
      }
      for (int j = threadIdx.x; j < BW * 256; j += BT) (&wcnt[0][0])[j] = 0;
      __syncthreads();
      const uint32_t rank = (uint32_t)__popcll(peer & lanes_below());
      if (valid && (peer & lanes_below()) == 0ull) wcnt[w][d] = (uint32_t)__popcll(peer);
      __syncthreads();
      if (valid) {
        uint32_t before = 0;
        for (int k = 0; k < w; ++k) before += wcnt[k][d];
        const uint32_t dest = run[d] + before + rank;
        dst[dest] = key;
        dv[dest] = val;
      }
      __syncthreads();
      if (digit_thread) {
        uint32_t t = 0;
        for (int k = 0; k < BW; ++k) t += wcnt[k][threadIdx.x];
        run[threadIdx.x] += t;
      }
      __syncthreads();
      }
    }
    flipped = !flipped;
  }
  return flipped;
}

}  // namespace ahf
