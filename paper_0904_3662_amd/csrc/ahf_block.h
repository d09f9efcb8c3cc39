// ahf_block.h -- workgroup-wide primitives of 256 threads (4 waves of 64):
// fixed-order sums, scans and extrema, and a stable LSD radix sort of a
// segment held in global memory.  Every thread of the workgroup calls them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ahf {

constexpr int kBT = 256;        // threads of the workgroups that use these
constexpr int kBW = kBT / 64;   // their waves
static_assert(kBT == 256, "the radix sort ranks one 8-bit digit per thread");

__device__ inline uint64_t lanes_below() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// sum over the workgroup in a fixed order (wave butterflies, then waves in order)
__device__ inline double block_sum(double x, double* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < kBW; ++i) t += red[i];
  return t;
}

__device__ inline uint64_t block_or(uint64_t x, uint64_t* red) {
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = x;
  __syncthreads();
  uint64_t t = 0;
  for (int i = 0; i < kBW; ++i) t |= red[i];
  return t;
}

__device__ inline uint64_t block_and(uint64_t x, uint64_t* red) {
  for (int o = 32; o > 0; o >>= 1) x &= __shfl_xor(x, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = x;
  __syncthreads();
  uint64_t t = ~0ull;
  for (int i = 0; i < kBW; ++i) t &= red[i];
  return t;
}

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
  for (int i = 1; i < kBW; ++i) t = red[i] > t ? red[i] : t;
  return t;
}

// inclusive scan of one value per thread over the workgroup, in thread
// order; returns the thread's prefix and sets *total
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
  for (int i = 0; i < kBW; ++i) {
    if (i < w) before += red[i];
    all += red[i];
  }
  *total = all;
  return before + x;
}

// Stable LSD radix sort of n (key, val) pairs of a segment: the pairs are in
// (ka, va); kb, vb are as large.  Digits of 8 bits; a digit that every key
// shares is skipped.  Returns true when the result is in (kb, vb).
template <class K>
__device__ bool block_sort(K* ka, uint32_t* va, K* kb, uint32_t* vb, uint32_t n) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kBW][256];
  __shared__ uint64_t red[kBW];
  uint64_t o = 0, a = ~0ull;
  for (uint32_t i = threadIdx.x; i < n; i += kBT) {
    o |= (uint64_t)ka[i];
    a &= (uint64_t)ka[i];
  }
  const uint64_t any = block_or(o, red);
  const uint64_t all = block_and(a, red);
  const uint64_t vary = any ^ all;
  bool flipped = false;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  for (int p = 0; p < (int)sizeof(K); ++p) {
    if (((vary >> (8 * p)) & 255u) == 0) continue;  // same digit everywhere
    K* src = flipped ? kb : ka;
    uint32_t* sv = flipped ? vb : va;
    K* dst = flipped ? ka : kb;
    uint32_t* dv = flipped ? va : vb;
    // digit counts, then each digit's first slot
    hist[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += kBT)
      atomicAdd(&hist[((uint64_t)src[i] >> (8 * p)) & 255u], 1u);
    __syncthreads();
    {
      const uint32_t c = hist[threadIdx.x];
      uint32_t x = c;
      for (int s = 1; s < 64; s <<= 1) {
        const uint32_t y = __shfl_up(x, s);
        if (lane >= s) x += y;
      }
      __shared__ uint32_t wt[kBW];
      if (lane == 63) wt[w] = x;
      __syncthreads();
      uint32_t before = 0;
      for (int i = 0; i < w; ++i) before += wt[i];
      run[threadIdx.x] = before + x - c;  // exclusive: the digit's first slot
    }
    __syncthreads();
    // chunks of kBT in order; within a chunk, ranks by thread order
    for (uint32_t c0 = 0; c0 < n; c0 += kBT) {
      const uint32_t i = c0 + threadIdx.x;
      const bool valid = i < n;
      K key = valid ? src[i] : K(0);
      const uint32_t val = valid ? sv[i] : 0u;
      const uint32_t d = (uint32_t)(((uint64_t)key >> (8 * p)) & 255u);
      // lanes of this wave with the same digit
      uint64_t peer = __ballot(valid);
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = (d >> bit) & 1u;
        const uint64_t bm = __ballot(on);
        peer &= on ? bm : ~bm;
      }
      for (int j = threadIdx.x; j < kBW * 256; j += kBT) (&wcnt[0][0])[j] = 0;
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
      {
        uint32_t t = 0;
        for (int k = 0; k < kBW; ++k) t += wcnt[k][threadIdx.x];
        run[threadIdx.x] += t;
      }
      __syncthreads();
    }
    flipped = !flipped;
  }
  return flipped;
}

}  // namespace ahf
