// ahf_dev.h -- device-side helpers of the hierarchy library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ahf {

constexpr int kQBits = 21;          // bits per axis of the quantized positions
constexpr int kMaxLevels = 22;      // levels 0..21
constexpr int kHeavy = 64;          // default: cells with more particles take the chunked path
constexpr int kHeavyMax = 64;       // largest light cell a thread may sum on its own
constexpr int kChunk = 1024;        // particles per chunk of a heavy cell (64 lanes x 16)

// device error flags (bit mask in a uint32 the host reads after the build)
constexpr uint32_t kErrCoord = 1u;     // a coordinate >= 2^21
constexpr uint32_t kErrLookup = 2u;    // a cell that must exist was not found
constexpr uint32_t kErrInternal = 4u;
constexpr uint32_t kErrCapacity = 8u;  // a planned level outgrew its capacity

// The number of elements a kernel works on: the host's bound `cap`, and,
// when the true count is only known on the device (a build whose levels are
// sized without waiting for the host), the count at p times mult, clamped
// to cap.  Without p the count is cap itself.
struct Cnt {
  const uint32_t* p;
  uint32_t mult;
  uint64_t cap;
};
__host__ __device__ inline Cnt host_cnt(uint64_t n) { return Cnt{nullptr, 1u, n}; }
__device__ inline uint64_t cnt_of(const Cnt& c) {
  if (!c.p) return c.cap;
  const uint64_t v = (uint64_t)(*c.p) * c.mult;
  return v < c.cap ? v : c.cap;
}

// 21-bit value -> every third bit of a 63-bit word (Morton spreading)
__host__ __device__ inline uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__host__ __device__ inline uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}

// Morton key: bit 3j+2 = x_j, bit 3j+1 = y_j, bit 3j = z_j
__host__ __device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

__host__ __device__ inline void unmorton3(uint64_t k, uint32_t& x, uint32_t& y, uint32_t& z) {
  x = compact3(k >> 2);
  y = compact3(k >> 1);
  z = compact3(k);
}

// One axis of a Morton key (its bits under mask m) moved by d in {-1, 0, 1},
// periodic, without leaving the interleaved form: +1 sets the other axes'
// bits so that the carry runs through them, -1 borrows through their zeros,
// and the mask drops what leaves the top.
__host__ __device__ inline uint64_t dilated_step(uint64_t k, uint64_t m, int d) {
  const uint64_t a = k & m;
  const uint64_t low = m & (~m + 1ull);
  const uint64_t b = d > 0 ? (((a | ~m) + low) & m) : (d < 0 ? ((a - low) & m) : a);
  return (k & ~m) | b;
}

// key of the cell displaced by (dx,dy,dz), each in {-1, 0, 1}, periodic on a
// grid of `bits` (<= 21) bits per axis
__host__ __device__ inline uint64_t shift_key(uint64_t k, int bits, int dx, int dy, int dz) {
  const uint64_t mz = 0x1249249249249249ull & ((1ull << (3 * bits)) - 1ull);
  k = dilated_step(k, mz << 2, dx);
  k = dilated_step(k, mz << 1, dy);
  return dilated_step(k, mz, dz);
}

// Per-level descent table: slot_child[l][s] is the brick (of level l+1) made
// of the children of slot s of level l, or -1.  Level-0 slots are level-0 keys.
struct Tree {
  const int32_t* slot_child[kMaxLevels];
};

// slot of the level-L cell with key `key` in its level's brick field, or -1
__device__ inline int64_t tree_lookup(const Tree& t, int L, uint64_t key) {
  int64_t slot = (int64_t)(key >> (3 * L));
  for (int l = 1; l <= L; ++l) {
    const int32_t d = t.slot_child[l - 1][slot];
    if (d < 0) return -1;
    slot = (int64_t)d * 8 + (int64_t)((key >> (3 * (L - l))) & 7u);
  }
  return slot;
}

// slots of K level-L keys at once (-1 where a key is not in the field, or
// where its slot is given as -1 on entry, i.e. skipped): all keys descend one
// level at a time, so their K loads per level are in flight together
template <int K>
__device__ inline void tree_lookup_k(const Tree& t, int L, const uint64_t (&key)[K],
                                     int64_t (&slot)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (slot[k] >= 0) slot[k] = (int64_t)(key[k] >> (3 * L));
  for (int l = 1; l <= L; ++l) {
    const int32_t* sc = t.slot_child[l - 1];
    int32_t dv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) dv[k] = slot[k] >= 0 ? sc[slot[k]] : -1;
#pragma unroll
    for (int k = 0; k < K; ++k)
      slot[k] = dv[k] < 0 ? -1 : (int64_t)dv[k] * 8 + (int64_t)((key[k] >> (3 * (L - l))) & 7u);
  }
}

// Blocks go to the GPU's 8 XCDs in turn (block b runs on XCD b mod 8), and
// every XCD has its own L2.  xcd_tile maps block b to a tile so that each XCD
// takes one contiguous run of tiles: neighbouring tiles, which share cache
// lines at their edges, then meet in one L2.  A bijection on [0, ntiles).
__device__ inline uint32_t xcd_tile(uint32_t b, uint32_t ntiles) {
  const uint32_t q = ntiles >> 3, r = ntiles & 7u;
  const uint32_t x = b & 7u, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// The same for work that varies from tile to tile: each XCD takes runs of C
// consecutive tiles, and the runs go to the XCDs in turn, so that no XCD is
// left with one dense region.  The tiles past the last whole round of 8 runs
// keep their block's index.  A bijection on [0, ntiles).
__device__ inline uint32_t xcd_tile_runs(uint32_t b, uint32_t ntiles, uint32_t C) {
  const uint32_t full = ntiles / (8u * C) * (8u * C);
  if (b >= full) return b;
  const uint32_t x = b & 7u, j = b >> 3;
  return ((j / C) * 8u + x) * C + j % C;
}

__device__ inline uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// Adds each active lane's key to h[p * 256 + digit_p] for the npass 8-bit
// digits p, with one LDS atomic per distinct digit of the wave (lanes with the
// same digit are matched by ballots).
__device__ inline void wave_digit_hist(uint64_t key, bool valid, int npass, uint32_t* h) {
  const uint64_t lt = lanemask_lt();
  const uint64_t act = __ballot(valid);
  // low digits of Morton keys are spread out: plain atomics rarely collide
  const int plain = npass > 2 ? npass - 2 : 0;
  for (int p = 0; p < plain; ++p)
    if (valid) atomicAdd(&h[p * 256 + ((uint32_t)(key >> (8 * p)) & 255u)], 1u);
  // the top digits take few values: match equal digits and add once per group
  for (int p = plain; p < npass; ++p) {
    const uint32_t d = (uint32_t)(key >> (8 * p)) & 255u;
    uint64_t peer = act;
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bm = __ballot(on);
      peer &= on ? bm : ~bm;
    }
    if (valid && (peer & lt) == 0ull) atomicAdd(&h[p * 256 + d], (uint32_t)__popcll(peer));
  }
}

}  // namespace ahf
