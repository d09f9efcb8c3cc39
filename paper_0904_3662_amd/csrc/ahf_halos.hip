// ahf_halos.hip -- particle collection and iterative unbinding of the halos of
// a classified grid tree (Sect. 2.1, the paragraphs after the classification;
// App. A).
//
// Every structure of the classification is a prospective halo:
//   - its leaf is its patch on the deepest level its main branch reaches, and
//     its centre is the centre of mass of the leaf patch's particles (periodic
//     minimum image relative to the lower corner of the leaf's smallest-key
//     cell);
//   - a host collects the particles of its main-branch patch on the deepest
//     level whose boundary contour (thr_{L-1} particles per level-(L-1) cell)
//     lies below Delta_vir times the background density; a substructure
//     collects every particle within half the distance to its host's centre;
//   - unbound particles are removed iteratively: with the particles ordered by
//     radius from the (fixed) centre, the potential is the integral of
//     M(<r')/r'^2 from r to r_vir plus G M_vir / r_vir (the halo truncated at
//     r_vir, App. A), -G M_vir / r beyond r_vir, and a particle whose kinetic
//     energy relative to the halo's mean velocity exceeds |phi| leaves; r_vir
//     is the radius of the last particle whose enclosed mean density is at
//     least Delta_vir times the background.
//
// Layout: one workgroup per structure for its centre and bound, and for the
// sphere query and unbinding of the small structures; the few structures with
// many possible candidates (the wide set) are collected and unbound by the
// whole grid together (chunk kernels and per-structure segment kernels).
// Every sum, sort and compaction has a fixed order, so reruns are
// bit-identical; the particle lists of the leaf and isodensity patches are made
// per cell with atomics (order-free counts and cursors, added once per wave)
// and ordered afterwards.  The centre does not move while a halo is unbound,
// so the candidates are sorted by (radius, index) once; each round then keeps
// that order while it drops the unbound particles.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "ahf_block.h"
#include "ahf_internal.h"

// the FP64 arithmetic of the distance and energy tests is done as written
// (no fused multiply-adds), as it is in the plain definition
#pragma clang fp contract(off)

namespace ahf {
namespace {

constexpr int kHT = kBT;             // threads per workgroup of the per-halo kernels
constexpr int kHW = kBW;             // waves per workgroup
constexpr int kHB = 256;             // threads per block of the per-cell kernels
constexpr int kHTBig = 1024;         // threads per workgroup of the largest structures
constexpr int kRows = 4;             // rows of a workgroup's width whose loads go out together
constexpr int kSeq = 4;              // consecutive particles per thread in the unbinding scans
constexpr int kRadiusBits = 40;      // top bits of a radius' bit pattern the sort orders by
constexpr uint32_t kShortTie = 64;   // longest run of tied truncated radii put in order in place
constexpr uint64_t kBigCand = 32768; // possible candidates from which a structure is wide (default)
constexpr double kQuantum = 1.0 / (double)(1u << kQBits);
constexpr double kHalfQuantum = 0.5 / (double)(1u << kQBits);

__global__ void k_fill_u64(uint64_t* a, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
__global__ void k_fill_u32(uint32_t* a, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

unsigned blocks_for(uint64_t n, int t = kHB) {
  uint64_t b = (n + t - 1) / t;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

// periodic minimum image of a displacement in the unit box
__device__ inline double mimg(double d) { return d - rint(d); }

// ---------------------------------------------------------------- leaves and patch lists

// leafkey[s] = max over the patches of structure s of (level << 32 | patch)
__global__ void k_leaf(int L, const int32_t* __restrict__ pstruct, uint64_t npatch,
                       unsigned long long* __restrict__ leafkey) {
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < npatch;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const int32_t s = pstruct[q];
    if (s < 0) continue;
    atomicMax(&leafkey[s], ((unsigned long long)L << 32) | (unsigned long long)q);
  }
}

// the isodensity patch of every host: its main-branch patch on the deepest
// level in [start, leaf] whose contour lies below Delta_vir (bit L of
// isomask), else its start level
__global__ void k_iso(int L, const int32_t* __restrict__ pstruct, uint64_t npatch,
                      const int32_t* __restrict__ s_depth, const int32_t* __restrict__ s_level,
                      const unsigned long long* __restrict__ leafkey, uint32_t isomask,
                      int32_t* __restrict__ iso_patch, int32_t* __restrict__ iso_level) {
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < npatch;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const int32_t s = pstruct[q];
    if (s < 0 || s_depth[s] != 0) continue;
    const int start = s_level[s];
    const int leafL = (int)(leafkey[s] >> 32);
    int li = start;
    for (int l = start; l <= leafL; ++l)
      if ((isomask >> l) & 1u) li = l;
    if (li == L) {
      iso_patch[s] = (int32_t)q;
      iso_level[s] = L;
    }
  }
}

// Per cell of level L: the cells of a structure's leaf patch count their
// particles into leaf_cnt (and the smallest key into leaf_min); the cells of a
// host's isodensity patch count into iso_cnt.  With fill, the particle indices
// are written into the lists at the structures' offsets instead (cursor order).
// Wave-aggregated atomics on per-structure counters: the lanes where `on` is
// set add v to ctr[key] (several lanes mostly share a key: neighbouring cells
// belong to one patch), one atomic per distinct key in the wave; each lane
// gets the counter's value before its own share (the lanes of a key in lane
// order).  Every lane of the wave calls it.
__device__ inline uint32_t wave_add(uint32_t* ctr, int32_t key, uint32_t v, bool on) {
  const int lane = __lane_id();
  uint64_t todo = __ballot(on);
  uint32_t mine = 0;
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int32_t kl = __shfl(key, leader);
    const bool peer = on && key == kl;
    const uint64_t peers = __ballot(peer);
    uint32_t inc = peer ? v : 0u;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    const uint32_t total = __shfl(inc, 63);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&ctr[kl], total);
    base = __shfl(base, leader);
    if (peer) mine = base + inc - v;
    todo &= ~peers;
  }
  return mine;
}

// the same for an integer maximum (or minimum, with `is_min`) of 64-bit values
__device__ inline void wave_extreme(unsigned long long* ctr, int32_t key, unsigned long long v,
                                    bool on, bool is_min) {
  const int lane = __lane_id();
  uint64_t todo = __ballot(on);
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int32_t kl = __shfl(key, leader);
    const bool peer = on && key == kl;
    const uint64_t peers = __ballot(peer);
    unsigned long long x = peer ? v : (is_min ? ~0ull : 0ull);
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long y = __shfl_xor(x, o);
      x = is_min ? (y < x ? y : x) : (y > x ? y : x);
    }
    if (lane == leader) {
      if (is_min) atomicMin(&ctr[kl], x);
      else atomicMax(&ctr[kl], x);
    }
    todo &= ~peers;
  }
}

__global__ void k_patch_lists(int L, uint64_t nS, uint64_t npatch, const uint64_t* __restrict__ Skey,
                              const uint32_t* __restrict__ Sstart,
                              const uint32_t* __restrict__ Scount,
                              const int32_t* __restrict__ Spatch,
                              const int32_t* __restrict__ pstruct,
                              const unsigned long long* __restrict__ leafkey,
                              const int32_t* __restrict__ iso_patch,
                              const int32_t* __restrict__ iso_level, const uint32_t* __restrict__ order,
                              uint32_t* __restrict__ leaf_cnt,
                              unsigned long long* __restrict__ leaf_min,
                              uint32_t* __restrict__ iso_cnt, int fill,
                              const uint64_t* __restrict__ leaf_off,
                              uint32_t* __restrict__ leaf_list,
                              const uint64_t* __restrict__ iso_off, uint32_t* __restrict__ iso_list) {
  // rounds of the whole grid, so that every lane of a wave takes part in the
  // wave-aggregated atomics
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < nS; base += stride) {
    const uint64_t c = base + threadIdx.x;
    int32_t s = -1;
    uint32_t cnt = 0;
    bool is_leaf = false, is_iso = false;
    if (c < nS) {
      const int32_t q = Spatch[c];
      if (q >= 0 && (uint64_t)q < npatch) {
        s = pstruct[q];
        if (s >= 0) {
          cnt = Scount[c];
          is_leaf = leafkey[s] == (((unsigned long long)L << 32) | (unsigned long long)q);
          is_iso = iso_level[s] == L && iso_patch[s] == q;
        }
      }
    }
    if (!fill) {
      (void)wave_add(leaf_cnt, s, cnt, is_leaf);
      wave_extreme(leaf_min, s, is_leaf ? (unsigned long long)Skey[c] : 0ull, is_leaf, true);
      (void)wave_add(iso_cnt, s, cnt, is_iso);
      continue;
    }
    const uint32_t la = wave_add(leaf_cnt, s, cnt, is_leaf && cnt);
    const uint32_t ia = wave_add(iso_cnt, s, cnt, is_iso && cnt);
    if ((is_leaf || is_iso) && cnt) {
      const uint32_t a = Sstart[c];
      for (uint32_t j = 0; j < cnt; ++j) {
        const uint32_t i = order[a + j];
        if (is_leaf) leaf_list[leaf_off[s] + la + j] = i;
        if (is_iso) iso_list[iso_off[s] + ia + j] = i;
      }
    }
  }
}
__global__ void k_extent(int L, int bits, uint64_t nS, uint64_t npatch,
                         const uint64_t* __restrict__ Skey, const int32_t* __restrict__ Spatch,
                         const int32_t* __restrict__ pstruct, const int32_t* __restrict__ s_depth,
                         const int32_t* __restrict__ s_level, const int32_t* __restrict__ s_patch,
                         const double* __restrict__ centre, unsigned long long* __restrict__ ext) {
  const double h = 1.0 / (double)(1ull << bits);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < nS; base += stride) {
    const uint64_t c = base + threadIdx.x;
    int32_t s = -1;
    bool on = false;
    unsigned long long ev = 0;
    if (c < nS) {
      const int32_t q = Spatch[c];
      if (q >= 0 && (uint64_t)q < npatch) {
        s = pstruct[q];
        on = s >= 0 && s_depth[s] != 0 && s_level[s] == L && s_patch[s] == q;
      }
    }
    if (on) {
      const uint64_t key = Skey[c];
      const uint32_t ix[3] = {compact3(key >> 2), compact3(key >> 1), compact3(key)};
      double dd[3];
      for (int k = 0; k < 3; ++k) {
        const double ck = centre[3 * (uint64_t)s + k];
        const double lo = (double)ix[k] / (double)(1ull << bits);
        const double a = fabs(mimg(lo - ck));
        const double hi = lo + h;
        const double b = fabs(mimg(hi - ck));
        dd[k] = a > b ? a : b;
      }
      const double e = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
      ev = (unsigned long long)__double_as_longlong(e);
    }
    wave_extreme(ext, s, ev, on, false);
  }
}

// Device-wide exclusive scans of integer values f(0..n-1) into n+1 offsets
// (off[n] = the total): the blocks' sums, one scan of those, then each
// block's own prefixes.  Integer sums, so the offsets do not depend on the
// order of the additions.
constexpr int kSB = 256, kSI = 16, kSC = kSB * kSI;  // threads, items each, items per block

struct CountOf {  // the values of a count array
  const uint32_t* c;
  __device__ uint64_t operator()(uint64_t i) const { return c[i]; }
};

// exclusive scan of one value per thread over a workgroup of BT threads;
// *total = the workgroup's sum
template <int BT>
__device__ inline uint64_t block_escan_u64(uint64_t x, uint64_t* red, uint64_t* total) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint64_t inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == 63) red[w] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int i = 0; i < BT / 64; ++i) {
    if (i < w) before += red[i];
    all += red[i];
  }
  *total = all;
  return before + inc - x;
}

template <class F>
__global__ __launch_bounds__(kSB) void k_scan_part(F f, uint64_t n, uint64_t* __restrict__ part) {
  __shared__ uint64_t red[kSB / 64];
  const uint64_t b0 = (uint64_t)blockIdx.x * kSC;
  uint64_t v = 0;
  for (int e = 0; e < kSI; ++e) {
    const uint64_t i = b0 + (uint64_t)e * kSB + threadIdx.x;
    if (i < n) v += f(i);
  }
  uint64_t total = 0;
  (void)block_escan_u64<kSB>(v, red, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// the blocks' sums scanned in place (one workgroup); *total = their sum
__global__ __launch_bounds__(1024) void k_scan_top(uint64_t* __restrict__ part, uint64_t nb,
                                                   uint64_t* __restrict__ total) {
  __shared__ uint64_t red[1024 / 64];
  uint64_t carry = 0;
  for (uint64_t c0 = 0; c0 < nb; c0 += 1024) {
    const uint64_t i = c0 + threadIdx.x;
    const uint64_t v = i < nb ? part[i] : 0;
    uint64_t t = 0;
    const uint64_t ex = block_escan_u64<1024>(v, red, &t);
    if (i < nb) part[i] = carry + ex;
    carry += t;
  }
  if (threadIdx.x == 0) *total = carry;
}

// each thread its kSI consecutive values
template <class F>
__global__ __launch_bounds__(kSB) void k_scan_apply(F f, uint64_t n, const uint64_t* __restrict__ part,
                                                    uint64_t* __restrict__ off) {
  __shared__ uint64_t red[kSB / 64];
  const uint64_t i0 = (uint64_t)blockIdx.x * kSC + (uint64_t)threadIdx.x * kSI;
  uint64_t v[kSI];
  uint64_t s = 0;
#pragma unroll
  for (int e = 0; e < kSI; ++e) {
    v[e] = i0 + e < n ? f(i0 + e) : 0;
    s += v[e];
  }
  uint64_t total = 0;
  uint64_t run = part[blockIdx.x] + block_escan_u64<kSB>(s, red, &total);
#pragma unroll
  for (int e = 0; e < kSI; ++e) {
    if (i0 + e < n) off[i0 + e] = run;
    run += v[e];
  }
}

template <class F>
static void scan_offsets(Ws& ws, F f, uint64_t n, uint64_t* off, hipStream_t st) {
  const uint64_t nb = n ? (n + kSC - 1) / kSC : 1;
  uint64_t* part = ws.get<uint64_t>(nb);
  k_scan_part<F><<<(unsigned)nb, kSB, 0, st>>>(f, n, part);
  k_scan_top<<<1, 1024, 0, st>>>(part, nb, off + n);
  k_scan_apply<F><<<(unsigned)nb, kSB, 0, st>>>(f, n, part, off);
  HIP_LAUNCH_CHECK();
}


// ---------------------------------------------------------------- per-halo kernels

// One particle as the halo kernels read it, in input order: its position as
// coordinates in box units (integer part plus fraction, times the quantum),
// then its velocity and mass (0 where the particles share mass_scalar).  The
// kernels reach particles by index, at random; one aligned 64-byte record
// per particle makes each such access one line instead of one per array.
struct alignas(64) PRec {
  double x, y, z, spare;
  float4 vm;  // vx, vy, vz, mass
  uint32_t pad[4];
};
static_assert(sizeof(PRec) == 64, "one record per 64-byte line");

struct PartIn {
  const uint32_t *X, *Y, *Z;
  const float *fx, *fy, *fz;  // may be null
  const float* mass;          // null: every particle has mass_scalar
  double mass_scalar;
  const float *vx, *vy, *vz;
  const PRec* R;              // the records (k_stage), n of them
};

__device__ inline double coord(const uint32_t* X, const float* f, uint32_t i) {
  return ((double)X[i] + (f ? (double)f[i] : 0.0)) * kQuantum;
}
// particle i's position, velocity and mass from its record
__device__ inline void ppos(const PartIn& P, uint32_t i, double& x, double& y, double& z) {
  const double2 a = *reinterpret_cast<const double2*>(&P.R[i].x);
  x = a.x;
  y = a.y;
  z = P.R[i].z;
}
__device__ inline float4 pvel(const PartIn& P, uint32_t i) { return P.R[i].vm; }
__device__ inline double pmass(const PartIn& P, uint32_t i) {
  return P.mass ? (double)P.R[i].vm.w : P.mass_scalar;
}

// LDS written by some lanes of a wave and read by others, within the wave
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the records of the n particles (F: all three fractions are given, else
// each may be null; M: the masses are given; as template arguments, so that
// every load of a particle is issued at once).  Each wave forms 64 records,
// one per lane, in LDS and writes them out as 4 KB of consecutive 16-byte
// pieces (lanes 16 bytes apart instead of 64).
constexpr int kStageBlocks = 1024;  // half the GPU's waves: the list kernels run beside it
template <bool F, bool M>
__global__ __launch_bounds__(256) void k_stage(PartIn P, uint64_t n, PRec* __restrict__ R) {
  __shared__ uint4 buf[4][64 * 4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint4* wb = buf[w];
  for (uint64_t base = ((uint64_t)blockIdx.x * 4 + w) * 64; base < n;
       base += (uint64_t)gridDim.x * 256) {
    const uint64_t i = base + lane;
    if (i < n) {
      const uint32_t X = P.X[i], Y = P.Y[i], Z = P.Z[i];
      const float fx = (F || P.fx) ? P.fx[i] : 0.0f;
      const float fy = (F || P.fy) ? P.fy[i] : 0.0f;
      const float fz = (F || P.fz) ? P.fz[i] : 0.0f;
      const float vx = P.vx[i], vy = P.vy[i], vz = P.vz[i];
      const float m = M ? P.mass[i] : 0.0f;
      const double x = ((double)X + (double)fx) * kQuantum;  // as coord()
      const double y = ((double)Y + (double)fy) * kQuantum;
      const double z = ((double)Z + (double)fz) * kQuantum;
      const uint64_t bx = (uint64_t)__double_as_longlong(x), by = (uint64_t)__double_as_longlong(y);
      const uint64_t bz = (uint64_t)__double_as_longlong(z);
      wb[lane * 4 + 0] = make_uint4((uint32_t)bx, (uint32_t)(bx >> 32), (uint32_t)by,
                                    (uint32_t)(by >> 32));
      wb[lane * 4 + 1] = make_uint4((uint32_t)bz, (uint32_t)(bz >> 32), 0u, 0u);
      wb[lane * 4 + 2] = make_uint4(__float_as_uint(vx), __float_as_uint(vy), __float_as_uint(vz),
                                    __float_as_uint(m));
      wb[lane * 4 + 3] = make_uint4(0u, 0u, 0u, 0u);
    }
    wave_lds_sync();
    uint4* out = reinterpret_cast<uint4*>(R + base);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = j * 64 + lane;  // piece q of the wave's 4 KB: record q / 4
      if (base + (uint64_t)(q >> 2) < n) out[q] = wb[q];
    }
    wave_lds_sync();
  }
}

// the fork and join events of the step's two streams, destroyed on every path
struct StreamEvents {
  hipEvent_t fork = nullptr, join = nullptr;
  StreamEvents() {
    HIP_CHECK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    const hipError_t e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (e != hipSuccess) {  // the destructor does not run for a constructor that throws
      (void)hipEventDestroy(fork);
      throw Error{AHF_EDEVICE, std::string("hipEventCreateWithFlags: ") + hipGetErrorString(e)};
    }
  }
  ~StreamEvents() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
  }
  StreamEvents(const StreamEvents&) = delete;
  StreamEvents& operator=(const StreamEvents&) = delete;
};

// centre of every structure: the leaf list sorted by particle index, then the
// mass-weighted mean of the minimum-image offsets from the lower corner of the
// leaf's smallest-key cell
__global__ __launch_bounds__(kHT) void k_centre(const uint64_t* __restrict__ leaf_off,
                                                const uint32_t* __restrict__ leaf_cnt,
                                                uint32_t* leaf_list, uint32_t* leaf_tmp,
                                                const unsigned long long* __restrict__ leafkey,
                                                const unsigned long long* __restrict__ leaf_min,
                                                int g, PartIn P, double* __restrict__ centre) {
  __shared__ double red[kHW];
  const uint32_t s = blockIdx.x;
  const uint32_t n = leaf_cnt[s];
  uint32_t* a = leaf_list + leaf_off[s];
  uint32_t* b = leaf_tmp + leaf_off[s];
  const bool fl = block_sort<uint32_t>(a, a, b, b, n);
  const uint32_t* idx = fl ? b : a;
  const int bits = g + (int)(leafkey[s] >> 32);
  const uint64_t key = leaf_min[s];
  double ref[3];
  ref[0] = (double)compact3(key >> 2) / (double)(1ull << bits);
  ref[1] = (double)compact3(key >> 1) / (double)(1ull << bits);
  ref[2] = (double)compact3(key) / (double)(1ull << bits);
  double sx = 0.0, sy = 0.0, sz = 0.0, sw = 0.0;
  for (uint32_t k = threadIdx.x; k < n; k += kHT) {
    const uint32_t i = idx[k];
    const double w = pmass(P, i);
    double x, y, z;
    ppos(P, i, x, y, z);
    sx += w * mimg(x - ref[0]);
    sy += w * mimg(y - ref[1]);
    sz += w * mimg(z - ref[2]);
    sw += w;
  }
  sx = block_sum(sx, red);
  sy = block_sum(sy, red);
  sz = block_sum(sz, red);
  sw = block_sum(sw, red);
  if (threadIdx.x == 0) {
    double c[3];
    if (sw == 0.0) {
      for (int d = 0; d < 3; ++d) c[d] = ref[d] + 0.5 / (double)(1ull << bits);
    } else {
      c[0] = ref[0] + sx / sw;
      c[1] = ref[1] + sy / sw;
      c[2] = ref[2] + sz / sw;
    }
    for (int d = 0; d < 3; ++d) centre[3 * s + d] = c[d] - floor(c[d]);
  }
}

// the level-0 cells a sphere may touch: per axis the cell range [lo, lo+n)
// (wrapped), the whole axis when the sphere is at least as wide as the box
__device__ inline void cube_of(const double* c, double R, int g, int64_t* lo, int64_t* nc) {
  const int64_t side = 1ll << g;
  for (int d = 0; d < 3; ++d) {
    int64_t a = (int64_t)floor((c[d] - R) * (double)side);
    int64_t b = (int64_t)floor((c[d] + R) * (double)side);
    if (b - a + 1 >= side) {
      a = 0;
      b = side - 1;
    }
    lo[d] = a;
    nc[d] = b - a + 1;
  }
}

__device__ inline uint64_t cube_cell(const int64_t* lo, const int64_t* nc, uint64_t k, int g) {
  const int64_t side = 1ll << g;
  const int64_t iz = (int64_t)(k % (uint64_t)nc[2]);
  const int64_t iy = (int64_t)((k / (uint64_t)nc[2]) % (uint64_t)nc[1]);
  const int64_t ix = (int64_t)(k / ((uint64_t)nc[2] * (uint64_t)nc[1]));
  const uint32_t x = (uint32_t)(((lo[0] + ix) % side + side) % side);
  const uint32_t y = (uint32_t)(((lo[1] + iy) % side + side) % side);
  const uint32_t z = (uint32_t)(((lo[2] + iz) % side + side) % side);
  return morton3(x, y, z);
}

// The cells of every built level (the hierarchy's device arrays), for the
// sphere queries; level 0 is dense (its S index is the key)
struct LevCells {
  const uint64_t* key[kMaxLevels];
  const uint32_t* start[kMaxLevels];
  const uint32_t* count[kMaxLevels];
  uint64_t n[kMaxLevels];
  int nlev;
  int g;
};

constexpr int kQCells = 125;  // cube cells of a query on a level whose cells are >= R/2 wide
constexpr int kCoarseMax = 4096;  // level-0 cube cells the grid's collection takes for a wide sphere

// The level a sphere of radius R is queried on: the deepest built level whose
// cells are at least R/2 wide, so that at most 5 per axis cover the sphere
// (level 0 when even its cells are narrower)
__device__ inline int query_level(const LevCells& LC, double R) {
  int L = LC.nlev - 1;
  while (L > 0 && ldexp(1.0, -(LC.g + L)) < 0.5 * R) --L;
  return L;
}

// The deepest cell of the hierarchy containing the level-L cell `key`: the
// cell itself when its parent was refined, else the nearest ancestor that
// exists (every level-0 cell does); its level and S index
__device__ inline void resolve_cell(const LevCells& LC, int L, uint64_t key, int* lout,
                                    uint64_t* iout) {
  for (;;) {
    if (L == 0) {
      *lout = 0;
      *iout = key;
      return;
    }
    const uint64_t* K = LC.key[L];
    uint64_t lo = 0, hi = LC.n[L];
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (K[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    if (lo < LC.n[L] && K[lo] == key) {
      *lout = L;
      *iout = lo;
      return;
    }
    key >>= 3;
    --L;
  }
}

// The particle ranges a sphere query scans when its cube on level L has at
// most kQCells cells: each cube cell resolved to the deepest cell containing
// it; the resolved cells are the leaves of the hierarchy cut at level L, so
// two are equal or disjoint, and the distinct ones cover the cube.  Their
// starts and counts go to qa, qc (LDS) in the order of their first cube cell
// (the same on every call); returns their number (every thread).
template <int BT>
__device__ inline uint32_t fine_cells(const LevCells& LC, int L, const int64_t* lo,
                                      const int64_t* nc, uint64_t ncell, uint32_t* qa,
                                      uint32_t* qc) {
  __shared__ int ql[kQCells];
  __shared__ uint64_t qi[kQCells];
  __shared__ double red[BT / 64];
  const uint32_t t = threadIdx.x;
  if (t < ncell) resolve_cell(LC, L, cube_cell(lo, nc, t, LC.g + L), &ql[t], &qi[t]);
  __syncthreads();
  bool keep = false;
  if (t < ncell) {
    keep = true;
    for (uint32_t u = 0; u < t; ++u) keep = keep && !(ql[u] == ql[t] && qi[u] == qi[t]);
  }
  double tot = 0.0;
  const double inc = block_scan<BT>(keep ? 1.0 : 0.0, red, &tot);
  if (keep) {
    const uint32_t at = (uint32_t)inc - 1u;
    qa[at] = LC.start[ql[t]][qi[t]];
    qc[at] = LC.count[ql[t]][qi[t]];
  }
  __syncthreads();
  return (uint32_t)tot;
}

// collection radius and an upper bound of the candidates: a host's
// isodensity patch count; a substructure's sphere (half the distance to its
// host's centre): the particles of the level-0 cells it may touch
__global__ __launch_bounds__(kHT) void k_bound(const int32_t* __restrict__ s_depth,
                                               const int32_t* __restrict__ s_host,
                                               const unsigned long long* __restrict__ ext,
                                               const double* __restrict__ centre,
                                               const uint32_t* __restrict__ iso_cnt,
                                               const LevCells LC,
                                               double* __restrict__ radius,
                                               uint32_t* __restrict__ bound,
                                               uint8_t* __restrict__ coarse) {
  __shared__ double red[kHW];
  __shared__ uint32_t qa[kQCells], qc[kQCells];
  const uint32_t s = blockIdx.x;
  if (s_depth[s] == 0) {
    if (threadIdx.x == 0) {
      radius[s] = 0.0;
      bound[s] = iso_cnt[s];
      coarse[s] = 0;
    }
    return;
  }
  const int32_t hh = s_host[s];
  if (hh < 0) {  // a substructure always has a host; nothing to collect otherwise
    if (threadIdx.x == 0) {
      radius[s] = 0.0;
      bound[s] = 0;
      coarse[s] = 0;
    }
    return;
  }
  const double* c = centre + 3 * (uint64_t)s;
  const double* ch = centre + 3 * (uint64_t)hh;
  const double sx = mimg(c[0] - ch[0]), sy = mimg(c[1] - ch[1]), sz = mimg(c[2] - ch[2]);
  const double half = 0.5 * sqrt(sx * sx + sy * sy + sz * sz);
  const double e = __longlong_as_double((long long)ext[s]);
  const double R = e < half ? e : half;  // capped by the start patch's extent
  // the particles of the cells the query scans (integers, exact in FP64)
  const int L = query_level(LC, R);
  int64_t lo[3], nc[3];
  cube_of(c, R, LC.g + L, lo, nc);
  const uint64_t ncell = (uint64_t)nc[0] * (uint64_t)nc[1] * (uint64_t)nc[2];
  double t = 0.0;
  if (ncell <= kQCells) {
    const uint32_t nq = fine_cells<kHT>(LC, L, lo, nc, ncell, qa, qc);
    for (uint32_t k = threadIdx.x; k < nq; k += kHT) t += (double)qc[k];
  } else {  // level 0, a sphere wider than several of its cells
    for (uint64_t k = threadIdx.x; k < ncell; k += kHT)
      t += (double)LC.count[0][cube_cell(lo, nc, k, LC.g)];
  }
  t = block_sum(t, red);
  if (threadIdx.x == 0) {
    radius[s] = R;
    bound[s] = (uint32_t)t;
    coarse[s] = ncell > kCoarseMax ? 1 : 0;
  }
}

// the candidates of every structure, unordered: a host's isodensity list, a
// substructure's particles within its radius.  A substructure scans the cells
// its query level gives (at most kQCells, else level-0 cells in chunks of one
// per thread); the particles of a chunk of cells are spread over all threads
// (a dense cell holds many), each finding its cell by a binary search of the
// chunk's particle offsets.
template <int BT>
__global__ __launch_bounds__(BT) void k_candidates(
    const int32_t* __restrict__ s_depth, const double* __restrict__ centre,
    const double* __restrict__ radius, const uint64_t* __restrict__ iso_off,
    const uint32_t* __restrict__ iso_cnt, const uint32_t* __restrict__ iso_list,
    const LevCells LC, const uint32_t* __restrict__ order, PartIn P,
    const uint64_t* __restrict__ cand_off,
    uint32_t* __restrict__ cand, uint32_t* __restrict__ cand_cnt, uint64_t big,
    const uint32_t* __restrict__ sel, const uint8_t* __restrict__ only) {
  constexpr int BW = BT / 64;
  // block b takes structure sel[b] (the wide list) or b; structures with at
  // least `big` possible candidates go to the wide workgroups (those with
  // `only` set: the rest of the wide set is collected by the grid)
  const uint32_t s = sel ? sel[blockIdx.x] : blockIdx.x;
  if ((cand_off[s + 1] - cand_off[s] >= big) != (BT > kHT)) return;
  if (only && !only[s]) return;
  __shared__ uint32_t cursor;
  __shared__ uint32_t cofs[BT + 1];  // the chunk's particle offsets per cell
  __shared__ uint32_t cst[BT];       // and each cell's first sorted position
  __shared__ double red[BW];
  uint32_t* out = cand + cand_off[s];
  if (s_depth[s] == 0) {
    const uint32_t n = iso_cnt[s];
    const uint32_t* in = iso_list + iso_off[s];
    for (uint32_t k = threadIdx.x; k < n; k += BT) out[k] = in[k];
    if (threadIdx.x == 0) cand_cnt[s] = n;
    return;
  }
  if (threadIdx.x == 0) cursor = 0;
  const double* c = centre + 3 * (uint64_t)s;
  const double R = radius[s];
  const double R2 = R * R;
  const int L = query_level(LC, R);
  int64_t lo[3], nc[3];
  cube_of(c, R, LC.g + L, lo, nc);
  const uint64_t ncube = (uint64_t)nc[0] * (uint64_t)nc[1] * (uint64_t)nc[2];
  const bool fine = ncube <= kQCells;
  __shared__ uint32_t qa[kQCells], qc[kQCells];
  const uint64_t ncell = fine ? fine_cells<BT>(LC, L, lo, nc, ncube, qa, qc) : ncube;
  for (uint64_t k0 = 0; k0 < ncell; k0 += BT) {
    const uint64_t k = k0 + threadIdx.x;
    uint32_t a = 0, cnt = 0;
    if (k < ncell) {
      if (fine) {
        a = qa[k];
        cnt = qc[k];
      } else {  // level 0
        const uint64_t cell = cube_cell(lo, nc, k, LC.g);
        a = LC.start[0][cell];
        cnt = LC.count[0][cell];
      }
    }
    // exclusive offsets (counts below 2^32 are exact in FP64)
    double tot = 0.0;
    const double inc = block_scan<BT>((double)cnt, red, &tot);
    cofs[threadIdx.x] = (uint32_t)inc - cnt;
    cst[threadIdx.x] = a;
    if (threadIdx.x == 0) cofs[BT] = (uint32_t)tot;
    __syncthreads();
    const uint32_t total = (uint32_t)tot;
    for (uint32_t f0 = threadIdx.x; f0 < total; f0 += kRows * BT) {
      // the particles of kRows rows, their loads out together
      uint32_t pi[kRows];
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const uint32_t f = f0 + j * BT;
        pi[j] = 0;
        if (f < total) {
          // the last cell whose offset is at most f (it holds particle f)
          uint32_t lo_c = 0, hi_c = BT - 1;
          while (lo_c < hi_c) {
            const uint32_t mid = (lo_c + hi_c + 1) >> 1;
            if (cofs[mid] <= f) lo_c = mid;
            else hi_c = mid - 1;
          }
          pi[j] = order[cst[lo_c] + (f - cofs[lo_c])];
        }
      }
      double px[kRows], py[kRows], pz[kRows];
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        if (f0 + j * BT < total) {
          ppos(P, pi[j], px[j], py[j], pz[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        if (f0 + j * BT >= total) break;
        const double dx = mimg(px[j] - c[0]);
        const double dy = mimg(py[j] - c[1]);
        const double dz = mimg(pz[j] - c[2]);
        if (dx * dx + dy * dy + dz * dz <= R2) out[atomicAdd(&cursor, 1u)] = pi[j];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) cand_cnt[s] = cursor;
}

// The radius and the velocity and mass of every candidate of the structures
// unbound by the wide workgroups, by candidate slot, computed by the whole
// grid (their loads by particle index are scattered; one workgroup on one
// compute unit would take them one after another): rad at the slot (the
// unbinding's msum scratch), vq at the slot.  Slots past a structure's count
// are left alone.
__global__ void k_big_data(const uint64_t* __restrict__ cand_off,
                           const uint32_t* __restrict__ cand_cnt,
                           const uint32_t* __restrict__ cand, const uint32_t* __restrict__ gs,
                           const uint64_t* __restrict__ boff, uint32_t nG,
                           const double* __restrict__ centre, PartIn P,
                           const uint8_t* __restrict__ only, double* __restrict__ rad,
                           float4* __restrict__ vq) {
  const uint64_t tb = boff[nG];
  for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < tb;
       p += (uint64_t)gridDim.x * blockDim.x) {
    // the wide structure of position p: the last g with boff[g] <= p
    uint32_t lo = 0, hi = nG - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (boff[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const uint64_t s = gs[lo];
    if (!only[s] || p - boff[lo] >= cand_cnt[s]) continue;
    const uint64_t j = cand_off[s] + (p - boff[lo]);
    const uint32_t i = cand[j];
    const double* c = centre + 3 * s;
    double x, y, z;
    ppos(P, i, x, y, z);
    const double dx = mimg(x - c[0]);
    const double dy = mimg(y - c[1]);
    const double dz = mimg(z - c[2]);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r < kHalfQuantum) r = kHalfQuantum;
    rad[j] = r;
    vq[j] = pvel(P, i);
  }
}

// inclusive scan of one value per thread over the workgroup, in thread
// order, with one barrier: consecutive calls alternate between the two
// halves of red (par), so a call never overwrites what the one before it
// is still reading
template <int BT>
__device__ inline double block_scan1(double x, double (*red)[BT / 64], int par, double* total) {
  constexpr int BW = BT / 64;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) red[par][w] = x;
  __syncthreads();
  double before = 0.0, all = 0.0;
  for (int i = 0; i < BW; ++i) {
    if (i < w) before += red[par][i];
    all += red[par][i];
  }
  *total = all;
  return before + x;
}

// exclusive scan of one value per thread over the workgroup, in thread
// order, with one barrier (alternating halves of red as block_scan1)
template <int BT>
__device__ inline double block_escan1(double x, double (*red)[BT / 64], int par, double* total) {
  constexpr int BW = BT / 64;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  double inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  double exc = __shfl_up(inc, 1);
  if (lane == 0) exc = 0.0;
  if (lane == 63) red[par][w] = inc;
  __syncthreads();
  double before = 0.0, all = 0.0;
  for (int i = 0; i < BW; ++i) {
    if (i < w) before += red[par][i];
    all += red[par][i];
  }
  *total = all;
  return before + exc;
}

__device__ inline double vmass(const PartIn& P, const float4& v) {
  return P.mass ? (double)v.w : P.mass_scalar;
}

// Unbinding of every structure's candidates.  Scratch per candidate (at the
// structure's offset): idx_a, idx_b (u32), key_a, key_b (u64), msum, tail
// (f64), and the velocity and mass (vbuf) in radius order, kept beside the
// radii while the rounds drop particles, so that the rounds read them in
// order instead of by particle index.  On exit cand holds the candidates in
// radius order, member the halo's particles in radius order.
template <int BT>
__global__ __launch_bounds__(BT) void k_unbind(
    const uint64_t* __restrict__ cand_off, const uint32_t* __restrict__ cand_cnt, uint32_t* cand,
    uint32_t* idx_a, uint32_t* idx_b, uint64_t* key_a, uint64_t* key_b, double* msum,
    double* tail, float4* vbuf, const float4* __restrict__ vslot,
    const double* __restrict__ centre, PartIn P, double rho_thr, double G,
    uint32_t max_iter, uint32_t* __restrict__ member, uint32_t* __restrict__ member_cnt,
    double* __restrict__ r_vir_out, double* __restrict__ m_vir_out, double* __restrict__ vel_out,
    uint32_t* __restrict__ iters_out, const uint32_t* __restrict__ mode,
    const uint32_t* __restrict__ sel) {
  constexpr int BW = BT / 64;
  // block b takes structure sel[b] (the wide list) or b; mode 0: the small
  // structures (kHT threads); mode 2: wide structures with long runs of tied
  // radii (kHTBig threads); mode 1 goes through the grid
  const uint32_t s = sel ? sel[blockIdx.x] : blockIdx.x;
  if (mode[s] != (BT > kHT ? 2u : 0u)) return;
  __shared__ double red[BW];
  __shared__ double rsc[2][BW];  // the scans, alternating halves
  __shared__ int64_t redi[BW];
  __shared__ uint32_t wkeep[2][BW], wgone[2][BW];  // the compaction, alternating halves
  const uint64_t off = cand_off[s];
  const uint32_t n = cand_cnt[s];
  uint32_t* cs = cand + off;
  uint32_t* ia = idx_a + off;
  uint32_t* ib = idx_b + off;
  uint64_t* ka = key_a + off;
  uint64_t* kb = key_b + off;
  double* M = msum + off;
  double* T = tail + off;
  float4* V = vbuf + off;
  const float4* VS = vslot + off;
  // the wide workgroups find radii and velocities by slot (k_big_data)
  constexpr bool kPre = BT > kHT;
  const double* c = centre + 3 * (uint64_t)s;
  const int lane = __lane_id(), w = threadIdx.x >> 6;

  // The candidates ordered by radius (bit patterns of non-negative doubles
  // order like the doubles), ties by particle index.  The sort takes the top
  // kRadiusBits bits of the radius (few passes) with the candidate's slot as
  // payload; particles whose truncated radii tie are then put in order by
  // (radius, index) by the first thread of their run.  A run longer than
  // kShortTie (near-coincident particles) sends the structure down the full
  // sort instead: by index, then stably by the whole radius.
  __shared__ uint32_t long_tie;
  if (threadIdx.x == 0) long_tie = 0;
  if (kPre) {
    for (uint32_t k = threadIdx.x; k < n; k += BT) {
      ka[k] = (uint64_t)__double_as_longlong(M[k]) >> (64 - kRadiusBits);
      ia[k] = k;
    }
  } else {
  for (uint32_t k0 = threadIdx.x; k0 < n; k0 += kRows * BT) {
    // kRows particles per thread, their (random) coordinate loads together
    uint32_t pi[kRows];
    double px[kRows], py[kRows], pz[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) pi[j] = (k0 + j * BT < n) ? cs[k0 + j * BT] : 0u;
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      if (k0 + j * BT < n) {
        ppos(P, pi[j], px[j], py[j], pz[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const uint32_t k = k0 + j * BT;
      if (k >= n) break;
      const double dx = mimg(px[j] - c[0]);
      const double dy = mimg(py[j] - c[1]);
      const double dz = mimg(pz[j] - c[2]);
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r < kHalfQuantum) r = kHalfQuantum;
      M[k] = r;  // the whole radius, by slot (M is free until the rounds)
      ka[k] = (uint64_t)__double_as_longlong(r) >> (64 - kRadiusBits);
      ia[k] = k;
    }
  }
  }
  __syncthreads();
  const bool ft = block_sort<uint64_t, BT>(ka, ia, kb, ib, n);
  const uint64_t* Kt = ft ? kb : ka;  // truncated radii, sorted
  const uint32_t* St = ft ? ib : ia;  // their slots
  uint64_t* K = ft ? ka : kb;         // whole radii in that order
  uint32_t* I = ft ? ia : ib;         // particle indices in that order
  // (each thread reads the slots it then overwrites in the other buffers)
  for (uint32_t k0 = threadIdx.x; k0 < n; k0 += kRows * BT) {
    uint32_t sl[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) sl[j] = (k0 + j * BT < n) ? St[k0 + j * BT] : 0u;
    double rv_[kRows];
    uint32_t iv[kRows];
    float4 qv[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      if (k0 + j * BT < n) {
        rv_[j] = M[sl[j]];
        iv[j] = cs[sl[j]];
      }
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      if (k0 + j * BT < n) {
        const uint32_t i = iv[j];
        qv[j] = kPre ? VS[sl[j]]
                     : pvel(P, i);
      }
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const uint32_t k = k0 + j * BT;
      if (k >= n) break;
      K[k] = (uint64_t)__double_as_longlong(rv_[j]);
      I[k] = iv[j];
      V[k] = qv[j];
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < n; k += BT) {
    if (k > 0 && Kt[k - 1] == Kt[k]) continue;  // not a run start
    uint32_t e = k + 1;
    while (e < n && Kt[e] == Kt[k] && e - k <= kShortTie) ++e;
    if (e - k > kShortTie) long_tie = 1u;
  }
  __syncthreads();
  if (long_tie == 0u) {
    // short ties: insertion sort by (radius, index); the truncated keys of
    // the other runs are not touched
    for (uint32_t k = threadIdx.x; k < n; k += BT) {
      if (k > 0 && Kt[k - 1] == Kt[k]) continue;
      uint32_t e = k + 1;
      while (e < n && Kt[e] == Kt[k]) ++e;
      for (uint32_t q = k + 1; q < e; ++q) {
        const uint64_t kq = K[q];
        const uint32_t iq = I[q];
        const float4 vq = V[q];
        uint32_t r = q;
        while (r > k && (K[r - 1] > kq || (K[r - 1] == kq && I[r - 1] > iq))) {
          K[r] = K[r - 1];
          I[r] = I[r - 1];
          V[r] = V[r - 1];
          --r;
        }
        K[r] = kq;
        I[r] = iq;
        V[r] = vq;
      }
    }
    __syncthreads();
  } else {
    // the full sort: the candidates by index, then a stable sort by radius
    uint32_t* sp1 = ft ? ib : ia;  // the free index buffer (the truncated sort's slots)
    if (block_sort<uint32_t, BT>(cs, cs, sp1, sp1, n))
      for (uint32_t k = threadIdx.x; k < n; k += BT) cs[k] = sp1[k];
    __syncthreads();
    uint64_t* kx = ft ? kb : ka;  // the truncated keys' buffer, now free
    for (uint32_t k = threadIdx.x; k < n; k += BT) {
      const uint32_t i = cs[k];
      double x, y, z;
      ppos(P, i, x, y, z);
      const double dx = mimg(x - c[0]);
      const double dy = mimg(y - c[1]);
      const double dz = mimg(z - c[2]);
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r < kHalfQuantum) r = kHalfQuantum;
      kx[k] = (uint64_t)__double_as_longlong(r);
      sp1[k] = i;
    }
    __syncthreads();
    if (block_sort<uint64_t, BT>(kx, sp1, K, I, n)) {
      // the result is in (K, I) already
    } else {
      for (uint32_t k = threadIdx.x; k < n; k += BT) {
        K[k] = kx[k];
        I[k] = sp1[k];
      }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < n; k += BT) {
      const uint32_t i = I[k];
      V[k] = pvel(P, i);
    }
    __syncthreads();
  }
  // the view's candidates: in radius order
  for (uint32_t k = threadIdx.x; k < n; k += BT) cs[k] = I[k];
  __syncthreads();
  int sc = 0;  // scans so far (their half of rsc)

  uint32_t na = n, iters = 0, nmem = 0;
  double r_vir = 0.0, m_vir = 0.0;
  double vh[3] = {0.0, 0.0, 0.0};
  bool done = false;
  for (uint32_t it = 1; it <= max_iter && na > 0; ++it) {
    iters = it;
    // the halo's velocity: mass-weighted mean
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, sm = 0.0;
    for (uint32_t k0 = threadIdx.x; k0 < na; k0 += kRows * BT) {
      float4 q[kRows];
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const uint32_t k = k0 + j * BT;
        q[j] = k < na ? V[k] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        if (k0 + j * BT >= na) break;
        const double m = vmass(P, q[j]);
        s0 += m * (double)q[j].x;
        s1 += m * (double)q[j].y;
        s2 += m * (double)q[j].z;
        sm += m;
      }
    }
    s0 = block_sum<BT>(s0, red);
    s1 = block_sum<BT>(s1, red);
    s2 = block_sum<BT>(s2, red);
    sm = block_sum<BT>(sm, red);
    vh[0] = s0 / sm;
    vh[1] = s1 / sm;
    vh[2] = s2 / sm;
    // enclosed masses along the radii, and the last particle dense enough:
    // each thread sums kSeq consecutive particles, the threads' sums are
    // scanned across the workgroup
    double carry = 0.0;
    int64_t v = -1;
    for (uint32_t c0 = 0; c0 < na; c0 += kSeq * BT) {
      const uint32_t b0 = c0 + threadIdx.x * kSeq;
      double pre[kSeq], rr[kSeq];
      double run = 0.0;
#pragma unroll
      for (int e = 0; e < kSeq; ++e) {
        const uint32_t k = b0 + e;
        const double m = k < na ? vmass(P, V[k]) : 0.0;
        rr[e] = k < na ? __longlong_as_double((long long)K[k]) : 1.0;
        run += m;
        pre[e] = run;
      }
      double tot = 0.0;
      const double before = carry + block_escan1<BT>(run, rsc, (sc++) & 1, &tot);
#pragma unroll
      for (int e = 0; e < kSeq; ++e) {
        const uint32_t k = b0 + e;
        if (k < na) {
          const double inc = before + pre[e];
          M[k] = inc;
          const double r = rr[e];
          const double dens = inc / (4.0 / 3.0 * M_PI * (r * r * r));
          if (dens >= rho_thr) v = (int64_t)k;
        }
      }
      carry += tot;
    }
    v = block_max_i64<BT>(v, redi);
    if (v < 0) {  // never dense enough: the halo dissolves
      na = 0;
      r_vir = 0.0;
      m_vir = 0.0;
      done = true;
      break;
    }
    __syncthreads();
    const double rv = __longlong_as_double((long long)K[v]);
    const double mv = M[v];
    // tail[k] = sum over j in [k, v) of M_j (1/r_j - 1/r_{j+1}), chunks from the end
    double tcarry = 0.0;
    const uint32_t nv = (uint32_t)v;  // terms 0 .. v-1
    for (int64_t c1 = (int64_t)nv; c1 > 0; c1 -= (int64_t)kSeq * BT) {
      // thread t takes the kSeq terms k = c1 - 1 - (t kSeq + e), from the top
      double pre[kSeq];
      double run = 0.0;
#pragma unroll
      for (int e = 0; e < kSeq; ++e) {
        const int64_t k = c1 - 1 - ((int64_t)threadIdx.x * kSeq + e);
        double term = 0.0;
        if (k >= 0) {
          const double r0 = __longlong_as_double((long long)K[k]);
          const double r1 = __longlong_as_double((long long)K[k + 1]);
          term = M[k] * (1.0 / r0 - 1.0 / r1);
        }
        run += term;
        pre[e] = run;
      }
      double tot = 0.0;
      const double before = tcarry + block_escan1<BT>(run, rsc, (sc++) & 1, &tot);
#pragma unroll
      for (int e = 0; e < kSeq; ++e) {
        const int64_t k = c1 - 1 - ((int64_t)threadIdx.x * kSeq + e);
        if (k >= 0) T[k] = before + pre[e];
      }
      tcarry += tot;
    }
    __syncthreads();
    // the unbound particles, then the others kept in radius order, in
    // place: one particle per thread and row, kRows rows whose loads go out
    // together; a row's writes land at or before its own reads, which all
    // come before its barrier, and before the later rows' reads
    uint32_t kept = 0;
    uint32_t ngone = 0;
    for (uint32_t s0r = 0; s0r < na; s0r += kRows * BT) {
      uint64_t keyr[kRows];
      uint32_t ir[kRows];
      float4 qr[kRows];
      double tr[kRows];
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const uint32_t k = s0r + j * BT + threadIdx.x;
        keyr[j] = 0;
        ir[j] = 0;
        qr[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        tr[j] = 0.0;
        if (k < na) {
          keyr[j] = K[k];
          ir[j] = I[k];
          qr[j] = V[k];
          tr[j] = k < nv ? T[k] : 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const uint32_t c0 = s0r + j * BT;
        if (c0 >= na) break;
        const uint32_t k = c0 + threadIdx.x;
        const int par = (int)((c0 / BT) & 1u);
        bool gone = false;
        if (k < na) {
          const double r = __longlong_as_double((long long)keyr[j]);
          const double phi = (int64_t)k <= v ? -G * (tr[j] + mv / rv) : -G * mv / r;
          const double dx = (double)qr[j].x - vh[0];
          const double dy = (double)qr[j].y - vh[1];
          const double dz = (double)qr[j].z - vh[2];
          const double ke = 0.5 * (dx * dx + dy * dy + dz * dz);
          gone = ke > fabs(phi);
        }
        const bool keep = k < na && !gone;
        const uint64_t kb_ = __ballot(keep);
        const uint64_t gb_ = __ballot(gone);
        if (lane == 0) {
          wkeep[par][w] = (uint32_t)__popcll(kb_);
          wgone[par][w] = (uint32_t)__popcll(gb_);
        }
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int q = 0; q < BW; ++q) {
          if (q < w) before += wkeep[par][q];
          all += wkeep[par][q];
          ngone += wgone[par][q];
        }
        if (keep) {
          const uint32_t at = kept + before + (uint32_t)__popcll(kb_ & lanes_below());
          K[at] = keyr[j];
          I[at] = ir[j];
          V[at] = qr[j];
        }
        kept += all;
      }
    }
    if (ngone == 0) {
      // converged: the particles within r_vir (the first v+1 in radius order)
      nmem = (uint32_t)v + 1;
      r_vir = rv;
      done = true;
      break;
    }
    na = kept;
    __syncthreads();
  }
  if (!done) {  // not converged within max_iter (or nothing collected)
    nmem = 0;
    r_vir = 0.0;
  }
  // the members: the first nmem in radius order
  uint32_t* out = member + off;
  double mm = 0.0;
  for (uint32_t k = threadIdx.x; k < nmem; k += BT) {
    out[k] = I[k];
    mm += vmass(P, V[k]);
  }
  mm = block_sum<BT>(mm, red);
  m_vir = nmem ? mm : 0.0;
  if (threadIdx.x == 0) {
    member_cnt[s] = nmem;
    r_vir_out[s] = r_vir;
    m_vir_out[s] = m_vir;
    vel_out[3 * s + 0] = vh[0];
    vel_out[3 * s + 1] = vh[1];
    vel_out[3 * s + 2] = vh[2];
    iters_out[s] = iters;
  }
}

// ---------------------------------------------------------------- wide unbinding
//
// The structures with many possible candidates (the "wide" set: a few hundred
// that hold most of the candidates) are unbound by the whole grid together
// instead of by one workgroup each: one global radix sort puts every wide
// structure's candidates in (structure, radius) order in one array, each
// structure at its own offset; then every round runs as chunk kernels over
// all still-active structures (a chunk is kWC consecutive particles of one
// structure) and segment kernels that combine a structure's chunks in chunk
// order, one wave per structure.  Every sum has a fixed order, so reruns are
// bit-identical; the host reads one count per round (the structures still
// active).

constexpr int kWT = 256;                 // threads of the chunk kernels
constexpr int kWE = 16;                  // particles per thread and chunk
constexpr uint32_t kWC = kWT * kWE;      // particles per chunk
constexpr uint32_t kRoundsPerCheck = 4;  // unbinding rounds per host read of the active count
// The grid's sort orders a radius r by (bits(r) - bits(kHalfQuantum)) >>
// shift: radii run from kHalfQuantum (the clamp) to below 1 (a minimum-image
// distance in the unit box), so the difference stays below 2^kRadSpan, and
// the radius part of a key is kRadSpan - shift bits wide.  The width is the
// widest that lets every sort pass move one packed word (key and index in 64
// bits), at most kRadiusBits, and kRadiusBits (with pairs in the first
// passes) where that would leave fewer than kMinRadBits.
constexpr int kRadSpan = 57;
static_assert(kQBits + 1 <= 32, "radii in [kHalfQuantum, 1) span at most 32 binary exponents");
constexpr int kMinRadBits = 28;
__device__ inline uint64_t wide_radius(double r, int shift) {
  return ((uint64_t)__double_as_longlong(r) - (uint64_t)__double_as_longlong(kHalfQuantum)) >> shift;
}

// segment (wide structure) and chunk of block b in this round's chunk table
// (cofs: nG + 1 exclusive chunk offsets); false past the table's end
__device__ inline bool chunk_of(const uint32_t* __restrict__ cofs, uint32_t nG, uint32_t b,
                                uint32_t* g, uint32_t* c) {
  if (b >= cofs[nG]) return false;
  uint32_t lo = 0, hi = nG - 1;
  while (lo < hi) {  // the last segment whose first chunk is at most b
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (cofs[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  *g = lo;
  *c = b - cofs[lo];
  return true;
}

// The wide set: the structures with at least `big` possible candidates, in
// structure order.  WideVal gives, for structure s, 0 below big, else 1, its
// possible count or its chunks (what = 0, 1, 2); k_w_place puts the wide
// ones in the list from the scans of those: gs[g] = s, boff[g] = the start
// of its segment, and sizes = (the set's size, its possible candidates, its
// chunks).
struct WideVal {
  const uint64_t* cand_off;
  uint64_t big;
  int what;
  __device__ uint64_t operator()(uint64_t s) const {
    const uint64_t b = cand_off[s + 1] - cand_off[s];
    if (b < big) return 0;
    return what == 0 ? 1 : (what == 1 ? b : (b + kWC - 1) / kWC);
  }
};

__global__ void k_w_place(const uint64_t* __restrict__ fo, const uint64_t* __restrict__ bo,
                          const uint64_t* __restrict__ co, uint64_t ns, uint32_t* __restrict__ gs,
                          uint64_t* __restrict__ boff, uint64_t* __restrict__ sizes) {
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < ns;
       s += (uint64_t)gridDim.x * blockDim.x) {
    if (fo[s + 1] != fo[s]) {
      gs[fo[s]] = (uint32_t)s;
      boff[fo[s]] = bo[s];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    boff[fo[ns]] = bo[ns];
    sizes[0] = fo[ns];
    sizes[1] = bo[ns];
    sizes[2] = co[ns];
  }
}

// sort keys of the wide arrays: (segment << rbits) | wide_radius for a
// candidate, all ones below the segment for the slack past its count (it
// sorts to the segment's end), and the digit histograms of the sort;
// word_ib >= 0: the sort starts on packed words (key << word_ib) | position
__global__ __launch_bounds__(256) void k_w_keys(const uint32_t* __restrict__ gs,
                                                const uint64_t* __restrict__ boff, uint32_t nG,
                                                const uint64_t* __restrict__ cand_off,
                                                const uint32_t* __restrict__ cand_cnt,
                                                const double* __restrict__ rad, int rbits,
                                                int npass, int word_ib,
                                                uint64_t* __restrict__ keys,
                                                uint32_t* __restrict__ ghist) {
  __shared__ uint32_t h[kRsMaxPass * 256];
  for (int i = threadIdx.x; i < kRsMaxPass * 256; i += 256) h[i] = 0u;
  __syncthreads();
  const uint64_t tb = boff[nG];
  for (uint64_t base = (uint64_t)blockIdx.x * 256; base < tb; base += (uint64_t)gridDim.x * 256) {
    const uint64_t p = base + threadIdx.x;
    const bool valid = p < tb;
    uint64_t key = 0;
    if (valid) {
      uint32_t lo = 0, hi = nG - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= p) lo = mid;
        else hi = mid - 1;
      }
      const uint64_t k = p - boff[lo];
      const uint32_t s = gs[lo];
      const uint64_t t = k < cand_cnt[s] ? wide_radius(rad[cand_off[s] + k], kRadSpan - rbits)
                                         : (1ull << rbits) - 1ull;
      key = ((uint64_t)lo << rbits) | t;
      keys[p] = word_ib >= 0 ? ((key << word_ib) | p) : key;
    }
    wave_digit_hist(key, valid, npass, h);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npass * 256; i += 256)
    if (h[i]) atomicAdd(&ghist[i], h[i]);
}

// sorted position p: its candidate (the sort's payload is the input position,
// whose segment is p's own): whole radius, particle, velocity and mass, and
// the sort key for the tie runs
__global__ void k_w_gather(const uint64_t* __restrict__ words, int ib, int rbits,
                           const uint32_t* __restrict__ gs, const uint64_t* __restrict__ boff,
                           uint32_t nG, const uint64_t* __restrict__ cand_off,
                           const uint32_t* __restrict__ cand_cnt,
                           const uint32_t* __restrict__ cand, const double* __restrict__ rad,
                           const float4* __restrict__ vq, uint64_t* __restrict__ K,
                           uint32_t* __restrict__ I, float4* __restrict__ V,
                           uint64_t* __restrict__ Kt) {
  const uint64_t tb = boff[nG];
  const uint64_t im = (1ull << ib) - 1ull;
  for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < tb;
       p += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = nG - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (boff[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t s = gs[lo];
    const uint64_t k = (words[p] & im) - boff[lo];  // the input position's place in the segment
    if (p - boff[lo] >= cand_cnt[s]) continue;      // slack at the segment's end
    const uint64_t slot = cand_off[s] + k;
    const uint64_t rb = (uint64_t)__double_as_longlong(rad[slot]);
    K[p] = rb;
    I[p] = cand[slot];
    V[p] = vq[slot];
    Kt[p] = ((uint64_t)lo << rbits) | wide_radius(rad[slot], kRadSpan - rbits);
  }
}

// runs of equal sort keys (within a segment): by (radius, index), insertion
// by the run's first thread; a run longer than kShortTie marks its structure
// for the one-workgroup path (mode 2)
__global__ void k_w_ties(const uint32_t* __restrict__ gs, const uint64_t* __restrict__ boff,
                         uint32_t nG, const uint32_t* __restrict__ cand_cnt,
                         const uint64_t* __restrict__ Kt, uint64_t* __restrict__ K,
                         uint32_t* __restrict__ I, float4* __restrict__ V,
                         uint32_t* __restrict__ mode) {
  const uint64_t tb = boff[nG];
  for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < tb;
       p += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = nG - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (boff[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const uint64_t b0 = boff[lo], end = b0 + cand_cnt[gs[lo]];
    if (p >= end) continue;
    if (p > b0 && Kt[p - 1] == Kt[p]) continue;  // not a run start
    uint64_t e = p + 1;
    while (e < end && Kt[e] == Kt[p]) ++e;
    if (e - p == 1) continue;
    if (e - p > kShortTie) {
      mode[gs[lo]] = 2u;
      continue;
    }
    for (uint64_t q = p + 1; q < e; ++q) {
      const uint64_t kq = K[q];
      const uint32_t iq = I[q];
      const float4 vv = V[q];
      uint64_t r = q;
      while (r > p && (K[r - 1] > kq || (K[r - 1] == kq && I[r - 1] > iq))) {
        K[r] = K[r - 1];
        I[r] = I[r - 1];
        V[r] = V[r - 1];
        --r;
      }
      K[r] = kq;
      I[r] = iq;
      V[r] = vv;
    }
  }
}

// state of the wide set after the sort: the view's candidates in radius
// order, every structure active with all its candidates (or handed to the
// one-workgroup path)
__global__ void k_w_start(const uint32_t* __restrict__ gs, const uint64_t* __restrict__ boff,
                          uint32_t nG, const uint64_t* __restrict__ cand_off,
                          const uint32_t* __restrict__ cand_cnt, const uint32_t* __restrict__ I,
                          const uint32_t* __restrict__ mode, uint32_t* __restrict__ cand,
                          uint32_t* __restrict__ na, uint32_t* __restrict__ act) {
  const uint64_t tb = boff[nG];
  for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < tb;
       p += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = nG - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (boff[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t s = gs[lo];
    const uint64_t k = p - boff[lo];
    if (k == 0) {
      const bool on = mode[s] == 1u && cand_cnt[s] > 0;
      na[lo] = on ? cand_cnt[s] : 0u;
      act[lo] = on ? 1u : 0u;
    }
    if (k < cand_cnt[s] && mode[s] == 1u) cand[cand_off[s] + k] = I[p];
  }
}

// this round's chunk table over the active segments (one workgroup)
__global__ __launch_bounds__(kHT) void k_w_chunks(const uint32_t* __restrict__ na,
                                                  const uint32_t* __restrict__ act, uint32_t nG,
                                                  uint32_t* __restrict__ cofs) {
  __shared__ double red[kHW];
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < nG; c0 += kHT) {
    const uint32_t g = c0 + threadIdx.x;
    const uint32_t v = (g < nG && act[g]) ? (na[g] + kWC - 1) / kWC : 0u;
    double tot = 0.0;
    const double inc = block_scan((double)v, red, &tot);
    if (g < nG) cofs[g] = carry + (uint32_t)inc - v;
    carry += (uint32_t)tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) cofs[nG] = carry;
}

// per chunk: the sums of m vx, m vy, m vz and m (each thread its kWE
// particles in row order, then the workgroup's fixed tree)
__global__ __launch_bounds__(kWT) void k_w_vel(const uint32_t* __restrict__ cofs, uint32_t nG,
                                               const uint64_t* __restrict__ boff,
                                               const uint32_t* __restrict__ na,
                                               const float4* __restrict__ V, PartIn P,
                                               double* __restrict__ part) {
  __shared__ double red[kWT / 64];
  uint32_t g, c;
  if (!chunk_of(cofs, nG, blockIdx.x, &g, &c)) return;
  const uint64_t k0 = (uint64_t)c * kWC, n = na[g], b0 = boff[g];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, sm = 0.0;
#pragma unroll 4
  for (int e = 0; e < kWE; ++e) {
    const uint64_t k = k0 + (uint64_t)e * kWT + threadIdx.x;
    if (k < n) {
      const float4 q = V[b0 + k];
      const double m = vmass(P, q);
      s0 += m * (double)q.x;
      s1 += m * (double)q.y;
      s2 += m * (double)q.z;
      sm += m;
    }
  }
  s0 = block_sum<kWT>(s0, red);
  s1 = block_sum<kWT>(s1, red);
  s2 = block_sum<kWT>(s2, red);
  sm = block_sum<kWT>(sm, red);
  if (threadIdx.x == 0) {
    double* o = part + 4 * (uint64_t)blockIdx.x;
    o[0] = s0;
    o[1] = s1;
    o[2] = s2;
    o[3] = sm;
  }
}

// per active segment (one wave): the halo velocity from its chunks' sums, and
// the exclusive offsets of its chunks' masses, in chunk order
__global__ void k_w_seg_vel(const uint32_t* __restrict__ cofs, uint32_t nG,
                            const uint32_t* __restrict__ act, const double* __restrict__ part,
                            double* __restrict__ vh, double* __restrict__ moff) {
  const uint32_t g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = __lane_id();
  if (g >= nG || !act[g]) return;
  const uint32_t a = cofs[g], e = cofs[g + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, carry = 0.0;
  for (uint32_t c0 = a; c0 < e; c0 += 64) {
    const uint32_t c = c0 + lane;
    double m = 0.0;
    if (c < e) {
      s0 += part[4 * (uint64_t)c];
      s1 += part[4 * (uint64_t)c + 1];
      s2 += part[4 * (uint64_t)c + 2];
      m = part[4 * (uint64_t)c + 3];
    }
    double inc = m;
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    double exc = __shfl_up(inc, 1);
    if (lane == 0) exc = 0.0;
    if (c < e) moff[c] = carry + exc;
    carry += __shfl(inc, 63);
  }
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o);
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
  }
  if (lane == 0) {
    vh[3 * (uint64_t)g] = s0 / carry;
    vh[3 * (uint64_t)g + 1] = s1 / carry;
    vh[3 * (uint64_t)g + 2] = s2 / carry;
  }
}

// LDS slot of chunk element i: one double of padding per 16, so that a
// thread reading its kWE consecutive elements and the lanes of a wave hit
// different banks
__device__ inline int wpad(int i) { return i + (i >> 4); }
constexpr int kWPad = kWC + kWC / 16;

// the exclusive suffix over the workgroup's threads (threads after this one)
// of one value per thread, with one barrier
template <int BT>
__device__ inline double block_esuffix(double x, double* red) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  double inc = x;  // inclusive suffix within the wave
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_down(inc, o);
    if (lane + o < 64) inc += y;
  }
  double exc = __shfl_down(inc, 1);
  if (lane == 63) exc = 0.0;
  if (lane == 0) red[w] = inc;
  __syncthreads();
  double after = 0.0;
  for (int i = BT / 64 - 1; i > w; --i) after += red[i];
  return after + exc;
}

// per chunk: the enclosed masses (each thread scans its kWE consecutive
// particles, the threads' sums are scanned over the workgroup, the chunk's
// offset from the segment's chunks before it), M, and the last particle of
// the chunk dense enough
__global__ __launch_bounds__(kWT) void k_w_enc(const uint32_t* __restrict__ cofs, uint32_t nG,
                                               const uint64_t* __restrict__ boff,
                                               const uint32_t* __restrict__ na,
                                               const uint64_t* __restrict__ K,
                                               const float4* __restrict__ V, PartIn P,
                                               const double* __restrict__ moff, double rho_thr,
                                               double* __restrict__ M,
                                               int64_t* __restrict__ vpart) {
  __shared__ double sv[kWPad];
  __shared__ double red[2][kWT / 64];
  __shared__ int64_t redi[kWT / 64];
  uint32_t g, c;
  if (!chunk_of(cofs, nG, blockIdx.x, &g, &c)) return;
  const uint64_t k0 = (uint64_t)c * kWC, n = na[g], b0 = boff[g];
  for (int e = 0; e < kWE; ++e) {
    const int i = e * kWT + threadIdx.x;
    const uint64_t k = k0 + i;
    sv[wpad(i)] = k < n ? vmass(P, V[b0 + k]) : 0.0;
  }
  __syncthreads();
  double pre[kWE];
  double run = 0.0;
#pragma unroll
  for (int e = 0; e < kWE; ++e) {
    run += sv[wpad(threadIdx.x * kWE + e)];
    pre[e] = run;
  }
  double tot = 0.0;
  const double base = moff[blockIdx.x] + block_escan1<kWT>(run, red, 0, &tot);
  __syncthreads();  // every thread's reads of sv are done
#pragma unroll
  for (int e = 0; e < kWE; ++e) sv[wpad(threadIdx.x * kWE + e)] = base + pre[e];
  __syncthreads();
  int64_t vl = -1;
  for (int e = 0; e < kWE; ++e) {
    const int i = e * kWT + threadIdx.x;
    const uint64_t k = k0 + i;
    if (k < n) {
      const double inc = sv[wpad(i)];
      M[b0 + k] = inc;
      const double r = __longlong_as_double((long long)K[b0 + k]);
      const double dens = inc / (4.0 / 3.0 * M_PI * (r * r * r));
      if (dens >= rho_thr) vl = (int64_t)k;
    }
  }
  vl = block_max_i64<kWT>(vl, redi);
  if (threadIdx.x == 0) vpart[blockIdx.x] = vl;
}

// per active segment (one wave): the last particle dense enough over its
// chunks; none: the halo dissolves (its results written); else r_vir and
// M(<r_vir) of the round
__global__ void k_w_seg_v(const uint32_t* __restrict__ cofs, uint32_t nG,
                          const uint32_t* __restrict__ gs, const uint64_t* __restrict__ boff,
                          uint32_t* __restrict__ act, const int64_t* __restrict__ vpart,
                          const uint64_t* __restrict__ K, const double* __restrict__ M,
                          const double* __restrict__ vh, uint32_t it,
                          int64_t* __restrict__ vseg, double* __restrict__ rvseg,
                          double* __restrict__ mvseg, uint32_t* __restrict__ member_cnt,
                          double* __restrict__ r_vir_out, double* __restrict__ m_vir_out,
                          double* __restrict__ vel_out, uint32_t* __restrict__ iters_out) {
  const uint32_t g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = __lane_id();
  if (g >= nG || !act[g]) return;
  int64_t v = -1;
  for (uint32_t c = cofs[g] + lane; c < cofs[g + 1]; c += 64) v = vpart[c] > v ? vpart[c] : v;
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t y = __shfl_xor(v, o);
    v = y > v ? y : v;
  }
  if (lane != 0) return;
  vseg[g] = v;
  if (v < 0) {  // never dense enough: the halo dissolves
    const uint32_t s = gs[g];
    act[g] = 0;
    member_cnt[s] = 0;
    r_vir_out[s] = 0.0;
    m_vir_out[s] = 0.0;
    for (int d = 0; d < 3; ++d) vel_out[3 * (uint64_t)s + d] = vh[3 * (uint64_t)g + d];
    iters_out[s] = it;
    return;
  }
  rvseg[g] = __longlong_as_double((long long)K[boff[g] + v]);
  mvseg[g] = M[boff[g] + v];
}

// the App. A term of particle k < v: M_k (1/r_k - 1/r_{k+1})
__device__ inline double tail_term(const uint64_t* K, const double* M, uint64_t k) {
  const double r0 = __longlong_as_double((long long)K[k]);
  const double r1 = __longlong_as_double((long long)K[k + 1]);
  return M[k] * (1.0 / r0 - 1.0 / r1);
}

// per chunk: the sum of its terms below v (each thread its kWE consecutive
// ones from the top, then the workgroup's fixed tree); the terms are formed
// from coalesced loads into LDS first, as in k_w_tail2 (the terms are not
// negative, so those past v add zeros that change no sum)
__global__ __launch_bounds__(kWT) void k_w_tail1(const uint32_t* __restrict__ cofs, uint32_t nG,
                                                 const uint64_t* __restrict__ boff,
                                                 const uint32_t* __restrict__ act,
                                                 const int64_t* __restrict__ vseg,
                                                 const uint64_t* __restrict__ K,
                                                 const double* __restrict__ M,
                                                 double* __restrict__ ttot) {
  __shared__ double sv[kWPad];
  __shared__ double red[kWT / 64];
  uint32_t g, c;
  if (!chunk_of(cofs, nG, blockIdx.x, &g, &c)) return;
  if (!act[g]) return;
  const uint64_t k0 = (uint64_t)c * kWC, b0 = boff[g];
  const int64_t v = vseg[g];
  if ((int64_t)k0 >= v) {  // the whole chunk at or past v (uniform): no terms
    if (threadIdx.x == 0) ttot[blockIdx.x] = 0.0;
    return;
  }
  for (int e = 0; e < kWE; ++e) {
    const int i = e * kWT + threadIdx.x;
    const uint64_t k = k0 + i;
    sv[wpad(i)] = (int64_t)k < v ? tail_term(K + b0, M + b0, k) : 0.0;
  }
  __syncthreads();
  double run = 0.0;
#pragma unroll
  for (int e = kWE - 1; e >= 0; --e) run += sv[wpad(threadIdx.x * kWE + e)];
  run = block_sum<kWT>(run, red);
  if (threadIdx.x == 0) ttot[blockIdx.x] = run;
}

// per active segment (one wave): each chunk's offset, the sum of the terms
// of the chunks after it
__global__ void k_w_seg_tail(const uint32_t* __restrict__ cofs, uint32_t nG,
                             const uint32_t* __restrict__ act, const double* __restrict__ ttot,
                             double* __restrict__ toff) {
  const uint32_t g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = __lane_id();
  if (g >= nG || !act[g]) return;
  const int64_t a = cofs[g], e = cofs[g + 1];
  double carry = 0.0;
  for (int64_t c0 = 0; c0 < e - a; c0 += 64) {
    const int64_t c = e - 1 - (c0 + lane);  // from the last chunk down
    const double x = c >= a ? ttot[c] : 0.0;
    double inc = x;
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    double exc = __shfl_up(inc, 1);
    if (lane == 0) exc = 0.0;
    if (c >= a) toff[c] = carry + exc;
    carry += __shfl(inc, 63);
  }
}

// per chunk: T_k = the sum of the terms j in [k, v) (each thread sums its
// kWE consecutive terms from the top, the threads after it in the workgroup
// and the chunks after this one come first)
__global__ __launch_bounds__(kWT) void k_w_tail2(const uint32_t* __restrict__ cofs, uint32_t nG,
                                                 const uint64_t* __restrict__ boff,
                                                 const uint32_t* __restrict__ act,
                                                 const int64_t* __restrict__ vseg,
                                                 const uint64_t* __restrict__ K,
                                                 const double* __restrict__ M,
                                                 const double* __restrict__ toff,
                                                 double* __restrict__ T) {
  __shared__ double sv[kWPad];
  __shared__ double red[kWT / 64];
  uint32_t g, c;
  if (!chunk_of(cofs, nG, blockIdx.x, &g, &c)) return;
  if (!act[g]) return;
  const uint64_t k0 = (uint64_t)c * kWC, b0 = boff[g];
  const int64_t v = vseg[g];
  if ((int64_t)k0 >= v) return;  // the whole chunk at or past v (uniform)
  for (int e = 0; e < kWE; ++e) {
    const int i = e * kWT + threadIdx.x;
    const uint64_t k = k0 + i;
    sv[wpad(i)] = (int64_t)k < v ? tail_term(K + b0, M + b0, k) : 0.0;
  }
  __syncthreads();
  double pre[kWE];
  double run = 0.0;
#pragma unroll
  for (int e = kWE - 1; e >= 0; --e) {
    run += sv[wpad(threadIdx.x * kWE + e)];
    pre[e] = run;
  }
  const double base = toff[blockIdx.x] + block_esuffix<kWT>(run, red);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kWE; ++e) sv[wpad(threadIdx.x * kWE + e)] = base + pre[e];
  __syncthreads();
  for (int e = 0; e < kWE; ++e) {
    const int i = e * kWT + threadIdx.x;
    const uint64_t k = k0 + i;
    if ((int64_t)k < v) T[b0 + k] = sv[wpad(i)];
  }
}

// per chunk: the escape test of every particle (as the one-workgroup path
// writes it), the kept ones as ballot words per row and wave, and the
// chunk's kept and unbound counts
__global__ __launch_bounds__(kWT) void k_w_esc1(const uint32_t* __restrict__ cofs, uint32_t nG,
                                                const uint64_t* __restrict__ boff,
                                                const uint32_t* __restrict__ na,
                                                const uint32_t* __restrict__ act,
                                                const int64_t* __restrict__ vseg,
                                                const double* __restrict__ rvseg,
                                                const double* __restrict__ mvseg,
                                                const double* __restrict__ vh, double G,
                                                const uint64_t* __restrict__ K,
                                                const float4* __restrict__ V,
                                                const double* __restrict__ T,
                                                uint64_t* __restrict__ kbits,
                                                uint32_t* __restrict__ ckeep,
                                                uint32_t* __restrict__ cgone) {
  __shared__ uint32_t wk[kWT / 64], wg[kWT / 64];
  uint32_t g, c;
  if (!chunk_of(cofs, nG, blockIdx.x, &g, &c)) return;
  if (!act[g]) return;
  const uint64_t k0 = (uint64_t)c * kWC, n = na[g], b0 = boff[g];
  const int64_t v = vseg[g];
  const uint64_t nv = (uint64_t)v;
  const double rv = rvseg[g], mv = mvseg[g];
  const double vx = vh[3 * (uint64_t)g], vy = vh[3 * (uint64_t)g + 1], vz = vh[3 * (uint64_t)g + 2];
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint32_t nk = 0, ng = 0;
  for (int e = 0; e < kWE; ++e) {
    const uint64_t k = k0 + (uint64_t)e * kWT + threadIdx.x;
    bool gone = false;
    if (k < n) {
      const double r = __longlong_as_double((long long)K[b0 + k]);
      const float4 q = V[b0 + k];
      const double phi = (int64_t)k <= v ? -G * ((k < nv ? T[b0 + k] : 0.0) + mv / rv) : -G * mv / r;
      const double dx = (double)q.x - vx;
      const double dy = (double)q.y - vy;
      const double dz = (double)q.z - vz;
      const double ke = 0.5 * (dx * dx + dy * dy + dz * dz);
      gone = ke > fabs(phi);
    }
    const uint64_t kb = __ballot(k < n && !gone);
    const uint64_t gb = __ballot(gone);
    if (lane == 0) kbits[((uint64_t)blockIdx.x * kWE + e) * (kWT / 64) + w] = kb;
    nk += (uint32_t)__popcll(kb);
    ng += (uint32_t)__popcll(gb);
  }
  if (lane == 0) {
    wk[w] = nk;
    wg[w] = ng;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0, b = 0;
    for (int i = 0; i < kWT / 64; ++i) {
      a += wk[i];
      b += wg[i];
    }
    ckeep[blockIdx.x] = a;
    cgone[blockIdx.x] = b;
  }
}

// per active segment (one wave): the kept particles' chunk offsets; nothing
// unbound: the halo converged (the first v + 1 particles; their list and mass
// are written at the end from this round's arrays, parity `par`); the last
// round, or nothing kept: it ends without members; else its particles are the
// kept ones.  Counts the segments still active.
__global__ void k_w_seg_esc(const uint32_t* __restrict__ cofs, uint32_t nG,
                            const uint32_t* __restrict__ gs, uint32_t* __restrict__ act,
                            const uint32_t* __restrict__ ckeep, const uint32_t* __restrict__ cgone,
                            const int64_t* __restrict__ vseg, const double* __restrict__ rvseg,
                            const double* __restrict__ vh, uint32_t it, uint32_t max_iter,
                            uint32_t par, uint32_t* __restrict__ koff, uint32_t* __restrict__ na,
                            uint32_t* __restrict__ nmem, uint32_t* __restrict__ mpar,
                            uint32_t* __restrict__ nact, uint32_t* __restrict__ member_cnt,
                            double* __restrict__ r_vir_out, double* __restrict__ m_vir_out,
                            double* __restrict__ vel_out, uint32_t* __restrict__ iters_out) {
  const uint32_t g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = __lane_id();
  if (g >= nG || !act[g]) return;
  const uint32_t a = cofs[g], e = cofs[g + 1];
  uint32_t carry = 0, gone = 0;
  for (uint32_t c0 = a; c0 < e; c0 += 64) {
    const uint32_t c = c0 + lane;
    const uint32_t x = c < e ? ckeep[c] : 0u;
    gone += c < e ? cgone[c] : 0u;
    uint32_t inc = x;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (c < e) koff[c] = carry + inc - x;
    carry += __shfl(inc, 63);
  }
  for (int o = 32; o > 0; o >>= 1) gone += __shfl_xor(gone, o);
  if (lane != 0) return;
  const uint32_t s = gs[g];
  const bool conv = gone == 0;
  // ends: converged, the last round, or every particle unbound (no members)
  if (conv || it == max_iter || carry == 0) {
    act[g] = 0;
    member_cnt[s] = conv ? (uint32_t)(vseg[g] + 1) : 0u;
    r_vir_out[s] = conv ? rvseg[g] : 0.0;
    if (!conv) m_vir_out[s] = 0.0;
    for (int d = 0; d < 3; ++d) vel_out[3 * (uint64_t)s + d] = vh[3 * (uint64_t)g + d];
    iters_out[s] = it;
    nmem[g] = conv ? (uint32_t)(vseg[g] + 1) : 0u;
    mpar[g] = par;
  } else {
    na[g] = carry;
    atomicAdd(nact, 1u);
  }
}

// per chunk of a segment still active: its kept particles to the other
// arrays, in order, at the chunk's offset
__global__ __launch_bounds__(kWT) void k_w_esc2(const uint32_t* __restrict__ cofs, uint32_t nG,
                                                const uint64_t* __restrict__ boff,
                                                const uint32_t* __restrict__ act,
                                                const uint64_t* __restrict__ kbits,
                                                const uint32_t* __restrict__ koff,
                                                const uint64_t* __restrict__ K,
                                                const uint32_t* __restrict__ I,
                                                const float4* __restrict__ V,
                                                uint64_t* __restrict__ Kn, uint32_t* __restrict__ In,
                                                float4* __restrict__ Vn) {
  __shared__ uint64_t kb[kWE * (kWT / 64)];
  uint32_t g, c;
  if (!chunk_of(cofs, nG, blockIdx.x, &g, &c)) return;
  if (!act[g]) return;
  if (threadIdx.x < kWE * (kWT / 64))
    kb[threadIdx.x] = kbits[(uint64_t)blockIdx.x * kWE * (kWT / 64) + threadIdx.x];
  __syncthreads();
  const uint64_t k0 = (uint64_t)c * kWC, b0 = boff[g];
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint32_t before = 0;  // kept particles of the rows before this one
  for (int e = 0; e < kWE; ++e) {
    const uint64_t mine = kb[e * (kWT / 64) + w];
    uint32_t wb = 0, rowall = 0;
    for (int i = 0; i < kWT / 64; ++i) {
      const uint32_t cnt = (uint32_t)__popcll(kb[e * (kWT / 64) + i]);
      if (i < w) wb += cnt;
      rowall += cnt;
    }
    if ((mine >> lane) & 1ull) {
      const uint64_t k = k0 + (uint64_t)e * kWT + threadIdx.x;
      const uint64_t at = b0 + koff[blockIdx.x] + before + wb +
                          (uint32_t)__popcll(mine & lanes_below());
      Kn[at] = K[b0 + k];
      In[at] = I[b0 + k];
      Vn[at] = V[b0 + k];
    }
    before += rowall;
  }
}

// the members of the converged segments: per chunk of their first nmem
// particles (in the arrays of their last round), the list and the sum of
// their masses
__global__ __launch_bounds__(kWT) void k_w_members(const uint32_t* __restrict__ cofs, uint32_t nG,
                                                   const uint32_t* __restrict__ gs,
                                                   const uint64_t* __restrict__ boff,
                                                   const uint32_t* __restrict__ nmem,
                                                   const uint32_t* __restrict__ mpar,
                                                   const uint64_t* __restrict__ cand_off,
                                                   const uint32_t* __restrict__ I0,
                                                   const uint32_t* __restrict__ I1,
                                                   const float4* __restrict__ V0,
                                                   const float4* __restrict__ V1, PartIn P,
                                                   uint32_t* __restrict__ member,
                                                   double* __restrict__ part) {
  __shared__ double red[kWT / 64];
  uint32_t g, c;
  if (!chunk_of(cofs, nG, blockIdx.x, &g, &c)) return;
  const uint64_t k0 = (uint64_t)c * kWC, n = nmem[g], b0 = boff[g];
  const uint32_t* I = mpar[g] ? I1 : I0;
  const float4* V = mpar[g] ? V1 : V0;
  uint32_t* out = member + cand_off[gs[g]];
  double sm = 0.0;
  for (int e = 0; e < kWE; ++e) {
    const uint64_t k = k0 + (uint64_t)e * kWT + threadIdx.x;
    if (k < n) {
      out[k] = I[b0 + k];
      sm += vmass(P, V[b0 + k]);
    }
  }
  sm = block_sum<kWT>(sm, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sm;
}

__global__ void k_w_seg_mvir(const uint32_t* __restrict__ cofs, uint32_t nG,
                             const uint32_t* __restrict__ gs, const uint32_t* __restrict__ nmem,
                             const double* __restrict__ part, double* __restrict__ m_vir_out) {
  const uint32_t g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = __lane_id();
  if (g >= nG || nmem[g] == 0) return;
  double sm = 0.0;
  for (uint32_t c = cofs[g] + lane; c < cofs[g + 1]; c += 64) sm += part[c];
  for (int o = 32; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
  if (lane == 0) m_vir_out[gs[g]] = sm;
}

// a candidate's distance from the centre c, clamped below at half a position
// quantum (as everywhere else in this file)
__device__ inline double cand_radius(const PartIn& P, uint32_t i, const double* c) {
  double x, y, z;
  ppos(P, i, x, y, z);
  const double dx = mimg(x - c[0]);
  const double dy = mimg(y - c[1]);
  const double dz = mimg(z - c[2]);
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (r < kHalfQuantum) r = kHalfQuantum;
  return r;
}

// bounds of the wide set, per segment
__global__ void k_w_bounds(const uint64_t* __restrict__ boff, uint32_t nG,
                           uint32_t* __restrict__ nb) {
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nG; g += gridDim.x * blockDim.x)
    nb[g] = (uint32_t)(boff[g + 1] - boff[g]);
}

// The candidates of the wide set (but the coarse substructures) collected by
// the whole grid: a chunk is kWC of a structure's possible candidates, a
// host's isodensity list (all of them candidates, at their own slots) or the
// particles of a substructure's query cells (every block resolves the same
// cells in the same order); a substructure's candidates get their slots from
// one atomic per block (in no particular order: the unbinding orders them).
// Each candidate's radius, velocity and mass are written beside it.
__global__ __launch_bounds__(kWT) void k_w_collect(
    const uint32_t* __restrict__ cofs, uint32_t nG, const uint32_t* __restrict__ gs,
    const int32_t* __restrict__ s_depth, const uint8_t* __restrict__ coarse,
    const double* __restrict__ centre, const double* __restrict__ radius,
    const uint64_t* __restrict__ iso_off, const uint32_t* __restrict__ iso_cnt,
    const uint32_t* __restrict__ iso_list, const LevCells LC, const uint32_t* __restrict__ order,
    PartIn P, const uint64_t* __restrict__ cand_off, uint32_t* __restrict__ wcnt,
    uint32_t* __restrict__ cand, double* __restrict__ rad, float4* __restrict__ vq) {
  __shared__ uint32_t qa[kCoarseMax], qc[kCoarseMax], qo[kCoarseMax + 1];
  __shared__ double red[kWT / 64];
  __shared__ uint32_t base;
  uint32_t g, c;
  if (!chunk_of(cofs, nG, blockIdx.x, &g, &c)) return;
  const uint32_t s = gs[g];
  if (coarse[s]) return;
  const double* ce = centre + 3 * (uint64_t)s;
  const uint64_t k0 = (uint64_t)c * kWC;
  uint32_t* out = cand + cand_off[s];
  double* ro = rad + cand_off[s];
  float4* vo = vq + cand_off[s];
  if (s_depth[s] == 0) {  // a host: its isodensity list
    const uint32_t n = iso_cnt[s];
    const uint32_t* in = iso_list + iso_off[s];
    for (int e = 0; e < kWE; ++e) {
      const uint64_t k = k0 + (uint64_t)e * kWT + threadIdx.x;
      if (k < n) {
        const uint32_t i = in[k];
        out[k] = i;
        ro[k] = cand_radius(P, i, ce);
        vo[k] = pvel(P, i);
      }
    }
    return;
  }
  const double R = radius[s];
  const double R2 = R * R;
  const int L = query_level(LC, R);
  int64_t lo[3], nc[3];
  cube_of(ce, R, LC.g + L, lo, nc);
  const uint64_t ncube = (uint64_t)nc[0] * (uint64_t)nc[1] * (uint64_t)nc[2];
  uint32_t nq;
  if (ncube <= kQCells) {
    nq = fine_cells<kWT>(LC, L, lo, nc, ncube, qa, qc);
  } else {  // level 0, at most kCoarseMax cube cells (else the structure is coarse)
    nq = (uint32_t)ncube;
    for (uint32_t k = threadIdx.x; k < nq; k += kWT) {
      const uint64_t cell = cube_cell(lo, nc, k, LC.g);
      qa[k] = LC.start[0][cell];
      qc[k] = LC.count[0][cell];
    }
    __syncthreads();
  }
  {  // the cells' particle offsets, in cell order
    uint32_t carry = 0;
    for (uint32_t k0c = 0; k0c < nq; k0c += kWT) {
      const uint32_t k = k0c + threadIdx.x;
      const uint32_t q = k < nq ? qc[k] : 0u;
      double tot = 0.0;
      const double inc = block_scan<kWT>((double)q, red, &tot);
      if (k < nq) qo[k] = carry + (uint32_t)inc - q;
      carry += (uint32_t)tot;
    }
    if (threadIdx.x == 0) qo[nq] = carry;
  }
  __syncthreads();
  const uint32_t total = qo[nq];
  uint32_t pi[kWE];
  uint32_t mask = 0, cnt = 0;
#pragma unroll
  for (int e = 0; e < kWE; ++e) {
    const uint64_t k = k0 + (uint64_t)e * kWT + threadIdx.x;
    pi[e] = 0;
    if (k < total) {
      uint32_t a = 0, b = nq - 1;  // the last cell whose offset is at most k
      while (a < b) {
        const uint32_t mid = (a + b + 1) >> 1;
        if (qo[mid] <= k) a = mid;
        else b = mid - 1;
      }
      const uint32_t i = order[qa[a] + (uint32_t)(k - qo[a])];
      pi[e] = i;
      double x, y, z;
      ppos(P, i, x, y, z);
      const double dx = mimg(x - ce[0]);
      const double dy = mimg(y - ce[1]);
      const double dz = mimg(z - ce[2]);
      if (dx * dx + dy * dy + dz * dz <= R2) {
        mask |= 1u << e;
        ++cnt;
      }
    }
  }
  double tot = 0.0;
  const double inc = block_scan<kWT>((double)cnt, red, &tot);
  if (threadIdx.x == 0) base = atomicAdd(&wcnt[g], (uint32_t)tot);
  __syncthreads();
  uint32_t at = base + (uint32_t)inc - cnt;
#pragma unroll
  for (int e = 0; e < kWE; ++e) {
    if ((mask >> e) & 1u) {
      const uint32_t i = pi[e];
      out[at] = i;
      ro[at] = cand_radius(P, i, ce);
      vo[at] = pvel(P, i);
      ++at;
    }
  }
}

// the candidate counts of the wide set collected by the grid
__global__ void k_w_setcnt(const uint32_t* __restrict__ gs, uint32_t nG,
                           const int32_t* __restrict__ s_depth, const uint8_t* __restrict__ coarse,
                           const uint32_t* __restrict__ iso_cnt, const uint32_t* __restrict__ wcnt,
                           uint32_t* __restrict__ cand_cnt) {
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nG; g += gridDim.x * blockDim.x) {
    const uint32_t s = gs[g];
    if (coarse[s]) continue;
    cand_cnt[s] = s_depth[s] == 0 ? iso_cnt[s] : wcnt[g];
  }
}

// mode of every structure: 1 for the wide set (at least `big` possible
// candidates), else 0 (its own workgroup); a wide one with a long run of tied
// radii is set to 2 later (one wide workgroup)
__global__ void k_w_mode(const uint64_t* __restrict__ cand_off, uint64_t ns, uint64_t big,
                         uint32_t* __restrict__ mode) {
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < ns;
       s += (uint64_t)gridDim.x * blockDim.x)
    mode[s] = (cand_off[s + 1] - cand_off[s] >= big) ? 1u : 0u;
}

// the candidate count of each wide structure, by its place in the wide list
__global__ void k_w_counts(const uint32_t* __restrict__ gs, uint32_t nG,
                           const uint32_t* __restrict__ cand_cnt, uint32_t* __restrict__ wc) {
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nG; g += gridDim.x * blockDim.x)
    wc[g] = cand_cnt[gs[g]];
}

// the results of the wide structures without candidates
__global__ void k_w_empty(const uint32_t* __restrict__ gs, uint32_t nG,
                          const uint32_t* __restrict__ cand_cnt, const uint32_t* __restrict__ mode,
                          uint32_t* __restrict__ member_cnt, double* __restrict__ r_vir_out,
                          double* __restrict__ m_vir_out, double* __restrict__ vel_out,
                          uint32_t* __restrict__ iters_out) {
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nG; g += gridDim.x * blockDim.x) {
    const uint32_t s = gs[g];
    if (mode[s] != 1u || cand_cnt[s] != 0) continue;
    member_cnt[s] = 0;
    r_vir_out[s] = 0.0;
    m_vir_out[s] = 0.0;
    for (int d = 0; d < 3; ++d) vel_out[3 * (uint64_t)s + d] = 0.0;
    iters_out[s] = 0;
  }
}

}  // namespace

// the halo set of one hierarchy: device arrays in an arena of the context
struct Halos {
  Owned mem;
  uint64_t n = 0;
  unsigned long long* leafkey = nullptr;
  double *centre = nullptr, *radius = nullptr, *r_vir = nullptr, *m_vir = nullptr,
         *vel = nullptr;
  uint64_t* cand_off = nullptr;
  uint32_t *cand_cnt = nullptr, *cand = nullptr, *member_cnt = nullptr, *member = nullptr,
           *iters = nullptr;
};

// Unbinding of the wide set by the whole grid (the kernels above): sort,
// then rounds until no structure is active, reading the number still active
// after each round; the members' lists and masses at the end.
template <class AfterTies>
static void wide_unbind(Ctx* ctx, Ws& ws, uint32_t nG, uint64_t tb, uint64_t maxch,
                        const uint32_t* gs, const uint64_t* boff, uint32_t* mode,
                        const double* rad, const float4* vslot, const PartIn& P, double rho_thr,
                        double G, uint32_t max_iter, hipStream_t st, Halos* out,
                        AfterTies after_ties) {
  int gbits = 1;
  while ((1ull << gbits) < nG) ++gbits;
  int ib = 1;  // the index width of the sort's packed words
  while (ib < 32 && (1ull << ib) < tb) ++ib;
  int rbits = std::min(kRadiusBits, 64 - ib - gbits);
  if (rbits < kMinRadBits) rbits = kRadiusBits;
  if (rbits + gbits > 64)  // the sort key is (structure, radius part)
    throw Error{AHF_ELIMIT, "too many structures for the grid's unbinding (raise large_from)"};
  const SortPlan sp = sort_plan(tb, rbits + gbits);
  uint64_t* keys = ws.get<uint64_t>(tb);
  uint32_t* ghist = ws.get<uint32_t>(kRsMaxPass * 256);
  k_fill_u32<<<blocks_for(kRsMaxPass * 256), kHB, 0, st>>>(ghist, kRsMaxPass * 256, 0);
  HIP_LAUNCH_CHECK();
  const unsigned kb = std::min<unsigned>(blocks_for(tb), 2048u);
  k_w_keys<<<kb, 256, 0, st>>>(gs, boff, nG, out->cand_off, out->cand_cnt, rad, rbits,
                               sp.npass, sp.q == 0 ? sp.ib : -1, keys, ghist);
  HIP_LAUNCH_CHECK();
  const uint64_t* words = sort_keys(ctx, ws, keys, tb, sp, ghist, st, nullptr);
  uint64_t* Kb[2] = {ws.get<uint64_t>(tb), ws.get<uint64_t>(tb)};
  uint32_t* Ib[2] = {ws.get<uint32_t>(tb), ws.get<uint32_t>(tb)};
  float4* Vb[2] = {ws.get<float4>(tb), ws.get<float4>(tb)};
  uint64_t* Kt = ws.get<uint64_t>(tb);
  double* M = ws.get<double>(tb);
  double* T = ws.get<double>(tb);
  k_w_gather<<<blocks_for(tb), kHB, 0, st>>>(words, sp.ib, rbits, gs, boff, nG, out->cand_off,
                                             out->cand_cnt, out->cand, rad, vslot, Kb[0], Ib[0],
                                             Vb[0], Kt);
  HIP_LAUNCH_CHECK();
  k_w_ties<<<blocks_for(tb), kHB, 0, st>>>(gs, boff, nG, out->cand_cnt, Kt, Kb[0], Ib[0], Vb[0],
                                           mode);
  HIP_LAUNCH_CHECK();
  after_ties();  // the modes are final from here on
  uint32_t* na = ws.get<uint32_t>(nG);
  uint32_t* act = ws.get<uint32_t>(nG);
  uint32_t* nmem = ws.get<uint32_t>(nG);
  uint32_t* mpar = ws.get<uint32_t>(nG);
  uint32_t* cofs = ws.get<uint32_t>(nG + 1);
  uint32_t* nact = ws.get<uint32_t>(1);
  double* vh = ws.get<double>(3 * (uint64_t)nG);
  int64_t* vseg = ws.get<int64_t>(nG);
  double* rvseg = ws.get<double>(nG);
  double* mvseg = ws.get<double>(nG);
  double* part = ws.get<double>(4 * maxch);
  double* moff = ws.get<double>(maxch);
  int64_t* vpart = ws.get<int64_t>(maxch);
  double* ttot = ws.get<double>(maxch);
  double* toff = ws.get<double>(maxch);
  uint64_t* kbits = ws.get<uint64_t>(maxch * kWE * (kWT / 64));
  uint32_t* ckeep = ws.get<uint32_t>(maxch);
  uint32_t* cgone = ws.get<uint32_t>(maxch);
  uint32_t* koff = ws.get<uint32_t>(maxch);
  k_fill_u32<<<blocks_for(nG), kHB, 0, st>>>(nmem, nG, 0);
  // a segment without candidates has no position to set its state from
  k_fill_u32<<<blocks_for(nG), kHB, 0, st>>>(na, nG, 0);
  k_fill_u32<<<blocks_for(nG), kHB, 0, st>>>(act, nG, 0);
  HIP_LAUNCH_CHECK();
  k_w_start<<<blocks_for(tb), kHB, 0, st>>>(gs, boff, nG, out->cand_off, out->cand_cnt, Ib[0],
                                            mode, out->cand, na, act);
  HIP_LAUNCH_CHECK();
  k_w_empty<<<blocks_for(nG), kHB, 0, st>>>(gs, nG, out->cand_cnt, mode, out->member_cnt,
                                            out->r_vir, out->m_vir, out->vel, out->iters);
  HIP_LAUNCH_CHECK();
  const unsigned ch = (unsigned)maxch;
  const unsigned sg = (nG + 3) / 4;  // one wave per segment
  for (uint32_t it = 1; it <= max_iter; ++it) {
    const uint32_t par = (it - 1) & 1u;
    const uint64_t* K = Kb[par];
    const uint32_t* I = Ib[par];
    const float4* V = Vb[par];
    k_fill_u32<<<1, 64, 0, st>>>(nact, 1, 0);
    k_w_chunks<<<1, kHT, 0, st>>>(na, act, nG, cofs);
    k_w_vel<<<ch, kWT, 0, st>>>(cofs, nG, boff, na, V, P, part);
    k_w_seg_vel<<<sg, 256, 0, st>>>(cofs, nG, act, part, vh, moff);
    k_w_enc<<<ch, kWT, 0, st>>>(cofs, nG, boff, na, K, V, P, moff, rho_thr, M, vpart);
    k_w_seg_v<<<sg, 256, 0, st>>>(cofs, nG, gs, boff, act, vpart, K, M, vh, it, vseg, rvseg,
                                  mvseg, out->member_cnt, out->r_vir, out->m_vir, out->vel,
                                  out->iters);
    k_w_tail1<<<ch, kWT, 0, st>>>(cofs, nG, boff, act, vseg, K, M, ttot);
    k_w_seg_tail<<<sg, 256, 0, st>>>(cofs, nG, act, ttot, toff);
    k_w_tail2<<<ch, kWT, 0, st>>>(cofs, nG, boff, act, vseg, K, M, toff, T);
    k_w_esc1<<<ch, kWT, 0, st>>>(cofs, nG, boff, na, act, vseg, rvseg, mvseg, vh, G, K, V, T,
                                 kbits, ckeep, cgone);
    k_w_seg_esc<<<sg, 256, 0, st>>>(cofs, nG, gs, act, ckeep, cgone, vseg, rvseg, vh, it,
                                    max_iter, par, koff, na, nmem, mpar, nact, out->member_cnt,
                                    out->r_vir, out->m_vir, out->vel, out->iters);
    k_w_esc2<<<ch, kWT, 0, st>>>(cofs, nG, boff, act, kbits, koff, K, I, V, Kb[par ^ 1u],
                                 Ib[par ^ 1u], Vb[par ^ 1u]);
    HIP_LAUNCH_CHECK();
    // the host looks at the active count every kRoundsPerCheck rounds only,
    // so that the rounds in between go to the GPU without a wait (a round
    // after the last segment has ended has no chunk and changes nothing)
    if (it % kRoundsPerCheck != 0 && it != max_iter) continue;
    uint32_t still = 0;
    HIP_CHECK(hipMemcpyAsync(&still, nact, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    if (still == 0) break;
  }
  // the members of the converged ones and their mass
  k_w_chunks<<<1, kHT, 0, st>>>(nmem, nmem, nG, cofs);
  k_w_members<<<ch, kWT, 0, st>>>(cofs, nG, gs, boff, nmem, mpar, out->cand_off, Ib[0], Ib[1],
                                  Vb[0], Vb[1], P, out->member, part);
  k_w_seg_mvir<<<sg, 256, 0, st>>>(cofs, nG, gs, nmem, part, out->m_vir);
  HIP_LAUNCH_CHECK();
}

static void find_halos(Ctx* ctx, Ws& ws, const Hier* h, const ahf_particles& p, const float* vx,
                       const float* vy, const float* vz, double delta_vir, double G,
                       uint32_t max_iter, uint64_t large, hipStream_t st, Halos* out) {
  const uint64_t ns = h->nStruct;
  const size_t nlev = h->lev.size();
  out->n = ns;
  Owned& mem = out->mem;
  out->leafkey = mem.get<unsigned long long>(ns);
  out->centre = mem.get<double>(3 * ns);
  out->radius = mem.get<double>(ns);
  out->r_vir = mem.get<double>(ns);
  out->m_vir = mem.get<double>(ns);
  out->vel = mem.get<double>(3 * ns);
  out->cand_off = mem.get<uint64_t>(ns + 1);
  out->cand_cnt = mem.get<uint32_t>(ns);
  out->member_cnt = mem.get<uint32_t>(ns);
  out->iters = mem.get<uint32_t>(ns);
  if (ns == 0) {
    k_fill_u64<<<1, kHB, 0, st>>>(out->cand_off, 1, 0);
    HIP_LAUNCH_CHECK();
    out->cand = mem.get<uint32_t>(1);
    out->member = mem.get<uint32_t>(1);
    return;
  }
  const uint64_t n = h->n;
  PartIn P{p.x, p.y, p.z, p.fx, p.fy, p.fz, p.mass, p.mass_scalar, vx, vy, vz, nullptr};
  if (!ctx->dep_st) HIP_CHECK(hipStreamCreateWithFlags(&ctx->dep_st, hipStreamNonBlocking));
  hipStream_t s2 = ctx->dep_st;
  StreamEvents ev;
  {  // the particles' records, on the second stream beside the lists below:
     // every kernel from the centres on reads particles from them
    PRec* R = ws.get<PRec>(n ? n : 1);
    HIP_CHECK(hipEventRecord(ev.fork, st));
    HIP_CHECK(hipStreamWaitEvent(s2, ev.fork, 0));
    const unsigned nb = std::min<unsigned>(blocks_for(n ? n : 1), kStageBlocks);
    const bool F = P.fx && P.fy && P.fz;
    if (F && P.mass) k_stage<true, true><<<nb, kHB, 0, s2>>>(P, n, R);
    else if (F) k_stage<true, false><<<nb, kHB, 0, s2>>>(P, n, R);
    else if (P.mass) k_stage<false, true><<<nb, kHB, 0, s2>>>(P, n, R);
    else k_stage<false, false><<<nb, kHB, 0, s2>>>(P, n, R);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipEventRecord(ev.join, s2));
    P.R = R;
  }
  unsigned long long* leaf_min = ws.get<unsigned long long>(ns);
  uint32_t* leaf_cnt = ws.get<uint32_t>(ns);
  uint32_t* iso_cnt = ws.get<uint32_t>(ns);
  int32_t* iso_patch = ws.get<int32_t>(ns);
  int32_t* iso_level = ws.get<int32_t>(ns);
  uint64_t* leaf_off = ws.get<uint64_t>(ns + 1);
  uint64_t* iso_off = ws.get<uint64_t>(ns + 1);
  uint32_t* bound = ws.get<uint32_t>(ns);
  uint32_t* leaf_list = ws.get<uint32_t>(n ? n : 1);
  uint32_t* leaf_tmp = ws.get<uint32_t>(n ? n : 1);
  uint32_t* iso_list = ws.get<uint32_t>(n ? n : 1);
  k_fill_u64<<<blocks_for(ns), kHB, 0, st>>>(reinterpret_cast<uint64_t*>(out->leafkey), ns, 0);
  k_fill_u64<<<blocks_for(ns), kHB, 0, st>>>(reinterpret_cast<uint64_t*>(leaf_min), ns, ~0ull);
  k_fill_u32<<<blocks_for(ns), kHB, 0, st>>>(leaf_cnt, ns, 0);
  k_fill_u32<<<blocks_for(ns), kHB, 0, st>>>(iso_cnt, ns, 0);
  k_fill_u32<<<blocks_for(ns), kHB, 0, st>>>(reinterpret_cast<uint32_t*>(iso_patch), ns, ~0u);
  k_fill_u32<<<blocks_for(ns), kHB, 0, st>>>(reinterpret_cast<uint32_t*>(iso_level), ns, ~0u);
  HIP_LAUNCH_CHECK();
  // leaves, then the hosts' isodensity patches: bit L of isomask when the
  // boundary contour of level-L patches lies below delta_vir * rho_b
  for (size_t L = 1; L < nlev; ++L) {
    const Level& lv = h->lev[L];
    if (!lv.nPatch) continue;
    k_leaf<<<blocks_for(lv.nPatch), kHB, 0, st>>>((int)L, lv.patch_struct, lv.nPatch,
                                                  out->leafkey);
    HIP_LAUNCH_CHECK();
  }
  uint32_t isomask = 0;
  for (size_t L = 1; L < nlev && L < 32; ++L) {
    const double thr = (L - 1 == 0) ? h->prm.dom_ref : h->prm.ref_ref;
    const double rho = thr * std::pow(8.0, (double)(L - 1)) * std::pow(2.0, 3.0 * h->prm.g) /
                       (double)n;
    if (rho < delta_vir) isomask |= 1u << L;
  }
  for (size_t L = 1; L < nlev; ++L) {
    const Level& lv = h->lev[L];
    if (!lv.nPatch) continue;
    k_iso<<<blocks_for(lv.nPatch), kHB, 0, st>>>((int)L, lv.patch_struct, lv.nPatch, h->s_depth,
                                                 h->s_level, out->leafkey, isomask, iso_patch,
                                                 iso_level);
    HIP_LAUNCH_CHECK();
  }
  // the particle lists of the leaf and isodensity patches: counts, offsets,
  // then the lists (cursor order)
  for (int fill = 0; fill < 2; ++fill) {
    if (fill) {
      scan_offsets(ws, CountOf{leaf_cnt}, ns, leaf_off, st);
      scan_offsets(ws, CountOf{iso_cnt}, ns, iso_off, st);
      k_fill_u32<<<blocks_for(ns), kHB, 0, st>>>(leaf_cnt, ns, 0);
      k_fill_u32<<<blocks_for(ns), kHB, 0, st>>>(iso_cnt, ns, 0);
      HIP_LAUNCH_CHECK();
    }
    for (size_t L = 1; L < nlev; ++L) {
      const Level& lv = h->lev[L];
      if (!lv.nS || !lv.nPatch) continue;
      k_patch_lists<<<blocks_for(lv.nS), kHB, 0, st>>>(
          (int)L, lv.nS, lv.nPatch, lv.Skey, lv.Sstart, lv.Scount, lv.Spatch, lv.patch_struct,
          out->leafkey,
          iso_patch, iso_level, h->order, leaf_cnt, leaf_min, iso_cnt, fill, leaf_off, leaf_list,
          iso_off, iso_list);
      HIP_LAUNCH_CHECK();
    }
  }
  HIP_CHECK(hipStreamWaitEvent(st, ev.join, 0));  // the records
  k_centre<<<(unsigned)ns, kHT, 0, st>>>(leaf_off, leaf_cnt, leaf_list, leaf_tmp, out->leafkey,
                                         leaf_min, h->prm.g, P, out->centre);
  HIP_LAUNCH_CHECK();
  unsigned long long* ext = ws.get<unsigned long long>(ns);
  k_fill_u64<<<blocks_for(ns), kHB, 0, st>>>(reinterpret_cast<uint64_t*>(ext), ns, 0);
  HIP_LAUNCH_CHECK();
  for (size_t L = 1; L < nlev; ++L) {
    const Level& lv = h->lev[L];
    if (!lv.nS || !lv.nPatch) continue;
    k_extent<<<blocks_for(lv.nS), kHB, 0, st>>>((int)L, (int)lv.b, lv.nS, lv.nPatch, lv.Skey,
                                                lv.Spatch, lv.patch_struct, h->s_depth,
                                                h->s_level, h->s_patch, out->centre, ext);
    HIP_LAUNCH_CHECK();
  }
  LevCells LC{};
  LC.nlev = (int)nlev;
  LC.g = h->prm.g;
  for (size_t L = 0; L < nlev; ++L) {
    const Level& lv = h->lev[L];
    LC.key[L] = lv.Skey;
    LC.start[L] = lv.Sstart;
    LC.count[L] = lv.Scount;
    LC.n[L] = lv.nS;
  }
  uint8_t* coarse = ws.get<uint8_t>(ns);
  k_bound<<<(unsigned)ns, kHT, 0, st>>>(h->s_depth, h->s_host, ext, out->centre, iso_cnt, LC,
                                        out->radius, bound, coarse);
  HIP_LAUNCH_CHECK();
  scan_offsets(ws, CountOf{bound}, ns, out->cand_off, st);
  HIP_LAUNCH_CHECK();
  // the wide set (structures with at least `large` possible candidates) and
  // every structure's mode
  uint32_t* gs = ws.get<uint32_t>(ns);
  uint64_t* boff = ws.get<uint64_t>(ns + 1);
  uint64_t* wsz = ws.get<uint64_t>(3);
  uint32_t* mode = ws.get<uint32_t>(ns);
  {
    uint64_t* fo = ws.get<uint64_t>(ns + 1);
    uint64_t* bo = ws.get<uint64_t>(ns + 1);
    uint64_t* co = ws.get<uint64_t>(ns + 1);
    scan_offsets(ws, WideVal{out->cand_off, large, 0}, ns, fo, st);
    scan_offsets(ws, WideVal{out->cand_off, large, 1}, ns, bo, st);
    scan_offsets(ws, WideVal{out->cand_off, large, 2}, ns, co, st);
    k_w_place<<<blocks_for(ns), kHB, 0, st>>>(fo, bo, co, ns, gs, boff, wsz);
  }
  HIP_LAUNCH_CHECK();
  k_w_mode<<<blocks_for(ns), kHB, 0, st>>>(out->cand_off, ns, large, mode);
  HIP_LAUNCH_CHECK();
  uint64_t total = 0, wide[3] = {0, 0, 0};
  HIP_CHECK(hipMemcpyAsync(&total, out->cand_off + ns, sizeof(uint64_t), hipMemcpyDeviceToHost,
                           st));
  HIP_CHECK(hipMemcpyAsync(wide, wsz, sizeof(wide), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  const uint32_t nG = (uint32_t)wide[0];
  const uint64_t tb = wide[1], maxch = wide[2];
  const uint64_t t1 = total ? total : 1;
  out->cand = mem.get<uint32_t>(t1);
  out->member = mem.get<uint32_t>(t1);
  uint32_t* idx_a = ws.get<uint32_t>(t1);
  uint32_t* idx_b = ws.get<uint32_t>(t1);
  uint64_t* key_a = ws.get<uint64_t>(t1);
  uint64_t* key_b = ws.get<uint64_t>(t1);
  double* msum = ws.get<double>(t1);
  double* tail = ws.get<double>(t1);
  float4* vbuf = ws.get<float4>(t1);
  float4* vslot = ws.get<float4>(t1);
  const double rho_b = h->lev.empty() ? 0.0 : h->lev[0].tot_part;
  // The small structures on a second stream, one workgroup of kHT threads
  // each; beside them, on st, the wide set's candidates (a workgroup of
  // kHTBig threads each), their radii and velocities found by the whole grid,
  // and their unbinding by the grid (wide_unbind).
  hipEvent_t fork = ev.fork, join = ev.join;
  if (nG) {
    // the coarse substructures' candidates (one wide workgroup each) before
    // the second stream starts: its many small workgroups would otherwise
    // hold the compute units these need
    k_candidates<kHTBig><<<nG, kHTBig, 0, st>>>(h->s_depth, out->centre, out->radius, iso_off,
                                                iso_cnt, iso_list, LC, h->order, P,
                                                out->cand_off, out->cand, out->cand_cnt, large,
                                                gs, coarse);
    HIP_LAUNCH_CHECK();
  }
  HIP_CHECK(hipEventRecord(fork, st));
  HIP_CHECK(hipStreamWaitEvent(s2, fork, 0));
  // the small structures first (the wide rounds below wait on the host)
  k_candidates<kHT><<<(unsigned)ns, kHT, 0, s2>>>(h->s_depth, out->centre, out->radius, iso_off,
                                                  iso_cnt, iso_list, LC, h->order, P,
                                                  out->cand_off, out->cand, out->cand_cnt,
                                                  large, nullptr, nullptr);
  HIP_LAUNCH_CHECK();
  k_unbind<kHT><<<(unsigned)ns, kHT, 0, s2>>>(out->cand_off, out->cand_cnt, out->cand, idx_a,
                                              idx_b, key_a, key_b, msum, tail, vbuf, vslot,
                                              out->centre, P, delta_vir * rho_b, G, max_iter,
                                              out->member, out->member_cnt, out->r_vir,
                                              out->m_vir, out->vel, out->iters, mode, nullptr);
  HIP_LAUNCH_CHECK();
  if (nG) {
    // the wide set's candidates with their radii and velocities: by the grid,
    // but the coarse substructures' (one wide workgroup each, then the grid)
    uint32_t* wnb = ws.get<uint32_t>(nG);
    uint32_t* wcnt = ws.get<uint32_t>(nG);
    uint32_t* ccofs = ws.get<uint32_t>(nG + 1);
    k_w_bounds<<<blocks_for(nG), kHB, 0, st>>>(boff, nG, wnb);
    k_fill_u32<<<blocks_for(nG), kHB, 0, st>>>(wcnt, nG, 0);
    k_w_chunks<<<1, kHT, 0, st>>>(wnb, wnb, nG, ccofs);
    HIP_LAUNCH_CHECK();
    k_w_collect<<<(unsigned)maxch, kWT, 0, st>>>(ccofs, nG, gs, h->s_depth, coarse, out->centre,
                                                 out->radius, iso_off, iso_cnt, iso_list, LC,
                                                 h->order, P, out->cand_off, wcnt, out->cand,
                                                 msum, vslot);
    HIP_LAUNCH_CHECK();
    k_w_setcnt<<<blocks_for(nG), kHB, 0, st>>>(gs, nG, h->s_depth, coarse, iso_cnt, wcnt,
                                               out->cand_cnt);
    HIP_LAUNCH_CHECK();
    k_big_data<<<blocks_for(tb), kHB, 0, st>>>(out->cand_off, out->cand_cnt, out->cand, gs,
                                               boff, nG, out->centre, P, coarse, msum, vslot);
    HIP_LAUNCH_CHECK();
    // the grid's unbinding, on the wide set's candidates packed (segments
    // as long as their counts, not their possible counts: the sort and the
    // rounds skip the slack); the wide structures whose tied radii were too
    // many for its sort go to one wide workgroup each, on the second stream
    // once the sort has marked them
    uint32_t* wc = ws.get<uint32_t>(nG);
    uint64_t* coff = ws.get<uint64_t>(nG + 1);
    k_w_counts<<<blocks_for(nG), kHB, 0, st>>>(gs, nG, out->cand_cnt, wc);
    scan_offsets(ws, CountOf{wc}, nG, coff, st);
    HIP_LAUNCH_CHECK();
    uint64_t tc = 0;
    HIP_CHECK(hipMemcpyAsync(&tc, coff + nG, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    if (tc == 0) {  // no wide structure has a candidate
      k_w_empty<<<blocks_for(nG), kHB, 0, st>>>(gs, nG, out->cand_cnt, mode, out->member_cnt,
                                                out->r_vir, out->m_vir, out->vel, out->iters);
      HIP_LAUNCH_CHECK();
    } else {
      wide_unbind(ctx, ws, nG, tc, maxch, gs, coff, mode, msum, vslot, P, delta_vir * rho_b, G,
                  max_iter, st, out, [&]() {
                    HIP_CHECK(hipEventRecord(fork, st));
                    HIP_CHECK(hipStreamWaitEvent(s2, fork, 0));
                    k_unbind<kHTBig><<<nG, kHTBig, 0, s2>>>(
                        out->cand_off, out->cand_cnt, out->cand, idx_a, idx_b, key_a, key_b,
                        msum, tail, vbuf, vslot, out->centre, P, delta_vir * rho_b, G, max_iter,
                        out->member, out->member_cnt, out->r_vir, out->m_vir, out->vel,
                        out->iters, mode, gs);
                    HIP_LAUNCH_CHECK();
                  });
    }
  }
  HIP_CHECK(hipEventRecord(join, s2));
  HIP_CHECK(hipStreamWaitEvent(st, join, 0));
  HIP_CHECK(hipStreamSynchronize(st));
}

}  // namespace ahf

struct ahf_halos {
  ahf::Halos h;
};

extern "C" {

ahf_status ahf_find_halos(ahf_ctx* ctx, const ahf_hierarchy* h, const ahf_particles* p,
                          const float* vx, const float* vy, const float* vz,
                          const ahf_halo_params* prm, void* stream, ahf_halos** out) {
  using namespace ahf;
  if (!out) {
    set_last_error("out is NULL");
    return AHF_EINVAL;
  }
  *out = nullptr;
  if (!ctx || !h || !p || !vx || !vy || !vz || !prm || prm->struct_size < sizeof(ahf_halo_params)) {
    set_last_error("ctx, h, particles, velocities and params are required");
    return AHF_EINVAL;
  }
  if (!h->h.classified) {
    set_last_error("the hierarchy is not classified (AHF_SUBSTRUCTURE or ahf_classify_substructure)");
    return AHF_EINVAL;
  }
  if (p->n != h->h.n || !p->x || !p->y || !p->z) {
    set_last_error("the particles are not those of the hierarchy");
    return AHF_EINVAL;
  }
  if (!(prm->delta_vir > 0.0) || !(prm->G > 0.0) || prm->max_iter == 0) {
    set_last_error("delta_vir and G must be positive, max_iter at least 1");
    return AHF_EINVAL;
  }
  ahf_halos* r = new (std::nothrow) ahf_halos();
  if (!r) {
    set_last_error("host allocation failed");
    return AHF_ENOMEM;
  }
  hipStream_t st = (hipStream_t)stream;
  r->h.mem.ctx = &ctx->c;
  r->h.mem.st = st;
  try {
    HIP_CHECK(hipSetDevice(ctx->c.device));
    ctx->ws.bind(&ctx->c, st);
    ctx->ws.reset();
    find_halos(&ctx->c, ctx->ws, &h->h, *p, vx, vy, vz, prm->delta_vir, prm->G, prm->max_iter,
               prm->large_from ? prm->large_from : kBigCand, st, &r->h);
    ctx->ws.reset();
  } catch (const Error& e) {
    (void)hipStreamSynchronize(st);
    if (ctx->c.dep_st) (void)hipStreamSynchronize(ctx->c.dep_st);
    ctx->ws.reset();
    r->h.mem.release_all();
    delete r;
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(st);
    if (ctx->c.dep_st) (void)hipStreamSynchronize(ctx->c.dep_st);
    ctx->ws.reset();
    r->h.mem.release_all();
    delete r;
    set_last_error("host allocation failed");
    return AHF_ENOMEM;
  }
  *out = r;
  return AHF_OK;
}

ahf_status ahf_halos_get(const ahf_halos* hs, ahf_halos_view* v) {
  if (!hs || !v) {
    ahf::set_last_error("bad arguments");
    return AHF_EINVAL;
  }
  const ahf::Halos& h = hs->h;
  v->n_halos = h.n;
  v->leaf = reinterpret_cast<const uint64_t*>(h.leafkey);
  v->centre = h.centre;
  v->radius = h.radius;
  v->cand_offset = h.cand_off;
  v->cand_count = h.cand_cnt;
  v->cand = h.cand;
  v->member_count = h.member_cnt;
  v->member = h.member;
  v->r_vir = h.r_vir;
  v->m_vir = h.m_vir;
  v->vel = h.vel;
  v->iterations = h.iters;
  return AHF_OK;
}

void ahf_halos_free(ahf_halos* hs) {
  if (!hs) return;
  hs->h.mem.release_all();
  delete hs;
}

}  // extern "C"
