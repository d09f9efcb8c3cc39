// ahf_internal.h -- host-side internals shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ahf.h"
#include "ahf_dev.h"

namespace ahf {

struct Error {
  ahf_status code;
  std::string msg;
};

#define HIP_CHECK(x)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw ::ahf::Error{AHF_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define HIP_LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

// device memory through the context's callbacks or its own caching pool
struct Pool {
  std::mutex mu;  // hierarchies may be freed from another thread (server)
  std::vector<std::pair<size_t, void*>> free_blocks;  // (size, ptr)
  std::vector<std::pair<size_t, void*>> all;          // everything hipMalloc'd
  size_t bytes_all = 0;       // sum of `all`: device memory the pool holds
  size_t bytes_outstanding = 0;  // through the callbacks: allocated, not yet freed
};

// HIP-event timing of selected kernels (profiling mode of a context)
// Events that only time work: recording one performs no system-scope fence
// (no L2 write-back between the kernels around it); their elapsed times are
// read once the stream has passed them.
constexpr unsigned kTimingEventFlags = hipEventDisableSystemFence;

struct Prof {
  bool on = false;
  std::vector<std::string> only;  // names to time; empty = all
  bool wants(const char* name) const {
    if (only.empty()) return true;
    for (auto& n : only)
      if (n == name) return true;
    return false;
  }
  struct Rec {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<std::pair<std::string, std::pair<uint64_t, double>>> acc;
  std::vector<hipEvent_t> spare;
  hipEvent_t take();
  void begin(const char* name, hipStream_t st, hipEvent_t* a);
  void end(const char* name, hipStream_t st, hipEvent_t a);
  void collect();   // fold finished events into acc
  void clear();
};

// Per-build tuning: the particle count above which a cell of level 0, of
// level 1 and of the deeper levels is summed by whole waves (chunks) instead
// of by one thread, and the records one thread has in flight on level 1.
struct Tuning {
  uint32_t heavy[3] = {64, 64, 64};
  uint32_t batch1 = 2;
  int32_t sort_skip = -1;  // low key digits left out of the sort (-1: by size)
};

struct Ctx {
  int device = 0;
  ahf_alloc_fn alloc = nullptr;
  ahf_free_fn free = nullptr;
  void* user = nullptr;
  Pool pool;
  Prof prof;
  uint32_t* dev_err = nullptr;  // device error flags of the running build
  // per-level counts read back while the level's deposit runs: pinned host
  // words, an event behind their copy, and events that time the build phases
  uint32_t* host_cnt = nullptr;
  double* host_tot = nullptr;  // level totals and the error word (same allocation)
  hipEvent_t cnt_ev = nullptr;
  hipEvent_t phase_ev[3] = {nullptr, nullptr, nullptr};
  // the second stream of a build: level L's deposit runs there while the
  // build stream makes the cells of level L+1; dep_ev hands a level to it,
  // join_ev hands the finished deposits back
  hipStream_t dep_st = nullptr;
  hipEvent_t dep_ev = nullptr, join_ev = nullptr;
  // the third stream: the labels of the first levels, run while the build
  // stream makes the last, small levels
  hipStream_t lab_st = nullptr;
  hipEvent_t lab_ev = nullptr;
  // builds keep to their one stream: set for the workers of a server with
  // several of them, whose concurrent builds already fill the GPU (and whose
  // streams would otherwise outnumber the hardware queues many times over)
  bool one_stream = false;
  // device bytes per particle of the last hierarchy built on this context:
  // sizes the first block of the next hierarchy's arena
  double hier_bpp = 0.0;
  // plans of builds sized ahead, learned from finished builds: per parameter
  // set and size class (half octaves of n), the depth and, per level, the
  // refined cells and next-level bricks per particle (largest seen)
  struct PlanRec {
    int g, Lmax, conn, bucket;
    double dom_ref, ref_ref;
    uint32_t flags;
    bool has_mass;
    int depth;
    double rF[kMaxLevels], rD[kMaxLevels];
    uint64_t last_use;
  };
  std::vector<PlanRec> plans;
  uint64_t plan_clock = 0;
  bool planning = false;
  // builds that run with no host involvement (the sub-volumes of a batch,
  // recorded into a graph): no timing events, no copy to pinned memory at the
  // end, the labels enqueued within the build; the host reads each build's
  // status block after the run (in_graph).  While a graph is being recorded
  // nothing may allocate (recording).
  bool in_graph = false;
  bool recording = false;
  // tuning by size: the entry with the largest min_n <= n applies to a build
  // of n particles (defaults when none does)
  std::vector<std::pair<uint64_t, Tuning>> tuning;
  Tuning tuning_for(uint64_t n) const {
    Tuning t;
    uint64_t best = 0;
    bool found = false;
    for (auto& e : tuning)
      if (e.first <= n && (!found || e.first >= best)) {
        best = e.first;
        t = e.second;
        found = true;
      }
    return t;
  }
};


// times one launch when the context profiles
#define AHF_TIMED(ctxp, name, st, launch)                  \
  do {                                                     \
    hipEvent_t ev_a_ = nullptr;                            \
    const bool tm_ = (ctxp)->prof.on && (ctxp)->prof.wants(name); \
    if (tm_) (ctxp)->prof.begin(name, st, &ev_a_);         \
    launch;                                                \
    HIP_LAUNCH_CHECK();                                    \
    if (tm_) (ctxp)->prof.end(name, st, ev_a_);            \
  } while (0)

void* ctx_alloc(Ctx* c, size_t bytes, hipStream_t s);  // throws AHF_ENOMEM
void ctx_free(Ctx* c, void* p, size_t bytes, hipStream_t s);
void ctx_release(Ctx* c, void* p, size_t bytes, hipStream_t s);  // not kept in the pool
void ctx_release_pool(Ctx* c);
// device memory the context holds: its pool (free blocks included), or what
// it has allocated through the callbacks and not yet freed
size_t ctx_device_bytes(Ctx* c);

// Stack-like scratch space for one build: chunks are never moved, so every
// pointer handed out stays valid until released.
class Ws {
 public:
  struct Mark {
    size_t chunk, off;
  };
  Ws() = default;
  void bind(Ctx* c, hipStream_t s) {
    ctx_ = c;
    st_ = s;
  }
  template <class T>
  T* get(uint64_t n) {
    return static_cast<T*>(raw(n * sizeof(T)));
  }
  void* raw(size_t bytes);
  Mark mark() const { return Mark{cur_, chunks_.empty() ? 0 : chunks_[cur_].used}; }
  void release(Mark m);
  void reset();        // drop every allocation (memory kept for the next build)
  // drop every allocation and keep every chunk as it is (memory that work
  // already recorded into a graph refers to must not move)
  void rewind() {
    for (auto& c : chunks_) c.used = 0;
    cur_ = 0;
  }
  void free_all();     // give the memory back to the context
  size_t high_water() const { return high_; }
  size_t capacity() const {
    size_t t = 0;
    for (auto& c : chunks_) t += c.size;
    return t;
  }
  Ctx* ctx() const { return ctx_; }

 private:
  struct Chunk {
    char* p;
    size_t size, used;
  };
  Ctx* ctx_ = nullptr;
  hipStream_t st_ = nullptr;
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
  size_t high_ = 0;
};

// Device memory of one hierarchy: an arena of a few large blocks from the
// context's allocator, each array a 256-byte aligned piece of one of them
// (so a build makes a handful of allocator calls, not one per array).  The
// first block is sized from the bytes the previous hierarchy of the context
// used per particle (not its blocks, so the size does not creep from build to
// build); a block that is full is followed by one of at least a quarter of
// everything so far.  Everything goes back at once.
struct Owned {
  Ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  std::vector<std::pair<void*, size_t>> list;  // blocks
  size_t used = 0, room = 0;                   // of the last block
  size_t handed = 0;                           // bytes handed out in all
  size_t first_hint = 0;                       // bytes for the first block
  template <class T>
  T* get(uint64_t n) {
    return static_cast<T*>(raw((n ? n : 1) * sizeof(T)));
  }
  void* raw(size_t b) {
    b = (b + 255) & ~size_t(255);
    if (list.empty() || used + b > room) {
      size_t tot = 0;
      for (auto& a : list) tot += a.second;
      size_t want = b;
      if (list.empty()) want = std::max(want, first_hint);
      want = std::max(want, tot / 4);
      want = std::max(want, size_t(1) << 20);
      want = (want + (size_t(1) << 16) - 1) & ~((size_t(1) << 16) - 1);
      void* p = ctx_alloc(ctx, want, st);
      list.emplace_back(p, want);
      used = 0;
      room = want;
    }
    char* p = static_cast<char*>(list.back().first) + used;
    used += b;
    handed += b;
    return p;
  }
  // the first block, of at least `bytes`, allocated now (before a build
  // that must not allocate while it is enqueued)
  void reserve(size_t bytes) {
    if (!list.empty()) return;
    const size_t hint = first_hint;
    first_hint = std::max(first_hint, bytes);
    (void)raw(1);
    used = 0;
    handed = 0;
    first_hint = hint;
  }
  // the same memory handed out again from the start (the work that used it
  // has finished): one block of at least `bytes`
  void reuse(size_t bytes) {
    if (list.size() == 1 && list[0].second >= bytes) {
      used = 0;
      room = list[0].second;
      handed = 0;
      return;
    }
    release_all();
    reserve(bytes);
  }
  void release_all() {
    for (auto& a : list) ctx_free(ctx, a.first, a.second, st);
    list.clear();
    used = room = handed = 0;
  }
  size_t bytes() const {
    size_t t = 0;
    for (auto& a : list) t += a.second;
    return t;
  }
};

// ---------------------------------------------------------------- primitives
// Indices of the nonzero bytes of flags[0, n) in increasing order: list[r]
// = index of the r-th flagged element and/or rank[i] = r for each flagged i
// (either may be null; an unflagged i keeps its value or becomes all ones);
// *count (device) = number of flagged elements.
void compact_flags(Ws& ws, const uint8_t* flags, uint64_t n, uint32_t* list, uint32_t* rank,
                   uint32_t* count, hipStream_t st);
// the same with a count known on the device only (laid out for nc.cap)
void compact_flags(Ws& ws, const uint8_t* flags, Cnt nc, uint32_t* list, uint32_t* rank,
                   uint32_t* count, hipStream_t st);
// Stable LSD sort of particles by Morton key (key_bits bits), ties by index,
// in 8-bit digits.  The first q passes move (key, index) pairs; from pass q on
// one packed word per element, ((key >> 8q) << ib) | index, with ib the index
// width.  sort_keys takes keys[i] = key of particle i (or, when q == 0, the
// packed word of particle i already) and ghist[p * 256 + d] = the number of
// keys whose digit p is d; it returns the sorted packed words (keys or a
// workspace buffer) and, in *spare, the other of the two buffers, free once
// the sort has run.
struct SortPlan {
  int key_bits = 0, npass = 0, ib = 1, q = 0;
};
SortPlan sort_plan(uint64_t n, int key_bits);
uint64_t* sort_keys(Ctx* ctx, Ws& ws, uint64_t* keys, uint64_t n, const SortPlan& sp,
                    const uint32_t* ghist, hipStream_t st, uint64_t** spare = nullptr);
constexpr int kRsMaxPass = 8;
template <typename T>
void sum_to_f64(Ws& ws, const T* a, uint64_t n, double* out, hipStream_t st);

// ---------------------------------------------------------------- hierarchy
struct Level {
  uint32_t b = 0;
  uint64_t nS = 0, nF = 0, nB = 0, nP = 0, nPatch = 0;
  uint64_t capF = 0;            // room for the refined cells (= nF once known)
  uint64_t* Skey = nullptr;     // [nS], null on level 0 (identity)
  uint32_t* Sstart = nullptr;   // [nS] (+1 sentinel on level 0)
  uint32_t* Scount = nullptr;   // [nS]
  uint8_t* Sflag = nullptr;     // [nS]
  double* Spmass = nullptr;     // [nS] particle mass per cell
  int32_t* Spatch = nullptr;    // [nS] after labelling (level >= 1)
  uint32_t* Fs = nullptr;       // [nF] S index of the refined cells
  uint64_t* Bkey = nullptr;     // [nB] parent key of each brick, null on level 0
  int32_t* Bcell = nullptr;     // [nB] S index of the brick's first cell or -1, null on level 0
  int32_t* Pbrick = nullptr;    // [nF of level-1] brick of each parent, null on level 0
  float* mass = nullptr;        // [8 nB]
  int32_t* slot_child = nullptr;  // [8 nB] brick of the next level made of the slot's children
  int32_t* slot_f = nullptr;      // [8 nB] index in F of the slot's cell, or -1
  int32_t* patch_parent = nullptr;
  uint32_t* patch_ncells = nullptr;
  uint64_t* patch_npart = nullptr;
  double* patch_mass = nullptr;
  int32_t* patch_struct = nullptr;  // [nPatch] structure of each patch (classified)
  double tot_cell = 0.0, tot_part = 0.0;
};

struct Params {
  int g = 0, Lmax = 0, conn = 26;
  double dom_ref = 0, ref_ref = 0;
  uint32_t flags = 0;
};

struct Hier {
  Ctx* ctx = nullptr;
  Owned mem;
  Params prm;
  uint64_t n = 0;
  int B = 0;
  uint32_t* order = nullptr;
  bool has_mass = false;
  double mass_scalar = 1.0;
  bool labelled = false;
  uint32_t* npatch_dev = nullptr;  // [kMaxLevels] patch counts on the device (labelled)
  uint32_t* lab_dev = nullptr;     // label error flags and counts (npatch_dev = lab_dev + 4)
  uint32_t lab_done = 0;           // levels whose refined cells were labelled during the build
  // host structures and substructures of the grid tree (classified)
  bool classified = false;
  uint64_t nStruct = 0;
  int32_t *s_host = nullptr, *s_level = nullptr, *s_patch = nullptr, *s_depth = nullptr;
  uint32_t* cls_base = nullptr;  // [kMaxLevels + 1] structures starting up to each level
  std::vector<Level> lev;
  bool planned = false;  // levels sized ahead (no host wait per level)
  bool sizes_known = true;  // the host knows every level's counts (after finish_build)
  const uint32_t* dev_lvcnt = nullptr;  // a planned build's level counts on the device
                                        // (2 per level: refined cells, next-level bricks)
  bool replanned = false;  // a planned attempt outgrew its capacities and was redone
  const uint64_t* dev_status = nullptr;  // the build's totals, counters and flags (in_graph)
  uint32_t host_waits = 0;  // times the host waited for the device during the build
  uint32_t sort_key_bits = 0, sort_passes = 0;  // what the radix sort ordered by
  double ms[4] = {0, 0, 0, 0};
  double t_start = 0.0;  // host clock at the start of the build
};

// Capacities of a build whose levels are all enqueued without waiting for the
// host: levels 0..depth, and per level the room for its refined cells (capF)
// and for the bricks of the next level (capD).
struct Plan {
  int depth = 0;
  uint64_t capF[kMaxLevels] = {};
  uint64_t capD[kMaxLevels] = {};
};
// internal status: a planned build outgrew its capacities and is redone
constexpr ahf_status kStatusReplan = -100;
// the capacities for a build of n particles from what the context learned
// from earlier builds of the same parameters and size class (false: none)
bool plan_for(Ctx* c, const Params& prm, bool has_mass, uint64_t n, Plan* out);

// Enqueues the build on st.  With finish, waits for it and completes h
// (totals, timings, device error flags); without, the caller must call
// finish_build once the stream has passed the build (labels may run first).
// With the count criterion every level's deposit runs on ctx->dep_st, with
// its scratch from wsd (kept until the build ends; the deposits are joined
// back into st before the build's last kernels).
void build_hierarchy(Ctx* ctx, Ws& ws, Ws& wsd, const ahf_particles& p, const Params& prm,
                     hipStream_t st, Hier* h, bool finish = true, const Plan* plan = nullptr);
void finish_build(Ctx* ctx, Hier* h);
void label_hierarchy(Ctx* ctx, Ws& ws, Hier* h, hipStream_t st);
// The status block of a build that runs with no host involvement (in_graph):
// kStatusWords 64-bit words (level totals, counters, device error flags, label
// counts) that enqueue_status copies to dst on st once the build and its
// labels are complete; finish_from_status completes h from a host copy
// (throws like finish_build and label_hierarchy; kStatusReplan when a level
// outgrew its capacity).
constexpr size_t kStatusWords = 160;
void enqueue_status(Hier* h, uint64_t* dst, hipStream_t st);
void finish_from_status(Hier* h, const uint64_t* status);
// joins the build's label stream into st and labels whatever is left, all
// enqueued (in_graph builds: nothing is left)
void label_enqueue(Ctx* ctx, Ws& ws, Hier* h, hipStream_t st);
// labels the refined cells of levels lab_done .. k1-1 on ctx->lab_st once st
// has passed their cells, with scratch from wsd (kept); label_hierarchy labels
// what is left
void label_early(Ctx* ctx, Ws& wsd, Hier* h, uint32_t k1, hipStream_t st);
// host structures and substructures of a labelled hierarchy (waits for it);
// classify_levels only enqueues, finish_classify waits and reads the count
void classify_hierarchy(Ctx* ctx, Ws& ws, Hier* h, hipStream_t st);
void classify_levels(Ctx* ctx, Ws& ws, Hier* h, hipStream_t st);
void finish_classify(Ctx* ctx, Hier* h, hipStream_t st);
// the device address of the library's static staging array on `device`
// (looked up once per device, with that device current)
void* static_scratch(int device);
// patch ids of level-L cells given by key (host arrays); level >= 1, labelled
void query_labels(Ws& ws, const Hier* h, int L, uint64_t n, const uint64_t* keys_host,
                  int32_t* out_host, hipStream_t st);
size_t hier_bytes(const Hier* h);
// validation of a build request before anything is launched (AHF_OK or an
// error status with the message set)
ahf_status check_request(const ahf_params* prm, const ahf_particles* p, Params* out);
void set_last_error(const std::string& msg);  // message returned by ahf_last_error

}  // namespace ahf

struct ahf_ctx {
  ahf::Ctx c;
  ahf::Ws ws;
  ahf::Ws ws_dep;  // scratch of the deposits running on the second stream
};

struct ahf_hierarchy {
  ahf::Hier h;
};
