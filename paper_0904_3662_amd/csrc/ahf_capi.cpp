// ahf_capi.cpp -- the extern "C" boundary: contexts, memory, validation, views.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "ahf_internal.h"

namespace ahf {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

static ahf_status fail(ahf_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// ---------------------------------------------------------------- memory

static size_t round_size(size_t b) {
  if (b < 4096) return (b + 255) & ~size_t(255);
  if (b < (size_t(2) << 20)) {
    size_t r = 4096;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t q = size_t(2) << 20;
  return (b + q - 1) / q * q;
}

static void release_free_blocks(Ctx* c);

void* ctx_alloc(Ctx* c, size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 1;
  // work being recorded into a graph must find all its memory in place
  if (c->recording) throw Error{AHF_EDEVICE, "a recorded build asked for device memory"};
  if (c->alloc) {
    void* p = c->alloc(c->user, bytes, (void*)s);
    if (!p) throw Error{AHF_ENOMEM, "device allocation callback failed"};
    std::lock_guard<std::mutex> lk(c->pool.mu);
    c->pool.bytes_outstanding += bytes;
    return p;
  }
  const size_t r = round_size(bytes);
  std::lock_guard<std::mutex> lk(c->pool.mu);
  // the smallest cached block that fits and wastes at most a quarter of it
  auto& fb = c->pool.free_blocks;
  size_t best = fb.size();
  for (size_t i = 0; i < fb.size(); ++i)
    if (fb[i].first >= r && fb[i].first - r <= fb[i].first / 4 &&
        (best == fb.size() || fb[i].first < fb[best].first))
      best = i;
  if (best < fb.size()) {
    void* p = fb[best].second;
    fb[best] = fb.back();
    fb.pop_back();
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, r) != hipSuccess) {
    (void)hipGetLastError();
    // give cached blocks back and retry once
    release_free_blocks(c);
    if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{AHF_ENOMEM, "hipMalloc of " + std::to_string(r) + " bytes failed"};
    }
  }
  c->pool.all.emplace_back(r, p);
  c->pool.bytes_all += r;
  return p;
}

// size the pool allocated for block p (caller holds the pool lock)
static size_t block_size(Ctx* c, void* p, size_t bytes) {
  for (auto& a : c->pool.all)
    if (a.second == p) return a.first;
  return round_size(bytes);
}

void ctx_free(Ctx* c, void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (bytes == 0) bytes = 1;
  if (c->free) {
    c->free(c->user, p, bytes, (void*)s);
    std::lock_guard<std::mutex> lk(c->pool.mu);
    c->pool.bytes_outstanding -= std::min(c->pool.bytes_outstanding, bytes);
    return;
  }
  std::lock_guard<std::mutex> lk(c->pool.mu);
  c->pool.free_blocks.emplace_back(block_size(c, p, bytes), p);
}

// gives one block back for good (not to the pool's cache): the workspace
// chunks that a reset folds into one would otherwise stay cached beside it
void ctx_release(Ctx* c, void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (c->free) {
    c->free(c->user, p, bytes ? bytes : 1, (void*)s);
    std::lock_guard<std::mutex> lk(c->pool.mu);
    c->pool.bytes_outstanding -= std::min(c->pool.bytes_outstanding, bytes ? bytes : 1);
    return;
  }
  std::lock_guard<std::mutex> lk(c->pool.mu);
  for (size_t i = 0; i < c->pool.all.size(); ++i)
    if (c->pool.all[i].second == p) {
      c->pool.bytes_all -= c->pool.all[i].first;
      c->pool.all[i] = c->pool.all.back();
      c->pool.all.pop_back();
      break;
    }
  (void)hipFree(p);
}

// caller holds the pool lock
static void release_free_blocks(Ctx* c) {
  auto& fb = c->pool.free_blocks;
  for (auto& b : fb) {
    (void)hipFree(b.second);
    for (size_t i = 0; i < c->pool.all.size(); ++i)
      if (c->pool.all[i].second == b.second) {
        c->pool.bytes_all -= c->pool.all[i].first;
        c->pool.all[i] = c->pool.all.back();
        c->pool.all.pop_back();
        break;
      }
  }
  fb.clear();
}

void ctx_release_pool(Ctx* c) {
  std::lock_guard<std::mutex> lk(c->pool.mu);
  release_free_blocks(c);
}

size_t ctx_device_bytes(Ctx* c) {
  std::lock_guard<std::mutex> lk(c->pool.mu);
  return c->alloc ? c->pool.bytes_outstanding : c->pool.bytes_all;
}

size_t hier_bytes(const Hier* h) { return h->mem.bytes(); }

void* Ws::raw(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  while (cur_ < chunks_.size()) {
    Chunk& c = chunks_[cur_];
    if (c.used + bytes <= c.size) {
      void* p = c.p + c.used;
      c.used += bytes;
      size_t tot = 0;
      for (size_t i = 0; i < cur_; ++i) tot += chunks_[i].size;
      if (tot + c.used > high_) high_ = tot + c.used;
      return p;
    }
    if (cur_ + 1 < chunks_.size()) {
      ++cur_;
      chunks_[cur_].used = 0;
      continue;
    }
    break;
  }
  size_t want = bytes;
  size_t have = 0;
  for (auto& c : chunks_) have += c.size;
  if (want < have) want = have;            // grow geometrically
  if (want < (size_t(64) << 20)) want = size_t(64) << 20;
  Chunk c{static_cast<char*>(ctx_alloc(ctx_, want, st_)), want, bytes};
  chunks_.push_back(c);
  cur_ = chunks_.size() - 1;
  if (have + bytes > high_) high_ = have + bytes;
  return c.p;
}

void Ws::release(Mark m) {
  if (chunks_.empty()) return;
  for (size_t i = m.chunk + 1; i < chunks_.size() && i <= cur_; ++i) chunks_[i].used = 0;
  cur_ = m.chunk;
  chunks_[cur_].used = m.off;
}

void Ws::reset() {
  // fold several chunks into one of the high-water size, so that the next
  // build of the same size needs a single chunk and nothing more (the old
  // chunks, which grew geometrically, go back for good; the callers have
  // waited for the work that used them).  Never throws: when the new chunk
  // cannot be had, the old ones stay.
  if (chunks_.size() > 1) {
    const size_t want = (high_ + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);
    char* p = nullptr;
    try {
      p = static_cast<char*>(ctx_alloc(ctx_, want, st_));
    } catch (const Error&) {
      p = nullptr;
    }
    if (p) {
      for (auto& c : chunks_) ctx_release(ctx_, c.p, c.size, st_);
      chunks_.clear();
      chunks_.push_back(Chunk{p, want, 0});
    }
  }
  for (auto& c : chunks_) c.used = 0;
  cur_ = 0;
}

void Ws::free_all() {
  for (auto& c : chunks_) ctx_free(ctx_, c.p, c.size, st_);
  chunks_.clear();
  cur_ = 0;
}

hipEvent_t Prof::take() {
  if (!spare.empty()) {
    hipEvent_t e = spare.back();
    spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  HIP_CHECK(hipEventCreateWithFlags(&e, kTimingEventFlags));
  return e;
}

void Prof::begin(const char* name, hipStream_t st, hipEvent_t* a) {
  (void)name;
  *a = take();
  HIP_CHECK(hipEventRecord(*a, st));
}

void Prof::end(const char* name, hipStream_t st, hipEvent_t a) {
  hipEvent_t b = take();
  HIP_CHECK(hipEventRecord(b, st));
  pending.push_back(Rec{name, a, b});
}

void Prof::collect() {
  for (auto& r : pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      bool found = false;
      for (auto& x : acc)
        if (x.first == r.name) {
          x.second.first += 1;
          x.second.second += ms;
          found = true;
          break;
        }
      if (!found) acc.push_back({r.name, {1, (double)ms}});
    } else {
      (void)hipGetLastError();
    }
    spare.push_back(r.a);
    spare.push_back(r.b);
  }
  pending.clear();
}

void Prof::clear() {
  collect();
  acc.clear();
}

// ---------------------------------------------------------------- validation

static ahf_status check_params(const ahf_params* prm, Params* out) {
  if (!prm || prm->struct_size < sizeof(ahf_params)) return fail(AHF_EINVAL, "bad ahf_params");
  const int g = (int)prm->dom_grid_log2;
  if (g < 1 || g > 10) return fail(AHF_EINVAL, "dom_grid_log2 must be in 1..10");
  if ((uint64_t)prm->dom_grid_log2 + prm->max_levels > 21)
    return fail(AHF_EINVAL, "dom_grid_log2 + max_levels must be <= 21");
  if (std::isnan(prm->dom_ref) || std::isnan(prm->ref_ref))
    return fail(AHF_EINVAL, "thresholds must not be NaN");
  const uint32_t conn = prm->connectivity ? prm->connectivity : 26;
  if (conn != 6 && conn != 18 && conn != 26) return fail(AHF_EINVAL, "connectivity must be 6, 18 or 26");
  out->g = g;
  out->Lmax = (int)prm->max_levels;
  out->conn = (int)conn;
  out->dom_ref = prm->dom_ref;
  out->ref_ref = prm->ref_ref;
  if ((prm->flags & AHF_SUBSTRUCTURE) && (prm->flags & AHF_NO_LABELS))
    return fail(AHF_EINVAL, "AHF_SUBSTRUCTURE needs the grid tree (not AHF_NO_LABELS)");
  out->flags = prm->flags;
  return AHF_OK;
}

static ahf_status check_particles(const ahf_particles* p) {
  if (!p) return fail(AHF_EINVAL, "particles is NULL");
  if (p->n >= (1ull << 32)) return fail(AHF_EINVAL, "at most 2^32 - 1 particles");
  if (p->n > 0 && (!p->x || !p->y || !p->z)) return fail(AHF_EINVAL, "x, y and z are required");
  if (!p->mass && !(std::isfinite(p->mass_scalar))) return fail(AHF_EINVAL, "mass_scalar must be finite");
  return AHF_OK;
}

ahf_status check_request(const ahf_params* prm, const ahf_particles* p, Params* out) {
  ahf_status s = check_params(prm, out);
  if (s != AHF_OK) return s;
  s = check_particles(p);
  if (s != AHF_OK) return s;
  if ((out->flags & AHF_DENSITY_CRITERION) && (p->mass || !(p->mass_scalar > 0.0)))
    return fail(AHF_EINVAL, "AHF_DENSITY_CRITERION needs equal masses (mass NULL, mass_scalar > 0)");
  return AHF_OK;
}

}  // namespace ahf

using namespace ahf;

extern "C" {

const char* ahf_last_error(void) { return g_last_error.c_str(); }

ahf_status ahf_ctx_create(const ahf_ctx_desc* desc, ahf_ctx** out) {
  if (!out) return fail(AHF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc || desc->struct_size < sizeof(ahf_ctx_desc)) return fail(AHF_EINVAL, "bad ahf_ctx_desc");
  if ((desc->alloc == nullptr) != (desc->free == nullptr))
    return fail(AHF_EINVAL, "alloc and free callbacks must be given together");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(AHF_EDEVICE, "no HIP device available");
  }
  if (desc->device < 0 || desc->device >= ndev) return fail(AHF_EINVAL, "device ordinal out of range");
  // the static staging array's address on this device, once per device
  try {
    if (hipSetDevice(desc->device) != hipSuccess) {
      (void)hipGetLastError();
      return fail(AHF_EDEVICE, "hipSetDevice failed");
    }
    (void)static_scratch(desc->device);
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  ahf_ctx* c = new (std::nothrow) ahf_ctx();
  if (!c) return fail(AHF_ENOMEM, "host allocation failed");
  c->c.device = desc->device;
  c->c.alloc = desc->alloc;
  c->c.free = desc->free;
  c->c.user = desc->user;
  c->ws.bind(&c->c, nullptr);
  c->ws_dep.bind(&c->c, nullptr);
  *out = c;
  return AHF_OK;
}

void ahf_ctx_destroy(ahf_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  ctx->ws.free_all();
  ctx->ws_dep.free_all();
  if (ctx->c.dep_st) (void)hipStreamDestroy(ctx->c.dep_st);
  if (ctx->c.lab_st) (void)hipStreamDestroy(ctx->c.lab_st);
  if (ctx->c.lab_ev) (void)hipEventDestroy(ctx->c.lab_ev);
  if (ctx->c.dep_ev) (void)hipEventDestroy(ctx->c.dep_ev);
  if (ctx->c.join_ev) (void)hipEventDestroy(ctx->c.join_ev);
  if (ctx->c.host_cnt) (void)hipHostFree(ctx->c.host_cnt);
  if (ctx->c.cnt_ev) (void)hipEventDestroy(ctx->c.cnt_ev);
  for (auto& e : ctx->c.phase_ev)
    if (e) (void)hipEventDestroy(e);
  ctx->c.prof.collect();
  for (auto e : ctx->c.prof.spare) (void)hipEventDestroy(e);
  ctx_release_pool(&ctx->c);
  for (auto& b : ctx->c.pool.all) (void)hipFree(b.second);
  delete ctx;
}

}  // extern "C"

namespace ahf {

static int size_class(uint64_t n) { return (int)std::floor(2.0 * std::log2((double)n)); }

static bool same_params(const Ctx::PlanRec& r, const Params& prm, bool has_mass, int bucket) {
  return r.g == prm.g && r.Lmax == prm.Lmax && r.conn == prm.conn && r.bucket == bucket &&
         r.dom_ref == prm.dom_ref && r.ref_ref == prm.ref_ref && r.flags == prm.flags &&
         r.has_mass == has_mass;
}

// capacities for a build of n particles from a learned plan: the per-particle
// counts seen, with a margin (15% and 64)
bool plan_for(Ctx* c, const Params& prm, bool has_mass, uint64_t n, Plan* out) {
  const int bucket = size_class(n);
  for (auto& r : c->plans)
    if (same_params(r, prm, has_mass, bucket)) {
      r.last_use = ++c->plan_clock;
      out->depth = r.depth;
      for (int L = 0; L < kMaxLevels; ++L) {
        out->capF[L] = L <= r.depth ? (uint64_t)std::ceil(r.rF[L] * (double)n * 1.15) + 64 : 0;
        out->capD[L] = L <= r.depth ? (uint64_t)std::ceil(r.rD[L] * (double)n * 1.15) + 64 : 0;
      }
      return true;
    }
  return false;
}

// learns from a finished build (the largest counts per particle win)
static void plan_record(Ctx* c, const Params& prm, bool has_mass, uint64_t n, const Hier* h) {
  if (n == 0 || h->lev.empty()) return;
  const int bucket = size_class(n);
  Ctx::PlanRec* r = nullptr;
  for (auto& x : c->plans)
    if (same_params(x, prm, has_mass, bucket)) r = &x;
  if (!r) {
    if (c->plans.size() >= 32) {  // forget the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < c->plans.size(); ++i)
        if (c->plans[i].last_use < c->plans[lru].last_use) lru = i;
      c->plans.erase(c->plans.begin() + (long)lru);
    }
    c->plans.push_back(Ctx::PlanRec{prm.g, prm.Lmax, prm.conn, bucket, prm.dom_ref, prm.ref_ref,
                                    prm.flags, has_mass, 0, {}, {}, 0});
    r = &c->plans.back();
  }
  r->last_use = ++c->plan_clock;
  const int depth = (int)h->lev.size() - 1;
  r->depth = std::max(r->depth, depth);
  for (int L = 0; L <= depth; ++L) {
    const double f = (double)h->lev[L].nF / (double)n;
    const double d = L + 1 <= depth ? (double)h->lev[L + 1].nB / (double)n : 0.0;
    r->rF[L] = std::max(r->rF[L], f);
    r->rD[L] = std::max(r->rD[L], d);
  }
}

// one attempt at a build (planned when plan is given): the hierarchy is
// complete, labels included, when this returns
static void build_once(ahf_ctx* ctx, const ahf_particles* particles, const Params& prm,
                       hipStream_t st, ahf_hierarchy* h, const Plan* plan) {
  HIP_CHECK(hipSetDevice(ctx->c.device));
  h->h.ctx = &ctx->c;
  h->h.mem.ctx = &ctx->c;
  h->h.mem.st = st;
  // the arena's first block from the last hierarchy of this context, in
  // steps of 2 MB so that builds of similar sizes reuse cached blocks
  h->h.mem.first_hint = (size_t)(ctx->c.hier_bpp * 1.05 * (double)particles->n);
  h->h.mem.first_hint = (h->h.mem.first_hint + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);
  ctx->ws.bind(&ctx->c, st);
  ctx->ws.reset();
  ctx->ws_dep.bind(&ctx->c, st);
  ctx->ws_dep.reset();
  // with equal masses the labels need nothing from the build's totals: they
  // are enqueued behind it, and one wait at the end covers both (a planned
  // build first reads its level sizes back, then labels)
  const bool labels = !(prm.flags & AHF_NO_LABELS);
  const bool defer = labels && particles->mass == nullptr && !plan;
  build_hierarchy(&ctx->c, ctx->ws, ctx->ws_dep, *particles, prm, st, &h->h, !defer, plan);
  if (labels) label_hierarchy(&ctx->c, ctx->ws, &h->h, st);
  if (defer) finish_build(&ctx->c, &h->h);
  ctx->ws.reset();
  ctx->ws_dep.reset();
}

// every stream of the context idle, the hierarchy's memory returned, the
// workspaces reset (after a failed attempt)
static void abandon(ahf_ctx* ctx, ahf_hierarchy* h, hipStream_t st) {
  if (ctx->c.dep_st) (void)hipStreamSynchronize(ctx->c.dep_st);
  if (ctx->c.lab_st) (void)hipStreamSynchronize(ctx->c.lab_st);
  (void)hipStreamSynchronize(st);
  h->h.mem.release_all();
  ctx->ws.reset();
  ctx->ws_dep.reset();
}

}  // namespace ahf

extern "C" {

ahf_status ahf_build_hierarchy(ahf_ctx* ctx, const ahf_particles* particles, const ahf_params* params,
                               void* stream, ahf_hierarchy** out) {
  if (!out) return fail(AHF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(AHF_EINVAL, "ctx is NULL");
  Params prm;
  ahf_status s = check_request(params, particles, &prm);
  if (s != AHF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const bool has_mass = particles->mass != nullptr;
  Plan plan;
  bool use_plan = ctx->c.planning && particles->n > 0 && !(prm.flags & AHF_DENSITY_CRITERION) &&
                  plan_for(&ctx->c, prm, has_mass, particles->n, &plan);
  bool replanned = false;
  for (;;) {
    ahf_hierarchy* h = new (std::nothrow) ahf_hierarchy();
    if (!h) return fail(AHF_ENOMEM, "host allocation failed");
    try {
      build_once(ctx, particles, prm, st, h, use_plan ? &plan : nullptr);
    } catch (const Error& e) {
      abandon(ctx, h, st);
      delete h;
      if (e.code == kStatusReplan && use_plan) {
        // the plan was too small for this snapshot: the synced build sizes
        // every level exactly and teaches the plan
        use_plan = false;
        replanned = true;
        continue;
      }
      return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
      abandon(ctx, h, st);
      delete h;
      return fail(AHF_ENOMEM, "host allocation failed");
    }
    h->h.replanned = replanned;
    if (particles->n > 0) ctx->c.hier_bpp = (double)h->h.mem.handed / (double)particles->n;
    if (!(prm.flags & AHF_DENSITY_CRITERION)) plan_record(&ctx->c, prm, has_mass, particles->n, &h->h);
    *out = h;
    return AHF_OK;
  }
}

ahf_status ahf_ctx_set_planning(ahf_ctx* ctx, int enable) {
  if (!ctx) return fail(AHF_EINVAL, "ctx is NULL");
  ctx->c.planning = enable != 0;
  if (!enable) ctx->c.plans.clear();
  return AHF_OK;
}

ahf_status ahf_hierarchy_build_info(const ahf_hierarchy* h, ahf_build_info* out) {
  if (!h || !out) return fail(AHF_EINVAL, "bad arguments");
  out->struct_size = sizeof(ahf_build_info);
  out->planned = h->h.planned ? 1u : 0u;
  out->replanned = h->h.replanned ? 1u : 0u;
  out->host_waits = h->h.host_waits;
  out->device_bytes = h->h.mem.bytes();
  out->sort_key_bits = h->h.sort_key_bits;
  out->sort_passes = h->h.sort_passes;
  return AHF_OK;
}

ahf_status ahf_label_refinements(ahf_ctx* ctx, ahf_hierarchy* h, void* stream) {
  if (!ctx || !h) return fail(AHF_EINVAL, "ctx and h are required");
  hipStream_t st = (hipStream_t)stream;
  try {
    HIP_CHECK(hipSetDevice(ctx->c.device));
    ctx->ws.bind(&ctx->c, st);
    ctx->ws.reset();
    h->h.mem.st = st;
    label_hierarchy(&ctx->c, ctx->ws, &h->h, st);
    ctx->ws.reset();
  } catch (const Error& e) {
    (void)hipStreamSynchronize(st);
    ctx->ws.reset();
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(AHF_ENOMEM, "host allocation failed");
  }
  return AHF_OK;
}

ahf_status ahf_hierarchy_num_levels(const ahf_hierarchy* h, uint32_t* out) {
  if (!out) return fail(AHF_EINVAL, "out is NULL");
  *out = 0;
  if (!h) return fail(AHF_EINVAL, "h is NULL");
  *out = (uint32_t)h->h.lev.size();
  return AHF_OK;
}

ahf_status ahf_level_get(const ahf_hierarchy* h, uint32_t level, ahf_level_view* v) {
  if (!v) return fail(AHF_EINVAL, "out is NULL");
  std::memset(v, 0, sizeof(*v));
  if (!h) return fail(AHF_EINVAL, "h is NULL");
  if (level >= h->h.lev.size()) return fail(AHF_EINVAL, "level out of range");
  const Level& L = h->h.lev[level];
  v->level = level;
  v->bits = L.b;
  v->n_cells = L.nS;
  v->n_refined = L.nF;
  v->n_particles = L.nP;
  v->n_bricks = L.nB;
  v->n_patches = (level >= 1 && h->h.labelled) ? L.nPatch : 0;
  v->cell_key = L.Skey;
  v->cell_start = L.Sstart;
  v->cell_count = L.Scount;
  v->cell_refined = L.Sflag;
  v->cell_patch = (level >= 1 && h->h.labelled) ? L.Spatch : nullptr;
  v->brick_key = L.Bkey;
  v->brick_cell = L.Bcell;
  v->brick_mass = L.mass;
  if (level >= 1 && h->h.labelled) {
    v->patch_parent = L.patch_parent;
    v->patch_ncells = L.patch_ncells;
    v->patch_nparticles = L.patch_npart;
    v->patch_mass = L.patch_mass;
  }
  v->total_cell_mass = L.tot_cell;
  v->total_particle_mass = L.tot_part;
  v->patch_struct = (level >= 1 && h->h.classified) ? L.patch_struct : nullptr;
  return AHF_OK;
}

ahf_status ahf_classify_substructure(ahf_ctx* ctx, ahf_hierarchy* h, void* stream) {
  if (!ctx || !h) return fail(AHF_EINVAL, "ctx and h are required");
  if (!h->h.labelled) return fail(AHF_EINVAL, "the hierarchy is not labelled");
  hipStream_t st = (hipStream_t)stream;
  try {
    HIP_CHECK(hipSetDevice(ctx->c.device));
    ctx->ws.bind(&ctx->c, st);
    ctx->ws.reset();
    h->h.mem.st = st;
    classify_hierarchy(&ctx->c, ctx->ws, &h->h, st);
    ctx->ws.reset();
  } catch (const Error& e) {
    (void)hipStreamSynchronize(st);
    ctx->ws.reset();
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(AHF_ENOMEM, "host allocation failed");
  }
  return AHF_OK;
}

ahf_status ahf_hierarchy_structures(const ahf_hierarchy* h, ahf_structures* out) {
  if (!out) return fail(AHF_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!h) return fail(AHF_EINVAL, "h is NULL");
  if (!h->h.classified) return fail(AHF_EINVAL, "the hierarchy is not classified");
  out->n_structures = h->h.nStruct;
  out->host = h->h.s_host;
  out->level = h->h.s_level;
  out->patch = h->h.s_patch;
  out->depth = h->h.s_depth;
  return AHF_OK;
}

ahf_status ahf_hierarchy_order(const ahf_hierarchy* h, const uint32_t** sorted_idx) {
  if (!sorted_idx) return fail(AHF_EINVAL, "out is NULL");
  *sorted_idx = nullptr;
  if (!h) return fail(AHF_EINVAL, "h is NULL");
  *sorted_idx = h->h.order;
  return AHF_OK;
}

ahf_status ahf_hierarchy_timings(const ahf_hierarchy* h, double* ms, uint32_t n) {
  if (!h || !ms || n > 4) return fail(AHF_EINVAL, "bad arguments");
  for (uint32_t i = 0; i < n; ++i) ms[i] = h->h.ms[i];
  return AHF_OK;
}

ahf_status ahf_hierarchy_query_label(ahf_ctx* ctx, const ahf_hierarchy* h, uint32_t level,
                                     uint64_t n, const uint64_t* keys, int32_t* out, void* stream) {
  if (!ctx || !h || (n && (!keys || !out))) return fail(AHF_EINVAL, "bad arguments");
  if (level >= h->h.lev.size()) return fail(AHF_EINVAL, "level out of range");
  if (level >= 1 && !h->h.labelled) return fail(AHF_EINVAL, "the hierarchy is not labelled");
  const uint32_t b = h->h.lev[level].b;
  for (uint64_t i = 0; i < n; ++i)
    if (3 * b < 64 && (keys[i] >> (3 * b)) != 0) return fail(AHF_EINVAL, "key beyond the level's bits");
  if (n == 0) return AHF_OK;
  if (level == 0) {
    for (uint64_t i = 0; i < n; ++i) out[i] = -1;
    return AHF_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  try {
    HIP_CHECK(hipSetDevice(ctx->c.device));
    ctx->ws.bind(&ctx->c, st);
    query_labels(ctx->ws, &h->h, (int)level, n, keys, out, st);
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  return AHF_OK;
}

ahf_status ahf_ctx_set_profiling(ahf_ctx* ctx, int enable) {
  if (!ctx) return fail(AHF_EINVAL, "ctx is NULL");
  try {
    HIP_CHECK(hipSetDevice(ctx->c.device));
    ctx->c.prof.clear();
    ctx->c.prof.on = enable != 0;
    // events for a few builds up front: creating them between launches
    // would slow the builds being timed
    while (enable && ctx->c.prof.spare.size() < 2048) {
      hipEvent_t e = nullptr;
      HIP_CHECK(hipEventCreateWithFlags(&e, kTimingEventFlags));
      ctx->c.prof.spare.push_back(e);
    }
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  return AHF_OK;
}

ahf_status ahf_ctx_set_tuning(ahf_ctx* ctx, uint32_t n_entries, const uint64_t* min_n,
                              const ahf_tuning* entries) {
  if (!ctx || (n_entries && (!min_n || !entries))) return fail(AHF_EINVAL, "bad arguments");
  std::vector<std::pair<uint64_t, Tuning>> tab;
  for (uint32_t i = 0; i < n_entries; ++i) {
    const ahf_tuning& e = entries[i];
    if (e.struct_size < sizeof(ahf_tuning)) return fail(AHF_EINVAL, "bad ahf_tuning");
    const uint32_t hv[3] = {e.heavy_level0, e.heavy_level1, e.heavy_deeper};
    Tuning t;
    for (int k = 0; k < 3; ++k) {
      if (hv[k] < 1 || hv[k] > (uint32_t)kHeavyMax)
        return fail(AHF_EINVAL, "heavy thresholds must be in 1..64");
      t.heavy[k] = hv[k];
    }
    if (e.batch_level1 != 2 && e.batch_level1 != 4) return fail(AHF_EINVAL, "batch_level1 must be 2 or 4");
    t.batch1 = e.batch_level1;
    if (e.sort_skip_digits < -1 || e.sort_skip_digits > 2)
      return fail(AHF_EINVAL, "sort_skip_digits must be -1..2");
    t.sort_skip = e.sort_skip_digits;
    tab.emplace_back(min_n[i], t);
  }
  ctx->c.tuning = tab;
  return AHF_OK;
}

ahf_status ahf_ctx_get_tuning(const ahf_ctx* ctx, uint64_t n, ahf_tuning* out) {
  if (!ctx || !out) return fail(AHF_EINVAL, "bad arguments");
  const Tuning t = ctx->c.tuning_for(n);
  out->struct_size = sizeof(ahf_tuning);
  out->heavy_level0 = t.heavy[0];
  out->heavy_level1 = t.heavy[1];
  out->heavy_deeper = t.heavy[2];
  out->batch_level1 = t.batch1;
  out->sort_skip_digits = t.sort_skip;
  return AHF_OK;
}

ahf_status ahf_ctx_profile_only(ahf_ctx* ctx, const char* names) {
  if (!ctx) return fail(AHF_EINVAL, "ctx is NULL");
  ctx->c.prof.only.clear();
  if (names) {
    std::string cur;
    for (const char* p = names;; ++p) {
      if (*p == ',' || *p == 0) {
        if (!cur.empty()) ctx->c.prof.only.push_back(cur);
        cur.clear();
        if (*p == 0) break;
      } else {
        cur.push_back(*p);
      }
    }
  }
  return AHF_OK;
}

ahf_status ahf_ctx_kernel_time(ahf_ctx* ctx, const char* kernel, uint64_t* launches,
                               double* total_ms) {
  if (!ctx || !kernel || !launches || !total_ms) return fail(AHF_EINVAL, "bad arguments");
  *launches = 0;
  *total_ms = 0.0;
  try {
    HIP_CHECK(hipSetDevice(ctx->c.device));
    ctx->c.prof.collect();
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  for (auto& x : ctx->c.prof.acc)
    if (x.first == kernel) {
      *launches = x.second.first;
      *total_ms = x.second.second;
    }
  return AHF_OK;
}

void ahf_hierarchy_free(ahf_hierarchy* h) {
  if (!h) return;
  // builds finish on their stream before they return, and the blocks go back
  // to the context's pool (or its free callback), so no wait is needed here
  h->h.mem.release_all();
  delete h;
}

}  // extern "C"
