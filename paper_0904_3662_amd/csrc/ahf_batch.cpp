// ahf_batch.cpp -- many independent sub-volume builds run with one host wait.
//
// Independent chunks of a volume are analysed separately (Sect. 2.2.3; the
// large runs of Sect. 5.3 are split into 64 chunks).  A batch builds a fixed
// set of sub-volumes again and again:
//   1. every sub-volume is built once on its chain's context, which learns
//      the level sizes of its parameter set and size class;
//   2. every sub-volume is built once more exactly as a run builds it (sized
//      ahead from the learned plan, labels within the build, the status block
//      copied on the device), and the host checks the results; this also
//      grows each chain's scratch memory and each hierarchy's arena to what
//      the builds need;
//   3. a run forks from the caller's stream into each chain, enqueues each
//      chain's builds one after another (each build itself on three streams:
//      cells, deposits, labels) and joins the chains back; nothing in it
//      waits for the host.  The host then reads one status block per
//      sub-volume and completes its hierarchy (level sizes, totals, patch
//      counts, device errors).
// The same enqueue can be recorded into one HIP graph (AHF_BATCH_GRAPH,
// record below); that recording is switched off: the HIP runtime faulted in
// hipStreamEndCapture on it.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <new>
#include <numeric>
#include <thread>

#include "ahf_internal.h"

using namespace ahf;

// AHF_TRACE=1 in the environment: one line on stderr per step of a batch's
// creation and runs
static void trace(const char* what, uint64_t a = 0, uint64_t b = 0) {
  static const bool on = [] {
    const char* e = std::getenv("AHF_TRACE");
    return e && e[0] == '1';
  }();
  if (!on) return;
  std::fprintf(stderr, "ahf_batch: %s %llu %llu\n", what, (unsigned long long)a,
               (unsigned long long)b);
  std::fflush(stderr);
}

struct ahf_batch {
  ahf_ctx* parent = nullptr;
  std::vector<ahf_ctx*> chains;       // a context per chain: streams, scratch, plans
  std::vector<hipStream_t> chain_st;  // the build stream of each chain
  std::vector<hipEvent_t> join_ev;
  hipEvent_t fork_ev = nullptr;
  hipStream_t origin = nullptr;       // the stream the graph is recorded from
  struct Item {
    ahf_particles p{};
    Params prm;
    uint32_t chain = 0;
    Plan plan;
    ahf_hierarchy* h = nullptr;
    std::vector<Level> lev;            // the levels as recorded (capacities)
    const uint32_t* dev_lvcnt = nullptr;
    size_t handed = 0;                 // arena bytes of the sub-volume's build
    ahf_status status = AHF_EINVAL;    // of the last completed run
  };
  std::vector<Item> items;
  std::vector<std::vector<uint32_t>> order;  // the sub-volumes of each chain, in order
  uint64_t* status_dev = nullptr;            // kStatusWords per sub-volume
  size_t status_bytes = 0;
  uint64_t* status_host = nullptr;           // pinned
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t run_st = nullptr;
  bool pending = false;  // a run was enqueued and not yet waited for
  bool ran = false;      // the hierarchies hold a completed run
};

namespace {

ahf_status fail_batch(ahf_status s, const std::string& m) {
  set_last_error(m);
  return s;
}

// enqueues sub-volume i's build, its labels and the copy of its status
// block on its chain's build stream
void enqueue_item(ahf_batch* b, uint32_t i) {
  ahf_batch::Item& it = b->items[i];
  ahf_ctx* c = b->chains[it.chain];
  const hipStream_t st = b->chain_st[it.chain];
  // the previous build of the chain is complete before this one's first
  // kernel (its deposit and label streams were joined back), so the same
  // scratch serves again
  c->ws.bind(&c->c, st);
  c->ws.rewind();
  c->ws_dep.bind(&c->c, st);
  c->ws_dep.rewind();
  Hier* h = &it.h->h;
  build_hierarchy(&c->c, c->ws, c->ws_dep, it.p, it.prm, st, h, false, &it.plan);
  if (!(it.prm.flags & AHF_NO_LABELS)) label_enqueue(&c->c, c->ws, h, st);
  enqueue_status(h, b->status_dev + (size_t)i * kStatusWords, st);
  // the levels as enqueued (sized by the plan): every run completes a copy
  it.lev = h->lev;
  it.dev_lvcnt = h->dev_lvcnt;
}

// sub-volume i's hierarchy emptied for the next build: its arena handed out
// again from the start (the previous build has finished), every other field
// as new
void reset_hier(ahf_batch* b, uint32_t i) {
  ahf_batch::Item& it = b->items[i];
  Hier& h = it.h->h;
  Owned mem = std::move(h.mem);
  Ctx* c = h.ctx;
  h = Hier{};
  h.mem = std::move(mem);
  h.ctx = c;
  h.mem.reuse(it.handed);
}

// a hierarchy object for sub-volume i, its arena on the chain's context
ahf_hierarchy* new_hier(ahf_batch* b, uint32_t i, size_t reserve) {
  ahf_batch::Item& it = b->items[i];
  ahf_ctx* c = b->chains[it.chain];
  ahf_hierarchy* h = new ahf_hierarchy();
  h->h.ctx = &c->c;
  h->h.mem.ctx = &c->c;
  h->h.mem.st = b->chain_st[it.chain];
  if (reserve) h->h.mem.reserve(reserve);
  return h;
}

void free_hiers(ahf_batch* b) {
  for (auto& it : b->items) {
    if (it.h) ahf_hierarchy_free(it.h);
    it.h = nullptr;
  }
}

void sync_chains(ahf_batch* b) {
  for (auto s : b->chain_st) (void)hipStreamSynchronize(s);
  for (auto c : b->chains) {
    if (c->c.dep_st) (void)hipStreamSynchronize(c->c.dep_st);
    if (c->c.lab_st) (void)hipStreamSynchronize(c->c.lab_st);
  }
}

// the status blocks to the host and every hierarchy completed from its own;
// the first failure's status (AHF_OK when none), kStatusReplan included
ahf_status complete_all(ahf_batch* b, std::string* msg) {
  HIP_CHECK(hipMemcpy(b->status_host, b->status_dev, b->status_bytes, hipMemcpyDeviceToHost));
  ahf_status first = AHF_OK;
  for (uint32_t i = 0; i < b->items.size(); ++i) {
    ahf_batch::Item& it = b->items[i];
    Hier* h = &it.h->h;
    // every run starts from the levels as recorded
    h->lev = it.lev;
    h->sizes_known = false;
    h->dev_lvcnt = it.dev_lvcnt;
    h->labelled = false;
    it.status = AHF_OK;
    try {
      finish_from_status(h, b->status_host + (size_t)i * kStatusWords);
    } catch (const Error& e) {
      it.status = e.code;
      if (first == AHF_OK) {
        first = e.code;
        *msg = "sub-volume " + std::to_string(i) + ": " + e.msg;
      }
    }
  }
  return first;
}

void destroy(ahf_batch* b) {
  if (!b) return;
  if (b->parent) (void)hipSetDevice(b->parent->c.device);
  if (b->pending && b->run_st) (void)hipStreamSynchronize(b->run_st);
  sync_chains(b);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto c : b->chains) c->c.recording = false;
  free_hiers(b);
  for (auto c : b->chains) ahf_ctx_destroy(c);
  for (auto s : b->chain_st) (void)hipStreamDestroy(s);
  for (auto e : b->join_ev) (void)hipEventDestroy(e);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->origin) (void)hipStreamDestroy(b->origin);
  if (b->status_dev) ctx_free(&b->parent->c, b->status_dev, b->status_bytes, nullptr);
  if (b->status_host) (void)hipHostFree(b->status_host);
  delete b;
}

ahf_status check_item(const ahf_particles* p, const ahf_params* prm, Params* out) {
  const ahf_status s = check_request(prm, p, out);
  if (s != AHF_OK) return s;
  if (p->n == 0) return fail_batch(AHF_EINVAL, "a sub-volume of a batch needs particles");
  if (p->mass) return fail_batch(AHF_EINVAL, "the sub-volumes of a batch have equal masses");
  if (out->flags & (AHF_DENSITY_CRITERION | AHF_SUBSTRUCTURE))
    return fail_batch(AHF_EINVAL,
                      "AHF_DENSITY_CRITERION and AHF_SUBSTRUCTURE are not available in a batch");
  return AHF_OK;
}

// steps 1 and 2: plans learned, then one rehearsal of the graph's builds;
// a rehearsal that outgrows its plan teaches the plan and runs again
void learn_and_rehearse(ahf_batch* b) {
  const uint32_t n = (uint32_t)b->items.size();
  for (uint32_t i = 0; i < n; ++i) {
    ahf_batch::Item& it = b->items[i];
    trace("learning build", i, it.p.n);
    ahf_params prm{};
    prm.struct_size = sizeof(ahf_params);
    prm.dom_grid_log2 = (uint32_t)it.prm.g;
    prm.dom_ref = it.prm.dom_ref;
    prm.ref_ref = it.prm.ref_ref;
    prm.max_levels = (uint32_t)it.prm.Lmax;
    prm.connectivity = (uint32_t)it.prm.conn;
    prm.flags = it.prm.flags;
    ahf_hierarchy* h = nullptr;
    ahf_ctx* c = b->chains[it.chain];
    const ahf_status s = ahf_build_hierarchy(c, &it.p, &prm, b->chain_st[it.chain], &h);
    if (s != AHF_OK) throw Error{s, ahf_last_error()};
    ahf_hierarchy_free(h);
  }
  for (int attempt = 0;; ++attempt) {
    for (auto& it : b->items) {
      ahf_ctx* c = b->chains[it.chain];
      if (!plan_for(&c->c, it.prm, false, it.p.n, &it.plan))
        throw Error{AHF_EDEVICE, "no plan learned for a sub-volume"};
    }
    for (auto c : b->chains) c->c.in_graph = true;
    for (uint32_t i = 0; i < n; ++i) b->items[i].h = new_hier(b, i, 0);
    for (uint32_t c = 0; c < b->chains.size(); ++c)
      for (uint32_t i : b->order[c]) {
        trace("rehearsal build", i, c);
        enqueue_item(b, i);
      }
    sync_chains(b);
    trace("rehearsal done", attempt);
    for (auto c : b->chains) c->c.in_graph = false;
    std::string msg;
    const ahf_status s = complete_all(b, &msg);
    if (s == AHF_OK) {
      for (auto& it : b->items) it.handed = it.h->h.mem.handed;
      return;
    }
    free_hiers(b);
    if (s != kStatusReplan || attempt >= 3) throw Error{s == kStatusReplan ? AHF_ELIMIT : s, msg};
    // a sub-volume outgrew the plan of its class: a build without a plan
    // sizes it exactly and teaches the plan
    for (auto& it : b->items) {
      if (it.status != kStatusReplan) continue;
      ahf_ctx* c = b->chains[it.chain];
      ahf_params prm{};
      prm.struct_size = sizeof(ahf_params);
      prm.dom_grid_log2 = (uint32_t)it.prm.g;
      prm.dom_ref = it.prm.dom_ref;
      prm.ref_ref = it.prm.ref_ref;
      prm.max_levels = (uint32_t)it.prm.Lmax;
      prm.connectivity = (uint32_t)it.prm.conn;
      prm.flags = it.prm.flags;
      ahf_hierarchy* h = nullptr;
      const ahf_status s2 = ahf_build_hierarchy(c, &it.p, &prm, b->chain_st[it.chain], &h);
      if (s2 != AHF_OK) throw Error{s2, ahf_last_error()};
      ahf_hierarchy_free(h);
    }
  }
}

// a run: fork from stream into the chains, every build enqueued (each
// chain's builds by a host thread of its own: one thread alone could not
// enqueue the launches as fast as the GPU runs them), the chains joined back
// into stream
void enqueue_run(ahf_batch* b, hipStream_t stream) {
  const uint32_t K = (uint32_t)b->chains.size();
  HIP_CHECK(hipEventRecord(b->fork_ev, stream));
  for (auto c : b->chains) c->c.in_graph = true;
  std::vector<std::exception_ptr> errs(K);
  auto chain = [&](uint32_t c) {
    try {
      HIP_CHECK(hipSetDevice(b->parent->c.device));
      HIP_CHECK(hipStreamWaitEvent(b->chain_st[c], b->fork_ev, 0));
      for (uint32_t i : b->order[c]) {
        reset_hier(b, i);
        enqueue_item(b, i);
      }
      HIP_CHECK(hipEventRecord(b->join_ev[c], b->chain_st[c]));
    } catch (...) {
      errs[c] = std::current_exception();
    }
  };
  if (K == 1) {
    chain(0);
  } else {
    std::vector<std::thread> th;
    th.reserve(K);
    for (uint32_t c = 0; c < K; ++c) th.emplace_back(chain, c);
    for (auto& t : th) t.join();
  }
  for (auto c : b->chains) c->c.in_graph = false;
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
  for (uint32_t c = 0; c < K; ++c) HIP_CHECK(hipStreamWaitEvent(stream, b->join_ev[c], 0));
}

// the same enqueue recorded into a graph (switched off: see the top)
void record(ahf_batch* b) {
  const uint32_t n = (uint32_t)b->items.size();
  free_hiers(b);
  for (uint32_t i = 0; i < n; ++i) b->items[i].h = new_hier(b, i, b->items[i].handed);
  for (auto c : b->chains) {
    c->c.in_graph = true;
    c->c.recording = true;
  }
  trace("recording");
  HIP_CHECK(hipStreamBeginCapture(b->origin, hipStreamCaptureModeRelaxed));
  try {
    HIP_CHECK(hipEventRecord(b->fork_ev, b->origin));
    for (uint32_t c = 0; c < b->chains.size(); ++c) {
      HIP_CHECK(hipStreamWaitEvent(b->chain_st[c], b->fork_ev, 0));
      for (uint32_t i : b->order[c]) {
        trace("recording build", i, c);
        enqueue_item(b, i);
      }
      HIP_CHECK(hipEventRecord(b->join_ev[c], b->chain_st[c]));
      HIP_CHECK(hipStreamWaitEvent(b->origin, b->join_ev[c], 0));
    }
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(b->origin, &g);
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    for (auto c : b->chains) c->c.in_graph = c->c.recording = false;
    throw;
  }
  for (auto c : b->chains) c->c.in_graph = c->c.recording = false;
  trace("recorded, ending the capture");
  HIP_CHECK(hipStreamEndCapture(b->origin, &b->graph));
  if (!b->graph) throw Error{AHF_EDEVICE, "the recording gave no graph"};
  trace("instantiating");
  // the error node and the log are written when instantiation fails
  hipGraphNode_t err_node = nullptr;
  char log[512] = {0};
  const hipError_t e = hipGraphInstantiate(&b->exec, b->graph, &err_node, log, sizeof(log) - 1);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b->exec = nullptr;
    throw Error{AHF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e) +
                                 (log[0] ? std::string(": ") + log : std::string())};
  }
  trace("instantiated");
  for (auto& it : b->items) it.status = AHF_EINVAL;
}

}  // namespace

extern "C" {

ahf_status ahf_batch_create(ahf_ctx* ctx, uint32_t n, const ahf_particles* parts,
                            const ahf_params* params, uint32_t n_chains, uint32_t flags,
                            void* stream, ahf_batch** out) {
  if (!out) return fail_batch(AHF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx || !parts || !params || n == 0)
    return fail_batch(AHF_EINVAL, "ctx, parts, params and n >= 1 are required");
  if (n_chains < 1 || n_chains > 16) return fail_batch(AHF_EINVAL, "n_chains must be 1..16");
  if (flags & ~AHF_BATCH_GRAPH) return fail_batch(AHF_EINVAL, "unknown flags");
  if (flags & AHF_BATCH_GRAPH)
    return fail_batch(AHF_EINVAL,
                      "recording a batch into a graph is switched off (the HIP runtime "
                      "faulted in hipStreamEndCapture on it)");
  ahf_batch* b = new (std::nothrow) ahf_batch();
  if (!b) return fail_batch(AHF_ENOMEM, "host allocation failed");
  b->parent = ctx;
  try {
    b->items.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
      const ahf_status s = check_item(&parts[i], &params[i], &b->items[i].prm);
      if (s != AHF_OK) {
        destroy(b);
        return s;
      }
      b->items[i].p = parts[i];
    }
    HIP_CHECK(hipSetDevice(ctx->c.device));
    // the chains: contexts on the parent's device and allocator, with its tuning
    const uint32_t K = std::min(n_chains, n);
    ahf_ctx_desc d{};
    d.struct_size = sizeof(ahf_ctx_desc);
    d.device = ctx->c.device;
    d.alloc = ctx->c.alloc;
    d.free = ctx->c.free;
    d.user = ctx->c.user;
    for (uint32_t c = 0; c < K; ++c) {
      ahf_ctx* cc = nullptr;
      const ahf_status s = ahf_ctx_create(&d, &cc);
      if (s != AHF_OK) throw Error{s, ahf_last_error()};
      cc->c.tuning = ctx->c.tuning;
      cc->c.planning = true;
      // with several chains each build keeps to its chain's stream (the
      // chains fill the GPU; more streams would only share its queues)
      cc->c.one_stream = K > 1;
      b->chains.push_back(cc);
      hipStream_t st = nullptr;
      HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      b->chain_st.push_back(st);
      hipEvent_t e = nullptr;
      HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->join_ev.push_back(e);
    }
    HIP_CHECK(hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
    // largest first, each to the chain with the fewest particles so far
    std::vector<uint32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0u);
    std::stable_sort(idx.begin(), idx.end(),
                     [&](uint32_t a, uint32_t c) { return parts[a].n > parts[c].n; });
    std::vector<uint64_t> load(K, 0);
    b->order.assign(K, {});
    for (uint32_t i : idx) {
      const uint32_t c = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
      b->items[i].chain = c;
      b->order[c].push_back(i);
      load[c] += parts[i].n;
    }
    for (auto& o : b->order) std::sort(o.begin(), o.end());
    b->status_bytes = (size_t)n * kStatusWords * sizeof(uint64_t);
    b->status_dev = static_cast<uint64_t*>(ctx_alloc(&ctx->c, b->status_bytes, nullptr));
    HIP_CHECK(hipHostMalloc((void**)&b->status_host, b->status_bytes, hipHostMallocDefault));
    // the particle arrays may still be in the making on the caller's stream
    HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
    learn_and_rehearse(b);
    if (flags & AHF_BATCH_GRAPH) record(b);
    trace("created", n, K);
  } catch (const Error& e) {
    destroy(b);
    return fail_batch(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    destroy(b);
    return fail_batch(AHF_ENOMEM, "host allocation failed");
  }
  *out = b;
  return AHF_OK;
}

ahf_status ahf_batch_run(ahf_batch* b, void* stream) {
  if (!b) return fail_batch(AHF_EINVAL, "b is NULL");
  if (b->pending) return fail_batch(AHF_EBUSY, "a run is pending: wait for it first");
  try {
    HIP_CHECK(hipSetDevice(b->parent->c.device));
    if (b->exec) {
      trace("launching the graph");
      HIP_CHECK(hipGraphLaunch(b->exec, (hipStream_t)stream));
    } else {
      trace("enqueueing a run");
      enqueue_run(b, (hipStream_t)stream);
    }
  } catch (const Error& e) {
    return fail_batch(e.code, e.msg);
  }
  b->run_st = (hipStream_t)stream;
  b->pending = true;
  b->ran = false;
  return AHF_OK;
}

ahf_status ahf_batch_wait(ahf_batch* b) {
  if (!b) return fail_batch(AHF_EINVAL, "b is NULL");
  if (!b->pending) return b->ran ? AHF_OK : fail_batch(AHF_EINVAL, "the batch has not run");
  std::string msg;
  ahf_status s = AHF_OK;
  try {
    HIP_CHECK(hipSetDevice(b->parent->c.device));
    HIP_CHECK(hipStreamSynchronize(b->run_st));
    b->pending = false;
    trace("run complete");
    s = complete_all(b, &msg);
  } catch (const Error& e) {
    b->pending = false;
    return fail_batch(e.code, e.msg);
  }
  b->ran = true;
  if (s == kStatusReplan) {
    for (auto& it : b->items)
      if (it.status == kStatusReplan) it.status = AHF_ELIMIT;
    return fail_batch(AHF_ELIMIT, msg + " (the batch must be created again)");
  }
  return s == AHF_OK ? AHF_OK : fail_batch(s, msg);
}

ahf_status ahf_batch_status(const ahf_batch* b, uint32_t i) {
  if (!b || i >= b->items.size()) return fail_batch(AHF_EINVAL, "bad arguments");
  if (!b->ran) return fail_batch(AHF_EINVAL, "the batch has not run");
  return b->items[i].status;
}

ahf_status ahf_batch_hierarchy(ahf_batch* b, uint32_t i, ahf_hierarchy** out) {
  if (!out) return fail_batch(AHF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!b || i >= b->items.size()) return fail_batch(AHF_EINVAL, "bad arguments");
  if (!b->ran || b->pending) return fail_batch(AHF_EINVAL, "no completed run");
  if (b->items[i].status != AHF_OK) return fail_batch(AHF_EINVAL, "that sub-volume failed");
  *out = b->items[i].h;
  return AHF_OK;
}

void ahf_batch_destroy(ahf_batch* b) { destroy(b); }

}  // extern "C"
