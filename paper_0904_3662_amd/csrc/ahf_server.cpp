// ahf_server.cpp -- continuous batching of hierarchy builds (ahf_submit/ahf_poll).
//
// n_streams worker threads each own a context (scratch space, memory pool)
// and a HIP stream of default priority.  Requests are admitted in submission
// order when a worker is idle and their footprint fits the HBM budget next to
// the device memory the workers already hold (their results, cached blocks
// and workspaces) and the builds in flight; finished results nobody holds are
// evicted least recently used first, and cached blocks and idle workspaces are
// given back, to make room.  Builds on different workers run concurrently, so
// their kernels overlap on the device.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "ahf_internal.h"

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Footprint of one build before it runs: the sort and record buffers
// (2 x 12 B pairs + 2 x 32 B records per particle), the dense domain grid
// arrays, the refined levels and labels, and the deposit scratch that the
// second stream keeps to the end of the build.  Measured on the device
// (memory in use after a build, result and the context's folded workspace
// included): 209 B per particle at 2^24, 230 at 2e6, 151 MB at 2e5
// particles; the margin covers a first build, whose workspace grows
// geometrically before it is folded to its high-water size.
uint64_t estimate_bytes(uint64_t n, uint32_t g) {
  const uint64_t dense = 1ull << (3 * g);
  return 300ull * n + 48ull * dense + (160ull << 20);
}

struct Request {
  enum State { QUEUED, RUNNING, DONE, FAILED, CANCELED };
  ahf_particles p{};
  ahf_params prm{};
  State state = QUEUED;
  ahf_status status = AHF_OK;
  ahf_hierarchy* h = nullptr;
  uint64_t est = 0;       // bytes charged while running
  uint64_t bytes = 0;     // bytes held once finished
  double t[4] = {0, 0, 0, 0};  // submit, admit, start, end
  uint64_t last_use = 0;
  int pins = 0;           // label queries in progress
  bool held = false;      // polled by the client: never evicted until released
  bool release_when_done = false;
  int worker = -1;        // the worker building or holding it
};

struct Worker {
  ahf_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  std::thread th;
  bool busy = false;      // a build is running (guarded by the server lock)
};

// canceled tickets remembered for ahf_poll (the most recent ones)
constexpr size_t kCanceledKept = 4096;

ahf_status fail(ahf_status c, const std::string& m) {
  ahf::set_last_error(m);
  return c;
}

}  // namespace

struct ahf_server {
  ahf_ctx* parent = nullptr;
  std::vector<Worker> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::map<uint64_t, Request> reqs;
  std::deque<uint64_t> canceled;
  uint64_t next_ticket = 1;
  uint64_t budget = 0, peak = 0, lru = 0;
  uint32_t max_queue = 1024;
  bool stop = false;
  ahf_server_stats st{};
  // label queries run on their own stream with the parent context
  std::mutex qmu;
  hipStream_t qstream = nullptr;
};

namespace {

// frees a finished result (its blocks go back to its worker's pool); caller
// holds the lock
void drop_result(ahf_server* s, Request& r) {
  (void)s;
  if (r.h) ahf_hierarchy_free(r.h);
  r.h = nullptr;
  r.bytes = 0;
}

// Device memory the server accounts for: what every worker's context holds
// (results, cached blocks, workspaces) plus, for each build in flight, what
// its estimate exceeds the workspace its worker already holds (the build
// reuses that first).  Caller holds the lock.
uint64_t in_use(ahf_server* s) {
  uint64_t t = 0;
  for (auto& w : s->workers) t += ahf::ctx_device_bytes(&w.ctx->c);
  for (auto& kv : s->reqs) {
    const Request& r = kv.second;
    if (r.state != Request::RUNNING) continue;
    ahf_ctx* c = s->workers[(size_t)r.worker].ctx;
    const uint64_t have = c->ws.capacity() + c->ws_dep.capacity();
    t += r.est > have ? r.est - have : 0;
  }
  return t;
}

void note_peak(ahf_server* s) { s->peak = std::max(s->peak, in_use(s)); }

// gives back memory that nothing uses: every worker's cached free blocks,
// and the workspaces of idle workers; caller holds the lock
void trim(ahf_server* s, bool workspaces) {
  for (auto& w : s->workers) {
    if (workspaces && !w.busy) {
      w.ctx->ws.free_all();
      w.ctx->ws_dep.free_all();
    }
    ahf::ctx_release_pool(&w.ctx->c);
  }
}

// Makes room for `need` more bytes: cached blocks go first, then the least
// recently used finished results that no client holds, then the idle
// workers' workspaces.  Caller holds the lock.
bool make_room(ahf_server* s, uint64_t need) {
  if (in_use(s) + need <= s->budget) return true;
  trim(s, false);
  while (in_use(s) + need > s->budget) {
    uint64_t best = 0, best_use = ~0ull;
    for (auto& kv : s->reqs) {
      const Request& r = kv.second;
      if (r.state == Request::DONE && r.pins == 0 && !r.held && r.last_use < best_use) {
        best = kv.first;
        best_use = r.last_use;
      }
    }
    if (!best) break;
    Request& r = s->reqs[best];
    drop_result(s, r);
    s->reqs.erase(best);
    s->st.evicted++;
    trim(s, false);
  }
  if (in_use(s) + need <= s->budget) return true;
  trim(s, true);
  return in_use(s) + need <= s->budget;
}

// a label query in progress holds a result that becomes evictable after it
bool any_pinned(ahf_server* s) {
  for (auto& kv : s->reqs)
    if (kv.second.pins > 0) return true;
  return false;
}

size_t running_builds(ahf_server* s) {
  size_t n = 0;
  for (auto& w : s->workers) n += w.busy ? 1 : 0;
  return n;
}

void worker_loop(ahf_server* s, Worker* w) {
  const int wi = (int)(w - s->workers.data());
  for (;;) {
    uint64_t ticket = 0;
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop) return;
        if (!s->queue.empty()) {
          Request& head = s->reqs[s->queue.front()];
          if (make_room(s, head.est)) break;
          if (running_builds(s) == 0 && !any_pinned(s)) {
            // nothing running and nothing left to evict: only results that
            // clients hold are in the way, and waiting would never end
            head.state = Request::FAILED;
            head.status = AHF_ELIMIT;
            head.t[3] = now_ms();
            s->queue.pop_front();
            s->st.failed++;
            s->cv_done.notify_all();
            continue;
          }
        }
        s->cv_work.wait(lk);
      }
      ticket = s->queue.front();
      s->queue.pop_front();
      r = &s->reqs[ticket];
      r->state = Request::RUNNING;
      r->worker = wi;
      r->t[1] = now_ms();
      w->busy = true;
      note_peak(s);
    }
    ahf_hierarchy* h = nullptr;
    const double t0 = now_ms();
    const ahf_status rc = ahf_build_hierarchy(w->ctx, &r->p, &r->prm, (void*)w->st, &h);
    const double t1 = now_ms();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      w->busy = false;
      r->t[2] = t0;
      r->t[3] = t1;
      if (rc == AHF_OK) {
        r->state = Request::DONE;
        r->h = h;
        r->bytes = ahf::hier_bytes(&h->h);
        s->st.completed++;
      } else {
        r->state = Request::FAILED;
        r->status = rc;
        s->st.failed++;
      }
      note_peak(s);
      r->last_use = ++s->lru;
      if (r->release_when_done) {
        drop_result(s, *r);
        s->reqs.erase(ticket);
        s->st.released++;
      }
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

ahf_status ahf_server_create(ahf_ctx* ctx, const ahf_server_desc* desc, ahf_server** out) {
  if (!out) return fail(AHF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx || !desc || desc->struct_size < sizeof(ahf_server_desc))
    return fail(AHF_EINVAL, "bad server description");
  if (desc->n_streams < 1 || desc->n_streams > 16) return fail(AHF_EINVAL, "n_streams must be 1..16");
  ahf_server* s = new (std::nothrow) ahf_server();
  if (!s) return fail(AHF_ENOMEM, "host allocation failed");
  s->parent = ctx;
  s->max_queue = desc->max_queue ? desc->max_queue : 1024;
  if (hipSetDevice(ctx->c.device) != hipSuccess) {
    delete s;
    return fail(AHF_EDEVICE, "hipSetDevice failed");
  }
  s->budget = desc->hbm_budget;
  if (!s->budget) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return fail(AHF_EDEVICE, "hipMemGetInfo failed");
    }
    s->budget = (uint64_t)(0.8 * (double)fr);
  }
  if (hipStreamCreateWithFlags(&s->qstream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return fail(AHF_EDEVICE, "hipStreamCreate failed");
  }
  s->workers.resize(desc->n_streams);
  for (auto& w : s->workers) {
    ahf_ctx_desc d{sizeof(ahf_ctx_desc), ctx->c.device, ctx->c.alloc, ctx->c.free, ctx->c.user};
    if (ahf_ctx_create(&d, &w.ctx) != AHF_OK ||
        hipStreamCreateWithFlags(&w.st, hipStreamNonBlocking) != hipSuccess) {
      for (auto& v : s->workers) {
        if (v.st) (void)hipStreamDestroy(v.st);
        if (v.ctx) ahf_ctx_destroy(v.ctx);
      }
      (void)hipStreamDestroy(s->qstream);
      delete s;
      return fail(AHF_EDEVICE, "worker set-up failed");
    }
  }
  // several workers: each build on its worker's one stream (measured on 64
  // sub-volumes: 2.8 against 2.0 G particles/s at 4 workers)
  for (auto& w : s->workers) {
    w.ctx->c.one_stream = s->workers.size() > 1;
    w.ctx->c.tuning = ctx->c.tuning;
  }
  for (auto& w : s->workers) w.th = std::thread(worker_loop, s, &w);
  *out = s;
  return AHF_OK;
}

ahf_status ahf_submit(ahf_server* s, const ahf_particles* p, const ahf_params* prm, uint64_t* ticket) {
  if (!ticket) return fail(AHF_EINVAL, "ticket is NULL");
  *ticket = 0;
  if (!s) return fail(AHF_EINVAL, "bad arguments");
  ahf::Params checked;
  const ahf_status cs = ahf::check_request(prm, p, &checked);
  if (cs != AHF_OK) return cs;
  const uint32_t g = prm->dom_grid_log2;
  const uint64_t est = estimate_bytes(p->n, g);
  std::lock_guard<std::mutex> lk(s->mu);
  if (est > s->budget) return fail(AHF_ELIMIT, "request footprint exceeds the HBM budget");
  if (s->queue.size() >= s->max_queue) return fail(AHF_EBUSY, "queue full");
  const uint64_t t = s->next_ticket++;
  Request& r = s->reqs[t];
  r.p = *p;
  r.prm = *prm;
  r.est = est;
  r.t[0] = now_ms();
  s->queue.push_back(t);
  s->st.submitted++;
  *ticket = t;
  s->cv_work.notify_one();
  return AHF_OK;
}

static ahf_status poll_locked(ahf_server* s, uint64_t ticket, ahf_hierarchy** h) {
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(AHF_ENOTFOUND, "unknown ticket");
  Request& r = it->second;
  if (r.state == Request::QUEUED || r.state == Request::RUNNING) return AHF_PENDING;
  if (r.state == Request::FAILED) return fail(r.status, "the build failed");
  if (r.state == Request::CANCELED) return fail(AHF_ECANCELED, "the request was canceled");
  // the client holds the result from here on: it is not evicted until
  // ahf_release, so the handle stays valid
  r.held = true;
  r.last_use = ++s->lru;
  *h = r.h;
  return AHF_OK;
}

ahf_status ahf_poll(ahf_server* s, uint64_t ticket, ahf_hierarchy** h) {
  if (!h) return fail(AHF_EINVAL, "h is NULL");
  *h = nullptr;
  if (!s) return fail(AHF_EINVAL, "s is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  return poll_locked(s, ticket, h);
}

ahf_status ahf_wait(ahf_server* s, uint64_t ticket, ahf_hierarchy** h) {
  if (!h) return fail(AHF_EINVAL, "h is NULL");
  *h = nullptr;
  if (!s) return fail(AHF_EINVAL, "s is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    const ahf_status rc = poll_locked(s, ticket, h);
    if (rc != AHF_PENDING) return rc;
    s->cv_done.wait(lk);
  }
}

ahf_status ahf_query_label(ahf_server* s, uint64_t ticket, uint32_t level, uint64_t n,
                           const uint64_t* keys, int32_t* out) {
  if (!s) return fail(AHF_EINVAL, "s is NULL");
  ahf_hierarchy* h = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(AHF_ENOTFOUND, "unknown ticket");
    Request& r = it->second;
    if (r.state != Request::DONE) return r.state == Request::FAILED ? fail(r.status, "the build failed")
                                                                    : AHF_PENDING;
    r.pins++;
    r.last_use = ++s->lru;
    h = r.h;
  }
  ahf_status rc;
  {
    std::lock_guard<std::mutex> qk(s->qmu);
    rc = ahf_hierarchy_query_label(s->parent, h, level, n, keys, out, (void*)s->qstream);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    Request& r = s->reqs[ticket];
    r.pins--;
    if (r.pins == 0 && r.release_when_done) {
      drop_result(s, r);
      s->reqs.erase(ticket);
      s->st.released++;
    }
  }
  s->cv_work.notify_all();
  return rc;
}

ahf_status ahf_release(ahf_server* s, uint64_t ticket) {
  if (!s) return fail(AHF_EINVAL, "s is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(AHF_ENOTFOUND, "unknown ticket");
  Request& r = it->second;
  if (r.state == Request::RUNNING || r.pins > 0) {
    r.release_when_done = true;
    return AHF_OK;
  }
  if (r.state == Request::QUEUED) {
    // canceled before it ran: its poll answers AHF_ECANCELED (the most
    // recent kCanceledKept canceled tickets are remembered)
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
    r.state = Request::CANCELED;
    r.t[3] = now_ms();
    s->canceled.push_back(ticket);
    if (s->canceled.size() > kCanceledKept) {
      s->reqs.erase(s->canceled.front());
      s->canceled.pop_front();
    }
    s->st.released++;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
    return AHF_OK;
  }
  if (r.state == Request::CANCELED) {
    s->canceled.erase(std::find(s->canceled.begin(), s->canceled.end(), ticket));
  } else {
    drop_result(s, r);
    s->st.released++;
  }
  s->reqs.erase(it);
  s->cv_work.notify_all();
  return AHF_OK;
}

ahf_status ahf_ticket_times(ahf_server* s, uint64_t ticket, double* t) {
  if (!s || !t) return fail(AHF_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(AHF_ENOTFOUND, "unknown ticket");
  for (int i = 0; i < 4; ++i) t[i] = it->second.t[i];
  return AHF_OK;
}

ahf_status ahf_server_get_stats(ahf_server* s, ahf_server_stats* out) {
  if (!s || !out) return fail(AHF_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queued = s->queue.size();
  out->running = 0;
  out->resident = 0;
  out->bytes_results = 0;
  for (auto& kv : s->reqs) {
    if (kv.second.state == Request::RUNNING) out->running++;
    if (kv.second.state == Request::DONE) {
      out->resident++;
      out->bytes_results += kv.second.bytes;
    }
  }
  out->bytes_in_use = in_use(s);
  out->bytes_peak = s->peak;
  return AHF_OK;
}

void ahf_server_destroy(ahf_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& w : s->workers)
    if (w.th.joinable()) w.th.join();
  for (auto& kv : s->reqs)
    if (kv.second.h) ahf_hierarchy_free(kv.second.h);
  s->reqs.clear();
  for (auto& w : s->workers) {
    (void)hipStreamSynchronize(w.st);
    (void)hipStreamDestroy(w.st);
    ahf_ctx_destroy(w.ctx);
  }
  (void)hipStreamDestroy(s->qstream);
  delete s;
}

}  // extern "C"
