// Batched solves and the serving loop (continuous batching).
//
// pf_solve_batch runs many cases through one launch sequence per Newton phase
// (newton.cpp).  The serving loop instead keeps a table of running requests,
// each an instance whose own launch plan (the case's single-case batch, its
// Newton step captured as a HIP graph) is replayed on one of a few streams, so
// that the requests' work overlaps on the device and admission or retirement
// changes nothing but the table:
//   - admission, first come first served: the head request is admitted when a
//     slot is free and the device pool can lend its working storage (factor
//     values and dense block; for Newton-Krylov also the Krylov storage), a
//     case that holds its own storage needing none; the pool is one
//     allocation of the configured budget, so the budget bounds what served
//     requests hold, and nothing is allocated while requests run;
//   - each admitted request starts its iteration and queues as many Newton
//     steps as its case's last LU solve took, then a gather of its state into
//     pinned host memory and an event;
//   - whenever a request's event has completed, the loop reads its state:
//     finished requests retire (result published, storage back to the pool),
//     the others get their next step.
// An instance's arithmetic is the same alone, in a batch and served.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <thread>

#include "internal.hpp"
#include "kernels.hpp"

namespace pfi {

namespace {

constexpr size_t kBatchCache = 4;  // batches of recent pf_solve_batch calls kept
constexpr int kStreams = 4;        // served requests spread over this many streams
constexpr size_t kAlign = 256;
constexpr size_t kGrowChunk = size_t(256) << 20;  // pool growth without a budget

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket;
  Case* c;
  pf_options opt;
  Clock::time_point submitted;
};

size_t al(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// Device memory lent to served requests: chunks with first-fit free lists
// (offset -> length), neighbours merged on return.  With a budget the pool is
// one chunk of that size, made when the budget is set; without one it grows
// by chunks of at least kGrowChunk as requests need them.
struct Pool {
  struct Chunk {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free;
  };
  std::vector<Chunk> chunks;
  size_t budget = 0;
  size_t lent = 0;

  char* take(Ctx* ctx, size_t bytes) {
    if (bytes == 0) return nullptr;
    bytes = al(bytes);
    for (auto& ch : chunks)
      for (auto it = ch.free.begin(); it != ch.free.end(); ++it)
        if (it->second >= bytes) {
          const size_t off = it->first, len = it->second;
          ch.free.erase(it);
          if (len > bytes) ch.free[off + bytes] = len - bytes;
          lent += bytes;
          return ch.base + off;
        }
    if (budget) return nullptr;
    Chunk ch;
    ch.size = std::max(bytes, kGrowChunk);
    ch.base = (char*)ctx->dalloc(ch.size);
    if (!ch.base) return nullptr;
    if (ch.size > bytes) ch.free[bytes] = ch.size - bytes;
    chunks.push_back(ch);
    lent += bytes;
    return chunks.back().base;
  }
  void give(char* p, size_t bytes) {
    if (!p) return;
    bytes = al(bytes);
    for (auto& ch : chunks) {
      if (p < ch.base || p >= ch.base + ch.size) continue;
      size_t off = (size_t)(p - ch.base), len = bytes;
      auto nx = ch.free.lower_bound(off);
      if (nx != ch.free.end() && nx->first == off + len) {
        len += nx->second;
        nx = ch.free.erase(nx);
      }
      if (nx != ch.free.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
          off = pv->first;
          len += pv->second;
          ch.free.erase(pv);
        }
      }
      ch.free[off] = len;
      lent -= bytes;
      return;
    }
  }
  void release(Ctx* ctx) {
    for (auto& ch : chunks) ctx->dfree(ch.base);
    chunks.clear();
    lent = 0;
  }
  bool make_budget(Ctx* ctx, size_t b) {
    release(ctx);
    budget = b;
    if (!b) return true;
    Chunk ch;
    ch.size = al(b);
    ch.base = (char*)ctx->dalloc(ch.size);
    if (!ch.base) {
      budget = 0;
      return false;
    }
    ch.free[0] = ch.size;
    chunks.push_back(ch);
    return true;
  }
};

// A running request.
struct Slot {
  Request r;
  Batch* b = nullptr;  // the case's own launch plan
  int si = 0;          // stream index
  int ei = 0;          // event index
  char* wlent = nullptr;
  size_t wl = 0;
  char* klent = nullptr;
  size_t kl = 0;
  Clock::time_point admitted;
};

// Working storage a request needs from the pool (its case's own storage, if
// any, is used instead).
void needs(const Request& r, size_t* w, size_t* k) {
  const Case* c = r.c;
  *w = c->wbase ? 0 : c->wbytes;
  *k = 0;
  if (r.opt.solver != PF_SOLVER_LU && !(c->kbase && c->km >= r.opt.gmres_m)) *k = krylov_bytes(c, r.opt.gmres_m);
}

}  // namespace

struct Server {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> queue;
  std::map<uint64_t, pf_result> done;
  std::map<uint64_t, int> state;  // 0 queued or running, 1 done
  uint64_t next = 1;
  bool stop = false;
  int max_slots = 32;
  int running = 0;
  Pool pool;  // guarded by mu
  std::thread worker;
};

pf_status step_batch(Batch* b, const pf_options* opt);   // newton.cpp
pf_status start_batch(Batch* b, const pf_options* opt);  // newton.cpp

namespace {

void publish(Server* sv, const Request& r, const pf_result& res) {
  r.c->busy.store(0);
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->done[r.ticket] = res;
  sv->state[r.ticket] = 1;
}

// a request that could not run: device or allocation failure
void fail(Server* sv, const Request& r, pf_status why) {
  pf_result res;
  std::memset(&res, 0, sizeof res);
  res.status = PF_FAILED;
  res.error = why;
  publish(sv, r, res);
}

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Loop {
  Ctx* ctx;
  Server* sv;
  hipStream_t streams[kStreams] = {};
  std::vector<hipEvent_t> events;
  std::vector<int> ev_free;
  std::vector<Slot> slots;
  int load[kStreams] = {};

  bool init() {
    if (hipSetDevice(ctx->device) != hipSuccess) return false;
    for (auto& s : streams)
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return false;
    return true;
  }
  void fini() {
    for (auto& s : streams)
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    for (auto e : events) (void)hipEventDestroy(e);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->pool.release(ctx);
  }
  int event() {
    if (!ev_free.empty()) {
      const int i = ev_free.back();
      ev_free.pop_back();
      return i;
    }
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return -1;
    events.push_back(e);
    return (int)events.size() - 1;
  }
  // lent storage back to the pool (a case's own storage stays with it)
  void give_back(Slot& s) {
    if (s.wlent) detach_work(s.r.c);
    if (s.klent) detach_krylov(s.r.c);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->pool.give(s.wlent, s.wl);
    sv->pool.give(s.klent, s.kl);
    sv->running--;
  }
  // ... and the plan back on the context's stream, the slot's event free
  void release(Slot& s) {
    give_back(s);
    s.b->stream = ctx->stream;
    load[s.si]--;
    ev_free.push_back(s.ei);
  }
  // the state gather and the event that tells the host it has landed
  bool mark(Slot& s) {
    pfd::launch_gather_red(s.b->stream, s.b->d_insts, 1, s.b->h_reds);
    return hipEventRecord(events[s.ei], s.b->stream) == hipSuccess && launch_status("pf_submit") == PF_OK;
  }
  bool start(Slot& s) {
    int si = 0;
    for (int i = 1; i < kStreams; ++i)
      if (load[i] < load[si]) si = i;
    s.si = si;
    s.ei = event();
    if (s.ei < 0) return false;
    load[si]++;
    Batch* b = s.b;
    b->stream = streams[si];
    Case* c = s.r.c;
    if (s.wlent) attach_work(c, s.wlent, false, b->stream);
    if (s.klent && !attach_krylov(c, s.r.opt.gmres_m, s.klent, false, b->stream)) return false;
    if (start_batch(b, &s.r.opt) != PF_OK) return false;
    if (s.r.opt.solver == PF_SOLVER_LU)
      for (int k = 0; k < std::min(b->lu_steps, s.r.opt.max_iter); ++k)
        if (step_batch(b, &s.r.opt) != PF_OK) return false;
    return mark(s);
  }

  void run() {
    for (;;) {
      std::vector<Slot> fresh;
      std::vector<std::pair<Request, pf_status>> refused;
      {
        std::unique_lock<std::mutex> lk(sv->mu);
        if (slots.empty()) sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
        if (sv->stop && sv->queue.empty() && slots.empty()) return;
        // first come, first served: the head waits until it fits
        while (!sv->queue.empty() && (int)(slots.size() + fresh.size()) < sv->max_slots) {
          const Request& r = sv->queue.front();
          size_t w, k;
          needs(r, &w, &k);
          if (sv->pool.budget && al(w) + al(k) > sv->pool.budget) {
            refused.push_back({r, PF_E_NOMEM});
            sv->queue.pop_front();
            continue;
          }
          Slot s;
          s.wlent = sv->pool.take(ctx, w);
          s.klent = sv->pool.take(ctx, k);
          if ((w && !s.wlent) || (k && !s.klent)) {
            sv->pool.give(s.wlent, w);
            sv->pool.give(s.klent, k);
            if (!sv->pool.budget) {  // the growth allocation itself failed
              refused.push_back({r, PF_E_NOMEM});
              sv->queue.pop_front();
              continue;
            }
            break;
          }
          s.wl = s.wlent ? w : 0;
          s.kl = s.klent ? k : 0;
          s.r = r;
          s.b = r.c->single;
          sv->queue.pop_front();
          sv->running++;
          fresh.push_back(s);
        }
      }
      for (auto& f : refused) fail(sv, f.first, f.second);
      bool progress = !fresh.empty() || !refused.empty();
      {
        std::lock_guard<std::mutex> lk(ctx->launch_mu);
        ctx->prof_off = true;
        for (auto& s : fresh) {
          s.admitted = Clock::now();
          if (!start(s)) {
            if (s.ei >= 0) (void)hipStreamSynchronize(s.b->stream);
            const pf_status why = launch_status("pf_submit") == PF_OK ? PF_E_NOMEM : PF_E_DEVICE;
            if (s.ei < 0)
              give_back(s);
            else
              release(s);
            fail(sv, s.r, why);
            continue;
          }
          slots.push_back(s);
        }
        // every request whose queued work has landed: retire or step
        for (size_t i = 0; i < slots.size();) {
          Slot& s = slots[i];
          const hipError_t q = hipEventQuery(events[s.ei]);
          if (q == hipErrorNotReady) {
            ++i;
            continue;
          }
          progress = true;
          pfd::Red red;
          std::memcpy(&red, (const void*)s.b->h_reds, sizeof red);
          pf_status bad = PF_OK;
          if (q != hipSuccess) {
            (void)hipGetLastError();
            bad = PF_E_DEVICE;
          } else if (red.timeout) {
            bad = PF_E_DEVICE;
          } else if (red.active) {
            if (step_batch(s.b, &s.r.opt) != PF_OK || !mark(s)) bad = PF_E_DEVICE;
            if (bad == PF_OK) {
              ++i;
              continue;
            }
          }
          if (bad != PF_OK) {
            (void)hipStreamSynchronize(s.b->stream);
            release(s);
            fail(sv, s.r, bad);
          } else {
            pf_result res;
            std::memset(&res, 0, sizeof res);
            res.status = red.status;
            res.iters = red.it;
            res.linear_iters = red.linear_iters;
            res.mismatch_inf = red.last_norm;
            res.max_step = red.last_step;
            const auto now = Clock::now();
            res.device_ms = ms_between(s.admitted, now);
            res.wait_ms = ms_between(s.r.submitted, s.admitted);
            if (s.r.opt.solver == PF_SOLVER_LU) s.b->lu_steps = red.it;
            release(s);
            publish(sv, s.r, res);
          }
          slots.erase(slots.begin() + i);
        }
        ctx->prof_off = false;
      }
      if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
};

void serve_loop(Ctx* ctx) {
  Loop L;
  L.ctx = ctx;
  L.sv = ctx->server.get();
  if (!L.init()) {
    // no streams: every request fails until shutdown
    for (;;) {
      std::unique_lock<std::mutex> lk(L.sv->mu);
      L.sv->cv.wait(lk, [&] { return L.sv->stop || !L.sv->queue.empty(); });
      if (L.sv->queue.empty()) break;
      Request r = L.sv->queue.front();
      L.sv->queue.pop_front();
      lk.unlock();
      fail(L.sv, r, PF_E_DEVICE);
    }
    L.fini();
    return;
  }
  L.run();
  L.fini();
}

}  // namespace

}  // namespace pfi

using namespace pfi;

extern "C" {

void pf_serve_shutdown(pf_ctx* ctx) {
  if (!ctx || !ctx->server) return;
  {
    std::lock_guard<std::mutex> lk(ctx->server->mu);
    ctx->server->stop = true;
  }
  ctx->server->cv.notify_all();
  if (ctx->server->worker.joinable()) ctx->server->worker.join();
  {
    std::lock_guard<std::mutex> lk(ctx->server->mu);
    ctx->server->pool.release(ctx);
  }
  ctx->server.reset();
}

pf_status pf_solve_batch(pf_ctx* ctx, pf_case* const* cases, int32_t count, const pf_options* opt,
                         pf_result* results) {
  if (!ctx || (count > 0 && (!cases || !results)) || count < 0) {
    set_error("pf_solve_batch: bad argument");
    return PF_E_INVALID;
  }
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  std::vector<Case*> cs;
  for (int i = 0; i < count; ++i) {
    if (!cases[i] || cases[i]->ctx != ctx) {
      set_error("pf_solve_batch: case belongs to another context");
      return PF_E_INVALID;
    }
    if (cases[i]->busy.load()) {
      set_error("pf_solve_batch: a case is queued or running");
      return PF_E_BUSY;
    }
    for (int k = 0; k < i; ++k)
      if (cases[k] == cases[i]) {
        set_error("pf_solve_batch: a case appears twice");
        return PF_E_INVALID;
      }
    cs.push_back(cases[i]);
  }
  if (count == 0) return PF_OK;
  std::lock_guard<std::mutex> lk(ctx->launch_mu);
  // reuse the batch of an earlier call over the same cases (its work lists,
  // Krylov lists and captured graphs), else build one and keep it
  Batch* b = nullptr;
  for (size_t i = 0; i < ctx->bcache.size(); ++i)
    if (ctx->bcache[i]->cases == cs) {
      b = ctx->bcache[i];
      ctx->bcache.erase(ctx->bcache.begin() + i);
      break;
    }
  if (!b) {
    b = new Batch();
    if (!b->build(ctx, cs)) {
      delete b;
      set_error("pf_solve_batch: batch set-up failed");
      return PF_E_NOMEM;
    }
    b->allow_graph = true;
  }
  ctx->bcache.insert(ctx->bcache.begin(), b);
  while (ctx->bcache.size() > kBatchCache) {
    delete ctx->bcache.back();
    ctx->bcache.pop_back();
  }
  return run_batch(b, &o, results);
}

pf_status pf_serve_config(pf_ctx* ctx, size_t max_bytes, int32_t max_slots) {
  if (!ctx || max_slots < 0) {
    set_error("pf_serve_config: bad argument");
    return PF_E_INVALID;
  }
  if (!ctx->server) ctx->server = std::make_shared<Server>();
  Server* sv = ctx->server.get();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (max_slots > 0) sv->max_slots = max_slots;
  if (max_bytes == sv->pool.budget && !(max_bytes && sv->pool.chunks.empty())) return PF_OK;
  if (!sv->queue.empty() || sv->running > 0) {
    set_error("pf_serve_config: the budget changes only while no request is queued or running");
    return PF_E_BUSY;
  }
  if (!sv->pool.make_budget(ctx, max_bytes)) {
    set_error("pf_serve_config: device allocation of the pool failed");
    return PF_E_NOMEM;
  }
  return PF_OK;
}

pf_status pf_serve_stats(pf_ctx* ctx, size_t* pool_bytes, size_t* lent_bytes, int32_t* queued, int32_t* running) {
  if (!ctx || !pool_bytes || !lent_bytes || !queued || !running) {
    set_error("pf_serve_stats: NULL argument");
    return PF_E_INVALID;
  }
  *pool_bytes = *lent_bytes = 0;
  *queued = *running = 0;
  if (!ctx->server) return PF_OK;
  Server* sv = ctx->server.get();
  std::lock_guard<std::mutex> lk(sv->mu);
  for (const auto& ch : sv->pool.chunks) *pool_bytes += ch.size;
  *lent_bytes = sv->pool.lent;
  *queued = (int32_t)sv->queue.size();
  *running = sv->running;
  return PF_OK;
}

pf_status pf_submit(pf_ctx* ctx, pf_case* c, const pf_options* opt, uint64_t* ticket) {
  if (!ctx || !c || !ticket || c->ctx != ctx) {
    set_error("pf_submit: bad argument");
    return PF_E_INVALID;
  }
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  if (check_opts(&o) != PF_OK) return PF_E_INVALID;
  int expect = 0;
  if (!c->busy.compare_exchange_strong(expect, 1)) {
    set_error("pf_submit: case already queued or running");
    return PF_E_BUSY;
  }
  {
    // the case's own launch plan (and, for Newton-Krylov, its Krylov launch
    // lists), made here so that the serving loop allocates nothing
    std::lock_guard<std::mutex> lk(ctx->launch_mu);
    if (!c->single) {
      auto* b = new Batch();
      if (!b->build(ctx, {c})) {
        delete b;
        c->busy.store(0);
        set_error("pf_submit: launch-plan set-up failed");
        return PF_E_NOMEM;
      }
      b->allow_graph = true;
      c->single = b;
    }
    if (o.solver != PF_SOLVER_LU && !c->single->kbuilt && !c->single->build_krylov()) {
      c->busy.store(0);
      set_error("pf_submit: Krylov launch-list set-up failed");
      return PF_E_NOMEM;
    }
  }
  if (!ctx->server) ctx->server = std::make_shared<Server>();
  Server* sv = ctx->server.get();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->worker.joinable()) sv->worker = std::thread(serve_loop, (Ctx*)ctx);
    *ticket = sv->next++;
    Request r;
    r.ticket = *ticket;
    r.c = c;
    r.opt = o;
    r.submitted = Clock::now();
    sv->queue.push_back(r);
    sv->state[*ticket] = 0;
  }
  sv->cv.notify_one();
  return PF_OK;
}

pf_status pf_poll(pf_ctx* ctx, uint64_t ticket, pf_result* out, int32_t* done) {
  if (!ctx || !out || !done) {
    set_error("pf_poll: bad argument");
    return PF_E_INVALID;
  }
  *done = 0;
  if (!ctx->server) {
    set_error("pf_poll: unknown ticket");
    return PF_E_NOTFOUND;
  }
  Server* sv = ctx->server.get();
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->state.find(ticket);
  if (it == sv->state.end()) {
    set_error("pf_poll: unknown ticket");
    return PF_E_NOTFOUND;
  }
  if (it->second == 1) {
    *out = sv->done[ticket];
    *done = 1;
    sv->done.erase(ticket);
    sv->state.erase(it);
  } else {
    std::memset(out, 0, sizeof *out);
    out->status = PF_PENDING;
  }
  return PF_OK;
}

}  // extern "C"
