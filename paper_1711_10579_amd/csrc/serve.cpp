// Batched solves and the serving loop (continuous batching).
//
// The server thread keeps a running batch.  At every Newton-step boundary it
// retires the instances whose iteration has finished (their results become
// visible to pf_poll), admits queued requests while batch slots and the
// device-byte budget allow (requests of one batch share their options), runs
// the start of the iteration for the newcomers, rebuilds the batch schedule
// and launches the next Newton step of every active instance together.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>

#include "internal.hpp"
#include "kernels.hpp"

namespace pfi {

namespace {

constexpr size_t kBatchCache = 4;  // batches of recent pf_solve_batch calls kept

struct Request {
  uint64_t ticket;
  Case* c;
  pf_options opt;
  hipEvent_t start_ev = nullptr;
};

bool same_opts(const pf_options& a, const pf_options& b) {
  return a.tol == b.tol && a.max_iter == b.max_iter && a.solver == b.solver && a.precision == b.precision &&
         a.precond == b.precond && a.gmres_m == b.gmres_m && a.gmres_max_restarts == b.gmres_max_restarts &&
         a.flat_start == b.flat_start && a.eta_max == b.eta_max;
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
  size_t max_bytes = 0;
  int max_slots = 64;
  std::thread worker;
};

pf_status step_batch(Batch* b, const pf_options* opt);                      // newton.cpp
pf_status start_batch(Batch* b, const pf_options* opt);                     // newton.cpp
pf_status read_batch(Batch* b, std::vector<pfd::Red>* h);                   // newton.cpp

static void finish(Server* sv, const Request& r, const pfd::Red& red) {
  pf_result res;
  std::memset(&res, 0, sizeof res);
  res.status = red.status;
  res.iters = red.it;
  res.linear_iters = red.linear_iters;
  res.mismatch_inf = red.last_norm;
  res.max_step = red.last_step;
  r.c->busy.store(0);
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->done[r.ticket] = res;
  sv->state[r.ticket] = 1;
}

static void fail(Server* sv, const Request& r) {
  pfd::Red red;
  std::memset(&red, 0, sizeof red);
  red.status = PF_DIVERGED;
  finish(sv, r, red);
}

static void serve_loop(Ctx* ctx) {
  Server* sv = ctx->server.get();
  std::vector<Request> run;  // instances in the running batch
  std::unique_ptr<Batch> batch;
  pf_options bopt;
  std::vector<pfd::Red> h;
  for (;;) {
    // admit
    std::vector<Request> fresh;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (run.empty()) sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop && sv->queue.empty() && run.empty()) return;
      size_t bytes = 0;
      for (auto& r : run) bytes += r.c->bytes;
      for (auto it = sv->queue.begin(); it != sv->queue.end();) {
        if ((int)(run.size() + fresh.size()) >= sv->max_slots) break;
        if (run.empty() && fresh.empty()) bopt = it->opt;
        if (!same_opts(it->opt, bopt)) {
          ++it;
          continue;
        }
        if (sv->max_bytes && bytes + it->c->bytes > sv->max_bytes && !(run.empty() && fresh.empty())) break;
        bytes += it->c->bytes;
        fresh.push_back(*it);
        it = sv->queue.erase(it);
      }
    }
    std::lock_guard<std::mutex> lk(ctx->launch_mu);
    if (!fresh.empty()) {
      std::vector<Case*> fc;
      for (auto& r : fresh) fc.push_back(r.c);
      Batch nb;
      if (!nb.build(ctx, fc) || start_batch(&nb, &bopt) != PF_OK) {
        for (auto& r : fresh) fail(sv, r);
        fresh.clear();
      }
    }
    if (!fresh.empty() || !batch) {
      for (auto& r : fresh) run.push_back(r);
      std::vector<Case*> cs;
      for (auto& r : run) cs.push_back(r.c);
      batch.reset(new Batch());
      if (!run.empty() && !batch->build(ctx, cs)) {
        for (auto& r : run) fail(sv, r);
        run.clear();
        batch.reset();
        continue;
      }
    }
    if (run.empty()) {
      batch.reset();
      continue;
    }
    // retire finished instances (after the newcomers' first convergence test)
    if (read_batch(batch.get(), &h) != PF_OK) {
      for (auto& r : run) fail(sv, r);
      run.clear();
      batch.reset();
      continue;
    }
    std::vector<Request> keep;
    for (size_t i = 0; i < run.size(); ++i) {
      if (h[i].active)
        keep.push_back(run[i]);
      else
        finish(sv, run[i], h[i]);
    }
    if (keep.size() != run.size()) {
      run.swap(keep);
      batch.reset();
      if (run.empty()) continue;
      std::vector<Case*> cs;
      for (auto& r : run) cs.push_back(r.c);
      batch.reset(new Batch());
      if (!batch->build(ctx, cs)) {
        for (auto& r : run) fail(sv, r);
        run.clear();
        batch.reset();
        continue;
      }
    }
    // one Newton step of every active instance
    if (step_batch(batch.get(), &bopt) != PF_OK) {
      for (auto& r : run) fail(sv, r);
      run.clear();
      batch.reset();
    }
  }
}

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
  std::lock_guard<std::mutex> lk(ctx->server->mu);
  ctx->server->max_bytes = max_bytes;
  if (max_slots > 0) ctx->server->max_slots = max_slots;
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
