// Batched solves and the serving loop.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>

#include "internal.hpp"

namespace pfi {

struct Request {
  uint64_t ticket;
  Case* c;
  pf_options opt;
};

struct Server {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> queue;
  std::map<uint64_t, pf_result> done;
  std::map<uint64_t, int> state;  // 0 queued/running, 1 done
  uint64_t next = 1;
  bool stop = false;
  size_t max_bytes = 0;
  int max_slots = 64;
  std::thread worker;
};

static void serve_loop(Ctx* ctx) {
  Server* sv = ctx->server.get();
  for (;;) {
    Request r;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop && sv->queue.empty()) return;
      r = sv->queue.front();
      sv->queue.pop_front();
    }
    pf_result res;
    {
      std::lock_guard<std::mutex> lk(ctx->launch_mu);
      if (solve_case(r.c, &r.opt, &res) != PF_OK) {
        std::memset(&res, 0, sizeof res);
        res.status = PF_DIVERGED;
      }
    }
    r.c->busy.store(0);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->done[r.ticket] = res;
    sv->state[r.ticket] = 1;
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
  for (int i = 0; i < count; ++i) {
    if (!cases[i] || cases[i]->ctx != ctx) {
      set_error("pf_solve_batch: case belongs to another context");
      return PF_E_INVALID;
    }
  }
  std::lock_guard<std::mutex> lk(ctx->launch_mu);
  for (int i = 0; i < count; ++i) {
    pf_status st = solve_case(cases[i], &o, &results[i]);
    if (st != PF_OK) return st;
  }
  return PF_OK;
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
  int expect = 0;
  if (!c->busy.compare_exchange_strong(expect, 1)) {
    set_error("pf_submit: case already queued or running");
    return PF_E_BUSY;
  }
  if (!ctx->server) ctx->server = std::make_shared<Server>();
  Server* sv = ctx->server.get();
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->worker.joinable()) sv->worker = std::thread(serve_loop, (Ctx*)ctx);
    *ticket = sv->next++;
    sv->queue.push_back({*ticket, c, o});
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
