// The outer Newton iteration (Sec. II-A and II-B iteration tables; both inner
// solvers share it, Sec. III) run on the device for a batch of cases, and the
// launch sequence of the LU inner solve (Sec. III-A).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>

#include "internal.hpp"
#include "kernels.hpp"

namespace pfi {

namespace {

constexpr int NB = 64;

}  // namespace

Batch::~Batch() {
  if (ctx) {
    // the graphs' timing events may still be queued for reading
    (void)hipStreamSynchronize(stream);
    ctx->prof_flush();
    if (dmem) ctx->dfree(dmem);
    if (kmem) ctx->dfree(kmem);
  }
  if (h_reds) (void)hipHostFree(h_reds);
  for (auto& g : graphs) g.reset();
}

void Batch::Graph::reset() {
  if (exec) (void)hipGraphExecDestroy(exec);
  exec = nullptr;
  for (auto& p : prof) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  prof.clear();
}

bool Batch::build(Ctx* cx, const std::vector<Case*>& cs) {
  std::vector<int2> work;
  plan(cx, cs, &work);
  // device buffer: instance table | work items
  dmem = (char*)ctx->dalloc(plan_bytes(work.size()));
  if (!dmem) return false;
  {
    void* hp = nullptr;
    const size_t hr = (sizeof(pfd::Red) * std::max(nslots, 1) + 255) & ~(size_t)255;
    if (hipHostMalloc(&hp, hr + 2 * sizeof(int) * std::max(nslots, 1), hipHostMallocCoherent) != hipSuccess) return false;
    h_reds = (pfd::Red*)hp;
    h_kstate = (int*)((char*)hp + hr);
  }
  return place(dmem, work);
}

size_t Batch::plan_bytes(size_t nwork) const {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return al(sizeof(void*) * std::max(nslots, 1)) + al(sizeof(int2) * std::max<size_t>(nwork, 1));
}

bool Batch::place(char* mem, const std::vector<int2>& work) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_tab = al(sizeof(void*) * std::max(nslots, 1));
  d_insts = (const pfd::Inst* const*)mem;
  d_work = (int2*)(mem + b_tab);
  std::vector<const pfd::Inst*> tab(nslots);
  for (int s = 0; s < nslots; ++s) tab[s] = cases[s]->d_inst;
  hipStream_t st = stream;
  bool ok = hipMemcpyAsync((void*)d_insts, tab.data(), sizeof(void*) * nslots, hipMemcpyHostToDevice, st) == hipSuccess;
  if (!work.empty())
    ok &= hipMemcpyAsync(d_work, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipStreamSynchronize(st) == hipSuccess;
  return ok;
}

void Batch::plan(Ctx* cx, const std::vector<Case*>& cs, std::vector<int2>* out) {
  ctx = cx;
  stream = cx->stream;
  cases = cs;
  nslots = (int)cs.size();
  std::vector<int2>& work = *out;
  work.clear();
  seq.clear();
  auto emit = [&](int kind, int cls, int G, int k0, const std::vector<int2>& items, double flops, double bytes) {
    if (items.empty()) return;
    Launch l;
    l.kind = kind;
    l.cls = cls;
    l.G = G;
    l.k0 = k0;
    l.nflag = 0;
    l.off = (int64_t)work.size();
    l.count = (int)items.size();
    l.flops = flops;
    l.bytes = bytes;
    work.insert(work.end(), items.begin(), items.end());
    seq.push_back(l);
  };
  max_n = max_nnz = max_nu = max_heavy = 0;
  max_lu = max_tail = 0;
  int max_lev = 0, max_blev = 0, max_M = 0;
  for (Case* c : cs) {
    max_n = std::max(max_n, c->n);
    max_heavy = std::max(max_heavy, c->nheavy);
    max_nnz = std::max(max_nnz, c->nnz);
    max_nu = std::max(max_nu, c->an.nu);
    max_lu = std::max(max_lu, c->lu_count());
    if (c->an.nt > 0) max_tail = std::max(max_tail, c->tail_count());
    max_lev = std::max(max_lev, c->nlev);
    max_blev = std::max(max_blev, c->nbl);
    max_M = std::max(max_M, c->M);
  }
  // sparse refactorisation, level by level, one launch per lane-group size;
  // each column's launch also runs the forward row of its node (the rows of
  // a level depend only on earlier levels' L blocks and solution entries)
  // (factor launches whose columns all fit one wave's lane groups in one
  // pass run a column per wave: k0 = 1)
  for (int l = 0; l < max_lev; ++l) {
    std::map<int, std::vector<int2>> byG;
    std::map<int, double> fl, by;
    std::map<int, int> maxt;  // most targets of a column's first pass
    for (int s = 0; s < nslots; ++s) {
      Case* c = cs[s];
      if (l >= c->nlev) continue;
      const int G = c->fac_g[l];
      auto& v = byG[G];
      int& mt = maxt[G];
      for (int k = c->an.col_lev_ptr[l]; k < c->an.col_lev_ptr[l + 1]; ++k) {
        const int j = c->an.col_order[k];
        v.push_back(make_int2(s, j));
        // first pass: D, the U blocks and the forward row
        mt = std::max(mt, 2 + c->an.colptr[j + 1] - c->an.colptr[j]);
      }
      fl[G] += c->fac_flops[l];
      by[G] += c->fac_bytes[l];
    }
    for (auto& kv : byG) {
      // k0 = 1: a column per wave when its targets fit one pass of the
      // wave's lane groups; 2: 1024 threads per column when the level has
      // few columns and they need several passes of 256 threads
      int wave = maxt[kv.first] * kv.first <= 64 ? 1 : 0;
      if (!wave && kv.second.size() < 128 && maxt[kv.first] * kv.first > 256) wave = 2;
      emit(L_FACTOR, PF_K_SPARSE_FACTOR, kv.first, wave, kv.second, fl[kv.first], by[kv.first]);
    }
  }
  // forward rows of the dense block, then the Schur complement into it
  {
    std::map<int, std::vector<int2>> byG, schur;
    std::map<int, double> sfl, sby;
    for (int s = 0; s < nslots; ++s) {
      Case* c = cs[s];
      if (c->an.nt == 0) continue;
      auto& v = byG[c->tailfwd_g];
      for (int i = c->an.ns; i < c->an.nu; ++i) v.push_back(make_int2(s, i));
      // lanes per Schur target from the case's own mean update-list length
      // (they set the summation order, so they must not depend on the batch)
      const double nupd = (double)(c->an.tail_uptr.empty() ? 0 : c->an.tail_uptr.back());
      int gs = 1;
      while (gs < 32 && 4.0 * gs * c->ntt < nupd) gs *= 2;
      const int per_wg = 256 / gs;
      for (int t = 0; t < c->ntt; t += per_wg) schur[gs].push_back(make_int2(s, t));
      sfl[gs] += 16.0 * nupd;
      sby[gs] += 8.0 * nupd + 64.0 * nupd + 64.0 * c->ntt;
    }
    for (auto& kv : byG) emit(L_FWD, PF_K_SPARSE_FWD, kv.first, 0, kv.second, 0, 0);
    for (auto& kv : schur) emit(L_SCHUR, PF_K_TAIL_SCHUR, kv.first, 0, kv.second, sfl[kv.first], sby[kv.first]);
  }
  // dense block, per 64-wide step k0: one launch with the panel of step k0
  // (which also applies step k0's update to the next block column) and the
  // previous step's update of every other tile right of and below it
  {
    std::vector<int> Ms(nslots);
    for (int s = 0; s < nslots; ++s) Ms[s] = cs[s]->M;
    std::vector<int2> items;
    for (int k0 = 0; k0 < max_M; k0 += NB) {
      int nflag = 0, npanel = 0;
      dense_plan_step(Ms, k0, &items, &nflag, &npanel);
      double fl = 0, by = 0;
      int kb, nrt, nct;
      for (int s = 0; s < nslots; ++s) {
        if (Ms[s] <= k0) continue;
        dense_grid(Ms[s], k0, &kb, &nrt, &nct);
        const double rr = Ms[s] - (k0 + kb);
        const double nc = std::min(NB, Ms[s] + 1 - (k0 + kb));
        // inverse of the diagonal block (Gauss-Jordan, 2 kb^3), the row
        // tiles times it and the next block column's update; reads the
        // block once, reads and writes the row tiles and the next block
        // column, reads its block row tile once per row tile, writes the
        // inverse
        fl += 2.0 * kb * kb * kb + 2.0 * kb * kb * rr + 2.0 * rr * kb * nc;
        by += 8.0 * (2.0 * kb * kb + 2.0 * kb * rr + 2.0 * rr * nc + nrt * kb * nc);
      }
      // per update of a tile: 2 NB^3 flops, read L_ik and A_kj, read and
      // write A_ij (once per item)
      const double nupd = (double)(items.size() - npanel);
      fl += nupd * 2.0 * NB * NB * NB;
      by += nupd * 8.0 * 4.0 * NB * NB;
      emit(L_PANEL, PF_K_DENSE_PANEL, npanel, k0, items, fl, by);
      if (!items.empty()) seq.back().nflag = nflag;
    }
  }
  // backward solve, one launch: the dense blocks (one work-group per block,
  // each waiting on the solution entries of the blocks after it; or one
  // work-group per instance running its blocks in order, when the batch has
  // more blocks than half the work-groups the device holds at once), then the
  // sparse rows by backward level
  {
    int total = 0;
    for (Case* c : cs) total += c->M > 0 ? c->nblk() : 0;
    int mode = cs.empty() ? 0 : cs[0]->sched.trsv_mode;
    for (Case* c : cs)
      if (c->sched.trsv_mode != mode) mode = 0;
    trsv_single = mode == 1 ? 0 : mode == 2 ? 1 : (total > 1024 ? 1 : 0);
    std::vector<BwdInput> in(nslots);
    double tfl = 0, tby = 0;
    for (int s = 0; s < nslots; ++s) {
      Case* c = cs[s];
      in[s].M = c->M;
      in[s].lev_ptr = &c->an.bwd_lev_ptr;
      in[s].rows = &c->an.bwd_rows;
      in[s].g = &c->bwd_g;
      tfl += (double)c->M * c->M;
      tby += 8.0 * ((double)c->M * c->M / 2 + 2.0 * c->M);
    }
    std::vector<int2> items;
    int nd = 0, nrw = 0;
    bwd_plan(in, trsv_single != 0, &items, &nd, &nrw);
    emit(L_BWD, PF_K_DENSE_TRSV, nd, nrw, items, tfl, tby);
  }

  // zeroing chunks of every instance's factor storage
  {
    const int64_t z = pfd::zero_chunk_values();
    zero_off = (int64_t)work.size();
    for (int s = 0; s < nslots; ++s) {
      Case* c = cs[s];
      for (int64_t k = 0; k * z < c->lu_count(); ++k) work.push_back(make_int2(s, (int)k));
      if (c->an.nt > 0)
        for (int64_t k = 0; k * z < c->tail_count(); ++k) work.push_back(make_int2(s, (int)(-1 - k)));
    }
    nzero = (int)((int64_t)work.size() - zero_off);
  }
}

namespace {

template <typename T>
void lu_solve(Batch* b) {
  Ctx* ctx = b->ctx;
  hipStream_t s = b->stream;
  const auto* I = b->d_insts;
  {
    Prof p(ctx, PF_K_JFILL, 0.0, 0.0);
    pfd::launch_fill<T>(s, I, b->nslots, 2 * b->max_nu, b->d_work + b->zero_off, b->nzero, b->max_nnz);
  }
  auto launch = [&](const Launch& l) {
    const int2* w = b->d_work + l.off;
    switch (l.kind) {
      case L_FACTOR:
        if (l.k0 == 1)
          pfd::launch_factor_cols_wave<T>(s, I, w, l.count, l.G);
        else
          pfd::launch_factor_cols<T>(s, I, w, l.count, l.G, l.k0 == 2);
        break;
      case L_FWD:
        pfd::launch_fwd_rows<T>(s, I, w, l.count, l.G);
        break;
      case L_SCHUR:
        pfd::launch_tail_schur<T>(s, I, w, l.count, l.G);
        break;
      case L_PANEL:
        pfd::launch_dense_step<T>(s, I, w, l.count, l.nflag, l.G, l.k0);
        break;
      case L_BWD:
        // G: dense items, k0: sparse row work-groups
        pfd::launch_bwd_solve<T>(s, I, w, l.G, l.k0, b->trsv_single);
        break;
    }
  };
  const bool spans = (ctx->mask() & PF_PROFILE_SPANS) != 0;
  for (size_t i = 0; i < b->seq.size();) {
    const int cls = b->seq[i].cls;
    size_t j = i + 1;
    if (spans && (ctx->mask() & (1 << cls)))
      while (j < b->seq.size() && b->seq[j].cls == cls) ++j;
    // one event pair around launches i..j-1 (one launch unless spans are on)
    hipEvent_t ev;
    ctx->prof_begin(cls, &ev);
    double fl = 0, by = 0;
    for (size_t q = i; q < j; ++q) {
      launch(b->seq[q]);
      fl += b->seq[q].flops;
      by += b->seq[q].bytes * sizeof(T) / 8.0;
    }
    ctx->prof_end(cls, ev, fl, by, (int)(j - i));
    i = j;
  }
  {
    Prof p(ctx, PF_K_UPDATE, 0.0, 0.0);
    pfd::launch_update<T>(s, I, b->nslots, b->max_nu);
  }
}

}  // namespace

pf_status check_opts(const pf_options* opt) {
  if (opt->solver != PF_SOLVER_LU && opt->solver != PF_SOLVER_GMRES && opt->solver != PF_SOLVER_BICGSTAB) {
    set_error("pf_solve: unknown solver");
    return PF_E_INVALID;
  }
  if (opt->precision != PF_PREC_FP64 && opt->precision != PF_PREC_MIXED) {
    set_error("pf_solve: unknown precision");
    return PF_E_INVALID;
  }
  if (!(opt->tol > 0) || opt->max_iter < 0) {
    set_error("pf_solve: tol must be > 0 and max_iter >= 0");
    return PF_E_INVALID;
  }
  if (opt->solver != PF_SOLVER_LU) {
    if (opt->gmres_m < 1 || opt->gmres_m > pfd::krylov_max_restart() || opt->gmres_max_restarts < 0 ||
        !(opt->eta_max > 0 && opt->eta_max < 1) ||
        (opt->precond != PF_PRECOND_ILU0 && opt->precond != PF_PRECOND_BJACOBI) ||
        (opt->nk_fallback != 0 && opt->nk_fallback != 1)) {
      set_error("pf_solve: Newton-Krylov needs 1 <= gmres_m <= 128, gmres_max_restarts >= 0, 0 < eta_max < 1, a "
                "known preconditioner and nk_fallback 0 or 1");
      return PF_E_INVALID;
    }
  }
  return PF_OK;
}

static pfd::DevOpts dev_opts(const pf_options* opt) {
  pfd::DevOpts d;
  d.tol = opt->tol;
  d.max_iter = opt->max_iter;
  d.pad = 0;
  return d;
}

// Start of the iteration: initial voltages, state reset, first mismatch and
// its convergence test.
pf_status start_batch(Batch* b, const pf_options* opt) {
  pf_status st = check_opts(opt);
  if (st != PF_OK) return st;
  for (Case* c : b->cases)
    if (!ensure_work(c)) return PF_E_NOMEM;
  if (opt->solver != PF_SOLVER_LU) {
    for (Case* c : b->cases)
      if (!ensure_krylov(c, opt->gmres_m)) return PF_E_NOMEM;
    if (!b->kbuilt && !b->build_krylov()) {
      set_error("pf_solve: Krylov batch set-up failed");
      return PF_E_NOMEM;
    }
  }
  hipStream_t s = b->stream;
  pfd::launch_init(s, b->d_insts, b->nslots, b->max_n, opt->flat_start ? 1 : 0);
  pfd::launch_start(s, b->d_insts, b->nslots);
  {
    Prof p(b->ctx, PF_K_MISMATCH, 0.0, 0.0);
    pfd::launch_mismatch(s, b->d_insts, b->nslots, b->max_n, b->max_heavy);
  }
  pfd::launch_decide(s, b->d_insts, b->nslots, dev_opts(opt));
  return launch_status("pf_solve");
}

// One Newton step of every active instance: linear solve, update, mismatch
// and the convergence test.
static void enqueue_lu_step(Batch* b, const pf_options* opt) {
  hipStream_t s = b->stream;
  if (opt->precision == PF_PREC_MIXED)
    lu_solve<float>(b);
  else
    lu_solve<double>(b);
  {
    Prof p(b->ctx, PF_K_MISMATCH, 0.0, 0.0);
    pfd::launch_mismatch(s, b->d_insts, b->nslots, b->max_n, b->max_heavy);
  }
  pfd::launch_decide(s, b->d_insts, b->nslots, dev_opts(opt));
}

// The LU Newton step of a reused batch as a HIP graph: captured on first use
// (kernels, and the timing events of the classes being timed), then
// replayed; each replay queues the graph's event pairs for reading.
static bool graph_step(Batch* b, const pf_options* opt) {
  Ctx* ctx = b->ctx;
  hipStream_t s = b->stream;
  if (!b->allow_graph || b->graph_failed || !ctx->use_graphs || s == nullptr) return false;
  Batch::Graph& g = b->graphs[opt->precision == PF_PREC_MIXED ? 1 : 0];
  if (g.exec && (g.tol != opt->tol || g.max_iter != opt->max_iter || g.prof_mask != ctx->mask())) {
    if (!ctx->pending.empty()) {
      (void)hipStreamSynchronize(s);
      ctx->prof_flush();
    }
    g.reset();
  }
  if (!g.exec) {
    // timing events for the graph, made before the capture (two per timed
    // launch at most)
    ctx->cap_pool.clear();
    if (ctx->mask() != 0)
      for (size_t i = 0; i < 2 * (b->seq.size() + 8); ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) break;
        ctx->cap_pool.push_back(e);
      }
    auto drop_pool = [&]() {
      for (auto e : ctx->cap_pool) (void)hipEventDestroy(e);
      ctx->cap_pool.clear();
    };
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      drop_pool();
      b->graph_failed = true;
      return false;
    }
    ctx->capture = &g.prof;
    ctx->capture_bad = false;
    enqueue_lu_step(b, opt);
    ctx->capture = nullptr;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess || !graph || ctx->capture_bad ||
        hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      g.exec = nullptr;
      b->graph_failed = true;
    }
    drop_pool();
    if (graph) (void)hipGraphDestroy(graph);
    if (b->graph_failed) {
      g.reset();
      (void)hipGetLastError();
      return false;
    }
    g.tol = opt->tol;
    g.max_iter = opt->max_iter;
    g.prof_mask = ctx->mask();
  }
  if (hipGraphLaunch(g.exec, s) != hipSuccess) return false;
  for (const auto& p : g.prof) ctx->pending.push_back(p);
  return true;
}

pf_status step_batch(Batch* b, const pf_options* opt) {
  if (opt->solver != PF_SOLVER_LU) {
    pf_status st = nk_step(b, opt);
    if (st != PF_OK) return st;
    {
      Prof p(b->ctx, PF_K_MISMATCH, 0.0, 0.0);
      pfd::launch_mismatch(b->stream, b->d_insts, b->nslots, b->max_n, b->max_heavy);
    }
    pfd::launch_decide(b->stream, b->d_insts, b->nslots, dev_opts(opt));
  } else if (!graph_step(b, opt)) {
    enqueue_lu_step(b, opt);
  }
  return launch_status("pf_solve");
}

// Copy every instance's state to the host (synchronises the stream).
pf_status read_batch(Batch* b, std::vector<pfd::Red>* h) {
  hipStream_t s = b->stream;
  h->resize(b->nslots);
  // the gather writes straight into pinned host memory
  pfd::launch_gather_red(s, b->d_insts, b->nslots, b->h_reds);
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_error("pf_solve: device failure during the Newton iteration");
    return PF_E_DEVICE;
  }
  std::memcpy(h->data(), b->h_reds, sizeof(pfd::Red) * b->nslots);
  b->ctx->prof_flush();
  for (const auto& r : *h)
    if (r.timeout) {
      set_error("pf_solve: an inter-work-group wait on the device timed out");
      return PF_E_DEVICE;
    }
  return PF_OK;
}

pf_status run_batch(Batch* b, const pf_options* opt, pf_result* results) {
  Ctx* ctx = b->ctx;
  hipStream_t s = b->stream;
  const int B = b->nslots;
  for (int i = 0; i < B; ++i) std::memset(&results[i], 0, sizeof(pf_result));
  if (B == 0) return PF_OK;
  b->nk_step_index = 0;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("pf_solve: hipSetDevice failed");
    return PF_E_DEVICE;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("pf_solve: event creation failed");
    return PF_E_DEVICE;
  }
  (void)hipEventRecord(e0, s);
  pf_status st = start_batch(b, opt);
  // LU Newton steps queued ahead of the first read-back of the instances'
  // state: as many as the batch's last LU solve took.  The device masks the
  // instances that finish earlier, so a step past convergence changes no
  // result; the loop below then reads and continues as long as any instance
  // is active.
  int queued = 0;
  if (opt->solver == PF_SOLVER_LU)
    for (; st == PF_OK && queued < std::min(b->lu_steps, opt->max_iter); ++queued) st = step_batch(b, opt);
  std::vector<pfd::Red> h;
  for (int guard = queued; st == PF_OK && guard <= opt->max_iter + 1; ++guard) {
    st = read_batch(b, &h);
    if (st != PF_OK) break;
    bool any = false;
    for (const auto& r : h) any |= r.active != 0;
    if (!any) break;
    st = step_batch(b, opt);
  }
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->prof_flush();
  if (st != PF_OK) return st;
  if (opt->solver == PF_SOLVER_LU) {
    int most = 0;
    for (const auto& r : h) most = std::max(most, r.it);
    b->lu_steps = most;
  }
  for (int i = 0; i < B; ++i) {
    results[i].status = h[i].status;
    results[i].iters = h[i].it;
    results[i].linear_iters = h[i].linear_iters;
    results[i].mismatch_inf = h[i].last_norm;
    results[i].max_step = h[i].last_step;
    results[i].device_ms = ms;
  }
  // Newton-Krylov with fallback: the cases whose Krylov step failed go on
  // with LU from the voltage they have reached (a batch of their own)
  if (opt->solver != PF_SOLVER_LU && opt->nk_fallback) {
    std::vector<Case*> failed;
    std::vector<int> where;
    for (int i = 0; i < B; ++i)
      if (results[i].status == PF_LINEAR_FAIL) {
        failed.push_back(b->cases[i]);
        where.push_back(i);
      }
    if (!failed.empty()) {
      Batch fb;
      if (!fb.build(ctx, failed)) {
        set_error("pf_solve: batch set-up for the LU fallback failed");
        return PF_E_NOMEM;
      }
      pf_options lo = *opt;
      lo.solver = PF_SOLVER_LU;
      lo.flat_start = 0;
      lo.nk_fallback = 0;
      std::vector<pf_result> fr(failed.size());
      st = run_batch(&fb, &lo, fr.data());
      if (st != PF_OK) return st;
      for (size_t k = 0; k < failed.size(); ++k) {
        pf_result& r = results[where[k]];
        const int its = r.iters, lin = r.linear_iters;
        const double dm = r.device_ms;
        r = fr[k];
        r.iters += its;
        r.linear_iters = lin;
        r.device_ms += dm;
        r.lu_fallback = 1;
      }
    }
  }
  return PF_OK;
}

pf_status solve_case(Case* c, const pf_options* opt, pf_result* res) {
  if (!c->single) {
    auto* b = new Batch();
    if (!b->build(c->ctx, {c})) {
      delete b;
      set_error("pf_solve: batch set-up failed");
      return PF_E_NOMEM;
    }
    b->allow_graph = true;
    c->single = b;
  }
  return run_batch(c->single, opt, res);
}

}  // namespace pfi
