// C ABI: contexts, case creation (validation, host analysis, upload), data
// access and profiling.  The Newton driver is in newton.cpp, the serving loop
// in serve.cpp.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace pfi {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

#define PF_HIP(call)                                                                \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call); \
      return PF_E_DEVICE;                                                           \
    }                                                                               \
  } while (0)

void* Ctx::dalloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (alloc) return alloc(bytes, user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void Ctx::dfree(void* p) {
  if (!p) return;
  if (freef)
    freef(p, user);
  else
    (void)hipFree(p);
}

void Ctx::prof_begin(int cls, hipEvent_t* a) {
  *a = nullptr;
  if (!(mask() & (1 << cls))) return;
  hipEvent_t e;
  if (capture) {
    if (cap_pool.empty()) {
      capture_bad = true;
      return;
    }
    e = cap_pool.back();
    cap_pool.pop_back();
  } else if (!evpool.empty()) {
    e = evpool.back();
    evpool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return;
  }
  // inside a stream capture the record becomes an event node of the graph
  if (capture) {
    if (hipEventRecordWithFlags(e, stream, hipEventRecordExternal) != hipSuccess) capture_bad = true;
  } else {
    (void)hipEventRecord(e, stream);
  }
  *a = e;
}

void Ctx::prof_end(int cls, hipEvent_t a, double flops, double bytes, int nl) {
  if (!a) return;
  hipEvent_t b;
  if (capture) {
    if (cap_pool.empty()) {
      capture_bad = true;
      cap_pool.push_back(a);
      return;
    }
    b = cap_pool.back();
    cap_pool.pop_back();
  } else if (!evpool.empty()) {
    b = evpool.back();
    evpool.pop_back();
  } else if (hipEventCreate(&b) != hipSuccess) {
    evpool.push_back(a);
    return;
  }
  if (capture) {
    if (hipEventRecordWithFlags(b, stream, hipEventRecordExternal) != hipSuccess) capture_bad = true;
    capture->push_back({cls, a, b, flops, bytes, false, nl});
  } else {
    (void)hipEventRecord(b, stream);
    pending.push_back({cls, a, b, flops, bytes, true, nl});
  }
}

void Ctx::prof_flush() {
  for (auto& p : pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      stats[p.cls].launches += p.nl;
      stats[p.cls].ms += ms;
      stats[p.cls].flops += p.flops;
      stats[p.cls].bytes += p.bytes;
    } else {
      (void)hipGetLastError();  // an unread pair is dropped, not a device failure
    }
    if (p.pooled) {
      evpool.push_back(p.a);
      evpool.push_back(p.b);
    }
  }
  pending.clear();
}

pf_status launch_status(const char* where) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return PF_OK;
  set_error(std::string(where) + ": device error " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return PF_E_DEVICE;
}

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

pf_status validate_desc(const pf_case_desc* d) {
  if (!d) {
    set_error("pf_create: desc is NULL");
    return PF_E_INVALID;
  }
  if (d->model != PF_MODEL_POLAR_1PH && d->model != PF_MODEL_CIM_3PH) {
    set_error("pf_create: unknown model");
    return PF_E_INVALID;
  }
  const int n = d->n, nnz = d->nnz;
  if (n < 1 || nnz < n || !d->row_ptr || !d->col_idx || !d->y || !d->bus_type || !d->v_mag || !d->v_ang) {
    set_error("pf_create: n < 1, nnz < n or a required array is NULL");
    return PF_E_INVALID;
  }
  if (d->model == PF_MODEL_POLAR_1PH && (!d->p_sp || !d->q_sp)) {
    set_error("pf_create: polar model needs p_sp and q_sp");
    return PF_E_INVALID;
  }
  if (d->model == PF_MODEL_CIM_3PH && !d->zip) {
    set_error("pf_create: CIM model needs zip");
    return PF_E_INVALID;
  }
  if (d->row_ptr[0] != 0 || d->row_ptr[n] != nnz) {
    set_error("pf_create: row_ptr must start at 0 and end at nnz");
    return PF_E_INVALID;
  }
  for (int i = 0; i < n; ++i) {
    int a = d->row_ptr[i], b = d->row_ptr[i + 1];
    if (b < a) {
      set_error("pf_create: row_ptr not non-decreasing");
      return PF_E_INVALID;
    }
    bool diag = false;
    for (int q = a; q < b; ++q) {
      int j = d->col_idx[q];
      if (j < 0 || j >= n) {
        set_error("pf_create: column index out of range");
        return PF_E_INVALID;
      }
      if (q > a && j <= d->col_idx[q - 1]) {
        set_error("pf_create: columns not strictly increasing within a row (unsorted or duplicate)");
        return PF_E_INVALID;
      }
      if (j == i) diag = true;
    }
    if (!diag) {
      set_error("pf_create: diagonal entry missing in row " + std::to_string(i));
      return PF_E_INVALID;
    }
  }
  // structural symmetry: every (i,j) has (j,i)
  for (int i = 0; i < n; ++i)
    for (int q = d->row_ptr[i]; q < d->row_ptr[i + 1]; ++q) {
      int j = d->col_idx[q];
      const int* b = d->col_idx + d->row_ptr[j];
      const int* e = d->col_idx + d->row_ptr[j + 1];
      if (!std::binary_search(b, e, i)) {
        set_error("pf_create: Ybus pattern is not structurally symmetric");
        return PF_E_INVALID;
      }
    }
  if (!finite_all(d->y, 2LL * nnz) || !finite_all(d->v_mag, n) || !finite_all(d->v_ang, n) ||
      (d->p_sp && !finite_all(d->p_sp, n)) || (d->q_sp && !finite_all(d->q_sp, n)) ||
      (d->zip && !finite_all(d->zip, 6LL * n))) {
    set_error("pf_create: non-finite input value");
    return PF_E_INVALID;
  }
  int nslack = 0;
  for (int i = 0; i < n; ++i) {
    int t = d->bus_type[i];
    if (t != PF_PQ && t != PF_PV && t != PF_SLACK) {
      set_error("pf_create: bus type outside {PQ, PV, SLACK}");
      return PF_E_INVALID;
    }
    if (t == PF_SLACK) ++nslack;
    if (t != PF_PQ && !(d->v_mag[i] > 0.0)) {
      set_error("pf_create: PV or slack magnitude not positive at node " + std::to_string(i));
      return PF_E_INVALID;
    }
  }
  if ((d->delta_to == nullptr) != (d->zip_delta == nullptr)) {
    set_error("pf_create: delta_to and zip_delta must be given together");
    return PF_E_INVALID;
  }
  if (d->delta_to) {
    if (d->model != PF_MODEL_CIM_3PH) {
      set_error("pf_create: delta loads need the current-injection model");
      return PF_E_INVALID;
    }
    if (!finite_all(d->zip_delta, 6LL * n)) {
      set_error("pf_create: non-finite input value");
      return PF_E_INVALID;
    }
    std::vector<char> into(n, 0);
    for (int k = 0; k < n; ++k) {
      const int t = d->delta_to[k];
      if (t == -1) continue;
      if (t < -1 || t >= n || t == k) {
        set_error("pf_create: delta_to out of range or equal to its node at node " + std::to_string(k));
        return PF_E_INVALID;
      }
      if (into[t]) {
        set_error("pf_create: node " + std::to_string(t) + " receives two delta loads");
        return PF_E_INVALID;
      }
      into[t] = 1;
      const int* b = d->col_idx + d->row_ptr[k];
      const int* e = d->col_idx + d->row_ptr[k + 1];
      if (!std::binary_search(b, e, t)) {
        set_error("pf_create: delta load " + std::to_string(k) + " -> " + std::to_string(t) +
                  " has no Ybus pattern entry");
        return PF_E_INVALID;
      }
    }
  }
  if (d->model == PF_MODEL_POLAR_1PH && nslack != 1) {
    set_error("pf_create: polar model needs exactly one slack bus");
    return PF_E_INVALID;
  }
  if (d->model == PF_MODEL_CIM_3PH && nslack < 1) {
    set_error("pf_create: CIM model needs source (slack) phase-nodes");
    return PF_E_INVALID;
  }
  if (nslack == n) {
    set_error("pf_create: no unknowns");
    return PF_E_INVALID;
  }
  return PF_OK;
}

}  // namespace pfi

using namespace pfi;

template <typename X>
static X* carve(char*& p, int64_t count) {
  X* r = reinterpret_cast<X*>(p);
  size_t b = (size_t)std::max<int64_t>(count, 1) * sizeof(X);
  b = (b + 255) & ~(size_t)255;
  p += b;
  return r;
}

template <typename X>
static size_t carve_size(int64_t count) {
  size_t b = (size_t)std::max<int64_t>(count, 1) * sizeof(X);
  return (b + 255) & ~(size_t)255;
}

extern "C" {

const char* pf_last_error(void) { return g_err.c_str(); }
const char* pf_version(void) { return "exagridpf-mi355x 0.1"; }

void pf_default_options(pf_options* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->max_iter = 20;
  o->solver = PF_SOLVER_LU;
  o->precision = PF_PREC_FP64;
  o->precond = PF_PRECOND_ILU0;
  o->gmres_m = 30;
  o->gmres_max_restarts = 10;
  o->flat_start = 1;
  o->nk_fallback = 0;
  o->eta_max = 0.1;
}

pf_status pf_ctx_create(int32_t device, void* hip_stream, pf_alloc_fn alloc, pf_free_fn free_, void* user,
                        pf_ctx** out) {
  if (!out) {
    set_error("pf_ctx_create: out is NULL");
    return PF_E_INVALID;
  }
  *out = nullptr;
  if ((alloc == nullptr) != (free_ == nullptr)) {
    set_error("pf_ctx_create: give both allocator callbacks or neither");
    return PF_E_INVALID;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    set_error("pf_ctx_create: no HIP device");
    return PF_E_DEVICE;
  }
  if (device < 0 || device >= count) {
    set_error("pf_ctx_create: device index out of range");
    return PF_E_INVALID;
  }
  hipDeviceProp_t prop;
  PF_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(std::string("pf_ctx_create: device is ") + prop.gcnArchName + ", this library is built for gfx950");
    return PF_E_DEVICE;
  }
  PF_HIP(hipSetDevice(device));
  auto* c = new pf_ctx();
  c->device = device;
  c->alloc = alloc;
  c->freef = free_;
  c->user = user;
  // the device address of pf_solve_noalloc's scratch array, once per device
  // (with the device current); a failure is reported by that call alone
  (void)scratch_init(device);
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      set_error("pf_ctx_create: stream creation failed");
      return PF_E_DEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return PF_OK;
}

void pf_serve_shutdown(pf_ctx* ctx);  // serve.cpp

void pf_ctx_destroy(pf_ctx* ctx) {
  if (!ctx) return;
  pf_serve_shutdown(ctx);
  (void)hipStreamSynchronize(ctx->stream);
  for (Batch* b : ctx->bcache) delete b;
  ctx->bcache.clear();
  ctx->prof_flush();
  for (auto e : ctx->evpool) (void)hipEventDestroy(e);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

pf_status pf_ctx_use_graphs(pf_ctx* ctx, int32_t on) {
  if (!ctx) {
    set_error("pf_ctx_use_graphs: NULL context");
    return PF_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(ctx->launch_mu);
  ctx->use_graphs = on != 0;
  return PF_OK;
}

}  // extern "C"

namespace pfi {

bool valid_schedule(const pf_schedule& s) {
  return s.dense_switch > 0 && s.dense_switch <= 1 && s.min_dense >= 1 &&
         (s.lane_scale == 1 || s.lane_scale == 2 || s.lane_scale == 4) && s.trsv_mode >= 0 && s.trsv_mode <= 2;
}

uint64_t topology_hash(const pf_case_desc* d) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a
  auto mix = [&](const void* p, size_t bytes) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < bytes; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  };
  mix(&d->model, sizeof d->model);
  mix(&d->n, sizeof d->n);
  mix(&d->nnz, sizeof d->nnz);
  mix(d->row_ptr, sizeof(int32_t) * ((size_t)d->n + 1));
  mix(d->col_idx, sizeof(int32_t) * (size_t)d->nnz);
  mix(d->bus_type, (size_t)d->n);
  return h;
}

pf_status create_case(Ctx* ctx, const pf_case_desc* d, const pf_schedule& sched, Case** out) {
  *out = nullptr;
  PF_HIP(hipSetDevice(ctx->device));
  auto t0 = std::chrono::steady_clock::now();
  const int n = d->n, nnz = d->nnz;
  pfh::GraphInput g;
  g.n_nodes = n;
  g.unknown.resize(n);
  g.adj.resize(n);
  for (int i = 0; i < n; ++i) {
    g.unknown[i] = d->bus_type[i] != PF_SLACK;
    for (int q = d->row_ptr[i]; q < d->row_ptr[i + 1]; ++q)
      if (d->col_idx[q] != i) g.adj[i].push_back(d->col_idx[q]);
  }
  auto* c = new pf_case();
  c->ctx = ctx;
  c->model = d->model;
  c->n = n;
  c->nnz = nnz;
  c->sched = sched;
  try {
    c->an = pfh::analyze(g, sched.dense_switch, sched.min_dense, 64);
  } catch (const std::exception& ex) {
    delete c;
    set_error(std::string("pf_create: analysis failed: ") + ex.what());
    return PF_E_INVALID;
  }
  auto& an = c->an;
  c->nlev = (int)an.col_lev_ptr.size() - 1;
  c->nbl = (int)an.bwd_lev_ptr.size() - 1;
  c->ntg = (int64_t)an.ns + 2 * an.nnzl;
  c->ntt = (int)an.tail_tgt.size();
  c->M = 2 * an.nt;
  c->type.assign(d->bus_type, d->bus_type + n);
  {
    auto pick = [&](int64_t m) {
      int g = 1;
      while (g < 64 && 4LL * g < m) g *= 2;
      return std::min(64, g * sched.lane_scale);
    };
    c->fac_g.resize(c->nlev);
    c->fac_flops.resize(c->nlev);
    c->fac_bytes.resize(c->nlev);
    for (int l = 0; l < c->nlev; ++l) {
      int64_t mf = 0, mr = 0;
      double upd = 0, blocks = 0;
      for (int k = an.col_lev_ptr[l]; k < an.col_lev_ptr[l + 1]; ++k) {
        int j = an.col_order[k];
        int len = an.colptr[j + 1] - an.colptr[j];
        int64_t t0 = j + 2LL * an.colptr[j];
        for (int t = 0; t <= 2 * len; ++t) mf = std::max(mf, an.uptr[t0 + t + 1] - an.uptr[t0 + t]);
        mr = std::max<int64_t>(mr, an.lrow_ptr[j + 1] - an.lrow_ptr[j]);
        upd += (double)(an.uptr[t0 + 1 + 2 * len] - an.uptr[t0]);
        blocks += 1 + 2 * len;
      }
      // one lane count for the level's update lists and its forward rows
      // (run by the same launch)
      c->fac_g[l] = pick(std::max(mf, mr));
      c->fac_flops[l] = 16.0 * upd + 40.0 * blocks;
      c->fac_bytes[l] = 8.0 * upd + 2 * 32.0 * blocks;  // index pairs + read/write of target blocks (FP64)
    }
    int64_t mt = 0;
    for (int i = an.ns; i < an.nu; ++i) mt = std::max<int64_t>(mt, an.lrow_ptr[i + 1] - an.lrow_ptr[i]);
    c->tailfwd_g = pick(mt);
    c->bwd_g.resize(c->nbl);
    for (int l = 0; l < c->nbl; ++l) {
      int64_t m = 0;
      for (int k = an.bwd_lev_ptr[l]; k < an.bwd_lev_ptr[l + 1]; ++k) {
        int i = an.bwd_rows[k];
        m = std::max<int64_t>(m, an.colptr[i + 1] - an.colptr[i]);
      }
      c->bwd_g[l] = pick(m);
    }
  }

  // Ybus entry -> LU destination
  std::vector<int> yrow, jmap;
  try {
    pfh::build_jmap(c->an, n, d->row_ptr, d->col_idx, &yrow, &jmap);
  } catch (const std::exception& ex) {
    delete c;
    set_error(std::string("pf_create: ") + ex.what());
    return PF_E_INVALID;
  }
  try {
    c->ka.reset(new pfh::KAnalysis(pfh::analyze_krylov(an, n, d->row_ptr, d->col_idx, 32)));
    pfh::build_kmap(an, *c->ka, n, d->row_ptr, d->col_idx, &c->kmap_host);
  } catch (const std::exception& ex) {
    delete c;
    set_error(std::string("pf_create: Krylov analysis failed: ") + ex.what());
    return PF_E_INVALID;
  }
  const int ns = an.ns;
  // rows the mismatch gives a work-group of their own
  std::vector<int> heavy;
  for (int i = 0; i < n; ++i)
    if (d->row_ptr[i + 1] - d->row_ptr[i] > pfd::kHeavyRow) heavy.push_back(i);
  c->nheavy = (int)heavy.size();
  // device layout
  const int nu = an.nu;
  const int64_t nupd = (int64_t)an.upd_l.size(), ntail = (int64_t)an.tail_l.size();
  size_t total = 0;
  total += carve_size<int>(n + 1) + 3 * carve_size<int>(nnz) + carve_size<double>(2LL * nnz);
  total += carve_size<int8_t>(n) + 4 * carve_size<double>(n) + carve_size<double>(6LL * n);
  total += carve_size<int>(n) + carve_size<int>(nu);
  total += 2 * carve_size<double>(n) + 2 * carve_size<double>(2LL * n) + carve_size<double>(2LL * nu);
  total += carve_size<double>(2LL * nu);
  total += carve_size<int>(ns + 1) + carve_size<int>(an.nnzl) + carve_size<int64_t>(c->ntg + 1) +
           2 * carve_size<int>(nupd) + carve_size<int>(ns);
  total += carve_size<int>(c->ntt) + carve_size<int64_t>(c->ntt + 1) + 2 * carve_size<int>(ntail);
  total += carve_size<int>(nu + 1) + 2 * carve_size<int>(an.nnzl) + carve_size<int>(ns);
  total += carve_size<double>(n) + carve_size<int>(2LL * n) + carve_size<double>(6LL * n);
  const int nmpart = (n + 63) / 64, nupart = (nu + 255) / 256;
  total += carve_size<pfd::Red>(1) + carve_size<pfd::Inst>(1) + carve_size<int>(c->nheavy);
  total += carve_size<double>(nmpart) + carve_size<double>(nupart);
  c->bytes = total;
  c->wbytes = work_bytes(c);
  c->base = (char*)ctx->dalloc(total);
  if (!c->base) {
    delete c;
    set_error("pf_create: device allocation failed");
    return PF_E_NOMEM;
  }
  char* p = c->base;
  c->row_ptr = carve<int>(p, n + 1);
  c->col = carve<int>(p, nnz);
  c->yrow = carve<int>(p, nnz);
  c->jmap = carve<int>(p, nnz);
  c->y = carve<double>(p, 2LL * nnz);
  c->dtype = carve<int8_t>(p, n);
  c->psp = carve<double>(p, n);
  c->qsp = carve<double>(p, n);
  c->vmag = carve<double>(p, n);
  c->vang = carve<double>(p, n);
  c->zip = carve<double>(p, 6LL * n);
  c->qg = carve<double>(p, n);
  c->dlink = carve<int>(p, 2LL * n);
  c->zipd = carve<double>(p, 6LL * n);
  c->pos = carve<int>(p, n);
  c->node = carve<int>(p, nu);
  c->vm = carve<double>(p, n);
  c->va = carve<double>(p, n);
  c->v = carve<double>(p, 2LL * n);
  c->ibus = carve<double>(p, 2LL * n);
  c->F = carve<double>(p, 2LL * nu);
  c->x = carve<double>(p, 2LL * nu);
  c->colptr = carve<int>(p, ns + 1);
  c->rowidx = carve<int>(p, an.nnzl);
  c->uptr = carve<int64_t>(p, c->ntg + 1);
  c->upd_l = carve<int>(p, nupd);
  c->upd_u = carve<int>(p, nupd);
  c->col_order = carve<int>(p, ns);
  c->tail_tgt = carve<int>(p, c->ntt);
  c->tail_uptr = carve<int64_t>(p, c->ntt + 1);
  c->tail_l = carve<int>(p, ntail);
  c->tail_u = carve<int>(p, ntail);
  c->lrow_ptr = carve<int>(p, nu + 1);
  c->lrow_blk = carve<int>(p, an.nnzl);
  c->lrow_col = carve<int>(p, an.nnzl);
  c->bwd_rows = carve<int>(p, ns);
  c->red = carve<pfd::Red>(p, 1);
  c->d_inst = carve<pfd::Inst>(p, 1);
  int* d_heavy = carve<int>(p, c->nheavy);
  double* d_mpart = carve<double>(p, nmpart);
  double* d_upart = carve<double>(p, nupart);
  if ((size_t)(p - c->base) != total) {
    ctx->dfree(c->base);
    delete c;
    set_error("pf_create: internal layout error");
    return PF_E_DEVICE;
  }

  std::vector<double> zeros(n, 0.0);
  hipStream_t s = ctx->stream;
  auto up = [&](void* dst, const void* src, size_t b) -> bool {
    if (b == 0) return true;
    return hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  bool ok = true;
  ok &= up(c->row_ptr, d->row_ptr, sizeof(int) * (n + 1));
  ok &= up(c->col, d->col_idx, sizeof(int) * nnz);
  ok &= up(c->yrow, yrow.data(), sizeof(int) * nnz);
  ok &= up(c->jmap, jmap.data(), sizeof(int) * nnz);
  ok &= up(c->y, d->y, sizeof(double) * 2 * nnz);
  ok &= up(c->dtype, d->bus_type, n);
  ok &= up(c->psp, d->p_sp ? d->p_sp : zeros.data(), sizeof(double) * n);
  ok &= up(c->qsp, d->q_sp ? d->q_sp : zeros.data(), sizeof(double) * n);
  ok &= up(c->vmag, d->v_mag, sizeof(double) * n);
  ok &= up(c->vang, d->v_ang, sizeof(double) * n);
  if (d->zip) ok &= up(c->zip, d->zip, sizeof(double) * 6 * n);
  ok &= up(c->qg, d->q_sp ? d->q_sp : zeros.data(), sizeof(double) * n);
  c->has_delta = false;
  if (d->delta_to) {
    // per node: the node its delta load draws into, and the node whose
    // delta load it receives (-1: none)
    std::vector<int> link(2 * (size_t)n, -1);
    for (int k = 0; k < n; ++k) {
      const int t = d->delta_to[k];
      if (t < 0) continue;
      link[2 * k] = t;
      link[2 * t + 1] = k;
      c->has_delta = true;
    }
    ok &= up(c->dlink, link.data(), sizeof(int) * 2 * n);
    ok &= up(c->zipd, d->zip_delta, sizeof(double) * 6 * n);
  }
  ok &= up(c->pos, an.pos_of_node.data(), sizeof(int) * n);
  ok &= up(c->node, an.node_of_pos.data(), sizeof(int) * nu);
  ok &= up(c->colptr, an.colptr.data(), sizeof(int) * (ns + 1));
  ok &= up(c->rowidx, an.rowidx.data(), sizeof(int) * an.nnzl);
  ok &= up(c->uptr, an.uptr.data(), sizeof(int64_t) * (c->ntg + 1));
  ok &= up(c->upd_l, an.upd_l.data(), sizeof(int) * nupd);
  ok &= up(c->upd_u, an.upd_u.data(), sizeof(int) * nupd);
  ok &= up(c->col_order, an.col_order.data(), sizeof(int) * ns);
  ok &= up(c->tail_tgt, an.tail_tgt.data(), sizeof(int) * c->ntt);
  ok &= up(c->tail_uptr, an.tail_uptr.data(), sizeof(int64_t) * (c->ntt + 1));
  ok &= up(c->tail_l, an.tail_l.data(), sizeof(int) * ntail);
  ok &= up(c->tail_u, an.tail_u.data(), sizeof(int) * ntail);
  ok &= up(c->lrow_ptr, an.lrow_ptr.data(), sizeof(int) * (nu + 1));
  ok &= up(c->lrow_blk, an.lrow_blk.data(), sizeof(int) * an.nnzl);
  ok &= up(c->lrow_col, an.lrow_col.data(), sizeof(int) * an.nnzl);
  ok &= up(c->bwd_rows, an.bwd_rows.data(), sizeof(int) * ns);
  ok &= up(d_heavy, heavy.data(), sizeof(int) * heavy.size());
  ok &= hipMemsetAsync(c->red, 0, sizeof(pfd::Red), s) == hipSuccess;
  {
    pfd::Inst hi;
    std::memset(&hi, 0, sizeof hi);
    hi.model = c->model;
    hi.n = n;
    hi.nnz = nnz;
    hi.nu = nu;
    hi.ns = ns;
    hi.nt = an.nt;
    hi.ldt = an.ldt;
    hi.M = c->M;
    hi.ntt = c->ntt;
    hi.nblk = c->nblk();
    hi.nnzl = an.nnzl;
    hi.lu_count = c->lu_count();
    hi.tail_count = an.nt > 0 ? c->tail_count() : 0;
    hi.row_ptr = c->row_ptr;
    hi.col = c->col;
    hi.yrow = c->yrow;
    hi.jmap = c->jmap;
    hi.y = c->y;
    hi.type = c->dtype;
    hi.psp = c->psp;
    hi.qsp = c->qsp;
    hi.vmag = c->vmag;
    hi.vang = c->vang;
    hi.zip = c->zip;
    hi.qg = c->qg;
    hi.dlink = c->has_delta ? (const int2*)c->dlink : nullptr;
    hi.zipd = c->zipd;
    hi.pos = c->pos;
    hi.node = c->node;
    hi.nheavy = c->nheavy;
    hi.heavy = d_heavy;
    hi.nmpart = nmpart;
    hi.nupart = nupart;
    hi.mpart = d_mpart;
    hi.upart = d_upart;
    hi.vm = c->vm;
    hi.va = c->va;
    hi.v = c->v;
    hi.ibus = c->ibus;
    hi.F = c->F;
    hi.x = c->x;
    hi.colptr = c->colptr;
    hi.rowidx = c->rowidx;
    hi.upd_l = c->upd_l;
    hi.upd_u = c->upd_u;
    hi.uptr = c->uptr;
    hi.tail_tgt = c->tail_tgt;
    hi.tail_l = c->tail_l;
    hi.tail_u = c->tail_u;
    hi.tail_uptr = c->tail_uptr;
    hi.lrow_ptr = c->lrow_ptr;
    hi.lrow_blk = c->lrow_blk;
    hi.lrow_col = c->lrow_col;
    hi.red = c->red;
    c->hinst = hi;
    ok &= up(c->d_inst, &hi, sizeof hi);
    // flat-start voltages so that pf_get_voltage is defined before a solve
    std::vector<double> v0(2 * (size_t)n), vm0(n), va0(n);
    for (int i = 0; i < n; ++i) {
      const int t = d->bus_type[i];
      double m, a;
      if (c->model == PF_MODEL_POLAR_1PH) {
        m = t == PF_PQ ? 1.0 : d->v_mag[i];
        a = t == PF_SLACK ? d->v_ang[i] : 0.0;
      } else {
        m = t == PF_PQ ? 1.0 : d->v_mag[i];
        a = d->v_ang[i];
      }
      vm0[i] = m;
      va0[i] = a;
      v0[2 * i] = m * std::cos(a);
      v0[2 * i + 1] = m * std::sin(a);
    }
    ok &= up(c->v, v0.data(), sizeof(double) * 2 * n);
    ok &= up(c->vm, vm0.data(), sizeof(double) * n);
    ok &= up(c->va, va0.data(), sizeof(double) * n);
  }
  ok &= hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    ctx->dfree(c->base);
    delete c;
    set_error("pf_create: upload failed");
    return PF_E_DEVICE;
  }
  // the upload is done: drop the host copies the device now owns
  an.upd_l.clear();
  an.upd_l.shrink_to_fit();
  an.upd_u.clear();
  an.upd_u.shrink_to_fit();
  an.tail_l.clear();
  an.tail_l.shrink_to_fit();
  an.tail_u.clear();
  an.tail_u.shrink_to_fit();
  c->analysis_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ctx->ncases++;
  *out = c;
  return PF_OK;
}

// Working storage of a solve: factor values (D | L | U blocks), the inverted
// 2x2 diagonal blocks, the dense block with its right-hand side column, its
// 64x64 diagonal-block inverses, the block step's flags, and the backward
// solve's published copy of the solution.
size_t work_bytes(const Case* c) {
  return carve_size<double>(c->lu_count()) + carve_size<double>(4LL * c->an.ns) +
         carve_size<double>(c->tail_count()) + carve_size<double>(c->dinvu_count()) +
         carve_size<unsigned long long>(c->nblk()) + carve_size<double>(2LL * c->an.nu);
}

void attach_work(Case* c, char* base, bool own, hipStream_t s) {
  char* p = base;
  c->lu = carve<double>(p, c->lu_count());
  c->dinv = carve<double>(p, 4LL * c->an.ns);
  c->tail = carve<double>(p, c->tail_count());
  c->dinvu = carve<double>(p, c->dinvu_count());
  c->pflags = carve<unsigned long long>(p, c->nblk());
  c->xs = carve<double>(p, 2LL * c->an.nu);
  c->wbase = base;
  c->wown = own;
  pfd::Inst& h = c->hinst;
  h.lu = c->lu;
  h.dinv = c->dinv;
  h.tail = c->tail;
  h.dinvu = c->dinvu;
  h.xs = c->xs;
  h.pflags = c->pflags;
  // the flags carry Newton-step epochs, which only grow within one case:
  // storage that another case used starts from zero (below every epoch)
  pfd::launch_zero_words(s, c->pflags, 2LL * std::max(c->nblk(), 1));
  pfd::launch_set_inst(s, c->d_inst, h);
}

bool ensure_work(Case* c) {
  if (c->wbase) return true;
  char* p = (char*)c->ctx->dalloc(c->wbytes);
  if (!p) {
    set_error("pf_solve: device allocation of the working storage failed");
    return false;
  }
  attach_work(c, p, true, c->ctx->stream);
  return true;
}

void detach_work(Case* c) {
  if (c->wown && c->wbase) c->ctx->dfree(c->wbase);
  c->wbase = nullptr;
  c->wown = false;
  c->lu = c->dinv = c->tail = c->dinvu = nullptr;
  c->xs = nullptr;
  c->pflags = nullptr;
}

}  // namespace pfi

extern "C" {

void pf_default_schedule(pf_schedule* s) {
  if (!s) return;
  std::memset(s, 0, sizeof *s);
  s->dense_switch = 0.15;
  s->min_dense = 32;
  s->lane_scale = 1;
  s->trsv_mode = 0;
}

pf_status pf_create_scheduled(pf_ctx* ctx, const pf_case_desc* d, const pf_schedule* sched, pf_case** out) {
  if (!ctx || !out || !sched) {
    set_error("pf_create_scheduled: NULL argument");
    return PF_E_INVALID;
  }
  *out = nullptr;
  if (!valid_schedule(*sched)) {
    set_error("pf_create_scheduled: schedule out of range");
    return PF_E_INVALID;
  }
  pf_status st = validate_desc(d);
  if (st != PF_OK) return st;
  Case* c = nullptr;
  st = create_case(ctx, d, *sched, &c);
  *out = static_cast<pf_case*>(c);
  return st;
}

pf_status pf_create(pf_ctx* ctx, const pf_case_desc* d, pf_case** out) {
  if (!ctx || !out) {
    set_error("pf_create: NULL context or out");
    return PF_E_INVALID;
  }
  *out = nullptr;
  pf_status st = validate_desc(d);
  if (st != PF_OK) return st;
  pf_schedule sc;
  pf_default_schedule(&sc);
  {
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    if (!ctx->tuned.empty()) {
      auto it = ctx->tuned.find(topology_hash(d));
      if (it != ctx->tuned.end()) sc = it->second;
    }
  }
  Case* c = nullptr;
  st = create_case(ctx, d, sc, &c);
  *out = static_cast<pf_case*>(c);
  return st;
}

pf_status pf_case_schedule(const pf_case* c, pf_schedule* out) {
  if (!c || !out) {
    set_error("pf_case_schedule: NULL argument");
    return PF_E_INVALID;
  }
  *out = c->sched;
  return PF_OK;
}

pf_status pf_destroy(pf_case* c) {
  if (!c) return PF_OK;
  if (c->busy.load()) {
    set_error("pf_destroy: case is queued or running");
    return PF_E_BUSY;
  }
  (void)hipStreamSynchronize(c->ctx->stream);
  {
    // cached batches that hold the case go with it
    std::lock_guard<std::mutex> lk(c->ctx->launch_mu);
    auto& bc = c->ctx->bcache;
    for (size_t i = 0; i < bc.size();) {
      if (std::find(bc[i]->cases.begin(), bc[i]->cases.end(), static_cast<Case*>(c)) != bc[i]->cases.end()) {
        delete bc[i];
        bc.erase(bc.begin() + i);
      } else {
        ++i;
      }
    }
  }
  delete c->single;
  c->single = nullptr;
  free_krylov(c);
  if (c->wown) c->ctx->dfree(c->wbase);
  c->ctx->dfree(c->base);
  c->ctx->ncases--;
  delete c;
  return PF_OK;
}

pf_status pf_case_info_get(const pf_case* c, pf_case_info* o) {
  if (!c || !o) {
    set_error("pf_case_info_get: NULL argument");
    return PF_E_INVALID;
  }
  const auto& an = c->an;
  o->n = c->n;
  o->n_unknown = an.nu;
  o->n_sparse = an.ns;
  o->n_dense = an.nt;
  o->levels = c->nlev;
  o->bwd_levels = c->nbl;
  o->nnz_l_blocks = an.nnzl;
  o->updates = an.uptr.empty() ? 0 : an.uptr.back();
  o->tail_updates = an.tail_uptr.empty() ? 0 : an.tail_uptr.back();
  o->flops_factor = an.flops_sparse + an.flops_tail_schur + an.flops_dense;
  o->device_bytes = c->bytes + (c->wown ? c->wbytes : 0);
  o->resident_bytes = c->bytes - (c->kown ? c->kbytes : 0);
  o->work_bytes = c->wbytes;
  o->krylov_bytes = krylov_bytes(c, 30);
  o->analysis_ms = c->analysis_ms;
  return PF_OK;
}

pf_status pf_case_footprint(const pf_case* c, size_t* bytes) {
  if (!c || !bytes) {
    set_error("pf_case_footprint: NULL argument");
    return PF_E_INVALID;
  }
  *bytes = (c->bytes - (c->kown ? c->kbytes : 0)) + c->wbytes;
  return PF_OK;
}

pf_status pf_set_injections(pf_case* c, const double* p_sp, const double* q_sp, const double* zip) {
  if (!c) {
    set_error("pf_set_injections: NULL case");
    return PF_E_INVALID;
  }
  if (c->busy.load()) {
    set_error("pf_set_injections: case is queued or running");
    return PF_E_BUSY;
  }
  const int n = c->n;
  if ((p_sp && !finite_all(p_sp, n)) || (q_sp && !finite_all(q_sp, n)) || (zip && !finite_all(zip, 6LL * n))) {
    set_error("pf_set_injections: non-finite value");
    return PF_E_INVALID;
  }
  if (zip && c->model != PF_MODEL_CIM_3PH) {
    set_error("pf_set_injections: zip given for a polar case");
    return PF_E_INVALID;
  }
  hipStream_t s = c->ctx->stream;
  if (p_sp) PF_HIP(hipMemcpyAsync(c->psp, p_sp, sizeof(double) * n, hipMemcpyHostToDevice, s));
  if (q_sp) PF_HIP(hipMemcpyAsync(c->qsp, q_sp, sizeof(double) * n, hipMemcpyHostToDevice, s));
  if (zip) PF_HIP(hipMemcpyAsync(c->zip, zip, sizeof(double) * 6 * n, hipMemcpyHostToDevice, s));
  PF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}

pf_status pf_get_voltage(const pf_case* c, double* re, double* im) {
  if (!c || !re || !im) {
    set_error("pf_get_voltage: NULL argument");
    return PF_E_INVALID;
  }
  std::vector<double> v(2 * (size_t)c->n);
  hipStream_t s = c->ctx->stream;
  PF_HIP(hipMemcpyAsync(v.data(), c->v, sizeof(double) * 2 * c->n, hipMemcpyDeviceToHost, s));
  PF_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < c->n; ++i) {
    re[i] = v[2 * i];
    im[i] = v[2 * i + 1];
  }
  return PF_OK;
}

pf_status pf_set_voltage(pf_case* c, const double* re, const double* im) {
  if (!c || !re || !im) {
    set_error("pf_set_voltage: NULL argument");
    return PF_E_INVALID;
  }
  if (c->busy.load()) {
    set_error("pf_set_voltage: case is queued or running");
    return PF_E_BUSY;
  }
  const int n = c->n;
  std::vector<double> v(2 * (size_t)n), vm(n), va(n);
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(re[i]) || !std::isfinite(im[i])) {
      set_error("pf_set_voltage: non-finite value");
      return PF_E_INVALID;
    }
    v[2 * i] = re[i];
    v[2 * i + 1] = im[i];
    vm[i] = std::hypot(re[i], im[i]);
    va[i] = std::atan2(im[i], re[i]);
  }
  hipStream_t s = c->ctx->stream;
  PF_HIP(hipMemcpyAsync(c->v, v.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice, s));
  PF_HIP(hipMemcpyAsync(c->vm, vm.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  PF_HIP(hipMemcpyAsync(c->va, va.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  PF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}

pf_status pf_profile_enable(pf_ctx* ctx, int32_t class_mask) {
  if (!ctx) {
    set_error("pf_profile_enable: NULL context");
    return PF_E_INVALID;
  }
  // -1: every class, one event pair per launch
  ctx->profile_mask = class_mask == -1 ? (1 << PF_K_COUNT) - 1 : class_mask;
  return PF_OK;
}

pf_status pf_profile_reset(pf_ctx* ctx) {
  if (!ctx) {
    set_error("pf_profile_reset: NULL context");
    return PF_E_INVALID;
  }
  (void)hipStreamSynchronize(ctx->stream);
  ctx->prof_flush();
  for (auto& s : ctx->stats) s = pf_kernel_stat{};
  return PF_OK;
}

pf_status pf_kernel_stats(pf_ctx* ctx, int32_t cls, pf_kernel_stat* out) {
  if (!ctx || !out || cls < 0 || cls >= PF_K_COUNT) {
    set_error("pf_kernel_stats: bad argument");
    return PF_E_INVALID;
  }
  PF_HIP(hipStreamSynchronize(ctx->stream));
  ctx->prof_flush();
  *out = ctx->stats[cls];
  return PF_OK;
}

pf_status pf_solve(pf_case* c, const pf_options* opt, pf_result* res) {
  if (!c || !res) {
    set_error("pf_solve: NULL argument");
    return PF_E_INVALID;
  }
  if (c->busy.load()) {
    set_error("pf_solve: case is queued or running");
    return PF_E_BUSY;
  }
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  std::lock_guard<std::mutex> lk(c->ctx->launch_mu);
  return solve_case(c, &o, res);
}

}  // extern "C"
