// The outer Newton iteration (Sec. II-A and II-B iteration tables; both
// solvers share it, Sec. III) and the LU inner solve (Sec. III-A).

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.hpp"
#include "kernels.hpp"

namespace pfi {

namespace {

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

struct Prof {
  Ctx* ctx;
  int cls;
  hipEvent_t a;
  double flops, bytes;
  Prof(Ctx* c, int k, double f, double b) : ctx(c), cls(k), a(nullptr), flops(f), bytes(b) {
    ctx->prof_begin(cls, &a);
  }
  ~Prof() { ctx->prof_end(cls, a, flops, bytes); }
};

template <typename T>
void lu_solve(Case* c) {
  Ctx* ctx = c->ctx;
  hipStream_t s = ctx->stream;
  const auto& an = c->an;
  const int ns = an.ns, nt = an.nt, nu = an.nu, M = c->M, ldt = an.ldt;
  T* x = (T*)c->x;
  T* lu = (T*)c->lu;
  T* dinv = (T*)c->dinv;
  T* tail = (T*)c->tail;
  const double tb = sizeof(T);
  pfd::Sched sc = c->sched();

  {
    Prof p(ctx, PF_K_JFILL, 0.0, tb * (c->lu_count() + c->tail_count()) + 28.0 * c->nnz + 16.0 * nu);
    pfd::launch_copy_rhs<T>(s, 2 * nu, c->F, x);
    pfd::launch_zero<T>(s, lu, c->lu_count());
    if (nt > 0) pfd::launch_zero<T>(s, tail, c->tail_count());
    if (c->model == PF_MODEL_POLAR_1PH)
      pfd::launch_jfill_polar<T>(s, c->nnz, c->yrow, c->col, c->y, c->v, c->ibus, c->vm, c->dtype, c->jmap,
                                 lu, tail, ldt, nt);
    else
      pfd::launch_jfill_cim<T>(s, c->nnz, c->yrow, c->col, c->y, c->v, c->psp, c->qsp, c->zip, c->jmap, lu,
                               tail, ldt, nt);
  }
  // sparse refactorisation by elimination-tree level
  for (int l = 0; l < c->nlev; ++l) {
    int b = an.col_lev_ptr[l], e = an.col_lev_ptr[l + 1];
    double upd = 0, blocks = 0;
    for (int k = b; k < e; ++k) {
      int j = an.col_order[k];
      int64_t t0 = j + 2LL * an.colptr[j];
      int len = an.colptr[j + 1] - an.colptr[j];
      upd += (double)(an.uptr[t0 + 1 + 2 * len] - an.uptr[t0]);
      blocks += 1 + 2 * len;
    }
    Prof p(ctx, PF_K_SPARSE_FACTOR, 16.0 * upd + 40.0 * blocks, tb * 4 * (2 * upd + 2 * blocks) + 8.0 * upd);
    pfd::launch_factor_cols<T>(s, c->col_order + b, e - b, sc, lu, dinv, c->red);
  }
  // forward solve over sparse rows (same levels as the factorisation)
  for (int l = 0; l < c->nlev; ++l) {
    int b = an.col_lev_ptr[l], e = an.col_lev_ptr[l + 1];
    Prof p(ctx, PF_K_SPARSE_FWD, 0.0, 0.0);
    pfd::launch_fwd_rows<T>(s, c->col_order + b, e - b, 0, c->lrow_ptr, c->lrow_blk, c->lrow_col, lu, x,
                            nullptr, ns);
  }
  if (nt > 0) {
    T* rhs = tail + (int64_t)M * ldt;
    {
      Prof p(ctx, PF_K_SPARSE_FWD, 0.0, 0.0);
      pfd::launch_fwd_rows<T>(s, nullptr, nt, ns, c->lrow_ptr, c->lrow_blk, c->lrow_col, lu, x, rhs, ns);
    }
    {
      double nupd = (double)(an.tail_uptr.empty() ? 0 : an.tail_uptr.back());
      Prof p(ctx, PF_K_TAIL_SCHUR, 16.0 * nupd, tb * (8.0 * nupd + 8.0 * c->ntt) + 8.0 * nupd);
      pfd::launch_tail_schur<T>(s, c->ntt, c->tail_tgt, c->tail_uptr, c->tail_l, c->tail_u, lu, tail, ldt, nt);
    }
    for (int k0 = 0; k0 < M; k0 += 64) {
      const double kb = std::min(64, M - k0);
      const double rr = M - (k0 + kb), rc = M + 1 - (k0 + kb);
      {
        Prof p(ctx, PF_K_DENSE_PANEL, (2.0 / 3.0) * kb * kb * kb + kb * kb * (rr + rc),
               tb * (2 * kb * kb + 2 * kb * (rr + rc)));
        pfd::launch_dense_lu_step<T>(s, tail, ldt, M, k0, c->red, 0);
        pfd::launch_dense_lu_step<T>(s, tail, ldt, M, k0, c->red, 1);
      }
      if (rr > 0) {
        Prof p(ctx, PF_K_DENSE_UPDATE, 2.0 * rr * rc * kb, tb * (rr * kb + kb * rc + 2.0 * rr * rc));
        pfd::launch_dense_lu_step<T>(s, tail, ldt, M, k0, c->red, 2);
      }
    }
    {
      Prof p(ctx, PF_K_DENSE_TRSV, (double)M * M, tb * ((double)M * M / 2 + 2.0 * M));
      pfd::launch_dense_trsv_upper<T>(s, tail, ldt, M, x + 2 * ns);
    }
  }
  for (int l = 0; l < c->nbl; ++l) {
    int b = an.bwd_lev_ptr[l], e = an.bwd_lev_ptr[l + 1];
    Prof p(ctx, PF_K_SPARSE_BWD, 0.0, 0.0);
    pfd::launch_bwd_rows<T>(s, c->bwd_rows + b, e - b, sc, lu, dinv, x);
  }
}

template <typename T>
void update(Case* c) {
  Ctx* ctx = c->ctx;
  hipStream_t s = ctx->stream;
  Prof p(ctx, PF_K_UPDATE, 0.0, 2.0 * sizeof(T) * c->an.nu + 48.0 * c->an.nu);
  if (c->model == PF_MODEL_POLAR_1PH)
    pfd::launch_update_polar<T>(s, c->an.nu, c->node, c->dtype, (const T*)c->x, c->vm, c->va, c->v, c->red);
  else
    pfd::launch_update_cim<T>(s, c->an.nu, c->node, (const T*)c->x, c->v, c->red);
}

void mismatch(Case* c) {
  Ctx* ctx = c->ctx;
  hipStream_t s = ctx->stream;
  Prof p(ctx, PF_K_MISMATCH, 8.0 * c->nnz, 24.0 * c->nnz + 60.0 * c->n + 16.0 * c->an.nu);
  if (c->model == PF_MODEL_POLAR_1PH)
    pfd::launch_mismatch_polar(s, c->n, c->row_ptr, c->col, c->y, c->v, c->dtype, c->psp, c->qsp, c->pos,
                               c->ibus, c->F, c->red);
  else
    pfd::launch_mismatch_cim(s, c->n, c->row_ptr, c->col, c->y, c->v, c->psp, c->qsp, c->zip, c->pos, c->F,
                             c->red);
}

}  // namespace

pf_status solve_case(Case* c, const pf_options* opt, pf_result* res) {
  Ctx* ctx = c->ctx;
  hipStream_t s = ctx->stream;
  std::memset(res, 0, sizeof *res);
  if (opt->solver != PF_SOLVER_LU) {
    set_error("pf_solve: only the LU inner solver is available in this build");
    return PF_E_INVALID;
  }
  if (!(opt->tol > 0) || opt->max_iter < 0) {
    set_error("pf_solve: tol must be > 0 and max_iter >= 0");
    return PF_E_INVALID;
  }
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
  if (opt->flat_start) {
    if (c->model == PF_MODEL_POLAR_1PH)
      pfd::launch_init_polar(s, c->n, c->dtype, c->vmag, c->vang, c->vm, c->va, c->v, 1);
    else
      pfd::launch_init_cim(s, c->n, c->dtype, c->vmag, c->vang, c->v);
  }
  const bool mixed = opt->precision == PF_PREC_MIXED;
  pfd::launch_reset_red(s, c->red);
  mismatch(c);
  double norm0 = 0;
  int status = PF_MAXITER;
  int it = 0;
  pfd::Red h;
  for (;; ++it) {
    if (hipMemcpyAsync(&h, c->red, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("pf_solve: device failure during the Newton iteration");
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return PF_E_DEVICE;
    }
    double norm = bits_to_double(h.norm_bits);
    res->mismatch_inf = norm;
    if (it > 0) res->max_step = bits_to_double(h.step_bits);
    if (it > 0 && h.singular) {
      status = PF_SINGULAR;
      break;
    }
    if (!std::isfinite(norm) || (it > 0 && !std::isfinite(res->max_step))) {
      status = PF_DIVERGED;
      break;
    }
    if (it == 0) norm0 = norm;
    if (norm <= opt->tol) {
      status = PF_CONVERGED;
      break;
    }
    if (it > 0 && norm > 1e6 * norm0) {
      status = PF_DIVERGED;
      break;
    }
    if (it >= opt->max_iter) {
      status = PF_MAXITER;
      break;
    }
    pfd::launch_reset_red(s, c->red);
    if (mixed) {
      lu_solve<float>(c);
      update<float>(c);
    } else {
      lu_solve<double>(c);
      update<double>(c);
    }
    mismatch(c);
  }
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->prof_flush();
  res->status = status;
  res->iters = it;
  res->device_ms = ms;
  return PF_OK;
}

}  // namespace pfi
