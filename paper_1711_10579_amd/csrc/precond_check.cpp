// Device check of the Newton-Krylov preconditioner set-up (Sec. III-B).
//
// Builds the Jacobian of a case at its flat start on the device, runs the
// preconditioner set-up kernels exactly as a Krylov Newton step does (ILU(0)
// factor or block-Jacobi group inverses), copies the results back and checks
// them on the host against their definitions: ILU(0) reproduces A on its
// pattern, (L U)_ij = A_ij, with U's inverted diagonal blocks the inverses of
// U's diagonal; a block-Jacobi group's inverse X satisfies A_bb X = I.  A test
// of the kernels; the solve path never calls it.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/pf_debug.h"
#include "internal.hpp"
#include "kernels.hpp"

namespace pfi {
pf_status start_batch(Batch* b, const pf_options* opt);  // newton.cpp
}

using namespace pfi;

namespace {

struct B2 {
  double a = 0, b = 0, c = 0, d = 0;
};
B2 add(const B2& x, const B2& y) { return {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; }
B2 mul(const B2& x, const B2& y) {
  return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
double nrm(const B2& m) {
  return std::max(std::max(std::fabs(m.a), std::fabs(m.b)), std::max(std::fabs(m.c), std::fabs(m.d)));
}
B2 at(const std::vector<double>& v, int64_t q) { return {v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]}; }

}  // namespace

extern "C" pf_status pf_debug_precond_check(pf_case* c, int32_t precond, double* deviation, int32_t* max_order) {
  if (!c || !deviation || !max_order || (precond != PF_PRECOND_ILU0 && precond != PF_PRECOND_BJACOBI)) {
    set_error("pf_debug_precond_check: bad argument");
    return PF_E_INVALID;
  }
  if (c->busy.load()) {
    set_error("pf_debug_precond_check: case is queued or running");
    return PF_E_BUSY;
  }
  Ctx* ctx = c->ctx;
  std::lock_guard<std::mutex> lk(ctx->launch_mu);
  if (hipSetDevice(ctx->device) != hipSuccess) {
    set_error("pf_debug_precond_check: hipSetDevice failed");
    return PF_E_DEVICE;
  }
  pf_options o;
  pf_default_options(&o);
  o.solver = PF_SOLVER_BICGSTAB;
  o.precond = precond;
  o.flat_start = 1;
  Batch b;
  if (!b.build(ctx, {c})) {
    set_error("pf_debug_precond_check: batch set-up failed");
    return PF_E_NOMEM;
  }
  pf_status st = start_batch(&b, &o);
  if (st != PF_OK) return st;
  hipStream_t s = b.stream;
  const bool ilu = precond == PF_PRECOND_ILU0;
  pfd::launch_kfill<double>(s, b.d_insts, 1, b.max_nnz, ilu ? 1 : 0);
  if (ilu && b.k_narrow)
    pfd::launch_ilu_factor_wg<double>(s, b.d_insts, 1);
  else if (ilu)
    for (const auto& l : b.k_lev) pfd::launch_ilu_rows<double>(s, b.d_insts, b.d_kwork + l.first, l.second);
  else
    pfd::launch_bj_inv<double>(s, b.d_insts, b.d_kwork + b.k_blocks.first, b.k_blocks_big,
                                b.k_blocks.second - b.k_blocks_big);
  st = launch_status("pf_debug_precond_check");
  if (st != PF_OK) return st;
  const pfh::KAnalysis& ka = *c->ka;
  const int nu = ka.nu;
  const int64_t knnz = ka.nnz();
  const pfd::Inst& h = c->hinst;
  std::vector<double> A(4 * knnz), P, Dinv;
  pfd::Red red;
  bool ok = hipMemcpyAsync(A.data(), h.jval, sizeof(double) * 4 * knnz, hipMemcpyDeviceToHost, s) == hipSuccess;
  if (ilu) {
    P.resize(4 * knnz);
    Dinv.resize(4LL * nu);
    ok &= hipMemcpyAsync(P.data(), h.pval, sizeof(double) * 4 * knnz, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok &= hipMemcpyAsync(Dinv.data(), h.pdinv, sizeof(double) * 4 * nu, hipMemcpyDeviceToHost, s) == hipSuccess;
  } else {
    P.resize((size_t)ka.bj_off.back());
    ok &= hipMemcpyAsync(P.data(), h.bjinv, sizeof(double) * P.size(), hipMemcpyDeviceToHost, s) == hipSuccess;
  }
  ok &= hipMemcpyAsync(&red, c->red, sizeof red, hipMemcpyDeviceToHost, s) == hipSuccess;
  ok &= hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    set_error("pf_debug_precond_check: device failure");
    return PF_E_DEVICE;
  }
  if (red.singular) {
    set_error("pf_debug_precond_check: the set-up met a singular pivot");
    return PF_E_INVALID;
  }
  double dev = 0;
  int order = 0;
  if (ilu) {
    // (L U)(r, j) = sum over k of L(r, k) U(k, j), L unit block-lower, U
    // block-upper, both on the pattern; compare with A on the pattern
    double amax = 0;
    for (int64_t q = 0; q < knnz; ++q) amax = std::max(amax, nrm(at(A, q)));
    auto find = [&](int r, int col) -> int64_t {
      const int* b0 = ka.col.data() + ka.row_ptr[r];
      const int* e0 = ka.col.data() + ka.row_ptr[r + 1];
      const int* it = std::lower_bound(b0, e0, col);
      return (it != e0 && *it == col) ? (int64_t)(it - ka.col.data()) : -1;
    };
    for (int r = 0; r < nu; ++r) {
      for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q) {
        const int j = ka.col[q];
        B2 sum;
        for (int p = ka.row_ptr[r]; p < ka.diag[r]; ++p) {
          const int k = ka.col[p];
          if (k > j) break;
          const int64_t u = find(k, j);
          if (u >= 0) sum = add(sum, mul(at(P, p), at(P, u)));
        }
        if (j >= r) sum = add(sum, at(P, q));
        const B2 a = at(A, q);
        dev = std::max(dev, nrm({sum.a - a.a, sum.b - a.b, sum.c - a.c, sum.d - a.d}) / amax);
      }
      // the stored inverse of U's diagonal block
      const B2 e = mul(at(P, ka.diag[r]), at(Dinv, r));
      dev = std::max(dev, nrm({e.a - 1, e.b, e.c, e.d - 1}));
      order = 2;
    }
  } else {
    // every group: X (column-major) against its gathered block A_bb
    for (int g = 0; g < ka.nblocks(); ++g) {
      const int r0 = ka.bj_ptr[g], sz = ka.bj_ptr[g + 1] - r0, N = 2 * sz;
      order = std::max(order, N);
      std::vector<double> M((size_t)N * N, 0.0);
      for (int a = 0; a < sz; ++a) {
        const int r = ka.bj_rows[r0 + a];
        for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q) {
          const int cl = ka.col[q];
          const int l = ka.bj_loc[cl];
          if (l < sz && ka.bj_rows[r0 + l] == cl) {
            const B2 v = at(A, q);
            M[(size_t)(2 * a) * N + 2 * l] = v.a;
            M[(size_t)(2 * a) * N + 2 * l + 1] = v.b;
            M[(size_t)(2 * a + 1) * N + 2 * l] = v.c;
            M[(size_t)(2 * a + 1) * N + 2 * l + 1] = v.d;
          }
        }
      }
      const double* X = P.data() + ka.bj_off[g];
      for (int i = 0; i < N; ++i)
        for (int col = 0; col < N; ++col) {
          double sum = 0;
          for (int k = 0; k < N; ++k) sum += M[(size_t)i * N + k] * X[(size_t)col * N + k];
          dev = std::max(dev, std::fabs(sum - (i == col ? 1.0 : 0.0)));
        }
    }
  }
  *deviation = dev;
  *max_order = order;
  return PF_OK;
}
