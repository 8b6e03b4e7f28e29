// Device-side data layout shared by the kernels and the host driver.
//
// Every kernel works on a batch of instances: it receives the device table
// of per-instance descriptors (Inst) and either a 2D grid (y = batch slot) for
// element-wise work or a flattened work list of (slot, item) pairs.  A solve
// of one case is a batch of one; each item's arithmetic depends only on its
// own instance, so an instance gives bit-identical results alone and in any
// batch.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pfd {

// Per-instance Newton state driven on the device.
struct Red {
  unsigned long long norm_bits;  // max |F| of the last mismatch, IEEE bits (non-negative values order as integers)
  unsigned long long step_bits;  // max |dx| of the last step
  double norm0;                  // max |F| at the flat start
  double last_norm;              // max |F| seen by the last convergence test
  double last_step;              // max |dx| seen by the last convergence test
  int singular;                  // set when a pivot is zero or non-finite
  int timeout;                   // a bounded inter-work-group wait expired
  int epoch;                     // step counter for inter-work-group flags
  int it;                        // Newton steps taken
  int status;                    // pf_solve_status (PF_PENDING while active)
  int active;                    // 1 while Newton steps remain
  int linear_iters;              // Krylov iterations summed over the steps
  int pad;
};

// Per-instance descriptor (device memory, one per case).
//
// Factor storage, block ids of the sparse part:
//   D_j: j;  L(rowidx[colptr[j]+p], j): ns + colptr[j] + p;
//   U(j, rowidx[colptr[j]+p]): ns + nnzl + colptr[j] + p;
// 4 values per block, row-major [a00 a01 a10 a11].  Targets of column j:
// tb = j + 2 colptr[j]; D: tb, U(j, r_p): tb + 1 + p, L(r_p, j): tb + 1 +
// len + p; updates of target t: [uptr[t], uptr[t+1]).  The dense trailing
// block (positions ns..nu-1) is a column-major scalar matrix of order M = 2 nt
// with leading dimension ldt and the right-hand side in column M.
struct Inst {
  int model, n, nnz, nu, ns, nt, ldt, M, ntt, nblk;
  int64_t nnzl;
  int64_t lu_count, tail_count;
  const int *row_ptr, *col, *yrow, *jmap;
  const double* y;
  const int8_t* type;
  const double *psp, *qsp, *vmag, *vang, *zip;
  const int *pos, *node;
  double *vm, *va, *v, *ibus, *F;
  void *x, *lu, *dinv, *tail, *dfac, *dinvu;
  int* dflags;
  const int *colptr, *rowidx, *upd_l, *upd_u;
  const int64_t* uptr;
  const int *tail_tgt, *tail_l, *tail_u;
  const int64_t* tail_uptr;
  const int *lrow_ptr, *lrow_blk, *lrow_col;
  // Krylov (NK) storage: J in CSR over block rows (same pattern as Ybus on
  // the unknowns), its ILU(0) / block-Jacobi factor and the GMRES basis
  const int *jrow_ptr, *jcol, *jdiag, *jmap_k;
  void *jval, *pval, *kry, *kh;
  Red* red;
};

// Options the device-side convergence test needs.
struct DevOpts {
  double tol;
  int max_iter;
  int pad;
};

}  // namespace pfd
