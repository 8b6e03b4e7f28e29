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
struct KState;

struct Inst {
  int model, n, nnz, nu, ns, nt, ldt, M, ntt, nblk;
  int64_t nnzl;
  int64_t lu_count, tail_count;
  const int *row_ptr, *col, *yrow, *jmap;
  const double* y;
  const int8_t* type;
  const double *psp, *qsp, *vmag, *vang, *zip;
  // CIM: per node {node its delta load draws into, node whose delta load it
  // receives} (-1: none; null without delta loads), the delta ZIP
  // coefficients [6n], and the generator Q of PV nodes (their Newton state
  // in place of |V|, which stays at the set-point)
  const int2* dlink;
  const double* zipd;
  double* qg;
  const int *pos, *node;
  // rows of more than kHeavyRow Ybus entries (the mismatch gives each a
  // work-group of its own)
  int nheavy;
  const int* heavy;
  // partial maxima of the mismatch (one per 64 rows) and of the update (one
  // per 256 unknown nodes), reduced by the convergence test
  int nmpart, nupart;
  double *mpart, *upart;
  double *vm, *va, *v, *ibus, *F;
  void *x, *lu, *dinv, *tail, *dinvu;
  // the backward solve's published copy of the solution (2 nu values),
  // marked unsolved before each solve: a row or block waits for the entries
  // it needs to lose the mark
  void* xs;
  // per 64-row block i of the dense block: (epoch << 20) | (k + 1) once the
  // panel of block step k has stored its tile L_ik
  unsigned long long* pflags;
  const int *colptr, *rowidx, *upd_l, *upd_u;
  const int64_t* uptr;
  const int *tail_tgt, *tail_l, *tail_u;
  const int64_t* tail_uptr;
  const int *lrow_ptr, *lrow_blk, *lrow_col;
  // Newton-Krylov storage (allocated on the first Krylov solve of the case;
  // null before).  Krylov vectors: 2 values per node with unknowns, nodes in
  // Krylov order r (kp_of_r[r] = factor position); the Jacobian as 2x2
  // blocks on the block CSR pattern krow_ptr/kcol (diagonal at kdiag), its
  // ILU(0) factor on the same pattern (pval) with the inverted diagonal
  // blocks (pdinv), or the block-Jacobi inverses (bjinv, bj_off).
  int km;        // restart length the basis storage holds
  int kchunks;   // vector chunks of KCH rows
  int knb;       // block-Jacobi blocks
  int knl, knul; // ILU(0) forward and backward levels
  int kwide;     // some level is wider than one work-group pass: the ILU(0)
                 // factor and sweeps run one launch per level, not in one
                 // work-group
  const int *kp_of_r, *krow_ptr, *kcol, *kdiag, *kmap, *kup_ptr, *kup_t, *kup_s;
  // rows by forward / backward level: level pointers, and per position
  // {row, first, end, 0} of the row's lower (forward) or upper (backward)
  // entries
  const int *kl_ptr, *ku_ptr;
  const int4 *kl_info, *ku_info;
  const int *bj_ptr, *bj_rows, *bj_loc;
  const int64_t* bj_off;
  int* bjbad;  // per group: 1 when its inverse needs partial pivoting
  void *jval, *pval, *pdinv, *bjinv;
  void *kv;      // basis [(km+1) x 2 nu]
  void *kw, *kz, *kx;  // work vectors [2 nu]
  double* kh;    // H [(km+1) x km] row-major, cs [km], sn [km], g [km+1], y [km]
  double* kpart; // partial sums [3][kchunks][km+1]
  KState* ks;
  Red* red;
};

// Per-instance state of the Krylov inner solve of the current Newton step.
struct KState {
  double bnorm;  // ||F||_2
  double eta;    // forcing term (relative residual target)
  double scale;  // factor that normalises the next basis vector
  double rel;    // residual estimate relative to bnorm
  double rho[2];  // BiCGStab: <r0, r> for the iteration of that parity
  double alpha, omega, beta;  // BiCGStab: the step factors
  int j;         // Arnoldi steps of the current cycle (BiCGStab: iterations done)
  int cycle;     // restarts done
  int state;     // KS_* below
  int met;       // forcing term met
  int total;     // Arnoldi steps of this Newton step
  int pad;
};
// KS_BP, KS_BS: the two halves of a BiCGStab iteration; KS_BH: the first
// half met the tolerance (its update of x pending)
enum { KS_DONE = 0, KS_ITER = 1, KS_CYCLE = 2, KS_RESTART = 3, KS_FINISH = 4, KS_BP = 5, KS_BS = 6, KS_BH = 7 };

// Options of the Krylov inner solve.
struct KOpts {
  double eta_max, eta_floor;
  int m, max_restarts;
};

// rows of a Krylov vector chunk (one work-group of KCH threads)
constexpr int KCH = 256;

// Options the device-side convergence test needs.
struct DevOpts {
  double tol;
  int max_iter;
  int pad;
};

}  // namespace pfd
