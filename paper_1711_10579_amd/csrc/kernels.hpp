// Launchers of the device kernels (kernels.hip, dense.hip, krylov.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "device.hpp"

namespace pfd {

void launch_init_polar(hipStream_t, int n, const int8_t* type, const double* vmag, const double* vang,
                       double* vm, double* va, double* v, int flat);
void launch_init_cim(hipStream_t, int n, const int8_t* type, const double* vmag, const double* vang,
                     double* v);
void launch_reset_red(hipStream_t, Red* r);
void launch_mismatch_polar(hipStream_t, int n, const int* row_ptr, const int* col, const double* y,
                           const double* v, const int8_t* type, const double* psp, const double* qsp,
                           const int* pos, double* ibus, double* F, Red* red);
void launch_mismatch_cim(hipStream_t, int n, const int* row_ptr, const int* col, const double* y,
                         const double* v, const double* pg, const double* qg, const double* zip,
                         const int* pos, double* F, Red* red);

template <typename T>
void launch_zero(hipStream_t, T* p, int64_t count);
template <typename T>
void launch_jfill_polar(hipStream_t, int nnz, const int* yrow, const int* col, const double* y,
                        const double* v, const double* ibus, const double* vm, const int8_t* type,
                        const int* jmap, T* lu, T* tail, int ldt, int nt);
template <typename T>
void launch_jfill_cim(hipStream_t, int nnz, const int* yrow, const int* col, const double* y,
                      const double* v, const double* pg, const double* qg, const double* zip,
                      const int* jmap, T* lu, T* tail, int ldt, int nt);
template <typename T>
void launch_factor_cols(hipStream_t, const int* cols, int ncols, const Sched& s, T* lu, T* dinv, Red* red);
template <typename T>
void launch_tail_schur(hipStream_t, int ntt, const int* tgt, const int64_t* uptr, const int* ul,
                       const int* uu, const T* lu, T* tail, int ldt, int nt);
template <typename T>
void launch_copy_rhs(hipStream_t, int m, const double* F, T* x);
template <typename T>
void launch_fwd_rows(hipStream_t, const int* rows, int nrows, int row_base, const int* lrow_ptr,
                     const int* lrow_blk, const int* lrow_col, const T* lu, T* x, T* tail_rhs, int ns);
template <typename T>
void launch_bwd_rows(hipStream_t, const int* rows, int nrows, const Sched& s, const T* lu, const T* dinv,
                     T* x);
template <typename T>
void launch_update_polar(hipStream_t, int nu, const int* node, const int8_t* type, const T* x, double* vm,
                         double* va, double* v, Red* red);
template <typename T>
void launch_update_cim(hipStream_t, int nu, const int* node, const T* x, double* v, Red* red);

// dense trailing block; part 0: diagonal factor, 1: panel solves, 2: update
template <typename T>
void launch_dense_lu_step(hipStream_t, T* A, int ld, int M, int k0, Red* red, int part);
template <typename T>
void launch_dense_trsv_upper(hipStream_t, const T* A, int ld, int M, T* out);

}  // namespace pfd
