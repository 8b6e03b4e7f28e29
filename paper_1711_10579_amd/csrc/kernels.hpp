// Launchers of the device kernels (kernels.hip, dense.hip, krylov.hip).  All
// take the batch's device table of instance descriptors.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "device.hpp"

namespace pfd {

// descriptor upload (by value, stream-ordered) and a zero fill of 32-bit words
void launch_set_inst(hipStream_t, Inst* dst, const Inst& src);
void launch_zero_words(hipStream_t, void* p, int64_t words);

// Newton driver
void launch_init(hipStream_t, const Inst* const* insts, int nslots, int max_n, int flat);
void launch_start(hipStream_t, const Inst* const* insts, int nslots);
void launch_decide(hipStream_t, const Inst* const* insts, int nslots, DevOpts o);
void launch_gather_red(hipStream_t, const Inst* const* insts, int nslots, Red* out);
// rows of more than kHeavyRow Ybus entries run one work-group each (max_heavy:
// the most such rows of an instance in the batch)
constexpr int kHeavyRow = 64;
void launch_mismatch(hipStream_t, const Inst* const* insts, int nslots, int max_n, int max_heavy);
template <typename T>
void launch_update(hipStream_t, const Inst* const* insts, int nslots, int max_nu);

// Jacobian fill: RHS copy, zero the factor storage (chunk items, see
// zero_chunk_values), scatter J
template <typename T>
void launch_fill(hipStream_t, const Inst* const* insts, int nslots, int max_nu2, const int2* zero_work, int nzero,
                 int max_nnz);
int zero_chunk_values();

// sparse part (work items (slot, column) or (slot, row); G lanes per list)
// (wide: 1024 threads per column instead of 256, for levels of few columns
// with many targets each)
template <typename T>
void launch_factor_cols(hipStream_t, const Inst* const* insts, const int2* work, int nwork, int G, int wide);
template <typename T>
void launch_fwd_rows(hipStream_t, const Inst* const* insts, const int2* work, int nwork, int G);
template <typename T>
void launch_tail_schur(hipStream_t, const Inst* const* insts, const int2* work, int nwork, int G);
// one column per wave; for levels whose columns have at most 64/G targets
template <typename T>
void launch_factor_cols_wave(hipStream_t, const Inst* const* insts, const int2* work, int nwork, int G);

// dense trailing block
template <typename T>
void launch_dense_step(hipStream_t, const Inst* const* insts, const int2* work, int nwork, int nflag, int npanel,
                       int k0);
// backward solve of the whole factorisation in one launch: nd dense items
// (slot, w) (single: (slot, 0), one work-group per instance), then nrw
// work-groups of sparse rows, each described by work[nd + k] = (offset of its
// first row item in work, rows | G << 16), row items (slot, row)
template <typename T>
void launch_bwd_solve(hipStream_t, const Inst* const* insts, const int2* work, int nd, int nrw, int single);

// Newton-Krylov inner solve (krylov.hip); preconditioner mode 0 = Arnoldi
// step, 1 = end of a GMRES cycle, 2 and 3 = the halves of a BiCGStab
// iteration
template <typename T>
void launch_kfill(hipStream_t, const Inst* const* insts, int nslots, int max_nnz, int ilu);
template <typename T>
void launch_ilu_rows(hipStream_t, const Inst* const* insts, const int2* work, int nwork);
template <typename T>
void launch_bj_inv(hipStream_t, const Inst* const* insts, const int2* work, int nbig, int nsmall);
int bj_small_nodes();  // groups of at most this many nodes are inverted one per wave
template <typename T>
void launch_ilu_fwd(hipStream_t, const Inst* const* insts, const int2* work, int nwork, int mode);
template <typename T>
void launch_ilu_bwd(hipStream_t, const Inst* const* insts, const int2* work, int nwork, int mode);
template <typename T>
void launch_ilu_factor_wg(hipStream_t, const Inst* const* insts, int nslots);
template <typename T>
void launch_ilu_apply_wg(hipStream_t, const Inst* const* insts, int nslots, int mode, int min_nu, int max_nu);
template <typename T>
void launch_bj_apply(hipStream_t, const Inst* const* insts, const int2* work, int nbig, int nwork, int mode);
template <typename T>
void launch_karnoldi(hipStream_t, const Inst* const* insts, int nslots, int max_chunks, KOpts o);
template <typename T>
void launch_kbegin(hipStream_t, const Inst* const* insts, int nslots, int max_chunks, KOpts o);
template <typename T>
void launch_kycomb(hipStream_t, const Inst* const* insts, int nslots, int max_chunks);
template <typename T>
void launch_kcycle_end(hipStream_t, const Inst* const* insts, int nslots, int max_chunks, KOpts o);
template <typename T>
void launch_kfinish(hipStream_t, const Inst* const* insts, int nslots, int max_chunks);
// BiCGStab: start and the first direction, then per iteration it [apply
// mode 2], v = J p^ and s, [apply mode 3], the first half's test with
// t = J s^, the update of x and r, and the test with the next direction
template <typename T>
void launch_bcg_begin(hipStream_t, const Inst* const* insts, int nslots, int max_chunks, KOpts o);
template <typename T>
void launch_bcg_dir(hipStream_t, const Inst* const* insts, int nslots, int max_chunks);
template <typename T>
void launch_bcg_half(hipStream_t, const Inst* const* insts, int nslots, int max_chunks, int it);
template <typename T>
void launch_bcg_end(hipStream_t, const Inst* const* insts, int nslots, int max_chunks, KOpts o, int it);
void launch_kgather(hipStream_t, const Inst* const* insts, int nslots, int* out);
int krylov_max_restart();

}  // namespace pfd
