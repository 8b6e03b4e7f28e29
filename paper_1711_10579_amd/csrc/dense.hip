// Dense trailing block of the factorisation (the nearly complete graph left
// by the minimum-degree elimination): right-looking block LU with static
// pivots and 64-wide blocks in block-LDU form -- the diagonal blocks are
// inverted outright and the block-lower factor keeps identity diagonal
// blocks:
//   P_k = A_kk^{-1},  L_ik = A_ik P_k (i > k),  A_ij -= L_ik A_kj (i, j > k),
// the block row A_kj (j > k) staying as it is.  The block is a column-major
// scalar matrix A of order M with leading dimension ld; column M holds the
// right-hand side, so the trailing updates carry the block forward
// substitution along.  The backward solve x_k = P_k (z_k - sum_{j>k} A_kj x_j)
// finishes the block.
//
// One launch per 64-wide block step k: the previous step's update of the
// tiles right of the diagonal block and below its block row (k-1 <- the
// tiles' last but one step), beside the panel of step k: every panel
// work-group inverts the diagonal block on the matrix cores (block
// Gauss-Jordan over 16x16 blocks), multiplies one 64-row tile below it by
// the inverse and applies this step's update to that row's tile of the next
// block column, so that the next launch's panel finds its block column up
// to date.  The rest of this step's update runs in the next launch, beside
// the next panel.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "blk.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "mfma16.hpp"

namespace pfd {

constexpr int NB = 64;

// LDS of a dense launch (elements of T): the larger of the panel's (staged
// blocks, a quarter row tile and its L rows) and the update's (two operand
// tiles)
constexpr int kQuarterLd = 17;
constexpr int kGemmLd = NB + 2;
constexpr int kPanelSmem = 8 * kStage + 2 * NB * kQuarterLd;
constexpr int kDenseSmem = 2 * NB * kGemmLd > kPanelSmem ? 2 * NB * kGemmLd : kPanelSmem;

// Value of a row block's flag once the previous step's update of its tile
// in the next block column of step k0 is stored, in Newton step `epoch`
// (epochs only grow, so every earlier value is smaller).
__device__ inline unsigned long long panel_flag(int epoch, int k0) {
  return ((unsigned long long)(unsigned)epoch << 20) | (unsigned long long)(k0 / NB + 1);
}

// A tile handed over inside a launch goes through device-coherent accesses
// (relaxed atomics at agent scope: stores write through, loads bypass the
// caches not coherent across the device), so no cache of any compute unit
// is written back or invalidated.  The writer waits for its stores to
// complete before the flag is set; the reader loads after seeing the flag.
template <typename T>
__device__ inline T ld_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void st_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long flag_ld(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// s_waitcnt vmcnt(0): every vector memory access of the wave, stores
// included, has completed
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Bound of an inter-work-group wait in ticks of the device's constant
// real-time counter (100 MHz): about one second.  Every wait here is on a
// work-group listed earlier in the same launch; work-groups are dispatched
// in index order, so the earliest unfinished one waits on nothing and the
// launch drains whatever else shares the device (the bound only turns a
// broken invariant into a recorded timeout instead of a hang).
constexpr unsigned long long kWaitTicks = 100000000ull;
__device__ inline unsigned long long rt_now() { return __builtin_amdgcn_s_memrealtime(); }

// Panel step k0 of every instance in the work list: item (slot, g), one of
// four work-groups h of four waves.  Every work-group inverts the diagonal
// block D = A_kk (identity-padded to 64x64) by block Gauss-Jordan over 4x4
// blocks of 16: wave j keeps block column j in N-form; at pivot block p wave
// p inverts D_pp (P) and stages P and its other blocks D_ip in LDS, then
// after one barrier every other wave j forms D_pj <- P D_pj and
// D_ij -= D_ip D_pj (i != p) and wave p D_ip <- -D_ip P.  Then
//   g = 0:        (h = 0 only) P is stored, column-major, for the backward
//                 solve;
//   g in 1..nrt:  rows 16h..16h+15 of row tile i = g - 1 below the block:
//                 L_ik = A_ik P, computed transposed (P^T A_ik^T) so that
//                 consecutive lanes store consecutive rows; then the same
//                 rows of the row's tile C in the next block column take this
//                 step's update, C -= L_ik A_{k,k+1}, once the previous step's
//                 update of C and of A_{k,k+1} is stored (the flags of both
//                 row blocks, set by work-groups earlier in the launch).  Each
//                 wave reads the flags as it starts and loads its part of C
//                 and A_{k,k+1} as soon as both are seen, while the inverse
//                 is still being formed.
template <typename T>
__device__ __forceinline__ void panel_step(const Inst* const* insts, const int2 w, int h, int k0, T* smem) {
  T* stage = smem;                    // two sets of four staged blocks
  T* xs = smem + 8 * kStage;          // the work-group's rows of A_ik, column-major [NB][kQuarterLd]
  T* ls = xs + NB * kQuarterLd;       // the same rows of L_ik
  const Inst& I = *insts[w.x];
  if (I.red->active == 0) return;
  // the launch is uniform per work-group: keep these in scalar registers
  const int g = __builtin_amdgcn_readfirstlane(w.y);
  if (g == 0 && h != 0) return;
  // the panel is the launch's critical path: its waves issue first on a
  // SIMD shared with update work-groups
  __builtin_amdgcn_s_setprio(3);
  T* A = (T*)I.tail;
  const int ld = I.ldt, M = I.M;
  const int kb = __builtin_amdgcn_readfirstlane(min(NB, M - k0));
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, c = lane & 15;
  int r0 = 0, nr = 0;  // this work-group's rows, nr <= 16
  if (g > 0) {
    r0 = k0 + kb + (g - 1) * NB + 16 * h;
    nr = M - r0 < 16 ? M - r0 : 16;
    if (nr <= 0) return;
  }
  const int c1 = k0 + kb;  // the next block column; may be the right-hand side column M
  const int nc = min(NB, M + 1 - c1);
  const auto G = gp((const T*)A);
  // the flags of this row block and of the block row, read as each phase
  // of the inverse starts and tested as it ends, then polled after it
  const bool wait = g > 0 && k0 > 0;
  unsigned long long want = 0, f1 = 0, f2 = 0;
  if (wait) {
    want = panel_flag(I.red->epoch, k0);
    f1 = flag_ld(&I.pflags[r0 / NB]);
    f2 = flag_ld(&I.pflags[k0 / NB]);
  }
  // the diagonal block's column block wv, identity outside kb x kb
  V4<T> d[4];
  {
    const int cc = 16 * wv + c;
    const int64_t cb = (int64_t)(k0 + min(cc, kb - 1)) * ld + k0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) d[i][e] = G[cb + min(16 * i + Mfma<T>::row(lane, e), kb - 1)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * i + Mfma<T>::row(lane, e);
        if (!(r < kb && cc < kb)) d[i][e] = r == cc ? T(1) : T(0);
      }
  }
  // the rows of A_ik (zero outside nr x kb), staged column-major
  if (g > 0) {
    const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
    T v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = G[(int64_t)(k0 + min(tc + 16 * q, kb - 1)) * ld + r0 + min(tr, nr - 1)];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int cc = tc + 16 * q;
      xs[cc * kQuarterLd + tr] = (tr < nr && cc < kb) ? v[q] : T(0);
    }
  }
  // this wave's part of the update: C^T block (wv) of the rows, N-form, and
  // the blocks (q, wv) of U = A_{k,k+1}, N-form
  V4<T> ct, un[4];
  auto fetch = [&]() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
    for (int e = 0; e < 4; ++e)
      ct[e] = ld_dev(&A[(int64_t)(c1 + min(16 * wv + Mfma<T>::row(lane, e), nc - 1)) * ld + r0 + min(c, nr - 1)]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        un[q][e] = ld_dev(&A[(int64_t)(c1 + min(16 * wv + c, nc - 1)) * ld + k0 + min(16 * q + Mfma<T>::row(lane, e), kb - 1)]);
  };
  bool have = false;
  if (g > 0 && !wait) {
    fetch();
    have = true;
  }
  const V4<T> zero = {T(0), T(0), T(0), T(0)};
  // the pivot wave of each phase has inverted its block before the phase:
  // wave 0 here, wave p + 1 during phase p, right after the update of its
  // own block and together with its other updates (matrix-core work beside
  // the inverse's vector work), its other blocks staged before the inverse
  if (wv == 0) {
    blk_inverse<T>(d[0], lane);
#pragma unroll
    for (int i = 1; i < 4; ++i) blk_put<T>(stage + i * kStage, d[i], lane);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    T* st = stage + (p & 1) * 4 * kStage;
    if (p > 0 && wait && !have) {
      f1 = flag_ld(&I.pflags[r0 / NB]);
      f2 = flag_ld(&I.pflags[k0 / NB]);
    }
    if (wv == p) blk_put<T>(st + p * kStage, d[p], lane);
    // one barrier per pivot block: a set of staged blocks is rewritten
    // (from the phase before its next use) after every wave has passed the
    // barrier of the phase that read it
    __syncthreads();
    if (wv == p) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i != p) d[i] = mm16<T>(-blk_get_t<T>(st + i * kStage, lane), d[p], zero);
    } else {
      const V4<T> npj = mm16<T>(blk_get_t<T>(st + p * kStage, lane), d[p], zero);
      if (wv == p + 1) {
        T* sn = stage + ((p + 1) & 1) * 4 * kStage;
        d[p + 1] = mm16<T>(-blk_get_t<T>(st + (p + 1) * kStage, lane), npj, d[p + 1]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i != p && i != p + 1) d[i] = mm16<T>(-blk_get_t<T>(st + i * kStage, lane), npj, d[i]);
        d[p] = npj;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i != p + 1) blk_put<T>(sn + i * kStage, d[i], lane);
        blk_inverse<T>(d[p + 1], lane);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i != p) d[i] = mm16<T>(-blk_get_t<T>(st + i * kStage, lane), npj, d[i]);
        d[p] = npj;
      }
    }
    if (wait && !have && __builtin_amdgcn_readfirstlane((f1 >= want && f2 >= want) ? 1 : 0)) {
      fetch();
      have = true;
    }
  }
  // d[i] = P_{i,wv}
  if (g == 0) {
    // a zero or non-finite pivot anywhere leaves no finite value in P
    bool bad = false;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
      for (int e = 0; e < 4; ++e) bad = bad || !isfinite((double)d[ib][e]);
    if (__builtin_amdgcn_ballot_w64(bad) != 0 && lane == 0) I.red->singular = 1;
    T* ui = (T*)I.dinvu + (int64_t)(k0 / NB) * NB * NB;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) ui[(int64_t)(16 * wv + c) * NB + 16 * i + Mfma<T>::row(lane, e)] = d[i][e];
    return;
  }
  bool expired = false;
  if (!have) {
    // bounded in device time: on expiry the instance records a timeout and
    // the update is not stored
    const unsigned long long t_start = rt_now();
    for (;;) {
      f1 = flag_ld(&I.pflags[r0 / NB]);
      f2 = flag_ld(&I.pflags[k0 / NB]);
      if (__builtin_amdgcn_readfirstlane((f1 >= want && f2 >= want) ? 1 : 0)) break;
      if (rt_now() - t_start > kWaitTicks) {
        expired = true;
        if (lane == 0) I.red->timeout = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    fetch();
  }
  // (A_ik P)_{wv}^T = sum_q P_{q,wv}^T (A_ik)_q^T over the rows
  V4<T> acc = zero;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    V4<T> xn;
#pragma unroll
    for (int e = 0; e < 4; ++e) xn[e] = xs[(16 * q + Mfma<T>::row(lane, e)) * kQuarterLd + c];
    acc = mm16<T>(d[q], xn, acc);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int col = 16 * wv + Mfma<T>::row(lane, e);
    if (c < nr && col < kb) st_dev(&A[(int64_t)(k0 + col) * ld + r0 + c], acc[e]);
    ls[col * kQuarterLd + c] = acc[e];
  }
  __syncthreads();
  // C -= L_ik U, transposed like the product above
  V4<T> cu = ct;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    V4<T> yn;
#pragma unroll
    for (int e = 0; e < 4; ++e) yn[e] = ls[(16 * q + Mfma<T>::row(lane, e)) * kQuarterLd + c];
    cu = mm16<T>(-un[q], yn, cu);
  }
  if (!expired)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int col = 16 * wv + Mfma<T>::row(lane, e);
      if (c < nr && col < nc) st_dev(&A[(int64_t)(c1 + col) * ld + r0 + c], cu[e]);
    }
}

// The previous block step's update of one 64x64 tile, A_ij -= L_{i,k-1}
// A_{k-1,j} (k-1 at column k0 - 64; the tile's columns may include the
// right-hand side column M), on the matrix cores: four waves, each a 32x32
// quarter of the tile as 2x2 blocks of 16x16, K = 64 in steps of 4.  Item
// (slot, j | i << 12 | flag << 24) for block row i and block column j; with
// the flag the tile is announced in pflags[i] once stored.  The tile is
// loaded with the operands, straight into the accumulators; operands sit
// k-major in LDS (L negated) so that each quarter-wave reads 16 consecutive
// values.
template <typename T>
__device__ __forceinline__ void gemm_tile(const Inst* const* insts, const int2 wk, int k0, T* smem) {
  T(*sa)[kGemmLd] = (T(*)[kGemmLd])smem;                   // [k][row]
  T(*sb)[kGemmLd] = (T(*)[kGemmLd])(smem + NB * kGemmLd);  // [k][col]
  const Inst& I = *insts[wk.x];
  if (I.red->active == 0) return;
  T* A = (T*)I.tail;
  const int ld = I.ldt, M = I.M;
  const int bi0 = __builtin_amdgcn_readfirstlane((wk.y >> 12) & 0xfff);
  const int bj0 = __builtin_amdgcn_readfirstlane(wk.y & 0xfff);
  const bool flag = (wk.y >> 24) != 0;
  if (flag) __builtin_amdgcn_s_setprio(2);
  const int kp = k0 - NB;
  const int tid = threadIdx.x;
  const int r0 = bi0 * NB, c0 = bj0 * NB;
  const int nr = min(NB, M - r0);
  const int nc = min(NB, M + 1 - c0);
  const int lane = tid % 64, w = tid / 64;
  const int rb = (w / 2) * 32, cb = (w % 2) * 32;
  const int li = lane % 16, lk = lane / 16;
  typedef typename Mfma<T>::v4 v4;
  const auto G = gp((const T*)A);
  // every load of a thread in flight at once (addresses clamped into the
  // tiles, values masked afterwards)
  v4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rb + bi * 16 + li, c = cb + bj * 16 + Mfma<T>::row(lane, e);
        acc[bi][bj][e] = G[(int64_t)(c0 + min(c, nc - 1)) * ld + r0 + min(r, nr - 1)];
      }
  T va[16], vb[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q;
    const int r = idx % NB, k = idx / NB;
    va[q] = G[(int64_t)(kp + k) * ld + r0 + min(r, nr - 1)];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q;
    const int k = idx % NB, c = idx / NB;
    vb[q] = G[(int64_t)(c0 + min(c, nc - 1)) * ld + kp + k];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q;
    const int r = idx % NB, k = idx / NB;
    sa[k][r] = r < nr ? -va[q] : T(0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q;
    const int k = idx % NB, c = idx / NB;
    sb[k][c] = c < nc ? vb[q] : T(0);
  }
  __syncthreads();
  // the transposed product (L U)^T = U^T L^T: the matrix core's first
  // operand is the column block, so a lane's result row is a tile column and
  // its lane index within 16 a tile row -- consecutive lanes then update
  // consecutive rows of the column-major tile
#pragma unroll 4
  for (int ks = 0; ks < NB; ks += 4) {
    T a0 = sa[ks + lk][rb + li], a1 = sa[ks + lk][rb + 16 + li];
    T b0 = sb[ks + lk][cb + li], b1 = sb[ks + lk][cb + 16 + li];
    acc[0][0] = Mfma<T>::run(b0, a0, acc[0][0]);
    acc[0][1] = Mfma<T>::run(b1, a0, acc[0][1]);
    acc[1][0] = Mfma<T>::run(b0, a1, acc[1][0]);
    acc[1][1] = Mfma<T>::run(b1, a1, acc[1][1]);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int r = rb + bi * 16 + li;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = cb + bj * 16 + Mfma<T>::row(lane, e);
        if (r < nr && c < nc) st_dev(&A[(int64_t)(c0 + c) * ld + r0 + r], acc[bi][bj][e]);
      }
    }
  if (flag) {
    // every wave's stores have completed before the flag is set
    wait_vmem();
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&I.pflags[bi0], panel_flag(I.red->epoch, k0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Block step k0 in one launch: items [0, nflag) the previous step's update
// of the tiles of the next block column (and of the block row's tile
// there), which announce themselves; then the npanel panel items of step
// k0, four work-groups each (a quarter of the item's row tile apiece), which
// wait for those; then the rest of the previous step's update.  Work-groups
// start in index order, so every wait is on a work-group that already runs.
// The items write disjoint tiles except the next block column's, written by
// its flagged update and then, after the flag, by its panel work-groups.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_dense_step(const Inst* const* insts, const int2* __restrict__ work,
                                                    int nflag, int npanel, int k0) {
  __shared__ T smem[kDenseSmem];
  const int b = blockIdx.x;
  if (b < nflag)
    gemm_tile<T>(insts, work[b], k0, smem);
  else if (b < nflag + 4 * npanel)
    panel_step<T>(insts, work[nflag + (b - nflag) / 4], (b - nflag) % 4, k0, smem);
  else
    gemm_tile<T>(insts, work[b - 3 * npanel], k0, smem);
}

// Block backward solve (z in column M): by 64-row blocks, acc = z_b -
// sum_{c > b} A_bc x_c (columns taken from the last block down), then x_b =
// P_b acc with the diagonal block's inverse made by the panel step.
// Flag mode, item (slot, w): work-group w owns block b = nblk-1-w and waits
// only for blocks of the same instance listed before it (dispatched before
// it, so the earliest unfinished block waits on nothing); results are
// published with an agent-scope release of dflags[b] = epoch, acquired by
// readers; the U tile of the next block is loaded before waiting for its
// flag; a wait is bounded in device time and records a timeout on expiry.  Single mode, item (slot, 0): one work-group runs all
// blocks of its instance in order.  Both modes do the same arithmetic.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_trsv(const Inst* const* insts, const int2* __restrict__ work,
                                                    int single) {
  __shared__ T part[4][NB];
  __shared__ T acc[NB];
  __shared__ int abort_flag;
  const int2 wk = work[blockIdx.x];
  const Inst& I = *insts[wk.x];
  if (I.red->active == 0) return;
  const T* A = (const T*)I.tail;
  const int ld = I.ldt, M = I.M;
  T* out = (T*)I.x + 2 * I.ns;
  const int tid = threadIdx.x;
  const int nblk = (M + NB - 1) / NB;
  const int lane_r = tid % NB, quarter = tid / NB;
  const int epoch = I.red->epoch;
  const int bfirst = single ? nblk - 1 : nblk - 1 - wk.y;
  const int blast = single ? 0 : bfirst;
  if (tid == 0) abort_flag = 0;
  for (int b = bfirst; b >= blast; --b) {
    const int b0 = b * NB;
    const int bl = min(NB, M - b0);
    // this block's U^{-1} entries (independent of the solve): loaded first
    T uiv[16];
    {
      const T* ui = (const T*)I.dinvu + (int64_t)b * NB * NB;
#pragma unroll
      for (int q = 0; q < 16; ++q) uiv[q] = ui[(int64_t)(quarter + 4 * q) * NB + lane_r];
    }
    __syncthreads();
    if (tid < NB) acc[tid] = tid < bl ? A[(int64_t)M * ld + b0 + tid] : T(0);
    __syncthreads();
    for (int cb = nblk - 1; cb > b; --cb) {
      const int c0 = cb * NB;
      const int cl = min(NB, M - c0);
      T u[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = quarter + 4 * q;
        u[q] = (lane_r < bl && c < cl) ? A[(int64_t)(c0 + c) * ld + b0 + lane_r] : T(0);
      }
      if (!single) {
        if (tid == 0) {
          // poll without ordering, then one acquire once the flag is seen
          const unsigned long long t_start = rt_now();
          while (__hip_atomic_load(&I.dflags[cb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            if (rt_now() - t_start > kWaitTicks) {
              abort_flag = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (abort_flag) break;
      }
      T sum = T(0);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = quarter + 4 * q;
        if (c < cl) sum += u[q] * out[c0 + c];
      }
      part[quarter][lane_r] = sum;
      __syncthreads();
      if (tid < NB) acc[tid] -= part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
      __syncthreads();
    }
    if (abort_flag) {
      if (tid == 0) I.red->timeout = 1;
      return;
    }
    T sum = T(0);
#pragma unroll
    for (int q = 0; q < 16; ++q) sum += uiv[q] * acc[quarter + 4 * q];
    part[quarter][lane_r] = sum;
    __syncthreads();
    if (tid < bl) out[b0 + tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
    __syncthreads();
    if (!single && tid == 0) __hip_atomic_store(&I.dflags[b], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------

template <typename T>
void launch_dense_step(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int nflag, int npanel,
                       int k0) {
  if (nwork <= 0) return;
  k_dense_step<T><<<dim3((unsigned)(nwork + 3 * npanel)), 256, 0, st>>>(insts, work, nflag, npanel, k0);
}

template <typename T>
void launch_dense_trsv(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int single) {
  if (nwork <= 0) return;
  k_dense_trsv<T><<<dim3((unsigned)nwork), 256, 0, st>>>(insts, work, single);
}

#define PF_DINST(T)                                                                        \
  template void launch_dense_step<T>(hipStream_t, const Inst* const*, const int2*, int, int, int, int); \
  template void launch_dense_trsv<T>(hipStream_t, const Inst* const*, const int2*, int, int);

PF_DINST(double)
PF_DINST(float)

}  // namespace pfd
