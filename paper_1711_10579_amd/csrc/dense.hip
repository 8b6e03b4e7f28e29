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
// (ld_dev / st_dev), so no cache of any compute unit is written back or
// invalidated.  The writer waits for its stores to complete before the flag
// is set; the reader loads after seeing the flag.
__device__ inline unsigned long long flag_ld(const unsigned long long* p) {
  return __hip_atomic_load((const PF_AS1 unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every inter-work-group wait here (bounded by kWaitTicks) is on a
// work-group listed earlier in the same launch; work-groups are dispatched
// in index order, so the earliest unfinished one waits on nothing and the
// launch drains whatever else shares the device (the bound only turns a
// broken invariant into a recorded timeout instead of a hang).

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
  const auto& I = *gp(gp(insts)[w.x]);
  if (gp(I.red)->active == 0) return;
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
    want = panel_flag(gp(I.red)->epoch, k0);
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
    if (__builtin_amdgcn_ballot_w64(bad) != 0 && lane == 0) gp(I.red)->singular = 1;
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
        if (lane == 0) gp(I.red)->timeout = 1;
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
  const auto& I = *gp(gp(insts)[wk.x]);
  if (gp(I.red)->active == 0) return;
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
    if (tid == 0)
      __hip_atomic_store((PF_AS1 unsigned long long*)&I.pflags[bi0], panel_flag(gp(I.red)->epoch, k0), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
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
    gemm_tile<T>(insts, ld_item(work, b), k0, smem);
  else if (b < nflag + 4 * npanel)
    panel_step<T>(insts, ld_item(work, nflag + (b - nflag) / 4), (b - nflag) % 4, k0, smem);
  else
    gemm_tile<T>(insts, ld_item(work, b - 3 * npanel), k0, smem);
}

// ---------------------------------------------------------------------------
// Backward solve of the whole factorisation in one launch (the triangular
// solve that follows the refactorisation, Sec. III-A): the dense block's
// 64-row blocks, then the sparse rows by backward level.  Every solution
// entry is published in xs (marked unsolved before the solve) with a
// device-coherent store of the value itself; a reader polls the entries it
// needs until they lose the mark, so one memory round trip hands a value
// over (no flag, no fence).  Every wait is on a work-group listed earlier in
// the launch (or on the same work-group's earlier block in single mode);
// work-groups are dispatched in index order, so the earliest unfinished one
// waits on nothing.  A wait is bounded in device time: on expiry the
// instance records a timeout, and every other wait of the instance gives up
// as soon as it sees that.

// The entries p[0..n) of the published solution once none is marked
// unsolved (all loads in flight at once, then only the missing ones again);
// false when the instance has timed out or the bound passed.
template <typename T, int N, typename IR>
__device__ inline bool await_solved(const T* p, const bool (&use)[N], T (&v)[N], const IR& I,
                                    unsigned long long t0) {
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = use[j] ? ld_dev(p + j) : T(0);
  for (;;) {
    bool miss = false;
#pragma unroll
    for (int j = 0; j < N; ++j) miss = miss || unsolved(v[j]);
    if (!miss) return true;
    if (ld_dev(&I.red->timeout) != 0) return false;
    if (rt_now() - t0 > kWaitTicks) {
      st_dev(&I.red->timeout, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (unsolved(v[j])) v[j] = ld_dev(p + j);
  }
}

constexpr int kBwdLd = NB + 1;

// One entry per lane of the published solution (lanes with use false take
// 0), waited for with four loads in flight: each round takes the oldest load
// as it returns and issues a new one, so an entry is seen within about a
// quarter of a round trip of landing.  The rounds are wave-uniform (they end
// when no lane still sees the mark) and hold only global loads and the
// clock read, so each round waits for the oldest load alone; the wait ends
// on the device-time bound, which every waiter of a timed-out instance
// reaches within the same bound of its own start.  false when the bound
// passed.
template <typename T>
__device__ inline T ld_dev_g(const PF_AS1 T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T, typename IR>
__device__ inline bool await_lanes(const T* pf, bool use, T& v, const IR& I, unsigned long long t0) {
  const PF_AS1 T* p = gp(use ? pf : (const T*)I.xs);  // unused lanes read a valid address
  v = use ? ld_dev_g(p) : T(0);
  auto pending = [&]() { return __builtin_amdgcn_ballot_w64(unsolved(v)) != 0; };
  if (!pending()) return true;
  T a0 = ld_dev_g(p);
  __builtin_amdgcn_s_sleep(2);
  T a1 = ld_dev_g(p);
  __builtin_amdgcn_s_sleep(2);
  T a2 = ld_dev_g(p);
  __builtin_amdgcn_s_sleep(2);
  T a3 = ld_dev_g(p);
  // the first 32 rounds straight-line (exact waits on the oldest load),
  // then the same rounds in a loop with the device-time bound
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    __builtin_amdgcn_s_sleep(2);
    if (unsolved(v)) v = a0;
    if (!pending()) return true;
    a0 = ld_dev_g(p);
    __builtin_amdgcn_s_sleep(2);
    if (unsolved(v)) v = a1;
    if (!pending()) return true;
    a1 = ld_dev_g(p);
    __builtin_amdgcn_s_sleep(2);
    if (unsolved(v)) v = a2;
    if (!pending()) return true;
    a2 = ld_dev_g(p);
    __builtin_amdgcn_s_sleep(2);
    if (unsolved(v)) v = a3;
    if (!pending()) return true;
    a3 = ld_dev_g(p);
  }
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    if (unsolved(v)) v = a0;
    if (!pending()) return true;
    a0 = ld_dev_g(p);
    __builtin_amdgcn_s_sleep(2);
    if (unsolved(v)) v = a1;
    if (!pending()) return true;
    a1 = ld_dev_g(p);
    __builtin_amdgcn_s_sleep(2);
    if (unsolved(v)) v = a2;
    if (!pending()) return true;
    a2 = ld_dev_g(p);
    __builtin_amdgcn_s_sleep(2);
    if (unsolved(v)) v = a3;
    if (!pending()) return true;
    a3 = ld_dev_g(p);
    if (rt_now() - t0 > kWaitTicks) {
      st_dev(&I.red->timeout, 1);
      return false;
    }
  }
}

// Q = P A for 64x64 P and A staged in LDS (sP[j][r] = P(r, j), sA[j][r] =
// A(r, j)) on the matrix cores: wave wv forms block column wv, Q_{i,wv} =
// sum_q P_{i,q} A_{q,wv}, in N-form
template <typename T>
__device__ inline void bwd_qprod(T (*sP)[kBwdLd], T (*sA)[kBwdLd], V4<T>* qd, int wv, int lane) {
  const int c = lane & 15;
  const V4<T> zero = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    V4<T> acc4 = zero;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      V4<T> xt, y;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rw = Mfma<T>::row(lane, e);
        xt[e] = sP[16 * q + rw][16 * i + c];
        y[e] = sA[16 * wv + c][16 * q + rw];
      }
      acc4 = mm16<T>(xt, y, acc4);
    }
    qd[i] = acc4;
  }
}
template <typename T>
__device__ inline void bwd_qstore(T (*sQ)[kBwdLd], const V4<T>* qd, int wv, int lane) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) sQ[16 * wv + (lane & 15)][16 * i + Mfma<T>::row(lane, e)] = qd[i][e];
}

// One 64-row block b of the dense block, 256 threads:
//   x_b = y' - Q2 x_{b+2} - Q1 x_{b+1},
//   y' = P_b (z_b - sum_{c > b+2} A_bc x_c),  Qk = P_b A_{b,b+k}
// with P_b the diagonal block's inverse from the block step and z in column
// M (the same solution as P_b (z_b - sum_{c > b} A_bc x_c), regrouped: the
// solutions of the two blocks above arrive last, one after the other, and
// each then costs one product in one wave).  Q1 and Q2 are formed on the
// matrix cores while the block waits; the blocks right of b + 2 are summed
// as their solutions arrive, wave wv taking columns 16 wv .. 16 wv + 15 of
// each (a partial sum per row); y' over the four waves with P_b's columns
// in registers; then wave 0 waits for x_{b+2}, then for x_{b+1}, and stores
// x_b (no barrier between the waits and the store).
template <typename T, typename IR>
__device__ __forceinline__ void bwd_block(const IR& I, int b, T* smem, int* abort_flag, unsigned long long t0) {
  T(*sX)[kBwdLd] = (T(*)[kBwdLd])smem;                  // P_b, then Q1
  T(*sY)[kBwdLd] = (T(*)[kBwdLd])(smem + NB * kBwdLd);  // A_{b,b+1}, A_{b,b+2}, then Q2
  T* part = smem + 2 * NB * kBwdLd;                     // [4][NB] partial sums
  T* al = part + 4 * NB;                                // [NB] z - the sums right of b + 2
  T* x2 = al + NB;                                      // [NB] x_{b+2}
  T* x1 = x2 + NB;                                      // [NB] x_{b+1}
  const auto G = gp((const T*)I.tail);
  const int ld = I.ldt, M = I.M;
  const int nblk = (M + NB - 1) / NB;
  const int b0 = b * NB, bl = min(NB, M - b0);
  T* xs = (T*)I.xs + 2 * I.ns;
  const auto out = gp((T*)I.x) + 2 * I.ns;
  const int tid = threadIdx.x, r = tid & 63, wv = tid >> 6, lane = tid & 63;
  const auto ui = gp((const T*)I.dinvu + (int64_t)b * NB * NB);
  const bool has1 = b + 1 < nblk, has2 = b + 2 < nblk;
  const int c1 = b0 + NB, cl1 = has1 ? min(NB, M - c1) : 0;
  const int c2 = b0 + 2 * NB, cl2 = has2 ? min(NB, M - c2) : 0;
  // the block's right-hand side and this thread's columns of P_b first (on
  // the top block they are on the chain)
  const T z = (wv == 0 && r < bl) ? G[(int64_t)M * ld + b0 + r] : T(0);
  T pr[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) pr[j] = ui[(int64_t)(16 * wv + j) * NB + r];
  if (has1) {
    // Q1 = P_b A_{b,b+1}, Q2 = P_b A_{b,b+2}: P_b and one A block at a time
    // staged, the products kept in registers until P_b is no longer read
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
      const int idx = tid + 256 * q, j = idx >> 6, rr = idx & 63;
      sX[j][rr] = ui[(int64_t)j * NB + rr];
      sY[j][rr] = (rr < bl && j < cl1) ? G[(int64_t)(c1 + j) * ld + b0 + rr] : T(0);
    }
    __syncthreads();
    V4<T> q1[4], q2[4];
    bwd_qprod<T>(sX, sY, q1, wv, lane);
    if (has2) {
      __syncthreads();  // every wave has read A_{b,b+1}
#pragma unroll 4
      for (int q = 0; q < 16; ++q) {
        const int idx = tid + 256 * q, j = idx >> 6, rr = idx & 63;
        sY[j][rr] = (rr < bl && j < cl2) ? G[(int64_t)(c2 + j) * ld + b0 + rr] : T(0);
      }
      __syncthreads();
      bwd_qprod<T>(sX, sY, q2, wv, lane);
    }
    __syncthreads();  // every wave has read P_b and the A block
    bwd_qstore<T>(sX, q1, wv, lane);
    if (has2) bwd_qstore<T>(sY, q2, wv, lane);
  }
  // the blocks right of b + 2
  T pacc = T(0);
  bool ok = true;
  for (int cb = nblk - 1; cb >= b + 3 && ok; --cb) {
    const int c0 = cb * NB, cl = min(NB, M - c0);
    T a[16], xv[16];
    bool use[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int col = 16 * wv + j;
      use[j] = col < cl;
      a[j] = (r < bl && use[j]) ? G[(int64_t)(c0 + col) * ld + b0 + r] : T(0);
    }
    ok = await_solved<T, 16>(xs + c0 + 16 * wv, use, xv, I, t0);
#pragma unroll
    for (int j = 0; j < 16; ++j) pacc = fma(a[j], xv[j], pacc);
  }
  part[wv * NB + r] = pacc;
  if (!ok) *abort_flag = 1;
  __syncthreads();
  if (*abort_flag != 0) return;  // uniform: read after the barrier
  if (wv == 0) al[r] = z - (((part[r] + part[NB + r]) + part[2 * NB + r]) + part[3 * NB + r]);
  __syncthreads();
  // y' = P_b al over the four waves
  {
    T s4 = T(0);
#pragma unroll
    for (int j = 0; j < 16; ++j) s4 = fma(pr[j], al[16 * wv + j], s4);
    part[wv * NB + r] = s4;
  }
  __syncthreads();
  if (wv == 0) {
    T y = ((part[r] + part[NB + r]) + part[2 * NB + r]) + part[3 * NB + r];
    if (has2) {
      T v;
      ok = await_lanes<T>(xs + c2 + r, r < cl2, v, I, t0);
      x2[r] = v;
      __builtin_amdgcn_wave_barrier();
      T t4[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int j0 = 0; j0 < NB; j0 += 16) {
        T xv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) xv[j] = x2[j0 + j];
#pragma unroll
        for (int j = 0; j < 16; ++j) t4[j & 3] = fma(sY[j0 + j][r], xv[j], t4[j & 3]);
        __builtin_amdgcn_sched_barrier(0);
      }
      y -= (t4[0] + t4[1]) + (t4[2] + t4[3]);
    }
    if (has1 && ok) {
      // the first half of this row of Q1 in registers, then the wait
      T qr[NB / 2];
#pragma unroll
      for (int j = 0; j < NB / 2; ++j) qr[j] = sX[j][r];
      T v;
      ok = await_lanes<T>(xs + c1 + r, r < cl1, v, I, t0);
      x1[r] = v;
      __builtin_amdgcn_wave_barrier();
      T t4[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int j0 = 0; j0 < NB; j0 += 16) {
        T xv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) xv[j] = x1[j0 + j];
#pragma unroll
        for (int j = 0; j < 16; ++j) t4[j & 3] = fma(j0 < NB / 2 ? qr[j0 + j] : sX[j0 + j][r], xv[j], t4[j & 3]);
        __builtin_amdgcn_sched_barrier(0);
      }
      y -= (t4[0] + t4[1]) + (t4[2] + t4[3]);
    }
    if (__builtin_amdgcn_ballot_w64(!ok) != 0) {
      if (r == 0) *abort_flag = 1;
    } else if (r < bl) {
      out[b0 + r] = y;
      st_dev(xs + b0 + r, y);
    }
  }
  __syncthreads();
}

// Rows of one backward level, G lanes per row:
//   x_i = D_i^{-1} (y_i - sum_j U(i,j) x_j)
// (y_i in x, the entries x_j of the published solution, waited for; the
// result into both).
template <typename T, int G>
__device__ __forceinline__ void bwd_rows(const Inst* const* insts, const int2* __restrict__ rows, int count, unsigned long long t0) {
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  if (g >= count) return;  // whole groups leave together
  const int2 w = ld_item(rows, g);
  const auto& I = *gp(gp(insts)[w.x]);
  if (gp(I.red)->active == 0) return;
  const auto lu = gp((const T*)I.lu);
  const auto x = gp((T*)I.x);
  T* xs = (T*)I.xs;
  const auto colptr = gp(I.colptr), rowidx = gp(I.rowidx);
  const int i = w.y;
  Blk<T> acc = {T(0), T(0), T(0), T(0)};
  if (lane == 0) {
    acc.a = x[2 * i];
    acc.c = x[2 * i + 1];
  }
  // the inverted diagonal block first (it does not depend on the solve)
  Blk<T> D = {T(0), T(0), T(0), T(0)};
  if (lane == 0) D = ld_blk(gp((const T*)I.dinv), i);
  bool ok = true;
  {
    // four entries' loads at once, applied in order
    const int q1 = colptr[i + 1];
    for (int q = colptr[i] + lane; q < q1 && ok; q += 4 * G) {
      int jj[4];
      Blk<T> U[4];
      bool use[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        use[u] = q + u * G < q1;
        jj[u] = use[u] ? rowidx[q + u * G] : 0;
        if (use[u]) U[u] = ld_blk(lu, (int64_t)I.ns + I.nnzl + q + u * G);
      }
      T xv[8];
      bool use2[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) use2[2 * u] = use2[2 * u + 1] = use[u];
      // the entries of the four columns, waited for together
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = use2[u] ? ld_dev(xs + 2 * jj[u / 2] + (u & 1)) : T(0);
      for (;;) {
        bool miss = false;
#pragma unroll
        for (int u = 0; u < 8; ++u) miss = miss || unsolved(xv[u]);
        if (!miss) break;
        if (ld_dev(&I.red->timeout) != 0) {
          ok = false;
          break;
        }
        if (rt_now() - t0 > kWaitTicks) {
          st_dev(&I.red->timeout, 1);
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (unsolved(xv[u])) xv[u] = ld_dev(xs + 2 * jj[u / 2] + (u & 1));
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (use[u]) {
          acc.a -= U[u].a * xv[2 * u] + U[u].b * xv[2 * u + 1];
          acc.c -= U[u].c * xv[2 * u] + U[u].d * xv[2 * u + 1];
        }
    }
  }
  acc = group_sum<T, G>(acc);
  if (__builtin_amdgcn_ballot_w64(!ok) != 0) return;
  if (lane == 0) {
    const T x0 = D.a * acc.a + D.b * acc.c;
    const T x1 = D.c * acc.a + D.d * acc.c;
    x[2 * i] = x0;
    x[2 * i + 1] = x1;
    st_dev(xs + 2 * i, x0);
    st_dev(xs + 2 * i + 1, x1);
  }
}

// Work-groups [0, nd): dense blocks (item (slot, w): block nblk - 1 - w, or
// in single mode (slot, 0): every block of the instance in order); then one
// work-group per descriptor work[b] = (offset of its first row item,
// rows | G << 16): rows of one backward level and one lane-group size.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_bwd_solve(const Inst* const* insts, const int2* __restrict__ work, int nd,
                                                   int single) {
  __shared__ T smem[2 * NB * kBwdLd + 7 * NB];
  __shared__ int abort_flag;
  const unsigned long long t0 = rt_now();
  const int2 wk = ld_item(work, blockIdx.x);
  if ((int)blockIdx.x < nd) {
    const auto& I = *gp(gp(insts)[wk.x]);
    if (gp(I.red)->active == 0 || I.M == 0) return;
    const int nblk = (I.M + NB - 1) / NB;
    if (threadIdx.x == 0) abort_flag = 0;
    __syncthreads();
    // single mode: every block of the instance in order; else one block
    const int bfirst = single ? nblk - 1 : nblk - 1 - wk.y;
    const int blast = single ? 0 : bfirst;
#pragma unroll 1
    for (int b = bfirst; b >= blast && abort_flag == 0; --b) bwd_block<T>(I, b, smem, &abort_flag, t0);
    return;
  }
  const int2* rows = work + wk.x;
  const int count = wk.y & 0xffff, G = wk.y >> 16;
  switch (G) {
    case 1: bwd_rows<T, 1>(insts, rows, count, t0); break;
    case 2: bwd_rows<T, 2>(insts, rows, count, t0); break;
    case 4: bwd_rows<T, 4>(insts, rows, count, t0); break;
    case 8: bwd_rows<T, 8>(insts, rows, count, t0); break;
    case 16: bwd_rows<T, 16>(insts, rows, count, t0); break;
    case 32: bwd_rows<T, 32>(insts, rows, count, t0); break;
    default: bwd_rows<T, 64>(insts, rows, count, t0); break;
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
void launch_bwd_solve(hipStream_t st, const Inst* const* insts, const int2* work, int nd, int nrw, int single) {
  if (nd + nrw <= 0) return;
  k_bwd_solve<T><<<dim3((unsigned)(nd + nrw)), 256, 0, st>>>(insts, work, nd, single);
}

#define PF_DINST(T)                                                                        \
  template void launch_dense_step<T>(hipStream_t, const Inst* const*, const int2*, int, int, int, int); \
  template void launch_bwd_solve<T>(hipStream_t, const Inst* const*, const int2*, int, int, int);

PF_DINST(double)
PF_DINST(float)

}  // namespace pfd
