// Dense trailing block of the factorisation (the nearly complete graph left
// by the minimum-degree elimination): right-looking blocked LU with static
// diagonal pivots and 64-wide panels.  The block is a column-major scalar
// matrix A of order M with leading dimension ld; column M holds the
// right-hand side, so the trailing updates carry the forward substitution
// along and that column ends up as L^{-1} b.  A backward solve with U
// finishes the block.
//
// Per panel step two launches: the panel (every work-group factors the
// diagonal block in LDS, then solves one 64-row tile of L or one 64-column
// tile of U) together with the previous step's trailing update away from the
// panel's block row and column, then the update of the next panel's block row
// and column (look-ahead: the bulk of the update runs beside the next panel).  Inside a 64x64 tile each of the 256
// threads keeps a 4x4 register block (rows ty+16i, columns tx+16j), and the
// pivot row / column of each elimination step goes through double-buffered
// LDS, so one barrier separates consecutive steps.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "kernels.hpp"

namespace pfd {

constexpr int NB = 64;

// Reciprocal from the hardware estimate refined by Newton steps
// r <- r + r (1 - x r) (two for FP64, one for FP32).
__device__ inline double fast_recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline float fast_recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

template <typename T>
struct Tile {
  T v[4][4];
};

// load a (nr x nc) tile at (r0, c0) into registers; outside -> identity pad
template <typename T>
__device__ inline void tile_load(Tile<T>& t, const T* A, int ld, int r0, int c0, int nr, int nc, int tx, int ty,
                                 bool ident_pad) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int r = ty + 16 * i, c = tx + 16 * j;
      T x = T(0);
      if (r < nr && c < nc)
        x = A[(int64_t)(c0 + c) * ld + r0 + r];
      else if (ident_pad && r == c)
        x = T(1);
      t.v[i][j] = x;
    }
}

template <typename T>
__device__ inline void tile_store(const Tile<T>& t, T* A, int ld, int r0, int c0, int nr, int nc, int tx, int ty) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int r = ty + 16 * i, c = tx + 16 * j;
      if (r < nr && c < nc) A[(int64_t)(c0 + c) * ld + r0 + r] = t.v[i][j];
    }
}

// Panel step k0 of every instance in the work list: item (slot, g).
//
// Every work-group factors the 64x64 diagonal block A_kk (identity-padded)
// in registers, one pivot per step: the pivot row and column go through
// double-buffered LDS, and each element update is one FMA with multipliers
// and pivot row zeroed outside the active part.  Row k of U and column k of L
// are final at step k, so in the same step each work-group also advances its
// own triangular solve:
//   g = 0:        Y = U^{-T} by forward substitution (U^T Y = I; row k of Y
//                 is final at step k); the factored block goes to dfac and
//                 U^{-1} = Y^T to dinvu (the other work-groups still read the
//                 unfactored block from A);
//   g in 1..nrt:  a 64-row tile below the block, x U = a (L_ik = A_ik U^{-1});
//   g > nrt:      a 64-column tile right of it, the last one holding the RHS
//                 column M, L y = a (U_kj = L_kk^{-1} A_kj).
// Divisions by U_kk are applied once after the loop (columns of L and of x,
// rows of Y are not touched after their step).
template <typename T>
__device__ __forceinline__ void panel_step(const Inst* const* insts, const int2 w, int k0) {
  __shared__ T row[2][NB], col[2][NB];    // pivot row / column of the block
  __shared__ T trow[2][NB], tcol[2][NB];  // published row / column of the tile
  __shared__ T rdiag[NB];
  __shared__ int bad;
  const Inst& I = *insts[w.x];
  if (I.red->active == 0) return;
  T* A = (T*)I.tail;
  const int ld = I.ldt, M = I.M;
  // the launch is uniform per work-group: keep these in scalar registers
  const int kb = __builtin_amdgcn_readfirstlane(min(NB, M - k0));
  const int nrt = __builtin_amdgcn_readfirstlane((M - (k0 + kb) + NB - 1) / NB);
  const int g = __builtin_amdgcn_readfirstlane(w.y);
  const int role = g == 0 ? 0 : (g <= nrt ? 1 : 2);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16, tid = threadIdx.x;
  if (tid == 0) bad = 0;
  if (tid < NB) rdiag[tid] = T(1);
  Tile<T> d, t;
  tile_load(d, A, ld, k0, k0, kb, kb, tx, ty, true);
  int r0 = 0, c0 = 0, nr = 0, nc = 0;
  if (role == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) t.v[i][j] = (ty + 16 * i == tx + 16 * j) ? T(1) : T(0);
  } else if (role == 1) {
    r0 = k0 + kb + (g - 1) * NB;
    nr = min(NB, M - r0);
    tile_load(t, A, ld, r0, k0, nr, kb, tx, ty, false);
  } else {
    c0 = k0 + kb + (g - 1 - nrt) * NB;
    nc = min(NB, M + 1 - c0);
    tile_load(t, A, ld, k0, c0, kb, nc, tx, ty, false);
  }
  // publish step 0: row/column 0 of the block, row 0 (roles 0, 2) or column 0
  // (role 1) of the tile
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ty + 16 * i, c = tx + 16 * j;
      if (c == 0) col[0][r] = d.v[i][j];
      if (r == 0) row[0][c] = d.v[i][j];
      if (role == 1 && c == 0) tcol[0][r] = t.v[i][j];
      if (role != 1 && r == 0) trow[0][c] = t.v[i][j];
    }
  __syncthreads();
  for (int k = 0; k < kb; ++k) {
    const int b = k & 1, nb = b ^ 1;
    T rv[4], cv[4], tv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) rv[j] = row[b][tx + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i) cv[i] = col[b][ty + 16 * i];
    if (role == 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) tv[i] = tcol[b][ty + 16 * i];
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) tv[j] = trow[b][tx + 16 * j];
    }
    T ur[4];
    if (role == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) ur[i] = row[b][ty + 16 * i];
    }
    T piv = row[b][k];
    if (tid == 0 && (!(piv != T(0)) || !isfinite((double)piv))) bad = 1;
    piv = (piv != T(0)) ? piv : T(1);
    const T rinv = fast_recip(piv);
    if (tid == 0) rdiag[k] = rinv;
    T l[4], u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) l[i] = (ty + 16 * i > k) ? cv[i] * rinv : T(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = (tx + 16 * j > k) ? rv[j] : T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) d.v[i][j] = fma(-l[i], u[j], d.v[i][j]);
    if (role == 0) {
      // rows r > k of Y: Y(r,:) -= U(k,r) Y(k,:), Y(k,:) = Yacc(k,:) / U_kk
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T m = (ty + 16 * i > k) ? ur[i] : T(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) t.v[i][j] = fma(-m, tv[j] * rinv, t.v[i][j]);
      }
    } else if (role == 1) {
      // columns c > k of x: a(:,c) -= x(:,k) U(k,c), x(:,k) = a(:,k) / U_kk
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T xk = tv[i] * rinv;
#pragma unroll
        for (int j = 0; j < 4; ++j) t.v[i][j] = fma(-xk, u[j], t.v[i][j]);
      }
    } else {
      // rows r > k of y: a(r,:) -= L(r,k) y(k,:)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) t.v[i][j] = fma(-l[i], tv[j], t.v[i][j]);
    }
    // publish row and column k+1 of the block and of the tile.  Their owners
    // are the threads with tx (ty) == (k+1) % 16, register column (row)
    // (k+1) / 16 (uniform); entries outside the active part are stored too:
    // they are finite and the next step masks them out.
    const int k1 = k + 1;
    if (k1 < kb) {
      const bool own_c = tx == (k1 & 15), own_r = ty == (k1 & 15);
#define PF_PUB(J)                                                                  \
  {                                                                                \
    if (own_c) {                                                                   \
      for (int i = 0; i < 4; ++i) col[nb][ty + 16 * i] = d.v[i][J];                \
      if (role == 1)                                                               \
        for (int i = 0; i < 4; ++i) tcol[nb][ty + 16 * i] = t.v[i][J];             \
    }                                                                              \
    if (own_r) {                                                                   \
      for (int j = 0; j < 4; ++j) row[nb][tx + 16 * j] = d.v[J][j];                \
      if (role != 1)                                                               \
        for (int j = 0; j < 4; ++j) trow[nb][tx + 16 * j] = t.v[J][j];             \
    }                                                                              \
  }
      switch (k1 >> 4) {
        case 0:
          PF_PUB(0);
          break;
        case 1:
          PF_PUB(1);
          break;
        case 2:
          PF_PUB(2);
          break;
        default:
          PF_PUB(3);
          break;
      }
#undef PF_PUB
    }
    __syncthreads();
  }
  if (role == 0) {
    // L below the diagonal: divide the stored columns by their pivots
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = ty + 16 * i, c = tx + 16 * j;
        if (r > c) d.v[i][j] *= rdiag[c];
      }
    tile_store(d, (T*)I.dfac + (int64_t)(k0 / NB) * NB * NB, NB, 0, 0, NB, NB, tx, ty);
    if (tid == 0 && bad) I.red->singular = 1;
    // U^{-1} = Y^T, rows of Y divided by their pivots
    T* ui = (T*)I.dinvu + (int64_t)(k0 / NB) * NB * NB;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ty + 16 * i;
      const T sc = rdiag[r];
#pragma unroll
      for (int j = 0; j < 4; ++j) ui[(int64_t)r * NB + tx + 16 * j] = t.v[i][j] * sc;
    }
  } else if (role == 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T sc = rdiag[tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i) t.v[i][j] *= sc;
    }
    tile_store(t, A, ld, r0, k0, nr, kb, tx, ty);
  } else {
    tile_store(t, A, ld, k0, c0, kb, nc, tx, ty);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dense_panel(const Inst* const* insts, const int2* __restrict__ work,
                                                     int k0) {
  panel_step<T>(insts, work[blockIdx.x], k0);
}

// Matrix-core 16x16x4 step: D = A B + C on a wave, one value of A and of B per
// lane (lane l holds A[l%16][l/16] and B[l/16][l%16]).  Element e of lane l
// of the result is D[row(l, e)][l%16]: row (l/16) + 4e for FP64, 4(l/16) + e
// for FP32.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int e) { return lane / 16 + 4 * e; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int e) { return 4 * (lane / 16) + e; }
};

// Trailing update A_ij -= A_ik A_kj on 64x64 tiles (rows and columns after
// the panel, the right-hand side column included), on the matrix cores: four
// waves, each a 32x32 quarter of the tile as 2x2 blocks of 16x16, K = 64 in
// steps of 4 (zero-padded past kb).  Both operands sit k-major in LDS so that
// each quarter-wave reads 16 consecutive values.
template <typename T>
__device__ __forceinline__ void gemm_tile(const Inst* const* insts, const int2 wk, int k0) {
  __shared__ T sa[NB][NB + 2];  // [k][row]
  __shared__ T sb[NB][NB + 2];  // [k][col]
  const Inst& I = *insts[wk.x];
  if (I.red->active == 0) return;
  T* A = (T*)I.tail;
  const int ld = I.ldt, M = I.M;
  const int kb = __builtin_amdgcn_readfirstlane(min(NB, M - k0));
  const int nrt = __builtin_amdgcn_readfirstlane((M - (k0 + kb) + NB - 1) / NB);
  const int tid = threadIdx.x;
  const int r0 = k0 + kb + (wk.y % nrt) * NB;
  const int c0 = k0 + kb + (wk.y / nrt) * NB;
  const int nr = min(NB, M - r0);
  const int nc = min(NB, M + 1 - c0);
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    int r = idx % NB, k = idx / NB;
    sa[k][r] = (r < nr && k < kb) ? A[(int64_t)(k0 + k) * ld + r0 + r] : T(0);
  }
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    int k = idx % NB, c = idx / NB;
    sb[k][c] = (c < nc && k < kb) ? A[(int64_t)(c0 + c) * ld + k0 + k] : T(0);
  }
  __syncthreads();
  const int lane = tid % 64, w = tid / 64;
  const int rb = (w / 2) * 32, cb = (w % 2) * 32;
  const int li = lane % 16, lk = lane / 16;
  typedef typename Mfma<T>::v4 v4;
  v4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll 4
  for (int ks = 0; ks < NB; ks += 4) {
    T a0 = sa[ks + lk][rb + li], a1 = sa[ks + lk][rb + 16 + li];
    T b0 = sb[ks + lk][cb + li], b1 = sb[ks + lk][cb + 16 + li];
    acc[0][0] = Mfma<T>::run(a0, b0, acc[0][0]);
    acc[0][1] = Mfma<T>::run(a0, b1, acc[0][1]);
    acc[1][0] = Mfma<T>::run(a1, b0, acc[1][0]);
    acc[1][1] = Mfma<T>::run(a1, b1, acc[1][1]);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int c = cb + bj * 16 + li;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rb + bi * 16 + Mfma<T>::row(lane, e);
        if (r < nr && c < nc) A[(int64_t)(c0 + c) * ld + r0 + r] -= acc[bi][bj][e];
      }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dense_gemm(const Inst* const* insts, const int2* __restrict__ work,
                                                    int k0) {
  gemm_tile<T>(insts, work[blockIdx.x], k0);
}

// Look-ahead: the panel of step k0 (items [0, npanel)) together with the
// trailing update of step k0 - 64 outside the block row and column of panel
// k0 (the other items).  The two touch disjoint tiles: the panel reads and
// writes only its block row and column, which the previous launch brought up
// to date; the update writes only tiles right of and below them.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_panel_gemm(const Inst* const* insts, const int2* __restrict__ work,
                                                          int npanel, int k0) {
  if ((int)blockIdx.x < npanel)
    panel_step<T>(insts, work[blockIdx.x], k0);
  else
    gemm_tile<T>(insts, work[blockIdx.x], k0 - NB);
}

// Backward solve U x = z (z in column M, U upper with its diagonal) by 64-row
// blocks: acc = z_b - sum_{c > b} U_bc x_c (columns taken from the last block
// down), then x_b = U_bb^{-1} acc through the inverse made by the panel step.
// Flag mode, item (slot, w): work-group w owns block b = nblk-1-w and waits
// only for blocks of the same instance listed before it (all work-groups of
// the launch are resident); results are published with an agent-scope
// release of dflags[b] = epoch, acquired by readers; the U tile of the next
// block is loaded before waiting for its flag; spins are bounded and record a
// timeout on expiry.  Single mode, item (slot, 0): one work-group runs all
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
          long spins = 0;
          while (__hip_atomic_load(&I.dflags[cb], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            if (++spins > (1l << 24)) {
              abort_flag = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
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
    const T* ui = (const T*)I.dinvu + (int64_t)b * NB * NB;
    T sum = T(0);
    for (int c = quarter; c < NB; c += 4) sum += ui[(int64_t)c * NB + lane_r] * acc[c];
    part[quarter][lane_r] = sum;
    __syncthreads();
    if (tid < bl) out[b0 + tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
    __syncthreads();
    if (!single && tid == 0) __hip_atomic_store(&I.dflags[b], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------

template <typename T>
void launch_dense_panel(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int k0) {
  if (nwork <= 0) return;
  k_dense_panel<T><<<dim3((unsigned)nwork), 256, 0, st>>>(insts, work, k0);
}

template <typename T>
void launch_dense_gemm(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int k0) {
  if (nwork <= 0) return;
  k_dense_gemm<T><<<dim3((unsigned)nwork), 256, 0, st>>>(insts, work, k0);
}

template <typename T>
void launch_dense_panel_gemm(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int npanel,
                             int k0) {
  if (nwork <= 0) return;
  k_dense_panel_gemm<T><<<dim3((unsigned)nwork), 256, 0, st>>>(insts, work, npanel, k0);
}

template <typename T>
void launch_dense_trsv(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int single) {
  if (nwork <= 0) return;
  k_dense_trsv<T><<<dim3((unsigned)nwork), 256, 0, st>>>(insts, work, single);
}

#define PF_DINST(T)                                                                        \
  template void launch_dense_panel<T>(hipStream_t, const Inst* const*, const int2*, int, int); \
  template void launch_dense_gemm<T>(hipStream_t, const Inst* const*, const int2*, int, int);  \
  template void launch_dense_panel_gemm<T>(hipStream_t, const Inst* const*, const int2*, int, int, int); \
  template void launch_dense_trsv<T>(hipStream_t, const Inst* const*, const int2*, int, int);

PF_DINST(double)
PF_DINST(float)

}  // namespace pfd
