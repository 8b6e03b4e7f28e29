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

#include "blk.hpp"
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
  // every load issued at once (addresses clamped into the tile), then masked
  const auto G = gp(A);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ty + 16 * i, c = tx + 16 * j;
      t.v[i][j] = G[(int64_t)(c0 + min(c, nc - 1)) * ld + r0 + min(r, nr - 1)];
    }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ty + 16 * i, c = tx + 16 * j;
      if (!(r < nr && c < nc)) t.v[i][j] = (ident_pad && r == c) ? T(1) : T(0);
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
// in registers, two pivots per step: the pivot rows and columns go through
// double-buffered LDS, and each element update is two FMAs with multipliers
// and pivot rows zeroed outside the active part.  Rows k, k+1 of U and
// columns k, k+1 of L are final after the step, so in the same step each
// work-group also advances its own triangular solve:
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
  // rows / columns k and k+1 of the block and of the tile, double-buffered
  __shared__ T row[2][2][NB], col[2][2][NB];
  __shared__ T trow[2][2][NB], tcol[2][2][NB];
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
  // threads 0..255 hold the diagonal block, threads 256..511 the tile (each
  // a 4x4 register block of rows ty+16i, columns tx+16j)
  const bool blk = threadIdx.x < 256;
  const int tid = threadIdx.x & 255;
  const int tx = tid % 16, ty = tid / 16;
  if (threadIdx.x == 0) bad = 0;
  if (threadIdx.x < NB) rdiag[threadIdx.x] = T(1);
  Tile<T> v;
  int r0 = 0, c0 = 0, nr = 0, nc = 0;
  if (role == 1) {
    r0 = k0 + kb + (g - 1) * NB;
    nr = min(NB, M - r0);
  } else if (role == 2) {
    c0 = k0 + kb + (g - 1 - nrt) * NB;
    nc = min(NB, M + 1 - c0);
  }
  if (blk) {
    tile_load(v, A, ld, k0, k0, kb, kb, tx, ty, true);
  } else if (role == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) v.v[i][j] = (ty + 16 * i == tx + 16 * j) ? T(1) : T(0);
  } else if (role == 1) {
    tile_load(v, A, ld, r0, k0, nr, kb, tx, ty, false);
  } else {
    tile_load(v, A, ld, k0, c0, kb, nc, tx, ty, false);
  }
  // publish rows / columns 0 and 1 of the block, and rows (roles 0, 2) or
  // columns (role 1) 0 and 1 of the tile
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ty + 16 * i, c = tx + 16 * j;
      if (blk) {
        if (c < 2) col[0][c][r] = v.v[i][j];
        if (r < 2) row[0][r][c] = v.v[i][j];
      } else {
        if (role == 1 && c < 2) tcol[0][c][r] = v.v[i][j];
        if (role != 1 && r < 2) trow[0][r][c] = v.v[i][j];
      }
    }
  __syncthreads();
  // Pivots k and k+1 per step (one barrier per pair).  With a = the block
  // before step k: l0(r) = a(r,k)/a(k,k), u0(c) = a(k,c) (r, c > k); after
  // pivot k the row and column k+1 are a'(k+1,c) = a(k+1,c) - l0(k+1) a(k,c)
  // and a'(r,k+1) = a(r,k+1) - l0(r) a(k,k+1), with pivot a'(k+1,k+1) =
  // det / a(k,k), det = a(k,k) a(k+1,k+1) - a(k+1,k) a(k,k+1); l1(r) =
  // a'(r,k+1)/a'(k+1,k+1), u1(c) = a'(k+1,c) (r, c > k+1); the block takes the
  // rank-2 update a -= l0 u0 + l1 u1.  The two reciprocals 1/a(k,k) and 1/det
  // are independent.  An odd kb pairs its last pivot with the identity
  // padding, which leaves everything unchanged.
  const int kpair = (kb + 1) & ~1;
  for (int k = 0; k < kpair; k += 2) {
    const int b = (k >> 1) & 1, nb = b ^ 1;
    const T a00 = row[b][0][k], a01 = row[b][0][k + 1], a10 = col[b][0][k + 1], a11 = row[b][1][k + 1];
    const T det = a00 * a11 - a10 * a01;
    const T p0 = (a00 != T(0)) ? a00 : T(1);
    const T dd = (det != T(0)) ? det : T(1);
    const T rinv0 = fast_recip(p0);
    const T rinv1 = p0 * fast_recip(dd);
    const T lk1 = a10 * rinv0;  // l0(k+1)
    // multipliers of the thread's rows / new U rows of its columns
    auto lmult = [&](T (&l0)[4], T (&l1)[4]) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = ty + 16 * i;
        const T cv0 = col[b][0][r], cv1 = col[b][1][r];
        l0[i] = r > k ? cv0 * rinv0 : T(0);
        l1[i] = r > k + 1 ? (cv1 - l0[i] * a01) * rinv1 : T(0);
      }
    };
    auto urows = [&](T (&u0)[4], T (&u1)[4]) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = tx + 16 * j;
        const T rv0 = row[b][0][c], rv1 = row[b][1][c];
        u0[j] = c > k ? rv0 : T(0);
        u1[j] = c > k + 1 ? rv1 - lk1 * rv0 : T(0);
      }
    };
    if (blk) {
      if (tid == 0) {
        if (!(a00 != T(0)) || !isfinite((double)a00) || !(det != T(0)) || !isfinite((double)det)) bad = 1;
        rdiag[k] = rinv0;
        rdiag[k + 1] = rinv1;
      }
      T l0[4], l1[4], u0[4], u1[4];
      lmult(l0, l1);
      urows(u0, u1);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v.v[i][j] = fma(-l1[i], u1[j], fma(-l0[i], u0[j], v.v[i][j]));
    } else if (role == 0) {
      // Y = U^{-T}: rows k, k+1 final (y0 = Y(k,:)/U_kk, y1 = (Y(k+1,:) -
      // U(k,k+1) y0)/U'_{k+1,k+1}); rows r > k take -U(k,r) y0, rows r > k+1
      // also -U'(k+1,r) y1
      T y0[4], y1[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        y0[j] = trow[b][0][tx + 16 * j] * rinv0;
        y1[j] = (trow[b][1][tx + 16 * j] - a01 * y0[j]) * rinv1;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = ty + 16 * i;
        const T ur0 = row[b][0][r], ur1 = row[b][1][r];
        const T m0 = r > k ? ur0 : T(0);
        const T m1 = r > k + 1 ? ur1 - lk1 * ur0 : T(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) v.v[i][j] = fma(-m1, y1[j], fma(-m0, y0[j], v.v[i][j]));
      }
    } else if (role == 1) {
      // x U = a: x(:,k) = a(:,k)/U_kk, x(:,k+1) = (a(:,k+1) - x(:,k) U(k,k+1))
      // / U'_{k+1,k+1}; columns c > k take -x(:,k) u0, c > k+1 also -x(:,k+1) u1
      T u0[4], u1[4], x0[4], x1[4];
      urows(u0, u1);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        x0[i] = tcol[b][0][ty + 16 * i] * rinv0;
        x1[i] = (tcol[b][1][ty + 16 * i] - x0[i] * a01) * rinv1;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v.v[i][j] = fma(-x1[i], u1[j], fma(-x0[i], u0[j], v.v[i][j]));
    } else {
      // L y = a: rows r > k take -L(r,k) y(k,:), rows r > k+1 also
      // -L(r,k+1) y(k+1,:) with y(k+1,:) = a(k+1,:) - L(k+1,k) y(k,:)
      T l0[4], l1[4], y0[4], y1[4];
      lmult(l0, l1);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        y0[j] = trow[b][0][tx + 16 * j];
        y1[j] = trow[b][1][tx + 16 * j] - lk1 * y0[j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v.v[i][j] = fma(-l1[i], y1[j], fma(-l0[i], y0[j], v.v[i][j]));
    }
    // publish rows and columns k+2 and k+3 (same register index (k+2) / 16,
    // owners tx or ty == (k+2) % 16 and (k+3) % 16): the block half its rows
    // and columns, the tile half its rows (roles 0, 2) or columns (role 1)
    const int k2 = k + 2;
    if (k2 < kpair) {
      const int s0 = k2 & 15;
      const bool c_0 = tx == s0, c_1 = tx == s0 + 1, r_0 = ty == s0, r_1 = ty == s0 + 1;
      const bool pc = blk ? (c_0 || c_1) : (role == 1 && (c_0 || c_1));
      const bool pr = blk ? (r_0 || r_1) : (role != 1 && (r_0 || r_1));
      T* cdst = blk ? &col[nb][c_1 ? 1 : 0][0] : &tcol[nb][c_1 ? 1 : 0][0];
      T* rdst = blk ? &row[nb][r_1 ? 1 : 0][0] : &trow[nb][r_1 ? 1 : 0][0];
#define PF_PUB(J)                                                       \
  {                                                                     \
    if (pc)                                                             \
      for (int i = 0; i < 4; ++i) cdst[ty + 16 * i] = v.v[i][J];        \
    if (pr)                                                             \
      for (int j = 0; j < 4; ++j) rdst[tx + 16 * j] = v.v[J][j];        \
  }
      switch (k2 >> 4) {
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
  if (blk) {
    if (role == 0 && tid == 0 && bad) I.red->singular = 1;
  } else if (role == 0) {
    // U^{-1} = Y^T, rows of Y divided by their pivots
    T* ui = (T*)I.dinvu + (int64_t)(k0 / NB) * NB * NB;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ty + 16 * i;
      const T sc = rdiag[r];
#pragma unroll
      for (int j = 0; j < 4; ++j) ui[(int64_t)r * NB + tx + 16 * j] = v.v[i][j] * sc;
    }
  } else if (role == 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T sc = rdiag[tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i) v.v[i][j] *= sc;
    }
    tile_store(v, A, ld, r0, k0, nr, kb, tx, ty);
  } else {
    tile_store(v, A, ld, k0, c0, kb, nc, tx, ty);
  }
}

template <typename T>
__global__ __launch_bounds__(512) void k_dense_panel(const Inst* const* insts, const int2* __restrict__ work,
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
  // in a 512-thread launch (beside the panel) threads 256.. only take the
  // barrier
  const bool work = threadIdx.x < 256;
  if (work) {
    // all 32 loads of a thread in flight before the LDS stores (addresses
    // clamped into the tile, values masked afterwards)
    const auto G = gp((const T*)A);
    T va[16], vb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx % NB, k = idx / NB;
      va[q] = G[(int64_t)(k0 + min(k, kb - 1)) * ld + r0 + min(r, nr - 1)];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = tid + 256 * q;
      const int k = idx % NB, c = idx / NB;
      vb[q] = G[(int64_t)(c0 + min(c, nc - 1)) * ld + k0 + min(k, kb - 1)];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx % NB, k = idx / NB;
      sa[k][r] = (r < nr && k < kb) ? va[q] : T(0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = tid + 256 * q;
      const int k = idx % NB, c = idx / NB;
      sb[k][c] = (c < nc && k < kb) ? vb[q] : T(0);
    }
  }
  __syncthreads();
  if (!work) return;
  const int lane = tid % 64, w = tid / 64;
  const int rb = (w / 2) * 32, cb = (w % 2) * 32;
  const int li = lane % 16, lk = lane / 16;
  typedef typename Mfma<T>::v4 v4;
  v4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4{T(0), T(0), T(0), T(0)};
  // the transposed product (A_ik A_kj)^T = A_kj^T A_ik^T: the matrix core's
  // first operand is the column block, so a lane's result row is a tile
  // column and its lane index within 16 a tile row -- consecutive lanes then
  // update consecutive rows of the column-major tile
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
__global__ __launch_bounds__(512) void k_dense_panel_gemm(const Inst* const* insts, const int2* __restrict__ work,
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
          long spins = 0;
          while (__hip_atomic_load(&I.dflags[cb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            if (++spins > (1l << 24)) {
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
void launch_dense_panel(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int k0) {
  if (nwork <= 0) return;
  k_dense_panel<T><<<dim3((unsigned)nwork), 512, 0, st>>>(insts, work, k0);
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
  k_dense_panel_gemm<T><<<dim3((unsigned)nwork), 512, 0, st>>>(insts, work, npanel, k0);
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
