// Dense trailing block of the factorisation (the nearly complete graph left
// by the minimum-degree elimination): right-looking blocked LU with static
// diagonal pivots and 64-wide panels.  The block is a column-major scalar
// matrix A of order M with leading dimension ld; column M holds the
// right-hand side, so the trailing updates carry the forward substitution
// along and that column ends up as L^{-1} b.  A backward solve with U
// finishes the block.
//
// Per panel step two launches: the panel kernel (every work-group factors the
// diagonal block in LDS, then solves one 64-row tile of L or one 64-column
// tile of U) and the trailing update.  Inside a 64x64 tile each of the 256
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

// LU without pivoting of the 64x64 register tile d (padded with identity).
// Step k applies the rank-1 update with multipliers and pivot row zeroed
// outside the active part, so each element costs one FMA; the pivot column
// is kept unscaled and divided by its pivot at the end.  On return d (and
// the LDS copy s) hold unit-lower L below the diagonal and U.
template <typename T>
__device__ inline void tile_lu(Tile<T>& d, T (*s)[NB + 1], T (*col)[NB], T (*row)[NB], int tx, int ty,
                               int* bad) {
  const int tid = ty * 16 + tx;
  if (tx == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) col[0][ty + 16 * i] = d.v[i][0];
  }
  if (ty == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) row[0][tx + 16 * j] = d.v[0][j];
  }
  __syncthreads();
  for (int k = 0; k < NB; ++k) {
    const int b = k & 1, nb = b ^ 1;
    T rv[4], cv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) rv[j] = row[b][tx + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i) cv[i] = col[b][ty + 16 * i];
    T piv = row[b][k];
    if (tid == 0 && (!(piv != T(0)) || !isfinite((double)piv))) *bad = 1;
    piv = (piv != T(0)) ? piv : T(1);
    const T rinv = T(1) / piv;
    T l[4], u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) l[i] = (ty + 16 * i > k) ? cv[i] * rinv : T(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = (tx + 16 * j > k) ? rv[j] : T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) d.v[i][j] = fma(-l[i], u[j], d.v[i][j]);
    const int k1 = k + 1;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = ty + 16 * i, c = tx + 16 * j;
        if (c == k1 && r > k) col[nb][r] = d.v[i][j];
        if (r == k1 && c > k) row[nb][c] = d.v[i][j];
      }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) s[ty + 16 * i][tx + 16 * j] = d.v[i][j];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ty + 16 * i, c = tx + 16 * j;
      if (r > c) {
        T dc = s[c][c];
        dc = (dc != T(0)) ? dc : T(1);
        d.v[i][j] = d.v[i][j] / dc;
      }
    }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (ty + 16 * i > tx + 16 * j) s[ty + 16 * i][tx + 16 * j] = d.v[i][j];
  __syncthreads();
}

// Inverse of the upper triangle held in s (identity-padded): U X = I solved
// by rows from the bottom (row r of X is final once the rows below it have
// been applied; it is divided by U_rr at the end).  X is returned in x.
template <typename T>
__device__ inline void tile_upper_inverse(Tile<T>& x, T (*s)[NB + 1], T (*row)[NB], int tx, int ty) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) x.v[i][j] = (ty + 16 * i == tx + 16 * j) ? T(1) : T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (ty + 16 * i == NB - 1) row[0][tx + 16 * j] = x.v[i][j];
  __syncthreads();
  for (int st = 0; st < NB; ++st) {
    const int r = NB - 1 - st;
    const int b = st & 1, nb = b ^ 1;
    T urr = s[r][r];
    urr = (urr != T(0)) ? urr : T(1);
    const T rinv = T(1) / urr;
    T xv[4], ul[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) xv[j] = row[b][tx + 16 * j] * rinv;
#pragma unroll
    for (int i = 0; i < 4; ++i) ul[i] = (ty + 16 * i < r) ? s[ty + 16 * i][r] : T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) x.v[i][j] = fma(-ul[i], xv[j], x.v[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (r > 0 && ty + 16 * i == r - 1) row[nb][tx + 16 * j] = x.v[i][j];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T urr = s[ty + 16 * i][ty + 16 * i];
    urr = (urr != T(0)) ? urr : T(1);
#pragma unroll
    for (int j = 0; j < 4; ++j) x.v[i][j] = x.v[i][j] / urr;
  }
}

// Panel step k0 of every instance in the work list: item (slot, g).  g = 0
// writes the factored diagonal block to dfac and the inverse of its U to dinvu
// (the other work-groups still read the unfactored block from A); g in
// 1..nrt takes a 64-row tile below it (L_ik = A_ik U_kk^{-1}); the rest take
// 64-column tiles right of it, the last one holding the RHS column M
// (U_kj = L_kk^{-1} A_kj).
template <typename T>
__global__ __launch_bounds__(256) void k_dense_panel(const Inst* const* insts, const int2* __restrict__ work,
                                                     int k0) {
  __shared__ T s[NB][NB + 1];
  __shared__ T col[2][NB];
  __shared__ T row[2][NB];
  __shared__ int bad;
  const int2 w = work[blockIdx.x];
  const Inst& I = *insts[w.x];
  if (I.red->active == 0) return;
  T* A = (T*)I.tail;
  const int ld = I.ldt, M = I.M;
  const int kb = min(NB, M - k0);
  const int nrt = (M - (k0 + kb) + NB - 1) / NB;
  T* dfac = (T*)I.dfac + (int64_t)(k0 / NB) * NB * NB;
  T* dinvu = (T*)I.dinvu + (int64_t)(k0 / NB) * NB * NB;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  if (threadIdx.x == 0) bad = 0;
  Tile<T> d;
  tile_load(d, A, ld, k0, k0, kb, kb, tx, ty, true);
  tile_lu(d, s, col, row, tx, ty, &bad);
  const int b = w.y;
  if (b == 0) {
    tile_store(d, dfac, NB, 0, 0, NB, NB, tx, ty);
    if (threadIdx.x == 0 && bad) I.red->singular = 1;
    Tile<T> xi;
    tile_upper_inverse(xi, s, row, tx, ty);
    tile_store(xi, dinvu, NB, 0, 0, NB, NB, tx, ty);
    return;
  }
  Tile<T> t;
  if (b <= nrt) {
    // rows r0..r0+nr-1: x U = a by a column sweep on the unscaled columns
    const int r0 = k0 + kb + (b - 1) * NB;
    const int nr = min(NB, M - r0);
    tile_load(t, A, ld, r0, k0, nr, kb, tx, ty, false);
    if (tx == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) col[0][ty + 16 * i] = t.v[i][0];
    }
    __syncthreads();
    for (int c = 0; c < kb; ++c) {
      const int bb = c & 1, nb2 = bb ^ 1;
      T ucc = s[c][c];
      ucc = (ucc != T(0)) ? ucc : T(1);
      const T rinv = T(1) / ucc;
      T xc[4], u[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xc[i] = col[bb][ty + 16 * i] * rinv;
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = (tx + 16 * j > c) ? s[c][tx + 16 * j] : T(0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) t.v[i][j] = fma(-xc[i], u[j], t.v[i][j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (tx + 16 * j == c + 1) col[nb2][ty + 16 * i] = t.v[i][j];
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      T ucc = s[tx + 16 * j][tx + 16 * j];
      ucc = (ucc != T(0)) ? ucc : T(1);
#pragma unroll
      for (int i = 0; i < 4; ++i) t.v[i][j] = t.v[i][j] / ucc;
    }
    tile_store(t, A, ld, r0, k0, nr, kb, tx, ty);
  } else {
    // columns c0..c0+nc-1: L y = a (unit lower) by a row sweep
    const int c0 = k0 + kb + (b - 1 - nrt) * NB;
    const int nc = min(NB, M + 1 - c0);
    tile_load(t, A, ld, k0, c0, kb, nc, tx, ty, false);
    if (ty == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) row[0][tx + 16 * j] = t.v[0][j];
    }
    __syncthreads();
    for (int r = 0; r < kb; ++r) {
      const int bb = r & 1, nb2 = bb ^ 1;
      T yv[4], l[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) yv[j] = row[bb][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i) l[i] = (ty + 16 * i > r) ? s[ty + 16 * i][r] : T(0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) t.v[i][j] = fma(-l[i], yv[j], t.v[i][j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (ty + 16 * i == r + 1) row[nb2][tx + 16 * j] = t.v[i][j];
      __syncthreads();
    }
    tile_store(t, A, ld, k0, c0, kb, nc, tx, ty);
  }
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
__global__ __launch_bounds__(256) void k_dense_gemm(const Inst* const* insts, const int2* __restrict__ work,
                                                    int k0) {
  __shared__ T sa[NB][NB + 2];  // [k][row]
  __shared__ T sb[NB][NB + 2];  // [k][col]
  const int2 wk = work[blockIdx.x];
  const Inst& I = *insts[wk.x];
  if (I.red->active == 0) return;
  T* A = (T*)I.tail;
  const int ld = I.ldt, M = I.M;
  const int kb = min(NB, M - k0);
  const int nrt = (M - (k0 + kb) + NB - 1) / NB;
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
void launch_dense_trsv(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int single) {
  if (nwork <= 0) return;
  k_dense_trsv<T><<<dim3((unsigned)nwork), 256, 0, st>>>(insts, work, single);
}

#define PF_DINST(T)                                                                        \
  template void launch_dense_panel<T>(hipStream_t, const Inst* const*, const int2*, int, int); \
  template void launch_dense_gemm<T>(hipStream_t, const Inst* const*, const int2*, int, int);  \
  template void launch_dense_trsv<T>(hipStream_t, const Inst* const*, const int2*, int, int);

PF_DINST(double)
PF_DINST(float)

}  // namespace pfd
