// Dense trailing block of the factorisation (the nearly complete graph left
// by the minimum-degree elimination): right-looking blocked LU with static
// diagonal pivots, 64-wide panels.  The block is a column-major scalar matrix
// A of order M with leading dimension ld; column M holds the right-hand side,
// so the trailing updates carry the forward substitution along and the
// column ends up as L^{-1} b.  A backward solve with U finishes the block.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "kernels.hpp"

namespace pfd {

constexpr int NB = 64;

// Factor the kb x kb diagonal block at (k0, k0) in LDS (one work-group).
template <typename T>
__global__ __launch_bounds__(256) void k_dense_diag(T* A, int ld, int k0, int kb, Red* red) {
  __shared__ T s[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kb * kb; idx += blockDim.x) {
    int r = idx % kb, c = idx / kb;
    s[r][c] = A[(int64_t)(k0 + c) * ld + k0 + r];
  }
  __syncthreads();
  for (int k = 0; k < kb; ++k) {
    T piv = s[k][k];
    if (tid == 0 && (!(piv != T(0)) || !isfinite((double)piv))) red->singular = 1;
    if (!(piv != T(0))) piv = T(1);
    T rinv = T(1) / piv;
    for (int r = k + 1 + tid; r < kb; r += blockDim.x) s[r][k] *= rinv;
    __syncthreads();
    int w = kb - k - 1;
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      int r = k + 1 + idx % w, c = k + 1 + idx / w;
      s[r][c] -= s[r][k] * s[k][c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kb * kb; idx += blockDim.x) {
    int r = idx % kb, c = idx / kb;
    A[(int64_t)(k0 + c) * ld + k0 + r] = s[r][c];
  }
}

// Panel solves after the diagonal block is factored.  Work-groups [0, nrt)
// take 64-row tiles below the block: A_ip <- A_ip U_pp^{-1}; work-groups
// [nrt, nrt + nct) take 64-column tiles right of it (the last one holds the
// right-hand side column M): A_pj <- L_pp^{-1} A_pj.
template <typename T>
__global__ __launch_bounds__(64) void k_dense_trsm(T* A, int ld, int M, int k0, int kb, int nrt) {
  __shared__ T d[NB][NB + 1];
  __shared__ T t[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kb * kb; idx += blockDim.x) {
    int r = idx % kb, c = idx / kb;
    d[r][c] = A[(int64_t)(k0 + c) * ld + k0 + r];
  }
  const int b = blockIdx.x;
  if (b < nrt) {
    const int r0 = k0 + kb + b * NB;
    const int nr = min(NB, M - r0);
    for (int idx = tid; idx < nr * kb; idx += blockDim.x) {
      int r = idx % nr, c = idx / nr;
      t[r][c] = A[(int64_t)(k0 + c) * ld + r0 + r];
    }
    __syncthreads();
    if (tid < nr) {
      // row vector x with x U = a, U upper with diagonal
      for (int c = 0; c < kb; ++c) {
        T v = t[tid][c];
        for (int k = 0; k < c; ++k) v -= t[tid][k] * d[k][c];
        t[tid][c] = v / d[c][c];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nr * kb; idx += blockDim.x) {
      int r = idx % nr, c = idx / nr;
      A[(int64_t)(k0 + c) * ld + r0 + r] = t[r][c];
    }
  } else {
    const int c0 = k0 + kb + (b - nrt) * NB;
    const int nc = min(NB, M + 1 - c0);
    for (int idx = tid; idx < nc * kb; idx += blockDim.x) {
      int r = idx % kb, c = idx / kb;
      t[r][c] = A[(int64_t)(c0 + c) * ld + k0 + r];
    }
    __syncthreads();
    if (tid < nc) {
      // column y with L y = a, L unit lower
      for (int r = 1; r < kb; ++r) {
        T v = t[r][tid];
        for (int k = 0; k < r; ++k) v -= d[r][k] * t[k][tid];
        t[r][tid] = v;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nc * kb; idx += blockDim.x) {
      int r = idx % kb, c = idx / kb;
      A[(int64_t)(c0 + c) * ld + k0 + r] = t[r][c];
    }
  }
}

// Trailing update A_ij -= A_ip A_pj on 64x64 tiles (rows and columns after the
// panel, the right-hand side column included).  16x16 threads, 4x4 each.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_gemm(T* A, int ld, int M, int k0, int kb) {
  __shared__ T sa[NB][NB + 1];  // [row][k]
  __shared__ T sb[NB][NB + 1];  // [k][col]
  const int tid = threadIdx.x;
  const int r0 = k0 + kb + blockIdx.x * NB;
  const int c0 = k0 + kb + blockIdx.y * NB;
  const int nr = min(NB, M - r0);
  const int nc = min(NB, M + 1 - c0);
  for (int idx = tid; idx < NB * kb; idx += blockDim.x) {
    int r = idx % NB, k = idx / NB;
    sa[r][k] = r < nr ? A[(int64_t)(k0 + k) * ld + r0 + r] : T(0);
  }
  for (int idx = tid; idx < NB * kb; idx += blockDim.x) {
    int k = idx % kb, c = idx / kb;
    sb[k][c] = c < nc ? A[(int64_t)(c0 + c) * ld + k0 + k] : T(0);
  }
  __syncthreads();
  const int tx = tid % 16, ty = tid / 16;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
  for (int k = 0; k < kb; ++k) {
    T av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) av[i] = sa[ty + 16 * i][k];
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = sb[k][tx + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int c = tx + 16 * j;
    if (c >= nc) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r = ty + 16 * i;
      if (r < nr) A[(int64_t)(c0 + c) * ld + r0 + r] -= acc[i][j];
    }
  }
}

// Backward solve U x = z (z in column M, U upper with diagonal) by 64-row
// blocks from the bottom, one work-group; x goes to out[0..M).
template <typename T>
__global__ __launch_bounds__(256) void k_dense_trsv_upper(const T* A, int ld, int M, T* out) {
  __shared__ T xs[NB];
  __shared__ T zs[NB];
  const int tid = threadIdx.x;
  const T* z = A + (int64_t)M * ld;
  // work copy of z in out (updated in place)
  for (int i = tid; i < M; i += blockDim.x) out[i] = z[i];
  __syncthreads();
  const int nblk = (M + NB - 1) / NB;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int b0 = blk * NB;
    const int bl = min(NB, M - b0);
    if (tid < 64) {
      T zt = tid < bl ? out[b0 + tid] : T(0);
      for (int c = bl - 1; c >= 0; --c) {
        T ucc = A[(int64_t)(b0 + c) * ld + b0 + c];
        T zc = __shfl(zt, c, 64);
        T xc = zc / ucc;
        if (tid == c) zt = xc;
        if (tid < c) zt -= A[(int64_t)(b0 + c) * ld + b0 + tid] * xc;
      }
      if (tid < bl) {
        xs[tid] = zt;
        out[b0 + tid] = zt;
      }
    }
    __syncthreads();
    for (int r = tid; r < b0; r += blockDim.x) {
      T v = out[r];
      for (int c = 0; c < bl; ++c) v -= A[(int64_t)(b0 + c) * ld + r] * xs[c];
      out[r] = v;
    }
    __syncthreads();
  }
  (void)zs;
}

// ---------------------------------------------------------------------------

template <typename T>
void launch_dense_lu_step(hipStream_t st, T* A, int ld, int M, int k0, Red* red, int part) {
  const int kb = min(NB, M - k0);
  const int rest_r = M - (k0 + kb);
  const int rest_c = M + 1 - (k0 + kb);
  const int nrt = (rest_r + NB - 1) / NB;
  const int nct = (rest_c + NB - 1) / NB;
  if (part == 0) {
    k_dense_diag<T><<<1, 256, 0, st>>>(A, ld, k0, kb, red);
  } else if (part == 1) {
    if (nrt + nct > 0) k_dense_trsm<T><<<dim3((unsigned)(nrt + nct)), 64, 0, st>>>(A, ld, M, k0, kb, nrt);
  } else {
    if (nrt > 0 && nct > 0) k_dense_gemm<T><<<dim3((unsigned)nrt, (unsigned)nct), 256, 0, st>>>(A, ld, M, k0, kb);
  }
}

template <typename T>
void launch_dense_trsv_upper(hipStream_t st, const T* A, int ld, int M, T* out) {
  if (M <= 0) return;
  k_dense_trsv_upper<T><<<1, 256, 0, st>>>(A, ld, M, out);
}

template void launch_dense_lu_step<double>(hipStream_t, double*, int, int, int, Red*, int);
template void launch_dense_lu_step<float>(hipStream_t, float*, int, int, int, Red*, int);
template void launch_dense_trsv_upper<double>(hipStream_t, const double*, int, int, double*);
template void launch_dense_trsv_upper<float>(hipStream_t, const float*, int, int, float*);

}  // namespace pfd
