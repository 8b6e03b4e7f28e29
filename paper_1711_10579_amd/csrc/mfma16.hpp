// 16x16 blocks on the matrix cores (gfx950, wave64): the FP64 / FP32
// 16x16x4 matrix-core step, the N-form layout of a block on one wave, block
// products, staging through LDS, the Gauss-Jordan inverse of a 16x16 block
// with the pivot rows carried in registers, and the block Gauss-Jordan
// inverse of a 64x64 block on four waves.  Shared by the dense block of the
// refactorisation (dense.hip) and the block-Jacobi preconditioner
// (krylov.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace pfd {

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
  // the lane group and element holding row k
  static constexpr int grp(int k) { return k & 3; }
  static constexpr int elem(int k) { return k >> 2; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int e) { return 4 * (lane / 16) + e; }
  static constexpr int grp(int k) { return k >> 2; }
  static constexpr int elem(int k) { return k & 3; }
};

// ---------------------------------------------------------------------------
// 16x16 blocks on one wave.  The N-form of a block Z is the layout of a
// matrix-core result: lane l, element e holds Z[row(l, e)][l % 16].  Taking
// the summation index of k-step s in lane group g as row(16 g, s), element s
// of the N-form of Y is the right operand of that k-step of a product X Y,
// and element s of the N-form of X^T its left operand; the product comes out
// in N-form.

template <typename T>
using V4 = typename Mfma<T>::v4;

// C + X Y from the N-forms of X^T and of Y
template <typename T>
__device__ inline V4<T> mm16(const V4<T>& xt, const V4<T>& y, V4<T> c) {
#pragma unroll
  for (int s = 0; s < 4; ++s) c = Mfma<T>::run(xt[s], y[s], c);
  return c;
}

// a 16x16 block staged in LDS, row stride 17
constexpr int kStage = 16 * 17;
template <typename T>
__device__ inline void blk_put(T* st, const V4<T>& z, int lane) {
#pragma unroll
  for (int e = 0; e < 4; ++e) st[Mfma<T>::row(lane, e) * 17 + (lane & 15)] = z[e];
}
// N-form of the transpose of a staged block
template <typename T>
__device__ inline V4<T> blk_get_t(const T* st, int lane) {
  V4<T> z;
#pragma unroll
  for (int e = 0; e < 4; ++e) z[e] = st[(lane & 15) * 17 + Mfma<T>::row(lane, e)];
  return z;
}

// value of lane K of each 16-lane row in the whole row (DPP row broadcast;
// every lane's source is valid, so no old value is kept)
template <int K>
__device__ inline double row_bcast(double v) {
  const long long b = __builtin_amdgcn_update_dpp(0ll, __builtin_bit_cast(long long, v), 0x150 + K, 0xf, 0xf, true);
  return __builtin_bit_cast(double, b);
}
template <int K>
__device__ inline float row_bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x150 + K, 0xf, 0xf, true));
}

// value of 16-lane row R (R static) in every row of the wave, through the
// two lane-swap instructions
template <int R>
__device__ inline int grp_bcast32(int x) {
  const auto a = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows (0,0,2,2) | (1,1,3,3)
  const int h = (R & 1) ? a[1] : a[0];
  const auto b = __builtin_amdgcn_permlane32_swap(h, h, false, false);  // rows (r,r,r,r) | (r+2,...)
  return (R & 2) ? b[1] : b[0];
}
template <int R>
__device__ inline double grp_bcast(double v) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = grp_bcast32<R>((int)u), hi = grp_bcast32<R>((int)(u >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int R>
__device__ inline float grp_bcast(float v) {
  return __builtin_bit_cast(float, grp_bcast32<R>(__builtin_bit_cast(int, v)));
}
// row K of a block in N-form, for this lane's column, in every lane
template <int K, typename T>
__device__ inline T block_row(const V4<T>& z) {
  return grp_bcast<Mfma<T>::grp(K)>(z[Mfma<T>::elem(K)]);
}

// Gauss-Jordan step K (pivot K, no pivoting) on a 16x16 block Z in N-form:
// with piv = Z(K,K): Z(r,c) -= Z(r,K) Z(K,c) / piv off row and column K,
// Z(K,c) /= piv, Z(r,K) = -Z(r,K) / piv, Z(K,K) = 1 / piv.  After steps
// 0..15 the block holds its inverse.  Every lane carries the pivot row P =
// Z(K, c) and the next row Q = Z(K+1, c) of its column c; the step forms the
// next pivot row from them with the arithmetic the row's owners use, so the
// exchange of a row between lane groups happens a step ahead of its use.  A
// zero or non-finite pivot makes the reciprocal and with it every later
// value non-finite (the caller tests the result).
template <int K, typename T>
__device__ __forceinline__ void gj_step(V4<T>& z, T& P, T& Q, int lane) {
  constexpr int ek = Mfma<T>::elem(K), gk = Mfma<T>::grp(K);
  const bool ck = (lane & 15) == K;
  const T piv = row_bcast<K>(P);  // Z(K,K)
  const T mq = row_bcast<K>(Q);   // Z(K+1,K)
  T m[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) m[e] = row_bcast<K>(z[e]);  // Z(row(lane, e), K)
  const T inv = fast_recip(piv);
  // the new row K: Z(K,c) / piv, and 1 / piv in column K
  const T sel = ck ? inv : P * inv;
  const T al = ck ? T(0) : T(1);
#pragma unroll
  for (int e = 0; e < 4; ++e) z[e] = fma(-m[e], sel, al * z[e]);
  if ((lane >> 4) == gk) z[ek] = sel;
  if (K < 15) {
    P = fma(-mq, sel, al * Q);
    // row K + 2 for the step after next: an LDS permute, off the chain
    if (K < 14) {
      constexpr int K2 = K < 14 ? K + 2 : 0;
      Q = __shfl(z[Mfma<T>::elem(K2)], Mfma<T>::grp(K2) * 16 + (lane & 15));
    }
  }
}

template <typename T>
__device__ inline void blk_inverse(V4<T>& z, int lane) {
  T P = block_row<0, T>(z), Q = block_row<1, T>(z);
  gj_step<0, T>(z, P, Q, lane);
  gj_step<1, T>(z, P, Q, lane);
  gj_step<2, T>(z, P, Q, lane);
  gj_step<3, T>(z, P, Q, lane);
  gj_step<4, T>(z, P, Q, lane);
  gj_step<5, T>(z, P, Q, lane);
  gj_step<6, T>(z, P, Q, lane);
  gj_step<7, T>(z, P, Q, lane);
  gj_step<8, T>(z, P, Q, lane);
  gj_step<9, T>(z, P, Q, lane);
  gj_step<10, T>(z, P, Q, lane);
  gj_step<11, T>(z, P, Q, lane);
  gj_step<12, T>(z, P, Q, lane);
  gj_step<13, T>(z, P, Q, lane);
  gj_step<14, T>(z, P, Q, lane);
  gj_step<15, T>(z, P, Q, lane);
}

// Inverse of a 64x64 block in place by block Gauss-Jordan without pivoting
// over 4x4 blocks of 16: wave wv (of four) holds block column wv in N-form,
// d[i] = D_{i,wv}; `stage` holds two sets of four staged blocks (8 kStage
// values).  At pivot block p wave p inverts D_pp (done in the phase before)
// and stages it, then after one barrier every other wave j forms
// D_pj <- P D_pj and D_ij -= D_ip D_pj (i != p) and wave p D_ip <- -D_ip P;
// the wave that pivots next updates its own block first, stages its other
// blocks for that phase and inverts its pivot block beside the others'
// products.  On return d[i] = (D^{-1})_{i,wv}.  A zero or non-finite pivot
// leaves non-finite values (the caller tests the result).
template <typename T>
__device__ inline void inverse64(V4<T>* d, T* stage, int wv, int lane) {
  const V4<T> zero = {T(0), T(0), T(0), T(0)};
  if (wv == 0) {
    blk_inverse<T>(d[0], lane);
#pragma unroll
    for (int i = 1; i < 4; ++i) blk_put<T>(stage + i * kStage, d[i], lane);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    T* st = stage + (p & 1) * 4 * kStage;
    if (wv == p) blk_put<T>(st + p * kStage, d[p], lane);
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
  }
}

}  // namespace pfd
