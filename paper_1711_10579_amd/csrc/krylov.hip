// HIP kernels of the Newton-Krylov inner solve (Sec. III-B) for gfx950.
//
// Right-preconditioned restarted GMRES(m) on the 2x2-block Jacobian, batched
// over instances: every kernel takes the instance table and skips instances
// whose Krylov state is not the one the kernel serves, so one launch
// sequence drives instances that need different numbers of steps.
//
// One Arnoldi step (state KS_ITER):
//   z = M^{-1} (scale * w), writing the normalised basis vector v_j on the
//   way (ILU(0) forward/backward rows by level, or block-Jacobi) ->
//   w = J z with the partial dots <w, v_i> (k_kspmv_dot) -> two classical
//   Gram-Schmidt passes (k_korth; the second re-orthogonalises and yields
//   ||w||) -> Givens rotation and residual estimate (k_karnoldi_end).
// End of a cycle (KS_CYCLE): u = V y, z = M^{-1} u, x += z; then either the
// result is final (KS_FINISH) or the true residual F - J x starts the next
// cycle (KS_RESTART).
//
// Value type T of the Jacobian, the preconditioner and the basis is double
// (plain) or float (mixed precision); dot products, norms, the Hessenberg
// matrix and the rotations are double.  Partial sums are reduced in a fixed
// order, so an instance's arithmetic does not depend on the batch.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "blk.hpp"
#include "mfma16.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace pfd {

namespace {

constexpr int KMAX = 128;  // largest restart length the kernels accept

// Helpers over an instance descriptor reached through a generic or a global
// reference (kernels that read theirs through global pointers get scalar
// loads of its fields and vector loads counted by one wait counter).
template <typename IR>
__device__ inline bool kstate_is(const IR& I, int want) {
  return gp(I.red)->active && gp(I.ks)->state == want;
}

// the Krylov state a preconditioner application serves: mode 0 an Arnoldi
// step (scaled input stored as basis vector), 1 the end of a GMRES cycle,
// 2 and 3 the first and second half of a BiCGStab iteration
__device__ inline int apply_state(int mode) {
  return mode == 0 ? KS_ITER : mode == 1 ? KS_CYCLE : KS_BP;
}

template <typename IR>
__device__ inline double* kh_H(const IR& I) { return I.kh; }
template <typename IR>
__device__ inline double* kh_cs(const IR& I) { return I.kh + (int64_t)(I.km + 1) * I.km; }
template <typename IR>
__device__ inline double* kh_sn(const IR& I) { return kh_cs(I) + I.km; }
template <typename IR>
__device__ inline double* kh_g(const IR& I) { return kh_sn(I) + I.km; }
template <typename IR>
__device__ inline double* kh_y(const IR& I) { return kh_g(I) + I.km + 1; }
template <typename IR>
__device__ inline PF_AS1 double* kpart(const IR& I, int pass, int chunk) {
  return gp(I.kpart) + ((int64_t)pass * I.kchunks + chunk) * (I.km + 1);
}

// The inner solve failed: the Newton iteration of the instance ends with
// status linear failure and the step is not taken (not counted).
template <typename IR>
__device__ inline void linear_failure(const IR& I) {
  gp(I.red)->status = 4;
  gp(I.red)->active = 0;
  gp(I.red)->it -= 1;
  gp(I.ks)->state = KS_DONE;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums over the KCH threads of a work-group of the values f(i) for i <
// count, written to out[i] (thread-uniform count).  Fixed reduction order.
template <typename F>
__device__ inline void block_sums(int count, F f, double (*red)[KCH / 64], PF_AS1 double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = 0; i < count; ++i) {
    double s = wave_sum(f(i));
    if (lane == 0) red[i][wave] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += KCH) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < KCH / 64; ++w) s += red[i][w];
    out[i] = s;
  }
}

// Sums over the chunks of N entries of the partial sums (entry es[k] of
// pass ps[k]; |value| where bit k of AbsMask is set), each in a fixed order
// (the same value wherever it is formed).  Called by all 64 lanes of one
// wave: lane l adds chunks l, l + 64, l + 128, ... in turn, then the
// butterfly of wave_sum.  The loads for four such chunks of every entry are
// issued together; past the last chunk a load repeats chunk 0 and adds
// nothing.
template <int N, int AbsMask = 0, typename IR>
__device__ inline void chunk_sums(const IR& I, const int (&ps)[N], const int (&es)[N], double (&out)[N]) {
  const int lane = threadIdx.x & 63, nc = I.kchunks;
  double s[N];
#pragma unroll
  for (int k = 0; k < N; ++k) s[k] = 0.0;
  for (int c0 = 0; c0 < nc; c0 += 256) {
    double v[4][N];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + 64 * u + lane;
      const int cc = c < nc ? c : 0;
#pragma unroll
      for (int k = 0; k < N; ++k) v[u][k] = kpart(I, ps[k], cc)[es[k]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = c0 + 64 * u + lane < nc;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const double x = (AbsMask >> k) & 1 ? fabs(v[u][k]) : v[u][k];
        s[k] += in ? x : 0.0;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < N; ++k) out[k] = wave_sum(s[k]);
}
template <typename IR>
__device__ inline double chunk_sum(const IR& I, int pass, int e) {
  double o[1];
  chunk_sums<1>(I, {pass}, {e}, o);
  return o[0];
}

// acc -= (Sub) or += (not Sub) sum over entries q in [q0, q1) of block
// M(q) times entries col(q) of vector x, in order of q; the loads of four
// entries (their blocks, columns and the gathered x values) are issued
// together, so a row costs two round trips rather than two per entry (past
// the range's end a load repeats its first entry and adds nothing).
template <bool Sub, typename T, typename MP, typename CP, typename XP>
__device__ inline void blk_range_dot(MP M, CP col, int q0, int q1, XP x, double& acc0, double& acc1) {
  for (int q = q0; q < q1; q += 4) {
    int c[4];
    Blk<T> B[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int qq = q + u < q1 ? q + u : q0;
      c[u] = col[qq];
      B[u] = ld_blk(M, qq);
    }
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = (double)x[2 * c[u]];
      b[u] = (double)x[2 * c[u] + 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u < q1) {
        if (Sub) {
          acc0 -= (double)B[u].a * a[u] + (double)B[u].b * b[u];
          acc1 -= (double)B[u].c * a[u] + (double)B[u].d * b[u];
        } else {
          acc0 += (double)B[u].a * a[u] + (double)B[u].b * b[u];
          acc1 += (double)B[u].c * a[u] + (double)B[u].d * b[u];
        }
      }
  }
}

// acc -= (Sub) or += (not Sub) row r of the block Jacobian times x
template <bool Sub, typename T, typename IR, typename XP>
__device__ inline void spmv_row(const IR& I, int r, XP x, double& acc0, double& acc1) {
  blk_range_dot<Sub, T>(gp((const T*)I.jval), gp(I.kcol), gp(I.krow_ptr)[r], gp(I.krow_ptr)[r + 1], x, acc0, acc1);
}

}  // namespace

// ---------------------------------------------------------------------------
// preconditioner set-up

// ILU(0) rows of one level (IKJ form): each lower block of row r becomes
// L(r,k) = A(r,k) U(k,k)^{-1}, followed by its listed updates
// A(r,j) -= L(r,k) U(k,j); then the row's diagonal block is inverted.  One
// thread per row; rows of earlier levels are final.
// The updates of row r from one of its lower entries, L = L(r, k):
// P(t_u) -= L P(s_u) for u in [u0, u1).  The targets are distinct entries of
// row r and the sources lie in row k < r, so the loads of four updates are
// issued together; every target still sees its updates in the order of the
// row's lower entries.
template <typename T, typename PP, typename IP>
__device__ inline void ilu_updates(PP P, IP kup_t, IP kup_s, int u0, int u1, const Blk<T>& L) {
  for (int u = u0; u < u1; u += 4) {
    int t[4], sr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (u + e < u1) {
        t[e] = kup_t[u + e];
        sr[e] = kup_s[u + e];
      }
    Blk<T> a[4], b[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (u + e < u1) {
        a[e] = ld_blk<T>(P, t[e]);
        b[e] = ld_blk<T>(P, sr[e]);
      }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (u + e < u1) {
        blk_msub(a[e], L, b[e]);
        st_blk(P, t[e], a[e]);
      }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ilu_rows(const Inst* const* insts, const int2* __restrict__ work, int nwork) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nwork) return;
  const int2 wk = ld_item(work, idx);
  const auto& I = *gp(gp(insts)[wk.x]);
  if (!gp(I.red)->active) return;
  const int r = wk.y;
  const auto P = gp((T*)I.pval);
  const auto D = gp((T*)I.pdinv);
  const int qd = gp(I.kdiag)[r];
  const auto kcol = gp(I.kcol), kup_ptr = gp(I.kup_ptr), kup_t = gp(I.kup_t), kup_s = gp(I.kup_s);
  const int q0 = gp(I.krow_ptr)[r];
  // as in k_ilu_factor_wg: the next lower entry's column, update range and
  // diagonal inverse fetched during this entry's updates
  if (q0 < qd) {
    int u0 = kup_ptr[q0], u1 = kup_ptr[q0 + 1];
    Blk<T> Dk = ld_blk<T>(D, kcol[q0]);
    for (int q = q0; q < qd; ++q) {
      const int qn = q + 1 < qd ? q + 1 : q;
      const int cn = kcol[qn], un = kup_ptr[qn + 1];
      const Blk<T> L = blk_mul(ld_blk<T>(P, q), Dk);
      st_blk(P, q, L);
      const Blk<T> Dn = ld_blk<T>(D, cn);
      ilu_updates<T>(P, kup_t, kup_s, u0, u1, L);
      u0 = u1;
      u1 = un;
      Dk = Dn;
    }
  }
  Blk<T> inv;
  if (!blk_inv(ld_blk(P, qd), &inv)) {
    gp(I.red)->singular = 1;
    inv.a = inv.b = inv.c = inv.d = T(0);
  }
  st_blk(D, r, inv);
}

// Block-Jacobi: inverse of the diagonal block A_bb of one node group (order
// N = 2 x nodes <= 64), stored column-major at bj_off[b], in three launches:
//   k_bj_inv_mfma (groups of more than kBjSmall nodes, a work-group each):
//     the block, padded with the identity to 64 x 64, inverted on the matrix
//     cores by block Gauss-Jordan without pivoting (FP64);
//   k_bj_inv_small (the other groups, a wave each, four to a work-group):
//     the block padded to 16 x 16, inverted by Gauss-Jordan without
//     pivoting on one wave (FP64);
//     in both the result is kept when it is finite and max |A_bb X - I| <=
//     1e-6, else the group is marked (bjbad[b] = 1);
//   k_bj_inv: the marked groups only, by Gauss-Jordan with partial pivoting
//     on [A | I] in LDS (FP64).
// All compute A_bb^{-1}; pivoting and the padding change only the rounding.
// Grouping the nodes leaves many groups of one or two nodes (a node whose
// neighbours all belong to earlier groups), which is why the small groups
// get a wave and not a work-group.
constexpr double kBjResidualTol = 1e-6;
constexpr int kBjSmall = 8;  // nodes: groups up to this size take k_bj_inv_small

// the entries of the group's rows that fall inside the group, stored into
// the row-major LDS array A (columns 0..2s-1).  Eight threads per member row
// (thread t of 8 s takes row t / 8), each taking every eighth entry of its
// row, so a row's chain of dependent loads (member -> row range -> column ->
// local index) is paid once rather than once per entry.  Distinct entries of
// a row have distinct columns, so no two threads store the same element.
template <typename T, int LD, typename IR>
__device__ inline void bj_scatter_rows(const IR& I, int r0, int s, double (*A)[LD], int t) {
  const int a = t >> 3, j = t & 7;
  if (a >= s) return;
  const auto rows = gp(I.bj_rows), loc = gp(I.bj_loc), kcol = gp(I.kcol), kptr = gp(I.krow_ptr);
  const auto jv = gp((const T*)I.jval);
  const int r = rows[r0 + a];
  const int q1 = kptr[r + 1];
  for (int q = kptr[r] + j; q < q1; q += 8) {
    const int c = kcol[q];
    const int l = loc[c];
    if (l < s && rows[r0 + l] == c) {
      const auto v = jv + 4 * (int64_t)q;
      A[2 * a][2 * l] = (double)v[0];
      A[2 * a][2 * l + 1] = (double)v[1];
      A[2 * a + 1][2 * l] = (double)v[2];
      A[2 * a + 1][2 * l + 1] = (double)v[3];
    }
  }
}

// the group's block gathered into a row-major 64 x (64 + pad) LDS array
// (identity outside N x N)
template <typename T, int LD, typename IR>
__device__ inline void bj_gather(const IR& I, int r0, int s, double (*A)[LD]) {
  const int tid = threadIdx.x;
  const int N = 2 * s;
  for (int e = tid; e < 64 * 64; e += blockDim.x) {
    const int i = e >> 6, c = e & 63;
    A[i][c] = (i == c && i >= N) ? 1.0 : 0.0;
  }
  __syncthreads();
  bj_scatter_rows<T, LD>(I, r0, s, A, threadIdx.x);
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_bj_inv_mfma(const Inst* const* insts, const int2* __restrict__ work) {
  __shared__ double A[64][65];
  __shared__ double stage[8 * kStage];
  __shared__ int bad_s;
  const int2 wk = work[blockIdx.x];
  const auto& I = *gp(gp(insts)[wk.x]);
  if (!gp(I.red)->active) return;
  const int b = wk.y;
  const int r0 = gp(I.bj_ptr)[b];
  const int s = gp(I.bj_ptr)[b + 1] - r0;
  const int N = 2 * s;
  if (threadIdx.x == 0) bad_s = 0;
  bj_gather<T, 65>(I, r0, s, A);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15;
  // wave wv: block column wv in N-form
  V4<double> d[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) d[i][e] = A[16 * i + Mfma<double>::row(lane, e)][16 * wv + c];
  inverse64<double>(d, stage, wv, lane);
  // residual A X - I of this block column: (A X)_{i,wv} = sum_q A_iq X_{q,wv},
  // A_iq^T in N-form read straight from the row-major array
  bool bad = false;
  const V4<double> zero = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    V4<double> acc = zero;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      V4<double> at;
#pragma unroll
      for (int e = 0; e < 4; ++e) at[e] = A[16 * i + c][16 * q + Mfma<double>::row(lane, e)];
      acc = mm16<double>(at, d[q], acc);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * i + Mfma<double>::row(lane, e), col = 16 * wv + c;
      const double r = acc[e] - (row == col ? 1.0 : 0.0);
      bad = bad || !(fabs(r) <= kBjResidualTol) || !isfinite(d[i][e]);
    }
  }
  if (__builtin_amdgcn_ballot_w64(bad) != 0 && lane == 0) bad_s = 1;
  __syncthreads();
  if (threadIdx.x == 0) I.bjbad[b] = bad_s;
  if (bad_s) return;
  // stored column-major: entry (i, col) at col N + i
  T* out = (T*)I.bjinv + gp(I.bj_off)[b];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * i + Mfma<double>::row(lane, e), col = 16 * wv + c;
      if (row < N && col < N) out[col * N + row] = (T)d[i][e];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bj_inv_small(const Inst* const* insts, const int2* __restrict__ work,
                                                      int nwork) {
  __shared__ double A[4][16][17];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15;
  const int k = blockIdx.x * 4 + wv;
  // every wave reaches both barriers; a wave without a group inverts the
  // identity and stores nothing
  int2 wk = make_int2(0, -1);
  if (k < nwork) wk = work[k];
  const auto ip = wk.y >= 0 ? gp(gp(insts)[wk.x]) : nullptr;
  const bool ok = ip && gp(ip->red)->active;
  const int b = wk.y;
  const int r0 = ok ? gp(ip->bj_ptr)[b] : 0;
  const int s = ok ? gp(ip->bj_ptr)[b + 1] - r0 : 0;
  const int N = 2 * s;
  double(*Aw)[17] = A[wv];
#pragma unroll
  for (int e = lane; e < 256; e += 64) {
    const int i = e >> 4, cc = e & 15;
    Aw[i][cc] = (i == cc && i >= N) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (ok) bj_scatter_rows<T, 17>(*ip, r0, s, Aw, lane);
  __syncthreads();
  V4<double> z;
#pragma unroll
  for (int e = 0; e < 4; ++e) z[e] = Aw[Mfma<double>::row(lane, e)][c];
  blk_inverse<double>(z, lane);
  // A X - I from the N-form of A^T read straight from the staged block
  const V4<double> zero = {0.0, 0.0, 0.0, 0.0};
  const V4<double> ax = mm16<double>(blk_get_t<double>(&Aw[0][0], lane), z, zero);
  bool bad = false;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = Mfma<double>::row(lane, e);
    const double r = ax[e] - (row == c ? 1.0 : 0.0);
    bad = bad || !(fabs(r) <= kBjResidualTol) || !isfinite(z[e]);
  }
  bad = __builtin_amdgcn_ballot_w64(bad) != 0;
  if (!ok) return;
  if (lane == 0) ip->bjbad[b] = bad ? 1 : 0;
  if (bad) return;
  T* out = (T*)ip->bjinv + gp(ip->bj_off)[b];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = Mfma<double>::row(lane, e);
    if (row < N && c < N) out[c * N + row] = (T)z[e];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bj_inv(const Inst* const* insts, const int2* __restrict__ work) {
  __shared__ double A[64][129];
  __shared__ double colk[64];
  __shared__ double rowk[128];
  __shared__ int piv;
  __shared__ int bad;
  const int2 wk = work[blockIdx.x];
  const auto& I = *gp(gp(insts)[wk.x]);
  if (!gp(I.red)->active) return;
  const int b = wk.y;
  if (b < 0 || !I.bjbad[b]) return;  // padding, or inverted without pivoting
  const int r0 = gp(I.bj_ptr)[b];
  const int s = gp(I.bj_ptr)[b + 1] - r0;
  const int N = 2 * s;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 128; e += 256) {
    const int i = e >> 7, c = e & 127;
    A[i][c] = (c >= 64 && c - 64 == i) ? 1.0 : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  bj_scatter_rows<T, 129>(I, r0, s, A, tid);  // the block beside the identity
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    if (tid < 64) {  // pivot search by the first wave
      double best = (tid >= k && tid < N) ? fabs(A[tid][k]) : -1.0;
      int who = tid;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        double ob = __shfl_xor(best, off, 64);
        int ow = __shfl_xor(who, off, 64);
        if (ob > best || (ob == best && ow < who)) {
          best = ob;
          who = ow;
        }
      }
      if (tid == 0) {
        piv = who;
        if (!(best > 0.0) || !isfinite(best)) bad = 1;
      }
    }
    __syncthreads();
    if (bad) break;
    const int p = piv;
    if (p != k && tid < 128) {
      double t = A[k][tid];
      A[k][tid] = A[p][tid];
      A[p][tid] = t;
    }
    __syncthreads();
    // the pivot column and the pivot row, read before any thread writes:
    // both threads of a column scale the pivot row's entry from the staged
    // copy, so the one that stores it cannot race the other's read
    if (tid < N) colk[tid] = A[tid][k];
    if (tid < 128) rowk[tid] = A[k][tid];
    __syncthreads();
    // thread (c, h) owns column c of [A | I] and the rows i = h mod 2: the
    // pivot row is scaled by 1/A[k][k] and every other row loses
    // A[i][k] times it (column k itself becomes exactly the unit column);
    // columns left of k are zero in the pivot row and are skipped
    {
      const int c = tid & 127, h = tid >> 7;
      if (c >= k) {
        const double ip = 1.0 / colk[k];
        const double akc = rowk[c] * ip;
        for (int i = h; i < N; i += 2)
          if (i != k) A[i][c] -= colk[i] * akc;
        if (h == 0) A[k][c] = akc;
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) gp(I.red)->singular = 1;
    return;
  }
  // stored column-major: entry (i, c) at c N + i, so that a wave applying the
  // block reads one contiguous column per step
  T* out = (T*)I.bjinv + gp(I.bj_off)[b];
  for (int e = tid; e < N * N; e += 256) {
    const int c = e / N, i = e - c * N;
    out[e] = (T)A[i][64 + c];
  }
}

// ---------------------------------------------------------------------------
// preconditioner application

// ILU(0) forward rows of one level: y_r = s w_r - sum_{k<r} L(r,k) y_k.  In
// an Arnoldi step (mode 0) the scaled input is also stored as basis vector
// v_j.  In the end-of-cycle solve (mode 1) the input is u and s = 1.
template <typename T>
__global__ __launch_bounds__(256) void k_ilu_fwd(const Inst* const* insts, const int2* __restrict__ work, int nwork,
                                                 int mode) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nwork) return;
  const int2 wk = ld_item(work, idx);
  const auto& I = *gp(gp(insts)[wk.x]);
  if (!kstate_is(I, apply_state(mode))) return;
  const int r = wk.y;
  const auto w = gp((const T*)I.kw);
  const auto z = gp((T*)I.kz);
  const auto P = gp((const T*)I.pval);
  T v0 = w[2 * r], v1 = w[2 * r + 1];
  if (mode == 0) {
    const double sc = gp(I.ks)->scale;
    v0 = (T)((double)v0 * sc);
    v1 = (T)((double)v1 * sc);
    const auto vj = gp((T*)I.kv) + (int64_t)gp(I.ks)->j * 2 * I.nu;
    vj[2 * r] = v0;
    vj[2 * r + 1] = v1;
  }
  double y0 = (double)v0, y1 = (double)v1;
  blk_range_dot<true, T>(P, gp(I.kcol), gp(I.krow_ptr)[r], gp(I.kdiag)[r], z, y0, y1);
  z[2 * r] = (T)y0;
  z[2 * r + 1] = (T)y1;
}

// ILU(0) backward rows of one level: z_r = U(r,r)^{-1} (y_r - sum_{j>r}
// U(r,j) z_j), in place over y.
template <typename T>
__global__ __launch_bounds__(256) void k_ilu_bwd(const Inst* const* insts, const int2* __restrict__ work, int nwork,
                                                 int mode) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nwork) return;
  const int2 wk = ld_item(work, idx);
  const auto& I = *gp(gp(insts)[wk.x]);
  if (!kstate_is(I, apply_state(mode))) return;
  const int r = wk.y;
  const auto z = gp((T*)I.kz);
  const auto P = gp((const T*)I.pval);
  double s0 = (double)z[2 * r], s1 = (double)z[2 * r + 1];
  blk_range_dot<true, T>(P, gp(I.kcol), gp(I.kdiag)[r] + 1, gp(I.krow_ptr)[r + 1], z, s0, s1);
  const Blk<T> D = ld_blk((const T*)I.pdinv, r);
  z[2 * r] = (T)((double)D.a * s0 + (double)D.b * s1);
  z[2 * r + 1] = (T)((double)D.c * s0 + (double)D.d * s1);
}

// The whole ILU(0) factor of an instance in one work-group: the rows of
// each level as in k_ilu_rows, a barrier between levels.  Used when the
// instance's levels are short (one launch instead of one per level).
template <typename T>
__global__ __launch_bounds__(1024) void k_ilu_factor_wg(const Inst* const* insts) {
  const auto& I = *gp(insts[blockIdx.x]);
  if (!gp(I.red)->active || I.kwide) return;
  auto P = gp((T*)I.pval);
  auto D = gp((T*)I.pdinv);
  const auto kl_ptr = gp(I.kl_ptr), kcol = gp(I.kcol), kup_ptr = gp(I.kup_ptr), kup_t = gp(I.kup_t),
             kup_s = gp(I.kup_s);
  const auto kl_info = (const PF_AS1 i4v*)I.kl_info;
  bool bad = false;
  for (int l = 0; l < I.knl; ++l) {
    const int k1 = kl_ptr[l + 1];
    for (int k = kl_ptr[l] + (int)threadIdx.x; k < k1; k += 1024) {
      const i4v inf = kl_info[k];
      const int r = inf.x, qd = inf.z;
      // the next lower entry's column, update range and diagonal inverse
      // (read-only, or final from earlier levels) are fetched during this
      // entry's updates; its own block is read after them, as they may
      // change it
      if (inf.y < qd) {
        int u0 = kup_ptr[inf.y], u1 = kup_ptr[inf.y + 1];
        Blk<T> Dk = ld_blk<T>(D, kcol[inf.y]);
        for (int q = inf.y; q < qd; ++q) {
          const int qn = q + 1 < qd ? q + 1 : q;
          const int cn = kcol[qn], un = kup_ptr[qn + 1];
          const Blk<T> L = blk_mul(ld_blk<T>(P, q), Dk);
          st_blk(P, q, L);
          const Blk<T> Dn = ld_blk<T>(D, cn);
          ilu_updates<T>(P, kup_t, kup_s, u0, u1, L);
          u0 = u1;
          u1 = un;
          Dk = Dn;
        }
      }
      Blk<T> inv;
      if (!blk_inv(ld_blk<T>(P, qd), &inv)) {
        bad = true;
        inv.a = inv.b = inv.c = inv.d = T(0);
      }
      st_blk(D, r, inv);
    }
    __syncthreads();
  }
  if (bad) gp(I.red)->singular = 1;
}

namespace {

constexpr int LPM = 256;  // level pointers kept in LDS (z takes the rest)

// Data of one row of a sweep with its first two off-diagonal entries.
template <typename T>
struct SweepData {
  T w0, w1;  // forward: right-hand side; backward: unused
  Blk<T> E[2];
  int c[2];
  Blk<T> D;  // backward: the inverted diagonal block
};

// the row info {row, first, end, 0} at position k of a level list, or row -1
__device__ inline i4v sweep_info(const PF_AS1 i4v* info, int k, int k1) {
  if (k < k1) return info[k];
  i4v none;
  none.x = -1;
  none.y = 0;
  none.z = 0;
  none.w = 0;
  return none;
}

template <typename T>
__device__ inline void sweep_data(const i4v& inf, const PF_AS1 T* P, const PF_AS1 int* kcol, const PF_AS1 T* w,
                                  const PF_AS1 T* dinv, SweepData<T>* s) {
  if (inf.x < 0) return;
  if (w) {
    s->w0 = w[2 * inf.x];
    s->w1 = w[2 * inf.x + 1];
  }
  if (dinv) s->D = ld_blk<T>(dinv, inf.x);
#pragma unroll
  for (int e = 0; e < 2; ++e)
    if (inf.y + e < inf.z) {
      s->E[e] = ld_blk<T>(P, inf.y + e);
      s->c[e] = kcol[inf.y + e];
    }
}

}  // namespace

// The ILU(0) application z = U^{-1} L^{-1} (s w) of an instance in one
// work-group, level by level with a barrier between levels (rows as in
// k_ilu_fwd / k_ilu_bwd).  Each thread's first row of a level is fetched in
// two stages: its row info two levels ahead, its data one level ahead, so
// that each dependent load has a level's time to arrive.  ZV > 0: the
// work-group keeps z in LDS (instances with 2 nu <= ZV values) and writes it
// out at the end; ZV = 0: z lives in device memory.  Instances of the other
// sizes are skipped.
template <typename T, int ZV>
__global__ __launch_bounds__(1024) void k_ilu_apply_wg(const Inst* const* insts, int mode, int zmin) {
  __shared__ T zl[ZV > 0 ? ZV : 1];
  __shared__ int lpf[LPM + 1], lpb[LPM + 1];
  const auto& I = *gp(insts[blockIdx.x]);
  const auto ks = gp(I.ks);
  if (!gp(I.red)->active || I.kwide || ks->state != (apply_state(mode))) return;
  const int nu = I.nu;
  if (2 * nu <= zmin || (ZV > 0 && 2 * nu > ZV)) return;
  T* z = ZV > 0 ? zl : (T*)I.kz;
  const auto P = gp((const T*)I.pval);
  const auto Dinv = gp((const T*)I.pdinv);
  const auto kcol = gp(I.kcol);
  const auto w = gp((const T*)I.kw);
  const auto kl_info = (const PF_AS1 i4v*)I.kl_info, ku_info = (const PF_AS1 i4v*)I.ku_info;
  const auto kl_ptr = gp(I.kl_ptr), ku_ptr = gp(I.ku_ptr);
  const int tid = threadIdx.x;
  const int nl = I.knl, nul = I.knul;
  const bool lds_ptr = nl <= LPM && nul <= LPM;
  if (lds_ptr) {
    for (int i = tid; i <= nl; i += 1024) lpf[i] = kl_ptr[i];
    for (int i = tid; i <= nul; i += 1024) lpb[i] = ku_ptr[i];
  }
  const double sc = mode == 0 ? ks->scale : 1.0;
  const auto vj = gp((T*)I.kv + (int64_t)ks->j * 2 * nu);
  __syncthreads();
  auto fp = [&](int l) { return lds_ptr ? lpf[l] : kl_ptr[l]; };
  auto bp = [&](int l) { return lds_ptr ? lpb[l] : ku_ptr[l]; };

  // entries [q0, q1) of a row: (y0, y1) -= B(q) z(col(q)) in order of q, the
  // loads issued four at a time
  auto sub_entries = [&](int q0, int q1, double& y0, double& y1) {
    for (int q = q0; q < q1; q += 4) {
      Blk<T> B[4];
      int cq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q + u < q1) {
          B[u] = ld_blk<T>(P, q + u);
          cq[u] = kcol[q + u];
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q + u < q1) {
          const double a = (double)z[2 * cq[u]], b = (double)z[2 * cq[u] + 1];
          y0 -= (double)B[u].a * a + (double)B[u].b * b;
          y1 -= (double)B[u].c * a + (double)B[u].d * b;
        }
    }
  };
  // forward: y_r = s w_r - sum_{k<r} L(r,k) y_k
  auto fwd_row = [&](const i4v& inf, const SweepData<T>& s) {
    const int r = inf.x;
    T v0 = s.w0, v1 = s.w1;
    if (mode == 0) {
      v0 = (T)((double)v0 * sc);
      v1 = (T)((double)v1 * sc);
      vj[2 * r] = v0;
      vj[2 * r + 1] = v1;
    }
    double y0 = (double)v0, y1 = (double)v1;
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (inf.y + e < inf.z) {
        const double a = (double)z[2 * s.c[e]], b = (double)z[2 * s.c[e] + 1];
        y0 -= (double)s.E[e].a * a + (double)s.E[e].b * b;
        y1 -= (double)s.E[e].c * a + (double)s.E[e].d * b;
      }
    sub_entries(inf.y + 2, inf.z, y0, y1);
    z[2 * r] = (T)y0;
    z[2 * r + 1] = (T)y1;
  };
  // backward: z_r = U(r,r)^{-1} (y_r - sum_{j>r} U(r,j) z_j)
  auto bwd_row = [&](const i4v& inf, const SweepData<T>& s) {
    const int r = inf.x;
    double s0 = (double)z[2 * r], s1 = (double)z[2 * r + 1];
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (inf.y + e < inf.z) {
        const double a = (double)z[2 * s.c[e]], b = (double)z[2 * s.c[e] + 1];
        s0 -= (double)s.E[e].a * a + (double)s.E[e].b * b;
        s1 -= (double)s.E[e].c * a + (double)s.E[e].d * b;
      }
    sub_entries(inf.y + 2, inf.z, s0, s1);
    const Blk<T> Dv = s.D;
    z[2 * r] = (T)((double)Dv.a * s0 + (double)Dv.b * s1);
    z[2 * r + 1] = (T)((double)Dv.c * s0 + (double)Dv.d * s1);
  };
  // one sweep over the levels of a list with the two-stage fetch
  auto sweep = [&](const PF_AS1 i4v* info, auto ptr, int nlev, const PF_AS1 T* wsrc, const PF_AS1 T* dsrc,
                   auto row_fn) {
    if (nlev <= 0) return;
    i4v i0 = sweep_info(info, ptr(0) + tid, ptr(1));
    i4v i1 = nlev > 1 ? sweep_info(info, ptr(1) + tid, ptr(2)) : i0;
    SweepData<T> d0, d1;
    sweep_data<T>(i0, P, kcol, wsrc, dsrc, &d0);
    for (int l = 0; l < nlev; ++l) {
      const int k0 = ptr(l), k1 = ptr(l + 1);
      i4v i2 = i1;
      if (l + 2 < nlev) i2 = sweep_info(info, ptr(l + 2) + tid, ptr(l + 3));
      if (l + 1 < nlev) sweep_data<T>(i1, P, kcol, wsrc, dsrc, &d1);
      if (i0.x >= 0) row_fn(i0, d0);
      for (int k = k0 + tid + 1024; k < k1; k += 1024) {
        const i4v ix = info[k];
        SweepData<T> dx;
        sweep_data<T>(ix, P, kcol, wsrc, dsrc, &dx);
        row_fn(ix, dx);
      }
      __syncthreads();
      i0 = i1;
      d0 = d1;
      i1 = i2;
    }
  };
  const PF_AS1 T* none = nullptr;
  sweep(kl_info, fp, nl, w, none, fwd_row);
  sweep(ku_info, bp, nul, none, Dinv, bwd_row);
  if (ZV > 0) {
    const auto zg = gp((T*)I.kz);
    for (int i = tid; i < 2 * nu; i += 1024) zg[i] = zl[i];
  }
}

// Block-Jacobi application z_b = A_bb^{-1} (s w_b) (mode 0 also stores s w_b
// as basis vector v_j).  Row t of a group of order N is the sum over the
// columns in order.  The inverse is stored column-major, so a column is one
// coalesced load across the group's lanes; all NC columns are issued at
// once, right behind the input's load, so that they arrive during its round
// trip.  Columns past N repeat column N - 1 and rows past N repeat row N - 1,
// so every load stays inside the group's inverse; those columns meet a zero
// input and those rows store nothing.  vg: the group's NC inputs in LDS.
template <typename T, int NC, typename IR>
__device__ inline void bj_apply_rows(const IR& I, int b, int r0, int N, int t, bool valid, int mode, double sc,
                                     double* vg) {
  const int tr = t < N ? t : N - 1;
  const int r = gp(I.bj_rows)[r0 + (tr >> 1)];
  T x = gp((const T*)I.kw)[2 * r + (tr & 1)];
  const auto inv = gp((const T*)I.bjinv) + gp(I.bj_off)[b] + tr;
  T col[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) col[c] = inv[(int64_t)(c < N ? c : N - 1) * N];
  const bool mine = valid && t < N;
  if (mode == 0) {
    x = (T)((double)x * sc);
    if (mine) gp((T*)I.kv)[(int64_t)gp(I.ks)->j * 2 * I.nu + 2 * r + (t & 1)] = x;
  }
  vg[t] = mine ? (double)x : 0.0;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) s += (double)col[c] * vg[c];
  if (mine) gp((T*)I.kz)[2 * r + (t & 1)] = (T)s;
}

// One wave per work-group.  Work-groups below nbig take one group of more
// than kBjSmall nodes each (64 lanes); the others take four consecutive
// entries of the small groups' list, 16 lanes per group (N <= 16).  The host
// lays that list out in fours of one instance each, padded with entries of
// group -1, so the instance is the same across the wave.
template <typename T>
__global__ __launch_bounds__(64) void k_bj_apply(const Inst* const* insts, const int2* __restrict__ work, int nbig,
                                                 int mode) {
  __shared__ double v[64];
  const auto wp = (const PF_AS1 int*)work;
  const bool big = (int)blockIdx.x < nbig;
  const int k0 = big ? (int)blockIdx.x : nbig + 4 * ((int)blockIdx.x - nbig);
  const auto& I = *gp(gp(insts)[wp[2 * k0]]);
  if (!kstate_is(I, apply_state(mode))) return;
  const double sc = mode == 0 ? gp(I.ks)->scale : 1.0;
  if (big) {
    const int b = wp[2 * k0 + 1];
    const int r0 = gp(I.bj_ptr)[b];
    const int N = 2 * (gp(I.bj_ptr)[b + 1] - r0);
    bj_apply_rows<T, 64>(I, b, r0, N, (int)threadIdx.x, true, mode, sc, v);
  } else {
    const int g = threadIdx.x >> 4;
    const int bw = wp[2 * (k0 + g) + 1];
    const int b = bw < 0 ? 0 : bw;
    const int r0 = gp(I.bj_ptr)[b];
    const int N = 2 * (gp(I.bj_ptr)[b + 1] - r0);
    bj_apply_rows<T, 16>(I, b, r0, N, (int)threadIdx.x & 15, bw >= 0, mode, sc, v + 16 * g);
  }
}

// ---------------------------------------------------------------------------
// Arnoldi step

// w = J z for the rows of one chunk, then the partial dots <w, v_i>, i <= j.
template <typename T>
__global__ __launch_bounds__(KCH) void k_kspmv_dot(const Inst* const* insts) {
  __shared__ double red[KMAX + 1][KCH / 64];
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_ITER) || (int)blockIdx.x >= I.kchunks) return;
  const int j = gp(I.ks)->j;
  const int r = blockIdx.x * KCH + threadIdx.x;
  const int64_t n2 = 2 * (int64_t)I.nu;
  double w0 = 0.0, w1 = 0.0;
  if (r < I.nu) {
    const auto z = gp((const T*)I.kz);
    spmv_row<false, T>(I, r, z, w0, w1);
    const auto w = gp((T*)I.kw);
    w[2 * r] = (T)w0;
    w[2 * r + 1] = (T)w1;
    w0 = (double)(T)w0;
    w1 = (double)(T)w1;
  }
  const auto V = gp((const T*)I.kv);
  block_sums(
      j + 1,
      [&](int i) {
        if (r >= I.nu) return 0.0;
        const auto vi = V + i * n2;
        return w0 * (double)vi[2 * r] + w1 * (double)vi[2 * r + 1];
      },
      red, kpart(I, 0, blockIdx.x));
}

// One classical Gram-Schmidt pass: h = sum over chunks of the partial dots
// of pass p; w -= V h; column j of H gets h (p = 0) or h added (p = 1).
// Pass 0 leaves the partial dots of the re-orthogonalisation, pass 1 the
// partial squared norm of w.
template <typename T>
__global__ __launch_bounds__(KCH) void k_korth(const Inst* const* insts, int pass) {
  __shared__ double red[KMAX + 1][KCH / 64];
  __shared__ double h[KMAX + 1];
  __shared__ double hg[8][KMAX + 1];
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_ITER) || (int)blockIdx.x >= I.kchunks) return;
  const int j = gp(I.ks)->j;
  // h_i = sum over chunks of the pass's partial dots: 8 interleaved groups
  // of chunks (group g adds chunks g, g + 8, ... in turn, the loads of eight
  // of them issued together; past the last chunk a load repeats chunk 0 and
  // adds nothing), then the groups in order
  const int ni = j + 1, nc = I.kchunks;
  for (int idx = threadIdx.x; idx < 8 * ni; idx += KCH) {
    const int i = idx % ni, grp = idx / ni;
    double s = 0.0;
    for (int c0 = grp; c0 < nc; c0 += 64) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + 8 * u;
        v[u] = kpart(I, pass, c < nc ? c : 0)[i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += c0 + 8 * u < nc ? v[u] : 0.0;
    }
    hg[grp][i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += KCH) {
    double s = 0.0;
#pragma unroll
    for (int grp = 0; grp < 8; ++grp) s += hg[grp][i];
    h[i] = s;
    if (blockIdx.x == 0) {
      double* H = kh_H(I) + (int64_t)i * I.km + j;
      *H = pass == 0 ? s : *H + s;
    }
  }
  __syncthreads();
  const int r = blockIdx.x * KCH + threadIdx.x;
  const int64_t n2 = 2 * (int64_t)I.nu;
  const auto V = gp((const T*)I.kv);
  double w0 = 0.0, w1 = 0.0;
  if (r < I.nu) {
    const auto w = gp((T*)I.kw);
    w0 = (double)w[2 * r];
    w1 = (double)w[2 * r + 1];
    for (int i = 0; i <= j; ++i) {
      const auto vi = V + i * n2;
      w0 -= h[i] * (double)vi[2 * r];
      w1 -= h[i] * (double)vi[2 * r + 1];
    }
    w[2 * r] = (T)w0;
    w[2 * r + 1] = (T)w1;
    w0 = (double)(T)w0;
    w1 = (double)(T)w1;
  }
  if (pass == 0) {
    block_sums(
        j + 1,
        [&](int i) {
          if (r >= I.nu) return 0.0;
          const auto vi = V + i * n2;
          return w0 * (double)vi[2 * r] + w1 * (double)vi[2 * r + 1];
        },
        red, kpart(I, 1, blockIdx.x));
  } else {
    block_sums(
        1, [&](int) { return w0 * w0 + w1 * w1; }, red, kpart(I, 2, blockIdx.x));
  }
}

// Per instance: h_{j+1,j} = ||w||, the earlier rotations and a new one on
// column j of H, the residual estimate |g_{j+1}| / ||F||.  The cycle ends
// when the forcing term is met, the basis is full or w vanished; then
// y = H^{-1} g by back substitution.
// One wave per instance: the chunk partial sums are reduced across the
// lanes (fixed order), the Hessenberg column and the rotations are staged in
// LDS for lane 0's sequential part, and the back substitution runs row by
// row with a wave reduction.
__global__ __launch_bounds__(64) void k_karnoldi_end(const Inst* const* insts, KOpts o) {
  __shared__ double hc[KMAX + 1], scs[KMAX], ssn[KMAX], y[KMAX];
  __shared__ int fin;
  const auto& I = *gp(gp(insts)[blockIdx.x]);
  if (!kstate_is(I, KS_ITER)) return;
  KState& ks = *I.ks;
  const int lane = threadIdx.x;
  const int j = ks.j, m = I.km;
  const double h = sqrt(chunk_sum(I, 2, 0));
  double* H = kh_H(I);
  double* cs = kh_cs(I);
  double* sn = kh_sn(I);
  double* g = kh_g(I);
  for (int i = lane; i <= j; i += 64) {
    hc[i] = H[(int64_t)i * m + j];
    if (i < j) {
      scs[i] = cs[i];
      ssn[i] = sn[i];
    }
  }
  __syncthreads();
  if (lane == 0) {
    for (int i = 0; i < j; ++i) {
      const double a = hc[i], b = hc[i + 1];
      hc[i] = scs[i] * a + ssn[i] * b;
      hc[i + 1] = -ssn[i] * a + scs[i] * b;
    }
    const double hjj = hc[j];
    const double d = hypot(hjj, h);
    if (!isfinite(d) || !(d > 0.0)) {
      linear_failure(I);
      fin = -1;
    } else {
      cs[j] = hjj / d;
      sn[j] = h / d;
      hc[j] = d;
      H[(int64_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      const double rel = fabs(g[j + 1]) / ks.bnorm;
      ks.rel = rel;
      ks.j = j + 1;
      ks.total += 1;
      gp(I.red)->linear_iters += 1;
      fin = (rel <= ks.eta || j + 1 >= o.m || !(h > 0.0)) ? 1 : 0;
      if (fin) ks.met = rel <= ks.eta;
      else ks.scale = 1.0 / h;
    }
  }
  __syncthreads();
  if (fin < 0) return;
  for (int i = lane; i <= j; i += 64) H[(int64_t)i * m + j] = hc[i];
  if (fin == 0) return;
  // end of the cycle: y = H^{-1} g over the k = j + 1 columns (H upper)
  const int k = j + 1;
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    double p = 0.0;
    for (int c = i + 1 + lane; c < k; c += 64) p += H[(int64_t)i * m + c] * y[c];
    p = wave_sum(p);
    if (lane == 0) y[i] = (g[i] - p) / (i == j ? hc[j] : H[(int64_t)i * m + i]);
    __syncthreads();
  }
  double* yo = kh_y(I);
  for (int i = lane; i < k; i += 64) yo[i] = y[i];
  if (lane == 0) ks.state = KS_CYCLE;
}

// ---------------------------------------------------------------------------
// start, end of cycle, restart, result

// Start of the inner solve: w = F in Krylov order, x = 0, partial ||F||^2.
template <typename T>
__global__ __launch_bounds__(KCH) void k_kbegin(const Inst* const* insts) {
  __shared__ double red[KMAX + 1][KCH / 64];
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!gp(I.red)->active || (int)blockIdx.x >= I.kchunks) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  double f0 = 0.0, f1 = 0.0;
  if (r < I.nu) {
    const int p = gp(I.kp_of_r)[r];
    f0 = I.F[2 * p];
    f1 = I.F[2 * p + 1];
    const auto w = gp((T*)I.kw);
    const auto x = gp((T*)I.kx);
    w[2 * r] = (T)f0;
    w[2 * r + 1] = (T)f1;
    x[2 * r] = T(0);
    x[2 * r + 1] = T(0);
  }
  block_sums(
      1, [&](int) { return f0 * f0 + f1 * f1; }, red, kpart(I, 2, blockIdx.x));
}

// Per instance: ||F||_2, the forcing term eta = max(min(eta_max,
// ||F||_inf), eta_floor) and the first cycle.  A singular preconditioner
// ends the instance's Newton iteration with status singular.
__global__ __launch_bounds__(64) void k_kbegin_fin(const Inst* const* insts, KOpts o) {
  const auto& I = *gp(gp(insts)[blockIdx.x]);
  if (!gp(I.red)->active) return;
  KState& ks = *I.ks;
  if (gp(I.red)->singular) {
    if (threadIdx.x == 0) {
      gp(I.red)->status = 3;
      gp(I.red)->active = 0;
      ks.state = KS_DONE;
    }
    return;
  }
  const double bn = sqrt(chunk_sum(I, 2, 0));
  if (threadIdx.x != 0) return;
  ks.bnorm = bn;
  ks.eta = fmax(fmin(o.eta_max, gp(I.red)->last_norm), o.eta_floor);
  ks.j = 0;
  ks.cycle = 0;
  ks.met = 0;
  ks.total = 0;
  ks.rel = 1.0;
  kh_g(I)[0] = bn;
  if (bn > 0.0) {
    ks.scale = 1.0 / bn;
    ks.state = KS_ITER;
  } else {
    ks.rel = 0.0;
    ks.met = 1;
    ks.state = KS_FINISH;
  }
}

// u = V y over the basis of the finished cycle (into w).
template <typename T>
__global__ __launch_bounds__(KCH) void k_kycomb(const Inst* const* insts) {
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_CYCLE) || (int)blockIdx.x >= I.kchunks) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  if (r >= I.nu) return;
  const int k = gp(I.ks)->j;
  const double* y = kh_y(I);
  const int64_t n2 = 2 * (int64_t)I.nu;
  const auto V = gp((const T*)I.kv);
  double u0 = 0.0, u1 = 0.0;
  for (int i = 0; i < k; ++i) {
    u0 += y[i] * (double)V[i * n2 + 2 * r];
    u1 += y[i] * (double)V[i * n2 + 2 * r + 1];
  }
  const auto w = gp((T*)I.kw);
  w[2 * r] = (T)u0;
  w[2 * r + 1] = (T)u1;
}

// x += z (the preconditioned correction of the cycle).
template <typename T>
__global__ __launch_bounds__(KCH) void k_kxadd(const Inst* const* insts) {
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_CYCLE) || (int)blockIdx.x >= I.kchunks) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  if (r >= I.nu) return;
  const auto x = gp((T*)I.kx);
  const auto z = gp((const T*)I.kz);
  x[2 * r] = (T)((double)x[2 * r] + (double)z[2 * r]);
  x[2 * r + 1] = (T)((double)x[2 * r + 1] + (double)z[2 * r + 1]);
}

// Per instance, after a cycle: done when the forcing term is met; after the
// last allowed cycle the step is still taken when its relative residual is
// at most eta_max, else the Newton iteration ends with a linear failure;
// otherwise restart.
__global__ void k_kcycle_fin(const Inst* const* insts, int nslots, KOpts o) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslots) return;
  const auto& I = *gp(gp(insts)[sl]);
  if (!kstate_is(I, KS_CYCLE)) return;
  KState& ks = *I.ks;
  if (ks.met) {
    ks.state = KS_FINISH;
  } else if (ks.cycle >= o.max_restarts) {
    if (ks.rel <= o.eta_max)
      ks.state = KS_FINISH;
    else
      linear_failure(I);
  } else {
    ks.cycle += 1;
    ks.state = KS_RESTART;
  }
}

// Restart: w = F - J x for the rows of one chunk, partial ||w||^2.
template <typename T>
__global__ __launch_bounds__(KCH) void k_kresid(const Inst* const* insts) {
  __shared__ double red[KMAX + 1][KCH / 64];
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_RESTART) || (int)blockIdx.x >= I.kchunks) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  double w0 = 0.0, w1 = 0.0;
  if (r < I.nu) {
    const int p = gp(I.kp_of_r)[r];
    w0 = I.F[2 * p];
    w1 = I.F[2 * p + 1];
    const auto x = gp((const T*)I.kx);
    spmv_row<true, T>(I, r, x, w0, w1);
    const auto w = gp((T*)I.kw);
    w[2 * r] = (T)w0;
    w[2 * r + 1] = (T)w1;
    w0 = (double)(T)w0;
    w1 = (double)(T)w1;
  }
  block_sums(
      1, [&](int) { return w0 * w0 + w1 * w1; }, red, kpart(I, 2, blockIdx.x));
}

// Per instance: the true residual starts the next cycle, or ends the solve
// when it already meets the forcing term.
__global__ __launch_bounds__(64) void k_krestart_fin(const Inst* const* insts) {
  const auto& I = *gp(gp(insts)[blockIdx.x]);
  if (!kstate_is(I, KS_RESTART)) return;
  KState& ks = *I.ks;
  const double beta = sqrt(chunk_sum(I, 2, 0));
  if (threadIdx.x != 0) return;
  ks.rel = beta / ks.bnorm;
  if (ks.rel <= ks.eta || !(beta > 0.0)) {
    ks.met = 1;
    ks.state = KS_FINISH;
    return;
  }
  kh_g(I)[0] = beta;
  ks.j = 0;
  ks.scale = 1.0 / beta;
  ks.state = KS_ITER;
}

// The Newton step in the factor layout that the voltage update reads.
template <typename T>
__global__ __launch_bounds__(KCH) void k_kfinish(const Inst* const* insts) {
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_FINISH) || (int)blockIdx.x >= I.kchunks) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  if (r >= I.nu) return;
  const int p = gp(I.kp_of_r)[r];
  const auto x = gp((const T*)I.kx);
  const auto out = gp((T*)I.x);
  out[2 * p] = x[2 * r];
  out[2 * p + 1] = x[2 * r + 1];
}

// ---------------------------------------------------------------------------
// BiCGStab (van der Vorst), the Krylov method the paper tested (Sec. III-B),
// right-preconditioned, from x = 0 with the shadow residual r0 = F.  Vectors
// in the basis storage: r (0; s overwrites it), r0 (1), p (2), v (3),
// p^ = M^-1 p (4), s^ = M^-1 s (5), t (6).  The first direction p = r =
// r0 = F goes into w at the start; then one iteration is the launch
// sequence
//   KS_BP: z = M^-1 w; p^ = z, v = J p^ with partial <r0, v>;
//          alpha = <r0, r> / <r0, v>, s = r - alpha v into w with partial
//          ||s||^2; z = M^-1 w; the first half meets the tolerance
//          (-> KS_BH) or not (-> KS_BS), and in KS_BS s^ = z, t = J s^ with
//          partial <t, s>, <t, t>
//   KS_BS: omega = <t, s> / <t, t>, x += alpha p^ + omega s^,
//          r = s - omega t with partial <r0, r>, ||r||^2; the convergence
//          test, beta and the next direction p = r + beta (p - omega v)
//          into w (-> KS_BP)
//   KS_BH: x += alpha p^, done.
// The tests run in every work-group of the launch that follows the partial
// sums they need (the same sums in the same order everywhere), the first
// work-group setting the state; seven launches per iteration.
// A zero <r0, r>, <r0, v>, <t, t> or omega, or the iteration limit, ends the
// solve with x as it stands: the step is taken when its relative residual
// is at most eta_max, else the Newton iteration ends with a linear failure.

template <typename T, typename IR>
__device__ inline PF_AS1 T* kvec(const IR& I, int i) {
  return gp((T*)I.kv) + (int64_t)i * 2 * I.nu;
}


// The solve ends as it stands.
template <typename IR>
__device__ inline void bcg_stop(const IR& I, KOpts o) {
  if (gp(I.ks)->rel <= o.eta_max)
    gp(I.ks)->state = KS_FINISH;
  else
    linear_failure(I);
}

// Per instance, after k_kbegin (w = F, x = 0, partial ||F||^2): ||F||_2,
// the forcing term, <r0, r> = ||F||^2 and the first iteration.
__global__ __launch_bounds__(64) void k_bcg_begin_fin(const Inst* const* insts, KOpts o) {
  const auto& I = *gp(gp(insts)[blockIdx.x]);
  if (!gp(I.red)->active) return;
  KState& ks = *I.ks;
  if (gp(I.red)->singular) {
    if (threadIdx.x == 0) {
      gp(I.red)->status = 3;
      gp(I.red)->active = 0;
      ks.state = KS_DONE;
    }
    return;
  }
  const double b2 = chunk_sum(I, 2, 0);
  if (threadIdx.x != 0) return;
  const double bn = sqrt(b2);
  ks.bnorm = bn;
  ks.eta = fmax(fmin(o.eta_max, gp(I.red)->last_norm), o.eta_floor);
  ks.j = 0;
  ks.cycle = 0;
  ks.met = 0;
  ks.total = 0;
  ks.rel = 1.0;
  ks.rho[0] = b2;
  ks.alpha = ks.omega = 1.0;
  ks.beta = 0.0;
  if (bn > 0.0) {
    ks.state = KS_BP;
  } else {
    ks.rel = 0.0;
    ks.met = 1;
    ks.state = KS_FINISH;
  }
}

// p = r + beta (p - omega v), or r = r0 = p = F in the first iteration; w = p.
template <typename T>
__global__ __launch_bounds__(KCH) void k_bcg_dir(const Inst* const* insts) {
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_BP) || (int)blockIdx.x >= I.kchunks) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  if (r >= I.nu) return;
  const auto& ks = *gp(I.ks);
  const auto w = gp((T*)I.kw);
  const auto R = kvec<T>(I, 0);
  const auto P = kvec<T>(I, 2);
  const auto V = kvec<T>(I, 3);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = 2 * r + e;
    T p;
    if (ks.j == 0) {
      p = w[i];
      R[i] = p;
      kvec<T>(I, 1)[i] = p;
    } else {
      p = (T)((double)R[i] + ks.beta * ((double)P[i] - ks.omega * (double)V[i]));
    }
    P[i] = p;
    w[i] = p;
  }
}

// p^ = z, v = J p^ for the rows of one chunk, partial <r0, v>.
template <typename T>
__global__ __launch_bounds__(KCH) void k_bcg_v(const Inst* const* insts) {
  __shared__ double red[KMAX + 1][KCH / 64];
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_BP) || (int)blockIdx.x >= I.kchunks) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  double d = 0.0;
  if (r < I.nu) {
    const auto z = gp((const T*)I.kz);
    const auto Ph = kvec<T>(I, 4);
    Ph[2 * r] = z[2 * r];
    Ph[2 * r + 1] = z[2 * r + 1];
    double v0 = 0.0, v1 = 0.0;
    spmv_row<false, T>(I, r, z, v0, v1);
    const auto V = kvec<T>(I, 3);
    V[2 * r] = (T)v0;
    V[2 * r + 1] = (T)v1;
    const auto R0 = kvec<T>(I, 1);
    d = (double)R0[2 * r] * (double)(T)v0 + (double)R0[2 * r + 1] * (double)(T)v1;
  }
  block_sums(
      1, [&](int) { return d; }, red, kpart(I, 0, blockIdx.x));
}

// alpha = <r0, r> / <r0, v>; s = r - alpha v into r and w; partial ||s||^2
// (it: the iteration, counted from 0 in the inner solve).
template <typename T>
__global__ __launch_bounds__(KCH) void k_bcg_s(const Inst* const* insts, int it) {
  __shared__ double red[KMAX + 1][KCH / 64];
  __shared__ double alpha_s;
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (!kstate_is(I, KS_BP) || (int)blockIdx.x >= I.kchunks) return;
  if (threadIdx.x < 64) {
    const double a = gp(I.ks)->rho[it & 1] / chunk_sum(I, 0, 0);
    if (threadIdx.x == 0) {
      alpha_s = a;
      if (blockIdx.x == 0) gp(I.ks)->alpha = a;
    }
  }
  __syncthreads();
  const double alpha = alpha_s;
  const int r = blockIdx.x * KCH + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (r < I.nu) {
    const auto R = kvec<T>(I, 0);
    const auto V = kvec<T>(I, 3);
    const auto w = gp((T*)I.kw);
    const T a = (T)((double)R[2 * r] - alpha * (double)V[2 * r]);
    const T b = (T)((double)R[2 * r + 1] - alpha * (double)V[2 * r + 1]);
    R[2 * r] = a;
    R[2 * r + 1] = b;
    w[2 * r] = a;
    w[2 * r + 1] = b;
    s0 = (double)a;
    s1 = (double)b;
  }
  block_sums(
      1, [&](int) { return s0 * s0 + s1 * s1; }, red, kpart(I, 1, blockIdx.x));
}

// The first half of the iteration, decided in every work-group from the
// chunk partials (the same sums in the same order, so every work-group
// decides alike): a zero <r0, v> or a non-finite alpha ends the solve as it
// stands, a small enough ||s|| takes x += alpha p^ only (KS_BH); otherwise
// (KS_BS) s^ = z, t = J s^ for the rows of one chunk, partial <t, s>,
// <t, t>.  The first work-group counts the iteration and sets the state;
// the others accept the state it sets as the one they started from.
template <typename T>
__global__ __launch_bounds__(KCH) void k_bcg_t(const Inst* const* insts, KOpts o) {
  __shared__ double red[KMAX + 1][KCH / 64];
  __shared__ int decision;  // 0 second half, 1 first half met, 2 breakdown
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if ((!kstate_is(I, KS_BP) && !kstate_is(I, KS_BS)) || (int)blockIdx.x >= I.kchunks) return;
  auto& ks = *gp(I.ks);
  if (threadIdx.x < 64) {
    double sum[2];
    chunk_sums<2, 1>(I, {0, 1}, {0, 0}, sum);
    const double sv = sum[0], ss = sum[1];
    if (threadIdx.x == 0) {
      const double srel = sqrt(ss) / ks.bnorm;
      const int dec = (!(sv > 0.0) || !isfinite(ks.alpha)) ? 2 : srel <= ks.eta ? 1 : 0;
      decision = dec;
      if (blockIdx.x == 0) {
        ks.total += 1;
        gp(I.red)->linear_iters += 1;
        if (dec == 2) {
          bcg_stop(I, o);
        } else if (dec == 1) {
          ks.rel = srel;
          ks.met = 1;
          ks.state = KS_BH;
        } else {
          ks.state = KS_BS;
        }
      }
    }
  }
  __syncthreads();
  if (decision != 0) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  double ts = 0.0, tt = 0.0;
  if (r < I.nu) {
    const auto z = gp((const T*)I.kz);
    const auto Sh = kvec<T>(I, 5);
    Sh[2 * r] = z[2 * r];
    Sh[2 * r + 1] = z[2 * r + 1];
    double t0 = 0.0, t1 = 0.0;
    spmv_row<false, T>(I, r, z, t0, t1);
    const auto Tv = kvec<T>(I, 6);
    Tv[2 * r] = (T)t0;
    Tv[2 * r + 1] = (T)t1;
    t0 = (double)(T)t0;
    t1 = (double)(T)t1;
    const auto S = kvec<T>(I, 0);
    ts = t0 * (double)S[2 * r] + t1 * (double)S[2 * r + 1];
    tt = t0 * t0 + t1 * t1;
  }
  block_sums(
      2, [&](int e) { return e == 0 ? ts : tt; }, red, kpart(I, 2, blockIdx.x));
}

// KS_BS: omega = <t, s> / <t, t>, x += alpha p^ + omega s^, r = s - omega t,
// partial <r0, r> and ||r||^2 (nothing when <t, t> = 0).  KS_BH:
// x += alpha p^.
template <typename T>
__global__ __launch_bounds__(KCH) void k_bcg_x(const Inst* const* insts) {
  __shared__ double red[KMAX + 1][KCH / 64];
  __shared__ double omega_s;
  __shared__ bool skip_s;
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  const bool half = kstate_is(I, KS_BH);
  if ((!half && !kstate_is(I, KS_BS)) || (int)blockIdx.x >= I.kchunks) return;
  const auto& ks = *gp(I.ks);
  const int r = blockIdx.x * KCH + threadIdx.x;
  const auto x = gp((T*)I.kx);
  const auto Ph = kvec<T>(I, 4);
  if (half) {
    if (r < I.nu) {
#pragma unroll
      for (int e = 0; e < 2; ++e) x[2 * r + e] = (T)((double)x[2 * r + e] + ks.alpha * (double)Ph[2 * r + e]);
    }
    return;
  }
  if (threadIdx.x < 64) {
    double sum[2];
    chunk_sums<2>(I, {2, 2}, {1, 0}, sum);
    const double tt = sum[0], ts = sum[1];
    if (threadIdx.x == 0) {
      skip_s = !(tt > 0.0);
      omega_s = skip_s ? 0.0 : ts / tt;
      if (blockIdx.x == 0) gp(I.ks)->omega = omega_s;
    }
  }
  __syncthreads();
  if (skip_s) return;  // <t, t> = 0: the solve ends as it stands
  const double omega = omega_s;
  double d = 0.0, q = 0.0;
  if (r < I.nu) {
    const auto Sh = kvec<T>(I, 5);
    const auto Tv = kvec<T>(I, 6);
    const auto R0 = kvec<T>(I, 1);
    const auto R = kvec<T>(I, 0);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = 2 * r + e;
      x[i] = (T)((double)x[i] + ks.alpha * (double)Ph[i] + omega * (double)Sh[i]);
      const T rn = (T)((double)R[i] - omega * (double)Tv[i]);
      R[i] = rn;
      d += (double)R0[i] * (double)rn;
      q += (double)rn * (double)rn;
    }
  }
  block_sums(
      2, [&](int e) { return e == 0 ? d : q; }, red, kpart(I, 1, blockIdx.x));
}

// The end of iteration it, decided in every work-group from the chunk
// partials (alike everywhere): the first half met ends the solve
// (KS_FINISH); a zero <t, t> ends it as it stands; then the convergence
// test; then, unless omega or <r0, r> is zero, the iteration limit is
// reached or the residual is not finite, beta = (rho' / rho)(alpha / omega)
// and the next direction p = r + beta (p - omega v) into p and w for the
// rows of one chunk.  The first work-group sets the instance's scalars and
// state (<r0, r> goes to the other parity, so no work-group reads a value
// this launch writes); the others accept the state it sets.
template <typename T>
__global__ __launch_bounds__(KCH) void k_bcg_next(const Inst* const* insts, KOpts o, int it) {
  __shared__ double beta_s;
  __shared__ int go;
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  const bool half = kstate_is(I, KS_BH);
  if ((!half && !kstate_is(I, KS_BS) && !kstate_is(I, KS_BP)) || (int)blockIdx.x >= I.kchunks) return;
  auto& ks = *gp(I.ks);
  if (threadIdx.x < 64) {
    double sum[3];
    chunk_sums<3>(I, {2, 1, 1}, {1, 0, 1}, sum);
    const double tt = sum[0], rho = sum[1], rr = sum[2];
    if (threadIdx.x == 0) {
      const double rel = sqrt(rr) / ks.bnorm;
      const int max_it = max(1, (1 + o.max_restarts) * o.m / 2);
      // 0 finish, 1 stop as it stands (the relative residual set first or
      // not), 2 go on
      int dec;
      bool set_rel = false;
      if (half) {
        dec = 0;
      } else if (!(tt > 0.0)) {
        dec = 1;
      } else if (rel <= ks.eta) {
        dec = 0;
        set_rel = true;
      } else if (ks.omega == 0.0 || rho == 0.0 || it + 1 >= max_it || !isfinite(rel)) {
        dec = 1;
        set_rel = true;
      } else {
        dec = 2;
        set_rel = true;
      }
      const double beta = (rho / ks.rho[it & 1]) * (ks.alpha / ks.omega);
      go = dec == 2;
      beta_s = beta;
      if (blockIdx.x == 0) {
        if (set_rel) ks.rel = rel;
        if (set_rel && dec != 0) ks.j = it + 1;
        if (dec == 0) {
          if (!half) ks.met = 1;
          ks.state = KS_FINISH;
        } else if (dec == 1) {
          bcg_stop(I, o);
        } else {
          ks.beta = beta;
          ks.rho[(it + 1) & 1] = rho;
          ks.state = KS_BP;
        }
      }
    }
  }
  __syncthreads();
  if (!go) return;
  const int r = blockIdx.x * KCH + threadIdx.x;
  if (r >= I.nu) return;
  const double beta = beta_s, omega = ks.omega;
  const auto w = gp((T*)I.kw);
  const auto R = kvec<T>(I, 0);
  const auto P = kvec<T>(I, 2);
  const auto V = kvec<T>(I, 3);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = 2 * r + e;
    const T p = (T)((double)R[i] + beta * ((double)P[i] - omega * (double)V[i]));
    P[i] = p;
    w[i] = p;
  }
}

// Per instance: a written result retires the solve (KS_FINISH -> KS_DONE).
__global__ void k_kretire(const Inst* const* insts, int nslots) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslots) return;
  const auto& I = *gp(gp(insts)[sl]);
  if (kstate_is(I, KS_FINISH)) gp(I.ks)->state = KS_DONE;
}

// Krylov state of every instance for the host (KS_DONE once the Newton
// iteration of the instance has ended) in out[0, nslots), and the steps or
// iterations of its current inner solve in out[nslots, 2 nslots).
__global__ void k_kgather(const Inst* const* insts, int nslots, int* out) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslots) return;
  const auto& I = *gp(gp(insts)[sl]);
  out[sl] = gp(I.red)->active ? gp(I.ks)->state : KS_DONE;
  out[nslots + sl] = gp(I.ks)->total;
}

// ---------------------------------------------------------------------------
// host launchers

static inline dim3 chunk_grid(int max_chunks, int nslots) {
  return dim3((unsigned)(max_chunks > 0 ? max_chunks : 1), (unsigned)nslots);
}
static inline dim3 slot_grid(int nslots) { return dim3((unsigned)((nslots + 63) / 64)); }
static inline dim3 item_grid(int nwork) { return dim3((unsigned)((nwork + 255) / 256)); }

template <typename T>
void launch_ilu_rows(hipStream_t st, const Inst* const* insts, const int2* work, int nwork) {
  if (nwork > 0) k_ilu_rows<T><<<item_grid(nwork), 256, 0, st>>>(insts, work, nwork);
}
template <typename T>
void launch_bj_inv(hipStream_t st, const Inst* const* insts, const int2* work, int nbig, int nsmall) {
  if (nbig > 0) k_bj_inv_mfma<T><<<dim3((unsigned)nbig), 256, 0, st>>>(insts, work);
  if (nsmall > 0) k_bj_inv_small<T><<<dim3((unsigned)((nsmall + 3) / 4)), 256, 0, st>>>(insts, work + nbig, nsmall);
  if (nbig + nsmall > 0) k_bj_inv<T><<<dim3((unsigned)(nbig + nsmall)), 256, 0, st>>>(insts, work);
}
int bj_small_nodes() { return kBjSmall; }
template <typename T>
void launch_ilu_fwd(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int mode) {
  if (nwork > 0) k_ilu_fwd<T><<<item_grid(nwork), 256, 0, st>>>(insts, work, nwork, mode);
}
template <typename T>
void launch_ilu_bwd(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int mode) {
  if (nwork > 0) k_ilu_bwd<T><<<item_grid(nwork), 256, 0, st>>>(insts, work, nwork, mode);
}
template <typename T>
void launch_ilu_factor_wg(hipStream_t st, const Inst* const* insts, int nslots) {
  k_ilu_factor_wg<T><<<dim3((unsigned)nslots), 1024, 0, st>>>(insts);
}
// z in LDS up to 160,000 bytes of values per work-group, in two sizes so that
// small instances keep several work-groups per CU
template <typename T>
void launch_ilu_apply_wg(hipStream_t st, const Inst* const* insts, int nslots, int mode, int min_nu, int max_nu) {
  constexpr int small = 8192 / sizeof(T) * 4;   // 32 KiB
  constexpr int big = 160000 / sizeof(T);
  const dim3 g((unsigned)nslots);
  // only the size classes some instance of the batch falls in
  if (2 * min_nu <= small) k_ilu_apply_wg<T, small><<<g, 1024, 0, st>>>(insts, mode, 0);
  if (2 * max_nu > small && 2 * min_nu <= big) k_ilu_apply_wg<T, big><<<g, 1024, 0, st>>>(insts, mode, small);
  if (2 * max_nu > big) k_ilu_apply_wg<T, 0><<<g, 1024, 0, st>>>(insts, mode, big);
}
template <typename T>
void launch_bj_apply(hipStream_t st, const Inst* const* insts, const int2* work, int nbig, int nwork, int mode) {
  if (nwork > 0) k_bj_apply<T><<<dim3((unsigned)(nbig + (nwork - nbig) / 4)), 64, 0, st>>>(insts, work, nbig, mode);
}
template <typename T>
void launch_karnoldi(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks, KOpts o) {
  const dim3 g = chunk_grid(max_chunks, nslots);
  k_kspmv_dot<T><<<g, KCH, 0, st>>>(insts);
  k_korth<T><<<g, KCH, 0, st>>>(insts, 0);
  k_korth<T><<<g, KCH, 0, st>>>(insts, 1);
  k_karnoldi_end<<<dim3((unsigned)nslots), 64, 0, st>>>(insts, o);
}
template <typename T>
void launch_kbegin(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks, KOpts o) {
  k_kbegin<T><<<chunk_grid(max_chunks, nslots), KCH, 0, st>>>(insts);
  k_kbegin_fin<<<dim3((unsigned)nslots), 64, 0, st>>>(insts, o);
}
template <typename T>
void launch_kycomb(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks) {
  k_kycomb<T><<<chunk_grid(max_chunks, nslots), KCH, 0, st>>>(insts);
}
template <typename T>
void launch_kcycle_end(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks, KOpts o) {
  const dim3 g = chunk_grid(max_chunks, nslots);
  k_kxadd<T><<<g, KCH, 0, st>>>(insts);
  k_kcycle_fin<<<slot_grid(nslots), 64, 0, st>>>(insts, nslots, o);
  k_kresid<T><<<g, KCH, 0, st>>>(insts);
  k_krestart_fin<<<dim3((unsigned)nslots), 64, 0, st>>>(insts);
}
template <typename T>
void launch_kfinish(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks) {
  k_kfinish<T><<<chunk_grid(max_chunks, nslots), KCH, 0, st>>>(insts);
  k_kretire<<<slot_grid(nslots), 64, 0, st>>>(insts, nslots);
}
template <typename T>
void launch_bcg_begin(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks, KOpts o) {
  k_kbegin<T><<<chunk_grid(max_chunks, nslots), KCH, 0, st>>>(insts);
  k_bcg_begin_fin<<<dim3((unsigned)nslots), 64, 0, st>>>(insts, o);
}
template <typename T>
void launch_bcg_dir(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks) {
  k_bcg_dir<T><<<chunk_grid(max_chunks, nslots), KCH, 0, st>>>(insts);
}
template <typename T>
void launch_bcg_half(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks, int it) {
  const dim3 g = chunk_grid(max_chunks, nslots);
  k_bcg_v<T><<<g, KCH, 0, st>>>(insts);
  k_bcg_s<T><<<g, KCH, 0, st>>>(insts, it);
}
template <typename T>
void launch_bcg_end(hipStream_t st, const Inst* const* insts, int nslots, int max_chunks, KOpts o, int it) {
  const dim3 g = chunk_grid(max_chunks, nslots);
  k_bcg_t<T><<<g, KCH, 0, st>>>(insts, o);
  k_bcg_x<T><<<g, KCH, 0, st>>>(insts);
  k_bcg_next<T><<<g, KCH, 0, st>>>(insts, o, it);
}
void launch_kgather(hipStream_t st, const Inst* const* insts, int nslots, int* out) {
  k_kgather<<<slot_grid(nslots), 64, 0, st>>>(insts, nslots, out);
}
int krylov_max_restart() { return KMAX; }

#define PF_KINST(T)                                                                    \
  template void launch_ilu_rows<T>(hipStream_t, const Inst* const*, const int2*, int);      \
  template void launch_bj_inv<T>(hipStream_t, const Inst* const*, const int2*, int, int);   \
  template void launch_ilu_fwd<T>(hipStream_t, const Inst* const*, const int2*, int, int);  \
  template void launch_ilu_bwd<T>(hipStream_t, const Inst* const*, const int2*, int, int);  \
  template void launch_bj_apply<T>(hipStream_t, const Inst* const*, const int2*, int, int, int);\
  template void launch_ilu_factor_wg<T>(hipStream_t, const Inst* const*, int);              \
  template void launch_ilu_apply_wg<T>(hipStream_t, const Inst* const*, int, int, int, int);\
  template void launch_karnoldi<T>(hipStream_t, const Inst* const*, int, int, KOpts);       \
  template void launch_kbegin<T>(hipStream_t, const Inst* const*, int, int, KOpts);         \
  template void launch_kycomb<T>(hipStream_t, const Inst* const*, int, int);                \
  template void launch_kcycle_end<T>(hipStream_t, const Inst* const*, int, int, KOpts);     \
  template void launch_kfinish<T>(hipStream_t, const Inst* const*, int, int);                  \
  template void launch_bcg_begin<T>(hipStream_t, const Inst* const*, int, int, KOpts);        \
  template void launch_bcg_dir<T>(hipStream_t, const Inst* const*, int, int);                 \
  template void launch_bcg_half<T>(hipStream_t, const Inst* const*, int, int, int);           \
  template void launch_bcg_end<T>(hipStream_t, const Inst* const*, int, int, KOpts, int);

PF_KINST(double)
PF_KINST(float)

}  // namespace pfd
