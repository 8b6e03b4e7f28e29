// HIP kernels of the Newton power-flow iteration for gfx950 (wave64).
//
// Per Newton step (Sec. II-A and II-B iteration tables, Sec. III-A solve):
//   mismatch (FP64) -> Jacobian fill into LU storage -> sparse block
//   refactorisation by elimination-tree levels -> forward solve -> Schur
//   update of the dense trailing block -> dense LU of that block with the
//   right-hand side appended -> dense backward solve -> sparse backward
//   solve -> voltage update (FP64).
// Value type T of the factor and the inner solves is double (plain) or float
// (mixed precision); the mismatch, the update and the convergence test are
// always double.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "kernels.hpp"

namespace pfd {

// ---------------------------------------------------------------------------
// helpers

__device__ inline void atomic_max_nonneg(unsigned long long* slot, double v) {
  // |x| and NaN (positive quiet NaN bits) both order correctly as integers
  atomicMax(slot, (unsigned long long)__double_as_longlong(v));
}

template <typename T>
struct Blk {
  T a, b, c, d;  // [[a b] [c d]]
};

template <typename T>
__device__ inline Blk<T> ld_blk(const T* p, int64_t id) {
  const T* q = p + 4 * id;
  Blk<T> r;
  r.a = q[0];
  r.b = q[1];
  r.c = q[2];
  r.d = q[3];
  return r;
}

template <typename T>
__device__ inline void st_blk(T* p, int64_t id, const Blk<T>& v) {
  T* q = p + 4 * id;
  q[0] = v.a;
  q[1] = v.b;
  q[2] = v.c;
  q[3] = v.d;
}

// acc -= X * Y
template <typename T>
__device__ inline void blk_msub(Blk<T>& acc, const Blk<T>& X, const Blk<T>& Y) {
  acc.a -= X.a * Y.a + X.b * Y.c;
  acc.b -= X.a * Y.b + X.b * Y.d;
  acc.c -= X.c * Y.a + X.d * Y.c;
  acc.d -= X.c * Y.b + X.d * Y.d;
}

template <typename T>
__device__ inline Blk<T> blk_mul(const Blk<T>& X, const Blk<T>& Y) {
  Blk<T> r;
  r.a = X.a * Y.a + X.b * Y.c;
  r.b = X.a * Y.b + X.b * Y.d;
  r.c = X.c * Y.a + X.d * Y.c;
  r.d = X.c * Y.b + X.d * Y.d;
  return r;
}

// ---------------------------------------------------------------------------
// state initialisation and update

// Polar flat start: |V| = 1 on PQ buses, set-point elsewhere; angle 0 but the
// slack's set-point.  Also writes the rectangular voltage v[2i], v[2i+1].
__global__ void k_init_polar(int n, const int8_t* __restrict__ type, const double* __restrict__ vmag,
                             const double* __restrict__ vang, double* vm, double* va, double* v,
                             int flat) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m, a;
  if (flat) {
    m = type[i] == 1 ? 1.0 : vmag[i];
    a = type[i] == 3 ? vang[i] : 0.0;
    vm[i] = m;
    va[i] = a;
  } else {
    m = vm[i];
    a = va[i];
  }
  double s, c;
  sincos(a, &s, &c);
  v[2 * i] = m * c;
  v[2 * i + 1] = m * s;
}

// CIM flat start: |V| = 1 (source magnitude on source nodes) at the node's
// nominal phase angle.
__global__ void k_init_cim(int n, const int8_t* __restrict__ type, const double* __restrict__ vmag,
                           const double* __restrict__ vang, double* v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m = type[i] == 3 ? vmag[i] : 1.0;
  double s, c;
  sincos(vang[i], &s, &c);
  v[2 * i] = m * c;
  v[2 * i + 1] = m * s;
}

__global__ void k_reset_red(Red* r) {
  if (threadIdx.x == 0) {
    r->norm_bits = 0ull;
    r->step_bits = 0ull;
    r->singular = 0;
  }
}

// ---------------------------------------------------------------------------
// mismatch (FP64)

// Polar: I = Y V (eq. 1), S = V conj(I) (eq. 5 conjugated), dP = P_sp - Re S
// for non-slack buses, dQ = Q_sp - Im S for PQ buses (eq. 8-9).  F is written
// at the bus's LU position (2 rows per node); the |V| row of a PV bus is 0.
__global__ void k_mismatch_polar(int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
                                 const double2* __restrict__ y, const double2* __restrict__ v,
                                 const int8_t* __restrict__ type, const double* __restrict__ psp,
                                 const double* __restrict__ qsp, const int* __restrict__ pos,
                                 double2* ibus, double* F, Red* red) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double local = 0.0;
  if (i < n) {
    double ir = 0.0, ii = 0.0;
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      double2 yy = y[q];
      double2 vv = v[col[q]];
      ir += yy.x * vv.x - yy.y * vv.y;
      ii += yy.x * vv.y + yy.y * vv.x;
    }
    ibus[i] = make_double2(ir, ii);
    int p = pos[i];
    if (p >= 0) {
      double2 vi = v[i];
      double sr = vi.x * ir + vi.y * ii;  // Re(V conj I)
      double si = vi.y * ir - vi.x * ii;  // Im(V conj I)
      double dp = psp[i] - sr;
      double dq = type[i] == 1 ? qsp[i] - si : 0.0;
      F[2 * p] = dp;
      F[2 * p + 1] = dq;
      local = fmax(fabs(dp), fabs(dq));
      if (!(dp == dp) || !(dq == dq)) local = __longlong_as_double(0x7ff8000000000000ll);
    }
  }
  // wave max then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(local, off, 64);
    local = (o > local || o != o) ? o : local;
  }
  if ((threadIdx.x & 63) == 0 && local != 0.0) atomic_max_nonneg(&red->norm_bits, local);
}

// CIM: I_calc = sum_j Y_ij V_j (eq. 18); P_l, Q_l from the ZIP model (eq.
// 14-15); P_sp = P_g - P_l (eq. 12-13); I_sp = conj((P_sp + jQ_sp)/V)
// (eq. 17); dI = I_sp - I_calc (eq. 16).  Rows per node: [Im dI, Re dI]
// (eq. 19 order within the node).
__global__ void k_mismatch_cim(int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
                               const double2* __restrict__ y, const double2* __restrict__ v,
                               const double* __restrict__ pg, const double* __restrict__ qg,
                               const double* __restrict__ zip, const int* __restrict__ pos, double* F,
                               Red* red) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double local = 0.0;
  if (i < n) {
    int p = pos[i];
    if (p >= 0) {
      double ir = 0.0, ii = 0.0;
      for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
        double2 yy = y[q];
        double2 vv = v[col[q]];
        ir += yy.x * vv.x - yy.y * vv.y;
        ii += yy.x * vv.y + yy.y * vv.x;
      }
      double2 vi = v[i];
      double w = vi.x * vi.x + vi.y * vi.y;
      double vm = sqrt(w);
      const double* z = zip + 6 * i;
      double pl = z[2] + z[1] * vm + z[0] * w;
      double ql = z[5] + z[4] * vm + z[3] * w;
      double ps = pg[i] - pl, qs = qg[i] - ql;
      // conj((ps + j qs) / V) = (ps - j qs) / conj(V) = (ps - j qs) V / w
      double spr = (ps * vi.x + qs * vi.y) / w;
      double spi = (ps * vi.y - qs * vi.x) / w;
      double dr = spr - ir, di = spi - ii;
      F[2 * p] = di;
      F[2 * p + 1] = dr;
      local = fmax(fabs(dr), fabs(di));
      if (!(dr == dr) || !(di == di)) local = __longlong_as_double(0x7ff8000000000000ll);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(local, off, 64);
    local = (o > local || o != o) ? o : local;
  }
  if ((threadIdx.x & 63) == 0 && local != 0.0) atomic_max_nonneg(&red->norm_bits, local);
}

// ---------------------------------------------------------------------------
// Jacobian fill into LU storage

template <typename T>
__global__ void k_zero(T* p, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = T(0);
}

template <typename T>
__device__ inline void jstore(T* lu, T* tail, int ldt, int nt, int code, double a, double b, double c,
                              double d) {
  if (code >= 0) {
    T* q = lu + 4 * (int64_t)code;
    q[0] = (T)a;
    q[1] = (T)b;
    q[2] = (T)c;
    q[3] = (T)d;
  } else if (code <= -2) {
    int t = -2 - code;
    int ta = t / nt, tb = t - ta * nt;
    T* q = tail + (int64_t)(2 * tb) * ldt + 2 * ta;
    q[0] = (T)a;
    q[1] = (T)c;
    q[ldt] = (T)b;
    q[ldt + 1] = (T)d;
  }
}

// Polar J (eq. 10) from the rectangular form of eq. 6-7.  For j != i, with
// W = V_i conj(Y_ij V_j):  dS_i/dangle_j = -jW,  dS_i/d|V_j| = W/|V_j|.
// Diagonal, with W_d = |V_i|^2 conj(Y_ii):  dS_i/dangle_i = j(S_i - W_d),
// dS_i/d|V_i| = (S_i + W_d)/|V_i|.  Block = [[Re dS/dangle, Re dS/d|V|],
// [Im dS/dangle, Im dS/d|V|]]; the |V| row and column of a PV bus are
// replaced by the identity (that unknown is fixed).
template <typename T>
__global__ void k_jfill_polar(int nnz, const int* __restrict__ yrow, const int* __restrict__ col,
                              const double2* __restrict__ y, const double2* __restrict__ v,
                              const double2* __restrict__ ibus, const double* __restrict__ vm,
                              const int8_t* __restrict__ type, const int* __restrict__ jmap, T* lu,
                              T* tail, int ldt, int nt) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int code = jmap[e];
  if (code == -1) return;
  int i = yrow[e], j = col[e];
  double2 yy = y[e];
  double2 vi = v[i];
  double a, b, c, d;
  if (i != j) {
    double2 vj = v[j];
    double tr = yy.x * vj.x - yy.y * vj.y;  // Y_ij V_j
    double ti = yy.x * vj.y + yy.y * vj.x;
    double wr = vi.x * tr + vi.y * ti;  // V_i conj(t)
    double wi = vi.y * tr - vi.x * ti;
    double inv = 1.0 / vm[j];
    a = wi;
    b = wr * inv;
    c = -wr;
    d = wi * inv;
  } else {
    double2 ii = ibus[i];
    double sr = vi.x * ii.x + vi.y * ii.y;
    double si = vi.y * ii.x - vi.x * ii.y;
    double w = vm[i] * vm[i];
    double wdr = w * yy.x, wdi = -w * yy.y;
    double inv = 1.0 / vm[i];
    a = -(si - wdi);
    c = sr - wdr;
    b = (sr + wdr) * inv;
    d = (si + wdi) * inv;
  }
  if (type[i] == 2) {  // PV row: |V| equation is the identity
    c = 0.0;
    d = (i == j) ? 1.0 : 0.0;
  }
  if (type[j] == 2) {  // PV column
    b = 0.0;
    if (i != j) d = 0.0;
  }
  jstore(lu, tail, ldt, nt, code, a, b, c, d);
}

// CIM J (eq. 21-23): [[B, G], [G, -B]] for every admittance entry between
// unknown nodes, minus the ZIP adjustments a, b, c, d on the node's own
// diagonal (derived: a load component with coefficient s and exponent e
// draws I = conj(s) V |V|^(e-2)).
template <typename T>
__global__ void k_jfill_cim(int nnz, const int* __restrict__ yrow, const int* __restrict__ col,
                            const double2* __restrict__ y, const double2* __restrict__ v,
                            const double* __restrict__ pg, const double* __restrict__ qg,
                            const double* __restrict__ zip, const int* __restrict__ jmap, T* lu,
                            T* tail, int ldt, int nt) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int code = jmap[e];
  if (code == -1) return;
  int i = yrow[e], j = col[e];
  double2 yy = y[e];
  double G = yy.x, B = yy.y;
  double a = B, b = G, c = G, d = -B;
  if (i == j) {
    double2 vv = v[i];
    double w = vv.x * vv.x + vv.y * vv.y;
    const double* z = zip + 6 * i;
    // components (s_re, s_im, exponent): loads enter with a minus sign
    double sr[4] = {-z[0], -z[1], -z[2], pg[i]};
    double sim[4] = {-z[3], -z[4], -z[5], qg[i]};
    double ex[4] = {2.0, 1.0, 0.0, 0.0};
    double drr = 0, dri = 0, dir = 0, dii = 0;  // dI/dVre (re, im), dI/dVim (re, im)
    for (int k = 0; k < 4; ++k) {
      double g = pow(w, 0.5 * (ex[k] - 2.0));
      double gp = 0.5 * (ex[k] - 2.0) * pow(w, 0.5 * (ex[k] - 4.0));
      double cr = sr[k], ci = -sim[k];  // conj(s)
      // dI/dVre = conj(s) * (g + 2 Vre V g')
      double ur = g + 2.0 * vv.x * vv.x * gp, ui = 2.0 * vv.x * vv.y * gp;
      drr += cr * ur - ci * ui;
      dri += cr * ui + ci * ur;
      // dI/dVim = conj(s) * (j g + 2 Vim V g')
      double tr = 2.0 * vv.y * vv.x * gp, ti = g + 2.0 * vv.y * vv.y * gp;
      dir += cr * tr - ci * ti;
      dii += cr * ti + ci * tr;
    }
    a -= dri;  // Im dI/dVre
    b -= dii;  // Im dI/dVim
    c -= drr;  // Re dI/dVre
    d -= dir;  // Re dI/dVim
  }
  jstore(lu, tail, ldt, nt, code, a, b, c, d);
}

// ---------------------------------------------------------------------------
// sparse block refactorisation: one work-group per column of a level

template <typename T>
__global__ void k_factor_cols(const int* __restrict__ cols, Sched s, T* lu, T* dinv, Red* red) {
  __shared__ T sdinv[4];
  const int j = cols[blockIdx.x];
  const int c0 = s.colptr[j];
  const int len = s.colptr[j + 1] - c0;
  const int64_t tb = (int64_t)j + 2LL * c0;
  // D_j and U(j, .): gather their updates
  for (int t = threadIdx.x; t <= len; t += blockDim.x) {
    int64_t dest = t == 0 ? (int64_t)j : (int64_t)s.ns + s.nnzl + c0 + (t - 1);
    Blk<T> acc = ld_blk(lu, dest);
    for (int64_t q = s.uptr[tb + t]; q < s.uptr[tb + t + 1]; ++q)
      blk_msub(acc, ld_blk(lu, s.upd_l[q]), ld_blk(lu, s.upd_u[q]));
    st_blk(lu, dest, acc);
    if (t == 0) {
      T det = acc.a * acc.d - acc.b * acc.c;
      bool bad = !(det != T(0)) || !isfinite((double)det);
      if (bad) {
        red->singular = 1;
        det = T(1);
      }
      T r = T(1) / det;
      sdinv[0] = acc.d * r;
      sdinv[1] = -acc.b * r;
      sdinv[2] = -acc.c * r;
      sdinv[3] = acc.a * r;
      T* q = dinv + 4 * (int64_t)j;
      q[0] = sdinv[0];
      q[1] = sdinv[1];
      q[2] = sdinv[2];
      q[3] = sdinv[3];
    }
  }
  __syncthreads();
  Blk<T> di = {sdinv[0], sdinv[1], sdinv[2], sdinv[3]};
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    int64_t dest = (int64_t)s.ns + c0 + t;
    int64_t tg = tb + 1 + len + t;
    Blk<T> acc = ld_blk(lu, dest);
    for (int64_t q = s.uptr[tg]; q < s.uptr[tg + 1]; ++q)
      blk_msub(acc, ld_blk(lu, s.upd_l[q]), ld_blk(lu, s.upd_u[q]));
    st_blk(lu, dest, blk_mul(acc, di));
  }
}

// Schur complement of the sparse part into the dense trailing block:
// T(a,b) -= sum_k L(a,k) U(k,b)
template <typename T>
__global__ void k_tail_schur(int ntt, const int* __restrict__ tgt, const int64_t* __restrict__ uptr,
                             const int* __restrict__ ul, const int* __restrict__ uu, const T* __restrict__ lu,
                             T* tail, int ldt, int nt) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntt) return;
  Blk<T> acc = {T(0), T(0), T(0), T(0)};
  for (int64_t q = uptr[t]; q < uptr[t + 1]; ++q) blk_msub(acc, ld_blk(lu, ul[q]), ld_blk(lu, uu[q]));
  int g = tgt[t];
  int ta = g / nt, tb = g - ta * nt;
  T* p = tail + (int64_t)(2 * tb) * ldt + 2 * ta;
  p[0] += acc.a;
  p[1] += acc.c;
  p[ldt] += acc.b;
  p[ldt + 1] += acc.d;
}

// ---------------------------------------------------------------------------
// triangular solves over sparse rows

template <typename T>
__global__ void k_copy_rhs(int m, const double* __restrict__ F, T* x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] = (T)F[i];
}

// y_i = b_i - sum_k L(i,k) y_k for the rows of one level (in place in x); rows
// of the dense block also copy their result into the appended RHS column.
template <typename T>
__global__ void k_fwd_rows(const int* __restrict__ rows, int nrows, int row_base,
                           const int* __restrict__ lrow_ptr, const int* __restrict__ lrow_blk,
                           const int* __restrict__ lrow_col, const T* __restrict__ lu, T* x, T* tail_rhs,
                           int ns) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int i = rows ? rows[r] : row_base + r;
  T y0 = x[2 * i], y1 = x[2 * i + 1];
  for (int q = lrow_ptr[i]; q < lrow_ptr[i + 1]; ++q) {
    Blk<T> L = ld_blk(lu, lrow_blk[q]);
    int k = lrow_col[q];
    T x0 = x[2 * k], x1 = x[2 * k + 1];
    y0 -= L.a * x0 + L.b * x1;
    y1 -= L.c * x0 + L.d * x1;
  }
  x[2 * i] = y0;
  x[2 * i + 1] = y1;
  if (tail_rhs && i >= ns) {
    tail_rhs[2 * (i - ns)] = y0;
    tail_rhs[2 * (i - ns) + 1] = y1;
  }
}

// x_i = D_i^{-1} (y_i - sum_j U(i,j) x_j) for the rows of one level
template <typename T>
__global__ void k_bwd_rows(const int* __restrict__ rows, int nrows, Sched s, const T* __restrict__ lu,
                           const T* __restrict__ dinv, T* x) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int i = rows[r];
  T z0 = x[2 * i], z1 = x[2 * i + 1];
  for (int q = s.colptr[i]; q < s.colptr[i + 1]; ++q) {
    Blk<T> U = ld_blk(lu, (int64_t)s.ns + s.nnzl + q);
    int j = s.rowidx[q];
    T x0 = x[2 * j], x1 = x[2 * j + 1];
    z0 -= U.a * x0 + U.b * x1;
    z1 -= U.c * x0 + U.d * x1;
  }
  Blk<T> D = ld_blk(dinv, i);
  x[2 * i] = D.a * z0 + D.b * z1;
  x[2 * i + 1] = D.c * z0 + D.d * z1;
}

// ---------------------------------------------------------------------------
// voltage update (FP64)

// Polar: angle += dx[2p] (non-slack), |V| += dx[2p+1] (PQ only); refresh the
// rectangular voltage.
template <typename T>
__global__ void k_update_polar(int nu, const int* __restrict__ node, const int8_t* __restrict__ type,
                               const T* __restrict__ x, double* vm, double* va, double2* v, Red* red) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  double local = 0.0;
  if (p < nu) {
    int i = node[p];
    double da = (double)x[2 * p];
    double dm = type[i] == 1 ? (double)x[2 * p + 1] : 0.0;
    double a = va[i] + da, m = vm[i] + dm;
    va[i] = a;
    vm[i] = m;
    double s, c;
    sincos(a, &s, &c);
    v[i] = make_double2(m * c, m * s);
    local = fmax(fabs(da), fabs(dm));
    if (!(local == local)) local = __longlong_as_double(0x7ff8000000000000ll);
  }
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(local, off, 64);
    local = (o > local || o != o) ? o : local;
  }
  if ((threadIdx.x & 63) == 0 && local != 0.0) atomic_max_nonneg(&red->step_bits, local);
}

// CIM: Re V += dx[2p], Im V += dx[2p+1] (eq. 20 pairing; Alg. steps 6-7).
template <typename T>
__global__ void k_update_cim(int nu, const int* __restrict__ node, const T* __restrict__ x, double2* v,
                             Red* red) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  double local = 0.0;
  if (p < nu) {
    int i = node[p];
    double dr = (double)x[2 * p], di = (double)x[2 * p + 1];
    double2 vv = v[i];
    v[i] = make_double2(vv.x + dr, vv.y + di);
    local = fmax(fabs(dr), fabs(di));
    if (!(local == local)) local = __longlong_as_double(0x7ff8000000000000ll);
  }
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(local, off, 64);
    local = (o > local || o != o) ? o : local;
  }
  if ((threadIdx.x & 63) == 0 && local != 0.0) atomic_max_nonneg(&red->step_bits, local);
}

// ---------------------------------------------------------------------------
// host launchers

#define PF_GRID(n, b) dim3((unsigned)(((n) + (b)-1) / (b)))

void launch_init_polar(hipStream_t st, int n, const int8_t* type, const double* vmag, const double* vang,
                       double* vm, double* va, double* v, int flat) {
  if (n <= 0) return;
  k_init_polar<<<PF_GRID(n, 256), 256, 0, st>>>(n, type, vmag, vang, vm, va, v, flat);
}
void launch_init_cim(hipStream_t st, int n, const int8_t* type, const double* vmag, const double* vang,
                     double* v) {
  if (n <= 0) return;
  k_init_cim<<<PF_GRID(n, 256), 256, 0, st>>>(n, type, vmag, vang, v);
}
void launch_reset_red(hipStream_t st, Red* r) { k_reset_red<<<1, 64, 0, st>>>(r); }

void launch_mismatch_polar(hipStream_t st, int n, const int* row_ptr, const int* col, const double* y,
                           const double* v, const int8_t* type, const double* psp, const double* qsp,
                           const int* pos, double* ibus, double* F, Red* red) {
  k_mismatch_polar<<<PF_GRID(n, 256), 256, 0, st>>>(n, row_ptr, col, (const double2*)y, (const double2*)v,
                                                    type, psp, qsp, pos, (double2*)ibus, F, red);
}
void launch_mismatch_cim(hipStream_t st, int n, const int* row_ptr, const int* col, const double* y,
                         const double* v, const double* pg, const double* qg, const double* zip,
                         const int* pos, double* F, Red* red) {
  k_mismatch_cim<<<PF_GRID(n, 256), 256, 0, st>>>(n, row_ptr, col, (const double2*)y, (const double2*)v, pg,
                                                  qg, zip, pos, F, red);
}

template <typename T>
void launch_zero(hipStream_t st, T* p, int64_t count) {
  if (count <= 0) return;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_zero<T><<<dim3((unsigned)blocks), 256, 0, st>>>(p, count);
}

template <typename T>
void launch_jfill_polar(hipStream_t st, int nnz, const int* yrow, const int* col, const double* y,
                        const double* v, const double* ibus, const double* vm, const int8_t* type,
                        const int* jmap, T* lu, T* tail, int ldt, int nt) {
  k_jfill_polar<T><<<PF_GRID(nnz, 256), 256, 0, st>>>(nnz, yrow, col, (const double2*)y, (const double2*)v,
                                                      (const double2*)ibus, vm, type, jmap, lu, tail, ldt,
                                                      nt);
}
template <typename T>
void launch_jfill_cim(hipStream_t st, int nnz, const int* yrow, const int* col, const double* y,
                      const double* v, const double* pg, const double* qg, const double* zip,
                      const int* jmap, T* lu, T* tail, int ldt, int nt) {
  k_jfill_cim<T><<<PF_GRID(nnz, 256), 256, 0, st>>>(nnz, yrow, col, (const double2*)y, (const double2*)v, pg,
                                                    qg, zip, jmap, lu, tail, ldt, nt);
}

template <typename T>
void launch_factor_cols(hipStream_t st, const int* cols, int ncols, const Sched& s, T* lu, T* dinv,
                        Red* red) {
  if (ncols <= 0) return;
  k_factor_cols<T><<<dim3((unsigned)ncols), 64, 0, st>>>(cols, s, lu, dinv, red);
}

template <typename T>
void launch_tail_schur(hipStream_t st, int ntt, const int* tgt, const int64_t* uptr, const int* ul,
                       const int* uu, const T* lu, T* tail, int ldt, int nt) {
  if (ntt <= 0) return;
  k_tail_schur<T><<<PF_GRID(ntt, 256), 256, 0, st>>>(ntt, tgt, uptr, ul, uu, lu, tail, ldt, nt);
}

template <typename T>
void launch_copy_rhs(hipStream_t st, int m, const double* F, T* x) {
  if (m <= 0) return;
  k_copy_rhs<T><<<PF_GRID(m, 256), 256, 0, st>>>(m, F, x);
}

template <typename T>
void launch_fwd_rows(hipStream_t st, const int* rows, int nrows, int row_base, const int* lrow_ptr,
                     const int* lrow_blk, const int* lrow_col, const T* lu, T* x, T* tail_rhs, int ns) {
  if (nrows <= 0) return;
  k_fwd_rows<T><<<PF_GRID(nrows, 64), 64, 0, st>>>(rows, nrows, row_base, lrow_ptr, lrow_blk, lrow_col, lu, x,
                                                   tail_rhs, ns);
}

template <typename T>
void launch_bwd_rows(hipStream_t st, const int* rows, int nrows, const Sched& s, const T* lu, const T* dinv,
                     T* x) {
  if (nrows <= 0) return;
  k_bwd_rows<T><<<PF_GRID(nrows, 64), 64, 0, st>>>(rows, nrows, s, lu, dinv, x);
}

template <typename T>
void launch_update_polar(hipStream_t st, int nu, const int* node, const int8_t* type, const T* x, double* vm,
                         double* va, double* v, Red* red) {
  if (nu <= 0) return;
  k_update_polar<T><<<PF_GRID(nu, 256), 256, 0, st>>>(nu, node, type, x, vm, va, (double2*)v, red);
}
template <typename T>
void launch_update_cim(hipStream_t st, int nu, const int* node, const T* x, double* v, Red* red) {
  if (nu <= 0) return;
  k_update_cim<T><<<PF_GRID(nu, 256), 256, 0, st>>>(nu, node, x, (double2*)v, red);
}

#define PF_INST(T)                                                                                          \
  template void launch_zero<T>(hipStream_t, T*, int64_t);                                                   \
  template void launch_jfill_polar<T>(hipStream_t, int, const int*, const int*, const double*, const double*, \
                                      const double*, const double*, const int8_t*, const int*, T*, T*, int,  \
                                      int);                                                                 \
  template void launch_jfill_cim<T>(hipStream_t, int, const int*, const int*, const double*, const double*,   \
                                    const double*, const double*, const double*, const int*, T*, T*, int,    \
                                    int);                                                                   \
  template void launch_factor_cols<T>(hipStream_t, const int*, int, const Sched&, T*, T*, Red*);            \
  template void launch_tail_schur<T>(hipStream_t, int, const int*, const int64_t*, const int*, const int*,   \
                                     const T*, T*, int, int);                                               \
  template void launch_copy_rhs<T>(hipStream_t, int, const double*, T*);                                    \
  template void launch_fwd_rows<T>(hipStream_t, const int*, int, int, const int*, const int*, const int*,    \
                                   const T*, T*, T*, int);                                                  \
  template void launch_bwd_rows<T>(hipStream_t, const int*, int, const Sched&, const T*, const T*, T*);     \
  template void launch_update_polar<T>(hipStream_t, int, const int*, const int8_t*, const T*, double*,       \
                                       double*, double*, Red*);                                             \
  template void launch_update_cim<T>(hipStream_t, int, const int*, const T*, double*, Red*);

PF_INST(double)
PF_INST(float)

}  // namespace pfd
