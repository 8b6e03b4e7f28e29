// HIP kernels of the Newton power-flow iteration for gfx950 (wave64).
//
// Per Newton step (Sec. II-A and II-B iteration tables, Sec. III-A solve):
//   convergence test -> Jacobian fill into LU storage -> sparse block
//   refactorisation by elimination-tree levels -> forward solve -> Schur
//   update of the dense trailing block -> dense LU of that block with the
//   right-hand side appended (dense.hip) -> dense backward solve -> sparse
//   backward solve -> voltage update -> mismatch.
// Value type T of the factor and the inner solves is double (plain) or float
// (mixed precision); the mismatch, the update and the convergence test are
// always double.  Every kernel takes the batch's instance table; instances
// whose Newton iteration has finished are skipped.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "blk.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace pfd {

// ---------------------------------------------------------------------------
// helpers

__device__ inline void atomic_max_nonneg(unsigned long long* slot, double v) {
  // |x| and NaN (positive quiet NaN bits) both order correctly as integers
  atomicMax(slot, (unsigned long long)__double_as_longlong(v));
}

__device__ inline double wave_max(double local) {
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(local, off, 64);
    local = (o > local || o != o) ? o : local;
  }
  return local;
}

template <typename IR>
__device__ inline bool inactive(const IR& I) { return gp(I.red)->active == 0; }

// max over a work-group of 256 threads (every thread calls it), stored by
// thread 0 as the work-group's partial maximum (the instance's convergence
// test reduces the partials; atomics on one address would serialise at the
// cache)
__device__ inline void block_max_store(double local, double* out) {
  __shared__ double wmax[4];
  local = wave_max(local);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
#pragma unroll
    for (int w = 1; w < 4; ++w) m = (wmax[w] > m || wmax[w] != wmax[w]) ? wmax[w] : m;
    *out = m;
  }
}

// ---------------------------------------------------------------------------
// Newton driver on the device

// Start of a solve: flat start (polar: |V| = 1 on PQ buses, set-point
// elsewhere, angle 0 but the slack's set-point; CIM: magnitude 1, the
// set-point on source and PV nodes, at the node's nominal phase angle, and a
// PV node's generator Q at its given starting value) or the stored voltage,
// and the rectangular voltage v.
__global__ void k_init(const Inst* const* insts, int flat) {
  const Inst& I = *insts[blockIdx.y];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= I.n) return;
  double m, a;
  if (I.model == 0) {
    if (flat) {
      m = I.type[i] == 1 ? 1.0 : I.vmag[i];
      a = I.type[i] == 3 ? I.vang[i] : 0.0;
      I.vm[i] = m;
      I.va[i] = a;
    } else {
      m = I.vm[i];
      a = I.va[i];
    }
    double s, c;
    sincos(a, &s, &c);
    I.v[2 * i] = m * c;
    I.v[2 * i + 1] = m * s;
  } else if (flat) {
    const int t = I.type[i];
    m = t == 1 ? 1.0 : I.vmag[i];
    double s, c;
    sincos(I.vang[i], &s, &c);
    I.v[2 * i] = m * c;
    I.v[2 * i + 1] = m * s;
    if (t == 2) I.qg[i] = I.qsp[i];
  }
}

__global__ void k_start(const Inst* const* insts, int nslots) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  Red& r = *insts[s]->red;
  r.norm_bits = 0ull;
  r.step_bits = 0ull;
  r.norm0 = 0.0;
  r.last_norm = 0.0;
  r.last_step = 0.0;
  r.singular = 0;
  r.timeout = 0;
  r.it = 0;
  r.status = 5;  // pending
  r.active = 1;
  r.linear_iters = 0;
}

// max that keeps a NaN
__device__ inline double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

// max of a[k] over k = tid, tid + 256, ... < n, eight loads in flight
// (issued whatever k, past the end re-reading a[0]: the values are >= 0)
__device__ inline double strided_max(const double* a, int n) {
  const PF_AS1 double* g = (const PF_AS1 double*)a;
  double m = 0.0;
  for (int k = threadIdx.x; k < n; k += 2048) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = g[k + 256 * u < n ? k + 256 * u : 0];
#pragma unroll
    for (int u = 0; u < 8; ++u) m = nanmax(m, v[u]);
  }
  return m;
}

// Convergence test of the Newton iteration (the loop condition of both
// iteration tables, on the FP64 mismatch max-norm), divergence and limits,
// one work-group per instance: the max-norms of the mismatch and of the
// last step are reduced from the work-groups' partial maxima (the rows of
// the mismatch that run a work-group each fold theirs into norm_bits).
// Sets status and active; prepares the step counters for the next step.
__global__ __launch_bounds__(256) void k_decide(const Inst* const* insts, DevOpts o) {
  __shared__ double wm[2][4];
  const Inst& I = *insts[blockIdx.x];
  Red& r = *I.red;
  if (!r.active) return;
  const int it = r.it;
  double nm = strided_max(I.mpart, I.nmpart);
  double st = it > 0 ? strided_max(I.upart, I.nupart) : 0.0;
  nm = wave_max(nm);
  st = wave_max(st);
  if ((threadIdx.x & 63) == 0) {
    wm[0][threadIdx.x >> 6] = nm;
    wm[1][threadIdx.x >> 6] = st;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  nm = nanmax(nanmax(wm[0][0], wm[0][1]), nanmax(wm[0][2], wm[0][3]));
  st = nanmax(nanmax(wm[1][0], wm[1][1]), nanmax(wm[1][2], wm[1][3]));
  const double norm = nanmax(nm, __longlong_as_double((long long)r.norm_bits));
  const double step = st;
  r.last_norm = norm;
  if (it > 0) r.last_step = step;
  int status = -1;
  if (it > 0 && r.singular) {
    status = 3;
  } else if (!isfinite(norm) || (it > 0 && !isfinite(step))) {
    status = 2;
  } else {
    if (it == 0) r.norm0 = norm;
    if (norm <= o.tol)
      status = 0;
    else if (it > 0 && norm > 1e6 * r.norm0)
      status = 2;
    else if (it >= o.max_iter)
      status = 1;
  }
  if (status >= 0) {
    r.status = status;
    r.active = 0;
    return;
  }
  r.it = it + 1;
  r.epoch += 1;
  r.singular = 0;
  r.norm_bits = 0ull;
  r.step_bits = 0ull;
}

// Store a descriptor passed by value (the launch captures it, so the host
// copy may change as soon as the launch is queued).
__global__ void k_set_inst(Inst* dst, Inst src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = src;
}

// Zero `words` 32-bit words with vector stores (flags and counters; a fill
// kernel rather than a memset node, so that it is safe inside captured graphs).
__global__ void k_zero_words(unsigned* p, int64_t words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0u;
}

// copy every instance's state into one contiguous array for the host
__global__ void k_gather_red(const Inst* const* insts, int nslots, Red* out) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nslots) out[s] = *insts[s]->red;
}

// ---------------------------------------------------------------------------
// mismatch (FP64)

// Polar: I = Y V (eq. 1), S = V conj(I) (eq. 5 conjugated), dP = P_sp - Re S
// for non-slack buses, dQ = Q_sp - Im S for PQ buses (eq. 8-9).  F is written
// at the bus's LU position (2 rows per node); the |V| row of a PV bus is 0.
// CIM: I_calc = sum_j Y_ij V_j (eq. 18); P_l, Q_l from the ZIP model (eq.
// 14-15); P_sp = P_g - P_l (eq. 12-13); I_sp = conj((P_sp + jQ_sp)/V)
// (eq. 17), a PV node's Q_g being its Newton state; minus the current of the
// node's own delta load, plus that of the delta load it receives;
// dI = I_sp - I_calc (eq. 16); rows per node [Im dI, Re dI].

// Current conj(S(|Vd|)/Vd) a delta load of ZIP coefficients z (at the
// nominal line-to-line voltage sqrt(3) pu) draws across Vd.
__device__ inline double2 delta_current(const PF_AS1 double* z, double2 vd) {
  const double w = vd.x * vd.x + vd.y * vd.y;
  const double m = sqrt(w);
  const double r3 = 0.57735026918962576;  // 1/sqrt(3)
  const double sr = z[0] * w * (1.0 / 3.0) + z[1] * m * r3 + z[2];
  const double si = z[3] * w * (1.0 / 3.0) + z[4] * m * r3 + z[5];
  return make_double2((sr * vd.x + si * vd.y) / w, (sr * vd.y - si * vd.x) / w);
}

// The mismatch reads every array through global (not generic) pointers, so
// that its loads are counted by the vector-memory counter alone and each
// wait is for the loads it needs.
__device__ inline double2 ld_c(const double* p, int64_t i) {
  const PF_AS1 double* q = (const PF_AS1 double*)p + 2 * i;
  return make_double2(q[0], q[1]);
}
__device__ inline void st_c(double* p, int64_t i, double re, double im) {
  PF_AS1 double* q = (PF_AS1 double*)p + 2 * i;
  q[0] = re;
  q[1] = im;
}

// A row's own data besides its Ybus entries (its voltage, set-points, type,
// ZIP coefficients and delta-load links), loaded before the row's sum so
// that these loads do not wait behind it.
struct RowSide {
  double2 vi;
  double psp, qsp, qg;
  int type;
  double z[6];
  int2 dl;
};
template <typename InstRef>
__device__ inline RowSide load_side(const InstRef& I, int i) {
  RowSide s;
  s.vi = ld_c((const double*)I.v, i);
  s.psp = gp(I.psp)[i];
  s.qsp = gp(I.qsp)[i];
  s.type = gp(I.type)[i];
  s.qg = 0.0;
  s.dl = make_int2(-1, -1);
  if (I.model != 0) {
    const auto zip = gp(I.zip) + 6 * i;
#pragma unroll
    for (int k = 0; k < 6; ++k) s.z[k] = zip[k];
    s.qg = gp(I.qg)[i];  // used for PV nodes only; loaded whatever the type so that no load waits for it
    if (I.dlink) {
      const PF_AS1 int* dl = (const PF_AS1 int*)I.dlink + 2 * i;
      s.dl = make_int2(dl[0], dl[1]);
    }
  }
  return s;
}

// The rest of row i's mismatch once I_i = sum_j Y_ij V_j is known: polar dP,
// dQ; CIM the ZIP load, the specified current, the delta loads and dI.
// Writes F at the node's position (and the bus current for polar) and
// returns the row's |F| (NaN when a value is NaN).
template <typename InstRef>
__device__ inline double mismatch_row(const InstRef& I, int i, int p, double ir, double ii, const RowSide& sd) {
  const double2 vi = sd.vi;
  const auto F = gp(I.F);
  double local = 0.0;
  if (I.model == 0) {
    st_c((double*)I.ibus, i, ir, ii);
    if (p >= 0) {
      double sr = vi.x * ir + vi.y * ii;  // Re(V conj I)
      double si = vi.y * ir - vi.x * ii;  // Im(V conj I)
      double dp = sd.psp - sr;
      double dq = sd.type == 1 ? sd.qsp - si : 0.0;
      F[2 * p] = dp;
      F[2 * p + 1] = dq;
      local = fmax(fabs(dp), fabs(dq));
      if (!(dp == dp) || !(dq == dq)) local = __longlong_as_double(0x7ff8000000000000ll);
    }
  } else {
    double w = vi.x * vi.x + vi.y * vi.y;
    double vm = sqrt(w);
    const double* z = sd.z;
    double pl = z[2] + z[1] * vm + z[0] * w;
    double ql = z[5] + z[4] * vm + z[3] * w;
    const double qgen = sd.type == 2 ? sd.qg : sd.qsp;
    double ps = sd.psp - pl, qs = qgen - ql;
    // conj((ps + j qs) / V) = (ps - j qs) V / |V|^2
    double spr = (ps * vi.x + qs * vi.y) / w;
    double spi = (ps * vi.y - qs * vi.x) / w;
    if (I.dlink) {
      const int2 L = sd.dl;
      if (L.x >= 0) {
        const double2 vt = ld_c((const double*)I.v, L.x);
        const double2 id = delta_current(gp(I.zipd) + 6 * i, make_double2(vi.x - vt.x, vi.y - vt.y));
        spr -= id.x;
        spi -= id.y;
      }
      if (L.y >= 0) {
        const double2 vk = ld_c((const double*)I.v, L.y);
        const double2 id = delta_current(gp(I.zipd) + 6 * L.y, make_double2(vk.x - vi.x, vk.y - vi.y));
        spr += id.x;
        spi += id.y;
      }
    }
    double dr = spr - ir, di = spi - ii;
    F[2 * p] = di;
    F[2 * p + 1] = dr;
    local = fmax(fabs(dr), fabs(di));
    if (!(dr == dr) || !(di == di)) local = __longlong_as_double(0x7ff8000000000000ll);
  }
  return local;
}

// Partial sum of Y_iq V_col(q) over q = q0, q0 + S, ... < q1 (the loads of
// two entries issued at once)
template <int S, typename InstRef>
__device__ inline void ydot_part(const InstRef& I, int q0, int q1, double& ir, double& ii) {
  const double* y = (const double*)I.y;
  const double* v = (const double*)I.v;
  const auto col = gp(I.col);
  for (int q = q0; q < q1; q += 2 * S) {
    const bool two = q + S < q1;
    const int c0 = col[q];
    const int c1 = two ? col[q + S] : c0;
    const double2 y0 = ld_c(y, q), y1 = two ? ld_c(y, q + S) : make_double2(0.0, 0.0);
    const double2 v0 = ld_c(v, c0), v1 = ld_c(v, c1);
    ir += y0.x * v0.x - y0.y * v0.y;
    ii += y0.x * v0.y + y0.y * v0.x;
    if (two) {
      ir += y1.x * v1.x - y1.y * v1.y;
      ii += y1.x * v1.y + y1.y * v1.x;
    }
  }
}

// A row of more than kHeavyRow entries (listed per instance in I.heavy): one
// work-group of 256 threads, block-strided partial sums reduced by a wave
// butterfly and then over the four waves in order; its |F| goes into the
// instance's maximum directly.
template <typename InstRef>
__device__ inline void mismatch_heavy_row(const InstRef& I, int h) {
  __shared__ double part[2][4];
  const int i = gp(I.heavy)[h];
  const int p = gp(I.pos)[i];
  if (!(I.model == 0 || p >= 0)) return;
  double ir = 0.0, ii = 0.0;
  ydot_part<256>(I, gp(I.row_ptr)[i] + (int)threadIdx.x, gp(I.row_ptr)[i + 1], ir, ii);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ir += __shfl_xor(ir, off, 64);
    ii += __shfl_xor(ii, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = ir;
    part[1][threadIdx.x >> 6] = ii;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ir = (part[0][0] + part[0][1]) + (part[0][2] + part[0][3]);
    ii = (part[1][0] + part[1][1]) + (part[1][2] + part[1][3]);
    const double local = mismatch_row(I, i, p, ir, ii, load_side(I, i));
    if (local != 0.0) atomic_max_nonneg(&I.red->norm_bits, local);
  }
}

// The mismatch of every row in one launch.  Blocks are renumbered so that
// each XCD takes a contiguous range of rows (the voltages a row gathers are
// mostly its neighbours').  The first nh renumbered work-groups take the
// heavy rows (one each; they are dispatched early, so these long sums
// overlap the rest); the others take the rows of at most kHeavyRow entries,
// S = 4 lanes per row splitting the row's entries (lane-strided partial
// sums, then a fixed-order butterfly), and store the work-group's partial
// maximum.
constexpr int kMisLanes = 4;
template <int S>
__global__ __launch_bounds__(256) void k_mismatch(const Inst* const* insts, int nh) {
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  // whether the instance is still iterating is tested only before the
  // first store: the row's loads need not wait for that flag
  const bool active = gp(I.red)->active != 0;
  const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
  if (blk < nh) {
    if (blk < I.nheavy && active) mismatch_heavy_row(I, blk);
    return;
  }
  const int bx = blk - nh;
  constexpr int kRows = 256 / S;
  if (bx * kRows >= I.n) return;
  const int lane = threadIdx.x % S;
  const int i = bx * kRows + (int)threadIdx.x / S;
  double local = 0.0;
  bool mine = false;
  int p = -1;
  double ir = 0.0, ii = 0.0;
  RowSide side;
  if (i < I.n) {
    p = gp(I.pos)[i];
    const int q0 = gp(I.row_ptr)[i], q1 = gp(I.row_ptr)[i + 1];
    // the lane's first three entries (rows of up to 3 S entries, such as
    // the three-phase rows of a feeder, then need no further round trip),
    // loaded whatever the row (indices past the row read its first entry,
    // which every row has: the diagonal), so that nothing waits for the
    // row's kind or for the side data
    const double* y = (const double*)I.y;
    const double* v = (const double*)I.v;
    const auto col = gp(I.col);
    const int qa = q0 + lane, qb = qa + S, qc = qb + S;
    const bool ha = qa < q1, hb = qb < q1, hc = qc < q1;
    const int ca = col[ha ? qa : q0], cb = col[hb ? qb : q0], cc = col[hc ? qc : q0];
    const double2 ya = ld_c(y, ha ? qa : q0), yb = ld_c(y, hb ? qb : q0), yc = ld_c(y, hc ? qc : q0);
    const double2 va = ld_c(v, ca), vb = ld_c(v, cb), vc = ld_c(v, cc);
    if (lane == 0) side = load_side(I, i);
    mine = (I.model == 0 || p >= 0) && q1 - q0 <= kHeavyRow;
    if (mine) {
      if (ha) {
        ir += ya.x * va.x - ya.y * va.y;
        ii += ya.x * va.y + ya.y * va.x;
      }
      if (hb) {
        ir += yb.x * vb.x - yb.y * vb.y;
        ii += yb.x * vb.y + yb.y * vb.x;
      }
      if (hc) {
        ir += yc.x * vc.x - yc.y * vc.y;
        ii += yc.x * vc.y + yc.y * vc.x;
      }
      if (qc + S < q1) ydot_part<S>(I, qc + S, q1, ir, ii);
    }
  }
#pragma unroll
  for (int off = S / 2; off > 0; off >>= 1) {
    ir += __shfl_xor(ir, off, 64);
    ii += __shfl_xor(ii, off, 64);
  }
  if (!active) return;  // uniform over the work-group
  if (mine && lane == 0) local = mismatch_row(I, i, p, ir, ii, side);
  block_max_store(local, (double*)I.mpart + bx);
}

// ---------------------------------------------------------------------------
// Jacobian fill into LU storage

// Zero the factor storage by chunks of ZCH values: item (slot, c) clears
// chunk c of the sparse factor values, item (slot, -1 - c) chunk c of the
// dense block.  The batch lists each instance's own chunks, so the grid is
// proportional to the storage actually cleared.
constexpr int ZCH = 8192;

template <typename T>
__global__ __launch_bounds__(256) void k_zero_chunks(const Inst* const* insts, const int2* __restrict__ work) {
  const int2 w = ld_item(work, blockIdx.x);
  const auto& I = *gp(gp(insts)[w.x]);
  if (inactive(I)) return;
  const bool tail = w.y < 0;
  const int64_t c = tail ? -1 - (int64_t)w.y : (int64_t)w.y;
  const auto p = gp((T*)(tail ? I.tail : I.lu));
  const int64_t n = tail ? I.tail_count : I.lu_count;
  const int64_t b = c * ZCH, e = min(n, b + ZCH);
  for (int64_t i = b + threadIdx.x; i < e; i += 256) p[i] = T(0);
}

template <typename T, typename IR>
__device__ inline void jstore(const IR& I, int code, double a, double b, double c, double d) {
  if (code >= 0) {
    const auto q = gp((T*)I.lu) + 4 * (int64_t)code;
    q[0] = (T)a;
    q[1] = (T)b;
    q[2] = (T)c;
    q[3] = (T)d;
  } else if (code <= -2) {
    int t = -2 - code;
    int ta = t / I.nt, tb = t - ta * I.nt;
    const auto q = gp((T*)I.tail) + (int64_t)(2 * tb) * I.ldt + 2 * ta;
    q[0] = (T)a;
    q[1] = (T)c;
    q[I.ldt] = (T)b;
    q[I.ldt + 1] = (T)d;
  }
}

// The 2x2 Jacobian block of Ybus entry e (row i, column j).
//
// Polar J (eq. 10) from the rectangular form of eq. 6-7.  For j != i, with
// W = V_i conj(Y_ij V_j):  dS_i/dangle_j = -jW,  dS_i/d|V_j| = W/|V_j|.
// Diagonal, with W_d = |V_i|^2 conj(Y_ii):  dS_i/dangle_i = j(S_i - W_d),
// dS_i/d|V_i| = (S_i + W_d)/|V_i|.  Block = [[Re dS/dangle, Re dS/d|V|],
// [Im dS/dangle, Im dS/d|V|]]; the |V| row and column of a PV bus are
// replaced by the identity (that unknown is fixed).
//
// CIM J (eq. 21-23): [[B, G], [G, -B]] for every admittance entry between
// unknown nodes, minus the ZIP adjustments a, b, c, d on the node's own
// diagonal (derived: a load component with coefficient s and exponent e
// draws I = conj(s) V |V|^(e-2)), plus the delta loads' blocks, with the
// columns of PV nodes taken in (angle, Q).
// dI/dVre and dI/dVim, as D = {Re dI/dVre, Im dI/dVre, Re dI/dVim,
// Im dI/dVim}, of the current sum_k conj(s_k) V |V|^(e_k - 2): with w = |V|^2,
// g = w^((e-2)/2), g' = ((e-2)/2) w^((e-4)/2), dI/dVre = conj(s)(g + 2 Vre V
// g') and dI/dVim = conj(s)(j g + 2 Vim V g').
__device__ inline void load_derivative(const double* sr, const double* sim, const double* ex, int cnt, double2 vv,
                                       double* D) {
  const double w = vv.x * vv.x + vv.y * vv.y;
  double drr = 0, dri = 0, dir = 0, dii = 0;
  for (int k = 0; k < cnt; ++k) {
    double g = pow(w, 0.5 * (ex[k] - 2.0));
    double gp = 0.5 * (ex[k] - 2.0) * pow(w, 0.5 * (ex[k] - 4.0));
    double cr = sr[k], ci = -sim[k];  // conj(s)
    double ur = g + 2.0 * vv.x * vv.x * gp, ui = 2.0 * vv.x * vv.y * gp;
    drr += cr * ur - ci * ui;
    dri += cr * ui + ci * ur;
    double tr = 2.0 * vv.y * vv.x * gp, ti = g + 2.0 * vv.y * vv.y * gp;
    dir += cr * tr - ci * ti;
    dii += cr * ti + ci * tr;
  }
  D[0] = drr;
  D[1] = dri;
  D[2] = dir;
  D[3] = dii;
}

// D = dI_d/dV_d of the delta load z between nodes at voltages vk and vt
// (V_d = vk - vt): its components are s / sqrt(3)^e.
template <typename P>
__device__ inline void delta_derivative(P z, double2 vk, double2 vt, double* D) {
  const double r3 = 0.57735026918962576;
  const double sr[3] = {z[0] * (1.0 / 3.0), z[1] * r3, z[2]};
  const double sim[3] = {z[3] * (1.0 / 3.0), z[4] * r3, z[5]};
  const double ex[3] = {2.0, 1.0, 0.0};
  load_derivative(sr, sim, ex, 3, make_double2(vk.x - vt.x, vk.y - vt.y), D);
}

template <typename IR>
__device__ inline void jblock(const IR& I, int e, double* out) {
  const int i = gp(I.yrow)[e], j = gp(I.col)[e];
  const double2 yy = ld_c(I.y, e);
  const double* v = I.v;  // complex, as pairs
  double a, b, c, d;
  if (I.model == 0) {
    const double2 vi = ld_c(v, i);
    if (i != j) {
      double2 vj = ld_c(v, j);
      double tr = yy.x * vj.x - yy.y * vj.y;  // Y_ij V_j
      double ti = yy.x * vj.y + yy.y * vj.x;
      double wr = vi.x * tr + vi.y * ti;  // V_i conj(t)
      double wi = vi.y * tr - vi.x * ti;
      double inv = 1.0 / gp(I.vm)[j];
      a = wi;
      b = wr * inv;
      c = -wr;
      d = wi * inv;
    } else {
      double2 ii = ld_c(I.ibus, i);
      double sr = vi.x * ii.x + vi.y * ii.y;
      double si = vi.y * ii.x - vi.x * ii.y;
      double w = gp(I.vm)[i] * gp(I.vm)[i];
      double wdr = w * yy.x, wdi = -w * yy.y;
      double inv = 1.0 / gp(I.vm)[i];
      a = -(si - wdi);
      c = sr - wdr;
      b = (sr + wdr) * inv;
      d = (si + wdi) * inv;
    }
    if (gp(I.type)[i] == 2) {  // PV row: the |V| equation is the identity
      c = 0.0;
      d = (i == j) ? 1.0 : 0.0;
    }
    if (gp(I.type)[j] == 2) {  // PV column
      b = 0.0;
      if (i != j) d = 0.0;
    }
  } else {
    const double G = yy.x, Bv = yy.y;
    a = Bv;
    b = G;
    c = G;
    d = -Bv;
    if (i == j) {
      const double2 vv = ld_c(v, i);
      const auto z = gp(I.zip) + 6 * i;
      // components (s_re, s_im, exponent): loads enter with a minus sign
      const double sr[4] = {-z[0], -z[1], -z[2], gp(I.psp)[i]};
      const double sim[4] = {-z[3], -z[4], -z[5], gp(I.type)[i] == 2 ? gp(I.qg)[i] : gp(I.qsp)[i]};
      const double ex[4] = {2.0, 1.0, 0.0, 0.0};
      double D[4];
      load_derivative(sr, sim, ex, 4, vv, D);
      a -= D[1];  // Im dI/dVre
      b -= D[3];  // Im dI/dVim
      c -= D[0];  // Re dI/dVre
      d -= D[2];  // Re dI/dVim
    }
    if (I.dlink) {
      // delta loads: the load k -> t draws I_d(V_k - V_t); with D = dI_d/dV_d
      // it adds +D at (k, k) and (t, t), -D at (k, t) and (t, k)
      const int2 L = ld_item(I.dlink, i);
      double D[4];
      if (L.x >= 0 && (j == i || j == L.x)) {
        delta_derivative(gp(I.zipd) + 6 * i, ld_c(v, i), ld_c(v, L.x), D);
        const double sg = j == i ? 1.0 : -1.0;
        a += sg * D[1];
        b += sg * D[3];
        c += sg * D[0];
        d += sg * D[2];
      }
      if (L.y >= 0 && (j == i || j == L.y)) {
        delta_derivative(gp(I.zipd) + 6 * L.y, ld_c(v, L.y), ld_c(v, i), D);
        const double sg = j == i ? 1.0 : -1.0;
        a += sg * D[1];
        b += sg * D[3];
        c += sg * D[0];
        d += sg * D[2];
      }
    }
    if (gp(I.type)[j] == 2) {
      // PV column: the node's unknowns are (angle, generator Q) with |V| at
      // its set-point.  d/dangle = -Vim d/dVre + Vre d/dVim; the Q column is
      // -dI_sp/dQ = -(Vim - j Vre)/|V|^2 on the node's own rows only.
      const double2 vj = ld_c(v, j);
      const double na = -vj.y * a + vj.x * b;
      const double nc = -vj.y * c + vj.x * d;
      a = na;
      c = nc;
      if (i == j) {
        const double w = vj.x * vj.x + vj.y * vj.y;
        b = vj.x / w;
        d = -vj.y / w;
      } else {
        b = 0.0;
        d = 0.0;
      }
    }
  }
  out[0] = a;
  out[1] = b;
  out[2] = c;
  out[3] = d;
}

// Work-groups below nj: the Jacobian blocks into the factor storage; the
// others: the right-hand side F into x, with every entry of the backward
// solve's published copy of the solution marked unsolved.
template <typename T>
__global__ void k_jfill(const Inst* const* insts, int nj) {
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (inactive(I)) return;
  if ((int)blockIdx.x >= nj) {
    const int i = ((int)blockIdx.x - nj) * blockDim.x + threadIdx.x;
    if (i < 2 * I.nu) {
      gp((T*)I.x)[i] = (T)gp(I.F)[i];
      gp((T*)I.xs)[i] = unsolved_value<T>();
    }
    return;
  }
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= I.nnz) return;
  int code = gp(I.jmap)[e];
  if (code == -1) return;
  double blk[4];
  jblock(I, e, blk);
  jstore<T>(I, code, blk[0], blk[1], blk[2], blk[3]);
}

// Jacobian fill for the Krylov inner solve: every Ybus entry between nodes
// with unknowns gives one 2x2 block of the block CSR Jacobian; with ILU(0)
// the block is also the starting value of the factor.
template <typename T>
__global__ void k_kfill(const Inst* const* insts, int ilu) {
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (inactive(I)) return;
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= I.nnz) return;
  const int q = gp(I.kmap)[e];
  if (q < 0) return;
  double b[4];
  jblock(I, e, b);
  const auto jv = gp((T*)I.jval) + 4 * (int64_t)q;
  jv[0] = (T)b[0];
  jv[1] = (T)b[1];
  jv[2] = (T)b[2];
  jv[3] = (T)b[3];
  if (ilu) {
    const auto pv = gp((T*)I.pval) + 4 * (int64_t)q;
    pv[0] = (T)b[0];
    pv[1] = (T)b[1];
    pv[2] = (T)b[2];
    pv[3] = (T)b[3];
  }
}

// ---------------------------------------------------------------------------
// sparse block refactorisation: one work-group per (instance, column) of a
// level; each target block (D_j, U(j, .), L(., j)) is reduced by a group of G
// lanes that split its update list (lane-strided partial sums, fixed-order
// tree).

// acc -= sum over updates q = q0, q0 + G, ... < q1 of L(q) U(q) (block ids
// from il / iu), in that order, the loads of four updates issued at once
template <typename T, int G>
__device__ inline void sub_updates(Blk<T>& acc, const T* lu_, const int* il_, const int* iu_, int64_t q0, int64_t q1) {
  const auto lu = gp(lu_);
  const auto il = gp(il_), iu = gp(iu_);
  for (int64_t q = q0; q < q1; q += 4 * G) {
    int a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u * G < q1) {
        a[u] = il[q + u * G];
        b[u] = iu[q + u * G];
      }
    Blk<T> L[4], U[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u * G < q1) {
        L[u] = ld_blk<T>(lu, a[u]);
        U[u] = ld_blk<T>(lu, b[u]);
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u * G < q1) blk_msub(acc, L[u], U[u]);
  }
}

// Forward row of node i by a group of G lanes: y_i = b_i - sum_k L(i,k) y_k
// over the row's L blocks (in place in x, which holds b_i before), lane-
// strided partial sums with the loads of four entries issued at once, then
// the fixed-order tree.  Every L(i,k) and y_k lies in an earlier level.
// Rows of the dense block also copy the result into its right-hand side
// column.
template <typename T, int G, typename IR>
__device__ inline void fwd_row(const IR& I, const T* lu_, T* x_, int i, int lane) {
  const auto lu = gp(lu_);
  const auto x = gp(x_);
  const auto lrow_ptr = gp(I.lrow_ptr), lrow_blk = gp(I.lrow_blk), lrow_col = gp(I.lrow_col);
  Blk<T> acc = {T(0), T(0), T(0), T(0)};  // (a, c) carry the 2-vector
  if (lane == 0) {
    acc.a = x[2 * i];
    acc.c = x[2 * i + 1];
  }
  const int q1 = lrow_ptr[i + 1];
  for (int q = lrow_ptr[i] + lane; q < q1; q += 4 * G) {
    int bk[4], kk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u * G < q1) {
        bk[u] = lrow_blk[q + u * G];
        kk[u] = lrow_col[q + u * G];
      }
    Blk<T> L[4];
    T x0[4], x1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u * G < q1) {
        L[u] = ld_blk(lu, bk[u]);
        x0[u] = x[2 * kk[u]];
        x1[u] = x[2 * kk[u] + 1];
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u * G < q1) {
        acc.a -= L[u].a * x0[u] + L[u].b * x1[u];
        acc.c -= L[u].c * x0[u] + L[u].d * x1[u];
      }
  }
  acc = group_sum<T, G>(acc);
  if (lane == 0) {
    x[2 * i] = acc.a;
    x[2 * i + 1] = acc.c;
    if (i >= I.ns) {
      const auto rhs = gp((T*)I.tail) + (int64_t)I.M * I.ldt;
      rhs[2 * (i - I.ns)] = acc.a;
      rhs[2 * (i - I.ns) + 1] = acc.c;
    }
  }
}

template <typename T, int G, typename IR>
__device__ inline Blk<T> gather_target(const IR& I, const T* lu, int64_t dest, int64_t tg, int lane) {
  Blk<T> acc = {T(0), T(0), T(0), T(0)};
  if (lane == 0) acc = ld_blk<T>(gp(lu), dest);
  sub_updates<T, G>(acc, lu, I.upd_l, I.upd_u, gp(I.uptr)[tg] + lane, gp(I.uptr)[tg + 1]);
  return group_sum<T, G>(acc);
}

// One column per wave (four per work-group) for levels whose columns have at
// most 64/G targets: the targets of a column then take one pass of the
// wave's lane groups, and the diagonal inverse goes to the wave by a
// shuffle instead of a work-group barrier.  Same arithmetic as k_factor_cols.
// Both kernels also run the forward row of the column's node (target len + 1
// of the first pass), so the forward substitution of the sparse part needs
// no launches of its own.
template <typename T, int G>
__global__ __launch_bounds__(256) void k_factor_cols_wave(const Inst* const* insts, const int2* __restrict__ work,
                                                          int nwork) {
  const int item = blockIdx.x * 4 + (int)(threadIdx.x / 64);
  if (item >= nwork) return;
  const int2 w = ld_item(work, item);
  const auto& I = *gp(gp(insts)[w.x]);
  if (inactive(I)) return;
  T* lu = (T*)I.lu;
  const int j = w.y;
  const int c0 = gp(I.colptr)[j];
  const int len = gp(I.colptr)[j + 1] - c0;
  const int64_t tb = (int64_t)j + 2LL * c0;
  const int wl = threadIdx.x % 64;
  const int lane = wl % G, grp = wl / G;
  constexpr int ngrp = 64 / G;
  T d0 = T(0), d1 = T(0), d2 = T(0), d3 = T(0);
  for (int t = grp; t <= len + 1; t += ngrp) {
    if (t == len + 1) {
      fwd_row<T, G>(I, lu, (T*)I.x, j, lane);
      continue;
    }
    int64_t dest = t == 0 ? (int64_t)j : (int64_t)I.ns + I.nnzl + c0 + (t - 1);
    Blk<T> acc = gather_target<T, G>(I, lu, dest, tb + t, lane);
    if (lane == 0) {
      st_blk(gp(lu), dest, acc);
      if (t == 0) {
        T det = acc.a * acc.d - acc.b * acc.c;
        bool bad = !(det != T(0)) || !isfinite((double)det);
        if (bad) {
          gp(I.red)->singular = 1;
          det = T(1);
        }
        T r = T(1) / det;
        d0 = acc.d * r;
        d1 = -acc.b * r;
        d2 = -acc.c * r;
        d3 = acc.a * r;
        const auto q = gp((T*)I.dinv) + 4 * (int64_t)j;
        q[0] = d0;
        q[1] = d1;
        q[2] = d2;
        q[3] = d3;
      }
    }
  }
  // the diagonal target was group 0's first, lane 0 of the wave holds it
  const Blk<T> di = {__shfl(d0, 0, 64), __shfl(d1, 0, 64), __shfl(d2, 0, 64), __shfl(d3, 0, 64)};
  for (int t = grp; t < len; t += ngrp) {
    int64_t dest = (int64_t)I.ns + c0 + t;
    Blk<T> acc = gather_target<T, G>(I, lu, dest, tb + 1 + len + t, lane);
    if (lane == 0) st_blk(gp(lu), dest, blk_mul(acc, di));
  }
}

template <typename T, int G, int NT>
__global__ __launch_bounds__(NT) void k_factor_cols(const Inst* const* insts, const int2* __restrict__ work) {
  __shared__ T sdinv[4];
  const int2 w = ld_item(work, blockIdx.x);
  const auto& I = *gp(gp(insts)[w.x]);
  if (inactive(I)) return;
  T* lu = (T*)I.lu;
  const int j = w.y;
  const int c0 = gp(I.colptr)[j];
  const int len = gp(I.colptr)[j + 1] - c0;
  const int64_t tb = (int64_t)j + 2LL * c0;
  const int lane = threadIdx.x % G, grp = threadIdx.x / G, ngrp = blockDim.x / G;
  // D_j and U(j, .), and the forward row of node j (t = len + 1)
  for (int t = grp; t <= len + 1; t += ngrp) {
    if (t == len + 1) {
      fwd_row<T, G>(I, lu, (T*)I.x, j, lane);
      continue;
    }
    int64_t dest = t == 0 ? (int64_t)j : (int64_t)I.ns + I.nnzl + c0 + (t - 1);
    Blk<T> acc = gather_target<T, G>(I, lu, dest, tb + t, lane);
    if (lane == 0) {
      st_blk(gp(lu), dest, acc);
      if (t == 0) {
        T det = acc.a * acc.d - acc.b * acc.c;
        bool bad = !(det != T(0)) || !isfinite((double)det);
        if (bad) {
          gp(I.red)->singular = 1;
          det = T(1);
        }
        T r = T(1) / det;
        sdinv[0] = acc.d * r;
        sdinv[1] = -acc.b * r;
        sdinv[2] = -acc.c * r;
        sdinv[3] = acc.a * r;
        const auto q = gp((T*)I.dinv) + 4 * (int64_t)j;
        q[0] = sdinv[0];
        q[1] = sdinv[1];
        q[2] = sdinv[2];
        q[3] = sdinv[3];
      }
    }
  }
  __syncthreads();
  const Blk<T> di = {sdinv[0], sdinv[1], sdinv[2], sdinv[3]};
  for (int t = grp; t < len; t += ngrp) {
    int64_t dest = (int64_t)I.ns + c0 + t;
    Blk<T> acc = gather_target<T, G>(I, lu, dest, tb + 1 + len + t, lane);
    if (lane == 0) st_blk(gp(lu), dest, blk_mul(acc, di));
  }
}

// Schur complement of the sparse part into the dense trailing block:
// T(a,b) -= sum_k L(a,k) U(k,b); work item = (instance, first target of a
// chunk of 256).
template <typename T, int G>
__global__ __launch_bounds__(256) void k_tail_schur(const Inst* const* insts, const int2* __restrict__ work) {
  const int2 w = ld_item(work, blockIdx.x);
  const auto& I = *gp(gp(insts)[w.x]);
  // the activity flag is tested only before the store, so that the loads
  // need not wait for it
  const bool active = !inactive(I);
  // G lanes per target split its update list (lane-strided, fixed-order tree)
  const int lane = threadIdx.x % G;
  const int t = w.y + (int)threadIdx.x / G;
  const bool live = t < I.ntt;
  const T* lu = (const T*)I.lu;
  // the target's own values, fetched before its sum (no other thread of
  // the launch writes them)
  const bool own = live && lane == 0;
  const int g = own ? gp(I.tail_tgt)[t] : 0;
  const int ta = g / I.nt, tb = g - ta * I.nt;
  const auto p = gp((T*)I.tail) + (int64_t)(2 * tb) * I.ldt + 2 * ta;
  Blk<T> old = {T(0), T(0), T(0), T(0)};
  if (own) old = {p[0], p[I.ldt], p[1], p[I.ldt + 1]};
  Blk<T> acc = {T(0), T(0), T(0), T(0)};
  if (live) sub_updates<T, G>(acc, lu, I.tail_l, I.tail_u, gp(I.tail_uptr)[t] + lane, gp(I.tail_uptr)[t + 1]);
  acc = group_sum<T, G>(acc);
  if (!active || !own) return;
  p[0] = old.a + acc.a;
  p[1] = old.c + acc.c;
  p[I.ldt] = old.b + acc.b;
  p[I.ldt + 1] = old.d + acc.d;
}

// ---------------------------------------------------------------------------
// triangular solves over sparse rows

// Forward rows of the dense block's nodes (after every sparse level): one
// (instance, row) per group of G lanes.
template <typename T, int G>
__global__ __launch_bounds__(256) void k_fwd_rows(const Inst* const* insts, const int2* __restrict__ work,
                                                  int nwork) {
  const int gid = (blockIdx.x * blockDim.x + threadIdx.x) / G, lane = threadIdx.x % G;
  if (gid >= nwork) return;  // whole groups leave together
  const int2 w = ld_item(work, gid);
  const auto& I = *gp(gp(insts)[w.x]);
  if (inactive(I)) return;
  fwd_row<T, G>(I, (const T*)I.lu, (T*)I.x, w.y, lane);
}

// ---------------------------------------------------------------------------
// voltage update (FP64)

// Polar: angle += dx[2p] (non-slack), |V| += dx[2p+1] (PQ only) (single-phase
// iteration table, update line); CIM: Re V += dx[2p], Im V += dx[2p+1]
// (eq. 20 pairing; three-phase iteration table, update and complex-form
// lines), on PV nodes angle += dx[2p] and Q_g += dx[2p+1].  Refreshes the rectangular voltage and records max |dx|.
template <typename T>
__global__ __launch_bounds__(256) void k_update(const Inst* const* insts) {
  const auto& I = *gp(gp(insts)[blockIdx.y]);
  if (inactive(I) || (int)(blockIdx.x * blockDim.x) >= I.nu) return;
  double local = 0.0;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < I.nu) {
    const auto x = gp((const T*)I.x);
    const int i = gp(I.node)[p];
    const auto type = gp(I.type);
    const auto va = gp(I.va), vm = gp(I.vm);
    double* v = I.v;  // complex, as pairs
    double d0 = (double)x[2 * p], d1 = (double)x[2 * p + 1];
    if (I.model == 0) {
      if (type[i] != 1) d1 = 0.0;
      double a = va[i] + d0, m = vm[i] + d1;
      va[i] = a;
      vm[i] = m;
      double s, c;
      sincos(a, &s, &c);
      st_c(v, i, m * c, m * s);
    } else if (type[i] == 2) {
      // PV node: rotate by the angle step at the set-point magnitude; the
      // second unknown is the generator Q
      double2 vv = ld_c(v, i);
      double s, c;
      sincos(d0, &s, &c);
      double nr = vv.x * c - vv.y * s, ni = vv.x * s + vv.y * c;
      double sc = gp(I.vmag)[i] / sqrt(nr * nr + ni * ni);
      st_c(v, i, nr * sc, ni * sc);
      gp(I.qg)[i] += d1;
    } else {
      double2 vv = ld_c(v, i);
      st_c(v, i, vv.x + d0, vv.y + d1);
    }
    double m = fmax(fabs(d0), fabs(d1));
    if (!(m == m)) m = __longlong_as_double(0x7ff8000000000000ll);
    local = m;
  }
  block_max_store(local, I.upart + blockIdx.x);
}

// ---------------------------------------------------------------------------
// host launchers

static inline dim3 grid2(int64_t count, int nslots, int block = 256, int64_t cap = 1 << 20) {
  int64_t gx = (count + block - 1) / block;
  if (gx < 1) gx = 1;
  if (gx > cap) gx = cap;
  return dim3((unsigned)gx, (unsigned)nslots);
}

void launch_set_inst(hipStream_t st, Inst* dst, const Inst& src) { k_set_inst<<<1, 64, 0, st>>>(dst, src); }

void launch_zero_words(hipStream_t st, void* p, int64_t words) {
  if (words <= 0) return;
  k_zero_words<<<dim3((unsigned)((words + 255) / 256)), 256, 0, st>>>((unsigned*)p, words);
}

void launch_init(hipStream_t st, const Inst* const* insts, int nslots, int max_n, int flat) {
  k_init<<<grid2(max_n, nslots), 256, 0, st>>>(insts, flat);
}
void launch_start(hipStream_t st, const Inst* const* insts, int nslots) {
  k_start<<<dim3((unsigned)((nslots + 63) / 64)), 64, 0, st>>>(insts, nslots);
}
void launch_decide(hipStream_t st, const Inst* const* insts, int nslots, DevOpts o) {
  k_decide<<<dim3((unsigned)nslots), 256, 0, st>>>(insts, o);
}
void launch_gather_red(hipStream_t st, const Inst* const* insts, int nslots, Red* out) {
  k_gather_red<<<dim3((unsigned)((nslots + 63) / 64)), 64, 0, st>>>(insts, nslots, out);
}
void launch_mismatch(hipStream_t st, const Inst* const* insts, int nslots, int max_n, int max_heavy) {
  const dim3 g = grid2((int64_t)max_n * kMisLanes, nslots);
  k_mismatch<kMisLanes><<<dim3(g.x + (unsigned)max_heavy, g.y), 256, 0, st>>>(insts, max_heavy);
}

template <typename T>
void launch_fill(hipStream_t st, const Inst* const* insts, int nslots, int max_nu2, const int2* zero_work,
                 int nzero, int max_nnz) {
  if (nzero > 0) k_zero_chunks<T><<<dim3((unsigned)nzero), 256, 0, st>>>(insts, zero_work);
  const dim3 gj = grid2(max_nnz, nslots), gc = grid2(max_nu2, nslots);
  k_jfill<T><<<dim3(gj.x + gc.x, (unsigned)nslots), 256, 0, st>>>(insts, (int)gj.x);
}

int zero_chunk_values() { return ZCH; }

template <typename T>
void launch_kfill(hipStream_t st, const Inst* const* insts, int nslots, int max_nnz, int ilu) {
  k_kfill<T><<<grid2(max_nnz, nslots), 256, 0, st>>>(insts, ilu);
}

#define PF_GSWITCH(G, CALL)                         \
  switch (G) {                                      \
    case 1: { constexpr int GG = 1; CALL; } break;   \
    case 2: { constexpr int GG = 2; CALL; } break;   \
    case 4: { constexpr int GG = 4; CALL; } break;   \
    case 8: { constexpr int GG = 8; CALL; } break;   \
    case 16: { constexpr int GG = 16; CALL; } break; \
    case 32: { constexpr int GG = 32; CALL; } break; \
    default: { constexpr int GG = 64; CALL; } break; \
  }

template <typename T>
void launch_factor_cols(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int G, int wide) {
  if (nwork <= 0) return;
  if (wide) {
    PF_GSWITCH(G, (k_factor_cols<T, GG, 1024><<<dim3((unsigned)nwork), 1024, 0, st>>>(insts, work)));
  } else {
    PF_GSWITCH(G, (k_factor_cols<T, GG, 256><<<dim3((unsigned)nwork), 256, 0, st>>>(insts, work)));
  }
}

template <typename T>
void launch_tail_schur(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int G) {
  if (nwork <= 0) return;
  PF_GSWITCH(G, (k_tail_schur<T, GG><<<dim3((unsigned)nwork), 256, 0, st>>>(insts, work)));
}

template <typename T>
void launch_factor_cols_wave(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int G) {
  if (nwork <= 0) return;
  PF_GSWITCH(G, (k_factor_cols_wave<T, GG><<<dim3((unsigned)((nwork + 3) / 4)), 256, 0, st>>>(insts, work, nwork)));
}

template <typename T>
void launch_fwd_rows(hipStream_t st, const Inst* const* insts, const int2* work, int nwork, int G) {
  if (nwork <= 0) return;
  PF_GSWITCH(G, (k_fwd_rows<T, GG><<<dim3((unsigned)(((int64_t)nwork * GG + 255) / 256)), 256, 0, st>>>(
                    insts, work, nwork)));
}

template <typename T>
void launch_update(hipStream_t st, const Inst* const* insts, int nslots, int max_nu) {
  k_update<T><<<grid2(max_nu, nslots), 256, 0, st>>>(insts);
}

#define PF_INST(T)                                                                                         \
  template void launch_fill<T>(hipStream_t, const Inst* const*, int, int, const int2*, int, int);          \
  template void launch_factor_cols<T>(hipStream_t, const Inst* const*, const int2*, int, int, int);        \
  template void launch_tail_schur<T>(hipStream_t, const Inst* const*, const int2*, int, int);              \
  template void launch_factor_cols_wave<T>(hipStream_t, const Inst* const*, const int2*, int, int);        \
  template void launch_fwd_rows<T>(hipStream_t, const Inst* const*, const int2*, int, int);                \
  template void launch_update<T>(hipStream_t, const Inst* const*, int, int);                                \
  template void launch_kfill<T>(hipStream_t, const Inst* const*, int, int, int);

PF_INST(double)
PF_INST(float)

}  // namespace pfd
