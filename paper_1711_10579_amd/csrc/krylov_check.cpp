// Host self-check of the Newton-Krylov analysis (no device involved).
//
// Rebuilds the Krylov analysis of a case exactly as pf_create does and checks
// every index the Krylov kernels derive from it: the ordering, the block
// pattern, the Ybus-to-block map, the ILU(0) update lists, both level
// schedules and the block-Jacobi groups.  It then runs the block ILU(0) of a
// random diagonally dominant matrix on that pattern through the update lists
// in level order, and applies it through the two level schedules, as the
// kernels do.  Reported: the largest relative deviation of (L U) from A on
// the pattern (zero in exact arithmetic for ILU(0)) and the relative residual
// of L U z = v.  A test of the host analysis; the solve path never calls it.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pf_debug.h"
#include "analysis.hpp"
#include "internal.hpp"

namespace pfi {
pf_status validate_desc(const pf_case_desc* d);
}

using namespace pfi;

namespace {

struct Fail : std::runtime_error {
  using std::runtime_error::runtime_error;
};

struct B2 {
  double a = 0, b = 0, c = 0, d = 0;
};
B2 mul(const B2& x, const B2& y) {
  return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
B2 inv(const B2& m) {
  const double det = m.a * m.d - m.b * m.c;
  if (det == 0 || !std::isfinite(det)) throw Fail("zero pivot block in the ILU(0) replay");
  return {m.d / det, -m.b / det, -m.c / det, m.a / det};
}
double nrm(const B2& m) { return std::max(std::max(std::fabs(m.a), std::fabs(m.b)), std::max(std::fabs(m.c), std::fabs(m.d))); }

}  // namespace

extern "C" pf_status pf_debug_krylov_check(const pf_case_desc* d, uint64_t seed, double* ilu_dev,
                                           double* rel_residual, int64_t* checks) {
  if (!ilu_dev || !rel_residual || !checks) {
    set_error("pf_debug_krylov_check: NULL output");
    return PF_E_INVALID;
  }
  pf_status st = validate_desc(d);
  if (st != PF_OK) return st;
  const int n = d->n;
  int64_t nchk = 0;
  auto req = [&](bool ok, const char* what) {
    ++nchk;
    if (!ok) throw Fail(what);
  };
  try {
    pfh::GraphInput g;
    g.n_nodes = n;
    g.unknown.resize(n);
    g.adj.resize(n);
    for (int i = 0; i < n; ++i) {
      g.unknown[i] = d->bus_type[i] != PF_SLACK;
      for (int q = d->row_ptr[i]; q < d->row_ptr[i + 1]; ++q)
        if (d->col_idx[q] != i) g.adj[i].push_back(d->col_idx[q]);
    }
    const pfh::Analysis an = pfh::analyze(g, 0.5, 32, 64);
    const pfh::KAnalysis ka = pfh::analyze_krylov(an, n, d->row_ptr, d->col_idx, 32);
    std::vector<int> kmap;
    pfh::build_kmap(an, ka, n, d->row_ptr, d->col_idx, &kmap);
    const int nu = ka.nu;
    const int64_t nnz = ka.nnz();
    // ordering
    req((int)ka.p_of_r.size() == nu && (int)ka.r_of_p.size() == nu, "ordering size");
    for (int r = 0; r < nu; ++r) {
      req(ka.p_of_r[r] >= 0 && ka.p_of_r[r] < nu, "ordering entry out of range");
      req(ka.r_of_p[ka.p_of_r[r]] == r, "ordering not a permutation");
    }
    // pattern: sorted, in range, diagonal, symmetric
    req(ka.row_ptr[0] == 0 && ka.row_ptr[nu] == nnz, "row pointer ends");
    std::vector<std::vector<int>> rows(nu);
    for (int r = 0; r < nu; ++r) {
      req(ka.row_ptr[r + 1] > ka.row_ptr[r], "empty row");
      for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q) {
        req(ka.col[q] >= 0 && ka.col[q] < nu, "column out of range");
        if (q > ka.row_ptr[r]) req(ka.col[q] > ka.col[q - 1], "columns not increasing");
        rows[r].push_back(ka.col[q]);
      }
      req(ka.diag[r] >= ka.row_ptr[r] && ka.diag[r] < ka.row_ptr[r + 1] && ka.col[ka.diag[r]] == r, "diagonal");
    }
    auto find = [&](int r, int c) -> int {
      auto it = std::lower_bound(rows[r].begin(), rows[r].end(), c);
      return (it != rows[r].end() && *it == c) ? ka.row_ptr[r] + (int)(it - rows[r].begin()) : -1;
    };
    for (int r = 0; r < nu; ++r)
      for (int c : rows[r]) req(find(c, r) >= 0, "pattern not symmetric");
    // Ybus -> block map: a bijection onto the pattern
    std::vector<int> hit(nnz, 0);
    for (int i = 0; i < n; ++i)
      for (int q = d->row_ptr[i]; q < d->row_ptr[i + 1]; ++q) {
        const int pi = an.pos_of_node[i], pj = an.pos_of_node[d->col_idx[q]];
        if (pi < 0 || pj < 0) {
          req(kmap[q] == -1, "map of an entry without unknowns");
          continue;
        }
        req(kmap[q] == find(ka.r_of_p[pi], ka.r_of_p[pj]), "map points at the wrong block");
        hit[kmap[q]]++;
      }
    for (int64_t q = 0; q < nnz; ++q) req(hit[q] == 1, "block not hit exactly once by the map");
    // ILU(0) update lists: exactly the pairs (r,j) in row r and (k,j) in row k, j > k
    for (int r = 0; r < nu; ++r)
      for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q) {
        const int k = ka.col[q];
        std::vector<std::pair<int, int>> want;
        if (q < ka.diag[r])
          for (int s = ka.diag[k] + 1; s < ka.row_ptr[k + 1]; ++s) {
            const int t = find(r, ka.col[s]);
            if (t >= 0) want.emplace_back(t, s);
          }
        req(ka.up_ptr[q + 1] - ka.up_ptr[q] == (int)want.size(), "update list length");
        for (int u = ka.up_ptr[q], w = 0; u < ka.up_ptr[q + 1]; ++u, ++w)
          req(ka.up_t[u] == want[w].first && ka.up_s[u] == want[w].second, "update list entry");
      }
    // level schedules
    auto check_levels = [&](const std::vector<int>& ptr, const std::vector<int>& lr, bool upper) {
      std::vector<int> lev(nu, -1);
      req(ptr.front() == 0 && ptr.back() == nu && (int)lr.size() == nu, "level list size");
      for (size_t l = 0; l + 1 < ptr.size(); ++l)
        for (int k = ptr[l]; k < ptr[l + 1]; ++k) {
          req(lr[k] >= 0 && lr[k] < nu && lev[lr[k]] < 0, "level rows not a permutation");
          lev[lr[k]] = (int)l;
        }
      for (int r = 0; r < nu; ++r)
        for (int c : rows[r])
          if (upper ? c > r : c < r) req(lev[c] < lev[r], "dependency not in an earlier level");
    };
    check_levels(ka.lev_ptr, ka.lev_rows, false);
    check_levels(ka.ulev_ptr, ka.ulev_rows, true);
    // block-Jacobi groups: a partition into connected groups of <= 32 nodes
    {
      std::vector<int> grp(nu, -1);
      req(ka.bj_ptr.front() == 0 && ka.bj_ptr.back() == nu, "group list size");
      for (int b = 0; b < ka.nblocks(); ++b) {
        const int s = ka.bj_ptr[b + 1] - ka.bj_ptr[b];
        req(s >= 1 && s <= 32, "group size");
        req(ka.bj_off[b + 1] - ka.bj_off[b] == 4LL * s * s, "group inverse offset");
        for (int a = 0; a < s; ++a) {
          const int r = ka.bj_rows[ka.bj_ptr[b] + a];
          req(r >= 0 && r < nu && grp[r] < 0, "group rows not a partition");
          grp[r] = b;
          req(ka.bj_loc[r] == a, "local index of a group row");
        }
        std::vector<char> seen(s, 0);
        std::deque<int> q{ka.bj_rows[ka.bj_ptr[b]]};
        seen[0] = 1;
        int reached = 1;
        while (!q.empty()) {
          const int u = q.front();
          q.pop_front();
          for (int c : rows[u])
            if (grp[c] == b && !seen[ka.bj_loc[c]]) {
              seen[ka.bj_loc[c]] = 1;
              ++reached;
              q.push_back(c);
            }
        }
        req(reached == s, "group not connected");
      }
    }
    // numeric replay: block ILU(0) through the lists, in level order
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    std::vector<B2> A(nnz), P;
    for (int r = 0; r < nu; ++r) {
      double off = 0;
      for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q)
        if (q != ka.diag[r]) {
          A[q] = {U(rng), U(rng), U(rng), U(rng)};
          off += nrm(A[q]);
        }
      A[ka.diag[r]] = {2 * off + 2 + U(rng), 0.5 * U(rng), 0.5 * U(rng), 2 * off + 2 + U(rng)};
    }
    P = A;
    std::vector<B2> Dinv(nu);
    for (size_t l = 0; l + 1 < ka.lev_ptr.size(); ++l)
      for (int k = ka.lev_ptr[l]; k < ka.lev_ptr[l + 1]; ++k) {
        const int r = ka.lev_rows[k];
        for (int q = ka.row_ptr[r]; q < ka.diag[r]; ++q) {
          const B2 L = mul(P[q], Dinv[ka.col[q]]);
          P[q] = L;
          for (int u = ka.up_ptr[q]; u < ka.up_ptr[q + 1]; ++u) {
            const B2 t = mul(L, P[ka.up_s[u]]);
            B2& a = P[ka.up_t[u]];
            a.a -= t.a;
            a.b -= t.b;
            a.c -= t.c;
            a.d -= t.d;
          }
        }
        Dinv[r] = inv(P[ka.diag[r]]);
      }
    // (L U)(r, c) = sum over k <= min(r, c) of L(r, k) U(k, c), L(r, r) = I
    double dev = 0, amax = 0;
    for (int r = 0; r < nu; ++r)
      for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q) {
        const int c = ka.col[q];
        B2 s;
        for (int p = ka.row_ptr[r]; p < ka.row_ptr[r + 1]; ++p) {
          const int k = ka.col[p];
          if (k > std::min(r, c)) break;
          const int kc = find(k, c);
          if (kc < 0) continue;
          const B2 t = k == r ? P[kc] : mul(P[p], P[kc]);
          s.a += t.a;
          s.b += t.b;
          s.c += t.c;
          s.d += t.d;
        }
        dev = std::max(dev, nrm({s.a - A[q].a, s.b - A[q].b, s.c - A[q].c, s.d - A[q].d}));
        amax = std::max(amax, nrm(A[q]));
      }
    *ilu_dev = amax > 0 ? dev / amax : dev;
    // apply through both level schedules, then check L (U z) = v
    std::vector<double> v(2 * (size_t)nu), z(2 * (size_t)nu);
    for (auto& x : v) x = U(rng);
    for (size_t l = 0; l + 1 < ka.lev_ptr.size(); ++l)
      for (int k = ka.lev_ptr[l]; k < ka.lev_ptr[l + 1]; ++k) {
        const int r = ka.lev_rows[k];
        double y0 = v[2 * r], y1 = v[2 * r + 1];
        for (int q = ka.row_ptr[r]; q < ka.diag[r]; ++q) {
          const int c = ka.col[q];
          y0 -= P[q].a * z[2 * c] + P[q].b * z[2 * c + 1];
          y1 -= P[q].c * z[2 * c] + P[q].d * z[2 * c + 1];
        }
        z[2 * r] = y0;
        z[2 * r + 1] = y1;
      }
    for (size_t l = 0; l + 1 < ka.ulev_ptr.size(); ++l)
      for (int k = ka.ulev_ptr[l]; k < ka.ulev_ptr[l + 1]; ++k) {
        const int r = ka.ulev_rows[k];
        double s0 = z[2 * r], s1 = z[2 * r + 1];
        for (int q = ka.diag[r] + 1; q < ka.row_ptr[r + 1]; ++q) {
          const int c = ka.col[q];
          s0 -= P[q].a * z[2 * c] + P[q].b * z[2 * c + 1];
          s1 -= P[q].c * z[2 * c] + P[q].d * z[2 * c + 1];
        }
        const B2& D = Dinv[r];
        z[2 * r] = D.a * s0 + D.b * s1;
        z[2 * r + 1] = D.c * s0 + D.d * s1;
      }
    std::vector<double> uz(2 * (size_t)nu, 0.0);
    for (int r = 0; r < nu; ++r)
      for (int q = ka.diag[r]; q < ka.row_ptr[r + 1]; ++q) {
        const int c = ka.col[q];
        uz[2 * r] += P[q].a * z[2 * c] + P[q].b * z[2 * c + 1];
        uz[2 * r + 1] += P[q].c * z[2 * c] + P[q].d * z[2 * c + 1];
      }
    double res = 0, vn = 0;
    for (int r = 0; r < nu; ++r) {
      double l0 = uz[2 * r], l1 = uz[2 * r + 1];
      for (int q = ka.row_ptr[r]; q < ka.diag[r]; ++q) {
        const int c = ka.col[q];
        l0 += P[q].a * uz[2 * c] + P[q].b * uz[2 * c + 1];
        l1 += P[q].c * uz[2 * c] + P[q].d * uz[2 * c + 1];
      }
      res = std::max(res, std::max(std::fabs(l0 - v[2 * r]), std::fabs(l1 - v[2 * r + 1])));
      vn = std::max(vn, std::max(std::fabs(v[2 * r]), std::fabs(v[2 * r + 1])));
    }
    *rel_residual = vn > 0 ? res / vn : res;
  } catch (const std::exception& ex) {
    set_error(std::string("pf_debug_krylov_check: ") + ex.what());
    *checks = nchk;
    return PF_E_INVALID;
  }
  *checks = nchk;
  return PF_OK;
}
