// Symbolic analysis: ordering, block LU structure, levels and update lists.

#include "analysis.hpp"

#include <algorithm>
#include <cstdio>
#include <numeric>
#include <stdexcept>

namespace pfh {

namespace {

inline int find_pos(const int* b, int len, int v) {
  const int* e = b + len;
  const int* it = std::lower_bound(b, e, v);
  if (it == e || *it != v) return -1;
  return (int)(it - b);
}

}  // namespace

std::string Analysis::summary() const {
  char buf[512];
  int nlev = (int)col_lev_ptr.size() - 1;
  snprintf(buf, sizeof buf,
           "nu=%d ns=%d nt=%d nnzl=%lld levels=%d upd=%zu tail_upd=%zu "
           "flops(sparse=%.3g schur=%.3g dense=%.3g)",
           nu, ns, nt, (long long)nnzl, nlev, upd_l.size(), tail_l.size(), flops_sparse,
           flops_tail_schur, flops_dense);
  return buf;
}

Analysis analyze(const GraphInput& g, double dense_switch, int min_dense, int tail_align) {
  Analysis A;
  const int n = g.n_nodes;
  std::vector<int> loc(n, -1), glob;
  for (int v = 0; v < n; ++v)
    if (g.unknown[v]) {
      loc[v] = (int)glob.size();
      glob.push_back(v);
    }
  const int nu = (int)glob.size();
  A.nu = nu;
  std::vector<std::vector<int>> adj(nu);
  for (int u = 0; u < nu; ++u) {
    for (int w : g.adj[glob[u]]) {
      int lw = loc[w];
      if (lw >= 0 && lw != u) adj[u].push_back(lw);
    }
    std::sort(adj[u].begin(), adj[u].end());
    adj[u].erase(std::unique(adj[u].begin(), adj[u].end()), adj[u].end());
  }

  Ordering ord = min_degree_order(nu, adj, dense_switch, min_dense);
  const int ns = ord.n_sparse;
  const int nt = nu - ns;
  A.ns = ns;
  A.nt = nt;
  A.ldt = nt == 0 ? 0 : ((2 * nt + tail_align - 1) / tail_align) * tail_align;
  A.node_of_pos.resize(nu);
  A.pos_of_node.assign(n, -1);
  std::vector<int> pos_of_loc(nu);
  for (int p = 0; p < nu; ++p) {
    A.node_of_pos[p] = glob[ord.perm[p]];
    pos_of_loc[ord.perm[p]] = p;
    A.pos_of_node[glob[ord.perm[p]]] = p;
  }

  // symbolic factorisation of the sparse columns by merging the structures
  // of elimination-tree children
  std::vector<std::vector<int>> R(ns);
  std::vector<std::vector<int>> kids(ns);
  A.parent.assign(ns, -1);
  for (int j = 0; j < ns; ++j) {
    std::vector<int>& s = R[j];
    for (int w : adj[ord.perm[j]]) {
      int pw = pos_of_loc[w];
      if (pw > j) s.push_back(pw);
    }
    for (int c : kids[j])
      for (int r : R[c])
        if (r != j) s.push_back(r);
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    if (!s.empty() && s[0] < ns) {
      A.parent[j] = s[0];
      kids[s[0]].push_back(j);
    }
  }
  A.colptr.assign(ns + 1, 0);
  for (int j = 0; j < ns; ++j) A.colptr[j + 1] = A.colptr[j] + (int)R[j].size();
  A.nnzl = A.colptr[ns];
  A.rowidx.resize(A.nnzl);
  for (int j = 0; j < ns; ++j) std::copy(R[j].begin(), R[j].end(), A.rowidx.begin() + A.colptr[j]);
  const int* cp = A.colptr.data();
  const int* ri = A.rowidx.data();
  auto len = [&](int j) { return cp[j + 1] - cp[j]; };
  const int64_t nnzl = A.nnzl;
  auto Lblk = [&](int k, int a) { return ns + cp[k] + a; };
  auto Ublk = [&](int k, int b) { return (int)(ns + nnzl + cp[k] + b); };

  // column levels = height in the elimination tree
  std::vector<int> lev(ns, 0);
  int nlev = 0;
  for (int j = 0; j < ns; ++j) {
    int l = 0;
    for (int c : kids[j]) l = std::max(l, lev[c] + 1);
    lev[j] = l;
    nlev = std::max(nlev, l + 1);
  }
  if (ns == 0) nlev = 0;
  A.col_lev_ptr.assign(nlev + 1, 0);
  for (int j = 0; j < ns; ++j) A.col_lev_ptr[lev[j] + 1]++;
  for (int l = 0; l < nlev; ++l) A.col_lev_ptr[l + 1] += A.col_lev_ptr[l];
  A.col_order.resize(ns);
  {
    std::vector<int> fill(A.col_lev_ptr.begin(), A.col_lev_ptr.end() - 1);
    for (int j = 0; j < ns; ++j) A.col_order[fill[lev[j]]++] = j;
  }

  // update lists: for every sparse column k and every pair (i, j) of its
  // structure, target (i, j) receives L(i,k) U(k,j); ascending k per target
  const int64_t ntg = (int64_t)ns + 2 * nnzl;
  std::vector<int64_t> cnt(ntg + 1, 0);
  std::vector<int> tcnt((size_t)nt * nt, 0);
  auto target_of = [&](int i, int j) -> int64_t {
    if (i == j) return (int64_t)i + 2LL * cp[i];
    if (i > j) {
      int p = find_pos(ri + cp[j], len(j), i);
      if (p < 0) throw std::runtime_error("symbolic: missing L entry");
      return (int64_t)j + 2LL * cp[j] + 1 + len(j) + p;
    }
    int p = find_pos(ri + cp[i], len(i), j);
    if (p < 0) throw std::runtime_error("symbolic: missing U entry");
    return (int64_t)i + 2LL * cp[i] + 1 + p;
  };
  for (int k = 0; k < ns; ++k) {
    const int lk = len(k);
    const int* rk = ri + cp[k];
    for (int a = 0; a < lk; ++a)
      for (int b = 0; b < lk; ++b) {
        int i = rk[a], j = rk[b];
        if (i >= ns && j >= ns)
          tcnt[(size_t)(i - ns) * nt + (j - ns)]++;
        else
          cnt[target_of(i, j) + 1]++;
      }
  }
  for (int64_t t = 0; t < ntg; ++t) cnt[t + 1] += cnt[t];
  A.uptr = cnt;
  A.upd_l.resize(cnt[ntg]);
  A.upd_u.resize(cnt[ntg]);
  std::vector<int> tidx((size_t)nt * nt, -1);
  int ntt = 0;
  for (size_t q = 0; q < tcnt.size(); ++q)
    if (tcnt[q]) tidx[q] = ntt++;
  A.tail_tgt.resize(ntt);
  A.tail_uptr.assign(ntt + 1, 0);
  for (size_t q = 0; q < tcnt.size(); ++q)
    if (tcnt[q]) {
      A.tail_tgt[tidx[q]] = (int)q;
      A.tail_uptr[tidx[q] + 1] = tcnt[q];
    }
  for (int t = 0; t < ntt; ++t) A.tail_uptr[t + 1] += A.tail_uptr[t];
  A.tail_l.resize(A.tail_uptr[ntt]);
  A.tail_u.resize(A.tail_uptr[ntt]);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    std::vector<int64_t> tfill(A.tail_uptr.begin(), A.tail_uptr.end() - 1);
    for (int k = 0; k < ns; ++k) {
      const int lk = len(k);
      const int* rk = ri + cp[k];
      for (int a = 0; a < lk; ++a)
        for (int b = 0; b < lk; ++b) {
          int i = rk[a], j = rk[b];
          if (i >= ns && j >= ns) {
            int t = tidx[(size_t)(i - ns) * nt + (j - ns)];
            int64_t s = tfill[t]++;
            A.tail_l[s] = Lblk(k, a);
            A.tail_u[s] = Ublk(k, b);
          } else {
            int64_t s = fill[target_of(i, j)]++;
            A.upd_l[s] = Lblk(k, a);
            A.upd_u[s] = Ublk(k, b);
          }
        }
    }
  }

  // row lists of L for the forward solve (all rows, sparse and tail)
  A.lrow_ptr.assign(nu + 1, 0);
  for (int64_t q = 0; q < nnzl; ++q) A.lrow_ptr[ri[q] + 1]++;
  for (int i = 0; i < nu; ++i) A.lrow_ptr[i + 1] += A.lrow_ptr[i];
  A.lrow_blk.resize(nnzl);
  A.lrow_col.resize(nnzl);
  {
    std::vector<int> fill(A.lrow_ptr.begin(), A.lrow_ptr.end() - 1);
    for (int k = 0; k < ns; ++k)
      for (int a = 0; a < len(k); ++a) {
        int i = ri[cp[k] + a];
        int s = fill[i]++;
        A.lrow_blk[s] = Lblk(k, a);
        A.lrow_col[s] = k;
      }
  }
  // forward levels over sparse rows equal the column levels
  A.fwd_lev_ptr = A.col_lev_ptr;
  A.fwd_rows = A.col_order;
  // backward levels: row i needs x_j for j in its structure
  std::vector<int> blev(ns, 0);
  int nb = 0;
  for (int i = ns - 1; i >= 0; --i) {
    int l = 0;
    for (int q = cp[i]; q < cp[i + 1]; ++q)
      if (ri[q] < ns) l = std::max(l, blev[ri[q]] + 1);
    blev[i] = l;
    nb = std::max(nb, l + 1);
  }
  if (ns == 0) nb = 0;
  A.bwd_lev_ptr.assign(nb + 1, 0);
  for (int i = 0; i < ns; ++i) A.bwd_lev_ptr[blev[i] + 1]++;
  for (int l = 0; l < nb; ++l) A.bwd_lev_ptr[l + 1] += A.bwd_lev_ptr[l];
  A.bwd_rows.resize(ns);
  {
    std::vector<int> fill(A.bwd_lev_ptr.begin(), A.bwd_lev_ptr.end() - 1);
    for (int i = 0; i < ns; ++i) A.bwd_rows[fill[blev[i]]++] = i;
  }

  A.flops_sparse = 16.0 * (double)A.upd_l.size() + 40.0 * (double)(ns + nnzl);
  A.flops_tail_schur = 16.0 * (double)A.tail_l.size();
  double m2 = 2.0 * nt;
  A.flops_dense = (2.0 / 3.0) * m2 * m2 * m2;
  return A;
}

void build_jmap(const Analysis& an, int n, const int* row_ptr, const int* col, std::vector<int>* yrow_out,
                std::vector<int>* jmap_out) {
  const int nnz = row_ptr[n];
  std::vector<int>& jmap = *jmap_out;
  std::vector<int>& yrow = *yrow_out;
  jmap.assign(nnz, -1);
  yrow.assign(nnz, 0);
  const int ns = an.ns, nt = an.nt;
  for (int i = 0; i < n; ++i)
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      yrow[q] = i;
      int j = col[q];
      int pi = an.pos_of_node[i], pj = an.pos_of_node[j];
      if (pi < 0 || pj < 0) continue;
      int code;
      if (pi >= ns && pj >= ns) {
        code = -2 - ((pi - ns) * nt + (pj - ns));
      } else if (pi == pj) {
        code = pi;
      } else if (pi > pj) {
        int p = find_pos(an.rowidx.data() + an.colptr[pj], an.colptr[pj + 1] - an.colptr[pj], pi);
        if (p < 0) throw std::runtime_error("jmap: Ybus entry outside the L structure");
        code = ns + an.colptr[pj] + p;
      } else {
        int p = find_pos(an.rowidx.data() + an.colptr[pi], an.colptr[pi + 1] - an.colptr[pi], pj);
        if (p < 0) throw std::runtime_error("jmap: Ybus entry outside the U structure");
        code = (int)(ns + an.nnzl + an.colptr[pi] + p);
      }
      jmap[q] = code;
    }
}

}  // namespace pfh
