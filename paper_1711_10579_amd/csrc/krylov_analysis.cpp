// Host analysis of the Newton-Krylov inner solve (Sec. III-B): ordering,
// block pattern, ILU(0) update lists, levels and block-Jacobi blocks.

#include <algorithm>
#include <deque>
#include <stdexcept>

#include "analysis.hpp"

namespace pfh {

namespace {

// breadth-first level structure from s inside the component; returns the
// eccentricity and fills last with the vertices of the deepest level
int bfs_levels(const std::vector<std::vector<int>>& adj, int s, std::vector<int>* mark, int stamp,
               std::vector<int>* last) {
  std::vector<int> cur{s}, next;
  (*mark)[s] = stamp;
  int depth = 0;
  for (;;) {
    next.clear();
    for (int u : cur)
      for (int w : adj[u])
        if ((*mark)[w] != stamp) {
          (*mark)[w] = stamp;
          next.push_back(w);
        }
    if (next.empty()) break;
    cur.swap(next);
    ++depth;
  }
  *last = cur;
  return depth;
}

}  // namespace

std::vector<int> rcm_order(const std::vector<std::vector<int>>& adj) {
  const int n = (int)adj.size();
  std::vector<int> deg(n), order;
  order.reserve(n);
  for (int v = 0; v < n; ++v) deg[v] = (int)adj[v].size();
  std::vector<char> seen(n, 0);
  std::vector<int> mark(n, -1), comp;
  int stamp = 0;
  for (int root = 0; root < n; ++root) {
    if (seen[root]) continue;
    // the component of root, and its vertex of smallest degree
    comp.clear();
    {
      std::deque<int> q{root};
      ++stamp;
      mark[root] = stamp;
      while (!q.empty()) {
        int u = q.front();
        q.pop_front();
        comp.push_back(u);
        for (int w : adj[u])
          if (mark[w] != stamp) {
            mark[w] = stamp;
            q.push_back(w);
          }
      }
    }
    int x = comp[0];
    for (int v : comp)
      if (deg[v] < deg[x] || (deg[v] == deg[x] && v < x)) x = v;
    // pseudo-peripheral vertex: move to a smallest-degree vertex of the
    // deepest level while the eccentricity grows
    std::vector<int> last;
    int ecc = bfs_levels(adj, x, &mark, ++stamp, &last);
    for (int round = 0; round < 16; ++round) {
      int y = last[0];
      for (int v : last)
        if (deg[v] < deg[y] || (deg[v] == deg[y] && v < y)) y = v;
      std::vector<int> ly;
      int ey = bfs_levels(adj, y, &mark, ++stamp, &ly);
      if (ey <= ecc) break;
      x = y;
      ecc = ey;
      last.swap(ly);
    }
    // Cuthill-McKee from x
    std::deque<int> q{x};
    seen[x] = 1;
    std::vector<int> nb;
    while (!q.empty()) {
      int u = q.front();
      q.pop_front();
      order.push_back(u);
      nb.clear();
      for (int w : adj[u])
        if (!seen[w]) {
          seen[w] = 1;
          nb.push_back(w);
        }
      std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; });
      for (int w : nb) q.push_back(w);
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

KAnalysis analyze_krylov(const Analysis& an, int n, const int* row_ptr, const int* col, int bj_cap) {
  KAnalysis ka;
  const int nu = an.nu;
  ka.nu = nu;
  // node graph over factor positions
  std::vector<std::vector<int>> adj(nu);
  for (int i = 0; i < n; ++i) {
    const int p = an.pos_of_node[i];
    if (p < 0) continue;
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      const int j = col[q];
      const int pj = an.pos_of_node[j];
      if (j != i && pj >= 0) adj[p].push_back(pj);
    }
  }
  for (auto& a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  ka.p_of_r = rcm_order(adj);
  ka.r_of_p.assign(nu, -1);
  for (int r = 0; r < nu; ++r) ka.r_of_p[ka.p_of_r[r]] = r;
  // block pattern in Krylov order
  ka.row_ptr.assign(nu + 1, 0);
  ka.diag.assign(nu, -1);
  for (int r = 0; r < nu; ++r) ka.row_ptr[r + 1] = ka.row_ptr[r] + 1 + (int)adj[ka.p_of_r[r]].size();
  ka.col.resize(ka.row_ptr[nu]);
  for (int r = 0; r < nu; ++r) {
    int* c = ka.col.data() + ka.row_ptr[r];
    int k = 0;
    c[k++] = r;
    for (int pj : adj[ka.p_of_r[r]]) c[k++] = ka.r_of_p[pj];
    std::sort(c, c + k);
    ka.diag[r] = ka.row_ptr[r] + (int)(std::lower_bound(c, c + k, r) - c);
  }
  // ILU(0) update lists
  ka.up_ptr.assign(ka.nnz() + 1, 0);
  std::vector<int> where(nu, -1);
  for (int r = 0; r < nu; ++r) {
    for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q) where[ka.col[q]] = q;
    for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q) {
      if (q < ka.diag[r]) {
        const int k = ka.col[q];
        for (int s = ka.diag[k] + 1; s < ka.row_ptr[k + 1]; ++s) {
          const int t = where[ka.col[s]];
          if (t >= 0) {
            ka.up_t.push_back(t);
            ka.up_s.push_back(s);
          }
        }
      }
      ka.up_ptr[q + 1] = (int)ka.up_t.size();
    }
    for (int q = ka.row_ptr[r]; q < ka.row_ptr[r + 1]; ++q) where[ka.col[q]] = -1;
  }
  // levels
  auto group = [&](const std::vector<int>& lev, std::vector<int>* ptr, std::vector<int>* rows) {
    int nl = 0;
    for (int v : lev) nl = std::max(nl, v + 1);
    ptr->assign(nl + 1, 0);
    for (int v : lev) (*ptr)[v + 1]++;
    for (int l = 0; l < nl; ++l) (*ptr)[l + 1] += (*ptr)[l];
    rows->resize(lev.size());
    std::vector<int> fill(ptr->begin(), ptr->end() - 1);
    for (int r = 0; r < (int)lev.size(); ++r) (*rows)[fill[lev[r]]++] = r;
  };
  {
    std::vector<int> lev(nu, 0);
    for (int r = 0; r < nu; ++r)
      for (int q = ka.row_ptr[r]; q < ka.diag[r]; ++q) lev[r] = std::max(lev[r], lev[ka.col[q]] + 1);
    group(lev, &ka.lev_ptr, &ka.lev_rows);
    std::vector<int> ulev(nu, 0);
    for (int r = nu - 1; r >= 0; --r)
      for (int q = ka.diag[r] + 1; q < ka.row_ptr[r + 1]; ++q) ulev[r] = std::max(ulev[r], ulev[ka.col[q]] + 1);
    group(ulev, &ka.ulev_ptr, &ka.ulev_rows);
  }
  // block-Jacobi blocks
  if (bj_cap < 1 || bj_cap > 32) throw std::invalid_argument("block-Jacobi block size must be 1..32 nodes");
  ka.bj_loc.assign(nu, -1);
  ka.bj_ptr.assign(1, 0);
  ka.bj_off.assign(1, 0);
  for (int seed = 0; seed < nu; ++seed) {
    if (ka.bj_loc[seed] >= 0) continue;
    const int start = (int)ka.bj_rows.size();
    std::deque<int> q{seed};
    ka.bj_loc[seed] = 0;
    ka.bj_rows.push_back(seed);
    int count = 1;
    while (!q.empty() && count < bj_cap) {
      const int u = q.front();
      q.pop_front();
      for (int e = ka.row_ptr[u]; e < ka.row_ptr[u + 1] && count < bj_cap; ++e) {
        const int w = ka.col[e];
        if (ka.bj_loc[w] < 0) {
          ka.bj_loc[w] = count++;
          ka.bj_rows.push_back(w);
          q.push_back(w);
        }
      }
    }
    const int s = (int)ka.bj_rows.size() - start;
    ka.bj_ptr.push_back((int)ka.bj_rows.size());
    ka.bj_off.push_back(ka.bj_off.back() + 4LL * s * s);
    ka.bj_max = std::max(ka.bj_max, s);
  }
  return ka;
}

void build_kmap(const Analysis& an, const KAnalysis& ka, int n, const int* row_ptr, const int* col,
                std::vector<int>* kmap) {
  kmap->assign(row_ptr[n], -1);
  for (int i = 0; i < n; ++i) {
    const int pi = an.pos_of_node[i];
    if (pi < 0) continue;
    const int r = ka.r_of_p[pi];
    const int* c0 = ka.col.data() + ka.row_ptr[r];
    const int* c1 = ka.col.data() + ka.row_ptr[r + 1];
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      const int pj = an.pos_of_node[col[q]];
      if (pj < 0) continue;
      const int rc = ka.r_of_p[pj];
      const int* f = std::lower_bound(c0, c1, rc);
      if (f == c1 || *f != rc) throw std::logic_error("Krylov pattern misses a Ybus entry");
      (*kmap)[q] = (int)(f - ka.col.data());
    }
  }
}

}  // namespace pfh
