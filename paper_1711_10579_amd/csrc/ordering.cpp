// Fill-reducing ordering of the node graph (the paper limits fill-in with an
// approximate minimum degree ordering, Sec. III-A).
//
// Quotient-graph minimum degree with approximate external degrees in the
// style of Amestoy, Davis and Duff's AMD: eliminated nodes become elements,
// elements adjacent to a pivot are absorbed into the new element, and a
// variable's degree is bounded by |A_i| + |L_p \ i| + sum_e |L_e \ L_p|.
// Elimination stops early once the remaining graph is nearly complete: those
// nodes form the dense trailing block that the GPU factors as one dense
// matrix.

#include "analysis.hpp"

#include <algorithm>
#include <set>
#include <stdexcept>

namespace pfh {

Ordering min_degree_order(int n, const std::vector<std::vector<int>>& adj,
                          double dense_switch, int min_dense) {
  Ordering out;
  out.perm.reserve(n);
  if (n == 0) {
    out.n_sparse = 0;
    return out;
  }
  std::vector<std::vector<int>> av(n);   // variable neighbours
  std::vector<std::vector<int>> ae(n);   // adjacent elements
  std::vector<std::vector<int>> le(n);   // element boundary (for elements)
  std::vector<char> is_elem(n, 0), dead(n, 0), alive_var(n, 1);
  std::vector<int> deg(n);
  for (int i = 0; i < n; ++i) {
    av[i] = adj[i];
    deg[i] = (int)av[i].size();
  }
  std::set<std::pair<int, int>> heap;
  for (int i = 0; i < n; ++i) heap.insert({deg[i], i});

  std::vector<int> mark(n, -1), wflag(n, -1), w(n, 0), inlp(n, -1);
  int remaining = n;
  int stamp = 0;
  while (remaining > 0) {
    auto it = heap.begin();
    int p = it->second;
    int dp = it->first;
    // dense switch: the rest of the graph is (almost) a clique
    if (remaining >= min_dense && dp >= dense_switch * (remaining - 1)) break;
    heap.erase(it);
    ++stamp;
    // L_p = (A_p u  U_{e in E_p} L_e) \ {p}
    std::vector<int> lp;
    mark[p] = stamp;
    for (int v : av[p])
      if (alive_var[v] && mark[v] != stamp) {
        mark[v] = stamp;
        lp.push_back(v);
      }
    for (int e : ae[p]) {
      if (dead[e]) continue;
      for (int v : le[e])
        if (alive_var[v] && mark[v] != stamp) {
          mark[v] = stamp;
          lp.push_back(v);
        }
      dead[e] = 1;  // absorbed into p
      le[e].clear();
      le[e].shrink_to_fit();
    }
    // p becomes an element
    alive_var[p] = 0;
    is_elem[p] = 1;
    av[p].clear();
    av[p].shrink_to_fit();
    ae[p].clear();
    ae[p].shrink_to_fit();
    le[p] = lp;
    out.perm.push_back(p);
    --remaining;
    for (int v : lp) inlp[v] = stamp;

    // update neighbour lists of every variable in L_p
    for (int i : lp) {
      auto& a = av[i];
      size_t k = 0;
      for (int v : a)
        if (alive_var[v] && inlp[v] != stamp && v != p) a[k++] = v;
      a.resize(k);
      auto& e = ae[i];
      k = 0;
      for (int x : e)
        if (!dead[x] && x != p) e[k++] = x;
      e.resize(k);
      e.push_back(p);
    }
    // |L_e \ L_p| for every element adjacent to L_p
    for (int i : lp)
      for (int x : ae[i]) {
        if (x == p) continue;
        if (wflag[x] != stamp) {
          int cnt = 0;
          auto& l = le[x];
          size_t k = 0;
          for (int v : l)
            if (alive_var[v]) {
              l[k++] = v;
              ++cnt;
            }
          l.resize(k);
          w[x] = cnt;
          wflag[x] = stamp;
        }
        w[x] -= 1;
      }
    int lsz = (int)lp.size();
    for (int i : lp) {
      long d = (long)av[i].size() + (lsz - 1);
      for (int x : ae[i])
        if (x != p) d += w[x];
      long bound = remaining - 1;
      long nd = std::min(d, bound);
      nd = std::min<long>(nd, (long)deg[i] + lsz);
      if (nd < 0) nd = 0;
      heap.erase({deg[i], i});
      deg[i] = (int)nd;
      heap.insert({deg[i], i});
    }
  }
  out.n_sparse = (int)out.perm.size();
  // the remaining nodes form the dense tail, in ascending degree order
  std::vector<std::pair<int, int>> rest(heap.begin(), heap.end());
  for (auto& pr : rest) out.perm.push_back(pr.second);
  if ((int)out.perm.size() != n) throw std::runtime_error("ordering lost nodes");
  return out;
}

}  // namespace pfh
