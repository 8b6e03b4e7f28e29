// Host self-check of the symbolic analysis (no device involved).
//
// Replays, on the CPU and in the same order, every index the device kernels
// will compute from the analysis of a case: the Ybus-to-factor map, the
// column levels with their update lists, the Schur lists of the dense block,
// the row lists of both triangular solves.  Each index is bounds-checked and
// each dependency is checked against the level schedule.  It then factors a
// random diagonally dominant 2x2-block matrix with the Ybus pattern through
// that schedule, solves one system and reports the relative residual.  This
// is a test of the host analysis; the solve path never calls it.

#include <algorithm>
#include <map>
#include <tuple>
#include <set>
#include <cmath>
#include <cstdint>
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

void req(bool ok, const char* what) {
  if (!ok) throw Fail(what);
}

// Replays the dense block's launch plan over instances of dense orders Ms
// on a tile state machine.  Tiles are named by the (row, column) offsets the
// kernels compute; updates are counted on the 64-aligned block holding a
// tile's first element (only the last, partial step starts a tile off the
// grid: its right-hand-side tile, which earlier steps updated as part of the
// diagonal block).  An aligned block (a, b) needs the trailing updates of
// steps 0..min(a,b)-1, then panel min(a,b) finishes it.  Every item of a
// launch is checked against the state before the launch (items of a launch
// run concurrently): a panel item needs its tile and the diagonal tile
// updated through the previous step; an update item of step k needs its tile
// updated through step k-1 and the L and U tiles of panel k finished.  The
// one ordering inside a launch is the row flag: a panel item's update of its
// row's tile in the next block column reads that tile and the block row's
// tile there after the flags of their rows, each set by the one flagged item
// of that row, listed earlier, which wrote the tile.  Apart from that no two
// items of a launch write one tile and no item reads a tile that another
// item of the launch writes.  At the end every block must be finished.
void check_dense_plan(const std::vector<int>& Ms, int64_t* nchk) {
  typedef std::tuple<int, int, int> Key;  // (slot, row offset, column offset)
  std::map<Key, int> cnt;                 // aligned blocks -> updates applied
  std::set<Key> fin;                      // finished tiles
  auto aligned = [](const Key& k) { return Key(std::get<0>(k), std::get<1>(k) / 64 * 64, std::get<2>(k) / 64 * 64); };
  const int ns = (int)Ms.size();
  int maxM = 0;
  for (int s = 0; s < ns; ++s) maxM = std::max(maxM, Ms[s]);
  std::vector<int2> items;
  for (int k0 = 0; k0 < maxM; k0 += 64) {
    int nflag = 0, npanel = 0;
    dense_plan_step(Ms, k0, &items, &nflag, &npanel);
    req(nflag >= 0 && npanel >= 0 && nflag + npanel <= (int)items.size(), "dense plan: item counts");
    const int p = k0 / 64;
    std::map<Key, std::vector<size_t>> writers;   // tile -> items writing it, in order
    std::map<std::pair<int, int>, size_t> flagged;  // (slot, row offset) -> flagged item
    std::vector<std::vector<Key>> rd(items.size());
    std::vector<std::pair<Key, size_t>> flag_rd;  // tiles read after their row's flag, with the reader
    std::vector<Key> upd, own;                    // tiles updated (once per update); panel tiles
    std::set<int> diag_slots;
    for (size_t i = 0; i < items.size(); ++i) {
      const int s = items[i].x;
      req(s >= 0 && s < ns && Ms[s] > k0, "dense plan: item of a finished instance");
      int kb, nrt, nct;
      dense_grid(Ms[s], k0, &kb, &nrt, &nct);
      ++*nchk;
      if ((int)i >= nflag && (int)i < nflag + npanel) {
        const int g = items[i].y;
        req(g >= 0 && g < 1 + nrt, "dense plan: panel item out of range");
        const Key d(s, k0, k0);
        req(cnt[aligned(d)] == p && !fin.count(d), "dense plan: diagonal block not up to date");
        if (g == 0) {
          req(diag_slots.insert(s).second, "dense plan: two diagonal items of an instance");
          rd[i] = {d};
          continue;
        }
        const int r0 = k0 + kb + 64 * (g - 1), c1 = k0 + kb;
        const Key o(s, r0, k0);
        req(r0 < Ms[s] && c1 <= Ms[s], "dense plan: tile out of range");
        req(cnt[aligned(o)] == p && !fin.count(o), "dense plan: panel tile not up to date");
        rd[i] = {d, o};
        writers[o].push_back(i);
        own.push_back(o);
        // this step's update of the row's tile in the next block column
        const Key nx(s, r0, c1), u(s, k0, c1);
        if (k0 == 0) {
          req(cnt[aligned(nx)] == 0 && cnt[aligned(u)] == 0 && !fin.count(nx) && !fin.count(u),
              "dense plan: next block column not up to date");
          rd[i].push_back(nx);
          rd[i].push_back(u);
        } else {
          flag_rd.push_back({nx, i});
          flag_rd.push_back({u, i});
        }
        writers[nx].push_back(i);
        upd.push_back(nx);
        continue;
      }
      // the previous step's update of a tile
      const int y = items[i].y, cb = y & 0xfff, rb = (y >> 12) & 0xfff, fl = y >> 24;
      req(fl == ((int)i < nflag ? 1 : 0), "dense plan: flag of an update item");
      req(k0 >= 64, "dense plan: update of a step before the first");
      const int r0 = 64 * rb, c0 = 64 * cb;
      req(r0 >= k0 && r0 < Ms[s] && c0 > k0 && c0 <= Ms[s], "dense plan: update tile off the grid");
      const Key x(s, r0, c0), l(s, r0, k0 - 64), u(s, k0 - 64, c0);
      req(cnt[x] == p - 1 && !fin.count(x), "dense plan: updated tile not up to date");
      req(fin.count(l) && fin.count(u), "dense plan: update before its panel");
      rd[i] = {x, l, u};
      writers[x].push_back(i);
      upd.push_back(x);
      if (fl) {
        req(c0 == k0 + 64, "dense plan: flagged update away from the next block column");
        req(flagged.emplace(std::make_pair(s, r0), i).second, "dense plan: two flagged items of one row block");
      }
    }
    // a tile read after a flag was written by that row's flagged item,
    // listed before the reader, and otherwise only by the reader
    std::set<std::pair<Key, size_t>> flag_ok;
    for (const auto& fr : flag_rd) {
      const Key& x = fr.first;
      auto f = flagged.find({std::get<0>(x), std::get<1>(x)});
      req(f != flagged.end() && f->second < fr.second, "dense plan: a flag wait on a later or missing work-group");
      const auto& w = writers[x];
      req(!w.empty() && w[0] == f->second, "dense plan: a flag that does not cover the tile read");
      for (size_t q = 1; q < w.size(); ++q) req(w[q] == fr.second, "dense plan: a tile read after a flag is written by another item");
      flag_ok.insert({x, fr.second});
    }
    for (const auto& kv : writers) {
      const auto& w = kv.second;
      req(w.size() == 1 || (w.size() == 2 && flag_ok.count({kv.first, w[1]})),
          "dense plan: two items of a launch write one tile");
    }
    for (size_t j = 0; j < items.size(); ++j)
      for (const Key& r : rd[j]) {
        auto it = writers.find(r);
        // (a flagged item reads its own tile before the flag)
        req(it == writers.end() ||
                (it->second[0] == j && (it->second.size() == 1 || flag_ok.count({r, it->second[1]}))),
            "dense plan: an item reads a tile written in its launch");
      }
    for (const Key& o : own) fin.insert(o);
    for (const Key& x : upd) cnt[aligned(x)] += 1;
    for (int s : diag_slots) {
      int kb, nrt, nct;
      dense_grid(Ms[s], k0, &kb, &nrt, &nct);
      fin.insert(Key(s, k0, k0));
      // the block row right of the diagonal block is final after the launch
      for (int j = 0; j < nct; ++j) {
        const Key u(s, k0, k0 + kb + 64 * j);
        req(cnt[aligned(u)] == p && !fin.count(u), "dense plan: block row not up to date");
        fin.insert(u);
      }
    }
    for (int s = 0; s < ns; ++s)
      req(Ms[s] <= k0 || diag_slots.count(s), "dense plan: an instance misses its panel");
  }
  for (int s = 0; s < ns; ++s) {
    const int R = (Ms[s] + 63) / 64, C = (Ms[s] + 1 + 63) / 64;
    for (int a = 0; a < R; ++a)
      for (int b = 0; b < C; ++b) {
        const Key x(s, 64 * a, 64 * b);
        req(fin.count(x) && cnt[x] == std::min(a, b), "dense plan: a block is not finished");
      }
    const int kl = (Ms[s] - 1) / 64 * 64;
    req(fin.count(Key(s, kl, Ms[s])) || Ms[s] % 64 == 0, "dense plan: right-hand side of the last step");
  }
}


// Replays the backward solve's launch plan (one launch) over copies of one
// analysed case with per-level lane counts gs.  Work-groups run in list
// order; every entry a work-group waits for must come from an earlier
// work-group: a dense block (flag mode) needs every block after it of its
// instance, a single-mode work-group runs its instance's blocks in order,
// and a sparse row needs its U columns, either rows of earlier work-groups
// (so never a row of its own work-group) or the dense blocks holding their
// entries.  Each work-group descriptor covers rows of one level and one lane
// count, at most 256 / G of them; every block and row is solved exactly once.
void check_bwd_plan(const pfh::Analysis& an, int M, const std::vector<int>& gs, int copies, bool single,
                    int64_t* nchk) {
  const int ns = an.ns;
  std::vector<BwdInput> in(copies);
  for (auto& x : in) {
    x.M = M;
    x.lev_ptr = &an.bwd_lev_ptr;
    x.rows = &an.bwd_rows;
    x.g = &gs;
  }
  std::vector<int2> items;
  int nd = 0, nrw = 0;
  bwd_plan(in, single, &items, &nd, &nrw);
  req(nd >= 0 && nrw >= 0 && (int64_t)nd + nrw <= (int64_t)items.size(), "backward plan: item counts");
  const int nblk = (M + 63) / 64;
  std::vector<std::vector<int>> blk_wg(copies, std::vector<int>(nblk, -1)), row_wg(copies, std::vector<int>(ns, -1));
  std::vector<int> blev(ns, -1);
  for (int l = 0; l + 1 < (int)an.bwd_lev_ptr.size(); ++l)
    for (int k = an.bwd_lev_ptr[l]; k < an.bwd_lev_ptr[l + 1]; ++k) blev[an.bwd_rows[k]] = l;
  for (int k = 0; k < nd; ++k) {
    const int s = items[k].x, w = items[k].y;
    ++*nchk;
    req(s >= 0 && s < copies && M > 0, "backward plan: dense item of an instance without a dense block");
    if (single) {
      req(w == 0, "backward plan: single-mode item");
      for (int b = nblk - 1; b >= 0; --b) {
        req(blk_wg[s][b] < 0, "backward plan: dense block solved twice");
        blk_wg[s][b] = k;
      }
      continue;
    }
    const int b = nblk - 1 - w;
    req(b >= 0 && b < nblk, "backward plan: dense block out of range");
    req(blk_wg[s][b] < 0, "backward plan: dense block solved twice");
    for (int c = b + 1; c < nblk; ++c)
      req(blk_wg[s][c] >= 0 && blk_wg[s][c] < k, "backward plan: a dense block waits on a later work-group");
    blk_wg[s][b] = k;
  }
  std::vector<int> covered(items.size(), 0);
  for (int k = nd; k < nd + nrw; ++k) {
    const int off = items[k].x, cnt = items[k].y & 0xffff, G = items[k].y >> 16;
    ++*nchk;
    req(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "backward plan: lanes per row");
    req(cnt >= 1 && cnt <= 256 / G, "backward plan: rows of a work-group");
    req(off >= nd + nrw && (int64_t)off + cnt <= (int64_t)items.size(), "backward plan: row items out of range");
    int lvl = -1;
    for (int g = 0; g < cnt; ++g) {
      req(covered[off + g]++ == 0, "backward plan: a row item in two work-groups");
      const int s = items[off + g].x, i = items[off + g].y;
      req(s >= 0 && s < copies && i >= 0 && i < ns, "backward plan: row out of range");
      req(row_wg[s][i] < 0, "backward plan: row solved twice");
      req(lvl < 0 || blev[i] == lvl, "backward plan: rows of two levels in one work-group");
      lvl = blev[i];
      req(gs[lvl] == G, "backward plan: lanes per row differ from the level's");
      for (int q = an.colptr[i]; q < an.colptr[i + 1]; ++q) {
        const int jj = an.rowidx[q];
        ++*nchk;
        if (jj >= ns) {
          const int p0 = 2 * (jj - ns);
          req(p0 + 1 < M, "backward plan: dense entry out of range");
          for (int b : {p0 / 64, (p0 + 1) / 64})
            req(blk_wg[s][b] >= 0 && blk_wg[s][b] < k, "backward plan: a row waits on a dense block of a later work-group");
        } else {
          req(row_wg[s][jj] >= 0 && row_wg[s][jj] < k, "backward plan: a row waits on its own or a later work-group");
        }
      }
    }
    for (int g = 0; g < cnt; ++g) row_wg[items[off + g].x][items[off + g].y] = k;
  }
  for (int s = 0; s < copies; ++s) {
    for (int b = 0; b < nblk; ++b) req(blk_wg[s][b] >= 0, "backward plan: dense block never solved");
    for (int i = 0; i < ns; ++i) req(row_wg[s][i] >= 0, "backward plan: row never solved");
  }
  for (size_t q = nd + nrw; q < items.size(); ++q) req(covered[q] == 1, "backward plan: row item outside every work-group");
}

}  // namespace

extern "C" pf_status pf_debug_schedule_check(const pf_case_desc* d, const pf_schedule* sched, uint64_t seed,
                                             double* rel_residual, int64_t* checks) {
  if (!rel_residual || !checks) {
    set_error("pf_debug_schedule_check: NULL output");
    return PF_E_INVALID;
  }
  pf_schedule sc;
  pf_default_schedule(&sc);
  if (sched) sc = *sched;
  if (!valid_schedule(sc)) {
    set_error("pf_debug_schedule_check: schedule out of range");
    return PF_E_INVALID;
  }
  pf_status st = validate_desc(d);
  if (st != PF_OK) return st;
  const int n = d->n;
  int64_t nchk = 0;
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
    pfh::Analysis an = pfh::analyze(g, sc.dense_switch, sc.min_dense, 64);
    std::vector<int> yrow, jmap;
    pfh::build_jmap(an, n, d->row_ptr, d->col_idx, &yrow, &jmap);
    const int ns = an.ns, nt = an.nt, nu = an.nu, M = 2 * nt, ldt = an.ldt;
    const int64_t nnzl = an.nnzl;
    const int64_t nblk = ns + 2 * nnzl;
    const int64_t ntail = (int64_t)ldt * (M + 1);
    req(nu == ns + nt, "nu != ns + nt");
    req(ldt >= M, "ldt < M");

    // level of every sparse column and the column of every L/U block
    std::vector<int> lev(ns, -1);
    for (int l = 0; l + 1 < (int)an.col_lev_ptr.size(); ++l)
      for (int k = an.col_lev_ptr[l]; k < an.col_lev_ptr[l + 1]; ++k) {
        int j = an.col_order[k];
        req(j >= 0 && j < ns, "col_order out of range");
        req(lev[j] == -1, "column listed twice");
        lev[j] = l;
      }
    for (int j = 0; j < ns; ++j) req(lev[j] >= 0, "column missing from the level lists");
    auto col_of_block = [&](int64_t id) {
      int64_t q = id < ns + nnzl ? id - ns : id - ns - nnzl;
      return (int)(std::upper_bound(an.colptr.begin(), an.colptr.end(), (int)q) - an.colptr.begin()) - 1;
    };

    // random diagonally dominant block matrix on the pattern (position space)
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    const int nnz = d->row_ptr[n];
    std::vector<double> A(4 * (size_t)nnz, 0.0);
    for (int q = 0; q < nnz; ++q) {
      for (int r = 0; r < 4; ++r) A[4 * q + r] = U(rng);
      if (yrow[q] == d->col_idx[q]) {
        int deg = d->row_ptr[yrow[q] + 1] - d->row_ptr[yrow[q]];
        A[4 * q + 0] += 4.0 * deg;
        A[4 * q + 3] += 4.0 * deg;
      }
    }
    std::vector<double> lu(4 * (size_t)nblk, 0.0), dinv(4 * (size_t)ns, 0.0);
    std::vector<double> tail((size_t)std::max<int64_t>(ntail, 1), 0.0);
    // scatter (the fill kernel's destinations)
    for (int q = 0; q < nnz; ++q) {
      int code = jmap[q];
      ++nchk;
      if (code == -1) {
        req(an.pos_of_node[yrow[q]] < 0 || an.pos_of_node[d->col_idx[q]] < 0, "skipped entry has unknowns");
        continue;
      }
      if (code >= 0) {
        req(code < nblk, "jmap block id out of range");
        for (int r = 0; r < 4; ++r) lu[4 * (size_t)code + r] = A[4 * q + r];
      } else {
        int t = -2 - code;
        req(t >= 0 && t < nt * nt, "jmap tail code out of range");
        int ta = t / nt, tb = t % nt;
        int64_t base = (int64_t)(2 * tb) * ldt + 2 * ta;
        req(base + ldt + 1 < ntail, "tail index out of range");
        tail[base] = A[4 * q + 0];
        tail[base + 1] = A[4 * q + 2];
        tail[base + ldt] = A[4 * q + 1];
        tail[base + ldt + 1] = A[4 * q + 3];
      }
    }
    auto msub = [&](double* acc, const double* X, const double* Y) {
      acc[0] -= X[0] * Y[0] + X[1] * Y[2];
      acc[1] -= X[0] * Y[1] + X[1] * Y[3];
      acc[2] -= X[2] * Y[0] + X[3] * Y[2];
      acc[3] -= X[2] * Y[1] + X[3] * Y[3];
    };
    auto chk_src = [&](int64_t l_id, int64_t u_id, int lev_target) {
      nchk += 2;
      req(l_id >= ns && l_id < ns + nnzl, "update L id out of range");
      req(u_id >= ns + nnzl && u_id < nblk, "update U id out of range");
      req(lev[col_of_block(l_id)] < lev_target, "update L source not finished at its level");
      req(lev[col_of_block(u_id)] < lev_target, "update U source not finished at its level");
    };
    // sparse refactorisation in level order (k_factor_cols)
    for (int l = 0; l + 1 < (int)an.col_lev_ptr.size(); ++l)
      for (int k = an.col_lev_ptr[l]; k < an.col_lev_ptr[l + 1]; ++k) {
        const int j = an.col_order[k];
        const int c0 = an.colptr[j], len = an.colptr[j + 1] - c0;
        const int64_t tb = (int64_t)j + 2LL * c0;
        req(tb + 2 * len + 1 < (int64_t)an.uptr.size(), "target id out of range");
        for (int t = 0; t <= len; ++t) {
          int64_t dest = t == 0 ? j : ns + nnzl + c0 + (t - 1);
          req(dest < nblk, "factor dest out of range");
          double* acc = &lu[4 * dest];
          for (int64_t q = an.uptr[tb + t]; q < an.uptr[tb + t + 1]; ++q) {
            chk_src(an.upd_l[q], an.upd_u[q], l);
            msub(acc, &lu[4 * (size_t)an.upd_l[q]], &lu[4 * (size_t)an.upd_u[q]]);
          }
        }
        double* D = &lu[4 * (size_t)j];
        double det = D[0] * D[3] - D[1] * D[2];
        req(det != 0.0, "zero pivot block");
        double* di = &dinv[4 * (size_t)j];
        di[0] = D[3] / det;
        di[1] = -D[1] / det;
        di[2] = -D[2] / det;
        di[3] = D[0] / det;
        for (int t = 0; t < len; ++t) {
          int64_t dest = ns + c0 + t;
          int64_t tg = tb + 1 + len + t;
          double acc[4] = {lu[4 * dest], lu[4 * dest + 1], lu[4 * dest + 2], lu[4 * dest + 3]};
          for (int64_t q = an.uptr[tg]; q < an.uptr[tg + 1]; ++q) {
            chk_src(an.upd_l[q], an.upd_u[q], l);
            msub(acc, &lu[4 * (size_t)an.upd_l[q]], &lu[4 * (size_t)an.upd_u[q]]);
          }
          lu[4 * dest + 0] = acc[0] * di[0] + acc[1] * di[2];
          lu[4 * dest + 1] = acc[0] * di[1] + acc[1] * di[3];
          lu[4 * dest + 2] = acc[2] * di[0] + acc[3] * di[2];
          lu[4 * dest + 3] = acc[2] * di[1] + acc[3] * di[3];
        }
      }
    // right-hand side in position space
    std::vector<double> b(2 * (size_t)nu), x(2 * (size_t)nu);
    for (auto& v : b) v = U(rng);
    x = b;
    auto fwd_row = [&](int i, int lev_i) {
      req(i >= 0 && i < nu, "forward row out of range");
      for (int q = an.lrow_ptr[i]; q < an.lrow_ptr[i + 1]; ++q) {
        int id = an.lrow_blk[q], k = an.lrow_col[q];
        ++nchk;
        req(id >= ns && id < ns + nnzl && k >= 0 && k < ns, "forward list out of range");
        req(lev_i < 0 || lev[k] < lev_i, "forward dependency not finished at its level");
        const double* L = &lu[4 * (size_t)id];
        x[2 * i] -= L[0] * x[2 * k] + L[1] * x[2 * k + 1];
        x[2 * i + 1] -= L[2] * x[2 * k] + L[3] * x[2 * k + 1];
      }
    };
    for (int l = 0; l + 1 < (int)an.col_lev_ptr.size(); ++l)
      for (int k = an.col_lev_ptr[l]; k < an.col_lev_ptr[l + 1]; ++k) fwd_row(an.col_order[k], l);
    for (int i = ns; i < nu; ++i) fwd_row(i, -1);
    if (nt > 0) {
      double* rhs = &tail[(size_t)M * ldt];
      for (int i = ns; i < nu; ++i) {
        rhs[2 * (i - ns)] = x[2 * i];
        rhs[2 * (i - ns) + 1] = x[2 * i + 1];
      }
      // Schur complement into the dense block
      for (size_t t = 0; t < an.tail_tgt.size(); ++t) {
        int g2 = an.tail_tgt[t];
        req(g2 >= 0 && g2 < nt * nt, "tail target out of range");
        double acc[4] = {0, 0, 0, 0};
        for (int64_t q = an.tail_uptr[t]; q < an.tail_uptr[t + 1]; ++q) {
          chk_src(an.tail_l[q], an.tail_u[q], 1 << 30);
          msub(acc, &lu[4 * (size_t)an.tail_l[q]], &lu[4 * (size_t)an.tail_u[q]]);
        }
        int ta = g2 / nt, tb = g2 % nt;
        double* p = &tail[(size_t)(2 * tb) * ldt + 2 * ta];
        p[0] += acc[0];
        p[1] += acc[2];
        p[ldt] += acc[1];
        p[ldt + 1] += acc[3];
      }
      // dense LU with static pivots on [A | rhs]
      for (int k = 0; k < M; ++k) {
        double piv = tail[(size_t)k * ldt + k];
        req(piv != 0.0, "zero dense pivot");
        for (int r = k + 1; r < M; ++r) tail[(size_t)k * ldt + r] /= piv;
        for (int c = k + 1; c <= M; ++c) {
          double u = tail[(size_t)c * ldt + k];
          for (int r = k + 1; r < M; ++r) tail[(size_t)c * ldt + r] -= tail[(size_t)k * ldt + r] * u;
        }
      }
      for (int r = M - 1; r >= 0; --r) {
        double v = rhs[r];
        for (int c = r + 1; c < M; ++c) v -= tail[(size_t)c * ldt + r] * x[2 * ns + c];
        x[2 * ns + r] = v / tail[(size_t)r * ldt + r];
      }
    }
    // backward rows by level
    std::vector<int> blev(ns, -1);
    for (int l = 0; l + 1 < (int)an.bwd_lev_ptr.size(); ++l)
      for (int k = an.bwd_lev_ptr[l]; k < an.bwd_lev_ptr[l + 1]; ++k) {
        int i = an.bwd_rows[k];
        req(i >= 0 && i < ns && blev[i] == -1, "backward row list broken");
        blev[i] = l;
      }
    for (int l = 0; l + 1 < (int)an.bwd_lev_ptr.size(); ++l)
      for (int k = an.bwd_lev_ptr[l]; k < an.bwd_lev_ptr[l + 1]; ++k) {
        int i = an.bwd_rows[k];
        double z0 = x[2 * i], z1 = x[2 * i + 1];
        for (int q = an.colptr[i]; q < an.colptr[i + 1]; ++q) {
          int jj = an.rowidx[q];
          ++nchk;
          req(jj > i && jj < nu, "backward column out of range");
          req(jj >= ns || blev[jj] < l, "backward dependency not finished at its level");
          const double* Ub = &lu[4 * (size_t)(ns + nnzl + q)];
          z0 -= Ub[0] * x[2 * jj] + Ub[1] * x[2 * jj + 1];
          z1 -= Ub[2] * x[2 * jj] + Ub[3] * x[2 * jj + 1];
        }
        const double* di = &dinv[4 * (size_t)i];
        x[2 * i] = di[0] * z0 + di[1] * z1;
        x[2 * i + 1] = di[2] * z0 + di[3] * z1;
      }
    // residual of A x = b in position space
    std::vector<double> r(b.size());
    for (size_t i = 0; i < r.size(); ++i) r[i] = -b[i];
    double anorm = 0;
    for (int q = 0; q < nnz; ++q) {
      int pi = an.pos_of_node[yrow[q]], pj = an.pos_of_node[d->col_idx[q]];
      if (pi < 0 || pj < 0) continue;
      const double* a = &A[4 * (size_t)q];
      r[2 * pi] += a[0] * x[2 * pj] + a[1] * x[2 * pj + 1];
      r[2 * pi + 1] += a[2] * x[2 * pj] + a[3] * x[2 * pj + 1];
      anorm = std::max(anorm, std::fabs(a[0]) + std::fabs(a[1]) + std::fabs(a[2]) + std::fabs(a[3]));
    }
    double rn = 0, xn = 0, bn = 0;
    for (size_t i = 0; i < r.size(); ++i) {
      rn = std::max(rn, std::fabs(r[i]));
      xn = std::max(xn, std::fabs(x[i]));
      bn = std::max(bn, std::fabs(b[i]));
    }
    *rel_residual = rn / (anorm * xn + bn);
    // the backward solve's launch plan: one lane count everywhere, then
    // mixed per level; alone, batched, and in single mode
    {
      const int nbl = (int)an.bwd_lev_ptr.size() - 1;
      std::vector<int> g1(nbl, 1), g64(nbl, 64), gmix(nbl);
      for (int l = 0; l < nbl; ++l) gmix[l] = 1 << (l % 7);
      for (const auto* gs : {&g1, &g64, &gmix})
        for (int copies : {1, 3})
          for (bool single : {false, true}) check_bwd_plan(an, M, *gs, copies, single, &nchk);
    }
    // the dense block's launch plan, alone and batched with other orders
    if (M > 0) {
      check_dense_plan({M}, &nchk);
      check_dense_plan({M, std::max(1, M / 2), 64, 65, 1, M + 64}, &nchk);
    }
  } catch (const std::exception& e) {
    set_error(std::string("pf_debug_schedule_check: ") + e.what());
    *checks = nchk;
    return PF_E_INVALID;
  }
  *checks = nchk;
  return PF_OK;
}
