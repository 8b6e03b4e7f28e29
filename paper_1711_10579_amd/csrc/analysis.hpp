// Host-side symbolic analysis of the Newton Jacobian (runs once per topology).
//
// The Jacobian of both formulations is a sparse matrix of 2x2 blocks over a
// node graph: buses for the single-phase polar form (unknowns angle and |V|,
// eq. 10) and phase-nodes for the three-phase current-injection form
// (unknowns Re V and Im V, eq. 19-22).  Its block pattern is the pattern of
// Ybus restricted to the nodes with unknowns, so the analysis works on that
// graph: fill-reducing ordering (Sec. III-A), symbolic block LU with a dense
// trailing block, column levels for the refactorisation and row levels for
// the two triangular solves, and the map from Ybus entries to LU storage.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pfh {

struct Ordering {
  std::vector<int> perm;  // position -> node
  int n_sparse = 0;       // leading positions eliminated as sparse columns
};

Ordering min_degree_order(int n, const std::vector<std::vector<int>>& adj,
                          double dense_switch, int min_dense);

// Block ids of the sparse factor storage:
//   D_j          : id j                         (j < ns)
//   L(r_p, j)    : id ns + colptr[j] + p        (r_p = rowidx[colptr[j]+p] > j)
//   U(j, r_p)    : id ns + nnzl + colptr[j] + p
// Each block holds 4 values, row-major [a00 a01 a10 a11].
// The dense trailing block (positions ns..nu-1) is a column-major scalar
// matrix of order 2*nt with leading dimension ldt.
struct Analysis {
  int nu = 0, ns = 0, nt = 0;
  std::vector<int> node_of_pos;  // [nu]
  std::vector<int> pos_of_node;  // [n_nodes], -1 for fixed nodes
  std::vector<int> colptr;       // [ns+1]
  std::vector<int> rowidx;       // [nnzl]
  std::vector<int> parent;       // elimination tree over sparse columns (-1: root or tail)
  int64_t nnzl = 0;
  int ldt = 0;

  // refactorisation: columns grouped by level
  std::vector<int> col_lev_ptr;  // [nlev+1]
  std::vector<int> col_order;    // [ns]
  // per column target list: D, U(j, r_0..), L(r_0.., j) -> target id
  // tbase[j] = j + 2*colptr[j]; target t's updates are upd[uptr[t]..uptr[t+1])
  std::vector<int64_t> uptr;     // [ntargets+1]
  std::vector<int> upd_l, upd_u; // source block ids
  // Schur complement into the dense tail: tail block (a,b) -> list of
  // (L block, U block) pairs; only blocks with a non-empty list are listed
  std::vector<int> tail_tgt;     // a*nt + b
  std::vector<int64_t> tail_uptr;
  std::vector<int> tail_l, tail_u;

  // forward solve (L y = b) over sparse rows, by level: row i gathers
  // L(i,k) y_k for the listed (block id, k) pairs
  std::vector<int> fwd_lev_ptr, fwd_rows;
  std::vector<int> lrow_ptr, lrow_blk, lrow_col;  // [nu+1], by row position
  // backward solve (U x = y) over sparse rows, by level (tail first)
  std::vector<int> bwd_lev_ptr, bwd_rows;

  // statistics
  double flops_sparse = 0, flops_tail_schur = 0, flops_dense = 0;
  std::string summary() const;
};

struct GraphInput {
  int n_nodes = 0;
  std::vector<char> unknown;          // [n_nodes]
  std::vector<std::vector<int>> adj;  // node graph over all nodes
};

Analysis analyze(const GraphInput& g, double dense_switch, int min_dense, int tail_align);

// Destination of every Ybus entry (i, j) in the factor storage: the block id
// of D/L/U, or -2 - (a*nt + b) for block (a, b) of the dense tail, or -1 when
// i or j has no unknowns.  yrow[q] is the row of entry q.
void build_jmap(const Analysis& an, int n, const int* row_ptr, const int* col, std::vector<int>* yrow,
                std::vector<int>* jmap);

}  // namespace pfh

namespace pfh {

// Host analysis of the Newton-Krylov inner solve (Sec. III-B), once per
// topology.  The Krylov vectors hold the two unknowns of every node with
// unknowns, nodes in reverse Cuthill-McKee order of the node graph (row r).
// The Jacobian is kept as 2x2 blocks on that graph's pattern (block CSR,
// sorted columns); ILU(0) works on the same pattern.
struct KAnalysis {
  int nu = 0;
  std::vector<int> p_of_r, r_of_p;       // Krylov row <-> factor position of the node
  std::vector<int> row_ptr, col, diag;   // block CSR pattern in Krylov order
  // ILU(0) in its IKJ form: lower entry q of row r (column k < r) is
  // followed by the updates A(r, j) -= L(r, k) U(k, j) for the listed pairs
  // (t = position of (r, j), s = position of (k, j)), j > k
  std::vector<int> up_ptr;               // [nnz+1], non-empty only for lower entries
  std::vector<int> up_t, up_s;
  // rows by level: a row's lower neighbours are in earlier levels (factor
  // and forward solve); its upper neighbours are in earlier levels of the
  // backward order
  std::vector<int> lev_ptr, lev_rows, ulev_ptr, ulev_rows;
  // block-Jacobi blocks: connected groups of at most bj_cap nodes grown
  // breadth-first from seeds in Krylov order; rows of each block in that
  // growth order, dense (2s)x(2s) inverse at bj_off[b]
  std::vector<int> bj_ptr, bj_rows, bj_loc;
  std::vector<int64_t> bj_off;
  int bj_max = 0;
  int64_t nnz() const { return (int64_t)col.size(); }
  int64_t nup() const { return (int64_t)up_t.size(); }
  int nblocks() const { return (int)bj_ptr.size() - 1; }
};

// The reverse Cuthill-McKee order of an undirected graph (adjacency lists,
// no self loops): breadth-first from a pseudo-peripheral start in every
// connected component, neighbours taken by increasing degree, the whole
// sequence reversed.  Returns order[r] = vertex.
std::vector<int> rcm_order(const std::vector<std::vector<int>>& adj);

KAnalysis analyze_krylov(const Analysis& an, int n, const int* row_ptr, const int* col, int bj_cap);

// Ybus entry -> block position in the Krylov pattern, -1 when the row or the
// column node has no unknowns.
void build_kmap(const Analysis& an, const KAnalysis& ka, int n, const int* row_ptr, const int* col,
                std::vector<int>* kmap);

}  // namespace pfh
