"""Newton-Krylov inner solve (Sec. III-B): the Jacobian system of each Newton
step is solved only approximately, by an iterative Krylov method.

The paper tested the bi-conjugate gradient stabilized method (BiCGStab, its
reference [20]) and names the parallel building blocks (sparse
matrix-vector products and vector updates), but no preconditioner.  Two
methods are given here: BiCGStab and restarted GMRES(m), both with right
preconditioning, the preconditioner being either ILU(0) or block-Jacobi, and
the inner tolerance being the forcing term eta_k = min(eta_max,
||F_k||_inf) of inexact Newton methods (Dembo, Eisenstat and Steihaug;
Eisenstat and Walker) relative to ||F_k||_2.

Written from the textbook definitions (Saad, "Iterative Methods for Sparse
Linear Systems": GMRES with modified Gram-Schmidt Arnoldi and Givens
rotations, and BiCGStab as van der Vorst gave it, both right-preconditioned;
ILU(0) in its IKJ form), for clarity rather than speed.  Test infrastructure
only: nothing on the GPU path imports it.
"""

from collections import deque

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee


# ---------------------------------------------------------------------------
# orderings

def unknown_order(node_of_unknown, comp_of_unknown, node_graph):
    """Permutation of the unknowns that keeps the (at most two) unknowns of a
    node adjacent, nodes in reverse Cuthill-McKee order of the node graph
    restricted to nodes with unknowns.  Returns (perm, node_rank) where
    perm[k] is the unknown placed at position k and node_rank[node] is the
    node's position in the node order (-1 for nodes without unknowns)."""
    node_of_unknown = np.asarray(node_of_unknown)
    nodes = np.unique(node_of_unknown)
    G = sp.csr_matrix(node_graph)[nodes][:, nodes]
    rcm = reverse_cuthill_mckee(G.tocsr(), symmetric_mode=True)
    node_rank = -np.ones(int(node_graph.shape[0]), dtype=np.int64)
    node_rank[nodes[rcm]] = np.arange(len(nodes))
    key = node_rank[node_of_unknown] * 2 + np.asarray(comp_of_unknown)
    return np.argsort(key, kind="stable"), node_rank


def aggregates(node_rank, node_graph, cap):
    """Block-Jacobi blocks: nodes are grouped by breadth-first growth from
    seeds taken in node order, each group holding at most ``cap`` nodes.
    Returns the group of every node (-1 for nodes without unknowns)."""
    G = sp.csr_matrix(node_graph)
    order = np.argsort(np.where(node_rank < 0, np.iinfo(np.int64).max, node_rank), kind="stable")
    order = order[node_rank[order] >= 0]
    group = -np.ones(G.shape[0], dtype=np.int64)
    ng = 0
    for seed in order:
        if group[seed] >= 0:
            continue
        group[seed] = ng
        count, queue = 1, deque([seed])
        while queue and count < cap:
            u = queue.popleft()
            for w in G.indices[G.indptr[u]:G.indptr[u + 1]]:
                if count >= cap:
                    break
                if node_rank[w] >= 0 and group[w] < 0:
                    group[w] = ng
                    count += 1
                    queue.append(w)
        ng += 1
    return group


# ---------------------------------------------------------------------------
# preconditioners

def ilu0(A):
    """Incomplete LU with zero fill: L (unit lower) and U (upper) on the
    pattern of A such that (L U)_ij = A_ij at every (i, j) of the pattern.
    IKJ form: row i is reduced by the earlier rows k of its lower pattern in
    increasing k, keeping only entries already in row i."""
    A = sp.csr_matrix(A, dtype=np.float64, copy=True)
    A.sort_indices()
    ip, ix, a = A.indptr, A.indices, A.data
    n = A.shape[0]
    where = [dict(zip(ix[ip[i]:ip[i + 1]].tolist(), range(ip[i], ip[i + 1]))) for i in range(n)]
    diag = np.empty(n, dtype=np.int64)
    for i in range(n):
        if i not in where[i]:
            raise ArithmeticError(f"ILU(0): diagonal entry missing in row {i}")
        diag[i] = where[i][i]
    for i in range(n):
        for p in range(ip[i], diag[i]):
            k = ix[p]
            if a[diag[k]] == 0:
                raise ArithmeticError(f"ILU(0): zero pivot in row {k}")
            a[p] = a[p] / a[diag[k]]
            for q in range(diag[k] + 1, ip[k + 1]):
                t = where[i].get(ix[q])
                if t is not None:
                    a[t] -= a[p] * a[q]
        if a[diag[i]] == 0 or not np.isfinite(a[diag[i]]):
            raise ArithmeticError(f"ILU(0): zero pivot in row {i}")
    LU = sp.csr_matrix((a, ix, ip), shape=A.shape)
    L = (sp.tril(LU, -1) + sp.identity(n)).tocsr()
    U = sp.triu(LU).tocsr()
    return L, U


def ilu0_apply(L, U):
    """z = U^{-1} L^{-1} v."""
    from scipy.sparse.linalg import spsolve_triangular

    def apply(v):
        y = spsolve_triangular(L, v, lower=True, unit_diagonal=True)
        return spsolve_triangular(U, y, lower=False)

    return apply


def block_jacobi(A, blocks):
    """Inverse of every diagonal block A[b, b] (``blocks``: index arrays that
    partition the unknowns).  Returns the apply function and the inverses."""
    A = sp.csr_matrix(A)
    invs = []
    for b in blocks:
        Ab = A[b][:, b].toarray()
        invs.append(np.linalg.inv(Ab))

    def apply(v):
        out = np.empty_like(v)
        for b, Bi in zip(blocks, invs):
            out[b] = Bi @ v[b]
        return out

    return apply, invs


# ---------------------------------------------------------------------------
# GMRES

def gmres(A, b, apply_m, m, rtol, max_restarts):
    """Right-preconditioned restarted GMRES(m) from x0 = 0.

    Each cycle builds the Arnoldi basis of A M^{-1} with modified
    Gram-Schmidt, reduces the Hessenberg matrix with Givens rotations and
    stops once |g_{j+1}| <= rtol ||b||_2; then x += M^{-1} V y.  At most
    1 + max_restarts cycles.  Returns x, the number of Arnoldi steps, the
    final relative residual estimate, whether rtol was met and the estimate
    after every step (the history)."""
    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.float64)
    N = b.shape[0]
    x = np.zeros(N)
    bnorm = float(np.linalg.norm(b))
    hist = []
    if bnorm == 0.0:
        return x, 0, 0.0, True, hist
    total = 0
    rel = 1.0
    for _cycle in range(max_restarts + 1):
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        rel = beta / bnorm
        if rel <= rtol:
            return x, total, rel, True, hist
        V = np.zeros((m + 1, N))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = A @ apply_m(V[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # earlier rotations on the new column
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -sn[i] * hi + cs[i] * hi1
            d = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j], H[j + 1, j] = d, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            rel = abs(g[j + 1]) / bnorm
            hist.append(rel)
            if rel <= rtol or breakdown:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):  # back substitution with upper H
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + apply_m(V[:k].T @ y)
        if rel <= rtol:
            return x, total, rel, True, hist
    return x, total, rel, False, hist


def bicgstab(A, b, apply_m, rtol, max_iter, record=None):
    """Right-preconditioned BiCGStab from x0 = 0 (van der Vorst): the shadow
    residual is r0 = b; each iteration takes a bi-conjugate gradient step
    along the preconditioned direction and then a one-dimensional minimal
    residual step, and stops once the residual's 2-norm is at most rtol
    ||b||_2 -- already after the first half when that half's residual s
    meets it.  At most max_iter iterations; a zero <r0, r>, <r0, v> or
    <t, t> ends the solve as it stands.  Returns x, the iterations begun, the
    final relative residual of the recurrence, whether rtol was met and the
    relative residual after every iteration.  ``record``: a list that
    receives, per completed iteration, the vectors s and t and the step
    omega (for tests)."""
    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.float64)
    N = b.shape[0]
    x = np.zeros(N)
    bnorm = float(np.linalg.norm(b))
    hist = []
    if bnorm == 0.0:
        return x, 0, 0.0, True, hist
    r = b.copy()
    rs = b.copy()  # shadow residual
    p = np.zeros(N)
    v = np.zeros(N)
    rho_prev = alpha = omega = 1.0
    rel = 1.0
    its = 0
    for i in range(max_iter):
        rho = float(rs @ r)
        if rho == 0.0:
            break
        its = i + 1
        if i == 0:
            p = r.copy()
        else:
            beta = (rho / rho_prev) * (alpha / omega)
            p = r + beta * (p - omega * v)
        ph = apply_m(p)
        v = A @ ph
        sv = float(rs @ v)
        if sv == 0.0:
            break
        alpha = rho / sv
        s = r - alpha * v
        srel = float(np.linalg.norm(s)) / bnorm
        if srel <= rtol:
            x = x + alpha * ph
            rel = srel
            hist.append(rel)
            return x, its, rel, True, hist
        sh = apply_m(s)
        t = A @ sh
        tt = float(t @ t)
        if tt == 0.0:
            break
        omega = float(t @ s) / tt
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        if record is not None:
            record.append({"s": s, "t": t, "omega": omega})
        if rel <= rtol:
            return x, its, rel, True, hist
        if omega == 0.0:
            break
        rho_prev = rho
    return x, its, rel, False, hist


# ---------------------------------------------------------------------------
# the inexact Newton step

def bicgstab_max_iter(m, max_restarts):
    """BiCGStab's iteration limit: two products with J per iteration, as many
    products in all as GMRES(m) with max_restarts restarts may take."""
    return max(1, (1 + max_restarts) * m // 2)


def forcing(nrm_inf, eta_max):
    """eta_k = min(eta_max, ||F_k||_inf)."""
    return min(eta_max, nrm_inf)


def inexact_step(J, F, nrm_inf, node_of_unknown, comp_of_unknown, node_graph, precond="ilu0", m=30,
                 max_restarts=10, eta_max=0.1, bj_cap=32, method="gmres"):
    """Solve J dx = F to the relative residual eta_k with right-preconditioned
    GMRES(m) (at most 1 + max_restarts cycles) or BiCGStab (at most
    (1 + max_restarts) m / 2 iterations: the same number of products with
    J) in the node-interleaved reverse Cuthill-McKee order.  Returns dx (in
    the original unknown order) and an info dict with the iterations, the
    forcing term, the achieved relative residual and whether it was met."""
    perm, node_rank = unknown_order(node_of_unknown, comp_of_unknown, node_graph)
    A = sp.csr_matrix(J)[perm][:, perm]
    rhs = np.asarray(F)[perm]
    if precond == "ilu0":
        L, U = ilu0(A)
        apply_m = ilu0_apply(L, U)
    elif precond == "bjacobi":
        grp = aggregates(node_rank, node_graph, bj_cap)
        ug = grp[np.asarray(node_of_unknown)[perm]]
        blocks = [np.flatnonzero(ug == q) for q in np.unique(ug)]
        apply_m, _ = block_jacobi(A, blocks)
    elif precond == "none":
        apply_m = lambda v: v  # noqa: E731
    else:
        raise ValueError(precond)
    eta = forcing(nrm_inf, eta_max)
    if method == "gmres":
        y, its, rel, ok, hist = gmres(A, rhs, apply_m, m, eta, max_restarts)
    elif method == "bicgstab":
        y, its, rel, ok, hist = bicgstab(A, rhs, apply_m, eta, bicgstab_max_iter(m, max_restarts))
    else:
        raise ValueError(method)
    dx = np.empty_like(y)
    dx[perm] = y
    return dx, {"iters": its, "eta": eta, "rel": rel, "met": ok, "history": hist}
