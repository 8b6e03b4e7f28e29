"""Pins of the oracle's Newton-Krylov inner solve (Sec. III-B) against facts
that do not depend on its code: the defining property of ILU(0), exactness
where elimination makes no fill, finite termination and the minimal-residual
property of GMRES (brute-force least squares over the Krylov space), exact
block-Jacobi with one block, the forcing term met by the true residual, and
Newton-Krylov reaching the root of the direct Newton iteration."""

import numpy as np
import pytest
import scipy.sparse as sp

import pfgen
from oracle import cim, krylov, polar
from oracle.result import CONVERGED, LINEAR_FAIL


def _random_pattern_matrix(n, extra, seed, dominance=4.0):
    rng = np.random.default_rng(seed)
    rows, cols = list(range(n)), list(range(n))
    for _ in range(extra):
        i, j = rng.integers(0, n, 2)
        if i != j:
            rows += [i, j]
            cols += [j, i]
    A = sp.csr_matrix((rng.uniform(-1, 1, len(rows)), (rows, cols)), shape=(n, n))
    A.sum_duplicates()
    A = A + sp.diags(dominance + np.abs(A).sum(axis=1).A1 * rng.uniform(0.2, 0.6, n))
    return A.tocsr()


def test_ilu0_reproduces_a_on_its_pattern():
    A = _random_pattern_matrix(80, 160, 1, dominance=0.5)
    L, U = krylov.ilu0(A)
    P = (L @ U).tocsr()
    Ad = A.toarray()
    Pd = P.toarray()
    mask = Ad != 0
    assert np.max(np.abs(Pd[mask] - Ad[mask])) <= 1e-12 * np.max(np.abs(Ad))
    # and it is not the exact LU: the product has entries off the pattern
    assert np.max(np.abs(Pd[~mask])) > 1e-6
    # L unit lower and U upper on the pattern of A
    assert np.all(L.diagonal() == 1.0)
    assert set(zip(*sp.tril(L, -1).nonzero())) <= set(zip(*A.nonzero()))
    assert set(zip(*sp.triu(U).nonzero())) <= set(zip(*A.nonzero()))


def test_ilu0_is_exact_lu_when_elimination_makes_no_fill():
    # a tree whose every node comes before its parent: eliminating a leaf
    # touches only its parent, so the exact LU has the pattern of A
    rng = np.random.default_rng(2)
    n = 60
    parent = [None] + [int(rng.integers(0, k)) for k in range(1, n)]
    order = list(range(n))[::-1]  # children have larger labels: reversed is leaf-first
    pos = {v: i for i, v in enumerate(order)}
    rows, cols, vals = [], [], []
    for v in range(1, n):
        a, b = pos[v], pos[parent[v]]
        rows += [a, b]
        cols += [b, a]
        vals += list(rng.uniform(-1, 1, 2))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n)) + sp.diags(rng.uniform(3, 4, n))
    L, U = krylov.ilu0(A)
    assert np.max(np.abs((L @ U - A).toarray())) <= 1e-13
    b = rng.normal(size=n)
    x, its, rel, ok, _ = krylov.gmres(A, b, krylov.ilu0_apply(L, U), 10, 1e-12, 0)
    assert ok and its == 1
    assert np.max(np.abs(A @ x - b)) <= 1e-12


def test_gmres_terminates_in_n_steps_without_preconditioner():
    rng = np.random.default_rng(3)
    n = 14
    A = sp.csr_matrix(rng.normal(size=(n, n)) + 6 * np.eye(n))
    b = rng.normal(size=n)
    x, its, rel, ok, hist = krylov.gmres(A, b, lambda v: v, n, 1e-13, 0)
    assert ok and its <= n
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=0, atol=1e-11)
    # the residual estimate never grows (minimal residual over nested spaces)
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))


@pytest.mark.parametrize("pre", ["none", "jacobi"])
def test_gmres_is_the_minimal_residual_over_the_krylov_space(pre):
    # brute force: x_k minimises ||b - A x|| over x in M^{-1} K_k(A M^{-1}, b)
    rng = np.random.default_rng(4)
    n = 25
    A = sp.csr_matrix(rng.normal(size=(n, n)) + 3 * np.eye(n))
    d = np.abs(A.diagonal()) + 1.0
    Minv = (lambda v: v) if pre == "none" else (lambda v: v / d)
    b = rng.normal(size=n)
    for k in range(1, 6):
        x, its, rel, ok, hist = krylov.gmres(A, b, Minv, k, 1e-300, 0)
        assert its == k
        K = [b]
        for _ in range(k - 1):
            K.append(A @ Minv(K[-1]))
        K = np.array(K).T
        AMK = np.column_stack([A @ Minv(K[:, i]) for i in range(k)])
        c, *_ = np.linalg.lstsq(AMK, b, rcond=None)
        best = np.linalg.norm(b - AMK @ c)
        assert abs(np.linalg.norm(b - A @ x) - best) <= 1e-10 * np.linalg.norm(b)
        assert abs(hist[-1] * np.linalg.norm(b) - best) <= 1e-10 * np.linalg.norm(b)


def test_block_jacobi_with_one_block_is_exact_and_blocks_invert():
    A = _random_pattern_matrix(40, 60, 5)
    b = np.random.default_rng(5).normal(size=40)
    apply, invs = krylov.block_jacobi(A, [np.arange(40)])
    x, its, rel, ok, _ = krylov.gmres(A, b, apply, 10, 1e-12, 0)
    assert ok and its == 1
    blocks = [np.arange(0, 13), np.arange(13, 29), np.arange(29, 40)]
    _, invs = krylov.block_jacobi(A, blocks)
    for blk, Bi in zip(blocks, invs):
        np.testing.assert_allclose(Bi @ A[blk][:, blk].toarray(), np.eye(len(blk)), atol=1e-12)


def test_orderings_are_node_interleaved_permutations():
    case = pfgen.make_polar_grid(200, 60, 20, 7, balanced=True)
    pvpq, pq = polar.index_sets(case)
    node_of = np.concatenate([pvpq, pq])
    comp_of = np.concatenate([np.zeros(len(pvpq), int), np.ones(len(pq), int)])
    G = sp.csr_matrix((np.ones(case.nnz), case.col, case.row_ptr), shape=(case.n, case.n))
    perm, rank = krylov.unknown_order(node_of, comp_of, G)
    assert sorted(perm.tolist()) == list(range(len(node_of)))
    nodes = node_of[perm]
    # non-decreasing node rank, angle before magnitude within a node
    assert np.all(np.diff(rank[nodes]) >= 0)
    same = np.diff(rank[nodes]) == 0
    assert np.all(comp_of[perm][1:][same] == 1)
    grp = krylov.aggregates(rank, G, 8)
    assert grp[rank < 0].tolist() == [-1] * int((rank < 0).sum())
    sizes = np.bincount(grp[grp >= 0])
    assert sizes.max() <= 8 and sizes.sum() == int((rank >= 0).sum())
    # every group is connected in the node graph
    import scipy.sparse.csgraph as csg
    for q in np.unique(grp[grp >= 0])[:40]:
        members = np.flatnonzero(grp == q)
        ncomp, _ = csg.connected_components(G[members][:, members], directed=False)
        assert ncomp == 1


@pytest.mark.parametrize("precond", ["ilu0", "bjacobi"])
def test_inexact_step_meets_its_forcing_term(precond):
    case = pfgen.make_polar_grid(400, 120, 40, 9, balanced=True)
    pvpq, pq = polar.index_sets(case)
    vm, va = polar.flat_start(case)
    F = polar.mismatch(case, vm, va)
    J = polar.jacobian(case, vm, va)
    node_of = np.concatenate([pvpq, pq])
    comp_of = np.concatenate([np.zeros(len(pvpq), int), np.ones(len(pq), int)])
    G = sp.csr_matrix((np.ones(case.nnz), case.col, case.row_ptr), shape=(case.n, case.n))
    nrm = float(np.max(np.abs(F)))
    for eta_max in (0.1, 1e-3, 1e-8):
        dx, info = krylov.inexact_step(J, F, nrm, node_of, comp_of, G, precond=precond, eta_max=eta_max,
                                       max_restarts=40)
        assert info["eta"] == min(eta_max, nrm)
        true_rel = np.linalg.norm(F - J @ dx) / np.linalg.norm(F)
        assert info["met"]
        assert true_rel <= info["eta"] * 1.001 + 1e-14


@pytest.mark.parametrize("precond", ["ilu0", "bjacobi"])
def test_newton_krylov_reaches_the_direct_newton_root(precond):
    for case, mod in [(pfgen.config_case(0), polar),
                      (pfgen.make_polar_grid(500, 150, 50, 3, balanced=True), polar),
                      (pfgen.make_feeder(80, 4), cim)]:
        ref = mod.newton(case)
        r = mod.newton(case, linear="gmres", precond=precond)
        assert r.status == CONVERGED
        assert np.max(np.abs(r.V - ref.V)) <= 1e-10
        assert len(r.linear_iters) == r.iters


def test_linear_fail_status_when_the_inner_solve_cannot_progress():
    case = pfgen.make_polar_grid(300, 90, 30, 12, balanced=True)
    r = polar.newton(case, linear="gmres", precond="none", m=1, max_restarts=0, eta_max=1e-6)
    assert r.status == LINEAR_FAIL


# ---------------------------------------------------------------------------
# BiCGStab


def _exact_solver(A):
    lu = sp.linalg.splu(sp.csc_matrix(A))
    return lu.solve


@pytest.mark.parametrize("n,seed", [(2, 1), (5, 2), (8, 3), (12, 4)])
def test_bicgstab_finite_termination(n, seed):
    # a bi-conjugate gradient method ends within n steps in exact
    # arithmetic: on small well-conditioned systems the residual is at
    # rounding level after n iterations at most
    A = _random_pattern_matrix(n, 3 * n, seed, dominance=1.0).toarray()
    b = np.random.default_rng(seed).uniform(-1, 1, n)
    x, its, rel, ok, _ = krylov.bicgstab(A, b, lambda v: v, 1e-13, n)
    assert ok and its <= n, (its, rel)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-10 * np.max(np.abs(x)))


def test_bicgstab_with_the_exact_inverse_ends_in_one_half_step():
    # right preconditioning by A^{-1}: v = A A^{-1} p = r, so alpha = 1,
    # s = 0 and x = A^{-1} b after the first half of the first iteration
    A = _random_pattern_matrix(60, 120, 5)
    b = np.random.default_rng(5).uniform(-1, 1, 60)
    x, its, rel, ok, hist = krylov.bicgstab(A, b, _exact_solver(A), 1e-10, 10)
    assert ok and its == 1 and len(hist) == 1 and rel <= 1e-12
    assert np.allclose(A @ x, b, atol=1e-12)


def test_bicgstab_recurrence_is_the_true_residual_and_omega_minimises_it():
    A = _random_pattern_matrix(150, 400, 6, dominance=0.8)
    b = np.random.default_rng(6).uniform(-1, 1, 150)
    L, U = krylov.ilu0(A)
    rec = []
    x, its, rel, ok, hist = krylov.bicgstab(A, b, krylov.ilu0_apply(L, U), 1e-9, 200, record=rec)
    assert ok and its >= 2
    true_rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(true_rel - rel) <= 1e-9
    # the second half-step minimises ||s - omega t||: the new residual is
    # orthogonal to t, and moving omega either way makes it longer
    for it in rec:
        s, t, w = it["s"], it["t"], it["omega"]
        r = s - w * t
        assert abs(t @ r) <= 1e-10 * np.linalg.norm(t) * np.linalg.norm(s)
        for dw in (1e-3, -1e-3):
            assert np.linalg.norm(s - (w + dw) * t) > np.linalg.norm(r)
    # residuals after each iteration are those the history reports
    assert len(hist) == its


@pytest.mark.parametrize("precond", ["ilu0", "bjacobi"])
def test_bicgstab_newton_reaches_the_direct_root(precond):
    case = pfgen.make_polar_grid(300, 90, 30, 11, balanced=True)
    ref = polar.newton(case)
    res = polar.newton(case, linear="bicgstab", precond=precond)
    assert ref.status == CONVERGED and res.status == CONVERGED
    assert np.max(np.abs(res.V - ref.V)) <= 1e-8
    assert all(k >= 1 for k in res.linear_iters)


def test_bicgstab_cim_newton_reaches_the_direct_root():
    case = pfgen.make_feeder(80, 4)
    ref = cim.newton(case)
    res = cim.newton(case, linear="bicgstab")
    assert ref.status == CONVERGED and res.status == CONVERGED
    assert np.max(np.abs(res.V - ref.V)) <= 1e-8


@pytest.mark.parametrize("linear", ["gmres", "bicgstab"])
def test_fallback_finishes_a_failed_krylov_iteration_at_the_direct_root(linear):
    # a starved inner solve (one Krylov step, no restarts, a forcing term
    # the step cannot meet) fails the first Newton step; with the fallback
    # the direct solve takes that step and the rest and reaches the same
    # root as direct Newton from the flat start
    case = pfgen.make_polar_grid(300, 90, 30, 11, balanced=True)
    opts = dict(precond="bjacobi", m=2, max_restarts=0, eta_max=1e-3)
    bad = polar.newton(case, linear=linear, **opts)
    assert bad.status == LINEAR_FAIL and not bad.lu_fallback
    res = polar.newton(case, linear=linear, fallback=True, **opts)
    ref = polar.newton(case)
    assert res.status == CONVERGED and res.lu_fallback
    assert np.max(np.abs(res.V - ref.V)) <= 1e-8
    assert res.iters == ref.iters  # the failed step is not taken, the direct ones are the same
