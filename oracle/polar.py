"""Single-phase polar Newton-Raphson power flow (Sec. II-A).

Unknowns are the angles of every non-slack bus and the magnitudes of the PQ
buses; equations are the active-power mismatch of every non-slack bus and the
reactive-power mismatch of every PQ bus (the buses whose P or Q is specified,
eq. 8-10).  Injections use the polar sums of eq. 6-7 directly; the Jacobian
blocks J1-J4 of eq. 10 are the first derivatives of eq. 6-7, written out
element by element below.
"""

import numpy as np

from . import linalg
from .result import OracleResult, CONVERGED, MAXITER, DIVERGED, SINGULAR, LINEAR_FAIL
from .ybus import as_csr

PQ, PV, SLACK = 1, 2, 3


def index_sets(case):
    """Non-slack buses (rows of dP, columns of d-angle) and PQ buses (rows of
    dQ, columns of d|V|), each in ascending bus order."""
    t = np.asarray(case.bus_type)
    pvpq = np.flatnonzero(t != SLACK)
    pq = np.flatnonzero(t == PQ)
    return pvpq, pq


def flat_start(case):
    """|V| = 1 on PQ buses and the set-point elsewhere; angle 0 except the
    slack's set-point."""
    t = np.asarray(case.bus_type)
    vm = np.where(t == PQ, 1.0, case.v_mag).astype(np.float64)
    va = np.where(t == SLACK, case.v_ang, 0.0).astype(np.float64)
    return vm, va


def _entries(case):
    Y = as_csr(case)
    rows = np.repeat(np.arange(case.n), np.diff(Y.indptr))
    return Y, rows, Y.indices, np.abs(Y.data), np.angle(Y.data)


def injections(case, vm, va):
    """Eq. 6-7: P_i = sum_j |V_i||V_j||Y_ij| cos(theta_ij - d_i + d_j),
    Q_i = -sum_j |V_i||V_j||Y_ij| sin(theta_ij - d_i + d_j)."""
    _, i, j, ymag, th = _entries(case)
    arg = th - va[i] + va[j]
    w = vm[i] * vm[j] * ymag
    P = np.bincount(i, w * np.cos(arg), minlength=case.n)
    Q = -np.bincount(i, w * np.sin(arg), minlength=case.n)
    return P, Q


def mismatch(case, vm, va):
    """Eq. 8-9 stacked as [dP over non-slack buses; dQ over PQ buses]."""
    pvpq, pq = index_sets(case)
    P, Q = injections(case, vm, va)
    return np.concatenate([case.p_sp[pvpq] - P[pvpq], case.q_sp[pq] - Q[pq]])


def jacobian(case, vm, va):
    """Eq. 10: J = d(P, Q)/d(angle, |V|) restricted to the index sets.

    Off the diagonal (i != j), with a_ij = theta_ij - d_i + d_j:
      dP_i/dd_j   = -|V_i||V_j||Y_ij| sin a_ij
      dP_i/d|V_j| =  |V_i||Y_ij| cos a_ij
      dQ_i/dd_j   = -|V_i||V_j||Y_ij| cos a_ij
      dQ_i/d|V_j| = -|V_i||Y_ij| sin a_ij
    On the diagonal, with G + jB = Y_ii:
      dP_i/dd_i   = -Q_i - B|V_i|^2      dP_i/d|V_i| = P_i/|V_i| + G|V_i|
      dQ_i/dd_i   =  P_i - G|V_i|^2      dQ_i/d|V_i| = Q_i/|V_i| - B|V_i|
    """
    import scipy.sparse as sp

    n = case.n
    Y, i, j, ymag, th = _entries(case)
    P, Q = injections(case, vm, va)
    arg = th - va[i] + va[j]
    off = i != j
    s, c = np.sin(arg), np.cos(arg)
    j11 = np.where(off, -vm[i] * vm[j] * ymag * s, 0.0)
    j12 = np.where(off, vm[i] * ymag * c, 0.0)
    j21 = np.where(off, -vm[i] * vm[j] * ymag * c, 0.0)
    j22 = np.where(off, -vm[i] * ymag * s, 0.0)
    d = np.flatnonzero(~off)
    ii = i[d]
    G, B = Y.data[d].real, Y.data[d].imag
    j11[d] = -Q[ii] - B * vm[ii] ** 2
    j12[d] = P[ii] / vm[ii] + G * vm[ii]
    j21[d] = P[ii] - G * vm[ii] ** 2
    j22[d] = Q[ii] / vm[ii] - B * vm[ii]

    def mat(v):
        return sp.csr_matrix((v, (i, j)), shape=(n, n))

    pvpq, pq = index_sets(case)
    J1 = mat(j11)[pvpq][:, pvpq]
    J2 = mat(j12)[pvpq][:, pq]
    J3 = mat(j21)[pq][:, pvpq]
    J4 = mat(j22)[pq][:, pq]
    return sp.bmat([[J1, J2], [J3, J4]], format="csr")


def newton(case, tol=1e-12, max_iter=20, linear="sparse", floor_tol=1e-8, vm0=None, va0=None, fallback=False,
           **krylov_opts):
    """The single-phase Newton-Raphson iteration of Sec. II-A.

    Each step evaluates the mismatch (eq. 8-9), stops if its max-norm is at
    most ``tol``, else builds J (eq. 10), solves J dx = F and adds dx to the
    angles of non-slack buses and the magnitudes of PQ buses.  The loop also
    stops at the rounding floor: once the max-norm is at most ``floor_tol`` and
    two steps in a row bring no tenfold decrease below the best earlier norm,
    the result is reported as converged.

    ``linear="gmres"`` or ``"bicgstab"`` makes it the Newton-Krylov
    iteration of Sec. III-B: the step is solved inexactly by
    ``krylov.inexact_step`` with that method (options
    ``precond``, ``m``, ``max_restarts``, ``eta_max``); a step whose relative
    residual misses its forcing term but is at most ``eta_max`` is taken, a
    worse one ends the iteration with status LINEAR_FAIL, or, with
    ``fallback``, hands the iteration to the direct solve from that step on.
    """
    pvpq, pq = index_sets(case)
    npv = pvpq.shape[0]
    vm, va = flat_start(case)
    if vm0 is not None:
        vm = np.array(vm0, np.float64)
        va = np.array(va0, np.float64)
    history, steps, lin = [], [], []
    fell_back = False
    status = MAXITER
    if linear in ("gmres", "bicgstab"):
        from . import krylov

        node_of = np.concatenate([pvpq, pq])
        comp_of = np.concatenate([np.zeros(npv, np.int64), np.ones(pq.shape[0], np.int64)])
        graph = as_csr(case)
    for k in range(max_iter + 1):
        F = mismatch(case, vm, va)
        nrm = float(np.max(np.abs(F))) if F.size else 0.0
        history.append(nrm)
        if not np.isfinite(nrm) or nrm > 1e6 * max(history[0], 1e-300):
            status = DIVERGED
            break
        if nrm <= tol:
            status = CONVERGED
            break
        if nrm <= floor_tol and k >= 2 and min(history[-2:]) >= 0.1 * min(history[:-2]):
            # below the acceptance bound and no tenfold progress over two
            # steps: the rounding floor
            status = CONVERGED
            break
        if k == max_iter:
            status = MAXITER
            break
        J = jacobian(case, vm, va)
        if linear in ("gmres", "bicgstab"):
            try:
                dx, info = krylov.inexact_step(J, F, nrm, node_of, comp_of, graph, method=linear,
                                               **krylov_opts)
            except (ArithmeticError, np.linalg.LinAlgError):
                status = SINGULAR
                break
            lin.append(info["iters"])
            if not info["met"] and not info["rel"] <= krylov_opts.get("eta_max", 0.1):
                if not fallback:
                    status = LINEAR_FAIL
                    break
                # the direct method takes over from the failed step on
                # (Sec. III-A: it solves where the Krylov method fails)
                linear, fell_back = "sparse", True
        if linear not in ("gmres", "bicgstab"):
            try:
                dx = linalg.solve(J, F, linear)
            except linalg.SingularError:
                status = SINGULAR
                break
        steps.append(float(np.max(np.abs(dx))))
        va[pvpq] += dx[:npv]
        vm[pq] += dx[npv:]
    V = vm * np.exp(1j * va)
    return OracleResult(status=status, iters=len(steps), V=V, history=history,
                        steps=steps, mismatch_inf=history[-1], linear_iters=lin, lu_fallback=fell_back)


def mismatch_at(case, V):
    """Max-norm of eq. 8-9 at a given complex voltage vector."""
    F = mismatch(case, np.abs(V), np.angle(V))
    return float(np.max(np.abs(F))) if F.size else 0.0
