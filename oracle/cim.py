"""Three-phase current-injection-method (CIM) Newton power flow (Sec. II-B).

Phase-nodes are the phases present at each bus; the source bus's phase-nodes
hold fixed voltages and carry no equations.  Every other phase-node has two
real unknowns (Re V, Im V) and two real equations (Im dI, Re dI).  Per bus the
order follows eq. 19-20: the equations are [Im dI of the bus's phases; Re dI of
the bus's phases] and the unknowns [Re dV of its phases; Im dV of its phases].

Specified power comes from the ZIP loads (eq. 12-15), the specified current
from eq. 17, the calculated current from the nodal sum of eq. 18 and the
mismatch from eq. 16.  The Jacobian has the blocks [B G; G -B] of eq. 21 for
every admittance entry and, on each phase-node's own diagonal, the ZIP
adjustments a, b, c, d of eq. 23:

  a = Im dI_sp/dVre, b = Im dI_sp/dVim, c = Re dI_sp/dVre, d = Re dI_sp/dVim.

Their closed form is derived here (the paper takes it from its ref. [18]): a
load component with complex coefficient s and voltage exponent e (2 for
constant impedance, 1 for constant current, 0 for constant power) draws the
current I = conj(s) V |V|^(e-2); with w = |V|^2, g = w^((e-2)/2) and
g' = ((e-2)/2) w^((e-4)/2),

  dI/dVre = conj(s) (g + 2 Vre V g'),   dI/dVim = conj(s) (j g + 2 Vim V g').
"""

import numpy as np
import scipy.sparse as sp

from . import linalg
from .result import OracleResult, CONVERGED, MAXITER, DIVERGED, SINGULAR, LINEAR_FAIL
from .ybus import as_csr

SLACK = 3


def unknown_layout(case):
    """Row and column positions of every non-source phase-node (eq. 19-20)."""
    n = case.n
    row_im = -np.ones(n, np.int64)
    row_re = -np.ones(n, np.int64)
    col_re = -np.ones(n, np.int64)
    col_im = -np.ones(n, np.int64)
    pos = 0
    nb = np.asarray(case.node_bus)
    unknown = np.asarray(case.node_type) != SLACK
    for bus in np.unique(nb[unknown]):
        nodes = np.flatnonzero((nb == bus) & unknown)
        k = nodes.shape[0]
        row_im[nodes] = pos + np.arange(k)
        row_re[nodes] = pos + k + np.arange(k)
        col_re[nodes] = pos + np.arange(k)
        col_im[nodes] = pos + k + np.arange(k)
        pos += 2 * k
    return unknown, row_im, row_re, col_re, col_im, pos


def flat_start(case):
    """Magnitude 1 (the source's set-point on source nodes) at the phase's
    nominal angle 0, -120 or +120 degrees."""
    mag = np.where(np.asarray(case.node_type) == SLACK, case.v_mag, 1.0)
    return mag * np.exp(1j * np.asarray(case.v_ang))


def specified_power(case, V):
    """Eq. 12-15: P_sp = P_g - (P_P + P_I|V| + P_Z|V|^2), same for Q."""
    vm = np.abs(V)
    z = case.zip
    p_l = z[:, 2] + z[:, 1] * vm + z[:, 0] * vm ** 2
    q_l = z[:, 5] + z[:, 4] * vm + z[:, 3] * vm ** 2
    return case.p_gen - p_l, case.q_gen - q_l


def current_mismatch_complex(case, V):
    """Eq. 16-18: dI = conj((P_sp + jQ_sp)/V) - sum_j Y_ij V_j."""
    Y = as_csr(case)
    i_calc = Y @ V
    p_sp, q_sp = specified_power(case, V)
    i_sp = np.conj((p_sp + 1j * q_sp) / V)
    return i_sp - i_calc


def mismatch(case, V):
    """The real augmented mismatch of eq. 19, over non-source phase-nodes."""
    unknown, row_im, row_re, _, _, dim = unknown_layout(case)
    dI = current_mismatch_complex(case, V)
    F = np.zeros(dim)
    u = np.flatnonzero(unknown)
    F[row_im[u]] = dI[u].imag
    F[row_re[u]] = dI[u].real
    return F


def zip_derivatives(case, V):
    """a, b, c, d of eq. 23 for every phase-node (derivation in the module
    docstring)."""
    z = case.zip
    vr, vi = V.real, V.imag
    w = vr * vr + vi * vi
    dr = np.zeros(case.n, np.complex128)
    di = np.zeros(case.n, np.complex128)
    comps = [  # (complex power coefficient s, exponent e); loads enter with -
        (-(z[:, 0] + 1j * z[:, 3]), 2),
        (-(z[:, 1] + 1j * z[:, 4]), 1),
        (-(z[:, 2] + 1j * z[:, 5]), 0),
        (case.p_gen + 1j * case.q_gen, 0),
    ]
    for s, e in comps:
        g = w ** ((e - 2) / 2.0)
        gp = ((e - 2) / 2.0) * w ** ((e - 4) / 2.0)
        cs = np.conj(s)
        dr += cs * (g + 2.0 * vr * V * gp)
        di += cs * (1j * g + 2.0 * vi * V * gp)
    return dr.imag, di.imag, dr.real, di.real


def jacobian(case, V):
    """Eq. 21-23 in the row/column order of eq. 19-20."""
    unknown, row_im, row_re, col_re, col_im, dim = unknown_layout(case)
    Y = as_csr(case)
    p = np.repeat(np.arange(case.n), np.diff(Y.indptr))
    q = Y.indices
    keep = unknown[p] & unknown[q]
    p, q = p[keep], q[keep]
    G, B = Y.data[keep].real, Y.data[keep].imag
    rows = [row_im[p], row_im[p], row_re[p], row_re[p]]
    cols = [col_re[q], col_im[q], col_re[q], col_im[q]]
    vals = [B, G, G, -B]
    a, b, c, d = zip_derivatives(case, V)
    u = np.flatnonzero(unknown)
    rows += [row_im[u], row_im[u], row_re[u], row_re[u]]
    cols += [col_re[u], col_im[u], col_re[u], col_im[u]]
    vals += [-a[u], -b[u], -c[u], -d[u]]
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim, dim))
    J.sum_duplicates()
    return J


def newton(case, tol=1e-12, max_iter=20, linear="sparse", floor_tol=1e-8, V0=None, fallback=False,
           **krylov_opts):
    """The three-phase Newton-Raphson (CIM) iteration of Sec. II-B: mismatch
    by eq. 12-20, Jacobian by eq. 21-23, solve, add dV to the real and
    imaginary parts (eq. 20 order) and convert back to complex form.  Stops on
    the max-norm of the current mismatch (and at the rounding floor as in the
    single-phase loop).  ``linear="gmres"`` or ``"bicgstab"`` solves each step inexactly as in
    the single-phase loop (Sec. III-B), with the same ``fallback`` to the
    direct solve."""
    unknown, _, _, col_re, col_im, _ = unknown_layout(case)
    u = np.flatnonzero(unknown)
    V = flat_start(case) if V0 is None else np.array(V0, np.complex128)
    history, steps, lin = [], [], []
    fell_back = False
    status = MAXITER
    if linear in ("gmres", "bicgstab"):
        from . import krylov

        node_of = np.empty(2 * u.shape[0], np.int64)
        comp_of = np.empty(2 * u.shape[0], np.int64)
        node_of[col_re[u]], comp_of[col_re[u]] = u, 0
        node_of[col_im[u]], comp_of[col_im[u]] = u, 1
        graph = as_csr(case)
    for k in range(max_iter + 1):
        F = mismatch(case, V)
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
        J = jacobian(case, V)
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
        vr = V.real.copy()
        vi = V.imag.copy()
        vr[u] += dx[col_re[u]]
        vi[u] += dx[col_im[u]]
        V = vr + 1j * vi
    return OracleResult(status=status, iters=len(steps), V=V, history=history,
                        steps=steps, mismatch_inf=history[-1], linear_iters=lin, lu_fallback=fell_back)


def mismatch_at(case, V):
    F = mismatch(case, np.asarray(V, np.complex128))
    return float(np.max(np.abs(F))) if F.size else 0.0
