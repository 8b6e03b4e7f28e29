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

Two additions the paper names but leaves out (Sec. II-B: distributed
generation as PV buses is "not yet added"), written here in the
current-injection form of its ref. [18]:

* PV phase-nodes (voltage-controlled generation): the generator's Q is one
  more unknown per PV node and |V| = set-point one more equation.  The
  augmented system appends, after the rows and columns of eq. 19-20, one row
  per PV node, d|V| = (Vre dVre + Vim dVim)/|V| against the residual
  |V|_sp - |V|, and one column per PV node, the node's current response to
  its Q: -dI_sp/dQ = -(Vim - j Vre)/|V|^2 (from I_sp = conj((P + jQ)/V)).
* Delta-connected ZIP loads between two phase-nodes k and t of one bus: the
  load draws I_d = conj(S(|V_d|)/V_d) from k into t, with V_d = V_k - V_t and
  S = s_Z (|V_d|/sqrt3)^2 + s_I |V_d|/sqrt3 + s_P (coefficients at the nominal
  line-to-line voltage sqrt(3) pu); it enters I_sp with -I_d at k and +I_d at
  t, and the Jacobian with the 2x2 derivative D = dI_d/dV_d as +D, -D in
  row k and -D, +D in row t (columns k, t).
"""

import numpy as np
import scipy.sparse as sp

from . import linalg
from .result import OracleResult, CONVERGED, MAXITER, DIVERGED, SINGULAR, LINEAR_FAIL
from .ybus import as_csr

SLACK = 3
PV = 2
SQRT3 = np.sqrt(3.0)


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
    """Magnitude 1 (the set-point on source and PV nodes) at the phase's
    nominal angle 0, -120 or +120 degrees."""
    t = np.asarray(case.node_type)
    mag = np.where((t == SLACK) | (t == PV), case.v_mag, 1.0)
    return mag * np.exp(1j * np.asarray(case.v_ang))


def pv_nodes(case):
    return np.flatnonzero(np.asarray(case.node_type) == PV)


def specified_power(case, V, q_gen=None):
    """Eq. 12-15: P_sp = P_g - (P_P + P_I|V| + P_Z|V|^2), same for Q (wye
    loads; ``q_gen`` replaces the case's generator Q when given)."""
    vm = np.abs(V)
    z = case.zip
    p_l = z[:, 2] + z[:, 1] * vm + z[:, 0] * vm ** 2
    q_l = z[:, 5] + z[:, 4] * vm + z[:, 3] * vm ** 2
    return case.p_gen - p_l, (case.q_gen if q_gen is None else q_gen) - q_l


def _delta_links(case):
    if case.delta_to is None:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    dt = np.asarray(case.delta_to, np.int64)
    k = np.flatnonzero(dt >= 0)
    return k, dt[k]


def _delta_components(zd):
    """(complex coefficient, exponent) of delta loads, scaled so that the load
    is s (|V_d| / sqrt3)^e."""
    return [((zd[:, 0] + 1j * zd[:, 3]) / 3.0, 2),
            ((zd[:, 1] + 1j * zd[:, 4]) / SQRT3, 1),
            (zd[:, 2] + 1j * zd[:, 5], 0)]


def delta_currents(case, V):
    """Current I_d each delta load draws from its first node into its second."""
    k, t = _delta_links(case)
    if not k.size:
        return k, t, np.zeros(0, np.complex128)
    Vd = V[k] - V[t]
    w = np.abs(Vd)
    S = sum(s * w ** e for s, e in _delta_components(case.zip_delta[k]))
    return k, t, np.conj(S / Vd)


def specified_current(case, V, q_gen=None):
    """Eq. 17 for the wye loads and generation, plus the delta loads."""
    p_sp, q_sp = specified_power(case, V, q_gen)
    i_sp = np.conj((p_sp + 1j * q_sp) / V)
    k, t, Id = delta_currents(case, V)
    np.add.at(i_sp, k, -Id)
    np.add.at(i_sp, t, Id)
    return i_sp


def pv_reactive(case, V):
    """Generator Q of every node: the case's value, and on PV nodes the Q that
    balances the node's reactive power at V exactly,
    Q_g = Im(V conj(I_calc - I_delta)) + Q_l(|V|), I_delta the delta loads'
    net current into the node (the remaining current mismatch of a PV node is
    then its active-power mismatch over conj(V))."""
    q = np.array(case.q_gen, np.float64)
    pv = pv_nodes(case)
    if pv.size:
        i_calc = as_csr(case) @ V
        idn = np.zeros(case.n, np.complex128)
        k, t, Id = delta_currents(case, V)
        np.add.at(idn, k, -Id)
        np.add.at(idn, t, Id)
        vm = np.abs(V[pv])
        z = case.zip[pv]
        q_l = z[:, 5] + z[:, 4] * vm + z[:, 3] * vm ** 2
        q[pv] = (V[pv] * np.conj(i_calc[pv] - idn[pv])).imag + q_l
    return q


def current_mismatch_complex(case, V, q_gen=None):
    """Eq. 16-18: dI = I_sp - sum_j Y_ij V_j (PV nodes at ``q_gen``, by
    default the balancing Q of pv_reactive)."""
    Y = as_csr(case)
    i_calc = Y @ V
    if q_gen is None:
        q_gen = pv_reactive(case, V)
    return specified_current(case, V, q_gen) - i_calc


def mismatch(case, V, q_gen=None):
    """The real augmented mismatch of eq. 19 over non-source phase-nodes,
    followed by |V|_sp - |V| of every PV node."""
    unknown, row_im, row_re, _, _, dim = unknown_layout(case)
    dI = current_mismatch_complex(case, V, q_gen)
    pv = pv_nodes(case)
    F = np.zeros(dim + pv.shape[0])
    u = np.flatnonzero(unknown)
    F[row_im[u]] = dI[u].imag
    F[row_re[u]] = dI[u].real
    F[dim:] = case.v_mag[pv] - np.abs(V[pv])
    return F


def _load_derivative(comps, V):
    """dI/dVre and dI/dVim of the current sum_k conj(s_k) V |V|^(e_k - 2)."""
    vr, vi = V.real, V.imag
    w = vr * vr + vi * vi
    dr = np.zeros(V.shape[0], np.complex128)
    di = np.zeros(V.shape[0], np.complex128)
    for s, e in comps:
        g = w ** ((e - 2) / 2.0)
        gp = ((e - 2) / 2.0) * w ** ((e - 4) / 2.0)
        cs = np.conj(s)
        dr += cs * (g + 2.0 * vr * V * gp)
        di += cs * (1j * g + 2.0 * vi * V * gp)
    return dr, di


def zip_derivatives(case, V, q_gen=None):
    """a, b, c, d of eq. 23 for every phase-node (derivation in the module
    docstring)."""
    z = case.zip
    comps = [  # (complex power coefficient s, exponent e); loads enter with -
        (-(z[:, 0] + 1j * z[:, 3]), 2),
        (-(z[:, 1] + 1j * z[:, 4]), 1),
        (-(z[:, 2] + 1j * z[:, 5]), 0),
        (case.p_gen + 1j * (case.q_gen if q_gen is None else q_gen), 0),
    ]
    dr, di = _load_derivative(comps, V)
    return dr.imag, di.imag, dr.real, di.real


def jacobian(case, V, q_gen=None):
    """Eq. 21-23 in the row/column order of eq. 19-20, with the delta loads'
    blocks, and the PV rows and columns appended (module docstring)."""
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
    a, b, c, d = zip_derivatives(case, V, q_gen)
    u = np.flatnonzero(unknown)
    rows += [row_im[u], row_im[u], row_re[u], row_re[u]]
    cols += [col_re[u], col_im[u], col_re[u], col_im[u]]
    vals += [-a[u], -b[u], -c[u], -d[u]]
    k, t = _delta_links(case)
    if k.size:
        Vd = V[k] - V[t]
        dr, di = _load_derivative(_delta_components(case.zip_delta[k]), Vd)
        for r_node, c_node, sgn in ((k, k, 1.0), (k, t, -1.0), (t, k, -1.0), (t, t, 1.0)):
            m = unknown[r_node] & unknown[c_node]
            rn, cn = r_node[m], c_node[m]
            rows += [row_im[rn], row_im[rn], row_re[rn], row_re[rn]]
            cols += [col_re[cn], col_im[cn], col_re[cn], col_im[cn]]
            vals += [sgn * dr[m].imag, sgn * di[m].imag, sgn * dr[m].real, sgn * di[m].real]
    pv = pv_nodes(case)
    npv = pv.shape[0]
    if npv:
        j = dim + np.arange(npv)
        vr, vi = V[pv].real, V[pv].imag
        w = vr * vr + vi * vi
        vm = np.sqrt(w)
        rows += [j, j, row_re[pv], row_im[pv]]
        cols += [col_re[pv], col_im[pv], j, j]
        vals += [vr / vm, vi / vm, -vi / w, vr / w]
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim + npv, dim + npv))
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
    direct solve.  PV nodes carry their generator Q as one more unknown
    each (module docstring), starting from the case's q_gen; the Krylov
    methods here take cases without PV nodes."""
    unknown, _, _, col_re, col_im, dim = unknown_layout(case)
    u = np.flatnonzero(unknown)
    pv = pv_nodes(case)
    if pv.size and linear in ("gmres", "bicgstab"):
        raise NotImplementedError("the oracle's Krylov steps take cases without PV nodes")
    qg = np.array(case.q_gen, np.float64)
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
        F = mismatch(case, V, qg)
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
        J = jacobian(case, V, qg)
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
        qg[pv] += dx[dim:]
    return OracleResult(status=status, iters=len(steps), V=V, history=history,
                        steps=steps, mismatch_inf=history[-1], linear_iters=lin, lu_fallback=fell_back,
                        q_gen=qg)


def mismatch_at(case, V):
    F = mismatch(case, np.asarray(V, np.complex128))
    return float(np.max(np.abs(F))) if F.size else 0.0
