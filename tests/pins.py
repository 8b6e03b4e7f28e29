"""Independent reference results that pin the oracle.

None of these reuse the oracle's Newton code: they are closed forms, a ladder
(backward/forward sweep) solver for radial feeders and small case builders.
"""

import math

import numpy as np

import pfgen
from pfgen.grids import PolarCase, PQ, PV, SLACK, _stamp_csr


def polar_case(n, f, t, r, x, b, bus_type, p_sp, q_sp, v_mag, v_ang=None, name="hand"):
    """A PolarCase from a branch list (Ybus by the generator's stamping)."""
    f = np.asarray(f, np.int32)
    t = np.asarray(t, np.int32)
    r = np.asarray(r, float)
    x = np.asarray(x, float)
    b = np.asarray(b, float)
    ys = 1.0 / (r + 1j * x)
    sh = 0.5j * b
    rows = np.concatenate([f, t, f, t])
    cols = np.concatenate([f, t, t, f])
    vals = np.concatenate([ys + sh, ys + sh, -ys, -ys])
    row_ptr, col, y = _stamp_csr(n, rows, cols, vals)
    return PolarCase(name=name, n=n, f=f, t=t, r=r, x=x, b=b, row_ptr=row_ptr,
                     col=col, y=y, bus_type=np.asarray(bus_type, np.int8),
                     p_sp=np.asarray(p_sp, float), q_sp=np.asarray(q_sp, float),
                     v_mag=np.asarray(v_mag, float),
                     v_ang=np.zeros(n) if v_ang is None else np.asarray(v_ang, float))


def two_bus_pq(r, x, P, Q, U1=1.0):
    """Closed form of a slack bus feeding a PQ load P + jQ over z = r + jx.

    With w = |V2|^2:  U1^2 w = (w + rP + xQ)^2 + (xP - rQ)^2, i.e.
    w^2 + (2(rP + xQ) - U1^2) w + |z|^2 (P^2 + Q^2) = 0; the high-voltage
    ("+") root is the flat-start Newton solution, and
    angle2 = -atan2(xP - rQ, w + rP + xQ).
    """
    bq = 2.0 * (r * P + x * Q) - U1 ** 2
    cq = (r * r + x * x) * (P * P + Q * Q)
    w = (-bq + math.sqrt(bq * bq - 4.0 * cq)) / 2.0
    ang = -math.atan2(x * P - r * Q, w + r * P + x * Q)
    return math.sqrt(w), ang


def two_bus_pq_charging(r, x, b, P, Q, U1=1.0):
    """Same with total line charging b: the bus-2 half shunt (b/2) adds
    -(b/2) w to the reactive load, so U1^2 w = (w + rP + xQ')^2 + (xP - rQ')^2
    with Q' = Q - (b/2) w; solved by bisection on the high-voltage branch."""

    def g(w):
        q = Q - 0.5 * b * w
        return (w + r * P + x * q) ** 2 + (x * P - r * q) ** 2 - U1 ** 2 * w

    lo, hi = 0.5, 1.5
    assert g(lo) < 0 < g(hi) or g(lo) > 0 > g(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (g(mid) > 0) == (g(hi) > 0):
            hi = mid
        else:
            lo = mid
    w = 0.5 * (lo + hi)
    q = Q - 0.5 * b * w
    ang = -math.atan2(x * P - r * q, w + r * P + x * q)
    return math.sqrt(w), ang


def two_bus_pv(r, x, P2, U, U1=1.0):
    """Closed form of a PV bus (|V2| = U, injection P2) behind z = r + jx:
    P2 = U^2 g - U U1 (g cos d + b sin d) with y = g + jb = 1/z, so
    d = phi +- arccos(rho / R), R = |y|, phi = atan2(b, g),
    rho = (U^2 g - P2) / (U U1); the root of smaller |d| is the solution."""
    z2 = r * r + x * x
    g, b = r / z2, -x / z2
    R = math.hypot(g, b)
    phi = math.atan2(b, g)
    rho = (U * U * g - P2) / (U * U1)
    c = math.acos(rho / R)
    cands = [phi + c, phi - c]
    cands = [math.atan2(math.sin(d), math.cos(d)) for d in cands]
    return min(cands, key=abs)


def ladder_sweep(case, tol=1e-13, max_iter=500):
    """Backward/forward sweep of a radial three-phase feeder.

    Backward: every branch carries the sum of the load currents of the
    subtree below it.  Forward: each child voltage is its parent's minus the
    branch impedance times the branch current.  Load current of a phase-node
    is conj(S_load / V) with S_load from the ZIP model.
    """
    nb = case.n_bus
    node_of = -np.ones((nb, 3), np.int64)
    node_of[case.node_bus, case.node_phase] = np.arange(case.n)
    parent = -np.ones(nb, np.int64)
    zbr_of = [None] * nb
    for e in range(case.f.shape[0]):
        parent[case.t[e]] = case.f[e]
        zbr_of[case.t[e]] = case.zbr[e]
    order = np.argsort(_depths(parent))  # parents before children
    V = case.v_mag * np.exp(1j * case.v_ang)
    V = V.astype(np.complex128)
    z = case.zip
    for _ in range(max_iter):
        vm = np.abs(V)
        s_load = (z[:, 2] + z[:, 1] * vm + z[:, 0] * vm ** 2) + 1j * (
            z[:, 5] + z[:, 4] * vm + z[:, 3] * vm ** 2)
        s_load = s_load - (case.p_gen + 1j * case.q_gen)
        i_load = np.conj(s_load / V)
        i_load[case.node_type == SLACK] = 0.0
        # bus-level 3-vectors of subtree current
        J = np.zeros((nb, 3), np.complex128)
        for bus in range(nb):
            for ph in range(3):
                k = node_of[bus, ph]
                if k >= 0:
                    J[bus, ph] = i_load[k]
        for bus in order[::-1]:
            p = parent[bus]
            if p >= 0:
                J[p] += J[bus]
        Vn = V.copy()
        for bus in order:
            p = parent[bus]
            if p < 0:
                continue
            ph = [q for q in range(3) if node_of[bus, q] >= 0]
            zs = zbr_of[bus][np.ix_(ph, ph)]
            drop = zs @ J[bus, ph]
            for u, q in enumerate(ph):
                Vn[node_of[bus, q]] = Vn[node_of[p, q]] - drop[u]
        delta = np.max(np.abs(Vn - V))
        V = Vn
        if delta < tol:
            return V
    raise RuntimeError("ladder sweep did not converge")


def _depths(parent):
    nb = parent.shape[0]
    d = np.zeros(nb, np.int64)
    for i in range(nb):
        k, c = i, 0
        while parent[k] >= 0:
            k = parent[k]
            c += 1
        d[i] = c
    return d


def polar_equivalent_of_balanced_feeder(fc):
    """Single-phase grid with the positive-sequence impedance of a balanced
    feeder (self minus mutual) and its per-phase constant-power loads."""
    nb = fc.n_bus
    z1 = np.array([fc.zbr[e][0, 0] - fc.zbr[e][0, 1] for e in range(fc.f.shape[0])])
    node_a = np.flatnonzero(fc.node_phase == 0)
    p = -fc.zip[node_a, 2]
    q = -fc.zip[node_a, 5]
    bt = np.full(nb, PQ)
    bt[0] = SLACK
    return polar_case(nb, fc.f, fc.t, z1.real, z1.imag, np.zeros(nb - 1), bt, p, q,
                      np.ones(nb), name="balanced-equivalent")


def random_small_grid(n, extra, n_pv, seed):
    return pfgen.make_polar_grid(n, extra, n_pv, seed, balanced=False)
