"""Nodal admittance matrix, assembled from branch data (Sec. II, eq. 1-3, 11).

The assembly here uses the branch-incidence form Y = A^T y_prim A + Y_shunt:
the voltage drop across branch e is (A V)_e, its current is y_e (A V)_e, and
summing branch currents at each node gives the off-diagonal -y_ij of eq. 3 and
the diagonal sum of eq. 2 (including the j=0 ground term, the line charging).
"""

import numpy as np
import scipy.sparse as sp


def polar_ybus(case):
    """Ybus of a single-phase grid (pi-model branches, charging b/2 per end)."""
    n, m = case.n, case.m
    e = np.arange(m)
    A = sp.csr_matrix((np.concatenate([np.ones(m), -np.ones(m)]),
                       (np.concatenate([e, e]), np.concatenate([case.f, case.t]))),
                      shape=(m, n))
    y_series = 1.0 / (case.r + 1j * case.x)
    Y = (A.T @ sp.diags(y_series) @ A).tocsr()
    # ground branches (j = 0 in eq. 2): half the line charging at each end
    shunt = np.zeros(n, np.complex128)
    np.add.at(shunt, case.f, 0.5j * case.b)
    np.add.at(shunt, case.t, 0.5j * case.b)
    Y = (Y + sp.diags(shunt)).tocsr()
    Y.sort_indices()
    return Y


def feeder_ybus(case):
    """Ybus over the present phase-nodes of a three-phase feeder.

    Each branch carries the 3x3 series impedance of eq. 11 restricted to the
    phases present on the branch; its primitive admittance is the inverse of
    that sub-matrix.  Rows of the incidence matrix are (branch, phase) pairs.
    """
    node_of = -np.ones((case.n_bus, 3), np.int64)
    node_of[case.node_bus, case.node_phase] = np.arange(case.n)
    rows, cols, vals = [], [], []
    blocks = []
    r = 0
    for e in range(case.f.shape[0]):
        ch = case.t[e]
        ph = [q for q in range(3) if case.bus_phases[ch, q]]
        for q in ph:
            rows += [r, r]
            cols += [node_of[case.f[e], q], node_of[ch, q]]
            vals += [1.0, -1.0]
            r += 1
        blocks.append(np.linalg.inv(case.zbr[e][np.ix_(ph, ph)]))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(r, case.n))
    yprim = sp.block_diag(blocks, format="csr")
    Y = (A.T @ yprim @ A).tocsr()
    Y.sort_indices()
    return Y


def as_csr(case):
    """The case's own Ybus (the generator's stamping) as a SciPy matrix."""
    n = case.n
    return sp.csr_matrix((case.y, case.col, case.row_ptr), shape=(n, n))
