"""Pins of the CPU oracle against results fixed by the paper's equations and by
mathematics, independent of the oracle's own Newton code."""

import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import pfgen
from oracle import cim, polar, ybus, linalg, CONVERGED, MAXITER, DIVERGED, SINGULAR
import pins


# ---------------------------------------------------------------- Ybus (eq. 1-3, 11)


@pytest.mark.parametrize("maker", [lambda: pfgen.config_case(0),
                                   lambda: pfgen.make_polar_grid(100, 30, 10, 5),
                                   lambda: pfgen.config_case(1)])
def test_polar_ybus_stamping_equals_incidence_assembly(maker):
    c = maker()
    Ya = ybus.as_csr(c)
    Yb = ybus.polar_ybus(c)
    d = (Ya - Yb).toarray() if c.n <= 200 else (Ya - Yb).data
    assert np.max(np.abs(d)) <= 1e-12 * np.max(np.abs(Ya.data))
    assert abs(Ya - Ya.T).max() == 0.0  # eq. 3: Y_ij = Y_ji


@pytest.mark.parametrize("n_bus,seed", [(30, 1), (200, 2)])
def test_feeder_ybus_stamping_equals_incidence_assembly(n_bus, seed):
    c = pfgen.make_feeder(n_bus, seed)
    Ya = ybus.as_csr(c)
    Yb = ybus.feeder_ybus(c)
    assert abs(Ya - Yb).max() <= 1e-12 * abs(Ya).max()
    assert abs(Ya - Ya.T).max() <= 1e-12 * abs(Ya).max()


def test_csr_layout_sorted_with_diagonal():
    for c in [pfgen.config_case(0), pfgen.make_feeder(50, 3)]:
        for i in range(c.n):
            cols = c.col[c.row_ptr[i]:c.row_ptr[i + 1]]
            assert np.all(np.diff(cols) > 0)
            assert i in cols


# ---------------------------------------------------------------- closed forms


@pytest.mark.parametrize("r,x,P,Q", [(0.02, 0.1, 0.5, 0.2), (0.05, 0.05, 1.0, 0.6),
                                     (0.01, 0.2, 0.3, -0.1), (0.03, 0.08, 2.0, 1.0)])
def test_two_bus_pq_closed_form(r, x, P, Q):
    c = pins.polar_case(2, [0], [1], [r], [x], [0.0], [3, 1], [0.0, -P], [0.0, -Q], [1.0, 1.0])
    res = polar.newton(c)
    assert res.status == CONVERGED
    vm, va = pins.two_bus_pq(r, x, P, Q)
    assert abs(res.vm[1] - vm) < 1e-12
    assert abs(res.va[1] - va) < 1e-12


@pytest.mark.parametrize("r,x,b,P,Q", [(0.02, 0.1, 0.04, 0.5, 0.2), (0.04, 0.15, 0.03, 1.2, 0.4)])
def test_two_bus_pq_with_charging(r, x, b, P, Q):
    c = pins.polar_case(2, [0], [1], [r], [x], [b], [3, 1], [0.0, -P], [0.0, -Q], [1.0, 1.0])
    res = polar.newton(c)
    vm, va = pins.two_bus_pq_charging(r, x, b, P, Q)
    assert abs(res.vm[1] - vm) < 1e-12
    assert abs(res.va[1] - va) < 1e-12


@pytest.mark.parametrize("r,x,P,U", [(0.02, 0.1, 0.5, 1.02), (0.05, 0.2, 0.8, 1.0),
                                     (0.01, 0.08, -0.4, 1.05)])
def test_two_bus_pv_closed_form(r, x, P, U):
    c = pins.polar_case(2, [0], [1], [r], [x], [0.0], [3, 2], [0.0, P], [0.0, 0.0], [1.0, U])
    res = polar.newton(c)
    assert res.status == CONVERGED
    assert abs(res.vm[1] - U) == 0.0  # PV magnitude is held
    assert abs(res.va[1] - pins.two_bus_pv(r, x, P, U)) < 1e-12


# ---------------------------------------------------------------- Jacobians by finite differences


def _fd(fun, x0, h=1e-6):
    cols = []
    for k in range(x0.shape[0]):
        e = np.zeros_like(x0)
        e[k] = h
        cols.append((fun(x0 + e) - fun(x0 - e)) / (2 * h))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("maker", [lambda: pfgen.config_case(0),
                                   lambda: pfgen.make_polar_grid(100, 30, 10, 11)])
def test_polar_jacobian_matches_finite_differences(maker):
    c = maker()
    rng = np.random.default_rng(7)
    pvpq, pq = polar.index_sets(c)
    vm, va = polar.flat_start(c)
    vm = vm + np.where(c.bus_type == 1, rng.uniform(-0.05, 0.05, c.n), 0)
    va = va + np.where(c.bus_type != 3, rng.uniform(-0.2, 0.2, c.n), 0)
    npv = pvpq.shape[0]

    def F(xv):
        a, m = va.copy(), vm.copy()
        a[pvpq] = xv[:npv]
        m[pq] = xv[npv:]
        return polar.mismatch(c, m, a)

    x0 = np.concatenate([va[pvpq], vm[pq]])
    J = polar.jacobian(c, vm, va).toarray()
    Jfd = -_fd(F, x0)  # F = S_sp - S_calc, so dF/dx = -J
    assert np.max(np.abs(J - Jfd)) <= 1e-7 * np.max(np.abs(J))


@pytest.mark.parametrize("zip_mode", ["random", "Z", "I", "P"])
def test_cim_jacobian_matches_finite_differences(zip_mode):
    c = pfgen.make_feeder(25, 4, zip_mode=zip_mode, load_scale=200.0)
    c = c.with_zip(c.zip)
    rng = np.random.default_rng(3)
    unknown, _, _, col_re, col_im, dim = cim.unknown_layout(c)
    u = np.flatnonzero(unknown)
    V0 = cim.flat_start(c) * np.where(unknown, 1 + rng.uniform(-0.05, 0.05, c.n), 1)
    V0 = V0 * np.exp(1j * np.where(unknown, rng.uniform(-0.05, 0.05, c.n), 0))

    def F(xv):
        V = V0.copy()
        V[u] = xv[col_re[u]] + 1j * xv[col_im[u]]
        return cim.mismatch(c, V)

    x0 = np.zeros(dim)
    x0[col_re[u]] = V0[u].real
    x0[col_im[u]] = V0[u].imag
    J = cim.jacobian(c, V0).toarray()
    Jfd = -_fd(F, x0, h=1e-7)
    assert np.max(np.abs(J - Jfd)) <= 1e-7 * np.max(np.abs(J))
    # the ZIP adjustment is really exercised: it changes the diagonal
    a, b, cc, d = cim.zip_derivatives(c, V0)
    assert np.max(np.abs(np.concatenate([a, b, cc, d])[np.tile(unknown, 4)])) > 1e-3


# ---------------------------------------------------------------- power balance / KCL


def _branch_flows_polar(c, V):
    ys = 1.0 / (c.r + 1j * c.x)
    Vf, Vt = V[c.f], V[c.t]
    I_ft = ys * (Vf - Vt) + 0.5j * c.b * Vf
    I_tf = ys * (Vt - Vf) + 0.5j * c.b * Vt
    S = np.zeros(c.n, np.complex128)
    np.add.at(S, c.f, Vf * np.conj(I_ft))
    np.add.at(S, c.t, Vt * np.conj(I_tf))
    return S


@pytest.mark.parametrize("maker", [lambda: pfgen.config_case(0), lambda: pfgen.config_case(1)])
def test_polar_power_balance_any_voltage(maker):
    c = maker()
    rng = np.random.default_rng(1)
    vm = rng.uniform(0.9, 1.1, c.n)
    va = rng.uniform(-0.5, 0.5, c.n)
    P, Q = polar.injections(c, vm, va)
    S = _branch_flows_polar(c, vm * np.exp(1j * va))
    assert np.max(np.abs(P - S.real)) < 1e-9
    assert np.max(np.abs(Q - S.imag)) < 1e-9


def test_polar_power_balance_at_solution():
    c = pfgen.config_case(0)
    res = polar.newton(c)
    S = _branch_flows_polar(c, res.V)
    losses = np.sum(S).real
    assert losses > 0
    P, Q = polar.injections(c, res.vm, res.va)
    # slack injection = total load - PV generation + losses
    assert abs(P[0] - (-np.sum(c.p_sp[1:]) + losses)) < 1e-9


def test_cim_kcl_any_voltage():
    c = pfgen.make_feeder(60, 9)
    rng = np.random.default_rng(2)
    V = cim.flat_start(c) * (1 + 0.05 * rng.standard_normal(c.n)) * np.exp(0.05j * rng.standard_normal(c.n))
    i_calc = ybus.as_csr(c) @ V
    node_of = -np.ones((c.n_bus, 3), np.int64)
    node_of[c.node_bus, c.node_phase] = np.arange(c.n)
    I = np.zeros(c.n, np.complex128)
    for e in range(c.f.shape[0]):
        ph = [q for q in range(3) if c.bus_phases[c.t[e], q]]
        yb = np.linalg.inv(c.zbr[e][np.ix_(ph, ph)])
        kf = node_of[c.f[e], ph]
        kt = node_of[c.t[e], ph]
        ib = yb @ (V[kf] - V[kt])
        I[kf] += ib
        I[kt] -= ib
    assert np.max(np.abs(I - i_calc)) < 1e-9 * np.max(np.abs(i_calc))


# ---------------------------------------------------------------- brute force


@settings(max_examples=25, deadline=None)
@given(n=st.integers(3, 14), extra=st.integers(0, 6), npv=st.integers(0, 3),
       seed=st.integers(0, 10_000))
def test_dense_brute_force_equals_sparse_path(n, extra, npv, seed):
    c = pins.random_small_grid(n, extra, min(npv, n - 1), seed)
    a = polar.newton(c, linear="dense")
    b = polar.newton(c, linear="sparse")
    assert a.status == b.status
    assert len(a.history) == len(b.history)
    if a.status == CONVERGED:
        assert np.max(np.abs(a.V - b.V)) < 1e-12


def test_dense_lu_solve_matches_library():
    rng = np.random.default_rng(0)
    for n in [1, 2, 5, 30, 60]:
        A = rng.standard_normal((n, n)) + n * np.eye(n) * rng.uniform(0, 1)
        b = rng.standard_normal(n)
        x = linalg.dense_lu_solve(A, b)
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    # a matrix that needs row exchanges
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    assert np.allclose(linalg.dense_lu_solve(A, np.array([2.0, 3.0])), [3.0, 2.0])


def test_cim_dense_equals_sparse():
    c = pfgen.make_feeder(12, 5)
    a = cim.newton(c, linear="dense")
    b = cim.newton(c, linear="sparse")
    assert a.status == b.status == CONVERGED
    assert np.max(np.abs(a.V - b.V)) < 1e-12


# ---------------------------------------------------------------- three-phase cross checks


def test_balanced_feeder_equals_single_phase_solution():
    fc = pfgen.make_feeder(80, 13, laterals=False, balanced=True, zip_mode="P", load_scale=30.0)
    pc = pins.polar_equivalent_of_balanced_feeder(fc)
    r3 = cim.newton(fc)
    r1 = polar.newton(pc)
    assert r3.status == r1.status == CONVERGED
    rot = np.exp(-2j * math.pi / 3 * np.array([0, 1, -1]))
    V3 = r1.V[fc.node_bus] * rot[fc.node_phase]
    assert np.max(np.abs(r3.V - V3)) < 1e-10


def test_all_impedance_loads_converge_in_one_step():
    c = pfgen.make_feeder(120, 17, zip_mode="Z", load_scale=40.0)
    res = cim.newton(c)
    assert res.status == CONVERGED
    assert res.history[1] < 1e-10
    Y = ybus.as_csr(c).toarray()
    u = np.flatnonzero(c.node_type != 3)
    s = np.flatnonzero(c.node_type == 3)
    A = Y[np.ix_(u, u)] + np.diag(c.zip[u, 0] - 1j * c.zip[u, 3])
    Vs = cim.flat_start(c)[s]
    Vu = np.linalg.solve(A, -Y[np.ix_(u, s)] @ Vs)
    assert np.max(np.abs(res.V[u] - Vu)) < 1e-11


@pytest.mark.parametrize("n_bus,seed,zip_mode", [(40, 21, "random"), (150, 22, "P"), (300, 23, "random")])
def test_ladder_sweep_equals_cim(n_bus, seed, zip_mode):
    c = pfgen.make_feeder(n_bus, seed, zip_mode=zip_mode)
    res = cim.newton(c)
    assert res.status == CONVERGED
    V = pins.ladder_sweep(c)
    assert np.max(np.abs(res.V - V)) < 1e-9


# ---------------------------------------------------------------- invariances and convergence


def test_permutation_invariance():
    c = pfgen.make_polar_grid(60, 20, 6, 31)
    rng = np.random.default_rng(4)
    perm = rng.permutation(c.n)  # new index of old bus i is perm[i]
    inv = np.argsort(perm)
    f, t = perm[c.f], perm[c.t]
    cp = pins.polar_case(c.n, f, t, c.r, c.x, c.b, c.bus_type[inv], c.p_sp[inv],
                         c.q_sp[inv], c.v_mag[inv], c.v_ang[inv])
    a = polar.newton(c)
    b = polar.newton(cp)
    assert a.status == b.status == CONVERGED
    assert np.max(np.abs(b.V[perm] - a.V)) < 1e-12


@pytest.mark.parametrize("cfg", [0, 1])
def test_quadratic_convergence(cfg):
    c = pfgen.config_case(cfg)
    h = polar.newton(c).history
    for a, b in zip(h[:-1], h[1:]):
        if a < 1e-2 and b > 1e-12:
            assert b <= 10.0 * a * a


def test_cim_quadratic_convergence():
    h = cim.newton(pfgen.config_case(2)).history
    for a, b in zip(h[:-1], h[1:]):
        if a < 1e-2 and b > 1e-10:
            assert b <= 100.0 * a * a


# ---------------------------------------------------------------- outcome statuses


def test_status_maxiter():
    assert polar.newton(pfgen.config_case(0), max_iter=1).status == MAXITER


def test_status_singular_islanded_bus():
    c = pins.polar_case(3, [0], [1], [0.02], [0.1], [0.0], [3, 1, 1],
                        [0, -0.3, -0.1], [0, -0.1, -0.05], [1, 1, 1])
    # bus 2 has no branch: its row of Y holds only an explicit zero diagonal
    c.row_ptr = np.array([0, 2, 4, 5], np.int32)
    c.col = np.array([0, 1, 0, 1, 2], np.int32)
    c.y = np.concatenate([c.y, [0j]])
    assert polar.newton(c).status == SINGULAR


def test_status_diverged_or_no_solution_when_overloaded():
    c = pfgen.config_case(0)
    c = c.with_injections(c.p_sp * 50, c.q_sp * 50)
    assert polar.newton(c).status in (DIVERGED, MAXITER)


def test_reference_workloads_converge():
    r0 = polar.newton(pfgen.config_case(0))
    assert r0.status == CONVERGED and r0.mismatch_inf < 1e-12
    r2 = cim.newton(pfgen.config_case(2))
    assert r2.status == CONVERGED and r2.mismatch_inf < 1e-10
    vmin = r2.vm[pfgen.config_case(2).node_type != 3].min()
    assert 0.93 <= vmin <= 0.96
