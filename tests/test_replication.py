"""Replication-scale cases (Sec. IV): the seeded copies of a 30-bus block
joined by random links, and the copies of a 906-bus feeder behind one
substation branch.  Checks the generators' structure, their admittance
matrices against the oracle's own assembly from branch data, and the oracle's
Newton roots on them against facts that do not come from the oracle: branch
power flows, the ladder (forward-backward sweep) method on the radial feeder,
and the symmetry of identical feeder copies.
"""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import pfgen
from pfgen import grids
from oracle import cim, polar, ybus

from pins import ladder_sweep

SEED_P = grids.REPLICATION_SEED_POLAR
SEED_F = grids.REPLICATION_SEED_FEEDER


def _base_block():
    return pfgen.make_polar_grid(30, 12, 5, SEED_P, balanced=True)


def test_polar_replica_structure():
    R = 40
    c = pfgen.replicate_polar(R, SEED_P)
    base = _base_block()
    mb = base.m
    assert (c.n, c.m) == (30 * R, mb * R + 2 * (R - 1))
    assert mb == 41
    assert c.bus_type[0] == pfgen.SLACK and (c.bus_type == pfgen.SLACK).sum() == 1
    # each copy keeps its 5 PV buses; the former slack of copies 1.. is one more
    assert (c.bus_type == pfgen.PV).sum() == 5 * R + (R - 1)
    for r in (0, 1, 17, R - 1):
        sl = slice(30 * r, 30 * r + 30)
        np.testing.assert_array_equal(c.f[mb * r:mb * (r + 1)] - 30 * r, base.f)
        np.testing.assert_array_equal(c.t[mb * r:mb * (r + 1)] - 30 * r, base.t)
        np.testing.assert_array_equal(c.r[mb * r:mb * (r + 1)], base.r)
        np.testing.assert_array_equal(c.q_sp[sl][1:], base.q_sp[1:])
        np.testing.assert_array_equal(c.p_sp[sl][1:], base.p_sp[1:])
    load = -base.p_sp[base.bus_type == pfgen.PQ].sum()
    np.testing.assert_allclose(c.p_sp[30::30], grids.REPLICA_LOSS_FRAC * load, rtol=0, atol=1e-15)
    # links: from an earlier copy to a later one, each repeating a base branch
    # (its ends and its impedance)
    lf, lt = c.f[mb * R:], c.t[mb * R:]
    assert (lf // 30 < lt // 30).all()
    assert np.array_equal(np.sort(lt // 30), np.repeat(np.arange(1, R), 2))
    branch = {(int(a), int(b)): (ra, xa, ba) for a, b, ra, xa, ba in zip(base.f, base.t, base.r, base.x, base.b)}
    for k in range(lf.shape[0]):
        key = (int(lf[k] % 30), int(lt[k] % 30))
        assert key in branch
        assert branch[key] == (c.r[mb * R + k], c.x[mb * R + k], c.b[mb * R + k])
    # one connected grid with loops across copies
    A = sp.coo_matrix((np.ones(c.m), (c.f, c.t)), shape=(c.n, c.n))
    assert connected_components(A, directed=False)[0] == 1
    assert c.m > c.n - 1


def test_polar_replica_ybus_matches_branch_assembly():
    c = pfgen.replicate_polar(200, SEED_P)
    Y = ybus.polar_ybus(c)
    A = ybus.as_csr(c)
    assert abs(Y - A).max() <= 1e-12 * abs(A).max()


def test_polar_replica_root_balances_branch_flows():
    # at the oracle's root of a 3,000-bus replica, the power leaving every
    # bus through its branches (computed from branch data alone) equals the
    # specified injection at PQ buses and the specified P at PV buses
    c = pfgen.replicate_polar(100, SEED_P)
    res = polar.newton(c)
    assert res.status == 0
    V = res.V
    ys = 1.0 / (c.r + 1j * c.x)
    Vf, Vt = V[c.f], V[c.t]
    S = np.zeros(c.n, np.complex128)
    np.add.at(S, c.f, Vf * np.conj(ys * (Vf - Vt) + 0.5j * c.b * Vf))
    np.add.at(S, c.t, Vt * np.conj(ys * (Vt - Vf) + 0.5j * c.b * Vt))
    pq = c.bus_type == pfgen.PQ
    pv = c.bus_type == pfgen.PV
    assert np.max(np.abs(S.real[pq | pv] - c.p_sp[pq | pv])) < 1e-8
    assert np.max(np.abs(S.imag[pq] - c.q_sp[pq])) < 1e-8
    np.testing.assert_allclose(np.abs(V[pv]), c.v_mag[pv], rtol=0, atol=1e-12)
    # the loss allowance of the copies keeps the one slack's output small
    assert abs(S[0].real) < 0.05


def test_feeder_replica_structure():
    R = 3
    c = pfgen.replicate_feeder(R, SEED_F)
    base = pfgen.make_feeder(906, SEED_F)
    assert c.n_bus == 2 + 905 * R and c.n == 6 + (base.n - 3) * R
    assert c.f.shape[0] == c.n_bus - 1
    assert (c.node_type == pfgen.SLACK).sum() == 3 and (c.node_type[:3] == pfgen.SLACK).all()
    np.testing.assert_allclose(c.zbr[0], np.eye(3) * grids.SUBSTATION_Z / R)
    per = base.n - 3
    for r in range(R):
        sl = slice(6 + r * per, 6 + (r + 1) * per)
        np.testing.assert_array_equal(c.zip[sl], base.zip[3:])
        np.testing.assert_array_equal(c.node_phase[sl], base.node_phase[3:])
    # a tree: every bus but the source has one parent
    assert np.array_equal(np.sort(c.t), np.arange(1, c.n_bus))
    A = sp.coo_matrix((np.ones(c.f.shape[0]), (c.f, c.t)), shape=(c.n_bus, c.n_bus))
    assert connected_components(A, directed=False)[0] == 1


def test_feeder_replica_ybus_matches_branch_assembly():
    c = pfgen.replicate_feeder(4, SEED_F)
    Y = ybus.feeder_ybus(c)
    A = ybus.as_csr(c)
    assert abs(Y - A).max() <= 1e-12 * abs(A).max()


def test_feeder_replica_root_matches_ladder_sweep():
    c = pfgen.replicate_feeder(2, SEED_F)
    res = cim.newton(c)
    assert res.status == 0
    V_ladder = ladder_sweep(c)
    assert np.max(np.abs(res.V - V_ladder)) < 1e-9


@pytest.mark.parametrize("R", [2, 5])
def test_feeder_copies_repeat_the_one_copy_root(R):
    # the substation branch is divided by R, so R identical copies drawing R
    # times the current see the one-copy drop across it: every copy's
    # voltages are the one-copy root
    one = cim.newton(pfgen.replicate_feeder(1, SEED_F))
    c = pfgen.replicate_feeder(R, SEED_F)
    res = cim.newton(c)
    assert one.status == 0 and res.status == 0
    per = one.V.shape[0] - 6
    np.testing.assert_allclose(res.V[3:6], one.V[3:6], rtol=0, atol=1e-10)
    for r in range(R):
        np.testing.assert_allclose(res.V[6 + r * per:6 + (r + 1) * per], one.V[6:], rtol=0, atol=1e-10)
    # the lowest voltage stays in a plausible band
    assert 0.9 < np.abs(one.V).min() < 0.99


def test_feeder_rounding_floor_grows_with_copies():
    # the mismatch of the exact one-copy root repeated over R copies is pure
    # FP64 rounding; it grows with the first bus's row of Ybus, which is why
    # the 256-copy case stops at 1e-7 instead of 1e-8
    one = cim.newton(pfgen.replication_feeder(1), tol=1e-14)
    floors = []
    for R in (4, 64):
        c = pfgen.replication_feeder(R)
        V = np.concatenate([one.V[:6], np.tile(one.V[6:], R)])
        floors.append(float(np.max(np.abs(cim.mismatch(c, V)))))
    assert floors[0] < 1e-10 < floors[1] < 1e-8
    assert pfgen.replication_feeder_tol(128) == 1e-8 and pfgen.replication_feeder_tol(256) == 1e-7
