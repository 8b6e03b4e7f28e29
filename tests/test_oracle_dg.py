"""Pins of the oracle's voltage-controlled generation (PV phase-nodes) and
delta-connected loads in the three-phase current-injection model.

Independent references: the closed forms of a PV bus and of a PQ load behind
an impedance (applied to a generator on every phase of a bus, and to one
delta load between two phases fed over two wires), the single-phase polar
Newton with a PV bus on the positive-sequence equivalent of a balanced feeder,
the identity of a balanced delta load and the wye load of the same
coefficients, and finite differences of the augmented mismatch.
"""

import math

import numpy as np
import pytest

import pfgen
from pfgen.grids import CimCase, PQ, PV, SLACK, _stamp_csr
from oracle import cim, polar

import pins

NOMINAL = np.array([0.0, -2.0 * math.pi / 3.0, 2.0 * math.pi / 3.0])


def _two_bus_feeder(phases, z, zip_load=None, name="two-bus"):
    """Source bus (three phases) feeding one bus with the given phases over an
    uncoupled branch of impedance z per phase."""
    ph = list(phases)
    k = len(ph)
    n = 3 + k
    node_bus = np.array([0, 0, 0] + [1] * k, np.int32)
    node_phase = np.array([0, 1, 2] + ph, np.int32)
    ys = 1.0 / z
    rows, cols, vals = [], [], []
    for u, q in enumerate(ph):
        a, b = q, 3 + u
        rows += [a, b, a, b]
        cols += [a, b, b, a]
        vals += [ys, ys, -ys, -ys]
    # explicit zero couplings between the load bus's phases (delta loads
    # need those entries in the pattern)
    for u in range(k):
        for v in range(k):
            if u != v:
                rows.append(3 + u)
                cols.append(3 + v)
                vals.append(0.0)
    row_ptr, col, y = _stamp_csr(n, rows, cols, vals)
    zbr = np.zeros((1, 3, 3), np.complex128)
    zbr[0] = np.eye(3) * z
    bus_phases = np.zeros((2, 3), np.int8)
    bus_phases[0] = 1
    bus_phases[1, ph] = 1
    node_type = np.array([SLACK] * 3 + [PQ] * k, np.int8)
    zip_ = np.zeros((n, 6)) if zip_load is None else zip_load
    return CimCase(name=name, n_bus=2, n=n, node_bus=node_bus, node_phase=node_phase,
                   f=np.zeros(1, np.int32), t=np.ones(1, np.int32), zbr=zbr, bus_phases=bus_phases,
                   row_ptr=row_ptr, col=col, y=y, node_type=node_type, zip=zip_,
                   p_gen=np.zeros(n), q_gen=np.zeros(n), v_mag=np.ones(n), v_ang=NOMINAL[node_phase])


@pytest.mark.parametrize("P,Q", [(0.3, 0.1), (0.8, 0.4), (0.05, -0.02)])
def test_delta_load_between_two_wires_closed_form(P, Q):
    # a constant-power delta load S between phases a and b of a bus fed over
    # two wires of impedance z: the loop is one source E_ab = sqrt3 at +30
    # degrees, a series impedance 2z and the load S
    z = 0.02 + 0.06j
    c = _two_bus_feeder([0, 1], z)
    c.delta_to = np.array([-1, -1, -1, 4, -1], np.int32)
    c.zip_delta = np.zeros((5, 6))
    c.zip_delta[3, 2] = P
    c.zip_delta[3, 5] = Q
    res = cim.newton(c)
    assert res.status == 0
    vm, va = pins.two_bus_pq(2 * z.real, 2 * z.imag, P, Q, U1=math.sqrt(3.0))
    Vab = res.V[3] - res.V[4]
    assert abs(abs(Vab) - vm) < 1e-10
    assert abs(np.angle(Vab) - (math.pi / 6 + va)) < 1e-10
    # the loop current leaves a and returns on b: the common mode is the
    # source's
    Ea, Eb = np.exp(1j * NOMINAL[:2])
    assert abs(res.V[3] + res.V[4] - (Ea + Eb)) < 1e-10


@pytest.mark.parametrize("P,U", [(0.3, 1.0), (0.6, 1.03), (-0.2, 0.99)])
def test_pv_generator_on_every_phase_closed_form(P, U):
    # a PV generator on each phase behind an uncoupled impedance: each phase
    # is the two-bus PV problem, at its own nominal angle
    z = 0.03 + 0.09j
    c = _two_bus_feeder([0, 1, 2], z)
    c.node_type[3:] = PV
    c.v_mag[3:] = U
    c.p_gen[3:] = P
    res = cim.newton(c)
    assert res.status == 0
    d = pins.two_bus_pv(z.real, z.imag, P, U)
    for ph in range(3):
        assert abs(abs(res.V[3 + ph]) - U) < 1e-12
        ang = np.angle(res.V[3 + ph] * np.exp(-1j * NOMINAL[ph]))
        assert abs(ang - d) < 1e-10
    # its Q: the power the generator must send over z to hold U
    I = (res.V[3:] - np.exp(1j * NOMINAL)) / z
    np.testing.assert_allclose(res.q_gen[3:], (res.V[3:] * np.conj(I)).imag, rtol=0, atol=1e-10)


def _balanced_feeder(nb, seed, mode):
    fc = pfgen.make_feeder(nb, seed, laterals=False, balanced=True, zip_mode="P")
    if mode == "zip":
        p = fc.zip[:, 2].copy()
        q = fc.zip[:, 5].copy()
        fc.zip[:, :3] = (p / 3.0)[:, None]
        fc.zip[:, 3:] = (q / 3.0)[:, None]
    return fc


@pytest.mark.parametrize("mode", ["P", "zip"])
def test_balanced_delta_loads_equal_wye_loads(mode):
    # on a balanced feeder the delta load of coefficients s between every
    # pair of phases draws, at each phase, the current of the wye load s
    fc = _balanced_feeder(40, 3, mode)
    dl = pfgen.add_dg_and_delta(fc, 5, n_dg=0, delta_frac=1.0, single_phase_dg=False)
    assert (dl.delta_to[3:] >= 0).all() and not dl.zip[3:].any()
    a = cim.newton(fc)
    b = cim.newton(dl)
    assert a.status == 0 and b.status == 0
    assert np.max(np.abs(a.V - b.V)) < 1e-10


def test_balanced_feeder_with_generator_equals_polar_pv_bus():
    # a three-phase generator on a balanced feeder is, per phase, a PV bus of
    # the positive-sequence equivalent (single-phase Newton, pinned on its
    # own)
    fc = _balanced_feeder(30, 11, "P")
    b = 17
    nodes = np.flatnonzero(fc.node_bus == b)
    c = pfgen.add_dg_and_delta(fc, 1, n_dg=0, delta_frac=0.0, single_phase_dg=False)
    c.node_type[nodes] = PV
    c.v_mag[nodes] = 1.01
    c.p_gen[nodes] = 0.25
    res = cim.newton(c)
    assert res.status == 0
    pc = pins.polar_equivalent_of_balanced_feeder(fc)
    pc.bus_type[b] = PV
    pc.v_mag[b] = 1.01
    pc.p_sp[b] += 0.25
    ref = polar.newton(pc)
    assert ref.status == 0
    node_a = np.flatnonzero(c.node_phase == 0)
    np.testing.assert_allclose(np.abs(res.V[node_a]), ref.vm, rtol=0, atol=1e-10)
    np.testing.assert_allclose(np.angle(res.V[node_a]), ref.va, rtol=0, atol=1e-10)
    # Q per phase: the polar bus's Q plus the phase's load Q
    P, Q = polar.injections(pc, ref.vm, ref.va)
    assert abs(res.q_gen[nodes[0]] - (Q[b] + fc.zip[nodes[0], 5])) < 1e-9


def _fd(fun, x0, h):
    f0 = fun(x0)
    J = np.zeros((f0.shape[0], x0.shape[0]))
    for j in range(x0.shape[0]):
        e = np.zeros_like(x0)
        e[j] = h
        J[:, j] = (fun(x0 + e) - fun(x0 - e)) / (2 * h)
    return J


def test_augmented_jacobian_matches_finite_differences():
    fc = pfgen.make_feeder(25, 4)
    c = pfgen.add_dg_and_delta(fc, 9, n_dg=2, delta_frac=0.5)
    pv = cim.pv_nodes(c)
    assert pv.size >= 6 and (c.delta_to >= 0).sum() >= 4
    unknown, _, _, col_re, col_im, dim = cim.unknown_layout(c)
    u = np.flatnonzero(unknown)
    rng = np.random.default_rng(3)
    V0 = cim.flat_start(c) * (1 + 0.03 * rng.standard_normal(c.n)) * np.exp(0.03j * rng.standard_normal(c.n))
    q0 = rng.uniform(-0.1, 0.1, c.n)

    def F(x):
        V = V0.copy()
        V[u] = x[col_re[u]] + 1j * x[col_im[u]]
        q = q0.copy()
        q[pv] = x[dim:]
        return cim.mismatch(c, V, q)

    x0 = np.zeros(dim + pv.size)
    x0[col_re[u]] = V0[u].real
    x0[col_im[u]] = V0[u].imag
    x0[dim:] = q0[pv]
    J = cim.jacobian(c, V0, q0).toarray()
    Jfd = -_fd(F, x0, 1e-7)
    assert np.max(np.abs(J - Jfd)) <= 1e-7 * np.max(np.abs(J))
    # the delta blocks and the PV rows and columns are exercised
    assert np.abs(J[dim:, :]).max() > 0.5 and np.abs(J[:, dim:]).max() > 0.5


def test_pv_mismatch_at_the_root_and_balancing_q():
    c = pfgen.add_dg_and_delta(pfgen.make_feeder(400, 8), 9)
    res = cim.newton(c)
    assert res.status == 0
    # mismatch_at solves each PV node's Q from V alone: the Newton Q
    np.testing.assert_allclose(cim.pv_reactive(c, res.V)[cim.pv_nodes(c)], res.q_gen[cim.pv_nodes(c)],
                               rtol=0, atol=1e-9)
    assert cim.mismatch_at(c, res.V) < 1e-10
    # and a voltage off the root shows a mismatch
    V = res.V.copy()
    V[cim.pv_nodes(c)[0]] *= np.exp(1e-4j)
    assert cim.mismatch_at(c, V) > 1e-6
