"""GPU solves of three-phase feeders with voltage-controlled generation (PV
phase-nodes) and delta-connected ZIP loads, against the CPU oracle through
the C ABI.

The GPU takes a PV node's unknowns as (angle, generator Q) with |V| at its
set-point; the oracle appends a Q column and a |V| row per PV node.  The two
Newton iterations differ, their root does not: the GPU's voltages must be
within 1e-7 of the oracle's root, their PV magnitudes at the set-point, and
the oracle's FP64 mismatch at them (PV nodes at their balancing Q) at most
1e-8.  Batched solves equal solves alone bit for bit.
"""

import sys

import numpy as np
import pytest

import pfgen
from oracle import cim

pytestmark = pytest.mark.gpu

TOL = 1e-8
VTOL = 1e-7


@pytest.fixture(scope="module")
def B():
    from paper_1711_10579_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    c = B.pf_ctx_create(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    ("feeder60+dg", lambda: pfgen.add_dg_and_delta(pfgen.make_feeder(60, 2), 3)),
    ("feeder400+dg", lambda: pfgen.add_dg_and_delta(pfgen.make_feeder(400, 8), 9)),
    ("feeder2000+dg", lambda: pfgen.add_dg_and_delta(pfgen.config_case(2), 21, n_dg=6)),
    ("feeder400+pv-only", lambda: pfgen.add_dg_and_delta(pfgen.make_feeder(400, 8), 4, delta_frac=0.0)),
    ("feeder400+delta-only", lambda: pfgen.add_dg_and_delta(pfgen.make_feeder(400, 8), 5, n_dg=0,
                                                            single_phase_dg=False, delta_frac=0.6)),
    ("replica4+dg", lambda: pfgen.add_dg_and_delta(pfgen.replication_feeder(4), 6, n_dg=8)),
]
_ROOTS = {}


def _root(name, case):
    if name not in _ROOTS:
        ref = cim.newton(case)
        assert ref.status == 0
        _ROOTS[name] = ref.V
    return _ROOTS[name]


def _check(name, case, r, V):
    assert r.status == 0, (name, r.as_dict())
    assert r.mismatch_inf <= TOL
    assert cim.mismatch_at(case, V) <= TOL
    pv = cim.pv_nodes(case)
    if pv.size:
        assert np.max(np.abs(np.abs(V[pv]) - case.v_mag[pv])) <= 1e-12
    ref = _root(name, case)
    assert np.max(np.abs(np.abs(V) - np.abs(ref))) <= VTOL
    assert np.max(np.abs(np.angle(V * np.conj(ref)))) <= VTOL


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("solver", [0, 1, 2], ids=["lu", "gmres", "bicgstab"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_dg_feeder_parity(B, ctx, name, maker, solver, precision):
    case = maker()
    _say(f"dg {name} solver={solver} precision={precision}")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=solver, precision=precision, max_iter=40, gmres_max_restarts=40)
    V = B.pf_get_voltage(h)
    _say(f"  iters={r.iters} linear={r.linear_iters} mismatch={r.mismatch_inf:.2e}")
    _check(name, case, r, V)
    if solver == 0 and precision == 0:
        # Newton's quadratic convergence: no more steps than the oracle's
        # to its tighter tolerance
        assert r.iters <= cim.newton(case).iters
    h.close()


def test_dg_warm_start_keeps_the_root(B, ctx):
    # a second solve from the stored state (voltages and PV generator Q)
    # starts at the root: zero or one step, same voltages
    name, maker = CASES[1]
    case = maker()
    h = B.pf_create_from(ctx, case)
    r1 = B.pf_solve(h)
    V1 = B.pf_get_voltage(h)
    r2 = B.pf_solve(h, flat_start=0)
    V2 = B.pf_get_voltage(h)
    assert r1.status == 0 and r2.status == 0 and r2.iters <= 1
    assert np.max(np.abs(V2 - V1)) <= 1e-9
    _check(name, case, r2, V2)
    h.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_dg_batch_bit_identical_to_alone(B, ctx, precision):
    cases = [m() for _, m in CASES[:2]] + [pfgen.make_feeder(300, 12), pfgen.config_case(0)]
    opts = B.pf_default_options(precision=precision, max_iter=40)
    alone = []
    for c in cases:
        h = B.pf_create_from(ctx, c)
        B.pf_solve(h, opts)
        alone.append(B.pf_get_voltage(h))
        h.close()
    hs = [B.pf_create_from(ctx, c) for c in cases]
    rs = B.pf_solve_batch(ctx, hs, opts)
    for c, h, r, Va in zip(cases, hs, rs, alone):
        assert r.status == 0, (c.name, r.as_dict())
        assert np.array_equal(B.pf_get_voltage(h), Va), c.name
        h.close()


def _edge_case_feeder():
    # a feeder whose delta links include a load from a source node into an
    # unknown node, and two unknown nodes drawing loads into each other, with
    # a generator on a bus right behind the source
    fc = pfgen.make_feeder(40, 17, laterals=False)
    c = pfgen.add_dg_and_delta(fc, 2, n_dg=0, delta_frac=0.0, single_phase_dg=False)
    child = int(c.t[np.flatnonzero(c.f == 0)[0]])
    kids = np.flatnonzero(c.node_bus == child)
    src_a = 0
    assert kids.size == 3
    # source phase a -> child phase b (a coupled branch gives the entry)
    assert kids[1] in c.col[c.row_ptr[src_a]:c.row_ptr[src_a + 1]]
    c.delta_to[src_a] = kids[1]
    c.zip_delta[src_a] = [0.0, 0.0, 0.004, 0.0, 0.0, 0.002]
    # a two-node cycle on another bus
    other = np.flatnonzero(c.node_bus == 25)
    c.delta_to[other[0]] = other[2]
    c.delta_to[other[2]] = other[0]
    c.zip_delta[other[0]] = [0.003, 0.0, 0.002, 0.001, 0.0, 0.001]
    c.zip_delta[other[2]] = [0.0, 0.004, 0.0, 0.0, 0.002, 0.0]
    # generator on every phase of the source's child
    c.node_type[kids] = pfgen.PV
    c.v_mag[kids] = 1.005
    c.p_gen[kids] = 0.01
    return c


@pytest.mark.parametrize("solver", [0, 2], ids=["lu", "bicgstab"])
def test_dg_degenerate_links(B, ctx, solver):
    case = _edge_case_feeder()
    _say(f"dg edge cases solver={solver}")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=solver, max_iter=40)
    V = B.pf_get_voltage(h)
    _say(f"  iters={r.iters} linear={r.linear_iters} mismatch={r.mismatch_inf:.2e}")
    _check("edge", case, r, V)
    h.close()
