"""GPU solves of the replication-scale cases (Sec. IV) through the C ABI.

At a size the oracle solves in well under a second (100 copies of the 30-bus
block, 2 feeder copies) the GPU's roots are compared with the oracle's node by
node for LU, GMRES and BiCGStab.  At the paper's sizes: the 48,000-bus grid
against the oracle's root (one oracle solve, ~15 s), and the 230K-bus feeder
(256 copies) through a property that holds at any size: every copy's voltages
equal the oracle's root of the one-copy feeder, since the substation branch is
divided by the number of copies.  The oracle's FP64 mismatch at every GPU root
is at most the stop tolerance: 1e-8, except 1e-7 for the 256-copy feeder,
whose first bus has an FP64 rounding floor of 2.2e-8 at the exact root.
"""

import sys

import numpy as np
import pytest

import pfgen
from oracle import cim, polar

pytestmark = pytest.mark.gpu

TOL = 1e-8
VTOL = 1e-7
SOLVERS = [("lu", 0, 0), ("gmres", 1, 0), ("bicgstab", 2, 0), ("bicgstab-bjacobi", 2, 1)]


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


def _same_root(V, ref):
    assert np.max(np.abs(np.abs(V) - np.abs(ref))) <= VTOL
    assert np.max(np.abs(np.angle(V * np.conj(ref)))) <= VTOL


@pytest.mark.parametrize("solver", SOLVERS, ids=[s[0] for s in SOLVERS])
def test_polar_replica_3000_buses(B, ctx, solver):
    case = pfgen.replication_polar(100)
    _say(f"replica {case.name} solver={solver[0]}")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=solver[1], precond=solver[2], max_iter=40)
    V = B.pf_get_voltage(h)
    assert r.status == 0, r.as_dict()
    assert polar.mismatch_at(case, V) <= TOL
    _same_root(V, polar.newton(case).V)
    h.close()


@pytest.mark.parametrize("solver", SOLVERS, ids=[s[0] for s in SOLVERS])
def test_feeder_replica_two_copies(B, ctx, solver):
    case = pfgen.replication_feeder(2)
    _say(f"replica {case.name} solver={solver[0]}")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=solver[1], precond=solver[2], max_iter=40, nk_fallback=1)
    V = B.pf_get_voltage(h)
    _say(f"  status={r.status} iters={r.iters} linear={r.linear_iters} fallback={r.lu_fallback}")
    assert r.status == 0, r.as_dict()
    assert cim.mismatch_at(case, V) <= TOL
    _same_root(V, cim.newton(case).V)
    h.close()


@pytest.fixture(scope="module")
def grid48k():
    case = pfgen.replication_polar()
    ref = polar.newton(case)
    assert ref.status == 0
    return case, ref.V


@pytest.mark.parametrize("solver", SOLVERS, ids=[s[0] for s in SOLVERS])
def test_polar_replica_48000_buses(B, ctx, grid48k, solver):
    case, ref = grid48k
    _say(f"replica {case.name} solver={solver[0]}")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=solver[1], precond=solver[2], max_iter=40)
    V = B.pf_get_voltage(h)
    _say(f"  status={r.status} iters={r.iters} linear={r.linear_iters} mismatch={r.mismatch_inf:.2e}")
    assert r.status == 0, r.as_dict()
    assert polar.mismatch_at(case, V) <= TOL
    _same_root(V, ref)
    h.close()


@pytest.mark.parametrize("copies,solver", [(256, 0), (16, 2)], ids=["230k-lu", "14k-bicgstab"])
def test_feeder_copies_repeat_the_one_copy_root(B, ctx, copies, solver):
    one = cim.newton(pfgen.replication_feeder(1))
    assert one.status == 0
    case = pfgen.replication_feeder(copies)
    tol = pfgen.replication_feeder_tol(copies)
    _say(f"replica {case.name} ({case.n} phase-nodes) solver={solver} tol={tol}")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=solver, max_iter=40, nk_fallback=1, tol=tol)
    V = B.pf_get_voltage(h)
    _say(f"  status={r.status} iters={r.iters} linear={r.linear_iters} fallback={r.lu_fallback}")
    assert r.status == 0, r.as_dict()
    assert cim.mismatch_at(case, V) <= tol
    per = one.V.shape[0] - 6
    _same_root(V[:6], one.V[:6])
    _same_root(V[6:].reshape(copies, per), np.broadcast_to(one.V[6:], (copies, per)))
    h.close()
