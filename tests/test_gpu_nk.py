"""GPU parity of the Newton-Krylov iteration (Sec. III-B: GMRES inner solve with
ILU(0) or block-Jacobi preconditioning, forcing term eta_k) against the CPU
oracle, through the C ABI.

The root does not depend on the inner solver: the GPU's voltages must be
within 1e-7 pu / rad of the oracle's Newton root and the oracle's FP64
mismatch at them at most 1e-8.  Batched Krylov solves must equal the solves
of each instance alone bit for bit.
"""

import sys

import numpy as np
import pytest

import pfgen
from oracle import cim, polar

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


def _check(case, r, V):
    assert r.status == 0, (case.name, r.as_dict())
    assert r.mismatch_inf <= TOL
    assert r.linear_iters > 0
    if hasattr(case, "bus_type"):
        assert polar.mismatch_at(case, V) <= TOL
        ref = polar.newton(case)
        assert np.max(np.abs(np.abs(V) - ref.vm)) <= VTOL
        assert np.max(np.abs(np.angle(V) - ref.va)) <= VTOL
    else:
        assert cim.mismatch_at(case, V) <= TOL
        ref = cim.newton(case)
        assert np.max(np.abs(np.abs(V) - ref.vm)) <= VTOL
        assert np.max(np.abs(np.angle(V * np.conj(ref.V)))) <= VTOL


CASES = [
    ("grid2", lambda: pfgen.make_polar_grid(2, 0, 0, 1)),
    ("grid3pv", lambda: pfgen.make_polar_grid(3, 1, 1, 1003, balanced=False)),
    ("grid30", lambda: pfgen.config_case(0)),
    ("grid257", lambda: pfgen.make_polar_grid(257, 77, 25, 1257, balanced=True)),
    ("grid1000", lambda: pfgen.make_polar_grid(1000, 300, 100, 2000, balanced=True)),
    ("grid3001", lambda: pfgen.make_polar_grid(3001, 900, 300, 4001, balanced=True)),
    ("feeder2", lambda: pfgen.make_feeder(2, 5)),
    ("feeder60", lambda: pfgen.make_feeder(60, 2)),
    ("feeder400", lambda: pfgen.make_feeder(400, 8)),
]


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precond", [0, 1], ids=["ilu0", "bjacobi"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_nk_parity(B, ctx, name, maker, precond, precision):
    case = maker()
    _say(f"nk {name} precond={precond} precision={precision}")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=B.PF_SOLVER_GMRES, precond=precond, precision=precision,
                   max_iter=40, gmres_max_restarts=40)
    V = B.pf_get_voltage(h)
    _check(case, r, V)
    h.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_nk_10k_bus_grid(B, ctx, precision):
    case = pfgen.config_case(1)
    _say(f"nk 10k precision={precision}")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=B.PF_SOLVER_GMRES, precision=precision, max_iter=40)
    V = B.pf_get_voltage(h)
    _say(f"  iters={r.iters} linear={r.linear_iters} mismatch={r.mismatch_inf:.2e}")
    _check(case, r, V)
    # the same root as the direct inner solve
    r2 = B.pf_solve(h)
    V2 = B.pf_get_voltage(h)
    assert r2.status == 0
    assert np.max(np.abs(V - V2)) <= VTOL
    h.close()


def test_nk_feeder_2000_buses(B, ctx):
    case = pfgen.config_case(2)
    _say("nk feeder 2000")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=B.PF_SOLVER_GMRES)
    _check(case, r, B.pf_get_voltage(h))
    h.close()


@pytest.mark.parametrize("precond", [0, 1], ids=["ilu0", "bjacobi"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_nk_batch_bit_identical_to_alone(B, ctx, precond, precision):
    rng = np.random.default_rng(8)
    cases = [pfgen.config_case(0), pfgen.make_feeder(120, 7)]
    for i in range(6):
        n = int(np.exp(rng.uniform(np.log(100), np.log(2500))))
        base = pfgen.make_polar_grid(n, int(0.3 * n), max(1, n // 10), 700 + i, balanced=True)
        cases.append(pfgen.perturb_loads(base, 70 + i))
    _say(f"nk batch precond={precond} precision={precision}")
    hs = [B.pf_create_from(ctx, c) for c in cases]
    opts = dict(solver=B.PF_SOLVER_GMRES, precond=precond, precision=precision, max_iter=40,
                gmres_max_restarts=40)
    alone = []
    for h in hs:
        r = B.pf_solve(h, **opts)
        alone.append((r, B.pf_get_voltage(h)))
    res = B.pf_solve_batch(ctx, hs, **opts)
    for c, h, (ra, va), rb in zip(cases, hs, alone, res):
        vb = B.pf_get_voltage(h)
        assert rb.status == ra.status and rb.iters == ra.iters, c.name
        assert rb.linear_iters == ra.linear_iters, c.name
        assert np.array_equal(va, vb), c.name
        _check(c, rb, vb)
    for h in hs:
        h.close()


def test_nk_restart_length_and_restarts(B, ctx):
    # a short restart length forces several cycles per Newton step; the root
    # is unchanged
    case = pfgen.make_polar_grid(1000, 300, 100, 2000, balanced=True)
    _say("nk short restarts")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=B.PF_SOLVER_GMRES, gmres_m=4, gmres_max_restarts=200, max_iter=40)
    _check(case, r, B.pf_get_voltage(h))
    r64 = B.pf_solve(h, solver=B.PF_SOLVER_GMRES, gmres_m=64, max_iter=40)
    _check(case, r64, B.pf_get_voltage(h))
    h.close()


def test_nk_linear_fail_status(B, ctx):
    # two block-Jacobi steps and no restart cannot reach a forcing term of
    # 1e-3 on the first step: the iteration ends with a linear failure
    case = pfgen.make_polar_grid(1000, 300, 100, 2000, balanced=True)
    _say("nk linear failure")
    h = B.pf_create_from(ctx, case)
    r = B.pf_solve(h, solver=B.PF_SOLVER_GMRES, precond=1, gmres_m=2, gmres_max_restarts=0, eta_max=1e-3)
    assert r.status == B.PF_LINEAR_FAIL, r.as_dict()
    assert r.iters == 0
    h.close()


@pytest.mark.parametrize("precond", [0, 1], ids=["ilu0", "bjacobi"])
def test_nk_singular_islanded_bus(B, ctx, precond):
    import pins

    island = pins.polar_case(3, [0], [1], [0.02], [0.1], [0.0], [3, 1, 1],
                             [0, -0.3, -0.1], [0, -0.1, -0.05], [1, 1, 1])
    island.row_ptr = np.array([0, 2, 4, 5], np.int32)
    island.col = np.array([0, 1, 0, 1, 2], np.int32)
    island.y = np.concatenate([island.y, [0j]])
    h = B.pf_create_from(ctx, island)
    r = B.pf_solve(h, solver=B.PF_SOLVER_GMRES, precond=precond)
    assert r.status == B.PF_SINGULAR, r.as_dict()
    h.close()


def test_nk_served_matches_alone(B, ctx):
    # Krylov requests through the serving loop give the results of solving
    # each case alone
    import time

    cases = [pfgen.make_polar_grid(n, int(0.3 * n), n // 10, 3000 + n, balanced=True) for n in (150, 600, 1400)]
    cases.append(pfgen.make_feeder(200, 9))
    hs = [B.pf_create_from(ctx, c) for c in cases]
    opts = B.pf_default_options(solver=B.PF_SOLVER_GMRES, precision=1, max_iter=40)
    alone = []
    for h in hs:
        r = B.pf_solve(h, opts)
        alone.append((r, B.pf_get_voltage(h)))
    _say("nk serving")
    tickets = [B.pf_submit(ctx, h, opts) for h in hs]
    got = {}
    t0 = time.perf_counter()
    while len(got) < len(hs):
        for i, t in enumerate(tickets):
            if i not in got:
                d, r = B.pf_poll(ctx, t)
                if d:
                    got[i] = r
        assert time.perf_counter() - t0 < 120
        time.sleep(0.001)
    for i, h in enumerate(hs):
        assert got[i].status == alone[i][0].status and got[i].iters == alone[i][0].iters
        assert np.array_equal(B.pf_get_voltage(h), alone[i][1])
    for h in hs:
        h.close()


def test_nk_option_validation(B, ctx):
    h = B.pf_create_from(ctx, pfgen.config_case(0))
    for bad in [dict(gmres_m=0), dict(gmres_m=129), dict(eta_max=0.0), dict(eta_max=1.0),
                dict(precond=7), dict(gmres_max_restarts=-1)]:
        with pytest.raises(B.PFError):
            B.pf_solve(h, solver=B.PF_SOLVER_GMRES, **bad)
    h.close()
