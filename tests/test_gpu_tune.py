"""GPU tests of case schedules and the autotuner: every schedule gives the
oracle's root (the schedule reorders the work, not what is computed), the
autotuner returns a converging schedule no slower than the default, and
later cases of the same topology are created with it."""

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
    if hasattr(case, "bus_type"):
        assert polar.mismatch_at(case, V) <= TOL
        ref = polar.newton(case)
        assert np.max(np.abs(np.abs(V) - ref.vm)) <= VTOL
        assert np.max(np.abs(np.angle(V) - ref.va)) <= VTOL
    else:
        assert cim.mismatch_at(case, V) <= TOL
        ref = cim.newton(case)
        assert np.max(np.abs(V - ref.V)) <= VTOL


SCHEDULES = [(0.3, 32, 1, 0), (0.8, 32, 2, 1), (1.0, 1, 4, 2), (0.5, 10 ** 6, 1, 0), (0.4, 8, 2, 2)]


@pytest.mark.parametrize("sched", SCHEDULES, ids=[f"s{i}" for i in range(len(SCHEDULES))])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_scheduled_cases_reach_the_oracle_root(B, ctx, sched, precision):
    ds, md, ls, tm = sched
    sc = B.pf_default_schedule(dense_switch=ds, min_dense=md, lane_scale=ls, trsv_mode=tm)
    for case in [pfgen.make_polar_grid(1000, 300, 100, 2000, balanced=True), pfgen.make_feeder(400, 8),
                 pfgen.config_case(0)]:
        _say(f"schedule {sched} {case.name} precision={precision}")
        h = B.pf_create_from(ctx, case, schedule=sc)
        assert B.pf_case_schedule(h).as_dict() == sc.as_dict()
        r = B.pf_solve(h, precision=precision, max_iter=40 if precision else 20)
        _check(case, r, B.pf_get_voltage(h))
        h.close()


def test_scheduled_10k_bus_grid(B, ctx):
    case = pfgen.config_case(1)
    for ds in (0.3, 0.8):
        sc = B.pf_default_schedule(dense_switch=ds)
        _say(f"10k dense_switch={ds}")
        h = B.pf_create_from(ctx, case, schedule=sc)
        info = B.pf_case_info_get(h)
        r = B.pf_solve(h)
        _say(f"  n_dense={info['n_dense']} ms={r.device_ms:.2f}")
        _check(case, r, B.pf_get_voltage(h))
        h.close()


def test_forced_flag_mode_on_a_large_batch(B, ctx):
    # flag-synchronised dense backward solves over more work-groups than the
    # automatic rule allows: every wait is on an earlier work-group
    sc = B.pf_default_schedule(trsv_mode=1)
    cases = [pfgen.perturb_loads(pfgen.make_polar_grid(1500, 450, 150, 60 + i, balanced=True), i)
             for i in range(24)]
    _say("forced flag mode, 24 x 1500")
    hs = [B.pf_create_from(ctx, c, schedule=sc) for c in cases]
    res = B.pf_solve_batch(ctx, hs)
    for c, h, r in zip(cases[:3], hs[:3], res[:3]):
        _check(c, r, B.pf_get_voltage(h))
    assert all(r.status == 0 for r in res)
    for h in hs:
        h.close()


def test_autotune_chooses_and_remembers_a_schedule(B, ctx):
    case = pfgen.make_polar_grid(2000, 600, 200, 77, balanced=True)
    _say("autotune 2000-bus grid")
    best, rep = B.pf_autotune(ctx, case, trials=2)
    _say(f"  best={best.as_dict()} report={rep}")
    # the default, eight dense_switch values, two lane_scale and two trsv_mode values
    assert rep["candidates"] == 13 and rep["trials"] == 2
    assert 0 < rep["best_ms"] <= rep["default_ms"]
    h = B.pf_create_from(ctx, case)
    assert B.pf_case_schedule(h).as_dict() == best.as_dict()
    r = B.pf_solve(h)
    _check(case, r, B.pf_get_voltage(h))
    h.close()
    # another topology keeps the default
    other = pfgen.make_polar_grid(2000, 600, 200, 78, balanced=True)
    h2 = B.pf_create_from(ctx, other)
    assert B.pf_case_schedule(h2).as_dict() == B.pf_default_schedule().as_dict()
    h2.close()


def test_autotune_rejects_bad_input(B, ctx):
    case = pfgen.config_case(0)
    with pytest.raises(B.PFError):
        B.pf_autotune(ctx, case, trials=1, tol=-1.0)
