"""GPU test of pf_solve_noalloc, the LU solve for callers that cannot
allocate, through the C ABI: on two calls in a row (the second a smaller case)
its results equal pf_solve's bit for bit (status, iterations, final mismatch,
voltages), the cases' own storage is left as it was, and a case too large for
the fixed array is rejected with a clear error."""

import sys

import numpy as np
import pytest

import pfgen
from oracle import polar

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1711_10579_amd import binding

    return binding


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_noalloc_matches_pf_solve(B, precision):
    ctx = B.pf_ctx_create(0)
    opts = dict(precision=precision, max_iter=40 if precision else 20)
    big = pfgen.config_case(1)
    small = pfgen.perturb_loads(pfgen.make_polar_grid(2500, 750, 250, 5, balanced=True), 3)
    feeder = pfgen.make_feeder(300, 4)
    # reference: pf_solve on handles of their own
    ref = {}
    for name, c in (("big", big), ("small", small), ("feeder", feeder)):
        h = B.pf_create_from(ctx, c)
        r = B.pf_solve(h, **opts)
        ref[name] = (r.status, r.iters, r.mismatch_inf, B.pf_get_voltage(h))
        h.close()
    # two calls in a row, the second with a smaller input, then a feeder on a
    # case that already holds its own working storage
    for name, c in (("big", big), ("small", small)):
        h = B.pf_create_from(ctx, c)
        _say(f"noalloc {name} precision={precision}")
        r, used = B.pf_solve_noalloc(h, **opts)
        assert (r.status, r.iters, r.mismatch_inf) == ref[name][:3], name
        assert np.array_equal(B.pf_get_voltage(h), ref[name][3]), name
        assert r.status == B.PF_CONVERGED
        info = B.pf_case_info_get(h)
        assert info["work_bytes"] < used <= 64 << 20
        # no working storage was allocated for the case
        assert info["device_bytes"] == info["resident_bytes"]
        h.close()
    h = B.pf_create_from(ctx, feeder)
    B.pf_solve(h, **opts)
    before = B.pf_case_info_get(h)["device_bytes"]
    r, _ = B.pf_solve_noalloc(h, **opts)
    assert (r.status, r.iters, r.mismatch_inf) == ref["feeder"][:3]
    assert np.array_equal(B.pf_get_voltage(h), ref["feeder"][3])
    assert B.pf_case_info_get(h)["device_bytes"] == before
    # ... and its own storage still serves pf_solve
    r2 = B.pf_solve(h, **opts)
    assert (r2.status, r2.iters, r2.mismatch_inf) == ref["feeder"][:3]
    h.close()
    # against the oracle once (the reference solve is pf_solve's own parity)
    assert polar.mismatch_at(small, ref["small"][3]) <= 1e-8
    ctx.close()


def test_noalloc_rejects_too_large_and_krylov(B):
    ctx = B.pf_ctx_create(0)
    big = pfgen.make_polar_grid(20000, 6000, 2000, 77, balanced=True)
    h = B.pf_create_from(ctx, big)
    with pytest.raises(B.PFError) as ei:
        B.pf_solve_noalloc(h)
    assert ei.value.code == B.PF_E_INVALID and "bytes of scratch" in str(ei.value)
    with pytest.raises(B.PFError) as ei:
        B.pf_solve_noalloc(h, solver=B.PF_SOLVER_GMRES)
    assert ei.value.code == B.PF_E_INVALID
    h.close()
    ctx.close()
