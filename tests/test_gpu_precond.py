"""GPU check of the Newton-Krylov preconditioner set-up kernels (Sec. III-B)
against their definitions, on the device's own Jacobian at the flat start:

- block-Jacobi: every node group's stored inverse X of its diagonal block
  A_bb satisfies A_bb X = I (groups of 1 to 32 nodes, orders 2 to 64);
- ILU(0): the stored factor reproduces A on its pattern, (L U)_ij = A_ij, and
  the stored inverted diagonal blocks invert U's diagonal.

The check is repeated to catch results that change from run to run (a race
in a set-up kernel would show as a large deviation in some run).
"""

import sys

import pytest

import pfgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1711_10579_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    c = B.pf_ctx_create(0)
    yield c
    c.close()


CASES = [
    ("grid30", lambda: pfgen.config_case(0)),
    ("grid1000", lambda: pfgen.make_polar_grid(1000, 300, 100, 4, balanced=True)),
    ("tree500", lambda: pfgen.make_polar_grid(500, 0, 50, 7)),
    ("feeder400", lambda: pfgen.make_feeder(400, 8)),
    ("feeder_dg_delta", lambda: pfgen.add_dg_and_delta(pfgen.make_feeder(300, 9), 5)),
    ("grid10k", lambda: pfgen.config_case(1)),
    ("grid48k", lambda: pfgen.replication_polar()),
]


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
def test_precond_setup_matches_definition(B, ctx, name, maker):
    case = maker()
    h = B.pf_create_from(ctx, case)
    for rep in range(3):
        dev_bj, order = B.pf_debug_precond_check(h, B.PF_PRECOND_BJACOBI)
        dev_ilu, _ = B.pf_debug_precond_check(h, B.PF_PRECOND_ILU0)
        print(f"{name} rep {rep}: block-Jacobi |A X - I| {dev_bj:.2e} (largest order {order}), "
              f"ILU(0) |LU - A| / |A| {dev_ilu:.2e}", flush=True)
        sys.stdout.flush()
        assert 2 <= order <= 64
        assert dev_bj <= 1e-9, (name, rep, dev_bj)
        assert dev_ilu <= 1e-12, (name, rep, dev_ilu)
    h.close()
