"""CPU tests of the native library: exported symbols, input validation and
the host symbolic analysis (replayed on the CPU through pf_debug_schedule_check)."""

import os
import re

import numpy as np
import pytest

import pfgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

B = pytest.importorskip("paper_1711_10579_amd.binding",
                        reason="build the library first (python -m paper_1711_10579_amd.build)")


def _declared_functions():
    names = []
    for h in ["pf.h", "pf_debug.h"]:
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(pf_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import ctypes

    lib = ctypes.CDLL(B.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(B.EXPORTED) | {"pf_default_options"}


def test_version_and_error_string():
    assert B.pf_version().startswith("exagridpf")
    assert isinstance(B.pf_last_error(), str)


CASES = [
    ("grid30", lambda: pfgen.config_case(0)),
    ("grid2", lambda: pfgen.make_polar_grid(2, 0, 0, 1)),
    ("grid3pv", lambda: pfgen.make_polar_grid(3, 1, 2, 2)),
    ("grid257", lambda: pfgen.make_polar_grid(257, 77, 25, 3, balanced=True)),
    ("grid1000", lambda: pfgen.make_polar_grid(1000, 300, 100, 4, balanced=True)),
    ("grid10k", lambda: pfgen.config_case(1)),
    ("feeder2", lambda: pfgen.make_feeder(2, 5)),
    ("feeder30", lambda: pfgen.make_feeder(30, 6)),
    ("feeder2k", lambda: pfgen.config_case(2)),
    ("tree_only", lambda: pfgen.make_polar_grid(500, 0, 50, 7)),
    ("dense_small", lambda: pfgen.make_polar_grid(80, 800, 8, 8)),
]


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
def test_schedule_replay(name, maker):
    c = maker()
    res, checks = B.pf_debug_schedule_check(**B.case_arrays(c), seed=11)
    assert checks > 0
    assert res < 1e-13


@pytest.mark.parametrize("ds,md", [(0.3, 32), (0.8, 32), (1.0, 1), (0.5, 1000000)],
                         ids=["switch0.3", "switch0.8", "switch1", "no_dense"])
@pytest.mark.parametrize("name", ["grid257", "grid1000", "grid10k", "feeder2k", "dense_small"])
def test_schedule_replay_under_other_schedules(name, ds, md):
    # every schedule the autotuner may choose gives a valid analysis
    c = dict(CASES)[name]()
    sc = B.pf_default_schedule(dense_switch=ds, min_dense=md)
    res, checks = B.pf_debug_schedule_check(**B.case_arrays(c), seed=3, schedule=sc)
    assert checks > 0
    assert res < 1e-12


@pytest.mark.parametrize("bad", [dict(dense_switch=0.0), dict(dense_switch=1.5), dict(min_dense=0),
                                 dict(lane_scale=3), dict(trsv_mode=3)])
def test_schedule_validation(bad):
    sc = B.pf_default_schedule(**bad)
    with pytest.raises(B.PFError) as ei:
        B.pf_debug_schedule_check(**B.case_arrays(pfgen.config_case(0)), schedule=sc)
    assert ei.value.code == B.PF_E_INVALID


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
def test_krylov_analysis_replay(name, maker):
    # every index of the Newton-Krylov analysis, and block ILU(0) through its
    # update lists and level schedules reproduces A on the pattern
    c = maker()
    dev, res, checks = B.pf_debug_krylov_check(**B.case_arrays(c), seed=5)
    assert checks > 0
    assert dev < 1e-13
    assert res < 1e-12


def test_dense_block_appears_on_meshed_grids():
    # the 10k-bus meshed grid leaves a dense trailing block; a radial feeder not
    c1 = pfgen.config_case(1)
    res, _ = B.pf_debug_schedule_check(**B.case_arrays(c1), seed=1)
    assert res < 1e-13


def _bad(**over):
    c = pfgen.config_case(0)
    kw = B.case_arrays(c)
    kw.update(over)
    return kw


@pytest.mark.parametrize("what,kw", [
    ("two slacks", lambda c: dict(bus_type=np.where(np.arange(c.n) < 2, 3, c.bus_type))),
    ("no slack", lambda c: dict(bus_type=np.where(c.bus_type == 3, 1, c.bus_type))),
    ("nan setpoint", lambda c: dict(p_sp=np.where(np.arange(c.n) == 4, np.nan, c.p_sp))),
    ("bad type", lambda c: dict(bus_type=np.where(np.arange(c.n) == 5, 7, c.bus_type))),
    ("unsorted", lambda c: dict(col_idx=_swap_first_row(c))),
    ("missing diagonal", lambda c: _drop_diagonal(c)),
    ("asymmetric", lambda c: _asymmetric(c)),
])
def test_invalid_inputs_rejected(what, kw):
    c = pfgen.config_case(0)
    args = B.case_arrays(c)
    args.update(kw(c))
    with pytest.raises(B.PFError) as ei:
        B.pf_debug_schedule_check(**args)
    assert ei.value.code == B.PF_E_INVALID


def _swap_first_row(c):
    col = c.col.copy()
    a, b = c.row_ptr[0], c.row_ptr[1]
    col[a], col[a + 1] = col[a + 1], col[a]
    return col


def _drop_diagonal(c):
    import scipy.sparse as sp

    Y = sp.csr_matrix((c.y, c.col, c.row_ptr), shape=(c.n, c.n)).tolil()
    Y[7, 7] = 0
    Y = sp.csr_matrix(Y)
    Y.eliminate_zeros()
    Y.sort_indices()
    return dict(row_ptr=Y.indptr, col_idx=Y.indices, y=Y.data)


def _asymmetric(c):
    import scipy.sparse as sp

    Y = sp.csr_matrix((c.y, c.col, c.row_ptr), shape=(c.n, c.n)).tolil()
    i, j = 3, 20
    assert Y[i, j] == 0
    Y[i, j] = 1.0 + 1.0j
    Y = sp.csr_matrix(Y)
    Y.sort_indices()
    return dict(row_ptr=Y.indptr, col_idx=Y.indices, y=Y.data)


def _dg_feeder():
    return pfgen.add_dg_and_delta(pfgen.make_feeder(60, 2), 3)


def test_dg_feeder_analysis_replay():
    c = _dg_feeder()
    assert (c.node_type == 2).sum() > 0 and (c.delta_to >= 0).sum() > 0
    res, chk = B.pf_debug_schedule_check(**B.case_arrays(c), seed=2)
    assert res < 1e-12 and chk > 0
    dev, kres, _ = B.pf_debug_krylov_check(**B.case_arrays(c), seed=2)
    assert dev < 1e-12 and kres < 1e-12


def _with(c, **over):
    args = B.case_arrays(c)
    args.update(over)
    return args


def _two_into_one(c):
    dt = c.delta_to.copy()
    k = int(np.flatnonzero(dt >= 0)[0])
    other = int(np.flatnonzero((dt < 0) & (np.arange(c.n) != dt[k]) & (np.arange(c.n) != k))[-1])
    # a second load into the same node needs the pattern entry: pick a
    # neighbour of that node
    t = int(dt[k])
    nb = [int(j) for j in c.col[c.row_ptr[t]:c.row_ptr[t + 1]] if j != t and dt[j] < 0 and j != k]
    dt[nb[0] if nb else other] = t
    return dt


@pytest.mark.parametrize("what,over", [
    ("delta_to without zip_delta", lambda c: dict(zip_delta=None)),
    ("zip_delta without delta_to", lambda c: dict(delta_to=None)),
    ("target out of range", lambda c: dict(delta_to=np.where(c.delta_to >= 0, c.n, -1))),
    ("target is the node", lambda c: dict(delta_to=np.where(c.delta_to >= 0, np.arange(c.n), -1))),
    ("node receives two", lambda c: dict(delta_to=_two_into_one(c))),
    ("no pattern entry", lambda c: dict(delta_to=np.where(np.arange(c.n) == 5, c.n - 1, c.delta_to))),
    ("pv magnitude zero", lambda c: dict(v_mag=np.where(c.node_type == 2, 0.0, c.v_mag))),
    ("nan delta coefficient", lambda c: dict(zip_delta=np.where(np.arange(6 * c.n).reshape(c.n, 6) == 30,
                                                                 np.nan, c.zip_delta))),
])
def test_dg_and_delta_inputs_rejected(what, over):
    c = _dg_feeder()
    with pytest.raises(B.PFError) as ei:
        B.pf_debug_schedule_check(**_with(c, **over(c)))
    assert ei.value.code == B.PF_E_INVALID, what


def test_polar_rejects_delta_loads():
    c = pfgen.config_case(0)
    args = B.case_arrays(c)
    args.update(delta_to=-np.ones(c.n, np.int32), zip_delta=np.zeros((c.n, 6)))
    with pytest.raises(B.PFError) as ei:
        B.pf_debug_schedule_check(**args)
    assert ei.value.code == B.PF_E_INVALID


def test_footprint_and_debug_calls_reject_null():
    import ctypes

    b = ctypes.c_size_t()
    assert B._lib.pf_case_footprint(None, ctypes.byref(b)) == B.PF_E_INVALID
    d = ctypes.c_double()
    o = ctypes.c_int32()
    assert B._lib.pf_debug_precond_check(None, 0, ctypes.byref(d), ctypes.byref(o)) == B.PF_E_INVALID
    s1, s2 = ctypes.c_size_t(), ctypes.c_size_t()
    q, r = ctypes.c_int32(), ctypes.c_int32()
    assert B._lib.pf_serve_stats(None, ctypes.byref(s1), ctypes.byref(s2), ctypes.byref(q),
                                 ctypes.byref(r)) == B.PF_E_INVALID
