"""ctypes binding of the C ABI declared in ``include/pf.h``.

Argument marshalling only: every step of the power-flow iteration runs in the
HIP library.  Importing this module loads ``_lib/libexagridpf.so`` and raises
if it is missing; there is no fallback.  PyTorch, when used, provides the
device allocator and the stream (``pf_ctx_create(use_torch=True)``).
"""

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PF_LIB selects another build of the same library (the host-sanitizer
# variant, see sanitize.py)
LIB_PATH = os.environ.get("PF_LIB") or os.path.join(_HERE, "_lib", "libexagridpf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_1711_10579_amd.build)")


def _preload_torch_hip_runtime():
    """Load PyTorch's HIP runtime (if PyTorch is installed) before the library,
    so that the library and PyTorch share one HIP runtime in this process."""
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return
    p = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
    if os.path.exists(p):
        C.CDLL(p, mode=C.RTLD_GLOBAL)


_preload_torch_hip_runtime()
_lib = C.CDLL(LIB_PATH)

PF_OK, PF_E_INVALID, PF_E_NOMEM, PF_E_DEVICE, PF_E_BUSY, PF_E_NOTFOUND = range(6)
PF_CONVERGED, PF_MAXITER, PF_DIVERGED, PF_SINGULAR, PF_LINEAR_FAIL, PF_PENDING, PF_FAILED = range(7)
PF_MODEL_POLAR_1PH, PF_MODEL_CIM_3PH = 0, 1
PF_PQ, PF_PV, PF_SLACK = 1, 2, 3
PF_SOLVER_LU, PF_SOLVER_GMRES, PF_SOLVER_BICGSTAB = 0, 1, 2
PF_PREC_FP64, PF_PREC_MIXED = 0, 1
PF_PRECOND_ILU0, PF_PRECOND_BJACOBI = 0, 1
(PF_K_MISMATCH, PF_K_JFILL, PF_K_SPARSE_FACTOR, PF_K_TAIL_SCHUR, PF_K_DENSE_PANEL,
 PF_K_DENSE_UPDATE, PF_K_SPARSE_FWD, PF_K_SPARSE_BWD, PF_K_DENSE_TRSV, PF_K_UPDATE,
 PF_K_KRYLOV, PF_K_PRECOND_SETUP, PF_K_PRECOND_APPLY, PF_K_COUNT) = range(14)
KERNEL_CLASS_NAMES = ["mismatch", "jfill", "sparse_factor", "tail_schur", "dense_panel",
                      "dense_update", "sparse_fwd", "sparse_bwd", "dense_trsv", "update",
                      "krylov", "precond_setup", "precond_apply"]

STATUS_NAMES = {0: "converged", 1: "maxiter", 2: "diverged", 3: "singular",
                4: "linear_fail", 5: "pending", 6: "failed"}


class pf_case_desc(C.Structure):
    _fields_ = [("model", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int32)), ("col_idx", C.POINTER(C.c_int32)),
                ("y", C.POINTER(C.c_double)), ("bus_type", C.POINTER(C.c_int8)),
                ("p_sp", C.POINTER(C.c_double)), ("q_sp", C.POINTER(C.c_double)),
                ("v_mag", C.POINTER(C.c_double)), ("v_ang", C.POINTER(C.c_double)),
                ("zip", C.POINTER(C.c_double)), ("delta_to", C.POINTER(C.c_int32)),
                ("zip_delta", C.POINTER(C.c_double))]


class pf_options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("solver", C.c_int32),
                ("precision", C.c_int32), ("precond", C.c_int32), ("gmres_m", C.c_int32),
                ("gmres_max_restarts", C.c_int32), ("flat_start", C.c_int32),
                ("nk_fallback", C.c_int32), ("eta_max", C.c_double)]


class pf_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("linear_iters", C.c_int32),
                ("lu_fallback", C.c_int32), ("mismatch_inf", C.c_double), ("max_step", C.c_double),
                ("device_ms", C.c_double), ("error", C.c_int32), ("reserved", C.c_int32),
                ("wait_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class pf_schedule(C.Structure):
    _fields_ = [("dense_switch", C.c_double), ("min_dense", C.c_int32), ("lane_scale", C.c_int32),
                ("trsv_mode", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class pf_tune_report(C.Structure):
    _fields_ = [("candidates", C.c_int32), ("trials", C.c_int32), ("default_ms", C.c_double),
                ("best_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pf_case_info(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_unknown", C.c_int32), ("n_sparse", C.c_int32),
                ("n_dense", C.c_int32), ("levels", C.c_int32), ("bwd_levels", C.c_int32),
                ("nnz_l_blocks", C.c_int64), ("updates", C.c_int64), ("tail_updates", C.c_int64),
                ("flops_factor", C.c_double), ("device_bytes", C.c_size_t),
                ("analysis_ms", C.c_double), ("resident_bytes", C.c_size_t), ("work_bytes", C.c_size_t),
                ("krylov_bytes", C.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class pf_kernel_stat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_P = C.c_void_p
_sig = {
    "pf_default_options": (None, [C.POINTER(pf_options)]),
    "pf_ctx_create": (C.c_int, [C.c_int32, _P, ALLOC_FN, FREE_FN, _P, C.POINTER(_P)]),
    "pf_ctx_destroy": (None, [_P]),
    "pf_create": (C.c_int, [_P, C.POINTER(pf_case_desc), C.POINTER(_P)]),
    "pf_default_schedule": (None, [C.POINTER(pf_schedule)]),
    "pf_ctx_use_graphs": (C.c_int, [_P, C.c_int32]),
    "pf_create_scheduled": (C.c_int, [_P, C.POINTER(pf_case_desc), C.POINTER(pf_schedule), C.POINTER(_P)]),
    "pf_case_schedule": (C.c_int, [_P, C.POINTER(pf_schedule)]),
    "pf_autotune": (C.c_int, [_P, C.POINTER(pf_case_desc), C.POINTER(pf_options), C.c_int32,
                              C.POINTER(pf_schedule), C.POINTER(pf_tune_report)]),
    "pf_destroy": (C.c_int, [_P]),
    "pf_case_info_get": (C.c_int, [_P, C.POINTER(pf_case_info)]),
    "pf_case_footprint": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "pf_set_injections": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "pf_solve": (C.c_int, [_P, C.POINTER(pf_options), C.POINTER(pf_result)]),
    "pf_solve_noalloc": (C.c_int, [_P, C.POINTER(pf_options), C.POINTER(pf_result), C.POINTER(C.c_size_t)]),
    "pf_solve_batch": (C.c_int, [_P, C.POINTER(_P), C.c_int32, C.POINTER(pf_options),
                                 C.POINTER(pf_result)]),
    "pf_submit": (C.c_int, [_P, _P, C.POINTER(pf_options), C.POINTER(C.c_uint64)]),
    "pf_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(pf_result), C.POINTER(C.c_int32)]),
    "pf_serve_config": (C.c_int, [_P, C.c_size_t, C.c_int32]),
    "pf_serve_stats": (C.c_int, [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]),
    "pf_get_voltage": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pf_set_voltage": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pf_profile_enable": (C.c_int, [_P, C.c_int32]),
    "pf_kernel_stats": (C.c_int, [_P, C.c_int32, C.POINTER(pf_kernel_stat)]),
    "pf_profile_reset": (C.c_int, [_P]),
    "pf_debug_schedule_check": (C.c_int, [C.POINTER(pf_case_desc), C.POINTER(pf_schedule), C.c_uint64,
                                          C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "pf_debug_krylov_check": (C.c_int, [C.POINTER(pf_case_desc), C.c_uint64, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "pf_debug_precond_check": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "pf_last_error": (C.c_char_p, []),
    "pf_version": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_sig)


class PFError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: status {code}: {_lib.pf_last_error().decode()}")


def _check(code, where):
    if code != PF_OK:
        raise PFError(code, where)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def pf_version():
    return _lib.pf_version().decode()


def pf_last_error():
    return _lib.pf_last_error().decode()


def pf_default_options(**kw):
    o = pf_options()
    _lib.pf_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Context:
    """A pf_ctx handle; ``use_torch`` routes device memory through PyTorch's
    caching allocator and launches on torch's current stream."""

    def __init__(self, device=0, stream=None, use_torch=False):
        self._keep = []
        alloc = ALLOC_FN()
        free = FREE_FN()
        if use_torch:
            import torch

            torch.cuda.set_device(device)
            if stream is None:
                stream = torch.cuda.current_stream(device).cuda_stream

            def _alloc(nbytes, _user):
                return torch.cuda.caching_allocator_alloc(nbytes, device)

            def _free(ptr, _user):
                torch.cuda.caching_allocator_delete(ptr)

            alloc, free = ALLOC_FN(_alloc), FREE_FN(_free)
            self._keep += [alloc, free]
        self.device = device
        h = C.c_void_p()
        _check(_lib.pf_ctx_create(device, C.c_void_p(stream) if stream else None, alloc, free,
                                  None, C.byref(h)), "pf_ctx_create")
        self.handle = h

    def close(self):
        if self.handle:
            _lib.pf_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pf_ctx_create(device=0, stream=None, use_torch=False):
    return Context(device, stream, use_torch)


def pf_ctx_destroy(ctx):
    ctx.close()


class Case:
    def __init__(self, ctx, handle, n, model):
        self.ctx = ctx
        self.handle = handle
        self.n = n
        self.model = model

    def close(self):
        if self.handle:
            _check(_lib.pf_destroy(self.handle), "pf_destroy")
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                _lib.pf_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def _desc(model, row_ptr, col_idx, y, bus_type, v_mag, v_ang, p_sp, q_sp, zip, delta_to=None, zip_delta=None):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    yv = np.ascontiguousarray(np.asarray(y, np.complex128).view(np.float64))
    bt = np.ascontiguousarray(bus_type, np.int8)
    vm = np.ascontiguousarray(v_mag, np.float64)
    va = np.ascontiguousarray(v_ang, np.float64)
    ps = None if p_sp is None else np.ascontiguousarray(p_sp, np.float64)
    qs = None if q_sp is None else np.ascontiguousarray(q_sp, np.float64)
    zp = None if zip is None else np.ascontiguousarray(np.asarray(zip, np.float64).reshape(-1))
    dt = None if delta_to is None else np.ascontiguousarray(delta_to, np.int32)
    zd = None if zip_delta is None else np.ascontiguousarray(np.asarray(zip_delta, np.float64).reshape(-1))
    n = bt.shape[0]
    d = pf_case_desc(model=model, n=n, nnz=ci.shape[0],
                     row_ptr=rp.ctypes.data_as(C.POINTER(C.c_int32)),
                     col_idx=ci.ctypes.data_as(C.POINTER(C.c_int32)),
                     y=_dptr(yv), bus_type=bt.ctypes.data_as(C.POINTER(C.c_int8)),
                     p_sp=_dptr(ps), q_sp=_dptr(qs), v_mag=_dptr(vm), v_ang=_dptr(va),
                     zip=_dptr(zp),
                     delta_to=None if dt is None else dt.ctypes.data_as(C.POINTER(C.c_int32)),
                     zip_delta=_dptr(zd))
    keep = (rp, ci, yv, bt, vm, va, ps, qs, zp, dt, zd)
    return d, n, keep


def pf_ctx_use_graphs(ctx, on):
    _check(_lib.pf_ctx_use_graphs(ctx.handle, int(bool(on))), "pf_ctx_use_graphs")


def pf_default_schedule(**kw):
    sc = pf_schedule()
    _lib.pf_default_schedule(C.byref(sc))
    for k, v in kw.items():
        if not hasattr(sc, k):
            raise TypeError(f"unknown schedule field {k}")
        setattr(sc, k, v)
    return sc


def pf_create(ctx, model, row_ptr, col_idx, y, bus_type, v_mag, v_ang, p_sp=None, q_sp=None,
              zip=None, schedule=None, delta_to=None, zip_delta=None):
    """Create a case from host arrays (Ybus CSR with complex values ``y``);
    ``schedule`` (a pf_schedule) selects pf_create_scheduled."""
    d, n, keep = _desc(model, row_ptr, col_idx, y, bus_type, v_mag, v_ang, p_sp, q_sp, zip, delta_to,
                       zip_delta)
    if schedule is not None:
        h = _P()
        _check(_lib.pf_create_scheduled(ctx.handle, C.byref(d), C.byref(schedule), C.byref(h)),
               "pf_create_scheduled")
        del keep
        return Case(ctx, h, n, model)
    h = C.c_void_p()
    _check(_lib.pf_create(ctx.handle, C.byref(d), C.byref(h)), "pf_create")
    del keep
    return Case(ctx, h, n, model)


def case_arrays(case):
    """Keyword arguments of pf_create for a seeded grid object."""
    if hasattr(case, "bus_type"):
        return dict(model=PF_MODEL_POLAR_1PH, row_ptr=case.row_ptr, col_idx=case.col, y=case.y,
                    bus_type=case.bus_type, v_mag=case.v_mag, v_ang=case.v_ang,
                    p_sp=case.p_sp, q_sp=case.q_sp, zip=None)
    out = dict(model=PF_MODEL_CIM_3PH, row_ptr=case.row_ptr, col_idx=case.col, y=case.y,
               bus_type=case.node_type, v_mag=case.v_mag, v_ang=case.v_ang,
               p_sp=case.p_gen, q_sp=case.q_gen, zip=case.zip)
    if getattr(case, "delta_to", None) is not None:
        out.update(delta_to=case.delta_to, zip_delta=case.zip_delta)
    return out


def pf_debug_schedule_check(model, row_ptr, col_idx, y, bus_type, v_mag, v_ang, p_sp=None,
                            q_sp=None, zip=None, seed=0, schedule=None, delta_to=None, zip_delta=None):
    """Host-only replay of the analysis schedule (include/pf_debug.h).
    Returns (relative residual, number of index checks)."""
    d, _, keep = _desc(model, row_ptr, col_idx, y, bus_type, v_mag, v_ang, p_sp, q_sp, zip, delta_to,
                       zip_delta)
    res = C.c_double()
    chk = C.c_int64()
    sp_ = C.byref(schedule) if schedule is not None else None
    _check(_lib.pf_debug_schedule_check(C.byref(d), sp_, C.c_uint64(seed), C.byref(res), C.byref(chk)),
           "pf_debug_schedule_check")
    del keep
    return res.value, chk.value


def pf_debug_krylov_check(model, row_ptr, col_idx, y, bus_type, v_mag, v_ang, p_sp=None,
                          q_sp=None, zip=None, seed=0, delta_to=None, zip_delta=None):
    """Host-only check of the Krylov analysis (include/pf_debug.h).
    Returns (ILU(0) deviation on the pattern, relative residual, checks)."""
    d, _, keep = _desc(model, row_ptr, col_idx, y, bus_type, v_mag, v_ang, p_sp, q_sp, zip, delta_to,
                       zip_delta)
    dev = C.c_double()
    res = C.c_double()
    chk = C.c_int64()
    _check(_lib.pf_debug_krylov_check(C.byref(d), C.c_uint64(seed), C.byref(dev), C.byref(res),
                                      C.byref(chk)), "pf_debug_krylov_check")
    del keep
    return dev.value, res.value, chk.value


def pf_debug_precond_check(case, precond):
    """Device check of the preconditioner set-up kernels at the case's flat
    start (include/pf_debug.h).  Returns (deviation, largest block order)."""
    dev = C.c_double()
    order = C.c_int32()
    _check(_lib.pf_debug_precond_check(case.handle, int(precond), C.byref(dev), C.byref(order)),
           "pf_debug_precond_check")
    return dev.value, order.value


def pf_create_from(ctx, case, schedule=None):
    """Convenience: create from a seeded grid object (single-phase or feeder)."""
    return pf_create(ctx, **case_arrays(case), schedule=schedule)


def pf_case_schedule(case):
    sc = pf_schedule()
    _check(_lib.pf_case_schedule(case.handle, C.byref(sc)), "pf_case_schedule")
    return sc


def pf_autotune(ctx, case, options=None, trials=3, **kw):
    """Autotune the schedule of a seeded grid object's topology (stored in the
    context for later pf_create calls).  Returns (pf_schedule, report dict)."""
    o = options if options is not None else pf_default_options(**kw)
    d, _, keep = _desc(**case_arrays(case))
    best = pf_schedule()
    rep = pf_tune_report()
    _check(_lib.pf_autotune(ctx.handle, C.byref(d), C.byref(o), int(trials), C.byref(best), C.byref(rep)),
           "pf_autotune")
    del keep
    return best, rep.as_dict()


def pf_destroy(case):
    case.close()


def pf_case_info_get(case):
    info = pf_case_info()
    _check(_lib.pf_case_info_get(case.handle, C.byref(info)), "pf_case_info_get")
    return info.as_dict()


def pf_case_footprint(case):
    """Device bytes of an LU solve of the case: resident plus working storage."""
    b = C.c_size_t()
    _check(_lib.pf_case_footprint(case.handle if case is not None else None, C.byref(b)), "pf_case_footprint")
    return b.value


def pf_set_injections(case, p_sp=None, q_sp=None, zip=None):
    ps = None if p_sp is None else np.ascontiguousarray(p_sp, np.float64)
    qs = None if q_sp is None else np.ascontiguousarray(q_sp, np.float64)
    zp = None if zip is None else np.ascontiguousarray(np.asarray(zip, np.float64).reshape(-1))
    _check(_lib.pf_set_injections(case.handle, _dptr(ps), _dptr(qs), _dptr(zp)),
           "pf_set_injections")


def pf_solve(case, options=None, **kw):
    o = options if options is not None else pf_default_options(**kw)
    r = pf_result()
    _check(_lib.pf_solve(case.handle, C.byref(o), C.byref(r)), "pf_solve")
    return r


def pf_solve_noalloc(case, options=None, **kw):
    """The LU solve in the library's fixed per-device array.  Returns
    (pf_result, scratch bytes the case needs)."""
    o = options if options is not None else pf_default_options(**kw)
    r = pf_result()
    used = C.c_size_t()
    _check(_lib.pf_solve_noalloc(case.handle, C.byref(o), C.byref(r), C.byref(used)), "pf_solve_noalloc")
    return r, used.value


def pf_solve_batch(ctx, cases, options=None, **kw):
    o = options if options is not None else pf_default_options(**kw)
    arr = (C.c_void_p * len(cases))(*[c.handle.value for c in cases])
    res = (pf_result * len(cases))()
    _check(_lib.pf_solve_batch(ctx.handle, arr, len(cases), C.byref(o), res), "pf_solve_batch")
    return list(res)


def pf_submit(ctx, case, options=None, **kw):
    o = options if options is not None else pf_default_options(**kw)
    t = C.c_uint64()
    _check(_lib.pf_submit(ctx.handle, case.handle, C.byref(o), C.byref(t)), "pf_submit")
    return t.value


def pf_poll(ctx, ticket):
    """Returns (done, pf_result)."""
    r = pf_result()
    d = C.c_int32()
    _check(_lib.pf_poll(ctx.handle, C.c_uint64(ticket), C.byref(r), C.byref(d)), "pf_poll")
    return bool(d.value), r


def pf_serve_config(ctx, max_bytes=0, max_slots=0):
    _check(_lib.pf_serve_config(ctx.handle, max_bytes, max_slots), "pf_serve_config")


def pf_serve_stats(ctx):
    """Serving pool bytes, bytes lent now, requests queued and running."""
    pool, lent = C.c_size_t(), C.c_size_t()
    q, r = C.c_int32(), C.c_int32()
    _check(_lib.pf_serve_stats(ctx.handle, C.byref(pool), C.byref(lent), C.byref(q), C.byref(r)),
           "pf_serve_stats")
    return {"pool_bytes": pool.value, "lent_bytes": lent.value, "queued": q.value, "running": r.value}


def pf_get_voltage(case):
    re = np.empty(case.n)
    im = np.empty(case.n)
    _check(_lib.pf_get_voltage(case.handle, _dptr(re), _dptr(im)), "pf_get_voltage")
    return re + 1j * im


def pf_set_voltage(case, V):
    V = np.asarray(V, np.complex128)
    re = np.ascontiguousarray(V.real)
    im = np.ascontiguousarray(V.imag)
    _check(_lib.pf_set_voltage(case.handle, _dptr(re), _dptr(im)), "pf_set_voltage")


PF_PROFILE_SPANS = 1 << 30


def pf_profile_enable(ctx, mask=-1):
    """Instrument the kernel classes whose bit (1 << class) is set in mask
    (with PF_PROFILE_SPANS: one event pair per run of consecutive launches)."""
    _check(_lib.pf_profile_enable(ctx.handle, int(mask)), "pf_profile_enable")


def pf_profile_reset(ctx):
    _check(_lib.pf_profile_reset(ctx.handle), "pf_profile_reset")


def pf_kernel_stats(ctx, kernel_class):
    s = pf_kernel_stat()
    _check(_lib.pf_kernel_stats(ctx.handle, kernel_class, C.byref(s)), "pf_kernel_stats")
    return {"launches": s.launches, "ms": s.ms, "flops": s.flops, "bytes": s.bytes}
