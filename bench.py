#!/usr/bin/env python3
"""Throughput of converged Newton power-flow solves on one MI355X.

Default workload: a step is one complete power-flow solve (flat start to
max-norm FP64 mismatch <= 1e-8 pu) of the 10,000-bus meshed transmission grid
(seeded synthetic; tree + 3,000 uniform chords, 1,000 PV buses, balanced
dispatch), with every Newton phase on the GPU: mismatch, Jacobian fill, sparse
refactorisation with its dense trailing block, triangular solves, voltage
update and the convergence test.  Inputs are resident in device memory before
the timed region.  Prints one JSON line with solves/s, latency percentiles,
the batched form on the same grid, the roofline of the dominant kernel (timed
with HIP events inside the timed region) and the CPU oracle timed on a
bounded sample of the same work.

The default line also carries the two target forms as fields: 512 grids of
100-5,000 buses with FP32 inner solves in one pf_solve_batch, and the served
mix (Poisson arrivals, admission by the serving pool's budget) beside the
plain FP64 one-at-a-time GPU Newton on the same requests; every leg reports
max |V - V_oracle| against the oracle's root on a stated sample.

Other modes (each prints its own JSON line):
  --workload scenarios512   512 grids of 100-5,000 buses, FP32 inner solves,
                            one pf_solve_batch per step
  --workload served         Poisson-arriving requests on a pool of single- and
                            three-phase grids through pf_submit/pf_poll
  --workload replication    the paper's replication-scale cases (Sec. IV):
                            the 48,000-bus grid (LU, GMRES, BiCGStab) and the
                            0.9K-230K-bus feeders of Table 1 (LU), solve
                            times beside the paper's CPU times (context);
                            with --feeder-copies 256 (say) only those feeders
  --calibrate-copy          a plain 256 MiB device copy (for scaling the
                            FETCH_SIZE / WRITE_SIZE counters)
"""

import argparse
import json
import os
import random
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks: HBM 8 TB/s; FP64 vector and FP64 matrix 78.6 TFLOP/s (vector:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz); FP32 matrix and FP32
# vector (packed) 157.3 TFLOP/s.  The dominant kernel's flops are mostly its
# matrix-core products; its time is set by the dependent chain of the
# diagonal block's inverse and of the next panel's tiles.
PEAK = {"hbm_gbs": 8000.0, "fp64_tflops": 78.6, "fp32_mfma_tflops": 157.3, "fp32_valu_tflops": 157.3}
METRIC = "converged PF solves/s at 1e-8 pu mismatch, batched vs plain; p50/p99 latency"


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def _cpu_worker(args):
    """One CPU worker of the all-cores baseline (a fresh interpreter): whole
    oracle solves of the 10,000-bus grid, one thread, until the budget is
    spent (at least one).  Returns (solves, seconds)."""
    budget_s, start_at = args
    from threadpoolctl import threadpool_limits

    import pfgen
    from oracle import polar

    case = pfgen.config_case(1)
    while time.time() < start_at:  # every worker starts together
        time.sleep(0.01)
    done, t0 = 0, time.perf_counter()
    with threadpool_limits(limits=1):
        while True:
            r = polar.newton(case, tol=1e-8)
            assert r.status == 0
            done += 1
            if time.perf_counter() - t0 >= budget_s:
                break
    return done, time.perf_counter() - t0


def cpu_baseline(case, budget_s=8.0, one_core_max=5):
    """The CPU oracle as it stands on whole solves of the same grid (tol 1e-8):
    one thread for up to `one_core_max` solves, then one single-threaded
    process per host core (at most 16, the host share of one GPU) over the
    same grid, each until `budget_s` is spent."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import polar

    done, t0 = 0, time.perf_counter()
    with threadpool_limits(limits=1):
        while True:
            r = polar.newton(case, tol=1e-8)
            assert r.status == 0
            done += 1
            if time.perf_counter() - t0 >= 20.0 or done >= one_core_max:
                break
    el = time.perf_counter() - t0
    one = {"value": done / el, "unit": "solves/s", "cores": 1,
           "sample": f"{done} full solves of the 10,000-bus grid (tol 1e-8), {el:.1f} s, 1 thread"}
    procs = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        start_at = time.time() + 8.0  # after every interpreter has imported NumPy and SciPy
        res = pool.map(_cpu_worker, [(budget_s, start_at)] * procs)
    total = sum(d for d, _ in res)
    span = max(t for _, t in res)
    return {"value": total / span, "unit": "solves/s", "cores": procs, "kind": "oracle",
            "sample": f"{total} full solves of the 10,000-bus grid (tol 1e-8) by {procs} single-threaded "
                      f"processes in {span:.1f} s (host nproc {os.cpu_count()}), FP64 NumPy/SciPy SuperLU",
            "one_core": one}


def _schedule_key(sc):
    return (f"dense_switch={sc['dense_switch']:g} min_dense={sc['min_dense']} "
            f"lane_scale={sc['lane_scale']} trsv_mode={sc['trsv_mode']}")


def _measured_traffic(kernel, schedule):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary (already scaled by the plain-copy calibration), or None
    when the kernel source or the case's schedule (which sets the dense block's
    size) differ from those the counters were taken with."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_grid10k_pmc.md")
    src = os.path.join(ROOT, "paper_1711_10579_amd", "csrc", "dense.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    val, cap, sched = None, None, None
    for line in text.splitlines():
        if line.startswith(f"traffic_bytes_per_launch {kernel}:"):
            val = float(line.split(":")[1])
        if line.startswith("dense.hip sha256 prefix at capture:"):
            cap = line.split(":")[1].strip()
        if line.startswith("schedule at capture:"):
            sched = line.split(":", 1)[1].strip()
    return val if cap == sha and sched == _schedule_key(schedule) else None


def _dense_roof(st, M, peak, mixed, sched):
    """Roofline of the dense block's step launches on the matrix cores.

    Algorithmic flops of the dense block's factorisation are (2/3) M^3 for
    dense order M (LU of the trailing block; the right-hand side column and
    the explicit diagonal-block inverses the library forms are not counted),
    spread over its ceil(M / 64) step launches; the library's own count,
    which includes the inverses (2 kb^3 per step) and the products by them,
    is reported beside it."""
    n = max(st["launches"], 1)
    avg_ms = st["ms"] / n
    steps = -(-M // 64)
    per = (2.0 / 3.0) * M ** 3 / steps
    achieved = per / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    lib_per = st["flops"] / n
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None if mixed else _measured_traffic("k_dense_step", sched),
            "kernel": "k_dense_step (block step k of the dense block: diagonal-block inverse by block "
                      "Gauss-Jordan, row tiles times it, and the matrix-core trailing update)",
            "avg_launch_ms": avg_ms, "launches": st["launches"], "dense_order": M,
            "launches_per_factorisation": steps,
            "flops_per_launch": per, "flops_basis": "(2/3) M^3 per factorisation / launches",
            "library_flops_per_launch": lib_per,
            "library_achieved": lib_per / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0,
            "timing": "HIP events on the library stream around each Newton step's run of k_dense_step "
                      "launches inside the replayed graph; per launch = span / launches (includes the gaps "
                      "between them)"}


def _vm_va_err(V, ref_vm, ref_va):
    import numpy as np

    return float(max(np.max(np.abs(np.abs(V) - ref_vm)), np.max(np.abs(np.angle(V) - ref_va))))


def _oracle_err(case, V):
    """max |V - V_oracle| against the oracle's own root (magnitudes in pu and
    angles in rad for single-phase grids, complex phase voltages for feeders)."""
    import numpy as np

    from oracle import cim, polar

    if hasattr(case, "bus_type"):
        ref = polar.newton(case)
        assert ref.status == 0
        return _vm_va_err(V, ref.vm, ref.va)
    ref = cim.newton(case)
    assert ref.status == 0
    return float(np.max(np.abs(V - ref.V)))


def _with_hbm(roof):
    """Add the HBM rate the measured traffic implies (bytes per launch over
    the average launch time) against the 8 TB/s peak."""
    if roof.get("traffic") and roof.get("avg_launch_ms"):
        gbs = roof["traffic"] / (roof["avg_launch_ms"] * 1e-3) / 1e9
        roof["hbm"] = {"achieved": gbs, "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": gbs / PEAK["hbm_gbs"]}
    return roof


def _breakdown(B, ctx, h, opts, tag, solves=3):
    """Every kernel class timed with HIP events over a few extra solves
    (stderr)."""
    B.pf_profile_enable(ctx, -1)
    B.pf_profile_reset(ctx)
    for _ in range(solves):
        B.pf_solve(h, opts)
    rows = [(name, B.pf_kernel_stats(ctx, k)) for k, name in enumerate(B.KERNEL_CLASS_NAMES)]
    tot = sum(s["ms"] for _, s in rows)
    for name, s in rows:
        if s["launches"]:
            print(f"[breakdown {tag}] {name:14s} launches/solve={s['launches'] / solves:8.1f} "
                  f"ms/solve={s['ms'] / solves:8.4f} ({100 * s['ms'] / tot:5.1f}%) "
                  f"GFLOP/s={s['flops'] / max(s['ms'], 1e-12) / 1e6:9.1f}", file=sys.stderr)
    B.pf_profile_enable(ctx, 0)


def calibrate_copy():
    import torch

    nbytes = 256 << 20
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(json.dumps({"mode": "calibrate-copy", "bytes_read_per_copy": nbytes,
                      "bytes_written_per_copy": nbytes, "copies": reps,
                      "GBps": 2 * nbytes * reps / el / 1e9}), flush=True)


def bench_grid10k(args):
    import numpy as np
    import torch

    import pfgen
    from oracle import polar
    from paper_1711_10579_amd import binding as B

    case = pfgen.config_case(1)
    ctx = B.pf_ctx_create(0)
    mixed = args.precision == "mixed"
    opts = B.pf_default_options(precision=int(mixed), max_iter=40 if mixed else 20)
    # the autotuner picks this topology's schedule (set-up, outside the timed
    # region); pf_create then uses it
    tuned = None
    fixed = None
    if args.schedule:
        ds, md, ls, tm = args.schedule.split(",")
        fixed = B.pf_default_schedule(dense_switch=float(ds), min_dense=int(md), lane_scale=int(ls),
                                      trsv_mode=int(tm))
    elif not args.no_autotune:
        t0 = time.perf_counter()
        best, rep = B.pf_autotune(ctx, case, opts, trials=3)
        tuned = {"schedule": best.as_dict(), "report": rep, "tune_s": time.perf_counter() - t0}
    h = B.pf_create_from(ctx, case, schedule=fixed)
    info = B.pf_case_info_get(h)
    sched = B.pf_case_schedule(h).as_dict()

    for _ in range(args.warmup):
        r = B.pf_solve(h, opts)
        assert r.status == B.PF_CONVERGED, r.as_dict()

    if args.breakdown:
        _breakdown(B, ctx, h, opts, "lu")

    # the dominant kernel (the dense block's step launches) is timed with HIP
    # events on the library's stream inside the timed region (captured into
    # the replayed Newton-step graph with the kernels): one event pair around
    # each Newton step's run of block-step launches
    dom = B.PF_K_DENSE_PANEL
    B.pf_profile_enable(ctx, (1 << dom) | B.PF_PROFILE_SPANS)
    B.pf_profile_reset(ctx)
    torch.cuda.synchronize()
    lat, conv, iters = [], 0, []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        r = B.pf_solve(h, opts)
        lat.append(time.perf_counter() - s0)
        conv += r.status == B.PF_CONVERGED
        iters.append(r.iters)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st_dom = B.pf_kernel_stats(ctx, dom)
    B.pf_profile_enable(ctx, 0)
    V_lu = B.pf_get_voltage(h)
    mism = polar.mismatch_at(case, V_lu)
    # the oracle's root of the same grid (run to its floor), for the error of
    # every leg on this grid
    ref = polar.newton(case)
    assert ref.status == 0
    err = lambda V: _vm_va_err(V, ref.vm, ref.va)  # noqa: E731

    # Newton-Krylov on the same grid, forcing term min(0.1, ||F||_inf):
    # GMRES(30) and BiCGStab (the method the paper tested), right
    # preconditioned with block ILU(0) or block-Jacobi
    def krylov_run(solver, label, precond=B.PF_PRECOND_ILU0):
        nopts = B.pf_default_options(solver=solver, precision=int(mixed), max_iter=40, precond=precond)
        for _ in range(max(1, args.warmup)):
            r = B.pf_solve(h, nopts)
            assert r.status == B.PF_CONVERGED, r.as_dict()
        if args.breakdown:
            _breakdown(B, ctx, h, nopts, label)
        torch.cuda.synchronize()
        nlat, nconv, nlin, nit = [], 0, [], []
        t0 = time.perf_counter()
        for _ in range(args.nk_steps):
            s0 = time.perf_counter()
            r = B.pf_solve(h, nopts)
            nlat.append(time.perf_counter() - s0)
            nconv += r.status == B.PF_CONVERGED
            nlin.append(r.linear_iters)
            nit.append(r.iters)
        torch.cuda.synchronize()
        nel = time.perf_counter() - t0
        V = B.pf_get_voltage(h)
        return {"value": nconv / nel, "unit": "solves/s", "steps": args.nk_steps, "converged": nconv,
                "latency_ms": {"p50": 1000 * _pct(nlat, 50), "p99": 1000 * _pct(nlat, 99)},
                "solver": label + ("+ilu0" if precond == B.PF_PRECOND_ILU0 else "+block-jacobi"),
                "newton_iters": int(np.median(nit)),
                "inner_iters_per_solve": int(np.median(nlin)),
                "final_mismatch_oracle": polar.mismatch_at(case, V), "max_err_vs_oracle": err(V)}

    nk = nk_bcg = nk_bcg_bj = None
    if args.nk_steps > 0:
        nk = krylov_run(B.PF_SOLVER_GMRES, "gmres(30)")
        nk_bcg = krylov_run(B.PF_SOLVER_BICGSTAB, "bicgstab")
        nk_bcg_bj = krylov_run(B.PF_SOLVER_BICGSTAB, "bicgstab", B.PF_PRECOND_BJACOBI)

    # batched form: the same grid under seeded load scenarios, one
    # pf_solve_batch per step
    batched = None
    if args.batch > 1:
        scen = [pfgen.perturb_loads(case, 7000 + i) for i in range(args.batch)]
        hb = [B.pf_create_from(ctx, sc) for sc in scen]
        for _ in range(max(1, args.warmup)):
            B.pf_solve_batch(ctx, hb, opts)
        bsteps = max(2, args.steps // 4)
        torch.cuda.synchronize()
        blat, bconv = [], 0
        t0 = time.perf_counter()
        for _ in range(bsteps):
            s0 = time.perf_counter()
            rs = B.pf_solve_batch(ctx, hb, opts)
            blat.append(time.perf_counter() - s0)
            bconv += sum(r.status == B.PF_CONVERGED for r in rs)
        torch.cuda.synchronize()
        bel = time.perf_counter() - t0
        berr = [_oracle_err(scen[i], B.pf_get_voltage(hb[i])) for i in (0, len(scen) - 1)]
        batched = {"instances": args.batch, "value": bconv / bel, "unit": "solves/s",
                   "batch_latency_ms": {"p50": 1000 * _pct(blat, 50), "p99": 1000 * _pct(blat, 99)},
                   "steps": bsteps, "converged": bconv,
                   "final_mismatch_oracle": polar.mismatch_at(scen[-1], B.pf_get_voltage(hb[-1])),
                   "max_err_vs_oracle": max(berr), "oracle_sample": "scenarios 0 and last"}
        for x in hb:
            x.close()

    # the target forms: 512 mixed-precision scenarios in one batch, and the
    # served mix against the plain FP64 one-at-a-time GPU Newton
    s512 = run_scenarios512(args, B, ctx) if args.with_targets else None
    served = run_served(args, B, ctx) if args.with_targets else None

    mfma_peak = PEAK["fp32_mfma_tflops"] if mixed else PEAK["fp64_tflops"]
    out = {
        "metric": METRIC,
        "value": conv / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not mixed else "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": "10,000-bus meshed grid, plain Newton-Raphson with sparse LU "
                               "(one solve per step, flat start to 1e-8 pu)",
                   "buses": case.n, "branches": case.m, "pv_buses": int((case.bus_type == 2).sum()),
                   "solver": "lu", "precision": args.precision,
                   "dense_block": info["n_dense"], "levels": info["levels"],
                   "schedule": _schedule_key(sched),
                   "newton_iters": int(np.median(iters))},
        "latency_ms": {"p50": 1000 * _pct(lat, 50), "p99": 1000 * _pct(lat, 99)},
        "converged": conv,
        "final_mismatch_oracle": mism,
        "max_err_vs_oracle": err(V_lu),
        "roofline": _with_hbm(_dense_roof(st_dom, 2 * info["n_dense"], mfma_peak, mixed, sched)),
        "batched": batched,
        "scenarios512": s512,
        "served": served,
        "newton_krylov": nk,
        "newton_krylov_bicgstab": nk_bcg,
        "newton_krylov_bicgstab_bjacobi": nk_bcg_bj,
        "autotune": tuned,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


def run_scenarios512(args, B, ctx):
    """512 grids of 100-5,000 buses (log-uniform, own topologies, +-20 %
    loads), FP32 inner solves with FP64 mismatch, update and test, one
    pf_solve_batch per step; FP64-oracle error on the 8 largest scenarios and
    8 others."""
    import numpy as np
    import torch

    import pfgen

    t0 = time.perf_counter()
    scen = pfgen.c3_scenarios(args.instances)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    hs = [B.pf_create_from(ctx, c) for c in scen]
    t_setup = time.perf_counter() - t0
    mixed = args.target_precision != "fp64"
    opts = B.pf_default_options(precision=int(mixed), max_iter=40 if mixed else 20)
    B.pf_solve_batch(ctx, hs, opts)
    torch.cuda.synchronize()
    conv, steps, lat = 0, max(2, args.steps // 10), []
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        rs = B.pf_solve_batch(ctx, hs, opts)
        lat.append(time.perf_counter() - s0)
        conv += sum(r.status == B.PF_CONVERGED for r in rs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    order = list(np.argsort([c.n for c in scen]))
    rng = np.random.default_rng(1)
    sample = order[-8:] + list(rng.choice(order[:-8], size=min(args.oracle_sample, len(order) - 8), replace=False))
    errs = [_oracle_err(scen[i], B.pf_get_voltage(hs[i])) for i in sample]
    for h in hs:
        h.close()
    return {"value": conv / el, "unit": "solves/s", "instances": len(scen), "steps": steps, "converged": conv,
            "sum_buses": int(sum(c.n for c in scen)), "ms_per_batch": 1000 * el / steps,
            "batch_latency_ms": {"p50": 1000 * _pct(lat, 50), "p99": 1000 * _pct(lat, 99)},
            "precision": "f32-inner/f64-outer" if mixed else "f64", "setup_s": t_setup, "generate_s": t_gen,
            "iters": {"p50": float(np.median([r.iters for r in rs])), "max": int(max(r.iters for r in rs))},
            "final_mismatch_max": float(max(r.mismatch_inf for r in rs)),
            "max_err_vs_oracle": max(errs), "oracle_sample": f"{len(sample)} scenarios: the 8 largest and "
                                                              f"{len(sample) - 8} seeded others"}


def bench_scenarios512(args):
    from paper_1711_10579_amd import binding as B

    ctx = B.pf_ctx_create(0)
    out = {"mode": "scenarios512", "metric": METRIC}
    out.update(run_scenarios512(args, B, ctx))
    print(json.dumps(out), flush=True)


def run_served(args, B, ctx):
    """Poisson-arriving requests on a pool of 32 single-phase grids of
    1,000-20,000 buses and 16 feeders of 500-3,000 buses (70 % / 30 %), each
    with a fresh +-20 % load perturbation, mixed-precision LU through
    pf_submit / pf_poll at 0.8 x the plain FP64 serial rate; beside it the
    plain FP64 one-at-a-time GPU Newton on the same requests (its service
    times, and its FIFO queue under the same arrivals)."""
    import pfgen

    pool = pfgen.c4_pool(n_polar=args.pool_polar, n_feeder=args.pool_feeder)
    reps = 2
    t0 = time.perf_counter()
    # served handles (two replicas per grid) hold no working storage of their
    # own: every request borrows it from the serving pool at admission; the
    # plain serial baseline runs on handles of its own
    cases = [[B.pf_create_from(ctx, g) for _ in range(reps)] for g in pool]
    serial = [B.pf_create_from(ctx, g) for g in pool]
    setup_s = time.perf_counter() - t0
    mixed = args.target_precision != "fp64"
    opts = B.pf_default_options(precision=int(mixed), max_iter=40 if mixed else 20)
    plain = B.pf_default_options(precision=0, max_iter=20)
    rng = random.Random(11)
    n_req = args.requests
    n_pol = args.pool_polar
    reqs = []
    for k in range(n_req):
        g = rng.randrange(n_pol) if rng.random() < 0.7 else n_pol + rng.randrange(args.pool_feeder)
        reqs.append((g, 50000 + k))
    pert = [pfgen.perturb_loads(pool[g], s) for g, s in reqs]

    def prepare(h, p):
        if hasattr(p, "bus_type"):
            B.pf_set_injections(h, p.p_sp, p.q_sp)
        else:
            B.pf_set_injections(h, None, None, p.zip)

    for h in serial:  # warm the serial handles (device code, launch plans, graphs)
        B.pf_solve(h, plain)
    # warm the served handles through the serving loop itself (launch plans
    # built at their first submit, graphs captured at their first step)
    B.pf_serve_config(ctx, max_bytes=args.max_bytes, max_slots=args.slots)
    for row in cases:
        for h in row:
            t = B.pf_submit(ctx, h, opts)
            while not B.pf_poll(ctx, t)[0]:
                time.sleep(0.0002)
    # the plain FP64 one-at-a-time GPU Newton over the same requests: service
    # times (host clock around each pf_solve, injections included)
    service, serial_conv = [], 0
    for (g, _), p in zip(reqs, pert):
        h = serial[g]
        s0 = time.perf_counter()
        prepare(h, p)
        r = B.pf_solve(h, plain)
        service.append(time.perf_counter() - s0)
        serial_conv += r.status == B.PF_CONVERGED
    serial_rate = n_req / sum(service)
    lam = args.load_factor * serial_rate if args.rate <= 0 else args.rate
    arrivals = []
    t = 0.0
    for _ in range(n_req):
        t += rng.expovariate(lam)
        arrivals.append(t)
    # that serial server under the same arrivals: FIFO, one solve at a time
    done_t, q_lat = 0.0, []
    for a, sv in zip(arrivals, service):
        done_t = max(done_t, a) + sv
        q_lat.append(done_t - a)

    # requests whose voltages are compared with the oracle's root: feeders and
    # grids up to 5,000 buses (the oracle solves them in about a second)
    small = [k for k, (g, _) in enumerate(reqs) if getattr(pool[g], "n", 0) <= 5000 or not hasattr(pool[g], "bus_type")]
    check = set(small[:8])

    def run(arr, keep):
        free = {g: list(range(reps)) for g in range(len(pool))}
        inflight = {}
        lat, conv, done_n, waits = [], 0, 0, []
        volts = {}
        lent = 0
        waiting = []  # arrived but no free replica yet
        start = time.perf_counter()
        nxt = 0
        while done_n < n_req:
            now = time.perf_counter() - start
            while nxt < n_req and arr[nxt] <= now:
                waiting.append(nxt)
                nxt += 1
            still = []
            for k in waiting:
                g = reqs[k][0]
                if free[g]:
                    r_ = free[g].pop()
                    h = cases[g][r_]
                    prepare(h, pert[k])
                    inflight[B.pf_submit(ctx, h, opts)] = (k, g, r_)
                else:
                    still.append(k)
            waiting = still
            for tk in list(inflight):
                d, res = B.pf_poll(ctx, tk)
                if d:
                    k, g, r_ = inflight.pop(tk)
                    if keep and k in check:
                        volts[k] = B.pf_get_voltage(cases[g][r_])
                    free[g].append(r_)
                    lat.append(time.perf_counter() - start - arr[k])
                    waits.append(res.wait_ms)
                    conv += res.status == B.PF_CONVERGED
                    done_n += 1
            lent = max(lent, B.pf_serve_stats(ctx)["lent_bytes"])
            time.sleep(0.0002)
        return conv, time.perf_counter() - start, lat, volts, waits, lent

    conv, el, lat, volts, waits, lent = run(arrivals, True)
    # saturation: every request arrives at once (replicas still bound a grid's
    # concurrency)
    sconv, sel, _, _, _, slent = run([0.0] * n_req, False)
    pool_bytes = B.pf_serve_stats(ctx)["pool_bytes"]
    errs = [_oracle_err(pert[k], V) for k, V in volts.items()]
    for row in cases:
        for h in row:
            h.close()
    for h in serial:
        h.close()
    B.pf_serve_config(ctx, max_bytes=0)
    return {"value": conv / el, "unit": "solves/s", "requests": n_req, "converged": conv,
            "arrival_rate_per_s": lam, "load_factor": args.load_factor,
            "latency_ms": {"p50": 1000 * _pct(lat, 50), "p99": 1000 * _pct(lat, 99)},
            "admission_wait_ms": {"p50": _pct(waits, 50), "p99": _pct(waits, 99)},
            "precision": "f32-inner/f64-outer" if mixed else "f64",
            "saturation": {"value": sconv / sel, "converged": sconv},
            "plain_fp64_serial": {"value": serial_rate, "converged": serial_conv,
                                  "service_ms": {"p50": 1000 * _pct(service, 50), "p99": 1000 * _pct(service, 99)},
                                  "queued_latency_ms_same_arrivals": {"p50": 1000 * _pct(q_lat, 50),
                                                                      "p99": 1000 * _pct(q_lat, 99)}},
            "max_err_vs_oracle": max(errs) if errs else None,
            "oracle_sample": f"{len(errs)} served requests (feeders and grids up to 5,000 buses)",
            "pool": {"single_phase": args.pool_polar, "feeders": args.pool_feeder, "replicas": reps,
                     "setup_s": setup_s},
            "slots": args.slots,
            "memory": {"budget_bytes": args.max_bytes, "pool_bytes": pool_bytes, "max_lent_bytes": lent,
                       "max_lent_bytes_saturation": slent,
                       "note": "working storage of running requests, lent by the serving pool at admission"}}


def bench_served(args):
    from paper_1711_10579_amd import binding as B

    ctx = B.pf_ctx_create(0)
    out = {"mode": "served", "metric": METRIC}
    out.update(run_served(args, B, ctx))
    print(json.dumps(out), flush=True)


# the paper's CPU times (Sec. IV; Cori node): Krylov solve of the 48,000-bus
# grid on 1 and 32 threads, and Table 1's Solving / Other seconds of the
# Newton-Raphson (SuperLU) three-phase solves by feeder size
PAPER_NK_48K_S = {"threads_1": 1.2, "threads_32": 0.21}
PAPER_TABLE1_S = {1: (0.319107, 0.047195), 2: (0.389616, 0.059578), 4: (0.799942, 0.092241),
                  8: (1.12324, 0.218415), 16: (2.31822, 0.450141), 32: (4.9977, 0.954925),
                  64: (11.8052, 2.047031), 128: (26.0988, 4.346155), 256: (55.291, 9.980889)}


def bench_replication(args):
    import numpy as np
    import torch

    import pfgen
    from oracle import cim, polar
    from paper_1711_10579_amd import binding as B

    ctx = B.pf_ctx_create(0)
    k = max(3, min(args.steps, 10))

    def timed(h, opts, check):
        for _ in range(max(1, args.warmup)):
            r = B.pf_solve(h, opts)
            assert r.status == B.PF_CONVERGED, r.as_dict()
        torch.cuda.synchronize()
        lat, conv = [], 0
        for _ in range(k):
            s0 = time.perf_counter()
            r = B.pf_solve(h, opts)
            lat.append(time.perf_counter() - s0)
            conv += r.status == B.PF_CONVERGED
        return {"solve_ms": {"p50": 1000 * _pct(lat, 50), "min": 1000 * min(lat)}, "converged": conv,
                "solves": k, "newton_iters": r.iters, "inner_iters": r.linear_iters,
                "lu_fallback": r.lu_fallback, "final_mismatch_oracle": check(B.pf_get_voltage(h))}

    if args.feeder_copies:
        # only the listed feeders (LU), e.g. for a kernel trace of one size
        feeders = []
        for copies in [int(c) for c in args.feeder_copies.split(",")]:
            tol = pfgen.replication_feeder_tol(copies)
            lu = B.pf_default_options(solver=B.PF_SOLVER_LU, max_iter=20, tol=tol)
            fc = pfgen.replication_feeder(copies)
            h = B.pf_create_from(ctx, fc)
            row = {"copies": copies, "buses": fc.n_bus, "phase_nodes": fc.n, "tol": tol}
            row.update(timed(h, lu, lambda V, fc=fc: cim.mismatch_at(fc, V)))
            feeders.append(row)
            h.close()
        print(json.dumps({"mode": "replication", "metric": "solve time of the listed replicated feeders (LU)",
                          "value": feeders[-1]["solve_ms"]["p50"], "unit": "ms", "n_gpus": 1, "steps": k,
                          "warmup": args.warmup, "higher_is_better": False, "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "feeders": feeders}), flush=True)
        return

    grid = pfgen.replication_polar()
    t0 = time.perf_counter()
    h = B.pf_create_from(ctx, grid)
    setup = time.perf_counter() - t0
    rows = {"buses": grid.n, "branches": grid.m, "setup_s": setup}
    for name, solver, pc in (("lu", B.PF_SOLVER_LU, 0), ("gmres", B.PF_SOLVER_GMRES, B.PF_PRECOND_ILU0),
                             ("bicgstab", B.PF_SOLVER_BICGSTAB, B.PF_PRECOND_ILU0),
                             ("bicgstab_bjacobi", B.PF_SOLVER_BICGSTAB, B.PF_PRECOND_BJACOBI)):
        opts = B.pf_default_options(solver=solver, max_iter=40, precond=pc)
        rows[name] = timed(h, opts, lambda V: polar.mismatch_at(grid, V))
        print(f"replication 48k {name}: {rows[name]['solve_ms']['p50']:.2f} ms", file=sys.stderr, flush=True)
    h.close()
    rows["paper_nk_s"] = PAPER_NK_48K_S

    feeders = []
    for copies in pfgen.FEEDER_COPIES:
        tol = pfgen.replication_feeder_tol(copies)
        lu = B.pf_default_options(solver=B.PF_SOLVER_LU, max_iter=20, tol=tol)
        fc = pfgen.replication_feeder(copies)
        t0 = time.perf_counter()
        h = B.pf_create_from(ctx, fc)
        setup = time.perf_counter() - t0
        row = {"copies": copies, "buses": fc.n_bus, "phase_nodes": fc.n, "tol": tol, "setup_s": setup}
        row.update(timed(h, lu, lambda V, fc=fc: cim.mismatch_at(fc, V)))
        row["paper_solving_s"], row["paper_other_s"] = PAPER_TABLE1_S[copies]
        feeders.append(row)
        print(f"replication feeder {fc.n_bus}: {row['solve_ms']['p50']:.2f} ms", file=sys.stderr, flush=True)
        h.close()

    # the 2,000-bus feeder with generators (PV phase-nodes) and delta loads
    dg = pfgen.add_dg_and_delta(pfgen.config_case(2), 21, n_dg=6)
    h = B.pf_create_from(ctx, dg)
    dg_rows = {"buses": dg.n_bus, "phase_nodes": dg.n, "pv_nodes": int((dg.node_type == 2).sum()),
               "delta_loads": int((dg.delta_to >= 0).sum())}
    for name, solver in (("lu", B.PF_SOLVER_LU), ("bicgstab", B.PF_SOLVER_BICGSTAB)):
        dg_rows[name] = timed(h, B.pf_default_options(solver=solver, max_iter=40),
                              lambda V: cim.mismatch_at(dg, V))
    h.close()

    out = {"mode": "replication",
           "metric": "solve time of the replication-scale cases (48,000-bus grid, Newton-Krylov BiCGStab + "
                     "block-Jacobi)",
           "value": rows["bicgstab_bjacobi"]["solve_ms"]["p50"], "unit": "ms", "n_gpus": 1, "steps": k,
           "warmup": args.warmup, "higher_is_better": False, "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "replicated 30-bus blocks (48,000 buses) and replicated 906-bus feeders "
                                  "(1-256 copies), flat start to 1e-8 pu (1e-7 for 256 copies, whose FP64 rounding "
                                  "floor at the first bus is 2.2e-8), one solve at a time"},
           "grid48k": rows, "feeders": feeders, "feeder2000_dg_delta": dg_rows,
           "note": "paper times are CPU seconds on a Cori node (context, another machine)"}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            r = polar.newton(grid, max_iter=20)
            el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1000 * el, "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": f"one oracle Newton-Raphson solve (sparse LU) of the 48,000-bus grid, "
                                         f"{r.iters} iterations"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--breakdown", action="store_true",
                    help="time every kernel class in an extra untimed pass (stderr)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default schedule instead of the autotuned one")
    ap.add_argument("--schedule", default="",
                    help="fixed schedule 'dense_switch,min_dense,lane_scale,trsv_mode' (no autotuning)")
    ap.add_argument("--nk-steps", type=int, default=10,
                    help="solves of the Newton-Krylov (GMRES + ILU(0)) leg on the same grid")
    ap.add_argument("--batch", type=int, default=16,
                    help="scenarios of the batched form (seeded +-20%% load perturbations)")
    ap.add_argument("--workload", choices=["grid10k", "scenarios512", "served", "replication"],
                    default="grid10k")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--feeder-copies", default="",
                    help="replication: only the feeders of these copy counts (comma-separated), LU")
    ap.add_argument("--oracle-sample", type=int, default=8)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--pool-polar", type=int, default=32)
    ap.add_argument("--pool-feeder", type=int, default=16)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--max-bytes", type=int, default=2 << 30,
                    help="serving pool budget in bytes (0: no limit)")
    ap.add_argument("--no-targets", action="store_true",
                    help="default workload without the scenarios512 and served legs")
    ap.add_argument("--target-precision", choices=["fp64", "mixed"], default="mixed",
                    help="precision of the scenarios512 and served legs")
    ap.add_argument("--rate", type=float, default=0.0, help="arrivals/s (0: load factor x serial rate)")
    ap.add_argument("--load-factor", type=float, default=0.8)
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
    args.with_targets = not args.no_targets
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent power-flow instances shard across GPUs without collectives)",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
    elif args.workload == "grid10k":
        args.precision = args.precision or "fp64"
        bench_grid10k(args)
    elif args.workload == "scenarios512":
        args.target_precision = args.precision or args.target_precision
        bench_scenarios512(args)
    elif args.workload == "replication":
        bench_replication(args)
    else:
        args.target_precision = args.precision or args.target_precision
        bench_served(args)


if __name__ == "__main__":
    main()
