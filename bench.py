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

Other modes (each prints its own JSON line):
  --workload scenarios512   512 grids of 100-5,000 buses, FP32 inner solves,
                            one pf_solve_batch per step
  --workload served         Poisson-arriving requests on a pool of single- and
                            three-phase grids through pf_submit/pf_poll
  --workload replication    the paper's replication-scale cases (Sec. IV):
                            the 48,000-bus grid (LU, GMRES, BiCGStab) and the
                            0.9K-230K-bus feeders of Table 1 (LU), solve
                            times beside the paper's CPU times (context)
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


def cpu_baseline(case, budget_s=20.0):
    """The CPU oracle as it stands, single-threaded, on whole solves of the
    same grid until the time budget is spent (at least one)."""
    from threadpoolctl import threadpool_limits

    from oracle import polar

    done, t0 = 0, time.perf_counter()
    with threadpool_limits(limits=1):
        while True:
            r = polar.newton(case, tol=1e-8)
            assert r.status == 0
            done += 1
            if time.perf_counter() - t0 >= budget_s or done >= 5:
                break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} full solves of the 10,000-bus grid (tol 1e-8), "
                      f"{el:.1f} s, FP64 NumPy/SciPy SuperLU, 1 thread"}


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


def _roof(st, bound, peak, unit, kernel):
    n = max(st["launches"], 1)
    avg_ms = st["ms"] / n
    if bound == "hbm":
        per = st["bytes"] / n
        achieved = per / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    else:
        per = st["flops"] / n
        achieved = per / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": None, "kernel": kernel,
            "avg_launch_ms": avg_ms, "launches": st["launches"],
            ("bytes_per_launch" if bound == "hbm" else "flops_per_launch"): per}


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
    # the replayed Newton-step graph with the kernels)
    dom = B.PF_K_DENSE_PANEL
    # one event pair around each Newton step's run of block-step launches
    # (its time includes the short gaps between them inside the graph)
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
    mism = polar.mismatch_at(case, B.pf_get_voltage(h))

    # Newton-Krylov on the same grid, right-preconditioned with block ILU(0),
    # forcing term min(0.1, ||F||_inf): GMRES(30), then BiCGStab (the method
    # the paper tested)
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
        return {"value": nconv / nel, "unit": "solves/s", "steps": args.nk_steps, "converged": nconv,
                "latency_ms": {"p50": 1000 * _pct(nlat, 50), "p99": 1000 * _pct(nlat, 99)},
                "solver": label + ("+ilu0" if precond == B.PF_PRECOND_ILU0 else "+block-jacobi"),
                "newton_iters": int(np.median(nit)),
                "inner_iters_per_solve": int(np.median(nlin)),
                "final_mismatch_oracle": polar.mismatch_at(case, B.pf_get_voltage(h))}

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
        batched = {"instances": args.batch, "value": bconv / bel, "unit": "solves/s",
                   "batch_latency_ms": {"p50": 1000 * _pct(blat, 50), "p99": 1000 * _pct(blat, 99)},
                   "steps": bsteps, "converged": bconv,
                   "final_mismatch_oracle": polar.mismatch_at(scen[-1], B.pf_get_voltage(hb[-1]))}
        for x in hb:
            x.close()

    valu_peak = PEAK["fp32_valu_tflops"] if mixed else PEAK["fp64_tflops"]
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
        "roofline": _with_hbm(dict(_roof(st_dom, "mfma", mfma_peak, "TFLOP/s",
                                         "k_dense_step (block step k of the dense block: diagonal-block inverse "
                                         "by block Gauss-Jordan, row tiles times it, and the matrix-core trailing "
                                         "update)"),
                                   traffic=None if mixed else _measured_traffic("k_dense_step", sched),
                                   timing="HIP events on the library stream around each Newton step's run of "
                                          "k_dense_step launches inside the replayed graph; per launch = span / "
                                          "launches (includes the gaps between them)")),
        "batched": batched,
        "newton_krylov": nk,
        "newton_krylov_bicgstab": nk_bcg,
        "newton_krylov_bicgstab_bjacobi": nk_bcg_bj,
        "autotune": tuned,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


def bench_scenarios512(args):
    import numpy as np
    import torch

    import pfgen
    from oracle import polar
    from paper_1711_10579_amd import binding as B

    t0 = time.perf_counter()
    scen = pfgen.c3_scenarios(args.instances)
    t_gen = time.perf_counter() - t0
    ctx = B.pf_ctx_create(0)
    t0 = time.perf_counter()
    hs = [B.pf_create_from(ctx, c) for c in scen]
    t_setup = time.perf_counter() - t0
    mixed = args.precision != "fp64"
    opts = B.pf_default_options(precision=int(mixed), max_iter=40 if mixed else 20)
    B.pf_solve_batch(ctx, hs, opts)
    torch.cuda.synchronize()
    conv, steps = 0, max(1, args.steps // 10)
    t0 = time.perf_counter()
    for _ in range(steps):
        rs = B.pf_solve_batch(ctx, hs, opts)
        conv += sum(r.status == B.PF_CONVERGED for r in rs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # FP64-oracle error on a sample of scenarios (the oracle's own roots)
    rng = np.random.default_rng(1)
    sample = sorted(rng.choice(len(scen), size=min(args.oracle_sample, len(scen)), replace=False))
    errs = []
    for i in sample:
        V = B.pf_get_voltage(hs[i])
        ref = polar.newton(scen[i])
        errs.append(float(max(np.max(np.abs(np.abs(V) - ref.vm)), np.max(np.abs(np.angle(V) - ref.va)))))
    out = {"mode": "scenarios512", "metric": METRIC, "value": conv / el, "unit": "solves/s",
           "instances": len(scen), "steps": steps, "converged": conv,
           "sum_buses": int(sum(c.n for c in scen)), "ms_per_batch": 1000 * el / steps,
           "precision": args.precision, "setup_s": t_setup, "generate_s": t_gen,
           "iters": {"p50": float(np.median([r.iters for r in rs])), "max": int(max(r.iters for r in rs))},
           "oracle_err_max": max(errs), "oracle_sample": len(sample),
           "final_mismatch_max": float(max(r.mismatch_inf for r in rs))}
    print(json.dumps(out), flush=True)


def bench_served(args):
    import numpy as np

    import pfgen
    from paper_1711_10579_amd import binding as B

    pool = pfgen.c4_pool(n_polar=args.pool_polar, n_feeder=args.pool_feeder)
    ctx = B.pf_ctx_create(0)
    reps = 2
    t0 = time.perf_counter()
    cases = [[B.pf_create_from(ctx, g) for _ in range(reps)] for g in pool]
    setup_s = time.perf_counter() - t0
    mixed = args.precision != "fp64"
    opts = B.pf_default_options(precision=int(mixed), max_iter=40 if mixed else 20)
    plain = B.pf_default_options(precision=0, max_iter=20)
    rng = random.Random(11)
    n_req = args.requests
    # request stream: 70 % single-phase, 30 % feeders, fresh perturbation each
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

    for row in cases:  # warm every case once (device code, cached launch plans)
        B.pf_solve(row[0], plain)
    # the plain FP64 one-at-a-time GPU Newton over the same requests: service
    # times (host clock around each pf_solve, injections included)
    service, serial_conv = [], 0
    for (g, _), p in zip(reqs, pert):
        h = cases[g][0]
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

    B.pf_serve_config(ctx, max_bytes=args.max_bytes, max_slots=args.slots)

    def run(arr):
        free = {g: list(range(reps)) for g in range(len(pool))}
        inflight = {}
        lat, conv, done_n = [], 0, 0
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
                    free[g].append(r_)
                    lat.append(time.perf_counter() - start - arr[k])
                    conv += res.status == B.PF_CONVERGED
                    done_n += 1
            time.sleep(0.0002)
        return conv, time.perf_counter() - start, lat

    conv, el, lat = run(arrivals)
    # saturation: every request arrives at once (replicas still bound a grid's
    # concurrency)
    sconv, sel, _ = run([0.0] * n_req)
    out = {"mode": "served", "metric": METRIC, "value": conv / el, "unit": "solves/s",
           "requests": n_req, "converged": conv, "arrival_rate_per_s": lam,
           "latency_ms": {"p50": 1000 * _pct(lat, 50), "p99": 1000 * _pct(lat, 99)},
           "saturation": {"value": sconv / sel, "converged": sconv},
           "plain_fp64_serial": {"value": serial_rate, "converged": serial_conv,
                                 "service_ms": {"p50": 1000 * _pct(service, 50), "p99": 1000 * _pct(service, 99)},
                                 "queued_latency_ms_same_arrivals": {"p50": 1000 * _pct(q_lat, 50),
                                                                     "p99": 1000 * _pct(q_lat, 99)}},
           "pool": {"single_phase": args.pool_polar, "feeders": args.pool_feeder, "replicas": reps,
                    "setup_s": setup_s},
           "slots": args.slots, "precision": args.precision}
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
    ap.add_argument("--oracle-sample", type=int, default=8)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--pool-polar", type=int, default=32)
    ap.add_argument("--pool-feeder", type=int, default=16)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--max-bytes", type=int, default=0)
    ap.add_argument("--rate", type=float, default=0.0, help="arrivals/s (0: load factor x serial rate)")
    ap.add_argument("--load-factor", type=float, default=0.8)
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
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
        args.precision = args.precision or "mixed"
        bench_scenarios512(args)
    elif args.workload == "replication":
        bench_replication(args)
    else:
        args.precision = args.precision or "mixed"
        bench_served(args)


if __name__ == "__main__":
    main()
