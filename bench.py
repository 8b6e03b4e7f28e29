#!/usr/bin/env python3
"""Throughput of converged Newton power-flow solves on one MI355X.

A step is one complete power-flow solve (flat start to max-norm FP64 mismatch
<= 1e-8 pu) of the 10,000-bus meshed transmission grid (seeded synthetic;
tree + 3,000 uniform chords, 1,000 PV buses, balanced dispatch), with every
Newton phase on the GPU: mismatch, Jacobian fill, sparse refactorisation with
its dense trailing block, triangular solves and voltage update.  Inputs are
resident in device memory before the timed region.

Prints one JSON line (rank 0) with solves/s, latency percentiles, the
roofline figures of the dominant kernel (timed with HIP events inside the
timed region) and the CPU oracle timed on a bounded sample of the same work.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_gbs": 8000.0, "fp64_tflops": 78.6, "fp32_tflops": 157.3}
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--breakdown", action="store_true",
                    help="time every kernel class in an extra untimed pass (stderr)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=16,
                    help="scenarios of the batched form (seeded +-20%% load perturbations)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent power-flow instances shard across GPUs without collectives)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import pfgen
    from paper_1711_10579_amd import binding as B

    case = pfgen.config_case(1)
    ctx = B.pf_ctx_create(0)
    h = B.pf_create_from(ctx, case)
    info = B.pf_case_info_get(h)
    mixed = args.precision == "mixed"
    opts = B.pf_default_options(precision=int(mixed), max_iter=40 if mixed else 20)

    for _ in range(args.warmup):
        r = B.pf_solve(h, opts)
        assert r.status == B.PF_CONVERGED, r.as_dict()

    if args.breakdown:
        B.pf_profile_enable(ctx, -1)
        B.pf_profile_reset(ctx)
        for _ in range(3):
            B.pf_solve(h, opts)
        tot = 0.0
        rows = []
        for k, name in enumerate(B.KERNEL_CLASS_NAMES):
            s = B.pf_kernel_stats(ctx, k)
            tot += s["ms"]
            rows.append((name, s))
        for name, s in rows:
            if s["launches"]:
                print(f"[breakdown] {name:14s} launches/solve={s['launches'] / 3:8.1f} "
                      f"ms/solve={s['ms'] / 3:8.4f} ({100 * s['ms'] / tot:5.1f}%) "
                      f"GFLOP/s={s['flops'] / max(s['ms'], 1e-12) / 1e6:9.1f} "
                      f"GB/s={s['bytes'] / max(s['ms'], 1e-12) / 1e6:9.1f}", file=sys.stderr)
        B.pf_profile_enable(ctx, 0)

    # dominant kernel: the trailing-block update of the dense LU
    dom = B.PF_K_DENSE_UPDATE
    B.pf_profile_enable(ctx, 1 << dom)
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
    st = B.pf_kernel_stats(ctx, dom)
    B.pf_profile_enable(ctx, 0)

    V = B.pf_get_voltage(h)
    from oracle import polar

    mism = polar.mismatch_at(case, V)

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
        Vb = B.pf_get_voltage(hb[-1])
        batched = {"instances": args.batch, "value": bconv / bel, "unit": "solves/s",
                   "batch_latency_ms": {"p50": 1000 * _pct(blat, 50), "p99": 1000 * _pct(blat, 99)},
                   "steps": bsteps, "converged": bconv,
                   "final_mismatch_oracle": polar.mismatch_at(scen[-1], Vb)}
        for x in hb:
            x.close()

    avg_ms = st["ms"] / max(st["launches"], 1)
    flops_per_launch = st["flops"] / max(st["launches"], 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    peak = PEAK["fp32_tflops"] if mixed else PEAK["fp64_tflops"]
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "kernel": "k_dense_gemm (trailing update of the dense block LU)",
                "avg_launch_ms": avg_ms, "launches": st["launches"],
                "flops_per_launch": flops_per_launch}

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
                   "newton_iters": int(np.median(iters))},
        "latency_ms": {"p50": 1000 * _pct(lat, 50), "p99": 1000 * _pct(lat, 99)},
        "converged": conv,
        "final_mismatch_oracle": mism,
        "roofline": roofline,
        "batched": batched,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
