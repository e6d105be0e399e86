"""Benchmark of the stochastic multiscale flux basis hot path on one MI355X.

One step = the whole hot path over one batch: the stochastic flux basis of
every (Darcy subdomain, local KL realization) unit, the interface CG to
rtol 1e-8 for every global collocation point, and the moment accumulation.
The Stokes basis (deterministic, one local realization) is built once before
the timed region and reported separately.

Prints one JSON line (see the keys below).  --gpus above 1 is refused: this
build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--single", action="store_true", help="time only --precision (profiling runs)")
    return ap.parse_args()


def gpu_step(ctx, prec, g, lam, rtol, torch):
    ctx.build_flux_basis(prec)
    ctx.solve_interface(g, lam, rtol=rtol, allow_notconv=True)
    ctx.accumulate_moments(g, lam)
    torch.cuda.synchronize()


def time_path(ctx, prec, g, lam, rtol, steps, warmup, torch):
    for _ in range(warmup):
        gpu_step(ctx, prec, g, lam, rtol, torch)
    ctx.reset_moments()
    torch.cuda.synchronize()
    basis_ms, solve_ms = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        gpu_step(ctx, prec, g, lam, rtol, torch)
        c = ctx.counters()
        basis_ms.append(c["ms_basis_darcy"])
        solve_ms.append(c["ms_solve"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, sum(basis_ms) / steps, sum(solve_ms) / steps


def cpu_baseline(prob, budget_s):
    """The oracle, untuned, on a bounded sample of the same workload."""
    import numpy as np
    from oracle.darcy import DarcyLocal
    from oracle.methods import Oracle
    t0 = time.perf_counter()
    o = Oracle(prob)
    o.stokes_basis()
    t_setup = time.perf_counter() - t0
    L = o.L
    # basis units: one local realization per Darcy subdomain, until the budget
    t1 = time.perf_counter()
    nu = 0
    for i in o.darcy_ids:
        r = L.subs[i]["region"]
        DarcyLocal(L, i, o.darcy_K(i, o.grid.local_points(r)[0])).basis()
        nu += 1
        if time.perf_counter() - t1 > 0.4 * budget_s:
            break
    t_unit = (time.perf_counter() - t1) / nu
    # realizations: S3 main loop (table from the units built above, reused)
    table = {}
    for i in o.darcy_ids:
        r = L.subs[i]["region"]
        table[(i, 0)] = None
    o.s3_table = {}
    for i in o.darcy_ids:
        r = L.subs[i]["region"]
        dl = DarcyLocal(L, i, o.darcy_K(i, o.grid.local_points(r)[0]))
        S = dl.basis()
        for k in range(o.grid.nlocal[r]):
            o.s3_table[(i, k)] = S
    for i, S in o.stokes_basis().items():
        o.s3_table[(i, 0)] = S
    t2 = time.perf_counter()
    nr = 0
    rng = np.random.default_rng(0)
    while True:
        o.realization_S3(int(rng.integers(0, o.grid.nreal)), rtol=1e-8)
        nr += 1
        if time.perf_counter() - t2 > 0.5 * budget_s:
            break
    t_real = (time.perf_counter() - t2) / nr
    n_units = sum(o.grid.nlocal[L.subs[i]["region"]] for i in o.darcy_ids)
    total = n_units * t_unit + o.grid.nreal * t_real
    return {"value": o.grid.nreal / total, "unit": "realizations/s", "cores": 1, "kind": "oracle",
            "sample": "%d Darcy flux bases (%.3f s each) and %d global realizations through CG rtol 1e-8 + "
                      "recovery (%.3f s each), extrapolated to %d units + %d realizations; Stokes basis "
                      "and setup (%.1f s) excluded" % (nu, t_unit, nr, t_real, n_units, o.grid.nreal, t_setup),
            "basis_builds_per_s": 1.0 / t_unit}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1802_06263_amd import sdmm
    from workloads import problem

    prob = problem(args.workload)
    ctx = sdmm.Context(0)
    ctx.set_problem(prob)
    sz = ctx.sizes()
    n, M = sz["n_real"], sz["M"]
    t0 = time.perf_counter()
    ctx.build_flux_basis("fp64")
    torch.cuda.synchronize()
    stokes_ms = ctx.counters()["ms_basis_stokes"]
    g = torch.arange(n, dtype=torch.int64, device="cuda")
    lam = torch.zeros((n, M), dtype=torch.float64, device="cuda")
    other = "fp64" if args.precision == "mixed" else "mixed"
    res = {}
    for prec in ((args.precision,) if args.single else (other, args.precision)):
        dt, bms, sms = time_path(ctx, prec, g, lam, args.rtol, args.steps, args.warmup, torch)
        c = ctx.counters()
        res[prec] = {"ms_per_step": dt * 1e3, "realizations_per_s": n / dt, "ms_basis": bms, "ms_cg": sms,
                     "basis_builds_per_s": sz["n_units"] / (bms * 1e-3),
                     "cg_iterations_mean": c["cg_iterations"] / max(1, c["realizations"])}
    main_r = res[args.precision]
    flops = sz["darcy_flops"]
    peak = PEAK_FP32 if args.precision == "mixed" else PEAK_FP64
    achieved = flops / (main_r["ms_basis"] * 1e-3)
    roof = {"kernel": "darcy_basis_%s" % args.precision, "bound": "mfma", "achieved": achieved / 1e12,
            "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None}
    out = {"metric": "collocation realizations/sec to CG rtol 1e-8 + basis builds/sec, FP64 vs mixed",
           "value": main_r["realizations_per_s"], "unit": "realizations/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_r["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
           "config": {"workload": args.workload, "n_real": n, "M": M, "basis_units": sz["n_units"],
                      "precision": args.precision, "rtol": args.rtol},
           "basis_builds_per_s": main_r["basis_builds_per_s"],
           "fp64": res.get("fp64"), "mixed": res.get("mixed"), "stokes_basis_ms": stokes_ms,
           "roofline": roof}
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
