"""Benchmark of the stochastic multiscale flux basis hot path on one MI355X.

One step = the whole hot path over one batch: the flux basis of every
(Darcy subdomain, local KL realization) unit and of every Stokes subdomain,
the interface CG to rtol 1e-8 for every global collocation point, the
moment accumulation and the expansion of the moments to the fine fields.
`value` is global realizations per second of that step, inputs resident in
HBM; the rate with both bases resident (CG and moments only) is reported
beside it.

Both precisions run on identical inputs; `value` is the one named by
--precision.  Each precision block states the error of every field's mean
and variance against the FP64 path at CG rtol 1e-11 (which the GPU tests tie
to the oracle), and the number of realizations that did not converge (the
bench exits non-zero if any did).  One CG iteration in every 16th
convergence-check group is timed with HIP events on its stream while the
other CG lane is idle, so each kernel's duration is its own; the dominant
kernel's algorithmic flops (or bytes) per launch over its average launch
duration give `roofline`, priced with the per-realization-iteration counts
of the scope table (2 sum_i R_i^2 flops; 5 M 8 bytes for the whole CG).  A
second workload block (`cfg3`: uneven subdomains, 54,273 realizations) runs
one step per precision, and a `methods` block times Methods S1 and S2 in FP64
on samples of the same collocation points beside Method S3's step.  The CPU baseline (the oracle, one thread, bounded
sample) runs in a child process started before the GPU is touched.

Prints one JSON line.  --gpus above 1 is refused: the library runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # FP64 vector and FP64 MFMA, dense
PEAK_HBM = 8.0e12

METRIC = "collocation realizations/sec to CG rtol 1e-8 + basis builds/sec, FP64 vs mixed"


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work in the CPU sample")
    ap.add_argument("--single", action="store_true", help="time only --precision (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device copy first (scale reference for HBM counters)")
    ap.add_argument("--cg-chunk", type=int, default=0, help="realizations in flight in the CG (0: autotune)")
    ap.add_argument("--cg-lanes", type=int, default=0, choices=[0, 1, 2],
                    help="CG lanes (0: the library default, two lanes whose kernels overlap)")
    ap.add_argument("--no-cfg3", action="store_true", help="skip the uneven-layout block")
    ap.add_argument("--no-methods", action="store_true", help="skip the Methods S1/S2 block")
    ap.add_argument("--methods-sample", type=int, default=512,
                    help="collocation points of the Method S2 sample (S1: at most 32 of them)")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the rtol-1e-11 reference solve and the moment errors (profiling runs)")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    return ap.parse_args()


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands


_POOL_ORACLE = None


def _pool_basis(unit):
    """The Darcy flux basis of unit (i, k), in a pool worker (forked oracle)."""
    from oracle.darcy import DarcyLocal
    o = _POOL_ORACLE
    i, k = unit
    r = o.L.subs[i]["region"]
    DarcyLocal(o.L, i, o.darcy_K(i, o.grid.local_points(r)[k])).basis()
    return i


def _pool_realizations(budget_s):
    """Realization 0 through CG, recovery and moments until the budget is
    spent, in a pool worker; returns how many were done."""
    o = _POOL_ORACLE
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        o.realization_S3(0, rtol=1e-8)
        n += 1
    return n


def _pool_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def cpu_pool_baseline(o, l0, n_units, workers, budget_s):
    """The sample on a process pool over independent units (forked workers,
    one thread each): up to 8 (subdomain, local realization) bases per worker,
    then realization l0 repeated in every worker."""
    import multiprocessing as mp
    global _POOL_ORACLE
    _POOL_ORACLE = o
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_pool_init) as pool:
        units = [(i, k) for i in o.darcy_ids for k in range(o.grid.nlocal[o.L.subs[i]["region"]])]
        units = units[:8 * workers]
        t0 = time.perf_counter()
        pool.map(_pool_basis, units, chunksize=1)
        t_unit = (time.perf_counter() - t0) / len(units)
        t1 = time.perf_counter()
        counts = pool.map(_pool_realizations, [budget_s] * workers, chunksize=1)
        t_real = (time.perf_counter() - t1) / max(1, sum(counts))
    _POOL_ORACLE = None
    total = n_units * t_unit + o.grid.nreal * t_real
    return {"value": o.grid.nreal / total, "unit": "realizations/s", "cores": workers, "kind": "oracle",
            "sample": "%d Darcy flux bases spread over %d worker processes (%.4f s per basis of wall time), then "
                      "realization %d through CG rtol 1e-8 + recovery + moments %d times in %d workers (%.4f s each "
                      "of wall time), one thread per worker, extrapolated to %d units + %d realizations"
                      % (len(units), workers, t_unit, l0, sum(counts), workers, t_real, n_units, o.grid.nreal),
            "basis_builds_per_s": 1.0 / t_unit}


def cpu_baseline(prob, budget_s):
    """The oracle, untuned and single-threaded, on a bounded sample of the workload.

    Sample: the Darcy flux bases that one global realization needs (one per
    Darcy subdomain, at that realization's local indices), then that
    realization through CG rtol 1e-8, recovery and moment accumulation,
    repeated while the budget lasts.  Extrapolated to every (subdomain, local
    realization) unit and every global realization.  Oracle set-up and the
    Stokes basis are excluded, as in the GPU step; the set-up factorizes the
    Stokes subdomains in threads to keep the run short, the timed sample is
    single-threaded.  The same sample is then timed on a process pool over
    independent units (``pool``).
    """
    from threadpoolctl import threadpool_limits
    from oracle.darcy import DarcyLocal
    from oracle.methods import Oracle
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        o = Oracle(prob, threads=6, progress=lambda i: log("cpu baseline: oracle Stokes subdomain %d set up "
                                                           "(%.0f s)" % (i, time.perf_counter() - t0)))
        stokes = o.stokes_basis()
        t_setup = time.perf_counter() - t0
        log("cpu baseline: oracle set-up done (%.0f s)" % t_setup)
        L = o.L
        l0 = 0
        kl = o.grid.g2l[l0]
        table = {(i, 0): S for i, S in stokes.items()}
        t1 = time.perf_counter()
        for i in o.darcy_ids:
            r = L.subs[i]["region"]
            k = int(kl[r])
            table[(i, k)] = DarcyLocal(L, i, o.darcy_K(i, o.grid.local_points(r)[k])).basis()
        t_unit = (time.perf_counter() - t1) / len(o.darcy_ids)
        log("cpu baseline: %d Darcy bases, %.3f s each" % (len(o.darcy_ids), t_unit))
        o.s3_table = table
        w = float(o.grid.weights[l0])
        acc1, acc2 = {}, {}
        t2 = t_log = time.perf_counter()
        nr = 0
        while True:
            fields, _, _, _ = o.realization_S3(l0, rtol=1e-8)
            for key, v in fields.items():
                acc1[key] = acc1.get(key, 0.0) + w * v
                acc2[key] = acc2.get(key, 0.0) + w * v * v
            nr += 1
            now = time.perf_counter()
            if now - t_log > 5.0:
                log("cpu baseline: %d realizations of the sample done" % nr)
                t_log = now
            if now - t1 > budget_s:
                break
        t_real = (time.perf_counter() - t2) / nr
    n_units = sum(o.grid.nlocal[L.subs[i]["region"]] for i in o.darcy_ids)
    total = n_units * t_unit + o.grid.nreal * t_real
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    log("cpu baseline: process pool of %d workers" % workers)
    pool = cpu_pool_baseline(o, l0, n_units, workers, budget_s / 2)
    return {"value": o.grid.nreal / total, "unit": "realizations/s", "cores": 1, "kind": "oracle",
            "sample": "%d Darcy flux bases of realization %d (%.3f s each) and that realization through CG "
                      "rtol 1e-8 + recovery + moments %d times (%.3f s each), one thread, extrapolated to "
                      "%d units + %d realizations; oracle set-up and Stokes basis (%.0f s) excluded"
                      % (len(o.darcy_ids), l0, t_unit, nr, t_real, n_units, o.grid.nreal, t_setup),
            "basis_builds_per_s": 1.0 / t_unit, "pool": pool}


def start_cpu_baseline(args):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--workload", args.workload,
           "--cpu-budget", str(args.cpu_budget)]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, env=env, cwd=ROOT)


# ---------------------------------------------------------------------------
# GPU path

FIELD_NAMES = ("lambda", "darcy_p", "darcy_u", "stokes_u", "stokes_p")
PEAK_FP32_MFMA = 157.3e12
TIME_EVERY = 16   # one timed CG iteration per 16 check groups of the first lane


def gpu_step(ctx, prec, g, lam, st, rtol, torch):
    """One pass of the hot path; returns the number of realizations that did
    not converge."""
    ctx.build_flux_basis(prec)            # Darcy units and Stokes subdomains
    ctx.solve_interface(g, lam, rtol=rtol, status=st, allow_notconv=True)
    ctx.reset_moments()
    ctx.accumulate_moments(g, lam)
    ctx.finalize_moments()                # moments expanded to the fine fields
    torch.cuda.synchronize()
    return int((st != 0).sum().item())


COUNTER_KEYS = ("cg_iterations", "realizations", "cg_launches", "cg_timed_launches", "cg_timed_active", "cg_timed_columns",
                "ms_cg_apply", "ms_cg_update", "basis_solves_darcy", "units_built")


def time_path(ctx, prec, g, lam, st, rtol, steps, warmup, torch):
    for _ in range(warmup):
        gpu_step(ctx, prec, g, lam, st, rtol, torch)
    torch.cuda.synchronize()
    c0 = ctx.counters()
    ms = {"basis_darcy": [], "basis_stokes": [], "basis_build": [], "cg": [], "moments": [], "step": []}
    bad = 0
    for s in range(steps):
        t0 = time.perf_counter()
        bad += gpu_step(ctx, prec, g, lam, st, rtol, torch)
        ms["step"].append((time.perf_counter() - t0) * 1e3)
        c = ctx.counters()
        ms["basis_darcy"].append(c["ms_basis_darcy"])
        ms["basis_stokes"].append(c["ms_basis_stokes"])
        ms["basis_build"].append(c["ms_basis_build"])
        ms["cg"].append(c["ms_solve"])
        ms["moments"].append(c["ms_moments"])
        log("%s step %d: %.1f ms (basis build %.1f: Darcy %.2f beside Stokes %.1f; CG %.1f, moments %.2f)"
            % (prec, s, ms["step"][-1], ms["basis_build"][-1], ms["basis_darcy"][-1], ms["basis_stokes"][-1],
               ms["cg"][-1], ms["moments"][-1]))
    c1 = ctx.counters()
    d = {k: c1[k] - c0[k] for k in COUNTER_KEYS}
    return {k: sum(v) / steps for k, v in ms.items()}, d, bad


def field_moments(ctx):
    return {f: ctx.get_moments(f) for f in FIELD_NAMES}


def moment_errors(mom, ref):
    """Per field: largest error of the mean relative to the largest |mean|, and
    of the variance relative to the largest |variance|."""
    out = {}
    for f in FIELD_NAMES:
        m, v = mom[f]
        mr, vr = ref[f]
        sm = max(abs(mr).max(), 1e-300)
        sv = max(abs(vr).max(), 1e-12 * sm * sm)
        out[f] = {"mean": float(abs(m - mr).max() / sm), "var": float(abs(v - vr).max() / sv)}
    return out


REF_RTOL = 1e-11


def reference_moments(ctx, g, lam, st, torch):
    """The FP64 path at CG rtol 1e-11 (iteration limit 50 M) over the whole
    grid: three orders of magnitude below the timed solves' stopping error."""
    ctx.build_flux_basis("fp64")
    ctx.solve_interface(g, lam, rtol=REF_RTOL, max_iter=50 * ctx.sizes()["M"], status=st, allow_notconv=True)
    ctx.reset_moments()
    ctx.accumulate_moments(g, lam)
    ctx.finalize_moments()
    torch.cuda.synchronize()
    if int((st != 0).sum().item()):
        raise RuntimeError("the reference solve did not converge everywhere")
    return field_moments(ctx)


def kernel_source_hash(kernel):
    """Hash of one CG kernel's source: its definition through its launcher,
    and the argument struct it takes."""
    csrc = os.path.join(ROOT, "paper_1802_06263_amd", "csrc")
    with open(os.path.join(csrc, "kernels.hip")) as fh:
        src = fh.read()
    with open(os.path.join(csrc, "kernels.hpp")) as fh:
        hdr = fh.read()
    i0 = src.index("void %s(" % kernel)
    i1 = src.index("return hipGetLastError();", i0)
    j0 = hdr.index("struct CgArgs")
    j1 = hdr.index("};", j0)
    h = hashlib.sha256()
    h.update(src[i0:i1].encode())
    h.update(hdr[j0:j1].encode())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload):
    """HBM bytes per realization-iteration from the committed counter summary,
    or None when there is none or the kernel sources changed since it was
    taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash(kernel + "_kernel"):
        return None
    try:
        return float(vals["hbm_bytes_per_unit"])
    except (KeyError, ValueError):
        return None


def cg_whole(M, sum_R2, real_iters, ms_cg):
    """The whole CG of a step against both peaks, priced with the scope
    table's counts per realization-iteration: 5 M 8 bytes (the CG vectors
    streamed once) and 2 sum_i R_i^2 flops (the basis products), over the CG
    wall time.  The two lanes' kernels overlap on the device, so this is the
    step-level figure; the per-kernel entries time each kernel alone."""
    b = 5.0 * M * 8
    f = 2.0 * sum_R2
    t = ms_cg * 1e-3
    return {"realization_iterations": real_iters, "bytes_per_unit": b, "flops_per_unit": f,
            "gbps": b * real_iters / t / 1e9, "frac_hbm": b * real_iters / t / PEAK_HBM,
            "tflops": f * real_iters / t / 1e12, "frac_fp64_mfma": f * real_iters / t / PEAK_FP64}


def kernel_rooflines(sz, M, sum_R2, d, ms, prec, workload):
    """Per-kernel roofline entries.  The algorithmic unit of the CG kernels is
    one realization-iteration (one CG iteration of one realization still
    iterating); the library times two consecutive (product, update) launch
    pairs per timed check group, with the other lane idle, and counts the
    realizations active in them.  The product is priced by its 2 sum_i R_i^2
    flops (FP64 MFMA; 2 M 8 bytes of vectors, above the ridge), the update by
    the 6 M 8 bytes it streams per iteration on average (the operator result,
    p and r read, r and p written, and lambda read and written in every other
    iteration).  The basis builds are one unit per step."""
    out = {}
    nl = d["cg_timed_launches"]
    if nl:
        act = d["cg_timed_active"] / nl
        b_upd = 6.0 * M * 8
        avg = d["ms_cg_update"] * 1e-3 / nl
        out["cg_update"] = {"kernel": "cg_update2_kernel", "bound": "hbm", "achieved": b_upd * act / avg / 1e9,
                            "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": b_upd * act / avg / PEAK_HBM,
                            "avg_launch_us": avg * 1e6, "timed_launches": nl, "active_per_launch": act,
                            "bytes_per_unit": b_upd, "algorithmic_bytes_per_launch": b_upd * act,
                            "sampled_ms": d["ms_cg_update"]}
        t = read_traffic("cg_update2", workload)
        out["cg_update"]["traffic"] = t * act if t is not None else None
        f_app = 2.0 * sum_R2
        b_app = 2.0 * M * 8
        avg = d["ms_cg_apply"] * 1e-3 / nl
        out["cg_apply"] = {"kernel": "cg_apply_mfma_kernel", "bound": "mfma", "achieved": f_app * act / avg / 1e12,
                           "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": f_app * act / avg / PEAK_FP64,
                           "avg_launch_us": avg * 1e6, "timed_launches": nl, "active_per_launch": act,
                           "columns_per_launch": d["cg_timed_columns"] / nl, "flops_per_unit": f_app,
                           "bytes_per_unit": b_app, "gbps": b_app * act / avg / 1e9,
                           "frac_hbm": b_app * act / avg / PEAK_HBM, "sampled_ms": d["ms_cg_apply"]}
        t = read_traffic("cg_apply_mfma", workload)
        out["cg_apply"]["traffic"] = t * act if t is not None else None
    # Darcy basis build: banded factor + forward/backward flops of every unit;
    # the mixed path computes them on FP32 MFMA, the FP64 path on FP64 MFMA
    peak = PEAK_FP32_MFMA if prec == "mixed" else PEAK_FP64
    ach = sz["darcy_flops"] / (ms["basis_darcy"] * 1e-3)
    out["darcy_basis"] = {"kernel": "darcy_factor_kernel + darcy_inverse_kernel + darcy_solve_%s_kernel" % prec,
                          "bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                          "frac": ach / peak, "avg_launch_us": ms["basis_darcy"] * 1e3,
                          "algorithmic_flops_per_launch": sz["darcy_flops"], "traffic": None}
    return out


def run_workload(ctx, args, workload, precs, steps, warmup, chunk, torch, np):
    """Both precisions on one workload: timing, rooflines, moment errors."""
    sz = ctx.sizes()
    n, M = sz["n_real"], sz["M"]
    R = np.diff(ctx.index_map("sub_ptr"))
    sum_R2 = int((R.astype(np.int64) ** 2).sum())
    g = torch.arange(n, dtype=torch.int64, device="cuda")
    lam = torch.zeros((n, M), dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    if chunk > 0:
        ctx.set_option("cg_chunk", chunk)
    else:
        ctx.build_flux_basis("fp64")
        chunk = ctx.autotune(g, rtol=args.rtol)
        log("%s: autotuned CG slots: %d realizations in flight" % (workload, chunk))
    ctx.set_option("stokes_rebuild", 1)
    ctx.set_option("kernel_timing", TIME_EVERY)
    res, kern = {}, {}
    for prec in precs:
        ms, d, bad = time_path(ctx, prec, g, lam, st, args.rtol, steps, warmup, torch)
        kern[prec] = kernel_rooflines(sz, M, sum_R2, d, ms, prec, workload)
        mom = field_moments(ctx)
        dt = ms["step"] * 1e-3
        res[prec] = {"ms_per_step": ms["step"], "realizations_per_s": n / dt,
                     "realizations_per_s_basis_resident": n / (dt - 1e-3 * ms["basis_build"]),
                     "ms_basis_darcy": ms["basis_darcy"], "ms_basis_stokes": ms["basis_stokes"],
                     "ms_basis_build": ms["basis_build"], "ms_cg": ms["cg"],
                     "ms_moments_expand": ms["moments"],
                     "basis_builds_per_s": sz["n_units"] / (ms["basis_darcy"] * 1e-3),
                     "local_solves_per_s": d["basis_solves_darcy"] / (steps * ms["basis_darcy"] * 1e-3),
                     "darcy_local_solves_per_step": d["basis_solves_darcy"] / steps,
                     "cg_iterations_mean": d["cg_iterations"] / max(1, d["realizations"]),
                     "not_converged": bad,
                     "refinement_group_steps_per_unit": (ctx.counters()["refinement_steps"] / sz["n_units"]
                                                         if prec == "mixed" else 0.0),
                     "max_refine_residual": ctx.counters()["max_refine_residual"] if prec == "mixed" else 0.0,
                     "cg_launches_per_step": d["cg_launches"] / steps,
                     "cg_whole": cg_whole(M, sum_R2, d["cg_iterations"] / steps, ms["cg"]),
                     "basis_roofline": {k: kern[prec]["darcy_basis"][k] for k in ("bound", "achieved", "peak",
                                                                                  "unit", "frac")},
                     "_mom": mom}
    ref = None if args.no_reference else reference_moments(ctx, g, lam, st, torch)
    for prec in precs:
        mom = res[prec].pop("_mom")
        res[prec]["moment_error_vs_fp64_rtol_1e-11"] = None if ref is None else moment_errors(mom, ref)
    info = {"n_real": n, "M": M, "basis_units": sz["n_units"], "cg_chunk": chunk}
    return res, kern, info


def main():
    args = parse()
    if args.cpu_baseline_only:
        from workloads import problem
        print(json.dumps(cpu_baseline(problem(args.workload), args.cpu_budget)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    # the oracle child starts before this process touches the GPU
    child = None if args.no_cpu_baseline else start_cpu_baseline(args)
    import numpy as np
    import torch
    from paper_1802_06263_amd import sdmm
    from workloads import problem

    if args.copy_probe:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)   # an elementwise kernel: 256 MiB read, 256 MiB written
        torch.cuda.synchronize()
        del src, dst
    other = "fp64" if args.precision == "mixed" else "mixed"
    precs = (args.precision,) if args.single else (other, args.precision)
    ctx = sdmm.Context(0)
    ctx.set_problem(problem(args.workload))
    if args.cg_lanes:
        ctx.set_option("cg_lanes", args.cg_lanes)
    log("%s: %d realizations, M = %d, %d basis units" % (args.workload, ctx.sizes()["n_real"], ctx.sizes()["M"],
                                                         ctx.sizes()["n_units"]))
    res, kern, info = run_workload(ctx, args, args.workload, precs, args.steps, args.warmup, args.cg_chunk, torch,
                                   np)
    ctx.close()
    main_r = res[args.precision]
    kmain = kern[args.precision]
    # dominant kernel: largest estimated share of the step (the sampled CG
    # launches scaled to every launch of the step; a basis build is one launch)
    share = {"darcy_basis": kmain["darcy_basis"]["avg_launch_us"]}
    for k in ("cg_update", "cg_apply"):
        if k in kmain:
            share[k] = kmain[k]["avg_launch_us"] * main_r["cg_launches_per_step"]
    for k in share:
        kmain[k]["est_ms_per_step"] = share[k] * 1e-3
    dom = max(share, key=share.get)
    r = kmain[dom]
    roof = {"kernel": r["kernel"], "bound": r["bound"], "achieved": r["achieved"], "peak": r["peak"],
            "unit": r["unit"], "frac": r["frac"], "traffic": r["traffic"], "avg_launch_us": r["avg_launch_us"]}
    out = {"metric": METRIC, "value": main_r["realizations_per_s"], "unit": "realizations/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_r["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
           "config": {"workload": args.workload, **info, "precision": args.precision, "rtol": args.rtol,
                      "cg_lanes": args.cg_lanes or 2},
           "basis_builds_per_s": main_r["basis_builds_per_s"],
           "fp64": res.get("fp64"), "mixed": res.get("mixed"), "roofline": roof, "kernels": kmain}
    if not args.no_cfg3 and args.workload != "cfg3":
        ctx = sdmm.Context(0)
        ctx.set_problem(problem("cfg3"))
        log("cfg3: %d realizations, M = %d, %d basis units" % (ctx.sizes()["n_real"], ctx.sizes()["M"],
                                                               ctx.sizes()["n_units"]))
        r3, k3, i3 = run_workload(ctx, args, "cfg3", precs, 1, 1, CFG3_CHUNK, torch, np)
        ctx.close()
        out["cfg3"] = {"config": i3, "fp64": r3.get("fp64"), "mixed": r3.get("mixed"),
                       "kernels": k3[args.precision]}
    if not args.no_methods and "fp64" in res:
        out["methods"] = methods_block(args, res["fp64"], info["n_real"], torch, np)
    bad = sum(res[p]["not_converged"] for p in precs)
    if "methods" in out:
        bad += sum(out["methods"][m]["not_converged"] for m in ("S1", "S2"))
    if child is not None:
        log("waiting for the CPU baseline")
        so, _ = child.communicate()
        if child.returncode == 0 and so.strip():
            out["cpu_baseline"] = json.loads(so.decode().strip().splitlines()[-1])
        else:
            log("CPU baseline failed (exit %d)" % child.returncode)
            out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    if bad:
        log("%d realizations did not converge" % bad)
        sys.exit(1)


CFG3_CHUNK = 5120   # CG slots on the uneven layout (what the autotuner picks there)


def methods_block(args, s3, n_real, torch, np):
    """Methods S2 (Section 5.3: each realization's own Darcy basis) and S1
    (Section 5.2: local Darcy solves in every CG iteration) on the same
    workload in FP64, beside Method S3's whole step: realizations per second
    of CG + moment accumulation on a sample of collocation points spread over
    the grid (the Stokes part, which no realization changes, is built before
    the timed region, as Method S3's build is counted in its step), and the
    Darcy local solves per realization that eqs. (S1-cost)-(S3-cost) count."""
    from paper_1802_06263_amd import sdmm
    from workloads import problem
    out = {}
    # S1 solves every Darcy subdomain of every realization in each CG
    # iteration (about 3,000 of them), a few seconds per 10 realizations on
    # cfg2, so its sample is kept to 32 (rate 2.6/s at 16, 3.5/s at 128)
    for name, method, n in (("S2", "deterministic", args.methods_sample),
                            ("S1", "per_iteration", min(32, args.methods_sample))):
        ctx = sdmm.Context(0)
        ctx.set_problem(problem(args.workload))
        ctx.build_flux_basis("fp64", method=method)
        M = ctx.sizes()["M"]
        idx = np.unique(np.linspace(0, n_real - 1, n).astype(np.int64))
        n = int(idx.size)
        g = torch.tensor(idx, device="cuda")
        lam = torch.zeros((n, M), dtype=torch.float64, device="cuda")
        st = torch.zeros(n, dtype=torch.int32, device="cuda")
        w = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
        # warm-up: the batch's device layout, two CG iterations
        ctx.solve_interface(g, lam, rtol=args.rtol, max_iter=2, allow_notconv=True)
        c0 = ctx.counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.solve_interface(g, lam, rtol=args.rtol, status=st, allow_notconv=True)
        ctx.reset_moments()
        ctx.accumulate_moments(g, lam, w)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        c1 = ctx.counters()
        bad = int((st != 0).sum().item())
        out[name] = {"realizations": n, "ms": t * 1e3, "realizations_per_s": n / t,
                     "darcy_local_solves_per_realization": (c1["basis_solves_darcy"] - c0["basis_solves_darcy"]) / n,
                     "cg_iterations_mean": (c1["cg_iterations"] - c0["cg_iterations"]) / n, "not_converged": bad}
        log("Method %s: %d realizations in %.0f ms (%.1f realizations/s)" % (name, n, t * 1e3, n / t))
        ctx.close()
    out["S3"] = {"realizations": n_real, "ms": s3["ms_per_step"], "realizations_per_s": s3["realizations_per_s"],
                 "darcy_local_solves_per_realization": s3["darcy_local_solves_per_step"] / n_real,
                 "cg_iterations_mean": s3["cg_iterations_mean"], "not_converged": s3["not_converged"]}
    out["note"] = ("FP64; S1 and S2: CG + moments of the sample after the Stokes build; S3: the whole fp64 step "
                   "(Darcy and Stokes basis builds included)")
    return out


if __name__ == "__main__":
    main()
