#!/usr/bin/env python3
"""Throughput of the two-level time-DD preconditioned KKT solve on one MI355X.

One step = FGMRES(30) solves, from x0 = 0 to a 1e-8 relative residual, of the grid128
workload at both of its regularisation parameters: 128x128 intervals (127^2 interior points),
nt = 256, T = 1, nu = 1, omega in {1e-2, 1e-4}, 16 time subdomains with overlap 2, constant +
linear coarse basis, seeded sine-mode target (12,387,072 KKT unknowns per problem).  The
right-hand sides are resident in HBM before the timed region.  `value` is the float64 path;
the float32-sweep path ("mixed": float32 sine-transform GEMMs and sweep state, float64 outer
FGMRES, matvec and coarse level) is timed the same way and reported beside it.

Prints one JSON line.  Extra objects:
  roofline      the kernel class with the largest share of the float64 solve time, its
                algorithmic bytes (or flops) over its launch durations, timed with HIP events
                on one extra step whose solves run one after another, against the MI355X
                peak; traffic from rocprofv3 counters when recorded
  cpu_baseline  the float64 CPU oracle timed on this host on a bounded sample of the same
                workload (the first FGMRES iterations), scaled to a whole solve
  hoisted       the same step with the transform-hoisted Schur block (sweeps as scalar
                recurrences per sine mode between one forward and one inverse batched
                transform), float64 and float32 transforms
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KKT space-time unknowns solved/s to 1e-8 rel. residual, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
WORKLOAD_SETS = {
    # the problems one step solves (one batch)
    "grid128": ("grid128", "grid128_w4"),
    "grid256": ("grid256",),
    "grid512": ("grid512",),
    "uneven64": "uneven64",
}
# restart length per workload: the Krylov basis of the largest ones must fit in HBM
DEFAULT_RESTART = {"grid512": 12, "uneven64": 12}
# reduced-precision paths timed per workload (the largest ones time a subset)
# ("auto": float32 sweeps per problem where kappa(D_sigma) <= 500, else float64)
DEFAULT_MIXED = {"grid512": ("fp32", "bf16x6"), "uneven64": ("auto",)}
DEFAULT_HOISTED = {"grid512": ("fp64", "fp32"), "uneven64": ("fp64", "auto")}


def workload_problems(key):
    """[(name, params, recipe)] of a workload set."""
    from paper_2305_04421_amd import workloads as wl
    if key == "uneven64":
        return [(f"uneven{i:02d}", params, recipe)
                for i, (params, recipe) in enumerate(wl.batch_uneven(64, seed=4))]
    return [(name,) + wl.config(name) for name in WORKLOAD_SETS[key]]
MIXED = ("fp32", "bf16x6", "bf16x3", "bf16")
DESCRIPTIONS = {
    "grid128": "grid128: 127x127 interior x nt=256, T=1, nu=1, omega {1e-2, 1e-4}, 16 time subdomains, "
               "overlap 2, constant+linear coarse basis",
    "grid256": "grid256: 255x255 interior x nt=1024, T=1, nu=0.1, omega 1e-3, 64 time subdomains, "
               "overlap 2, constant+linear coarse basis, target with 1e-3 noise",
    "grid512": "grid512: 511x511 interior x nt=2048, T=1, nu=1, omega 1e-4, 128 time subdomains, "
               "overlap 4, constant+linear coarse basis",
    "uneven64": "uneven64: 64 independent problems, n in {64,96,128,192,256}, nt = 16*U{4..32}, "
                "nu log-uniform [0.05,1], omega log-uniform [1e-4,1e-1], nt/16 time subdomains, overlap 2, "
                "constant+linear coarse basis",
}
# HBM bytes per dispatch from rocprofv3 FETCH_SIZE + WRITE_SIZE (FETCH_SIZE scaled by 2.0,
# WRITE_SIZE by 1.0: what a 1 GiB device copy reads on those counters), per workload and
# kernel class, as recorded in profiles/arnoldi_<workload>_fp64_hbm_counters.md for the
# current kernels.  A class whose kernels changed since the counters were taken, or a
# workload without counters, is absent (traffic null).
TRAFFIC = {"grid128": {"arnoldi": 496.85e6, "matvec": 215.83e6},
           "grid256": {"arnoldi": 8900.26e6, "matvec": 3687.70e6},
           "grid512": {"arnoldi": 34507.54e6, "matvec": 31325.91e6}}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--restart", type=int, default=None,
                    help="FGMRES restart length (default 30; 12 for grid512 and uneven64)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--cpu-iters", type=int, default=4,
                    help="FGMRES iterations of the CPU oracle sample (0: skip the CPU baseline)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the float32-sweep path")
    ap.add_argument("--no-hoisted", action="store_true", help="skip the transform-hoisted (modal) paths")
    ap.add_argument("--sequential", action="store_true",
                    help="solve the problems of a step one after another instead of as one batch")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device once (a known-size kernel for HBM counters)")
    ap.add_argument("--roofline-class", default=None,
                    choices=["matvec", "sweep_rows", "sweep_cols", "coarse", "arnoldi", "other"],
                    help="kernel class of the roofline object (default: the one with the most time)")
    ap.add_argument("--workload", default="grid128", choices=sorted(WORKLOAD_SETS),
                    help="problem set of one step (default: grid128 at omega 1e-2 and 1e-4)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver has no "
              "multi-GPU path.", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    from paper_2305_04421_amd import KKTSolver, solve_batched, workloads as wl

    torch.cuda.init()
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.restart is None:
        args.restart = DEFAULT_RESTART.get(args.workload, 30)
    probs = []
    recipes = {}
    for name, params, recipe in workload_problems(args.workload):
        u0, ut = wl.data(params, recipe)
        recipes[name] = recipe
        probs.append((name, params, torch.from_numpy(u0.reshape(-1)).to(dev), torch.from_numpy(ut.reshape(-1)).to(dev)))
        del u0, ut
    unknowns = [3 * p["nt"] * (p["nx"] - 1) * (p["ny"] - 1) for _, p, _, _ in probs]

    def run_path(precision, steps, warmup, profile, sweep="step", must_converge=True, keep_x=False):
        solvers = [KKTSolver(p, precision, sweep=sweep) for _, p, _, _ in probs]
        fs = [S.rhs(u0, ut) for S, (_, _, u0, ut) in zip(solvers, probs)]
        xs = [torch.zeros_like(f) for f in fs]
        stats = []

        def step():
            for x in xs:
                x.zero_()
            if args.sequential:
                out = [S.solve(f, x=x, restart=args.restart, maxit=600, rtol=args.rtol)[1]
                       for S, f, x in zip(solvers, fs, xs)]
            else:
                _, out = solve_batched(solvers, fs, xs, restart=args.restart, maxit=600, rtol=args.rtol)
            for (name, _, _, _), st in zip(probs, out):
                if st["status"] != 0 and must_converge:
                    raise RuntimeError(f"{precision} solve of {name} did not converge: {st}")
            return out

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            stats = step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = None
        if profile:
            # Kernel timer: the same step once more, its solves one after another, with HIP
            # events around every launch (concurrent solves would charge each kernel with
            # the time it shares the GPU with the other problem's kernels).
            for S in solvers:
                S.profile(True)
            for S, f, x in zip(solvers, fs, xs):
                x.zero_()
                S.solve(f, x=x, restart=args.restart, maxit=600, rtol=args.rtol)
            prof = {}
            for S in solvers:
                for k, v in S.profile_read().items():
                    acc = prof.setdefault(k, dict(ms=0.0, launches=0, bytes=0.0, flops=0.0))
                    for kk in acc:
                        acc[kk] += v[kk]
                S.profile(False)
        for S in solvers:
            S.close()
        return dt, stats, prof, (xs if keep_x else None)

    # float64 path; its solutions (host copies) are the reference of the other paths' errors
    others = not (args.no_mixed and args.no_hoisted)
    dt64, st64, prof64, xs64 = run_path("fp64", args.steps, args.warmup, profile=True, keep_x=others)
    x64 = [x.cpu() for x in xs64] if others else None
    del xs64
    value64 = args.steps * sum(unknowns) / dt64
    result = {
        "metric": METRIC, "value": value64, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt64 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[args.workload] + ", FGMRES(%d) to %g from x0=0, %s" % (
                                   args.restart, args.rtol,
                                   "solved one after another" if args.sequential else "solved as one batch"),
                   "unknowns_per_step": sum(unknowns), "problems": [name for name, _, _, _ in probs]},
        "iterations": {name: st["iters"] for (name, _, _, _), st in zip(probs, st64)},
        "reorthogonalised_steps": {name: st["reorth"] for (name, _, _, _), st in zip(probs, st64)},
        "batched": not args.sequential,
        "relres_true": {name: st["relres_true"] for (name, _, _, _), st in zip(probs, st64)},
        # ||f_b - (K x)_b|| / ||f_b|| per block (u, z, w; 0 where f_b = 0)
        "relres_block": {name: st["relres_block"] for (name, _, _, _), st in zip(probs, st64)},
    }

    # roofline of the dominant kernel class (or the one asked for)
    def class_roof(cls):
        d = prof64[cls]
        if cls in ("sweep_rows", "sweep_cols"):
            achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12 if d["ms"] else 0.0
            r = {"bound": "mfma", "achieved": achieved, "peak": MFMA_PEAK_TFLOPS["fp64"], "unit": "TFLOP/s"}
        else:
            achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] else 0.0
            r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        r["frac"] = r["achieved"] / r["peak"]
        return r

    dom = args.roofline_class or max(prof64, key=lambda k: prof64[k]["ms"])
    d = prof64[dom]
    total_ms = sum(v["ms"] for v in prof64.values())
    roof = class_roof(dom)
    roof["traffic"] = TRAFFIC.get(args.workload, {}).get(dom)
    roof["kernel_class"] = dom
    roof["launches"] = d["launches"]
    roof["avg_launch_us"] = 1e3 * d["ms"] / max(d["launches"], 1)
    roof["algorithmic_bytes_per_launch"] = d["bytes"] / max(d["launches"], 1)
    roof["algorithmic_flops_per_launch"] = d["flops"] / max(d["launches"], 1)
    roof["share_of_kernel_time"] = d["ms"] / total_ms if total_ms else None
    roof["classes_ms_per_step"] = {k: v["ms"] for k, v in prof64.items()}
    roof["classes"] = {}
    for k, v in prof64.items():
        if v["launches"]:
            r = class_roof(k)
            roof["classes"][k] = {"launches": v["launches"], "avg_launch_us": 1e3 * v["ms"] / v["launches"],
                                  "achieved": r["achieved"], "unit": r["unit"], "frac": r["frac"]}
    roof["timed_on"] = "one extra step, its solves run one after another, HIP events around every launch"
    result["roofline"] = roof

    def err_vs_fp64(xs):
        # relative 2-norm distance of each solution from the float64 per-step path's
        out = {}
        for (name, _, _, _), x, ref in zip(probs, xs, x64):
            r = ref.to(dev)
            out[name] = float((x - r).norm() / r.norm())
            del r
        return out

    def summary(prec, sweep):
        dt, st, _, xs = run_path(prec, args.steps, args.warmup, profile=False, sweep=sweep,
                                 must_converge=False, keep_x=True)
        err = err_vs_fp64(xs)
        del xs
        failed = [name for (name, _, _, _), x in zip(probs, st) if x["status"] != 0]
        if failed:
            return {"value": None, "not_converged": failed, "ms_per_step": 1e3 * dt / args.steps,
                    "iterations": {name: x["iters"] for (name, _, _, _), x in zip(probs, st)},
                    "err_vs_fp64": err}
        v = args.steps * sum(unknowns) / dt
        return {"value": v, "ms_per_step": 1e3 * dt / args.steps, "ratio_vs_fp64": v / value64,
                "iterations": {name: x["iters"] for (name, _, _, _), x in zip(probs, st)},
                "relres_true": {name: x["relres_true"] for (name, _, _, _), x in zip(probs, st)},
                "err_vs_fp64": err}

    if not args.no_mixed:
        # reduced-precision sweeps and sine-transform GEMMs; FGMRES, matvec and coarse level
        # stay float64 (FGMRES acting as iterative refinement)
        result["mixed"] = {prec: summary(prec, "step") for prec in DEFAULT_MIXED.get(args.workload, MIXED)}

    if not args.no_hoisted:
        # transform-hoisted Schur block (sine-mode sweeps), measured beside the per-step path
        result["hoisted"] = {prec: summary(prec, "modal")
                             for prec in DEFAULT_HOISTED.get(args.workload, ("fp64",) + MIXED)}

    if args.cpu_iters > 0:
        result["cpu_baseline"] = cpu_baseline(args, probs[0][0], probs[0][1], recipes[probs[0][0]],
                                              st64[0]["iters"])

    print(json.dumps(result), flush=True)
    return 0


# Above this many KKT unknowns the CPU sample is a time-truncated copy of the problem.
CPU_FULL_LIMIT = 50_000_000


def cpu_baseline(args, name, params, recipe, iters_full):
    """The CPU oracle on a bounded sample: its first `cpu_iters` FGMRES iterations of the
    step's first problem, scaled to the iteration count of the full solve.  Problems above
    CPU_FULL_LIMIT unknowns are sampled on their first 64 time steps (same grid, time step,
    steps per subdomain and overlap) and scaled per unknown-iteration."""
    import numpy as np
    from oracle.problem import Problem
    from oracle import operators as op, precond as pc, gmres as gm
    from paper_2305_04421_amd import workloads as wl
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = None
    full = Problem(**params).validate()
    sample_params = dict(params)
    truncated = full.size > CPU_FULL_LIMIT
    if truncated:
        k = params["nt"] // params["n_sub"]
        nt = 64
        sample_params.update(nt=nt, T=params["T"] * nt / params["nt"], n_sub=nt // k)
    p = Problem(**sample_params).validate()
    u0, ut = wl.data(sample_params, recipe)
    f = op.rhs(p, u0, ut)
    t0 = time.perf_counter()
    res = gm.gmres(lambda v: op.apply_K(p, v), lambda v: pc.apply_Pinv(p, v), f,
                   restart=args.restart, maxit=args.cpu_iters, rtol=args.rtol)
    dt = time.perf_counter() - t0
    per_iter = dt / max(res.iterations, 1)
    what = (f"the first {p.nt} time steps ({p.n_sub} subdomains) of the {name} problem"
            if truncated else f"the {name} solve")
    return {"value": p.size / (per_iter * iters_full), "unit": "unknowns/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {res.iterations} FGMRES({args.restart}) iterations of {what} "
                      f"({dt:.1f} s incl. the initial residual), scaled to the {iters_full} "
                      f"iterations of the full solve"
                      + (" and per unknown-iteration to the full problem" if truncated else "")
                      + f"; numpy float64 with {threads} BLAS threads"}


if __name__ == "__main__":
    sys.exit(main())
