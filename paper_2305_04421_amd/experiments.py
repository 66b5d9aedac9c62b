"""The numerical experiments of Sec. 4 run on the HIP solver: iteration counts of the one-level
(RASQ, Eq. 13) and two-level (Eq. 15) preconditioners on the paper's closed-form problem.

    python -m paper_2305_04421_amd.experiments weak  [--mesh 17] [--sweep step|modal] [--out F]
    python -m paper_2305_04421_amd.experiments omega [--nt 800]
    python -m paper_2305_04421_amd.experiments mesh
    python -m paper_2305_04421_amd.experiments ablation

Studies (each one solve per row; GMRES unrestarted, right-preconditioned, stopped at a
relative residual of 1e-6 or after 420 iterations, as in Sec. 4):
  weak   Fig. 1: N_t in {100, ..., 3200}, 80 / 20 / 5 time steps per subdomain, omega in
         {1e-2, 1e-3, 1e-4}, one- and two-level.  N_t values not divisible by the steps per
         subdomain are skipped, so the 80-step series starts at N_t = 400.
  omega  Fig. 2: omega over five orders of magnitude (1e-1 ... 1e-5) at a fixed N_t.
  mesh   the mesh-size remark of Sec. 4: 9, 17 and 33 mesh points per direction.
  ablation  variants of the preconditioner against the paper's choices, on the float64
         modal path: symmetric overlap, additive Schwarz, the exact local inverse of Eq. (9),
         fine-first and additive two-level combinations, the constant-only coarse space,
         and overlap 0 / 2, over N_t at 20 and 5 steps per subdomain.

Each row is printed as one JSON object; --out also writes the rows as a markdown table.
"""

import argparse
import json
import sys

from . import workloads as wl

NT_SERIES = (100, 200, 400, 800, 1600, 3200)
STEPS_PER_SUB = (80, 20, 5)
OMEGAS_WEAK = (1e-2, 1e-3, 1e-4)
OMEGAS_ROBUST = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5)
MESHES = (9, 17, 33)
RTOL = 1e-6
MAXIT = 420


def weak_cases(n_points=17, nt_series=NT_SERIES, steps=STEPS_PER_SUB, omegas=OMEGAS_WEAK):
    for k in steps:
        for omega in omegas:
            for nt in nt_series:
                if nt % k or nt // k < 1:
                    continue
                for coarse in (0, 2):
                    yield dict(study="weak", nt=nt, steps_per_sub=k, omega=omega, coarse=coarse,
                               mesh=n_points)


def omega_cases(nt=800, n_points=17, steps=STEPS_PER_SUB, omegas=OMEGAS_ROBUST):
    for k in steps:
        for omega in omegas:
            for coarse in (0, 2):
                yield dict(study="omega", nt=nt, steps_per_sub=k, omega=omega, coarse=coarse,
                           mesh=n_points)


def mesh_cases(nt=800, steps=20, omegas=OMEGAS_WEAK, meshes=MESHES):
    for n_points in meshes:
        for omega in omegas:
            for coarse in (0, 2):
                yield dict(study="mesh", nt=nt, steps_per_sub=steps, omega=omega, coarse=coarse,
                           mesh=n_points)


# name -> parameter changes against the paper's method (overlap 1 to the left, RAS, RASQ
# local solves, coarse first, constant + linear coarse basis)
ABLATIONS = {
    "paper": {},
    "one-level": dict(coarse=0),
    "constant coarse": dict(coarse=1),
    "overlap 0": dict(overlap=0),
    "overlap 2": dict(overlap=2),
    "overlap both sides": dict(overlap_side="both"),
    "ASM": dict(schwarz="asm"),
    "exact local (Eq. 9)": dict(local="exact"),
    "fine first": dict(combine="fine_first"),
    "additive": dict(combine="additive"),
    "one-level ASM": dict(coarse=0, schwarz="asm"),
    "one-level exact local": dict(coarse=0, local="exact"),
}


def ablation_cases(n_points=17, nt_series=(100, 200, 400, 800, 1600), steps=(20, 5),
                   omegas=(1e-2, 1e-4)):
    for k in steps:
        for omega in omegas:
            for name in ABLATIONS:
                for nt in nt_series:
                    yield dict(study="ablation", variant=name, nt=nt, steps_per_sub=k, omega=omega,
                               coarse=ABLATIONS[name].get("coarse", 2), mesh=n_points)


def run_case(case, sweep="step", precision="fp64", rtol=RTOL, maxit=MAXIT):
    """One unrestarted GMRES solve of the Sec. 4 problem on the device; returns the row."""
    import torch
    from . import KKTSolver
    params = wl.paper_problem(case["nt"], case["steps_per_sub"], case["omega"],
                              coarse=case["coarse"], overlap=1, n_points=case["mesh"])
    if "variant" in case:
        params.update(ABLATIONS[case["variant"]])
        sweep, precision = "modal", "fp64"   # the variants run on the float64 modal path
    u0, ut = wl.paper_data(params)
    with KKTSolver(params, precision, sweep=sweep) as S:
        f = S.rhs(torch.from_numpy(u0.reshape(-1)).cuda(), torch.from_numpy(ut.reshape(-1)).cuda())
        _, st = S.solve(f, restart=maxit, maxit=maxit, rtol=rtol)
    row = dict(case)
    row.update(n_sub=params["n_sub"], iters=st["iters"], converged=st["status"] == 0,
               relres_true=st["relres_true"], solve_s=st["solve_s"], sweep=sweep,
               precision=precision)
    return row


def markdown(rows):
    """Rows grouped as the paper's figures: one line per (study, mesh, k, omega, level)."""
    out = []
    keyed = {}
    ablation = [r for r in rows if r["study"] == "ablation"]
    rows = [r for r in rows if r["study"] != "ablation"]
    if ablation:
        out.append(ablation_table(ablation))
    for r in rows:
        key = (r["study"], r["mesh"], r["steps_per_sub"], r["omega"], r["coarse"])
        keyed.setdefault(key, []).append(r)
    by_study = {}
    for key, rs in keyed.items():
        by_study.setdefault(key[0], []).append((key, rs))
    for study, groups in by_study.items():
        xs = sorted({(r["nt"], r["omega"], r["mesh"]) for _, rs in groups for r in rs})
        if study == "weak":
            out.append("| mesh | steps/sub | omega | level | " +
                       " | ".join(f"N_t={nt}" for nt in sorted({x[0] for x in xs})) + " |")
            cols = sorted({x[0] for x in xs})
            colkey = "nt"
        elif study == "omega":
            cols = sorted({x[1] for x in xs}, reverse=True)
            out.append("| mesh | steps/sub | N_t | level | " +
                       " | ".join(f"omega={w:g}" for w in cols) + " |")
            colkey = "omega"
        else:
            cols = sorted({x[2] for x in xs})
            out.append("| N_t | steps/sub | omega | level | " +
                       " | ".join(f"{m}x{m} points" for m in cols) + " |")
            colkey = "mesh"
        out.append("|" + "---|" * (4 + len(cols)))
        if study == "omega":
            merged = {}
            for (st, mesh, k, omega, coarse), rs in groups:
                merged.setdefault((mesh, k, coarse), []).extend(rs)
            items = sorted(merged.items(), key=lambda kv: (kv[0][0], -kv[0][1], kv[0][2]))
            for (mesh, k, coarse), rs in items:
                cells = _cells(rs, cols, colkey)
                out.append(f"| {mesh} | {k} | {rs[0]['nt']} | {_level(coarse)} | " + " | ".join(cells) + " |")
        elif study == "mesh":
            merged = {}
            for (st, mesh, k, omega, coarse), rs in groups:
                merged.setdefault((k, omega, coarse), []).extend(rs)
            for (k, omega, coarse), rs in sorted(merged.items(), key=lambda kv: (-kv[0][1], kv[0][2])):
                cells = _cells(rs, cols, colkey)
                out.append(f"| {rs[0]['nt']} | {k} | {omega:g} | {_level(coarse)} | " + " | ".join(cells) + " |")
        else:
            for (st, mesh, k, omega, coarse), rs in sorted(groups, key=lambda g: (g[0][1], -g[0][2], -g[0][3], g[0][4])):
                cells = _cells(rs, cols, colkey)
                out.append(f"| {mesh} | {k} | {omega:g} | {_level(coarse)} | " + " | ".join(cells) + " |")
        out.append("")
    return "\n".join(out)


def ablation_table(rows):
    nts = sorted({r["nt"] for r in rows})
    out = ["| steps/sub | omega | variant | " + " | ".join(f"N_t={nt}" for nt in nts) + " |",
           "|" + "---|" * (3 + len(nts))]
    groups = {}
    for r in rows:
        groups.setdefault((r["steps_per_sub"], r["omega"], r["variant"]), []).append(r)
    order = list(ABLATIONS)
    for (k, omega, name), rs in sorted(groups.items(), key=lambda kv: (-kv[0][0], -kv[0][1],
                                                                        order.index(kv[0][2]))):
        out.append(f"| {k} | {omega:g} | {name} | " + " | ".join(_cells(rs, nts, "nt")) + " |")
    out.append("")
    return "\n".join(out)


def _level(coarse):
    return "one-level" if coarse == 0 else "two-level"


def _cells(rs, cols, colkey):
    got = {r[colkey]: r for r in rs}
    cells = []
    for c in cols:
        r = got.get(c)
        if r is None:
            cells.append("")
        elif r["converged"]:
            cells.append(str(r["iters"]))
        else:
            cells.append(f">{r['iters']}")
    return cells


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("study", choices=["weak", "omega", "mesh", "ablation", "all"])
    ap.add_argument("--mesh", type=int, default=17, help="mesh points per direction")
    ap.add_argument("--nt", type=int, default=800, help="N_t of the omega and mesh studies")
    ap.add_argument("--max-nt", type=int, default=3200)
    ap.add_argument("--sweep", choices=["step", "modal"], default="step")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--out", default=None, help="markdown table of the rows")
    args = ap.parse_args(argv)
    series = tuple(n for n in NT_SERIES if n <= args.max_nt)
    cases = []
    if args.study in ("weak", "all"):
        cases += list(weak_cases(args.mesh, series))
    if args.study in ("omega", "all"):
        cases += list(omega_cases(args.nt, args.mesh))
    if args.study in ("mesh", "all"):
        cases += list(mesh_cases(args.nt))
    if args.study == "ablation":
        cases += list(ablation_cases(args.mesh, tuple(n for n in (100, 200, 400, 800, 1600)
                                                      if n <= args.max_nt)))
    rows = []
    for case in cases:
        row = run_case(case, sweep=args.sweep, precision=args.precision)
        rows.append(row)
        print(json.dumps(row), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(markdown(rows) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
