"""Parity of the HIP library with the CPU oracle, element by element, on seeded inputs.

Float64 path: the matvec and right-hand side to 1e-13 relative, the spatial solve and the
preconditioner to 1e-11 relative (rounding of four dense transforms per step, chained over
a sweep), the FGMRES iterate to 1e-10 relative at equal iteration counts.  Float32 sweeps:
the spatial solve to 1e-4 relative and the solve itself to the same 1e-8 relative residual
within two more iterations than float64.
"""

import numpy as np
import pytest

from oracle.problem import Problem
from oracle import operators as op
from oracle import precond as pc
from oracle import spatial as sp
from oracle import gmres as gm
from paper_2305_04421_amd import workloads as wl
from common import CASES, relerr, relerr_blocks, relerr_blocks_2norm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def host(t, shape):
    return t.detach().cpu().numpy().reshape(shape)


def solver(params, precision="fp64", sweep="step"):
    from paper_2305_04421_amd import KKTSolver
    return KKTSolver(params, precision, sweep=sweep)


@pytest.mark.parametrize("name", list(CASES))
def test_kkt_apply_matches_oracle(name):
    params = CASES[name]
    p = Problem(**params).validate()
    x = wl.random_field((3,) + p.field_shape, 101)
    with solver(params) as S:
        y = host(S.apply(dev(x)), x.shape)
    assert relerr(y, op.apply_K(p, x)) <= 1e-13


@pytest.mark.parametrize("name", ["ragged_tiles", "tiny32"])
def test_rhs_matches_oracle(name):
    params = CASES[name]
    p = Problem(**params).validate()
    u0, ut = wl.sine_mode_data(params, 5, 4)
    with solver(params) as S:
        f = host(S.rhs(dev(u0), dev(ut)), (3,) + p.field_shape)
    assert relerr(f, op.rhs(p, u0, ut)) <= 1e-15


PRECISION_TOL = [("fp64", 1e-11), ("fp32", 1e-4), ("bf16x6", 1e-4), ("bf16x3", 1e-3), ("bf16", 5e-2)]


@pytest.mark.parametrize("precision,tol", PRECISION_TOL)
@pytest.mark.parametrize("name", list(CASES))
def test_spatial_solve_matches_oracle(name, precision, tol):
    params = CASES[name]
    p = Problem(**params).validate()
    b = wl.random_field((3,) + p.slice_shape, 102)
    with solver(params, precision) as S:
        x = host(S.spatial_solve(dev(b), p.sigma), b.shape)
    assert relerr(x, sp.solve_diag_block(p, b, p.sigma)) <= tol


@pytest.mark.parametrize("nx,ny", [(81, 100), (200, 17), (600, 33), (1024, 9), (9, 1024), (129, 257),
                                   (385, 512), (512, 385)])
@pytest.mark.parametrize("precision,tol", PRECISION_TOL)
def test_spatial_solve_tile_shapes(nx, ny, precision, tol):
    """Padded extents whose tile counts need 1..8 tiles per wave and up to 8 waves, and
    workgroups needing more than 64 KiB of LDS; 384 and 512 are the three- and four-tile
    row kernels that share a CU between two workgroups (every grid512 sweep launch)."""
    params = wl.problem(nx=nx, ny=ny, nt=4, Lx=1.0, Ly=1.7, nu=0.05, omega=1e-3, n_sub=1, overlap=0, coarse=0)
    p = Problem(**params).validate()
    b = wl.random_field((2,) + p.slice_shape, 106)
    with solver(params, precision) as S:
        x = host(S.spatial_solve(dev(b), 1.3), b.shape)
    assert relerr(x, sp.solve_diag_block(p, b, 1.3)) <= tol


@pytest.mark.parametrize("sweep", ["step", "modal"])
@pytest.mark.parametrize("coarse", [0, 1, 2])
@pytest.mark.parametrize("name", ["tiny_ragged", "ragged_tiles", "full_tiles_overlap_k", "tiny32", "long_subdomains",
                                  "reg24", "reg32_overlap_k"])
def test_precond_matches_oracle(name, coarse, sweep):
    params = dict(CASES[name], coarse=coarse)
    p = Problem(**params).validate()
    r = wl.random_field((3,) + p.field_shape, 103)
    with solver(params, sweep=sweep) as S:
        z = host(S.precond(dev(r)), r.shape)
    want = pc.apply_Pinv(p, r)
    assert relerr_blocks(z, want) <= 1e-11


@pytest.mark.parametrize("precision,tol", PRECISION_TOL[1:])
@pytest.mark.parametrize("sweep", ["step", "modal"])
def test_precond_reduced_precision_close_to_oracle(sweep, precision, tol):
    params = CASES["tiny32"]
    p = Problem(**params).validate()
    r = wl.random_field((3,) + p.field_shape, 107)
    with solver(params, precision, sweep=sweep) as S:
        z = host(S.precond(dev(r)), r.shape)
    assert relerr_blocks(z, pc.apply_Pinv(p, r)) <= 10 * tol


@pytest.mark.parametrize("sweep", ["step", "modal"])
def test_precond_degenerate_one_level(sweep):
    params = CASES["degenerate"]
    p = Problem(**params).validate()
    r = wl.random_field((3,) + p.field_shape, 104)
    with solver(params, sweep=sweep) as S:
        z = host(S.precond(dev(r)), r.shape)
    assert relerr_blocks(z, pc.apply_Pinv(p, r)) <= 1e-12


# (waves, deep ring, blocks per workgroup) of the row kernel and of the column kernel
SHAPE_PAIRS = [((8, 0, 1), (4, 1, 1)), ((8, 1, 1), (2, 0, 1)), ((4, 1, 1), (2, 1, 1)), ((2, 0, 1), (4, 0, 1)),
               ((4, 0, 1), (2, 1, 1)), ((8, 0, 2), (4, 0, 2)), ((4, 0, 4), (2, 0, 4)), ((2, 0, 2), (4, 0, 4)),
               ((8, 0, 4), (2, 0, 2))]


def _shape_sweep(lib, prec, extents, ns, run, pairs):
    """run() under every (rows, cols) launch shape of `pairs`; restores the table after."""
    import ctypes
    saved = []
    for kind, M in ((0, extents[0]), (1, extents[1])):
        w, d, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert lib.kkt_tune_get(kind, prec, M, ns, ctypes.byref(w), ctypes.byref(d), ctypes.byref(b)) == 0
        saved.append((kind, M, w.value, d.value, b.value))
    out = []
    try:
        for rows_shape, cols_shape in pairs:
            assert lib.kkt_tune_set(0, prec, extents[0], ns, *rows_shape) == 0
            assert lib.kkt_tune_set(1, prec, extents[1], ns, *cols_shape) == 0
            out.append(((rows_shape, cols_shape), run()))
    finally:
        for kind, M, w, d, b in saved:
            lib.kkt_tune_set(kind, prec, M, ns, w, d, b)
    return out


@pytest.mark.parametrize("precision,sweep", [(p, "step") for p in ("fp64", "fp32", "bf16x6", "bf16x3", "bf16")] +
                                            [("fp64", "modal"), ("fp32", "modal")])
@pytest.mark.parametrize("name", ["full_tiles_overlap_k", "ragged_tiles"])
def test_launch_shapes_give_identical_results(name, precision, sweep):
    """Every launch shape of the transform kernels (waves per workgroup, prefetch depth, 16-row
    or 16-column blocks per workgroup) performs the same operations in the same order: the
    preconditioner is bitwise equal.  ragged_tiles has fewer row blocks than some widths."""
    from paper_2305_04421_amd import _lib
    lib = _lib.load()
    params = CASES[name]    # padded extents 128 x 64 (4 subdomains), 64 x 32 (3 subdomains)
    p = Problem(**params).validate()
    r = dev(wl.random_field((3,) + p.field_shape, 21))
    prec = _lib.PRECISIONS[precision]
    extents = (128, 64) if name == "full_tiles_overlap_k" else (64, 32)
    pairs = SHAPE_PAIRS if name == "full_tiles_overlap_k" else [
        ((4, 0, 1), (2, 0, 1)), ((4, 0, 2), (2, 0, 2)), ((4, 0, 4), (2, 0, 4)), ((2, 0, 4), (2, 0, 1))]
    with solver(params, precision, sweep=sweep) as S:
        ns = p.nt if sweep == "modal" else p.n_sub
        ref = S.precond(r).clone()
        for shapes, z in _shape_sweep(lib, prec, extents, ns, lambda: S.precond(r).clone(), pairs):
            assert torch.equal(z, ref), shapes


# (nx, ny) -> padded extents (rows, cols) and the shape pairs tried there; 16-wave workgroups
# (two tiles per wave) exist where an extent has a multiple of 16 tiles (512 here)
WIDTH_GEOMETRIES = {
    (385, 512): ((384, 512), [((8, 0, 1), (8, 0, 1)), ((8, 0, 2), (8, 0, 2)), ((8, 0, 4), (8, 0, 4)),
                              ((8, 0, 2), (8, 0, 1)), ((8, 0, 2), (16, 0, 2)), ((8, 0, 1), (16, 0, 1))]),
    (512, 385): ((512, 384), [((8, 0, 1), (8, 0, 1)), ((16, 0, 2), (8, 0, 2)), ((16, 0, 1), (8, 0, 4))]),
}
# 16-wave workgroups of four blocks: the engines whose two-tile kernels fit them
WIDTH_PAIRS_16x4 = {(385, 512): [((8, 0, 4), (16, 0, 4))], (512, 385): [((16, 0, 4), (8, 0, 2))]}


@pytest.mark.parametrize("geometry", list(WIDTH_GEOMETRIES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x6", "bf16x3", "bf16"])
def test_block_widths_give_identical_results_at_the_largest_extents(precision, geometry):
    """The spatial solve at padded extents 384 and 512 (three and four tiles per wave at 8
    waves, every grid512 sweep launch; two tiles per wave at 16 waves) under each workgroup
    width and wave count: bitwise equal to one block per 8-wave group."""
    from paper_2305_04421_amd import _lib
    lib = _lib.load()
    nx, ny = geometry
    extents, pairs = WIDTH_GEOMETRIES[geometry]
    if precision in ("fp32", "bf16x3", "bf16"):
        pairs = pairs + WIDTH_PAIRS_16x4[geometry]
    params = wl.problem(nx=nx, ny=ny, nt=4, Lx=1.0, Ly=1.7, nu=0.05, omega=1e-3, n_sub=1, overlap=0, coarse=0)
    p = Problem(**params).validate()
    b = dev(wl.random_field((3,) + p.slice_shape, 108))
    prec = _lib.PRECISIONS[precision]
    with solver(params, precision) as S:
        out = _shape_sweep(lib, prec, extents, 3, lambda: S.spatial_solve(b, 1.3).clone(), pairs)
    ref = out[0][1]
    for shapes, x in out[1:]:
        assert torch.equal(x, ref), shapes


PLACEMENT_CASES = dict(CASES, eleven_subdomains=wl.problem(nx=40, ny=33, nt=22, Lx=1.0, Ly=0.8, nu=0.4,
                                                           omega=1e-3, n_sub=11, overlap=1, coarse=2))


@pytest.mark.parametrize("case,sweep", [("full_tiles_overlap_k", "step"), ("full_tiles_overlap_k", "modal"),
                                        ("tiny32", "step"), ("eleven_subdomains", "step")])
def test_workgroup_placement_gives_identical_results(case, sweep, monkeypatch):
    """Both workgroup placements of the transform kernels (slices spread over the XCDs, or one
    XCD per slice with a one-dimensional grid whose surplus workgroups exit) compute every
    tile the same way: the preconditioner is bitwise equal, also for slice counts that are not
    multiples of eight."""
    params = PLACEMENT_CASES[case]
    p = Problem(**params).validate()
    r = wl.random_field((3,) + p.field_shape, 23)
    rd = dev(r)
    with solver(params, sweep=sweep) as S:
        out = {}
        for mode in ("0", "1"):
            monkeypatch.setenv("KKTDD_XCD_MAP", mode)
            out[mode] = S.precond(rd).clone()
        monkeypatch.delenv("KKTDD_XCD_MAP")
        out["auto"] = S.precond(rd).clone()
    assert torch.equal(out["0"], out["1"])
    assert torch.equal(out["0"], out["auto"])
    assert relerr_blocks(host(out["1"], r.shape), pc.apply_Pinv(p, r)) <= 1e-11


def test_precond_is_deterministic():
    params = CASES["tiny32"]
    p = Problem(**params).validate()
    r = dev(wl.random_field((3,) + p.field_shape, 105))
    with solver(params) as S:
        a = S.precond(r).clone()
        b = S.precond(r)
    assert torch.equal(a, b)


def _oracle_solve(p, f, restart, maxit, rtol):
    return gm.gmres(lambda v: op.apply_K(p, v), lambda v: pc.apply_Pinv(p, v), f,
                    restart=restart, maxit=maxit, rtol=rtol)


@pytest.mark.parametrize("sweep", ["step", "modal"])
@pytest.mark.parametrize("name", ["ragged_tiles", "tiny32"])
def test_fgmres_matches_oracle_at_fixed_iterations(name, sweep):
    params = CASES[name]
    p = Problem(**params).validate()
    u0, ut = wl.sine_mode_data(params, 7, 8)
    f = op.rhs(p, u0, ut)
    ref = _oracle_solve(p, f, restart=4, maxit=7, rtol=1e-15)
    with solver(params, sweep=sweep) as S:
        x, st = S.solve(dev(f), restart=4, maxit=7, rtol=1e-15)
    assert st["iters"] == ref.iterations == 7
    assert st["status"] == 1
    xs = host(x, f.shape)
    assert relerr_blocks_2norm(xs, ref.x) <= 1e-10, relerr_blocks_2norm(xs, ref.x)


@pytest.mark.parametrize("sweep", ["step", "modal"])
def test_fgmres_converges_like_oracle_tiny32(sweep):
    params, recipe = wl.config("tiny32")
    p = Problem(**params).validate()
    u0, ut = wl.data(params, recipe)
    f = op.rhs(p, u0, ut)
    ref = _oracle_solve(p, f, restart=30, maxit=300, rtol=1e-8)
    with solver(params, sweep=sweep) as S:
        fd = S.rhs(dev(u0), dev(ut))
        x, st = S.solve(fd, restart=30, maxit=300, rtol=1e-8)
    assert st["status"] == 0 and ref.converged
    assert st["iters"] == ref.iterations
    assert st["relres_true"] <= 1e-8
    xs = host(x, f.shape)
    assert relerr_blocks_2norm(xs, ref.x) <= 1e-10, relerr_blocks_2norm(xs, ref.x)
    # the oracle's own residual of the GPU iterate
    assert np.linalg.norm(f - op.apply_K(p, xs)) <= 1e-8 * np.linalg.norm(f)


# Iterations allowed above float64 for each inner precision (float64 FGMRES recovers the
# 1e-8 residual; the inner rounding, amplified by the condition number of D_sigma, costs
# iterations).  Plain bfloat16 only has to converge.
EXTRA_ITERS = {"fp32": 2, "bf16x6": 2, "bf16x3": 4, "bf16": 60}


@pytest.mark.parametrize("precision", list(EXTRA_ITERS))
@pytest.mark.parametrize("sweep", ["step", "modal"])
def test_reduced_precision_sweeps_reach_float64_tolerance(sweep, precision):
    params, recipe = wl.config("tiny32")
    p = Problem(**params).validate()
    u0, ut = wl.data(params, recipe)
    f = op.rhs(p, u0, ut)
    with solver(params, "fp64", sweep=sweep) as S64, solver(params, precision, sweep=sweep) as Sr:
        fd = dev(f)
        x64, st64 = S64.solve(fd, restart=30, maxit=300, rtol=1e-8)
        xr, str_ = Sr.solve(fd, restart=30, maxit=300, rtol=1e-8)
    assert str_["status"] == 0 and str_["iters"] <= st64["iters"] + EXTRA_ITERS[precision], (st64, str_)
    xrh = host(xr, f.shape)
    assert np.linalg.norm(f - op.apply_K(p, xrh)) <= 1e-8 * np.linalg.norm(f)


def test_auto_precision_resolves_by_kappa():
    from paper_2305_04421_amd import kappa
    params, recipe = wl.config("tiny32")            # kappa 133: float32 sweeps
    assert kappa(params) < 500
    with solver(params, "auto") as S:
        assert S.resolved_precision == "fp32"
    stiff, recipe = wl.batch_uneven(64, seed=4)[50]  # kappa 1617: float32 sweeps stall here
    assert kappa(stiff) > 500
    u0, ut = wl.data(stiff, recipe)
    with solver(stiff, "auto") as Sa, solver(stiff, "fp64") as S64:
        assert Sa.resolved_precision == "fp64"
        fa = Sa.rhs(dev(u0), dev(ut))
        xa, sta = Sa.solve(fa, restart=12, maxit=100, rtol=1e-8)
        x64, st64 = S64.solve(fa, restart=12, maxit=100, rtol=1e-8)
    assert sta["status"] == 0 and sta["iters"] == st64["iters"]
    assert torch.equal(xa, x64)


def test_fgmres_edge_cases():
    params = CASES["tiny_ragged"]
    p = Problem(**params).validate()
    with solver(params) as S:
        zero = torch.zeros(S.size, dtype=torch.float64, device="cuda")
        x = torch.ones(S.size, dtype=torch.float64, device="cuda")
        x, st = S.solve(zero, x=x)
        assert st["status"] == 0 and st["iters"] == 0 and not bool(x.any())
        u0, ut = wl.sine_mode_data(params, 9, 3)
        f = dev(op.rhs(p, u0, ut))
        _, st = S.solve(f, restart=5, maxit=3, rtol=1e-14)
        assert st["status"] == 1 and st["iters"] == 3
        bad = f.clone()
        bad[5] = float("nan")
        from paper_2305_04421_amd import KKTDDError
        with pytest.raises(KKTDDError) as ei:
            S.solve(bad)
        assert ei.value.code == -4


def test_batched_solve_equals_individual_solves():
    """Uneven problems solved together give bitwise the same iterates as solved one by one."""
    from paper_2305_04421_amd import solve_batched
    names = ["ragged_tiles", "tiny32", "full_tiles_overlap_k"]
    fs, solvers, single = [], [], []
    for k, name in enumerate(names):
        params = CASES[name]
        p = Problem(**params).validate()
        u0, ut = wl.sine_mode_data(params, 20 + k, 5)
        S = solver(params)
        solvers.append(S)
        fs.append(dev(op.rhs(p, u0, ut)))
        x, st = S.solve(fs[-1], restart=10, maxit=60, rtol=1e-9)
        single.append((x.clone(), st))
    xs, sts = solve_batched(solvers, fs, restart=10, maxit=60, rtol=1e-9)
    for (x1, st1), x2, st2 in zip(single, xs, sts):
        assert st1["iters"] == st2["iters"] and st1["status"] == st2["status"] == 0
        assert torch.equal(x1, x2)
    for S in solvers:
        S.close()
