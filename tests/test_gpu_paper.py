"""The experiment of Sec. 4 on the HIP path: unrestarted GMRES (one Arnoldi cycle of up to 420
vectors) with the one-level and the two-level preconditioner on the closed-form problem.

Iteration counts equal the oracle's; iterates after a fixed number of steps of a long cycle
agree with the oracle's to 1e-9 relative; and the qualitative claims of Sec. 4 hold as
properties: the two-level count stays flat as N_t (and N_D with it) grows, the one-level
count grows with N_D.
"""

import numpy as np
import pytest

from oracle.problem import Problem
from oracle import operators as op
from oracle import precond as pc
from oracle import gmres as gm
from paper_2305_04421_amd import workloads as wl
from common import relerr, relerr_blocks, relerr_blocks_2norm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def oracle_solve(params, f, restart, maxit, rtol):
    p = Problem(**params).validate()
    return gm.gmres(lambda v: op.apply_K(p, v), lambda v: pc.apply_Pinv(p, v), f,
                    restart=restart, maxit=maxit, rtol=rtol)


def paper_rhs(params):
    p = Problem(**params).validate()
    u0, ut = wl.paper_data(params)
    return op.rhs(p, u0, ut)


@pytest.mark.parametrize("sweep", ["step", "modal"])
@pytest.mark.parametrize("steps,coarse", [(20, 0), (20, 2), (5, 0), (5, 2)])
def test_paper_workload_iterations_equal_oracle(steps, coarse, sweep):
    from paper_2305_04421_amd import KKTSolver
    params = wl.paper_problem(100, steps, 1e-2, coarse=coarse, n_points=9)
    f = paper_rhs(params)
    ref = oracle_solve(params, f, restart=420, maxit=420, rtol=1e-6)
    with KKTSolver(params, sweep=sweep) as S:
        x, st = S.solve(dev(f), restart=420, maxit=420, rtol=1e-6)
    assert ref.converged and st["status"] == 0
    assert st["iters"] == ref.iterations, (st["iters"], ref.iterations)
    xs = x.cpu().numpy().reshape(f.shape)
    assert relerr_blocks_2norm(xs, ref.x) <= 1e-9, relerr_blocks_2norm(xs, ref.x)
    assert st["relres_true"] <= 1e-6


@pytest.mark.parametrize("restart", [33, 100])
def test_long_cycle_matches_oracle_at_fixed_iterations(restart):
    """A cycle longer than one 32-vector chunk of the inner-product kernel, stopped early."""
    from paper_2305_04421_amd import KKTSolver
    params = wl.paper_problem(400, 5, 1e-2, coarse=0, n_points=9)   # 80 subdomains, one level
    f = paper_rhs(params)
    iters = 100
    ref = oracle_solve(params, f, restart=restart, maxit=iters, rtol=1e-15)
    with KKTSolver(params) as S:
        x, st = S.solve(dev(f), restart=restart, maxit=iters, rtol=1e-15)
    assert st["status"] == 1 and st["iters"] == ref.iterations == iters
    xs = x.cpu().numpy().reshape(f.shape)
    assert relerr_blocks_2norm(xs, ref.x) <= 1e-9, relerr_blocks_2norm(xs, ref.x)


def test_restart_bounds():
    from paper_2305_04421_amd import KKTSolver, KKTDDError, _lib
    params = wl.paper_problem(100, 20, 1e-2, n_points=9)
    with KKTSolver(params) as S:
        f = dev(paper_rhs(params))
        for bad in (0, _lib.MAX_RESTART + 1):
            with pytest.raises(KKTDDError) as ei:
                S.solve(f, restart=bad)
            assert ei.value.code == _lib.EINVAL
        # growing the cycle reallocates the basis; the solve still converges
        _, st1 = S.solve(f, restart=5, maxit=420, rtol=1e-6)
        _, st2 = S.solve(f, restart=200, maxit=420, rtol=1e-6)
        assert st1["status"] == st2["status"] == 0
        assert st2["restarts"] == 0 and st2["iters"] <= st1["iters"]


def test_two_level_is_flat_and_one_level_grows():
    """Sec. 4 (Fig. 1): at fixed steps per subdomain the two-level count does not grow with
    N_t, the one-level count does."""
    from paper_2305_04421_amd import KKTSolver
    counts = {0: [], 2: []}
    for nt in (100, 200, 400, 800):
        for coarse in (0, 2):
            params = wl.paper_problem(nt, 5, 1e-2, coarse=coarse, n_points=9)
            f = paper_rhs(params)
            with KKTSolver(params, sweep="modal") as S:
                _, st = S.solve(dev(f), restart=420, maxit=420, rtol=1e-6)
            assert st["status"] == 0
            counts[coarse].append(st["iters"])
    two, one = counts[2], counts[0]
    assert max(two) - min(two) <= 4, two
    assert all(b > a for a, b in zip(one, one[1:])), one
    assert one[-1] >= 4 * two[-1], (one, two)


def test_mesh_size_is_not_a_factor():
    """Sec. 4: the two-level count barely changes between 9x9, 17x17 and 33x33 mesh points."""
    from paper_2305_04421_amd import KKTSolver
    counts = []
    for n_points in (9, 17, 33):
        params = wl.paper_problem(200, 20, 1e-2, coarse=2, n_points=n_points)
        f = paper_rhs(params)
        with KKTSolver(params, sweep="modal") as S:
            _, st = S.solve(dev(f), restart=420, maxit=420, rtol=1e-6)
        assert st["status"] == 0
        counts.append(st["iters"])
    assert max(counts) - min(counts) <= 2, counts


def test_two_level_is_robust_in_omega():
    """Sec. 4 (Fig. 2): over five orders of magnitude of omega the two-level count stays within
    a narrow band while the one-level count varies strongly."""
    from paper_2305_04421_amd import KKTSolver
    two, one = [], []
    for omega in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5):
        for coarse, out in ((2, two), (0, one)):
            params = wl.paper_problem(400, 5, omega, coarse=coarse, n_points=9)
            f = paper_rhs(params)
            with KKTSolver(params, sweep="modal") as S:
                _, st = S.solve(dev(f), restart=420, maxit=420, rtol=1e-6)
            assert st["status"] == 0
            out.append(st["iters"])
    assert max(two) - min(two) <= 6, two
    assert max(one) >= 3 * max(two), (one, two)
