"""Failure paths, debug modes and the restart boundary on the device.

- Memory-plan refusals: kkt_create of a problem larger than the device, and fgmres_solve of
  the grid512 workload with restart 30 (its Krylov basis needs more than the 288 GB of one
  MI355X), both return KKTDD_ENOMEM before allocating anything, and the handle stays usable.
- KKTDD_DEBUG_POISON=1 fills every work buffer with NaN bytes before use: preconditioner and
  solve results stay bitwise equal, so no kernel reads workspace it has not written.
- A solve stopped after whole cycles and resumed from its iterate equals one solve, bitwise.
- The residual history (kkt_residual_history) has one entry per Arnoldi step and follows
  the oracle's Givens estimates.
"""

import numpy as np
import pytest

from oracle.problem import Problem
from oracle import operators as op
from oracle import precond as pc
from oracle import gmres as gm
from paper_2305_04421_amd import workloads as wl
from common import CASES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_create_refuses_a_problem_larger_than_the_device():
    from paper_2305_04421_amd import KKTSolver, KKTDDError, memory_plan, _lib
    params = wl.problem(nx=1024, ny=1024, nt=60000, n_sub=3750, overlap=2)
    assert memory_plan(params) > torch.cuda.get_device_properties(0).total_memory
    before = free_bytes()
    with pytest.raises(KKTDDError) as ei:
        KKTSolver(params)
    assert ei.value.code == _lib.ENOMEM
    assert free_bytes() == before


def test_grid512_solve_with_restart_30_is_refused_before_allocating():
    from paper_2305_04421_amd import KKTSolver, KKTDDError, memory_plan, _lib
    params, recipe = wl.config("grid512")
    total = torch.cuda.get_device_properties(0).total_memory
    assert memory_plan(params, "fp64", 30) > total >= memory_plan(params, "fp64", 12)
    u0, ut = wl.data(params, recipe)
    with KKTSolver(params) as S:
        f = S.rhs(dev(u0), dev(ut))
        del u0, ut
        x = torch.zeros_like(f)
        before = free_bytes()
        with pytest.raises(KKTDDError) as ei:
            S.solve(f, x=x, restart=30, maxit=5, rtol=1e-8)
        assert ei.value.code == _lib.ENOMEM
        assert b"restart 30" in _lib.load().kkt_last_error()
        assert free_bytes() == before
        assert not bool(x.any())
        # the handle is intact: a matvec after the refusal is exact on a sampled node
        y = S.apply(f)
        assert torch.isfinite(y).all()
        del f, x, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision,sweep", [("fp64", "step"), ("fp32", "step"), ("bf16x6", "step"),
                                             ("fp64", "modal"), ("fp32", "modal")])
@pytest.mark.parametrize("name", ["ragged_tiles", "tiny_ragged", "long_subdomains"])
def test_nan_poisoned_workspace_changes_nothing(name, precision, sweep, monkeypatch):
    from paper_2305_04421_amd import KKTSolver
    params = CASES[name]
    p = Problem(**params).validate()
    r = dev(wl.random_field((3,) + p.field_shape, 31))
    u0, ut = wl.sine_mode_data(params, 32, 4)
    f = dev(op.rhs(p, u0, ut))
    out = {}
    for poison in ("0", "1"):
        monkeypatch.setenv("KKTDD_DEBUG_POISON", poison)
        with KKTSolver(params, precision, sweep=sweep) as S:
            z = S.precond(r).clone()
            x, st = S.solve(f, restart=5, maxit=40, rtol=1e-10)
            out[poison] = (z, x.clone(), st["iters"])
    assert torch.isfinite(out["1"][0]).all() and torch.isfinite(out["1"][1]).all()
    assert torch.equal(out["0"][0], out["1"][0])
    assert torch.equal(out["0"][1], out["1"][1])
    assert out["0"][2] == out["1"][2]


@pytest.mark.parametrize("sweep", ["step", "modal"])
def test_solve_resumed_at_a_cycle_boundary_equals_one_solve(sweep):
    from paper_2305_04421_amd import KKTSolver
    params, recipe = wl.config("tiny32")
    p = Problem(**params).validate()
    u0, ut = wl.data(params, recipe)
    f = dev(op.rhs(p, u0, ut))
    with KKTSolver(params, sweep=sweep) as S:
        x_whole, st_whole = S.solve(f, restart=5, maxit=300, rtol=1e-8)
        assert st_whole["status"] == 0 and st_whole["iters"] > 10
        x_part, st_first = S.solve(f, restart=5, maxit=10, rtol=1e-8)
        assert st_first["status"] == 1 and st_first["iters"] == 10
        hist_first = S.residual_history()
        x_part, st_rest = S.solve(f, x=x_part, restart=5, maxit=300, rtol=1e-8)
        hist_rest = S.residual_history()
    assert st_rest["status"] == 0
    assert st_first["iters"] + st_rest["iters"] == st_whole["iters"]
    assert torch.equal(x_part, x_whole)
    assert len(hist_first) == 10 and len(hist_first) + len(hist_rest) == st_whole["iters"]


def test_residual_history_follows_the_oracle():
    from paper_2305_04421_amd import KKTSolver
    params, recipe = wl.config("tiny32")
    p = Problem(**params).validate()
    u0, ut = wl.data(params, recipe)
    f = op.rhs(p, u0, ut)
    ref = gm.gmres(lambda v: op.apply_K(p, v), lambda v: pc.apply_Pinv(p, v), f, restart=30, maxit=300,
                   rtol=1e-8)
    with KKTSolver(params) as S:
        _, st = S.solve(dev(f), restart=30, maxit=300, rtol=1e-8)
        hist = S.residual_history()
    assert len(hist) == st["iters"] == ref.iterations
    assert np.allclose(hist, ref.history, rtol=1e-6, atol=0.0), (hist, ref.history)
    assert hist[-1] <= 1e-8 < hist[-2]
