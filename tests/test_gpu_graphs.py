"""Arnoldi steps replayed from HIP graphs give bitwise the results of the same launches issued
from the stream.

fgmres_solve runs each basis slot's step (Schur-block application, matvec, DCGS2 passes)
eagerly the first time, records it as a HIP graph the second time and replays it afterwards,
on any stream but the NULL stream (which cannot be captured): the handles here get a private
torch stream.
Here short restarts make every slot run several times within one solve; the solves are
repeated with the program's own eager work (a preconditioner application, a matvec) and
synchronisations between them, and every replay is compared with the eager solve.
"""

import numpy as np
import pytest

from oracle.problem import Problem
from oracle import operators as op
from paper_2305_04421_amd import workloads as wl
from common import CASES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


@pytest.mark.parametrize("precision,sweep", [("fp64", "step"), ("fp32", "step"), ("bf16x3", "step"),
                                             ("fp64", "modal"), ("fp32", "modal")])
@pytest.mark.parametrize("name", ["ragged_tiles", "tiny32", "long_subdomains"])
def test_graph_replays_equal_stream_launches(name, precision, sweep, monkeypatch):
    from paper_2305_04421_amd import KKTSolver
    params = CASES[name]
    p = Problem(**params).validate()
    u0, ut = wl.sine_mode_data(params, 41, 6)
    f = dev(op.rhs(p, u0, ut))
    r = dev(wl.random_field((3,) + p.field_shape, 42))
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    monkeypatch.setenv("KKTDD_GRAPH", "0")
    with torch.cuda.stream(stream), KKTSolver(params, precision, sweep=sweep) as S:
        x_ref, st_ref = S.solve(f, restart=4, maxit=40, rtol=1e-12)
        x_ref = x_ref.clone()
        z_ref = S.precond(r).clone()
        stream.synchronize()
    monkeypatch.setenv("KKTDD_GRAPH", "1")
    with torch.cuda.stream(stream), KKTSolver(params, precision, sweep=sweep) as S:
        for rep in range(4):
            x, st = S.solve(f, restart=4, maxit=40, rtol=1e-12)
            stream.synchronize()
            assert st["iters"] == st_ref["iters"] and st["status"] == st_ref["status"], rep
            assert torch.equal(x, x_ref), (name, precision, sweep, rep)
            # eager work on the same handle between the replays
            assert torch.equal(S.precond(r), z_ref), rep
            S.apply(f)
            stream.synchronize()


def test_graph_replays_in_a_batch_equal_single_solves(monkeypatch):
    from paper_2305_04421_amd import KKTSolver, solve_batched
    names = ["ragged_tiles", "tiny32", "full_tiles_overlap_k"]
    fs, solvers, single = [], [], []
    monkeypatch.setenv("KKTDD_GRAPH", "0")
    for k, name in enumerate(names):
        params = CASES[name]
        p = Problem(**params).validate()
        u0, ut = wl.sine_mode_data(params, 50 + k, 5)
        fs.append(dev(op.rhs(p, u0, ut)))
        with KKTSolver(params) as S:
            x, st = S.solve(fs[-1], restart=6, maxit=60, rtol=1e-10)
            single.append((x.clone(), st))
    monkeypatch.setenv("KKTDD_GRAPH", "1")
    solvers = [KKTSolver(CASES[name]) for name in names]
    try:
        for rep in range(3):
            xs, sts = solve_batched(solvers, fs, restart=6, maxit=60, rtol=1e-10)
            for (x1, st1), x2, st2 in zip(single, xs, sts):
                assert st1["iters"] == st2["iters"] and st1["status"] == st2["status"], rep
                assert torch.equal(x1, x2), rep
    finally:
        for S in solvers:
            S.close()
