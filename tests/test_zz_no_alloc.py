"""kkt_spatial_solve_noalloc, called through the C ABI: bitwise the results of kkt_spatial_solve
on two calls in a row (the second smaller, with another shift), within the oracle's tolerance,
no change of free device memory, and a clear refusal beyond its fixed scratch array."""

import ctypes

import numpy as np
import pytest

from oracle.problem import Problem
from oracle import spatial as sp
from paper_2305_04421_amd import workloads as wl
from common import CASES, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-11, "fp32": 1e-4, "bf16x6": 1e-4, "bf16x3": 1e-3, "bf16": 5e-2}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def noalloc(S, b, x, nslices, shift):
    from paper_2305_04421_amd import _lib
    lib = _lib.load()
    return lib.kkt_spatial_solve_noalloc(S._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                         int(nslices), float(shift))


@pytest.mark.parametrize("precision", list(TOL))
@pytest.mark.parametrize("name", ["ragged_tiles", "full_tiles_overlap_k", "tiny_ragged"])
def test_noalloc_spatial_solve_equals_the_allocating_one(name, precision):
    from paper_2305_04421_amd import KKTSolver
    params = CASES[name]
    p = Problem(**params).validate()
    with KKTSolver(params, precision) as S:
        for nslices, shift, seed in ((7, p.sigma, 61), (3, 1.7, 62)):   # the second call is smaller
            b_host = wl.random_field((nslices,) + p.slice_shape, seed)
            b = dev(b_host)
            want = S.spatial_solve(b, shift)
            x = torch.full_like(b, float("nan"))
            torch.cuda.synchronize()
            free = torch.cuda.mem_get_info()[0]
            assert noalloc(S, b, x, nslices, shift) == 0
            torch.cuda.synchronize()
            assert torch.cuda.mem_get_info()[0] == free
            assert torch.equal(x, want), (name, precision, nslices)
            xh = x.cpu().numpy().reshape(b_host.shape)
            assert relerr(xh, sp.solve_diag_block(p, b_host, shift)) <= TOL[precision]


def test_noalloc_refuses_more_than_its_scratch_array():
    from paper_2305_04421_amd import KKTSolver, _lib
    params = wl.problem(nx=512, ny=512, nt=4, n_sub=1, overlap=0, coarse=0)   # 2 MiB per float64 slice
    p = Problem(**params).validate()
    with KKTSolver(params) as S:
        ok = dev(wl.random_field((15,) + p.slice_shape, 63))
        x = torch.empty_like(ok)
        assert noalloc(S, ok, x, 15, 1.3) == 0          # 2 MiB table + 2 x 15 x 2 MiB = 62 MiB
        assert torch.equal(x, S.spatial_solve(ok, 1.3))
        big = dev(wl.random_field((16,) + p.slice_shape, 64))
        y = torch.zeros_like(big)
        assert noalloc(S, big, y, 16, 1.3) == _lib.EINVAL
        assert b"at most 15 slices" in _lib.load().kkt_last_error()
        assert not bool(y.any())
        assert noalloc(S, big, y, 0, 1.3) == 0 and noalloc(S, big, y, 2, -1.0) == _lib.EINVAL
