"""Host-only checks of the test metrics, the stats layout of the C ABI and the memory plan.

The parity metric compares KKT vectors block by block.  Here the oracle alone shows, on every
operator-level case, that a wrong Schur block (z_w = 0, z_w doubled, or one entry off by a
relative 1e-9) fails the 1e-11 bound of the preconditioner tests, while a whole-vector metric
lets some of these mistakes through because the z block r_z/(omega h) of Eq. (7) dominates.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle.problem import Problem
from oracle import precond as pc
from paper_2305_04421_amd import workloads as wl
from common import CASES, relerr, relerr_blocks, relerr_blocks_2norm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = 1e-11   # the bound of the float64 preconditioner parity tests


def _plants(want):
    zero = want.copy()
    zero[2] = 0.0
    double = want.copy()
    double[2] *= 2.0
    one = want.copy()
    k = np.unravel_index(np.argmax(np.abs(want[2])), want[2].shape)
    one[2][k] += 1e-9 * np.abs(want[2]).max()
    return {"z_w = 0": zero, "z_w doubled": double, "one z_w entry off by 1e-9": one}


@pytest.mark.parametrize("name", list(CASES))
def test_block_metric_rejects_a_wrong_schur_block(name):
    params = CASES[name]
    p = Problem(**params).validate()
    r = wl.random_field((3,) + p.field_shape, 103)
    want = pc.apply_Pinv(p, r)
    assert relerr_blocks(want, want) == 0.0
    for what, bad in _plants(want).items():
        assert relerr_blocks(bad, want) > TOL, (name, what)
        assert relerr_blocks_2norm(bad, want) > TOL, (name, what)


def test_whole_vector_metric_misses_the_schur_block():
    """The reason for the block metric: on ragged_tiles the z block is so much larger than
    z_w that dropping z_w entirely stays under the bound of a whole-vector comparison."""
    p = Problem(**CASES["ragged_tiles"]).validate()
    want = pc.apply_Pinv(p, wl.random_field((3,) + p.field_shape, 103))
    bad = _plants(want)["z_w = 0"]
    assert relerr(bad, want) <= TOL
    assert relerr_blocks(bad, want) == 1.0


def test_block_metric_handles_zero_blocks():
    a = np.zeros((3, 2, 2))
    b = np.zeros((3, 2, 2))
    assert relerr_blocks(a, b) == 0.0
    a[1, 0, 0] = 1e-300
    assert relerr_blocks(a, b) == np.inf


def test_stats_struct_matches_the_header():
    """The ctypes mirror of kktdd_stats has the header's fields, in order, with their types."""
    from paper_2305_04421_amd import _lib
    text = open(os.path.join(ROOT, "include", "kktdd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct kktdd_stats \{(.*?)\} kktdd_stats;", text, flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, name = decl.split()
        m = re.match(r"(\w+)\[(\d+)\]", name)
        fields.append((m.group(1), typ, int(m.group(2))) if m else (name, typ, 1))
    ct = {"int32_t": ctypes.c_int32, "double": ctypes.c_double}
    mirror = _lib.Stats._fields_
    assert [f[0] for f in fields] == [f[0] for f in mirror]
    for (name, typ, n), (_, ctyp) in zip(fields, mirror):
        want = ct[typ] if n == 1 else ct[typ] * n
        assert ctypes.sizeof(ctyp) == ctypes.sizeof(want) and getattr(ctyp, "_type_", ctyp) == getattr(
            want, "_type_", want), name


def test_memory_plan_of_the_largest_workload():
    """grid512 (1.6e9 unknowns): FGMRES(30) needs more than the 288 GB of one MI355X, which is
    why the bench runs it with restart 12; FGMRES(12) fits."""
    from paper_2305_04421_amd import memory_plan
    params, _ = wl.config("grid512")
    hbm = 288e9
    assert memory_plan(params, "fp64", 30) > hbm
    assert memory_plan(params, "fp64", 12) < 0.85 * hbm
    assert memory_plan(params, "fp32", 12) < memory_plan(params, "fp64", 12)
