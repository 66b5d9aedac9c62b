"""The C-ABI library: it loads, exports every entry point its header declares, and rejects
bad problems in host-only validation.  No device call is made here."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kktdd.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2305_04421_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2305_04421_amd import build
        build.build()
    return _lib.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kkt_\w+|precond_apply|fgmres_solve)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ("kkt_create", "kkt_destroy", "kkt_size", "kkt_rhs", "kkt_apply", "precond_apply",
                 "fgmres_solve", "kkt_last_error", "kkt_validate", "kkt_memory_plan", "kkt_spatial_solve"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2305_04421_amd import _lib
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(_declared_functions()) == set(_lib.EXPORTED)


def _prob(**kw):
    from paper_2305_04421_amd import _lib
    base = dict(nx=32, ny=32, nt=32, Lx=1.0, Ly=1.0, T=1.0, nu=1.0, omega=1e-2, n_sub=4, overlap=2, coarse=2)
    base.update(kw)
    prec = base.pop("precision", "fp64")
    sweep = base.pop("sweep", "step")
    return _lib.make_problem(base, prec, sweep)


def test_validate_accepts_the_configurations(lib):
    from paper_2305_04421_amd import workloads as wl
    for name in ("tiny32", "grid128", "grid128_w4", "grid256", "grid512"):
        params, _ = wl.config(name)
        for prec in ("fp64", "fp32", "bf16", "bf16x3", "bf16x6", "auto"):
            p = _prob(**dict(params, precision=prec))
            assert lib.kkt_validate(ctypes.byref(p)) == 0, name


@pytest.mark.parametrize("bad", [dict(nx=1), dict(ny=0), dict(nx=1025), dict(nt=0), dict(nt=65536, n_sub=4), dict(omega=0.0),
                                 dict(nu=-1.0), dict(T=float("inf")), dict(Lx=0.0), dict(n_sub=5),
                                 dict(overlap=9), dict(overlap=-1), dict(coarse=3), dict(n_sub=32, coarse=2),
                                 dict(precision=6), dict(sweep=2)])
def test_validate_rejects_bad_problems(lib, bad):
    from paper_2305_04421_amd import _lib
    p = _prob(**bad)
    assert lib.kkt_validate(ctypes.byref(p)) == _lib.EINVAL
    assert len(lib.kkt_last_error()) > 0


def test_header_constants_match_the_binding():
    from paper_2305_04421_amd import _lib
    text = open(HEADER).read()
    assert int(re.search(r"#define KKTDD_MAX_RESTART (\d+)", text).group(1)) == _lib.MAX_RESTART
    for name, val in (("KKTDD_OK", _lib.OK), ("KKTDD_NOT_CONVERGED", _lib.NOT_CONVERGED),
                      ("KKTDD_EINVAL", _lib.EINVAL), ("KKTDD_EBREAKDOWN", _lib.EBREAKDOWN),
                      ("KKTDD_BF16X6", _lib.BF16X6), ("KKTDD_SWEEP_MODAL", _lib.SWEEP_MODAL)):
        assert int(re.search(name + r"\s*=\s*(-?\d+)", text).group(1)) == val, name


def test_kappa_matches_the_sine_mode_eigenvalues(lib):
    import math
    from oracle.problem import Problem
    from oracle.spatial import laplacian_eigenvalues_1d
    from paper_2305_04421_amd import kappa, workloads as wl
    for name in ("tiny32", "grid128", "grid256", "grid512"):
        params, _ = wl.config(name)
        p = Problem(**params).validate()
        lx = laplacian_eigenvalues_1d(p.nx, p.dx)
        ly = laplacian_eigenvalues_1d(p.ny, p.dy)
        d = p.sigma + p.dt * p.nu * (ly[:, None] + lx[None, :])
        assert math.isclose(kappa(params), d.max() / d.min(), rel_tol=1e-12), name
    assert lib.kkt_kappa(ctypes.byref(_prob(nx=1))) == -1.0


def test_auto_precision_is_accepted_and_planned_like_its_resolution(lib):
    from paper_2305_04421_amd import memory_plan
    stiff = dict(nx=256, ny=256, nt=240, nu=0.81, omega=2.1e-2, n_sub=15, overlap=2)   # kappa > 500
    mild = dict(nx=32, ny=32, nt=32, n_sub=4, overlap=2)                                # kappa 133
    for kw, want in ((stiff, "fp64"), (mild, "fp32")):
        p = _prob(**dict(kw, precision="auto"))
        assert lib.kkt_validate(ctypes.byref(p)) == 0
        params = dict(Lx=1.0, Ly=1.0, T=1.0, coarse=2, nu=1.0, omega=1e-2)
        params.update(kw)
        assert memory_plan(params, "auto", 10) == memory_plan(params, want, 10)


@pytest.mark.parametrize("bad", [dict(overlap_side="both"), dict(schwarz="asm", precision="fp32", sweep="modal"),
                                 dict(local="exact", sweep="step"), dict(combine="additive", precision="bf16x3",
                                                                         sweep="modal")])
def test_variants_are_rejected_off_the_float64_modal_path(lib, bad):
    from paper_2305_04421_amd import _lib
    p = _prob(**bad)
    assert lib.kkt_validate(ctypes.byref(p)) == _lib.EINVAL
    assert b"modal" in lib.kkt_last_error()


def test_variant_fields_out_of_range_are_rejected(lib):
    from paper_2305_04421_amd import _lib
    for field, value in (("overlap_side", 2), ("schwarz", -1), ("local", 2), ("combine", 3)):
        p = _prob(sweep="modal")
        setattr(p, field, value)
        assert lib.kkt_validate(ctypes.byref(p)) == _lib.EINVAL, field


def test_variant_memory_plan():
    from paper_2305_04421_amd import memory_plan
    base = dict(nx=32, ny=32, nt=64, n_sub=4, overlap=2, coarse=2)
    plain = memory_plan(base, "fp64", 0, sweep="modal")
    asm = memory_plan(dict(base, schwarz="asm", overlap_side="both"), "fp64", 0, sweep="modal")
    exact = memory_plan(dict(base, local="exact"), "fp64", 0, sweep="modal")
    MM = 32 * 32   # padded 31 -> 32
    assert asm - plain == 4 * 2 * 2 * MM * 8            # extension slots: N_D * 2 delta * MM
    assert exact - plain == 2 * 4 * (16 + 2) * MM * 8   # pivots and values: 2 * N_D * L * MM
    assert memory_plan(dict(base, local="exact"), "auto", 0, sweep="modal") == exact


def test_launch_shape_table(lib):
    from paper_2305_04421_amd import _lib
    w, d, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    # no entry: the default shape (8 waves for 32 tiles, shallow ring, one block)
    assert lib.kkt_tune_get(1, _lib.FP32, 512, 7, ctypes.byref(w), ctypes.byref(d), ctypes.byref(b)) == 0
    assert (w.value, d.value, b.value) == (8, 0, 1)
    assert lib.kkt_tune_set(1, _lib.FP32, 512, 7, 4, 1, 1) == 0
    assert lib.kkt_tune_get(1, _lib.FP32, 512, 7, ctypes.byref(w), ctypes.byref(d), ctypes.byref(b)) == 0
    assert (w.value, d.value, b.value) == (4, 1, 1)
    assert lib.kkt_tune_set(0, _lib.BF16X3, 512, 7, 8, 0, 4) == 0
    assert lib.kkt_tune_get(0, _lib.BF16X3, 512, 7, ctypes.byref(w), ctypes.byref(d), ctypes.byref(b)) == 0
    assert (w.value, d.value, b.value) == (8, 0, 4)
    # 16 waves: two tiles per wave (32 tiles), one or two blocks, shallow ring
    assert lib.kkt_tune_set(1, _lib.FP64, 512, 7, 16, 0, 2) == 0
    assert lib.kkt_tune_get(1, _lib.FP64, 512, 7, ctypes.byref(w), ctypes.byref(d), ctypes.byref(b)) == 0
    assert (w.value, d.value, b.value) == (16, 0, 2)
    assert lib.kkt_tune_set(0, _lib.BF16X6, 256, 7, 16, 0, 1) == 0
    # four blocks in 16 waves where the two-tile kernels fit: not float64 or bf16x6
    assert lib.kkt_tune_set(0, _lib.BF16X3, 512, 7, 16, 0, 4) == 0
    assert lib.kkt_tune_set(1, _lib.FP32, 512, 7, 16, 0, 4) == 0
    assert lib.kkt_tune_set(0, _lib.FP64, 512, 7, 16, 0, 4) == _lib.EINVAL
    assert lib.kkt_tune_set(0, _lib.BF16X6, 512, 7, 16, 0, 4) == _lib.EINVAL
    # wave counts must be even (each wave stays inside one half of the folded transform),
    # extents multiples of 32, at most 8 tiles per wave; widths 1, 2 or 4, and a width above 1
    # takes the shallow ring and at most 4 tiles per wave; more than 8 waves only as 16 waves
    # of at most two tiles with the shallow ring
    for bad in [(2, 0, 128, 4, 8, 0, 1), (0, 9, 128, 4, 8, 0, 1), (0, 0, 100, 4, 4, 0, 1),
                (0, 0, 128, 4, 3, 0, 1), (0, 0, 128, 4, 1, 0, 1), (0, 0, 16, 4, 2, 0, 1),
                (0, 0, 512, 4, 2, 0, 1), (0, 0, 128, 0, 8, 0, 1), (0, 0, 128, 4, 8, 2, 1),
                (0, 0, 128, 4, 8, 0, 3), (0, 0, 128, 4, 8, 1, 2), (0, 0, 512, 4, 4, 0, 2),
                (0, 0, 128, 4, 8, 0, 0), (0, 0, 768, 4, 16, 0, 1), (0, 0, 512, 4, 16, 0, 8),
                (0, 0, 512, 4, 16, 1, 1), (0, 0, 512, 4, 12, 0, 1), (0, 0, 1024, 4, 32, 0, 1),
                (0, 0, 384, 4, 16, 0, 1)]:
        assert lib.kkt_tune_set(*bad) == _lib.EINVAL, bad


def test_memory_plan_of_a_long_cycle(lib):
    # the unrestarted solves of the weak-scaling experiment keep up to 421 basis vectors
    p = _prob(nx=16, ny=16, nt=256, n_sub=16)
    b = ctypes.c_size_t()
    assert lib.kkt_memory_plan(ctypes.byref(p), 420, ctypes.byref(b)) == 0
    P = 15 * 15 * 256
    assert b.value >= (421 * 3 + 420) * P * 8


def test_memory_plan_grows_with_restart(lib):
    p = _prob(nx=128, ny=128, nt=256, n_sub=16)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.kkt_memory_plan(ctypes.byref(p), 0, ctypes.byref(a)) == 0
    assert lib.kkt_memory_plan(ctypes.byref(p), 30, ctypes.byref(b)) == 0
    P = 127 * 127 * 256
    # the basis holds 31 three-field vectors and 30 w-blocks in float64
    assert b.value - a.value >= (31 * 3 + 30) * P * 8
    assert lib.kkt_memory_plan(ctypes.byref(p), -1, ctypes.byref(b)) < 0


def test_null_arguments_are_rejected_without_a_device(lib):
    from paper_2305_04421_amd import _lib
    assert lib.kkt_create(None, None, None) == _lib.EINVAL
    assert lib.kkt_apply(None, None, None) == _lib.EINVAL
    assert lib.precond_apply(None, None, None) == _lib.EINVAL
    assert lib.kkt_size(None) == 0
    lib.kkt_destroy(None)
