"""ctypes binding of libkktdd.so (argument marshalling only; every step runs in the HIP library).

The names follow include/kktdd.h.  Arrays are torch.float64 tensors on the HIP device; only
their data pointers cross the boundary.  The library is loaded on first use and its absence
is an error: there is no fallback path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkktdd.so")

# enum kktdd_status
OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, EBREAKDOWN = 0, 1, -1, -2, -3, -4
# enum kktdd_precision
FP64, FP32, BF16, BF16X3, BF16X6, AUTO = 0, 1, 2, 3, 4, 5
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16x3": BF16X3, "bf16x6": BF16X6, "auto": AUTO}
PRECISION_NAMES = {v: k for k, v in PRECISIONS.items()}
# enum kktdd_sweep
SWEEP_STEP, SWEEP_MODAL = 0, 1
SWEEPS = {"step": SWEEP_STEP, "modal": SWEEP_MODAL}
# variants of the method (ablations); the first value of each is the paper's method
VARIANTS = {
    "overlap_side": {"left": 0, "both": 1},
    "schwarz": {"ras": 0, "asm": 1},
    "local": {"rasq": 0, "exact": 1},
    "combine": {"coarse_first": 0, "fine_first": 1, "additive": 2},
}
# longest Arnoldi cycle of fgmres_solve
MAX_RESTART = 1024

EXPORTED = ("kkt_validate", "kkt_memory_plan", "kkt_create", "kkt_destroy", "kkt_size", "kkt_precision",
            "kkt_kappa", "kkt_tune_set", "kkt_tune_get", "kkt_rhs",
            "kkt_apply", "precond_apply", "kkt_spatial_solve", "kkt_spatial_solve_noalloc", "fgmres_solve", "kkt_solve_batched", "kkt_profile",
            "kkt_profile_read", "kkt_residual_history", "kkt_last_error")

# enum kktdd_kernel_class
KERNEL_CLASSES = ("matvec", "sweep_rows", "sweep_cols", "coarse", "arnoldi", "other")


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
                ("nt", ctypes.c_int32), ("T", ctypes.c_double),
                ("nu", ctypes.c_double), ("omega", ctypes.c_double),
                ("n_sub", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("coarse", ctypes.c_int32), ("precision", ctypes.c_int32), ("sweep", ctypes.c_int32),
                ("overlap_side", ctypes.c_int32), ("schwarz", ctypes.c_int32),
                ("local", ctypes.c_int32), ("combine", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("status", ctypes.c_int32), ("reorth", ctypes.c_int32),
                ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("relres_block", ctypes.c_double * 3), ("solve_s", ctypes.c_double),
                ("setup_s", ctypes.c_double)]

    def as_dict(self):
        return dict(iters=self.iters, restarts=self.restarts, status=self.status, reorth=self.reorth,
                    relres_est=self.relres_est, relres_true=self.relres_true,
                    relres_block=list(self.relres_block), solve_s=self.solve_s, setup_s=self.setup_s)


_lib = None


def load():
    """Load libkktdd.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_04421_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER(Problem)
    lib.kkt_validate.argtypes = [P]
    lib.kkt_memory_plan.argtypes = [P, i32, ctypes.POINTER(sz)]
    lib.kkt_create.argtypes = [P, vp, ctypes.POINTER(vp)]
    lib.kkt_destroy.argtypes = [vp]
    lib.kkt_destroy.restype = None
    lib.kkt_size.argtypes = [vp]
    lib.kkt_size.restype = sz
    lib.kkt_precision.argtypes = [vp]
    lib.kkt_precision.restype = ctypes.c_int
    lib.kkt_kappa.argtypes = [P]
    lib.kkt_kappa.restype = dbl
    lib.kkt_tune_set.argtypes = [i32] * 7
    lib.kkt_tune_get.argtypes = [i32] * 4 + [ctypes.POINTER(i32)] * 3
    lib.kkt_rhs.argtypes = [vp, vp, vp, vp]
    lib.kkt_apply.argtypes = [vp, vp, vp]
    lib.precond_apply.argtypes = [vp, vp, vp]
    lib.kkt_spatial_solve.argtypes = [vp, vp, vp, i32, dbl]
    lib.kkt_spatial_solve_noalloc.argtypes = [vp, vp, vp, i32, dbl]
    lib.fgmres_solve.argtypes = [vp, vp, vp, i32, i32, dbl, ctypes.POINTER(Stats)]
    lib.kkt_solve_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      i32, i32, dbl, ctypes.POINTER(Stats)]
    lib.kkt_profile.argtypes = [vp, ctypes.c_int]
    lib.kkt_profile_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.kkt_residual_history.argtypes = [vp, ctypes.POINTER(dbl), i32]
    lib.kkt_residual_history.restype = ctypes.c_int
    lib.kkt_last_error.argtypes = []
    lib.kkt_last_error.restype = ctypes.c_char_p
    for name in ("kkt_validate", "kkt_memory_plan", "kkt_create", "kkt_tune_set", "kkt_tune_get", "kkt_rhs", "kkt_apply",
                 "precond_apply", "kkt_spatial_solve", "kkt_spatial_solve_noalloc", "fgmres_solve", "kkt_solve_batched", "kkt_profile",
                 "kkt_profile_read"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def make_problem(params, precision="fp64", sweep="step"):
    """Problem struct from a parameter dict (keys nx, ny, nt, Lx, Ly, T, nu, omega, n_sub, overlap,
    coarse, and optionally the variant keys overlap_side, schwarz, local, combine)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    swp = SWEEPS[sweep] if isinstance(sweep, str) else int(sweep)
    return Problem(int(params["nx"]), int(params["ny"]), float(params.get("Lx", 1.0)),
                   float(params.get("Ly", 1.0)), int(params["nt"]), float(params.get("T", 1.0)),
                   float(params.get("nu", 1.0)), float(params.get("omega", 1e-2)),
                   int(params.get("n_sub", 1)), int(params.get("overlap", 1)),
                   int(params.get("coarse", 2)), prec, swp,
                   *[VARIANTS[key][params.get(key, next(iter(VARIANTS[key])))] for key in VARIANTS])


class KKTDDError(RuntimeError):
    def __init__(self, code, where):
        msg = load().kkt_last_error().decode(errors="replace")
        super().__init__(f"{where} returned {code}: {msg}")
        self.code = code


def check(code, where):
    if code < 0:
        raise KKTDDError(code, where)
    return code
