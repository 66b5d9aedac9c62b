"""MI355X (gfx950) two-level time-domain-decomposition KKT solver.

Thin Python layer over libkktdd.so (include/kktdd.h): it checks tensor arguments and passes
device pointers; all arithmetic runs in the library's HIP kernels.  Tensors are torch.float64
on the current HIP device, laid out as in the header (u | z | w, time-node-major, x fastest).

    from paper_2305_04421_amd import KKTSolver, workloads
    params, recipe = workloads.config("grid128")
    with KKTSolver(params) as S:
        f = S.rhs(u0, utilde)
        x, stats = S.solve(f, restart=30, rtol=1e-8)
"""

import ctypes

from . import _lib
from ._lib import KKTDDError  # noqa: F401

__all__ = ["KKTSolver", "KKTDDError", "validate", "memory_plan", "kappa", "library_path", "solve_batched"]


def library_path():
    return _lib.LIB_PATH


def validate(params, precision="fp64", sweep="step"):
    """Host-only parameter check (no device); raises KKTDDError on a bad problem."""
    prob = _lib.make_problem(params, precision, sweep)
    _lib.check(_lib.load().kkt_validate(ctypes.byref(prob)), "kkt_validate")


def kappa(params):
    """Condition number of the sweeps' spatial block D_sigma (host-only)."""
    prob = _lib.make_problem(params, "fp64", "step")
    v = _lib.load().kkt_kappa(ctypes.byref(prob))
    if v < 0:
        raise _lib.KKTDDError(_lib.EINVAL, "kkt_kappa: invalid problem")
    return v


def memory_plan(params, precision="fp64", restart=0, sweep="step"):
    """Device bytes a handle (plus a Krylov basis of `restart` vectors) needs; host-only."""
    prob = _lib.make_problem(params, precision, sweep)
    out = ctypes.c_size_t(0)
    _lib.check(_lib.load().kkt_memory_plan(ctypes.byref(prob), int(restart), ctypes.byref(out)),
               "kkt_memory_plan")
    return out.value


def _ptr(t, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a torch.float64 tensor on the HIP device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class KKTSolver:
    """One problem handle on the current device and torch's current stream.

    precision: "fp64", "fp32", "bf16x6", "bf16x3", "bf16" (sweeps and their sine-transform
        GEMMs), or "auto" (float32 when the spatial block is well conditioned, else float64);
    sweep: "step" (a spatial solve at every sweep step) or "modal" (transforms hoisted).
    """

    def __init__(self, params, precision="fp64", stream=None, sweep="step"):
        import torch
        lib = _lib.load()
        self.params = dict(params)
        self.precision = precision
        self.sweep = sweep
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        prob = _lib.make_problem(params, precision, sweep)
        handle = ctypes.c_void_p()
        _lib.check(lib.kkt_create(ctypes.byref(prob), ctypes.c_void_p(self._stream.cuda_stream),
                                  ctypes.byref(handle)), "kkt_create")
        self._h = handle
        self.mx = params["nx"] - 1
        self.my = params["ny"] - 1
        self.nt = params["nt"]
        self.size = lib.kkt_size(self._h)
        # the precision the sweeps run in ("auto" resolved by the library)
        self.resolved_precision = _lib.PRECISION_NAMES[lib.kkt_precision(self._h)]

    # ---- lifetime -------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().kkt_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- entry points ----------------------------------------------------------------------
    def _new(self, n):
        import torch
        return torch.empty(n, dtype=torch.float64, device="cuda")

    def rhs(self, u0, utilde, out=None):
        f = self._new(self.size) if out is None else out
        nxy = self.mx * self.my
        _lib.check(_lib.load().kkt_rhs(self._h, _ptr(u0, nxy, "u0"), _ptr(utilde, nxy * self.nt, "utilde"),
                                       _ptr(f, self.size, "f")), "kkt_rhs")
        return f

    def apply(self, x, out=None):
        y = self._new(self.size) if out is None else out
        _lib.check(_lib.load().kkt_apply(self._h, _ptr(x, self.size, "x"), _ptr(y, self.size, "y")), "kkt_apply")
        return y

    def precond(self, r, out=None):
        z = self._new(self.size) if out is None else out
        _lib.check(_lib.load().precond_apply(self._h, _ptr(r, self.size, "r"), _ptr(z, self.size, "z")),
                   "precond_apply")
        return z

    def spatial_solve(self, b, shift, out=None):
        nxy = self.mx * self.my
        if b.numel() % nxy:
            raise ValueError("b must hold whole slices")
        ns = b.numel() // nxy
        x = self._new(b.numel()) if out is None else out
        _lib.check(_lib.load().kkt_spatial_solve(self._h, _ptr(b, ns * nxy, "b"), _ptr(x, ns * nxy, "x"),
                                                 ns, float(shift)), "kkt_spatial_solve")
        return x

    def profile(self, enable=True):
        """Start (clearing the counters) or stop the per-launch kernel timer."""
        _lib.check(_lib.load().kkt_profile(self._h, 1 if enable else 0), "kkt_profile")

    def profile_read(self):
        """{class: dict(ms, launches, bytes, flops)} summed over the launches timed so far."""
        out = {}
        for i, name in enumerate(_lib.KERNEL_CLASSES):
            ms, n, b, f = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            _lib.check(_lib.load().kkt_profile_read(self._h, i, ctypes.byref(ms), ctypes.byref(n),
                                                    ctypes.byref(b), ctypes.byref(f)), "kkt_profile_read")
            out[name] = dict(ms=ms.value, launches=n.value, bytes=b.value, flops=f.value)
        return out

    def residual_history(self):
        """Rotated residual estimates |g_{j+1}|/||f|| after every Arnoldi step of the last solve."""
        lib = _lib.load()
        n = _lib.check(lib.kkt_residual_history(self._h, None, 0), "kkt_residual_history")
        buf = (ctypes.c_double * max(n, 1))()
        _lib.check(lib.kkt_residual_history(self._h, buf, n), "kkt_residual_history")
        return list(buf[:n])

    def solve(self, f, x=None, restart=30, maxit=500, rtol=1e-8):
        """FGMRES(restart) from x (zero if None); returns (x, stats dict)."""
        import torch
        if x is None:
            x = torch.zeros(self.size, dtype=torch.float64, device="cuda")
        st = _lib.Stats()
        code = _lib.load().fgmres_solve(self._h, _ptr(f, self.size, "f"), _ptr(x, self.size, "x"),
                                        int(restart), int(maxit), float(rtol), ctypes.byref(st))
        _lib.check(code, "fgmres_solve")
        return x, st.as_dict()


def solve_batched(solvers, fs, xs=None, restart=30, maxit=500, rtol=1e-8):
    """Solve independent problems concurrently (kkt_solve_batched); returns (xs, [stats])."""
    import torch
    n = len(solvers)
    if len(fs) != n or (xs is not None and len(xs) != n):
        raise ValueError("solvers, fs and xs must have the same length")
    if xs is None:
        xs = [torch.zeros(S.size, dtype=torch.float64, device="cuda") for S in solvers]
    hs = (ctypes.c_void_p * n)(*[S._h.value for S in solvers])
    fp = (ctypes.c_void_p * n)(*[_ptr(f, S.size, "f").value for S, f in zip(solvers, fs)])
    xp = (ctypes.c_void_p * n)(*[_ptr(x, S.size, "x").value for S, x in zip(solvers, xs)])
    st = (_lib.Stats * n)()
    code = _lib.load().kkt_solve_batched(n, hs, fp, xp, int(restart), int(maxit), float(rtol), st)
    _lib.check(code, "kkt_solve_batched")
    return xs, [s.as_dict() for s in st]
