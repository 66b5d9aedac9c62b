"""Right-preconditioned restarted GMRES (oracle; test infrastructure only).

Sec. 4 solves K u = f with right-preconditioned GMRES to a relative residual
tolerance.  The paper does not state the restart length, the norm or the starting
guess; here: restart length R, Euclidean norm of the full (u, z, w) residual
relative to ||f||, x0 given (zero by default), modified Gram-Schmidt Arnoldi with
Givens rotations (Saad, Iterative Methods for Sparse Linear Systems, Alg. 6.9 with
right preconditioning, Alg. 9.5 storing the preconditioned vectors).

Stopping rule: inside a cycle, stop at the first j whose rotated residual estimate
|g_{j+1}| <= rtol*||f||; then form x and check the true residual ||f - K x||; if it
is still above rtol*||f|| (rounding) a new cycle starts.  `maxit` counts Arnoldi
steps over all cycles.
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    restarts: int
    converged: bool
    relres_est: float
    relres_true: float
    history: list = field(default_factory=list)   # |g_{j+1}|/||f|| after every Arnoldi step


def gmres(apply_A, apply_Minv, f, x0=None, restart=30, maxit=300, rtol=1e-8):
    """Solve A x = f with right preconditioner M^{-1}: A M^{-1} t = f, x = M^{-1} t."""
    f = np.asarray(f, dtype=np.float64)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    fnorm = float(np.linalg.norm(f))
    if fnorm == 0.0:
        return GmresResult(np.zeros_like(f), 0, 0, True, 0.0, 0.0, [])
    tol = rtol * fnorm
    its, cycles, history = 0, 0, []
    est = float("inf")
    while True:
        r = f - apply_A(x)
        beta = float(np.linalg.norm(r))
        if beta <= tol:
            return GmresResult(x, its, max(cycles - 1, 0), True, est, beta / fnorm, history)
        if its >= maxit:
            return GmresResult(x, its, max(cycles - 1, 0), False, est, beta / fnorm, history)
        cycles += 1
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j_end = 0
        for j in range(restart):
            Z.append(apply_Minv(V[j]))
            w = apply_A(Z[j])
            for i in range(j + 1):                         # modified Gram-Schmidt
                H[i, j] = float(np.vdot(V[i], w))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):                             # previous rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, b = H[j, j], H[j + 1, j]
            rho = float(np.hypot(a, b))
            cs[j], sn[j] = (1.0, 0.0) if rho == 0.0 else (a / rho, b / rho)
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            est = abs(g[j + 1]) / fnorm
            history.append(est)
            j_end = j + 1
            breakdown = b == 0.0
            if not breakdown:
                V.append(w / b)
            if abs(g[j + 1]) <= tol or its >= maxit or breakdown:
                break
        # least-squares solution of the rotated (upper triangular) system
        y = np.zeros(j_end)
        for i in range(j_end - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:j_end], y[i + 1:j_end])) / H[i, i]
        for i in range(j_end):
            x = x + y[i] * Z[i]
