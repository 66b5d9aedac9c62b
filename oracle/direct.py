"""Exact discrete KKT solutions by two routes independent of the iteration (oracle; test infrastructure only).

dense_* : assemble the matrices of Eqs. (2)-(7) with Kronecker products (tiny grids only)
          and solve with LAPACK.  This construction shares no code with operators.py.
modal_solve : every block of K commutes with the 2-D sine transform, so the KKT system
          splits into one 2*nt banded system per sine mode (any grid size).
modal_solve_modes : the same banded systems for a sample of modes (the largest grids).
"""

import numpy as np
import scipy.linalg

from .problem import Problem


# ---- dense assembly (Eqs. (2)-(5), (7)) ------------------------------------------------

def _second_difference(m, d):
    """(1/d^2) tridiag(-1, 2, -1) of size m: the 1-D part of the 5-point stencil of Eq. (2)."""
    return (2.0 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)) / d ** 2


def dense_Ah(p: Problem):
    """A_h on the flattened slice (index (j-1)*(nx-1) + (i-1), x fastest)."""
    Ax = _second_difference(p.mx, p.dx)
    Ay = _second_difference(p.my, p.dy)
    return np.kron(np.eye(p.my), Ax) + np.kron(Ay, np.eye(p.mx))


def dense_J(p: Problem, shift=1.0):
    """J of Eq. (4): block diagonal shift*I + dt*nu*A_h, block sub-diagonal -I (shift=sigma: J_hat)."""
    nxy = p.mx * p.my
    blk = shift * np.eye(nxy) + p.dt * p.nu * dense_Ah(p)
    return np.kron(np.eye(p.nt), blk) - np.kron(np.eye(p.nt, k=-1), np.eye(nxy))


def dense_K(p: Problem):
    """The KKT matrix of Eq. (5) with M_u = M_z = h*I and L = -dt*I."""
    n = p.nt * p.mx * p.my
    I = np.eye(n)
    J = dense_J(p)
    L = -p.dt * I
    Z = np.zeros((n, n))
    return np.block([[p.h * I, Z, J.T], [Z, p.omega * p.h * I, L.T], [J, L, Z]])


def dense_schur(p: Problem):
    """Exact Schur complement S = J M_u^{-1} J^T + omega^{-1} L M_z^{-1} L^T (Eq. (6))."""
    J = dense_J(p)
    n = J.shape[0]
    return (J @ J.T + (p.dt ** 2 / p.omega) * np.eye(n)) / p.h


def dense_schur_hat(p: Problem):
    """S_hat = J_hat M_u^{-1} J_hat^T of Eq. (7)."""
    Jh = dense_J(p, p.sigma)
    return Jh @ Jh.T / p.h


def dense_solve(p: Problem, f):
    """Solve K x = f densely; f and the result have shape (3, nt, ny-1, nx-1)."""
    x = np.linalg.solve(dense_K(p), np.asarray(f, dtype=np.float64).reshape(-1))
    return x.reshape((3,) + p.field_shape)


# ---- per-sine-mode direct solve ----------------------------------------------------------

def _sine(n):
    idx = np.arange(1, n, dtype=np.float64)
    return np.sin(np.pi * np.outer(idx, idx) / n)


def _mode_band(p: Problem):
    """Band storage of one mode's system (see modal_solve) with the diagonal left to fill."""
    nt, h, dt = p.nt, p.h, p.dt
    c = dt * dt / (p.omega * h)
    N = 2 * nt
    # band storage ab[2 + i - j, j] = A[i, j] (two sub- and two super-diagonals);
    # every mode has the same pattern, only the diagonal d0 changes.
    ab = np.zeros((5, N))
    iu = 2 * np.arange(nt)        # row/column of u_n: constraint row d0 u_n - u_{n-1} - c w_n
    iw = iu + 1                   # row/column of w_n: adjoint row h u_n + d0 w_n - w_{n+1}
    ab[4, iu[:-1]] = -1.0         # A[iu_n, iu_{n-1}]
    ab[1, iw] = -c                # A[iu_n, iw_n]
    ab[3, iu] = h                 # A[iw_n, iu_n]
    ab[0, iw[1:]] = -1.0          # A[iw_n, iw_{n+1}]
    return ab


def _eigenvalues(p: Problem):
    lx = 4.0 / p.dx ** 2 * np.sin(np.arange(1, p.nx) * np.pi / (2 * p.nx)) ** 2
    ly = 4.0 / p.dy ** 2 * np.sin(np.arange(1, p.ny) * np.pi / (2 * p.ny)) ** 2
    return lx, ly


def _solve_mode(p: Problem, ab, lam, u0_coef, ut_coef):
    """(u_n, w_n) sine coefficients of one mode with eigenvalue lam of A_h."""
    ab[2, :] = 1.0 + p.dt * p.nu * lam
    b = np.zeros(2 * p.nt)
    b[0] = u0_coef
    b[1::2] = p.h * ut_coef
    sol = scipy.linalg.solve_banded((2, 2), ab, b)
    return sol[0::2], sol[1::2]


def modal_solve(p: Problem, u0, utilde):
    """Exact solution of K x = f for f = (h*utilde, 0, (u0, 0, ...)), mode by mode.

    With d0 = 1 + dt*nu*lambda_pq the rows of Eq. (5) for one mode read
        h u_n + d0 w_n - w_{n+1}        = h utilde_n
        omega*h z_n - dt w_n            = 0
        d0 u_n - u_{n-1} - dt z_n       = u0 * [n == 1]
    Eliminating z_n = dt w_n/(omega h) leaves a banded system in (u_n, w_n), ordered
    (u_1, w_1, u_2, w_2, ...), solved with LAPACK's banded LU.
    """
    Sx, Sy = _sine(p.nx), _sine(p.ny)
    nrm = 4.0 / (p.nx * p.ny)
    ut_hat = Sy @ np.asarray(utilde, dtype=np.float64) @ Sx     # (nt, my, mx)
    u0_hat = Sy @ np.asarray(u0, dtype=np.float64) @ Sx
    lx, ly = _eigenvalues(p)
    ab = _mode_band(p)
    uh = np.empty((p.nt, p.my, p.mx))
    wh = np.empty((p.nt, p.my, p.mx))
    for q in range(p.my):
        for pp in range(p.mx):
            uh[:, q, pp], wh[:, q, pp] = _solve_mode(p, ab, ly[q] + lx[pp], u0_hat[q, pp],
                                                     ut_hat[:, q, pp])
    u = nrm * (Sy @ uh @ Sx)
    w = nrm * (Sy @ wh @ Sx)
    z = p.dt * w / (p.omega * p.h)
    return np.stack([u, z, w])


def sine_coefficients(p: Problem, v, modes):
    """2-D sine coefficients of a field v (shape (..., ny-1, nx-1)) at the listed modes.

    Mode (q, pm), 0-based, has the coefficient sum_{j,i} sin(pi (q+1)(j+1)/ny) v[..., j, i]
    sin(pi (pm+1)(i+1)/nx); a field equals (4/(nx ny)) times the inverse transform of its
    coefficients.  Returns shape (len(modes),) + v.shape[:-2].
    """
    v = np.asarray(v, dtype=np.float64)
    j = np.arange(1, p.ny)
    i = np.arange(1, p.nx)
    out = []
    for q, pm in modes:
        sy = np.sin(np.pi * (q + 1) * j / p.ny)
        sx = np.sin(np.pi * (pm + 1) * i / p.nx)
        out.append(np.einsum("...ji,j,i->...", v, sy, sx))
    return np.array(out)


def modal_solve_modes(p: Problem, u0, utilde, modes):
    """Sine coefficients of the exact solution of K x = f (f as in modal_solve) at the listed
    modes only: shape (len(modes), 3, nt) for (u, z, w).  Each mode costs one banded solve,
    so the exact solution can be sampled on grids too large for modal_solve."""
    lx, ly = _eigenvalues(p)
    ab = _mode_band(p)
    u0c = sine_coefficients(p, u0, modes)
    utc = sine_coefficients(p, utilde, modes)
    out = np.empty((len(modes), 3, p.nt))
    for k, (q, pm) in enumerate(modes):
        uh, wh = _solve_mode(p, ab, ly[q] + lx[pm], u0c[k], utc[k])
        out[k, 0] = uh
        out[k, 1] = p.dt * wh / (p.omega * p.h)
        out[k, 2] = wh
    return out
