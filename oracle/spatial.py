"""Dirichlet spatial solve (oracle; test infrastructure only).

Every time step of a forward or adjoint sweep solves (s*I + dt*nu*A_h) x = b on one
slice.  The paper inverts this operator "with a direct solve" (Sec. 4).  Here the
direct solve is the discrete sine transform written out by its definition: the
vectors phi_pq(i,j) = sin(p*pi*i/nx) sin(q*pi*j/ny) are exact eigenvectors of the
5-point A_h with eigenvalues lambda^x_p + lambda^y_q,
    lambda^x_p = (4/dx^2) sin^2(p*pi/(2 nx)),  lambda^y_q = (4/dy^2) sin^2(q*pi/(2 ny)),
and the (nx-1)x(nx-1) matrix S_x[p,i] = sin(pi*p*i/nx) satisfies S_x S_x = (nx/2) I.
"""

import numpy as np

from .problem import Problem


def sine_matrix(n):
    """S[p-1, i-1] = sin(pi*p*i/n) for p, i = 1..n-1 (symmetric)."""
    idx = np.arange(1, n, dtype=np.float64)
    return np.sin(np.pi * np.outer(idx, idx) / n)


def laplacian_eigenvalues_1d(n, d):
    """(4/d^2) sin^2(p*pi/(2n)), p = 1..n-1: eigenvalues of the 1-D 3-point negative Laplacian."""
    p = np.arange(1, n, dtype=np.float64)
    return 4.0 / d ** 2 * np.sin(p * np.pi / (2.0 * n)) ** 2


def mode_eigenvalues(p: Problem):
    """lambda_pq of A_h on the (ny-1, nx-1) mode grid: [q-1, p-1] -> lambda^y_q + lambda^x_p."""
    lx = laplacian_eigenvalues_1d(p.nx, p.dx)
    ly = laplacian_eigenvalues_1d(p.ny, p.dy)
    return ly[:, None] + lx[None, :]


def dst2(p: Problem, x):
    """Forward 2-D sine transform of slices: xhat = S_y x S_x (no normalisation)."""
    return sine_matrix(p.ny) @ x @ sine_matrix(p.nx)


def idst2(p: Problem, xhat):
    """Inverse of dst2: x = (2/ny)(2/nx) S_y xhat S_x."""
    return (4.0 / (p.nx * p.ny)) * (sine_matrix(p.ny) @ xhat @ sine_matrix(p.nx))


def solve_diag_block(p: Problem, b, shift):
    """x = (shift*I + dt*nu*A_h)^{-1} b for every slice of b (..., ny-1, nx-1).

    Transform, divide each mode by shift + dt*nu*lambda_pq, transform back.
    """
    d = shift + p.dt * p.nu * mode_eigenvalues(p)
    return idst2(p, dst2(p, b) / d)
