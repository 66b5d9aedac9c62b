"""Discrete operators of the KKT system (oracle; test infrastructure only).

Storage: a field is a float64 array of shape (nt, ny-1, nx-1): index [n-1, j-1, i-1]
holds the value at time-node n and interior point (x_i, y_j), x fastest.  A KKT
vector is an array of shape (3, nt, ny-1, nx-1) holding (u, z, w).

Sec. 2, Eq. (2): one backward-Euler step of the heat equation reads
    u^{n+1} - u^n + dt*nu*A_h u^{n+1} = dt*z^{n+1},
with A_h the 5-point negative Laplacian.  Moving everything to the left gives
Eq. (3) with blocks J_{n,n} = B = I + dt*nu*A_h, J_{n,n-1} = -I and L = -dt*I,
so the constraint rows of Eq. (4) are J u + L z = f with f = (u0, 0, ..., 0).
"""

import numpy as np

from .problem import Problem


def apply_Ah(p: Problem, x):
    """5-point negative Laplacian of Eq. (2) on every slice of x (..., ny-1, nx-1).

    (A_h x)_{ij} = (2x_ij - x_{i+1,j} - x_{i-1,j})/dx^2 + (2x_ij - x_{i,j+1} - x_{i,j-1})/dy^2,
    with zero values outside the interior (homogeneous Dirichlet data).
    """
    pad = [(0, 0)] * (x.ndim - 2) + [(1, 1), (1, 1)]
    xp = np.pad(x, pad)
    c = xp[..., 1:-1, 1:-1]
    east, west = xp[..., 1:-1, 2:], xp[..., 1:-1, :-2]
    north, south = xp[..., 2:, 1:-1], xp[..., :-2, 1:-1]
    return (2.0 * c - east - west) / p.dx ** 2 + (2.0 * c - north - south) / p.dy ** 2


def apply_diag_block(p: Problem, x, shift):
    """(shift*I + dt*nu*A_h) x slice by slice: shift=1 gives J's block B, shift=sigma J_hat's D_sigma."""
    return shift * x + p.dt * p.nu * apply_Ah(p, x)


def shift_back(x):
    """x^{n-1} at node n (zero at n = 1, where the initial condition was moved to f)."""
    out = np.zeros_like(x)
    out[1:] = x[:-1]
    return out


def shift_forward(x):
    """x^{n+1} at node n (zero at n = nt: nothing follows the last node)."""
    out = np.zeros_like(x)
    out[:-1] = x[1:]
    return out


# ---- the space-time blocks of Eq. (4)/(5) and of Eq. (7) --------------------------

def apply_J(p: Problem, u, shift=1.0):
    """(J u)^n = B u^n - u^{n-1}: Eq. (3) for every step; shift=sigma gives J_hat of Eq. (7)."""
    return apply_diag_block(p, u, shift) - shift_back(u)


def apply_JT(p: Problem, w, shift=1.0):
    """(J^T w)^n = B w^n - w^{n+1} (B is symmetric); shift=sigma gives J_hat^T."""
    return apply_diag_block(p, w, shift) - shift_forward(w)


def apply_L(p: Problem, z):
    """L z = -dt z (Eq. (2): the control enters the step as dt*z^{n+1} on the right)."""
    return -p.dt * z


def apply_K(p: Problem, x):
    """KKT matvec of Eq. (5): K = [[M_u, 0, J^T], [0, omega*M_z, L^T], [J, L, 0]], M = h*I."""
    u, z, w = x
    y = np.empty_like(x)
    y[0] = p.h * u + apply_JT(p, w)
    y[1] = p.omega * p.h * z + apply_L(p, w)   # L^T = L
    y[2] = apply_J(p, u) + apply_L(p, z)
    return y


def rhs(p: Problem, u0, utilde):
    """Right-hand side (f_u, f_z, f) of Eq. (5).

    f = (u0, 0, ..., 0): the initial condition moved to the right of the first step
    (Sec. 2, below Eq. (4)).  f_u = h*utilde(t_n) and f_z = 0 make the first two
    block rows the stationarity conditions of Eq. (1) with the objective's time and
    space integrals taken with the same weights as the mass matrices (the paper does
    not print f_u and f_z).
    u0: (ny-1, nx-1) samples of u_0; utilde: (nt, ny-1, nx-1) samples of the target at t_n = n*dt.
    """
    f = np.zeros((3,) + p.field_shape)
    f[0] = p.h * np.asarray(utilde, dtype=np.float64)
    f[2, 0] = np.asarray(u0, dtype=np.float64)
    return f


def objective(p: Problem, u, z, utilde):
    """Discrete objective of Eq. (1): 1/2 sum h|u - utilde|^2 + omega/2 sum h|z|^2."""
    return 0.5 * p.h * np.sum((u - utilde) ** 2) + 0.5 * p.omega * p.h * np.sum(z ** 2)
