"""Block preconditioner and its two-level time-DD Schur approximation (oracle; test infrastructure only).

P = diag(M_u, omega*M_z, S_hat) with S_hat = J_hat M_u^{-1} J_hat^T (Eq. (7)).
S_hat^{-1} is approximated by the one-level RASQ preconditioner of Eq. (13)
combined multiplicatively with the Nicolaides coarse level of Eqs. (14)-(15).

J_hat is block lower bidiagonal with diagonal blocks D_sigma = sigma*I + dt*nu*A_h
and sub-diagonal blocks -I, so J_hat y = r is a forward sweep
y^n = D_sigma^{-1}(r^n + y^{n-1}) and J_hat^T x = b an adjoint sweep
x^n = D_sigma^{-1}(b^n + x^{n+1}).
"""

import numpy as np

from .problem import Problem, subdomain_nodes, owned_nodes
from .operators import apply_J, apply_JT
from .spatial import solve_diag_block, dst2, idst2, mode_eigenvalues


# ---- S_hat itself ------------------------------------------------------------------

def apply_S_hat(p: Problem, c):
    """S_hat c = (1/h) J_hat (J_hat^T c) (Eq. (7) with M_u = h*I)."""
    return apply_J(p, apply_JT(p, c, p.sigma), p.sigma) / p.h


# ---- one-level RASQ (Eq. (13)) -------------------------------------------------------

def forward_sweep(p: Problem, r, nodes):
    """Solve J_hat y = r restricted to `nodes` with a zero state before the first node.

    Returns {node: y^node}.  This is J_hat_s^{-1} of Eq. (13) applied to Q_s R_s^T r:
    the extra node W_s in front of the subdomain carries a zero right-hand side and a
    zero initial condition, so its value is zero and it drops out.
    """
    y, prev = {}, np.zeros(p.slice_shape)
    for n in nodes:
        prev = solve_diag_block(p, r[n - 1] + prev, p.sigma)
        y[n] = prev
    return y


def adjoint_sweep(p: Problem, b, nodes):
    """Solve J_hat^T x = b restricted to `nodes` with zero after the last node; returns {node: x^node}."""
    x, nxt = {}, np.zeros(p.slice_shape)
    for n in reversed(nodes):
        nxt = solve_diag_block(p, b[n] + nxt, p.sigma)
        x[n] = nxt
    return x


def exact_local_solve(p: Problem, r, nodes):
    """x = (R_s S_hat R_s^T)^{-1} R_s r on `nodes`: the local inverse of Eq. (9), with
    S_hat = J_hat M_u^{-1} J_hat^T = (1/h) J_hat J_hat^T.  Returns {node: x^node}.

    J_hat J_hat^T is block tridiagonal in time with blocks that are polynomials in A_h:
    D_sigma^2 + I on the diagonal (D_sigma^2 at node 1, which has no earlier step) and
    -D_sigma off it.  Every block is diagonal in the sine modes, so the restricted system
    splits into one tridiagonal system per mode (d = sigma + dt*nu*lambda_pq).
    """
    L = len(nodes)
    d = p.sigma + p.dt * p.nu * mode_eigenvalues(p)                  # (my, mx)
    rhat = np.stack([dst2(p, r[n - 1]) for n in nodes])               # (L, my, mx)
    T = np.zeros(d.shape + (L, L))
    for i, n in enumerate(nodes):
        T[..., i, i] = d * d + (1.0 if n >= 2 else 0.0)
        if i > 0:
            T[..., i, i - 1] = -d
            T[..., i - 1, i] = -d
    rhs = np.moveaxis(rhat, 0, -1)[..., None]                         # (my, mx, L, 1)
    xhat = np.moveaxis(np.linalg.solve(T / p.h, rhs)[..., 0], -1, 0)   # (L, my, mx)
    return {n: idst2(p, xhat[i]) for i, n in enumerate(nodes)}


def rasq(p: Problem, r):
    """One-level RASQ of Eq. (13): sum_s R_s^T D_s (J_hat_s^{-T} M_s J_hat_s^{-1}) R_s r.

    Per subdomain: forward sweep, scale by the mass h, adjoint sweep, keep the owned nodes.
    Variants: local == "exact" replaces the two sweeps by the local inverse of Eq. (9);
    schwarz == "asm" keeps every node of the subdomain (no partition of unity), so
    overlapping nodes receive the sum of their subdomains' values.
    """
    out = np.zeros(p.field_shape)
    for s in range(1, p.n_sub + 1):
        nodes = subdomain_nodes(p, s)
        if p.local == "exact":
            x = exact_local_solve(p, r, nodes)
        else:
            y = forward_sweep(p, r, nodes)
            hy = {n: p.h * y[n] for n in nodes}
            x = adjoint_sweep(p, hy, nodes)
        for n in (owned_nodes(p, s) if p.schwarz == "ras" else nodes):
            out[n - 1] += x[n]
    return out


# ---- Nicolaides coarse level (Eq. (14)) ---------------------------------------------

def coarse_time_basis(p: Problem):
    """Z_t: nt x (nb*N_D) time factor of the coarse basis Z = Z_t (x) I (Eq. (14)).

    Subdomain s contributes a constant column and (coarse == 2) a linear column, both
    supported on its owned nodes (D_s R_s^T Phi_s).  The linear column is
    -1 + 2 (n - (s-1)k)/k on owned node n.  Any other affine normalisation spans the
    same space, and the coarse correction Z (Z^T S Z)^{-1} Z^T depends only on that span.
    The basis acts on every spatial point separately (tensor product with the spatial
    identity), one coarse unknown per basis function and interior point.
    """
    nb = p.coarse
    Zt = np.zeros((p.nt, nb * p.n_sub))
    for s in range(1, p.n_sub + 1):
        for n in owned_nodes(p, s):
            Zt[n - 1, nb * (s - 1)] = 1.0
            if nb == 2:
                Zt[n - 1, nb * (s - 1) + 1] = -1.0 + 2.0 * (n - (s - 1) * p.k) / p.k
    return Zt


def lower_bidiagonal_gram(n, diag, sub):
    """G = J J^T for the n x n lower-bidiagonal J with constant diagonal `diag` and sub-diagonal `sub`.

    G[0,0] = diag^2, G[i,i] = diag^2 + sub^2 (i > 0), G[i,i-1] = G[i-1,i] = diag*sub.
    Sec. 3 shows this product for a forward-Euler step; for one sine mode of J_hat it is
    J_hat_lambda J_hat_lambda^T with diag = sigma + dt*nu*lambda and sub = -1.
    """
    J = np.diag(np.full(n, float(diag))) + np.diag(np.full(n - 1, float(sub)), -1)
    return J @ J.T


def coarse_operator_modes(p: Problem, q=None):
    """S_hat_0 = Z^T S_hat Z (Sec. 3) for every sine mode: array (ny-1, nx-1, nc, nc),
    or for the modes of row q only: (nx-1, nc, nc).

    In sine-mode space S_hat is block diagonal: mode lambda sees
    (1/h) T(d), T(d) = J_l J_l^T, J_l = lower bidiagonal(d, -1), d = sigma + dt*nu*lambda.
    T(d) = d^2 I + diag(0,1,..,1) - d (E + E^T) with E the sub-diagonal shift, so
    Z_t^T T(d) Z_t = d^2 G2 + G0 - d G1 with the three fixed Gram matrices below.
    """
    Zt = coarse_time_basis(p)
    nt = p.nt
    E = np.diag(np.ones(nt - 1), -1)
    G2 = Zt.T @ Zt
    G0 = Zt.T @ np.diag(np.r_[0.0, np.ones(nt - 1)]) @ Zt
    G1 = Zt.T @ (E + E.T) @ Zt
    d = p.sigma + p.dt * p.nu * mode_eigenvalues(p)
    if q is not None:
        d = d[q]
    d = d[..., None, None]
    return (d * d * G2 + G0 - d * G1) / p.h


def coarse_correction(p: Problem, r):
    """c = Z (Z^T S_hat Z)^{-1} Z^T r (the R_0^T S_hat_0^{-1} R_0 factor of Eq. (15)).

    Restrict (R_0 = Z^T sums over each subdomain's owned nodes), transform the coarse
    slices to sine modes, solve the small SPD system of every mode, transform back,
    prolong (Z = Z_t (x) I).
    """
    Zt = coarse_time_basis(p)
    r0 = np.einsum("nc,nyx->cyx", Zt, r)
    r0_hat = dst2(p, r0)
    c0_hat = np.empty_like(r0_hat)
    for q in range(p.my):                                       # one row of modes at a time
        S0 = coarse_operator_modes(p, q)                        # (mx, nc, nc)
        rhs = np.moveaxis(r0_hat[:, q, :], 0, -1)[..., None]    # (mx, nc, 1)
        c0_hat[:, q, :] = np.moveaxis(np.linalg.solve(S0, rhs)[..., 0], -1, 0)
    c0 = idst2(p, c0_hat)
    return np.einsum("nc,cyx->nyx", Zt, c0)


# ---- two-level combination (Eq. (15)) and the block preconditioner (Eq. (7)) --------

def schur_inverse(p: Problem, r):
    """Approximate S_hat^{-1} r.

    coarse == 0: one-level RASQ (Eq. (13)).
    coarse >= 1: Eq. (15) is printed as the product S_RASQ^{-1} R_0^T S_0^{-1} R_0, which
    has the rank of the coarse space and cannot precondition alone; the text calls the
    coarse solve "applied in a multiplicative way", read here as coarse first, then
    the fine level on the remaining residual:
        c = Q_0 r,  z = c + S_RASQ^{-1} (r - S_hat c),
    whose error propagator is (I - S_RASQ^{-1} S_hat)(I - Q_0 S_hat).
    Variants: combine == "fine_first" applies the fine level first,
        y = S_RASQ^{-1} r,  z = y + Q_0 (r - S_hat y),
    and combine == "additive" adds the two, z = Q_0 r + S_RASQ^{-1} r.
    """
    if p.coarse == 0:
        return rasq(p, r)
    if p.combine == "fine_first":
        y = rasq(p, r)
        return y + coarse_correction(p, r - apply_S_hat(p, y))
    if p.combine == "additive":
        return coarse_correction(p, r) + rasq(p, r)
    c = coarse_correction(p, r)
    return c + rasq(p, r - apply_S_hat(p, c))


def apply_Pinv(p: Problem, r, schur=None):
    """P^{-1} r for P = diag(M_u, omega*M_z, S_hat) of Eq. (7).

    The third block applies `schur` (default: the approximation schur_inverse above);
    tests pass the exact Schur complement here to check the block structure.
    """
    z = np.empty_like(r)
    z[0] = r[0] / p.h
    z[1] = r[1] / (p.omega * p.h)
    z[2] = (schur or (lambda v: schur_inverse(p, v)))(r[2])
    return z
