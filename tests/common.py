"""Shared parity metrics and operator-level cases of the tests (no GPU needed to import).

The KKT blocks differ in scale by many orders of magnitude: in P^{-1} r (Eq. (7)) the z block
r_z/(omega h) exceeds the Schur block z_w by 1e10 or more on the workloads here.  A relative
error taken over the whole vector therefore cannot see the Schur block, which is where the
sweeps, the sine-transform GEMMs and the coarse level act.  Every comparison of KKT vectors
below is made block by block, each block relative to its own scale.
"""

import numpy as np

from paper_2305_04421_amd import workloads as wl


def relerr(a, b):
    """max|a - b| / max|b| over the whole array (for single-block quantities)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def relerr_blocks(a, b):
    """Largest over the KKT blocks (the leading axis of length 3: u, z, w) of
    max|a_k - b_k| / max|b_k|.  A block of b that is exactly zero must be zero in a."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape and a.shape[0] == 3, (a.shape, b.shape)
    worst = 0.0
    for k in range(3):
        d = float(np.abs(a[k] - b[k]).max())
        s = float(np.abs(b[k]).max())
        worst = max(worst, d / s if s > 0 else (0.0 if d == 0 else np.inf))
    return worst


def relerr_blocks_2norm(a, b):
    """Largest over the KKT blocks of ||a_k - b_k||_2 / ||b_k||_2 (iterates of a solve)."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape and a.shape[0] == 3, (a.shape, b.shape)
    worst = 0.0
    for k in range(3):
        d = float(np.linalg.norm(a[k] - b[k]))
        s = float(np.linalg.norm(b[k]))
        worst = max(worst, d / s if s > 0 else (0.0 if d == 0 else np.inf))
    return worst


# Operator-level parity cases: ragged extents (padding inside the last tile), the degenerate
# one-node problem, full tiles with overlap = k, the tiny32 workload, long subdomains, and
# sweeps of 22 and 32 nodes.
CASES = {
    "tiny_ragged": wl.problem(nx=6, ny=5, nt=8, Lx=1.0, Ly=2.0, nu=0.7, omega=1e-2, n_sub=4, overlap=1, coarse=2),
    "ragged_tiles": wl.problem(nx=37, ny=21, nt=12, Lx=1.3, Ly=0.7, nu=0.3, omega=1e-3, n_sub=3, overlap=2, coarse=2),
    "degenerate": wl.problem(nx=2, ny=3, nt=1, nu=1.0, omega=1e-1, n_sub=1, overlap=0, coarse=0),
    "full_tiles_overlap_k": wl.problem(nx=129, ny=65, nt=16, Lx=1.0, Ly=0.5, nu=0.2, omega=1e-4, n_sub=4, overlap=4,
                                       coarse=1),
    "tiny32": wl.config("tiny32")[0],
    "long_subdomains": wl.problem(nx=10, ny=12, nt=80, Lx=1.0, Ly=2.0, nu=1.0, omega=1e-2, n_sub=2, overlap=1,
                                  coarse=2),
    # sweeps of 22 and 32 nodes (the longer register forms of the mode-space sweep), the
    # second with overlap = k
    "reg24": wl.problem(nx=9, ny=7, nt=80, Lx=1.0, Ly=0.8, nu=0.4, omega=1e-3, n_sub=4, overlap=2, coarse=2),
    "reg32_overlap_k": wl.problem(nx=7, ny=8, nt=64, Lx=0.9, Ly=1.1, nu=1.3, omega=1e-2, n_sub=4, overlap=16,
                                  coarse=2),
}
