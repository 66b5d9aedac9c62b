"""Seeded synthetic workloads: problem parameters and sampled input data.

This module draws random numbers and samples closed-form functions on the grid;
it holds none of the solver's arithmetic.  Tests, the smoke check and the benchmark
feed the same arrays to the HIP library and to the CPU oracle.

Problem parameters are plain dicts with the keys
    nx, ny, nt, Lx, Ly, T, nu, omega, n_sub, overlap, coarse
(nx, ny are grid intervals; interior points per slice (nx-1)*(ny-1)).

Input data for one problem:
    u0      (ny-1, nx-1) float64: the initial condition at the interior points
    utilde  (nt, ny-1, nx-1) float64: the target at t_n = n*dt, n = 1..nt
Point (i, j) is x_i = i*Lx/nx, y_j = j*Ly/ny; index [n-1, j-1, i-1], x fastest.

Targets of the synthetic configurations: a sum of seeded sine modes
sin(p*pi*x/Lx) sin(q*pi*y/Ly) with (p, q) uniform on {1..min(16, n-1)} and N(0,1)
amplitudes, times exp(-t); optionally plus iid uniform noise.  The paper's own
experiment (Sec. 4) uses u0 = -x y (x-1)(y-2) and utilde = sin(2 pi t) sin(2 pi x) sin(2 pi y)
on (0,1)x(0,2), T = 1.
"""

import math

import numpy as np

DEFAULTS = dict(Lx=1.0, Ly=1.0, T=1.0, nu=1.0, omega=1e-2, n_sub=1, overlap=1, coarse=2)


def problem(**kw):
    """Complete a parameter dict with the defaults above."""
    d = dict(DEFAULTS)
    d.update(kw)
    return d


# ---- named configurations ------------------------------------------------------------

def config(name):
    """(params, data recipe) of a named workload.

    tiny32     32x32 intervals, nt=32, nu=1, omega=1e-2, 4 subdomains, overlap 2
    grid128    128x128, nt=256, nu=1, omega=1e-2 (grid128_w4: omega=1e-4), 16 subdomains, overlap 2
    grid256    256x256, nt=1024, nu=0.1, omega=1e-3, 64 subdomains, overlap 2, noisy target
    grid512    512x512, nt=2048, nu=1, omega=1e-4, 128 subdomains, overlap 4
    """
    table = {
        "tiny32": (problem(nx=32, ny=32, nt=32, nu=1.0, omega=1e-2, n_sub=4, overlap=2),
                   dict(seed=1, n_modes=8, noise=0.0)),
        "grid128": (problem(nx=128, ny=128, nt=256, nu=1.0, omega=1e-2, n_sub=16, overlap=2),
                    dict(seed=2, n_modes=8, noise=0.0)),
        "grid128_w4": (problem(nx=128, ny=128, nt=256, nu=1.0, omega=1e-4, n_sub=16, overlap=2),
                       dict(seed=2, n_modes=8, noise=0.0)),
        "grid256": (problem(nx=256, ny=256, nt=1024, nu=0.1, omega=1e-3, n_sub=64, overlap=2),
                    dict(seed=3, n_modes=16, noise=1e-3)),
        "grid512": (problem(nx=512, ny=512, nt=2048, nu=1.0, omega=1e-4, n_sub=128, overlap=4),
                    dict(seed=5, n_modes=32, noise=0.0)),
    }
    params, recipe = table[name]
    return dict(params), dict(recipe)


def paper_problem(nt, steps_per_sub, omega, coarse=2, overlap=1, n_points=17):
    """The experiment of Sec. 4: (0,1)x(0,2), T=1, n_points x n_points mesh points.

    nu is not stated in the paper; nu = 1 is used.
    """
    return problem(nx=n_points - 1, ny=n_points - 1, nt=nt, Lx=1.0, Ly=2.0, T=1.0, nu=1.0,
                   omega=omega, n_sub=nt // steps_per_sub, overlap=overlap, coarse=coarse)


def batch_uneven(count=64, seed=4):
    """Uneven batch: n from {64,96,128,192,256}, nt = 16*U{4..32}, nu log-uniform in [0.05, 1],
    omega log-uniform in [1e-4, 1e-1], nt/16 subdomains, overlap 2; problem i's data seed 4000+i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice([64, 96, 128, 192, 256]))
        nt = 16 * int(rng.integers(4, 33))
        nu = float(math.exp(rng.uniform(math.log(0.05), math.log(1.0))))
        omega = float(10.0 ** rng.uniform(-4.0, -1.0))
        out.append((problem(nx=n, ny=n, nt=nt, nu=nu, omega=omega, n_sub=nt // 16, overlap=2),
                    dict(seed=4000 + i, n_modes=8, noise=0.0)))
    return out


# ---- sampled data -------------------------------------------------------------------

def grid_coordinates(params):
    """Interior coordinates x_i = i*Lx/nx (i=1..nx-1), y_j, and time-nodes t_n = n*T/nt (n=1..nt)."""
    x = np.arange(1, params["nx"]) * (params["Lx"] / params["nx"])
    y = np.arange(1, params["ny"]) * (params["Ly"] / params["ny"])
    t = np.arange(1, params["nt"] + 1) * (params["T"] / params["nt"])
    return x, y, t


def sine_mode_data(params, seed, n_modes, noise=0.0):
    """u0 = sin(pi x/Lx) sin(pi y/Ly); utilde = exp(-t) * sum_k a_k sin(p_k pi x/Lx) sin(q_k pi y/Ly) [+ noise]."""
    x, y, t = grid_coordinates(params)
    Lx, Ly = params["Lx"], params["Ly"]
    rng = np.random.default_rng(seed)
    pmax = min(16, params["nx"] - 1)
    qmax = min(16, params["ny"] - 1)
    pk = rng.integers(1, pmax + 1, n_modes)
    qk = rng.integers(1, qmax + 1, n_modes)
    ak = rng.standard_normal(n_modes)
    spatial = np.zeros((y.size, x.size))
    for p, q, a in zip(pk, qk, ak):
        spatial += a * np.outer(np.sin(q * np.pi * y / Ly), np.sin(p * np.pi * x / Lx))
    utilde = np.exp(-t)[:, None, None] * spatial[None, :, :]
    if noise > 0.0:
        utilde = utilde + rng.uniform(-noise, noise, utilde.shape)
    u0 = np.outer(np.sin(np.pi * y / Ly), np.sin(np.pi * x / Lx))
    return np.ascontiguousarray(u0), np.ascontiguousarray(utilde)


def paper_data(params):
    """Sec. 4 data: u0 = -x y (x-1)(y-2), utilde = sin(2 pi t) sin(2 pi x) sin(2 pi y)."""
    x, y, t = grid_coordinates(params)
    X, Y = np.meshgrid(x, y)
    u0 = -X * Y * (X - 1.0) * (Y - 2.0)
    spatial = np.sin(2.0 * np.pi * X) * np.sin(2.0 * np.pi * Y)
    utilde = np.sin(2.0 * np.pi * t)[:, None, None] * spatial[None, :, :]
    return np.ascontiguousarray(u0), np.ascontiguousarray(utilde)


def data(params, recipe):
    """Sample the inputs of a (params, recipe) pair from config() or batch_uneven()."""
    return sine_mode_data(params, recipe["seed"], recipe["n_modes"], recipe.get("noise", 0.0))


def random_field(shape, seed):
    """iid N(0,1) float64 array, for operator-level parity cases."""
    return np.random.default_rng(seed).standard_normal(shape)
