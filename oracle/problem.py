"""Problem parameters, derived constants and time subdomains (oracle; test infrastructure only).

Discretisation (Sec. 2, Eq. (2)): a Cartesian grid on (0,Lx)x(0,Ly) with nx, ny
*intervals*; the unknowns at each time-node are the interior points
i = 1..nx-1, j = 1..ny-1 (boundary values are zero and eliminated).  Time-nodes
run 0..nt with dt = T/nt; node 0 carries the initial condition and is not an
unknown, so u, z and w live on nodes 1..nt.  The mass matrices are
h*I with h = dt*dx*dy (Sec. 2, below Eq. (5)).

Readings where the paper is silent (all listed in the design notes):
  * sigma = 1 + dt/sqrt(omega) is the diagonal shift of J_hat (Eq. (7)), i.e.
    J_hat = J - omega^{-1/2} L with L = -dt*I, the sign that makes J_hat's
    diagonal block larger than J's (Pearson-Wathen); the literal sign would make
    J_hat's diagonal indefinite for small omega.
  * overlap delta extends each subdomain delta nodes to the LEFT; delta = 1 gives
    the paper's example {1,2,3},{3,4,5,6},{6,7,8,9} for nt=9, N_D=3 (Sec. 3).
  * the boolean partition of unity D_s gives each node to the subdomain whose own
    time steps end there: s owns (s-1)k+1 .. sk.

Variants of the method (ablations; the defaults are the paper's method):
  overlap_side  "left" (paper) | "both": the overlap also extends delta nodes to the right
  schwarz       "ras" (paper, R_s^T D_s) | "asm": additive Schwarz, R_s^T without D_s
  local         "rasq" (Eq. (13): two sweeps) | "exact": the local inverse of Eq. (9),
                (R_s J_hat M_u^{-1} J_hat^T R_s^T)^{-1}
  combine       "coarse_first" (the reading of Eq. (15)) | "fine_first" | "additive"
"""

from dataclasses import dataclass
import math


@dataclass(frozen=True)
class Problem:
    nx: int            # grid intervals in x; interior points per row nx-1
    ny: int            # grid intervals in y
    nt: int            # time steps N_t; time-nodes 0..nt
    Lx: float = 1.0
    Ly: float = 1.0
    T: float = 1.0
    nu: float = 1.0    # heat conductivity
    omega: float = 1e-2  # regularisation parameter
    n_sub: int = 1     # number of time subdomains N_D
    overlap: int = 1   # delta: extra time-nodes to the left of each subdomain
    coarse: int = 2    # 0: one-level RASQ; 1: constant coarse basis; 2: constant+linear (paper)
    overlap_side: str = "left"
    schwarz: str = "ras"
    local: str = "rasq"
    combine: str = "coarse_first"

    # ---- derived quantities -------------------------------------------------
    @property
    def mx(self):
        return self.nx - 1

    @property
    def my(self):
        return self.ny - 1

    @property
    def dx(self):
        return self.Lx / self.nx

    @property
    def dy(self):
        return self.Ly / self.ny

    @property
    def dt(self):
        return self.T / self.nt

    @property
    def h(self):
        """Mass-matrix scale: M_u = M_z = dt*dx*dy*I (Sec. 2, below Eq. (5))."""
        return self.dt * self.dx * self.dy

    @property
    def sigma(self):
        """Diagonal shift of J_hat's blocks: D_sigma = sigma*I + dt*nu*A_h (Eq. (7), sign reading above)."""
        return 1.0 + self.dt / math.sqrt(self.omega)

    @property
    def k(self):
        """Time steps per subdomain."""
        return self.nt // self.n_sub

    @property
    def slice_shape(self):
        return (self.my, self.mx)

    @property
    def field_shape(self):
        return (self.nt, self.my, self.mx)

    @property
    def size(self):
        """Number of KKT unknowns: three fields (u, z, w) on every interior point and time-node 1..nt."""
        return 3 * self.nt * self.my * self.mx

    def validate(self):
        """Raise ValueError for parameters outside the method's domain."""
        if self.nx < 2 or self.ny < 2:
            raise ValueError("nx and ny must be >= 2 (at least one interior point)")
        if self.nt < 1:
            raise ValueError("nt must be >= 1")
        for name in ("Lx", "Ly", "T", "nu", "omega"):
            v = getattr(self, name)
            if not (v > 0 and math.isfinite(v)):
                raise ValueError(f"{name} must be positive and finite")
        if self.n_sub < 1 or self.nt % self.n_sub != 0:
            raise ValueError("n_sub must be >= 1 and divide nt")
        if self.overlap < 0 or self.overlap > self.k:
            raise ValueError("overlap must satisfy 0 <= overlap <= nt/n_sub")
        if self.coarse not in (0, 1, 2):
            raise ValueError("coarse must be 0, 1 or 2")
        if self.coarse == 2 and self.k < 2:
            raise ValueError("a linear coarse basis needs at least 2 time steps per subdomain")
        if self.overlap_side not in ("left", "both"):
            raise ValueError("overlap_side must be 'left' or 'both'")
        if self.schwarz not in ("ras", "asm"):
            raise ValueError("schwarz must be 'ras' or 'asm'")
        if self.local not in ("rasq", "exact"):
            raise ValueError("local must be 'rasq' or 'exact'")
        if self.combine not in ("coarse_first", "fine_first", "additive"):
            raise ValueError("combine must be 'coarse_first', 'fine_first' or 'additive'")
        return self


def subdomain_nodes(p: Problem, s: int):
    """Time-nodes of subdomain s (1-based), Sec. 3: its own steps plus `overlap` earlier nodes
    (and, with overlap_side "both", `overlap` later nodes)."""
    first = max(1, (s - 1) * p.k + 1 - p.overlap)
    last = s * p.k if p.overlap_side == "left" else min(p.nt, s * p.k + p.overlap)
    return list(range(first, last + 1))


def owned_nodes(p: Problem, s: int):
    """Nodes kept by the partition of unity D_s (Eq. (9)): (s-1)k+1 .. sk."""
    return list(range((s - 1) * p.k + 1, s * p.k + 1))
