"""FP64 CPU oracle for the two-level time-domain-decomposition KKT solve.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 implementation
of the method in Cyr, "A 2-Level Domain
Decomposition Preconditioner for KKT Systems with Heat-Equation Constraints"
(DD27, arXiv 2305.04421).  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it.  The HIP library never calls it and
it shares no code, tables or helpers with the HIP library.

Modules
-------
problem   -- problem parameters, derived constants, time subdomains (Sec. 2, Sec. 3)
operators -- 5-point A_h, J, L, K matvec, right-hand side (Eqs. (2)-(5))
spatial   -- Dirichlet spatial solve by the discrete sine transform (Sec. 4 "direct solve")
precond   -- RASQ fine level (Eq. (13)), Nicolaides coarse level (Eq. (14)),
             multiplicative two-level combination (Eq. (15)), block P (Eq. (7))
gmres     -- right-preconditioned restarted GMRES (Sec. 4)
direct    -- exact discrete solution: dense assembly on tiny grids and the
             per-sine-mode direct solve on any grid

Every floating point operation is float64.  Where the paper is silent or its
printed formula cannot be taken literally, the reading used is stated in the
docstring of the function that applies it.
"""

from .problem import Problem, subdomain_nodes, owned_nodes  # noqa: F401
