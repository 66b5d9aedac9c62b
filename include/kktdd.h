/*
 * kktdd.h -- C ABI of the MI355X (gfx950) two-level time-domain-decomposition KKT solver.
 *
 * Method: E. C. Cyr, "A 2-Level Domain Decomposition Preconditioner for KKT Systems with
 * Heat-Equation Constraints" (DD27, arXiv 2305.04421).
 *
 * The library solves the KKT system of Eq. (5),
 *     K = [[M_u, 0, J^T], [0, omega*M_z, L^T], [J, L, 0]],  unknowns (u, z, w),
 * that backward Euler in time and the 5-point stencil in space (Eq. (2)) produce for the
 * heat-equation-constrained control problem of Eq. (1), by flexible GMRES right-preconditioned
 * with P = diag(M_u, omega*M_z, S_hat) (Eq. (7)), where S_hat^{-1} is approximated by the
 * one-level RASQ time-subdomain sweeps of Eq. (13) combined multiplicatively with the
 * Nicolaides coarse time level of Eqs. (14)-(15).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid: nx, ny are grid INTERVALS on (0,Lx)x(0,Ly); the unknowns of one time-node are the
 *    (nx-1)*(ny-1) interior points (Sec. 2).  Time-nodes 1..nt carry unknowns (node 0 is the
 *    initial condition); dt = T/nt; the mass matrices are h*I with h = dt*(Lx/nx)*(Ly/ny).
 *  - Layout of a KKT vector (3*nt*(ny-1)*(nx-1) doubles, contiguous): field-major u | z | w;
 *    inside a field time-node-major (n = 1..nt), inside a slice row-major with x fastest:
 *        offset(f, n, j, i) = ((f*nt + n-1)*(ny-1) + j-1)*(nx-1) + i-1.
 *  - Every array argument is a DEVICE pointer to float64 data on the device the handle was
 *    created on, owned by the caller, and must not alias another argument unless stated.
 *  - Calls are ordered on the handle's HIP stream and return once the work is enqueued,
 *    except fgmres_solve and kkt_solve_batched, which synchronise before returning.
 *  - Return codes: KKTDD_OK (0), KKTDD_NOT_CONVERGED (1, x holds the last iterate), or a
 *    negative error; no C++ exception crosses this boundary.  kkt_last_error() gives a
 *    human-readable message for the last failing call of the calling thread.
 *  - Sign reading: J_hat = J + (dt/sqrt(omega)) I, i.e. the diagonal shift of Eq. (7) that
 *    enlarges J_hat's diagonal blocks (sigma = 1 + dt/sqrt(omega)).
 */
#ifndef KKTDD_H
#define KKTDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Longest Arnoldi cycle fgmres_solve takes: enough to run the unrestarted GMRES of the
 * experiments of Sec. 4 (at most 420 iterations) as a single cycle. */
#define KKTDD_MAX_RESTART 1024

enum kktdd_status {
  KKTDD_OK = 0,
  KKTDD_NOT_CONVERGED = 1, /* maxit reached; x holds the last iterate                        */
  KKTDD_EINVAL = -1,       /* parameter outside the method's domain (see kkt_validate)        */
  KKTDD_ENOMEM = -2,       /* the memory plan does not fit the device's free memory          */
  KKTDD_EHIP = -3,         /* a HIP runtime call failed (message in kkt_last_error)           */
  KKTDD_EBREAKDOWN = -4    /* non-finite residual or Hessenberg entry                         */
};

/* Arithmetic of the fine-level sweeps and their sine-transform GEMMs.  The KKT matvec, the
 * Krylov vectors, the coarse level and every reduction stay float64. */
enum kktdd_precision {
  KKTDD_FP64 = 0,   /* float64 MFMA                                                        */
  KKTDD_FP32 = 1,   /* float32 MFMA, float32 sweep state; float64 outer refinement          */
  KKTDD_BF16 = 2,   /* bfloat16 MFMA, float32 accumulation and sweep state                  */
  KKTDD_BF16X3 = 3, /* each float32 operand split into 2 bfloat16 parts, 3 part products    */
  KKTDD_BF16X6 = 4, /* each float32 operand split into 3 bfloat16 parts, 6 part products    */
  KKTDD_AUTO = 5    /* resolved by kkt_create: FP32 if kkt_kappa(prob) <= 500, else FP64    */
};

/* Placement of the spatial transforms in the fine-level sweeps.  Both compute the same
 * two-level Schur block (Eqs. (13)-(15)) up to rounding. */
enum kktdd_sweep {
  KKTDD_SWEEP_STEP = 0,  /* every sweep step is a spatial solve: 4 sine-transform GEMMs per
                            step, forward then adjoint, as the time integrator would do it     */
  KKTDD_SWEEP_MODAL = 1  /* transforms hoisted out of the time loop: one batched forward
                            transform of all slices, scalar recurrences per sine mode for the
                            coarse solve, residual and both sweeps, one inverse transform      */
};

/* Problem of Eq. (1) discretised as in Sec. 2, and the time decomposition of Sec. 3. */
typedef struct kktdd_problem {
  int32_t nx, ny;     /* grid intervals, >= 2                                              */
  double Lx, Ly;      /* domain extents, > 0                                               */
  int32_t nt;         /* time steps N_t, >= 1                                              */
  double T;           /* final time, > 0                                                   */
  double nu;          /* heat conductivity, > 0                                            */
  double omega;       /* regularisation parameter, > 0                                    */
  int32_t n_sub;      /* time subdomains N_D >= 1, must divide nt                         */
  int32_t overlap;    /* delta: nodes each subdomain extends to the left, 0..nt/n_sub      */
  int32_t coarse;     /* 0: one-level RASQ; 1: constant coarse basis; 2: constant+linear   */
  int32_t precision;  /* enum kktdd_precision                                              */
  int32_t sweep;      /* enum kktdd_sweep                                                  */
  /* Variants of the method for ablation studies (0 = the paper's method in every field).
   * Any nonzero variant needs sweep = KKTDD_SWEEP_MODAL and precision = KKTDD_FP64. */
  int32_t overlap_side; /* enum kktdd_overlap_side                                         */
  int32_t schwarz;      /* enum kktdd_schwarz                                              */
  int32_t local;        /* enum kktdd_local                                                */
  int32_t combine;      /* enum kktdd_combine                                              */
} kktdd_problem;

/* Subdomain extent (Sec. 3): delta nodes to the left (the paper's example), or to both sides. */
enum kktdd_overlap_side { KKTDD_OVERLAP_LEFT = 0, KKTDD_OVERLAP_BOTH = 1 };
/* Schwarz sum (Eqs. (9), (13)): restricted (R_s^T D_s, the paper) or additive (R_s^T). */
enum kktdd_schwarz { KKTDD_SCHWARZ_RAS = 0, KKTDD_SCHWARZ_ASM = 1 };
/* Local operator: the two sweeps of Eq. (13) (RASQ, the paper) or the exact local inverse
 * (R_s J_hat M_u^{-1} J_hat^T R_s^T)^{-1} of Eq. (9). */
enum kktdd_local { KKTDD_LOCAL_RASQ = 0, KKTDD_LOCAL_EXACT = 1 };
/* Two-level combination (Eq. (15)): coarse level first, then the fine level on the remaining
 * residual (the default reading); fine level first; or the sum of both. */
enum kktdd_combine { KKTDD_COMBINE_COARSE_FIRST = 0, KKTDD_COMBINE_FINE_FIRST = 1,
                     KKTDD_COMBINE_ADDITIVE = 2 };

typedef struct kktdd_stats {
  int32_t iters;          /* Arnoldi steps over all cycles                                 */
  int32_t restarts;       /* cycles after the first                                        */
  int32_t status;         /* return code of the solve                                      */
  int32_t reorth;         /* Arnoldi steps that needed a second Gram-Schmidt pass          */
  double relres_est;      /* Givens estimate |g_{j+1}| / ||f|| at exit                     */
  double relres_true;     /* ||f - K x|| / ||f|| at exit                                   */
  double relres_block[3]; /* per-block ||f_b - (K x)_b|| / ||f_b|| (u, z, w; 0 if f_b = 0) */
  double solve_s;         /* wall time of the solve                                        */
  double setup_s;         /* wall time of kkt_create for this handle: tables, coarse
                             factors, work buffers and the launch-shape measurements        */
} kktdd_stats;

typedef struct kktdd_handle kktdd_handle;

/* Host-only check of a problem description; touches no device.  Rules: nx, ny >= 2;
 * nt >= 1; Lx, Ly, T, nu, omega positive and finite; n_sub >= 1 dividing nt;
 * 0 <= overlap <= nt/n_sub; coarse in {0,1,2}; coarse == 2 needs nt/n_sub >= 2 (the linear
 * basis function of Eq. (14) is constant on a one-step subdomain); nx, ny <= 1024;
 * precision and sweep known.
 * Returns KKTDD_OK or KKTDD_EINVAL. */
int kkt_validate(const kktdd_problem* prob);

/* Device bytes kkt_create allocates for `prob`, plus what fgmres_solve adds for restart
 * length `restart` (0: creation only).  Host-only.  Returns KKTDD_OK or KKTDD_EINVAL. */
int kkt_memory_plan(const kktdd_problem* prob, int32_t restart, size_t* bytes);

/* Create a handle on the current HIP device: validate, check the memory plan against the
 * free device memory (KKTDD_ENOMEM before any allocation), build the sine and eigenvalue
 * tables and factor the coarse operator of every sine mode (Sec. 3, S_hat_0 = R_0 S_hat R_0^T).
 * `hip_stream` is a hipStream_t (NULL: the default stream).  On error *out is NULL. */
int kkt_create(const kktdd_problem* prob, void* hip_stream, kktdd_handle** out);

/* Release every device buffer of the handle (NULL is ignored).  Synchronises its stream. */
void kkt_destroy(kktdd_handle* h);

/* Number of KKT unknowns, 3*nt*(nx-1)*(ny-1); 0 for NULL. */
size_t kkt_size(const kktdd_handle* h);

/* The precision the handle's sweeps run in (KKTDD_AUTO resolved); KKTDD_EINVAL for NULL. */
int kkt_precision(const kktdd_handle* h);

/* Launch shapes of the sine-transform GEMM kernels (row kernel: kind 0, column kernel: kind 1)
 * for a padded extent (multiple of 32) and slice count, per precision: waves per workgroup
 * (even, at most 8, dividing extent/16 with at most 8 tiles per wave; or 16 with at most 2
 * tiles per wave, no deep ring and a width of at most 2 for KKTDD_FP64 and KKTDD_BF16X6, at
 * most 4 for the other precisions), a deep L2 prefetch ring (0/1), and the
 * width: blocks of 16 rows (row kernel) or 16 columns (column kernel) per workgroup, 1, 2 or
 * 4, each table fragment a wave loads serving all of them (width > 1: at most 4 tiles per
 * wave, no deep ring; a width whose workgroup would not fit the LDS, or whose column blocks do
 * not divide the x extent, runs as width 1).  kkt_create measures the candidates on its own
 * extents and keeps the fastest for the process (disable with KKTDD_AUTOTUNE=0;
 * KKTDD_TUNE_CACHE=<file> keeps them across processes, one JSON object per line).  Every
 * shape performs the same operations in the same order, so results do not depend on it;
 * neither do they on the workgroup placement (one XCD per slice when a launch's slices take
 * at most 8 MiB, else slices spread over the XCDs; KKTDD_XCD_MAP=0|1 forces it).
 * Host-only; set returns KKTDD_EINVAL for an invalid shape. */
int kkt_tune_set(int32_t kind, int32_t precision, int32_t extent, int32_t nslices, int32_t waves,
                 int32_t deep, int32_t width);
int kkt_tune_get(int32_t kind, int32_t precision, int32_t extent, int32_t nslices, int32_t* waves,
                 int32_t* deep, int32_t* width);

/* Condition number of the spatial block D_sigma = sigma*I + dt*nu*A_h of the preconditioner's
 * sweeps (Eq. (7) with the shift of Sec. 2), from the extreme sine-mode eigenvalues of A_h.
 * Float32 rounding in the sweeps is amplified by it.  Host-only; -1 for an invalid problem. */
double kkt_kappa(const kktdd_problem* prob);

/* Right-hand side of Eq. (5): f_u = h*utilde(t_n), f_z = 0, f_w = (u0, 0, ..., 0)
 * (Sec. 2: f carries the initial condition).
 * u0: (ny-1)*(nx-1) doubles, x fastest; utilde: nt slices, slice n-1 sampled at t_n = n*dt;
 * f: kkt_size doubles. */
int kkt_rhs(kktdd_handle* h, const double* u0, const double* utilde, double* f);

/* y = K x, the KKT matvec of Eq. (5) in float64.  x and y: kkt_size doubles; no aliasing. */
int kkt_apply(kktdd_handle* h, const double* x, double* y);

/* z = P^{-1} r for the block preconditioner of Eq. (7): z_u = r_u/h, z_z = r_z/(omega h),
 * z_w = S_2level^{-1} r_w (Eqs. (13)-(15); coarse = 0 gives the one-level RASQ).
 * r and z: kkt_size doubles; no aliasing. */
int precond_apply(kktdd_handle* h, const double* r, double* z);

/* x = D^{-1} b slice by slice, D = shift*I + dt*nu*A_h: the Dirichlet spatial solve done at
 * every step of a time sweep (Sec. 4 "direct solve"), as sine-transform GEMMs in the
 * handle's precision.  b, x: nslices*(ny-1)*(nx-1) doubles; may alias. */
int kkt_spatial_solve(kktdd_handle* h, const double* b, double* x, int32_t nslices, double shift);

/* Allocation-free variant of kkt_spatial_solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).  Same
 * operation, arguments and results as kkt_spatial_solve (bitwise), but its eigenvalue table and
 * work slices live in a fixed 64 MiB device array that the library holds per device until the
 * process ends (its address is resolved by kkt_create), it calls no hipMalloc or hipFree, and
 * it returns once the work is enqueued on the handle's stream (no synchronisation).
 * Limit: one padded eigenvalue table plus 2*nslices padded slices in the handle's sweep
 * element type (8 bytes for KKTDD_FP64, else 4) must fit 64 MiB; larger calls return
 * KKTDD_EINVAL with the limit in kkt_last_error.  All calls on one device share the array:
 * calls that overlap in time on one device (other streams or threads) race. */
int kkt_spatial_solve_noalloc(kktdd_handle* h, const double* b, double* x, int32_t nslices,
                              double shift);

/* Solve K x = f by flexible GMRES(restart) right-preconditioned with P (Sec. 4).  x holds the
 * initial guess on entry and the iterate on exit.  Stops at the first Arnoldi step whose
 * rotated residual estimate is <= rtol*||f||, confirmed by the true residual (a new cycle
 * starts otherwise), or after maxit Arnoldi steps (KKTDD_NOT_CONVERGED).  f = 0 returns x = 0.
 * 1 <= restart <= KKTDD_MAX_RESTART (31 with the KKTDD_ARNOLDI=cgs passes); the basis of
 * restart+1 vectors and restart stored w-blocks is allocated on first use of a longer cycle
 * (kkt_memory_plan gives its size).  `stats` may be NULL. */
int fgmres_solve(kktdd_handle* h, const double* f, double* x, int32_t restart, int32_t maxit,
                 double rtol, kktdd_stats* stats);

/* Solve n independent problems, each by fgmres_solve with the same restart, maxit and rtol.
 * hs: n distinct handles (grid sizes, nt and parameters may all differ); f[i], x[i]: device
 * vectors of kkt_size(hs[i]) doubles (x[i] is the initial guess, then the iterate).  The
 * problems run concurrently, each on a private stream ordered after the work already queued
 * on its handle's stream; the call returns when all are done.  stats: NULL or n entries.
 * Returns KKTDD_OK if every problem converged, KKTDD_NOT_CONVERGED if some did not, else the
 * most severe error (message names the problem). */
int kkt_solve_batched(int32_t n, kktdd_handle* const* hs, const double* const* f,
                      double* const* x, int32_t restart, int32_t maxit, double rtol,
                      kktdd_stats* stats);

/* Residual history of the handle's last fgmres_solve (or kkt_solve_batched member): the
 * rotated estimate |g_{j+1}| / ||f|| after every Arnoldi step, over all cycles (Sec. 4's
 * stopping quantity).  Copies min(count, cap) values to out (host memory) and returns the
 * count, or KKTDD_EINVAL for a NULL handle, cap < 0, or out NULL with cap > 0.  Host-only.
 * With the environment variable KKTDD_LOG=1 every solve also prints it to stderr. */
int kkt_residual_history(const kktdd_handle* h, double* out, int32_t cap);

/* Kernel classes of the per-launch timer below. */
enum kktdd_kernel_class {
  KKTDD_K_MATVEC = 0,      /* KKT matvec of Eq. (5), also the residual f - K x              */
  KKTDD_K_SWEEP_ROWS = 1,  /* row-block sine-transform GEMMs of the sweeps (Eq. (13))       */
  KKTDD_K_SWEEP_COLS = 2,  /* column-block sine-transform GEMMs of the sweeps               */
  KKTDD_K_COARSE = 3,      /* coarse level of Eqs. (14)-(15) and the residual r - S_hat c   */
  KKTDD_K_ARNOLDI = 4,     /* Gram-Schmidt passes and their reductions                      */
  KKTDD_K_OTHER = 5,       /* solution update, norms, block scalings, diagnostics           */
  KKTDD_K_COUNT = 6
};

/* Per-launch kernel timer.  enable != 0 clears the counters and brackets every later launch
 * made through this handle with HIP events on the handle's stream; enable == 0 stops
 * recording.  kkt_profile_read synchronises the stream and returns, for one class, the summed
 * event time in milliseconds, the launch count, and the algorithmic HBM bytes and flops of
 * those launches (bytes: vectors the kernels must read and write; flops: 2*m*m*m' per dense
 * product with the unpadded grid sizes).  Any pointer may be NULL. */
int kkt_profile(kktdd_handle* h, int enable);
int kkt_profile_read(kktdd_handle* h, int kclass, double* ms, int64_t* launches, double* bytes,
                     double* flops);

/* Message of the calling thread's last failing call ("" if none). */
const char* kkt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KKTDD_H */
