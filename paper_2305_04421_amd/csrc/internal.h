// Internal declarations shared by the kernel files and the host driver of libkktdd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "kktdd.h"

namespace kktdd {

// ---------------------------------------------------------------------------------------
// Geometry of one problem, passed by value to kernels.
// A slice is (ny-1) x (nx-1) interior points, x fastest.  Sine-transform work buffers pad
// both extents (Mx, My; pad_extent) so every MFMA tile is full.  Along a transformed extent
// they hold sine modes in the folded order of mode_pos; along an untransformed one, the
// interior points followed by padding.  The half-transform tables and the eigenvalue tables
// are zero at padding positions, so padding modes stay zero; padding points are never read.
// ---------------------------------------------------------------------------------------
struct Geom {
  int mx, my;          // interior points per row / per column
  int Mx, My;          // padded extents (multiples of 16)
  int nt;              // time-nodes carrying unknowns
  int nxy;             // mx*my
  long long P;         // nt*nxy: points of one field
  double cx, cy;       // dt*nu/dx^2, dt*nu/dy^2
  double h;            // dt*dx*dy (mass scale)
  double omega, dt;
  double sigma;        // 1 + dt/sqrt(omega): J_hat's diagonal shift
  int nd, k, delta;    // time subdomains, steps per subdomain, overlap
  int L;               // sweep length k + delta (+ delta with overlap on both sides);
                       // subdomain 1 is padded with zero nodes in front
  int sym;             // overlap on both sides (enum kktdd_overlap_side)
  int asm_sum;         // additive Schwarz sum (enum kktdd_schwarz)
  int exact_local;     // exact local inverse of Eq. (9) (enum kktdd_local)
  int combine;         // two-level combination (enum kktdd_combine)
  int nb;              // coarse basis functions per subdomain (0, 1, 2)
  int nc;              // nb*nd coarse slots per point
  __host__ __device__ long long padded() const { return (long long)Mx * My; }
};

// Padded sine-transform extent.  The transforms are folded by parity: with n = m + 1
// intervals, sin(pi p (n-i)/n) = (-1)^(p+1) sin(pi p i/n), so mirrored points i and n-i enter
// the odd frequencies as a sum and the even ones as a difference, and each 1-D transform
// splits into two half-size products.  The padded extent M is twice a half extent H that holds
// the A = ceil(m/2) sums (or odd frequencies) in [0, H) and the B = floor(m/2) differences (or
// even frequencies) in [H, 2H).  H is a multiple of 16 (of 32 for the bfloat16 engines, which
// step k by 32), and the tile count t = M/16 splits evenly over the waves of a workgroup with
// every wave inside one half (t <= 8, or a multiple of 4 up to 32, or of 8 above).
inline int pad_extent(int m, bool bf16 = false) {
  int tb = ((m + 1) / 2 + 15) / 16;   // tiles per half
  if (bf16 && (tb & 1)) ++tb;
  if (2 * tb > 8) tb = (tb + 1) / 2 * 2;
  if (2 * tb > 32) tb = (tb + 3) / 4 * 4;
  return 32 * tb;
}

// Sine mode a (0-based; frequency a+1) sits at position mode_pos(a, M) of a padded extent M:
// odd frequencies in the first half, even ones in the second.  mode_at inverts it; a position
// whose mode_at is >= m is padding.
__host__ __device__ inline int mode_pos(int a, int M) { return (a & 1) * (M >> 1) + (a >> 1); }
__host__ __device__ inline int mode_at(int pos, int M) {
  const int H = M >> 1;
  return pos < H ? 2 * pos : 2 * (pos - H) + 1;
}
// The j-th non-padding position (j < m), in increasing order.
__host__ __device__ inline int live_pos(int j, int m, int M) {
  const int A = (m + 1) / 2;
  return j < A ? j : (M >> 1) + (j - A);
}

// Launch helpers report through this; the host driver converts to KKTDD_EHIP.
#define KKT_HIP(call)                                       \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return ::kktdd::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

int hip_fail(hipError_t e, const char* what, const char* file, int line);
int set_error(int code, const std::string& msg);

// Per-launch timing (enabled per handle through kkt_profile): no-ops unless the calling
// thread is inside an entry point of a handle whose timer is on.
void prof_begin(int kclass, hipStream_t s);
void prof_end(int kclass, hipStream_t s, double bytes, double flops);
long long prof_mark();                          // index of the next record (-1: timer off)
void prof_add_bytes(long long record, double bytes);

// ---- stencil.hip: KKT matvec, right-hand side, block scalings, D_sigma stencil ----------
// y = K [su*xu; sz*xz; sw*xw] (Eq. (5)); su and sz are further multiplied by the optional
// device scalar *dscale (nullptr: 1).  If f != nullptr, y = f - K x instead.
int launch_kkt_apply(const Geom& g, const double* xu, const double* xz, const double* xw,
                     double su, double sz, double sw, const double* dscale,
                     const double* f, double* yu, double* yz, double* yw, hipStream_t s);
int launch_rhs(const Geom& g, const double* u0, const double* ut, double* f, hipStream_t s);
// out = a*in (+ optional device scalar factor), n doubles
int launch_scale(long long n, const double* in, double a, const double* dscale, double* out,
                 hipStream_t s);
// out = (shift I + dt nu A_h) in on nslices unpadded slices
int launch_apply_D(const Geom& g, const double* in, double* out, int nslices, double shift,
                   hipStream_t s);

// ---- dst.hip: sine-transform GEMMs and the fine-level sweeps ---------------------------
int launch_spatial_solve(const Geom& g, int precision, const void* Sx, const void* Sy,
                         const void* invlam, const double* b, double* x, int nslices,
                         void* work1, void* work2, hipStream_t s);
// Fine-level RASQ sweeps of Eq. (13) for every subdomain: reads r' (nt slices, float64 for
// the float64 engine, else float32), writes z_w (nt slices) = c + x at owned nodes, c from the
// coarse slots c0 (nullptr: 0).
int launch_sweeps(const Geom& g, int precision, const void* Sx, const void* Sy,
                  const void* invlam, const void* rprime, const double* c0, double* zw,
                  void* Tbuf, void* Ubuf, void* Ybuf, hipStream_t s);
// Coarse sine transforms (float64): forward r0 (nc unpadded slices) -> rhat (padded), and
// inverse chat (padded) -> c0 (unpadded, with the 4/(nx ny) normalisation).
int launch_coarse_dst(const Geom& g, const double* Sx, const double* Sy, const double* r0,
                      double* rhat, double* tmp, hipStream_t s);
int launch_coarse_idst(const Geom& g, const double* Sx, const double* Sy, const double* chat,
                       double* c0, double* tmp, double norm, hipStream_t s);

// Batched 2-D sine transforms of nslices slices in the handle's precision (folded products;
// padded mode space in the order of mode_pos):
//   forward  out = S_y (scale*in) S_x   (in: unpadded float64 slices, or in32: float32 ones
//            for the reduced-precision engines; out, tmp: padded)
//   inverse  out = norm * S_y in S_x    (in, tmp: padded; out: unpadded float64 slices),
//            plus the coarse part Z c0 when c0 != nullptr (the slices are time-nodes 1..nt)
int launch_dst_forward(const Geom& g, int precision, const void* Sx, const void* Sy,
                       const double* in, const double* dscale, void* tmp, void* out, int nslices,
                       hipStream_t s, const float* in32 = nullptr);
int launch_dst_inverse(const Geom& g, int precision, const void* Sx, const void* Sy,
                       const void* in, void* tmp, double* out, int nslices, double norm,
                       const double* c0, hipStream_t s);

// ---- modal.hip: transform-hoisted Schur block (sine-mode space) --------------------------
// Autotuner: measure the launch shapes of the row and column kernels for this extent and
// slice count on two work buffers (each nslices padded slices) and keep the fastest.  With
// r' (nt slices in the sweep precision, zeroed) and the forward-sweep store, the row launches are timed as
// forward-sweep steps (reading r', storing y); else as plain chained products.
int launch_autotune(const Geom& g, int precision, const void* Sx, const void* Sy,
                    const void* invlam, void* bufA, void* bufB, int nslices, const void* rprime,
                    void* ybuf, hipStream_t s);

int tune_set(int kind, int precision, int extent, int nslices, int waves, int deep, int width);
int tune_get(int kind, int precision, int extent, int nslices, int* waves, int* deep, int* width);
// Counter that kkt_tune_set advances: work recorded with older launch shapes is stale.
int tune_generation();

int launch_modal_restrict(const Geom& g, int precision, const void* rhat, double* r0,
                          hipStream_t s);
int launch_modal_sweeps(const Geom& g, int precision, const void* rhat, const double* c0,
                        int sub_coarse, const double* lamx, const double* lamy, double* yscratch,
                        void* zhat, double* ext, hipStream_t s);
int launch_modal_asm_add(const Geom& g, const double* ext, double* zhat, hipStream_t s);
int launch_modal_residual(const Geom& g, const double* zhat, const double* lamx,
                          const double* lamy, double* rhat, hipStream_t s);
int launch_modal_prolong_add(const Geom& g, const double* c0, double* zhat, hipStream_t s);

// ---- coarse.hip: Nicolaides coarse level --------------------------------------------------
int launch_restrict(const Geom& g, const double* rw, const double* dscale, double* r0,
                    hipStream_t s);
// Factor the banded SPD coarse operator of every sine mode; band (nc x (bw+1)) Gram pieces.
int launch_coarse_factor(const Geom& g, const double* G2, const double* G0, const double* G1,
                         const double* lamx, const double* lamy, double* fac, int* info,
                         hipStream_t s);
int launch_coarse_solve(const Geom& g, const double* fac, double* xhat, hipStream_t s);
// r' = scale*r_w - S_hat c with c prolonged from c0; c0/Dc0/DDc0 may be nullptr (no coarse).
// Computed in float64 and stored as float32 (f32 != 0: the reduced-precision sweeps, which
// round it to float32 when they read it) or float64.
int launch_residual_prime(const Geom& g, const double* rw, const double* dscale,
                          const double* c0, const double* Dc0, const double* DDc0,
                          void* rprime, int f32, hipStream_t s);

// ---- krylov.hip: Arnoldi and vector kernels ------------------------------------------------
// Per-block partial sums of the raw products <V_i, w> for i < nv and, if want_norm, <w, w>
// at slot nv (the scales vinv are applied after the reduction).
int launch_multidot(long long n, const double* V, long long ldv, int nv, const double* vinv,
                    const double* w, int want_norm, double* partials, int nblocks,
                    hipStream_t s);
// w_out = w - sum_i coef[i] * vinv[i] * v_i, and partial sums of <v_i vinv[i], w_out> and
// <w_out, w_out>.  If gate != nullptr and *gate == 0 the kernel does nothing.
int launch_update_dot(long long n, const double* V, long long ldv, int nv, const double* vinv,
                      const double* coef, const double* w, double* wout, int want_dots,
                      double* partials, int nblocks, const int* gate, hipStream_t s);
int launch_reduce_partials(const double* partials, int nblocks, int nsums, double* out,
                           hipStream_t s);
// Arnoldi bookkeeping on the device (one thread): see krylov.hip.
int launch_arnoldi_finish(int j, const double* sums1, const double* sums2, const double* sums3,
                          int* gate, double* hcol, double* vinv, double eta, int stage,
                          hipStream_t s);
// x_f += sum_i yv[i] * fscale_f * vinv[i] * V_i,f for f = u, z; x_w += sum_i yw[i] * Zw_i.
int launch_update_solution(const Geom& g, const double* V, long long ldv, const double* Zw,
                           long long ldz, int nv, const double* yv, const double* yw,
                           const double* vinv, double su, double sz, double* x, hipStream_t s);
// DCGS2 Arnoldi (see krylov.hip): inner products, bookkeeping, combined update pass.
int launch_dcgs_dots(long long n, const double* V, long long ldv, int j, const double* Vc,
                     const double* W, double* partials, int nblocks, hipStream_t s);
int launch_dcgs_finish(int j, const double* sums, double* vinv, double* coef, double* rec,
                       int* gate, int stage, hipStream_t s);
int launch_dcgs_update(long long n, double* V, long long ldv, int j, const double* coef,
                       const int* gate, double* partials, int nblocks, hipStream_t s);
int launch_sumsq_blocks(const Geom& g, const double* r, double* partials, int nblocks,
                        hipStream_t s);

// ---- noalloc.hip: the allocation-free spatial solve ----------------------------------------
// Resolve the device address of the library's scratch array on `device` (current).
int noalloc_setup(int device);

// ---- per-launch timer ------------------------------------------------------------------
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;   // events are created once and reused
  size_t used = 0;
  struct Rec { int cls; size_t ev; double bytes, flops; };
  std::vector<Rec> recs;
  size_t open_ev = 0;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      pool.push_back(e);
    }
    return pool[used++];
  }
};

}  // namespace kktdd

// Handle of one problem (opaque in the C ABI): its geometry, stream, tables and buffers.
struct kktdd_handle {
  kktdd_problem prob{};
  kktdd::Geom g{};
  hipStream_t stream = nullptr;
  int device = 0;
  int elem = 8;                       // bytes per element of the sweep work buffers
  double setup_s = 0.0;               // wall time of kkt_create
  std::vector<double> history;        // residual estimates of the last fgmres_solve
  // Arnoldi steps recorded as HIP graphs, one per basis slot j (see run_step in api.hip)
  std::vector<hipGraphExec_t> graph_exec;
  std::vector<char> graph_ran;         // slot j has run eagerly once (its next run is captured)
  int graph_gen = 0;                   // tune_generation() the graphs were recorded under
  std::vector<void*> allocations;

  // tables: per extent the forward then inverse half-transform blocks (see dst.hip), and
  // the inverse eigenvalues in the folded mode order
  double *Sx64 = nullptr, *Sy64 = nullptr, *invlam64 = nullptr;
  float *Sx32 = nullptr, *Sy32 = nullptr, *invlam32 = nullptr;
  double *lamx = nullptr, *lamy = nullptr;     // dt*nu*lambda (unpadded)
  // per-step sweeps
  void *Tbuf = nullptr, *Ubuf = nullptr, *Ybuf = nullptr;
  void* rprime = nullptr;                      // r', P elements of the sweep precision
  // modal (transform-hoisted) sweeps
  void *Rhat = nullptr, *Mtmp = nullptr;
  double* Ysc = nullptr;
  double* ext = nullptr;                       // additive-Schwarz extension values
  // coarse
  double *r0 = nullptr, *c0 = nullptr, *Dc0 = nullptr, *DDc0 = nullptr;
  double *chat = nullptr, *ctmp = nullptr, *cfac = nullptr;
  // reductions
  double *partials = nullptr, *sums = nullptr;
  double* host_sums = nullptr;                 // pinned
  // Krylov basis and its bookkeeping, sized for restart length R (see krylov_small)
  int R = 0;
  double *V = nullptr, *Zw = nullptr;
  double *kpart = nullptr, *ksums = nullptr, *hcol = nullptr, *vinv = nullptr, *ydev = nullptr;
  int* gate = nullptr;
  double* host_hcol = nullptr;                 // pinned, KrylovSmall(R).host doubles
  kktdd::Prof prof;

  uint16_t *SxBF = nullptr, *SyBF = nullptr;  // three bfloat16 parts of each table (transposed blocks)

  // half-transform tables and eigenvalue table of the handle's GEMM engine
  const void* Sx() const {
    switch (prob.precision) {
      case KKTDD_FP64: return Sx64;
      case KKTDD_FP32: return Sx32;
      default: return SxBF;
    }
  }
  const void* Sy() const {
    switch (prob.precision) {
      case KKTDD_FP64: return Sy64;
      case KKTDD_FP32: return Sy32;
      default: return SyBF;
    }
  }
  const void* invlam() const {
    return prob.precision == KKTDD_FP64 ? (const void*)invlam64 : (const void*)invlam32;
  }
};

