// Transform-hoisted Schur block: the two-level preconditioner of Eqs. (13)-(15) applied in
// sine-mode space.
//
// Every operator of the Schur block commutes with the 2-D sine transform: D_sigma becomes the
// scalar d = sigma + dt*nu*(lam^y_q + lam^x_p) on mode (q,p), J_hat a lower-bidiagonal
// (d, -1) recurrence in time, S_hat = (1/h) J_hat J_hat^T the tridiagonal
// (1/h) tridiag(-d; d^2 + [n>=2]; -d), and the coarse basis Z = Z_t (x) I acts on each mode
// separately.  So with r_hat = S_y r S_x (all nt slices at once, one batched GEMM pair):
//     restrict   r0_hat[s,b] = sum over owned n of phi_b(n) r_hat[n]
//     coarse     c0_hat = S_hat_0(d)^{-1} r0_hat             (band Cholesky per mode)
//     residual   r'_hat = r_hat - S_hat c_hat, c_hat^n = sum_b phi_b(n) c0_hat[s(n),b]
//     sweeps     y_j = (r'_j + y_{j-1})/d, x_j = (h y_j + x_{j+1})/d   (per subdomain)
//     output     z_hat^n = c_hat^n + x^n on owned nodes
// and z = (4/(nx ny)) S_y z_hat S_x (one batched GEMM pair).  The result equals the per-step
// sweeps up to rounding; only the placement of the transforms differs.
#include "internal.h"

namespace kktdd {

namespace {

constexpr int kBlock = 256;
constexpr int kRegSteps = 32;   // sweep lengths up to this keep the forward states in registers

__device__ inline double phi1m(int node, int s, int k) {
  return -1.0 + 2.0 * (double)(node - s * k) / (double)k;
}

// coarse restriction in mode space: r0[nb*s + b][q*Mx + p] (float64, padded layout)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_modal_restrict(Geom g, const T* __restrict__ rhat, double* __restrict__ r0) {
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (m >= MM) return;
  double a0 = 0.0, a1 = 0.0;
  for (int n = s * g.k + 1; n <= (s + 1) * g.k; ++n) {
    const double v = (double)rhat[(long long)(n - 1) * MM + m];
    a0 += v;
    a1 += phi1m(n, s, g.k) * v;
  }
  r0[(long long)(g.nb * s) * MM + m] = a0;
  if (g.nb == 2) r0[(long long)(g.nb * s + 1) * MM + m] = a1;
}

// prolonged coarse value c_hat^n of one mode (0 outside 1..nt)
__device__ inline double chat_at(const Geom& g, const double* __restrict__ c0, long long MM,
                                 long long m, int node) {
  if (node < 1 || node > g.nt) return 0.0;
  const int s = (node - 1) / g.k;
  const double* c = c0 + (long long)(g.nb * s) * MM + m;
  double v = c[0];
  if (g.nb == 2) v += phi1m(node, s, g.k) * c[MM];
  return v;
}

// One thread = one sine mode of one subdomain: residual, forward sweep, adjoint sweep,
// owned-node output.  Padded modes write zeros.
template <typename T, bool REG>
__global__ void __launch_bounds__(kBlock)
k_modal_sweep(Geom g, const T* __restrict__ rhat, const double* __restrict__ c0,
              const double* __restrict__ lamx, const double* __restrict__ lamy,
              double* __restrict__ yscratch, T* __restrict__ zhat) {
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (m >= MM) return;
  const int q = (int)(m / g.Mx), p = (int)(m % g.Mx);
  const int first = s * g.k + 1 - g.delta;
  if (q >= g.my || p >= g.mx) {
    for (int n = s * g.k + 1; n <= (s + 1) * g.k; ++n) zhat[(long long)(n - 1) * MM + m] = (T)0;
    return;
  }
  const double d = g.sigma + lamy[q] + lamx[p];
  const double invd = 1.0 / d, invh = 1.0 / g.h;
  double yreg[REG ? kRegSteps : 1];
  double* ysc = REG ? nullptr : yscratch + ((long long)s * g.L) * MM + m;
  // forward sweep over the subdomain's nodes (zero right-hand side below node 1)
  double y = 0.0;
  for (int j = 0; j < g.L; ++j) {
    const int n = first + j;
    double r = 0.0;
    if (n >= 1) {
      r = (double)rhat[(long long)(n - 1) * MM + m];
      if (c0) {
        // (S_hat c)^n = (1/h) ((d^2 + [n>=2]) c^n - d c^{n-1} [n>=2] - d c^{n+1})
        const double cn = chat_at(g, c0, MM, m, n);
        double sc = d * d * cn - d * chat_at(g, c0, MM, m, n + 1);
        if (n >= 2) sc += cn - d * chat_at(g, c0, MM, m, n - 1);
        r -= sc * invh;
      }
    }
    y = (r + y) * invd;
    if (REG) {
#pragma unroll
      for (int i = 0; i < kRegSteps; ++i)
        if (i == j) yreg[i] = y;
    } else {
      ysc[(long long)j * MM] = y;
    }
  }
  // adjoint sweep with the mass scale, output on owned nodes
  double x = 0.0;
  for (int j = g.L - 1; j >= 0; --j) {
    double yj = 0.0;
    if (REG) {
#pragma unroll
      for (int i = 0; i < kRegSteps; ++i)
        if (i == j) yj = yreg[i];
    } else {
      yj = ysc[(long long)j * MM];
    }
    x = (g.h * yj + x) * invd;
    if (j >= g.delta) {
      const int n = first + j;
      const double c = c0 ? chat_at(g, c0, MM, m, n) : 0.0;
      zhat[(long long)(n - 1) * MM + m] = (T)(c + x);
    }
  }
}

template <typename T>
int modal_t(const Geom& g, const void* rhat, const double* c0, const double* lamx,
            const double* lamy, double* yscratch, void* zhat, hipStream_t s) {
  const long long MM = g.padded();
  const dim3 grid((unsigned)((MM + kBlock - 1) / kBlock), g.nd);
  prof_begin(KKTDD_K_COARSE, s);
  if (g.L <= kRegSteps)
    hipLaunchKernelGGL((k_modal_sweep<T, true>), grid, dim3(kBlock), 0, s, g,
                       static_cast<const T*>(rhat), c0, lamx, lamy, yscratch, static_cast<T*>(zhat));
  else
    hipLaunchKernelGGL((k_modal_sweep<T, false>), grid, dim3(kBlock), 0, s, g,
                       static_cast<const T*>(rhat), c0, lamx, lamy, yscratch, static_cast<T*>(zhat));
  KKT_HIP(hipGetLastError());
  // read r_hat over the subdomain nodes, write z_hat once
  const double el = sizeof(T);
  prof_end(KKTDD_K_COARSE, s, el * MM * ((double)g.nd * g.L + g.nt), 0.0);
  return 0;
}

}  // namespace

int launch_modal_restrict(const Geom& g, int precision, const void* rhat, double* r0,
                          hipStream_t s) {
  const long long MM = g.padded();
  const dim3 grid((unsigned)((MM + kBlock - 1) / kBlock), g.nd);
  prof_begin(KKTDD_K_COARSE, s);
  if (precision != KKTDD_FP64)
    hipLaunchKernelGGL((k_modal_restrict<float>), grid, dim3(kBlock), 0, s, g,
                       static_cast<const float*>(rhat), r0);
  else
    hipLaunchKernelGGL((k_modal_restrict<double>), grid, dim3(kBlock), 0, s, g,
                       static_cast<const double*>(rhat), r0);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, (precision != KKTDD_FP64 ? 4.0 : 8.0) * MM * g.nt + 8.0 * MM * g.nc, 0.0);
  return 0;
}

int launch_modal_sweeps(const Geom& g, int precision, const void* rhat, const double* c0,
                        const double* lamx, const double* lamy, double* yscratch, void* zhat,
                        hipStream_t s) {
  if (precision != KKTDD_FP64) return modal_t<float>(g, rhat, c0, lamx, lamy, yscratch, zhat, s);
  return modal_t<double>(g, rhat, c0, lamx, lamy, yscratch, zhat, s);
}

}  // namespace kktdd
