// Nicolaides coarse time level (Sec. 3, Eq. (14)) and the multiplicative two-level residual.
//
// Coarse basis Z = Z_t (x) I: subdomain s (0-based, owned nodes s*k+1..(s+1)*k) has a
// constant function and, with two functions per subdomain, the linear one
// phi_1(n) = -1 + 2 (n - s*k)/k, both zero off its owned nodes.  Slot nb*s + b of a coarse
// vector holds one full slice (every interior point) for basis function b of subdomain s.
//
// In sine-mode space S_hat = J_hat M^{-1} J_hat^T is block diagonal: mode (q,p) sees
// (1/h) T(d) with d = sigma + dt*nu*(lam^y_q + lam^x_p) and T(d) = J_d J_d^T, J_d lower
// bidiagonal (d on the diagonal, -1 below).  Hence S_hat_0 = Z^T S_hat Z is, mode by mode,
// the small SPD band matrix (1/h)(d^2 G2 + G0 - d G1) with fixed Gram matrices
// G2 = Z_t^T Z_t, G0 = Z_t^T diag(0,1,..,1) Z_t, G1 = Z_t^T (E + E^T) Z_t (E: time shift),
// of half-bandwidth 2*nb - 1.  One thread factors / solves one mode.
#include "internal.h"

namespace kktdd {

namespace {

constexpr int kBlock = 256;

__device__ inline double phi1(int node, int s, int k) {
  return -1.0 + 2.0 * (double)(node - s * k) / (double)k;
}

// r0[nb*s + b][pt] = sum over owned nodes n of s of phi_b(n) * scale * r_w[n][pt]
__global__ void __launch_bounds__(kBlock)
k_restrict(Geom g, const double* __restrict__ rw, const double* __restrict__ dscale,
           double* __restrict__ r0) {
  const int pt = blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (pt >= g.nxy) return;
  double a0 = 0.0, a1 = 0.0;
  constexpr int kReg = 32;
  if (g.k <= kReg) {
    // the subdomain's values are loaded together, then summed in node order
    double v[kReg];
#pragma unroll
    for (int i = 0; i < kReg; ++i) v[i] = i < g.k ? rw[(long long)(s * g.k + i) * g.nxy + pt] : 0.0;
#pragma unroll
    for (int i = 0; i < kReg; ++i)
      if (i < g.k) {
        a0 += v[i];
        a1 += phi1(s * g.k + 1 + i, s, g.k) * v[i];
      }
  } else {
    for (int n = s * g.k + 1; n <= (s + 1) * g.k; ++n) {
      const double v = rw[(long long)(n - 1) * g.nxy + pt];
      a0 += v;
      a1 += phi1(n, s, g.k) * v;
    }
  }
  const double sc = dscale ? *dscale : 1.0;
  r0[(long long)(g.nb * s) * g.nxy + pt] = sc * a0;
  if (g.nb == 2) r0[(long long)(g.nb * s + 1) * g.nxy + pt] = sc * a1;
}

// Band storage of the Gram matrices: G[i*(hb+1) + b] = G(i, i-b), b = 0..hb.
// Factor: fac[(i*(hb+1) + b) * nmodes + mode] = L(i, i-b) (lower Cholesky factor) for b >= 1,
// and 1 / L(i, i) for b = 0 (the solves multiply by it).
__global__ void __launch_bounds__(kBlock)
k_coarse_factor(Geom g, const double* __restrict__ G2, const double* __restrict__ G0,
                const double* __restrict__ G1, const double* __restrict__ lamx,
                const double* __restrict__ lamy, double* __restrict__ fac, int* info) {
  const int mode = blockIdx.x * kBlock + threadIdx.x;
  const int nmodes = g.nxy;
  if (mode >= nmodes) return;
  // mode enumeration shared with k_coarse_solve: the live positions of the padded mode space
  const int q = mode_at(live_pos(mode / g.mx, g.my, g.My), g.My);
  const int p = mode_at(live_pos(mode % g.mx, g.mx, g.Mx), g.Mx);
  const double d = g.sigma + lamy[q] + lamx[p];   // tables hold dt*nu*lambda
  const int hb = 2 * g.nb - 1, w = hb + 1;
  const double invh = 1.0 / g.h;
  auto L = [&](int i, int j) -> double& { return fac[((long long)i * w + (i - j)) * nmodes + mode]; };
  for (int i = 0; i < g.nc; ++i) {
    const int j0 = i - hb > 0 ? i - hb : 0;
    for (int j = j0; j <= i; ++j) {
      const int b = i - j;
      double a = (d * d * G2[i * w + b] + G0[i * w + b] - d * G1[i * w + b]) * invh;
      for (int m = (i - hb > 0 ? i - hb : 0); m < j; ++m) {
        if (j - m > hb) continue;
        a -= L(i, m) * L(j, m);
      }
      if (j < i) {
        L(i, j) = a * L(j, j);   // L(j, j) holds the reciprocal diagonal
      } else {
        if (!(a > 0.0)) {
          *info = 1;
          a = 1.0;
        }
        L(i, i) = 1.0 / sqrt(a);
      }
    }
  }
}

// In-place solve of every mode's band system on padded sine-mode slices xhat[slot][q][p]:
// forward L y = r, then backward L^T c = y column by column (once c_i is known, its
// contributions L(i, i-b) c_i leave the pending values of rows i-1 .. i-hb), so both passes
// need only row i of the factor at step i.  Rows and right-hand sides come through a register
// ring kRing steps ahead of the chain, which runs through registers; the loads do not depend
// on it.
template <int NB>
__global__ void __launch_bounds__(64)
k_coarse_solve(Geom g, const double* __restrict__ fac, double* __restrict__ xhat) {
  constexpr int hb = 2 * NB - 1, w = hb + 1, kRing = 8;
  const int mode = blockIdx.x * 64 + threadIdx.x;
  const int nmodes = g.nxy;
  if (mode >= nmodes) return;
  const long long MM = g.padded();
  double* x = xhat + (long long)live_pos(mode / g.mx, g.my, g.My) * g.Mx + live_pos(mode % g.mx, g.mx, g.Mx);
  const double* Lm = fac + mode;
  const long long ld = nmodes;
  const int nc = g.nc;
  // row i of the factor: 1/L(i,i), then L(i,i-b), b = 1..hb, at Lm[(i*w + b)*ld]
  auto load_row = [&](int i, double (&row)[w]) {
#pragma unroll
    for (int b = 0; b < w; ++b) row[b] = (i >= 0 && i < nc) ? Lm[((long long)i * w + b) * ld] : 0.0;
  };
  auto load_x = [&](int i) { return (i >= 0 && i < nc) ? x[(long long)i * MM] : 0.0; };
  double ring[kRing][w], rv[kRing];

  // forward: y_i = (r_i - sum_b L(i,i-b) y_{i-b}) / L(i,i);  win[b] = y_{i-1-b}
  double win[hb];
#pragma unroll
  for (int b = 0; b < hb; ++b) win[b] = 0.0;
#pragma unroll
  for (int d = 0; d < kRing; ++d) {
    load_row(d, ring[d]);
    rv[d] = load_x(d);
  }
  for (int i0 = 0; i0 < nc; i0 += kRing) {
#pragma unroll
    for (int d = 0; d < kRing; ++d) {
      const int i = i0 + d;
      if (i >= nc) break;
      double a = rv[d];
#pragma unroll
      for (int b = 1; b <= hb; ++b)
        if (i - b >= 0) a -= ring[d][b] * win[b - 1];   // entries before row 0 are not stored
      const double y = a * ring[d][0];
      x[(long long)i * MM] = y;
#pragma unroll
      for (int b = hb - 1; b > 0; --b) win[b] = win[b - 1];
      win[0] = y;
      load_row(i + kRing, ring[d]);
      rv[d] = load_x(i + kRing);
    }
  }

  // backward: c_i = pend_i / L(i,i), then pend_{i-b} -= L(i,i-b) c_i.  cur = pend_i,
  // acc[b] = pend_{i-1-b}; the value entering the window at step i is y_{i-1-hb}.
  double cur = win[0], acc[hb];
#pragma unroll
  for (int b = 0; b < hb; ++b) acc[b] = b + 1 < hb ? win[b + 1] : load_x(nc - 1 - hb);
#pragma unroll
  for (int d = 0; d < kRing; ++d) {
    load_row(nc - 1 - d, ring[d]);
    rv[d] = load_x(nc - 2 - hb - d);
  }
  for (int i0 = nc - 1; i0 >= 0; i0 -= kRing) {
#pragma unroll
    for (int d = 0; d < kRing; ++d) {
      const int i = i0 - d;
      if (i < 0) break;
      const double c = cur * ring[d][0];
      x[(long long)i * MM] = c;
#pragma unroll
      for (int b = 1; b <= hb; ++b)
        if (i - b >= 0) acc[b - 1] -= ring[d][b] * c;
      cur = acc[0];
#pragma unroll
      for (int b = 0; b + 1 < hb; ++b) acc[b] = acc[b + 1];
      acc[hb - 1] = rv[d];
      load_row(i - kRing, ring[d]);
      rv[d] = load_x(i - 1 - hb - kRing);
    }
  }
}

// r'^n = scale*r_w^n - (S_hat c)^n, c^n = sum_b phi_b(n) c0[slot(n,b)] (prolongation Z c0).
// With g^n = (J_hat^T c)^n = D c^n - c^{n+1} and (J_hat g)^n = D g^n - g^{n-1}:
//     (S_hat c)^n = (1/h) (D^2 c^n - D c^{n+1} - [n>=2] (D c^{n-1} - c^n)),
// where D c and D^2 c are prolonged from the precomputed D c0 and D^2 c0 (Z commutes with D).
// One thread per interior point and subdomain marches over the subdomain's owned nodes.  The
// coarse slots of the subdomain (and the D c0 slots of its neighbours, needed at its first and
// last node) are loaded once, so the per-node work is one load of r_w and one store.
template <typename TO>
__global__ void __launch_bounds__(kBlock)
k_residual_prime(Geom g, const double* __restrict__ rw, const double* __restrict__ dscale,
                 const double* __restrict__ c0, const double* __restrict__ Dc0,
                 const double* __restrict__ DDc0, TO* __restrict__ rp) {
  const int pt = blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (pt >= g.nxy) return;
  const double sc = dscale ? *dscale : 1.0;
  const long long nxy = g.nxy;
  const int n0 = s * g.k + 1, n1 = (s + 1) * g.k;
  if (!c0) {
    for (int n = n0; n <= n1; ++n) {
      const long long e = (long long)(n - 1) * nxy + pt;
      rp[e] = (TO)(sc * rw[e]);
    }
    return;
  }
  const bool lin = g.nb == 2;
  auto slot = [&](const double* X, int sd, int b) { return X[(long long)(g.nb * sd + b) * nxy + pt]; };
  const double C0 = slot(c0, s, 0), C1 = lin ? slot(c0, s, 1) : 0.0;
  const double D0 = slot(Dc0, s, 0), D1 = lin ? slot(Dc0, s, 1) : 0.0;
  const double E0 = slot(DDc0, s, 0), E1 = lin ? slot(DDc0, s, 1) : 0.0;
  const bool hasP = s > 0, hasN = s + 1 < g.nd;
  const double P0 = hasP ? slot(Dc0, s - 1, 0) : 0.0, P1 = (hasP && lin) ? slot(Dc0, s - 1, 1) : 0.0;
  const double N0 = hasN ? slot(Dc0, s + 1, 0) : 0.0, N1 = (hasN && lin) ? slot(Dc0, s + 1, 1) : 0.0;
  const double invh = 1.0 / g.h;
  for (int n = n0; n <= n1; ++n) {
    const double ph = lin ? phi1(n, s, g.k) : 0.0;
    // (S_hat c)^n = (1/h) (D^2 c^n - D c^{n+1} - [n>=2] (D c^{n-1} - c^n)), prolonged from slots
    double Dnext = 0.0;
    if (n < n1) Dnext = D0 + (lin ? phi1(n + 1, s, g.k) : 0.0) * D1;
    else if (hasN) Dnext = N0 + (lin ? phi1(n + 1, s + 1, g.k) : 0.0) * N1;
    double Sc = (E0 + ph * E1) - Dnext;
    if (n >= 2) {
      double Dprev = 0.0;
      if (n > n0) Dprev = D0 + (lin ? phi1(n - 1, s, g.k) : 0.0) * D1;
      else if (hasP) Dprev = P0 + (lin ? phi1(n - 1, s - 1, g.k) : 0.0) * P1;
      Sc -= Dprev - (C0 + ph * C1);
    }
    const long long e = (long long)(n - 1) * nxy + pt;
    rp[e] = (TO)(sc * rw[e] - Sc * invh);
  }
}

}  // namespace

int launch_restrict(const Geom& g, const double* rw, const double* dscale, double* r0,
                    hipStream_t s) {
  const dim3 grid((g.nxy + kBlock - 1) / kBlock, g.nd);
  prof_begin(KKTDD_K_COARSE, s);
  hipLaunchKernelGGL(k_restrict, grid, dim3(kBlock), 0, s, g, rw, dscale, r0);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, 8.0 * g.P + 8.0 * g.nc * g.nxy, 0.0);
  return 0;
}

int launch_coarse_factor(const Geom& g, const double* G2, const double* G0, const double* G1,
                         const double* lamx, const double* lamy, double* fac, int* info,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_factor, dim3((g.nxy + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g,
                     G2, G0, G1, lamx, lamy, fac, info);
  KKT_HIP(hipGetLastError());
  return 0;
}

int launch_coarse_solve(const Geom& g, const double* fac, double* xhat, hipStream_t s) {
  prof_begin(KKTDD_K_COARSE, s);
  // 64-thread workgroups spread the (latency-bound) per-mode solves over more CUs
  const dim3 grid((g.nxy + 63) / 64), block(64);
  if (g.nb == 2)
    hipLaunchKernelGGL(k_coarse_solve<2>, grid, block, 0, s, g, fac, xhat);
  else
    hipLaunchKernelGGL(k_coarse_solve<1>, grid, block, 0, s, g, fac, xhat);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, 8.0 * g.nxy * g.nc * (2.0 * g.nb + 2.0), 0.0);
  return 0;
}

int launch_residual_prime(const Geom& g, const double* rw, const double* dscale,
                          const double* c0, const double* Dc0, const double* DDc0,
                          void* rprime, int f32, hipStream_t s) {
  prof_begin(KKTDD_K_COARSE, s);
  const dim3 grid((g.nxy + kBlock - 1) / kBlock, g.nd);
  if (f32)
    hipLaunchKernelGGL(k_residual_prime<float>, grid, dim3(kBlock), 0, s, g, rw, dscale, c0, Dc0, DDc0,
                       static_cast<float*>(rprime));
  else
    hipLaunchKernelGGL(k_residual_prime<double>, grid, dim3(kBlock), 0, s, g, rw, dscale, c0, Dc0, DDc0,
                       static_cast<double*>(rprime));
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, (f32 ? 12.0 : 16.0) * g.P, 0.0);
  return 0;
}

}  // namespace kktdd
