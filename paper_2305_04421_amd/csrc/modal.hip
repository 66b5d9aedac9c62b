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
//
// The variants of the method (ablations) run here, in float64:
//   overlap on both sides   the sweep also covers delta nodes after the owned ones
//   additive Schwarz        non-owned outputs go to extension slots and are added to
//                           their owners by a second kernel (fixed order)
//   exact local inverse     Eq. (9): the restricted tridiagonal (1/h) T solved by LDL^T per
//                           mode instead of the two sweeps
//   fine first / additive   two-level combinations other than coarse first: the sweeps see
//                           r itself; fine first then forms r - S_hat y in mode space,
//                           restricts, solves and adds the prolonged correction
#include "internal.h"

namespace kktdd {

namespace {

constexpr int kBlock = 256;
constexpr int kRegSteps = 32;   // sweep lengths up to this keep the forward states in registers

__device__ inline double phi1m(int node, int s, int k) {
  return -1.0 + 2.0 * (double)(node - s * k) / (double)k;
}

// coarse restriction in mode space: r0[nb*s + b][q*Mx + p] (float64, padded layout).  With
// k <= R the subdomain's values are loaded together (unconditionally, the node index clamped
// to the last owned node; entries past k are not used), then summed in node order.
template <typename T, int R>
__global__ void __launch_bounds__(kBlock)
k_modal_restrict(Geom g, const T* __restrict__ rhat, double* __restrict__ r0) {
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (m >= MM) return;
  double a0 = 0.0, a1 = 0.0;
  if (R > 0) {
    double v[R > 0 ? R : 1];
#pragma unroll
    for (int i = 0; i < R; ++i)
      v[i] = (double)rhat[(long long)(s * g.k + (i < g.k ? i : g.k - 1)) * MM + m];
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (i < g.k) {
        a0 += v[i];
        a1 += phi1m(s * g.k + 1 + i, s, g.k) * v[i];
      }
  } else {
    for (int n = s * g.k + 1; n <= (s + 1) * g.k; ++n) {
      const double v = (double)rhat[(long long)(n - 1) * MM + m];
      a0 += v;
      a1 += phi1m(n, s, g.k) * v;
    }
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

// Node ranges of subdomain s (0-based): owned nodes s*k+1 .. (s+1)*k; the sweep covers
// first .. last, first = s*k+1-delta (slot 0 of the forward store), last = (s+1)*k
// (+ delta with overlap on both sides), both clipped to 1..nt.  Nodes left of the owned
// range map to extension slots 0..delta-1, nodes right of it to slots delta..2*delta-1.
struct Range {
  int own_lo, own_hi, first, lo, hi;
};
__device__ inline Range node_range(const Geom& g, int s) {
  Range r;
  r.own_lo = s * g.k + 1;
  r.own_hi = (s + 1) * g.k;
  r.first = r.own_lo - g.delta;
  r.lo = r.first < 1 ? 1 : r.first;
  const int last = r.own_hi + (g.sym ? g.delta : 0);
  r.hi = last > g.nt ? g.nt : last;
  return r;
}

// r'_n of one mode: r_hat_n, minus (S_hat c_hat)_n / h when the coarse correction comes first
//   (S_hat c)^n = (1/h) ((d^2 + [n>=2]) c^n - d c^{n-1} [n>=2] - d c^{n+1})
template <typename T>
__device__ inline double rprime_at(const Geom& g, const T* __restrict__ rhat,
                                   const double* __restrict__ c0, int sub, double d, long long MM,
                                   long long m, int n) {
  double r = (double)rhat[(long long)(n - 1) * MM + m];
  if (c0 && sub) {
    const double cn = chat_at(g, c0, MM, m, n);
    double sc = d * d * cn - d * chat_at(g, c0, MM, m, n + 1);
    if (n >= 2) sc += cn - d * chat_at(g, c0, MM, m, n - 1);
    r -= sc / g.h;
  }
  return r;
}

// Output of node n of subdomain s: owned nodes get c_hat + x, the others (additive Schwarz)
// go to the extension slots, which a second kernel adds to their owners.
template <typename T>
__device__ inline void put_out(const Geom& g, const Range& rg, const double* __restrict__ c0,
                               long long MM, long long m, int s, int n, double x,
                               T* __restrict__ zhat, double* __restrict__ ext) {
  if (n >= rg.own_lo && n <= rg.own_hi) {
    const double c = c0 ? chat_at(g, c0, MM, m, n) : 0.0;
    zhat[(long long)(n - 1) * MM + m] = (T)(c + x);
  } else if (ext) {
    const int E = g.delta * (1 + g.sym);
    const int slot = n < rg.own_lo ? n - rg.first : g.delta + (n - rg.own_hi - 1);
    ext[((long long)s * E + slot) * MM + m] = x;
  }
}

// Every lane of the wave gets the value that lane `lane` holds (a wave-uniform result).
__device__ inline double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

template <int W>
__device__ inline double pick(const double (&a)[W], int j) {
  double r = a[0];
#pragma unroll
  for (int t = 1; t < W; ++t) r = j == t ? a[t] : r;
  return r;
}

// One thread = one sine mode of one subdomain whose sweep covers at most R nodes: residual,
// forward sweep, adjoint sweep, output, with the states in registers.  Every load is issued
// before any arithmetic and none sits under a branch, so they are all in flight together:
//   - R values of r_hat, the node index clamped to the sweep's last node (entries past the
//     sweep are loaded but not used);
//   - with the coarse level (W > 0), the coarse values of the W subdomains s-W/2 .. s+W/2
//     (clamped to 0..nd-1), which own every node lo-1 .. hi+1 the residual and the output read:
//     W = 3 when delta < k, 5 when delta = k.
// The owner slot and linear basis value of node lo-1+i sit in lane i of every wave (all lanes
// active) and are read back as wave-uniform values, so c_hat of a node is one select chain
// and one multiply-add, recomputed where it is used rather than held through the sweeps
// (with R <= 24 the kernel then fits four waves per SIMD).  `sub` subtracts S_hat c_hat / h
// from r_hat (coarse level first); with W > 0 the output adds c_hat on owned nodes either
// way.  Padded modes compute on an in-range eigenvalue entry and write zeros.  The padded mode
// count is a multiple of the workgroup size, so every thread has a mode.
template <typename T, int R, int W>
__global__ void __launch_bounds__(kBlock, (W > 0 && R <= 24) ? 4 : 1)
k_modal_sweep_reg(Geom g, const T* __restrict__ rhat, const double* __restrict__ c0, int sub,
                  const double* __restrict__ lamx, const double* __restrict__ lamy,
                  T* __restrict__ zhat, double* __restrict__ ext) {
  static_assert(R + 2 <= 64, "the node table needs a lane per node");
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  const Range rg = node_range(g, s);
  const int cnt = rg.hi - rg.lo + 1;
  int tslot = -1;
  double tphi = 0.0;
  if constexpr (W > 0) {
    const int node = rg.lo - 1 + (int)__lane_id();
    if (node >= 1 && node <= g.nt) {
      const int o = (node - 1) / g.k;
      tslot = o - s + W / 2;
      if (g.nb == 2) tphi = phi1m(node, o, g.k);
    }
  }
  const int q = mode_at((int)(m / g.Mx), g.My), p = mode_at((int)(m % g.Mx), g.Mx);
  const bool pad = q >= g.my || p >= g.mx;
  const double d = g.sigma + lamy[pad ? 0 : q] + lamx[pad ? 0 : p];
  const double invd = 1.0 / d;
  double v[R];
#pragma unroll
  for (int i = 0; i < R; ++i)
    v[i] = (double)rhat[(long long)(rg.lo - 1 + (i < cnt ? i : cnt - 1)) * MM + m];
  // c_hat of node lo-1+i, recomputed where it is used (the same operations every time)
  double ca[W > 0 ? W : 1], cb[W > 0 ? W : 1];
  if constexpr (W > 0) {
#pragma unroll
    for (int j = 0; j < W; ++j) {
      int o = s - W / 2 + j;
      o = o < 0 ? 0 : (o >= g.nd ? g.nd - 1 : o);
      ca[j] = c0[(long long)(g.nb * o) * MM + m];
      cb[j] = c0[(long long)(g.nb * o + g.nb - 1) * MM + m];
    }
  }
  const bool lin = g.nb == 2;
  auto chat = [&](int i) -> double {
    if constexpr (W > 0) {
      const int j = __builtin_amdgcn_readlane(tslot, i);
      const double ph = lane_value(tphi, i);
      const double a = pick<W>(ca, j);
      const double c = lin ? a + ph * pick<W>(cb, j) : a;
      return j < 0 ? 0.0 : c;
    } else {
      return 0.0;
    }
  };
  if constexpr (W > 0) {
    if (sub) {
      double cm = chat(0), cn = chat(1);
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (i < cnt) {
          // (S_hat c)^n h = (d^2 + [n>=2]) c^n - d c^{n+1} - [n>=2] d c^{n-1}, n = lo + i
          const double cp = chat(i + 2);
          double sc = d * d * cn - d * cp;
          if (rg.lo + i >= 2) sc += cn - d * cm;
          v[i] -= sc / g.h;
          cm = cn;
          cn = cp;
        }
    }
  }
  double y = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i)
    if (i < cnt) {
      y = (v[i] + y) * invd;
      v[i] = y;
    }
  double x = 0.0;
#pragma unroll
  for (int i = R - 1; i >= 0; --i)
    if (i < cnt) {
      x = (g.h * v[i] + x) * invd;
      v[i] = x;
    }
  const int E = g.delta * (1 + g.sym);
#pragma unroll
  for (int i = 0; i < R; ++i)
    if (i < cnt) {
      const int n = rg.lo + i;
      if (n >= rg.own_lo && n <= rg.own_hi) {
        zhat[(long long)(n - 1) * MM + m] = pad ? (T)0 : (T)(chat(i + 1) + v[i]);
      } else if (ext && !pad) {
        const int slot = n < rg.own_lo ? n - rg.first : g.delta + (n - rg.own_hi - 1);
        ext[((long long)s * E + slot) * MM + m] = v[i];
      }
    }
}

// One thread = one sine mode of one subdomain: residual, forward sweep, adjoint sweep,
// output, for sweeps longer than the register form takes; the forward states go to a
// float64 store.  Padded modes write zeros on their owned nodes.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_modal_sweep(Geom g, const T* __restrict__ rhat, const double* __restrict__ c0, int sub,
              const double* __restrict__ lamx, const double* __restrict__ lamy,
              double* __restrict__ yscratch, T* __restrict__ zhat, double* __restrict__ ext) {
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (m >= MM) return;
  const int q = mode_at((int)(m / g.Mx), g.My), p = mode_at((int)(m % g.Mx), g.Mx);
  const Range rg = node_range(g, s);
  if (q >= g.my || p >= g.mx) {
    for (int n = rg.own_lo; n <= rg.own_hi; ++n) zhat[(long long)(n - 1) * MM + m] = (T)0;
    return;
  }
  const double d = g.sigma + lamy[q] + lamx[p];
  const double invd = 1.0 / d;
  double* ysc = yscratch + ((long long)s * g.L) * MM + m;
  // forward sweep over the subdomain's nodes (zero state before the first)
  double y = 0.0;
  for (int n = rg.lo; n <= rg.hi; ++n) {
    y = (rprime_at(g, rhat, c0, sub, d, MM, m, n) + y) * invd;
    ysc[(long long)(n - rg.first) * MM] = y;
  }
  // adjoint sweep with the mass scale (zero state after the last node)
  double x = 0.0;
  for (int n = rg.hi; n >= rg.lo; --n) {
    x = (g.h * ysc[(long long)(n - rg.first) * MM] + x) * invd;
    put_out(g, rg, c0, MM, m, s, n, x, zhat, ext);
  }
}

// Exact local inverse of Eq. (9) for one sine mode of one subdomain: the restricted system
// (1/h) T x = r' with T tridiagonal, T_nn = d^2 + [n>=2], T_{n,n+-1} = -d, solved by its
// LDL^T factorisation (forward elimination, then back substitution).  The store holds
// y_n / D_n and the multiplier -d / D_n of every node.
__global__ void __launch_bounds__(kBlock)
k_modal_exact(Geom g, const double* __restrict__ rhat, const double* __restrict__ c0, int sub,
              const double* __restrict__ lamx, const double* __restrict__ lamy,
              double* __restrict__ store, double* __restrict__ zhat, double* __restrict__ ext) {
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (m >= MM) return;
  const int q = mode_at((int)(m / g.Mx), g.My), p = mode_at((int)(m % g.Mx), g.Mx);
  const Range rg = node_range(g, s);
  if (q >= g.my || p >= g.mx) {
    for (int n = rg.own_lo; n <= rg.own_hi; ++n) zhat[(long long)(n - 1) * MM + m] = 0.0;
    return;
  }
  const double d = g.sigma + lamy[q] + lamx[p];
  const double e = -d;
  double* zs = store + ((long long)s * g.L) * MM + m;
  double* ls = store + ((long long)(g.nd + s) * g.L) * MM + m;
  double Dprev = 0.0, yprev = 0.0;
  for (int n = rg.lo; n <= rg.hi; ++n) {
    const double a = d * d + (n >= 2 ? 1.0 : 0.0);
    const double b = g.h * rprime_at(g, rhat, c0, sub, d, MM, m, n);
    double Dn, yn;
    if (n == rg.lo) {
      Dn = a;
      yn = b;
    } else {
      const double l = e / Dprev;
      Dn = a - l * e;
      yn = b - l * yprev;
    }
    const int j = n - rg.first;
    zs[(long long)j * MM] = yn / Dn;
    ls[(long long)j * MM] = e / Dn;
    Dprev = Dn;
    yprev = yn;
  }
  double x = 0.0;
  for (int n = rg.hi; n >= rg.lo; --n) {
    const int j = n - rg.first;
    x = zs[(long long)j * MM] - (n < rg.hi ? ls[(long long)j * MM] * x : 0.0);
    put_out(g, rg, c0, MM, m, s, n, x, zhat, ext);
  }
}

// Additive Schwarz: add the extension values of the neighbours to the owned nodes of s
// (left extension of s+1, then right extension of s-1), one thread per mode and subdomain.
__global__ void __launch_bounds__(kBlock)
k_modal_asm_add(Geom g, const double* __restrict__ ext, double* __restrict__ zhat) {
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (m >= MM) return;
  if (mode_at((int)(m / g.Mx), g.My) >= g.my || mode_at((int)(m % g.Mx), g.Mx) >= g.mx) return;
  const int E = g.delta * (1 + g.sym);
  if (s + 1 < g.nd)
    for (int i = 0; i < g.delta; ++i) {
      const int n = (s + 1) * g.k + 1 - g.delta + i;
      zhat[(long long)(n - 1) * MM + m] += ext[((long long)(s + 1) * E + i) * MM + m];
    }
  if (g.sym && s > 0)
    for (int i = 0; i < g.delta; ++i) {
      const int n = s * g.k + 1 + i;
      zhat[(long long)(n - 1) * MM + m] += ext[((long long)(s - 1) * E + g.delta + i) * MM + m];
    }
}

// r_hat <- r_hat - S_hat z_hat over all nodes, one thread per mode (fine level first).
__global__ void __launch_bounds__(kBlock)
k_modal_residual(Geom g, const double* __restrict__ zhat, const double* __restrict__ lamx,
                 const double* __restrict__ lamy, double* __restrict__ rhat) {
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (m >= MM) return;
  const int q = mode_at((int)(m / g.Mx), g.My), p = mode_at((int)(m % g.Mx), g.Mx);
  if (q >= g.my || p >= g.mx) return;
  const double d = g.sigma + lamy[q] + lamx[p];
  double zp = 0.0, zc = zhat[m];
  for (int n = 1; n <= g.nt; ++n) {
    const double zn = n < g.nt ? zhat[(long long)n * MM + m] : 0.0;
    double sc = d * d * zc - d * zn;
    if (n >= 2) sc += zc - d * zp;
    rhat[(long long)(n - 1) * MM + m] -= sc / g.h;
    zp = zc;
    zc = zn;
  }
}

// z_hat <- z_hat + Z c0 (prolongation of the coarse solution), one thread per mode.
__global__ void __launch_bounds__(kBlock)
k_modal_prolong_add(Geom g, const double* __restrict__ c0, double* __restrict__ zhat) {
  const long long MM = g.padded();
  const long long m = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (m >= MM) return;
  if (mode_at((int)(m / g.Mx), g.My) >= g.my || mode_at((int)(m % g.Mx), g.Mx) >= g.mx) return;
  for (int n = 1; n <= g.nt; ++n) zhat[(long long)(n - 1) * MM + m] += chat_at(g, c0, MM, m, n);
}

template <typename T, int R>
void reg_sweep_r(int W, dim3 grid, hipStream_t s, const Geom& g, const T* rhat, const double* c0,
                 int sub, const double* lamx, const double* lamy, T* zhat, double* ext) {
  if (W == 0)
    hipLaunchKernelGGL((k_modal_sweep_reg<T, R, 0>), grid, dim3(kBlock), 0, s, g, rhat, c0, sub,
                       lamx, lamy, zhat, ext);
  else if (W == 3)
    hipLaunchKernelGGL((k_modal_sweep_reg<T, R, 3>), grid, dim3(kBlock), 0, s, g, rhat, c0, sub,
                       lamx, lamy, zhat, ext);
  else
    hipLaunchKernelGGL((k_modal_sweep_reg<T, R, 5>), grid, dim3(kBlock), 0, s, g, rhat, c0, sub,
                       lamx, lamy, zhat, ext);
}

template <typename T>
void reg_sweep(int R, int W, dim3 grid, hipStream_t s, const Geom& g, const T* rhat,
               const double* c0, int sub, const double* lamx, const double* lamy, T* zhat,
               double* ext) {
  if (R == 12)
    reg_sweep_r<T, 12>(W, grid, s, g, rhat, c0, sub, lamx, lamy, zhat, ext);
  else if (R == 24)
    reg_sweep_r<T, 24>(W, grid, s, g, rhat, c0, sub, lamx, lamy, zhat, ext);
  else
    reg_sweep_r<T, 32>(W, grid, s, g, rhat, c0, sub, lamx, lamy, zhat, ext);
}

template <typename T>
int modal_t(const Geom& g, const void* rhat, const double* c0, int sub, const double* lamx,
            const double* lamy, double* yscratch, void* zhat, double* ext, hipStream_t s) {
  const long long MM = g.padded();
  const dim3 grid((unsigned)((MM + kBlock - 1) / kBlock), g.nd);
  prof_begin(KKTDD_K_COARSE, s);
  if (g.exact_local)
    hipLaunchKernelGGL(k_modal_exact, grid, dim3(kBlock), 0, s, g,
                       static_cast<const double*>(rhat), c0, sub, lamx, lamy, yscratch,
                       static_cast<double*>(zhat), ext);
  else if (g.L <= kRegSteps) {
    if (MM % kBlock) return set_error(KKTDD_EINVAL, "padded mode count is not a multiple of 256");
    const int W = !c0 ? 0 : (g.delta < g.k ? 3 : 5);
    const int R = g.L <= 12 ? 12 : (g.L <= 24 ? 24 : 32);
    reg_sweep<T>(R, W, grid, s, g, static_cast<const T*>(rhat), c0, sub, lamx, lamy,
                 static_cast<T*>(zhat), ext);
  } else {
    hipLaunchKernelGGL((k_modal_sweep<T>), grid, dim3(kBlock), 0, s, g,
                       static_cast<const T*>(rhat), c0, sub, lamx, lamy, yscratch,
                       static_cast<T*>(zhat), ext);
  }
  KKT_HIP(hipGetLastError());
  // read r_hat over the subdomain nodes, write z_hat once
  const double el = sizeof(T);
  prof_end(KKTDD_K_COARSE, s, el * MM * ((double)g.nd * g.L + g.nt), 0.0);
  return 0;
}

template <typename T>
void restrict_t(int R, dim3 grid, hipStream_t s, const Geom& g, const T* rhat, double* r0) {
  if (R == 16)
    hipLaunchKernelGGL((k_modal_restrict<T, 16>), grid, dim3(kBlock), 0, s, g, rhat, r0);
  else if (R == kRegSteps)
    hipLaunchKernelGGL((k_modal_restrict<T, kRegSteps>), grid, dim3(kBlock), 0, s, g, rhat, r0);
  else
    hipLaunchKernelGGL((k_modal_restrict<T, 0>), grid, dim3(kBlock), 0, s, g, rhat, r0);
}

}  // namespace

int launch_modal_restrict(const Geom& g, int precision, const void* rhat, double* r0,
                          hipStream_t s) {
  const long long MM = g.padded();
  const dim3 grid((unsigned)((MM + kBlock - 1) / kBlock), g.nd);
  prof_begin(KKTDD_K_COARSE, s);
  const int R = g.k <= 16 ? 16 : (g.k <= kRegSteps ? kRegSteps : 0);
  if (precision != KKTDD_FP64)
    restrict_t<float>(R, grid, s, g, static_cast<const float*>(rhat), r0);
  else
    restrict_t<double>(R, grid, s, g, static_cast<const double*>(rhat), r0);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, (precision != KKTDD_FP64 ? 4.0 : 8.0) * MM * g.nt + 8.0 * MM * g.nc, 0.0);
  return 0;
}

int launch_modal_sweeps(const Geom& g, int precision, const void* rhat, const double* c0,
                        int sub_coarse, const double* lamx, const double* lamy, double* yscratch,
                        void* zhat, double* ext, hipStream_t s) {
  if (g.exact_local && precision != KKTDD_FP64)
    return set_error(KKTDD_EINVAL, "the exact local inverse runs in float64 only");
  if (g.asm_sum && !ext) return set_error(KKTDD_EINVAL, "additive Schwarz needs its extension buffer");
  if (precision != KKTDD_FP64)
    return modal_t<float>(g, rhat, c0, sub_coarse, lamx, lamy, yscratch, zhat, ext, s);
  return modal_t<double>(g, rhat, c0, sub_coarse, lamx, lamy, yscratch, zhat, ext, s);
}

int launch_modal_asm_add(const Geom& g, const double* ext, double* zhat, hipStream_t s) {
  const long long MM = g.padded();
  const dim3 grid((unsigned)((MM + kBlock - 1) / kBlock), g.nd);
  prof_begin(KKTDD_K_COARSE, s);
  hipLaunchKernelGGL(k_modal_asm_add, grid, dim3(kBlock), 0, s, g, ext, zhat);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, 24.0 * MM * g.nd * g.delta * (1 + g.sym), 0.0);
  return 0;
}

int launch_modal_residual(const Geom& g, const double* zhat, const double* lamx,
                          const double* lamy, double* rhat, hipStream_t s) {
  const long long MM = g.padded();
  prof_begin(KKTDD_K_COARSE, s);
  hipLaunchKernelGGL(k_modal_residual, dim3((unsigned)((MM + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, g, zhat, lamx, lamy, rhat);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, 24.0 * MM * g.nt, 0.0);
  return 0;
}

int launch_modal_prolong_add(const Geom& g, const double* c0, double* zhat, hipStream_t s) {
  const long long MM = g.padded();
  prof_begin(KKTDD_K_COARSE, s);
  hipLaunchKernelGGL(k_modal_prolong_add, dim3((unsigned)((MM + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, g, c0, zhat);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, 16.0 * MM * g.nt + 8.0 * MM * g.nc, 0.0);
  return 0;
}

}  // namespace kktdd
