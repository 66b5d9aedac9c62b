// KKT matvec (Eq. (5)), right-hand side, block scalings and the D_sigma stencil.
//
// Block rows of K x for x = (u, z, w), with B = I + dt*nu*A_h the diagonal block of J
// (Eq. (2)-(3)), J's sub-diagonal block -I, L = -dt*I and M = h*I:
//     y_u^n = h u^n + B w^n - w^{n+1}
//     y_z^n = omega h z^n - dt w^n
//     y_w^n = B u^n - u^{n-1} - dt z^n
// (w^{nt+1} = 0, u^0 = 0: the initial condition lives in the right-hand side.)
//
// HBM-bound: 3 fields in, 3 out, 48 bytes per space-time point.  One thread owns one
// interior point and marches over a block of time-nodes, carrying u^{n-1} and w^{n+1} in
// registers so each centre value is fetched once; the four in-slice neighbours come from
// L1/L2.  Work tiles (slice chunk, time block) are ordered so that the tiles one XCD runs
// are neighbours in space, which keeps the neighbour rows inside that XCD's L2.
#include "internal.h"

namespace kktdd {

namespace {

constexpr int kBlock = 256;

__device__ inline int xcd_tile(int b, int nblk) {
  // Workgroups are dispatched round-robin over the 8 XCDs; give XCD x a contiguous range
  // of logical tiles.  Bijection of [0, nblk).
  const int q = nblk / 8, r = nblk % 8;
  const int xcd = b % 8, idx = b / 8;
  return xcd * q + (xcd < r ? xcd : r) + idx;
}

__global__ void __launch_bounds__(kBlock)
k_kkt_apply(Geom g, const double* __restrict__ xu, const double* __restrict__ xz,
            const double* __restrict__ xw, double su, double sz, double sw,
            const double* __restrict__ dscale, const double* __restrict__ f,
            double* __restrict__ yu, double* __restrict__ yz, double* __restrict__ yw, int tb,
            int nchunks) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int chunk = tile % nchunks, tblock = tile / nchunks;
  const int pt = chunk * kBlock + threadIdx.x;
  if (pt >= g.nxy) return;
  const int i = pt % g.mx, j = pt / g.mx;
  const bool hasE = i + 1 < g.mx, hasW = i > 0, hasN = j + 1 < g.my, hasS = j > 0;
  const int n0 = tblock * tb;
  const int n1 = min(g.nt, n0 + tb);
  if (dscale) {   // device factor of the u and z inputs (the Krylov vector's scale)
    const double d = *dscale;
    su *= d;
    sz *= d;
  }
  const double cx = g.cx, cy = g.cy, h = g.h, oh = g.omega * g.h, dt = g.dt;
  const long long nxy = g.nxy;
  // Operands of one time-node.  Those of node n+1 are requested before node n is computed,
  // so every thread keeps two nodes' loads in flight.
  struct Node {
    double u, uE, uW, uN, uS, wE, wW, wN, wS, z, w_next;
  };
  auto load = [&](int n, Node& v) {
    const long long b = n * nxy + pt;
    v.u = xu[b];
    v.uE = hasE ? xu[b + 1] : 0.0;
    v.uW = hasW ? xu[b - 1] : 0.0;
    v.uN = hasN ? xu[b + g.mx] : 0.0;
    v.uS = hasS ? xu[b - g.mx] : 0.0;
    v.wE = hasE ? xw[b + 1] : 0.0;
    v.wW = hasW ? xw[b - 1] : 0.0;
    v.wN = hasN ? xw[b + g.mx] : 0.0;
    v.wS = hasS ? xw[b - g.mx] : 0.0;
    v.z = xz[b];
    v.w_next = n + 1 < g.nt ? xw[b + nxy] : 0.0;
  };
  double u_prev = n0 > 0 ? xu[(n0 - 1) * nxy + pt] : 0.0;
  double w_c = xw[n0 * nxy + pt];
  Node cur, nxt;
  load(n0, cur);
  for (int n = n0; n < n1; ++n) {
    if (n + 1 < n1) load(n + 1, nxt);
    const long long b = n * nxy + pt;
    const double u_c = cur.u;
    const double Bu = u_c + cx * (2.0 * u_c - cur.uE - cur.uW) + cy * (2.0 * u_c - cur.uN - cur.uS);
    const double Bw = w_c + cx * (2.0 * w_c - cur.wE - cur.wW) + cy * (2.0 * w_c - cur.wN - cur.wS);
    double ru = h * su * u_c + sw * (Bw - cur.w_next);
    double rz = oh * sz * cur.z - dt * sw * w_c;
    double rw = su * (Bu - u_prev) - dt * sz * cur.z;
    if (f) {
      ru = f[b] - ru;
      rz = f[g.P + b] - rz;
      rw = f[2 * g.P + b] - rw;
    }
    yu[b] = ru;
    yz[b] = rz;
    yw[b] = rw;
    u_prev = u_c;
    w_c = cur.w_next;
    cur = nxt;
  }
}

__global__ void __launch_bounds__(kBlock)
k_rhs(Geom g, const double* __restrict__ u0, const double* __restrict__ ut, double* __restrict__ f) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= g.P) return;
  f[e] = g.h * ut[e];
  f[g.P + e] = 0.0;
  f[2 * g.P + e] = e < g.nxy ? u0[e] : 0.0;
}

__global__ void __launch_bounds__(kBlock)
k_scale(long long n, const double* __restrict__ in, double a, const double* __restrict__ dscale,
        double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const double s = dscale ? a * *dscale : a;
  out[e] = s * in[e];
}

__global__ void __launch_bounds__(kBlock)
k_apply_D(Geom g, const double* __restrict__ in, double* __restrict__ out, int nslices,
          double shift) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (long long)nslices * g.nxy) return;
  const int pt = (int)(e % g.nxy);
  const int i = pt % g.mx, j = pt / g.mx;
  const double c = in[e];
  const double E = i + 1 < g.mx ? in[e + 1] : 0.0, W = i > 0 ? in[e - 1] : 0.0;
  const double N = j + 1 < g.my ? in[e + g.mx] : 0.0, S = j > 0 ? in[e - g.mx] : 0.0;
  out[e] = shift * c + g.cx * (2.0 * c - E - W) + g.cy * (2.0 * c - N - S);
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int launch_kkt_apply(const Geom& g, const double* xu, const double* xz, const double* xw,
                     double su, double sz, double sw, const double* dscale, const double* f,
                     double* yu, double* yz, double* yw, hipStream_t s) {
  const int nchunks = (g.nxy + kBlock - 1) / kBlock;
  // Enough time blocks for a few waves of workgroups per CU, at most 16 nodes each.
  int tb = 16;
  while (tb > 1 && (long long)nchunks * ((g.nt + tb - 1) / tb) < 2048) tb /= 2;
  const int ntb = (g.nt + tb - 1) / tb;
  prof_begin(KKTDD_K_MATVEC, s);
  hipLaunchKernelGGL(k_kkt_apply, dim3(nchunks * ntb), dim3(kBlock), 0, s, g, xu, xz, xw, su, sz,
                     sw, dscale, f, yu, yz, yw, tb, nchunks);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_MATVEC, s, (f ? 72.0 : 48.0) * g.P, 0.0);
  return 0;
}

int launch_rhs(const Geom& g, const double* u0, const double* ut, double* f, hipStream_t s) {
  prof_begin(KKTDD_K_OTHER, s);
  hipLaunchKernelGGL(k_rhs, dim3(blocks_for(g.P)), dim3(kBlock), 0, s, g, u0, ut, f);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_OTHER, s, 32.0 * g.P, 0.0);
  return 0;
}

int launch_scale(long long n, const double* in, double a, const double* dscale, double* out,
                 hipStream_t s) {
  if (n == 0) return 0;
  prof_begin(KKTDD_K_OTHER, s);
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, in, a, dscale, out);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_OTHER, s, 16.0 * n, 0.0);
  return 0;
}

int launch_apply_D(const Geom& g, const double* in, double* out, int nslices, double shift,
                   hipStream_t s) {
  const long long n = (long long)nslices * g.nxy;
  if (n == 0) return 0;
  prof_begin(KKTDD_K_COARSE, s);
  hipLaunchKernelGGL(k_apply_D, dim3(blocks_for(n)), dim3(kBlock), 0, s, g, in, out, nslices,
                     shift);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_COARSE, s, 16.0 * n, 0.0);
  return 0;
}

}  // namespace kktdd
