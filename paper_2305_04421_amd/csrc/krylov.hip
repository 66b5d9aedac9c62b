// Flexible GMRES vector kernels (float64): Arnoldi Gram-Schmidt passes, reductions,
// solution update.
//
// Krylov vectors are stored unnormalised: the basis vector is v_i = vinv[i] * V_i with the
// scale vinv[i] kept on the device, so normalising a new vector costs no extra pass.
//
// Default orthogonalisation: delayed classical Gram-Schmidt with reorthogonalisation (DCGS2,
// the one-synchronisation CGS2 of Swirydowicz, Langou, Ananthan, Yang and Thomas).  Step j
// holds the not yet reorthogonalised candidate of v_j and W = K z_j; one inner-product pass
// forms <V_i, candidate>, <V_i, W>, ||candidate||^2, <candidate, W> and ||W||^2, and one
// update pass finishes v_j (second projection) and projects W once, which becomes the next
// candidate.  The basis is walked in chunks, so a cycle may hold any number of vectors.
//
// Alternative: classical Gram-Schmidt with selective reorthogonalisation
// (Daniel-Gragg-Kaufman-Stewart, at most 32 vectors per pass): pass A forms <v_i, w> and
// ||w||; pass B subtracts the projections and, reading the same V, also forms <v_i, w1>
// and ||w1||; only if ||w1|| < eta ||w|| does pass C subtract the second projections.
//
// Every reduction is two-stage and in a fixed order, so results are deterministic.
#include "internal.h"

namespace kktdd {

namespace {

constexpr int kBlock = 256;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum `count` per-thread values over the block; thread 0 writes out[0..count).
template <int MAXS>
__device__ inline void block_sums(double (&acc)[MAXS], int count, double* out) {
  __shared__ double red[kBlock / 64][MAXS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < MAXS; ++i) {
    if (i < count) {
      const double v = wave_sum(acc[i]);
      if (lane == 0) red[wave][i] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < count) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += red[w][threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// Vectors are streamed as double2 (16-byte loads); V's leading dimension and the vector
// pointers are 16-byte aligned, and an odd tail element is handled by thread 0 of block 0.
template <int MAXV>
__global__ void __launch_bounds__(kBlock)
k_multidot(long long n, const double* __restrict__ V, long long ldv, int nv,
           const double* __restrict__ w, int want_norm, double* __restrict__ partials) {
  double acc[MAXV + 1];
#pragma unroll
  for (int i = 0; i <= MAXV; ++i) acc[i] = 0.0;
  const long long n2 = n >> 1, ld2 = ldv >> 1;
  const double2* __restrict__ V2 = reinterpret_cast<const double2*>(V);
  const double2* __restrict__ w2 = reinterpret_cast<const double2*>(w);
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n2; e += stride) {
    const double2 wv = w2[e];
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      if (i < nv) {
        const double2 v = V2[i * ld2 + e];
        acc[i] += v.x * wv.x + v.y * wv.y;
      }
    acc[MAXV] += wv.x * wv.x + wv.y * wv.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double wv = w[n - 1];
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      if (i < nv) acc[i] += V[i * ldv + n - 1] * wv;
    acc[MAXV] += wv * wv;
  }
  // compact: slot nv holds the norm
  double out[MAXV + 1];
#pragma unroll
  for (int i = 0; i <= MAXV; ++i) out[i] = i < nv ? acc[i] : 0.0;
  if (want_norm) {
#pragma unroll
    for (int i = 0; i <= MAXV; ++i)
      if (i == nv) out[i] = acc[MAXV];
  }
  block_sums<MAXV + 1>(out, nv + (want_norm ? 1 : 0), partials + (long long)blockIdx.x * (nv + (want_norm ? 1 : 0)));
}

template <int MAXV>
__global__ void __launch_bounds__(kBlock)
k_update_dot(long long n, const double* __restrict__ V, long long ldv, int nv,
             const double* __restrict__ vinv, const double* __restrict__ coef,
             const double* w, double* wout, int want_dots, double* __restrict__ partials,
             const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  double cf[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) cf[i] = i < nv ? coef[i] * vinv[i] : 0.0;
  double acc[MAXV + 1];
#pragma unroll
  for (int i = 0; i <= MAXV; ++i) acc[i] = 0.0;
  const long long n2 = n >> 1, ld2 = ldv >> 1;
  const double2* __restrict__ V2 = reinterpret_cast<const double2*>(V);
  const double2* w2 = reinterpret_cast<const double2*>(w);
  double2* o2 = reinterpret_cast<double2*>(wout);
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n2; e += stride) {
    double2 vv[MAXV];
    double2 x = w2[e];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      vv[i] = i < nv ? V2[i * ld2 + e] : double2{0.0, 0.0};
      x.x -= cf[i] * vv[i].x;
      x.y -= cf[i] * vv[i].y;
    }
    o2[e] = x;
    if (want_dots) {
#pragma unroll
      for (int i = 0; i < MAXV; ++i) acc[i] += vv[i].x * x.x + vv[i].y * x.y;
    }
    acc[MAXV] += x.x * x.x + x.y * x.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double vv[MAXV];
    double x = w[n - 1];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      vv[i] = i < nv ? V[i * ldv + n - 1] : 0.0;
      x -= cf[i] * vv[i];
    }
    wout[n - 1] = x;
    if (want_dots) {
#pragma unroll
      for (int i = 0; i < MAXV; ++i) acc[i] += vv[i] * x;
    }
    acc[MAXV] += x * x;
  }
  const int ns = (want_dots ? nv : 0) + 1;
  double out[MAXV + 1];
#pragma unroll
  for (int i = 0; i <= MAXV; ++i) out[i] = (want_dots && i < nv) ? acc[i] : 0.0;
#pragma unroll
  for (int i = 0; i <= MAXV; ++i)
    if (i == ns - 1) out[i] = acc[MAXV];
  block_sums<MAXV + 1>(out, ns, partials + (long long)blockIdx.x * ns);
}

// ---- delayed classical Gram-Schmidt with reorthogonalisation (DCGS2) -------------------
// Arnoldi step j holds final basis vectors in slots 0..j-1, the once-orthogonalised
// candidate of basis vector j in slot j and the new product W = K z_j in slot j+1.  One
// pass forms every inner product the step needs,
//     A_i = <V_i, Vc>, B_i = <V_i, W> (i < j), C = <Vc, Vc>, E = <Vc, W>, F = <W, W>,
// and one pass applies them: the candidate is reorthogonalised into the final v_j and W is
// projected once against v_0..v_j, becoming the next candidate.  So each step reads the basis
// twice instead of three times (Swirydowicz et al. 2021; Bielich et al. 2022).
// Inner products of a DCGS2 step for any j.  Per-block partial sums are laid out as
// [A_0..A_{j-1}, B_0..B_{j-1}, C, E, F].  The basis is processed in chunks of CH vectors held
// in register accumulators; each further chunk re-streams the candidate and W.
template <int CH>
__global__ void __launch_bounds__(kBlock)
k_dcgs_dots(long long n, const double* __restrict__ V, long long ldv, int j,
            const double* __restrict__ Vc, const double* __restrict__ W,
            double* __restrict__ partials) {
  constexpr int NS = 2 * CH + 3;
  __shared__ double red[kBlock / 64][NS];
  const int ns = 2 * j + 3;
  const long long n2 = n >> 1, ld2 = ldv >> 1;
  const double2* __restrict__ V2 = reinterpret_cast<const double2*>(V);
  const double2* __restrict__ c2 = reinterpret_cast<const double2*>(Vc);
  const double2* __restrict__ w2 = reinterpret_cast<const double2*>(W);
  const bool hasW = W != nullptr;
  const long long stride = (long long)gridDim.x * kBlock;
  const bool tail = (n & 1) && blockIdx.x == 0 && threadIdx.x == 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* out = partials + (long long)blockIdx.x * ns;
  const int nchunks = j == 0 ? 1 : (j + CH - 1) / CH;
  for (int c = 0; c < nchunks; ++c) {
    const int i0 = c * CH;
    const int cnt = j - i0 < CH ? j - i0 : CH;   // <= 0 only when j == 0
    const bool first = c == 0;
    double acc[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) acc[i] = 0.0;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n2; e += stride) {
      const double2 cv = c2[e];
      const double2 w = hasW ? w2[e] : double2{0.0, 0.0};
#pragma unroll
      for (int i = 0; i < CH; ++i)
        if (i < cnt) {
          const double2 v = V2[(long long)(i0 + i) * ld2 + e];
          acc[i] += v.x * cv.x + v.y * cv.y;
          acc[CH + i] += v.x * w.x + v.y * w.y;
        }
      acc[2 * CH] += cv.x * cv.x + cv.y * cv.y;
      acc[2 * CH + 1] += cv.x * w.x + cv.y * w.y;
      acc[2 * CH + 2] += w.x * w.x + w.y * w.y;
    }
    if (tail) {
      const double cv = Vc[n - 1], w = hasW ? W[n - 1] : 0.0;
#pragma unroll
      for (int i = 0; i < CH; ++i)
        if (i < cnt) {
          const double v = V[(long long)(i0 + i) * ldv + n - 1];
          acc[i] += v * cv;
          acc[CH + i] += v * w;
        }
      acc[2 * CH] += cv * cv;
      acc[2 * CH + 1] += cv * w;
      acc[2 * CH + 2] += w * w;
    }
    // wave sums, then thread t adds the four waves' value of slot t and stores it
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const bool used = (i < CH && i < cnt) || (i >= CH && i < 2 * CH && i - CH < cnt) ||
                        (i >= 2 * CH && first);
      if (used) {
        const double v = wave_sum(acc[i]);
        if (lane == 0) red[wave][i] = v;
      }
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NS) {
      int dst = -1;
      if (t < CH) dst = t < cnt ? i0 + t : -1;
      else if (t < 2 * CH) dst = t - CH < cnt ? j + i0 + (t - CH) : -1;
      else if (first) dst = 2 * j + (t - 2 * CH);
      if (dst >= 0) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) v += red[w][t];
        out[dst] = v;
      }
    }
    __syncthreads();
  }
}

// coef = [cv, hjj, p_0..p_{j-1}, q_0..q_{j-1}]:
//   slot j   <- v  = cv * Vc - sum_i p_i V_i
//   slot j+1 <- W' = W - sum_i q_i V_i - hjj * v,  with partial sums of ||W'||^2.
// MAXV > 0: j <= MAXV, coefficients in registers.  MAXV == 0: any j, coefficients read per
// use (wave-uniform loads).
template <int MAXV>
__global__ void __launch_bounds__(kBlock)
k_dcgs_update(long long n, double* V, long long ldv, int j, const double* __restrict__ coef,
              const int* __restrict__ gate, double* __restrict__ partials) {
  if (gate && *gate == 0) return;
  const double cv = coef[0], hjj = coef[1];
  constexpr int NR = MAXV > 0 ? MAXV : 1;
  double p[NR], q[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    p[i] = (MAXV > 0 && i < j) ? coef[2 + i] : 0.0;
    q[i] = (MAXV > 0 && i < j) ? coef[2 + j + i] : 0.0;
  }
  const long long n2 = n >> 1, ld2 = ldv >> 1;
  double2* V2 = reinterpret_cast<double2*>(V);
  double2* c2 = V2 + (long long)j * ld2;
  double2* w2 = c2 + ld2;
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n2; e += stride) {
    const double2 c = c2[e];
    double2 w = w2[e];
    double2 v = {cv * c.x, cv * c.y};
    if constexpr (MAXV > 0) {
#pragma unroll
      for (int i = 0; i < MAXV; ++i)
        if (i < j) {
          const double2 b = V2[(long long)i * ld2 + e];
          v.x -= p[i] * b.x;
          v.y -= p[i] * b.y;
          w.x -= q[i] * b.x;
          w.y -= q[i] * b.y;
        }
    } else {
      const double* pc = coef + 2;
      const double* qc = coef + 2 + j;
      int i = 0;
      for (; i + 8 <= j; i += 8) {
        double2 b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = V2[(long long)(i + u) * ld2 + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          v.x -= pc[i + u] * b[u].x;
          v.y -= pc[i + u] * b[u].y;
          w.x -= qc[i + u] * b[u].x;
          w.y -= qc[i + u] * b[u].y;
        }
      }
      for (; i < j; ++i) {
        const double2 b = V2[(long long)i * ld2 + e];
        v.x -= pc[i] * b.x;
        v.y -= pc[i] * b.y;
        w.x -= qc[i] * b.x;
        w.y -= qc[i] * b.y;
      }
    }
    w.x -= hjj * v.x;
    w.y -= hjj * v.y;
    // streaming stores (measured 4-7% faster for this pass than cached stores)
    double* cp = reinterpret_cast<double*>(c2 + e);
    double* wp = reinterpret_cast<double*>(w2 + e);
    __builtin_nontemporal_store(v.x, cp);
    __builtin_nontemporal_store(v.y, cp + 1);
    __builtin_nontemporal_store(w.x, wp);
    __builtin_nontemporal_store(w.y, wp + 1);
    acc += w.x * w.x + w.y * w.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double* c = V + (long long)j * ldv;
    double* w = c + ldv;
    double v = cv * c[n - 1], x = w[n - 1];
    for (int i = 0; i < j; ++i) {
      const double b = V[(long long)i * ldv + n - 1];
      v -= coef[2 + i] * b;
      x -= coef[2 + j + i] * b;
    }
    x -= hjj * v;
    c[n - 1] = v;
    w[n - 1] = x;
    acc += x * x;
  }
  double out[1] = {acc};
  block_sums<1>(out, 1, partials + blockIdx.x);
}

// Bookkeeping of a DCGS2 step by one wave (lane l handles entries l, l+64, ...; the two
// inner sums are reduced in a fixed order).  vinv[i] scales slot i (1 for final vectors).
// rec (host-visible) = [alpha, nu, a_0..a_{j-1}, b_0..b_{j-1}, hjj, nu_next, breakdown]
//   stage 1 (sums of a full step):   reorthogonalisation of the candidate, projection of W,
//                                    update coefficients; gate = 0 on breakdown
//   stage 2 (sum of ||W'||^2):       normalisation scales of slots j and j+1
//   stage 3 (sums without W):        reorthogonalisation coefficients only (closing a column)
__global__ void __launch_bounds__(64)
k_dcgs_finish(int j, const double* __restrict__ sums, double* __restrict__ vinv,
              double* __restrict__ coef, double* __restrict__ rec, int* __restrict__ gate,
              int stage) {
  if (blockIdx.x != 0) return;
  const int l = threadIdx.x;
  double* a = rec + 2;
  double* b = rec + 2 + j;
  if (stage == 1 || stage == 3) {
    const double sc = vinv[j];
    double sa = 0.0;
    for (int i = l; i < j; i += 64) {
      const double ai = vinv[i] * sc * sums[i];
      a[i] = ai;
      sa += ai * ai;
    }
    sa = wave_sum(sa);
    const double c = sc * sc * sums[2 * j];
    const double al2 = c - sa;
    const bool brk = !(al2 > 1e-24 * c) || !(c > 0.0);
    const double alpha = brk ? 0.0 : sqrt(al2);
    if (l == 0) {
      rec[0] = alpha;
      rec[1] = sc > 0.0 ? 1.0 / sc : 0.0;
      rec[2 * j + 4] = brk ? 1.0 : 0.0;
    }
    if (stage == 3) return;
    double ab = 0.0;
    for (int i = l; i < j; i += 64) {
      const double bi = vinv[i] * sums[j + i];
      b[i] = bi;
      ab += a[i] * bi;
    }
    ab = wave_sum(ab);
    const double e = sc * sums[2 * j + 1];
    const double hjj = brk ? 0.0 : (e - ab) / alpha;
    for (int i = l; i < j; i += 64) {
      coef[2 + i] = brk ? 0.0 : a[i] * vinv[i] / alpha;
      coef[2 + j + i] = b[i] * vinv[i];
    }
    if (l == 0) {
      rec[2 * j + 2] = hjj;
      coef[0] = brk ? 0.0 : sc / alpha;
      coef[1] = hjj;
      *gate = brk ? 0 : 1;
    }
  } else if (l == 0 && *gate) {
    const double nu = sqrt(sums[0]);
    rec[2 * j + 3] = nu;
    vinv[j] = 1.0;
    vinv[j + 1] = nu > 0.0 ? 1.0 / nu : 0.0;
  }
}

// out[i] = sum over blocks of partials[b*nsums + i] in a fixed order: workgroup i sums
// column i, thread t taking blocks t, t+256, ..., then a fixed-shape tree over the threads.
__global__ void __launch_bounds__(kBlock)
k_reduce_partials(const double* __restrict__ partials, int nblocks, int nsums,
                  double* __restrict__ out) {
  __shared__ double red[kBlock / 64];
  const int i = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) t += partials[(long long)b * nsums + i];
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) out[i] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Arnoldi bookkeeping for step j (one thread).
//   hcol[0..j]   : Hessenberg column (projections, accumulated over both passes)
//   hcol[j+1]    : ||w|| after orthogonalisation = H(j+1, j)
//   hcol[j+2]    : 1 if a second pass was taken
//   coef[0..j]   : coefficients of the next update pass (stored right after hcol)
// stage 1: sums1 = raw <V_i, w>, ||w||^2      -> coef = h, hcol = h, keep ||w||
// stage 2: sums2 = raw <V_i, w1>, ||w1||^2    -> reorthogonalise if ||w1|| < eta ||w||
// stage 3: sums3 = ||w2||^2 (only if gated)
__global__ void k_arnoldi_finish(int j, const double* sums1, const double* sums2,
                                 const double* sums3, int* gate, double* hcol, double* vinv,
                                 double eta, int stage) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* coef = hcol + (j + 3);
  double* wnorm = hcol + 2 * (j + 3);   // scratch: ||w|| of pass A
  if (stage == 1) {
    for (int i = 0; i <= j; ++i) {
      const double h = vinv[i] * sums1[i];
      hcol[i] = h;
      coef[i] = h;
    }
    wnorm[0] = sqrt(sums1[j + 1]);
    hcol[j + 2] = 0.0;
    *gate = 0;
  } else if (stage == 2) {
    const double n1 = sqrt(sums2[j + 1]);
    if (n1 < eta * wnorm[0]) {
      for (int i = 0; i <= j; ++i) {
        const double h = vinv[i] * sums2[i];
        hcol[i] += h;
        coef[i] = h;
      }
      hcol[j + 2] = 1.0;
      *gate = 1;
    } else {
      hcol[j + 1] = n1;
      vinv[j + 1] = n1 > 0.0 ? 1.0 / n1 : 0.0;
      *gate = 0;
    }
  } else if (*gate) {
    const double n2 = sqrt(sums3[0]);
    hcol[j + 1] = n2;
    vinv[j + 1] = n2 > 0.0 ? 1.0 / n2 : 0.0;
  }
}

// x_u += su * sum_i yv[i] vinv[i] V_i,u;  x_z += sz * (same with V_i,z);  x_w += sum_i yw[i] Zw_i
// (yv and yw are the coefficients of the basis vectors and of the stored w-blocks).
__global__ void __launch_bounds__(kBlock)
k_update_solution(Geom g, const double* __restrict__ V, long long ldv,
                  const double* __restrict__ Zw, long long ldz, int nv,
                  const double* __restrict__ yv, const double* __restrict__ yw,
                  const double* __restrict__ vinv, double su, double sz, double* __restrict__ x) {
  const long long n3 = 3 * g.P;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n3; e += stride) {
    const int f = (int)(e / g.P);
    double acc = 0.0;
    if (f < 2) {
      const double sf = f == 0 ? su : sz;
      for (int i = 0; i < nv; ++i) acc += (yv[i] * vinv[i] * sf) * V[i * ldv + e];
    } else {
      const long long off = e - 2 * g.P;
      for (int i = 0; i < nv; ++i) acc += yw[i] * Zw[i * ldz + off];
    }
    x[e] += acc;
  }
}

// partials[b*3 + f] = sum of squares of field f over this block's share.
__global__ void __launch_bounds__(kBlock)
k_sumsq_blocks(Geom g, const double* __restrict__ r, double* __restrict__ partials) {
  double acc[3] = {0.0, 0.0, 0.0};
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < g.P; e += stride) {
    const double a = r[e], b = r[g.P + e], c = r[2 * g.P + e];
    acc[0] += a * a;
    acc[1] += b * b;
    acc[2] += c * c;
  }
  block_sums<3>(acc, 3, partials + (long long)blockIdx.x * 3);
}

}  // namespace

int launch_multidot(long long n, const double* V, long long ldv, int nv, const double* vinv,
                    const double* w, int want_norm, double* partials, int nblocks,
                    hipStream_t s) {
  (void)vinv;
  const dim3 grid(nblocks), block(kBlock);
  prof_begin(KKTDD_K_ARNOLDI, s);
  if (nv <= 8)
    hipLaunchKernelGGL((k_multidot<8>), grid, block, 0, s, n, V, ldv, nv, w, want_norm, partials);
  else if (nv <= 16)
    hipLaunchKernelGGL((k_multidot<16>), grid, block, 0, s, n, V, ldv, nv, w, want_norm, partials);
  else if (nv <= 24)
    hipLaunchKernelGGL((k_multidot<24>), grid, block, 0, s, n, V, ldv, nv, w, want_norm, partials);
  else if (nv <= 32)
    hipLaunchKernelGGL((k_multidot<32>), grid, block, 0, s, n, V, ldv, nv, w, want_norm, partials);
  else
    return set_error(KKTDD_EINVAL, "more than 32 Krylov vectors per pass");
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_ARNOLDI, s, 8.0 * (nv + 1) * n, 0.0);
  return 0;
}

int launch_update_dot(long long n, const double* V, long long ldv, int nv, const double* vinv,
                      const double* coef, const double* w, double* wout, int want_dots,
                      double* partials, int nblocks, const int* gate, hipStream_t s) {
  const dim3 grid(nblocks), block(kBlock);
  prof_begin(KKTDD_K_ARNOLDI, s);
  if (nv <= 8)
    hipLaunchKernelGGL((k_update_dot<8>), grid, block, 0, s, n, V, ldv, nv, vinv, coef, w, wout,
                       want_dots, partials, gate);
  else if (nv <= 16)
    hipLaunchKernelGGL((k_update_dot<16>), grid, block, 0, s, n, V, ldv, nv, vinv, coef, w, wout,
                       want_dots, partials, gate);
  else if (nv <= 24)
    hipLaunchKernelGGL((k_update_dot<24>), grid, block, 0, s, n, V, ldv, nv, vinv, coef, w, wout,
                       want_dots, partials, gate);
  else if (nv <= 32)
    hipLaunchKernelGGL((k_update_dot<32>), grid, block, 0, s, n, V, ldv, nv, vinv, coef, w, wout,
                       want_dots, partials, gate);
  else
    return set_error(KKTDD_EINVAL, "more than 32 Krylov vectors per pass");
  KKT_HIP(hipGetLastError());
  // a gated pass counts its bytes only once the host knows it ran
  prof_end(KKTDD_K_ARNOLDI, s, gate ? 0.0 : 8.0 * (nv + 2) * n, 0.0);
  return 0;
}

int launch_reduce_partials(const double* partials, int nblocks, int nsums, double* out,
                           hipStream_t s) {
  prof_begin(KKTDD_K_ARNOLDI, s);
  hipLaunchKernelGGL(k_reduce_partials, dim3(nsums), dim3(kBlock), 0, s, partials, nblocks,
                     nsums, out);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_ARNOLDI, s, 8.0 * nblocks * nsums, 0.0);
  return 0;
}

int launch_arnoldi_finish(int j, const double* sums1, const double* sums2, const double* sums3,
                          int* gate, double* hcol, double* vinv, double eta, int stage,
                          hipStream_t s) {
  prof_begin(KKTDD_K_ARNOLDI, s);
  hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(64), 0, s, j, sums1, sums2, sums3, gate, hcol,
                     vinv, eta, stage);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_ARNOLDI, s, 0.0, 0.0);
  return 0;
}

int launch_dcgs_dots(long long n, const double* V, long long ldv, int j, const double* Vc,
                     const double* W, double* partials, int nblocks, hipStream_t s) {
  const dim3 grid(nblocks), block(kBlock);
  prof_begin(KKTDD_K_ARNOLDI, s);
  // 8- and 16-vector chunks keep the accumulators in few enough registers for full
  // occupancy; wider chunks read the candidate and W fewer times but stream more slowly.
  const int ch = j <= 8 ? 8 : 16;
  if (ch == 8)
    hipLaunchKernelGGL((k_dcgs_dots<8>), grid, block, 0, s, n, V, ldv, j, Vc, W, partials);
  else
    hipLaunchKernelGGL((k_dcgs_dots<16>), grid, block, 0, s, n, V, ldv, j, Vc, W, partials);
  KKT_HIP(hipGetLastError());
  const int nchunks = j == 0 ? 1 : (j + ch - 1) / ch;
  prof_end(KKTDD_K_ARNOLDI, s, 8.0 * (j + nchunks * (W ? 2 : 1)) * n, 0.0);
  return 0;
}

int launch_dcgs_update(long long n, double* V, long long ldv, int j, const double* coef,
                       const int* gate, double* partials, int nblocks, hipStream_t s) {
  const dim3 grid(nblocks), block(kBlock);
  prof_begin(KKTDD_K_ARNOLDI, s);
  if (j <= 8)
    hipLaunchKernelGGL((k_dcgs_update<8>), grid, block, 0, s, n, V, ldv, j, coef, gate, partials);
  else if (j <= 16)
    hipLaunchKernelGGL((k_dcgs_update<16>), grid, block, 0, s, n, V, ldv, j, coef, gate, partials);
  else if (j <= 24)
    hipLaunchKernelGGL((k_dcgs_update<24>), grid, block, 0, s, n, V, ldv, j, coef, gate, partials);
  else if (j <= 32)
    hipLaunchKernelGGL((k_dcgs_update<32>), grid, block, 0, s, n, V, ldv, j, coef, gate, partials);
  else
    hipLaunchKernelGGL((k_dcgs_update<0>), grid, block, 0, s, n, V, ldv, j, coef, gate, partials);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_ARNOLDI, s, 8.0 * (j + 4) * n, 0.0);
  return 0;
}

int launch_dcgs_finish(int j, const double* sums, double* vinv, double* coef, double* rec,
                       int* gate, int stage, hipStream_t s) {
  prof_begin(KKTDD_K_ARNOLDI, s);
  hipLaunchKernelGGL(k_dcgs_finish, dim3(1), dim3(64), 0, s, j, sums, vinv, coef, rec, gate, stage);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_ARNOLDI, s, 0.0, 0.0);
  return 0;
}

int launch_update_solution(const Geom& g, const double* V, long long ldv, const double* Zw,
                           long long ldz, int nv, const double* yv, const double* yw,
                           const double* vinv, double su, double sz, double* x, hipStream_t s) {
  const long long n3 = 3 * g.P;
  long long nb = (n3 + kBlock - 1) / kBlock;
  if (nb > 8192) nb = 8192;
  prof_begin(KKTDD_K_OTHER, s);
  hipLaunchKernelGGL(k_update_solution, dim3((unsigned)nb), dim3(kBlock), 0, s, g, V, ldv, Zw, ldz,
                     nv, yv, yw, vinv, su, sz, x);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_OTHER, s, 8.0 * g.P * (2.0 * nv + nv + 6.0), 0.0);
  return 0;
}

int launch_sumsq_blocks(const Geom& g, const double* r, double* partials, int nblocks,
                        hipStream_t s) {
  prof_begin(KKTDD_K_OTHER, s);
  hipLaunchKernelGGL(k_sumsq_blocks, dim3(nblocks), dim3(kBlock), 0, s, g, r, partials);
  KKT_HIP(hipGetLastError());
  prof_end(KKTDD_K_OTHER, s, 24.0 * g.P, 0.0);
  return 0;
}

}  // namespace kktdd
