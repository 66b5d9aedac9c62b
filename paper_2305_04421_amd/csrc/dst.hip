// Dirichlet spatial solves as sine-transform GEMMs on MFMA, and the RASQ time sweeps.
//
// Spatial solve (every step of a sweep, Sec. 3-4): D = shift*I + dt*nu*A_h is diagonalised by
// the 2-D discrete sine transform,
//     D^{-1} b = (4/(nx ny)) S_y [ (S_y b S_x) ./ (shift + dt*nu*(lam^y_q + lam^x_p)) ] S_x,
// with S_x[p][i] = sin(pi (p+1)(i+1)/nx) symmetric and S_x S_x = (nx/2) I.  The 4/(nx ny)
// factor is folded into the inverse eigenvalue table.  A solve is four dense GEMMs.
//
// Work split.  A slice b is (my x mx), rows = y.  Right products (. S_x) only mix within a
// row, left products (S_y .) only within a column.  A solve is therefore arranged as
//     row kernel:    T  = b S_x                               (row blocks of 16)
//     column kernel: X  = (S_y T) ./ lambda ;  U = S_y X      (column blocks of 16)
//     row kernel:    y  = U S_x                               (row blocks of 16)
// and in a sweep the last row product of step j and the first of step j+1 run in the same
// row kernel (b_{j+1} = r'_{j+1} + y_j is formed row-locally), so one step costs one row and
// one column launch, each doing two chained 16 x M x M GEMMs.
//
// MFMA: 16x16x4 (f64 or f32).  Lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator
// element r (0..3) holds D[row][l%16] with row = 4*(l/16)+r for f32 and row = l/16 + 4*r for
// f64 (checked on gfx950).  The sine matrices are read straight from
// L2 (they are shared by every workgroup) using their symmetry so that each MFMA operand load
// is four 64-byte or 128-byte row segments; the other operand sits in LDS.
#include <cstdlib>

#include "internal.h"

namespace kktdd {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct AccT;
template <> struct AccT<double> { using type = v4d; };
template <> struct AccT<float> { using type = v4f; };

__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row (within the 16x16 tile) of accumulator element r in lane group lk = l/16.
template <typename T> __device__ inline int acc_row(int lk, int r);
template <> __device__ inline int acc_row<float>(int lk, int r) { return 4 * lk + r; }
template <> __device__ inline int acc_row<double>(int lk, int r) { return lk + 4 * r; }

// ---- tile GEMMs ------------------------------------------------------------------------
// Work split inside a workgroup: the M/16 column (or row) tiles of a 16-wide block are dealt
// to nw waves, TPW tiles each, with nw * TPW == M/16 exactly (the padded extents are chosen so
// that this holds).  The sine-matrix operand comes from L2 through a register ring that runs
// kPD k-steps ahead of the MFMAs, hiding the L2 latency; the LDS operand is read in place.
constexpr int kPD = 4;

// acc[t] += A (16 x M, in LDS with row stride lda) * S(:, tile wave + t*nw), S symmetric M x M.
template <typename T, int TPW, typename Acc>
__device__ inline void gemm_right(const T* A, int lda, const T* __restrict__ S, int M, int wave,
                                  int nw, int li, int lk, Acc (&acc)[TPW]) {
  const T* Sp = S + (long long)lk * M + wave * 16 + li;
  const long long tstride = (long long)nw * 16;
  T bq[kPD][TPW];
#pragma unroll
  for (int p = 0; p < kPD; ++p)
#pragma unroll
    for (int t = 0; t < TPW; ++t) bq[p][t] = Sp[(long long)(4 * p) * M + t * tstride];
  const int nks = M >> 2;
  for (int ks0 = 0; ks0 < nks; ks0 += kPD) {
#pragma unroll
    for (int p = 0; p < kPD; ++p) {
      const int ks = ks0 + p;
      const T a = A[li * lda + 4 * ks + lk];
#pragma unroll
      for (int t = 0; t < TPW; ++t) acc[t] = mfma16(a, bq[p][t], acc[t]);
      const int kn = ks + kPD;
      if (kn < nks) {
#pragma unroll
        for (int t = 0; t < TPW; ++t) bq[p][t] = Sp[(long long)(4 * kn) * M + t * tstride];
      }
    }
  }
}

// acc[t] += S(row tile wave + t*nw, :) * B (M x 16, in LDS with row stride ldb).
template <typename T, int TPW, typename Acc>
__device__ inline void gemm_left(const T* __restrict__ S, const T* B, int ldb, int M, int wave,
                                 int nw, int li, int lk, Acc (&acc)[TPW]) {
  // A(row = li, k = lk) of tile rt is S[rt*16 + li][k0 + lk] = S[k0 + lk][rt*16 + li].
  const T* Sp = S + (long long)lk * M + wave * 16 + li;
  const long long tstride = (long long)nw * 16;
  T aq[kPD][TPW];
#pragma unroll
  for (int p = 0; p < kPD; ++p)
#pragma unroll
    for (int t = 0; t < TPW; ++t) aq[p][t] = Sp[(long long)(4 * p) * M + t * tstride];
  const int nks = M >> 2;
  for (int ks0 = 0; ks0 < nks; ks0 += kPD) {
#pragma unroll
    for (int p = 0; p < kPD; ++p) {
      const int ks = ks0 + p;
      const T b = B[(4 * ks + lk) * ldb + li];
#pragma unroll
      for (int t = 0; t < TPW; ++t) acc[t] = mfma16(aq[p][t], b, acc[t]);
      const int kn = ks + kPD;
      if (kn < nks) {
#pragma unroll
        for (int t = 0; t < TPW; ++t) aq[p][t] = Sp[(long long)(4 * kn) * M + t * tstride];
      }
    }
  }
}

// ---- row kernel ------------------------------------------------------------------------
// One workgroup = 16 rows of one slice.  Optional GEMM1 (y = g1_scale * U S_x) with its
// epilogue stores, then optional formation of b and GEMM2 (T = b S_x).
enum BMode { B_NONE = 0, B_RPRIME_PLUS_Y = 1, B_H_YBUF_PLUS_Y = 2, B_H_Y = 3, B_INPUT = 4 };
enum OutMode { OUT_NONE = 0, OUT_OWNED = 1, OUT_PLAIN = 2 };

template <typename T>
struct RowArgs {
  const T* Sx;
  const T* g1_in;            // padded slices (nullptr: y = 0)
  long long g1_stride;
  double g1_scale;
  T* ystore;                 // padded; nullptr: no store
  long long ystore_stride;
  int out_mode;
  double* out64;             // OUT_OWNED: z_w field (nt slices); OUT_PLAIN: nslices slices
  const double* c0;          // coarse slots added to OUT_OWNED / OUT_PLAIN field output (nullptr: none)
  int g1_step;               // sweep step of the GEMM1 result (OUT_OWNED)
  int b_mode;
  int b_step;                // sweep step whose right-hand side is formed (B_RPRIME_PLUS_Y)
  const double* rin;         // r' field (nt slices) or plain input slices (B_INPUT)
  const double* in_scale;    // device factor of the B_INPUT slices (nullptr: 1)
  const T* ybuf_in;          // padded (B_H_YBUF_PLUS_Y)
  long long ybuf_stride;
  T* g2_out;                 // padded
  long long g2_stride;
};

template <typename T, int TPW>
__global__ void __launch_bounds__(512)
k_rows(Geom g, RowArgs<T> a) {
  using acc_t = typename AccT<T>::type;
  extern __shared__ unsigned char smem_raw[];
  T* A = reinterpret_cast<T*>(smem_raw);          // [16][Mx+1]
  const int Mx = g.Mx, lda = Mx + 1;
  const int rb = blockIdx.x, s = blockIdx.y;
  const int nthr = blockDim.x, nw = nthr >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  acc_t acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = acc_t{0, 0, 0, 0};

  // node of a sweep step in this subdomain (0-based subdomain s): first = s*k + 1 - delta
  const int first = s * g.k + 1 - g.delta;

  // Right-hand-side operands of b, fetched before GEMM1 so their latency hides behind it.
  T pre[TPW][4];
  if (a.b_mode == B_RPRIME_PLUS_Y || a.b_mode == B_H_YBUF_PLUS_Y || a.b_mode == B_INPUT) {
    const int bnode = first + a.b_step;
    const double isc = (a.b_mode == B_INPUT && a.in_scale) ? *a.in_scale : 1.0;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int col = (wave + t * nw) * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb * 16 + acc_row<T>(lk, r);
        const bool in = row < g.my && col < g.mx;
        T v = 0;
        if (a.b_mode == B_RPRIME_PLUS_Y) {
          if (in && bnode >= 1) v = (T)a.rin[(long long)(bnode - 1) * g.nxy + row * g.mx + col];
        } else if (a.b_mode == B_H_YBUF_PLUS_Y) {
          v = a.ybuf_in[s * a.ybuf_stride + (long long)row * Mx + col];
        } else if (in) {
          v = (T)(isc * a.rin[(long long)s * g.nxy + row * g.mx + col]);
        }
        pre[t][r] = v;
      }
    }
  }

  // ---- GEMM1: y = U S_x ------------------------------------------------------------------
  if (a.g1_in) {
    const T* src = a.g1_in + s * a.g1_stride + (long long)rb * 16 * Mx;
    for (int e = threadIdx.x; e < 16 * Mx; e += nthr) A[(e / Mx) * lda + e % Mx] = src[e];
    __syncthreads();
    gemm_right<T, TPW>(A, lda, a.Sx, Mx, wave, nw, li, lk, acc);
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[t][r] = (T)(acc[t][r] * a.g1_scale);
  }

  // ---- GEMM1 epilogue stores -------------------------------------------------------------
  if (a.g1_in) {
    const int node = first + a.g1_step;
    const bool owned = a.g1_step >= g.delta;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int col = (wave + t * nw) * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb * 16 + acc_row<T>(lk, r);
        const T v = acc[t][r];
        if (a.ystore) a.ystore[s * a.ystore_stride + (long long)row * Mx + col] = v;
        if (row < g.my && col < g.mx) {
          if (a.out_mode == OUT_PLAIN) {
            double val = (double)v;
            if (a.c0) {   // slice s is time-node s+1 of a field: add the prolonged coarse part
              const int n = s + 1, sd = s / g.k;
              const double* c = a.c0 + (long long)(g.nb * sd) * g.nxy + row * g.mx + col;
              val += c[0];
              if (g.nb == 2) val += (-1.0 + 2.0 * (double)(n - sd * g.k) / g.k) * c[g.nxy];
            }
            a.out64[(long long)s * g.nxy + row * g.mx + col] = val;
          } else if (a.out_mode == OUT_OWNED && owned) {
            const long long pt = row * g.mx + col;
            double val = (double)v;
            if (a.c0) {
              const double* c = a.c0 + (long long)(g.nb * s) * g.nxy + pt;
              val += c[0];
              if (g.nb == 2) val += (-1.0 + 2.0 * (double)(node - s * g.k) / g.k) * c[g.nxy];
            }
            a.out64[(long long)(node - 1) * g.nxy + pt] = val;
          }
        }
      }
    }
  }
  if (a.b_mode == B_NONE) return;

  // ---- form b (row-local) into LDS -------------------------------------------------------
  __syncthreads();  // every wave has finished reading A for GEMM1
  {
    const T hT = (T)g.h;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int col = (wave + t * nw) * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rloc = acc_row<T>(lk, r);
        T b = 0;
        switch (a.b_mode) {
          case B_RPRIME_PLUS_Y: b = pre[t][r] + acc[t][r]; break;
          case B_H_YBUF_PLUS_Y: b = hT * pre[t][r] + acc[t][r]; break;
          case B_H_Y: b = hT * acc[t][r]; break;
          case B_INPUT: b = pre[t][r]; break;
        }
        A[rloc * lda + col] = b;
      }
    }
  }
  __syncthreads();

  // ---- GEMM2: T = b S_x ------------------------------------------------------------------
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = acc_t{0, 0, 0, 0};
  gemm_right<T, TPW>(A, lda, a.Sx, Mx, wave, nw, li, lk, acc);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int col = (wave + t * nw) * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rb * 16 + acc_row<T>(lk, r);
      a.g2_out[s * a.g2_stride + (long long)row * Mx + col] = acc[t][r];
    }
  }
}

// ---- column kernel ---------------------------------------------------------------------
// One workgroup = 16 columns of one slice: X = S_y T (optionally ./ lambda), and optionally
// U = S_y X chained through LDS.
template <typename T>
struct ColArgs {
  const T* Sy;
  const T* in;
  long long in_stride;
  const T* invlam;     // nullptr: no scaling
  int two;             // chain the second product
  T* out;
  long long out_stride;
};

template <typename T, int TPW>
__global__ void __launch_bounds__(512)
k_cols(Geom g, ColArgs<T> a) {
  using acc_t = typename AccT<T>::type;
  extern __shared__ unsigned char smem_raw[];
  T* B = reinterpret_cast<T*>(smem_raw);          // [My][17]
  constexpr int ldb = 17;
  const int Mx = g.Mx, My = g.My;
  const int cb = blockIdx.x, s = blockIdx.y;
  const int nthr = blockDim.x, nw = nthr >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;

  const T* src = a.in + s * a.in_stride + cb * 16;
  for (int e = threadIdx.x; e < My * 16; e += nthr) B[(e >> 4) * ldb + (e & 15)] = src[(long long)(e >> 4) * Mx + (e & 15)];
  __syncthreads();

  acc_t acc[TPW];
  for (int pass = 0; pass < 1 + a.two; ++pass) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = acc_t{0, 0, 0, 0};
    gemm_left<T, TPW>(a.Sy, B, ldb, My, wave, nw, li, lk, acc);
    if (pass == 0 && a.invlam) {
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[t][r] *= a.invlam[(long long)((wave + t * nw) * 16 + acc_row<T>(lk, r)) * Mx + cb * 16 + li];
    }
    if (pass == 0 && a.two) {
      __syncthreads();
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) B[((wave + t * nw) * 16 + acc_row<T>(lk, r)) * ldb + li] = acc[t][r];
      __syncthreads();
    }
  }
  T* dst = a.out + s * a.out_stride + cb * 16;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      dst[(long long)((wave + t * nw) * 16 + acc_row<T>(lk, r)) * Mx + li] = acc[t][r];
}

// ---- launch helpers ----------------------------------------------------------------------
// Waves per workgroup for M/16 tiles: every wave gets the same number of tiles (<= 8).
// The preferred width is 8 waves (KKTDD_GEMM_WAVES=4 selects 4).
inline int wave_cap() {
  static const int cap = [] {
    const char* v = std::getenv("KKTDD_GEMM_WAVES");
    return (v && std::atoi(v) == 4) ? 4 : 8;
  }();
  return cap;
}

inline int waves_for(int M) {
  const int t = M / 16, cap = wave_cap();
  if (t <= 4) return t;
  if (t <= 8) return (t == 8 && cap == 4) ? 4 : t;
  if (t % cap == 0 && t / cap <= 8) return cap;
  if (t % 4 == 0 && t / 4 <= 8) return 4;
  return 8;   // padded extents make t a multiple of 8 here
}

// Dynamic LDS above 64 KiB has to be enabled per kernel before the first launch.
template <typename F>
int allow_lds(F* kernel, size_t lds) {
  if (lds > 65536)
    KKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return 0;
}

// Algorithmic flops of one launch: 2*my*mx*mx per right product, 2*my*my*mx per left product.
template <typename T, int TPW>
int rows_t(const Geom& g, const RowArgs<T>& a, int nslices, int nw, int kclass, hipStream_t s) {
  const size_t lds = (size_t)16 * (g.Mx + 1) * sizeof(T);
  if (int e = allow_lds(k_rows<T, TPW>, lds)) return e;
  const int ngemm = (a.g1_in ? 1 : 0) + (a.b_mode != B_NONE ? 1 : 0);
  prof_begin(kclass, s);
  hipLaunchKernelGGL((k_rows<T, TPW>), dim3(g.My / 16, nslices), dim3(64 * nw), lds, s, g, a);
  KKT_HIP(hipGetLastError());
  prof_end(kclass, s, 0.0, 2.0 * ngemm * nslices * (double)g.my * g.mx * g.mx);
  return 0;
}

template <typename T, int TPW>
int cols_t(const Geom& g, const ColArgs<T>& a, int nslices, int nw, int kclass, hipStream_t s) {
  const size_t lds = (size_t)g.My * 17 * sizeof(T);
  if (int e = allow_lds(k_cols<T, TPW>, lds)) return e;
  prof_begin(kclass, s);
  hipLaunchKernelGGL((k_cols<T, TPW>), dim3(g.Mx / 16, nslices), dim3(64 * nw), lds, s, g, a);
  KKT_HIP(hipGetLastError());
  prof_end(kclass, s, 0.0, 2.0 * (1 + a.two) * nslices * (double)g.my * g.my * g.mx);
  return 0;
}

#define KKT_TPW_DISPATCH(FN, TPWV, ...)                  \
  switch (TPWV) {                                        \
    case 1: return FN<T, 1>(__VA_ARGS__);                \
    case 2: return FN<T, 2>(__VA_ARGS__);                \
    case 3: return FN<T, 3>(__VA_ARGS__);                \
    case 4: return FN<T, 4>(__VA_ARGS__);                \
    case 5: return FN<T, 5>(__VA_ARGS__);                \
    case 6: return FN<T, 6>(__VA_ARGS__);                \
    case 7: return FN<T, 7>(__VA_ARGS__);                \
    case 8: return FN<T, 8>(__VA_ARGS__);                \
    default: return set_error(KKTDD_EINVAL, "unsupported tile count"); \
  }

template <typename T>
int rows(const Geom& g, const RowArgs<T>& a, int nslices, int kclass, hipStream_t s) {
  const int nw = waves_for(g.Mx);
  KKT_TPW_DISPATCH(rows_t, g.Mx / 16 / nw, g, a, nslices, nw, kclass, s)
}

template <typename T>
int cols(const Geom& g, const ColArgs<T>& a, int nslices, int kclass, hipStream_t s) {
  const int nw = waves_for(g.My);
  KKT_TPW_DISPATCH(cols_t, g.My / 16 / nw, g, a, nslices, nw, kclass, s)
}

template <typename T>
RowArgs<T> row_args(const void* Sx) {
  RowArgs<T> a{};
  a.Sx = static_cast<const T*>(Sx);
  a.g1_scale = 1.0;
  return a;
}

template <typename T>
int spatial_solve_t(const Geom& g, const void* Sx, const void* Sy, const void* invlam,
                    const double* b, double* x, int nslices, void* w1, void* w2, hipStream_t s) {
  const long long MM = g.padded();
  RowArgs<T> r1 = row_args<T>(Sx);
  r1.b_mode = B_INPUT;
  r1.rin = b;
  r1.g2_out = static_cast<T*>(w1);
  r1.g2_stride = MM;
  if (int e = rows<T>(g, r1, nslices, KKTDD_K_OTHER, s)) return e;
  ColArgs<T> c{static_cast<const T*>(Sy), static_cast<const T*>(w1), MM,
               static_cast<const T*>(invlam), 1, static_cast<T*>(w2), MM};
  if (int e = cols<T>(g, c, nslices, KKTDD_K_OTHER, s)) return e;
  RowArgs<T> r2 = row_args<T>(Sx);
  r2.g1_in = static_cast<const T*>(w2);
  r2.g1_stride = MM;
  r2.out_mode = OUT_PLAIN;
  r2.out64 = x;
  return rows<T>(g, r2, nslices, KKTDD_K_OTHER, s);
}

// RASQ sweeps (Eq. (13)) of all subdomains in lockstep.  Subdomain s (0-based) covers the
// nodes s*k+1-delta .. (s+1)*k (sweep steps j = 0..L-1, L = k+delta); for s = 0 the nodes
// below 1 carry a zero right-hand side, which keeps the state exactly zero there, so every
// subdomain runs the same L steps.
template <typename T>
int sweeps_t(const Geom& g, const void* Sx, const void* Sy, const void* invlam,
             const double* rprime, const double* c0, double* zw, void* Tb, void* Ub, void* Yb,
             hipStream_t s) {
  const long long MM = g.padded();
  T* Tbuf = static_cast<T*>(Tb);
  T* Ubuf = static_cast<T*>(Ub);
  T* Ybuf = static_cast<T*>(Yb);
  const long long ystride = (long long)g.L * MM;
  const int nd = g.nd, L = g.L;
  ColArgs<T> c{static_cast<const T*>(Sy), Tbuf, MM, static_cast<const T*>(invlam), 1, Ubuf, MM};

  // forward sweep: y_j = D^{-1}(r'_j + y_{j-1})
  for (int j = 0; j < L; ++j) {
    RowArgs<T> r = row_args<T>(Sx);
    if (j > 0) {
      r.g1_in = Ubuf;
      r.g1_stride = MM;
      r.ystore = Ybuf + (long long)(j - 1) * MM;
      r.ystore_stride = ystride;
    }
    r.b_mode = B_RPRIME_PLUS_Y;
    r.b_step = j;
    r.rin = rprime;
    r.g2_out = Tbuf;
    r.g2_stride = MM;
    if (int e = rows<T>(g, r, nd, KKTDD_K_SWEEP_ROWS, s)) return e;
    if (int e = cols<T>(g, c, nd, KKTDD_K_SWEEP_COLS, s)) return e;
  }
  // junction: y_{L-1} from the last solve; adjoint right-hand side h*y_{L-1}
  {
    RowArgs<T> r = row_args<T>(Sx);
    r.g1_in = Ubuf;
    r.g1_stride = MM;
    r.b_mode = B_H_Y;
    r.g2_out = Tbuf;
    r.g2_stride = MM;
    if (int e = rows<T>(g, r, nd, KKTDD_K_SWEEP_ROWS, s)) return e;
    if (int e = cols<T>(g, c, nd, KKTDD_K_SWEEP_COLS, s)) return e;
  }
  // adjoint sweep: x_j = D^{-1}(h y_j + x_{j+1}); owned x_{j+1} written with the coarse part
  for (int j = L - 2; j >= 0; --j) {
    RowArgs<T> r = row_args<T>(Sx);
    r.g1_in = Ubuf;
    r.g1_stride = MM;
    r.out_mode = OUT_OWNED;
    r.out64 = zw;
    r.c0 = c0;
    r.g1_step = j + 1;
    r.b_mode = B_H_YBUF_PLUS_Y;
    r.b_step = j;
    r.ybuf_in = Ybuf + (long long)j * MM;
    r.ybuf_stride = ystride;
    r.g2_out = Tbuf;
    r.g2_stride = MM;
    if (int e = rows<T>(g, r, nd, KKTDD_K_SWEEP_ROWS, s)) return e;
    if (int e = cols<T>(g, c, nd, KKTDD_K_SWEEP_COLS, s)) return e;
  }
  RowArgs<T> r = row_args<T>(Sx);
  r.g1_in = Ubuf;
  r.g1_stride = MM;
  r.out_mode = OUT_OWNED;
  r.out64 = zw;
  r.c0 = c0;
  r.g1_step = 0;
  r.b_mode = B_NONE;
  return rows<T>(g, r, nd, KKTDD_K_SWEEP_ROWS, s);
}

template <typename T>
int dst_forward_t(const Geom& g, const void* Sx, const void* Sy, const double* in,
                  const double* dscale, void* tmp, void* out, int nslices, hipStream_t s) {
  const long long MM = g.padded();
  RowArgs<T> r = row_args<T>(Sx);
  r.b_mode = B_INPUT;
  r.rin = in;
  r.in_scale = dscale;
  r.g2_out = static_cast<T*>(tmp);
  r.g2_stride = MM;
  if (int e = rows<T>(g, r, nslices, KKTDD_K_SWEEP_ROWS, s)) return e;
  ColArgs<T> c{static_cast<const T*>(Sy), static_cast<const T*>(tmp), MM, nullptr, 0,
               static_cast<T*>(out), MM};
  return cols<T>(g, c, nslices, KKTDD_K_SWEEP_COLS, s);
}

template <typename T>
int dst_inverse_t(const Geom& g, const void* Sx, const void* Sy, const void* in, void* tmp,
                  double* out, int nslices, double norm, const double* c0, hipStream_t s) {
  const long long MM = g.padded();
  ColArgs<T> c{static_cast<const T*>(Sy), static_cast<const T*>(in), MM, nullptr, 0,
               static_cast<T*>(tmp), MM};
  if (int e = cols<T>(g, c, nslices, KKTDD_K_SWEEP_COLS, s)) return e;
  RowArgs<T> r = row_args<T>(Sx);
  r.g1_in = static_cast<const T*>(tmp);
  r.g1_stride = MM;
  r.g1_scale = norm;
  r.out_mode = OUT_PLAIN;
  r.out64 = out;
  r.c0 = c0;
  return rows<T>(g, r, nslices, KKTDD_K_SWEEP_ROWS, s);
}

}  // namespace

int launch_dst_forward(const Geom& g, int precision, const void* Sx, const void* Sy,
                       const double* in, const double* dscale, void* tmp, void* out, int nslices,
                       hipStream_t s) {
  if (precision == KKTDD_FP32) return dst_forward_t<float>(g, Sx, Sy, in, dscale, tmp, out, nslices, s);
  return dst_forward_t<double>(g, Sx, Sy, in, dscale, tmp, out, nslices, s);
}

int launch_dst_inverse(const Geom& g, int precision, const void* Sx, const void* Sy,
                       const void* in, void* tmp, double* out, int nslices, double norm,
                       const double* c0, hipStream_t s) {
  if (precision == KKTDD_FP32) return dst_inverse_t<float>(g, Sx, Sy, in, tmp, out, nslices, norm, c0, s);
  return dst_inverse_t<double>(g, Sx, Sy, in, tmp, out, nslices, norm, c0, s);
}

int launch_spatial_solve(const Geom& g, int precision, const void* Sx, const void* Sy,
                         const void* invlam, const double* b, double* x, int nslices,
                         void* work1, void* work2, hipStream_t s) {
  if (nslices <= 0) return 0;
  if (precision == KKTDD_FP32)
    return spatial_solve_t<float>(g, Sx, Sy, invlam, b, x, nslices, work1, work2, s);
  return spatial_solve_t<double>(g, Sx, Sy, invlam, b, x, nslices, work1, work2, s);
}

int launch_sweeps(const Geom& g, int precision, const void* Sx, const void* Sy,
                  const void* invlam, const double* rprime, const double* c0, double* zw,
                  void* Tbuf, void* Ubuf, void* Ybuf, hipStream_t s) {
  if (precision == KKTDD_FP32)
    return sweeps_t<float>(g, Sx, Sy, invlam, rprime, c0, zw, Tbuf, Ubuf, Ybuf, s);
  return sweeps_t<double>(g, Sx, Sy, invlam, rprime, c0, zw, Tbuf, Ubuf, Ybuf, s);
}

int launch_coarse_dst(const Geom& g, const double* Sx, const double* Sy, const double* r0,
                      double* rhat, double* tmp, hipStream_t s) {
  const long long MM = g.padded();
  RowArgs<double> r = row_args<double>(Sx);
  r.b_mode = B_INPUT;
  r.rin = r0;
  r.g2_out = tmp;
  r.g2_stride = MM;
  if (int e = rows<double>(g, r, g.nc, KKTDD_K_COARSE, s)) return e;
  ColArgs<double> c{Sy, tmp, MM, nullptr, 0, rhat, MM};
  return cols<double>(g, c, g.nc, KKTDD_K_COARSE, s);
}

int launch_coarse_idst(const Geom& g, const double* Sx, const double* Sy, const double* chat,
                       double* c0, double* tmp, double norm, hipStream_t s) {
  const long long MM = g.padded();
  ColArgs<double> c{Sy, chat, MM, nullptr, 0, tmp, MM};
  if (int e = cols<double>(g, c, g.nc, KKTDD_K_COARSE, s)) return e;
  RowArgs<double> r = row_args<double>(Sx);
  r.g1_in = tmp;
  r.g1_stride = MM;
  r.g1_scale = norm;
  r.out_mode = OUT_PLAIN;
  r.out64 = c0;
  return rows<double>(g, r, g.nc, KKTDD_K_COARSE, s);
}

}  // namespace kktdd
