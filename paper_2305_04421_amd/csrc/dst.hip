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
// GEMM engines (one per arithmetic):
//   f64, f32      16x16x4 MFMA.  Lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator
//                 element r holds D[row][l%16], row = 4*(l/16)+r (f32) or l/16 + 4*r (f64).
//   bf16 x1/x3/x6 16x16x32 bf16 MFMA with float32 accumulation.  Lane l supplies
//                 A[l%16][8*(l/16)+i] and B[8*(l/16)+i][l%16], i = 0..7; D as for f32.  A
//                 float32 operand a is split into bfloat16 parts a0 + a1 + a2 (each part the
//                 rounded remainder of the previous ones) and a product is accumulated from
//                 the part products a0b0 (x1); a0b0 + a0b1 + a1b0 (x3); and those plus
//                 a0b2 + a1b1 + a2b0 (x6) (Henry, Tang, Heinecke, ARITH 2019).
// All layouts were checked on gfx950.  The sine matrices (pre-split into bf16 parts for the
// bf16 engines) are read straight from L2 using their symmetry, so every operand load is a
// run of contiguous row segments; the other operand sits in LDS.  Work buffers are float64
// for the f64 engine and float32 otherwise.
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include "internal.h"

namespace kktdd {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T> struct AccT;
template <> struct AccT<double> { using type = v4d; };
template <> struct AccT<float> { using type = v4f; };

__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma_bf(bf16x8 a, bf16x8 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Work split inside a workgroup: the M/16 column (or row) tiles of a 16-wide block are dealt
// to nw waves, TPW tiles each, with nw * TPW == M/16 exactly (the padded extents are chosen so
// that this holds).  The sine-matrix operand comes from L2 through a register ring that runs
// ahead of the MFMAs, hiding the L2 latency; the LDS operand is read in place.  The ring is
// PD k-steps deep: 4 by default, deeper (16 for one tile per wave, 8 for two to four) where
// the autotuner measured it faster.
constexpr int kPDDefault = 4;
template <int TPW>
constexpr int deep_prefetch() { return TPW == 1 ? 16 : (TPW <= 4 ? 8 : kPDDefault); }

// ---- plain engines (f64, f32) ----------------------------------------------------------
template <typename T>
struct EngPlain {
  using data_t = T;
  using acc_t = typename AccT<T>::type;
  using s_t = T;
  static __host__ __device__ size_t rows_lds(int M) { return (size_t)16 * (M + 1) * sizeof(T); }
  static __host__ __device__ size_t cols_lds(int M) { return (size_t)M * 17 * sizeof(T); }
  static __device__ int acc_row(int lk, int r) {
    if constexpr (sizeof(T) == 8) return lk + 4 * r; else return 4 * lk + r;
  }
  // rows operand A[16][M+1]
  static __device__ void put_a(unsigned char* lds, int M, int r, int c, T v) {
    reinterpret_cast<T*>(lds)[r * (M + 1) + c] = v;
  }
  // cols operand B[M][17]
  static __device__ void put_b(unsigned char* lds, int M, int k, int c, T v) {
    (void)M;
    reinterpret_cast<T*>(lds)[k * 17 + c] = v;
  }
  // acc[t] += A (16 x M) * S(:, tile wave + t*nw), S symmetric M x M.
  template <int TPW, int kPD>
  static __device__ void gemm_right(const unsigned char* lds, const T* __restrict__ S, int M,
                                    int wave, int nw, int li, int lk, acc_t (&acc)[TPW]) {
    const T* A = reinterpret_cast<const T*>(lds);
    const int lda = M + 1;
    const T* Sp = S + (long long)lk * M + wave * 16 + li;
    const long long tstride = (long long)nw * 16;
    const int nks = M >> 2;
    T bq[kPD][TPW];
#pragma unroll
    for (int p = 0; p < kPD; ++p)
      if (p < nks) {
#pragma unroll
        for (int t = 0; t < TPW; ++t) bq[p][t] = Sp[(long long)(4 * p) * M + t * tstride];
      }
    for (int ks0 = 0; ks0 < nks; ks0 += kPD) {
#pragma unroll
      for (int p = 0; p < kPD; ++p) {
        const int ks = ks0 + p;
        if (ks >= nks) break;
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
  // acc[t] += S(row tile wave + t*nw, :) * B (M x 16).
  template <int TPW, int kPD>
  static __device__ void gemm_left(const T* __restrict__ S, const unsigned char* lds, int M,
                                   int wave, int nw, int li, int lk, acc_t (&acc)[TPW]) {
    const T* B = reinterpret_cast<const T*>(lds);
    // A(row = li, k = lk) of tile rt is S[rt*16 + li][k0 + lk] = S[k0 + lk][rt*16 + li].
    const T* Sp = S + (long long)lk * M + wave * 16 + li;
    const long long tstride = (long long)nw * 16;
    const int nks = M >> 2;
    T aq[kPD][TPW];
#pragma unroll
    for (int p = 0; p < kPD; ++p)
      if (p < nks) {
#pragma unroll
        for (int t = 0; t < TPW; ++t) aq[p][t] = Sp[(long long)(4 * p) * M + t * tstride];
      }
    for (int ks0 = 0; ks0 < nks; ks0 += kPD) {
#pragma unroll
      for (int p = 0; p < kPD; ++p) {
        const int ks = ks0 + p;
        if (ks >= nks) break;
        const T b = B[(4 * ks + lk) * 17 + li];
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
};

// ---- split-bfloat16 engines -------------------------------------------------------------
template <int SPLIT>
struct EngBF {
  static constexpr int NP = SPLIT == 1 ? 1 : (SPLIT == 3 ? 2 : 3);   // parts per operand
  using data_t = float;
  using acc_t = v4f;
  using s_t = __bf16;    // NP parts of an M x M matrix, part p at offset p*M*M
  static __host__ __device__ size_t rows_lds(int M) { return (size_t)NP * 16 * (M + 8) * 2; }
  static __host__ __device__ size_t cols_lds(int M) { return (size_t)NP * 16 * (M + 8) * 2; }
  static __device__ int acc_row(int lk, int r) { return 4 * lk + r; }
  static __device__ void split(float v, __bf16 (&part)[NP]) {
    part[0] = (__bf16)v;
    if constexpr (NP > 1) {
      const float r1 = v - (float)part[0];
      part[1] = (__bf16)r1;
      if constexpr (NP > 2) part[2] = (__bf16)(r1 - (float)part[1]);
    }
  }
  // rows operand: NP arrays A_p[16][M+8] (k contiguous)
  static __device__ void put_a(unsigned char* lds, int M, int r, int c, float v) {
    __bf16 part[NP];
    split(v, part);
    __bf16* A = reinterpret_cast<__bf16*>(lds);
#pragma unroll
    for (int p = 0; p < NP; ++p) A[(p * 16 + r) * (M + 8) + c] = part[p];
  }
  // cols operand stored transposed: NP arrays Bt_p[16][M+8], Bt_p[c][k] = part_p(B[k][c])
  static __device__ void put_b(unsigned char* lds, int M, int k, int c, float v) {
    __bf16 part[NP];
    split(v, part);
    __bf16* B = reinterpret_cast<__bf16*>(lds);
#pragma unroll
    for (int p = 0; p < NP; ++p) B[(p * 16 + c) * (M + 8) + k] = part[p];
  }
  static __device__ v4f mma(const bf16x8 (&a)[NP], const bf16x8 (&b)[NP], v4f acc) {
    if constexpr (SPLIT == 6) {
      acc = mfma_bf(a[2], b[0], acc);
      acc = mfma_bf(a[1], b[1], acc);
      acc = mfma_bf(a[0], b[2], acc);
    }
    if constexpr (SPLIT >= 3) {
      acc = mfma_bf(a[1], b[0], acc);
      acc = mfma_bf(a[0], b[1], acc);
    }
    return mfma_bf(a[0], b[0], acc);
  }
  static constexpr int ring(int TPW) { return TPW * NP <= 8 ? 2 : 1; }
  // acc[t] += A (16 x M) * S(:, tile wave + t*nw); the B fragment of tile ct is
  // S[32ks + 8lk + i][ct*16 + li] = S[ct*16 + li][32ks + 8lk + i]: 16 contiguous bytes.
  template <int TPW, int PD_unused>
  static __device__ void gemm_right(const unsigned char* lds, const __bf16* __restrict__ S, int M,
                                    int wave, int nw, int li, int lk, acc_t (&acc)[TPW]) {
    constexpr int RD = ring(TPW);
    const __bf16* A = reinterpret_cast<const __bf16*>(lds);
    const long long MM = (long long)M * M;
    const int lda = M + 8;
    auto bload = [&](int ks, int t, int p) {
      const long long row = (long long)(wave + t * nw) * 16 + li;
      return *reinterpret_cast<const bf16x8*>(S + p * MM + row * M + 32 * ks + 8 * lk);
    };
    bf16x8 bq[RD][TPW][NP];
#pragma unroll
    for (int d = 0; d < RD; ++d)
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int p = 0; p < NP; ++p) bq[d][t][p] = bload(d, t, p);
    const int nks = M >> 5;
    for (int ks0 = 0; ks0 < nks; ks0 += RD) {
#pragma unroll
      for (int d = 0; d < RD; ++d) {
        const int ks = ks0 + d;
        if (ks >= nks) break;
        bf16x8 af[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p)
          af[p] = *reinterpret_cast<const bf16x8*>(A + (p * 16 + li) * lda + 32 * ks + 8 * lk);
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[t] = mma(af, bq[d][t], acc[t]);
        const int kn = ks + RD;
        if (kn < nks) {
#pragma unroll
          for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int p = 0; p < NP; ++p) bq[d][t][p] = bload(kn, t, p);
        }
      }
    }
  }
  // acc[t] += S(row tile wave + t*nw, :) * B (M x 16, stored transposed in LDS).
  template <int TPW, int PD_unused>
  static __device__ void gemm_left(const __bf16* __restrict__ S, const unsigned char* lds, int M,
                                   int wave, int nw, int li, int lk, acc_t (&acc)[TPW]) {
    constexpr int RD = ring(TPW);
    const __bf16* Bt = reinterpret_cast<const __bf16*>(lds);
    const long long MM = (long long)M * M;
    const int ldb = M + 8;
    auto aload = [&](int ks, int t, int p) {
      const long long row = (long long)(wave + t * nw) * 16 + li;
      return *reinterpret_cast<const bf16x8*>(S + p * MM + row * M + 32 * ks + 8 * lk);
    };
    bf16x8 aq[RD][TPW][NP];
#pragma unroll
    for (int d = 0; d < RD; ++d)
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int p = 0; p < NP; ++p) aq[d][t][p] = aload(d, t, p);
    const int nks = M >> 5;
    for (int ks0 = 0; ks0 < nks; ks0 += RD) {
#pragma unroll
      for (int d = 0; d < RD; ++d) {
        const int ks = ks0 + d;
        if (ks >= nks) break;
        bf16x8 bf[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p)
          bf[p] = *reinterpret_cast<const bf16x8*>(Bt + (p * 16 + li) * ldb + 32 * ks + 8 * lk);
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[t] = mma(aq[d][t], bf, acc[t]);
        const int kn = ks + RD;
        if (kn < nks) {
#pragma unroll
          for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int p = 0; p < NP; ++p) aq[d][t][p] = aload(kn, t, p);
        }
      }
    }
  }
};

// ---- row kernel ------------------------------------------------------------------------
// One workgroup = 16 rows of one slice.  Optional GEMM1 (y = g1_scale * U S_x) with its
// epilogue stores, then optional formation of b and GEMM2 (T = b S_x).
enum BMode { B_NONE = 0, B_RPRIME_PLUS_Y = 1, B_H_YBUF_PLUS_Y = 2, B_H_Y = 3, B_INPUT = 4 };
enum OutMode { OUT_NONE = 0, OUT_OWNED = 1, OUT_PLAIN = 2 };

template <typename T>
struct RowArgs {
  const void* Sx;            // engine's sine-matrix operand
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

template <typename Eng, int TPW, int PD>
__global__ void __launch_bounds__(512)
k_rows(Geom g, RowArgs<typename Eng::data_t> a) {
  using T = typename Eng::data_t;
  using acc_t = typename Eng::acc_t;
  using S_t = typename Eng::s_t;
  extern __shared__ unsigned char smem_raw[];
  const int Mx = g.Mx;
  const S_t* Sx = static_cast<const S_t*>(a.Sx);
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
        const int row = rb * 16 + Eng::acc_row(lk, r);
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
    for (int e = threadIdx.x; e < 16 * Mx; e += nthr) Eng::put_a(smem_raw, Mx, e / Mx, e % Mx, src[e]);
    __syncthreads();
    Eng::template gemm_right<TPW, PD>(smem_raw, Sx, Mx, wave, nw, li, lk, acc);
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
        const int row = rb * 16 + Eng::acc_row(lk, r);
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
  __syncthreads();  // every wave has finished reading the LDS operand of GEMM1
  {
    const T hT = (T)g.h;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int col = (wave + t * nw) * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rloc = Eng::acc_row(lk, r);
        T b = 0;
        switch (a.b_mode) {
          case B_RPRIME_PLUS_Y: b = pre[t][r] + (T)acc[t][r]; break;
          case B_H_YBUF_PLUS_Y: b = hT * pre[t][r] + (T)acc[t][r]; break;
          case B_H_Y: b = hT * (T)acc[t][r]; break;
          case B_INPUT: b = pre[t][r]; break;
        }
        Eng::put_a(smem_raw, Mx, rloc, col, b);
      }
    }
  }
  __syncthreads();

  // ---- GEMM2: T = b S_x ------------------------------------------------------------------
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = acc_t{0, 0, 0, 0};
  Eng::template gemm_right<TPW, PD>(smem_raw, Sx, Mx, wave, nw, li, lk, acc);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int col = (wave + t * nw) * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rb * 16 + Eng::acc_row(lk, r);
      a.g2_out[s * a.g2_stride + (long long)row * Mx + col] = (T)acc[t][r];
    }
  }
}

// ---- column kernel ---------------------------------------------------------------------
// One workgroup = 16 columns of one slice: X = S_y T (optionally ./ lambda), and optionally
// U = S_y X chained through LDS.
template <typename T>
struct ColArgs {
  const void* Sy;      // engine's sine-matrix operand
  const T* in;
  long long in_stride;
  const T* invlam;     // nullptr: no scaling
  int two;             // chain the second product
  T* out;
  long long out_stride;
};

template <typename Eng, int TPW, int PD>
__global__ void __launch_bounds__(512)
k_cols(Geom g, ColArgs<typename Eng::data_t> a) {
  using T = typename Eng::data_t;
  using acc_t = typename Eng::acc_t;
  using S_t = typename Eng::s_t;
  extern __shared__ unsigned char smem_raw[];
  const int Mx = g.Mx, My = g.My;
  const S_t* Sy = static_cast<const S_t*>(a.Sy);
  const int cb = blockIdx.x, s = blockIdx.y;
  const int nthr = blockDim.x, nw = nthr >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;

  const T* src = a.in + s * a.in_stride + cb * 16;
  for (int e = threadIdx.x; e < My * 16; e += nthr)
    Eng::put_b(smem_raw, My, e >> 4, e & 15, src[(long long)(e >> 4) * Mx + (e & 15)]);
  __syncthreads();

  acc_t acc[TPW];
  for (int pass = 0; pass < 1 + a.two; ++pass) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = acc_t{0, 0, 0, 0};
    Eng::template gemm_left<TPW, PD>(Sy, smem_raw, My, wave, nw, li, lk, acc);
    if (pass == 0 && a.invlam) {
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[t][r] *= a.invlam[(long long)((wave + t * nw) * 16 + Eng::acc_row(lk, r)) * Mx + cb * 16 + li];
    }
    if (pass == 0 && a.two) {
      __syncthreads();
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Eng::put_b(smem_raw, My, (wave + t * nw) * 16 + Eng::acc_row(lk, r), li, (T)acc[t][r]);
      __syncthreads();
    }
  }
  T* dst = a.out + s * a.out_stride + cb * 16;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      dst[(long long)((wave + t * nw) * 16 + Eng::acc_row(lk, r)) * Mx + li] = (T)acc[t][r];
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

// ---- autotuned launch shapes ---------------------------------------------------------------
// A launch shape is (waves per workgroup, deep prefetch ring).  Every shape runs the same
// multiply-adds in the same order, so the choice changes the speed only, never the result.
// Choices are measured per (kernel, engine, extent, slices) and kept for the process (and in
// the file KKTDD_TUNE_CACHE names, one JSON object per line, when that is set).
struct Shape {
  int nw;
  int deep;
};
using TuneKey = std::array<int, 4>;   // kind (0 rows, 1 cols), engine, M, slices
std::mutex g_tune_mu;
std::map<TuneKey, Shape> g_tuned;
bool g_tune_loaded = false;

const char* tune_path() {
  const char* p = std::getenv("KKTDD_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    int kind, eng, M, ns, nw, deep;
    if (std::sscanf(line, "{\"kind\": %d, \"engine\": %d, \"M\": %d, \"slices\": %d, \"waves\": %d, "
                    "\"deep\": %d", &kind, &eng, &M, &ns, &nw, &deep) == 6)
      g_tuned[{kind, eng, M, ns}] = Shape{nw, deep};
  }
  std::fclose(f);
}

Shape tuned_shape(int kind, int eng, int M, int nslices) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tuned.find({kind, eng, M, nslices});
  if (it != g_tuned.end()) return it->second;
  return Shape{waves_for(M), 0};
}

template <typename Eng> constexpr int engine_id();
template <> constexpr int engine_id<EngPlain<double>>() { return KKTDD_FP64; }
template <> constexpr int engine_id<EngPlain<float>>() { return KKTDD_FP32; }
template <> constexpr int engine_id<EngBF<1>>() { return KKTDD_BF16; }
template <> constexpr int engine_id<EngBF<3>>() { return KKTDD_BF16X3; }
template <> constexpr int engine_id<EngBF<6>>() { return KKTDD_BF16X6; }

// Dynamic LDS above 64 KiB has to be enabled per kernel before the first launch.
template <typename F>
int allow_lds(F* kernel, size_t lds) {
  if (lds > 65536)
    KKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return 0;
}

// Algorithmic flops of one launch: 2*my*mx*mx per right product, 2*my*my*mx per left product.
template <typename Eng, int TPW, int PD>
int rows_t(const Geom& g, const RowArgs<typename Eng::data_t>& a, int nslices, int nw, int kclass,
           hipStream_t s) {
  const size_t lds = Eng::rows_lds(g.Mx);
  if (int e = allow_lds(k_rows<Eng, TPW, PD>, lds)) return e;
  const int ngemm = (a.g1_in ? 1 : 0) + (a.b_mode != B_NONE ? 1 : 0);
  prof_begin(kclass, s);
  hipLaunchKernelGGL((k_rows<Eng, TPW, PD>), dim3(g.My / 16, nslices), dim3(64 * nw), lds, s, g, a);
  KKT_HIP(hipGetLastError());
  prof_end(kclass, s, 0.0, 2.0 * ngemm * nslices * (double)g.my * g.mx * g.mx);
  return 0;
}

template <typename Eng, int TPW, int PD>
int cols_t(const Geom& g, const ColArgs<typename Eng::data_t>& a, int nslices, int nw, int kclass,
           hipStream_t s) {
  const size_t lds = Eng::cols_lds(g.My);
  if (int e = allow_lds(k_cols<Eng, TPW, PD>, lds)) return e;
  prof_begin(kclass, s);
  hipLaunchKernelGGL((k_cols<Eng, TPW, PD>), dim3(g.Mx / 16, nslices), dim3(64 * nw), lds, s, g, a);
  KKT_HIP(hipGetLastError());
  prof_end(kclass, s, 0.0, 2.0 * (1 + a.two) * nslices * (double)g.my * g.my * g.mx);
  return 0;
}

// (tiles per wave, deep ring) -> instantiation; deep rings exist for up to four tiles.
#define KKT_TPW_DISPATCH(FN, TPWV, DEEP, ...)                                            \
  switch (TPWV) {                                                                        \
    case 1: return (DEEP) ? FN<Eng, 1, deep_prefetch<1>()>(__VA_ARGS__)                  \
                          : FN<Eng, 1, kPDDefault>(__VA_ARGS__);                         \
    case 2: return (DEEP) ? FN<Eng, 2, deep_prefetch<2>()>(__VA_ARGS__)                  \
                          : FN<Eng, 2, kPDDefault>(__VA_ARGS__);                         \
    case 3: return (DEEP) ? FN<Eng, 3, deep_prefetch<3>()>(__VA_ARGS__)                  \
                          : FN<Eng, 3, kPDDefault>(__VA_ARGS__);                         \
    case 4: return (DEEP) ? FN<Eng, 4, deep_prefetch<4>()>(__VA_ARGS__)                  \
                          : FN<Eng, 4, kPDDefault>(__VA_ARGS__);                         \
    case 5: return FN<Eng, 5, kPDDefault>(__VA_ARGS__);                                  \
    case 6: return FN<Eng, 6, kPDDefault>(__VA_ARGS__);                                  \
    case 7: return FN<Eng, 7, kPDDefault>(__VA_ARGS__);                                  \
    case 8: return FN<Eng, 8, kPDDefault>(__VA_ARGS__);                                  \
    default: return set_error(KKTDD_EINVAL, "unsupported tile count");                   \
  }

template <typename Eng>
int rows_shape(const Geom& g, const RowArgs<typename Eng::data_t>& a, int nslices, Shape sh,
               int kclass, hipStream_t s) {
  KKT_TPW_DISPATCH(rows_t, g.Mx / 16 / sh.nw, sh.deep, g, a, nslices, sh.nw, kclass, s)
}

template <typename Eng>
int cols_shape(const Geom& g, const ColArgs<typename Eng::data_t>& a, int nslices, Shape sh,
               int kclass, hipStream_t s) {
  KKT_TPW_DISPATCH(cols_t, g.My / 16 / sh.nw, sh.deep, g, a, nslices, sh.nw, kclass, s)
}

template <typename Eng>
int rows(const Geom& g, const RowArgs<typename Eng::data_t>& a, int nslices, int kclass, hipStream_t s) {
  return rows_shape<Eng>(g, a, nslices, tuned_shape(0, engine_id<Eng>(), g.Mx, nslices), kclass, s);
}

template <typename Eng>
int cols(const Geom& g, const ColArgs<typename Eng::data_t>& a, int nslices, int kclass, hipStream_t s) {
  return cols_shape<Eng>(g, a, nslices, tuned_shape(1, engine_id<Eng>(), g.My, nslices), kclass, s);
}

template <typename T>
RowArgs<T> row_args(const void* Sx) {
  RowArgs<T> a{};
  a.Sx = Sx;
  a.g1_scale = 1.0;
  return a;
}

template <typename Eng>
int spatial_solve_t(const Geom& g, const void* Sx, const void* Sy, const void* invlam,
                    const double* b, double* x, int nslices, void* w1, void* w2, hipStream_t s) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  RowArgs<T> r1 = row_args<T>(Sx);
  r1.b_mode = B_INPUT;
  r1.rin = b;
  r1.g2_out = static_cast<T*>(w1);
  r1.g2_stride = MM;
  if (int e = rows<Eng>(g, r1, nslices, KKTDD_K_OTHER, s)) return e;
  ColArgs<T> c{Sy, static_cast<const T*>(w1), MM,
               static_cast<const T*>(invlam), 1, static_cast<T*>(w2), MM};
  if (int e = cols<Eng>(g, c, nslices, KKTDD_K_OTHER, s)) return e;
  RowArgs<T> r2 = row_args<T>(Sx);
  r2.g1_in = static_cast<const T*>(w2);
  r2.g1_stride = MM;
  r2.out_mode = OUT_PLAIN;
  r2.out64 = x;
  return rows<Eng>(g, r2, nslices, KKTDD_K_OTHER, s);
}

// RASQ sweeps (Eq. (13)) of all subdomains in lockstep.  Subdomain s (0-based) covers the
// nodes s*k+1-delta .. (s+1)*k (sweep steps j = 0..L-1, L = k+delta); for s = 0 the nodes
// below 1 carry a zero right-hand side, which keeps the state exactly zero there, so every
// subdomain runs the same L steps.
template <typename Eng>
int sweeps_t(const Geom& g, const void* Sx, const void* Sy, const void* invlam,
             const double* rprime, const double* c0, double* zw, void* Tb, void* Ub, void* Yb,
             hipStream_t s) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  T* Tbuf = static_cast<T*>(Tb);
  T* Ubuf = static_cast<T*>(Ub);
  T* Ybuf = static_cast<T*>(Yb);
  const long long ystride = (long long)g.L * MM;
  const int nd = g.nd, L = g.L;
  ColArgs<T> c{Sy, Tbuf, MM, static_cast<const T*>(invlam), 1, Ubuf, MM};

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
    if (int e = rows<Eng>(g, r, nd, KKTDD_K_SWEEP_ROWS, s)) return e;
    if (int e = cols<Eng>(g, c, nd, KKTDD_K_SWEEP_COLS, s)) return e;
  }
  // junction: y_{L-1} from the last solve; adjoint right-hand side h*y_{L-1}
  {
    RowArgs<T> r = row_args<T>(Sx);
    r.g1_in = Ubuf;
    r.g1_stride = MM;
    r.b_mode = B_H_Y;
    r.g2_out = Tbuf;
    r.g2_stride = MM;
    if (int e = rows<Eng>(g, r, nd, KKTDD_K_SWEEP_ROWS, s)) return e;
    if (int e = cols<Eng>(g, c, nd, KKTDD_K_SWEEP_COLS, s)) return e;
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
    if (int e = rows<Eng>(g, r, nd, KKTDD_K_SWEEP_ROWS, s)) return e;
    if (int e = cols<Eng>(g, c, nd, KKTDD_K_SWEEP_COLS, s)) return e;
  }
  RowArgs<T> r = row_args<T>(Sx);
  r.g1_in = Ubuf;
  r.g1_stride = MM;
  r.out_mode = OUT_OWNED;
  r.out64 = zw;
  r.c0 = c0;
  r.g1_step = 0;
  r.b_mode = B_NONE;
  return rows<Eng>(g, r, nd, KKTDD_K_SWEEP_ROWS, s);
}

template <typename Eng>
int dst_forward_t(const Geom& g, const void* Sx, const void* Sy, const double* in,
                  const double* dscale, void* tmp, void* out, int nslices, hipStream_t s) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  RowArgs<T> r = row_args<T>(Sx);
  r.b_mode = B_INPUT;
  r.rin = in;
  r.in_scale = dscale;
  r.g2_out = static_cast<T*>(tmp);
  r.g2_stride = MM;
  if (int e = rows<Eng>(g, r, nslices, KKTDD_K_SWEEP_ROWS, s)) return e;
  ColArgs<T> c{Sy, static_cast<const T*>(tmp), MM, nullptr, 0,
               static_cast<T*>(out), MM};
  return cols<Eng>(g, c, nslices, KKTDD_K_SWEEP_COLS, s);
}

template <typename Eng>
int dst_inverse_t(const Geom& g, const void* Sx, const void* Sy, const void* in, void* tmp,
                  double* out, int nslices, double norm, const double* c0, hipStream_t s) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  ColArgs<T> c{Sy, static_cast<const T*>(in), MM, nullptr, 0,
               static_cast<T*>(tmp), MM};
  if (int e = cols<Eng>(g, c, nslices, KKTDD_K_SWEEP_COLS, s)) return e;
  RowArgs<T> r = row_args<T>(Sx);
  r.g1_in = static_cast<const T*>(tmp);
  r.g1_stride = MM;
  r.g1_scale = norm;
  r.out_mode = OUT_PLAIN;
  r.out64 = out;
  r.c0 = c0;
  return rows<Eng>(g, r, nslices, KKTDD_K_SWEEP_ROWS, s);
}

// Measure every launch shape of the row and column kernels on one sweep step's worth of
// slices (both products of each kernel, on the handle's work buffers) and keep the fastest.
template <typename Eng>
int autotune_t(const Geom& g, const void* Sx, const void* Sy, const void* invlam, void* bufA,
               void* bufB, int nslices, hipStream_t s) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  RowArgs<T> r = row_args<T>(Sx);
  r.g1_in = static_cast<const T*>(bufA);
  r.g1_stride = MM;
  r.b_mode = B_H_Y;
  r.g2_out = static_cast<T*>(bufB);
  r.g2_stride = MM;
  ColArgs<T> c{Sy, static_cast<const T*>(bufA), MM, static_cast<const T*>(invlam), 1,
               static_cast<T*>(bufB), MM};
  hipEvent_t e0, e1;
  KKT_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(KKTDD_EHIP, "hipEventCreate failed");
  }
  int rc = 0;
  for (int kind = 0; kind < 2 && rc == 0; ++kind) {
    const int M = kind == 0 ? g.Mx : g.My;
    const TuneKey key{kind, engine_id<Eng>(), M, nslices};
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      tune_load_locked();
      if (g_tuned.count(key)) continue;
    }
    const int t = M / 16;
    // candidates: the default shape first, then every other valid shape
    Shape cand[32];
    int nc = 0;
    cand[nc++] = Shape{waves_for(M), 0};
    for (int nw : {2, 4, 8, t}) {
      if (nw < 1 || nw > 8 || t % nw != 0 || t / nw > 8) continue;
      for (int deep = 0; deep <= (t / nw <= 4 ? 1 : 0); ++deep) {
        bool seen = false;
        for (int i = 0; i < nc; ++i) seen = seen || (cand[i].nw == nw && cand[i].deep == deep);
        if (!seen && nc < 32) cand[nc++] = Shape{nw, deep};
      }
    }
    // rounds of 4 launches per candidate, candidates interleaved; a candidate's time is its
    // fastest round.  The default shape is kept unless another is at least 5% faster.
    float best_round[32];
    for (int i = 0; i < nc; ++i) best_round[i] = 1e30f;
    for (int round = 0; round < 3 && rc == 0; ++round) {
      for (int ci = 0; ci < nc && rc == 0; ++ci) {
        const Shape sh = cand[ci];
        auto launch = [&]() {
          return kind == 0 ? rows_shape<Eng>(g, r, nslices, sh, KKTDD_K_OTHER, s)
                           : cols_shape<Eng>(g, c, nslices, sh, KKTDD_K_OTHER, s);
        };
        if ((rc = launch())) break;
        if (hipEventRecord(e0, s) != hipSuccess) {
          rc = set_error(KKTDD_EHIP, "hipEventRecord failed");
          break;
        }
        for (int rep = 0; rep < 4 && rc == 0; ++rep) rc = launch();
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = set_error(KKTDD_EHIP, "autotune timing failed");
          break;
        }
        best_round[ci] = std::min(best_round[ci], 1e3f * ms / 4.f);
      }
    }
    Shape best = cand[0];
    float best_us = best_round[0];
    for (int ci = 1; ci < nc; ++ci)
      if (best_round[ci] < 0.95f * best_round[0] && best_round[ci] < best_us) {
        best_us = best_round[ci];
        best = cand[ci];
      }
    if (rc) break;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
    if (const char* path = tune_path()) {
      if (FILE* f = std::fopen(path, "a")) {
        std::fprintf(f, "{\"kind\": %d, \"engine\": %d, \"M\": %d, \"slices\": %d, \"waves\": %d, "
                        "\"deep\": %d, \"us\": %.2f}\n", kind, engine_id<Eng>(), M, nslices, best.nw,
                     best.deep, best_us);
        std::fclose(f);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

#define KKT_ENGINE_DISPATCH(PREC, FN, ...)                                    \
  switch (PREC) {                                                             \
    case KKTDD_FP64: return FN<EngPlain<double>>(__VA_ARGS__);                \
    case KKTDD_FP32: return FN<EngPlain<float>>(__VA_ARGS__);                 \
    case KKTDD_BF16: return FN<EngBF<1>>(__VA_ARGS__);                        \
    case KKTDD_BF16X3: return FN<EngBF<3>>(__VA_ARGS__);                      \
    case KKTDD_BF16X6: return FN<EngBF<6>>(__VA_ARGS__);                      \
    default: return set_error(KKTDD_EINVAL, "unknown precision");            \
  }

int launch_dst_forward(const Geom& g, int precision, const void* Sx, const void* Sy,
                       const double* in, const double* dscale, void* tmp, void* out, int nslices,
                       hipStream_t s) {
  KKT_ENGINE_DISPATCH(precision, dst_forward_t, g, Sx, Sy, in, dscale, tmp, out, nslices, s)
}

int launch_dst_inverse(const Geom& g, int precision, const void* Sx, const void* Sy,
                       const void* in, void* tmp, double* out, int nslices, double norm,
                       const double* c0, hipStream_t s) {
  KKT_ENGINE_DISPATCH(precision, dst_inverse_t, g, Sx, Sy, in, tmp, out, nslices, norm, c0, s)
}

int launch_spatial_solve(const Geom& g, int precision, const void* Sx, const void* Sy,
                         const void* invlam, const double* b, double* x, int nslices,
                         void* work1, void* work2, hipStream_t s) {
  if (nslices <= 0) return 0;
  KKT_ENGINE_DISPATCH(precision, spatial_solve_t, g, Sx, Sy, invlam, b, x, nslices, work1, work2, s)
}

int launch_sweeps(const Geom& g, int precision, const void* Sx, const void* Sy,
                  const void* invlam, const double* rprime, const double* c0, double* zw,
                  void* Tbuf, void* Ubuf, void* Ybuf, hipStream_t s) {
  KKT_ENGINE_DISPATCH(precision, sweeps_t, g, Sx, Sy, invlam, rprime, c0, zw, Tbuf, Ubuf, Ybuf, s)
}

int launch_coarse_dst(const Geom& g, const double* Sx, const double* Sy, const double* r0,
                      double* rhat, double* tmp, hipStream_t s) {
  const long long MM = g.padded();
  RowArgs<double> r = row_args<double>(Sx);
  r.b_mode = B_INPUT;
  r.rin = r0;
  r.g2_out = tmp;
  r.g2_stride = MM;
  if (int e = rows<EngPlain<double>>(g, r, g.nc, KKTDD_K_COARSE, s)) return e;
  ColArgs<double> c{Sy, tmp, MM, nullptr, 0, rhat, MM};
  return cols<EngPlain<double>>(g, c, g.nc, KKTDD_K_COARSE, s);
}

int launch_coarse_idst(const Geom& g, const double* Sx, const double* Sy, const double* chat,
                       double* c0, double* tmp, double norm, hipStream_t s) {
  const long long MM = g.padded();
  ColArgs<double> c{Sy, chat, MM, nullptr, 0, tmp, MM};
  if (int e = cols<EngPlain<double>>(g, c, g.nc, KKTDD_K_COARSE, s)) return e;
  RowArgs<double> r = row_args<double>(Sx);
  r.g1_in = tmp;
  r.g1_stride = MM;
  r.g1_scale = norm;
  r.out_mode = OUT_PLAIN;
  r.out64 = c0;
  return rows<EngPlain<double>>(g, r, g.nc, KKTDD_K_COARSE, s);
}

}  // namespace kktdd

namespace kktdd {

int tune_set(int kind, int precision, int extent, int nslices, int waves, int deep) {
  const int t = extent / 16;
  if (kind < 0 || kind > 1 || precision < KKTDD_FP64 || precision > KKTDD_BF16X6 || extent < 16 ||
      extent % 16 != 0 || nslices < 1 || waves < 1 || waves > 8 || t % waves != 0 ||
      t / waves > 8 || deep < 0 || deep > 1)
    return set_error(KKTDD_EINVAL, "invalid launch shape");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tuned[{kind, precision, extent, nslices}] = Shape{waves, deep};
  return 0;
}

int tune_get(int kind, int precision, int extent, int nslices, int* waves, int* deep) {
  if (!waves || !deep || extent < 16 || extent % 16 != 0)
    return set_error(KKTDD_EINVAL, "invalid launch-shape query");
  const Shape sh = tuned_shape(kind, precision, extent, nslices);
  *waves = sh.nw;
  *deep = sh.deep;
  return 0;
}

int launch_autotune(const Geom& g, int precision, const void* Sx, const void* Sy,
                    const void* invlam, void* bufA, void* bufB, int nslices, hipStream_t s) {
  if (nslices <= 0) return 0;
  KKT_ENGINE_DISPATCH(precision, autotune_t, g, Sx, Sy, invlam, bufA, bufB, nslices, s)
}

}  // namespace kktdd
