// Dirichlet spatial solves as sine-transform GEMMs on MFMA, and the RASQ time sweeps.
//
// Spatial solve (every step of a sweep, Sec. 3-4): D = shift*I + dt*nu*A_h is diagonalised by
// the 2-D discrete sine transform,
//     D^{-1} b = (4/(nx ny)) S_y [ (S_y b S_x) ./ (shift + dt*nu*(lam^y_q + lam^x_p)) ] S_x,
// with S_x[p][i] = sin(pi (p+1)(i+1)/nx) symmetric and S_x S_x = (nx/2) I.  The 4/(nx ny)
// factor is folded into the inverse eigenvalue table.  A solve is four sine-transform products.
//
// Work split.  A slice b is (my x mx), rows = y.  Right products (. S_x) only mix within a
// row, left products (S_y .) only within a column.  A solve is therefore arranged as
//     row kernel:    T  = b S_x                               (row blocks of 16)
//     column kernel: X  = (S_y T) ./ lambda ;  U = S_y X      (column blocks of 16)
//     row kernel:    y  = U S_x                               (row blocks of 16)
// and in a sweep the last row product of step j and the first of step j+1 run in the same
// row kernel (b_{j+1} = r'_{j+1} + y_j is formed row-locally), so one step costs one row and
// one column launch, each doing two chained products.
//
// Folding.  With n = m+1 intervals, S[p][n-i] = (-1)^(p+1) S[p][i] (1-based p, i).  A forward
// transform therefore takes the sums b_i + b_{n-i} (i <= n/2, the middle point once) to the
// odd frequencies and the differences b_i - b_{n-i} to the even ones, through two half-size
// blocks F_odd[k][j] = sin(pi (2j+1)(k+1)/n) and F_even[k][j] = sin(pi (2j+2)(k+1)/n); an
// inverse transform computes E = F_odd x_odd and O = F_even x_even and writes E + O at point i
// and E - O at point n-i.  Each 1-D transform costs half the multiply-adds of the dense one.
// Mode space keeps the odd frequencies in the first half of the padded extent and the even
// ones in the second (mode_pos).
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
// All layouts were checked on gfx950.  The half-size blocks (pre-split into bf16 parts for the
// bf16 engines) are read straight from L2, stored in whichever orientation makes every
// operand load a run of contiguous row segments; the other operand sits in LDS.  Work buffers are float64
// for the f64 engine and float32 otherwise.
#include <algorithm>
#include <array>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <type_traits>

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
// to nw waves (nw even), TPW tiles each, with nw * TPW == M/16 exactly (the padded extents
// are chosen so that this holds).  Even waves take tiles of the odd-frequency half, odd waves
// tiles of the even-frequency half, so every wave's tiles share one half of the operand.
// The table operand comes from L2 through a register ring that runs ahead of the MFMAs,
// hiding the L2 latency; the LDS operand is read in place.  The ring is PD k-steps deep: 4 by
// default; deeper rings (16 for one tile per wave, 8 for two to four) can be selected with
// kkt_tune_set.
constexpr int kPDDefault = 4;
template <int TPW>
constexpr int deep_prefetch() { return TPW == 1 ? 16 : (TPW <= 4 ? 8 : kPDDefault); }

// Workgroup size bound of a kernel: those with at most two tiles per wave and at most
// Eng::kMaxW16 blocks per workgroup (the kernels that stay within 128 VGPRs) also run as
// 16-wave workgroups, which fill a CU alone; the others take at most 8 waves.
template <typename Eng, int TPW, int PD, int W>
constexpr int max_threads() { return (TPW <= 2 && W <= Eng::kMaxW16 && PD == kPDDefault) ? 1024 : 512; }

// A launch shape for t tiles per transformed extent: nw waves (even, dividing t, at most 8
// tiles each; 16 only with at most two tiles each and at most max_w16 blocks), the default or
// the deep ring, 1, 2 or 4 blocks per workgroup (several blocks: at most 4 tiles per wave,
// default ring).
inline bool shape_valid(int t, int nw, int deep, int width, int max_w16) {
  if (nw < 2 || (nw & 1) || t % nw != 0 || t / nw > 8) return false;
  if (deep < 0 || deep > 1 || (width != 1 && width != 2 && width != 4)) return false;
  if (width > 1 && (deep || t / nw > 4)) return false;
  if (nw > 8 && (nw != 16 || t / nw > 2 || width > max_w16 || deep)) return false;
  return true;
}

// ---- plain engines (f64, f32) ----------------------------------------------------------
// A half-transform table Q holds two H x H blocks (H = M/2), block b at Q + b*H*H, its rows
// stored in k-step groups (see the table loads below).
// gemm_right: acc[w][t] += A_w(:, half blk) * Q[blk](:, tile), A_w = row block w (16 rows) of
//             the 16W x M operand in LDS.
// gemm_left:  acc[w][t] += Q[blk](:, tile)^T * B_w(half blk, :), B_w = column block w (16
//             columns) of the M x 16W operand in LDS.
// Output tile t of a wave is local tile lt0 + t*lts of half blk.  A wave loads each table
// fragment once and uses it for all W blocks of the workgroup, so a workgroup of W blocks reads
// the table W times less per row (or column) than W workgroups of one block; every output
// element still sums over k in the same order, so W never changes a result.
template <typename T>
struct EngPlain {
  using data_t = T;
  using acc_t = typename AccT<T>::type;
  using s_t = T;
  static constexpr int kTableParts = 1;
  static constexpr int kMaxW16 = sizeof(T) == 8 ? 2 : 4;   // blocks of a 16-wave workgroup
  template <int W> static __host__ __device__ size_t rows_lds(int M) { return (size_t)16 * W * (M + 1) * sizeof(T); }
  template <int W> static __host__ __device__ size_t cols_lds(int M) { return (size_t)M * (16 * W + 1) * sizeof(T); }
  // The combine buffer of the inverse products is the operand buffer itself, in the same
  // layout, so a thread may overwrite the combine values it has just read.
  static constexpr bool kCombInPlace = true;
  template <int W> static __host__ __device__ size_t rows_lds_total(int M) { return rows_lds<W>(M); }
  template <int W> static __host__ __device__ size_t cols_lds_total(int M) { return cols_lds<W>(M); }
  // Three or four tiles per wave with the default ring, one block (or two in float32): two
  // 8-wave workgroups share a CU, their registers capped.
  template <int TPW, int PD, int W>
  static constexpr bool two_per_cu() {
    return (TPW == 3 || TPW == 4) && PD == kPDDefault && (W == 1 || (W == 2 && sizeof(T) == 4));
  }
  static __device__ int acc_row(int lk, int r) {
    if constexpr (sizeof(T) == 8) return lk + 4 * r; else return 4 * lk + r;
  }
  // rows operand A[16W][M+1]
  template <int W>
  static __device__ void put_a(unsigned char* lds, int M, int r, int c, T v) {
    reinterpret_cast<T*>(lds)[r * (M + 1) + c] = v;
  }
  // cols operand B[M][16W+1]
  template <int W>
  static __device__ void put_b(unsigned char* lds, int M, int k, int c, T v) {
    (void)M;
    reinterpret_cast<T*>(lds)[k * (16 * W + 1) + c] = v;
  }
  // Table loads: a wave-uniform base (block, k-step pair) plus a 32-bit per-lane offset per
  // tile.  The float64 tables store each block with k-steps interleaved in pairs: the element
  // of row 4ks + lk, column c sits at ((ks/2 * 4 + lk) H + c) * 2 + ks % 2, so one 16-byte
  // load brings a lane its operands of k-steps 2P and 2P + 1 (half the load instructions).
  // The float32 tables group four k-steps the same way (a quarter of the loads).
  using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
  template <int TPW, int kPD, int W>
  static __device__ void gemm_right2(const unsigned char* lds, const T* __restrict__ Q, int M,
                                     int blk, int lt0, int lts, int li, int lk, acc_t (&acc)[W][TPW]) {
    const int H = M >> 1, ldr = 16 * (M + 1);
    const T* Ab = reinterpret_cast<const T*>(lds) + li * (M + 1) + blk * H + lk;
    const T2* Qb = reinterpret_cast<const T2*>(Q + (long long)blk * H * H);
    int voff[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) voff[t] = lk * H + (lt0 + t * lts) * 16 + li;
    const int npr = H >> 3;           // k-step pairs
    constexpr int RP = kPD / 2;       // ring depth in pairs
    T2 bq[RP][TPW];
    // every ring slot is filled (a short extent repeats its last pair), so all loads are counted
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const T2* Qk = Qb + (long long)(4 * (p < npr ? p : npr - 1)) * H;
#pragma unroll
      for (int t = 0; t < TPW; ++t) bq[p][t] = Qk[voff[t]];
    }
    // one ring step: slot p holds the table operands of k-step pair pr
    auto step = [&](const int p, const int pr) __attribute__((always_inline)) {
      T a0[W], a1[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        a0[w] = Ab[w * ldr + 8 * pr];
        a1[w] = Ab[w * ldr + 8 * pr + 4];
      }
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(a0[w], bq[p][t].x, acc[w][t]);
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(a1[w], bq[p][t].y, acc[w][t]);
      // refilled on every step (past the end with the last pair again: in bounds, never used)
      const int kn = pr + RP < npr ? pr + RP : npr - 1;
      {
        const T2* Qk = Qb + (long long)(4 * kn) * H;
#pragma unroll
        for (int t = 0; t < TPW; ++t) bq[p][t] = Qk[voff[t]];
      }
    };
    // whole ring rounds, then the pairs left over: with no exit inside a round the compiler
    // counts the refills in flight instead of draining the ring on every round
    int pr0 = 0;
    for (; pr0 + RP <= npr; pr0 += RP) {
#pragma unroll
      for (int p = 0; p < RP; ++p) step(p, pr0 + p);
    }
#pragma unroll
    for (int p = 0; p < RP; ++p)
      if (pr0 + p < npr) step(p, pr0 + p);
  }
  template <int TPW, int kPD, int W>
  static __device__ void gemm_left2(const T* __restrict__ Q, const unsigned char* lds, int M,
                                    int blk, int lt0, int lts, int li, int lk, acc_t (&acc)[W][TPW]) {
    const int H = M >> 1, ldb = 16 * W + 1;
    const T* Bb = reinterpret_cast<const T*>(lds) + (blk * H + lk) * ldb + li;
    const T2* Qb = reinterpret_cast<const T2*>(Q + (long long)blk * H * H);
    int voff[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) voff[t] = lk * H + (lt0 + t * lts) * 16 + li;
    const int npr = H >> 3;
    constexpr int RP = kPD / 2;
    T2 aq[RP][TPW];
    // every ring slot is filled (a short extent repeats its last pair), so all loads are counted
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const T2* Qk = Qb + (long long)(4 * (p < npr ? p : npr - 1)) * H;
#pragma unroll
      for (int t = 0; t < TPW; ++t) aq[p][t] = Qk[voff[t]];
    }
    // one ring step: slot p holds the table operands of k-step pair pr
    auto step = [&](const int p, const int pr) __attribute__((always_inline)) {
      T b0[W], b1[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        b0[w] = Bb[8 * pr * ldb + 16 * w];
        b1[w] = Bb[(8 * pr + 4) * ldb + 16 * w];
      }
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(aq[p][t].x, b0[w], acc[w][t]);
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(aq[p][t].y, b1[w], acc[w][t]);
      // refilled on every step (past the end with the last pair again: in bounds, never used)
      const int kn = pr + RP < npr ? pr + RP : npr - 1;
      {
        const T2* Qk = Qb + (long long)(4 * kn) * H;
#pragma unroll
        for (int t = 0; t < TPW; ++t) aq[p][t] = Qk[voff[t]];
      }
    };
    // whole ring rounds, then the pairs left over: with no exit inside a round the compiler
    // counts the refills in flight instead of draining the ring on every round
    int pr0 = 0;
    for (; pr0 + RP <= npr; pr0 += RP) {
#pragma unroll
      for (int p = 0; p < RP; ++p) step(p, pr0 + p);
    }
#pragma unroll
    for (int p = 0; p < RP; ++p)
      if (pr0 + p < npr) step(p, pr0 + p);
  }
  // float32: k-steps in groups of four, one 16-byte load per lane brings four of them.
  template <int TPW, int kPD, int W>
  static __device__ void gemm_right4(const unsigned char* lds, const T* __restrict__ Q, int M,
                                     int blk, int lt0, int lts, int li, int lk, acc_t (&acc)[W][TPW]) {
    const int H = M >> 1, ldr = 16 * (M + 1);
    const T* Ab = reinterpret_cast<const T*>(lds) + li * (M + 1) + blk * H + lk;
    const float4* Qb = reinterpret_cast<const float4*>(Q + (long long)blk * H * H);
    int voff[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) voff[t] = lk * H + (lt0 + t * lts) * 16 + li;
    const int ngr = H >> 4;                          // groups of four k-steps
    constexpr int RP = kPD / 4 > 0 ? kPD / 4 : 1;    // ring depth in groups
    float4 bq[RP][TPW];
#pragma unroll
    for (int p = 0; p < RP; ++p)
      if (p < ngr) {
        const float4* Qk = Qb + (long long)(4 * p) * H;
#pragma unroll
        for (int t = 0; t < TPW; ++t) bq[p][t] = Qk[voff[t]];
      }
    for (int gr0 = 0; gr0 < ngr; gr0 += RP) {
#pragma unroll
      for (int p = 0; p < RP; ++p) {
        const int gr = gr0 + p;
        if (gr >= ngr) break;
        T a0[W], a1[W], a2[W], a3[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          a0[w] = Ab[w * ldr + 16 * gr];
          a1[w] = Ab[w * ldr + 16 * gr + 4];
          a2[w] = Ab[w * ldr + 16 * gr + 8];
          a3[w] = Ab[w * ldr + 16 * gr + 12];
        }
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(a0[w], bq[p][t].x, acc[w][t]);
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(a1[w], bq[p][t].y, acc[w][t]);
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(a2[w], bq[p][t].z, acc[w][t]);
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(a3[w], bq[p][t].w, acc[w][t]);
        const int kn = gr + RP;
        if (kn < ngr) {
          const float4* Qk = Qb + (long long)(4 * kn) * H;
#pragma unroll
          for (int t = 0; t < TPW; ++t) bq[p][t] = Qk[voff[t]];
        }
      }
    }
  }
  template <int TPW, int kPD, int W>
  static __device__ void gemm_left4(const T* __restrict__ Q, const unsigned char* lds, int M,
                                    int blk, int lt0, int lts, int li, int lk, acc_t (&acc)[W][TPW]) {
    const int H = M >> 1, ldb = 16 * W + 1;
    const T* Bb = reinterpret_cast<const T*>(lds) + (blk * H + lk) * ldb + li;
    const float4* Qb = reinterpret_cast<const float4*>(Q + (long long)blk * H * H);
    int voff[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) voff[t] = lk * H + (lt0 + t * lts) * 16 + li;
    const int ngr = H >> 4;
    constexpr int RP = kPD / 4 > 0 ? kPD / 4 : 1;
    float4 aq[RP][TPW];
#pragma unroll
    for (int p = 0; p < RP; ++p)
      if (p < ngr) {
        const float4* Qk = Qb + (long long)(4 * p) * H;
#pragma unroll
        for (int t = 0; t < TPW; ++t) aq[p][t] = Qk[voff[t]];
      }
    for (int gr0 = 0; gr0 < ngr; gr0 += RP) {
#pragma unroll
      for (int p = 0; p < RP; ++p) {
        const int gr = gr0 + p;
        if (gr >= ngr) break;
        T b0[W], b1[W], b2[W], b3[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          b0[w] = Bb[16 * gr * ldb + 16 * w];
          b1[w] = Bb[(16 * gr + 4) * ldb + 16 * w];
          b2[w] = Bb[(16 * gr + 8) * ldb + 16 * w];
          b3[w] = Bb[(16 * gr + 12) * ldb + 16 * w];
        }
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(aq[p][t].x, b0[w], acc[w][t]);
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(aq[p][t].y, b1[w], acc[w][t]);
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(aq[p][t].z, b2[w], acc[w][t]);
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[w][t] = mfma16(aq[p][t].w, b3[w], acc[w][t]);
        const int kn = gr + RP;
        if (kn < ngr) {
          const float4* Qk = Qb + (long long)(4 * kn) * H;
#pragma unroll
          for (int t = 0; t < TPW; ++t) aq[p][t] = Qk[voff[t]];
        }
      }
    }
  }
  // Table operand groups: kGroup k-steps per load (two in float64, four in float32).
  static constexpr int kGroup = sizeof(T) == 8 ? 2 : 4;
  template <int TPW, int kPD, int W>
  static __device__ void gemm_right(const unsigned char* lds, const T* __restrict__ Q, int M,
                                    int blk, int lt0, int lts, int li, int lk, acc_t (&acc)[W][TPW]) {
    if constexpr (sizeof(T) == 8) gemm_right2<TPW, kPD, W>(lds, Q, M, blk, lt0, lts, li, lk, acc);
    else gemm_right4<TPW, kPD, W>(lds, Q, M, blk, lt0, lts, li, lk, acc);
  }
  template <int TPW, int kPD, int W>
  static __device__ void gemm_left(const T* __restrict__ Q, const unsigned char* lds, int M,
                                   int blk, int lt0, int lts, int li, int lk, acc_t (&acc)[W][TPW]) {
    if constexpr (sizeof(T) == 8) gemm_left2<TPW, kPD, W>(Q, lds, M, blk, lt0, lts, li, lk, acc);
    else gemm_left4<TPW, kPD, W>(Q, lds, M, blk, lt0, lts, li, lk, acc);
  }
};

// ---- split-bfloat16 engines -------------------------------------------------------------
// Tables hold three bfloat16 parts, part p at offset p*M*M/2 (two H x H blocks each).  Here
// gemm_right reads Q[blk](tile, :) and gemm_left Q[blk](tile, :) as well (k contiguous, 16
// bytes per lane), so these engines take the transposes of the plain engines' tables.  The
// W row (or column) blocks of a workgroup share each table fragment as in the plain engines.
template <int SPLIT>
struct EngBF {
  static constexpr int NP = SPLIT == 1 ? 1 : (SPLIT == 3 ? 2 : 3);   // parts per operand
  using data_t = float;
  using acc_t = v4f;
  using s_t = __bf16;
  static constexpr int kTableParts = 3;
  static constexpr int kMaxW16 = NP <= 2 ? 4 : 2;          // blocks of a 16-wave workgroup
  template <int W> static __host__ __device__ size_t rows_lds(int M) { return (size_t)NP * 16 * W * (M + 8) * 2; }
  template <int W> static __host__ __device__ size_t cols_lds(int M) { return (size_t)NP * 16 * W * (M + 8) * 2; }
  // The float combine buffers ([16W][M+1] rows, [M][16W+1] cols) overlap the operand parts, so
  // every combine value is read before the operand is written again.
  static constexpr bool kCombInPlace = false;
  template <int W> static __host__ __device__ size_t rows_lds_total(int M) {
    const size_t c = (size_t)16 * W * (M + 1) * 4;
    return rows_lds<W>(M) > c ? rows_lds<W>(M) : c;
  }
  template <int W> static __host__ __device__ size_t cols_lds_total(int M) {
    const size_t c = (size_t)M * (16 * W + 1) * 4;
    return cols_lds<W>(M) > c ? cols_lds<W>(M) : c;
  }
  template <int TPW, int PD, int W>
  static constexpr bool two_per_cu() {
    return (TPW == 3 || TPW == 4) && PD == kPDDefault && (W == 1 || (W == 2 && NP <= 2));
  }
  static __device__ int acc_row(int lk, int r) { return 4 * lk + r; }
  static __device__ void split(float v, __bf16 (&part)[NP]) {
    part[0] = (__bf16)v;
    if constexpr (NP > 1) {
      const float r1 = v - (float)part[0];
      part[1] = (__bf16)r1;
      if constexpr (NP > 2) part[2] = (__bf16)(r1 - (float)part[1]);
    }
  }
  // rows operand: NP arrays A_p[16W][M+8] (k contiguous)
  template <int W>
  static __device__ void put_a(unsigned char* lds, int M, int r, int c, float v) {
    __bf16 part[NP];
    split(v, part);
    __bf16* A = reinterpret_cast<__bf16*>(lds);
#pragma unroll
    for (int p = 0; p < NP; ++p) A[(p * 16 * W + r) * (M + 8) + c] = part[p];
  }
  // cols operand stored transposed: NP arrays Bt_p[16W][M+8], Bt_p[c][k] = part_p(B[k][c])
  template <int W>
  static __device__ void put_b(unsigned char* lds, int M, int k, int c, float v) {
    __bf16 part[NP];
    split(v, part);
    __bf16* B = reinterpret_cast<__bf16*>(lds);
#pragma unroll
    for (int p = 0; p < NP; ++p) B[(p * 16 * W + c) * (M + 8) + k] = part[p];
  }
  // Part products of one product, in the order every accumulator receives them (smallest
  // first): a2b0, a1b1, a0b2 (x6), a1b0, a0b1 (x3, x6), a0b0.  The GEMM loops issue part
  // product q for all of a wave's accumulators before part product q+1, so consecutive MFMAs
  // never depend on each other; each accumulator still sums its part products in this order.
  static constexpr int kProducts = SPLIT;
  static __host__ __device__ constexpr int part_a(int q) {
    return SPLIT == 6 ? (q == 0 ? 2 : q == 1 ? 1 : q == 2 ? 0 : q == 3 ? 1 : 0)
                      : SPLIT == 3 ? (q == 0 ? 1 : 0) : 0;
  }
  static __host__ __device__ constexpr int part_b(int q) {
    return SPLIT == 6 ? (q == 0 ? 0 : q == 1 ? 1 : q == 2 ? 2 : q == 3 ? 0 : q == 4 ? 1 : 0)
                      : SPLIT == 3 ? (q == 1 ? 1 : 0) : 0;
  }
  // table fragments kept in flight per tile and part: two k-steps while the ring fits the
  // register budget of the launch shape, else one
  template <int TPW, int W>
  static constexpr int ring() { return TPW * NP <= (W == 1 ? 8 : 12) ? 2 : 1; }
  // fragment of local tile lt at k-step ks: Q_p[blk][lt*16 + li][32ks + 8lk .. +8], as a
  // wave-uniform base (part, block, k-step) plus a 32-bit per-lane offset
  static __device__ bf16x8 qload(const __bf16* __restrict__ Q, int M, int blk, int lt, int ks,
                                 int p, int li, int lk) {
    const int H = M >> 1;
    const __bf16* base = Q + (long long)p * M * H + (long long)blk * H * H + 32 * ks;
    return *reinterpret_cast<const bf16x8*>(base + ((lt * 16 + li) * H + 8 * lk));
  }
  template <int TPW, int PD_unused, int W>
  static __device__ void gemm_right(const unsigned char* lds, const __bf16* __restrict__ Q, int M,
                                    int blk, int lt0, int lts, int li, int lk, acc_t (&acc)[W][TPW]) {
    constexpr int RD = ring<TPW, W>();
    const int H = M >> 1, lda = M + 8;
    const __bf16* A = reinterpret_cast<const __bf16*>(lds) + blk * H + 8 * lk;
    bf16x8 bq[RD][TPW][NP];
    const int nks = H >> 5;
#pragma unroll
    for (int d = 0; d < RD; ++d)
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int p = 0; p < NP; ++p) bq[d][t][p] = d < nks ? qload(Q, M, blk, lt0 + t * lts, d, p, li, lk) : bf16x8{};
    for (int ks0 = 0; ks0 < nks; ks0 += RD) {
#pragma unroll
      for (int d = 0; d < RD; ++d) {
        const int ks = ks0 + d;
        if (ks >= nks) break;
        bf16x8 af[W][NP];
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int p = 0; p < NP; ++p)
            af[w][p] = *reinterpret_cast<const bf16x8*>(A + (p * 16 * W + w * 16 + li) * lda + 32 * ks);
#pragma unroll
        for (int q = 0; q < kProducts; ++q)
#pragma unroll
          for (int w = 0; w < W; ++w)
#pragma unroll
            for (int t = 0; t < TPW; ++t)
              acc[w][t] = mfma_bf(af[w][part_a(q)], bq[d][t][part_b(q)], acc[w][t]);
        const int kn = ks + RD;
        if (kn < nks) {
#pragma unroll
          for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int p = 0; p < NP; ++p) bq[d][t][p] = qload(Q, M, blk, lt0 + t * lts, kn, p, li, lk);
        }
      }
    }
  }
  template <int TPW, int PD_unused, int W>
  static __device__ void gemm_left(const __bf16* __restrict__ Q, const unsigned char* lds, int M,
                                   int blk, int lt0, int lts, int li, int lk, acc_t (&acc)[W][TPW]) {
    constexpr int RD = ring<TPW, W>();
    const int H = M >> 1, ldb = M + 8;
    const __bf16* Bt = reinterpret_cast<const __bf16*>(lds) + blk * H + 8 * lk;
    bf16x8 aq[RD][TPW][NP];
    const int nks = H >> 5;
#pragma unroll
    for (int d = 0; d < RD; ++d)
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int p = 0; p < NP; ++p) aq[d][t][p] = d < nks ? qload(Q, M, blk, lt0 + t * lts, d, p, li, lk) : bf16x8{};
    for (int ks0 = 0; ks0 < nks; ks0 += RD) {
#pragma unroll
      for (int d = 0; d < RD; ++d) {
        const int ks = ks0 + d;
        if (ks >= nks) break;
        bf16x8 bf[W][NP];
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int p = 0; p < NP; ++p)
            bf[w][p] = *reinterpret_cast<const bf16x8*>(Bt + (p * 16 * W + w * 16 + li) * ldb + 32 * ks);
#pragma unroll
        for (int q = 0; q < kProducts; ++q)
#pragma unroll
          for (int w = 0; w < W; ++w)
#pragma unroll
            for (int t = 0; t < TPW; ++t)
              acc[w][t] = mfma_bf(aq[d][t][part_a(q)], bf[w][part_b(q)], acc[w][t]);
        const int kn = ks + RD;
        if (kn < nks) {
#pragma unroll
          for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int p = 0; p < NP; ++p) aq[d][t][p] = qload(Q, M, blk, lt0 + t * lts, kn, p, li, lk);
        }
      }
    }
  }
};

// ---- row kernel ------------------------------------------------------------------------
// One workgroup = RB blocks of 16 rows of one slice.  Optional GEMM1 (inverse product
// y = g1_scale * U S_x, U in x-mode space) with its epilogue stores, then optional formation of
// b and GEMM2 (forward product T = b S_x, T in x-mode space).  Both products are folded: the
// workgroup works on mirrored column pairs (c, mx-1-c), 2*TPW pairs per thread and row block.
enum BMode { B_NONE = 0, B_RPRIME_PLUS_Y = 1, B_H_YBUF_PLUS_Y = 2, B_H_Y = 3, B_INPUT = 4 };
enum OutMode { OUT_NONE = 0, OUT_OWNED = 1, OUT_PLAIN = 2 };

template <typename T>
struct RowArgs {
  const void* Sx;            // engine's half-transform tables of x: forward, then inverse
  const T* g1_in;            // padded slices (nullptr: y = 0)
  long long g1_stride;
  double g1_scale;
  T* ystore;                 // padded layout, interior points written; nullptr: no store
  long long ystore_stride;
  int out_mode;
  double* out64;             // OUT_OWNED: z_w field (nt slices); OUT_PLAIN: nslices slices
  const double* c0;          // coarse slots added to OUT_OWNED / OUT_PLAIN field output (nullptr: none)
  int g1_step;               // sweep step of the GEMM1 result (OUT_OWNED)
  int b_mode;
  int b_step;                // sweep step whose right-hand side is formed (B_RPRIME_PLUS_Y)
  const double* rin;         // r' field (nt slices) or plain input slices (B_INPUT), float64
  const float* rin32;        // the same in float32 (read instead of rin when set)
  const double* in_scale;    // device factor of the B_INPUT slices (nullptr: 1)
  const T* ybuf_in;          // padded (B_H_YBUF_PLUS_Y)
  long long ybuf_stride;
  T* g2_out;                 // padded
  long long g2_stride;
  int nsl;                   // set by the launcher: slice count of the slice-per-XCD grid, or 0
};

// Workgroup placement of the row and column kernels.  Workgroups are dealt to the XCDs
// round-robin by linear id.  The two-dimensional grid (tile, slice) spreads every slice over
// all XCDs.  The slice-per-XCD grid is one-dimensional, kXcds * ceil(nslices / kXcds) * ntile
// workgroups: id = x + kXcds * q runs tile q % ntile of slice x + kXcds * (q / ntile) on XCD
// x, so the slice one launch writes is read by the next launch on the same XCD (from its L2
// while the slices fit there).  Ids past the last slice exit at once.
constexpr int kXcds = 8;
__device__ inline bool tile_and_slice(int ntile, int nsl, int& tile, int& slice) {
  if (nsl == 0) {
    tile = blockIdx.x;
    slice = blockIdx.y;
    return true;
  }
  const int q = blockIdx.x / kXcds, c = q / ntile;
  slice = blockIdx.x % kXcds + kXcds * c;
  tile = q - c * ntile;
  return slice < nsl;
}

template <typename Eng>
__device__ inline const typename Eng::s_t* table(const void* S, int M, int inverse) {
  return static_cast<const typename Eng::s_t*>(S) +
         (inverse ? (long long)Eng::kTableParts * M * (M >> 1) : 0);
}

// Three or four tiles per wave with the default ring (and the block counts listed in each
// engine's two_per_cu): registers are capped so that two 8-wave workgroups share a CU (one's
// loads and stores overlap the other's MFMAs), and the right-hand-side operands are fetched
// after the first product instead of before it.
template <typename Eng, int TPW, int PD, int RB>
__global__ void __launch_bounds__((max_threads<Eng, TPW, PD, RB>()), (Eng::template two_per_cu<TPW, PD, RB>() ? 4 : 1))
k_rows(Geom g, RowArgs<typename Eng::data_t> a) {
  using T = typename Eng::data_t;
  using acc_t = typename Eng::acc_t;
  constexpr bool kTwo = Eng::template two_per_cu<TPW, PD, RB>();
  extern __shared__ unsigned char smem_raw[];
  const int Mx = g.Mx, Hx = Mx >> 1, mx = g.mx, Ax = (mx + 1) / 2, ldc = Mx + 1;
  int rg, s;
  if (!tile_and_slice((g.my + 16 * RB - 1) / (16 * RB), a.nsl, rg, s)) return;
  const int row0 = rg * 16 * RB;       // first row of the workgroup's RB row blocks
  const int nthr = blockDim.x, nw = nthr >> 6;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int blk = wave & 1, lt0 = wave >> 1, lts = nw >> 1;
  T* comb = reinterpret_cast<T*>(smem_raw);
  constexpr int NPR = 2 * TPW;   // per row block: 16 rows x Hx pairs = NPR * blockDim.x
  acc_t acc[RB][TPW];

  // node of a sweep step in this subdomain (0-based subdomain s): first = s*k + 1 - delta
  const int first = s * g.k + 1 - g.delta;

  // Right-hand-side operands of b at both points of every pair, fetched before GEMM1 so their
  // latency hides behind it (after it where registers are capped).  With at most 8 pairs per
  // thread the source is chosen once per launch and every lane loads all of its pairs
  // unconditionally (rows and columns past the interior clamped to the last interior point,
  // their values replaced by zero), so the loads are in flight together; with more pairs that
  // form would keep every address live and spill, so the loads stay per pair.
  constexpr bool kBatchPre = RB * NPR <= 8;
  T pre[RB][NPR][2];
  auto fill_pre = [&](auto base, long long rstride, double isc) {
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
#pragma unroll
      for (int i = 0; i < NPR; ++i) {
        const int e = threadIdx.x + i * nthr;
        const int r = e / Hx, k = e - r * Hx;
        const int row = row0 + rr * 16 + r;
        const bool live = row < g.my && k < Ax;
        const int kc = k < Ax ? k : Ax - 1;
        const auto* src = base + (long long)(row < g.my ? row : g.my - 1) * rstride;
        const auto x1 = src[kc], x2 = src[mx - 1 - kc];
        pre[rr][i][0] = live ? (T)(isc * x1) : (T)0;
        pre[rr][i][1] = live ? (T)(isc * x2) : (T)0;
      }
  };
  auto load_pre_each = [&]() {
    if (a.b_mode == B_RPRIME_PLUS_Y || a.b_mode == B_H_YBUF_PLUS_Y || a.b_mode == B_INPUT) {
      const int bnode = first + a.b_step;
      const double isc = (a.b_mode == B_INPUT && a.in_scale) ? *a.in_scale : 1.0;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
#pragma unroll
        for (int i = 0; i < NPR; ++i) {
          const int e = threadIdx.x + i * nthr;
          const int r = e / Hx, k = e - r * Hx;
          const int row = row0 + rr * 16 + r;
          T v1 = 0, v2 = 0;
          if (row < g.my && k < Ax) {
            const int c2 = mx - 1 - k;
            if (a.b_mode == B_RPRIME_PLUS_Y) {
              if (bnode >= 1) {
                const long long o = (long long)(bnode - 1) * g.nxy + (long long)row * mx;
                if (a.rin32) {
                  v1 = (T)a.rin32[o + k];
                  v2 = (T)a.rin32[o + c2];
                } else {
                  v1 = (T)a.rin[o + k];
                  v2 = (T)a.rin[o + c2];
                }
              }
            } else if (a.b_mode == B_H_YBUF_PLUS_Y) {
              const T* src = a.ybuf_in + s * a.ybuf_stride + (long long)row * Mx;
              v1 = src[k];
              v2 = src[c2];
            } else if (a.rin32) {   // float32 input, never scaled
              const float* src = a.rin32 + (long long)s * g.nxy + (long long)row * mx;
              v1 = (T)src[k];
              v2 = (T)src[c2];
            } else {
              const double* src = a.rin + (long long)s * g.nxy + (long long)row * mx;
              v1 = (T)(isc * src[k]);
              v2 = (T)(isc * src[c2]);
            }
          }
          pre[rr][i][0] = v1;
          pre[rr][i][1] = v2;
        }
    }
  };
  auto load_pre = [&]() {
    if constexpr (!kBatchPre) {
      load_pre_each();
      return;
    }
    const bool from_r = a.b_mode == B_RPRIME_PLUS_Y, from_y = a.b_mode == B_H_YBUF_PLUS_Y;
    if (!from_r && !from_y && a.b_mode != B_INPUT) return;
    const int bnode = first + a.b_step;
    if (from_r && bnode < 1) {
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
#pragma unroll
        for (int i = 0; i < NPR; ++i) pre[rr][i][0] = pre[rr][i][1] = (T)0;
      return;
    }
    if (from_y) {
      fill_pre(a.ybuf_in + s * a.ybuf_stride, Mx, 1.0);
      return;
    }
    // r' of the node (B_RPRIME_PLUS_Y) or input slice s (B_INPUT); float32 input is never scaled
    const long long o = from_r ? (long long)(bnode - 1) * g.nxy : (long long)s * g.nxy;
    if (a.rin32)
      fill_pre(a.rin32 + o, mx, 1.0);
    else
      fill_pre(a.rin + o, mx, (!from_r && a.in_scale) ? *a.in_scale : 1.0);
  };
  if constexpr (!kTwo) load_pre();

  // ---- GEMM1: E | O = U(odd modes) F_odd^T | U(even modes) F_even^T, into the combine buffer
  if (a.g1_in) {
    // the workgroup's rows are one contiguous run of 16*RB*Mx elements; every thread issues
    // all of its loads before the first LDS write, so they are in flight together
    constexpr int NE = 4 * RB * TPW;   // elements per thread: 16*RB*Mx / blockDim.x
    const T* src = a.g1_in + s * a.g1_stride + (long long)row0 * Mx;
    const int live = (g.my - row0) * Mx;   // elements of live rows; rows past them read as zero
    T buf[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = threadIdx.x + j * nthr;
      buf[j] = e < live ? src[e] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int r = e / Mx;
      Eng::template put_a<RB>(smem_raw, Mx, r, e - r * Mx, buf[j]);
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
#pragma unroll
      for (int t = 0; t < TPW; ++t) acc[rr][t] = acc_t{0, 0, 0, 0};
    Eng::template gemm_right<TPW, PD, RB>(smem_raw, table<Eng>(a.Sx, Mx, 1), Mx, blk, lt0, lts, li, lk, acc);
    __syncthreads();  // every wave has read the operand, which the combine buffer overlays
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          comb[(rr * 16 + Eng::acc_row(lk, r)) * ldc + blk * Hx + (lt0 + t * lts) * 16 + li] =
              (T)(acc[rr][t][r] * a.g1_scale);
    __syncthreads();
  }

  // ---- per pair: y at both points (E +- O), its stores, and the folded b (sum | difference)
  const bool form_b = a.b_mode != B_NONE;
  const bool owned = a.g1_step >= g.delta;
  const int node = first + a.g1_step;
  const T hT = (T)g.h;
  // Field output with the prolonged coarse part: OUT_PLAIN slice s is time node s+1, OUT_OWNED
  // writes node `node`; both add c0 of the owning subdomain cs times (1, phi).  With at most 8
  // pairs per thread the coarse values of a group of GP pairs are loaded before the group's
  // stores, unconditionally (clamped like the right-hand side), so they are in flight
  // together; wider shapes read them per point (the grouped form spills there).
  const bool out_plain = a.out_mode == OUT_PLAIN, out_owned = a.out_mode == OUT_OWNED && owned;
  const bool add_c = a.g1_in && a.c0 && (out_plain || out_owned);
  const int cs = out_plain ? s / g.k : s;
  const double cphi = -1.0 + 2.0 * (double)((out_plain ? s + 1 : node) - cs * g.k) / g.k;
  const double* cb = a.c0 ? a.c0 + (long long)(g.nb * cs) * g.nxy : nullptr;
  const long long o1 = g.nb == 2 ? g.nxy : 0;   // second slot (the first again with nb = 1)
  auto store_y = [&](int row, int col, T v, double c_0, double c_1) {
    if (a.ystore) a.ystore[s * a.ystore_stride + (long long)row * Mx + col] = v;
    const long long pt = (long long)row * mx + col;
    if (out_plain || out_owned) {
      double val = (double)v;
      if (add_c) {
        val += c_0;
        if (g.nb == 2) val += cphi * c_1;
      }
      a.out64[(out_plain ? (long long)s : (long long)(node - 1)) * g.nxy + pt] = val;
    }
  };
  T yv[RB][NPR][2];
  if constexpr (kBatchPre) {
    constexpr int GP = NPR % 4 == 0 ? 4 : 2;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
#pragma unroll
      for (int i0 = 0; i0 < NPR; i0 += GP) {
        double cv[GP][4];
        if (add_c) {
#pragma unroll
          for (int q = 0; q < GP; ++q) {
            const int e = threadIdx.x + (i0 + q) * nthr;
            const int r = e / Hx, k = e - r * Hx;
            const int row = row0 + rr * 16 + r;
            const int kc = k < Ax ? k : Ax - 1;
            const double* c = cb + (long long)(row < g.my ? row : g.my - 1) * mx;
            cv[q][0] = c[kc];
            cv[q][1] = c[o1 + kc];
            cv[q][2] = c[mx - 1 - kc];
            cv[q][3] = c[o1 + mx - 1 - kc];
          }
        }
#pragma unroll
        for (int q = 0; q < GP; ++q) {
          const int i = i0 + q;
          const int e = threadIdx.x + i * nthr;
          const int r = e / Hx, k = e - r * Hx;
          const int row = row0 + rr * 16 + r;
          const int c2 = mx - 1 - k;
          T y1 = 0, y2 = 0;
          if (a.g1_in) {
            const T* cr = comb + (rr * 16 + r) * ldc;
            const T E = cr[k], O = cr[Hx + k];
            y1 = E + O;
            y2 = E - O;
            if (k < Ax && row < g.my) {
              store_y(row, k, y1, cv[q][0], cv[q][1]);
              if (k != c2) store_y(row, c2, y2, cv[q][2], cv[q][3]);
            }
          }
          yv[rr][i][0] = y1;
          yv[rr][i][1] = y2;
        }
      }
  } else {
    // per point: the coarse values are read where they are added
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
#pragma unroll
      for (int i = 0; i < NPR; ++i) {
        const int e = threadIdx.x + i * nthr;
        const int r = e / Hx, k = e - r * Hx;
        const int row = row0 + rr * 16 + r;
        const int c2 = mx - 1 - k;
        T y1 = 0, y2 = 0;
        if (a.g1_in) {
          const T* cr = comb + (rr * 16 + r) * ldc;
          const T E = cr[k], O = cr[Hx + k];
          y1 = E + O;
          y2 = E - O;
          if (k < Ax && row < g.my) {
            const double* c = add_c ? cb + (long long)row * mx : nullptr;
            store_y(row, k, y1, add_c ? c[k] : 0.0, add_c ? c[o1 + k] : 0.0);
            if (k != c2) store_y(row, c2, y2, add_c ? c[c2] : 0.0, add_c ? c[o1 + c2] : 0.0);
          }
        }
        yv[rr][i][0] = y1;
        yv[rr][i][1] = y2;
      }
  }
  if (!form_b) return;
  if constexpr (kTwo) load_pre();
  if constexpr (!Eng::kCombInPlace) __syncthreads();   // combine values read before the operand is written
#pragma unroll
  for (int rr = 0; rr < RB; ++rr)
#pragma unroll
    for (int i = 0; i < NPR; ++i) {
      const int e = threadIdx.x + i * nthr;
      const int r = e / Hx, k = e - r * Hx;
      const bool mid = k == mx - 1 - k;
      const T y1 = yv[rr][i][0], y2 = yv[rr][i][1];
      T b1 = 0, b2 = 0;
      switch (a.b_mode) {
        case B_RPRIME_PLUS_Y: b1 = pre[rr][i][0] + y1; b2 = pre[rr][i][1] + y2; break;
        case B_H_YBUF_PLUS_Y: b1 = hT * pre[rr][i][0] + y1; b2 = hT * pre[rr][i][1] + y2; break;
        case B_H_Y: b1 = hT * y1; b2 = hT * y2; break;
        case B_INPUT: b1 = pre[rr][i][0]; b2 = pre[rr][i][1]; break;
      }
      T sum = 0, dif = 0;
      if (k < Ax) {
        sum = mid ? b1 : b1 + b2;
        dif = mid ? (T)0 : b1 - b2;
      }
      Eng::template put_a<RB>(smem_raw, Mx, rr * 16 + r, k, sum);
      Eng::template put_a<RB>(smem_raw, Mx, rr * 16 + r, Hx + k, dif);
    }
  __syncthreads();

  // ---- GEMM2: T = [sums | differences] (F_odd | F_even), stored in x-mode order -------------
#pragma unroll
  for (int rr = 0; rr < RB; ++rr)
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[rr][t] = acc_t{0, 0, 0, 0};
  Eng::template gemm_right<TPW, PD, RB>(smem_raw, table<Eng>(a.Sx, Mx, 0), Mx, blk, lt0, lts, li, lk, acc);
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    if (row0 + rr * 16 >= g.my) break;   // row blocks wholly past the interior write nothing
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int col = blk * Hx + (lt0 + t * lts) * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + rr * 16 + Eng::acc_row(lk, r);
        a.g2_out[s * a.g2_stride + (long long)row * Mx + col] = (T)acc[rr][t][r];
      }
    }
  }
}

// ---- column kernel ---------------------------------------------------------------------
// One workgroup = CB blocks of 16 columns of one slice.  fold: the input rows are points and
// the first product is the forward transform X = S_y T (optionally ./ lambda); otherwise the
// input rows are y-modes.  two: the inverse product U = S_y X follows, chained through LDS.  An
// inverse last product writes point rows (mirrored pairs combined); a forward one writes mode
// rows.
template <typename T>
struct ColArgs {
  const void* Sy;      // engine's half-transform tables of y: forward, then inverse
  const T* in;
  long long in_stride;
  const T* invlam;     // nullptr: no scaling
  int fold;            // input rows are points (forward first product)
  int two;             // chain the inverse product (needs fold)
  T* out;
  long long out_stride;
  int nsl = 0;         // set by the launcher: slice count of the slice-per-XCD grid, or 0
};

template <typename Eng, int TPW, int PD, int CB>
__global__ void __launch_bounds__((max_threads<Eng, TPW, PD, CB>()))
k_cols(Geom g, ColArgs<typename Eng::data_t> a) {
  using T = typename Eng::data_t;
  using acc_t = typename Eng::acc_t;
  extern __shared__ unsigned char smem_raw[];
  constexpr int NC = 16 * CB;       // columns of the workgroup
  const int Mx = g.Mx, My = g.My, Hy = My >> 1, my = g.my, Ay = (my + 1) / 2;
  int cg, s;
  if (!tile_and_slice(g.Mx / NC, a.nsl, cg, s)) return;
  const int nthr = blockDim.x, nw = nthr >> 6;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int blk = wave & 1, lt0 = wave >> 1, lts = nw >> 1;
  T* comb = reinterpret_cast<T*>(smem_raw);

  // Staging: every thread issues all of its loads before the first LDS write, so they are in
  // flight together.  fold: Hy*NC (point, mirrored point) pairs; else My*NC mode values.
  const T* src = a.in + s * a.in_stride + cg * NC;
  if (a.fold) {
    constexpr int NE = 2 * TPW * CB;   // pairs per thread: Hy*NC / blockDim.x
    T v1[NE], v2[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int k = e / NC, c = e % NC, r2 = my - 1 - k;
      v1[j] = k < Ay ? src[(long long)k * Mx + c] : (T)0;
      v2[j] = (k < Ay && r2 != k) ? src[(long long)r2 * Mx + c] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int k = e / NC, c = e % NC;
      T sum = 0, dif = 0;
      if (k < Ay) {
        if (my - 1 - k == k) {
          sum = v1[j];
        } else {
          sum = v1[j] + v2[j];
          dif = v1[j] - v2[j];
        }
      }
      Eng::template put_b<CB>(smem_raw, My, k, c, sum);
      Eng::template put_b<CB>(smem_raw, My, Hy + k, c, dif);
    }
  } else {
    constexpr int NE = 4 * TPW * CB;   // values per thread: My*NC / blockDim.x
    T v[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = threadIdx.x + j * nthr;
      v[j] = src[(long long)(e / NC) * Mx + (e % NC)];
    }
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = threadIdx.x + j * nthr;
      Eng::template put_b<CB>(smem_raw, My, e / NC, e % NC, v[j]);
    }
  }
  __syncthreads();

  acc_t acc[CB][TPW];
  auto product = [&](int inverse) {
#pragma unroll
    for (int w = 0; w < CB; ++w)
#pragma unroll
      for (int t = 0; t < TPW; ++t) acc[w][t] = acc_t{0, 0, 0, 0};
    Eng::template gemm_left<TPW, PD, CB>(table<Eng>(a.Sy, My, inverse), smem_raw, My, blk, lt0, lts, li, lk, acc);
  };
  product(!a.fold);
  if (a.invlam) {
    const T* il = a.invlam + (long long)(blk * Hy + lt0 * 16) * Mx + cg * NC;
#pragma unroll
    for (int w = 0; w < CB; ++w)
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[w][t][r] *= il[(t * lts * 16 + Eng::acc_row(lk, r)) * Mx + w * 16 + li];
  }
  if (a.two) {
    __syncthreads();
#pragma unroll
    for (int w = 0; w < CB; ++w)
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Eng::template put_b<CB>(smem_raw, My, blk * Hy + (lt0 + t * lts) * 16 + Eng::acc_row(lk, r),
                                  w * 16 + li, (T)acc[w][t][r]);
    __syncthreads();
    product(1);
  }
  T* dst = a.out + s * a.out_stride + cg * NC;
  if (a.fold && !a.two) {   // forward only: y-mode rows
#pragma unroll
    for (int w = 0; w < CB; ++w)
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          dst[(long long)(blk * Hy + (lt0 + t * lts) * 16 + Eng::acc_row(lk, r)) * Mx + w * 16 + li] =
              (T)acc[w][t][r];
    return;
  }
  // inverse last: E (odd modes) and O (even modes) of each pair through LDS, then the points
  constexpr int ldc = NC + 1;
  __syncthreads();  // every wave has read the operand, which the combine buffer overlays
#pragma unroll
  for (int w = 0; w < CB; ++w)
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        comb[(blk * Hy + (lt0 + t * lts) * 16 + Eng::acc_row(lk, r)) * ldc + w * 16 + li] = (T)acc[w][t][r];
  __syncthreads();
  for (int e = threadIdx.x; e < Ay * NC; e += nthr) {
    const int k = e / NC, c = e % NC;
    const T E = comb[k * ldc + c], O = comb[(Hy + k) * ldc + c];
    const int r2 = my - 1 - k;
    dst[(long long)k * Mx + c] = E + O;
    if (r2 != k) dst[(long long)r2 * Mx + c] = E - O;
  }
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
// A launch shape is (waves per workgroup, deep prefetch ring, blocks per workgroup: 16-row
// blocks of the row kernel or 16-column blocks of the column kernel).  Every shape runs the
// same multiply-adds in the same order, so the choice changes the speed only, never the
// result.  Choices are measured per (kernel, engine, extent, slices) and kept for the process
// (and in the file KKTDD_TUNE_CACHE names, one JSON object per line, when that is set).
struct Shape {
  int nw;
  int deep;
  int width;
};

// LDS one workgroup may take on gfx950.
constexpr size_t kMaxLds = 160 * 1024;
using TuneKey = std::array<int, 4>;   // kind (0 rows, 1 cols), engine, M, slices
std::mutex g_tune_mu;
std::map<TuneKey, Shape> g_tuned;
bool g_tune_loaded = false;
std::atomic<int> g_tune_gen{0};   // changes whenever kkt_tune_set replaces a shape

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
    int kind, eng, M, ns, nw, deep, width;
    if (std::sscanf(line, "{\"kind\": %d, \"engine\": %d, \"M\": %d, \"slices\": %d, \"waves\": %d, "
                    "\"deep\": %d, \"width\": %d", &kind, &eng, &M, &ns, &nw, &deep, &width) == 7)
      g_tuned[{kind, eng, M, ns}] = Shape{nw, deep, width};
  }
  std::fclose(f);
}

Shape tuned_shape(int kind, int eng, int M, int nslices) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tuned.find({kind, eng, M, nslices});
  if (it != g_tuned.end()) return it->second;
  return Shape{waves_for(M), 0, 1};
}

template <typename Eng> constexpr int engine_id();
template <> constexpr int engine_id<EngPlain<double>>() { return KKTDD_FP64; }
template <> constexpr int engine_id<EngPlain<float>>() { return KKTDD_FP32; }
template <> constexpr int engine_id<EngBF<1>>() { return KKTDD_BF16; }
template <> constexpr int engine_id<EngBF<3>>() { return KKTDD_BF16X3; }
template <> constexpr int engine_id<EngBF<6>>() { return KKTDD_BF16X6; }

// Dynamic LDS above 64 KiB has to be enabled per kernel before its first launch; the largest
// size enabled so far is remembered per kernel, so later launches (also those recorded into a
// HIP graph) make no further runtime call.
template <auto Kernel>
int allow_lds(size_t lds) {
  static std::atomic<size_t> enabled{65536};
  if (lds <= enabled.load(std::memory_order_acquire)) return 0;
  KKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  size_t cur = enabled.load();
  while (lds > cur && !enabled.compare_exchange_weak(cur, lds)) {
  }
  return 0;
}

// The slice-per-XCD grid pays off while the slices of a launch fit the XCDs' L2 caches
// (measured at padded 128 x 128 x 16 slices in float64: a row + column step pair 17.7 ->
// 16.4 us; at 256 x 256 x 64 slices it was 0.5% slower).  KKTDD_XCD_MAP=0/1 forces it.
inline bool slice_per_xcd(const Geom& g, int nslices, size_t elem) {
  const char* v = std::getenv("KKTDD_XCD_MAP");
  if (v && *v) return std::atoi(v) != 0;
  return (double)nslices * g.Mx * g.My * (double)elem <= 8.0 * 1024 * 1024;
}

inline dim3 sweep_grid(int ntile, int nslices, int nsl) {
  return nsl ? dim3(kXcds * ((nslices + kXcds - 1) / kXcds) * ntile) : dim3(ntile, nslices);
}

// Flops of the folded products: a 1-D transform of extent m costs 2*(A^2 + B^2) per vector,
// A = ceil(m/2), B = floor(m/2) (about half of the unfolded 2*m^2).
inline double folded_flops(int m) {
  const double A = (m + 1) / 2, B = m / 2;
  return 2.0 * (A * A + B * B);
}

template <typename Eng, int TPW, int PD, int RB>
int rows_t(const Geom& g, const RowArgs<typename Eng::data_t>& a, int nslices, int nw, int kclass,
           hipStream_t s) {
  const size_t lds = Eng::template rows_lds_total<RB>(g.Mx);
  if (lds > kMaxLds) return set_error(KKTDD_EINVAL, "row-kernel shape needs more LDS than a CU has");
  if (64 * nw > max_threads<Eng, TPW, PD, RB>()) return set_error(KKTDD_EINVAL, "row-kernel shape has too many waves");
  if (int e = allow_lds<k_rows<Eng, TPW, PD, RB>>(lds)) return e;
  const int ngemm = (a.g1_in ? 1 : 0) + (a.b_mode != B_NONE ? 1 : 0);
  prof_begin(kclass, s);
  RowArgs<typename Eng::data_t> la = a;
  la.nsl = slice_per_xcd(g, nslices, sizeof(typename Eng::data_t)) ? nslices : 0;
  // row blocks past the interior would only write padding rows, which nothing reads
  hipLaunchKernelGGL((k_rows<Eng, TPW, PD, RB>), sweep_grid((g.my + 16 * RB - 1) / (16 * RB), nslices, la.nsl),
                     dim3(64 * nw), lds, s, g, la);
  KKT_HIP(hipGetLastError());
  prof_end(kclass, s, 0.0, ngemm * nslices * (double)g.my * folded_flops(g.mx));
  return 0;
}

template <typename Eng, int TPW, int PD, int CB>
int cols_t(const Geom& g, const ColArgs<typename Eng::data_t>& a, int nslices, int nw, int kclass,
           hipStream_t s) {
  const size_t lds = Eng::template cols_lds_total<CB>(g.My);
  if (lds > kMaxLds || (g.Mx / 16) % CB != 0 || 64 * nw > max_threads<Eng, TPW, PD, CB>())
    return set_error(KKTDD_EINVAL, "column-kernel shape does not fit the extent, the LDS or the waves");
  if (int e = allow_lds<k_cols<Eng, TPW, PD, CB>>(lds)) return e;
  prof_begin(kclass, s);
  ColArgs<typename Eng::data_t> la = a;
  la.nsl = slice_per_xcd(g, nslices, sizeof(typename Eng::data_t)) ? nslices : 0;
  hipLaunchKernelGGL((k_cols<Eng, TPW, PD, CB>), sweep_grid(g.Mx / (16 * CB), nslices, la.nsl), dim3(64 * nw),
                     lds, s, g, la);
  KKT_HIP(hipGetLastError());
  prof_end(kclass, s, 0.0, (1 + a.two) * nslices * (double)g.mx * folded_flops(g.my));
  return 0;
}

// Whether a workgroup of `width` blocks fits the LDS (and, for the column kernel, the tile
// count of the x extent).
template <typename Eng>
bool width_fits(int kind, const Geom& g, int width) {
  size_t lds = 0;
  switch (width) {
    case 1: lds = kind == 0 ? Eng::template rows_lds_total<1>(g.Mx) : Eng::template cols_lds_total<1>(g.My); break;
    case 2: lds = kind == 0 ? Eng::template rows_lds_total<2>(g.Mx) : Eng::template cols_lds_total<2>(g.My); break;
    case 4: lds = kind == 0 ? Eng::template rows_lds_total<4>(g.Mx) : Eng::template cols_lds_total<4>(g.My); break;
    default: return false;
  }
  return lds <= kMaxLds && (kind == 0 || (g.Mx / 16) % width == 0);
}

// (tiles per wave, deep ring, blocks per workgroup) -> instantiation; deep rings exist for up
// to four tiles and one block, several blocks for up to four tiles and the default ring.
#define KKT_W_DISPATCH(FN, TPWV, W, ...)                                                 \
  switch (W) {                                                                           \
    case 2: return FN<Eng, TPWV, kPDDefault, 2>(__VA_ARGS__);                            \
    case 4: return FN<Eng, TPWV, kPDDefault, 4>(__VA_ARGS__);                            \
    default: return set_error(KKTDD_EINVAL, "unsupported blocks per workgroup");         \
  }
#define KKT_TPW_DISPATCH(FN, TPWV, DEEP, W, ...)                                         \
  if ((W) != 1) {                                                                        \
    if (DEEP) return set_error(KKTDD_EINVAL, "deep rings take one block per workgroup"); \
    switch (TPWV) {                                                                      \
      case 1: KKT_W_DISPATCH(FN, 1, W, __VA_ARGS__)                                      \
      case 2: KKT_W_DISPATCH(FN, 2, W, __VA_ARGS__)                                      \
      case 3: KKT_W_DISPATCH(FN, 3, W, __VA_ARGS__)                                      \
      case 4: KKT_W_DISPATCH(FN, 4, W, __VA_ARGS__)                                      \
      default: return set_error(KKTDD_EINVAL, "several blocks need <= 4 tiles per wave"); \
    }                                                                                    \
  }                                                                                      \
  switch (TPWV) {                                                                        \
    case 1: return (DEEP) ? FN<Eng, 1, deep_prefetch<1>(), 1>(__VA_ARGS__)               \
                          : FN<Eng, 1, kPDDefault, 1>(__VA_ARGS__);                      \
    case 2: return (DEEP) ? FN<Eng, 2, deep_prefetch<2>(), 1>(__VA_ARGS__)               \
                          : FN<Eng, 2, kPDDefault, 1>(__VA_ARGS__);                      \
    case 3: return (DEEP) ? FN<Eng, 3, deep_prefetch<3>(), 1>(__VA_ARGS__)               \
                          : FN<Eng, 3, kPDDefault, 1>(__VA_ARGS__);                      \
    case 4: return (DEEP) ? FN<Eng, 4, deep_prefetch<4>(), 1>(__VA_ARGS__)               \
                          : FN<Eng, 4, kPDDefault, 1>(__VA_ARGS__);                      \
    case 5: return FN<Eng, 5, kPDDefault, 1>(__VA_ARGS__);                               \
    case 6: return FN<Eng, 6, kPDDefault, 1>(__VA_ARGS__);                               \
    case 7: return FN<Eng, 7, kPDDefault, 1>(__VA_ARGS__);                               \
    case 8: return FN<Eng, 8, kPDDefault, 1>(__VA_ARGS__);                               \
    default: return set_error(KKTDD_EINVAL, "unsupported tile count");                   \
  }

template <typename Eng>
int rows_shape(const Geom& g, const RowArgs<typename Eng::data_t>& a, int nslices, Shape sh,
               int kclass, hipStream_t s) {
  KKT_TPW_DISPATCH(rows_t, g.Mx / 16 / sh.nw, sh.deep, sh.width, g, a, nslices, sh.nw, kclass, s)
}

template <typename Eng>
int cols_shape(const Geom& g, const ColArgs<typename Eng::data_t>& a, int nslices, Shape sh,
               int kclass, hipStream_t s) {
  KKT_TPW_DISPATCH(cols_t, g.My / 16 / sh.nw, sh.deep, sh.width, g, a, nslices, sh.nw, kclass, s)
}

// A shape kept for another extent's geometry may not fit this one (same padded extent,
// other tile counts along the other axis): fall back to one block per workgroup.
template <typename Eng>
Shape fitted(int kind, const Geom& g, Shape sh) {
  if (sh.width != 1 && !width_fits<Eng>(kind, g, sh.width)) sh.width = 1;
  return sh;
}

template <typename Eng>
int rows(const Geom& g, const RowArgs<typename Eng::data_t>& a, int nslices, int kclass, hipStream_t s) {
  return rows_shape<Eng>(g, a, nslices, fitted<Eng>(0, g, tuned_shape(0, engine_id<Eng>(), g.Mx, nslices)),
                         kclass, s);
}

template <typename Eng>
int cols(const Geom& g, const ColArgs<typename Eng::data_t>& a, int nslices, int kclass, hipStream_t s) {
  return cols_shape<Eng>(g, a, nslices, fitted<Eng>(1, g, tuned_shape(1, engine_id<Eng>(), g.My, nslices)),
                         kclass, s);
}

// r' in the engine's sweep precision: float64 for the float64 engine, float32 otherwise.
template <typename T>
void set_rin(RowArgs<T>& r, const void* rprime) {
  if constexpr (sizeof(T) == 8) r.rin = static_cast<const double*>(rprime);
  else r.rin32 = static_cast<const float*>(rprime);
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
               static_cast<const T*>(invlam), 1, 1, static_cast<T*>(w2), MM};
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
             const void* rprime, const double* c0, double* zw, void* Tb, void* Ub, void* Yb,
             hipStream_t s) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  T* Tbuf = static_cast<T*>(Tb);
  T* Ubuf = static_cast<T*>(Ub);
  T* Ybuf = static_cast<T*>(Yb);
  const long long ystride = (long long)g.L * MM;
  const int nd = g.nd, L = g.L;
  ColArgs<T> c{Sy, Tbuf, MM, static_cast<const T*>(invlam), 1, 1, Ubuf, MM};

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
    set_rin<T>(r, rprime);
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
                  const double* dscale, void* tmp, void* out, int nslices, hipStream_t s,
                  const float* in32) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  RowArgs<T> r = row_args<T>(Sx);
  r.b_mode = B_INPUT;
  r.rin = in;
  r.rin32 = in32;
  r.in_scale = dscale;
  r.g2_out = static_cast<T*>(tmp);
  r.g2_stride = MM;
  if (int e = rows<Eng>(g, r, nslices, KKTDD_K_SWEEP_ROWS, s)) return e;
  ColArgs<T> c{Sy, static_cast<const T*>(tmp), MM, nullptr, 1, 0,
               static_cast<T*>(out), MM};
  return cols<Eng>(g, c, nslices, KKTDD_K_SWEEP_COLS, s);
}

template <typename Eng>
int dst_inverse_t(const Geom& g, const void* Sx, const void* Sy, const void* in, void* tmp,
                  double* out, int nslices, double norm, const double* c0, hipStream_t s) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  ColArgs<T> c{Sy, static_cast<const T*>(in), MM, nullptr, 0, 0,
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
               void* bufB, int nslices, const void* rprime, void* ybuf, hipStream_t s) {
  using T = typename Eng::data_t;
  const long long MM = g.padded();
  RowArgs<T> r = row_args<T>(Sx);
  r.g1_in = static_cast<const T*>(bufA);
  r.g1_stride = MM;
  r.b_mode = B_H_Y;
  r.g2_out = static_cast<T*>(bufB);
  r.g2_stride = MM;
  if (rprime && ybuf) {
    // the per-step sweeps: time the forward-sweep row launch, which also reads r' and stores y
    r.b_mode = B_RPRIME_PLUS_Y;
    r.b_step = g.delta;
    set_rin<T>(r, rprime);
    r.ystore = static_cast<T*>(ybuf);
    r.ystore_stride = (long long)g.L * MM;
  }
  ColArgs<T> c{Sy, static_cast<const T*>(bufA), MM, static_cast<const T*>(invlam), 1, 1,
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
    // (the deep rings are not candidates: with the folded products' half-length k-loops they
    // measured slower than the default ring at every extent; tune_set can still select them)
    cand[nc++] = Shape{waves_for(M), 0, 1};
    for (int width : {1, 2, 4}) {
      if (!width_fits<Eng>(kind, g, width)) continue;
      for (int nw : {waves_for(M), 2, 4, 8, 16, t}) {
        if (!shape_valid(t, nw, 0, width, Eng::kMaxW16)) continue;
        bool seen = false;
        for (int i = 0; i < nc; ++i) seen = seen || (cand[i].nw == nw && cand[i].width == width);
        if (!seen && nc < 32) cand[nc++] = Shape{nw, 0, width};
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
    if (const char* v = std::getenv("KKTDD_TUNE_LOG"); v && std::atoi(v) != 0)
      for (int ci = 0; ci < nc; ++ci)
        std::fprintf(stderr, "kktdd tune: kind %d engine %d M %d slices %d waves %d width %d: %.2f us\n", kind,
                     engine_id<Eng>(), M, nslices, cand[ci].nw, cand[ci].width, best_round[ci]);
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
                        "\"deep\": %d, \"width\": %d, \"us\": %.2f}\n", kind, engine_id<Eng>(), M, nslices,
                     best.nw, best.deep, best.width, best_us);
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
                       hipStream_t s, const float* in32) {
  if (in32 && (precision == KKTDD_FP64 || dscale))
    return set_error(KKTDD_EINVAL, "float32 transform input needs a reduced-precision engine and no scale");
  KKT_ENGINE_DISPATCH(precision, dst_forward_t, g, Sx, Sy, in, dscale, tmp, out, nslices, s, in32)
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
                  const void* invlam, const void* rprime, const double* c0, double* zw,
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
  ColArgs<double> c{Sy, tmp, MM, nullptr, 1, 0, rhat, MM};
  return cols<EngPlain<double>>(g, c, g.nc, KKTDD_K_COARSE, s);
}

int launch_coarse_idst(const Geom& g, const double* Sx, const double* Sy, const double* chat,
                       double* c0, double* tmp, double norm, hipStream_t s) {
  const long long MM = g.padded();
  ColArgs<double> c{Sy, chat, MM, nullptr, 0, 0, tmp, MM};
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

// Blocks a 16-wave workgroup of an engine may hold.
static int max_w16_for(int precision) {
  switch (precision) {
    case KKTDD_FP64: return EngPlain<double>::kMaxW16;
    case KKTDD_FP32: return EngPlain<float>::kMaxW16;
    case KKTDD_BF16: return EngBF<1>::kMaxW16;
    case KKTDD_BF16X3: return EngBF<3>::kMaxW16;
    default: return EngBF<6>::kMaxW16;
  }
}

int tune_set(int kind, int precision, int extent, int nslices, int waves, int deep, int width) {
  const int t = extent / 16;
  if (kind < 0 || kind > 1 || precision < KKTDD_FP64 || precision > KKTDD_BF16X6 || extent < 32 ||
      extent % 32 != 0 || nslices < 1 || !shape_valid(t, waves, deep, width, max_w16_for(precision)))
    return set_error(KKTDD_EINVAL, "invalid launch shape");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tuned[{kind, precision, extent, nslices}] = Shape{waves, deep, width};
  g_tune_gen.fetch_add(1);
  return 0;
}

int tune_generation() { return g_tune_gen.load(); }

int tune_get(int kind, int precision, int extent, int nslices, int* waves, int* deep, int* width) {
  if (!waves || !deep || !width || extent < 32 || extent % 32 != 0)
    return set_error(KKTDD_EINVAL, "invalid launch-shape query");
  const Shape sh = tuned_shape(kind, precision, extent, nslices);
  *waves = sh.nw;
  *deep = sh.deep;
  *width = sh.width;
  return 0;
}

int launch_autotune(const Geom& g, int precision, const void* Sx, const void* Sy,
                    const void* invlam, void* bufA, void* bufB, int nslices, const void* rprime,
                    void* ybuf, hipStream_t s) {
  if (nslices <= 0) return 0;
  KKT_ENGINE_DISPATCH(precision, autotune_t, g, Sx, Sy, invlam, bufA, bufB, nslices, rprime, ybuf, s)
}

}  // namespace kktdd
