// Host driver of libkktdd: the C ABI declared in include/kktdd.h.
//
// Owns the handle (tables, work buffers, Krylov storage), validates problems, plans memory,
// orchestrates the preconditioner (Eqs. (7), (13)-(15)) and runs flexible GMRES (Sec. 4).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <algorithm>
#include <thread>
#include <vector>

#include "internal.h"

namespace kktdd {

namespace {
thread_local std::string g_last_error;
// Arnoldi orthogonalisation: DCGS2 (default) or, with KKTDD_ARNOLDI=cgs, classical
// Gram-Schmidt with selective reorthogonalisation.
bool arnoldi_dcgs2() {
  static const bool v = [] {
    const char* e = std::getenv("KKTDD_ARNOLDI");
    return !(e && std::string(e) == "cgs");
  }();
  return v;
}
constexpr int kRedBlocks = 1024;   // most blocks of a two-stage reduction
constexpr long kBatchStaggerUs = 300;   // start offset of the odd members of a batch
constexpr int kFieldSums = 3;      // per-block partial sums of a field reduction
constexpr int kMaxCgsRestart = 31; // the CGS passes keep one accumulator per basis vector
constexpr double kReorthEta = 0.70710678118654752;  // 1/sqrt(2)

// KKTDD_ROCTX=1: a roctx range around every kernel launch (named by its timer class) and
// around every entry point, for rocprofv3 --marker-trace.  Read once per process.
bool roctx_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("KKTDD_ROCTX");
    return e && std::atoi(e) != 0;
  }();
  return v;
}
const char* const kClassNames[KKTDD_K_COUNT] = {"kktdd:matvec", "kktdd:sweep_rows", "kktdd:sweep_cols",
                                                "kktdd:coarse", "kktdd:arnoldi", "kktdd:other"};

// KKTDD_DEBUG_POISON=1: every device buffer the library allocates is filled with NaN bytes,
// and the work buffers of the preconditioner and of FGMRES are filled again at the start of
// every precond_apply and fgmres_solve.  A kernel that reads workspace it has not written
// first then produces NaN.  Read at every use, so a process can switch it.
bool poison_enabled() {
  const char* e = std::getenv("KKTDD_DEBUG_POISON");
  return e && std::atoi(e) != 0;
}

// KKTDD_GRAPH=0 runs every Arnoldi step's launches from the stream instead of replaying them
// as a HIP graph (default 1).  Read at every solve.
bool graphs_enabled() {
  const char* e = std::getenv("KKTDD_GRAPH");
  return !(e && std::atoi(e) == 0);
}

// KKTDD_LOG=1: every fgmres_solve prints its residual-estimate history to stderr when it ends.
bool log_enabled() {
  const char* e = std::getenv("KKTDD_LOG");
  return e && std::atoi(e) != 0;
}

// RAII roctx range (no-op unless KKTDD_ROCTX=1).
struct RoctxScope {
  bool on;
  explicit RoctxScope(const char* name) : on(roctx_enabled()) {
    if (on) roctxRangePushA(name);
  }
  ~RoctxScope() {
    if (on) roctxRangePop();
  }
};
}  // namespace

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  return set_error(KKTDD_EHIP, buf);
}


namespace {
thread_local Prof* t_prof = nullptr;
}

void prof_begin(int kclass, hipStream_t s) {
  if (roctx_enabled() && kclass >= 0 && kclass < KKTDD_K_COUNT) roctxRangePushA(kClassNames[kclass]);
  if (!t_prof || !t_prof->on) return;
  hipEvent_t e = t_prof->next();
  if (!e) return;
  t_prof->open_ev = t_prof->used - 1;
  (void)hipEventRecord(e, s);
}

void prof_end(int kclass, hipStream_t s, double bytes, double flops) {
  if (roctx_enabled() && kclass >= 0 && kclass < KKTDD_K_COUNT) roctxRangePop();
  if (!t_prof || !t_prof->on) return;
  hipEvent_t e = t_prof->next();
  if (!e) return;
  (void)hipEventRecord(e, s);
  t_prof->recs.push_back({kclass, t_prof->open_ev, bytes, flops});
}

long long prof_mark() { return (t_prof && t_prof->on) ? (long long)t_prof->recs.size() : -1; }

void prof_add_bytes(long long record, double bytes) {
  if (!t_prof || record < 0 || record >= (long long)t_prof->recs.size()) return;
  t_prof->recs[(size_t)record].bytes += bytes;
}

}  // namespace kktdd

using namespace kktdd;


namespace {

// Makes the handle's timer current for the calling thread during one entry point.
struct ProfScope {
  Prof* saved;
  explicit ProfScope(kktdd_handle* H) : saved(t_prof) { t_prof = H ? &H->prof : nullptr; }
  ~ProfScope() { t_prof = saved; }
};

template <typename T>
int dalloc(kktdd_handle* h, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return 0;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    char buf[160];
    std::snprintf(buf, sizeof buf, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                  hipGetErrorString(e));
    return set_error(e == hipErrorOutOfMemory ? KKTDD_ENOMEM : KKTDD_EHIP, buf);
  }
  h->allocations.push_back(q);
  *p = static_cast<T*>(q);
  if (poison_enabled()) {
    if (hipMemsetAsync(q, 0xFF, count * sizeof(T), h->stream) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(KKTDD_EHIP, "poisoning a new buffer failed");
    }
  }
  return 0;
}

int validate(const kktdd_problem* p) {
  if (!p) return set_error(KKTDD_EINVAL, "problem is NULL");
  auto bad = [](const char* m) { return set_error(KKTDD_EINVAL, m); };
  if (p->nx < 2 || p->ny < 2) return bad("nx and ny must be >= 2");
  if (p->nx > 1024 || p->ny > 1024) return bad("nx and ny must be <= 1024");
  if (p->nt < 1 || p->nt > 65535) return bad("nt must be in 1..65535 (one launch row per time node)");
  const double pos[] = {p->Lx, p->Ly, p->T, p->nu, p->omega};
  for (double v : pos)
    if (!(v > 0.0) || !std::isfinite(v)) return bad("Lx, Ly, T, nu, omega must be positive and finite");
  if (p->n_sub < 1 || p->nt % p->n_sub != 0) return bad("n_sub must be >= 1 and divide nt");
  if (p->n_sub > 65535) return bad("n_sub must be <= 65535 (one launch row per subdomain)");
  const int k = p->nt / p->n_sub;
  if (p->overlap < 0 || p->overlap > k) return bad("overlap must satisfy 0 <= overlap <= nt/n_sub");
  if (p->coarse < 0 || p->coarse > 2) return bad("coarse must be 0, 1 or 2");
  if (p->coarse == 2 && k < 2) return bad("a linear coarse basis needs nt/n_sub >= 2");
  if (p->precision < KKTDD_FP64 || p->precision > KKTDD_AUTO) return bad("unknown precision");
  if (p->sweep != KKTDD_SWEEP_STEP && p->sweep != KKTDD_SWEEP_MODAL) return bad("unknown sweep placement");
  if (p->overlap_side < 0 || p->overlap_side > 1 || p->schwarz < 0 || p->schwarz > 1 ||
      p->local < 0 || p->local > 1 || p->combine < 0 || p->combine > 2)
    return bad("unknown method variant");
  if ((p->overlap_side || p->schwarz || p->local || p->combine) &&
      (p->sweep != KKTDD_SWEEP_MODAL || (p->precision != KKTDD_FP64 && p->precision != KKTDD_AUTO)))
    return bad("method variants run on the float64 modal sweeps only");
  if ((long long)p->nt * (p->nx - 1) * (p->ny - 1) > (1LL << 40)) return bad("problem too large");
  return KKTDD_OK;
}

bool is_bf16(int precision) { return precision >= KKTDD_BF16 && precision <= KKTDD_BF16X6; }

// Condition number of D_sigma = sigma I + dt nu A_h: the ratio of its extreme eigenvalues
// sigma + dt nu (lambda^x_p + lambda^y_q), lambda_p = (4/dx^2) sin^2(p pi / (2 nx)).
double kappa_D(const kktdd_problem& p) {
  const double dx = p.Lx / p.nx, dy = p.Ly / p.ny, dt = p.T / p.nt;
  const double sigma = 1.0 + dt / std::sqrt(p.omega);
  auto lam = [](int i, int n, double d) {
    const double s = std::sin(i * 3.14159265358979323846 / (2.0 * n));
    return 4.0 / (d * d) * s * s;
  };
  const double lo = lam(1, p.nx, dx) + lam(1, p.ny, dy);
  const double hi = lam(p.nx - 1, p.nx, dx) + lam(p.ny - 1, p.ny, dy);
  return (sigma + dt * p.nu * hi) / (sigma + dt * p.nu * lo);
}

// KKTDD_AUTO: float32 sweeps while kappa(D_sigma) <= kAutoKappaFp32, else float64.  Rounding
// of the float32 transforms is amplified by kappa in the sweep output; up to this bound
// the float64 FGMRES iteration count stays within two of the float64 path on the uneven
// batch workload, beyond it float32 sweeps can stall the outer iteration.
constexpr double kAutoKappaFp32 = 500.0;

kktdd_problem resolve(const kktdd_problem& p) {
  kktdd_problem r = p;
  const bool variant = p.overlap_side || p.schwarz || p.local || p.combine;
  if (r.precision == KKTDD_AUTO)
    r.precision = !variant && kappa_D(p) <= kAutoKappaFp32 ? KKTDD_FP32 : KKTDD_FP64;
  return r;
}

Geom make_geom(const kktdd_problem& p) {
  Geom g{};
  g.mx = p.nx - 1;
  g.my = p.ny - 1;
  g.Mx = pad_extent(g.mx, is_bf16(p.precision));
  g.My = pad_extent(g.my, is_bf16(p.precision));
  g.nt = p.nt;
  g.nxy = g.mx * g.my;
  g.P = (long long)g.nt * g.nxy;
  const double dx = p.Lx / p.nx, dy = p.Ly / p.ny, dt = p.T / p.nt;
  g.cx = dt * p.nu / (dx * dx);
  g.cy = dt * p.nu / (dy * dy);
  g.h = dt * dx * dy;
  g.omega = p.omega;
  g.dt = dt;
  g.sigma = 1.0 + dt / std::sqrt(p.omega);
  g.nd = p.n_sub;
  g.k = p.nt / p.n_sub;
  g.delta = p.overlap;
  g.sym = p.overlap_side;
  g.asm_sum = p.schwarz;
  g.exact_local = p.local;
  g.combine = p.combine;
  g.L = g.k + g.delta * (1 + g.sym);
  g.nb = p.coarse;
  g.nc = g.nb * g.nd;
  return g;
}

// Leading dimension of the Krylov basis: 3P rounded up to 64 doubles, so every basis vector
// starts 512-byte aligned (the Arnoldi kernels stream them with 16-byte loads).
long long krylov_ld(const Geom& g) { return (3 * g.P + 63) / 64 * 64; }

// Blocks of the Arnoldi reductions: one element pair per thread at most, kRedBlocks at most.
int krylov_blocks(const Geom& g) {
  const long long pairs = (3 * g.P + 1) / 2;
  const long long b = (pairs + 255) / 256;
  return (int)(b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks);
}

// Small Krylov buffers for restart length R (doubles):
//   part  per-block partial sums, blocks x (2R+3)
//   sums  reduced sums: DCGS2 [0, 2R+3) plus the norm slot at 2R+4; CGS three runs of R+2
//   rec   Arnoldi record read back by the host (DCGS2 2j+5, CGS 2(j+3)+1 doubles, j < R)
//   vinv  basis scales, R+2
//   ydev  update coefficients [0, 2R+2), then the solution coefficients yv, yw at 2R+4
//   host  pinned: the record, then the staged yv, yw at 2R+8
struct KrylovSmall {
  size_t part, sums, rec, vinv, ydev, host;
  explicit KrylovSmall(int R)
      : part((size_t)kRedBlocks * (2 * R + 3)), sums(3 * (size_t)R + 8), rec(2 * (size_t)R + 8),
        vinv((size_t)R + 2), ydev(4 * (size_t)R + 4), host(4 * (size_t)R + 8) {}
  size_t device_bytes() const { return (part + sums + rec + vinv + ydev) * 8 + 256; }
};

struct Plan {
  size_t tables, sweeps, coarse, krylov;
  size_t total() const { return tables + sweeps + coarse + krylov; }
};

constexpr int kModalRegSteps = 32;   // must match the register sweep length in modal.hip

// Which buffers a configuration needs.  The coarse level runs in physical space (its own
// float64 transforms of 2N_D slices, r' formed pointwise in float64) for the per-step sweeps
// and for the reduced-precision modal sweeps: float32 or bfloat16 transforms of r itself would
// round r before the cancellation in r - S_hat c.  Float64 modal sweeps do the coarse level in
// mode space.
bool physical_coarse(const Geom& g, int precision, int sweep) {
  return g.nb > 0 && (sweep == KKTDD_SWEEP_STEP || precision != KKTDD_FP64);
}
bool needs_rprime(const Geom& g, int precision, int sweep) {
  return sweep == KKTDD_SWEEP_STEP || physical_coarse(g, precision, sweep);
}

// Modal sweep store (doubles): the forward states when a sweep is too long for registers, or
// the pivots and forward values of the exact local solves.
size_t modal_store(const Geom& g) {
  const size_t per = (size_t)g.nd * g.L * (size_t)g.padded();
  if (g.exact_local) return 2 * per;
  return g.L > kModalRegSteps ? per : 0;
}
// Additive-Schwarz extension values (doubles): delta nodes per side and subdomain.
size_t modal_ext(const Geom& g) {
  return g.asm_sum ? (size_t)g.nd * g.delta * (1 + g.sym) * (size_t)g.padded() : 0;
}

Plan plan(const Geom& g, int precision, int sweep, int R) {
  const size_t el = precision == KKTDD_FP64 ? 8 : 4;
  const size_t MM = (size_t)g.padded();
  Plan p{};
  p.tables = ((size_t)g.Mx * g.Mx + (size_t)g.My * g.My + MM) * 12 + (size_t)(g.mx + g.my) * 8;
  if (is_bf16(precision)) p.tables += ((size_t)g.Mx * g.Mx + (size_t)g.My * g.My) * 6;
  if (sweep == KKTDD_SWEEP_MODAL) {
    p.sweeps = 2 * (size_t)g.nt * MM * el + (modal_store(g) + modal_ext(g)) * 8;
  } else {
    p.sweeps = (2 * (size_t)g.nd * MM + (size_t)g.nd * g.L * MM) * el;
  }
  if (needs_rprime(g, precision, sweep)) p.sweeps += (size_t)g.P * el;
  if (g.nb > 0) {
    const int hb = 2 * g.nb - 1;
    p.coarse = (size_t)g.nc * MM * 8 * 2 + (size_t)g.nxy * g.nc * (hb + 1) * 8;
    if (physical_coarse(g, precision, sweep)) p.coarse += (size_t)g.nc * g.nxy * 8 * 4;
  }
  p.coarse += (size_t)kRedBlocks * kFieldSums * 8 + 128 * 8;
  if (R > 0)
    p.krylov = ((size_t)(R + 1) * (size_t)krylov_ld(g) + (size_t)R * (size_t)g.P) * 8 +
               KrylovSmall(R).device_bytes();
  return p;
}

// bfloat16 of a value: round its float32 image to nearest-even on the upper 16 bits.
uint16_t bf16_round(double v) {
  const float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// sin(pi * r / n) with r reduced modulo 2n first, so the argument stays in [0, 2 pi)
double sinpi_frac(long long r, long long n) {
  r %= 2 * n;
  return std::sin(M_PI * (double)r / (double)n);
}

int build_tables(kktdd_handle* H) {
  const Geom& g = H->g;
  const kktdd_problem& p = H->prob;
  // Half-size transform blocks of one extent (n intervals, padded extent M = 2H), block b at
  // b*H*H: F_b[k][j] = sin(pi f_b(j) (k+1) / n), f_0(j) = 2j+1 for k, j < ceil(m/2) and
  // f_1(j) = 2j+2 for k, j < floor(m/2), zero elsewhere; `transposed` stores F_b^T.
  auto half = [](int n, int M, bool transposed) {
    const int H = M / 2, m = n - 1, A = (m + 1) / 2, B = m / 2;
    std::vector<double> Q((size_t)M * H, 0.0);
    for (int b = 0; b < 2; ++b) {
      const int lim = b == 0 ? A : B;
      for (int k = 0; k < lim; ++k)
        for (int j = 0; j < lim; ++j)
          Q[(size_t)b * H * H + (transposed ? (size_t)j * H + k : (size_t)k * H + j)] =
              sinpi_frac((long long)(2 * j + 1 + b) * (k + 1), n);
    }
    return Q;
  };
  // The plain engines read each H x H block with k-steps (groups of four rows) interleaved in
  // groups of kg (2 for float64, 4 for float32): row 4ks + lk, column c goes to
  // ((ks/kg * 4 + lk) H + c) kg + ks % kg.
  auto group_rows = [](std::vector<double>& Q, int M, int kg) {
    const int H = M / 2;
    std::vector<double> out(Q.size());
    for (int b = 0; b < 2; ++b) {
      const size_t base = (size_t)b * H * H;
      for (int k = 0; k < H; ++k) {
        const int ks = k >> 2, lk = k & 3;
        for (int c = 0; c < H; ++c)
          out[base + ((size_t)((ks / kg) * 4 + lk) * H + c) * kg + (ks % kg)] = Q[base + (size_t)k * H + c];
      }
    }
    Q.swap(out);
  };
  // Engine operand of one extent: forward blocks, then inverse blocks.  The plain engines
  // reduce over the row index of what they read (forward F, inverse F^T); the bfloat16 engines
  // over the column index (forward F^T, inverse F).  kg > 0: the plain engines' k-step groups.
  auto sine = [&](int n, int M, bool bf, int kg) {
    std::vector<double> f = half(n, M, bf);
    std::vector<double> i = half(n, M, !bf);
    if (kg > 0) {
      group_rows(f, M, kg);
      group_rows(i, M, kg);
    }
    f.insert(f.end(), i.begin(), i.end());
    return f;
  };
  const double dx = p.Lx / p.nx, dy = p.Ly / p.ny, dtnu = g.dt * p.nu;
  std::vector<double> lx(g.mx), ly(g.my);
  for (int a = 0; a < g.mx; ++a) {
    const double s = std::sin(M_PI * (a + 1) / (2.0 * p.nx));
    lx[a] = dtnu * 4.0 / (dx * dx) * s * s;
  }
  for (int a = 0; a < g.my; ++a) {
    const double s = std::sin(M_PI * (a + 1) / (2.0 * p.ny));
    ly[a] = dtnu * 4.0 / (dy * dy) * s * s;
  }
  const std::vector<double> Sx = sine(p.nx, g.Mx, false, 2), Sy = sine(p.ny, g.My, false, 2);
  const std::vector<double> Sx4 = sine(p.nx, g.Mx, false, 4), Sy4 = sine(p.ny, g.My, false, 4);
  const double norm = 4.0 / ((double)p.nx * p.ny);
  std::vector<double> inv((size_t)g.padded(), 0.0);   // mode order of mode_pos
  for (int q = 0; q < g.my; ++q)
    for (int a = 0; a < g.mx; ++a)
      inv[(size_t)mode_pos(q, g.My) * g.Mx + mode_pos(a, g.Mx)] = norm / (g.sigma + ly[q] + lx[a]);
  auto to32 = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
  if (is_bf16(p.precision)) {
    auto parts = [](const std::vector<double>& S) {
      const size_t n = S.size();
      std::vector<uint16_t> out(3 * n);
      for (size_t i = 0; i < n; ++i) {
        double rest = S[i];
        for (int q = 0; q < 3; ++q) {
          const uint16_t b = bf16_round(rest);
          out[q * n + i] = b;
          rest -= bf16_value(b);
        }
      }
      return out;
    };
    // three parts of the forward blocks, then three of the inverse blocks
    auto parts2 = [&](const std::vector<double>& S) {
      const size_t h = S.size() / 2;
      std::vector<uint16_t> a = parts(std::vector<double>(S.begin(), S.begin() + h));
      const std::vector<uint16_t> b = parts(std::vector<double>(S.begin() + h, S.end()));
      a.insert(a.end(), b.begin(), b.end());
      return a;
    };
    const std::vector<uint16_t> bx = parts2(sine(p.nx, g.Mx, true, 0)), by = parts2(sine(p.ny, g.My, true, 0));
    if (int e = dalloc(H, &H->SxBF, bx.size())) return e;
    if (int e = dalloc(H, &H->SyBF, by.size())) return e;
    KKT_HIP(hipMemcpy(H->SxBF, bx.data(), bx.size() * 2, hipMemcpyHostToDevice));
    KKT_HIP(hipMemcpy(H->SyBF, by.data(), by.size() * 2, hipMemcpyHostToDevice));
  }

  if (int e = dalloc(H, &H->Sx64, Sx.size())) return e;
  if (int e = dalloc(H, &H->Sy64, Sy.size())) return e;
  if (int e = dalloc(H, &H->invlam64, inv.size())) return e;
  if (int e = dalloc(H, &H->Sx32, Sx.size())) return e;
  if (int e = dalloc(H, &H->Sy32, Sy.size())) return e;
  if (int e = dalloc(H, &H->invlam32, inv.size())) return e;
  if (int e = dalloc(H, &H->lamx, lx.size())) return e;
  if (int e = dalloc(H, &H->lamy, ly.size())) return e;
  KKT_HIP(hipMemcpy(H->Sx64, Sx.data(), Sx.size() * 8, hipMemcpyHostToDevice));
  KKT_HIP(hipMemcpy(H->Sy64, Sy.data(), Sy.size() * 8, hipMemcpyHostToDevice));
  KKT_HIP(hipMemcpy(H->invlam64, inv.data(), inv.size() * 8, hipMemcpyHostToDevice));
  const auto Sx32 = to32(Sx4), Sy32 = to32(Sy4), inv32 = to32(inv);
  KKT_HIP(hipMemcpy(H->Sx32, Sx32.data(), Sx32.size() * 4, hipMemcpyHostToDevice));
  KKT_HIP(hipMemcpy(H->Sy32, Sy32.data(), Sy32.size() * 4, hipMemcpyHostToDevice));
  KKT_HIP(hipMemcpy(H->invlam32, inv32.data(), inv32.size() * 4, hipMemcpyHostToDevice));
  KKT_HIP(hipMemcpy(H->lamx, lx.data(), lx.size() * 8, hipMemcpyHostToDevice));
  KKT_HIP(hipMemcpy(H->lamy, ly.data(), ly.size() * 8, hipMemcpyHostToDevice));
  return 0;
}

// Gram matrices of the coarse time basis in band storage G[i*(hb+1) + b] = G(i, i-b).
int build_coarse(kktdd_handle* H) {
  const Geom& g = H->g;
  if (g.nb == 0) return 0;
  const int hb = 2 * g.nb - 1, w = hb + 1, nc = g.nc;
  std::vector<double> G2((size_t)nc * w, 0.0), G0((size_t)nc * w, 0.0), G1((size_t)nc * w, 0.0);
  // basis values at node n (1-based): slots nb*s + b, s = (n-1)/k
  auto basis = [&](int n, double* v) {
    const int s = (n - 1) / g.k;
    v[0] = 1.0;
    v[1] = -1.0 + 2.0 * (double)(n - s * g.k) / g.k;
    return g.nb * s;
  };
  auto add = [&](std::vector<double>& G, int a, int b, double val) {
    if (a < b) std::swap(a, b);
    if (a - b <= hb) G[(size_t)a * w + (a - b)] += val;
  };
  for (int n = 1; n <= g.nt; ++n) {
    double va[2], vb[2];
    const int sa = basis(n, va);
    for (int a = 0; a < g.nb; ++a)
      for (int b = 0; b < g.nb; ++b) {
        if (sa + a < sa + b) continue;  // lower triangle once
        add(G2, sa + a, sa + b, va[a] * va[b]);
        if (n >= 2) add(G0, sa + a, sa + b, va[a] * va[b]);
      }
    if (n < g.nt) {
      const int sb = basis(n + 1, vb);
      // (E + E^T) couples n and n+1 symmetrically: Z(n,a) Z(n+1,b) + Z(n+1,a) Z(n,b)
      for (int a = 0; a < g.nb; ++a)
        for (int b = 0; b < g.nb; ++b) {
          const int ia = sa + a, ib = sb + b;
          // contributes to G1(ia, ib) and G1(ib, ia); store the lower one once
          if (ia == ib) add(G1, ia, ib, 2.0 * va[a] * vb[b]);
          else add(G1, ia, ib, va[a] * vb[b]);
        }
    }
  }
  double *dG2, *dG0, *dG1;
  int* dinfo;
  if (int e = dalloc(H, &dG2, G2.size())) return e;
  if (int e = dalloc(H, &dG0, G0.size())) return e;
  if (int e = dalloc(H, &dG1, G1.size())) return e;
  if (int e = dalloc(H, &dinfo, 1)) return e;
  KKT_HIP(hipMemcpy(dG2, G2.data(), G2.size() * 8, hipMemcpyHostToDevice));
  KKT_HIP(hipMemcpy(dG0, G0.data(), G0.size() * 8, hipMemcpyHostToDevice));
  KKT_HIP(hipMemcpy(dG1, G1.data(), G1.size() * 8, hipMemcpyHostToDevice));
  KKT_HIP(hipMemset(dinfo, 0, sizeof(int)));
  if (int e = dalloc(H, &H->cfac, (size_t)g.nxy * nc * w)) return e;
  if (int e = launch_coarse_factor(g, dG2, dG0, dG1, H->lamx, H->lamy, H->cfac, dinfo, H->stream)) return e;
  int info = 0;
  KKT_HIP(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, H->stream));
  KKT_HIP(hipStreamSynchronize(H->stream));
  if (info) return set_error(KKTDD_EINVAL, "coarse operator not positive definite");
  return 0;
}

// Coarse correction in physical space (float64): c0 = S_hat_0^{-1} Z^T r, then
// r' = scale*r - S_hat Z c0 pointwise.  Returns c0 (nullptr without a coarse level).
int coarse_physical(kktdd_handle* H, const double* rw, const double* dscale, const double** c0out) {
  const Geom& g = H->g;
  hipStream_t s = H->stream;
  const double* c0 = nullptr;
  if (g.nb > 0) {
    if (int e = launch_restrict(g, rw, dscale, H->r0, s)) return e;
    if (int e = launch_coarse_dst(g, H->Sx64, H->Sy64, H->r0, H->chat, H->ctmp, s)) return e;
    if (int e = launch_coarse_solve(g, H->cfac, H->chat, s)) return e;
    const double norm = 4.0 / ((double)H->prob.nx * H->prob.ny);
    if (int e = launch_coarse_idst(g, H->Sx64, H->Sy64, H->chat, H->c0, H->ctmp, norm, s)) return e;
    if (int e = launch_apply_D(g, H->c0, H->Dc0, g.nc, g.sigma, s)) return e;
    if (int e = launch_apply_D(g, H->Dc0, H->DDc0, g.nc, g.sigma, s)) return e;
    c0 = H->c0;
  }
  *c0out = c0;
  return launch_residual_prime(g, rw, dscale, c0, H->Dc0, H->DDc0, H->rprime, H->elem == 4, s);
}

// Transform-hoisted Schur block (sine-mode space): see modal.hip.
int schur_apply_modal(kktdd_handle* H, const double* rw, const double* dscale, double* zw) {
  const Geom& g = H->g;
  hipStream_t s = H->stream;
  const int prec = H->prob.precision;
  const double norm = 4.0 / ((double)H->prob.nx * H->prob.ny);
  if (physical_coarse(g, prec, KKTDD_SWEEP_MODAL)) {
    // float32 transforms: coarse level and r' in float64 physical space, sweeps in mode space
    const double* c0 = nullptr;
    if (int e = coarse_physical(H, rw, dscale, &c0)) return e;
    if (int e = launch_dst_forward(g, prec, H->Sx(), H->Sy(), nullptr, nullptr, H->Mtmp, H->Rhat, g.nt, s,
                                   static_cast<const float*>(H->rprime))) return e;
    if (int e = launch_modal_sweeps(g, prec, H->Rhat, nullptr, 0, H->lamx, H->lamy, H->Ysc, H->Mtmp,
                                    nullptr, s)) return e;
    return launch_dst_inverse(g, prec, H->Sx(), H->Sy(), H->Mtmp, H->Rhat, zw, g.nt, norm, c0, s);
  }
  // float64: everything in sine-mode space between one forward and one inverse transform
  double* rhat = static_cast<double*>(H->Rhat);
  double* zhat = static_cast<double*>(H->Mtmp);
  if (int e = launch_dst_forward(g, prec, H->Sx(), H->Sy(), rw, dscale, H->Mtmp, H->Rhat, g.nt, s)) return e;
  const bool coarse = g.nb > 0;
  const bool fine_first = coarse && g.combine == KKTDD_COMBINE_FINE_FIRST;
  const double* c0 = nullptr;
  if (coarse && !fine_first) {
    if (int e = launch_modal_restrict(g, prec, rhat, H->chat, s)) return e;
    if (int e = launch_coarse_solve(g, H->cfac, H->chat, s)) return e;
    c0 = H->chat;
  }
  // coarse first: the sweeps see r - S_hat c; additive: r itself; both add c to the output
  const int sub = g.combine == KKTDD_COMBINE_COARSE_FIRST ? 1 : 0;
  if (int e = launch_modal_sweeps(g, prec, rhat, c0, sub, H->lamx, H->lamy, H->Ysc, zhat, H->ext, s)) return e;
  if (g.asm_sum)
    if (int e = launch_modal_asm_add(g, H->ext, zhat, s)) return e;
  if (fine_first) {
    // y = fine level of r; z = y + Q_0 (r - S_hat y)
    if (int e = launch_modal_residual(g, zhat, H->lamx, H->lamy, rhat, s)) return e;
    if (int e = launch_modal_restrict(g, prec, rhat, H->chat, s)) return e;
    if (int e = launch_coarse_solve(g, H->cfac, H->chat, s)) return e;
    if (int e = launch_modal_prolong_add(g, H->chat, zhat, s)) return e;
  }
  return launch_dst_inverse(g, prec, H->Sx(), H->Sy(), H->Mtmp, H->Rhat, zw, g.nt, norm, nullptr, s);
}

int schur_apply(kktdd_handle* H, const double* rw, const double* dscale, double* zw) {
  if (H->prob.sweep == KKTDD_SWEEP_MODAL) return schur_apply_modal(H, rw, dscale, zw);
  const Geom& g = H->g;
  hipStream_t s = H->stream;
  const double* c0 = nullptr;
  if (int e = coarse_physical(H, rw, dscale, &c0)) return e;
  return launch_sweeps(g, H->prob.precision, H->Sx(), H->Sy(), H->invlam(), H->rprime, c0, zw,
                       H->Tbuf, H->Ubuf, H->Ybuf, s);
}

// KKTDD_DEBUG_POISON: NaN bytes into every work buffer that a kernel must write before it
// reads it (not the tables, the coarse factors, or the coarse mode slots whose padding must
// stay zero).  Stream-ordered before the work that follows.
int poison_workspace(kktdd_handle* H) {
  if (!poison_enabled()) return 0;
  const Geom& g = H->g;
  const size_t MM = (size_t)g.padded(), el = H->elem;
  auto fill = [&](void* p, size_t bytes) -> int {
    if (!p || !bytes) return 0;
    KKT_HIP(hipMemsetAsync(p, 0xFF, bytes, H->stream));
    return 0;
  };
  if (int e = fill(H->Tbuf, (size_t)g.nd * MM * el)) return e;
  if (int e = fill(H->Ubuf, (size_t)g.nd * MM * el)) return e;
  if (int e = fill(H->Ybuf, (size_t)g.nd * g.L * MM * el)) return e;
  if (int e = fill(H->rprime, (size_t)g.P * el)) return e;
  if (int e = fill(H->Rhat, (size_t)g.nt * MM * el)) return e;
  if (int e = fill(H->Mtmp, (size_t)g.nt * MM * el)) return e;
  if (int e = fill(H->Ysc, modal_store(g) * 8)) return e;
  if (int e = fill(H->ext, modal_ext(g) * 8)) return e;
  for (double* p : {H->r0, H->c0, H->Dc0, H->DDc0})
    if (int e = fill(p, (size_t)g.nc * g.nxy * 8)) return e;
  if (int e = fill(H->partials, (size_t)kRedBlocks * kFieldSums * 8)) return e;
  if (H->R > 0) {
    const KrylovSmall ks(H->R);
    if (int e = fill(H->V, (size_t)(H->R + 1) * (size_t)krylov_ld(g) * 8)) return e;
    if (int e = fill(H->Zw, (size_t)H->R * (size_t)g.P * 8)) return e;
    if (int e = fill(H->kpart, ks.part * 8)) return e;
    if (int e = fill(H->ksums, ks.sums * 8)) return e;
    if (int e = fill(H->hcol, ks.rec * 8)) return e;
    if (int e = fill(H->vinv, ks.vinv * 8)) return e;
    if (int e = fill(H->ydev, ks.ydev * 8)) return e;
  }
  return 0;
}

// squared norms of the three fields of a KKT vector, to the host (synchronises)
int field_sumsq(kktdd_handle* H, const double* r, double out[3]) {
  if (int e = launch_sumsq_blocks(H->g, r, H->partials, kRedBlocks, H->stream)) return e;
  if (int e = launch_reduce_partials(H->partials, kRedBlocks, kFieldSums, H->sums, H->stream)) return e;
  KKT_HIP(hipMemcpyAsync(H->host_sums, H->sums, 3 * sizeof(double), hipMemcpyDeviceToHost, H->stream));
  KKT_HIP(hipStreamSynchronize(H->stream));
  for (int i = 0; i < 3; ++i) out[i] = H->host_sums[i];
  return 0;
}

// Launch shapes of the sweep GEMM kernels for this handle's extents (unless KKTDD_AUTOTUNE=0):
// measured on the handle's zeroed work buffers, once per (extent, slices, engine) per process.
bool autotune_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("KKTDD_AUTOTUNE");
    return !(e && std::string(e) == "0");
  }();
  return v;
}

int autotune(kktdd_handle* H) {
  if (!autotune_enabled()) return 0;
  const Geom& g = H->g;
  const int prec = H->prob.precision;
  const size_t MM = (size_t)g.padded();
  void *a = nullptr, *b = nullptr;
  int nslices = 0;
  if (H->prob.sweep == KKTDD_SWEEP_MODAL) {
    a = H->Rhat;
    b = H->Mtmp;
    nslices = g.nt;
  } else {
    a = H->Tbuf;
    b = H->Ubuf;
    nslices = g.nd;
  }
  const size_t bytes = (size_t)nslices * MM * H->elem;
  KKT_HIP(hipMemsetAsync(a, 0, bytes, H->stream));
  KKT_HIP(hipMemsetAsync(b, 0, bytes, H->stream));
  const bool step = H->prob.sweep == KKTDD_SWEEP_STEP;
  if (step) KKT_HIP(hipMemsetAsync(H->rprime, 0, (size_t)g.P * H->elem, H->stream));
  if (int e = launch_autotune(g, prec, H->Sx(), H->Sy(), H->invlam(), a, b, nslices, step ? H->rprime : nullptr,
                              step ? H->Ybuf : nullptr, H->stream)) return e;
  KKT_HIP(hipStreamSynchronize(H->stream));
  return 0;
}

// Drop the recorded Arnoldi steps (their kernel arguments point into the Krylov storage).
void release_graphs(kktdd_handle* H) {
  for (hipGraphExec_t& e : H->graph_exec)
    if (e) (void)hipGraphExecDestroy(e);
  H->graph_exec.clear();
  H->graph_ran.clear();
}

// One Arnoldi step's launches (the Schur-block application, the matvec and the DCGS2 passes
// of basis slot j; no host synchronisation inside).  Its first run in a handle is eager; the
// next one is recorded as a HIP graph by stream capture and launched; later runs replay the
// graph.  The launches of slot j always take the same arguments (pointers into the handle's
// fixed storage, the slot index), so a replay performs exactly the work the stream would.
// Not used while the per-launch timer is on, with KKTDD_GRAPH=0, or on the NULL stream (which
// cannot be captured; kkt_solve_batched always runs on private streams).
template <typename F>
int run_step(kktdd_handle* H, int j, F&& work) {
  if (!graphs_enabled() || (t_prof && t_prof->on) || H->stream == nullptr) return work();
  if (H->graph_gen != tune_generation()) {
    release_graphs(H);   // launch shapes changed since the graphs were recorded
    H->graph_gen = tune_generation();
  }
  if ((int)H->graph_exec.size() <= j) {
    H->graph_exec.resize((size_t)j + 1, nullptr);
    H->graph_ran.resize((size_t)j + 1, 0);
  }
  hipStream_t s = H->stream;
  if (H->graph_exec[j]) {
    KKT_HIP(hipGraphLaunch(H->graph_exec[j], s));
    return 0;
  }
  if (!H->graph_ran[j]) {
    H->graph_ran[j] = 1;
    return work();
  }
  KKT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const int e = work();
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(s, &graph);
  if (e || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return e ? e : hip_fail(ce, "hipStreamEndCapture", __FILE__, __LINE__);
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate", __FILE__, __LINE__);
  H->graph_exec[j] = exec;
  KKT_HIP(hipGraphLaunch(exec, s));
  return 0;
}

int ensure_krylov(kktdd_handle* H, int R) {
  if (H->R >= R) return 0;
  release_graphs(H);
  const Geom& g = H->g;
  // free the previous basis
  auto release = [&](void* p) {
    if (!p) return;
    for (auto it = H->allocations.begin(); it != H->allocations.end(); ++it)
      if (*it == p) {
        (void)hipFree(p);
        H->allocations.erase(it);
        break;
      }
  };
  KKT_HIP(hipStreamSynchronize(H->stream));
  for (void* p : {(void*)H->V, (void*)H->Zw, (void*)H->kpart, (void*)H->ksums, (void*)H->hcol,
                  (void*)H->vinv, (void*)H->ydev, (void*)H->gate})
    release(p);
  H->V = H->Zw = H->kpart = H->ksums = H->hcol = H->vinv = H->ydev = nullptr;
  H->gate = nullptr;
  if (H->host_hcol) (void)hipHostFree(H->host_hcol);
  H->host_hcol = nullptr;
  H->R = 0;
  const KrylovSmall ks(R);
  size_t free_b = 0, total_b = 0;
  KKT_HIP(hipMemGetInfo(&free_b, &total_b));
  const size_t need = ((size_t)(R + 1) * (size_t)krylov_ld(g) + (size_t)R * (size_t)g.P) * 8 +
                      ks.device_bytes();
  if (need > free_b) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "Krylov basis for restart %d needs %zu bytes, %zu free", R, need, free_b);
    return set_error(KKTDD_ENOMEM, buf);
  }
  if (int e = dalloc(H, &H->V, (size_t)(R + 1) * (size_t)krylov_ld(g))) return e;
  if (int e = dalloc(H, &H->Zw, (size_t)R * g.P)) return e;
  if (int e = dalloc(H, &H->kpart, ks.part)) return e;
  if (int e = dalloc(H, &H->ksums, ks.sums)) return e;
  if (int e = dalloc(H, &H->hcol, ks.rec)) return e;
  if (int e = dalloc(H, &H->vinv, ks.vinv)) return e;
  if (int e = dalloc(H, &H->ydev, ks.ydev)) return e;
  if (int e = dalloc(H, &H->gate, 1)) return e;
  if (hipHostMalloc((void**)&H->host_hcol, ks.host * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    H->host_hcol = nullptr;
    return set_error(KKTDD_EHIP, "hipHostMalloc failed");
  }
  H->R = R;
  return 0;
}

}  // namespace

// ==========================================================================================
extern "C" {

int kkt_validate(const kktdd_problem* prob) { return validate(prob); }

int kkt_memory_plan(const kktdd_problem* prob, int32_t restart, size_t* bytes) {
  if (int e = validate(prob)) return e;
  if (!bytes || restart < 0) return set_error(KKTDD_EINVAL, "bad memory-plan arguments");
  const kktdd_problem rp = resolve(*prob);
  *bytes = plan(make_geom(rp), rp.precision, rp.sweep, restart).total();
  return KKTDD_OK;
}

int kkt_create(const kktdd_problem* prob_in, void* hip_stream, kktdd_handle** out) {
  const auto t_setup = std::chrono::steady_clock::now();
  if (!out) return set_error(KKTDD_EINVAL, "out is NULL");
  *out = nullptr;
  if (int e = validate(prob_in)) return e;
  const kktdd_problem resolved = resolve(*prob_in);
  const kktdd_problem* prob = &resolved;
  kktdd_handle* H = new (std::nothrow) kktdd_handle;
  if (!H) return set_error(KKTDD_ENOMEM, "host allocation failed");
  H->prob = *prob;
  H->g = make_geom(*prob);
  H->stream = static_cast<hipStream_t>(hip_stream);
  H->elem = prob->precision == KKTDD_FP64 ? 8 : 4;
  auto fail = [&](int code) {
    kkt_destroy(H);
    return code;
  };
  if (hipGetDevice(&H->device) != hipSuccess) {
    (void)hipGetLastError();
    delete H;
    return set_error(KKTDD_EHIP, "no HIP device");
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    delete H;
    return set_error(KKTDD_EHIP, "hipMemGetInfo failed");
  }
  const Geom& g = H->g;
  const Plan pl = plan(g, prob->precision, prob->sweep, 0);
  if (pl.total() > free_b) {
    delete H;
    char buf[160];
    std::snprintf(buf, sizeof buf, "problem needs %zu bytes, %zu free", pl.total(), free_b);
    return set_error(KKTDD_ENOMEM, buf);
  }
  // the allocation-free entry point's scratch array: its address on this device, once (after
  // the memory check, so that a refused problem loads nothing onto the device)
  if (int e = noalloc_setup(H->device)) {
    delete H;
    return e;
  }
  if (int e = build_tables(H)) return fail(e);
  const size_t MM = (size_t)g.padded();
  const size_t el = H->elem;
  if (prob->sweep == KKTDD_SWEEP_MODAL) {
    unsigned char *rh, *mt;
    if (int e = dalloc(H, &rh, (size_t)g.nt * MM * el)) return fail(e);
    if (int e = dalloc(H, &mt, (size_t)g.nt * MM * el)) return fail(e);
    H->Rhat = rh;
    H->Mtmp = mt;
    if (int e = dalloc(H, &H->Ysc, modal_store(g))) return fail(e);
    if (int e = dalloc(H, &H->ext, modal_ext(g))) return fail(e);
  } else {
    unsigned char *t, *u, *y;
    if (int e = dalloc(H, &t, (size_t)g.nd * MM * el)) return fail(e);
    if (int e = dalloc(H, &u, (size_t)g.nd * MM * el)) return fail(e);
    if (int e = dalloc(H, &y, (size_t)g.nd * g.L * MM * el)) return fail(e);
    H->Tbuf = t;
    H->Ubuf = u;
    H->Ybuf = y;
  }
  if (needs_rprime(g, prob->precision, prob->sweep)) {
    unsigned char* rp = nullptr;
    if (int e = dalloc(H, &rp, (size_t)g.P * el)) return fail(e);
    H->rprime = rp;
  }
  if (g.nb > 0) {
    if (physical_coarse(g, prob->precision, prob->sweep)) {
      if (int e = dalloc(H, &H->r0, (size_t)g.nc * g.nxy)) return fail(e);
      if (int e = dalloc(H, &H->c0, (size_t)g.nc * g.nxy)) return fail(e);
      if (int e = dalloc(H, &H->Dc0, (size_t)g.nc * g.nxy)) return fail(e);
      if (int e = dalloc(H, &H->DDc0, (size_t)g.nc * g.nxy)) return fail(e);
    }
    if (int e = dalloc(H, &H->chat, (size_t)g.nc * MM)) return fail(e);
    if (int e = dalloc(H, &H->ctmp, (size_t)g.nc * MM)) return fail(e);
    // padded sine-mode slices must start (and stay) zero outside the mode grid
    if (hipMemsetAsync(H->chat, 0, (size_t)g.nc * MM * 8, H->stream) != hipSuccess ||
        hipMemsetAsync(H->ctmp, 0, (size_t)g.nc * MM * 8, H->stream) != hipSuccess) {
      (void)hipGetLastError();
      return fail(set_error(KKTDD_EHIP, "hipMemsetAsync failed"));
    }
  }
  if (int e = dalloc(H, &H->partials, (size_t)kRedBlocks * kFieldSums)) return fail(e);
  if (int e = dalloc(H, &H->sums, 128)) return fail(e);
  if (hipHostMalloc((void**)&H->host_sums, 128 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    H->host_sums = nullptr;
    return fail(set_error(KKTDD_EHIP, "hipHostMalloc failed"));
  }
  if (int e = build_coarse(H)) return fail(e);
  if (int e = autotune(H)) return fail(e);
  if (hipStreamSynchronize(H->stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(set_error(KKTDD_EHIP, "setup failed"));
  }
  H->setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_setup).count();
  *out = H;
  return KKTDD_OK;
}

void kkt_destroy(kktdd_handle* H) {
  if (!H) return;
  (void)hipStreamSynchronize(H->stream);
  release_graphs(H);
  for (void* p : H->allocations) (void)hipFree(p);
  if (H->host_sums) (void)hipHostFree(H->host_sums);
  if (H->host_hcol) (void)hipHostFree(H->host_hcol);
  for (hipEvent_t e : H->prof.pool) (void)hipEventDestroy(e);
  delete H;
}

size_t kkt_size(const kktdd_handle* H) { return H ? (size_t)(3 * H->g.P) : 0; }

int kkt_precision(const kktdd_handle* H) { return H ? H->prob.precision : KKTDD_EINVAL; }

int kkt_tune_set(int32_t kind, int32_t precision, int32_t extent, int32_t nslices, int32_t waves,
                 int32_t deep, int32_t width) {
  return tune_set(kind, precision, extent, nslices, waves, deep, width);
}

int kkt_tune_get(int32_t kind, int32_t precision, int32_t extent, int32_t nslices, int32_t* waves,
                 int32_t* deep, int32_t* width) {
  return tune_get(kind, precision, extent, nslices, waves, deep, width);
}

double kkt_kappa(const kktdd_problem* prob) {
  if (!prob || validate(prob) != KKTDD_OK) return -1.0;
  return kappa_D(*prob);
}

int kkt_rhs(kktdd_handle* H, const double* u0, const double* utilde, double* f) {
  ProfScope ps(H);
  if (!H || !u0 || !utilde || !f) return set_error(KKTDD_EINVAL, "NULL argument");
  return launch_rhs(H->g, u0, utilde, f, H->stream);
}

int kkt_apply(kktdd_handle* H, const double* x, double* y) {
  ProfScope ps(H);
  if (!H || !x || !y) return set_error(KKTDD_EINVAL, "NULL argument");
  if (x == y) return set_error(KKTDD_EINVAL, "x and y must not alias");
  const Geom& g = H->g;
  return launch_kkt_apply(g, x, x + g.P, x + 2 * g.P, 1.0, 1.0, 1.0, nullptr, nullptr, y,
                          y + g.P, y + 2 * g.P, H->stream);
}

int precond_apply(kktdd_handle* H, const double* r, double* z) {
  ProfScope ps(H);
  RoctxScope rs("kktdd:precond_apply");
  if (!H || !r || !z) return set_error(KKTDD_EINVAL, "NULL argument");
  if (r == z) return set_error(KKTDD_EINVAL, "r and z must not alias");
  if (int e = poison_workspace(H)) return e;
  const Geom& g = H->g;
  if (int e = launch_scale(g.P, r, 1.0 / g.h, nullptr, z, H->stream)) return e;
  if (int e = launch_scale(g.P, r + g.P, 1.0 / (g.omega * g.h), nullptr, z + g.P, H->stream)) return e;
  return schur_apply(H, r + 2 * g.P, nullptr, z + 2 * g.P);
}

int kkt_spatial_solve(kktdd_handle* H, const double* b, double* x, int32_t nslices, double shift) {
  ProfScope ps(H);
  if (!H || !b || !x) return set_error(KKTDD_EINVAL, "NULL argument");
  if (nslices < 0 || !(shift > 0.0) || !std::isfinite(shift)) return set_error(KKTDD_EINVAL, "bad nslices or shift");
  if (nslices == 0) return KKTDD_OK;
  const Geom& g = H->g;
  const kktdd_problem& p = H->prob;
  const size_t MM = (size_t)g.padded();
  // eigenvalue table for this shift (this diagnostic entry point allocates and synchronises)
  const double dx = p.Lx / p.nx, dy = p.Ly / p.ny, dtnu = g.dt * p.nu;
  const double norm = 4.0 / ((double)p.nx * p.ny);
  std::vector<double> inv(MM, 0.0);
  for (int q = 0; q < g.my; ++q) {
    const double sy = std::sin(M_PI * (q + 1) / (2.0 * p.ny));
    for (int a = 0; a < g.mx; ++a) {
      const double sx = std::sin(M_PI * (a + 1) / (2.0 * p.nx));
      inv[(size_t)mode_pos(q, g.My) * g.Mx + mode_pos(a, g.Mx)] =
          norm / (shift + dtnu * 4.0 / (dx * dx) * sx * sx + dtnu * 4.0 / (dy * dy) * sy * sy);
    }
  }
  const size_t el = H->elem;
  void *tab = nullptr, *w1 = nullptr, *w2 = nullptr;
  int rc = 0;
  if (hipMalloc(&tab, MM * el) != hipSuccess || hipMalloc(&w1, (size_t)nslices * MM * el) != hipSuccess ||
      hipMalloc(&w2, (size_t)nslices * MM * el) != hipSuccess) {
    (void)hipGetLastError();
    rc = set_error(KKTDD_ENOMEM, "work allocation failed");
  }
  if (!rc) {
    hipError_t e;
    if (el == 4) {
      std::vector<float> f(inv.begin(), inv.end());
      e = hipMemcpyAsync(tab, f.data(), MM * 4, hipMemcpyHostToDevice, H->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(H->stream);
    } else {
      e = hipMemcpyAsync(tab, inv.data(), MM * 8, hipMemcpyHostToDevice, H->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(H->stream);
    }
    if (e != hipSuccess) rc = hip_fail(e, "table upload", __FILE__, __LINE__);
  }
  if (!rc) rc = launch_spatial_solve(g, p.precision, H->Sx(), H->Sy(), tab, b, x, nslices, w1, w2, H->stream);
  if (hipStreamSynchronize(H->stream) != hipSuccess && !rc) rc = set_error(KKTDD_EHIP, "spatial solve failed");
  if (tab) (void)hipFree(tab);
  if (w1) (void)hipFree(w1);
  if (w2) (void)hipFree(w2);
  return rc;
}

int fgmres_solve(kktdd_handle* H, const double* f, double* x, int32_t restart, int32_t maxit,
                 double rtol, kktdd_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  ProfScope ps(H);
  RoctxScope rs("kktdd:fgmres_solve");
  if (!H || !f || !x) return set_error(KKTDD_EINVAL, "NULL argument");
  if (f == x) return set_error(KKTDD_EINVAL, "f and x must not alias");
  H->history.clear();
  const bool dcgs = arnoldi_dcgs2();
  if (restart < 1 || restart > KKTDD_MAX_RESTART || maxit < 0 || !(rtol > 0.0))
    return set_error(KKTDD_EINVAL, "need 1 <= restart <= KKTDD_MAX_RESTART, maxit >= 0, rtol > 0");
  if (!dcgs && restart > kMaxCgsRestart)
    return set_error(KKTDD_EINVAL, "the CGS Arnoldi passes take restart <= 31");
  kktdd_stats st{};
  const Geom& g = H->g;
  hipStream_t s = H->stream;
  const long long n3 = 3 * g.P;
  const int nred = krylov_blocks(g);
  if (int e = ensure_krylov(H, restart)) return e;
  if (int e = poison_workspace(H)) return e;
  double fb[3];
  if (int e = field_sumsq(H, f, fb)) return e;
  const double fnorm = std::sqrt(fb[0] + fb[1] + fb[2]);
  auto finish = [&](int status, double est, const double rb[3]) {
    st.status = status;
    st.relres_est = est;
    const double rn = std::sqrt(rb[0] + rb[1] + rb[2]);
    st.relres_true = fnorm > 0 ? rn / fnorm : 0.0;
    for (int b = 0; b < 3; ++b) st.relres_block[b] = fb[b] > 0 ? std::sqrt(rb[b] / fb[b]) : 0.0;
    st.solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    st.setup_s = H->setup_s;
    if (stats) *stats = st;
    if (log_enabled()) {
      std::string line = "kktdd: fgmres_solve status " + std::to_string(status) + ", " +
                         std::to_string(st.iters) + " iterations, residual estimates";
      char buf[32];
      for (double v : H->history) {
        std::snprintf(buf, sizeof buf, " %.3e", v);
        line += buf;
      }
      std::snprintf(buf, sizeof buf, "; true %.3e\n", st.relres_true);
      line += buf;
      std::fputs(line.c_str(), stderr);
    }
    return status;
  };
  if (!(std::isfinite(fnorm))) {
    const double z[3] = {0, 0, 0};
    finish(KKTDD_EBREAKDOWN, NAN, z);
    return set_error(KKTDD_EBREAKDOWN, "non-finite right-hand side");
  }
  if (fnorm == 0.0) {
    KKT_HIP(hipMemsetAsync(x, 0, (size_t)n3 * 8, s));
    KKT_HIP(hipStreamSynchronize(s));
    const double z[3] = {0, 0, 0};
    return finish(KKTDD_OK, 0.0, z);
  }
  const double tol = rtol * fnorm;
  const int R = restart;
  const long long ldv = krylov_ld(g);
  double* V = H->V;
  double* Zw = H->Zw;
  double* part = H->kpart;
  // Hessenberg (R+1) x R row-major, Givens rotations, rotated right-hand side
  std::vector<double> Hm((size_t)(R + 1) * R), cs(R), sn(R), gv(R + 1), y(R), yv(R), yw(R);
  // DCGS2: alpha[j] and amat[i*(R+1)+j] = coefficients of the candidate of step j in the
  // final basis (candidate_j = alpha_j v_j + sum_{i<j} a_ij v_i)
  std::vector<double> alpha(R + 1), amat((size_t)(R + 1) * (R + 1));
  double est = INFINITY;
  int its = 0, cycles = 0;
  auto rotate_column = [&](int j) {
    for (int i = 0; i < j; ++i) {
      const double a = Hm[(size_t)i * R + j], b = Hm[(size_t)(i + 1) * R + j];
      Hm[(size_t)i * R + j] = cs[i] * a + sn[i] * b;
      Hm[(size_t)(i + 1) * R + j] = -sn[i] * a + cs[i] * b;
    }
    const double a = Hm[(size_t)j * R + j], b = Hm[(size_t)(j + 1) * R + j];
    const double rho = std::hypot(a, b);
    cs[j] = rho == 0.0 ? 1.0 : a / rho;
    sn[j] = rho == 0.0 ? 0.0 : b / rho;
    Hm[(size_t)j * R + j] = rho;
    Hm[(size_t)(j + 1) * R + j] = 0.0;
    gv[j + 1] = -sn[j] * gv[j];
    gv[j] = cs[j] * gv[j];
  };
  // provisional |g_{j+1}| if column j were cand (length j+2), without touching the state
  auto provisional = [&](int j, const std::vector<double>& cand) {
    std::vector<double> c(cand);
    for (int i = 0; i < j; ++i) {
      const double a = c[i], b = c[i + 1];
      c[i] = cs[i] * a + sn[i] * b;
      c[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double rho = std::hypot(c[j], c[j + 1]);
    return rho == 0.0 ? 0.0 : std::fabs(c[j + 1] / rho * gv[j]);
  };
  auto bad = [&](const char* what) {
    const double z3[3] = {NAN, NAN, NAN};
    st.iters = its;
    finish(KKTDD_EBREAKDOWN, est, z3);
    return set_error(KKTDD_EBREAKDOWN, what);
  };
  while (true) {
    // r = f - K x into V_0
    if (int e = launch_kkt_apply(g, x, x + g.P, x + 2 * g.P, 1.0, 1.0, 1.0, nullptr, f, V,
                                 V + g.P, V + 2 * g.P, s)) return e;
    double rb[3];
    if (int e = field_sumsq(H, V, rb)) return e;
    const double beta = std::sqrt(rb[0] + rb[1] + rb[2]);
    if (!std::isfinite(beta)) {
      finish(KKTDD_EBREAKDOWN, est, rb);
      return set_error(KKTDD_EBREAKDOWN, "non-finite residual");
    }
    if (beta <= tol) {
      st.iters = its;
      st.restarts = cycles > 0 ? cycles - 1 : 0;
      return finish(KKTDD_OK, cycles ? est : beta / fnorm, rb);
    }
    if (its >= maxit) {
      st.iters = its;
      st.restarts = cycles > 0 ? cycles - 1 : 0;
      return finish(KKTDD_NOT_CONVERGED, cycles ? est : beta / fnorm, rb);
    }
    ++cycles;
    H->host_sums[4] = 1.0 / beta;   // pinned staging slot
    KKT_HIP(hipMemcpyAsync(H->vinv, H->host_sums + 4, sizeof(double), hipMemcpyHostToDevice, s));
    std::fill(Hm.begin(), Hm.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int m = 0;   // columns of this cycle that enter the solution
    double* sums = H->ksums;
    double* norm_slot = H->ksums + 2 * R + 4;
    double* rec = H->hcol;
    const double* hrec = H->host_hcol;
    for (int j = 0; j < R; ++j) {
      double* vj = V + (long long)j * ldv;
      double* w = V + (long long)(j + 1) * ldv;
      double* zwj = Zw + (long long)j * g.P;
      // z_j = P^{-1} v_j: u and z blocks are v scaled (folded into the matvec), w block stored;
      // then w = K z_j
      auto front = [&]() -> int {
        if (int e = schur_apply(H, vj + 2 * g.P, H->vinv + j, zwj)) return e;
        return launch_kkt_apply(g, vj, vj + g.P, zwj, 1.0 / g.h, 1.0 / (g.omega * g.h), 1.0,
                                H->vinv + j, nullptr, w, w + g.P, w + 2 * g.P, s);
      };
      if (!dcgs) {
        if (int e = front()) return e;
        // ---- classical Gram-Schmidt with selective reorthogonalisation ------------------
        const int nv = j + 1;
        double* sums1 = H->ksums;
        double* sums2 = H->ksums + (R + 2);
        double* sums3 = H->ksums + 2 * (R + 2);
        if (int e = launch_multidot(n3, V, ldv, nv, H->vinv, w, 1, part, nred, s)) return e;
        if (int e = launch_reduce_partials(part, nred, nv + 1, sums1, s)) return e;
        if (int e = launch_arnoldi_finish(j, sums1, nullptr, nullptr, H->gate, H->hcol, H->vinv,
                                          kReorthEta, 1, s)) return e;
        if (int e = launch_update_dot(n3, V, ldv, nv, H->vinv, H->hcol + (j + 3), w, w, 1,
                                      part, nred, nullptr, s)) return e;
        if (int e = launch_reduce_partials(part, nred, nv + 1, sums2, s)) return e;
        if (int e = launch_arnoldi_finish(j, nullptr, sums2, nullptr, H->gate, H->hcol, H->vinv,
                                          kReorthEta, 2, s)) return e;
        const long long passC = prof_mark();
        if (int e = launch_update_dot(n3, V, ldv, nv, H->vinv, H->hcol + (j + 3), w, w, 0,
                                      part, nred, H->gate, s)) return e;
        if (int e = launch_reduce_partials(part, nred, 1, sums3, s)) return e;
        if (int e = launch_arnoldi_finish(j, nullptr, nullptr, sums3, H->gate, H->hcol,
                                          H->vinv, kReorthEta, 3, s)) return e;
        KKT_HIP(hipMemcpyAsync(H->host_hcol, H->hcol, (j + 3) * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        KKT_HIP(hipStreamSynchronize(s));
        const double* hc = H->host_hcol;
        if (hc[j + 2] != 0.0) {
          ++st.reorth;
          prof_add_bytes(passC, (double)(nv + 2) * n3 * 8.0);   // the gated pass ran
        }
        for (int i = 0; i <= j + 1; ++i) {
          if (!std::isfinite(hc[i])) return bad("non-finite Hessenberg entry");
          Hm[(size_t)i * R + j] = hc[i];
        }
        const double sub = Hm[(size_t)(j + 1) * R + j];
        rotate_column(j);
        alpha[j] = 1.0;
        for (int i = 0; i < j; ++i) amat[(size_t)i * (R + 1) + j] = 0.0;
        ++its;
        m = j + 1;
        est = std::fabs(gv[j + 1]) / fnorm;
        H->history.push_back(est);
        if (std::fabs(gv[j + 1]) <= tol || its >= maxit || sub == 0.0) break;
        continue;
      }
      // ---- DCGS2: slot j holds the candidate of v_j, slot j+1 the product W ---------------
      const int ns = 2 * j + 3;
      auto step_work = [&]() -> int {
        if (int e = front()) return e;
        if (int e = launch_dcgs_dots(n3, V, ldv, j, vj, w, part, nred, s)) return e;
        if (int e = launch_reduce_partials(part, nred, ns, sums, s)) return e;
        if (int e = launch_dcgs_finish(j, sums, H->vinv, H->ydev, rec, H->gate, 1, s)) return e;
        if (int e = launch_dcgs_update(n3, V, ldv, j, H->ydev, H->gate, part, nred, s)) return e;
        if (int e = launch_reduce_partials(part, nred, 1, norm_slot, s)) return e;
        return launch_dcgs_finish(j, norm_slot, H->vinv, H->ydev, rec, H->gate, 2, s);
      };
      if (int e = run_step(H, j, step_work)) return e;
      KKT_HIP(hipMemcpyAsync(H->host_hcol, rec, (2 * j + 5) * sizeof(double), hipMemcpyDeviceToHost, s));
      KKT_HIP(hipStreamSynchronize(s));
      for (int i = 0; i < 2 * j + 5; ++i)
        if (!std::isfinite(hrec[i])) return bad("non-finite Arnoldi coefficient");
      const double al = hrec[0], nu = hrec[1], hjj = hrec[2 * j + 2], nu1 = hrec[2 * j + 3];
      const bool brk = hrec[2 * j + 4] != 0.0;
      ++st.reorth;
      // close column j-1 with the reorthogonalisation of its candidate
      if (j == 0) {
        gv[0] = beta * al;
      } else {
        for (int i = 0; i < j; ++i) Hm[(size_t)i * R + (j - 1)] += nu * hrec[2 + i];
        Hm[(size_t)j * R + (j - 1)] = nu * al;
        rotate_column(j - 1);
        est = std::fabs(gv[j]) / fnorm;
        H->history.push_back(est);
      }
      alpha[j] = al;
      for (int i = 0; i < j; ++i) amat[(size_t)i * (R + 1) + j] = hrec[2 + i];
      if (brk || (j > 0 && std::fabs(gv[j]) <= tol)) {
        // the candidate lies in the span of v_0..v_{j-1}, or those columns already converged
        m = j;
        break;
      }
      // column j, projected once: b_i (i < j), hjj, and the norm of the next candidate
      for (int i = 0; i < j; ++i) Hm[(size_t)i * R + j] = hrec[2 + j + i];
      Hm[(size_t)j * R + j] = hjj;
      Hm[(size_t)(j + 1) * R + j] = nu1;
      ++its;
      std::vector<double> cand((size_t)j + 2);
      for (int i = 0; i <= j + 1; ++i) cand[i] = Hm[(size_t)i * R + j];
      const bool last = (j + 1 == R) || its >= maxit || nu1 == 0.0 || provisional(j, cand) <= tol;
      if (!last) continue;
      // close column j now: reorthogonalisation coefficients of the next candidate only
      if (nu1 > 0.0) {
        const int j1 = j + 1;
        if (int e = launch_dcgs_dots(n3, V, ldv, j1, w, nullptr, part, nred, s)) return e;
        if (int e = launch_reduce_partials(part, nred, 2 * j1 + 3, sums, s)) return e;
        if (int e = launch_dcgs_finish(j1, sums, H->vinv, H->ydev, rec, H->gate, 3, s)) return e;
        KKT_HIP(hipMemcpyAsync(H->host_hcol, rec, (2 * j1 + 5) * sizeof(double), hipMemcpyDeviceToHost, s));
        KKT_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < 2 + j1; ++i)
          if (!std::isfinite(hrec[i])) return bad("non-finite Arnoldi coefficient");
        for (int i = 0; i <= j; ++i) Hm[(size_t)i * R + j] += nu1 * hrec[2 + i];
        Hm[(size_t)(j + 1) * R + j] = nu1 * hrec[0];
      }
      rotate_column(j);
      est = std::fabs(gv[j + 1]) / fnorm;
      H->history.push_back(est);
      m = j + 1;
      break;
    }
    if (m == 0) return bad("Arnoldi breakdown on the first basis vector");
    // x += Z y with y from the rotated triangular system of the m closed columns
    for (int i = m - 1; i >= 0; --i) {
      double t = gv[i];
      for (int q = i + 1; q < m; ++q) t -= Hm[(size_t)i * R + q] * y[q];
      y[i] = t / Hm[(size_t)i * R + i];
    }
    // z_j's u and z blocks are its candidate alpha_j v_j + sum_{i<j} a_ij v_i, scaled
    for (int i = 0; i < m; ++i) {
      double c = y[i] * alpha[i];
      for (int q = i + 1; q < m; ++q) c += y[q] * amat[(size_t)i * (R + 1) + q];
      yv[i] = c;
      yw[i] = y[i];
    }
    if (m > 0) {
      double* stage = H->host_hcol + 2 * R + 8;   // pinned staging of yv, yw (2R doubles)
      double* ystage = H->ydev + 2 * R + 4;
      std::copy(yv.begin(), yv.begin() + m, stage);
      std::copy(yw.begin(), yw.begin() + m, stage + R);
      KKT_HIP(hipMemcpyAsync(ystage, stage, (size_t)(R + m) * sizeof(double), hipMemcpyHostToDevice, s));
      if (int e = launch_update_solution(g, V, ldv, Zw, g.P, m, ystage, ystage + R,
                                         H->vinv, 1.0 / g.h, 1.0 / (g.omega * g.h), x, s)) return e;
      KKT_HIP(hipStreamSynchronize(s));   // the staging buffer is reused by the next cycle
    }
  }
}

int kkt_solve_batched(int32_t n, kktdd_handle* const* hs, const double* const* f,
                      double* const* x, int32_t restart, int32_t maxit, double rtol,
                      kktdd_stats* stats) {
  if (n < 0 || (n > 0 && (!hs || !f || !x))) return set_error(KKTDD_EINVAL, "bad batch arguments");
  if (n == 0) return KKTDD_OK;
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !f[i] || !x[i]) return set_error(KKTDD_EINVAL, "NULL handle or vector in batch");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return set_error(KKTDD_EINVAL, "a handle appears twice in the batch");
  }
  // Every problem runs on a private stream of its own host thread, ordered after the work
  // already queued on its handle's stream and before anything queued there later.
  std::vector<hipStream_t> priv(n, nullptr), orig(n, nullptr);
  std::vector<hipEvent_t> ev(n, nullptr);
  int rc = KKTDD_OK;
  for (int i = 0; i < n && rc == KKTDD_OK; ++i) {
    orig[i] = hs[i]->stream;
    hipError_t e = hipStreamCreateWithFlags(&priv[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev[i], orig[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(priv[i], ev[i], 0);
    if (e != hipSuccess) rc = hip_fail(e, "batch stream setup", __FILE__, __LINE__);
  }
  std::vector<int> codes(n, KKTDD_OK);
  std::vector<std::string> msgs(n);
  if (rc == KKTDD_OK) {
    int device = 0;
    (void)hipGetDevice(&device);
    std::vector<std::thread> pool;
    pool.reserve(n);
    // Odd members start a little later, so that one problem's bandwidth-bound Arnoldi passes
    // tend to meet another's latency-bound sweeps rather than its own Arnoldi passes
    // (KKTDD_BATCH_STAGGER_US overrides; 0 starts every member at once).
    const char* stg = std::getenv("KKTDD_BATCH_STAGGER_US");
    const long stagger_us = stg ? std::atol(stg) : kBatchStaggerUs;
    for (int i = 0; i < n; ++i) {
      pool.emplace_back([&, i]() {
        if (stagger_us > 0 && (i & 1)) std::this_thread::sleep_for(std::chrono::microseconds(stagger_us));
        (void)hipSetDevice(device);
        hs[i]->stream = priv[i];
        codes[i] = fgmres_solve(hs[i], f[i], x[i], restart, maxit, rtol, stats ? stats + i : nullptr);
        if (codes[i] < 0) msgs[i] = g_last_error;
      });
    }
    for (auto& t : pool) t.join();
  }
  for (int i = 0; i < n; ++i) {
    if (priv[i]) {
      if (ev[i] && hipEventRecord(ev[i], priv[i]) == hipSuccess) (void)hipStreamWaitEvent(orig[i], ev[i], 0);
      (void)hipStreamSynchronize(priv[i]);
      (void)hipStreamDestroy(priv[i]);
    }
    if (ev[i]) (void)hipEventDestroy(ev[i]);
    hs[i]->stream = orig[i];
  }
  if (rc != KKTDD_OK) return rc;
  int worst = KKTDD_OK;
  for (int i = 0; i < n; ++i) {
    if (codes[i] < 0 && (worst >= 0 || codes[i] < worst)) {
      worst = codes[i];
      g_last_error = "problem " + std::to_string(i) + ": " + msgs[i];
    } else if (codes[i] == KKTDD_NOT_CONVERGED && worst == KKTDD_OK) {
      worst = KKTDD_NOT_CONVERGED;
    }
  }
  return worst;
}

int kkt_residual_history(const kktdd_handle* H, double* out, int32_t cap) {
  if (!H || cap < 0 || (cap > 0 && !out)) return set_error(KKTDD_EINVAL, "bad history arguments");
  const int n = (int)H->history.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = H->history[i];
  return n;
}

int kkt_profile(kktdd_handle* H, int enable) {
  if (!H) return set_error(KKTDD_EINVAL, "NULL handle");
  KKT_HIP(hipStreamSynchronize(H->stream));
  if (enable) {
    H->prof.recs.clear();
    H->prof.used = 0;
  }
  H->prof.on = enable != 0;
  return KKTDD_OK;
}

int kkt_profile_read(kktdd_handle* H, int kclass, double* ms, int64_t* launches, double* bytes,
                     double* flops) {
  if (!H || kclass < 0 || kclass >= KKTDD_K_COUNT) return set_error(KKTDD_EINVAL, "bad handle or class");
  KKT_HIP(hipStreamSynchronize(H->stream));
  double t = 0.0, b = 0.0, f = 0.0;
  int64_t n = 0;
  for (const Prof::Rec& r : H->prof.recs) {
    if (r.cls != kclass) continue;
    float e = 0.0f;
    KKT_HIP(hipEventElapsedTime(&e, H->prof.pool[r.ev], H->prof.pool[r.ev + 1]));
    t += e;
    b += r.bytes;
    f += r.flops;
    ++n;
  }
  if (ms) *ms = t;
  if (launches) *launches = n;
  if (bytes) *bytes = b;
  if (flops) *flops = f;
  return KKTDD_OK;
}

const char* kkt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
