// kkt_spatial_solve_noalloc: the Dirichlet spatial solve of kkt_spatial_solve with no device
// allocation at call time.
//
// Its eigenvalue table and the two padded work stacks live in one file-scope device array,
// `scratch`, of kScratchBytes per device.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol): kkt_create resolves the array's device
// address once per device with hipGetSymbolAddress, with that device current, and every
// launch takes that address.  All calls on one device share the array, so calls that overlap
// in time on one device (other streams, other threads) race; a call leaves its data there.
#include <cmath>
#include <cstdio>
#include <mutex>

#include "internal.h"

namespace kktdd {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Inverse eigenvalues of shift*I + dt*nu*A_h in the folded mode order, times the inverse-
// transform normalisation: position (row, col) of the padded grid holds mode (q, a) =
// (mode_at(row), mode_at(col)), norm / ((shift + lamx[a]) + lamy[q]), and zero at padding.
// The sum is taken in the same order as the host table of kkt_spatial_solve, so both tables
// hold the same values.
__global__ void k_invlam_table(Geom g, const double* __restrict__ lamx, const double* __restrict__ lamy,
                               double shift, double norm, int f32, void* out) {
  const long long MM = g.padded();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MM) return;
  const int row = (int)(i / g.Mx), col = (int)(i - (long long)row * g.Mx);
  const int q = mode_at(row, g.My), a = mode_at(col, g.Mx);
  double v = 0.0;
  if (q < g.my && a < g.mx) v = norm / ((shift + lamx[a]) + lamy[q]);
  if (f32)
    static_cast<float*>(out)[i] = (float)v;
  else
    static_cast<double*>(out)[i] = v;
}

}  // namespace

// Called by kkt_create with `device` current.
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return set_error(KKTDD_EHIP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return 0;
  void* p = nullptr;
  KKT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return set_error(KKTDD_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_dev[device] = p;
  return 0;
}

}  // namespace kktdd

using namespace kktdd;

extern "C" int kkt_spatial_solve_noalloc(kktdd_handle* H, const double* b, double* x, int32_t nslices,
                                         double shift) {
  if (!H || !b || !x) return set_error(KKTDD_EINVAL, "NULL argument");
  if (nslices < 0 || !(shift > 0.0) || !std::isfinite(shift)) return set_error(KKTDD_EINVAL, "bad nslices or shift");
  if (nslices == 0) return KKTDD_OK;
  const Geom& g = H->g;
  const size_t MM = (size_t)g.padded(), el = (size_t)H->elem;
  const size_t tab = round256(MM * el), work = round256((size_t)nslices * MM * el);
  if (tab + 2 * work > kScratchBytes) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "kkt_spatial_solve_noalloc: %d slices need %zu bytes of the %zu-byte scratch array "
                  "(at most %zu slices of this grid)", nslices, tab + 2 * work, kScratchBytes,
                  (kScratchBytes - tab) / 2 / (MM * el));
    return set_error(KKTDD_EINVAL, buf);
  }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (H->device >= 0 && H->device < kMaxDevices) base = g_scratch_dev[H->device];
  }
  if (!base) return set_error(KKTDD_EHIP, "scratch array not set up for this device");
  unsigned char* p = static_cast<unsigned char*>(base);
  void* table = p;
  void* w1 = p + tab;
  void* w2 = p + tab + work;
  const kktdd_problem& pr = H->prob;
  const double norm = 4.0 / ((double)pr.nx * pr.ny);
  const int threads = 256;
  const long long blocks = ((long long)MM + threads - 1) / threads;
  hipLaunchKernelGGL(k_invlam_table, dim3((unsigned)blocks), dim3(threads), 0, H->stream, g, H->lamx,
                     H->lamy, shift, norm, el == 4 ? 1 : 0, table);
  KKT_HIP(hipGetLastError());
  return launch_spatial_solve(g, pr.precision, H->Sx(), H->Sy(), table, b, x, nslices, w1, w2, H->stream);
}
