// y = A x with no device allocation: the staging buffers of oras_apply_A live
// in a fixed device array instead of context memory, for callers that cannot
// allocate (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).
//
// The array is a file-scope __device__ variable, so every GPU the library is
// loaded on holds its own copy until the process ends.  Its name is only a
// host-side handle: host code uses the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device when a context is created there.  Every call on a device shares that
// device's copy and leaves its last contents; each call overwrites all of the
// staging it reads before reading it, and calls that overlap on one device
// race.
#include <mutex>

#include "oras_internal.h"

namespace {

constexpr size_t NOALLOC_BYTES = size_t(64) << 20;   // 64 MiB per device
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};

}  // namespace

namespace oras {

oras_status noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return ORAS_E_HIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return ORAS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    g_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    return ORAS_E_HIP;
  }
  g_ptr[device] = p;
  return ORAS_OK;
}

}  // namespace oras

extern "C" size_t oras_noalloc_scratch_bytes(void) { return NOALLOC_BYTES; }

extern "C" oras_status oras_apply_A_noalloc(oras_ctx c, const void* x_dev, void* y_dev, int nrhs,
                                            int prec) {
  const oras_status st = oras::check_apply_A(c, x_dev, y_dev, nrhs, prec);
  if (st != ORAS_OK) return st;
  const size_t need = oras::apply_A_scratch_bytes(c, nrhs, prec);
  if (need > NOALLOC_BYTES) {
    const std::string msg = "apply_A_noalloc needs " + std::to_string(need) +
                            " bytes of staging, above the fixed " +
                            std::to_string(NOALLOC_BYTES) + " (n * pad8(nrhs) too large)";
    return oras::set_error(c, ORAS_E_ARG, msg.c_str());
  }
  const int dev = oras::ctx_device(c);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (dev >= 0 && dev < MAX_DEVICES) base = g_ptr[dev];
  }
  if (!base) return oras::set_error(c, ORAS_E_HIP, "no-alloc scratch address unavailable on this device");
  const size_t ns = need / (2 * sizeof(double2) + (prec == ORAS_C64 ? sizeof(float2) : 0));
  char* p = static_cast<char*>(base);
  double2* xin = reinterpret_cast<double2*>(p);
  double2* yout = reinterpret_cast<double2*>(p + ns * sizeof(double2));
  float2* x32 = prec == ORAS_C64 ? reinterpret_cast<float2*>(p + 2 * ns * sizeof(double2)) : nullptr;
  return oras::apply_A_staged(c, x_dev, y_dev, nrhs, prec, xin, yout, x32);
}
