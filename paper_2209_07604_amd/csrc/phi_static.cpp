// phi_power_iteration_static: the power method of phi_power_iteration with
// its scratch image in a fixed device array instead of a caller buffer, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid it).
//
// The array below is the scratch: every GPU the library runs on holds its own
// copy (kStaticScratchBytes) from module load until the process ends.  Host
// code never passes the array's name to a kernel or a copy (in host code that
// name is a host-side stand-in, not a device address): the device address is
// taken once per device with hipGetSymbolAddress, with that device current,
// and kept here.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "phi.h"
#include "phi_plan.h"

namespace {

constexpr size_t kStaticScratchBytes = (size_t)32 << 20;  // 32 MiB: L Ny Nx <= 8 Mi pixels
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

// Device address of this device's scratch array (looked up once per device).
phi_status scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PHI_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return PHI_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PHI_ERR_HIP;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return PHI_OK;
}

}  // namespace

extern "C" {

phi_status phi_power_iteration_static(phi_plan p, float* d_x, int32_t n_iter, double* d_nu, void* stream) {
  if (!p || !d_x || !d_nu) return PHI_ERR_ARG;
  if ((size_t)p->L * p->Ny * p->Nx * sizeof(float) > kStaticScratchBytes) return PHI_ERR_UNSUPPORTED;
  void* tmp = nullptr;
  const phi_status st = scratch_ptr(&tmp);
  if (st != PHI_OK) return st;
  return power_iteration_impl(p, d_x, static_cast<float*>(tmp), n_iter, d_nu, stream);
}

}  // extern "C"
