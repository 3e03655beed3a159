// Allocation-free variant of the step's vector--Jacobian product, for
// callers that cannot allocate device memory at call time (code under HIP
// graph capture, serving loops, harnesses that forbid hipMalloc).
//
// nsc_step_vjp allocates its four state-sized adjoint workspaces on its
// first call.  nsc_step_vjp_noalloc runs the same kernels in the same order
// with those workspaces in a file-scope device array of kNoallocBytes,
// which every context on a device shares: calls that overlap on one device
// race on it.  The host never uses the array's name as an address: nsc_init
// records, once per device and with that device current, the address
// hipGetSymbolAddress returns for it, and only that address reaches the
// kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nsc_internal.h"

namespace nsc {
namespace {

constexpr size_t kNoallocBytes = (size_t)128 << 20;  // four FP64 states of up to 32 MiB each
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoallocBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {nullptr};
bool g_tried[kMaxDevices] = {false};

}  // namespace

void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_tried[device]) return;
  g_tried[device] = true;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_ptr[device] = p;
  else (void)hipGetLastError();  // leave no sticky error behind; the entry point reports it
}

}  // namespace nsc

extern "C" int nsc_step_vjp_noalloc(nsc_ctx *c, const double *u, const double *stages,
                                    const double *ubar_next, double *ubar) {
  int st = nsc::step_vjp_check(c, u, stages, ubar_next, ubar);
  if (st != NSC_OK) return st;
  const size_t need = (size_t)4 * c->d.f * c->d.nr * c->d.nmodes * 2 * sizeof(double);
  if (need > nsc::kNoallocBytes) return NSC_ERR_ARG;
  if (c->device < 0 || c->device >= nsc::kMaxDevices) return NSC_ERR_DEVICE;
  void *p;
  {
    std::lock_guard<std::mutex> lock(nsc::g_mu);
    p = nsc::g_ptr[c->device];
  }
  if (!p) return NSC_ERR_DEVICE;
  return nsc::step_vjp_impl(c, u, stages, ubar_next, ubar, static_cast<double *>(p));
}
