// Allocation-free kernel product: krr_kernel_matmat with its scratch space in a file-scope
// device array instead of a caller workspace, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/krr.h"
#include "kernels.hpp"

namespace {

// One copy per GPU, held from module load until the process ends. Host code never passes
// this name to a kernel or a copy: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress below, once per device.
static __device__ __align__(256) unsigned char scratch[KRR_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first call there).
hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

krr_status krr_kernel_matmat_noalloc(const float* X1, int64_t n1, int64_t ldx1, const float* X2,
                                     int64_t n2, int64_t ldx2, int64_t d, double sigma,
                                     double shift, const double* V, int64_t m, int64_t ldv,
                                     double* OUT, int64_t ldo, int32_t deriv, int32_t prec,
                                     void* stream) {
  const size_t need = krr_workspace_bytes(KRR_OP_KERNEL_MATMAT, n1, n2, d, 0, m, prec);
  if (need > (size_t)KRR_NOALLOC_SCRATCH_BYTES) {
    char msg[256];
    snprintf(msg, sizeof(msg),
             "krr_kernel_matmat_noalloc: needs %zu bytes of scratch, the fixed maximum is %zu "
             "(use krr_kernel_matmat with a workspace)",
             need, (size_t)KRR_NOALLOC_SCRATCH_BYTES);
    return krr::report_error(KRR_E_WORKSPACE, msg);
  }
  if (!X1 || !X2 || !V || !OUT || n1 < 1 || n2 < 1 || d < 1 || m < 1)  // argument errors first
    return krr_kernel_matmat(X1, n1, ldx1, X2, n2, ldx2, d, sigma, shift, V, m, ldv, OUT, ldo,
                             deriv, prec, nullptr, 0, stream);
  void* ws = nullptr;
  const hipError_t e = scratch_ptr(&ws);
  if (e != hipSuccess) {
    char msg[256];
    snprintf(msg, sizeof(msg), "krr_kernel_matmat_noalloc: scratch address: %s",
             hipGetErrorString(e));
    return krr::report_error(KRR_E_HIP, msg);
  }
  return krr_kernel_matmat(X1, n1, ldx1, X2, n2, ldx2, d, sigma, shift, V, m, ldv, OUT, ldo,
                           deriv, prec, ws, (size_t)KRR_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
