// phdc_stedc_noalloc: phdc_stedc with its workspace in a static device array,
// for callers that cannot allocate device memory.
//
// The array `scratch` below is a file-scope device variable: each GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code the name is only a stand-in for the device symbol, never
// an address: the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept in g_scratch.
#include <cstring>
#include <mutex>

#include "phdc_internal.h"

namespace phdc {

static __device__ __align__(256) char scratch[PHDC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (nullptr on failure).
void* scratch_for_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return nullptr;
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

__global__ void k_copy_status(const int32_t* __restrict__ status, int32_t* info) { *info = *status; }

}  // namespace
}  // namespace phdc

using namespace phdc;

extern "C" int phdc_stedc_noalloc(int64_t n, const double* d, const double* e, double* lambda, double* Q,
                                  int64_t ldq, int32_t* info, const phdc_opts* o, void* stream) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (n < 0 || n > ((int64_t)1 << 30)) return -1;
  if (n > 0 && !d) return -2;
  if (n > 1 && !e) return -3;
  if (n > 0 && !lambda) return -4;
  if (n > 0 && !Q) return -5;
  if (ldq < std::max<int64_t>(1, n)) return -6;
  if (!info) return -7;
  if (o->gemm_mode == PHDC_GEMM_HSS) return -8;  // the HSS path uses pinned host memory
  size_t need = 0;
  const int rc = phdc_stedc_workspace(n, o, &need);  // (argument check)
  if (rc != 0) return rc == -2 ? -8 : -1;
  need = stedc_workspace_bytes(n, o, false);  // this path takes no zero fill, hence no third buffer
  if (need > PHDC_NOALLOC_SCRATCH_BYTES) return -1;  // too large for the static workspace
  void* work = scratch_for_current_device();
  if (!work) return PHDC_E_HIP;
  hipStream_t s = (hipStream_t)stream;
  const int r = stedc_impl(n, d, e, lambda, Q, ldq, work, PHDC_NOALLOC_SCRATCH_BYTES, o, s, true);
  if (r == PHDC_E_HIP) return r;
  // the status word of this call (also after an argument error found by the
  // check_finite scan, which sets it)
  hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(1), 0, s, (const int32_t*)work, info);
  if (hipGetLastError() != hipSuccess) return PHDC_E_HIP;
  return r;
}
