// Small utility kernels: status reset and the eigenvector sign convention;
// the library's auxiliary streams.
#include <algorithm>
#include <mutex>

#include "phdc_internal.h"

namespace phdc {

// One non-blocking stream per device, created on first use at the default
// priority, for work that runs beside the caller's stream between an event
// fork and join.  nullptr if it cannot be created (the caller then runs the
// work on its own stream).
hipStream_t aux_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
    streams[dev] = nullptr;
    (void)hipGetLastError();
  }
  return streams[dev];
}


// Zero the 256-byte status block with a kernel (not a memset node), so the
// call sequence stays safe to capture in a HIP graph.
__global__ void k_clear_status(int32_t* status) { status[threadIdx.x] = 0; }

void launch_clear_status(int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, status);
}

// Grid-stride scan for NaN or Inf; any lane that finds one raises the flag and
// the status word (first failure wins).  Race-free: both are only ever set.
__global__ void __launch_bounds__(256) k_scan_finite(const double* __restrict__ a, int64_t n, int32_t* flag,
                                                     int32_t* status) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) bad |= !isfinite(a[i]);
  if (__ballot(bad) != 0ULL && (threadIdx.x & 63) == 0) {
    atomicOr(flag, 1);
    set_status(status, PHDC_ERR_NONFINITE);
  }
}

void launch_scan_finite(const double* a, int64_t n, int32_t* flag, int32_t* status, hipStream_t s) {
  if (n <= 0 || a == nullptr) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_scan_finite, dim3((unsigned)blocks), dim3(256), 0, s, a, n, flag, status);
}

// Eigenvectors are defined up to sign; this fixes it: in every column the entry
// of largest magnitude (lowest row on ties) is made positive.  One block per
// column, columns of all matrices of a batch in one launch.
__global__ void __launch_bounds__(256) k_canonical_sign(const CanonDesc* __restrict__ descs,
                                                       const int32_t* __restrict__ pfx, int nmat) {
  __shared__ double sv[4];
  __shared__ int si[4];
  const int b = blockIdx.x;
  int lo = 0, hi = nmat - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pfx[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const CanonDesc D = descs[lo];
  const int col = b - pfx[lo];
  double* q = D.q + (int64_t)col * D.ld;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int r = threadIdx.x; r < D.n; r += 256) {
    double a = fabs(q[r]);
    if (a > best) { best = a; bi = r; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    double ob = __shfl_xor(best, o, 64);
    int oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sv[w] = best; si[w] = bi; }
  __syncthreads();
  best = sv[0];
  bi = si[0];
  for (int i = 1; i < 4; ++i)
    if (sv[i] > best || (sv[i] == best && si[i] < bi)) { best = sv[i]; bi = si[i]; }
  if (bi >= D.n) return;
  if (q[bi] < 0.0) {
    __syncthreads();
    for (int r = threadIdx.x; r < D.n; r += 256) q[r] = -q[r];
  }
}

void launch_canonical_sign(const void* descs, const int32_t* pfx, int nmat, int total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_canonical_sign, dim3(total), dim3(256), 0, s, (const CanonDesc*)descs, pfx, nmat);
}

}  // namespace phdc
