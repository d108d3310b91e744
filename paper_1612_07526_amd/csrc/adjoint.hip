// Adjoint of the tridiagonal eigen-decomposition: gradients on (d, e) from
// gradients on (lambda, Q).
//
// For T = Q diag(lambda) Q^T with simple eigenvalues, first-order perturbation
// theory gives dL/dT = Q (diag(lbar) + F o (Q^T Qbar)) Q^T with
// F_ij = 1/(lambda_j - lambda_i) off the diagonal.  d_i enters T once, e_i
// twice (at (i, i+1) and (i+1, i)), so only the band of dL/dT is needed:
//   M' = diag(lbar) + F o (Q^T Qbar)   (FP64 MFMA product, F fused in the epilogue)
//   W  = Q M'                          (FP64 MFMA product)
//   dbar_i = sum_a W_ia Q_ia,  ebar_i = sum_a W_ia Q_{i+1,a} + W_{i+1,a} Q_ia.
#include <algorithm>

#include "gemm_generic.h"
#include "profile.h"

namespace phdc {

constexpr int64_t kAdjChunk = 8;  // problems per pass through the workspace

// One thread per row i of one problem; W may be null (eigenvalue-only loss:
// W = Q diag(lbar)).
__global__ void __launch_bounds__(256) k_band(int n, const double* __restrict__ Q, int64_t strideQ,
                                              const double* __restrict__ W, int64_t strideW,
                                              const double* __restrict__ lbar, int64_t strideL, double* dbar,
                                              double* ebar) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double* q = Q + (int64_t)b * strideQ;
  const double* w = W ? W + (int64_t)b * strideW : nullptr;
  const double* lb = lbar ? lbar + (int64_t)b * strideL : nullptr;
  double sd = 0.0, se = 0.0;
  const bool last = (i == n - 1);
  for (int a = 0; a < n; ++a) {
    const int64_t o = (int64_t)a * n;
    const double qi = q[i + o];
    const double qn = last ? 0.0 : q[i + 1 + o];
    if (w) {
      const double wi = w[i + o];
      const double wn = last ? 0.0 : w[i + 1 + o];
      sd += wi * qi;
      se += wi * qn + wn * qi;
    } else {
      const double l = lb ? lb[a] : 0.0;
      sd += l * qi * qi;
      se += 2.0 * l * qi * qn;
    }
  }
  dbar[(int64_t)b * n + i] = sd;
  if (!last) ebar[(int64_t)b * (n - 1) + i] = se;
}

}  // namespace phdc

using namespace phdc;

extern "C" {

int phdc_stedc_backward_workspace(int64_t n, int64_t batch, size_t* bytes) {
  if (n < 0) return -1;
  if (batch < 0) return -2;
  if (!bytes) return -3;
  const int64_t c = std::min<int64_t>(std::max<int64_t>(batch, 1), kAdjChunk);
  *bytes = 256 + (size_t)2 * c * n * n * 8;
  return 0;
}

int phdc_stedc_backward(int64_t n, int64_t batch, const double* lambda, const double* Q, const double* lambda_bar,
                        const double* Q_bar, double* d_bar, double* e_bar, void* work, size_t lwork, void* stream) {
  if (n < 0 || n > (1 << 20)) return -1;
  if (batch < 0) return -2;
  if (n == 0 || batch == 0) return 0;
  if (!lambda) return -3;
  if (!Q) return -4;
  if (!d_bar) return -7;
  if (n > 1 && !e_bar) return -8;
  if (!work) return -9;
  size_t need = 0;
  phdc_stedc_backward_workspace(n, batch, &need);
  if (lwork < need) return -10;
  hipStream_t s = (hipStream_t)stream;
  double* Mp = (double*)((char*)work + 256);
  const int64_t nn = n * n;
  for (int64_t b0 = 0; b0 < batch; b0 += kAdjChunk) {
    const int cb = (int)std::min<int64_t>(kAdjChunk, batch - b0);
    const double* Qb = Q + b0 * nn;
    const double* lb = lambda_bar ? lambda_bar + b0 * n : nullptr;
    double* W = nullptr;
    if (Q_bar) {
      ProfScope ps(PH_ADJ_GEMM, s);
      double* W_ = Mp + (int64_t)cb * nn;
      GemmArgs g1{Qb, Q_bar + b0 * nn, n, n, nn, nn, (int32_t)n, (int32_t)n, (int32_t)n, 0};
      gemm_f64_adjoint_f(g1, cb, Mp, n, nn, lambda + b0 * n, lb, n, s);
      GemmArgs g2{Qb, Mp, n, n, nn, nn, (int32_t)n, (int32_t)n, (int32_t)n, 0};
      gemm_f64(false, false, g2, cb, W_, n, nn, s);
      W = W_;
    }
    ProfScope pb(PH_ADJ_BAND, s);
    dim3 grid((unsigned)((n + 255) / 256), cb);
    hipLaunchKernelGGL(k_band, grid, dim3(256), 0, s, (int)n, Qb, nn, W, nn, lb, n, d_bar + b0 * n,
                       n > 1 ? e_bar + b0 * (n - 1) : e_bar);
  }
  return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
}

}  // extern "C"
