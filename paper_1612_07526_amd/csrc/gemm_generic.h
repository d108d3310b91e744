// Generic FP64 MFMA product (gemm_generic.hip) and its fused epilogues.
#pragma once
#include "phdc_internal.h"

namespace phdc {

// op(A) is m x k, op(B) is k x n; all column-major; batch b uses A + b strideA, B + b strideB.
struct GemmArgs {
  const double* A;
  const double* B;
  int64_t lda, ldb, strideA, strideB;
  int32_t m, n, k;
  int32_t pad;
};

struct EpiStore {
  double* C;
  int64_t ldc, strideC;
  __device__ void operator()(int b, int i, int j, double v) const { C[(int64_t)b * strideC + i + (int64_t)j * ldc] = v; }
};

struct EpiAdjointF {
  double* C;
  int64_t ldc, strideC;
  const double* lam;
  const double* lbar;
  int64_t strideL;
  __device__ void operator()(int b, int i, int j, double v) const {
    const double* l = lam + (int64_t)b * strideL;
    double r;
    if (i == j) r = lbar ? lbar[(int64_t)b * strideL + i] : 0.0;
    else r = v / (l[j] - l[i]);
    C[(int64_t)b * strideC + i + (int64_t)j * ldc] = r;
  }
};

void gemm_f64(bool ta, bool tb, const GemmArgs& g, int batch, double* C, int64_t ldc, int64_t strideC,
              hipStream_t s);
void gemm_f64_adjoint_f(const GemmArgs& g, int batch, double* C, int64_t ldc, int64_t strideC, const double* lam,
                        const double* lbar, int64_t strideL, hipStream_t s);

}  // namespace phdc

namespace phdc {

// One product of a variable-size batch: C = alpha op(A) op(B) + beta C (column-major).
// If cmap is set, column j of C lives at C + cmap[j] * ldc.
struct VGemm {
  const double* A;
  const double* B;
  double* C;
  const int32_t* cmap;
  int64_t lda, ldb, ldc;
  double alpha, beta;
  int32_t m, n, k;
  int32_t ta, tb;
  int32_t pad;
};

// Launch a batch of products described by `descs` (device) with tile prefix
// `pfx` (device, nd + 1 entries, pfx[nd] == total tiles of 128 x 128).  The
// products are ordered by transposition group q = ta + 2 tb, whose tiles are
// [bound[q], bound[q + 1]) (host array of 5).
void vgemm_launch(const VGemm* descs, const int32_t* pfx, int nd, const int* bound, hipStream_t s);
int vgemm_tiles(int m, int n);

}  // namespace phdc
