// General FP64 matrix product on the gfx950 matrix cores, column-major
// operands with optional transposition, a batch index in blockIdx.y and a
// fused epilogue.  Same tiling as the merge update: 128x128 output tile per
// 256-thread block, 4 waves of 4x4 v_mfma_f64_16x16x4 blocks, k-steps of 16
// through double-buffered LDS.
#include "gemm_generic.h"

namespace phdc {

typedef double d4g_t __attribute__((ext_vector_type(4)));

constexpr int QT = 128, QK = 16, QLD = QT + 4;
// An operand whose k index is contiguous in memory is staged k-contiguous in LDS
// ([row][k], row stride QK + 1) so each thread's eight consecutive k values
// land in consecutive LDS words; the other layout is staged [k][row].
constexpr int QKP = QK + 1;
constexpr int QBUF = (QT * QKP > QK * QLD) ? QT * QKP : QK * QLD;

template <bool KC>
__device__ inline int lds_at(int k, int r) {
  return KC ? r * QKP + k : k * QLD + r;
}

// TN = 128 or 64 output columns per tile (64 for a product of at most 512
// columns whose last 128-column tile would be at most half used, such as the
// 192 sample columns of the HSS compression: each wave then holds 64 x 32).
template <bool TA, bool TB, class Epi, int TN = QT>
__global__ void __launch_bounds__(256) k_gemm_f64(GemmArgs g, Epi epi) {
  __shared__ double As[2][QBUF];
  __shared__ double Bs[2][QBUF];
  constexpr bool AKC = TA;   // op(A)(i, k) = A[k + i lda]: k contiguous
  constexpr bool BKC = !TB;  // op(B)(k, j) = B[k + j ldb]: k contiguous
  constexpr int NB = TN / 32;  // 16-column MFMA blocks per wave
  constexpr int BE = TN / 16;  // B entries staged per thread per k-step
  const int bz = blockIdx.y;
  const double* A = g.A + (int64_t)bz * g.strideA;
  const double* B = g.B + (int64_t)bz * g.strideB;
  const int tmn = (g.m + QT - 1) / QT;
  const int mt = blockIdx.x % tmn, nt = blockIdx.x / tmn;
  const int i0 = mt * QT, j0 = nt * TN;
  const int t = threadIdx.x;
  double ra[8], rb[BE];

  auto gload = [&](int kt) {
    const int kb = kt * QK;
    if (!TA) {  // A(i,k) = A[i + k lda]: thread stages k = t/16, rows i0 + 8*(t%16) ..
      const int k = kb + (t >> 4), i = i0 + (t & 15) * 8;
      const double* src = A + (int64_t)k * g.lda + i;
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = (k < g.k && i + e < g.m) ? src[e] : 0.0;
    } else {    // op(A)(i,k) = A[k + i lda]: thread stages row i = t/2, k = kb + 8*(t%2) ..
      const int i = i0 + (t >> 1), k = kb + (t & 1) * 8;
      const double* src = A + (int64_t)i * g.lda + k;
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = (i < g.m && k + e < g.k) ? src[e] : 0.0;
    }
    if (!TB) {  // B(k,j) = B[k + j ldb]: thread stages column j = t / (16 / BE), BE consecutive k
      const int j = j0 + t / (QK / BE), k = kb + (t % (QK / BE)) * BE;
      const double* src = B + (int64_t)j * g.ldb + k;
#pragma unroll
      for (int e = 0; e < BE; ++e) rb[e] = (j < g.n && k + e < g.k) ? src[e] : 0.0;
    } else {    // op(B)(k,j) = B[j + k ldb]: thread stages k = t/16, BE consecutive j
      const int k = kb + (t >> 4), j = j0 + (t & 15) * BE;
      const double* src = B + (int64_t)k * g.ldb + j;
#pragma unroll
      for (int e = 0; e < BE; ++e) rb[e] = (k < g.k && j + e < g.n) ? src[e] : 0.0;
    }
  };
  auto lstore = [&](int buf) {
    if (!TA) {
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][lds_at<AKC>(t >> 4, (t & 15) * 8 + e)] = ra[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][lds_at<AKC>((t & 1) * 8 + e, t >> 1)] = ra[e];
    }
    if (!TB) {
#pragma unroll
      for (int e = 0; e < BE; ++e) Bs[buf][lds_at<BKC>((t % (QK / BE)) * BE + e, t / (QK / BE))] = rb[e];
    } else {
#pragma unroll
      for (int e = 0; e < BE; ++e) Bs[buf][lds_at<BKC>(t >> 4, (t & 15) * BE + e)] = rb[e];
    }
  };

  const int w = t >> 6, lane = t & 63;
  const int wm = (w & 1) * 64, wn = (w >> 1) * (TN / 2);
  const int li = lane & 15, lk = lane >> 4;
  d4g_t acc[4][NB];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = d4g_t{0.0, 0.0, 0.0, 0.0};

  const int nkt = (g.k + QK - 1) / QK;
  if (nkt > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nkt) gload(kt + 1);
#pragma unroll
    for (int ks = 0; ks < QK / 4; ++ks) {
      const int kr = ks * 4 + lk;
      double av[4], bv[NB];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[buf][lds_at<AKC>(kr, wm + i * 16 + li)];
#pragma unroll
      for (int j = 0; j < NB; ++j) bv[j] = Bs[buf][lds_at<BKC>(kr, wn + j * 16 + li)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nkt) lstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int cj = j0 + wn + j * 16 + li;
    if (cj >= g.n) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ri = i0 + wm + i * 16 + lk + 4 * r;  // element r of a lane sits at row lk + 4 r
        if (ri < g.m) epi(bz, ri, cj, acc[i][j][r]);
      }
  }
}

template <bool TA, bool TB, class Epi>
void launch_gemm(const GemmArgs& g, int batch, const Epi& epi, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || batch <= 0) return;
  const int tm = (g.m + QT - 1) / QT;
  const int rem = g.n % QT, tn = (g.n + QT - 1) / QT;
  if (rem > 0 && rem <= QT / 2 && tn <= 4) {  // a narrow product whose last column tile would be mostly empty
    dim3 grid(tm * ((g.n + QT / 2 - 1) / (QT / 2)), batch);
    hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi, QT / 2>), grid, dim3(256), 0, s, g, epi);
    return;
  }
  dim3 grid(tm * ((g.n + QT - 1) / QT), batch);
  hipLaunchKernelGGL((k_gemm_f64<TA, TB, Epi, QT>), grid, dim3(256), 0, s, g, epi);
}

// C = op(A) op(B), plain store.
void gemm_f64(bool ta, bool tb, const GemmArgs& g, int batch, double* C, int64_t ldc, int64_t strideC,
              hipStream_t s) {
  EpiStore e{C, ldc, strideC};
  if (!ta && !tb) launch_gemm<false, false>(g, batch, e, s);
  else if (ta && !tb) launch_gemm<true, false>(g, batch, e, s);
  else if (!ta && tb) launch_gemm<false, true>(g, batch, e, s);
  else launch_gemm<true, true>(g, batch, e, s);
}

// M' = diag(lbar) + F o (Q^T Qbar), F_ij = 1/(lambda_j - lambda_i) off the diagonal.
void gemm_f64_adjoint_f(const GemmArgs& g, int batch, double* C, int64_t ldc, int64_t strideC, const double* lam,
                        const double* lbar, int64_t strideL, hipStream_t s) {
  EpiAdjointF e{C, ldc, strideC, lam, lbar, strideL};
  launch_gemm<true, false>(g, batch, e, s);
}

}  // namespace phdc

namespace phdc {

int vgemm_tiles(int m, int n) {
  if (m <= 0 || n <= 0) return 0;
  return ((m + QT - 1) / QT) * ((n + QT - 1) / QT);
}

// Variable-size batch: the products are grouped by their transpositions, one
// launch per group compiled for it (the staging layout is then fixed at compile
// time, as in k_gemm_f64); every block finds its product by binary search in the
// tile prefix and computes one 128 x 128 tile of it.  alpha scales the staged A entries and beta C
// enters through the matrix cores, so the epilogue is a plain store (arithmetic
// there would pull all 64 accumulators into VGPRs at once).
template <bool TA, bool TB>
__device__ __forceinline__ void vgemm_tile(const VGemm& g, int tile, double (*As)[QBUF], double (*Bs)[QBUF]) {
  constexpr bool AKC = TA, BKC = !TB;  // operands with k contiguous in memory are staged [row][k]
  const int tmn = (g.m + QT - 1) / QT;
  const int i0 = (tile % tmn) * QT, j0 = (tile / tmn) * QT;
  const int t = threadIdx.x;
  double ra[8], rb[8];
  auto gload = [&](int kt) {
    const int kb = kt * QK;
    if (!TA) {
      const int k = kb + (t >> 4), i = i0 + (t & 15) * 8;
      const double* src = g.A + (int64_t)k * g.lda + i;
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = (k < g.k && i + e < g.m) ? src[e] : 0.0;
    } else {
      const int i = i0 + (t >> 1), k = kb + (t & 1) * 8;
      const double* src = g.A + (int64_t)i * g.lda + k;
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = (i < g.m && k + e < g.k) ? src[e] : 0.0;
    }
    if (!TB) {
      const int j = j0 + (t >> 1), k = kb + (t & 1) * 8;
      const double* src = g.B + (int64_t)j * g.ldb + k;
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = (j < g.n && k + e < g.k) ? src[e] : 0.0;
    } else {
      const int k = kb + (t >> 4), j = j0 + (t & 15) * 8;
      const double* src = g.B + (int64_t)k * g.ldb + j;
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = (k < g.k && j + e < g.n) ? src[e] : 0.0;
    }
    if (g.alpha != 1.0)
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] *= g.alpha;
  };
  auto lstore = [&](int buf) {
    if (!TA) {
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][lds_at<AKC>(t >> 4, (t & 15) * 8 + e)] = ra[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][lds_at<AKC>((t & 1) * 8 + e, t >> 1)] = ra[e];
    }
    if (!TB) {
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][lds_at<BKC>((t & 1) * 8 + e, t >> 1)] = rb[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][lds_at<BKC>(t >> 4, (t & 15) * 8 + e)] = rb[e];
    }
  };
  const int w = t >> 6, lane = t & 63;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
  const int li = lane & 15, lk = lane >> 4;
  d4g_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4g_t{0.0, 0.0, 0.0, 0.0};
  const int nkt = (g.k + QK - 1) / QK;
  if (nkt > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nkt) gload(kt + 1);
#pragma unroll
    for (int ks = 0; ks < QK / 4; ++ks) {
      const int kr = ks * 4 + lk;
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[buf][lds_at<AKC>(kr, wm + i * 16 + li)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[buf][lds_at<BKC>(kr, wn + j * 16 + li)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nkt) lstore(buf ^ 1);
    __syncthreads();
  }
  {
    // acc += beta C on the matrix cores: four more k-steps per 16 x 16 block with
    // A = the columns 4q..4q+3 of the identity and B = rows 4q..4q+3 of beta C,
    // so each entry gains beta C(i, j) in one rounding, as acc + beta C would.
    // (Run for beta == 0 too, adding zeros: a branch around these steps makes the
    // compiler move the accumulators out of their registers.)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cj = j0 + wn + j * 16 + li;
      const double* col = (cj < g.n) ? g.C + (int64_t)(g.cmap ? g.cmap[cj] : cj) * g.ldc : nullptr;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ri = i0 + wm + i * 16 + 4 * q + lk;
          const double bq = (g.beta != 0.0 && col && ri < g.m) ? g.beta * col[ri] : 0.0;
          const double aq = (li == 4 * q + lk) ? 1.0 : 0.0;
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq, bq, acc[i][j], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int cj = j0 + wn + j * 16 + li;
    if (cj >= g.n) continue;
    double* col = g.C + (int64_t)(g.cmap ? g.cmap[cj] : cj) * g.ldc;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ri = i0 + wm + i * 16 + lk + 4 * r;
        if (ri < g.m) col[ri] = acc[i][j][r];
      }
  }
}

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_vgemm(const VGemm* __restrict__ descs, const int32_t* __restrict__ pfx,
                                               int nd, int base) {
  __shared__ double As[2][QBUF];
  __shared__ double Bs[2][QBUF];
  const int bid = base + blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pfx[mid] <= bid) lo = mid; else hi = mid - 1;
  }
  const VGemm g = descs[lo];
  vgemm_tile<TA, TB>(g, bid - pfx[lo], As, Bs);
}

void vgemm_launch(const VGemm* descs, const int32_t* pfx, int nd, const int* bound, hipStream_t s) {
  if (nd <= 0) return;
  for (int q = 0; q < 4; ++q) {
    const int nb = bound[q + 1] - bound[q];
    if (nb <= 0) continue;
    if (q == 0) hipLaunchKernelGGL((k_vgemm<false, false>), dim3(nb), dim3(256), 0, s, descs, pfx, nd, bound[q]);
    else if (q == 1) hipLaunchKernelGGL((k_vgemm<true, false>), dim3(nb), dim3(256), 0, s, descs, pfx, nd, bound[q]);
    else if (q == 2) hipLaunchKernelGGL((k_vgemm<false, true>), dim3(nb), dim3(256), 0, s, descs, pfx, nd, bound[q]);
    else hipLaunchKernelGGL((k_vgemm<true, true>), dim3(nb), dim3(256), 0, s, descs, pfx, nd, bound[q]);
  }
}

}  // namespace phdc
