// Eigenvector update of a merge (Eq. (6)) on the FP64 matrix cores.
//
// With Gu's grouping (Sec. 1) the product [Q G P](:, survivors) * Uhat splits
// into two dense products that skip the structural zeros:
//   U(rows of Q1, :) = Q(rows of Q1, cols of parts 1,2) * Uhat(grouped rows 0 .. k1+k2)
//   U(rows of Q2, :) = Q(rows of Q2, cols of parts 2,3) * Uhat(grouped rows k1 .. K)
// The A operand is gathered column by column straight from the merge's input
// block (no packed copy), Uhat is row-major, and column j of the result is
// written to its final (sorted) output column dest[j].
//
// Tiling for gfx950: 256 threads (4 waves) per 128x128 output tile, each wave a
// 64x64 quadrant made of 4x4 v_mfma_f64_16x16x4 blocks; k-steps of 16 staged
// through double-buffered LDS.
#include "phdc_internal.h"

namespace phdc {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int GT = 128;       // output tile edge
constexpr int GK = 16;        // k per LDS stage
constexpr int GPAD = 4;       // LDS row padding (doubles)
constexpr int GLD = GT + GPAD;

__global__ void __launch_bounds__(256) k_merge_gemm(BlockMap bm, Scratch S) {
  __shared__ double As[2][GK][GLD];
  __shared__ double Bs[2][GK][GLD];
  const int b = blockIdx.x;
  const int mi = find_merge(bm, b);
  const int lb = b - bm.pfx[mi];
  const MergeDesc M = bm.descs[mi];
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  if (cnt[C_PATH] != 0) return;  // formed by another update path
  const int K = cnt[C_K], k1 = cnt[C_K1], k2 = cnt[C_K2], k3 = cnt[C_K3];
  const int n1 = M.n1, n2 = M.m - M.n1;
  const int tmt = (n1 + GT - 1) / GT, tmb = (n2 + GT - 1) / GT;
  const int TM = tmt + tmb;
  const int mt = lb % TM, nt = lb / TM;
  if (nt * GT >= K) return;
  const bool top = mt < tmt;
  const int mrow0 = top ? mt * GT : (mt - tmt) * GT;  // first row of the tile within its half
  const int Mrows = top ? n1 : n2;
  const int rowoff = top ? 0 : n1;                    // half's first row within the merge block
  const int kd = top ? k1 + k2 : k2 + k3;
  const int64_t so = M.s_off;
  const int32_t* colA = top ? S.coltop + so : S.colbot + so;
  const double* Bm = S.uhat + M.u_off + (int64_t)(top ? 0 : k1) * K;  // row-major, ld = K
  const double* A = M.qin + rowoff;
  const int64_t lda = M.ldin;
  const int ncol0 = nt * GT;

  const int t = threadIdx.x;
  const int lkc = t >> 4;          // k index this thread stages (A column / B row)
  const int l8 = (t & 15) * 8;     // first of 8 consecutive rows (A) / columns (B)
  double ra[8], rb[8];

  auto gload = [&](int kt) {
    const int kk = kt * GK + lkc;
    if (kk < kd) {
      const double* src = A + (int64_t)colA[kk] * lda + mrow0 + l8;
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = (mrow0 + l8 + e < Mrows) ? src[e] : 0.0;
      const double* bs = Bm + (int64_t)kk * K + ncol0 + l8;
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = (ncol0 + l8 + e < K) ? bs[e] : 0.0;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) { ra[e] = 0.0; rb[e] = 0.0; }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[buf][lkc][l8 + e] = ra[e];
      Bs[buf][lkc][l8 + e] = rb[e];
    }
  };

  const int w = t >> 6, lane = t & 63;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
  const int li = lane & 15, lk = lane >> 4;
  d4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int nkt = (kd + GK - 1) / GK;
  if (nkt > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nkt) gload(kt + 1);
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      const int kr = ks * 4 + lk;
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[buf][kr][wm + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[buf][kr][wn + j * 16 + li];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nkt) lstore(buf ^ 1);
    __syncthreads();
  }

  // Epilogue: v_mfma_f64_16x16x4 leaves element r of lane (li, lk) of block
  // (i, j) at row lk + 4 r, column li (rows interleaved across lane groups).
  const int32_t* dest = S.dest + so;
  double* out = M.qout + rowoff;
  const int64_t ldo = M.ldout;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int cj = ncol0 + wn + j * 16 + li;
    if (cj >= K) continue;
    double* oc = out + (int64_t)dest[cj] * ldo;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mrow0 + wm + i * 16 + lk + 4 * r;
        if (row < Mrows) oc[row] = acc[i][j][r];
      }
    }
  }
}

void launch_merge_gemm_f64(const BlockMap& bm, int total, const Scratch& S, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_merge_gemm, dim3(total), dim3(256), 0, s, bm, S);
}

}  // namespace phdc
