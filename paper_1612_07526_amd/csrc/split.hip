// Split-precision merge update: the same Gu-grouped products as the FP64 path
// (Eq. (6)), with the bulk arithmetic on the BF16 matrix cores.
//
// Each row i of the Q operand A is scaled by 2^-e_i and each column j of Uhat
// (operand B) by 2^-f_j so that all entries lie in (-1, 1); the scaled values
// are cut into s slices of 8 bits,
//     x = sum_{p < s} 2^{-8(p+1)} a_p,   a_p integer, |a_p| <= 255,
// which BF16 (8 significant bits) holds exactly.  A slice product a_p b_q is an
// integer below 2^16, so an FP32 sum of up to 2^8 of them is exact.  Products
// with the same weight t = p + q are summed in FP32 over 32-deep k-steps
// (at most s * 32 * 255^2 < 2^24: exact), then scaled by 2^{-8(t+2)} and
// accumulated in FP64; pairs with p + q >= s are dropped (their weight is below
// 2^{-8(s+1)}).  Finally C_ij = 2^{e_i + f_j} * acc_ij.
#include "phdc_internal.h"
#include "split.h"

namespace phdc {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f4s_t __attribute__((ext_vector_type(4)));

__device__ inline int exp_above(double v) {
  // smallest e with |v| < 2^e (v == 0 -> 0)
  if (v == 0.0) return 0;
  int e;
  frexp(v, &e);  // v = m 2^e, m in [0.5, 1)
  return e;
}

// ------------------------------------------------------------ scales
// Row exponents of the gathered Q operand (both halves) and column exponents of
// the grouped Uhat (row-major, ld K).  One thread per row / column.
__global__ void __launch_bounds__(256) k_split_scales(BlockMap bm, Scratch S, SplitBufs B) {
  const int b = blockIdx.x;
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  const int K = cnt[C_K], k1 = cnt[C_K1], k2 = cnt[C_K2], k3 = cnt[C_K3];
  const int64_t so = M.s_off;
  const int x = lb * 256 + threadIdx.x;
  if (x < M.m) {  // row x of the merge block
    const bool top = x < M.n1;
    const int kd = top ? k1 + k2 : k2 + k3;
    const int32_t* cols = top ? S.coltop + so : S.colbot + so;
    const RowRange* rg = top ? S.rgtop + so : S.rgbot + so;
    double mx = 0.0;
    for (int k = 0; k < kd; ++k)
      if (x >= rg[k].lo && x < rg[k].hi) mx = fmax(mx, fabs(M.qin[x + (int64_t)cols[k] * M.ldin]));
    B.erow[so + x] = exp_above(mx);
  }
  if (x < K) {  // column x of Uhat
    const double* U = S.uhat + M.u_off;
    double mx = 0.0;
    for (int g = 0; g < K; ++g) mx = fmax(mx, fabs(U[(int64_t)g * K + x]));
    B.fcol[so + x] = exp_above(mx);
  }
}

// ------------------------------------------------------------ slicing
__device__ inline void cut(double v, int nsl, __bf16* out, int64_t stride) {
  // v in (-1, 1): 8 bits per slice, truncation toward zero keeps every slice's sign
  for (int p = 0; p < nsl; ++p) {
    v *= 256.0;
    const double a = trunc(v);
    v -= a;
    out[(int64_t)p * stride] = (__bf16)(float)a;
  }
}

// A slices: per half, row-major [slice][row][kdp] (kdp = kd rounded up to 8), zero-padded.
__global__ void __launch_bounds__(256) k_split_slice_a(BlockMap bm, Scratch S, SplitBufs B, int nsl) {
  const int b = blockIdx.x;
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  if (cnt[C_PATH] != 1) return;
  const int k1 = cnt[C_K1], k2 = cnt[C_K2], k3 = cnt[C_K3];
  const int64_t so = M.s_off;
  const int RB = (M.m + 255) / 256;
  const int rb = lb % RB, kg = lb / RB;
  const int x = rb * 256 + threadIdx.x;
  if (x >= M.m) return;
  const bool top = x < M.n1;
  const int kd = top ? k1 + k2 : k2 + k3;
  const int kdp = (kd + 7) & ~7;
  const int rows = top ? M.n1 : M.m - M.n1;
  const int row = top ? x : x - M.n1;
  const int32_t* cols = top ? S.coltop + so : S.colbot + so;
  const RowRange* rg = top ? S.rgtop + so : S.rgbot + so;
  __bf16* base = B.aslice + (int64_t)nsl * M.x_off + (top ? 0 : (int64_t)nsl * M.n1 * (((k1 + k2) + 7) & ~7));
  const int64_t stride = (int64_t)rows * kdp;
  const double sc = ldexp(1.0, -B.erow[so + x]);
  for (int k0 = kg * 8; k0 < kdp; k0 += 8 * B.kgroups) {
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + e;
      const double v = (k < kd && x >= rg[k].lo && x < rg[k].hi) ? M.qin[x + (int64_t)cols[k] * M.ldin] * sc : 0.0;
      cut(v, nsl, base + (int64_t)row * kdp + k, stride);
    }
  }
}

// B slices: row-major [slice][g][Kp] (Kp = K rounded up to 8), zero-padded.
__global__ void __launch_bounds__(256) k_split_slice_b(BlockMap bm, Scratch S, SplitBufs B, int nsl) {
  const int b = blockIdx.x;
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  if (cnt[C_PATH] != 1) return;
  const int K = cnt[C_K];
  const int Kp = (K + 7) & ~7;
  const int64_t so = M.s_off;
  const int CB = (M.m + 255) / 256;
  const int cb = lb % CB, rg = lb / CB;
  const int j = cb * 256 + threadIdx.x;
  if (j >= Kp) return;
  const double* U = S.uhat + M.u_off;
  __bf16* base = B.bslice + (int64_t)nsl * M.x_off;
  const int64_t stride = (int64_t)K * Kp;
  const double sc = (j < K) ? ldexp(1.0, -B.fcol[so + j]) : 0.0;
  for (int g = rg; g < K; g += B.rgroups) {
    const double v = (j < K) ? U[(int64_t)g * K + j] * sc : 0.0;
    cut(v, nsl, base + (int64_t)g * Kp + j, stride);
  }
}

// ------------------------------------------------------------ slice products
constexpr int XT = 128;  // output tile
constexpr int XK = 32;   // k per step (one BF16 MFMA depth)
constexpr int XLD = XK + 8;  // LDS row stride in bf16 (16-byte aligned rows)
constexpr int XMAXS = kSplitMaxSlices;

__global__ void __launch_bounds__(256) k_split_gemm(BlockMap bm, Scratch S, SplitBufs B, int nsl) {
  __shared__ __attribute__((aligned(16))) __bf16 As[XMAXS][XT][XLD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[XMAXS][XT][XLD];
  const int b = blockIdx.x;
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  if (cnt[C_PATH] != 1) return;
  const int K = cnt[C_K], k1 = cnt[C_K1], k2 = cnt[C_K2], k3 = cnt[C_K3];
  const int Kp = (K + 7) & ~7;
  const int n1 = M.n1, n2 = M.m - M.n1;
  const int tmt = (n1 + XT - 1) / XT, tmb = (n2 + XT - 1) / XT;
  const int TM = tmt + tmb;
  const int TN = (K + XT - 1) / XT;
  const int nact = TM * TN;
  if (lb >= nact) return;
  // A block computes tiles lb, lb + G, ... (G = the merge's blocks).
  const int G = merge_blocks(bm, mi);
  for (int tile = lb; tile < nact; tile += G) {
    // XCD-aware grouped tile order, as in the FP64 update GEMM
    const int n8 = nact - nact % 8;
    const int lid = (tile < n8) ? (tile % 8) * (n8 / 8) + tile / 8 : tile;
    const int width = 8 * TN;
    const int first = (lid / width) * 8;
    const int gsz = min(TM - first, 8);
    const int in = lid % width;
    const int mt = first + in % gsz, nt = in / gsz;
    const bool top = mt < tmt;
    const int mrow0 = top ? mt * XT : (mt - tmt) * XT;
    const int rows = top ? n1 : n2;
    const int rowoff = top ? 0 : n1;
    const int kd = top ? k1 + k2 : k2 + k3;
    const int kdp = (kd + 7) & ~7;
    const int64_t so = M.s_off;
    const __bf16* Abase = B.aslice + (int64_t)nsl * M.x_off + (top ? 0 : (int64_t)nsl * n1 * (((k1 + k2) + 7) & ~7));
    const int64_t astride = (int64_t)rows * kdp;
    const __bf16* Bbase = B.bslice + (int64_t)nsl * M.x_off + (int64_t)(top ? 0 : k1) * Kp;
    const int64_t bstride = (int64_t)K * Kp;
    const int ncol0 = nt * XT;
    const int t = threadIdx.x;
    const int w = t >> 6, lane = t & 63;
    const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
    const int li = lane & 15, lg = lane >> 4;

    double acc[4][4][4];
  #pragma unroll
    for (int i = 0; i < 4; ++i)
  #pragma unroll
      for (int j = 0; j < 4; ++j)
  #pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

    const int nks = (kd + XK - 1) / XK;
    for (int ks = 0; ks < nks; ++ks) {
      const int kb = ks * XK;
      __syncthreads();
      // stage: A slices (rows x 32 k, k contiguous in global), B slices (32 k x 128 j) transposed to [j][k]
      for (int e = t; e < nsl * XT * 4; e += 256) {
        const int p = e / (XT * 4), rem = e % (XT * 4), i = rem >> 2, kq = (rem & 3) * 8;
        const int row = mrow0 + i, k = kb + kq;
        bf8_t v;
        if (row < rows && k < kdp) v = *(const bf8_t*)(Abase + (int64_t)p * astride + (int64_t)row * kdp + k);
        else
          for (int q = 0; q < 8; ++q) v[q] = (__bf16)0.0f;
        *(bf8_t*)&As[p][i][kq] = v;
      }
      for (int e = t; e < nsl * XK * (XT / 8); e += 256) {
        const int p = e / (XK * (XT / 8)), rem = e % (XK * (XT / 8)), kk = rem / (XT / 8), j8 = (rem % (XT / 8)) * 8;
        const int k = kb + kk, col = ncol0 + j8;
        bf8_t v;
        if (k < kd && col < Kp) v = *(const bf8_t*)(Bbase + (int64_t)p * bstride + (int64_t)k * Kp + col);
        else
          for (int q = 0; q < 8; ++q) v[q] = (__bf16)0.0f;
        for (int q = 0; q < 8; ++q) Bs[p][j8 + q][kk] = v[q];
      }
      __syncthreads();
      for (int tw = 0; tw < nsl; ++tw) {  // weight group t = p + q
        f4s_t c[4][4];
  #pragma unroll
        for (int i = 0; i < 4; ++i)
  #pragma unroll
          for (int j = 0; j < 4; ++j) c[i][j] = f4s_t{0.f, 0.f, 0.f, 0.f};
        for (int p = 0; p <= tw; ++p) {
          const int q = tw - p;
          bf8_t av[4], bv[4];
  #pragma unroll
          for (int i = 0; i < 4; ++i) av[i] = *(const bf8_t*)&As[p][wm + i * 16 + li][lg * 8];
  #pragma unroll
          for (int j = 0; j < 4; ++j) bv[j] = *(const bf8_t*)&Bs[q][wn + j * 16 + li][lg * 8];
  #pragma unroll
          for (int i = 0; i < 4; ++i)
  #pragma unroll
            for (int j = 0; j < 4; ++j) c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], c[i][j], 0, 0, 0);
        }
        const double wt = ldexp(1.0, -8 * (tw + 2));
  #pragma unroll
        for (int i = 0; i < 4; ++i)
  #pragma unroll
          for (int j = 0; j < 4; ++j)
  #pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)c[i][j][r] * wt;
      }
    }
    // epilogue: undo the scales, write to the sorted output columns
    const int32_t* dest = S.dest + so;
    double* out = M.qout + rowoff;
  #pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cj = ncol0 + wn + j * 16 + li;
      if (cj >= K) continue;
      double* oc = out + (int64_t)dest[cj] * M.ldout;
      const int fe = B.fcol[so + cj];
  #pragma unroll
      for (int i = 0; i < 4; ++i)
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = mrow0 + wm + i * 16 + kSplitRow(lg, r);
          if (row < rows) oc[row] = ldexp(acc[i][j][r], B.erow[so + rowoff + row] + fe);
        }
    }
    __syncthreads();  // LDS reused by the next tile
  }
}

void launch_split_update(const MergeDesc* descs, int nm, const LevelMaps& maps, const Scratch& S,
                         const SplitBufs& B, int nsl, hipStream_t s) {
  auto bmap = [&](int kind) { return BlockMap{descs, maps.pfx[kind], nm, maps.per[kind]}; };
  hipLaunchKernelGGL(k_split_scales, dim3(maps.total[MAP_ROWS256]), dim3(256), 0, s, bmap(MAP_ROWS256), S, B);
  hipLaunchKernelGGL(k_split_slice_a, dim3(maps.total[MAP_SPLITA]), dim3(256), 0, s, bmap(MAP_SPLITA), S, B, nsl);
  hipLaunchKernelGGL(k_split_slice_b, dim3(maps.total[MAP_SPLITB]), dim3(256), 0, s, bmap(MAP_SPLITB), S, B, nsl);
  hipLaunchKernelGGL(k_split_gemm, dim3(maps.total[MAP_GEMM]), dim3(256), 0, s, bmap(MAP_GEMM), S, B, nsl);
}

}  // namespace phdc
