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
// Tiling for gfx950: 256 threads (4 waves) per GT x GT output tile (GT = 64 or
// 128, chosen per tree level from a table that phdc_autotune_gemm measures),
// each wave a quadrant of v_mfma_f64_16x16x4 blocks; k-steps of 16 staged
// through double-buffered LDS.
#include <algorithm>
#include <atomic>
#include <cstdint>

#include "phdc_internal.h"

namespace phdc {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) double gdouble_t;  // a double in global memory

constexpr int GK = 16;        // k per LDS stage
constexpr int GPAD = 4;       // LDS row padding (doubles)

// GT x GT output tiles, 256 threads (4 waves in 2 x 2), each wave a GT/2 x
// GT/2 quadrant of 16 x 16 MFMA blocks; block lb of the merge's G blocks
// computes tiles lb, lb + G, ...  lds holds the double-buffered A and B
// stages.  The k loop runs in the same order for every tile size, so the
// result does not depend on GT.
template <int GT>
__device__ __forceinline__ void gemm_merge_tiles(const MergeDesc& M, const Scratch& S, int K, int k1, int k2, int k3,
                                                 int lb, int G, int scale_cols, double* lds) {
  constexpr int GLD = GT + GPAD;
  constexpr int E = GT * GK / 256;  // elements of A (and of B) each thread stages per k-step
  constexpr int WT = GT / 2;        // wave tile edge
  constexpr int NB = WT / 16;       // MFMA blocks per wave tile edge
  double (*As)[GK][GLD] = reinterpret_cast<double (*)[GK][GLD]>(lds);
  double (*Bs)[GK][GLD] = reinterpret_cast<double (*)[GK][GLD]>(lds + 2 * GK * GLD);
  const int n1 = M.n1, n2 = M.m - M.n1;
  const int tmt = (n1 + GT - 1) / GT, tmb = (n2 + GT - 1) / GT;
  const int TM = tmt + tmb;
  const int TN = (K + GT - 1) / GT;  // column tiles with work (the grid covers m columns)
  const int nact = TM * TN;
  for (int tile = lb; tile < nact; tile += G) {
    // Tile order.  Workgroups are dispatched round-robin over the 8 XCDs, each
    // with its own L2: hand XCD (tile mod 8) a contiguous range of tiles, and walk
    // each range in groups of 8 row tiles so that the blocks in flight on one XCD
    // share A panels across columns and B panels across rows.
    const int n8 = nact - nact % 8;
    const int lid = (tile < n8) ? (tile % 8) * (n8 / 8) + tile / 8 : tile;
    constexpr int GM = 8;
    const int width = GM * TN;
    const int first = (lid / width) * GM;
    const int gsz = min(TM - first, GM);
    const int in = lid % width;
    const int mt = first + in % gsz, nt = in / gsz;
    const bool top = mt < tmt;
    const int mrow0 = top ? mt * GT : (mt - tmt) * GT;  // first row of the tile within its half
    const int Mrows = top ? n1 : n2;
    const int rowoff = top ? 0 : n1;                    // half's first row within the merge block
    const int kd = top ? k1 + k2 : k2 + k3;
    const int64_t so = M.s_off;
    const int32_t* colA = top ? S.coltop + so : S.colbot + so;
    const RowRange* rgA = top ? S.rgtop + so : S.rgbot + so;  // rows of each column that can be nonzero
    const double* Bm = S.uhat + M.u_off + (int64_t)(top ? 0 : k1) * K;  // row-major, ld = K
    const double* A = M.qin + rowoff;
    const int64_t lda = M.ldin;
    const int ncol0 = nt * GT;

    const int t = threadIdx.x;
    const int lkc = t >> 4;          // k index this thread stages (A column / B row)
    const int l8 = (t & 15) * E;     // first of E consecutive rows (A) / columns (B)
    double ra[E], rb[E];
    // Uhat written with unscaled columns: the B entries take their column's
    // scale (the reciprocal norm of Uhat's column) as they are staged, which
    // gives the bits of the normalized entries.  A thread stages the same E
    // columns at every k-step.
    double csc[E];
  #pragma unroll
    for (int e = 0; e < E; ++e)
      csc[e] = (scale_cols && ncol0 + l8 + e < K) ? S.cnorm[M.s_off + ncol0 + l8 + e] : 1.0;

    // With 64-wide (or 32-wide) tiles (merges with few columns: latency counts), the column
    // index and row range of the A column a thread stages are read two k-steps
    // ahead of its data (gidx), so the data load of a step waits on one memory
    // latency, not on two dependent ones.  With 128-wide tiles (large merges)
    // they are read with the data: the early reads would make a step's MFMAs
    // wait for that step's loads (measured: 10% slower at K = 16384).
    constexpr bool kIdxAhead = GT <= 64;
    int nxc = 0;
    RowRange nxg{0, 0};
    auto gidx = [&](int kt) {
      const int kk = kt * GK + lkc;
      if (kIdxAhead && kk < kd) {
        nxc = colA[kk];
        nxg = rgA[kk];
      }
    };
    // Rows outside the staged A column's range are not loaded (they read as 0).
    auto gload = [&](int kt) {
      const int kk = kt * GK + lkc;
      if (kk < kd) {
        // The input block is global memory: say so, so that the loads are
        // global (not flat) ones and the waits can count them separately.
        const int cidx = kIdxAhead ? nxc : colA[kk];
        const gdouble_t* src = (const gdouble_t*)(A + (int64_t)cidx * lda + mrow0 + l8);
        const RowRange g = kIdxAhead ? nxg : rgA[kk];
        const int lo = g.lo - (rowoff + mrow0 + l8), hi = min(g.hi - rowoff, Mrows) - (mrow0 + l8);
  #pragma unroll
        for (int e = 0; e < E; ++e) ra[e] = (e >= lo && e < hi) ? src[e] : 0.0;
        const double* bs = Bm + (int64_t)kk * K + ncol0 + l8;
  #pragma unroll
        for (int e = 0; e < E; ++e) rb[e] = (ncol0 + l8 + e < K) ? bs[e] : 0.0;
      } else {
  #pragma unroll
        for (int e = 0; e < E; ++e) { ra[e] = 0.0; rb[e] = 0.0; }
      }
    };
    // (the column scale is applied here, after the step's MFMAs, not right after
    // the load: there it would make the step wait for its loads before computing)
    auto lstore = [&](int buf) {
  #pragma unroll
      for (int e = 0; e < E; ++e) {
        As[buf][lkc][l8 + e] = ra[e];
        Bs[buf][lkc][l8 + e] = rb[e] * csc[e];
      }
    };

    const int w = t >> 6, lane = t & 63;
    const int wm = (w & 1) * WT, wn = (w >> 1) * WT;
    const int li = lane & 15, lk = lane >> 4;
    d4_t acc[NB][NB];
  #pragma unroll
    for (int i = 0; i < NB; ++i)
  #pragma unroll
      for (int j = 0; j < NB; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    const int nkt = (kd + GK - 1) / GK;
    if (nkt > 0) {
      gidx(0);
      gload(0);
      if (nkt > 1) gidx(1);
      lstore(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nkt) gload(kt + 1);
      if (kt + 2 < nkt) gidx(kt + 2);
  #pragma unroll
      for (int ks = 0; ks < GK / 4; ++ks) {
        const int kr = ks * 4 + lk;
        double av[NB], bv[NB];
  #pragma unroll
        for (int i = 0; i < NB; ++i) av[i] = As[buf][kr][wm + i * 16 + li];
  #pragma unroll
        for (int j = 0; j < NB; ++j) bv[j] = Bs[buf][kr][wn + j * 16 + li];
  #pragma unroll
        for (int i = 0; i < NB; ++i)
  #pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
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
    for (int j = 0; j < NB; ++j) {
      const int cj = ncol0 + wn + j * 16 + li;
      if (cj >= K) continue;
      double* oc = out + (int64_t)dest[cj] * ldo;
  #pragma unroll
      for (int i = 0; i < NB; ++i) {
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = mrow0 + wm + i * 16 + lk + 4 * r;
          if (row < Mrows) oc[row] = acc[i][j][r];
        }
      }
    }
    __syncthreads();  // LDS reused by the next tile
  }
}

// Tile edge of one merge: 128 (if the launch allows it) when the merge has at
// least kGemmWideTiles tiles of that edge, else 64: a merge that keeps few
// columns gets four times more, smaller, tiles, so that more CUs share it.  The
// grid of every merge is sized for edge 64 (at most kGemmBlockCap blocks).
constexpr int kGemmWideTiles = 512;

// GTMAX = 32 runs every merge of the launch in 32-wide tiles (more, smaller
// tiles for levels of many small merges; an autotuner candidate).
template <int GTMAX>
__global__ void __launch_bounds__(256) k_merge_gemm(BlockMap bm, Scratch S, int scale_cols) {
  __shared__ double lds[4 * GK * (GTMAX + GPAD)];
  const int b = blockIdx.x;
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  if (cnt[C_PATH] != 0) return;  // formed by another update path
  const int K = cnt[C_K], k1 = cnt[C_K1], k2 = cnt[C_K2], k3 = cnt[C_K3];
  const int G = merge_blocks(bm, mi);
  if constexpr (GTMAX == 32) {
    gemm_merge_tiles<32>(M, S, K, k1, k2, k3, lb, G, scale_cols, lds);
    return;
  }
  if constexpr (GTMAX == 128) {
    const int tiles128 = ((M.n1 + 127) / 128 + (M.m - M.n1 + 127) / 128) * ((K + 127) / 128);
    if (tiles128 >= kGemmWideTiles) {
      gemm_merge_tiles<128>(M, S, K, k1, k2, k3, lb, G, scale_cols, lds);
      return;
    }
  }
  gemm_merge_tiles<64>(M, S, K, k1, k2, k3, lb, G, scale_cols, lds);
}

void launch_merge_gemm_f64(const BlockMap& bm, int total, const Scratch& S, int tile, bool scale_cols,
                           hipStream_t s) {
  if (total <= 0) return;
  if (tile == 32) hipLaunchKernelGGL(k_merge_gemm<32>, dim3(total), dim3(256), 0, s, bm, S, scale_cols ? 1 : 0);
  else if (tile == 64) hipLaunchKernelGGL(k_merge_gemm<64>, dim3(total), dim3(256), 0, s, bm, S, scale_cols ? 1 : 0);
  else hipLaunchKernelGGL(k_merge_gemm<128>, dim3(total), dim3(256), 0, s, bm, S, scale_cols ? 1 : 0);
}

// ------------------------------------------------------------ tile choice
// Tile rule per merge-size bucket (bucket b holds 2^(b-1) < m <= 2^b): 32 or 64
// (every merge of the launch in tiles of that edge) or 128 (128-wide tiles for
// merges with at least kGemmWideTiles of them, 64 for the others); 0 means not
// measured, in which case 64 is used up to m = 256 and 128 above.
namespace {
std::atomic<int> g_tile[kTileBuckets];

int bucket_of(int64_t m) {
  int b = 0;
  while (b + 1 < kTileBuckets && ((int64_t)1 << b) < m) ++b;
  return b;
}

__global__ void k_autotune_fill(double* q, double* u, int64_t count, int32_t* cnt, int32_t* coltop, int32_t* colbot,
                                int32_t* dest, RowRange* rgtop, RowRange* rgbot, int m, int n1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = i; e < count; e += stride) {  // bounded values, no structure the GEMM could exploit
    q[e] = (double)((e * 2654435761LL) % 1000003) * 1e-6 - 0.5;
    u[e] = (double)((e * 40503LL + 17) % 999983) * 1e-6 - 0.5;
  }
  for (int64_t c = i; c < m; c += stride) {
    dest[c] = (int32_t)c;
    if (c < n1) {
      coltop[c] = (int32_t)c;
      rgtop[c] = RowRange{0, n1};
    }
    if (c < m - n1) {
      colbot[c] = (int32_t)(n1 + c);
      rgbot[c] = RowRange{n1, m};
    }
  }
  if (i == 0) {
    for (int k = 0; k < kCounters; ++k) cnt[k] = 0;
    cnt[C_K] = m;
    cnt[C_K1] = n1;
    cnt[C_K2] = 0;
    cnt[C_K3] = m - n1;
    cnt[C_PATH] = 0;
  }
}

size_t autotune_bytes(int64_t max_m) {
  const size_t mm = (size_t)max_m * max_m;
  return 3 * mm * 8 + (size_t)(3 * max_m + kCounters + 64) * 4 + (size_t)2 * max_m * sizeof(RowRange) + 3 * 256 +
         sizeof(MergeDesc);
}
}  // namespace

int gemm_tile_for(int64_t maxm) {
  const int v = g_tile[bucket_of(maxm)].load();
  if (v == 32 || v == 64 || v == 128) return v;
  return maxm <= 256 ? 64 : 128;
}

}  // namespace phdc

using namespace phdc;

extern "C" {

int phdc_autotune_gemm_workspace(int64_t max_m, size_t* bytes) {
  if (max_m < 2 || max_m > ((int64_t)1 << (kTileBuckets - 1))) return -1;
  if (!bytes) return -2;
  *bytes = autotune_bytes(max_m);
  return 0;
}

int phdc_autotune_gemm(int64_t max_m, void* work, size_t lwork, void* stream) {
  if (max_m < 2 || max_m > ((int64_t)1 << (kTileBuckets - 1))) return -1;
  if (!work) return -2;
  if (lwork < autotune_bytes(max_m)) return -3;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)work;
  const size_t mm = (size_t)max_m * max_m;
  double* q = (double*)base;
  double* qo = q + mm;
  double* u = qo + mm;
  int32_t* cnt = (int32_t*)(u + mm);
  int32_t* coltop = cnt + kCounters;
  int32_t* colbot = coltop + max_m;
  int32_t* dest = colbot + max_m;
  RowRange* rgtop = (RowRange*)(((uintptr_t)(dest + max_m) + 255) / 256 * 256);
  RowRange* rgbot = rgtop + max_m;
  char* tail = (char*)(rgbot + max_m);
  tail = (char*)(((uintptr_t)tail + 255) / 256 * 256);
  MergeDesc* desc = (MergeDesc*)tail;
  int32_t* pfx = (int32_t*)(tail + 256);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PHDC_E_HIP;
  int rc = 0;
  for (int64_t m = 64; m <= max_m && rc == 0; m *= 2) {
    const int n1 = (int)(m / 2);
    hipLaunchKernelGGL(k_autotune_fill, dim3(1024), dim3(256), 0, s, q, u, (int64_t)(m * m), cnt, coltop, colbot, dest,
                       rgtop, rgbot, (int)m, n1);
    MergeDesc D{};
    D.qin = q;
    D.qout = qo;
    D.ldin = m;
    D.ldout = m;
    D.m = (int32_t)m;
    D.n1 = n1;
    D.id = 0;
    Scratch S{};
    S.counters = cnt;
    S.coltop = coltop;
    S.colbot = colbot;
    S.rgtop = rgtop;
    S.rgbot = rgbot;
    S.dest = dest;
    S.uhat = u;
    constexpr int NC = 3;
    float best[NC] = {1e30f, 1e30f, 1e30f};
    const int tiles[NC] = {32, 64, 128};
    for (int v = 0; v < NC && rc == 0; ++v) {
      const int gt = tiles[v];
      const int total = map_blocks(MAP_GEMM, (int)m, n1, gt, false);
      const int32_t hp[2] = {0, total};
      if (hipMemcpyAsync(desc, &D, sizeof(D), hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(pfx, hp, sizeof(hp), hipMemcpyHostToDevice, s) != hipSuccess) {
        rc = PHDC_E_HIP;
        break;
      }
      BlockMap bm{desc, pfx, 1, 0};
      launch_merge_gemm_f64(bm, total, S, gt, false, s);  // warm-up
      for (int r = 0; r < 3; ++r) {
        hipEventRecord(e0, s);
        launch_merge_gemm_f64(bm, total, S, gt, false, s);
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = PHDC_E_HIP;
          break;
        }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        best[v] = std::min(best[v], ms);
      }
    }
    if (rc == 0) {
      int bv = 0;
      for (int v = 1; v < NC; ++v)
        if (best[v] < best[bv]) bv = v;
      g_tile[bucket_of(m)].store(tiles[bv]);
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc == 0 && hipGetLastError() != hipSuccess) rc = PHDC_E_HIP;
  return rc;
}

int phdc_gemm_tile_table(int32_t* tiles, int n) {
  if (!tiles || n <= 0) return -1;
  for (int b = 0; b < n && b < kTileBuckets; ++b) tiles[b] = g_tile[b].load();
  return std::min(n, kTileBuckets);
}

}  // extern "C"
