// HSS path of the merge update (Sec. 2.2): when a merge keeps K >= hss_min_K
// poles, the Cauchy-like eigenvector matrix Uhat (K x K) is compressed into
// hierarchically semiseparable form by randomized sampling (Algorithm 1) and
// the update U = X Uhat (Eq. (6), X = the merge's rotated input columns in
// pole order, no Gu grouping) is applied in that form.
//
// HSS form (Eq. (7)): on a binary tree over the pole order with leaves of at
// most hss_leaf poles, each leaf i has D_i = Uhat(t_i, t_i) and row / column
// interpolation bases U_i, V_i; each parent has transfer matrices U_p, V_p
// acting on its children's skeletons, and each sibling pair (c1, c2) has the
// couplings B_c1 = Uhat(I_c1, J_c2), B_c2 = Uhat(I_c2, J_c1) where I, J are
// skeleton row / column indices chosen by interpolative decompositions (IDs).
//
// Construction (Algorithm 1): Y = Uhat Omega1, Z = Uhat^T Omega2 with Gaussian
// Omega (K x d); bottom-up, Phi_i = Y_i - D_i Omega1_i (leaf) or the stacked
// child skeleton rows minus their couplings' contribution (parent), a row ID
// Phi_i ~ U_i Phi_i(I_i, :) and likewise Theta_i ~ V_i Theta_i(J_i, :) for Z,
// then Yhat_i = V_i^T Omega1_i (nested), Zhat_i = U_i^T Omega2_i (nested).
//
// Application of U = X Uhat (the transposed HSS product, all operands m rows):
//   leaves   Xh_i = X(:, t_i) U_i,       U(:, t_i) = X(:, t_i) D_i
//   up       Xh_p = [Xh_c1 Xh_c2] U_p
//   couple   Yh_c2 = Xh_c1 B_c1,         Yh_c1 = Xh_c2 B_c2
//   down     [Yh_c1 Yh_c2] += Yh_p V_p^T
//   leaves   U(:, t_i) += Yh_i V_i^T
// The IDs use column-pivoted Householder QR of Phi^T.  The rank ends at the
// first pivot with |R_kk| <= max(tol |R_00|, tol sqrt(d) ||Uhat||_2), tol =
// hss_rel_tol: relative to the node's own largest pivot, with a floor at the
// size a Gaussian sample of a block with singular value tol ||Uhat||_2 has.
// Uhat is orthogonal (||Uhat||_2 = 1).  Without the floor, the parents'
// samples, formed by subtracting the sibling coupling from the children's
// skeleton rows, carry rounding noise far above tol times their own (small)
// largest pivot, and the ranks grow to the sample count.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gemm_generic.h"
#include "hss.h"
#include "profile.h"

namespace phdc {

// ------------------------------------------------------------ random samples
// Counter-based Gaussian numbers: SplitMix64 (Steele, Lea, Flood 2014) on the
// counter, then the Box-Muller transform.
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

__global__ void __launch_bounds__(256) k_gauss(int64_t count, uint64_t seed, double* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const uint64_t a = splitmix64(seed + 2 * (uint64_t)i), b = splitmix64(seed + 2 * (uint64_t)i + 1);
  const double u1 = ((double)(a >> 11) + 0.5) * 1.1102230246251565e-16;  // (0, 1)
  const double u2 = (double)(b >> 11) * 1.1102230246251565e-16;          // [0, 1)
  out[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// ------------------------------------------------------------ gathers
// X(:, k) = input column of survivor k (pole order), rows outside its range as 0.
__global__ void __launch_bounds__(256) k_gather_x(const double* __restrict__ qin, int64_t ldin, int m, int K,
                                                  const int32_t* __restrict__ csort,
                                                  const RowRange* __restrict__ crng, double* X) {
  const int k = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (k >= K || r >= m) return;
  const int c = csort[k];
  const RowRange g = crng[c];
  X[r + (int64_t)k * m] = (r >= g.lo && r < g.hi) ? qin[r + (int64_t)c * ldin] : 0.0;
}

// Entries of the compressed matrix: either Uhat evaluated from the secular
// solution with the same arithmetic as the dense writer, zhat_i / ((d_i -
// dorg_j) - tau_j) * cnorm_j, or (A != nullptr) a dense column-major matrix.
__global__ void __launch_bounds__(256) k_ugather(const UGather* __restrict__ g, const double* __restrict__ ds,
                                                 const double* __restrict__ zh, const double* __restrict__ dorg,
                                                 const double* __restrict__ tau, const double* __restrict__ cn,
                                                 const double* __restrict__ A, int64_t lda) {
  const UGather G = g[blockIdx.x];
  for (int e = threadIdx.x; e < G.nr * G.nc; e += 256) {
    const int a = e % G.nr, b = e / G.nr;
    const int i = G.ri ? G.ri[a] : G.r0 + a;
    const int j = G.cj ? G.cj[b] : G.c0 + b;
    G.out[a + (int64_t)b * G.ld] = A ? A[i + (int64_t)j * lda] : zh[i] / ((ds[i] - dorg[j]) - tau[j]) * cn[j];
  }
}

__global__ void __launch_bounds__(256) k_rows(const RowCopy* __restrict__ rc) {
  const RowCopy R = rc[blockIdx.x];
  for (int e = threadIdx.x; e < R.nr * R.ncol; e += 256) {
    const int a = e % R.nr, b = e / R.nr;
    const int src = R.idx ? R.idx[a] : a;
    R.dst[R.dst_row0 + a + (int64_t)b * R.ldd] = R.src[src + (int64_t)b * R.lds];
  }
}

__global__ void __launch_bounds__(256) k_ints(const IntCopy* __restrict__ ic) {
  const IntCopy C = ic[blockIdx.x];
  for (int a = threadIdx.x; a < C.n; a += 256) C.dst[C.dst0 + a] = C.src[a];
}

__global__ void __launch_bounds__(256) k_skel(const SkelDesc* __restrict__ sd) {
  const SkelDesc S = sd[blockIdx.x];
  for (int a = threadIdx.x; a < S.rank; a += 256) {
    const int p = S.perm[a];
    S.out[a] = S.base ? S.base[p] : S.lo + p;
  }
}

// ------------------------------------------------------------ interpolative decomposition
// Row ID of Phi (p x d): Phi ~ U Phi(I, :), U (p x r) holding the identity on
// the skeleton rows I = perm[0:r].  Computed as the column-pivoted Householder
// QR of Phi^T, whose columns are Phi's rows: Phi^T P = Q [R11 R12]; the rank r
// is the number of pivots with |R_kk| > tol |R_00|; T = R11^{-1} R12 and
// U(perm[r + c], :) = T(:, c)^T.  One block per decomposition; the work copy
// keeps Phi's layout, so row c of Phi (a column of Phi^T) is W(c, :).
constexpr int kIdMax = kHssLeafMax;  // rows p of one decomposition; the sample count d <= 512 < kIdMax
constexpr int kIdThreads = 1024;
constexpr int kIdWaves = kIdThreads / 64;
constexpr int kIdLanes = 16;                    // lanes per column in the reflector update
constexpr int kIdCols = kIdThreads / kIdLanes;  // columns updated at a time
constexpr int kIdRegs = 16;                     // entries of a column a lane keeps in registers
constexpr int kIdSpan = kIdLanes * kIdRegs;     // rows j .. j + kIdSpan - 1 of a column stay in registers

__device__ inline double id_group_sum(double s) {
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 4, 64);
  s += __shfl_xor(s, 8, 64);
  return s;
}

__global__ void __launch_bounds__(kIdThreads) k_row_id(const IdDesc* __restrict__ ids, double tol, double abs_tol) {
  __shared__ double cn[kIdMax], cn0[kIdMax], v[kIdMax];
  __shared__ int pv[kIdMax];
  __shared__ double redv[kIdWaves];
  __shared__ int redi[kIdWaves];
  __shared__ double sh_norm, sh_r00;
  __shared__ int sh_piv, sh_stop;
  const IdDesc D = ids[blockIdx.x];
  const int p = D.p, d = D.d;
  double* W = D.work;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int sub = t % kIdLanes, cg = t / kIdLanes;
  for (int64_t e = t; e < (int64_t)p * d; e += kIdThreads) {
    const int c = (int)(e % p), k = (int)(e / p);
    W[c + (int64_t)k * p] = D.phi[c + (int64_t)k * D.ldphi];
  }
  __syncthreads();
  // Squared norms of Phi's rows (columns of Phi^T), four lanes per row; each
  // lane only touches the entries k = sub (mod 4) of its column.
  for (int c0 = 0; c0 < p; c0 += kIdCols) {
    const int c = c0 + cg;
    double s = 0.0;
    if (c < p)
      for (int k = sub; k < d; k += kIdLanes) {
        const double x = W[c + (int64_t)k * p];
        s += x * x;
      }
    s = id_group_sum(s);
    if (c < p && sub == 0) {
      cn[c] = s;
      cn0[c] = s;
      pv[c] = c;
    }
  }
  if (t == 0) {
    sh_r00 = 0.0;
    sh_stop = 0;
  }
  __syncthreads();
  const int kmax = min(p, d);
  int r = 0;
  for (int j = 0; j < kmax; ++j) {
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int c = j + t; c < p; c += kIdThreads)
      if (cn[c] > bv) {
        bv = cn[c];
        bi = c;
      }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > bv || (ob == bv && oi < bi)) {
        bv = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      redv[w] = bv;
      redi[w] = bi;
    }
    __syncthreads();
    if (t == 0) {
      double b0 = redv[0];
      int i0 = redi[0];
      for (int q = 1; q < kIdWaves; ++q)
        if (redv[q] > b0 || (redv[q] == b0 && redi[q] < i0)) {
          b0 = redv[q];
          i0 = redi[q];
        }
      sh_piv = i0;
      const double nrm = sqrt(fmax(b0, 0.0));
      if (j == 0) sh_r00 = nrm;
      sh_stop = (i0 >= p || sh_r00 == 0.0 || nrm <= fmax(tol * sh_r00, abs_tol)) ? 1 : 0;
    }
    __syncthreads();
    if (sh_stop) break;
    const int piv = sh_piv;
    if (piv != j) {
      for (int k = t; k < d; k += kIdThreads) {
        const double a = W[j + (int64_t)k * p];
        W[j + (int64_t)k * p] = W[piv + (int64_t)k * p];
        W[piv + (int64_t)k * p] = a;
      }
      if (t == 0) {
        double a = cn[j];
        cn[j] = cn[piv];
        cn[piv] = a;
        a = cn0[j];
        cn0[j] = cn0[piv];
        cn0[piv] = a;
        const int q = pv[j];
        pv[j] = pv[piv];
        pv[piv] = q;
      }
      __syncthreads();
    }
    // Householder reflector of x = W(j, j:d): v = x - alpha e_j, alpha = -sign(x_j) |x|
    double s = 0.0;
    for (int k = j + t; k < d; k += kIdThreads) {
      const double x = W[j + (int64_t)k * p];
      v[k] = x;
      s += x * x;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) redv[w] = s;
    __syncthreads();
    if (t == 0) {
      double tot = 0.0;
      for (int q = 0; q < kIdWaves; ++q) tot += redv[q];
      sh_norm = sqrt(tot);
    }
    __syncthreads();
    const double xn = sh_norm;
    const double x0 = W[j + (int64_t)j * p];
    const double alpha = (x0 >= 0.0) ? -xn : xn;
    const double vtv = 2.0 * xn * (xn + fabs(x0));  // |x - alpha e_j|^2
    __syncthreads();
    if (t == 0) v[j] = x0 - alpha;
    __syncthreads();
    if (vtv > 0.0) {
      // Apply the reflector to the remaining columns, kIdLanes lanes per column:
      // a lane loads its entries of the column's first kIdSpan rows (from j) once,
      // all in flight together, and keeps them in registers for the dot product,
      // the update and, when needed, the recomputed norm; rows beyond (only with
      // more than kIdSpan samples) are read again for the update.  (Offsets into
      // the work copy fit in 32 bits: p d <= kIdMax * 512.)
      for (int c0 = j + 1; c0 < p; c0 += kIdCols) {
        const int c = c0 + cg;
        const bool on = c < p;
        double x[kIdRegs];
#pragma unroll
        for (int u = 0; u < kIdRegs; ++u) {
          const int k = j + sub + u * kIdLanes;
          x[u] = (on && k < d) ? W[c + k * p] : 0.0;
        }
        double dot = 0.0;
#pragma unroll
        for (int u = 0; u < kIdRegs; ++u) {
          const int k = j + sub + u * kIdLanes;
          if (k < d) dot += v[k] * x[u];
        }
        if (on)
          for (int k = j + kIdSpan + sub; k < d; k += kIdLanes) dot += v[k] * W[c + k * p];
        dot = id_group_sum(dot);
        const double f = 2.0 * dot / vtv;
        double rjc = 0.0;
#pragma unroll
        for (int u = 0; u < kIdRegs; ++u) {
          const int k = j + sub + u * kIdLanes;
          if (on && k < d) {
            x[u] -= f * v[k];
            W[c + k * p] = x[u];
            if (k == j) rjc = x[u];  // R_jc, held by lane sub == 0
          }
        }
        if (on)
          for (int k = j + kIdSpan + sub; k < d; k += kIdLanes) W[c + k * p] -= f * v[k];
        rjc = id_group_sum(rjc);
        double nc = on ? cn[c] - rjc * rjc : 0.0;
        const bool redo = on && nc <= 1e-2 * cn0[c];  // same decision in all lanes of the group
        if (redo) {  // cancellation: recompute the remaining norm
          double q = 0.0;
#pragma unroll
          for (int u = 0; u < kIdRegs; ++u) {
            const int k = j + sub + u * kIdLanes;
            if (k > j && k < d) q += x[u] * x[u];
          }
          for (int k = j + kIdSpan + sub; k < d; k += kIdLanes) {
            const double y = W[c + k * p];
            q += y * y;
          }
          nc = q;
        }
        const double nred = id_group_sum(redo ? nc : 0.0);
        if (on && sub == 0) {
          if (redo) {
            cn0[c] = nred;
            cn[c] = nred;
          } else {
            cn[c] = nc;
          }
        }
      }
    }
    __syncthreads();
    if (t == 0) W[j + (int64_t)j * p] = alpha;  // R_jj; R_{j c} sits at W(c, j)
    __syncthreads();
    r = j + 1;
  }
  // T = R11^{-1} R12 by column-oriented back substitution: the thread of
  // column c (c >= r) overwrites W(c, 0:r) = R12(:, c) with T(:, c).
  for (int a = r - 1; a >= 0; --a) {
    const double raa = W[a + (int64_t)a * p];
    for (int c = r + t; c < p; c += kIdThreads) {
      const double x = W[c + (int64_t)a * p] / raa;
      W[c + (int64_t)a * p] = x;
      for (int b = 0; b < a; ++b) W[c + (int64_t)b * p] -= W[a + (int64_t)b * p] * x;  // R_ba at W(a, b)
    }
  }
  double* U = D.U;
  for (int64_t e = t; e < (int64_t)p * r; e += kIdThreads) U[e] = 0.0;
  __syncthreads();
  for (int a = t; a < r; a += kIdThreads) U[pv[a] + (int64_t)a * p] = 1.0;
  for (int c = r + t; c < p; c += kIdThreads) {
    const int row = pv[c];
    for (int a = 0; a < r; ++a) U[row + (int64_t)a * p] = W[c + (int64_t)a * p];
  }
  for (int c = t; c < p; c += kIdThreads) D.perm[c] = pv[c];
  if (t == 0) *D.rank = r;
}

// The same decomposition with the whole work matrix on chip, for p <= 32 NS
// rows of Phi and d <= 16 NR samples.  Column c of Phi^T (row c of Phi) is
// owned by a group of kRfLanes lanes; lane sub keeps its entries k = sub +
// kRfLanes u (u < NR) in registers for the whole factorization (zero past d), so a
// pivot step moves no matrix data through memory: the pivot's owners publish
// the reflector in LDS, zero outside rows j..d-1, and every lane then applies
// it to all of its columns at once (one LDS read of v per row for every slot,
// no per-row predicates), and downdates the norms (recomputing them on
// cancellation, as above); row j of a column is picked out by a dot product
// with the unit vector e_j, also in LDS.  Columns are not swapped: a
// pivoted column is only marked, and ties in the pivot choice go to the lowest
// column index.  R11 (the rows of the pivoted columns up to their step) goes
// to LDS -- to the work copy past kRfR11 pivots -- and every unpivoted column
// solves R11 t = R12(:, c) in its registers by back substitution.
constexpr int kRfThreads = 512;
constexpr int kRfLanes = 16;
constexpr int kRfGroups = kRfThreads / kRfLanes;  // columns in flight per slot
constexpr int kRfRowsMax = kRfLanes * 16;  // largest sample count d of the on-chip form
constexpr int kRfR11 = 128;

template <int CTRL>
__device__ __forceinline__ double rf_dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 16 lanes of a row (quad xor 1, quad xor 2, half-row mirror,
// row mirror): every lane receives the same total.
__device__ __forceinline__ double rf_sum16(double v) {
  v += rf_dpp<0xB1>(v);
  v += rf_dpp<0x4E>(v);
  v += rf_dpp<0x141>(v);
  v += rf_dpp<0x140>(v);
  return v;
}

// Value of lane `src` of the caller's 16-lane row.
__device__ __forceinline__ double rf_lane(double v, int src) {
  return __shfl(v, (int)(threadIdx.x & 48) + src, 64);
}

struct RfShared {
  double* cn;
  double* cn0;
  double* v;   // reflector, zero outside rows j..d-1
  double* ej;  // unit vector of row j
  int* stp;
  int* chosen;
  double* vtv;
};

// The pivot column's owners build the reflector of its rows j..: v = x -
// alpha e_j, alpha = -sign(x_j) |x|; the column keeps R_jj = alpha.
template <int NS, int NR>
__device__ __forceinline__ void rf_reflect(double (&x)[NS][NR], const RfShared& sh, int piv, int j, int cg,
                                           int sub) {
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (cg + kRfGroups * s == piv) {
      double q = 0.0, xj = 0.0;
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int k = sub + kRfLanes * u;
        q += (k >= j) ? x[s][u] * x[s][u] : 0.0;
        xj += (k == j) ? x[s][u] : 0.0;
      }
      q = rf_sum16(q);
      const double x0 = rf_sum16(xj);  // (one nonzero term: exact)
      const double xn = sqrt(q);
      const double alpha = (x0 >= 0.0) ? -xn : xn;
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int k = sub + kRfLanes * u;
        sh.v[k] = (k > j) ? x[s][u] : (k == j ? x0 - alpha : 0.0);
        sh.ej[k] = (k == j) ? 1.0 : 0.0;
        if (k == j) x[s][u] = alpha;
      }
      if (sub == 0) {
        *sh.vtv = 2.0 * xn * (xn + fabs(x0));  // |x - alpha e_j|^2
        sh.cn[piv] = -1.0;
        sh.stp[piv] = j;
        sh.chosen[j] = piv;
      }
    }
  }
}

// Every remaining column c: x -= (2 v.x / v.v) v, and the norm of its rows
// j+1.. downdated by R_jc^2.  The rows below j see v = 0 and stay unchanged;
// whole registers below row j are skipped.
template <int NS, int NR>
__device__ __forceinline__ void rf_update(double (&x)[NS][NR], const RfShared& sh, int j, int p, int cg,
                                          int sub) {
  const int uj = j / kRfLanes;
  double f[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) f[s] = 0.0;
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    if (u >= uj) {
      const double vk = sh.v[sub + kRfLanes * u];
#pragma unroll
      for (int s = 0; s < NS; ++s) f[s] = fma(vk, x[s][u], f[s]);
    }
  }
  const double g = 2.0 / *sh.vtv;
  bool on[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = cg + kRfGroups * s;
    on[s] = c < p && sh.stp[c] < 0;
    f[s] = on[s] ? rf_sum16(f[s]) * g : 0.0;
  }
  double xj[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) xj[s] = 0.0;
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    if (u >= uj) {
      const double vk = sh.v[sub + kRfLanes * u], ek = sh.ej[sub + kRfLanes * u];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        x[s][u] = fma(-f[s], vk, x[s][u]);
        xj[s] = fma(ek, x[s][u], xj[s]);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (on[s]) {  // (uniform in the group)
      const int c = cg + kRfGroups * s;
      const double rj = rf_sum16(xj[s]);  // R_jc (one nonzero term: exact)
      double nc = sh.cn[c] - rj * rj;
      const bool redo = nc <= 1e-2 * sh.cn0[c];
      if (redo) {  // cancellation: recompute the remaining norm
        double q = 0.0;
#pragma unroll
        for (int u = 0; u < NR; ++u) {
          const int k = sub + kRfLanes * u;
          q += (k > j) ? x[s][u] * x[s][u] : 0.0;
        }
        nc = rf_sum16(q);
      }
      if (sub == 0) {
        sh.cn[c] = nc;
        if (redo) sh.cn0[c] = nc;
      }
    }
  }
}

template <int NS, int NR>
__global__ void __launch_bounds__(kRfThreads) k_row_id_rf(const IdDesc* __restrict__ ids, double tol,
                                                          double abs_tol) {
  constexpr int PM = NS * kRfGroups;
  constexpr int RM = PM < kRfR11 ? PM : kRfR11;
  __shared__ double cn[PM], cn0[PM];
  __shared__ double v[kRfLanes * NR], ej[kRfLanes * NR];
  __shared__ int stp[PM];     // pivot step of column c, -1 while unpivoted
  __shared__ int chosen[PM];  // column pivoted at step j
  __shared__ int lpos[PM];    // rank of an unpivoted column among the unpivoted
  __shared__ double rl[RM * RM];
  __shared__ double sh_vtv, sh_r00;
  __shared__ int sh_piv, sh_stop;
  const RfShared sh{cn, cn0, v, ej, stp, chosen, &sh_vtv};
  const IdDesc D = ids[blockIdx.x];
  const int p = D.p, d = D.d;
  const int t = threadIdx.x;
  const int sub = t % kRfLanes, cg = t / kRfLanes;
  double x[NS][NR];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = cg + kRfGroups * s;
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int k = sub + kRfLanes * u;
      x[s][u] = (c < p && k < d) ? D.phi[c + (int64_t)k * D.ldphi] : 0.0;
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = cg + kRfGroups * s;
    double q = 0.0;
#pragma unroll
    for (int u = 0; u < NR; ++u) q += x[s][u] * x[s][u];
    q = rf_sum16(q);
    if (sub == 0) {
      cn[c] = (c < p) ? q : -1.0;  // -1: not a candidate
      cn0[c] = q;
      stp[c] = -1;
    }
  }
  if (t == 0) sh_r00 = 0.0;
  __syncthreads();
  const int kmax = min(p, d);
  int r = 0;
  for (int j = 0; j < kmax; ++j) {
    // pivot: the largest remaining norm (one wave)
    if (t < 64) {
      double bv = -1.0;
      int bi = 0x7fffffff;
      for (int c = t; c < p; c += 64) {
        const double q = cn[c];
        if (q > bv) {
          bv = q;
          bi = c;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > bv || (ob == bv && oi < bi)) {
          bv = ob;
          bi = oi;
        }
      }
      if (t == 0) {
        const double nrm = sqrt(fmax(bv, 0.0));
        if (j == 0) sh_r00 = nrm;
        sh_piv = bi;
        sh_stop = (bv < 0.0 || sh_r00 == 0.0 || nrm <= fmax(tol * sh_r00, abs_tol)) ? 1 : 0;
      }
    }
    __syncthreads();
    if (sh_stop) break;
    const int piv = sh_piv;
    rf_reflect<NS, NR>(x, sh, piv, j, cg, sub);
    __syncthreads();
    if (sh_vtv > 0.0) {
      rf_update<NS, NR>(x, sh, j, p, cg, sub);
    }
    __syncthreads();
    r = j + 1;
  }
  // R11 (column a = the column pivoted at step a, rows 0..a), in LDS or, past
  // RM pivots, in the work copy
  double* R11 = (r <= RM) ? rl : D.work;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = cg + kRfGroups * s;
    const int a = (c < p) ? stp[c] : -1;
    if (a >= 0) {
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int k = sub + kRfLanes * u;
        if (k <= a) R11[k + (int64_t)a * r] = x[s][u];
      }
    }
  }
  for (int c = t; c < p; c += kRfThreads)
    if (stp[c] < 0) {
      int q = 0;
      for (int c2 = 0; c2 < c; ++c2) q += (stp[c2] < 0) ? 1 : 0;
      lpos[c] = q;
    }
  __syncthreads();
  // T(:, c) = R11^{-1} R12(:, c) for the unpivoted columns, in place in rows
  // 0..r-1 (row a: register a / 16 of lane a % 16); the other slots compute
  // along and are ignored
#pragma unroll
  for (int ua = NR - 1; ua >= 0; --ua) {
    if (kRfLanes * ua >= r) continue;
    for (int sa = kRfLanes - 1; sa >= 0; --sa) {
      const int a = kRfLanes * ua + sa;
      if (a >= r) continue;
      const double inv = 1.0 / R11[a + (int64_t)a * r];
      double ta[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        ta[s] = rf_lane(x[s][ua], sa) * inv;
        if (sub == sa) x[s][ua] = ta[s];
      }
#pragma unroll
      for (int ub = 0; ub <= ua; ++ub) {
        const int b = sub + kRfLanes * ub;
        const double rba = (b < a) ? R11[b + (int64_t)a * r] : 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) x[s][ub] = fma(-rba, ta[s], x[s][ub]);
      }
    }
  }
  // U (p x r): the identity on the pivoted rows, T^T on the others
  double* U = D.U;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = cg + kRfGroups * s;
    if (c < p) {
      const int a0 = stp[c];
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int k = sub + kRfLanes * u;
        if (k < r) U[c + (int64_t)k * p] = (a0 >= 0) ? (k == a0 ? 1.0 : 0.0) : x[s][u];
      }
    }
  }
  for (int a = t; a < r; a += kRfThreads) D.perm[a] = chosen[a];
  for (int c = t; c < p; c += kRfThreads)
    if (stp[c] < 0) D.perm[r + lpos[c]] = c;
  if (t == 0) *D.rank = r;
}

// Forms of the decomposition: 0 the global-memory kernel, then the on-chip
// one by (slots, registers): d <= 192 takes 12 registers per lane (up to 256
// rows of Phi), d <= 256 takes 16 (up to 192 rows).
constexpr int kRfForms = 8;
static int row_id_form(int p, int d) {
  if (d <= 12 * kRfLanes) {
    for (int f = 1; f <= 4; ++f)
      if (p <= 2 * f * kRfGroups) return f;
  } else if (d <= 16 * kRfLanes) {
    for (int f = 5; f <= 7; ++f)
      if (p <= 2 * (f - 4) * kRfGroups) return f;
  }
  return 0;
}

static void launch_row_id(int form, int n, const IdDesc* ids, double tol, double atol, hipStream_t s) {
  if (n <= 0) return;
  switch (form) {
    case 0: hipLaunchKernelGGL(k_row_id, dim3(n), dim3(kIdThreads), 0, s, ids, tol, atol); break;
    case 1: hipLaunchKernelGGL((k_row_id_rf<2, 12>), dim3(n), dim3(kRfThreads), 0, s, ids, tol, atol); break;
    case 2: hipLaunchKernelGGL((k_row_id_rf<4, 12>), dim3(n), dim3(kRfThreads), 0, s, ids, tol, atol); break;
    case 3: hipLaunchKernelGGL((k_row_id_rf<6, 12>), dim3(n), dim3(kRfThreads), 0, s, ids, tol, atol); break;
    case 4: hipLaunchKernelGGL((k_row_id_rf<8, 12>), dim3(n), dim3(kRfThreads), 0, s, ids, tol, atol); break;
    case 5: hipLaunchKernelGGL((k_row_id_rf<2, 16>), dim3(n), dim3(kRfThreads), 0, s, ids, tol, atol); break;
    case 6: hipLaunchKernelGGL((k_row_id_rf<4, 16>), dim3(n), dim3(kRfThreads), 0, s, ids, tol, atol); break;
    default: hipLaunchKernelGGL((k_row_id_rf<6, 16>), dim3(n), dim3(kRfThreads), 0, s, ids, tol, atol); break;
  }
}

// ------------------------------------------------------------ host orchestration

namespace {

struct HNode {
  int lo, hi, c1, c2, level;
  bool leaf;
};

int build_hss_tree(std::vector<HNode>& T, int lo, int hi, int leaf, int level) {
  const int id = (int)T.size();
  T.push_back(HNode{lo, hi, -1, -1, level, hi - lo <= leaf});
  if (hi - lo > leaf) {
    const int mid = lo + (hi - lo) / 2;
    const int a = build_hss_tree(T, lo, mid, leaf, level + 1);
    const int b = build_hss_tree(T, mid, hi, leaf, level + 1);
    T[id].c1 = a;
    T[id].c2 = b;
  }
  return id;
}

// Descriptors of one stage, staged into the device descriptor area and
// uploaded once (kernels of the stage are launched after the upload).
struct Stage {
  char* dev;
  size_t cap;
  std::vector<char> host;
  template <class T>
  const T* push(const std::vector<T>& v) {
    if (v.empty()) return nullptr;
    const size_t at = (host.size() + 255) / 256 * 256;
    host.resize(at + v.size() * sizeof(T));
    std::memcpy(host.data() + at, v.data(), v.size() * sizeof(T));
    return (const T*)(dev + at);
  }
  // 0, kHssGaveUp (descriptor area too small) or PHDC_E_HIP
  int flush(const void* key, hipStream_t s) {
    if (host.empty()) return 0;
    if (host.size() > cap) return kHssGaveUp;
    int rc = hss_upload(key, dev, host, s);
    host.clear();
    return rc;
  }
};

// A batch of independent products, kept ordered by transposition group
// (ta + 2 tb) for vgemm_launch; bound[q] is the first tile of group q.
struct VBatch {
  std::vector<VGemm> g;
  std::vector<int32_t> pf{0};
  int bound[5] = {0, 0, 0, 0, 0};
  static int group(const VGemm& x) { return (x.ta ? 1 : 0) + (x.tb ? 2 : 0); }
  void add(const VGemm& x) {
    if (x.m <= 0 || x.n <= 0) return;
    const int q = group(x);
    size_t pos = 0;
    while (pos < g.size() && group(g[pos]) <= q) ++pos;
    g.insert(g.begin() + pos, x);
    pf.assign(1, 0);
    for (int b = 0; b < 5; ++b) bound[b] = 0;
    for (const VGemm& y : g) {
      pf.push_back(pf.back() + vgemm_tiles(y.m, y.n));
      for (int b = group(y) + 1; b < 5; ++b) bound[b] = pf.back();
    }
  }
};

VGemm mk(const double* A, int64_t lda, int ta, const double* B, int64_t ldb, int tb, double* C, int64_t ldc, int m,
         int n, int k, double alpha, double beta, const int32_t* cmap = nullptr) {
  VGemm g;
  std::memset(&g, 0, sizeof(g));
  g.A = A; g.B = B; g.C = C; g.cmap = cmap;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta;
  g.m = m; g.n = n; g.k = k; g.ta = ta; g.tb = tb;
  return g;
}

}  // namespace

size_t hss_arena_bytes(int64_t m, int64_t K, int leaf, int dmax, bool with_x) {
  if (K <= 0 || m <= 0) return 0;
  std::vector<HNode> T;
  build_hss_tree(T, 0, (int)K, std::max(8, leaf), 0);
  const int64_t pmax = std::max<int64_t>(std::max(8, leaf), 2 * (int64_t)dmax);
  size_t b = 0;
  auto take = [&](int64_t bytes) { b += ((size_t)bytes + 255) / 256 * 256; };
  if (with_x) take(m * K * 8);
  for (int q = 0; q < 4; ++q) take(K * dmax * 8);
  take((int64_t)(2 * T.size() + 2) * 4);
  for (auto& h : T) {
    const int64_t p = h.leaf ? h.hi - h.lo : pmax;
    if (h.leaf) take(p * p * 8);
    for (int q = 0; q < 6; ++q) take(p * dmax * 8);
    for (int q = 0; q < 4; ++q) take((int64_t)dmax * dmax * 8);
    if (!h.leaf) { take((int64_t)dmax * dmax * 8); take((int64_t)dmax * dmax * 8); }
    take(m * dmax * 8);
    take(m * dmax * 8);
    take(p * 4); take(p * 4); take(dmax * 4); take(dmax * 4); take(2 * dmax * 4); take(2 * dmax * 4);
  }
  return b + 4096;
}

__global__ void k_set_int(int32_t* dst, int32_t v) { *dst = v; }

// Compression of the K x K matrix of `src` (Algorithm 1) and the product
// out(:, cmap[j]) = (X A)(:, j) in HSS form (X: m x K, ld ldx; cmap == nullptr:
// column j at out + j ldo).  anorm scales the absolute floor of the ID
// truncation (||A||_2, or an estimate of it).  The largest ID rank goes to
// *rank_dev (device, may be null).  Returns 0, kHssGaveUp or PHDC_E_HIP.
int hss_core(const HssSource& src, int K, int m, const double* X, int64_t ldx, double* out, int64_t ldo,
             const int32_t* cmap, char* arena, size_t arena_bytes, char* descarea, size_t desc_bytes,
             const phdc_opts* o, double anorm, int32_t* rank_dev, const void* work, hipStream_t s) {
  const int leaf = std::max(8, o->hss_leaf);
  const int dmax = std::min(512, std::max(16, o->hss_samples) + 2 * std::max(16, o->hss_samples_inc));
  int d = std::min(std::max(16, o->hss_samples), 512);
  const double* ds = src.ds;
  const double* zh = src.zh;
  const double* dorg = src.dorg;
  const double* tau = src.tau;
  const double* cn = src.cn;
  std::vector<HNode> T;
  build_hss_tree(T, 0, K, leaf, 0);
  const int nn = (int)T.size();
  int maxlevel = 0;
  for (auto& h : T) maxlevel = std::max(maxlevel, h.level);
  const void* key = work;

  for (int attempt = 0; attempt < 3; ++attempt) {
    const int pmax = std::max(leaf, 2 * dmax);
    size_t off = 0;
    auto dtake = [&](int64_t count) {
      double* p = (double*)(arena + off);
      off += ((size_t)count * 8 + 255) / 256 * 256;
      return p;
    };
    auto itake = [&](int64_t count) {
      int32_t* p = (int32_t*)(arena + off);
      off += ((size_t)count * 4 + 255) / 256 * 256;
      return p;
    };
    double* Om1 = dtake((int64_t)K * dmax);
    double* Om2 = dtake((int64_t)K * dmax);
    double* Y = dtake((int64_t)K * dmax);
    double* Z = dtake((int64_t)K * dmax);
    int32_t* ranks = itake(2 * nn + 2);  // [2 i] row-ID rank, [2 i + 1] column-ID rank
    std::vector<double*> Dl(nn, nullptr), Phi(nn), Theta(nn), Wk(nn), Wk2(nn), Ub(nn), Vb(nn), Phisk(nn), Thsk(nn),
        Yhat(nn), Zhat(nn), B1(nn, nullptr), B2(nn, nullptr), Xh(nn), Yh(nn);
    std::vector<int32_t*> permU(nn), permV(nn), skI(nn), skJ(nn), stI(nn), stJ(nn);
    for (int i = 0; i < nn; ++i) {
      const int p = T[i].leaf ? T[i].hi - T[i].lo : pmax;
      if (T[i].leaf) Dl[i] = dtake((int64_t)p * p);
      Phi[i] = dtake((int64_t)p * dmax);
      Theta[i] = dtake((int64_t)p * dmax);
      Wk[i] = dtake((int64_t)p * dmax);
      Wk2[i] = dtake((int64_t)p * dmax);
      Ub[i] = dtake((int64_t)p * dmax);
      Vb[i] = dtake((int64_t)p * dmax);
      Phisk[i] = dtake((int64_t)dmax * dmax);
      Thsk[i] = dtake((int64_t)dmax * dmax);
      Yhat[i] = dtake((int64_t)dmax * dmax);
      Zhat[i] = dtake((int64_t)dmax * dmax);
      if (!T[i].leaf) {
        B1[i] = dtake((int64_t)dmax * dmax);
        B2[i] = dtake((int64_t)dmax * dmax);
      }
      Xh[i] = dtake((int64_t)m * dmax);
      Yh[i] = dtake((int64_t)m * dmax);
      permU[i] = itake(p);
      permV[i] = itake(p);
      skI[i] = itake(dmax);
      skJ[i] = itake(dmax);
      stI[i] = itake(2 * dmax);
      stJ[i] = itake(2 * dmax);
    }
    if (off > arena_bytes) return kHssGaveUp;
    Stage st{descarea, desc_bytes, {}};

    {
      ProfScope ps(PH_HSS_SAMPLE, s);
      const int64_t cnt = (int64_t)K * d;
      const uint64_t sd = o->seed + 0x9e3779b97f4a7c15ULL * (uint64_t)(attempt + 1);
      hipLaunchKernelGGL(k_gauss, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, cnt, sd, Om1);
      hipLaunchKernelGGL(k_gauss, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, cnt, sd ^ 0x5bd1e9955bd1e995ULL,
                         Om2);
      // Y = A Omega1, Z = A^T Omega2; a row-major A read column-major is A^T.
      // The two products (each K/128 x d/128 tiles: too few blocks to fill the
      // GPU alone) run side by side, Z on the auxiliary stream.
      const bool rm = src.sample_row_major;
      GemmArgs gy{src.sample, Om1, src.lds, K, 0, 0, K, d, K, 0};
      GemmArgs gz{src.sample, Om2, src.lds, K, 0, 0, K, d, K, 0};
      struct Events {  // destroyed on every exit (a destroyed event is released once its work completes)
        hipEvent_t fork = nullptr, join = nullptr;
        ~Events() {
          if (fork) (void)hipEventDestroy(fork);
          if (join) (void)hipEventDestroy(join);
        }
      } ev;
      hipStream_t a = aux_stream();
      if (a && (hipEventCreateWithFlags(&ev.fork, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&ev.join, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(ev.fork, s) != hipSuccess || hipStreamWaitEvent(a, ev.fork, 0) != hipSuccess))
        return PHDC_E_HIP;
      gemm_f64(rm, false, gy, 1, Y, K, 0, s);
      gemm_f64(!rm, false, gz, 1, Z, K, 0, a ? a : s);
      if (a && (hipEventRecord(ev.join, a) != hipSuccess || hipStreamWaitEvent(s, ev.join, 0) != hipSuccess))
        return PHDC_E_HIP;
    }

    std::vector<int32_t> hr(2 * nn + 2, 0), hp(2 * nn + 2, 0);
    int maxrank = 0;
    bool too_large = false;
    {
      ProfScope pc(PH_HSS_COMPRESS, s);
      for (int lev = maxlevel; lev >= 0 && !too_large; --lev) {
        std::vector<int> nodes;
        for (int i = 0; i < nn; ++i)
          if (T[i].level == lev) nodes.push_back(i);
        std::vector<UGather> ug;
        std::vector<RowCopy> rc;
        VBatch g1;
        std::vector<IdDesc> idd;
        const bool root_only = (lev == 0 && !T[0].leaf);
        for (int i : nodes) {
          const HNode& h = T[i];
          if (h.leaf) {
            const int p = h.hi - h.lo;
            hp[2 * i] = hp[2 * i + 1] = p;
            ug.push_back(UGather{nullptr, nullptr, Dl[i], p, h.lo, h.lo, p, p});
            rc.push_back(RowCopy{Y + h.lo, nullptr, Phi[i], K, p, p, d, 0, 0});
            rc.push_back(RowCopy{Z + h.lo, nullptr, Theta[i], K, p, p, d, 0, 0});
            g1.add(mk(Dl[i], p, 0, Om1 + h.lo, K, 0, Phi[i], p, p, d, p, -1.0, 1.0));
            g1.add(mk(Dl[i], p, 1, Om2 + h.lo, K, 0, Theta[i], p, p, d, p, -1.0, 1.0));
          } else {
            const int a = h.c1, b = h.c2;
            const int ra = hr[2 * a], rb = hr[2 * b], ca = hr[2 * a + 1], cb = hr[2 * b + 1];
            const int p = ra + rb, q = ca + cb;
            hp[2 * i] = p;
            hp[2 * i + 1] = q;
            // couplings of the children: B1 = Uhat(I_a, J_b), B2 = Uhat(I_b, J_a)
            ug.push_back(UGather{skI[a], skJ[b], B1[i], dmax, 0, 0, ra, cb});
            ug.push_back(UGather{skI[b], skJ[a], B2[i], dmax, 0, 0, rb, ca});
            if (root_only) continue;
            rc.push_back(RowCopy{Phisk[a], nullptr, Phi[i], dmax, p, ra, d, 0, 0});
            rc.push_back(RowCopy{Phisk[b], nullptr, Phi[i], dmax, p, rb, d, ra, 0});
            rc.push_back(RowCopy{Thsk[a], nullptr, Theta[i], dmax, q, ca, d, 0, 0});
            rc.push_back(RowCopy{Thsk[b], nullptr, Theta[i], dmax, q, cb, d, ca, 0});
          }
        }
        // the coupling products need B1/B2 and the stacked rows first: two stages
        const UGather* dug = st.push(ug);
        const RowCopy* drc = st.push(rc);
        const VGemm* dg1 = st.push(g1.g);
        const int32_t* dp1 = st.push(g1.pf);
        if (int rc = st.flush(key, s)) return rc;
        if (dug)
          hipLaunchKernelGGL(k_ugather, dim3((unsigned)ug.size()), dim3(256), 0, s, dug, ds, zh, dorg, tau, cn, src.A,
                             src.lda);
        if (root_only) break;
        if (drc) hipLaunchKernelGGL(k_rows, dim3((unsigned)rc.size()), dim3(256), 0, s, drc);
        if (dg1) vgemm_launch(dg1, dp1, (int)g1.g.size(), g1.bound, s);
        VBatch g2;
        for (int i : nodes) {
          const HNode& h = T[i];
          if (h.leaf) continue;
          const int a = h.c1, b = h.c2;
          const int ra = hr[2 * a], rb = hr[2 * b], ca = hr[2 * a + 1], cb = hr[2 * b + 1];
          const int p = ra + rb, q = ca + cb;
          // Phi rows of a -= B1 Yhat_b, rows of b -= B2 Yhat_a (Algorithm 1)
          g2.add(mk(B1[i], dmax, 0, Yhat[b], dmax, 0, Phi[i], p, ra, d, cb, -1.0, 1.0));
          g2.add(mk(B2[i], dmax, 0, Yhat[a], dmax, 0, Phi[i] + ra, p, rb, d, ca, -1.0, 1.0));
          // Theta rows of a -= B2^T Zhat_b, rows of b -= B1^T Zhat_a
          g2.add(mk(B2[i], dmax, 1, Zhat[b], dmax, 0, Theta[i], q, ca, d, rb, -1.0, 1.0));
          g2.add(mk(B1[i], dmax, 1, Zhat[a], dmax, 0, Theta[i] + ca, q, cb, d, ra, -1.0, 1.0));
        }
        for (int i : nodes) {
          idd.push_back(IdDesc{Phi[i], Wk[i], Ub[i], permU[i], &ranks[2 * i], hp[2 * i], hp[2 * i], d});
          idd.push_back(IdDesc{Theta[i], Wk2[i], Vb[i], permV[i], &ranks[2 * i + 1], hp[2 * i + 1], hp[2 * i + 1], d});
        }
        int cnt[kRfForms], first[kRfForms];
        std::vector<IdDesc> sorted;
        for (int f = 0; f < kRfForms; ++f) {
          first[f] = (int)sorted.size();
          for (const IdDesc& q : idd)
            if (row_id_form(q.p, q.d) == f) sorted.push_back(q);
          cnt[f] = (int)sorted.size() - first[f];
        }
        const VGemm* dg2 = st.push(g2.g);
        const int32_t* dp2 = st.push(g2.pf);
        const IdDesc* did = st.push(sorted);
        if (int rc = st.flush(key, s)) return rc;
        if (dg2) vgemm_launch(dg2, dp2, (int)g2.g.size(), g2.bound, s);
        // each decomposition by the on-chip form for its size, else by the
        // global-memory one (descriptors grouped by form)
        const double atol = o->hss_rel_tol * std::sqrt((double)d) * anorm;
        for (int f = 0; f < kRfForms; ++f) launch_row_id(f, cnt[f], did + first[f], o->hss_rel_tol, atol, s);
        if (hipMemcpyAsync(hr.data(), ranks, hr.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return PHDC_E_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return PHDC_E_HIP;
        for (int i : nodes) {
          maxrank = std::max(maxrank, std::max(hr[2 * i], hr[2 * i + 1]));
          if ((hr[2 * i] >= d - 8 && hr[2 * i] < hp[2 * i]) || (hr[2 * i + 1] >= d - 8 && hr[2 * i + 1] < hp[2 * i + 1]))
            too_large = true;
        }
        if (too_large) break;
        // skeleton rows and indices, nested Yhat / Zhat
        std::vector<RowCopy> rs;
        std::vector<IntCopy> ic;
        std::vector<SkelDesc> sk;
        VBatch g3, g4;
        for (int i : nodes) {
          const HNode& h = T[i];
          const int p = hp[2 * i], q = hp[2 * i + 1], r = hr[2 * i], c = hr[2 * i + 1];
          rs.push_back(RowCopy{Phi[i], permU[i], Phisk[i], p, dmax, r, d, 0, 0});
          rs.push_back(RowCopy{Theta[i], permV[i], Thsk[i], q, dmax, c, d, 0, 0});
          if (h.leaf) {
            sk.push_back(SkelDesc{permU[i], nullptr, skI[i], r, h.lo});
            sk.push_back(SkelDesc{permV[i], nullptr, skJ[i], c, h.lo});
            g3.add(mk(Vb[i], q, 1, Om1 + h.lo, K, 0, Yhat[i], dmax, c, d, q, 1.0, 0.0));
            g3.add(mk(Ub[i], p, 1, Om2 + h.lo, K, 0, Zhat[i], dmax, r, d, p, 1.0, 0.0));
          } else {
            const int a = h.c1, b = h.c2;
            const int ra = hr[2 * a], rb = hr[2 * b], ca = hr[2 * a + 1], cb = hr[2 * b + 1];
            ic.push_back(IntCopy{skI[a], stI[i], ra, 0});
            ic.push_back(IntCopy{skI[b], stI[i], rb, ra});
            ic.push_back(IntCopy{skJ[a], stJ[i], ca, 0});
            ic.push_back(IntCopy{skJ[b], stJ[i], cb, ca});
            sk.push_back(SkelDesc{permU[i], stI[i], skI[i], r, 0});
            sk.push_back(SkelDesc{permV[i], stJ[i], skJ[i], c, 0});
            g3.add(mk(Vb[i], q, 1, Yhat[a], dmax, 0, Yhat[i], dmax, c, d, ca, 1.0, 0.0));
            g4.add(mk(Vb[i] + ca, q, 1, Yhat[b], dmax, 0, Yhat[i], dmax, c, d, cb, 1.0, ca ? 1.0 : 0.0));
            g3.add(mk(Ub[i], p, 1, Zhat[a], dmax, 0, Zhat[i], dmax, r, d, ra, 1.0, 0.0));
            g4.add(mk(Ub[i] + ra, p, 1, Zhat[b], dmax, 0, Zhat[i], dmax, r, d, rb, 1.0, ra ? 1.0 : 0.0));
          }
        }
        const RowCopy* drs = st.push(rs);
        const IntCopy* dic = st.push(ic);
        const SkelDesc* dsk = st.push(sk);
        const VGemm* dg3 = st.push(g3.g);
        const int32_t* dp3 = st.push(g3.pf);
        const VGemm* dg4 = st.push(g4.g);
        const int32_t* dp4 = st.push(g4.pf);
        if (int rc = st.flush(key, s)) return rc;
        hipLaunchKernelGGL(k_rows, dim3((unsigned)rs.size()), dim3(256), 0, s, drs);
        if (dic) hipLaunchKernelGGL(k_ints, dim3((unsigned)ic.size()), dim3(256), 0, s, dic);
        hipLaunchKernelGGL(k_skel, dim3((unsigned)sk.size()), dim3(256), 0, s, dsk);
        if (dg3) vgemm_launch(dg3, dp3, (int)g3.g.size(), g3.bound, s);
        if (dg4) vgemm_launch(dg4, dp4, (int)g4.g.size(), g4.bound, s);
      }
    }
    if (too_large) {
      if (d >= dmax || attempt == 2) return kHssGaveUp;
      d = std::min(dmax, d + std::max(16, o->hss_samples_inc));  // adaptive sampling: more columns, start over
      continue;
    }
    if (rank_dev) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, rank_dev, (int32_t)maxrank);

    // ------------------------------------------------------------ apply out = X A
    ProfScope pa(PH_HSS_APPLY, s);
    // columns t_i of the result: cmap + lo (mapped) or out + lo ldo (plain)
    auto ocols = [&](int lo) { return cmap ? out : out + (int64_t)lo * ldo; };
    auto omap = [&](int lo) { return cmap ? cmap + lo : (const int32_t*)nullptr; };
    std::vector<VBatch> stages;
    {
      VBatch g;
      for (int i = 0; i < nn; ++i) {
        const HNode& h = T[i];
        if (!h.leaf) continue;
        const int p = h.hi - h.lo, r = hr[2 * i];
        if (nn > 1) g.add(mk(X + (int64_t)h.lo * ldx, ldx, 0, Ub[i], p, 0, Xh[i], m, m, r, p, 1.0, 0.0));
        g.add(mk(X + (int64_t)h.lo * ldx, ldx, 0, Dl[i], p, 0, ocols(h.lo), ldo, m, p, p, 1.0, 0.0, omap(h.lo)));
      }
      stages.push_back(g);
    }
    for (int lev = maxlevel - 1; lev >= 1; --lev) {  // up-sweep
      VBatch ga, gb;
      for (int i = 0; i < nn; ++i) {
        const HNode& h = T[i];
        if (h.leaf || h.level != lev) continue;
        const int a = h.c1, b = h.c2, ra = hr[2 * a], rb = hr[2 * b], p = ra + rb, r = hr[2 * i];
        ga.add(mk(Xh[a], m, 0, Ub[i], p, 0, Xh[i], m, m, r, ra, 1.0, 0.0));
        gb.add(mk(Xh[b], m, 0, Ub[i] + ra, p, 0, Xh[i], m, m, r, rb, 1.0, ra ? 1.0 : 0.0));
      }
      stages.push_back(ga);
      stages.push_back(gb);
    }
    {
      VBatch g;  // couplings of every sibling pair
      for (int i = 0; i < nn; ++i) {
        const HNode& h = T[i];
        if (h.leaf) continue;
        const int a = h.c1, b = h.c2, ra = hr[2 * a], rb = hr[2 * b], ca = hr[2 * a + 1], cb = hr[2 * b + 1];
        g.add(mk(Xh[a], m, 0, B1[i], dmax, 0, Yh[b], m, m, cb, ra, 1.0, 0.0));
        g.add(mk(Xh[b], m, 0, B2[i], dmax, 0, Yh[a], m, m, ca, rb, 1.0, 0.0));
      }
      stages.push_back(g);
    }
    for (int lev = 1; lev <= maxlevel - 1; ++lev) {  // down-sweep
      VBatch g;
      for (int i = 0; i < nn; ++i) {
        const HNode& h = T[i];
        if (h.leaf || h.level != lev) continue;
        const int a = h.c1, b = h.c2, ca = hr[2 * a + 1], cb = hr[2 * b + 1], q = ca + cb, c = hr[2 * i + 1];
        if (!c) continue;
        g.add(mk(Yh[i], m, 0, Vb[i], q, 1, Yh[a], m, m, ca, c, 1.0, 1.0));
        g.add(mk(Yh[i], m, 0, Vb[i] + ca, q, 1, Yh[b], m, m, cb, c, 1.0, 1.0));
      }
      stages.push_back(g);
    }
    if (nn > 1) {
      VBatch g;  // leaves: out(:, t) += Yh V^T
      for (int i = 0; i < nn; ++i) {
        const HNode& h = T[i];
        if (!h.leaf) continue;
        const int p = h.hi - h.lo, c = hr[2 * i + 1];
        if (c) g.add(mk(Yh[i], m, 0, Vb[i], p, 1, ocols(h.lo), ldo, m, p, c, 1.0, 1.0, omap(h.lo)));
      }
      stages.push_back(g);
    }
    std::vector<std::pair<const VGemm*, const int32_t*>> dptr;
    for (auto& g : stages) dptr.emplace_back(st.push(g.g), st.push(g.pf));
    if (int rc = st.flush(key, s)) return rc;
    for (size_t q = 0; q < stages.size(); ++q)
      if (!stages[q].g.empty())
        vgemm_launch(dptr[q].first, dptr[q].second, (int)stages[q].g.size(), stages[q].bound, s);
    return 0;
  }
  return kHssGaveUp;
}

// One HSS merge, with K known on the host: X = the merge's input columns of the
// survivors in pole order (rows outside a column's range as 0), A = Uhat
// (normalized, pole order; ||Uhat||_2 = 1), result columns at dest.
int run_hss_merge(const MergeDesc& M, int K, const Scratch& S, char* arena, size_t arena_bytes, char* descarea,
                  size_t desc_bytes, const phdc_opts* o, int32_t* counters_dev, const void* work, hipStream_t s) {
  if (o->force_fail & PHDC_FAIL_HSS) return kHssGaveUp;
  const int m = M.m;
  const int64_t so = M.s_off;
  const size_t xb = ((size_t)m * K * 8 + 255) / 256 * 256;
  if (xb > arena_bytes) return kHssGaveUp;
  double* X = (double*)arena;
  {
    ProfScope ps(PH_HSS_SAMPLE, s);
    hipLaunchKernelGGL(k_gather_x, dim3((m + 255) / 256, K), dim3(256), 0, s, M.qin, M.ldin, m, K, S.csort + so,
                       S.crng + so, X);
  }
  HssSource src{};
  src.ds = S.ds + so;
  src.zh = S.zhat + so;
  src.dorg = S.dorg + so;
  src.tau = S.tau + so;
  src.cn = S.cnorm + so;
  src.A = nullptr;
  src.sample = S.uhat + M.u_off;  // row-major K x K: Uhat(i, j) at i K + j
  src.lds = K;
  src.sample_row_major = true;
  return hss_core(src, K, m, X, m, M.qout, M.ldout, S.dest + so, arena + xb, arena_bytes - xb, descarea, desc_bytes,
                  o, 1.0, counters_dev + C_HSSRANK, work, s);
}

}  // namespace phdc

// ------------------------------------------------------------ dense matrices (Example 1)
namespace phdc {
namespace {

// Squares of column j summed by block j (fixed order: deterministic).
__global__ void __launch_bounds__(256) k_colsq(const double* __restrict__ A, int64_t lda, int K, double* colsq) {
  __shared__ double sh[4];
  const double* a = A + (int64_t)blockIdx.x * lda;
  double v = 0.0;
  for (int i = threadIdx.x; i < K; i += 256) v += a[i] * a[i];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) colsq[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_sum_seq(const double* __restrict__ x, int n, double* out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += x[i];
  *out = s;
}

constexpr size_t kHssDescBytes = (size_t)16 << 20;

struct DenseLayout {
  size_t status, colsq, desc, arena, total;
};

DenseLayout dense_layout(int64_t K, int64_t m, const phdc_opts* o) {
  DenseLayout L;
  size_t p = 0;
  auto take = [&](size_t bytes) {
    size_t at = p;
    p = (p + std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    return at;
  };
  const int dmax = std::min(512, std::max(16, o->hss_samples) + 2 * std::max(16, o->hss_samples_inc));
  L.status = take(256);
  L.colsq = take((size_t)(K + 1) * 8);
  L.desc = take(kHssDescBytes);
  L.arena = take(hss_arena_bytes(m, K, o->hss_leaf, dmax, false));
  L.total = p;
  return L;
}

bool hss_opts_ok(const phdc_opts* o) {
  return o->hss_leaf >= 8 && o->hss_leaf <= kHssLeafMax && o->hss_samples >= 16 && o->hss_samples <= 512 &&
         o->hss_samples_inc >= 0 && o->hss_rel_tol > 0.0 && o->hss_rel_tol < 1.0;
}

}  // namespace
}  // namespace phdc

using namespace phdc;

extern "C" {

int phdc_hss_gemm_workspace(int64_t K, int64_t m, const phdc_opts* o, size_t* bytes) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (K < 1 || K > (1 << 30)) return -1;
  if (m < 1 || m > (1 << 30)) return -2;
  if (!hss_opts_ok(o)) return -3;
  if (!bytes) return -4;
  *bytes = dense_layout(K, m, o).total;
  return 0;
}

int phdc_hss_gemm(int64_t K, const double* A, int64_t lda, int64_t m, const double* X, int64_t ldx, double* C,
                  int64_t ldc, int32_t* rank_host, void* work, size_t lwork, const phdc_opts* o, void* stream) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (K < 1 || K > (1 << 30)) return -1;
  if (!A) return -2;
  if (lda < K) return -3;
  if (m < 1 || m > (1 << 30)) return -4;
  if (!X) return -5;
  if (ldx < m) return -6;
  if (!C) return -7;
  if (ldc < m) return -8;
  if (!work || ((uintptr_t)work & 255) != 0) return -10;
  if (!hss_opts_ok(o)) return -12;
  const DenseLayout L = dense_layout(K, m, o);
  if (lwork < L.total) return -11;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)work;
  int32_t* status = (int32_t*)(base + L.status);
  double* colsq = (double*)(base + L.colsq);
  launch_clear_status(status, s);
  // ||A||_F / sqrt(K) (= 1 for an orthogonal A) scales the truncation floor
  hipLaunchKernelGGL(k_colsq, dim3((unsigned)K), dim3(256), 0, s, A, lda, (int)K, colsq);
  hipLaunchKernelGGL(k_sum_seq, dim3(1), dim3(64), 0, s, colsq, (int)K, colsq + K);
  double fro2 = 0.0;
  if (hipMemcpyAsync(&fro2, colsq + K, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return PHDC_E_HIP;
  const double anorm = std::sqrt(fro2 / (double)K);
  HssSource src{};
  src.A = A;
  src.lda = lda;
  src.sample = A;
  src.lds = lda;
  src.sample_row_major = false;
  int32_t* rank_dev = status + 8;
  int rc = (o->force_fail & PHDC_FAIL_HSS)
               ? kHssGaveUp
               : hss_core(src, (int)K, (int)m, X, ldx, C, ldc, nullptr, base + L.arena, L.total - L.arena,
                          base + L.desc, kHssDescBytes, o, anorm, rank_dev, work, s);
  if (rc == PHDC_E_HIP) return rc;
  int32_t rank = -1;
  if (rc == 0) {
    if (hipMemcpyAsync(&rank, rank_dev, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return PHDC_E_HIP;
  } else {  // the compression gave up: dense FP64 product
    ProfScope pa(PH_HSS_APPLY, s);
    GemmArgs g{X, A, ldx, lda, 0, 0, (int32_t)m, (int32_t)K, (int32_t)K, 0};
    gemm_f64(false, false, g, 1, C, ldc, 0, s);
  }
  if (rank_host) *rank_host = rank;
  return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
}

}  // extern "C"
