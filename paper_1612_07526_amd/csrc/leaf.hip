// Leaf eigensolves of the divide-and-conquer tree: one 64-lane wavefront per
// leaf (at most 64 rows), implicit QL with a Wilkinson shift.
//
// The paper leaves the leaf solver to ScaLAPACK; any exact symmetric
// tridiagonal eigensolver is a correct leaf.  Before solving, the leaf's first
// and last diagonal entries lose |e| of the coupling that the Cuppen split
// (Eq. (2)) removed on that side.
#include "phdc_internal.h"

namespace phdc {

// Z is stored column-major in LDS (column c at Z[c * kMaxLeaf]); lane t owns row t.
__global__ void __launch_bounds__(64) k_leaf_ql(const LeafArgs* __restrict__ leaves, int32_t* status) {
  __shared__ double sd[kMaxLeaf];
  __shared__ double se[kMaxLeaf];
  __shared__ double Z[kMaxLeaf * kMaxLeaf];
  const LeafArgs L = leaves[blockIdx.x];
  const int s = L.s;
  const int t = threadIdx.x;
  if (s <= 0) return;
  for (int c = 0; c < s; ++c) Z[c * kMaxLeaf + t] = (c == t) ? 1.0 : 0.0;
  if (t < s) {
    sd[t] = L.d[t];
    se[t] = (t < s - 1) ? L.e[t] : 0.0;
  }
  __syncthreads();
  // Corner updates of the split (the first/last row lost |e| of the removed coupling).
  double cl = (L.couple & 1) ? fabs(L.e[-1]) : 0.0;
  double cr = (L.couple & 2) ? fabs(L.e[s - 1]) : 0.0;
  __syncthreads();
  if (t == 0) {
    sd[0] -= cl;
    sd[s - 1] -= cr;
  }
  __syncthreads();

  // Every lane runs the scalar recurrence redundantly (uniform control flow);
  // only the eigenvector rotations are lane-parallel.
  bool failed = false;
  for (int l = 0; l < s && !failed; ++l) {
    int iter = 0;
    for (;;) {
      // First negligible off-diagonal entry at or below row l splits the matrix.
      int mm = l;
      while (mm < s - 1) {
        double dd = fabs(sd[mm]) + fabs(sd[mm + 1]);
        if (fabs(se[mm]) <= kUnitRoundoff * dd) break;
        ++mm;
      }
      if (mm == l) break;
      if (++iter > 64) {
        failed = true;
        break;
      }
      // Shift: the eigenvalue of the leading 2x2 block [d_l e_l; e_l d_{l+1}]
      // nearer d_l, folded into the starting value g of the bulge chase.
      double g = (sd[l + 1] - sd[l]) / (2.0 * se[l]);
      double r = hypot(g, 1.0);
      g = sd[mm] - sd[l] + se[l] / (g + copysign(r, g));
      double sn = 1.0, cs = 1.0, p = 0.0;
      bool restart = false;
      // Chase the bulge from the bottom of the unreduced block up to row l,
      // one plane rotation in rows/columns (i, i+1) at a time.
      for (int i = mm - 1; i >= l; --i) {
        double f = sn * se[i];
        double b = cs * se[i];
        r = hypot(f, g);
        __syncthreads();
        if (t == 0) se[i + 1] = r;
        __syncthreads();
        if (r == 0.0) {
          // The rotation underflowed: the block has split at i+1; undo the
          // pending shift correction and look for the split again.
          if (t == 0) {
            sd[i + 1] -= p;
            se[mm] = 0.0;
          }
          __syncthreads();
          restart = true;
          break;
        }
        sn = f / r;
        cs = g / r;
        g = sd[i + 1] - p;
        r = (sd[i] - g) * sn + 2.0 * cs * b;
        p = sn * r;
        __syncthreads();
        if (t == 0) sd[i + 1] = g + p;
        g = cs * r - b;
        if (t < s) {
          double zi = Z[i * kMaxLeaf + t];
          double zj = Z[(i + 1) * kMaxLeaf + t];
          Z[(i + 1) * kMaxLeaf + t] = sn * zi + cs * zj;
          Z[i * kMaxLeaf + t] = cs * zi - sn * zj;
        }
        __syncthreads();
      }
      if (restart) continue;
      __syncthreads();
      if (t == 0) {
        sd[l] -= p;
        se[l] = g;
        se[mm] = 0.0;
      }
      __syncthreads();
    }
  }
  if (failed) {
    if (t == 0) set_status(status, PHDC_ERR_LEAF);
  }
  __syncthreads();
  // Selection sort into ascending order, moving eigenvector columns along.
  for (int i = 0; i < s - 1; ++i) {
    int best = i;
    double bv = sd[i];
    for (int j = i + 1; j < s; ++j)
      if (sd[j] < bv) {
        bv = sd[j];
        best = j;
      }
    if (best != i) {
      __syncthreads();
      double a = sd[i];
      if (t < s) {
        double zi = Z[i * kMaxLeaf + t];
        Z[i * kMaxLeaf + t] = Z[best * kMaxLeaf + t];
        Z[best * kMaxLeaf + t] = zi;
      }
      __syncthreads();
      if (t == 0) {
        sd[i] = bv;
        sd[best] = a;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (t < s) {
    L.lam[t] = sd[t];
    for (int c = 0; c < s; ++c) L.q[t + (int64_t)c * L.ldq] = Z[c * kMaxLeaf + t];
  }
}

void launch_leaf_ql(const LeafArgs* leaves, int nleaves, int32_t* status, hipStream_t s) {
  if (nleaves <= 0) return;
  hipLaunchKernelGGL(k_leaf_ql, dim3(nleaves), dim3(64), 0, s, leaves, status);
}

}  // namespace phdc
