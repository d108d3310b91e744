// Leaf eigensolves of the divide-and-conquer tree: one 64-lane wavefront per
// leaf (at most 64 rows), implicit QL with a Wilkinson shift.
//
// The paper leaves the leaf solver to ScaLAPACK; any exact symmetric
// tridiagonal eigensolver is a correct leaf.  Before solving, the leaf's first
// and last diagonal entries lose |e| of the coupling that the Cuppen split
// (Eq. (2)) removed on that side.
#include "phdc_internal.h"

namespace phdc {

// Z is stored column-major in LDS (column c at Z[c * kMaxLeaf]); lane t owns
// row t.  The block is a single wavefront: every lane runs the scalar QL
// recurrence redundantly and stores the same values to LDS, so no barrier is
// needed (LDS instructions of one wavefront complete in program order); only
// the eigenvector rotations are lane-parallel.
// Store of a value every lane computed identically.  The wave barriers only
// keep the compiler from moving other LDS accesses across the store; on the
// hardware the lanes of a wavefront are in lockstep anyway.
__device__ inline void lockstep_store(double* a, double v) {
  __builtin_amdgcn_wave_barrier();
  *a = v;
  __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(64) k_leaf_ql(const LeafArgs* __restrict__ leaves, int32_t* status) {
  __shared__ double sd[kMaxLeaf];
  __shared__ double se[kMaxLeaf];
  __shared__ double Z[kMaxLeaf * kMaxLeaf];
  const LeafArgs L = leaves[blockIdx.x];
  const int s = L.s;
  const int t = threadIdx.x;
  if (s <= 0) return;
  for (int c = 0; c < s; ++c) Z[c * kMaxLeaf + t] = (c == t) ? 1.0 : 0.0;
  // Corner updates of the split: the first/last row lost |e| of the removed coupling.
  const double cl = (L.couple & 1) ? fabs(L.e[-1]) : 0.0;
  const double cr = (L.couple & 2) ? fabs(L.e[s - 1]) : 0.0;
  for (int i = 0; i < s; ++i) {
    double di = L.d[i];
    if (i == 0) di -= cl;
    if (i == s - 1) di -= cr;
    lockstep_store(&sd[i], di);
    lockstep_store(&se[i], (i < s - 1) ? L.e[i] : 0.0);
  }

  bool failed = false;
  for (int l = 0; l < s && !failed; ++l) {
    int iter = 0;
    for (;;) {
      // First negligible off-diagonal entry at or below row l splits the matrix.
      int mm = l;
      while (mm < s - 1) {
        const double dd = fabs(sd[mm]) + fabs(sd[mm + 1]);
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
        const double f = sn * se[i];
        const double b = cs * se[i];
        r = hypot(f, g);
        lockstep_store(&se[i + 1], r);
        if (r == 0.0) {
          // The rotation underflowed: the block has split at i+1; undo the
          // pending shift correction and look for the split again.
          lockstep_store(&sd[i + 1], sd[i + 1] - p);
          lockstep_store(&se[mm], 0.0);
          restart = true;
          break;
        }
        sn = f / r;
        cs = g / r;
        g = sd[i + 1] - p;
        r = (sd[i] - g) * sn + 2.0 * cs * b;
        p = sn * r;
        lockstep_store(&sd[i + 1], g + p);
        g = cs * r - b;
        if (t < s) {
          const double zi = Z[i * kMaxLeaf + t];
          const double zj = Z[(i + 1) * kMaxLeaf + t];
          Z[(i + 1) * kMaxLeaf + t] = sn * zi + cs * zj;
          Z[i * kMaxLeaf + t] = cs * zi - sn * zj;
        }
      }
      if (restart) continue;
      lockstep_store(&sd[l], sd[l] - p);
      lockstep_store(&se[l], g);
      lockstep_store(&se[mm], 0.0);
    }
  }
  if (failed && t == 0) set_status(status, PHDC_ERR_LEAF);
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
      const double a = sd[i];
      if (t < s) {
        const double zi = Z[i * kMaxLeaf + t];
        Z[i * kMaxLeaf + t] = Z[best * kMaxLeaf + t];
        Z[best * kMaxLeaf + t] = zi;
      }
      lockstep_store(&sd[i], bv);
      lockstep_store(&sd[best], a);
    }
  }
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
