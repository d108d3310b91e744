// Leaf eigensolves of the divide-and-conquer tree: one 64-lane wavefront per
// leaf (at most 64 rows), implicit QL with a Wilkinson shift.
//
// The paper leaves the leaf solver to ScaLAPACK; any exact symmetric
// tridiagonal eigensolver is a correct leaf.  Before solving, the leaf's first
// and last diagonal entries lose |e| of the coupling that the Cuppen split
// (Eq. (2)) removed on that side.
//
// Layout on the wavefront: lane t holds d_t and e_t in registers; the scalar
// recurrence of the bulge chase is computed identically by every lane, reading
// the entry it needs with a lane read and writing it back with a lane select
// (no LDS round trip on the critical path).  The eigenvector matrix Z sits in
// LDS, column-major, and lane t owns row t of it, so the rotations need no
// communication between lanes and no barrier.
#include <algorithm>

#include "phdc_internal.h"

namespace phdc {

namespace {

__device__ inline double lane_get(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double lane_put(double old, double v, int lane) {
  return (int)(threadIdx.x & 63) == lane ? v : old;
}

// sqrt(a^2 + b^2); the plain form is exact to rounding inside [1e-150, 1e150],
// the scaled library routine covers the rest.
__device__ inline double hyp(double a, double b) {
  const double mx = fmax(fabs(a), fabs(b));
  if (mx > 1e150 || mx < 1e-150) return hypot(a, b);
  return sqrt(a * a + b * b);
}

// Plane rotation with r = sqrt(f^2 + g^2), c = g / r, s = f / r (c, s unused
// when r == 0).  Inside [1e-150, 1e150] the reciprocal square root of
// f^2 + g^2 comes from the hardware estimate and two Newton steps
// y <- y (3/2 - (x/2) y^2), which leaves a few ulps; outside, the scaled
// library hypot and a division.
__device__ inline double rotation(double f, double g, double* c, double* s) {
  const double mx = fmax(fabs(f), fabs(g));
  if (mx > 1e150 || mx < 1e-150) {
    const double r = hypot(f, g);
    if (r != 0.0) {
      const double ri = 1.0 / r;
      *c = g * ri;
      *s = f * ri;
    }
    return r;
  }
  const double x = fma(f, f, g * g);
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  *c = g * y;
  *s = f * y;
  return x * y;
}

}  // namespace

// Each wavefront of a block solves one leaf; a block holds kLeavesPerBlock of
// them, so that the waves of a launch spread over the SIMDs of every CU (one
// 64-thread block per leaf stacks several waves on one SIMD).  Z is ls x ls in
// dynamic LDS per wave (ls = the largest leaf of the launch).
constexpr int kLeavesPerBlock = 4;

__global__ void __launch_bounds__(64 * kLeavesPerBlock) k_leaf_ql(const LeafArgs* __restrict__ leaves, int nleaves,
                                                                   int32_t* status, int ls, int maxit) {
  HIP_DYNAMIC_SHARED(double, Zall)
  const int wv = threadIdx.x >> 6;
  const int li = blockIdx.x * kLeavesPerBlock + wv;
  if (li >= nleaves) return;  // whole wave: no barrier below
  double* Z = Zall + (size_t)wv * ls * ls;
  const LeafArgs L = leaves[li];
  const int s = L.s;
  const int t = threadIdx.x & 63;
  if (s <= 0 || s > ls) return;
  const bool row = t < s;  // lane t owns row t of Z
  if (row)
    for (int c = 0; c < s; ++c) Z[c * ls + t] = (c == t) ? 1.0 : 0.0;
  // Corner updates of the split: the first/last row lost |e| of the removed coupling.
  double d = 0.0, e = 0.0;
  if (t < s) {
    d = L.d[t];
    if (t == 0 && (L.couple & 1)) d -= fabs(L.e[-1]);
    if (t == s - 1 && (L.couple & 2)) d -= fabs(L.e[s - 1]);
    e = (t < s - 1) ? L.e[t] : 0.0;
  }

  bool failed = false;
  for (int l = 0; l < s && !failed; ++l) {
    int iter = 0;
    for (;;) {
      // First negligible off-diagonal entry at or below row l splits the matrix
      // (row s-1 always ends it).
      const double dn = __shfl(d, (t + 1) & 63);
      const bool split = t >= l && t < s && (t == s - 1 || fabs(e) <= kUnitRoundoff * (fabs(d) + fabs(dn)));
      const int mm = __ffsll((unsigned long long)__ballot(split)) - 1;
      if (mm == l) break;
      if (++iter > maxit) {
        failed = true;
        break;
      }
      // Shift: the eigenvalue of the leading 2x2 block [d_l e_l; e_l d_{l+1}]
      // nearer d_l, folded into the starting value g of the bulge chase.
      const double dl = lane_get(d, l), el = lane_get(e, l);
      double g = (lane_get(d, l + 1) - dl) / (2.0 * el);
      double r = hyp(g, 1.0);
      g = lane_get(d, mm) - dl + el / (g + copysign(r, g));
      double sn = 1.0, cs = 1.0, p = 0.0;
      bool restart = false;
      // Chase the bulge from the bottom of the unreduced block up to row l,
      // one plane rotation in rows/columns (i, i+1) at a time.  Column i+1 of
      // Z is final after step i; column i is carried to the next step in a
      // register (zj), so each step reads one untouched column from LDS.
      double zj = row ? Z[mm * ls + t] : 0.0;
      for (int i = mm - 1; i >= l; --i) {
        const double zi = row ? Z[i * ls + t] : 0.0;
        const double ei = lane_get(e, i);
        const double f = sn * ei;
        const double b = cs * ei;
        double c2 = 1.0, s2 = 0.0;
        r = rotation(f, g, &c2, &s2);
        e = lane_put(e, r, i + 1);
        const double di1 = lane_get(d, i + 1);
        if (r == 0.0) {
          // The rotation underflowed: the block has split at i+1; undo the
          // pending shift correction and look for the split again.
          d = lane_put(d, di1 - p, i + 1);
          e = lane_put(e, 0.0, mm);
          if (row) Z[(i + 1) * ls + t] = zj;
          restart = true;
          break;
        }
        sn = s2;
        cs = c2;
        g = di1 - p;
        r = (lane_get(d, i) - g) * sn + 2.0 * cs * b;
        p = sn * r;
        d = lane_put(d, g + p, i + 1);
        g = cs * r - b;
        if (row) Z[(i + 1) * ls + t] = sn * zi + cs * zj;
        zj = cs * zi - sn * zj;
      }
      if (restart) continue;
      if (row) Z[l * ls + t] = zj;
      d = lane_put(d, lane_get(d, l) - p, l);
      e = lane_put(e, g, l);
      e = lane_put(e, 0.0, mm);
    }
  }
  if (failed && t == 0) set_status(status, PHDC_ERR_LEAF);
  // Ascending order: rank of each eigenvalue (ties by index), then column c of
  // Z goes to output column rank(c).
  int rank = 0;
  for (int j = 0; j < s; ++j) {
    const double dj = lane_get(d, j);
    rank += (dj < d || (dj == d && j < t)) ? 1 : 0;
  }
  if (row) L.lam[rank] = d;
  for (int c = 0; c < s; ++c) {
    const int rc = __builtin_amdgcn_readlane(rank, c);
    if (row) L.q[t + (int64_t)rc * L.ldq] = Z[c * ls + t];
  }
  if (row && L.rng) L.rng[t] = RowRange{L.r0, L.r0 + s};  // every column spans the leaf's rows
}

void launch_leaf_ql(const LeafArgs* leaves, int nleaves, int32_t* status, int max_leaf, int maxit, hipStream_t s) {
  if (nleaves <= 0) return;
  const int ls = std::max(1, std::min(max_leaf, kMaxLeaf));
  const int blocks = (nleaves + kLeavesPerBlock - 1) / kLeavesPerBlock;
  hipLaunchKernelGGL(k_leaf_ql, dim3(blocks), dim3(64 * kLeavesPerBlock),
                     (size_t)kLeavesPerBlock * ls * ls * sizeof(double), s, leaves, nleaves, status, ls, maxit);
}

}  // namespace phdc
