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

// Leaves of at most LG rows (LG = 8 or 16): LG lanes per leaf, 64 / LG leaves
// per wavefront.  Lane t of a group owns row t of the leaf's eigenvector matrix
// Z in registers (z[c] = Z(t, c)), so the rotation of columns (i, i+1) is two
// multiply-adds per lane with no communication.  d and e sit in LDS, one copy
// per group, and every lane of the group runs the same scalar recurrence on
// broadcast reads; lanes of one group compute bit-identical values, so each
// lane's reads follow its own writes.  The sweep is unrolled over i with the
// step taken under the mask l <= i < mm: groups in different states share one
// instruction stream, and a step that no group of the wave needs is branched
// over.  The whole iteration (find the unreduced block, shift, sweep) is one
// loop per group, so a group does not wait for the others between eigenvalues.
struct alignas(16) LeafDE {
  double d, e;
};

template <int LG>
__global__ void __launch_bounds__(64) k_leaf_ql_grouped(const LeafArgs* __restrict__ leaves, int nleaves,
                                                        int32_t* status, int maxit) {
  constexpr int GPW = 64 / LG;  // leaves per wavefront (= per block)
  __shared__ LeafDE desh[GPW][LG + 1];
  __shared__ int rsh[GPW][LG];
  const int gi = threadIdx.x / LG;
  const int t = threadIdx.x % LG;
  const int li = blockIdx.x * GPW + gi;
  if (li >= nleaves) return;  // whole group; no block barrier below
  const LeafArgs L = leaves[li];
  const int s = L.s;
  if (s <= 0 || s > LG) return;
  LeafDE* de = desh[gi];
  {
    double dv = 0.0, ev = 0.0;
    if (t < s) {
      dv = L.d[t];
      if (t == 0 && (L.couple & 1)) dv -= fabs(L.e[-1]);
      if (t == s - 1 && (L.couple & 2)) dv -= fabs(L.e[s - 1]);
      ev = (t < s - 1) ? L.e[t] : 0.0;
    }
    de[t] = LeafDE{dv, ev};
    if (t == 0) de[LG] = LeafDE{0.0, 0.0};
  }
  __builtin_amdgcn_wave_barrier();
  double z[LG];
#pragma unroll
  for (int c = 0; c < LG; ++c) z[c] = (c == t) ? 1.0 : 0.0;
  const int gshift = gi * LG;
  constexpr unsigned long long gmask = (1ull << LG) - 1;
  int l = 0, iter = 0;
  bool failed = false;
  for (;;) {
    // Bit k of U: row k < s-1 is still coupled to row k+1 (|e_k| above the
    // negligibility threshold).
    const double dk = de[t].d, ek = de[t].e, dk1 = de[t + 1].d;
    const bool coupled = t < s - 1 && !(fabs(ek) <= kUnitRoundoff * (fabs(dk) + fabs(dk1)));
    const unsigned U = (unsigned)((__ballot(coupled) >> gshift) & gmask);
    const unsigned rem = U & (~0u << l);
    if (rem == 0) break;  // every eigenvalue of the leaf has converged
    const int nl = __builtin_ctz(rem);
    if (nl != l) {
      l = nl;
      iter = 0;
    }
    // The unreduced block is rows l..mm.
    const int mm = __builtin_ctz(~U & (~0u << l));
    if (++iter > maxit) {
      failed = true;
      break;
    }
    // Shift: the eigenvalue of [d_l e_l; e_l d_{l+1}] nearer d_l, folded into
    // the starting value g of the bulge chase.
    const double dl = de[l].d, el = de[l].e;
    const double dmm = de[mm].d;
    double g = (de[l + 1].d - dl) / (2.0 * el);
    double r = hyp(g, 1.0);
    g = dmm - dl + el / (g + copysign(r, g));
    double sn = 1.0, cs = 1.0, p = 0.0;
    double dnext = dmm;  // d_{i+1} as it was before this sweep
    bool live = true;    // false once a rotation underflows
#pragma unroll
    for (int i = LG - 2; i >= 0; --i) {
      const LeafDE cur = de[i];  // untouched by this sweep so far
      if (live && i >= l && i < mm) {
        const double f = sn * cur.e, b = cs * cur.e;
        double c2 = 1.0, s2 = 0.0;
        const double rr = rotation(f, g, &c2, &s2);
        if (rr == 0.0) {
          // The block has split at i+1: undo the pending shift correction and
          // look for the split again (e_mm is cleared after the sweep).
          de[i + 1] = LeafDE{dnext - p, 0.0};
          live = false;
        } else {
          sn = s2;
          cs = c2;
          g = dnext - p;
          r = (cur.d - g) * sn + 2.0 * cs * b;
          p = sn * r;
          de[i + 1] = LeafDE{g + p, rr};
          g = cs * r - b;
          const double zi = z[i], zj = z[i + 1];
          z[i + 1] = sn * zi + cs * zj;
          z[i] = cs * zi - sn * zj;
        }
        dnext = cur.d;
      }
    }
    if (live) {
      de[l].d = de[l].d - p;
      de[l].e = g;
    }
    de[mm].e = 0.0;
  }
  if (failed && t == 0) set_status(status, PHDC_ERR_LEAF);
  // Ascending order: rank of each eigenvalue (ties by index); column c of Z
  // goes to output column rank(c).
  const double dt = de[t].d;
  int rank = 0;
#pragma unroll
  for (int j = 0; j < LG; ++j) {
    const double dj = de[j].d;
    rank += (j < s && (dj < dt || (dj == dt && j < t))) ? 1 : 0;
  }
  rsh[gi][t] = rank;
  __builtin_amdgcn_wave_barrier();
  if (t < s) {
    L.lam[rank] = dt;
#pragma unroll
    for (int c = 0; c < LG; ++c)
      if (c < s) L.q[t + (int64_t)rsh[gi][c] * L.ldq] = z[c];
    if (L.rng) L.rng[t] = RowRange{L.r0, L.r0 + s};
  }
}

void launch_leaf_ql(const LeafArgs* leaves, int nleaves, int32_t* status, int max_leaf, int maxit, hipStream_t s) {
  if (nleaves <= 0) return;
  if (max_leaf <= 8) {
    hipLaunchKernelGGL(k_leaf_ql_grouped<8>, dim3((nleaves + 7) / 8), dim3(64), 0, s, leaves, nleaves, status, maxit);
    return;
  }
  if (max_leaf <= 16) {
    hipLaunchKernelGGL(k_leaf_ql_grouped<16>, dim3((nleaves + 3) / 4), dim3(64), 0, s, leaves, nleaves, status, maxit);
    return;
  }
  const int ls = std::max(1, std::min(max_leaf, kMaxLeaf));
  const int blocks = (nleaves + kLeavesPerBlock - 1) / kLeavesPerBlock;
  hipLaunchKernelGGL(k_leaf_ql, dim3(blocks), dim3(64 * kLeavesPerBlock),
                     (size_t)kLeavesPerBlock * ls * ls * sizeof(double), s, leaves, nleaves, status, ls, maxit);
}

}  // namespace phdc
