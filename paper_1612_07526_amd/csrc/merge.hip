// Merge step of the divide-and-conquer eigensolver (Sec. 1, Eq. (3)-(6)):
// deflation, secular roots, Loewner z, the eigenvector matrix Uhat, the final
// ordering and the copy of deflated columns.  All merges of one level run in
// one launch per kernel; every kernel reads the data-dependent sizes (K, type
// counts) from device counters, so no host round trip is needed.
#include "phdc_internal.h"
#include "profile.h"
#include "split.h"

namespace phdc {

__device__ inline int cdiv_d(int a, int b) { return (a + b - 1) / b; }

// ------------------------------------------------------------ block utilities

template <int NT>
__device__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < NT / 64; ++i) r += sh[i];  // fixed order: deterministic
  return r;
}

template <int NT>
__device__ double block_max(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < NT / 64; ++i) r = fmax(r, sh[i]);
  return r;
}

// Exclusive scan of a 64-bit value over the block (used with packed counters).
template <int NT>
__device__ int64_t block_excl_scan(int64_t x, int64_t* total, int64_t* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t v = x;
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  __syncthreads();
  if (lane == 63) sh[w] = v;
  __syncthreads();
  int64_t before = 0, tot = 0;
  for (int i = 0; i < NT / 64; ++i) {
    if (i < w) before += sh[i];
    tot += sh[i];
  }
  *total = tot;
  return before + v - x;
}

// # of a[0:n) strictly below x / at most x (a ascending).
__device__ inline int count_lt(const double* a, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ inline int count_le(const double* a, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Type-2 deflation test for consecutive survivors p < j (Sec. 1, after Remark 1):
// the rotation that zeroes z_p leaves the off-diagonal residue (d_j - d_p) c s.
__device__ inline bool pair_deflates(double dp, double zp, double dj, double zj, double tol, double* c,
                                     double* s, double* tau) {
  double t = hypot(zp, zj);
  *c = zj / t;
  *s = -zp / t;
  *tau = t;
  return fabs((dj - dp) * (*c) * (*s)) <= tol;
}

// ------------------------------------------------------------ deflation
// One workgroup per merge (1024 threads; 256 on levels whose merges have at
// most kDefSmall rows).  The compactions in pole order give
// each wave a contiguous index segment and place elements with ballots, so a
// pass over m costs two block barriers however large m is.  The merge-path
// searches of step 2 read D from LDS when the level's merges fit
// (kDefLdsMax poles, dynamic LDS sized per launch).
constexpr int kDefThreads = 1024;
constexpr int kDefWaves = kDefThreads / 64;
constexpr int kDefLdsMax = 16384;
constexpr int kDefSmall = 256;

__device__ inline int lanes_below(uint64_t mask) {
  return __popcll(mask & ((1ULL << (threadIdx.x & 63)) - 1ULL));
}

// Sum over lanes 0..15 (lanes 16..63 hold 0), broadcast to the whole wave.
__device__ inline int sum16_bcast(int v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return __shfl(v, 0, 64);
}

// Exclusive prefix over the NW waves of the block of NC per-wave counts, and
// the block totals; lane i of every wave reads wave i's count.  Uses sh[NC][kDefWaves].
template <int NC, int NW>
__device__ inline void wave_prefix(const int (&c)[NC], int (&pre)[NC], int (&tot)[NC], int (*sh)[kDefWaves]) {
  static_assert(NW <= 16, "sum16_bcast covers 16 waves");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NC; ++q) sh[q][w] = c[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int v = (lane < NW) ? sh[q][lane] : 0;
    tot[q] = sum16_bcast(v);
    pre[q] = sum16_bcast(lane < w ? v : 0);
  }
}

// Steps 1 and 2 of the deflation below for merges of at least kDefPrepRows
// rows, one element per thread over many workgroups (one workgroup per merge
// spends most of its time on these two steps' memory round trips): the row
// range, the z entry, the sortedness check and the merged position of every
// element.  z is written unnormalised; each block leaves its partial |z|^2,
// max |D| and sortedness flags in the merge's slot of tau, dorg and org, which
// the secular roots overwrite only later.  If the runs are not ascending the
// positions may collide: the deflation kernel then places every element again.
constexpr int kPrepThreads = 256;

template <int NT>
__device__ double block_sum(double v, double* sh);
template <int NT>
__device__ double block_max(double v, double* sh);

__global__ void __launch_bounds__(kPrepThreads) k_deflate_prep(BlockMap bm, Scratch S) {
  __shared__ double shd[kPrepThreads / 64];
  __shared__ int shu;
  const int mi = find_merge(bm, blockIdx.x);
  const int lb = blockIdx.x - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int m = M.m, n1 = M.n1, t = threadIdx.x;
  const int64_t so = M.s_off;
  double zsign = M.zsign;
  if (M.ecoup != nullptr) zsign = (*M.ecoup < 0.0) ? -1.0 : 1.0;
  const int i = lb * kPrepThreads + t;
  double zi = 0.0, di = 0.0;
  int uns = 0;
  if (i < m) {
    RowRange g = (i < n1) ? RowRange{0, n1} : RowRange{n1, m};
    if (M.rin) g = RowRange{M.rin[i].lo - M.r0, M.rin[i].hi - M.r0};
    S.crng[so + i] = g;
    const int zr = (i < n1) ? n1 - 1 : n1;
    if (M.zgiven) zi = M.zgiven[i];
    else if (zr >= g.lo && zr < g.hi) zi = ((i < n1) ? 1.0 : zsign) * M.qin[zr + (int64_t)i * M.ldin];
    di = M.lin[i];
    const double dprev = (i > 0) ? M.lin[i - 1] : 0.0;
    S.zs[so + i] = zi;
    if (!isfinite(di)) uns = 2;
    else if (i > 0 && i != n1 && !(di >= dprev)) uns = 1;
    const int pos = (i < n1) ? i + count_lt(M.lin + n1, m - n1, di) : (i - n1) + count_le(M.lin, n1, di);
    S.dv[so + pos] = di;
    S.zv[so + pos] = zi;
    S.col[so + pos] = i;
    S.part[so + pos] = (i < n1) ? 1 : 3;
  }
  const double zzb = block_sum<kPrepThreads>(zi * zi, shd);
  const double dmb = block_max<kPrepThreads>(fabs(di), shd);
  if (t == 0) shu = 0;
  __syncthreads();
  if (uns) atomicOr(&shu, uns);
  __syncthreads();
  if (t == 0) {
    S.tau[so + lb] = zzb;
    S.dorg[so + lb] = dmb;
    S.org[so + lb] = shu;
  }
}

// The partial |z|^2, max |D| and sortedness flags of k_deflate_prep's blocks,
// combined by wave 0 in one fixed order, so that every kernel that combines
// them gets the same bits; sh2 and shu are LDS scratch.  All threads call it.
__device__ void prep_totals(const MergeDesc& M, const Scratch& S, double* sh2, int* shu, double* zz, double* dmx,
                            int* uns) {
  const int t = threadIdx.x;
  if (t < 64) {
    const int64_t so = M.s_off;
    const int nb = cdiv_d(M.m, kPrepThreads);
    double a = 0.0, b = 0.0;
    int u = 0;
    for (int i = t; i < nb; i += 64) {
      a += S.tau[so + i];
      b = fmax(b, S.dorg[so + i]);
      u |= S.org[so + i];
    }
    // (an xor butterfly leaves the same bits in every lane: IEEE addition commutes)
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o, 64);
      b = fmax(b, __shfl_xor(b, o, 64));
      u |= __shfl_xor(u, o, 64);
    }
    if (t == 0) {
      sh2[0] = a;
      sh2[1] = b;
      *shu = u;
    }
  }
  __syncthreads();
  *zz = sh2[0];
  *dmx = sh2[1];
  *uns = *shu;
  __syncthreads();
}

// Type-1 deflation of merges of at least kDefPrepRows rows across many
// workgroups (after k_deflate_prep): kDefT1Threads pole positions per
// workgroup.  Every workgroup combines the prep partials (prep_totals) into
// rho and the tolerance exactly as the one-workgroup deflation does, tests the
// positions before its own for survivors itself (a short redundant read, so
// that no workgroup waits for another), and writes its survivors (surv) and
// type-1 deflations (dfv1, dfc1) straight to their places in pole order.  It
// leaves normalised z in zhat (pole order), the 0/1 flags, and per workgroup
// j: its survivors (dest[j]), its deflations (destd1[j]), their counts by
// half (destd2[j]: Q1 rows only + 65536 x Q2 rows only) and their rows in
// range (cnorm[j]).  Workgroup 0 leaves rho, the tolerance and 1 (done) in
// the merge's mparam slots 0-2.  Input that is unsorted or not finite is left
// to the one-workgroup deflation (slot 2 = 0), which then does every step as
// for small merges.
constexpr int kDefT1Threads = 1024;
constexpr int kDefT1Loads = 16;  // loads of preceding z issued together per thread

template <int NT>
__device__ int block_isum(int v, int* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  int r = 0;
  for (int i = 0; i < NT / 64; ++i) r += sh[i];
  return r;
}

// sdl: LDS for D, used by the merge-path searches when m <= lds_cap.  UN: the
// elements per thread (chunks of 64 per wave) whose loads each pass issues
// together (more registers); 1 where a merge fits one pass anyway.
template <int NT, int UN = 4>
__device__ void deflate_body(const MergeDesc& M, const Scratch& S, int lds_cap, double* sdl) {
  constexpr int NW = NT / 64;
  static_assert(NW <= kDefWaves, "wave_prefix covers at most kDefWaves waves");
  __shared__ double shd[kDefWaves];
  __shared__ int shc[7][kDefWaves];
  __shared__ int shi[4];
  const int m = M.m, n1 = M.n1, t = threadIdx.x;
  const int64_t so = M.s_off;
  int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  double* dv = S.dv + so;
  double* zv = S.zv + so;  // (zhat after the many-workgroup type-1 deflation)
  int32_t* col = S.col + so;
  int32_t* part = S.part + so;
  int32_t* flag = S.flag + so;
  int32_t* surv = S.surv + so;

  double rho0 = M.rho, zsign = M.zsign;
  if (M.ecoup != nullptr) {
    // stedc: the coupling b_k of the split (Eq. (2)) lives in the off-diagonal
    // array: rho = |b_k| and the Q2 half of z carries sign(b_k).
    const double bk = *M.ecoup;
    rho0 = fabs(bk);
    zsign = (bk < 0.0) ? -1.0 : 1.0;
  }

  // 1. z (Eq. (3): last row of Q1, first row of Q2), |z|^2, max |D|, sortedness;
  // the row range of every input column, in rows of the merge block.  Large
  // merges ran this step and step 2 element-wise in k_deflate_prep (many
  // workgroups): here its per-block partial sums are combined.
  double zz = 0.0, dmx = 0.0;
  int uns = 0;  // bit 0: a descending step inside D1 or D2; bit 1: a NaN or Inf pole
  const bool prepared = (M.flags & kFlagPrepDeflate) != 0;  // block-uniform
  // k_deflate_t1 did step 3 (and left rho and the tolerance) unless the input
  // was unsorted or not finite
  const double* mp = S.mparam + (int64_t)M.id * 4;
  const bool split1 = prepared && mp[2] != 0.0;  // block-uniform
  constexpr int U1 = UN;  // loads of UN indices issued before their uses
  __shared__ double sh2[2];
  if (prepared && !split1) prep_totals(M, S, sh2, &shi[1], &zz, &dmx, &uns);
  for (int i0 = t; !prepared && i0 < m; i0 += U1 * NT) {
    double zi[U1], di[U1], dprev[U1];
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int i = i0 + u * NT;
      zi[u] = di[u] = dprev[u] = 0.0;
      if (i < m) {
        RowRange g = (i < n1) ? RowRange{0, n1} : RowRange{n1, m};
        if (M.rin) g = RowRange{M.rin[i].lo - M.r0, M.rin[i].hi - M.r0};
        S.crng[so + i] = g;
        const int zr = (i < n1) ? n1 - 1 : n1;  // the row of the column that enters z
        if (M.zgiven) zi[u] = M.zgiven[i];
        else if (zr >= g.lo && zr < g.hi) zi[u] = ((i < n1) ? 1.0 : zsign) * M.qin[zr + (int64_t)i * M.ldin];
        di[u] = M.lin[i];
        if (i > 0) dprev[u] = M.lin[i - 1];
      }
    }
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int i = i0 + u * NT;
      if (i < m) {
        S.zs[so + i] = zi[u];
        zz += zi[u] * zi[u];
        dmx = fmax(dmx, fabs(di[u]));
        // A non-finite pole or a descending step inside either run makes the
        // merge of the two runs ill-defined; such input is reported and merged
        // without sorting.
        if (!isfinite(di[u])) uns |= 2;
        else if (i > 0 && i != n1 && !(di[u] >= dprev[u])) uns |= 1;
      }
    }
  }
  if (!prepared) {
    zz = block_sum<NT>(zz, shd);
    dmx = block_max<NT>(dmx, shd);
  }
  __syncthreads();
  if (t == 0) shi[0] = 0;
  __syncthreads();
  if (uns) atomicOr(&shi[0], uns);
  __syncthreads();
  uns = shi[0];
  if (!isfinite(zz) || !isfinite(rho0)) uns |= 2;  // block-uniform
  const double rho = split1 ? mp[0] : rho0 * zz;
  const double zn = sqrt(zz);
  const double tol = split1 ? mp[1] : 8.0 * kUnitRoundoff * fmax(dmx, rho);
  if (t == 0 && !split1) {
    S.mparam[(int64_t)M.id * 4 + 0] = rho;
    S.mparam[(int64_t)M.id * 4 + 1] = tol;
    if (uns & 2) set_status(S.status, PHDC_ERR_NONFINITE);
    else if (uns) set_status(S.status, PHDC_ERR_UNSORTED);
  }

  // 2. merge the two ascending runs (ties: D1 first) and normalise z.  For
  // valid input the positions form a permutation of [0, m); otherwise keep the
  // input order so every slot is still written exactly once.  (Prepared merges:
  // already placed by k_deflate_prep, and step 3 done by k_deflate_t1, which
  // left normalised z in zhat; placed again here in input order if the runs
  // were not ascending, and every step done here.)
  if (split1) zv = S.zhat + so;
  auto place = [&](const double* D) {
    for (int i = t; i < m; i += NT) {
      const double di = D[i];
      const int pos = uns ? i : (i < n1) ? i + count_lt(D + n1, m - n1, di) : (i - n1) + count_le(D, n1, di);
      dv[pos] = di;
      zv[pos] = (zn > 0.0) ? S.zs[so + i] / zn : 0.0;
      col[pos] = i;
      part[pos] = (i < n1) ? 1 : 3;
    }
  };
  if (split1) {
  } else if (m <= lds_cap) {
    for (int i = t; i < m; i += NT) sdl[i] = M.lin[i];
    __syncthreads();
    place(sdl);
  } else {
    place(M.lin);
  }
  __syncthreads();

  // 3. type-1 deflation (rho |z_i| <= tol) and compaction of both lists in pole order.
  const int lane = t & 63, wv = t >> 6;
  const int seg = ((m + NW - 1) / NW + 63) / 64 * 64;
  const int seg0 = min(m, wv * seg), seg1 = min(m, seg0 + seg);
  int ns, nd1;
  int t1dp1 = 0, t1dp3 = 0;  // (split1) type-1 deflations by half, rows in range
  double t1rows = 0.0;
  // The passes below load UC chunks of 64 before using any of them (the chunks
  // are then consumed in order), so a wave waits on memory once per UC chunks.
  constexpr int UC = UN;
  if (split1) {  // k_deflate_t1's per-workgroup totals
    const int nb1 = cdiv_d(m, kDefT1Threads);
    int a = 0, b = 0, h1 = 0, h3 = 0;
    double r = 0.0;
    for (int j = t; j < nb1; j += NT) {
      a += S.dest[so + j];
      b += S.destd1[so + j];
      const int h = S.destd2[so + j];
      h1 += h & 0xFFFF;
      h3 += h >> 16;
      r += S.cnorm[so + j];
    }
    ns = block_isum<NT>(a, shc[0]);
    nd1 = block_isum<NT>(b, shc[1]);
    t1dp1 = block_isum<NT>(h1, shc[2]);
    t1dp3 = block_isum<NT>(h3, shc[3]);
    t1rows = block_sum<NT>(r, shd);
  } else {
    int c[2] = {0, 0}, pre[2], tot[2];
    for (int b0 = seg0; b0 < seg1; b0 += 64 * UC) {
      double zk[UC];
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int k = b0 + u * 64 + lane;
        zk[u] = (k < seg1) ? zv[k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int k = b0 + u * 64 + lane;
        const bool valid = k < seg1;
        const bool dfl = valid && rho * fabs(zk[u]) <= tol;
        if (valid) flag[k] = dfl ? 1 : 0;
        const uint64_t md = __ballot(dfl), mv = __ballot(valid);
        c[0] += __popcll(mv & ~md);
        c[1] += __popcll(md);
      }
    }
    wave_prefix<2, NW>(c, pre, tot, shc);
    int ps = pre[0], pd = pre[1];
    for (int b0 = seg0; b0 < seg1; b0 += 64 * UC) {
      double zk[UC], dk[UC];
      int ck[UC];
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int k = b0 + u * 64 + lane;
        const bool valid = k < seg1;
        zk[u] = valid ? zv[k] : 0.0;
        dk[u] = valid ? dv[k] : 0.0;
        ck[u] = valid ? col[k] : 0;
      }
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int k = b0 + u * 64 + lane;
        const bool valid = k < seg1;
        const bool dfl = valid && rho * fabs(zk[u]) <= tol;
        const uint64_t md = __ballot(dfl), ms = __ballot(valid && !dfl);
        if (valid && !dfl) surv[ps + lanes_below(ms)] = k;
        if (dfl) {
          const int q = pd + lanes_below(md);
          S.dfv1[so + q] = dk[u];
          S.dfc1[so + q] = ck[u];
        }
        ps += __popcll(ms);
        pd += __popcll(md);
      }
    }
    ns = tot[0];
    nd1 = tot[1];
  }
  __syncthreads();

  // 4. type-2 deflation: scan consecutive survivors in pole order.  Wave 0 tests
  // 64 survivors at a time speculatively (each against its unmodified
  // predecessor) and then replays the chunk in order, jumping straight to the
  // next pair that passes whenever the current predecessor is unmodified.
  if (t < 64) {
    const int lane = t;
    int nrot = 0, nchain = 0;
    bool have_p = false, pmod = false;
    int pk = -1, pp = 0;
    double pd = 0.0, pz = 0.0;
    for (int b0 = 0; b0 < ns; b0 += 64) {
      const int nv = min(64, ns - b0);
      int k = -1, kp = 0;
      double dk = 0.0, zk = 0.0;
      if (lane < nv) {
        k = surv[b0 + lane];
        dk = dv[k];
        zk = zv[k];
        kp = part[k];
      }
      double dprev = __shfl_up(dk, 1, 64), zprev = __shfl_up(zk, 1, 64);
      double c_, s_, t_;
      bool spec = (lane > 0) && (lane < nv) && pair_deflates(dprev, zprev, dk, zk, tol, &c_, &s_, &t_);
      const uint64_t mask = __ballot(spec);
      int L = 0;
      while (L < nv) {
        const double dL = __shfl(dk, L, 64), zL = __shfl(zk, L, 64);
        const int kL = __shfl(k, L, 64), partL = __shfl(kp, L, 64);
        if (!have_p) {
          have_p = true;
          pk = kL; pd = dL; pz = zL; pp = partL; pmod = false;
          ++L;
        } else {
          double c, s, tau;
          if (pair_deflates(pd, pz, dL, zL, tol, &c, &s, &tau)) {
            const double dpn = pd * c * c + dL * s * s;
            const double djn = pd * s * s + dL * c * c;
            const int np = (pp == partL) ? pp : 2;
            if (lane == 0) {
              if (!pmod) S.chain[so + nchain] = nrot;
              const int cp = col[pk], cj = col[kL];
              const RowRange gp = S.crng[so + cp], gj = S.crng[so + cj];
              const RowRange gh{min(gp.lo, gj.lo), max(gp.hi, gj.hi)};  // both results span the hull
              S.rcolp[so + nrot] = cp;
              S.rcolj[so + nrot] = cj;
              S.rc[so + nrot] = c;
              S.rs[so + nrot] = s;
              S.rrp[so + nrot] = gp;
              S.rrj[so + nrot] = gj;
              S.crng[so + cp] = gh;
              S.crng[so + cj] = gh;
              dv[pk] = dpn;
              zv[pk] = 0.0;
              flag[pk] = 2;
              part[pk] = np;
              dv[kL] = djn;
              zv[kL] = tau;
              part[kL] = np;
            }
            if (!pmod) ++nchain;
            ++nrot;
            pk = kL; pd = djn; pz = tau; pp = np; pmod = true;
            ++L;
            continue;
          }
          pk = kL; pd = dL; pz = zL; pp = partL; pmod = false;
          ++L;
        }
        // The predecessor is an unmodified survivor of this chunk: the
        // speculative results are exact until the next passing pair.
        const uint64_t rem = (L < 64) ? (mask & (~0ULL << L)) : 0ULL;
        if (rem == 0ULL) {
          if (L < nv) {
            const int q = nv - 1;
            pk = __shfl(k, q, 64); pd = __shfl(dk, q, 64); pz = __shfl(zk, q, 64); pp = __shfl(kp, q, 64);
            pmod = false;
          }
          L = nv;
        } else {
          const int h = __ffsll((unsigned long long)rem) - 1;
          if (h > L) {
            const int q = h - 1;
            pk = __shfl(k, q, 64); pd = __shfl(dk, q, 64); pz = __shfl(zk, q, 64); pp = __shfl(kp, q, 64);
            pmod = false;
          }
          L = h;
        }
      }
    }
    if (lane == 0) {
      cnt[C_NROT] = nrot;
      cnt[C_NCHAIN] = nchain;
    }
  }
  __syncthreads();

  // 5. final survivors in pole order, Gu's grouping by part (Sec. 1): rows of
  // Uhat ordered [part 1 | part 2 | part 3]; the Q1-row product uses columns of
  // parts 1,2 and the Q2-row product those of parts 2,3.  Type-2 deflated list.
  // (split1: only the survivors of step 3 are visited, through surv; the type-1
  // deflations were counted by k_deflate_t1.)
  const int n5 = split1 ? ns : m;
  const int sg5 = ((n5 + NW - 1) / NW + 63) / 64 * 64;
  const int s50 = min(n5, wv * sg5), s51 = min(n5, s50 + sg5);
  auto pole = [&](int i) { return split1 ? surv[i] : i; };
  // a wave whose segment is one batch keeps its indices, flags and halves in
  // registers for the second pass (block-uniform)
  const bool one5 = sg5 <= 64 * UC;
  int kA[UC], fA[UC], pA[UC];
  int c[7] = {0, 0, 0, 0, 0, 0, 0}, pre[7], tot[7];
  for (int b0 = s50; b0 < s51; b0 += 64 * UC) {
    int fu[UC], pu[UC], ku[UC];
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int i = b0 + u * 64 + lane;
      ku[u] = (i < s51) ? pole(i) : -1;
    }
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int k = ku[u];
      fu[u] = (k >= 0) ? flag[k] : -1;
      pu[u] = (k >= 0) ? part[k] : 0;
      kA[u] = k;
      fA[u] = fu[u];
      pA[u] = pu[u];
    }
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int f = fu[u], p = pu[u];
      c[0] += __popcll(__ballot(f == 0 && p == 1));
      c[1] += __popcll(__ballot(f == 0 && p == 2));
      c[2] += __popcll(__ballot(f == 0 && p == 3));
      c[3] += __popcll(__ballot(f == 2));
      c[4] += __popcll(__ballot(f > 0 && p == 1));  // deflated columns by nonzero half
      c[5] += __popcll(__ballot(f > 0 && p == 2));
      c[6] += __popcll(__ballot(f > 0 && p == 3));
    }
  }
  wave_prefix<7, NW>(c, pre, tot, shc);
  const int k1 = tot[0], k2 = tot[1], k3 = tot[2], nd2 = tot[3];
  const int dp1 = tot[4] + t1dp1, dp2 = tot[5], dp3 = tot[6] + t1dp3;
  const int K = k1 + k2 + k3;
  double drows = 0.0;  // rows in range over the deflated columns (exact: integers below 2^53)
  {
    int b1 = pre[0], b2 = pre[1], b3 = pre[2], b4 = pre[3];
    for (int b0 = s50; b0 < s51; b0 += 64 * UC) {
      int fu[UC], pu[UC], cu[UC], ku[UC];
      double du[UC], zu[UC];
      RowRange gu[UC];
      if (one5) {
#pragma unroll
        for (int u = 0; u < UC; ++u) {
          ku[u] = kA[u];
          fu[u] = fA[u];
          pu[u] = pA[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < UC; ++u) {
          const int i = b0 + u * 64 + lane;
          ku[u] = (i < s51) ? pole(i) : -1;
        }
#pragma unroll
        for (int u = 0; u < UC; ++u) {
          const int k = ku[u];
          fu[u] = (k >= 0) ? flag[k] : -1;
          pu[u] = (k >= 0) ? part[k] : 0;
        }
      }
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int k = ku[u];
        const bool valid = k >= 0;
        cu[u] = valid ? col[k] : 0;
        du[u] = valid ? dv[k] : 0.0;
        zu[u] = valid ? zv[k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UC; ++u) gu[u] = (fu[u] >= 0) ? S.crng[so + cu[u]] : RowRange{0, 0};
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int f = fu[u], p = pu[u];
        const uint64_t m1 = __ballot(f == 0 && p == 1), m2 = __ballot(f == 0 && p == 2);
        const uint64_t m3 = __ballot(f == 0 && p == 3), m4 = __ballot(f == 2);
        if (f == 0) {
          const int e1 = b1 + lanes_below(m1), e2 = b2 + lanes_below(m2), e3 = b3 + lanes_below(m3);
          const int ks = e1 + e2 + e3;
          S.ds[so + ks] = du[u];
          S.zs[so + ks] = zu[u];
          const int ck = cu[u];
          const RowRange gk = gu[u];
          S.csort[so + ks] = ck;
          int g;
          if (p == 1) {
            g = e1;
            S.coltop[so + e1] = ck;
            S.rgtop[so + e1] = gk;
          } else if (p == 2) {
            g = k1 + e2;
            S.coltop[so + k1 + e2] = ck;
            S.rgtop[so + k1 + e2] = gk;
            S.colbot[so + e2] = ck;
            S.rgbot[so + e2] = gk;
          } else {
            g = k1 + k2 + e3;
            S.colbot[so + k2 + e3] = ck;
            S.rgbot[so + k2 + e3] = gk;
          }
          S.grp[so + ks] = g;
          S.grpsrc[so + g] = ks;
        } else if (f == 2) {
          const int q = b4 + lanes_below(m4);
          S.dfv2[so + q] = du[u];
          S.dfc2[so + q] = cu[u];
        }
        if (f > 0) drows += (double)(gu[u].hi - gu[u].lo);
        b1 += __popcll(m1);
        b2 += __popcll(m2);
        b3 += __popcll(m3);
        b4 += __popcll(m4);
      }
    }
  }
  drows = block_sum<NT>(drows, shd) + t1rows;
  if (t == 0) {
    const int64_t dr = (int64_t)drows;
    cnt[C_DROWS_LO] = (int32_t)(uint32_t)(dr & 0xffffffffLL);
    cnt[C_DROWS_HI] = (int32_t)(dr >> 32);
    cnt[C_K] = K;
    cnt[C_K1] = k1;
    cnt[C_K2] = k2;
    cnt[C_K3] = k3;
    cnt[C_NT1] = nd1;
    cnt[C_NT2] = nd2;
    cnt[C_ND1] = nd1;
    cnt[C_ND2] = nd2;
    cnt[C_DP1] = dp1;
    cnt[C_DP2] = dp2;
    cnt[C_DP3] = dp3;
    cnt[C_PATH] = M.split_on ? 1 : (M.hss_min_k > 0 && K >= M.hss_min_k) ? 2 : 0;
    cnt[C_HSSRANK] = 0;
    cnt[C_WROWS] = 0;
    cnt[C_WROWS + 1] = 0;
  }
}

__global__ void __launch_bounds__(kDefT1Threads) k_deflate_t1(BlockMap bm, Scratch S) {
  constexpr int NT = kDefT1Threads, NW = NT / 64;
  static_assert(NW <= kDefWaves, "wave_prefix covers at most kDefWaves waves");
  __shared__ double shd[NW];
  __shared__ double sh2[2];
  __shared__ int shu;
  __shared__ int shc[2][kDefWaves];
  __shared__ int shs[4][NW];
  const int mi = find_merge(bm, blockIdx.x);
  const int lb = blockIdx.x - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  if (!(M.flags & kFlagPrepDeflate)) return;  // (the one-workgroup deflation does every step)
  const int m = M.m, t = threadIdx.x, lane = t & 63;
  const int64_t so = M.s_off;
  double zz, dmx;
  int uns;
  prep_totals(M, S, sh2, &shu, &zz, &dmx, &uns);
  double rho0 = M.rho;
  if (M.ecoup != nullptr) rho0 = fabs(*M.ecoup);
  if (!isfinite(zz) || !isfinite(rho0)) uns |= 2;
  // exactly the one-workgroup deflation's rho, normalisation and test
  const double rho = rho0 * zz;
  const double zn = sqrt(zz);
  const double tol = 8.0 * kUnitRoundoff * fmax(dmx, rho);
  if (lb == 0 && t == 0) {
    double* mp = S.mparam + (int64_t)M.id * 4;
    mp[0] = rho;
    mp[1] = tol;
    mp[2] = uns ? 0.0 : 1.0;
  }
  if (uns) return;  // (block-uniform)
  auto znorm = [&](double z) { return (zn > 0.0) ? z / zn : 0.0; };

  // survivors among the positions before this workgroup's
  const int k0 = lb * NT;
  int cs = 0;
  for (int b0 = t; b0 < k0; b0 += NT * kDefT1Loads) {
    double zb[kDefT1Loads];
#pragma unroll
    for (int u = 0; u < kDefT1Loads; ++u) {
      const int k = b0 + u * NT;
      zb[u] = (k < k0) ? S.zv[so + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kDefT1Loads; ++u)
      if (b0 + u * NT < k0 && !(rho * fabs(znorm(zb[u])) <= tol)) ++cs;
  }
  const int pre_s = block_isum<NT>(cs, shs[0]), pre_d = k0 - pre_s;

  // this workgroup's positions
  const int k = k0 + t;
  const bool valid = k < m;
  double zk = 0.0, dk = 0.0;
  int ck = 0, pk = 0;
  if (valid) {
    zk = znorm(S.zv[so + k]);
    dk = S.dv[so + k];
    ck = S.col[so + k];
    pk = S.part[so + k];
  }
  const bool dfl = valid && rho * fabs(zk) <= tol;
  if (valid) {
    S.zhat[so + k] = zk;
    S.flag[so + k] = dfl ? 1 : 0;
  }
  const uint64_t ms = __ballot(valid && !dfl), md = __ballot(dfl);
  int cw[2] = {(int)__popcll(ms), (int)__popcll(md)}, pre[2], tot[2];
  wave_prefix<2, NW>(cw, pre, tot, shc);
  if (valid && !dfl) S.surv[so + pre_s + pre[0] + lanes_below(ms)] = k;
  double rows = 0.0;
  if (dfl) {
    const int q = pre_d + pre[1] + lanes_below(md);
    S.dfv1[so + q] = dk;
    S.dfc1[so + q] = ck;
    const RowRange g = S.crng[so + ck];
    rows = (double)(g.hi - g.lo);
  }
  const int h1 = block_isum<NT>(dfl && pk == 1 ? 1 : 0, shs[1]);
  const int h3 = block_isum<NT>(dfl && pk == 3 ? 1 : 0, shs[2]);
  rows = block_sum<NT>(rows, shd);
  if (t == 0) {
    S.dest[so + lb] = tot[0];
    S.destd1[so + lb] = tot[1];
    S.destd2[so + lb] = h1 | (h3 << 16);
    S.cnorm[so + lb] = rows;
  }
  (void)lane;
}

template <int NT>
__global__ void __launch_bounds__(NT) k_deflate(const MergeDesc* __restrict__ descs, Scratch S, int lds_cap) {
  HIP_DYNAMIC_SHARED(double, sdl)
  const MergeDesc M = descs[blockIdx.x];
  if (M.flags & kFlagSmallMerge) return;  // deflated by k_merge_small
  deflate_body<NT>(M, S, lds_cap, sdl);
}

// ------------------------------------------------------------ rotations
// Applies the recorded rotation chains to the columns of the merge's input
// block, in place.  A chain's records share a column and run in order per row;
// distinct chains touch disjoint columns and run in parallel.  A rotation reads
// each column inside its recorded range only and writes both over the hull of
// the two ranges (zeros where neither column has rows), which is the range the
// rotated columns carry on.
constexpr int kRotGroups = 16;

// Row r of the chains g, g + G, ... of merge M.
// A chain is a run of rotations (c_0, c_1), (c_1, c_2), ... : the type-2 scan
// carries each rotated survivor on as the predecessor of the next test, so
// column cj of one rotation is column cp of the next and no column appears in
// two chains.  Row r keeps the running column in a register and reads each
// fresh column once; the reads of kRotBatch rotations are issued before their
// arithmetic, so a chain costs one memory round trip per batch rather than two
// dependent accesses per rotation.  Rows outside both ranges of a rotation
// are neither read nor written (they stay zero for every later reader).
constexpr int kRotBatch = 4;

__device__ void rotate_chains(const MergeDesc& M, const Scratch& S, int r, int g, int G) {
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  const int nrot = cnt[C_NROT], nchain = cnt[C_NCHAIN];
  const int64_t so = M.s_off;
  double* q = M.qin;
  const int64_t ld = M.ldin;
  for (int ci = g; ci < nchain; ci += G) {
    const int a = S.chain[so + ci];
    const int e = (ci + 1 < nchain) ? S.chain[so + ci + 1] : nrot;
    int cp = S.rcolp[so + a];
    RowRange gp = S.rrp[so + a];
    double xp = (r >= gp.lo && r < gp.hi) ? q[r + (int64_t)cp * ld] : 0.0;
    for (int x0 = a; x0 < e; x0 += kRotBatch) {
      int cj[kRotBatch];
      RowRange gj[kRotBatch];
      double cs[kRotBatch], sn[kRotBatch], xj[kRotBatch];
#pragma unroll
      for (int u = 0; u < kRotBatch; ++u) {
        const int x = x0 + u;
        cj[u] = 0;
        gj[u] = RowRange{0, 0};
        cs[u] = 1.0;
        sn[u] = 0.0;
        xj[u] = 0.0;
        if (x < e) {
          cj[u] = S.rcolj[so + x];
          gj[u] = S.rrj[so + x];
          cs[u] = S.rc[so + x];
          sn[u] = S.rs[so + x];
          if (r >= gj[u].lo && r < gj[u].hi) xj[u] = q[r + (int64_t)cj[u] * ld];
        }
      }
#pragma unroll
      for (int u = 0; u < kRotBatch; ++u) {
        if (x0 + u < e) {
          // rows of the hull of both ranges carry the rotated values on
          const bool in = r >= min(gp.lo, gj[u].lo) && r < max(gp.hi, gj[u].hi);
          const double np = cs[u] * xp + sn[u] * xj[u];
          const double nj = cs[u] * xj[u] - sn[u] * xp;
          if (in) q[r + (int64_t)cp * ld] = np;
          xp = in ? nj : 0.0;
          cp = cj[u];
          gp = RowRange{min(gp.lo, gj[u].lo), max(gp.hi, gj[u].hi)};
        }
      }
    }
    if (r >= gp.lo && r < gp.hi) q[r + (int64_t)cp * ld] = xp;
  }
}

__device__ void rotate_body(const BlockMap& bm, const Scratch& S, int b) {
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int RB = cdiv_d(M.m, 256);
  const int G = (merge_blocks(bm, mi)) / RB;
  const int rb = lb % RB, g = lb / RB;
  const int r = rb * 256 + threadIdx.x;
  if (r < M.m) rotate_chains(M, S, r, g, G);
}

// ------------------------------------------------------------ secular roots
// Root j of f(lambda) = 1 + rho sum_i z_i^2/(d_i - lambda) (Sec. 1, after
// Eq. (4)) is bracketed in (d_j, d_{j+1}) (last root: (d_K, d_K + rho|z|^2));
// its origin is the bracket end nearer to the root (sign of f at the midpoint).
// tau is then refined by the two-pole rational model of f (the "middle way" of
// R.-C. Li, 1993: psi = poles left of the bracket, phi = poles right of it,
// each matched in value and slope at the current iterate), with the bracket
// kept up to date and a bisection step whenever the model step leaves it.  All
// differences are formed as (d_i - d_org) - tau.
//
// Each root is owned by a group of G consecutive lanes that split the sums over
// the poles and combine them with shuffles, so every lane of the group takes
// the same decisions.  Reciprocals in the sums use the hardware estimate
// refined by two Newton-Raphson steps y <- y (2 - x y) (quadratic convergence
// from the ~2^-26 estimate: full double precision up to an ulp).
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

constexpr int kSecMaxIters = 120;  // bracketed steps per root (bisection alone needs at most ~64)

// A double moved between lanes of a 16-lane row by a DPP lane pattern (a VALU
// operand modifier: no LDS round trip, unlike a general shuffle).
template <int CTRL>
__device__ inline double dpp_row(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppQuadXor1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int kDppRowHalfMirror = 0x141; // lane i <-> 7 - i within each 8 lanes
constexpr int kDppRowMirror = 0x140;     // lane i <-> 15 - i within each 16 lanes

// Sum (product) over the G consecutive lanes of a group, every lane receiving
// the same value.  For G = 16 the partners are the lane's quad neighbours, then
// the mirrored quad and the mirrored half-row: the same pairing tree as xor 1,
// 2, 4, 8 (quads hold equal values by then), so the result does not depend on
// which form runs, and IEEE addition being commutative every lane holds the
// identical total.  G = 4 takes the first two steps; G = 32 adds the totals
// of its two rows (in either order: the same bits).
template <int G>
__device__ inline double group_sum(double v) {
  if constexpr (G == 32) {
    v += dpp_row<kDppQuadXor1>(v);
    v += dpp_row<kDppQuadXor2>(v);
    v += dpp_row<kDppRowHalfMirror>(v);
    v += dpp_row<kDppRowMirror>(v);
    v += __shfl_xor(v, 16, 64);
  } else if constexpr (G == 16 || G == 4) {
    v += dpp_row<kDppQuadXor1>(v);
    v += dpp_row<kDppQuadXor2>(v);
    if constexpr (G == 16) {
      v += dpp_row<kDppRowHalfMirror>(v);
      v += dpp_row<kDppRowMirror>(v);
    }
  } else {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
  }
  return v;
}

// Sums of the secular function at lambda = dorg + t over the poles, split at jl:
// psi = sum_{i <= jl} z_i^2/(d_i - lambda), phi = the rest, their derivatives and
// sum |z_i^2/(d_i - lambda)|; the G lanes of a group each take every G-th pole,
// two poles in flight per lane.  SQ: z holds the squares.
struct SecSums {
  double psi, dpsi, phi, dphi, eabs;
};

template <int G, bool SQ>
__device__ __forceinline__ SecSums secular_sums(int K, const double* __restrict__ d, const double* __restrict__ z,
                                                int jl, int sub, double dorg, double t) {
  auto z2 = [&](int i) { return SQ ? z[i] : z[i] * z[i]; };
  double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0, eabs = 0.0;
  double psi2 = 0.0, dpsi2 = 0.0, phi2 = 0.0, dphi2 = 0.0, eabs2 = 0.0;
  int i = sub;
  for (; i + G < K; i += 2 * G) {
    const int i2 = i + G;
    const double del = (d[i] - dorg) - t, del2 = (d[i2] - dorg) - t;
    const double rcp = rcp_nr(del), rcp2 = rcp_nr(del2);
    const double tt = z2(i) * rcp, tt2 = z2(i2) * rcp2;
    const double dt = tt * rcp, dt2 = tt2 * rcp2;
    if (i <= jl) { psi += tt; dpsi += dt; } else { phi += tt; dphi += dt; }
    if (i2 <= jl) { psi2 += tt2; dpsi2 += dt2; } else { phi2 += tt2; dphi2 += dt2; }
    eabs += fabs(tt);
    eabs2 += fabs(tt2);
  }
  if (i < K) {
    const double del = (d[i] - dorg) - t;
    const double rcp = rcp_nr(del);
    const double tt = z2(i) * rcp;
    const double dt = tt * rcp;
    if (i <= jl) { psi += tt; dpsi += dt; } else { phi += tt; dphi += dt; }
    eabs += fabs(tt);
  }
  return SecSums{group_sum<G>(psi + psi2), group_sum<G>(dpsi + dpsi2), group_sum<G>(phi + phi2),
                 group_sum<G>(dphi + dphi2), group_sum<G>(eabs + eabs2)};
}

// SQ: z holds the squares z_i^2 (staged copies) instead of z_i.  Interior roots
// first evaluate f, with its derivatives, at the middle of their bracket: the
// sign picks the origin, and the same sums give the first rational step.
template <int G, bool SQ>
__device__ __forceinline__ bool secular_root(int K, const double* __restrict__ d, const double* __restrict__ z,
                                             double rho, int j, int sub, int* org_out, double* tau_out,
                                             int maxit = kSecMaxIters, int* iters = nullptr) {
  auto z2 = [&](int i) { return SQ ? z[i] : z[i] * z[i]; };
  const double inv_rho = 1.0 / rho;
  if (K == 1) {
    *org_out = 0;
    *tau_out = rho * z2(0);
    return true;
  }
  const int jl = (j < K - 1) ? j : K - 2;
  const int jr = jl + 1;
  int org;
  double lo, hi, tau;
  SecSums f{};
  bool have = false;  // f holds the sums at tau
  if (j < K - 1) {
    const double dj = d[j], dj1 = d[j + 1];
    const double half = 0.5 * (dj1 - dj);
    f = secular_sums<G, SQ>(K, d, z, jl, sub, dj, half);
    if (inv_rho + f.psi + f.phi >= 0.0) {
      org = j; lo = 0.0; hi = half; tau = hi;
    } else {
      org = j + 1; lo = (dj - dj1) + half; hi = 0.0; tau = lo;
    }
    have = true;
  } else {
    org = K - 1;
    lo = 0.0;
    double zz = 0.0;
    for (int i = sub; i < K; i += G) zz += z2(i);
    hi = rho * group_sum<G>(zz);
    for (int guard = 0; guard < 64; ++guard) {
      double w = 0.0;
      for (int i = sub; i < K; i += G) w += z2(i) / ((d[i] - d[org]) - hi);
      w = inv_rho + group_sum<G>(w);
      if (w >= 0.0) break;
      hi *= 2.0;
    }
    tau = 0.5 * (lo + hi);
  }
  const double dorg = d[org];
  bool ok = false;
  int it = 0;
  for (; it < maxit; ++it) {
    if (!have) f = secular_sums<G, SQ>(K, d, z, jl, sub, dorg, tau);
    have = false;
    const double w = inv_rho + f.psi + f.phi;
    if (w > 0.0) hi = tau;
    else if (w < 0.0) lo = tau;
    else if (w == 0.0) { ok = true; break; }
    else break;  // NaN: not converged (reported as PHDC_ERR_SECULAR)
    if (fabs(w) <= 8.0 * kUnitRoundoff * (inv_rho + f.eabs)) { ok = true; break; }
    const double Dl = (d[jl] - dorg) - tau, Dr = (d[jr] - dorg) - tau;
    const double a = (Dl + Dr) * w - Dl * Dr * (f.dpsi + f.dphi);
    const double bb = Dl * Dr * w;
    const double c = w - Dl * f.dpsi - Dr * f.dphi;
    const double disc = sqrt(fabs(a * a - 4.0 * bb * c));
    double eta;
    if (c == 0.0) eta = bb / a;
    else if (j < K - 1) eta = (a <= 0.0) ? (a - disc) / (2.0 * c) : 2.0 * bb / (a + disc);
    else eta = (a >= 0.0) ? (a + disc) / (2.0 * c) : 2.0 * bb / (a - disc);
    double tn = tau + eta;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (tn == tau || !(hi > lo)) { ok = true; break; }
    tau = tn;
  }
  if (iters) *iters = it + 1;
  *org_out = org;
  *tau_out = tau;
  return ok;
}

constexpr int kSecThreads = 256;  // threads per block
constexpr int kSecLds = 2048;     // largest number of poles staged in LDS (d_i and z_i^2: 32 KB)
constexpr int kSecG = 16;         // lanes per root (crowded levels, small merges, standalone roots)
constexpr int kSecGWide = 32;     // lanes per root in levels of at most kSecWideRows rows (fastest of 4..64
                                  // on a random n = 16384 solve)

// The roots of one block: G lanes per root, kSecThreads / G roots per block.
// Merges with K <= cap stage the poles and squared weights in LDS once (cap:
// the launch's LDS, sized by its largest merge, at most kSecLds); larger ones
// read them from global memory (L2-resident).
template <int G>
__device__ __forceinline__ void secular_block(const MergeDesc& M, const Scratch& S, int K, int lb, int nb, double* sd,
                                              double* sz, int cap) {
  constexpr int R = kSecThreads / G;
  if (lb * R >= K) return;  // whole block idle (uniform)
  const int sub = threadIdx.x % G;
  const int64_t so = M.s_off;
  const double rho = S.mparam[(int64_t)M.id * 4 + 0];
  const int maxit = (M.flags & kFlagNoSecularIters) ? 0 : kSecMaxIters;
  const bool staged = K <= cap;  // block-uniform
  if (staged) {
    for (int i = threadIdx.x; i < K; i += kSecThreads) {
      sd[i] = S.ds[so + i];
      const double zi = S.zs[so + i];
      sz[i] = zi * zi;
    }
    __syncthreads();
  }
  // roots lb R .. lb R + R - 1, then nb R further on (nb: the merge's blocks)
  for (int j0 = lb * R; j0 < K; j0 += nb * R) {
    const int j = j0 + (int)threadIdx.x / G;
    const bool active = j < K;
    // inactive groups of a partly filled block run root K-1 redundantly so that
    // every lane takes part in the group shuffles; only active groups write
    const int jj = active ? j : K - 1;
    int org = 0;
    double tau = 0.0;
    const bool ok = staged ? secular_root<G, true>(K, sd, sz, rho, jj, sub, &org, &tau, maxit)
                           : secular_root<G, false>(K, S.ds + so, S.zs + so, rho, jj, sub, &org, &tau, maxit);
    if (active && sub == 0) {
      S.org[so + j] = org;
      S.tau[so + j] = tau;
      S.dorg[so + j] = S.ds[so + org];
      if (!ok) set_status(S.status, PHDC_ERR_SECULAR);
    }
  }
}

template <int G>
__device__ void secular_body(const BlockMap& bm, const Scratch& S, int b, double* sd, double* sz, int cap) {
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int K = S.counters[(int64_t)M.id * kCounters + C_K];
  secular_block<G>(M, S, K, lb, merge_blocks(bm, mi), sd, sz, cap);
}

__global__ void __launch_bounds__(64) k_secular_raw(int K, const double* d, const double* z, double rho,
                                                    int32_t* org, double* tau, int32_t* status) {
  const int j = blockIdx.x * (64 / kSecG) + (int)threadIdx.x / kSecG;
  const int sub = threadIdx.x % kSecG;
  const bool active = j < K;
  int o = 0, its = 0;
  double t = 0.0;
  bool ok = secular_root<kSecG, false>(K, d, z, rho, active ? j : K - 1, sub, &o, &t, kSecMaxIters, &its);
  if (active && sub == 0) {
    org[j] = o;
    tau[j] = t;
    if (!ok) set_status(status, PHDC_ERR_SECULAR);
    atomicMax(status + 1, its);  // largest number of evaluations of one root
  }
}

// ------------------------------------------------------------ Loewner z
// rho zhat_i^2 = prod_j (lambda_j - d_i) / prod_{k != i} (d_k - d_i) (Remark 1),
// paired so every factor is in (0, 1]: for j < i (d_i - lambda_j)/(d_i - d_j),
// for i <= j < K-1 (d_i - lambda_j)/(d_i - d_{j+1}), times lambda_{K-1} - d_i.
template <int G>
__device__ inline double group_prod(double v) {
  if constexpr (G == 16 || G == 32) {
    v *= dpp_row<kDppQuadXor1>(v);
    v *= dpp_row<kDppQuadXor2>(v);
    v *= dpp_row<kDppRowHalfMirror>(v);
    v *= dpp_row<kDppRowMirror>(v);
    if constexpr (G == 32) v *= __shfl_xor(v, 16, 64);  // (the two rows' products, in either order)
  } else {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v *= __shfl_xor(v, o, 64);
  }
  return v;
}

// Both kernels: 256-lane blocks, IG lanes per item (16, or 32 in levels of at
// most kSecWideRows rows, as for the secular roots) each taking every IG-th
// term, two terms in flight per lane.
constexpr int kItemG = 16;

// A lane's partial product is a product of factors in (0, 1], so none
// underflows before the full product does.  Item i0 of a merge with K poles,
// computed by the IG lanes of a group (sub = lane within the group).
template <int IG = kItemG>
__device__ inline void lowner_item(const MergeDesc& M, const Scratch& S, int K, int i0, int sub) {
  const bool active = i0 < K;
  const int i = active ? i0 : K - 1;  // idle groups repeat the last item (group shuffles)
  const int64_t so = M.s_off;
  const double* ds = S.ds + so;
  const double* dorg = S.dorg + so;
  const double* tau = S.tau + so;
  const double rho = S.mparam[(int64_t)M.id * 4 + 0];
  const double di = ds[i];
  double w1 = 1.0, w2 = 1.0;
  int j = sub;
  for (; j + IG < K - 1; j += 2 * IG) {
    const int j2 = j + IG;
    const double num = (di - dorg[j]) - tau[j], num2 = (di - dorg[j2]) - tau[j2];
    const double den = (j < i) ? (di - ds[j]) : (di - ds[j + 1]);
    const double den2 = (j2 < i) ? (di - ds[j2]) : (di - ds[j2 + 1]);
    w1 *= num / den;
    w2 *= num2 / den2;
  }
  if (j < K - 1) {
    const double num = (di - dorg[j]) - tau[j];
    const double den = (j < i) ? (di - ds[j]) : (di - ds[j + 1]);
    w1 *= num / den;
  }
  double w = group_prod<IG>(w1 * w2);
  w *= -((di - dorg[K - 1]) - tau[K - 1]);
  if (active && sub == 0) {
    const double mag = sqrt(fabs(w) / rho);
    S.zhat[so + i] = (S.zs[so + i] < 0.0) ? -mag : mag;
  }
}

template <int IG>
__device__ void lowner_body(const BlockMap& bm, const Scratch& S, int b) {
  constexpr int IPB = kSecThreads / IG;  // items per block
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int K = S.counters[(int64_t)M.id * kCounters + C_K];
  const int G = merge_blocks(bm, mi);
  for (int i0 = lb * IPB; i0 < K; i0 += G * IPB)  // (block-uniform bound)
    lowner_item<IG>(M, S, K, i0 + (int)threadIdx.x / IG, threadIdx.x % IG);
}

// Reciprocal 2-norms of the columns zhat_i / (d_i - lambda_j) of Uhat (Eq. (4)).
template <int IG = kItemG>
__device__ inline void unorm_item(const MergeDesc& M, const Scratch& S, int K, int j0, int sub) {
  const bool active = j0 < K;
  const int j = active ? j0 : K - 1;
  const int64_t so = M.s_off;
  const double* ds = S.ds + so;
  const double* zh = S.zhat + so;
  const double lj = S.dorg[so + j], tj = S.tau[so + j];
  double s1 = 0.0, s2 = 0.0;
  int i = sub;
  for (; i + IG < K; i += 2 * IG) {
    const int i2 = i + IG;
    const double v = zh[i] / ((ds[i] - lj) - tj), v2 = zh[i2] / ((ds[i2] - lj) - tj);
    s1 += v * v;
    s2 += v2 * v2;
  }
  if (i < K) {
    const double v = zh[i] / ((ds[i] - lj) - tj);
    s1 += v * v;
  }
  const double s = group_sum<IG>(s1 + s2);
  if (active && sub == 0) S.cnorm[so + j] = 1.0 / sqrt(s);
}

template <int IG>
__device__ void unorm_body(const BlockMap& bm, const Scratch& S, int b) {
  constexpr int IPB = kSecThreads / IG;  // items per block
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int K = S.counters[(int64_t)M.id * kCounters + C_K];
  const int G = merge_blocks(bm, mi);
  for (int j0 = lb * IPB; j0 < K; j0 += G * IPB)  // (block-uniform bound)
    unorm_item<IG>(M, S, K, j0 + (int)threadIdx.x / IG, threadIdx.x % IG);
}

// ... then the entries, written row-major (row g = grouped row, ld = K) so that
// the product's operand tiles are contiguous.  HSS merges keep the pole order
// (Gu's grouping would break the low-rank structure of the off-diagonal
// blocks, Sec. 2.2); plain merges use it.  With normalized == false the columns
// are left unscaled (the update GEMM applies the column scale in its
// epilogue), so that the writer need not wait for the norms.
__device__ inline double uhat_entry(const MergeDesc& M, const Scratch& S, bool pole_order, int g, double lj,
                                    double tj, double sc) {
  const int64_t so = M.s_off;
  const int i = pole_order ? g : S.grpsrc[so + g];
  return S.zhat[so + i] / ((S.ds[so + i] - lj) - tj) * sc;
}

// A block covers 256 columns and strides over rows.
constexpr int kUwRowGroups = 64;

__device__ void uwrite_body(const BlockMap& bm, const Scratch& S, int b, bool normalized) {
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int K = S.counters[(int64_t)M.id * kCounters + C_K];
  const int CB = cdiv_d(M.m, 256);
  const int RG = (merge_blocks(bm, mi)) / CB;
  const int cb = lb % CB, rg = lb / CB;
  const int j = cb * 256 + threadIdx.x;
  if (j >= K) return;
  const int64_t so = M.s_off;
  const bool pole_order = S.counters[(int64_t)M.id * kCounters + C_PATH] == 2;
  const double lj = S.dorg[so + j], tj = S.tau[so + j], sc = normalized ? S.cnorm[so + j] : 1.0;
  double* U = S.uhat + M.u_off;
  for (int g = rg; g < K; g += RG) U[(int64_t)g * K + j] = uhat_entry(M, S, pole_order, g, lj, tj, sc);
}

// Levels whose merges have at most kSmallUhat rows: one workgroup of NT
// threads per merge applies the rotations and forms the secular roots, zhat,
// the column norms, Uhat and the output ranks in turn (one launch instead of
// several whose fixed latency exceeds this work, and no grid sized for K = m),
// with G lanes per root or item.  With G = kSecG (the levels that take this
// step alone) the per-item arithmetic is that of the multi-block kernels, so a
// merge gives the same bits on either path.
constexpr int kSmallUhat = 64;
static_assert(kFillMinRows > kSmallUhat, "a zero-filled root never takes the small-merge branches");
constexpr int kStageSmallThreads = 1024;

__device__ int rank_item(const MergeDesc& M, const Scratch& S, int x);

template <int NT, int G>
__device__ void small_body(const MergeDesc& M, const Scratch& S, bool normalized, double* sd, double* sz) {
  static_assert(NT % 64 == 0 && NT / G >= kSmallUhat, "one pass over the roots");
  const int K = S.counters[(int64_t)M.id * kCounters + C_K];
  const int t = threadIdx.x;
  const int64_t so = M.s_off;
  // rotations of the input block (independent of the steps below): NT / 64 groups
  // of 64 threads, group g takes the chains g, g + NT / 64, ..., thread r of a group row r
  if ((t & 63) < M.m) rotate_chains(M, S, t & 63, t >> 6, NT / 64);
  if (K > 0) {  // block-uniform
    // secular roots, G lanes each, poles staged in LDS (K <= kSmallUhat)
    const double rho = S.mparam[(int64_t)M.id * 4 + 0];
    const int maxit = (M.flags & kFlagNoSecularIters) ? 0 : kSecMaxIters;
    for (int i = t; i < K; i += NT) {
      sd[i] = S.ds[so + i];
      const double zi = S.zs[so + i];
      sz[i] = zi * zi;
    }
    __syncthreads();
    const int sub = t % G;
    for (int j0 = 0; j0 < K; j0 += NT / G) {
      const int j = j0 + t / G;
      int org = 0;
      double tau = 0.0;
      const bool ok = secular_root<G, true>(K, sd, sz, rho, j < K ? j : K - 1, sub, &org, &tau, maxit);
      if (j < K && sub == 0) {
        S.org[so + j] = org;
        S.tau[so + j] = tau;
        S.dorg[so + j] = sd[org];
        if (!ok) set_status(S.status, PHDC_ERR_SECULAR);
      }
    }
    __syncthreads();
    const int grp = t / G, isub = t % G;
    for (int i0 = 0; i0 < K; i0 += NT / G) lowner_item<G>(M, S, K, i0 + grp, isub);
    __syncthreads();
    for (int j0 = 0; j0 < K; j0 += NT / G) unorm_item<G>(M, S, K, j0 + grp, isub);
    __syncthreads();
    const bool pole_order = S.counters[(int64_t)M.id * kCounters + C_PATH] == 2;
    double* U = S.uhat + M.u_off;
    const int nj = min(K, NT), rg = NT / nj;  // column j = t % nj, row group t / nj
    if (t < nj * rg) {
      for (int j = t % nj; j < K; j += nj) {
        const double lj = S.dorg[so + j], tj = S.tau[so + j], sc = normalized ? S.cnorm[so + j] : 1.0;
        for (int g = t / nj; g < K; g += rg) U[(int64_t)g * K + j] = uhat_entry(M, S, pole_order, g, lj, tj, sc);
      }
    }
  }
  for (int x = t; x < M.m; x += NT) rank_item(M, S, x);
}

// ------------------------------------------------------------ final order
// Output position of every eigenvalue of the merge: the ascending order of
// {roots} u {type-1 deflated} u {type-2 deflated}, ties broken by (class,
// index).  Roots and type-1 values are each non-decreasing (binary search);
// type-2 values are counted directly.
// Item x of merge M (x < M.m).
// Returns, for a deflated column of a zero-filled root, the rows its copy
// writes (its range), else 0.
__device__ int rank_item(const MergeDesc& M, const Scratch& S, int x) {
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  const int K = cnt[C_K], nd1 = cnt[C_ND1], nd2 = cnt[C_ND2];
  const int64_t so = M.s_off;
  const double* dorg = S.dorg + so;
  const double* tau = S.tau + so;
  const double* v1 = S.dfv1 + so;
  const double* v2 = S.dfv2 + so;
  int cls, idx;
  double v;
  if (x < K) { cls = 0; idx = x; v = dorg[x] + tau[x]; }
  else if (x < K + nd1) { cls = 1; idx = x - K; v = v1[idx]; }
  else { cls = 2; idx = x - K - nd1; v = v2[idx]; }
  int r;
  // roots
  if (cls == 0) r = idx;
  else {
    int lo = 0, hi = K;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (dorg[mid] + tau[mid] <= v) lo = mid + 1; else hi = mid;
    }
    r = lo;
  }
  // type-1 deflated
  if (cls == 1) r += idx;
  else if (cls == 0) r += count_lt(v1, nd1, v);
  else r += count_le(v1, nd1, v);
  // type-2 deflated
  for (int q = 0; q < nd2; ++q) {
    const double u = v2[q];
    r += (u < v) || (u == v && cls == 2 && q < idx);
  }
  M.lout[r] = v;
  if (cls == 0) S.dest[so + idx] = r;
  else if (cls == 1) S.destd1[so + idx] = r;
  else S.destd2[so + idx] = r;
  RowRange g{0, M.m};  // roots fill every row of the block; deflated columns keep their range
  if (cls > 0) g = S.crng[so + (cls == 1 ? S.dfc1[so + idx] : S.dfc2[so + idx])];
  if (M.rout) M.rout[r] = RowRange{g.lo + M.r0, g.hi + M.r0};
  if (cls == 0 || !(M.flags & kFlagPrefilled)) return 0;
  return g.hi - g.lo;
}

__device__ void rank_body(const BlockMap& bm, const Scratch& S, int b) {
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int x = lb * 256 + threadIdx.x;
  unsigned long long w = (x < M.m) ? (unsigned long long)rank_item(M, S, x) : 0ULL;
  if (M.flags & kFlagPrefilled) {  // (block-uniform) one atomic per wave
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
    if ((threadIdx.x & 63) == 0 && w)
      atomicAdd((unsigned long long*)(S.counters + (int64_t)M.id * kCounters + C_WROWS), w);
  }
}

// ------------------------------------------------------------ deflated columns
// Deflated columns of Q G P (Eq. (6), the identity block) go unchanged to
// their output position.  Only the rows of a column's range are read and, below
// the root of the tree, written: the next merge reads no other row.  The root
// merge writes every row (zeros outside the range), since its output is the
// caller's eigenvector matrix.
constexpr int kCopyBlocks = 16384;  // cap on column blocks per merge
constexpr int kCopyWideRows = 2048;  // root merges from this many rows copy a column per block

// Below the root, each block streams whole columns: a column group of RPT
// lanes (RPT = m rounded up to a power of two, at most 64) walks the range, 256
// / RPT columns per block at a time, four rows in flight per lane.
__device__ inline int copy_rpt(int m) {
  int rpt = 1;
  while (rpt < m && rpt < 64) rpt <<= 1;
  return rpt;
}

// Rows [x, y) of an output column, val(r) each: 16-byte nontemporal stores on
// the row pairs aligned to 16 bytes in memory, a scalar store at an unaligned
// end.  Lanes lane, lane + step, ... take the pairs; on a wavefront's short
// columns (!wide) four pairs per lane are read before any is written.
template <class V>
__device__ __forceinline__ void put_rows(double* out, int x, int y, int lane, int step, bool wide, V val) {
  typedef double d2_t __attribute__((ext_vector_type(2)));
  if (x >= y) return;
  const int a = (int)(((uintptr_t)out >> 3) & 1);  // rows a, a + 2, ... start 16-byte pairs
  const int p0 = (x - a + 1) >> 1, p1 = (y - a) >> 1;
  if (lane == 0) {
    if (x < a + 2 * p0) out[x] = val(x);
    if (a + 2 * p1 < y) out[y - 1] = val(y - 1);
  }
  d2_t* o2 = (d2_t*)(out + a);
  if (wide) {  // (long columns: this streaming loop keeps the memory system busy by itself)
#pragma unroll 4
    for (int p = p0 + lane; p < p1; p += step) {
      const int r = a + 2 * p;
      __builtin_nontemporal_store(d2_t{val(r), val(r + 1)}, &o2[p]);
    }
  } else {
    constexpr int U = 4;
    for (int pb = p0 + lane; pb < p1; pb += U * step) {
      d2_t v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = a + 2 * (pb + u * step);
        v[u] = (pb + u * step < p1) ? d2_t{val(r), val(r + 1)} : d2_t{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (pb + u * step < p1) __builtin_nontemporal_store(v[u], &o2[pb + u * step]);
    }
  }
}

__device__ void copy_body(const BlockMap& bm, const Scratch& S, int b) {
  const int mi = find_merge(bm, b);
  const int lb = b - merge_first_block(bm, mi);
  const int G = merge_blocks(bm, mi);
  const MergeDesc M = bm.descs[mi];
  const int m = M.m;
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  const int nd1 = cnt[C_ND1], nd = nd1 + cnt[C_ND2];
  const int64_t so = M.s_off;
  if (M.root) {
    // The caller's Q: every row is written -- rows [0, m), or, when Q was
    // zero-filled beforehand, only the rows of the column's range.  A
    // whole block per column (a wave per column below kCopyWideRows rows),
    // rows in pairs with 16-byte nontemporal stores (nothing here reads Q
    // again, so the lines need not stay in the caches).  On the short columns
    // of a wave, up to 4 row pairs per lane are read before any is written,
    // and the next column's list entry and destination are read while the
    // current one is in flight.
    const bool wide = m >= kCopyWideRows;
    const bool pre = (M.flags & kFlagPrefilled) != 0;
    const int lane = wide ? threadIdx.x : (threadIdx.x & 63), step = wide ? 256 : 64;
    const int q0 = wide ? lb : lb * 4 + (threadIdx.x >> 6), qs = wide ? G : G * 4;
    auto entry = [&](int q, int& c, int& dst) {
      if (q < nd1) { c = S.dfc1[so + q]; dst = S.destd1[so + q]; }
      else { const int q2 = q - nd1; c = S.dfc2[so + q2]; dst = S.destd2[so + q2]; }
    };
    int c = 0, dst = 0;
    if (q0 < nd) entry(q0, c, dst);
    for (int q = q0; q < nd; q += qs) {
      const RowRange g = S.crng[so + c];
      int cn = 0, dn = 0;
      if (!wide && q + qs < nd) entry(q + qs, cn, dn);
      const double* src = M.qin + (int64_t)c * M.ldin;
      double* out = M.qout + (int64_t)dst * M.ldout;
      auto val = [&](int r) { return (r >= g.lo && r < g.hi) ? src[r] : 0.0; };
      put_rows(out, pre ? g.lo : 0, pre ? g.hi : m, lane, step, wide, val);
      if (wide) {
        if (q + qs < nd) entry(q + qs, cn, dn);
      }
      c = cn;
      dst = dn;
    }
    return;
  }
  const int rpt = copy_rpt(m);
  const int cpb = 256 / rpt;
  const int lane = threadIdx.x % rpt, sub = threadIdx.x / rpt;
  for (int q = lb * cpb + sub; q < nd; q += G * cpb) {
    int c, dst;
    if (q < nd1) { c = S.dfc1[so + q]; dst = S.destd1[so + q]; }
    else { const int q2 = q - nd1; c = S.dfc2[so + q2]; dst = S.destd2[so + q2]; }
    const RowRange g = S.crng[so + c];
    const double* src = M.qin + (int64_t)c * M.ldin;
    double* out = M.qout + (int64_t)dst * M.ldout;
    const int w0 = M.root ? 0 : g.lo, w1 = M.root ? m : g.hi;  // rows written
    constexpr int U = 4;
    for (int r0 = w0 + lane; r0 < w1; r0 += U * rpt) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = r0 + u * rpt;
        v[u] = (r >= g.lo && r < g.hi) ? src[r] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = r0 + u * rpt;
        if (r < w1) out[r] = v[u];
      }
    }
  }
}

// ------------------------------------------------------------ block maps

bool small_merge(int m, const phdc_opts* o) {
  if (m > kSmallMergeMax || o->gemm_mode == PHDC_GEMM_SPLIT) return false;
  return !(o->gemm_mode == PHDC_GEMM_HSS && m >= std::max<int64_t>(o->hss_min_K, 1));
}

int map_blocks(int kind, int m, int n1, int gt, bool root, bool small, int nm, bool sec_wide) {
  auto cdiv = [](int a, int b) { return (a + b - 1) / b; };
  if (small || kind == MAP_SMALL) return (small && kind == MAP_SMALL) ? 1 : 0;
  const int share = cdiv(kLevelBlocks, std::max(nm, 1));  // this merge's part of a full level launch
  auto trim = [&](int full, int unit) {  // at least one unit, whole units, at most full
    return full <= share ? full : unit * std::max(1, share / unit);
  };
  switch (kind) {
    case MAP_SECULAR: return trim(cdiv(m, kSecThreads / (sec_wide ? kSecGWide : kSecG)), 1);
    case MAP_ROOTS16: return trim(cdiv(m, kSecThreads / (sec_wide ? kSecGWide : kItemG)), 1);
    case MAP_ROWS256: return cdiv(m, 256);
    case MAP_ROT: return trim(cdiv(m, 256) * std::max(1, std::min(m / 2, kRotGroups)), cdiv(m, 256));
    case MAP_UWRITE: return trim(cdiv(m, 256) * std::max(1, std::min(m, kUwRowGroups)), cdiv(m, 256));
    case MAP_GEMM:  // edge-64 tiles
      return trim(std::min((cdiv(n1, 64) + cdiv(m - n1, 64)) * cdiv(m, 64), kGemmBlockCap), 1);
    case MAP_COPY: {
      // root: a block per column from kCopyWideRows rows, else a wave per column;
      // below the root, 256 / (m rounded up to a power of two, at most 64) per block
      if (root) return trim(std::max(1, std::min(m >= kCopyWideRows ? m : cdiv(m, 4), kCopyBlocks)), 1);
      int rpt = 1;
      while (rpt < m && rpt < 64) rpt <<= 1;
      return trim(std::max(1, std::min(cdiv(m, 256 / rpt), kCopyBlocks)), 1);
    }
    case MAP_SPLITA: return cdiv(m, 256) * kSplitKGroups;
    case MAP_SPLITB: return cdiv(m + 8, 256) * kSplitRGroups;
    case MAP_PREP: return m >= kDefPrepRows ? cdiv(m, kPrepThreads) : 0;
    case MAP_DEFL1: return m >= kDefPrepRows ? cdiv(m, kDefT1Threads) : 0;
  }
  return 0;
}


// Zero fill of the caller's Q (FillDesc): every row of every column (k = 0),
// or the off-diagonal quadrants (column c < k gets zeros in rows [k, n),
// column c >= k in rows [0, k)), or with diag the diagonal halves (the other
// rows).  A block of NT threads per column (wide) or a wave per column; cpfx:
// prefix of the column counts of the nd matrices.
template <int NT>
__global__ void __launch_bounds__(NT) k_fill_zero(const FillDesc* __restrict__ fd, const int32_t* __restrict__ cpfx,
                                                  int nd, int total, int wide, int diag) {
  constexpr int W = NT / 64;
  const int first = wide ? (int)blockIdx.x : (int)blockIdx.x * W + (int)(threadIdx.x >> 6);
  const int stride = wide ? (int)gridDim.x : (int)gridDim.x * W;
  const int lane = wide ? (int)threadIdx.x : (int)(threadIdx.x & 63), step = wide ? NT : 64;
  auto zero = [](int) { return 0.0; };
  for (int col = first; col < total; col += stride) {  // (uniform per wave or block)
    int lo = 0, hi = nd - 1;  // the matrix holding col: cpfx[lo] <= col < cpfx[lo + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cpfx[mid] <= col) lo = mid;
      else hi = mid - 1;
    }
    const FillDesc F = fd[lo];
    const int c = col - cpfx[lo];
    double* out = F.q + (int64_t)c * F.ld;
    if (F.k == 0) put_rows(out, 0, F.n, lane, step, wide != 0, zero);
    else if ((c < F.k) != (diag != 0)) put_rows(out, F.k, F.n, lane, step, wide != 0, zero);
    else put_rows(out, 0, F.k, lane, step, wide != 0, zero);
  }
}

void launch_fill_zero(const FillDesc* fd, const int32_t* cpfx, int nd, int total, bool wide, bool diag,
                      int max_blocks, hipStream_t s) {
  if (nd <= 0 || total <= 0) return;
  constexpr int W = kFillThreads / 64;
  const int blocks = std::max(1, std::min(max_blocks, wide ? total : (total + W - 1) / W));
  hipLaunchKernelGGL(k_fill_zero<kFillThreads>, dim3(blocks), dim3(kFillThreads), 0, s, fd, cpfx, nd, total,
                     wide ? 1 : 0, diag ? 1 : 0);
}

__global__ void __launch_bounds__(256) k_copy_ints(const int32_t* __restrict__ src, int32_t* dst, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------ fused stages
// A tree level runs as a few launches, each the union of steps that depend on
// the same earlier ones (a launch costs a few microseconds of fixed latency,
// comparable to the work of the upper levels): the block index picks the step.
// The longest-running blocks come first in each launch, so that they are
// dispatched before the many short ones.
//   deflate | rotations + secular roots | Loewner z + output ranks |
//   column norms + Uhat (unscaled) + deflated-column copy | update GEMM
// Levels of merges with at most kSmallUhat rows do roots, Loewner z, norms, Uhat
// and ranks in one workgroup per merge.  When Uhat must hold normalized columns
// (a level with HSS candidates, whose compression samples Uhat itself, or the
// split-precision path), the norms come first in a launch of their own.

// Dynamic LDS: 2 cap doubles, cap = min(largest merge of the level, kSecLds).
template <int G>
__global__ void __launch_bounds__(256) k_stage_roots(BlockMap sec, int nsec, BlockMap rot, Scratch S, int cap) {
  HIP_DYNAMIC_SHARED(double, lds)
  const int b = blockIdx.x;
  if (b < nsec) secular_body<G>(sec, S, b, lds, lds + cap, cap);
  else rotate_body(rot, S, b - nsec);
}

__global__ void __launch_bounds__(kStageSmallThreads) k_stage_small(const MergeDesc* __restrict__ descs, Scratch S,
                                                                    int normalized) {
  __shared__ double sd[kSmallUhat];
  __shared__ double sz[kSmallUhat];
  const MergeDesc M = descs[blockIdx.x];
  if (M.flags & kFlagSmallMerge) return;  // done by k_merge_small
  small_body<kStageSmallThreads, kSecG>(M, S, normalized != 0, sd, sz);
}

// ------------------------------------------------------------ one-workgroup merges
// A merge of at most kSmallMergeMax rows on the FP64 path runs in one
// workgroup from deflation to the eigenvector update.  Three shapes: levels of
// many such merges (at least kSmallManyMerges: the GPU is full and throughput
// counts) take one wavefront per merge and one lane per secular root -- at
// these sizes every loop is a single pass, the block barriers cost nothing,
// and a CU holds up to twenty merges; levels of fewer merges take 1024
// threads and kSecG lanes per root, for the shortest latency per merge, or
// 256 threads and four lanes per root when the merges have at most 32 rows.
// The update product runs on the FP64 matrix cores, one wave per 16 x 16
// output tile: the two column lists are staged in LDS, Uhat (grouped rows)
// and the input columns are read directly; then the deflated columns are
// copied.
constexpr int kSmallManyMerges = 2048;
typedef double d4s_t __attribute__((ext_vector_type(4)));

// cl, rl: LDS for 2 kSmallMergeMax columns and row ranges (top list, then
// bottom list).  Uhat is read where this workgroup wrote it (cache-resident).
template <int NT>
__device__ void small_update(const MergeDesc& M, const Scratch& S, int32_t* cl, RowRange* rl) {
  const int t = threadIdx.x, m = M.m, n1 = M.n1, n2 = M.m - M.n1;
  const int32_t* cnt = S.counters + (int64_t)M.id * kCounters;
  const int K = cnt[C_K], k1 = cnt[C_K1], k2 = cnt[C_K2], k3 = cnt[C_K3];
  const int kt = k1 + k2, kb = k2 + k3;
  const int64_t so = M.s_off;
  for (int x = t; x < kt; x += NT) {
    cl[x] = S.coltop[so + x];
    rl[x] = S.rgtop[so + x];
  }
  for (int x = t; x < kb; x += NT) {
    cl[kSmallMergeMax + x] = S.colbot[so + x];
    rl[kSmallMergeMax + x] = S.rgbot[so + x];
  }
  const double* U = S.uhat + M.u_off;  // (written by this workgroup before the barrier)
  __syncthreads();
  // Row tiles of 16 per half (a tile never straddles the halves), column tiles
  // of 16 roots.  v_mfma_f64_16x16x4f64: A(i, k) from lane 16 k + i, B(k, j)
  // from lane 16 k + j, result element q of lane l at (l / 16 + 4 q, l % 16).
  const int tt = (n1 + 15) / 16, tb = (n2 + 15) / 16, TM = tt + tb, TN = (K + 15) / 16;
  const int lane = t & 63, li = lane & 15, lk = lane >> 4;
  constexpr int NS = kSmallMergeMax / 4;  // k-steps of 4
  for (int tile = t >> 6; tile < TM * TN; tile += NT / 64) {
    const int mt = tile % TM, nt = tile / TM;
    const bool top = mt < tt;
    const int r0 = top ? mt * 16 : n1 + (mt - tt) * 16;  // first merge row of the tile
    const int rend = top ? n1 : m;
    const int kd = top ? kt : kb;
    const int off = top ? 0 : k1;  // first grouped row of Uhat this half uses
    const int32_t* ca = cl + (top ? 0 : kSmallMergeMax);
    const RowRange* ra = rl + (top ? 0 : kSmallMergeMax);
    const int r = r0 + li, j = nt * 16 + li;
    d4s_t acc = {0.0, 0.0, 0.0, 0.0};
    // k-steps in two halves: each half's loads are issued together, then its MFMAs
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      constexpr int NH = NS / 2;
      double av[NH], bv[NH];
#pragma unroll
      for (int qq = 0; qq < NH; ++qq) {
        const int k = 4 * (h * NH + qq) + lk;
        av[qq] = 0.0;
        bv[qq] = 0.0;
        if (k < kd) {
          const RowRange g = ra[k];
          if (r < rend && r >= g.lo && r < g.hi) av[qq] = M.qin[r + (int64_t)ca[k] * M.ldin];
          if (j < K) bv[qq] = U[(off + k) * K + j];
        }
      }
#pragma unroll
      for (int qq = 0; qq < NH; ++qq)
        if (4 * (h * NH + qq) < kd)  // (wave-uniform)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[qq], bv[qq], acc, 0, 0, 0);
    }
    if (j < K) {
      double* oc = M.qout + (int64_t)S.dest[so + j] * M.ldout;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = r0 + lk + 4 * q;
        if (rr < rend) oc[rr] = acc[q];
      }
    }
  }
  // deflated columns: over their range (every row when the merge is a root)
  const int nd1 = cnt[C_ND1], nd = nd1 + cnt[C_ND2];
  for (int x = t; x < nd * kSmallMergeMax; x += NT) {
    const int q = x / kSmallMergeMax, r = x % kSmallMergeMax;
    if (r >= m) continue;
    int c, dst;
    if (q < nd1) { c = S.dfc1[so + q]; dst = S.destd1[so + q]; }
    else { c = S.dfc2[so + q - nd1]; dst = S.destd2[so + q - nd1]; }
    const RowRange g = S.crng[so + c];
    const bool in = r >= g.lo && r < g.hi;
    if (in || M.root) M.qout[r + (int64_t)dst * M.ldout] = in ? M.qin[r + (int64_t)c * M.ldin] : 0.0;
  }
}

// Dynamic LDS: kmax doubles, kmax = the largest such merge of the level (at
// most kSmallMergeMax); it holds the poles during deflation.  (Five waves per
// SIMD: the register budget that fits five 256-thread merges per CU, or twenty
// one-wave merges, without spilling.)
template <int NT, int G>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5))) k_merge_small(BlockMap bm, Scratch S) {
  HIP_DYNAMIC_SHARED(double, Us)
  __shared__ double sd[kSmallUhat];
  __shared__ double sz[kSmallUhat];
  __shared__ int32_t cl[2 * kSmallMergeMax];
  __shared__ RowRange rl[2 * kSmallMergeMax];
  const int mi = find_merge(bm, blockIdx.x);
  const MergeDesc M = bm.descs[mi];
  deflate_body<NT, 1>(M, S, M.m, Us);  // (m <= 64: one element per thread, one chunk per wave)
  __syncthreads();
  small_body<NT, G>(M, S, true, sd, sz);
  __syncthreads();
  small_update<NT>(M, S, cl, rl);
}

template <int IG>
__global__ void __launch_bounds__(256) k_stage_lowner(BlockMap low, int nlow, BlockMap rank, Scratch S) {
  const int b = blockIdx.x;
  if (b < nlow) lowner_body<IG>(low, S, b);
  else rank_body(rank, S, b - nlow);
}

template <int IG>
__global__ void __launch_bounds__(256) k_stage_uhat(BlockMap cp, int ncp, BlockMap uw, int nuw, BlockMap un, Scratch S,
                                                    int normalized) {
  const int b = blockIdx.x;
  if (b < ncp) copy_body(cp, S, b);
  else if (b < ncp + nuw) uwrite_body(uw, S, b - ncp, normalized != 0);
  else unorm_body<IG>(un, S, b - ncp - nuw);
}

void launch_merge_level(const MergeDesc* descs, int nm, const LevelMaps& maps, const Scratch& S, int gemm_mode,
                        const SplitBufs* split, int nsl, hipStream_t s, const LevelProbe* probe,
                        hipEvent_t qout_ready) {
  if (nm <= 0) return;
  auto bmap = [&](int kind) { return BlockMap{descs, maps.pfx[kind], nm, maps.per[kind]}; };
  const BlockMap none{descs, nullptr, 1, 1};
  const int normalized = maps.uhat_normalized ? 1 : 0;
  const int nsmall = maps.total[MAP_SMALL];
  if (nsmall > 0) {  // merges that run in one workgroup each, deflation included
    ProfScope p(PH_SMALL_MERGE, s);
    const int kmax = std::min(maps.maxm, kSmallMergeMax);
    const size_t lds = (size_t)kmax * sizeof(double);
    if (nsmall >= kSmallManyMerges)
      hipLaunchKernelGGL((k_merge_small<64, 1>), dim3(nsmall), dim3(64), lds, s, bmap(MAP_SMALL), S);
    else if (kmax <= 32)
      hipLaunchKernelGGL((k_merge_small<256, 4>), dim3(nsmall), dim3(256), lds, s, bmap(MAP_SMALL), S);
    else
      hipLaunchKernelGGL((k_merge_small<1024, kSecG>), dim3(nsmall), dim3(1024), lds, s, bmap(MAP_SMALL), S);
    if (nsmall == nm) return;  // (no HSS candidate in such a level: no probe needed)
  }
  { ProfScope p(PH_DEFLATE, s);
    if (maps.total[MAP_PREP] > 0)
      hipLaunchKernelGGL(k_deflate_prep, dim3(maps.total[MAP_PREP]), dim3(kPrepThreads), 0, s, bmap(MAP_PREP), S);
    if (maps.total[MAP_DEFL1] > 0)
      hipLaunchKernelGGL(k_deflate_t1, dim3(maps.total[MAP_DEFL1]), dim3(kDefT1Threads), 0, s, bmap(MAP_DEFL1), S);
    const int cap = maps.maxm <= kDefLdsMax ? maps.maxm : 0;
    if (maps.maxm <= kDefSmall)
      hipLaunchKernelGGL(k_deflate<256>, dim3(nm), dim3(256), (size_t)cap * sizeof(double), s, descs, S, cap);
    else
      hipLaunchKernelGGL(k_deflate<kDefThreads>, dim3(nm), dim3(kDefThreads), (size_t)cap * sizeof(double), s, descs,
                         S, cap); }
  if (probe && probe->count > 0) {
    hipLaunchKernelGGL(k_copy_ints, dim3((probe->count + 255) / 256), dim3(256), 0, s, probe->src, probe->dst,
                       probe->count);
    (void)hipEventRecord(probe->done, s);
  }
  const int nrot = maps.total[MAP_ROT];
  const int ncopy = maps.total[MAP_COPY];
  if (maps.maxm <= kSmallUhat) {
    { ProfScope p(PH_SECULAR, s);
      hipLaunchKernelGGL(k_stage_small, dim3(nm), dim3(kStageSmallThreads), 0, s, descs, S, normalized); }
    { ProfScope p(PH_UWRITE, s);  // (the copy phase times the lone root copy only)
      hipLaunchKernelGGL(k_stage_uhat<kItemG>, dim3(ncopy), dim3(256), 0, s, bmap(MAP_COPY), ncopy, none, 0, none, S, 0); }
  } else {
    const int nsec = maps.total[MAP_SECULAR], nitem = maps.total[MAP_ROOTS16], nrank = maps.total[MAP_ROWS256];
    const int nuw = maps.total[MAP_UWRITE];
    // items (Loewner z, column norms) take as many lanes as the level's secular roots
    const auto k_lowner = maps.sec_wide ? k_stage_lowner<kSecGWide> : k_stage_lowner<kItemG>;
    const auto k_uhat = maps.sec_wide ? k_stage_uhat<kSecGWide> : k_stage_uhat<kItemG>;
    { ProfScope p(PH_SECULAR, s);
      const int cap = std::min(maps.maxm, kSecLds);
      if (maps.sec_wide)
        hipLaunchKernelGGL(k_stage_roots<kSecGWide>, dim3(nsec + nrot), dim3(256), (size_t)2 * cap * sizeof(double),
                           s, bmap(MAP_SECULAR), nsec, bmap(MAP_ROT), S, cap);
      else
        hipLaunchKernelGGL(k_stage_roots<kSecG>, dim3(nsec + nrot), dim3(256), (size_t)2 * cap * sizeof(double), s,
                           bmap(MAP_SECULAR), nsec, bmap(MAP_ROT), S, cap); }
    { ProfScope p(PH_LOWNER, s);
      hipLaunchKernelGGL(k_lowner, dim3(nitem + nrank), dim3(256), 0, s, bmap(MAP_ROOTS16), nitem,
                         bmap(MAP_ROWS256), S); }
    const int nc = maps.copy_alone ? 0 : ncopy;
    // the launches below write output blocks: a zero fill of a root's output
    // (rows >= kFillMinRows, so never in the small branches above) ends first
    if (qout_ready) (void)hipStreamWaitEvent(s, qout_ready, 0);
    if (normalized) {
      { ProfScope p(PH_UNORM, s);
        hipLaunchKernelGGL(k_uhat, dim3(nitem), dim3(256), 0, s, none, 0, none, 0, bmap(MAP_ROOTS16), S, 1); }
      { ProfScope p(PH_UWRITE, s);
        hipLaunchKernelGGL(k_uhat, dim3(nc + nuw), dim3(256), 0, s, bmap(MAP_COPY), nc, bmap(MAP_UWRITE), nuw,
                           none, S, 1); }
    } else {
      ProfScope p(PH_UWRITE, s);
      hipLaunchKernelGGL(k_uhat, dim3(nc + nuw + nitem), dim3(256), 0, s, bmap(MAP_COPY), nc, bmap(MAP_UWRITE),
                         nuw, bmap(MAP_ROOTS16), S, 0);
    }
    if (maps.copy_alone) {
      ProfScope p(PH_COPY, s);
      hipLaunchKernelGGL(k_stage_uhat<kItemG>, dim3(ncopy), dim3(256), 0, s, bmap(MAP_COPY), ncopy, none, 0, none, S, 0);
    }
  }
  { ProfScope p(PH_GEMM, s);
    launch_merge_gemm_f64(bmap(MAP_GEMM), maps.total[MAP_GEMM], S, maps.gemm_tile, !normalized, s); }
  if (gemm_mode == PHDC_GEMM_SPLIT && split) {
    ProfScope p(PH_SPLIT_GEMM, s);
    launch_split_update(descs, nm, maps, S, *split, nsl, s);
  }
}

__global__ void k_mark_fallback(const MergeDesc* __restrict__ desc, int32_t* counters) {
  int32_t* cnt = counters + (int64_t)desc->id * kCounters;
  cnt[C_PATH] = 0;
  cnt[C_HSSRANK] = -1;
}

// Runs after the merge's level: the column norms exist, so Uhat is rewritten
// normalized, in the grouped row order of the FP64 product.
void launch_fp64_fallback(const MergeDesc* desc, const MergeDesc& M, const Scratch& S, hipStream_t s) {
  const int tile = gemm_tile_for(M.m);
  const int nuw = map_blocks(MAP_UWRITE, M.m, M.n1, tile, M.root != 0);
  const int ngm = map_blocks(MAP_GEMM, M.m, M.n1, tile, M.root != 0);
  const BlockMap none{desc, nullptr, 1, 1};
  hipLaunchKernelGGL(k_mark_fallback, dim3(1), dim3(1), 0, s, desc, S.counters);
  hipLaunchKernelGGL(k_stage_uhat<kItemG>, dim3(nuw), dim3(256), 0, s, none, 0, BlockMap{desc, nullptr, 1, nuw}, nuw, none,
                     S, 1);  // Uhat only
  launch_merge_gemm_f64(BlockMap{desc, nullptr, 1, ngm}, ngm, S, tile, false, s);
}

void launch_secular_standalone(int64_t K, const double* d, const double* z, double rho, int32_t* org, double* tau,
                               int32_t* status, hipStream_t s) {
  if (K <= 0) return;
  const int per = 64 / kSecG;
  hipLaunchKernelGGL(k_secular_raw, dim3((unsigned)((K + per - 1) / per)), dim3(64), 0, s, (int)K, d, z, rho, org, tau,
                     status);
}

}  // namespace phdc
