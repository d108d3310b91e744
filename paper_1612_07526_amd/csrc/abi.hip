// C-ABI entry points and the host-side planner of libphdc.so.
//
// The planner lays out the Cuppen split tree (Eq. (2)) of every matrix: blocks
// are halved (first half floor(m/2)) until they have at most leaf_size rows.
// Leaves are solved in one launch; merges are grouped by height (a leaf has
// height 0, a merge one more than its taller child) and each height is one
// batched launch per kernel.  A node at depth t writes its eigenvectors to the
// caller's buffers when t is even and to the workspace twin when t is odd, so
// a merge always reads its children from the other buffer than it writes --
// except that a matrix whose root is zero-filled ahead of time (see run_solve)
// keeps the eigenvectors of its even depths below the root in a third
// workspace buffer, so that nothing but the root writes the caller's Q.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "phdc_internal.h"
#include "profile.h"
#include "hss.h"
#include "split.h"

namespace phdc {

void launch_canonical_sign(const void* descs, const int32_t* pfx, int nmat, int total, hipStream_t s);
void launch_clear_status(int32_t* status, hipStream_t s);

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Node {
  int32_t b;      // matrix
  int64_t r0;     // first row within the matrix
  int32_t m, n1;  // size, first half (merges)
  int32_t depth, height;
};

struct Tree {
  std::vector<Node> leaves;
  std::vector<Node> merges;  // sorted by height, stable
  std::vector<int32_t> hstart;  // merges of height h: [hstart[h-1], hstart[h]) for h >= 1
  int32_t root_merge = -1;      // id of matrix 0's root merge (or -1)
};

int build_node(Tree& T, int32_t b, int64_t r0, int32_t m, int32_t depth, int leaf) {
  if (m <= leaf) {
    T.leaves.push_back(Node{b, r0, m, 0, depth, 0});
    return 0;
  }
  const int32_t k = m / 2;
  const int h1 = build_node(T, b, r0, k, depth + 1, leaf);
  const int h2 = build_node(T, b, r0 + k, m - k, depth + 1, leaf);
  const int h = 1 + std::max(h1, h2);
  T.merges.push_back(Node{b, r0, m, k, depth, h});
  return h;
}

Tree build_tree(const std::vector<int64_t>& n, int leaf) {
  Tree T;
  for (size_t b = 0; b < n.size(); ++b)
    if (n[b] > 0) build_node(T, (int32_t)b, 0, (int32_t)n[b], 0, leaf);
  std::stable_sort(T.merges.begin(), T.merges.end(),
                   [](const Node& a, const Node& c) { return a.height < c.height; });
  int H = T.merges.empty() ? 0 : T.merges.back().height;
  T.hstart.assign(H + 1, 0);
  for (int h = 1; h <= H; ++h) {
    T.hstart[h] = T.hstart[h - 1];
    while (T.hstart[h] < (int)T.merges.size() && T.merges[T.hstart[h]].height == h) ++T.hstart[h];
  }
  for (size_t i = 0; i < T.merges.size(); ++i)
    if (T.merges[i].b == 0 && T.merges[i].depth == 0) T.root_merge = (int32_t)i;
  return T;
}

// Sizes that determine the workspace.
struct Sizes {
  int64_t n_total = 0;     // rows over all matrices (scratch arrays)
  int64_t q_total = 0;     // elements of the eigenvector twin buffer
  int64_t q3_total = 0;    // elements of the third eigenvector buffer (zero-filled roots' even depths)
  int64_t nmerges = 0, nleaves = 0, nmats = 0;
  int64_t uhat = 0;        // elements of the Uhat arena
  int64_t map_ints = 0;    // block-map prefix entries
  int H = 0;
  size_t hss_arena = 0;    // HSS working storage (largest HSS-eligible merge)
  size_t hss_desc = 0;     // HSS descriptor staging area
  int64_t xslots = 0;      // split precision: max over levels of sum m (m + 8) (per slice, bf16)
  int nsl = 0;             // split precision: slices per operand (0: path off)
};

struct Layout {
  size_t status, hdr, counters, mparam, descs, leaves, canon, canon_pfx, maps, fill, fill_pfx, scratch, uhat, qtwin,
      ltwin, ranges, hss, hss_desc, sa, sb, serow, sfcol, qthird, total;
};

constexpr int kScratchD = 17, kScratchI = 18;  // 8-byte arrays (doubles, row ranges), int32 arrays

int32_t hss_threshold(const phdc_opts* o) {
  if (!o || o->gemm_mode != PHDC_GEMM_HSS) return 0;
  return (int32_t)std::min<int64_t>(std::max<int64_t>(o->hss_min_K, 1), 1 << 30);
}

int split_slices(const phdc_opts* o) {
  if (!o || o->gemm_mode != PHDC_GEMM_SPLIT) return 0;
  return std::min(kSplitMaxSlices, std::max(1, o->split_slices));
}

// split-precision slot of one merge (per slice, in bf16 elements), a multiple of 8
int64_t xslot(int64_t m) { return (m * (m + 8) + 7) / 8 * 8; }

int hss_dmax(const phdc_opts* o) {
  return std::min(512, std::max(16, o->hss_samples) + 2 * std::max(16, o->hss_samples_inc));
}

Sizes sizes_of(const Tree& T, const std::vector<int64_t>& n, int64_t q_total, const phdc_opts* o) {
  Sizes z;
  for (auto x : n) z.n_total += x;
  z.q_total = q_total;
  z.nmerges = (int64_t)T.merges.size();
  z.nleaves = (int64_t)T.leaves.size();
  z.nmats = (int64_t)n.size();
  z.H = (int)T.hstart.size() - 1;
  for (int h = 1; h <= z.H; ++h) {
    int64_t u = 0;
    for (int i = T.hstart[h - 1]; i < T.hstart[h]; ++i) u += (int64_t)T.merges[i].m * T.merges[i].m;
    z.uhat = std::max(z.uhat, u);
    z.map_ints += (int64_t)MAP_COUNT * (T.hstart[h] - T.hstart[h - 1] + 1);
    int64_t x = 0;
    for (int i = T.hstart[h - 1]; i < T.hstart[h]; ++i) x += xslot(T.merges[i].m);
    z.xslots = std::max(z.xslots, x);
  }
  z.nsl = split_slices(o);
  if (!z.nsl) z.xslots = 0;
  const int32_t thr = hss_threshold(o);
  if (thr > 0) {
    int64_t mh = 0;
    for (auto& nd : T.merges)
      if (nd.m >= thr) mh = std::max<int64_t>(mh, nd.m);
    if (mh > 0) {
      z.hss_arena = hss_arena_bytes(mh, mh, o->hss_leaf, hss_dmax(o), true);
      z.hss_desc = (size_t)16 << 20;
    }
  }
  return z;
}

Layout layout_of(const Sizes& z) {
  Layout L;
  size_t p = 0;
  auto take = [&](size_t bytes) {
    size_t at = p;
    p = align_up(p + std::max<size_t>(bytes, 1));
    return at;
  };
  L.status = take(256);
  L.hdr = take(256);
  L.counters = take((size_t)std::max<int64_t>(z.nmerges, 1) * kCounters * 4);
  L.mparam = take((size_t)std::max<int64_t>(z.nmerges, 1) * 4 * 8);
  L.descs = take((size_t)z.nmerges * sizeof(MergeDesc));
  L.leaves = take((size_t)z.nleaves * sizeof(LeafArgs));
  L.canon = take((size_t)z.nmats * sizeof(CanonDesc));
  L.canon_pfx = take((size_t)(z.nmats + 1) * 4);
  L.maps = take((size_t)z.map_ints * 4);
  L.fill = take((size_t)z.nmats * sizeof(FillDesc));
  L.fill_pfx = take((size_t)(z.nmats + 2) * 4);
  L.scratch = take((size_t)z.n_total * (kScratchD * 8 + kScratchI * 4) + kScratchD * kAlign + kScratchI * kAlign);
  L.uhat = take((size_t)z.uhat * 8);
  L.qtwin = take((size_t)z.q_total * 8);
  L.ltwin = take((size_t)z.n_total * 8);
  L.ranges = take((size_t)z.n_total * 2 * sizeof(RowRange));  // column ranges, one set per eigenvector buffer
  L.hss = take(z.hss_arena);
  L.hss_desc = take(z.hss_desc);
  L.sa = take((size_t)z.nsl * z.xslots * 2);
  L.sb = take((size_t)z.nsl * z.xslots * 2);
  L.serow = take(z.nsl ? (size_t)z.n_total * 4 : 0);
  L.sfcol = take(z.nsl ? (size_t)z.n_total * 4 : 0);
  L.qthird = take((size_t)z.q3_total * 8);
  L.total = p;
  return L;
}

Scratch scratch_of(char* base, const Layout& L, const Sizes& z) {
  Scratch S;
  char* p = base + L.scratch;
  auto dtake = [&]() {
    double* r = (double*)p;
    p += align_up((size_t)z.n_total * 8);
    return r;
  };
  auto itake = [&]() {
    int32_t* r = (int32_t*)p;
    p += align_up((size_t)z.n_total * 4);
    return r;
  };
  auto rtake = [&]() { return (RowRange*)dtake(); };  // 8 bytes per entry, like a double
  S.dv = dtake(); S.zv = dtake(); S.ds = dtake(); S.zs = dtake(); S.rc = dtake(); S.rs = dtake();
  S.dfv1 = dtake(); S.dfv2 = dtake(); S.tau = dtake(); S.dorg = dtake(); S.zhat = dtake(); S.cnorm = dtake();
  S.rgtop = rtake(); S.rgbot = rtake(); S.crng = rtake(); S.rrp = rtake(); S.rrj = rtake();
  S.col = itake(); S.part = itake(); S.flag = itake(); S.surv = itake(); S.grp = itake(); S.coltop = itake();
  S.colbot = itake(); S.rcolp = itake(); S.rcolj = itake(); S.chain = itake();
  S.dfc1 = itake(); S.dfc2 = itake(); S.org = itake(); S.dest = itake();
  S.destd1 = itake(); S.destd2 = itake(); S.grpsrc = itake(); S.csort = itake();
  S.mparam = (double*)(base + L.mparam);
  S.uhat = (double*)(base + L.uhat);
  S.counters = (int32_t*)(base + L.counters);
  S.status = (int32_t*)(base + L.status);
  return S;
}

SplitBufs split_of(char* base, const Layout& L) {
  SplitBufs B;
  B.aslice = (__bf16*)(base + L.sa);
  B.bslice = (__bf16*)(base + L.sb);
  B.erow = (int32_t*)(base + L.serow);
  B.fcol = (int32_t*)(base + L.sfcol);
  B.kgroups = kSplitKGroups;
  B.rgroups = kSplitRGroups;
  return B;
}

// Pinned staging buffer for an upload.  The next upload through the same
// buffer waits for the previous one to finish before reusing it.
struct Staging {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

// Pinned, device-mapped host memory for the counters the HSS path reads back
// (LevelProbe), and the event that marks their arrival.
struct Probe {
  int32_t* host = nullptr;
  int32_t* dev = nullptr;
  size_t cap = 0;  // int32 values
  hipEvent_t done = nullptr;
};

// Host-side state kept per workspace address: staging for the plan upload and
// for the HSS descriptors, the HSS counter probe, and the prepared plan of
// phdc_stedc_batched_prepare.  phdc_release frees it.
struct WorkState {
  Staging plan, hss;
  Probe probe;
  hipEvent_t fill_ev[4] = {};  // the zero fill's second stream: fork and join of its two phases
};
std::mutex g_mu;
std::unordered_map<const void*, WorkState> g_state;

// Fork and join events of phase `phase` (0 or 1) of the zero fill of a
// workspace (created once; false if they cannot be).
bool fill_events(const void* work, int phase, hipEvent_t* fork, hipEvent_t* join) {
  std::lock_guard<std::mutex> lk(g_mu);
  WorkState& w = g_state[work];
  hipEvent_t* ev = w.fill_ev + 2 * phase;
  for (int i = 0; i < 2; ++i)
    if (!ev[i] && hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
      ev[i] = nullptr;
      return false;
    }
  *fork = ev[0];
  *join = ev[1];
  return true;
}

void free_staging(Staging& st) {
  if (st.pending) hipEventSynchronize(st.done);
  if (st.host) hipHostFree(st.host);
  if (st.done) hipEventDestroy(st.done);
  st = Staging{};
}

int upload_through(Staging& st, void* dst, const std::vector<char>& bytes, hipStream_t s) {
  if (st.pending) {
    hipEventSynchronize(st.done);
    st.pending = false;
  }
  if (st.cap < bytes.size()) {
    if (st.host) hipHostFree(st.host);
    st.host = nullptr;
    st.cap = 0;
    if (hipHostMalloc(&st.host, bytes.size(), hipHostMallocDefault) != hipSuccess) return PHDC_E_HIP;
    st.cap = bytes.size();
  }
  if (!st.done && hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) return PHDC_E_HIP;
  std::memcpy(st.host, bytes.data(), bytes.size());
  if (hipMemcpyAsync(dst, st.host, bytes.size(), hipMemcpyHostToDevice, s) != hipSuccess) return PHDC_E_HIP;
  if (hipEventRecord(st.done, s) != hipSuccess) return PHDC_E_HIP;
  st.pending = true;
  return 0;
}

// Upload of a solve's plan through the workspace's staging buffer.
int upload(const void* work, void* dst, const std::vector<char>& bytes, hipStream_t s) {
  if (bytes.empty()) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  return upload_through(g_state[work].plan, dst, bytes, s);
}

template <class T>
void put(std::vector<char>& buf, size_t at, const T* src, size_t count) {
  if (count == 0) return;
  if (buf.size() < at + count * sizeof(T)) buf.resize(at + count * sizeof(T));
  std::memcpy(buf.data() + at, src, count * sizeof(T));
}

bool opts_ok(const phdc_opts* o) {
  return o->leaf_size >= 2 && o->leaf_size <= kMaxLeaf && o->gemm_mode >= 0 && o->gemm_mode <= 2 &&
         o->hss_leaf >= 8 && o->hss_leaf <= kHssLeafMax && o->hss_samples >= 16 && o->hss_samples <= 512 &&
         o->hss_samples_inc >= 0 && o->hss_rel_tol > 0.0 && o->hss_rel_tol < 1.0 && o->split_slices >= 1 &&
         o->split_slices <= kSplitMaxSlices;
}

// Everything one solve needs: tree, sizes and layout.
struct Setup {
  Tree T;
  Sizes z;
  Layout L;
  std::vector<int64_t> q3off;  // per matrix: its offset in the third eigenvector buffer, or -1
};

// The third eigenvector buffer of an m-row matrix: the blocks of its two
// depth-1 nodes (first half floor(m/2) rows), one after the other, each with
// its own leading dimension.
int64_t third_elems(int64_t m) {
  const int64_t m1 = m / 2;
  return m1 * m1 + (m - m1) * (m - m1);
}

// fill: roots of at least kFillMinRows rows in the last level are zero-filled
// ahead of time (their matrices take the third buffer); off for the
// allocation-free entry point, whose static workspace is sized without it.
Setup setup_for(const std::vector<int64_t>& n, int64_t q_total, const phdc_opts* o, bool fill = true) {
  Setup S;
  S.T = build_tree(n, o->leaf_size);
  S.z = sizes_of(S.T, n, q_total, o);
  S.q3off.assign(n.size(), -1);
  const int H = S.z.H;
  if (fill && H >= 1)
    for (int i = S.T.hstart[H - 1]; i < S.T.hstart[H]; ++i) {
      const Node& nd = S.T.merges[i];
      if (nd.depth != 0 || nd.m < kFillMinRows) continue;
      S.q3off[nd.b] = S.z.q3_total;
      S.z.q3_total += third_elems(nd.m);
    }
  S.L = layout_of(S.z);
  return S;
}

struct Buffers {
  const double* d;
  const double* e;
  int64_t nd = 0, ne = 0;  // entries of d and e over all matrices
  double* lam[2];
  double* q[2];
  RowRange* rng[2];                      // column ranges of q[0], q[1] (indexed like lam)
  std::vector<int64_t> off, eoff, qoff;  // per matrix
  std::vector<int64_t> ld[2];            // per matrix
  double* q3 = nullptr;                  // third eigenvector buffer
  std::vector<int64_t> q3off;            // per matrix (Setup::q3off)
};

// Eigenvector block of the node of matrix b (mb rows) at depth t whose rows
// start at r0, and its leading dimension: the caller's Q at even depth, the
// twin at odd depth, or, for the even depths below a zero-filled root, the
// third buffer (inside the block of the depth-1 node the rows belong to,
// blocks of one depth on that block's diagonal like everywhere else).
double* qblock(const Buffers& BF, int64_t b, int64_t mb, int t, int64_t r0, int64_t* ld) {
  if (t >= 2 && (t & 1) == 0 && BF.q3off[b] >= 0) {
    const int64_t m1 = mb / 2;
    const bool second = r0 >= m1;
    const int64_t w = second ? mb - m1 : m1, x = second ? r0 - m1 : r0;
    *ld = w;
    return BF.q3 + BF.q3off[b] + (second ? m1 * m1 : 0) + x + x * w;
  }
  const int p = t & 1;
  *ld = BF.ld[p][b];
  return BF.q[p] + BF.qoff[b] + r0 + r0 * *ld;
}


// The level's merges that may take the HSS path (m >= hss_min_K), as the id
// range [lo, hi] (ids of one level are consecutive).  False if there are none.
bool hss_candidates(const MergeDesc* hdescs, int nm, const phdc_opts* o, int32_t* lo, int32_t* hi) {
  const int32_t thr = hss_threshold(o);
  if (thr <= 0) return false;
  bool any = false;
  for (int i = 0; i < nm; ++i) {
    if (hdescs[i].m < thr) continue;
    *lo = any ? std::min(*lo, hdescs[i].id) : hdescs[i].id;
    *hi = any ? std::max(*hi, hdescs[i].id) : hdescs[i].id;
    any = true;
  }
  return any;
}

// A probe for the counters of merges lo..hi on the workspace's mapped buffer.
int make_probe(const void* work, const Scratch& S, int32_t lo, int32_t hi, LevelProbe* lp) {
  const size_t n = (size_t)(hi - lo + 1) * kCounters;
  std::lock_guard<std::mutex> lk(g_mu);
  Probe& p = g_state[work].probe;
  if (p.cap < n) {
    if (p.host) hipHostFree(p.host);
    p.host = p.dev = nullptr;
    p.cap = 0;
    if (hipHostMalloc((void**)&p.host, n * 4, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
      return PHDC_E_HIP;
    if (hipHostGetDevicePointer((void**)&p.dev, p.host, 0) != hipSuccess) return PHDC_E_HIP;
    p.cap = n;
  }
  if (!p.done && hipEventCreateWithFlags(&p.done, hipEventDisableTiming) != hipSuccess) return PHDC_E_HIP;
  *lp = LevelProbe{S.counters + (int64_t)lo * kCounters, p.dev, (int32_t)n, p.done};
  return 0;
}

// HSS update of the merges of one level that kept K >= hss_min_K poles.  The
// path was chosen on the device.  The host needs K: with a probe it waits for
// the counter copy made right after deflation (the rest of the level keeps the
// GPU busy meanwhile); without one it copies the counters and synchronises.
// A merge whose compression gives up (ranks beyond the largest sample count,
// an arena or descriptor area too small, or the PHDC_FAIL_HSS test hook) is
// finished with the FP64 product instead (Sec. 2.2: Gu's GEMMs whenever HSS
// does not apply).  ddev: the level's device descriptors (same order as hdescs).
int run_hss_level(const MergeDesc* hdescs, const MergeDesc* ddev, int nm, const Scratch& S, char* arena,
                  size_t arena_bytes, char* descarea, size_t desc_bytes, const phdc_opts* o, hipStream_t s,
                  const void* work, const LevelProbe* probe = nullptr) {
  int32_t lo = 0, hi = 0;
  if (!hss_candidates(hdescs, nm, o, &lo, &hi)) return 0;
  std::vector<int32_t> c((size_t)(hi - lo + 1) * kCounters);
  if (probe) {
    if (hipEventSynchronize(probe->done) != hipSuccess) return PHDC_E_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    std::memcpy(c.data(), g_state[work].probe.host, c.size() * 4);
  } else if (hipMemcpyAsync(c.data(), S.counters + (int64_t)lo * kCounters, c.size() * 4, hipMemcpyDeviceToHost,
                            s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess) {
    return PHDC_E_HIP;
  }
  for (int i = 0; i < nm; ++i) {
    if (hdescs[i].m < hss_threshold(o)) continue;
    const int32_t* ci = c.data() + (size_t)(hdescs[i].id - lo) * kCounters;
    if (ci[C_PATH] != 2) continue;
    int rc = run_hss_merge(hdescs[i], ci[C_K], S, arena, arena_bytes, descarea, desc_bytes, o,
                           S.counters + (int64_t)hdescs[i].id * kCounters, work, s);
    if (rc == PHDC_E_HIP) return rc;
    if (rc != 0) {
      launch_fp64_fallback(ddev + i, hdescs[i], S, s);
      if (hipGetLastError() != hipSuccess) return PHDC_E_HIP;
    }
  }
  return 0;
}

// Everything the kernel launches of a solve need once its plan is on the device.
struct Prepared {
  Scratch S;
  SplitBufs SB;
  Layout L;
  Sizes z;
  std::vector<int32_t> hstart;
  std::vector<LevelMaps> lm;
  int nleaves = 0, nmat = 0, ncols = 0;
  int nfill = 0, nfill_wide = 0;  // matrices of the off-block fill (the wide ones first)
  int fill_cols_wide = 0, fill_cols = 0;
  int fill_level = 1;   // the fill starts before this level
  int fill2_level = 1;  // its second phase (diagonal halves of the wide matrices) before this one
  phdc_opts o;
  const double* d = nullptr;  // inputs, for the optional non-finite scan
  const double* e = nullptr;
  int64_t nd = 0, ne = 0;
};
std::mutex g_pm_mu;
std::unordered_map<const void*, Prepared> g_prepared;

void forget_prepared(const void* work) {
  std::lock_guard<std::mutex> lk(g_pm_mu);
  g_prepared.erase(work);
}

int leaf_iters(const phdc_opts* o) { return (o->force_fail & PHDC_FAIL_LEAF) ? 0 : kLeafMaxIters; }

// Start phase `phase` of the zero fill: on the auxiliary stream after what s
// has queued, its completion recorded in *join (returns true: the last level
// waits for *join before writing output blocks), or on s itself when no second
// stream or event is available (returns false).  Phase 0: the off-diagonal
// quadrants of the wide matrices (kFillWideRows rows and more) and all of the
// narrow ones; phase 1: the diagonal halves of the wide ones.
bool start_fill(char* base, const Prepared& P, hipStream_t s, int phase, hipEvent_t* join) {
  const FillDesc* fd = (const FillDesc*)(base + P.L.fill);
  const int32_t* pfx = (const int32_t*)(base + P.L.fill_pfx);
  hipStream_t a = aux_stream();
  hipEvent_t fork = nullptr;
  const bool forked = a && fill_events(base, phase, &fork, join) && hipEventRecord(fork, s) == hipSuccess &&
                      hipStreamWaitEvent(a, fork, 0) == hipSuccess;
  hipStream_t fs = forked ? a : s;
  {
    ProfScope p(PH_FILL, fs);
    launch_fill_zero(fd, pfx, P.nfill_wide, P.fill_cols_wide, true, phase == 1, kFillBlocksWide, fs);
    if (phase == 0)
      launch_fill_zero(fd + P.nfill_wide, pfx + P.nfill_wide + 1, P.nfill - P.nfill_wide,
                       P.fill_cols - P.fill_cols_wide, false, false, kFillBlocksNarrow, fs);
  }
  return forked && hipEventRecord(*join, a) == hipSuccess;
}

// The zero fill around the levels of a solve: phase 0 starts before level
// P.fill_level, phase 1 before level P.fill2_level (queued after phase 0 on
// the same stream), and the last level waits for them before writing output
// blocks.
struct FillRun {
  hipEvent_t join[2] = {};
  bool joined[2] = {false, false};
  // before launching level h; returns the level's qout_ready event
  hipEvent_t before_level(char* base, const Prepared& P, hipStream_t s, int h) {
    if (P.nfill <= 0) return nullptr;
    if (h == P.fill_level) joined[0] = start_fill(base, P, s, 0, &join[0]);
    if (h == P.fill2_level && P.nfill_wide > 0) joined[1] = start_fill(base, P, s, 1, &join[1]);
    if (h != P.z.H) return nullptr;
    return joined[1] ? join[1] : joined[0] ? join[0] : nullptr;  // (phase 1 runs after phase 0)
  }
};

// Launch every kernel of a prepared solve: no host synchronisation, no memcpy,
// no memset -- safe to capture in a HIP graph and replay.
void launch_prepared_all(char* base, const Prepared& P, hipStream_t s) {
  launch_clear_status(P.S.status, s);
  if (P.o.check_finite) {  // graph-safe: the scan only sets the status word
    launch_scan_finite(P.d, P.nd, P.S.status + 1, P.S.status, s);
    launch_scan_finite(P.e, P.ne, P.S.status + 2, P.S.status, s);
  }
  {
    ProfScope p(PH_LEAF, s);
    launch_leaf_ql((const LeafArgs*)(base + P.L.leaves), P.nleaves, P.S.status, P.o.leaf_size, leaf_iters(&P.o), s);
  }
  FillRun fill;
  const MergeDesc* dd = (const MergeDesc*)(base + P.L.descs);
  for (int h = 1; h <= P.z.H; ++h) {
    const int a = P.hstart[h - 1], e = P.hstart[h];
    const hipEvent_t ready = fill.before_level(base, P, s, h);
    launch_merge_level(dd + a, e - a, P.lm[h], P.S, P.o.gemm_mode, &P.SB, P.z.nsl, s, nullptr, ready);
  }
  if (P.o.canonical_sign && P.ncols > 0) {
    ProfScope p(PH_CANON, s);
    launch_canonical_sign(base + P.L.canon, (const int32_t*)(base + P.L.canon_pfx), P.nmat, P.ncols, s);
  }
}

// Build the device plan (descriptors, leaves, block maps), upload it and
// launch every kernel of the solve.  With prepare_only the plan is uploaded
// synchronously and kept for phdc_launch_prepared instead.
// no_alloc: upload the plan from pageable host memory and wait for the upload
// (no pinned staging buffer is allocated); the HSS path is not taken.
int run_solve(const Setup& SU, const Buffers& BF, const std::vector<int64_t>& n, void* work, const phdc_opts* o,
              hipStream_t s, bool prepare_only = false, bool no_alloc = false) {
  const Tree& T = SU.T;
  const Sizes& z = SU.z;
  const Layout& L = SU.L;
  char* base = (char*)work;
  Scratch S = scratch_of(base, L, z);
  SplitBufs SB = split_of(base, L);

  std::vector<char> plan;
  const size_t plan0 = L.hdr;  // plan region spans hdr .. maps (contiguous)
  plan.resize(L.scratch - plan0, 0);
  put(plan, 0, &T.root_merge, 1);
  const int32_t nmerges32 = (int32_t)T.merges.size();
  put(plan, 4, &nmerges32, 1);

  std::vector<MergeDesc> descs(T.merges.size());
  std::vector<int64_t> uoff(T.merges.size(), 0), xoff(T.merges.size(), 0);
  for (int h = 1; h <= z.H; ++h) {
    int64_t u = 0, x = 0;
    for (int i = T.hstart[h - 1]; i < T.hstart[h]; ++i) {
      uoff[i] = u;
      xoff[i] = x;
      u += (int64_t)T.merges[i].m * T.merges[i].m;
      x += xslot(T.merges[i].m);
    }
  }
  for (size_t i = 0; i < T.merges.size(); ++i) {
    const Node& nd = T.merges[i];
    const int pout = nd.depth & 1, pin = pout ^ 1;
    MergeDesc& D = descs[i];
    std::memset(&D, 0, sizeof(D));
    const int64_t b = nd.b;
    D.qin = qblock(BF, b, n[b], nd.depth + 1, nd.r0, &D.ldin);
    D.qout = qblock(BF, b, n[b], nd.depth, nd.r0, &D.ldout);
    D.lin = BF.lam[pin] + BF.off[b] + nd.r0;
    D.lout = BF.lam[pout] + BF.off[b] + nd.r0;
    D.zgiven = nullptr;
    D.ecoup = BF.e + BF.eoff[b] + nd.r0 + nd.n1 - 1;
    D.rho = 0.0;
    D.zsign = 1.0;
    D.m = nd.m;
    D.n1 = nd.n1;
    D.s_off = BF.off[b] + nd.r0;
    D.u_off = uoff[i];
    D.id = (int32_t)i;
    D.hss_min_k = hss_threshold(o);
    D.x_off = xoff[i];
    D.split_on = z.nsl > 0 ? 1 : 0;
    D.flags = ((o->force_fail & PHDC_FAIL_SECULAR) ? kFlagNoSecularIters : 0) |
              (small_merge(nd.m, o) ? kFlagSmallMerge : 0) | (nd.m >= kDefPrepRows ? kFlagPrepDeflate : 0);
    D.rin = BF.rng[pin] + BF.off[b] + nd.r0;
    D.rout = BF.rng[pout] + BF.off[b] + nd.r0;
    D.r0 = (int32_t)nd.r0;
    D.root = nd.depth == 0 ? 1 : 0;
  }
  // Roots in the last level with a third buffer (Setup::q3off): nothing but
  // the root writes the caller's Q of such a matrix, so that Q is zero-filled
  // on a second stream while the tree below runs, and the root's copy of its
  // deflated columns then writes only the rows of each column's range.  The
  // fill holds about half the compute units while it runs, which slows the
  // levels beside it: a wide Q is filled in two phases, its off-diagonal
  // quadrants from the first levels on and its diagonal halves only a few
  // levels before the root, where they cost the least.  Wide matrices first,
  // then narrow ones.
  std::vector<FillDesc> fills;
  int nfw = 0;
  if (!no_alloc && z.H >= 1) {
    for (int pass = 0; pass < 2; ++pass)
      for (int i = T.hstart[z.H - 1]; i < T.hstart[z.H]; ++i) {
        const Node& nd = T.merges[i];
        if (nd.depth != 0 || nd.m < kFillMinRows) continue;
        if ((nd.m >= kFillWideRows) != (pass == 0)) continue;
        descs[i].flags |= kFlagPrefilled;
        fills.push_back(FillDesc{BF.q[0] + BF.qoff[nd.b], BF.ld[0][nd.b], nd.m, pass == 0 ? nd.n1 : 0});
        if (pass == 0) ++nfw;
      }
  }
  std::vector<int32_t> fpfx(fills.size() + 2, 0);  // wide group [0, nfw], narrow group [nfw + 1, ...]
  for (int i = 0; i < nfw; ++i) fpfx[i + 1] = fpfx[i] + fills[i].n;
  for (size_t i = nfw; i < fills.size(); ++i) fpfx[i + 2] = fpfx[i + 1] + fills[i].n;
  if (!fills.empty()) {
    put(plan, L.fill - plan0, fills.data(), fills.size());
    put(plan, L.fill_pfx - plan0, fpfx.data(), fpfx.size());
  }
  put(plan, L.descs - plan0, descs.data(), descs.size());

  std::vector<LeafArgs> leaves(T.leaves.size());
  for (size_t i = 0; i < T.leaves.size(); ++i) {
    const Node& nd = T.leaves[i];
    const int p = nd.depth & 1;
    const int64_t b = nd.b;
    LeafArgs& A = leaves[i];
    std::memset(&A, 0, sizeof(A));
    A.d = BF.d + BF.off[b] + nd.r0;
    A.e = BF.e + BF.eoff[b] + nd.r0;
    A.q = qblock(BF, b, n[b], nd.depth, nd.r0, &A.ldq);
    A.lam = BF.lam[p] + BF.off[b] + nd.r0;
    A.s = nd.m;
    A.couple = (nd.r0 > 0 ? 1 : 0) | (nd.r0 + nd.m < n[b] ? 2 : 0);
    A.rng = BF.rng[p] + BF.off[b] + nd.r0;
    A.r0 = (int32_t)nd.r0;
  }
  put(plan, L.leaves - plan0, leaves.data(), leaves.size());

  std::vector<CanonDesc> canon(n.size());
  std::vector<int32_t> cpfx(n.size() + 1, 0);
  for (size_t b = 0; b < n.size(); ++b) {
    canon[b] = CanonDesc{BF.q[0] + BF.qoff[b], BF.ld[0][b], (int32_t)n[b], 0};
    cpfx[b + 1] = cpfx[b] + (int32_t)n[b];
  }
  put(plan, L.canon - plan0, canon.data(), canon.size());
  put(plan, L.canon_pfx - plan0, cpfx.data(), cpfx.size());

  std::vector<int32_t> maps;
  maps.reserve((size_t)z.map_ints);
  std::vector<LevelMaps> lm(z.H + 1);
  std::vector<int32_t> blk;  // blocks per merge of a level, kind-major
  for (int h = 1; h <= z.H; ++h) {
    const int a = T.hstart[h - 1], e = T.hstart[h];
    for (int i = a; i < e; ++i) lm[h].maxm = std::max(lm[h].maxm, T.merges[i].m);
    lm[h].gemm_tile = (o->gemm_mode == PHDC_GEMM_SPLIT) ? 128 : gemm_tile_for(lm[h].maxm);
    // Uhat keeps unit columns where something other than the FP64 GEMM reads it:
    // the split-precision slicer, or the HSS sampling of a level with candidates
    lm[h].uhat_normalized = o->gemm_mode == PHDC_GEMM_SPLIT || (hss_threshold(o) > 0 && lm[h].maxm >= hss_threshold(o));
    lm[h].copy_alone = (e - a == 1) && T.merges[a].depth == 0;
    int64_t rows = 0;
    for (int i = a; i < e; ++i) rows += T.merges[i].m;
    lm[h].sec_wide = rows <= kSecWideRows;
    // a merge's block counts depend on its size, split and depth (and the
    // level): merges of a level mostly share them, so they are reused
    const int nm = e - a;
    blk.assign((size_t)MAP_COUNT * nm, 0);
    for (int i = a; i < e; ++i) {
      const Node& nd = T.merges[i];
      const bool same = i > a && nd.m == T.merges[i - 1].m && nd.n1 == T.merges[i - 1].n1 &&
                        (nd.depth == 0) == (T.merges[i - 1].depth == 0);
      for (int k = 0; k < MAP_COUNT; ++k)
        blk[(size_t)k * nm + (i - a)] =
            same ? blk[(size_t)k * nm + (i - a - 1)]
                 : map_blocks(k, nd.m, nd.n1, lm[h].gemm_tile, nd.depth == 0, small_merge(nd.m, o), nm, lm[h].sec_wide);
    }
    for (int k = 0; k < MAP_COUNT; ++k) {
      const size_t at = maps.size();
      int32_t acc = 0, first = -1;
      bool equal = true;
      maps.push_back(0);
      for (int i = 0; i < nm; ++i) {
        const int32_t bl = blk[(size_t)k * nm + i];
        if (first < 0) first = bl;
        else if (bl != first) equal = false;
        acc += bl;
        maps.push_back(acc);
      }
      lm[h].pfx[k] = (const int32_t*)(base + L.maps) + at;
      lm[h].total[k] = acc;
      lm[h].per[k] = (equal && first > 0) ? first : 0;
    }
  }
  put(plan, L.maps - plan0, maps.data(), maps.size());
  plan.resize(L.scratch - plan0);

  Prepared P;
  P.S = S;
  P.SB = SB;
  P.L = L;
  P.z = z;
  P.hstart = T.hstart;
  P.lm = lm;
  P.nleaves = (int)T.leaves.size();
  P.nmat = (int)n.size();
  P.ncols = cpfx.back();
  P.o = *o;
  P.d = BF.d;
  P.e = BF.e;
  P.nd = BF.nd;
  P.ne = BF.ne;
  P.nfill = (int)fills.size();
  P.nfill_wide = nfw;
  P.fill_cols_wide = fpfx[nfw];
  P.fill_cols = fpfx[nfw] + fpfx[fills.size() + 1];
  // the fill starts once the levels of one-workgroup merges are queued (its
  // traffic would stretch their steps), at the last level at latest
  P.fill_level = 1;
  while (P.fill_level < z.H && lm[P.fill_level].maxm <= kSmallMergeMax && small_merge(lm[P.fill_level].maxm, o))
    ++P.fill_level;
  P.fill2_level = std::max(P.fill_level, z.H - kFillLateLevels);
  if (prepare_only) {
    if (hipStreamSynchronize(s) != hipSuccess) return PHDC_E_HIP;
    if (hipMemcpy(base + plan0, plan.data(), plan.size(), hipMemcpyHostToDevice) != hipSuccess) return PHDC_E_HIP;
    std::lock_guard<std::mutex> lk(g_pm_mu);
    g_prepared[work] = P;
    return 0;
  }
  forget_prepared(work);  // the plan on the device is about to change
  P.o.check_finite = 0;   // the entry point has scanned the inputs already
  if (no_alloc) {
    if (hss_threshold(o) > 0) return -9;
    if (hipMemcpyAsync(base + plan0, plan.data(), plan.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PHDC_E_HIP;
    launch_prepared_all(base, P, s);
    return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
  }
  if (hss_threshold(o) <= 0) {
    if (upload(work, base + plan0, plan, s) != 0) return PHDC_E_HIP;
    launch_prepared_all(base, P, s);
    return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
  }
  // HSS: the host reads K back after each level that has eligible merges
  launch_clear_status(S.status, s);
  if (upload(work, base + plan0, plan, s) != 0) return PHDC_E_HIP;
  FillRun fill;
  {
    ProfScope p(PH_LEAF, s);
    launch_leaf_ql((const LeafArgs*)(base + L.leaves), (int)T.leaves.size(), S.status, o->leaf_size, leaf_iters(o),
                   s);
  }
  const MergeDesc* dd = (const MergeDesc*)(base + L.descs);
  for (int h = 1; h <= z.H; ++h) {
    const int a = T.hstart[h - 1], e = T.hstart[h];
    const hipEvent_t ready = fill.before_level(base, P, s, h);
    int32_t lo = 0, hi = 0;
    LevelProbe lp{};
    const bool cand = hss_candidates(descs.data() + a, e - a, o, &lo, &hi);
    if (cand && make_probe(work, S, lo, hi, &lp) != 0) return PHDC_E_HIP;
    launch_merge_level(dd + a, e - a, lm[h], S, o->gemm_mode, &SB, z.nsl, s, cand ? &lp : nullptr, ready);
    if (!cand) continue;
    int rc = run_hss_level(descs.data() + a, dd + a, e - a, S, base + L.hss, L.hss_desc - L.hss, base + L.hss_desc,
                           z.hss_desc, o, s, work, &lp);
    if (rc != 0) return rc;
  }
  if (o->canonical_sign && cpfx.back() > 0) {
    ProfScope p(PH_CANON, s);
    launch_canonical_sign(base + L.canon, (const int32_t*)(base + L.canon_pfx), (int)n.size(), cpfx.back(), s);
  }
  return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
}

// The optional input scan of an entry point: waits for it and returns the
// 1-based index of the first array argument holding a NaN or Inf (0: none, or
// PHDC_E_HIP).  On a hit the status word is PHDC_ERR_NONFINITE.
int scan_inputs(int32_t* status, const double* a0, int64_t n0, int arg0, const double* a1, int64_t n1, int arg1,
                hipStream_t s) {
  launch_clear_status(status, s);
  launch_scan_finite(a0, n0, status + 1, status, s);
  launch_scan_finite(a1, n1, status + 2, status, s);
  int32_t f[3] = {0, 0, 0};
  if (hipMemcpyAsync(f, status, sizeof(f), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return PHDC_E_HIP;
  return f[1] ? arg0 : f[2] ? arg1 : 0;
}

}  // namespace

int hss_upload(const void* work, void* dst, const std::vector<char>& bytes, hipStream_t s) {
  if (bytes.empty()) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  return upload_through(g_state[work].hss, dst, bytes, s);
}

}  // namespace phdc

using namespace phdc;

extern "C" {

void phdc_opts_default(phdc_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->leaf_size = 16;
  o->gemm_mode = PHDC_GEMM_FP64;
  o->hss_min_K = 4096;
  o->hss_rel_tol = 1e-14;
  o->hss_leaf = 256;
  o->hss_samples = 192;
  o->hss_samples_inc = 128;
  o->split_slices = 6;
  o->seed = 0x9e3779b97f4a7c15ULL;
  o->canonical_sign = 0;
  o->check_finite = 0;
  o->force_fail = 0;
}

int phdc_version(void) { return 1; }

}  // extern "C"

size_t phdc::stedc_workspace_bytes(int64_t n, const phdc_opts* o, bool fill) {
  return setup_for({n}, n * n, o, fill).L.total;
}

extern "C" {

int phdc_stedc_workspace(int64_t n, const phdc_opts* o, size_t* bytes) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (n < 0) return -1;
  if (!opts_ok(o)) return -2;
  if (!bytes) return -3;
  Setup SU = setup_for({n}, n * n, o);
  *bytes = SU.L.total;
  return 0;
}

int phdc_stedc(int64_t n, const double* d, const double* e, double* lambda, double* Q, int64_t ldq, void* work,
               size_t lwork, const phdc_opts* o, void* stream) {
  return stedc_impl(n, d, e, lambda, Q, ldq, work, lwork, o, (hipStream_t)stream, false);
}

}  // extern "C"

// phdc_stedc; no_alloc: the plan upload allocates nothing (phdc_stedc_noalloc).
int phdc::stedc_impl(int64_t n, const double* d, const double* e, double* lambda, double* Q, int64_t ldq, void* work,
                     size_t lwork, const phdc_opts* o, hipStream_t stream, bool no_alloc) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (n < 0) return -1;
  if (n > 0 && !d) return -2;
  if (n > 1 && !e) return -3;
  if (n > 0 && !lambda) return -4;
  if (n > 0 && !Q) return -5;
  if (ldq < std::max<int64_t>(1, n)) return -6;
  if (!work) return -7;
  if (!opts_ok(o)) return -9;
  if (n > (int64_t)1 << 30) return -1;
  Setup SU = setup_for({n}, n * n, o, !no_alloc);
  if (lwork < SU.L.total) return -8;
  if (((uintptr_t)work & (kAlign - 1)) != 0) return -7;
  if (n == 0) {
    forget_prepared(work);
    launch_clear_status((int32_t*)work, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
  }
  if (o->check_finite) {
    const int bad = scan_inputs((int32_t*)work, d, n, 2, e, n - 1, 3, (hipStream_t)stream);
    if (bad != 0) return bad == PHDC_E_HIP ? bad : -bad;
  }
  char* base = (char*)work;
  Buffers BF;
  BF.d = d;
  BF.e = e;
  BF.nd = n;
  BF.ne = n - 1;
  BF.lam[0] = lambda;
  BF.lam[1] = (double*)(base + SU.L.ltwin);
  BF.q[0] = Q;
  BF.q[1] = (double*)(base + SU.L.qtwin);
  BF.rng[0] = (RowRange*)(base + SU.L.ranges);
  BF.rng[1] = BF.rng[0] + n;
  BF.off = {0};
  BF.eoff = {0};
  BF.qoff = {0};
  BF.ld[0] = {ldq};
  BF.ld[1] = {n};
  BF.q3 = (double*)(base + SU.L.qthird);
  BF.q3off = SU.q3off;
  return run_solve(SU, BF, {n}, work, o, stream, false, no_alloc);
}

extern "C" {

int phdc_stedc_batched_workspace(int64_t B, const int64_t* n_host, const phdc_opts* o, size_t* bytes) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (B < 0) return -1;
  if (B > 0 && !n_host) return -2;
  if (!opts_ok(o)) return -3;
  if (!bytes) return -4;
  std::vector<int64_t> n(n_host, n_host + B);
  int64_t q = 0;
  for (auto x : n) {
    if (x < 0) return -2;
    q += x * x;
  }
  Setup SU = setup_for(n, q, o);
  *bytes = SU.L.total;
  return 0;
}

static int stedc_batched_impl(int64_t B, const int64_t* n_host, const int64_t* off_host, const int64_t* qoff_host,
                              const double* d, const double* e, double* lambda, double* Q, void* work, size_t lwork,
                              const phdc_opts* o, void* stream, bool prepare_only);

int phdc_stedc_batched(int64_t B, const int64_t* n_host, const int64_t* off_host, const int64_t* qoff_host,
                       const double* d, const double* e, double* lambda, double* Q, void* work, size_t lwork,
                       const phdc_opts* o, void* stream) {
  return stedc_batched_impl(B, n_host, off_host, qoff_host, d, e, lambda, Q, work, lwork, o, stream, false);
}

int phdc_stedc_batched_prepare(int64_t B, const int64_t* n_host, const int64_t* off_host, const int64_t* qoff_host,
                               const double* d, const double* e, double* lambda, double* Q, void* work,
                               size_t lwork, const phdc_opts* o, void* stream) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (o->gemm_mode == PHDC_GEMM_HSS) return -11;  // the HSS path reads sizes back on the host
  return stedc_batched_impl(B, n_host, off_host, qoff_host, d, e, lambda, Q, work, lwork, o, stream, true);
}

int phdc_launch_prepared(void* work, void* stream) {
  if (!work) return -1;
  Prepared P;
  {
    std::lock_guard<std::mutex> lk(g_pm_mu);
    auto it = g_prepared.find(work);
    if (it == g_prepared.end()) return -1;
    P = it->second;
  }
  launch_prepared_all((char*)work, P, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
}

int phdc_release(void* work) {
  if (!work) return -1;
  forget_prepared(work);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_state.find(work);
  if (it == g_state.end()) return 0;
  WorkState& w = it->second;
  free_staging(w.plan);
  free_staging(w.hss);
  if (w.probe.host) hipHostFree(w.probe.host);
  if (w.probe.done) {
    hipEventSynchronize(w.probe.done);
    hipEventDestroy(w.probe.done);
  }
  for (hipEvent_t ev : w.fill_ev)
    if (ev) {
      hipEventSynchronize(ev);
      hipEventDestroy(ev);
    }
  g_state.erase(it);
  return 0;
}

static int stedc_batched_impl(int64_t B, const int64_t* n_host, const int64_t* off_host, const int64_t* qoff_host,
                              const double* d, const double* e, double* lambda, double* Q, void* work, size_t lwork,
                              const phdc_opts* o, void* stream, bool prepare_only) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (B < 0) return -1;
  if (B > 0 && (!n_host)) return -2;
  if (B > 0 && (!off_host)) return -3;
  if (B > 0 && (!qoff_host)) return -4;
  std::vector<int64_t> n(n_host, n_host + B);
  int64_t acc = 0, qacc = 0;
  for (int64_t b = 0; b < B; ++b) {
    if (n[b] < 0 || n[b] > (1 << 30)) return -2;
    if (off_host[b] != acc) return -3;
    if (qoff_host[b] != qacc) return -4;
    acc += n[b];
    qacc += n[b] * n[b];
  }
  if (acc > 0 && !d) return -5;
  int64_t etot = 0;
  for (int64_t b = 0; b < B; ++b) etot += std::max<int64_t>(n[b] - 1, 0);
  if (etot > 0 && !e) return -6;
  if (acc > 0 && !lambda) return -7;
  if (acc > 0 && !Q) return -8;
  if (!work) return -9;
  if (!opts_ok(o)) return -11;
  Setup SU = setup_for(n, qacc, o);
  if (lwork < SU.L.total) return -10;
  if (((uintptr_t)work & (kAlign - 1)) != 0) return -9;
  if (acc == 0) {
    forget_prepared(work);
    launch_clear_status((int32_t*)work, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
  }
  if (o->check_finite && !prepare_only) {
    const int bad = scan_inputs((int32_t*)work, d, acc, 5, e, etot, 6, (hipStream_t)stream);
    if (bad != 0) return bad == PHDC_E_HIP ? bad : -bad;
  }
  char* base = (char*)work;
  Buffers BF;
  BF.d = d;
  BF.e = e;
  BF.nd = acc;
  BF.ne = etot;
  BF.lam[0] = lambda;
  BF.lam[1] = (double*)(base + SU.L.ltwin);
  BF.q[0] = Q;
  BF.q[1] = (double*)(base + SU.L.qtwin);
  BF.rng[0] = (RowRange*)(base + SU.L.ranges);
  BF.rng[1] = BF.rng[0] + acc;
  BF.off.assign(off_host, off_host + B);
  BF.qoff.assign(qoff_host, qoff_host + B);
  BF.eoff.resize(B);
  int64_t eacc = 0;
  for (int64_t b = 0; b < B; ++b) {
    BF.eoff[b] = eacc;
    eacc += std::max<int64_t>(n[b] - 1, 0);
  }
  BF.ld[0] = n;
  BF.ld[1] = n;
  BF.q3 = (double*)(base + SU.L.qthird);
  BF.q3off = SU.q3off;
  return run_solve(SU, BF, n, work, o, (hipStream_t)stream, prepare_only);
}

int phdc_merge_workspace(int64_t n1, int64_t n2, const phdc_opts* o, size_t* bytes) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  if (n1 < 0) return -1;
  if (n2 < 0) return -2;
  if (!opts_ok(o)) return -3;
  if (!bytes) return -4;
  const int64_t m = n1 + n2;
  Tree T;
  if (m > 0) {
    T.merges.push_back(Node{0, 0, (int32_t)m, (int32_t)n1, 0, 1});
    T.hstart = {0, 1};
  } else {
    T.hstart = {0};
  }
  Sizes z = sizes_of(T, {m}, m * m, o);
  *bytes = layout_of(z).total;
  return 0;
}

int phdc_merge(int64_t n1, int64_t n2, const double* D, const double* z, double rho, const double* Q1,
               int64_t ldq1, const double* Q2, int64_t ldq2, double* lambda, double* Q, int64_t ldq, void* work,
               size_t lwork, const phdc_opts* o, void* stream) {
  phdc_opts def;
  if (!o) { phdc_opts_default(&def); o = &def; }
  const int64_t m = n1 + n2;
  if (n1 < 0) return -1;
  if (n2 < 0) return -2;
  if (m > 0 && !D) return -3;
  if (m > 0 && !z) return -4;
  if (!(rho >= 0.0) || !std::isfinite(rho)) return -5;
  if (n1 > 0 && !Q1) return -6;
  if (ldq1 < std::max<int64_t>(1, n1)) return -7;
  if (n2 > 0 && !Q2) return -8;
  if (ldq2 < std::max<int64_t>(1, n2)) return -9;
  if (m > 0 && !lambda) return -10;
  if (m > 0 && !Q) return -11;
  if (ldq < std::max<int64_t>(1, m)) return -12;
  if (!work) return -13;
  if (!opts_ok(o)) return -15;
  if (m > (int64_t)1 << 30) return -1;
  Tree T;
  if (m > 0) {
    T.merges.push_back(Node{0, 0, (int32_t)m, (int32_t)n1, 0, 1});
    T.hstart = {0, 1};
    T.root_merge = 0;
  } else {
    T.hstart = {0};
  }
  Sizes zs = sizes_of(T, {m}, m * m, o);
  Layout L = layout_of(zs);
  if (lwork < L.total) return -14;
  if (((uintptr_t)work & (kAlign - 1)) != 0) return -13;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)work;
  forget_prepared(work);
  if (m == 0) {
    launch_clear_status((int32_t*)(base + L.status), s);
    return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
  }
  if (o->check_finite) {
    const int bad = scan_inputs((int32_t*)(base + L.status), D, m, 3, z, m, 4, s);
    if (bad != 0) return bad == PHDC_E_HIP ? bad : -bad;
  }
  Scratch S = scratch_of(base, L, zs);
  double* qin = (double*)(base + L.qtwin);
  if (n1 > 0 && hipMemcpy2DAsync(qin, m * 8, Q1, ldq1 * 8, n1 * 8, n1, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return PHDC_E_HIP;
  if (n2 > 0 && hipMemcpy2DAsync(qin + n1 + n1 * m, m * 8, Q2, ldq2 * 8, n2 * 8, n2, hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
    return PHDC_E_HIP;
  MergeDesc Dd;
  std::memset(&Dd, 0, sizeof(Dd));
  Dd.qin = qin;
  Dd.ldin = m;
  Dd.qout = Q;
  Dd.ldout = ldq;
  Dd.lin = D;
  Dd.lout = lambda;
  Dd.zgiven = z;
  Dd.ecoup = nullptr;
  Dd.rho = rho;
  Dd.zsign = 1.0;
  Dd.m = (int32_t)m;
  Dd.n1 = (int32_t)n1;
  Dd.s_off = 0;
  Dd.u_off = 0;
  Dd.id = 0;
  Dd.hss_min_k = hss_threshold(o);
  Dd.x_off = 0;
  Dd.split_on = zs.nsl > 0 ? 1 : 0;
  Dd.flags = ((o->force_fail & PHDC_FAIL_SECULAR) ? kFlagNoSecularIters : 0) |
             (small_merge((int)m, o) ? kFlagSmallMerge : 0) | (m >= kDefPrepRows ? kFlagPrepDeflate : 0);
  Dd.rin = nullptr;  // Q1 and Q2 fill their halves
  Dd.rout = nullptr;
  Dd.r0 = 0;
  Dd.root = 1;
  std::vector<char> plan(L.scratch - L.hdr, 0);
  const int32_t root_and_count[2] = {0, 1};
  std::memcpy(plan.data(), root_and_count, 8);
  std::memcpy(plan.data() + (L.descs - L.hdr), &Dd, sizeof(Dd));
  CanonDesc c{Q, ldq, (int32_t)m, 0};
  int32_t pf[2] = {0, (int32_t)m};
  std::memcpy(plan.data() + (L.canon - L.hdr), &c, sizeof(c));
  std::memcpy(plan.data() + (L.canon_pfx - L.hdr), pf, sizeof(pf));
  std::vector<int32_t> maps;
  LevelMaps lm;
  lm.maxm = (int32_t)m;
  lm.gemm_tile = (o->gemm_mode == PHDC_GEMM_SPLIT) ? 128 : gemm_tile_for(m);
  lm.uhat_normalized = o->gemm_mode == PHDC_GEMM_SPLIT || (hss_threshold(o) > 0 && m >= hss_threshold(o));
  lm.copy_alone = true;
  lm.sec_wide = m <= kSecWideRows;
  for (int k = 0; k < MAP_COUNT; ++k) {
    lm.pfx[k] = (const int32_t*)(base + L.maps) + maps.size();
    lm.total[k] = map_blocks(k, (int)m, (int)n1, lm.gemm_tile, true, small_merge((int)m, o), 1, lm.sec_wide);
    lm.per[k] = lm.total[k] > 0 ? lm.total[k] : 0;
    maps.push_back(0);
    maps.push_back(lm.total[k]);
  }
  std::memcpy(plan.data() + (L.maps - L.hdr), maps.data(), maps.size() * 4);
  launch_clear_status(S.status, s);
  if (upload(work, base + L.hdr, plan, s) != 0) return PHDC_E_HIP;
  SplitBufs SB = split_of(base, L);
  const MergeDesc* ddev = (const MergeDesc*)(base + L.descs);
  launch_merge_level(ddev, 1, lm, S, o->gemm_mode, &SB, zs.nsl, s);
  {
    int rc = run_hss_level(&Dd, ddev, 1, S, base + L.hss, L.hss_desc - L.hss, base + L.hss_desc, zs.hss_desc, o, s,
                           work);
    if (rc != 0) return rc;
  }
  if (o->canonical_sign) launch_canonical_sign(base + L.canon, (const int32_t*)(base + L.canon_pfx), 1, (int)m, s);
  return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
}

int phdc_secular(int64_t K, const double* d, const double* z, double rho, int32_t* org, double* tau, void* work,
                 size_t lwork, void* stream) {
  if (K < 0) return -1;
  if (K > 0 && !d) return -2;
  if (K > 0 && !z) return -3;
  if (!(rho > 0.0) || !std::isfinite(rho)) return -4;
  if (K > 0 && !org) return -5;
  if (K > 0 && !tau) return -6;
  if (!work) return -7;
  if (lwork < 256) return -8;
  hipStream_t s = (hipStream_t)stream;
  launch_clear_status((int32_t*)work, s);
  launch_secular_standalone(K, d, z, rho, org, tau, (int32_t*)work, s);
  return hipGetLastError() == hipSuccess ? 0 : PHDC_E_HIP;
}

int phdc_status(const void* work, void* stream) {
  if (!work) return -1;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PHDC_E_HIP;
  int32_t v = 0;
  if (hipMemcpy(&v, work, 4, hipMemcpyDeviceToHost) != hipSuccess) return PHDC_E_HIP;
  return v;
}

int phdc_merge_stats(const void* work, int32_t* stats_host) {
  if (!work || !stats_host) return -1;
  int32_t root = -1;
  if (hipMemcpy(&root, (const char*)work + 256, 4, hipMemcpyDeviceToHost) != hipSuccess) return -1;
  if (root < 0) {
    std::memset(stats_host, 0, 8 * 4);
    return 0;
  }
  int32_t c[kCounters];
  const char* cnt = (const char*)work + 512;  // counters follow the status and header blocks
  if (hipMemcpy(c, cnt + (size_t)root * kCounters * 4, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  stats_host[0] = c[C_K];
  stats_host[1] = c[C_K1];
  stats_host[2] = c[C_K2];
  stats_host[3] = c[C_K3];
  stats_host[4] = c[C_NT1];
  stats_host[5] = c[C_NT2];
  stats_host[6] = c[C_PATH];
  stats_host[7] = c[C_HSSRANK];
  return 0;
}

int phdc_merge_table(const void* work, int64_t max_rows, int32_t* table_host, int64_t* rows_out) {
  if (!work || !rows_out) return -1;
  int32_t hdr[2] = {-1, 0};
  if (hipMemcpy(hdr, (const char*)work + 256, 8, hipMemcpyDeviceToHost) != hipSuccess) return -1;
  const int64_t nm = hdr[1];
  *rows_out = nm;
  if (!table_host || max_rows <= 0 || nm <= 0) return 0;
  const int64_t rows = std::min<int64_t>(nm, max_rows);
  // counters start at 512; the descriptors follow counters and mparam (layout_of order)
  Sizes z;
  z.nmerges = nm;
  const size_t counters = 512;
  const size_t mparam = align_up(counters + (size_t)std::max<int64_t>(nm, 1) * kCounters * 4);
  const size_t descs = align_up(mparam + (size_t)std::max<int64_t>(nm, 1) * 4 * 8);
  std::vector<int32_t> c((size_t)rows * kCounters);
  std::vector<MergeDesc> d((size_t)rows);
  if (hipMemcpy(c.data(), (const char*)work + counters, c.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return -1;
  if (hipMemcpy(d.data(), (const char*)work + descs, d.size() * sizeof(MergeDesc), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return -1;
  for (int64_t i = 0; i < rows; ++i) {
    int32_t* r = table_host + i * PHDC_MERGE_TABLE_COLS;
    r[0] = d[i].m;
    r[1] = d[i].n1;
    for (int k = 0; k < 8; ++k) r[2 + k] = c[i * kCounters + k];
    r[10] = c[i * kCounters + C_DP1];
    r[11] = c[i * kCounters + C_DP2];
    r[12] = c[i * kCounters + C_DP3];
    r[13] = c[i * kCounters + C_DROWS_LO];
    r[14] = c[i * kCounters + C_DROWS_HI];
    r[15] = d[i].root;
    r[16] = (d[i].flags & kFlagPrefilled) ? 1 : 0;
    r[17] = c[i * kCounters + C_WROWS];
    r[18] = c[i * kCounters + C_WROWS + 1];
  }
  return 0;
}

}  // extern "C"
