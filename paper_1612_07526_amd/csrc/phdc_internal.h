// Internal declarations shared by the HIP translation units of libphdc.so.
// Not part of the public C-ABI (include/phdc.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/phdc.h"

namespace phdc {

constexpr double kUnitRoundoff = 1.1102230246251565e-16;  // 2^-53
constexpr int kMaxLeaf = 64;
constexpr int kHssLeafMax = 1024;    // largest HSS leaf (rows of one interpolative decomposition)
constexpr int kSplitMaxSlices = 7;   // BF16 slices per operand on the split-precision path
constexpr int kCounters = 20;  // per-merge int32 counters

// Counter slots (per merge).
enum : int {
  C_K = 0, C_K1 = 1, C_K2 = 2, C_K3 = 3, C_NT1 = 4, C_NT2 = 5, C_PATH = 6, C_HSSRANK = 7,
  C_NROT = 8, C_NCHAIN = 9, C_ND1 = 10, C_ND2 = 11,
  C_DP1 = 12, C_DP2 = 13, C_DP3 = 14,  // deflated columns nonzero in the Q1 half only / both / the Q2 half only
  C_DROWS_LO = 15, C_DROWS_HI = 16,    // sum over deflated columns of the rows in their range (64 bits)
  C_WROWS = 18                         // prefilled root: rows the deflated-column copy writes (uint64 at 18..19)
};

// Rows [lo, hi) of an eigenvector column that can be nonzero; rows outside
// are structurally zero and their storage is not read.  Columns leave a leaf
// with the leaf's rows, a root of a merge with all its rows, and a deflated
// column with the range it entered the merge with (after the type-2 rotations,
// which join the hulls of the two columns they combine).
struct alignas(8) RowRange {
  int32_t lo, hi;
};

// One rank-one merge of the divide-and-conquer tree.  All pointers are device pointers.
struct MergeDesc {
  double* qin;          // input block origin: rows/cols [0, m) hold diag(Q1, Q2); off-diagonal blocks are scratch
  double* qout;         // output block origin (m x m)
  int64_t ldin, ldout;  // leading dimensions
  const double* lin;    // child eigenvalues D = [D1; D2] (m), each half ascending
  double* lout;         // output eigenvalues (m)
  const double* zgiven; // merge(): caller's z (m); stedc: nullptr (z gathered from qin)
  const double* ecoup;  // stedc: the off-diagonal entry b_k coupling the halves; merge(): nullptr
  double rho;           // merge(): coupling rho >= 0 (stedc: taken from *ecoup)
  double zsign;         // merge(): 1 (stedc: sign of *ecoup)
  int32_t m, n1;        // merge size and size of the first half
  int64_t s_off;        // offset of this merge's m-long slot in the n-long scratch arrays
  int64_t u_off;        // offset of this merge's m*m slot in the Uhat arena
  int32_t id;           // row in the counters table
  int32_t hss_min_k;    // HSS update for this merge when K >= hss_min_k (0: never)
  int64_t x_off;        // offset of this merge's m*(m+8) slot (per slice) in the split-precision arenas
  int32_t split_on;     // split-precision update for this merge
  int32_t flags;        // kFlagNoSecularIters (test hook), kFlagSmallMerge
  const RowRange* rin;  // input column ranges in rows of the whole matrix (nullptr: [0, n1) / [n1, m) by half)
  RowRange* rout;       // output column ranges (nullptr: not recorded)
  int32_t r0;           // first row (= first column) of the merge block within the matrix
  int32_t root;         // 1: last merge of its matrix (every output entry is written, zeros included)
};

// One matrix whose caller-side eigenvector matrix is zero-filled, while the
// tree below its root runs, before the root merge writes it (nothing below the
// root touches that Q: the even depths below it use a workspace buffer of
// their own): all of it at once (k = 0), or in two parts split at row and
// column k (the root's n1): the off-diagonal quadrants, then the diagonal
// halves.
struct FillDesc {
  double* q;  // the matrix's Q (column-major)
  int64_t ld;
  int32_t n, k;  // size; 0, or the first half
};

// One leaf solve (one wavefront).
struct LeafArgs {
  const double* d;     // diagonal at the leaf's first row
  const double* e;     // off-diagonal at the leaf's first row (e[-1] valid if coupled left)
  double* q;           // eigenvector block origin
  int64_t ldq;
  double* lam;         // eigenvalue output
  int32_t s;           // rows
  int32_t couple;      // bit 0: coupled to the left, bit 1: coupled to the right
  RowRange* rng;       // column ranges of the leaf's eigenvectors (nullptr: not recorded)
  int32_t r0;          // first row of the leaf within the matrix
  int32_t pad;
};

// One matrix for the eigenvector sign pass.
struct CanonDesc {
  double* q;
  int64_t ld;
  int32_t n;
  int32_t pad;
};

// Scratch arrays (device pointers into the caller's workspace).  Unless noted
// each is n_total long and merge i uses [s_off, s_off + m).
struct Scratch {
  double* dv;      // poles sorted ascending (modified in place by rotations)
  double* zv;      // z in sorted order (normalised)
  int32_t* col;    // merge column of sorted pole
  int32_t* part;   // 1: rows of Q1 only, 3: rows of Q2 only, 2: both
  int32_t* flag;   // 0 survivor, 1 type-1, 2 type-2
  int32_t* surv;   // sorted indices of the type-1 survivors
  double* ds;      // final survivors: pole
  double* zs;      //                  z
  int32_t* grp;    //                  row of Uhat in Gu's grouped order
  int32_t* coltop; // GEMM column list for the Q1 rows (types 1, 2)
  int32_t* colbot; // GEMM column list for the Q2 rows (types 2, 3)
  RowRange* rgtop; // row range (merge rows) of each column of coltop
  RowRange* rgbot; //                                     of colbot
  RowRange* crng;  // row range (merge rows) of every merge column, after the rotations
  int32_t* rcolp;  // rotation records: column p
  int32_t* rcolj;  //                   column j
  double* rc;      //                   cosine
  double* rs;      //                   sine
  RowRange* rrp;   //                   row range of column p before the rotation (merge rows)
  RowRange* rrj;   //                   row range of column j before the rotation
  int32_t* chain;  // first record of each rotation chain
  double* dfv1;    // type-1 deflated: value (ascending)
  int32_t* dfc1;   //                  column
  double* dfv2;    // type-2 deflated: value
  int32_t* dfc2;   //                  column
  int32_t* org;    // secular root: origin pole
  double* tau;     //                offset
  double* dorg;    //                origin pole value d[org]
  double* zhat;    // Loewner z
  double* cnorm;   // 1 / column norm of Uhat
  int32_t* dest;   // output column of root j (K), then of deflated items
  int32_t* destd1; // output column of type-1 deflated item
  int32_t* destd2; // output column of type-2 deflated item
  int32_t* grpsrc; // survivor that fills grouped row g of Uhat
  int32_t* csort;  // input column of survivor k (pole order)
  double* mparam;  // per merge (4 doubles): normalised rho, deflation tolerance
  double* uhat;    // Uhat arena
  int32_t* counters;
  int32_t* status;
};

// Block map: launch of `total` blocks split over merges by prefix pfx[0..nm].
// When every merge of the launch has the same number of blocks (per > 0) the
// merge of a block is b / per, with no search through pfx.
struct BlockMap {
  const MergeDesc* descs;
  const int32_t* pfx;
  int32_t nm;
  int32_t per;
};

__device__ inline int find_merge(const BlockMap& bm, int b) {
  if (bm.per > 0) return b / bm.per;
  int lo = 0, hi = bm.nm - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (bm.pfx[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// First block of merge mi, and its number of blocks.
__device__ inline int merge_first_block(const BlockMap& bm, int mi) { return bm.per > 0 ? mi * bm.per : bm.pfx[mi]; }
__device__ inline int merge_blocks(const BlockMap& bm, int mi) {
  return bm.per > 0 ? bm.per : bm.pfx[mi + 1] - bm.pfx[mi];
}

__device__ inline void set_status(int32_t* status, int code) {
  // First error wins; written with a vector atomic.
  atomicCAS(status, 0, code);
}

constexpr int32_t kFlagNoSecularIters = 1;  // secular roots get no iterations (test hook)
constexpr int32_t kFlagSmallMerge = 2;      // the whole merge runs in one workgroup (k_merge_small)
constexpr int32_t kFlagPrepDeflate = 4;     // deflation's element-wise first steps run in k_deflate_prep
constexpr int kDefPrepRows = 4096;          // merges from this size take kFlagPrepDeflate
constexpr int32_t kFlagPrefilled = 8;       // root: the caller's Q was zero-filled beforehand
constexpr int kFillMinRows = 256;           // roots from this size take the zero fill
constexpr int kFillWideRows = 2048;         // matrices from this size fill in two phases, a column per block (else per wave)
// Merges of at most this many rows on the FP64 path run in one workgroup each.
constexpr int kSmallMergeMax = 64;
static_assert(kFillMinRows > kSmallMergeMax, "a zero-filled root is never a one-workgroup merge");

// Kernel launchers (defined in the .hip files).  maxit: iteration cap per
// eigenvalue of the leaf QL (0 under the PHDC_FAIL_LEAF test hook).
void launch_leaf_ql(const LeafArgs* leaves, int nleaves, int32_t* status, int max_leaf, int maxit, hipStream_t s);
constexpr int kLeafMaxIters = 64;

// Scan a[0:n) for NaN/Inf: on a hit, flag[0] = 1 and the status word is set to
// PHDC_ERR_NONFINITE.  The flag is only ever set, never cleared.
void launch_scan_finite(const double* a, int64_t n, int32_t* flag, int32_t* status, hipStream_t s);
// Zero the 256-byte status block (status word and the scan flags after it).
void launch_clear_status(int32_t* status, hipStream_t s);
hipStream_t aux_stream();

// Block maps of one merge level (device prefix arrays, nm + 1 entries each).
enum MapKind {
  MAP_SECULAR = 0, MAP_ROOTS16, MAP_ROWS256, MAP_ROT, MAP_UWRITE, MAP_GEMM, MAP_COPY, MAP_SPLITA, MAP_SPLITB, MAP_SMALL,
  MAP_PREP, MAP_DEFL1, MAP_COUNT
};
struct LevelMaps {
  const int32_t* pfx[MAP_COUNT];
  int32_t total[MAP_COUNT];
  int32_t per[MAP_COUNT] = {};  // blocks per merge when equal for all merges of the level, else 0
  int32_t maxm = 0;         // largest merge of the level
  int32_t gemm_tile = 128;  // output tile edge of the FP64 update GEMM (64 or 128)
  bool uhat_normalized = false;  // Uhat written with unit columns (else the GEMM epilogue scales them)
  bool copy_alone = false;       // the deflated-column copy gets a launch of its own (a lone root merge)
  bool sec_wide = false;         // 32 lanes per secular root (levels of at most kSecWideRows rows), else 16
};
// Blocks of one merge for a kernel class; gt is the FP64 GEMM tile edge (MAP_GEMM);
// root: the merge is the last one of its matrix (MAP_COPY: one column per block);
// small: the merge runs in one workgroup of k_merge_small (MAP_SMALL: 1 block,
// every other class 0).
// Blocks of merge (m, n1) in a level of nm merges.  Kinds whose blocks loop
// over their items get fewer blocks per merge once a level would launch more
// than kLevelBlocks (levels of many small merges: the trimmed blocks would
// mostly find no work, yet each costs a dispatch).
constexpr int kLevelBlocks = 16384;
// Levels of at most this many rows over all their merges give each secular
// root 32 lanes (short latency per root); crowded levels give it 16 (more roots
// in flight).
constexpr int kSecWideRows = 65536;
int map_blocks(int kind, int m, int n1, int gt, bool root, bool small = false, int nm = 1, bool sec_wide = false);
// Whether a merge of m rows takes the one-workgroup path for these options.
bool small_merge(int m, const phdc_opts* o);
constexpr int kGemmBlockCap = 1024;      // blocks per merge of the update GEMMs (they loop over tiles)
constexpr int kTileBuckets = 21;        // merge-size buckets of the GEMM tile table (m <= 2^20)
int gemm_tile_for(int64_t maxm);        // tile edge for a level whose largest merge is maxm
// scale_cols: multiply result column j by the column scale cnorm[j] of Uhat
// (Uhat was written unscaled).
void launch_merge_gemm_f64(const BlockMap& bm, int total, const Scratch& S, int tile, bool scale_cols,
                           hipStream_t s);

// Copy of a level's counters to host-visible memory, made right after the
// deflation kernel has fixed the sizes and the update path of every merge.
struct LevelProbe {
  const int32_t* src;  // device counters of the first merge of interest
  int32_t* dst;        // device address of pinned, mapped host memory
  int32_t count;       // int32 values to copy
  hipEvent_t done;     // recorded after the copy
};

struct SplitBufs;
// qout_ready: an event the level waits for before its first write of a
// merge's output block (nullptr: none).
void launch_merge_level(const MergeDesc* descs, int nm, const LevelMaps& maps, const Scratch& S,
                        int gemm_mode, const SplitBufs* split, int nsl, hipStream_t s,
                        const LevelProbe* probe = nullptr, hipEvent_t qout_ready = nullptr);
// Zero-fill the Q of nd matrices (FillDesc; with k > 0 its off-diagonal
// quadrants, or with diag its diagonal halves; cpfx: prefix of their column
// counts, total = cpfx[nd]); wide: a block per column, else a wave per column;
// at most max_blocks workgroups, looping over the columns.
void launch_fill_zero(const FillDesc* fd, const int32_t* cpfx, int nd, int total, bool wide, bool diag,
                      int max_blocks, hipStream_t s);
// Workgroup size and caps of the fill (a block per column / a wave per
// column): they set how many compute units it holds beside the levels it runs
// with.
constexpr int kFillThreads = 256;
// The diagonal halves of a wide Q are filled from this many levels before the
// root on.
constexpr int kFillLateLevels = 4;
constexpr int kFillBlocksWide = 128;
constexpr int kFillBlocksNarrow = 512;
void launch_secular_standalone(int64_t K, const double* d, const double* z, double rho, int32_t* org,
                               double* tau, int32_t* status, hipStream_t s);

// phdc_stedc; no_alloc: the plan is uploaded from pageable host memory (no
// pinned staging buffer), the call waits for it, and the HSS path is refused.
int stedc_impl(int64_t n, const double* d, const double* e, double* lambda, double* Q, int64_t ldq, void* work,
               size_t lwork, const phdc_opts* o, hipStream_t s, bool no_alloc);
// Workspace bytes of an n-row solve (o valid); fill: with the zero fill's third
// eigenvector buffer (phdc_stedc), else without (no_alloc).
size_t stedc_workspace_bytes(int64_t n, const phdc_opts* o, bool fill);

// FP64 product for one merge whose HSS compression gave up (Sec. 2.2: Gu's
// grouped products whenever HSS does not apply).  desc is the merge's device
// descriptor, M its host copy.  The merge is marked as FP64 (path 0, HSS rank
// -1), Uhat is rewritten in the grouped row order and the update GEMM runs for
// this merge alone; the rest of the merge (ranks, deflated columns) is done.
void launch_fp64_fallback(const MergeDesc* desc, const MergeDesc& M, const Scratch& S, hipStream_t s);

}  // namespace phdc
