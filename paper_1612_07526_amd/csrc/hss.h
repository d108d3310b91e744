// Descriptors of the HSS kernels (hss.hip).  All sizes are host-known: the
// host reads the ID ranks after each tree level before building the next one.
#pragma once
#include <vector>

#include "phdc_internal.h"

namespace phdc {

// out(a, b) = Uhat(row_a, col_b); row_a = ri ? ri[a] : r0 + a (same for columns).
struct UGather {
  const int32_t* ri;
  const int32_t* cj;
  double* out;
  int64_t ld;
  int32_t r0, c0, nr, nc;
};

// dst(row0 + a, b) = src(idx ? idx[a] : a, b) for a < nr, b < ncol (column-major).
struct RowCopy {
  const double* src;
  const int32_t* idx;
  double* dst;
  int64_t lds, ldd;
  int32_t nr, ncol, dst_row0, pad;
};

// dst[dst0 + a] = src[a] for a < n.
struct IntCopy {
  const int32_t* src;
  int32_t* dst;
  int32_t n, dst0;
};

// out[a] = base ? base[perm[a]] : lo + perm[a] for a < rank.
struct SkelDesc {
  const int32_t* perm;
  const int32_t* base;
  int32_t* out;
  int32_t rank, lo;
};

// Row ID of phi (p x d, ld ldphi): outputs rank, perm (p), U (p x rank, ld p).
struct IdDesc {
  const double* phi;
  double* work;  // p x d scratch (ld p)
  double* U;
  int32_t* perm;
  int32_t* rank;
  int64_t ldphi;
  int32_t p, d;
};

// Arena of one compression of a K x K matrix applied to m rows (with_x: plus
// the m x K gathered operand of a merge).
size_t hss_arena_bytes(int64_t m, int64_t K, int leaf, int dmax, bool with_x);

// Where the entries of the matrix A being compressed come from: the Cauchy form
// of a merge's Uhat (A == nullptr: A(i, j) = zh_i / ((ds_i - dorg_j) - tau_j) cn_j)
// or a dense column-major matrix; `sample` is a dense copy of A for the
// sampling products (row-major: it holds A^T column-major, ld lds).
struct HssSource {
  const double *ds, *zh, *dorg, *tau, *cn;
  const double* A;
  int64_t lda;
  const double* sample;
  int64_t lds;
  bool sample_row_major;
};
int hss_core(const HssSource& src, int K, int m, const double* X, int64_t ldx, double* out, int64_t ldo,
             const int32_t* cmap, char* arena, size_t arena_bytes, char* descarea, size_t desc_bytes,
             const phdc_opts* o, double anorm, int32_t* rank_dev, const void* work, hipStream_t s);
// One HSS merge, with K known on the host.  Returns 0, kHssGaveUp when the
// compression cannot be completed (the caller then forms the FP64 product; no
// part of the merge's output has been written), or PHDC_E_HIP.
constexpr int kHssGaveUp = 1;
int run_hss_merge(const MergeDesc& M, int K, const Scratch& S, char* arena, size_t arena_bytes, char* descarea,
                  size_t desc_bytes, const phdc_opts* o, int32_t* counters_dev, const void* work, hipStream_t s);
// Upload of HSS descriptors through the workspace's own pinned staging buffer.
int hss_upload(const void* work, void* dst, const std::vector<char>& bytes, hipStream_t s);

}  // namespace phdc
