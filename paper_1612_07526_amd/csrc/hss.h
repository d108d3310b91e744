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

size_t hss_arena_bytes(int64_t m, int64_t K, int leaf, int dmax);
int run_hss_merge(const MergeDesc& M, int K, const Scratch& S, char* arena, size_t arena_bytes, char* descarea,
                  size_t desc_bytes, const phdc_opts* o, int32_t* counters_dev, hipStream_t s);
int hss_upload(const void* key, void* dst, const std::vector<char>& bytes, hipStream_t s);

}  // namespace phdc
