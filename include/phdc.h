/*
 * phdc.h -- C-ABI of the MI355X (gfx950) tridiagonal divide-and-conquer
 * eigensolver library (libphdc.so).
 *
 * The problem (Sec. 1, Eq. (1)): given the symmetric tridiagonal T with
 * diagonal d[0:n] and off-diagonal e[0:n-1], compute T = Q diag(lambda) Q^T
 * with lambda ascending and Q orthogonal.  The method is Cuppen's divide and
 * conquer (Eq. (2)-(6)): split, solve the halves, and merge through the
 * rank-one update D + rho z z^T, whose eigenvector matrix Uhat is assembled
 * from secular-equation roots and the Loewner-recomputed z (Remark 1), then
 * applied as diag(Q1, Q2) * Uhat (Eq. (6)) -- as a plain FP64 product, as a
 * split-precision product, or through an HSS compression of Uhat (Sec. 2.2,
 * Algorithm 1).
 *
 * Conventions for every entry point:
 *  - Pointers named d, e, D, z, Q*, lambda*, *_bar and work are DEVICE
 *    pointers (hipMalloc / torch CUDA tensors); arrays named *_host are host
 *    pointers.  All matrices are column-major with the stated leading
 *    dimension.  The caller owns every buffer; the library never allocates or
 *    frees device memory.
 *  - `stream` is a hipStream_t (may be NULL for the default stream).  Work is
 *    only enqueued; nothing waits for the GPU except phdc_status().
 *  - Return value: 0 on success, -i if argument i (1-based) is invalid.  The
 *    argument checks are done on the host before anything is enqueued.
 *    Failures that can only be seen on the device (a leaf QL or secular
 *    iteration that does not converge, unsorted merge input, non-finite
 *    input) are reported through phdc_status().
 *  - Every call needs a workspace of at least the size returned by the
 *    matching *_workspace query; the same workspace must not be used by two
 *    calls that may run at the same time.
 */
#ifndef PHDC_H
#define PHDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* How the merge's eigenvector update diag(Q1,Q2) * Uhat (Eq. (6)) is formed. */
enum phdc_gemm_mode {
    PHDC_GEMM_FP64 = 0,  /* FP64 MFMA product with Gu's column grouping (Sec. 1) */
    PHDC_GEMM_SPLIT = 1, /* split-precision: BF16 slices on MFMA, FP32 accumulation, FP64 recombination */
    PHDC_GEMM_HSS = 2    /* HSS-compressed Uhat (Sec. 2.2, Algorithm 1) when K >= hss_min_K, else FP64 */
};

/* Device-side status codes returned by phdc_status(). */
enum phdc_info {
    PHDC_OK = 0,
    PHDC_ERR_LEAF = 1,     /* a leaf QL iteration did not converge */
    PHDC_ERR_SECULAR = 2,  /* a secular root did not converge */
    PHDC_ERR_UNSORTED = 3, /* merge(): D1 or D2 not ascending */
    PHDC_ERR_NONFINITE = 4 /* non-finite input */
};

typedef struct phdc_opts {
    int32_t leaf_size;      /* largest block solved directly (default 32, range 2..64) */
    int32_t gemm_mode;      /* enum phdc_gemm_mode (default PHDC_GEMM_FP64) */
    int64_t hss_min_K;      /* HSS only for merges with at least this many surviving poles (default 4096) */
    double hss_rel_tol;     /* ID truncation tolerance for HSS compression (default 1e-14): a node's
                               rank ends at |R_kk| <= tol * max(|R_00|, sqrt(d)), d samples */
    int32_t hss_leaf;       /* HSS leaf block size, 8..1024 (default 256) */
    int32_t hss_samples;    /* initial number of random sample columns d, 16..512 (default 256) */
    int32_t hss_samples_inc;/* extra sample columns when a rank reaches d - 8, >= 0 (default 128) */
    int32_t split_slices;   /* number of BF16 slices per operand for PHDC_GEMM_SPLIT, 1..7 (default 7) */
    uint64_t seed;          /* seed of the counter-based Gaussian generator used by HSS sampling */
    int32_t canonical_sign; /* if nonzero: each eigenvector's largest-magnitude entry is made positive */
    int32_t check_finite;   /* if nonzero: scan the inputs for NaN/Inf on the device */
} phdc_opts;

/* Fill *o with the defaults listed above. */
void phdc_opts_default(phdc_opts *o);

/* Library version; also a cheap call to check that the library loads. */
int phdc_version(void);

/* ---------------------------------------------------------------- stedc
 * All eigenpairs of the tridiagonal (d, e) of Eq. (1) by divide and conquer.
 *   n       order (n >= 0)
 *   d       device, n doubles, diagonal (read only)
 *   e       device, n-1 doubles, off-diagonal (read only; may be NULL if n <= 1)
 *   lambda  device, n doubles, output eigenvalues ascending
 *   Q       device, ldq*n doubles, output eigenvectors (column j for lambda[j])
 *   ldq     leading dimension of Q, ldq >= max(1, n)
 *   work    device workspace of lwork bytes (phdc_stedc_workspace), 256-byte aligned
 * Returns 0 or -(argument index). */
int phdc_stedc_workspace(int64_t n, const phdc_opts *o, size_t *bytes);
int phdc_stedc(int64_t n, const double *d, const double *e, double *lambda, double *Q, int64_t ldq,
               void *work, size_t lwork, const phdc_opts *o, void *stream);

/* ---------------------------------------------------------------- merge
 * One rank-one merge (Eq. (3)-(6)): the eigen-decomposition of
 *     diag(Q1, Q2) (D + rho z z^T) diag(Q1, Q2)^T,   D = diag(D[0:n1], D[n1:n1+n2]).
 *   D      device, n1+n2 doubles; D[0:n1] and D[n1:] must each be ascending
 *   z      device, n1+n2 doubles, any values (normalised internally)
 *   rho    rho >= 0 (rho == 0 or z == 0: every pole deflates)
 *   Q1     device, ldq1*n1 (n1 x n1), Q2 device, ldq2*n2 (n2 x n2); any matrices
 *   lambda device, n1+n2 doubles, output ascending
 *   Q      device, ldq*(n1+n2), output eigenvectors; must not overlap Q1/Q2
 * stats_host (may be NULL): after phdc_status(), phdc_merge_stats() returns
 * {K, k1, k2, k3, type-1 deflations, type-2 deflations, path, hss_rank}. */
int phdc_merge_workspace(int64_t n1, int64_t n2, const phdc_opts *o, size_t *bytes);
int phdc_merge(int64_t n1, int64_t n2, const double *D, const double *z, double rho, const double *Q1,
               int64_t ldq1, const double *Q2, int64_t ldq2, double *lambda, double *Q, int64_t ldq,
               void *work, size_t lwork, const phdc_opts *o, void *stream);

/* ---------------------------------------------------------------- batched stedc
 * B independent tridiagonals of orders n_host[b] (each >= 0), solved together:
 * all leaves in one launch, then every merge of equal height across the batch
 * in one launch per kernel.  Packed layout: matrix b's diagonal starts at
 * d[off_host[b]], its off-diagonal follows those of matrices 0..b-1 in e
 * (max(n_b - 1, 0) entries each), its eigenvalues at
 * lambda[off_host[b]], and its n_b x n_b eigenvector block at
 * Q[qoff_host[b]] with leading dimension n_b.  off_host must be the exclusive
 * prefix sum of n_host and qoff_host that of n_host[b]^2. */
int phdc_stedc_batched_workspace(int64_t B, const int64_t *n_host, const phdc_opts *o, size_t *bytes);
int phdc_stedc_batched(int64_t B, const int64_t *n_host, const int64_t *off_host, const int64_t *qoff_host,
                       const double *d, const double *e, double *lambda, double *Q, void *work,
                       size_t lwork, const phdc_opts *o, void *stream);

/* Two-step form of the batched solve for callers that replay it in a HIP
 * graph: phdc_stedc_batched_prepare builds the plan (split trees, level
 * schedule, block maps) and copies it into `work` synchronously (same
 * arguments as phdc_stedc_batched; PHDC_GEMM_HSS is rejected with -11 because
 * that path reads sizes back on the host).  phdc_launch_prepared then only
 * enqueues kernels (no memcpy, memset or host synchronisation), so it may be
 * captured on `stream` and the graph replayed; every replay recomputes the
 * solve from the current contents of d and e.  The prepared plan belongs to
 * `work` until the next prepare or solve call on it. */
int phdc_stedc_batched_prepare(int64_t B, const int64_t *n_host, const int64_t *off_host, const int64_t *qoff_host,
                               const double *d, const double *e, double *lambda, double *Q, void *work,
                               size_t lwork, const phdc_opts *o, void *stream);
int phdc_launch_prepared(void *work, void *stream);

/* ---------------------------------------------------------------- adjoint
 * Gradients of a loss L(lambda, Q) with respect to d and e, given lbar =
 * dL/dlambda and Qbar = dL/dQ at the eigenpairs (lambda, Q) of T:
 *   Tbar = Q (diag(lbar) + F o (Q^T Qbar)) Q^T, F_ij = 1/(lambda_j - lambda_i) (i != j), 0 (i == j);
 *   d_bar[i] = Tbar_ii, e_bar[i] = Tbar_{i,i+1} + Tbar_{i+1,i}.
 * Eigenvalues must be simple.  Q_bar may be NULL (eigenvalue-only loss).
 * Batched form: `batch` problems of equal order n, packed with strides n
 * (lambda, lbar, d_bar), n-1 (e_bar) and n*n (Q, Qbar; ld = n). */
int phdc_stedc_backward_workspace(int64_t n, int64_t batch, size_t *bytes);
int phdc_stedc_backward(int64_t n, int64_t batch, const double *lambda, const double *Q,
                        const double *lambda_bar, const double *Q_bar, double *d_bar, double *e_bar,
                        void *work, size_t lwork, void *stream);

/* ---------------------------------------------------------------- status
 * Waits for `stream`, then returns the device status word (enum phdc_info)
 * written by the last call that used `work`. */
int phdc_status(const void *work, void *stream);

/* After phdc_status(): statistics of the top-level merge of the last
 * stedc/merge call on `work` (8 int32, see phdc_merge). Returns 0 or -1. */
int phdc_merge_stats(const void *work, int32_t *stats_host);

/* ---------------------------------------------------------------- measurement
 * Opt-in timing: while enabled, every kernel class of a solve is bracketed by
 * HIP events on the launch stream (small overhead).  phdc_profile_read waits
 * for the recorded events, returns per-phase milliseconds and launch counts in
 * ms[0:nphase], count[0:nphase] (phase order: leaf, deflate, rotate, secular,
 * loewner, uhat-norm, uhat-write, rank, gemm, copy, sign, split-slice,
 * split-gemm, hss-sample, hss-compress, hss-apply, adjoint-gemm, adjoint-band)
 * and forgets them.  Returns 0. */
int phdc_profile_enable(int on);
int phdc_profile_read(double *ms, int64_t *count, int nphase);
/* Restrict the recorded phases to the set bits of mask (bit i = phase i in the
 * order above; default: all).  Fewer events perturb the timed work less.
 * Returns 0. */
int phdc_profile_select(uint32_t mask);

/* Sizes of every merge of the last stedc/merge call on `work` (call after
 * phdc_status): up to max_rows rows of PHDC_MERGE_TABLE_COLS int32 each:
 * {m, n1, K, k1, k2, k3, type-1 deflations, type-2 deflations,
 *  path (0 FP64, 1 split, 2 HSS), HSS rank,
 *  deflated columns nonzero in the Q1 rows only, in both halves, in the Q2 rows only,
 *  rows the deflated columns can be nonzero in, summed: low 32 bits (as unsigned), high bits,
 *  1 for the last merge of its matrix (which writes every row of its output) else 0}.
 * Rows are in the order the merges were planned (leaves upward, the root last).
 * *rows_out receives the number of merges.  Returns 0 or -1. */
#define PHDC_MERGE_TABLE_COLS 16
int phdc_merge_table(const void *work, int64_t max_rows, int32_t *table_host, int64_t *rows_out);

/* ---------------------------------------------------------------- secular roots
 * The K roots of f(lambda) = 1 + rho sum_i z_i^2/(d_i - lambda) (Sec. 1, after
 * Eq. (4)) for strictly ascending d, rho > 0 and nonzero z, one root per GPU
 * thread.  Root j is returned as origin pole org[j] (int32) and offset tau[j]
 * with lambda_j = d[org[j]] + tau[j].  All pointers are device pointers.
 * Non-convergence is reported through phdc_status(work). */
int phdc_secular(int64_t K, const double *d, const double *z, double rho, int32_t *org, double *tau,
                 void *work, size_t lwork, void *stream);

/* ---------------------------------------------------------------- GEMM tile autotuner
 * The FP64 update GEMM (Eq. (6)) of every tree level uses square output tiles
 * of edge 64 or 128, looked up per merge-size bucket (2^(b-1) < m <= 2^b) in a
 * process-wide table when a solve is planned.  phdc_autotune_gemm times both
 * edges with HIP events on a synthetic merge of each size m = 64, 128, ...,
 * max_m (no deflation, K = m) and records the faster one; untimed buckets use
 * 64 up to m = 256 and 128 above.  The tile changes the speed only: both edges
 * accumulate in the same k order, so results are bitwise identical.
 *   max_m   largest merge size to time, 2 <= max_m <= 2^20
 *   work    device scratch of at least phdc_autotune_gemm_workspace(max_m) bytes
 *           (three max_m x max_m FP64 arrays and index arrays), 256-byte aligned
 * Synchronises the stream; not for use under graph capture.  Returns 0 or a
 * negative code (-1 bad size, -2 null work, -3 lwork too small, < -3 HIP error).
 * phdc_gemm_tile_table copies the table (0 = not timed) into tiles[0:n) and
 * returns the number of buckets written. */
int phdc_autotune_gemm_workspace(int64_t max_m, size_t *bytes);
int phdc_autotune_gemm(int64_t max_m, void *work, size_t lwork, void *stream);
int phdc_gemm_tile_table(int32_t *tiles, int n);

#ifdef __cplusplus
}
#endif
#endif /* PHDC_H */
