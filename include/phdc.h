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
 *  - Return value: 0 on success; -i (1 <= i <= 99) if argument i (1-based) is
 *    invalid, found by host-side checks before anything is enqueued (with
 *    opts.check_finite set, also a NaN or Inf in an input array, found by a
 *    device scan the call waits for); PHDC_E_HIP (-100) if a HIP runtime call
 *    made by the library failed (launch, copy, synchronisation, event or
 *    pinned host allocation).  No other value is returned.
 *    Failures that can only be seen on the device (a leaf QL or secular
 *    iteration that does not converge, unsorted merge input, non-finite
 *    input) are reported through phdc_status() (enum phdc_info); the solve
 *    still runs to completion and every access stays inside the caller's
 *    buffers, but its results are then meaningless.
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

/* Device-side status codes returned by phdc_status().  The first failure of a
 * call is kept. */
enum phdc_info {
    PHDC_OK = 0,
    PHDC_ERR_LEAF = 1,     /* a leaf QL iteration did not converge (or opts.force_fail bit 0) */
    PHDC_ERR_SECULAR = 2,  /* a secular root did not converge, or the secular function was NaN
                              (or opts.force_fail bit 1) */
    PHDC_ERR_UNSORTED = 3, /* merge(): D1 or D2 not ascending */
    PHDC_ERR_NONFINITE = 4 /* a NaN or Inf among the merge's poles, z or coupling, or found by the
                              check_finite scan */
};

/* Host-side return code: a HIP runtime call made by the library failed. */
#define PHDC_E_HIP (-100)

/* Bits of phdc_opts.force_fail: test hooks that make a bounded device loop give
 * up at once, so that the failure path runs without any fault or hang. */
enum phdc_force_fail {
    PHDC_FAIL_LEAF = 1,    /* leaf QL gets no iterations: PHDC_ERR_LEAF for any leaf that needs one */
    PHDC_FAIL_SECULAR = 2, /* secular roots get no iterations: PHDC_ERR_SECULAR when a merge keeps K >= 2 */
    PHDC_FAIL_HSS = 4      /* every HSS compression reports rank overflow, so each HSS merge takes
                              the FP64 fall-back product (HSS rank -1 in the merge table) */
};

typedef struct phdc_opts {
    int32_t leaf_size;      /* largest block solved directly (default 16, range 2..64) */
    int32_t gemm_mode;      /* enum phdc_gemm_mode (default PHDC_GEMM_FP64) */
    int64_t hss_min_K;      /* HSS only for merges with at least this many surviving poles (default 4096) */
    double hss_rel_tol;     /* ID truncation tolerance for HSS compression (default 1e-14): a node's
                               rank ends at |R_kk| <= tol * max(|R_00|, sqrt(d)), d samples */
    int32_t hss_leaf;       /* HSS leaf block size, 8..1024 (default 256) */
    int32_t hss_samples;    /* initial number of random sample columns d, 16..512 (default 192) */
    int32_t hss_samples_inc;/* extra sample columns when a rank reaches d - 8, >= 0 (default 128) */
    int32_t split_slices;   /* number of BF16 slices per operand for PHDC_GEMM_SPLIT, 1..7 (default 6: the
                               fewest that meet 10x the FP64 bounds) */
    uint64_t seed;          /* seed of the counter-based Gaussian generator used by HSS sampling */
    int32_t canonical_sign; /* if nonzero: each eigenvector's largest-magnitude entry is made positive */
    int32_t check_finite;   /* if nonzero: scan the input arrays for NaN/Inf on the device first; the
                               call waits for the scan and, on a hit, sets PHDC_ERR_NONFINITE, enqueues
                               nothing else and returns -(index of the first such array argument).
                               phdc_launch_prepared (graph capture: no waiting) only sets the status. */
    int32_t force_fail;     /* test hook, bits of enum phdc_force_fail (default 0) */
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
 *           (about 2.5 n^2 doubles for large n: a second eigenvector buffer of
 *           n^2, a third of about n^2/2 for the even depths below a root that
 *           is zero-filled ahead of time (n >= 256), Uhat of the largest
 *           level, about n^2, and O(n) scratch)
 * Returns 0, -(argument index) or PHDC_E_HIP. */
int phdc_stedc_workspace(int64_t n, const phdc_opts *o, size_t *bytes);
int phdc_stedc(int64_t n, const double *d, const double *e, double *lambda, double *Q, int64_t ldq,
               void *work, size_t lwork, const phdc_opts *o, void *stream);

/* ---------------------------------------------------------------- stedc without allocation
 * For callers that cannot allocate memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same solve as phdc_stedc,
 * with the workspace taken from a static device array of
 * PHDC_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends (enough for n up to about 2450 in the FP64 form
 * and 1500 in the split-precision form).  The call makes no hipMalloc,
 * hipHostMalloc or hipFree and no other allocating library call; it uploads the
 * solve's plan from pageable host memory and waits for that upload, then
 * enqueues the kernels.  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents (each call starts by clearing what must start
 * at zero): calls that overlap on one GPU (two streams, two threads) race,
 * calls in sequence on one stream are safe.
 *   n, d, e, lambda, Q, ldq, o, stream: as for phdc_stedc
 *   info   device, 1 int32: receives the call's status word (enum phdc_info)
 * Returns 0; -1 if n < 0 or the solve needs more than PHDC_NOALLOC_SCRATCH_BYTES
 * of workspace; -(argument index) for other invalid arguments, -8 also for
 * PHDC_GEMM_HSS (whose host read-back uses pinned memory) or invalid options;
 * PHDC_E_HIP. */
#define PHDC_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
int phdc_stedc_noalloc(int64_t n, const double *d, const double *e, double *lambda, double *Q, int64_t ldq,
                       int32_t *info, const phdc_opts *o, void *stream);

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
/* Returns 0, -1 if `work` holds no prepared plan (never prepared, or another
 * solve, merge or phdc_release on `work` came after the prepare), or PHDC_E_HIP. */
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
 * written by the last call that used `work`, or PHDC_E_HIP. */
int phdc_status(const void *work, void *stream);

/* Forget the host-side state the library keeps for `work` (the prepared plan
 * of phdc_stedc_batched_prepare, and the pinned staging buffers and events of
 * the plan upload and of the HSS path), freeing its pinned memory and events.
 * Call it before freeing a workspace; a later call on the same address starts
 * afresh.  Waits for uploads still in flight.  Returns 0, or -1 if work is NULL. */
int phdc_release(void *work);

/* After phdc_status(): statistics of the top-level merge of the last
 * stedc/merge call on `work` (8 int32, see phdc_merge). Returns 0 or -1. */
int phdc_merge_stats(const void *work, int32_t *stats_host);

/* ---------------------------------------------------------------- measurement
 * Opt-in timing: while enabled, every launch of a solve is bracketed by HIP
 * events on the launch stream (small overhead).  phdc_profile_read waits for
 * the recorded events, returns per-phase milliseconds and launch counts in
 * ms[0:nphase], count[0:nphase] (phase order: leaf, deflate, rotate, secular,
 * loewner, uhat-norm, uhat-write, rank, gemm, copy, sign, split-slice,
 * split-gemm, hss-sample, hss-compress, hss-apply, adjoint-gemm, adjoint-band,
 * small-merge, fill) and forgets them.  A merge level runs some steps in one launch,
 * timed under one phase: "small-merge" = every step of the merges of at most 64
 * rows on the FP64 path (one workgroup each); "secular" = rotations + secular
 * roots (levels whose merges have at most 64 rows on the other paths: also
 * Loewner z, column norms, Uhat and output ranks); "loewner" = Loewner z +
 * output ranks; "uhat-write" = column norms + Uhat + the deflated-column copy
 * ("uhat-norm" when the norms run first, for normalized Uhat); "copy" = the
 * deflated-column copy of a lone root merge (the caller's whole Q); "fill" =
 * the zero fill of the caller's Q for a root merge of at least 256 rows in the
 * last level, on a second stream while the levels below run (from 2048 rows
 * in two parts: the off-diagonal quadrants from the first levels, the diagonal
 * halves from four levels before the root; its events are recorded on that
 * stream); "rotate" and "rank" are no longer recorded separately.
 * Returns 0. */
int phdc_profile_enable(int on);
int phdc_profile_read(double *ms, int64_t *count, int nphase);
/* Restrict the recorded phases to the set bits of mask (bit i = phase i in the
 * order above; default: all).  Fewer events perturb the timed work less.
 * Returns 0. */
int phdc_profile_select(uint32_t mask);

/* Sizes of every merge of the last stedc/merge call on `work` (call after
 * phdc_status): up to max_rows rows of PHDC_MERGE_TABLE_COLS int32 each:
 * {m, n1, K, k1, k2, k3, type-1 deflations, type-2 deflations,
 *  path (0 FP64, 1 split, 2 HSS), HSS rank (largest interpolative-decomposition
 *  rank; -1 when the HSS compression gave up -- ranks beyond the largest
 *  sample count, or opts.force_fail -- and the merge took the FP64 product),
 *  deflated columns nonzero in the Q1 rows only, in both halves, in the Q2 rows only,
 *  rows the deflated columns can be nonzero in, summed: low 32 bits (as unsigned), high bits,
 *  1 for the last merge of its matrix (which writes every row of its output) else 0,
 *  1 for a last merge whose output was zero-filled on a second stream while the
 *  tree below ran (its deflated-column copy then writes the rows of each
 *  column's range only), else 0,
 *  for such a merge: the rows its deflated-column copy writes, summed: low 32
 *  bits (as unsigned), high bits; else 0, 0}.
 * Rows are in the order the merges were planned (leaves upward, the root last).
 * *rows_out receives the number of merges.  Returns 0 or -1. */
#define PHDC_MERGE_TABLE_COLS 19
int phdc_merge_table(const void *work, int64_t max_rows, int32_t *table_host, int64_t *rows_out);

/* ---------------------------------------------------------------- HSS product of a dense matrix
 * The compression of the merge update (Sec. 2.2, Algorithm 1) applied to a
 * general dense K x K matrix, as in the paper's Example 1 (Table 1): A is
 * compressed into HSS form by randomized sampling and interpolative
 * decompositions (tolerance opts.hss_rel_tol relative to each node's largest
 * pivot, with an absolute floor of hss_rel_tol sqrt(d) ||A||_F / sqrt(K);
 * leaves of opts.hss_leaf rows; opts.hss_samples samples, growing by
 * opts.hss_samples_inc), then C = X A is formed in that form.
 *   K      order of A, 1 <= K <= 2^30
 *   A      device, K x K column-major, lda >= K, read only
 *   m      rows of X and C, 1 <= m <= 2^30
 *   X      device, m x K column-major, ldx >= m, read only
 *   C      device, m x K column-major output, ldc >= m; must not overlap A or X
 *   rank_host  host, may be NULL: the largest ID rank, or -1 when the compression
 *          gave up (ranks beyond the largest sample count, or opts.force_fail
 *          PHDC_FAIL_HSS) and C was formed by the dense FP64 MFMA product instead
 *   work   device workspace of phdc_hss_gemm_workspace(K, m) bytes, 256-byte aligned
 * Waits for the stream (the ID ranks of each tree level are read on the host).
 * Returns 0, -(argument index) or PHDC_E_HIP.  Timing phases: hss-sample,
 * hss-compress, hss-apply (also the dense product when the compression gave up). */
int phdc_hss_gemm_workspace(int64_t K, int64_t m, const phdc_opts *o, size_t *bytes);
int phdc_hss_gemm(int64_t K, const double *A, int64_t lda, int64_t m, const double *X, int64_t ldx, double *C,
                  int64_t ldc, int32_t *rank_host, void *work, size_t lwork, const phdc_opts *o, void *stream);

/* ---------------------------------------------------------------- secular roots
 * The K roots of f(lambda) = 1 + rho sum_i z_i^2/(d_i - lambda) (Sec. 1, after
 * Eq. (4)) for strictly ascending d, rho > 0 and nonzero z, one root per GPU
 * thread.  Root j is returned as origin pole org[j] (int32) and offset tau[j]
 * with lambda_j = d[org[j]] + tau[j].  All pointers are device pointers.
 * Non-convergence is reported through phdc_status(work); the int32 after the
 * status word in work receives the largest number of evaluations of the
 * secular function spent on one root. */
int phdc_secular(int64_t K, const double *d, const double *z, double rho, int32_t *org, double *tau,
                 void *work, size_t lwork, void *stream);

/* ---------------------------------------------------------------- GEMM tile autotuner
 * The FP64 update GEMM (Eq. (6)) of every tree level uses square output tiles
 * whose rule is looked up per merge-size bucket (2^(b-1) < m <= 2^b) in a
 * process-wide table when a solve is planned: 32 or 64 (every merge of the
 * level in tiles of that edge) or 128 (128-wide tiles for merges with at least
 * 512 of them, 64 for the others).  phdc_autotune_gemm times the three rules
 * with HIP events on a synthetic merge of each size m = 64, 128, ..., max_m (no
 * deflation, K = m) and records the fastest; untimed buckets use 64 up to
 * m = 256 and 128 above.  The tile changes the speed only: every edge
 * accumulates in the same k order, so results are bitwise identical.
 *   max_m   largest merge size to time, 2 <= max_m <= 2^20
 *   work    device scratch of at least phdc_autotune_gemm_workspace(max_m) bytes
 *           (three max_m x max_m FP64 arrays and index arrays), 256-byte aligned
 * Synchronises the stream; not for use under graph capture.  Returns 0 or a
 * negative code (-1 bad size, -2 null work, -3 lwork too small, PHDC_E_HIP).
 * phdc_gemm_tile_table copies the table (0 = not timed) into tiles[0:n) and
 * returns the number of buckets written. */
int phdc_autotune_gemm_workspace(int64_t max_m, size_t *bytes);
int phdc_autotune_gemm(int64_t max_m, void *work, size_t lwork, void *stream);
int phdc_gemm_tile_table(int32_t *tiles, int n);

#ifdef __cplusplus
}
#endif
#endif /* PHDC_H */
