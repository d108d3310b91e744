/*
 * oracle.c -- plain, slow, FP64 reference implementation of the symmetric
 * tridiagonal divide-and-conquer (DC) eigensolver described in
 *   S. Li, F.-H. Rouet, J. Liu, C. Huang, X. Gao, X. Chi, "An efficient hybrid
 *   tridiagonal divide-and-conquer algorithm on distributed memory
 *   architectures" (arXiv 1612.07526).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the yardstick the HIP library is
 * measured against; it is compiled on its own with gcc, shares no code, header
 * or constant with the HIP library, and is loaded only by the tests, by the
 * smoke check and by the benchmark's CPU-baseline leg.
 *
 * Every routine favours being checkable by eye over speed: no blocking, no
 * fusion, no reordering beyond what the definition states.  OpenMP is used only
 * across fully independent items (independent roots, independent columns).
 *
 * Conventions: all matrices are column-major, element (i,j) of a matrix with
 * leading dimension ld is at [i + j*ld]; indices are 0-based.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Unit roundoff of IEEE binary64 (2^-53), the "eps" of the deflation test. */
static const double OR_U = 1.1102230246251565e-16;

#define A_(M, ld, i, j) ((M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

int or_version(void) { return 3; }

/* ------------------------------------------------------------------------- */
/* Dense symmetric eigensolver used for the DC leaves: cyclic Jacobi.         */
/* The paper leaves the leaf solver unspecified; any exact eigensolver is a   */
/* correct leaf.  Jacobi is used here because it is short and obviously       */
/* correct, and because the HIP library uses a different method (QL).         */
/* ------------------------------------------------------------------------- */

/* Eigen-decomposition A = V diag(w) V^T of a symmetric n x n matrix.  A is
 * overwritten.  w is returned ascending, V's columns match w.  Returns the
 * number of sweeps used, or -1 if 100 sweeps did not converge. */
int or_jacobi(int n, double *A, int lda, double *w, double *V, int ldv)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) A_(V, ldv, i, j) = (i == j) ? 1.0 : 0.0;
    int sweep, converged = 0;
    for (sweep = 0; sweep < 100 && !converged; ++sweep) {
        converged = 1;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = A_(A, lda, p, q);
                double app = A_(A, lda, p, p), aqq = A_(A, lda, q, q);
                /* Skip entries that are negligible relative to their diagonal. */
                if (fabs(apq) <= OR_U * sqrt(fabs(app) * fabs(aqq)) || apq == 0.0) {
                    A_(A, lda, p, q) = 0.0;
                    A_(A, lda, q, p) = 0.0;
                    continue;
                }
                converged = 0;
                /* Symmetric Schur rotation that annihilates A(p,q). */
                double theta = (aqq - app) / (2.0 * apq);
                double t;
                if (fabs(theta) > 1e150)
                    t = 0.5 / theta;
                else
                    t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* A <- J^T A J with J = rotation in the (p,q) plane. */
                for (int k = 0; k < n; ++k) {
                    double akp = A_(A, lda, k, p), akq = A_(A, lda, k, q);
                    A_(A, lda, k, p) = c * akp - s * akq;
                    A_(A, lda, k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A_(A, lda, p, k), aqk = A_(A, lda, q, k);
                    A_(A, lda, p, k) = c * apk - s * aqk;
                    A_(A, lda, q, k) = s * apk + c * aqk;
                }
                A_(A, lda, p, q) = 0.0;
                A_(A, lda, q, p) = 0.0;
                for (int k = 0; k < n; ++k) {
                    double vkp = A_(V, ldv, k, p), vkq = A_(V, ldv, k, q);
                    A_(V, ldv, k, p) = c * vkp - s * vkq;
                    A_(V, ldv, k, q) = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = A_(A, lda, i, i);
    /* Selection sort into ascending order (stable for equal values). */
    for (int i = 0; i < n; ++i) {
        int best = i;
        for (int j = i + 1; j < n; ++j)
            if (w[j] < w[best]) best = j;
        if (best != i) {
            double tw = w[i];
            w[i] = w[best];
            w[best] = tw;
            for (int k = 0; k < n; ++k) {
                double tv = A_(V, ldv, k, i);
                A_(V, ldv, k, i) = A_(V, ldv, k, best);
                A_(V, ldv, k, best) = tv;
            }
        }
    }
    return converged ? sweep : -1;
}

/* ------------------------------------------------------------------------- */
/* Secular equation (Sec. 1, after Eq. (4)):                                  */
/*   f(lambda) = 1 + rho * sum_i z_i^2 / (d_i - lambda),                       */
/* with the sum over all i (the printed formula omits the summation sign).    */
/* ------------------------------------------------------------------------- */

/* f evaluated at lambda = d[o] + tau, using the differences (d_i - d[o]) - tau
 * so that the distance to the nearest pole keeps full relative accuracy. */
static double secular_f(int K, const double *d, const double *z, double rho, int o, double tau)
{
    double s = 0.0;
    for (int i = 0; i < K; ++i) s += z[i] * z[i] / ((d[i] - d[o]) - tau);
    return 1.0 + rho * s;
}

/* All K roots of the secular equation for strictly ascending d, rho > 0 and
 * nonzero z.  Root j lies in (d_j, d_{j+1}) (and in (d_{K-1}, d_{K-1} +
 * rho*|z|^2) for the last one).  It is returned as an origin pole o[j] and an
 * offset tau[j], lambda_j = d[o[j]] + tau[j].  The origin is the nearer end of
 * the bracket, decided by the sign of f at the bracket midpoint; tau is then
 * found by plain bisection, run until the bracket cannot shrink further in
 * binary64.  Returns the largest number of bisection steps used. */
int or_secular(int K, const double *d, const double *z, double rho, int *o, double *tau)
{
    double zz = 0.0;
    for (int i = 0; i < K; ++i) zz += z[i] * z[i];
    int maxit = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : maxit)
    for (int j = 0; j < K; ++j) {
        int org;
        double lo, hi;
        if (j < K - 1) {
            double half = 0.5 * (d[j + 1] - d[j]);
            double fmid = secular_f(K, d, z, rho, j, half);
            if (fmid >= 0.0) {
                org = j;
                lo = 0.0;
                hi = half;
            } else {
                org = j + 1;
                lo = (d[j] - d[j + 1]) + half; /* the midpoint, seen from d_{j+1} */
                hi = 0.0;
            }
        } else {
            org = K - 1;
            lo = 0.0;
            hi = rho * zz;
            while (secular_f(K, d, z, rho, org, hi) < 0.0) hi *= 2.0;
        }
        int it = 0;
        for (;;) {
            double mid = lo + 0.5 * (hi - lo);
            if (!(mid > lo && mid < hi)) break;
            double fm = secular_f(K, d, z, rho, org, mid);
            ++it;
            if (fm > 0.0)
                hi = mid;
            else if (fm < 0.0)
                lo = mid;
            else {
                lo = hi = mid;
                break;
            }
        }
        /* Keep whichever end of the final bracket gives the smaller |f|; the
         * end at a pole (tau == 0) is never a root. */
        double t;
        if (lo == 0.0 && org == j)
            t = hi;
        else if (hi == 0.0 && org == j + 1)
            t = lo;
        else {
            double flo = fabs(secular_f(K, d, z, rho, org, lo));
            double fhi = fabs(secular_f(K, d, z, rho, org, hi));
            t = (flo <= fhi) ? lo : hi;
        }
        o[j] = org;
        tau[j] = t;
        if (it > maxit) maxit = it;
    }
    return maxit;
}

/* d_i - lambda_j with lambda_j = d[o_j] + tau_j. */
static double dminus(const double *d, int i, const int *o, const double *tau, int j)
{
    return (d[i] - d[o[j]]) - tau[j];
}

/* ------------------------------------------------------------------------- */
/* Loewner recomputation of z (Sec. 1 and Remark 1).  Given the computed      */
/* eigenvalues lambda and the poles d, the vector zhat for which the lambdas  */
/* are the exact eigenvalues of D + rho*zhat*zhat^T satisfies                  */
/*   rho * zhat_i^2 = prod_j (lambda_j - d_i) / prod_{k != i} (d_k - d_i).      */
/* The products are paired so that every factor lies in (0, 1]:               */
/*   j <  i   : (d_i - lambda_j) / (d_i - d_j)                                  */
/*   i <= j < K-1 : (lambda_j - d_i) / (d_{j+1} - d_i)                          */
/* times the single unpaired numerator (lambda_{K-1} - d_i).                  */
/* The sign of zhat_i is taken from z_i.                                      */
/* ------------------------------------------------------------------------- */
void or_lowner(int K, const double *d, double rho, const int *o, const double *tau, const double *z,
               double *zhat)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < K; ++i) {
        double w = -dminus(d, i, o, tau, K - 1); /* lambda_{K-1} - d_i */
        for (int j = 0; j < i; ++j) w *= dminus(d, i, o, tau, j) / (d[i] - d[j]);
        for (int j = i; j < K - 1; ++j) w *= -dminus(d, i, o, tau, j) / (d[j + 1] - d[i]);
        double mag = sqrt(w / rho);
        zhat[i] = (z[i] < 0.0) ? -mag : mag;
    }
}

/* ------------------------------------------------------------------------- */
/* Eigenvectors of D + rho*zhat*zhat^T (Sec. 1, after Eq. (4)):               */
/*   qhat_j = (D - lambda_j I)^{-1} zhat, scaled to unit 2-norm.               */
/* U is K x K column-major: U(i,j) = zhat_i / (d_i - lambda_j) / norm_j.       */
/* ------------------------------------------------------------------------- */
void or_uhat(int K, const double *d, const int *o, const double *tau, const double *zhat, double *U,
             int ldu)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < K; ++j) {
        double nrm2 = 0.0;
        for (int i = 0; i < K; ++i) {
            double v = zhat[i] / dminus(d, i, o, tau, j);
            A_(U, ldu, i, j) = v;
            nrm2 += v * v;
        }
        double inv = 1.0 / sqrt(nrm2);
        for (int i = 0; i < K; ++i) A_(U, ldu, i, j) *= inv;
    }
}

/* ------------------------------------------------------------------------- */
/* One merge step: the spectral decomposition of                              */
/*     diag(Q1, Q2) (diag(D1, D2) + rho z z^T) diag(Q1, Q2)^T                  */
/* (Eq. (3)-(6)).  D1 = D[0:n1] and D2 = D[n1:m] must each be ascending.      */
/* z is any vector, rho >= 0.  Output: lam ascending (m), Q (m x m).          */
/*                                                                            */
/* Steps, in the paper's order:                                               */
/*  1. normalise: rho <- rho*|z|^2, z <- z/|z|;                               */
/*  2. sort the poles ascending (ties keep D1 before D2);                     */
/*  3. deflation (Sec. 1, after Remark 1):                                    */
/*     type 1: rho*|z_i| <= tol removes pole i with its column unchanged;     */
/*     type 2: for consecutive surviving poles p < j, the plane rotation that  */
/*     zeroes z_p is applied when its off-diagonal residue |(d_j-d_p) c s| is */
/*     <= tol; p is removed with value d_p c^2 + d_j s^2 and j carries on with */
/*     value d_p s^2 + d_j c^2 and z_j = hypot(z_p, z_j);                      */
/*     tol = 8 u max(max|d|, rho) with u the unit roundoff;                    */
/*  4. secular roots of the K survivors (or_secular);                         */
/*  5. Loewner zhat (or_lowner) and the eigenvector matrix Uhat (or_uhat);    */
/*  6. eigenvectors (Eq. (6)): [Q G P](:, survivors) * Uhat, and the removed  */
/*     columns of Q G P unchanged;                                            */
/*  7. all m eigenvalues sorted ascending with their columns (ties: secular   */
/*     roots first, then removed poles in pole order).                        */
/* stats (may be NULL) receives {K, k1, k2, k3, n_type1, n_type2, 0, 0}: K    */
/* survivors, of which k1 touch only Q1's rows, k3 only Q2's rows and k2 both. */
/* ------------------------------------------------------------------------- */
int or_merge(int n1, int n2, const double *D, const double *z, double rho, const double *Q1, int ldq1,
             const double *Q2, int ldq2, double *lam, double *Q, int ldq, int *stats)
{
    int m = n1 + n2;
    if (m == 0) return 0;
    /* X = diag(Q1, Q2) as a dense m x m matrix; rotations act on its columns. */
    double *X = calloc((size_t)m * m, sizeof(double));
    for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) A_(X, m, i, j) = A_(Q1, ldq1, i, j);
    for (int j = 0; j < n2; ++j)
        for (int i = 0; i < n2; ++i) A_(X, m, n1 + i, n1 + j) = A_(Q2, ldq2, i, j);

    /* 1. normalise */
    double zz = 0.0;
    for (int i = 0; i < m; ++i) zz += z[i] * z[i];
    double zn = sqrt(zz);
    double r = rho * zz;
    double *dv = malloc(sizeof(double) * m), *zv = malloc(sizeof(double) * m);
    int *col = malloc(sizeof(int) * m), *part = malloc(sizeof(int) * m);
    /* 2. sort ascending, stable: merge of the two ascending runs. */
    {
        int a = 0, b = 0, k = 0;
        while (a < n1 || b < n2) {
            int takeA = (b >= n2) || (a < n1 && D[a] <= D[n1 + b]);
            int src = takeA ? a++ : n1 + b++;
            dv[k] = D[src];
            zv[k] = (zn > 0.0) ? z[src] / zn : 0.0;
            col[k] = src;
            part[k] = takeA ? 1 : 3; /* 1: rows of Q1 only, 3: rows of Q2 only, 2: both */
            ++k;
        }
    }
    double dmax = 0.0;
    for (int i = 0; i < m; ++i)
        if (fabs(dv[i]) > dmax) dmax = fabs(dv[i]);
    double tol = 8.0 * OR_U * (dmax > r ? dmax : r);

    /* 3. deflation */
    int *defl = calloc(m, sizeof(int)); /* 0 survivor, 1 type-1, 2 type-2 */
    int ntype1 = 0, ntype2 = 0;
    for (int i = 0; i < m; ++i)
        if (r * fabs(zv[i]) <= tol) {
            defl[i] = 1;
            ++ntype1;
        }
    int p = -1;
    for (int j = 0; j < m; ++j) {
        if (defl[j]) continue;
        if (p < 0) {
            p = j;
            continue;
        }
        double tau = hypot(zv[p], zv[j]);
        double c = zv[j] / tau, s = -zv[p] / tau;
        double t = dv[j] - dv[p];
        if (fabs(t * c * s) <= tol) {
            /* rotate columns p and j of X: x_p' = c x_p + s x_j, x_j' = c x_j - s x_p */
            int cp = col[p], cj = col[j];
            for (int i = 0; i < m; ++i) {
                double xp = A_(X, m, i, cp), xj = A_(X, m, i, cj);
                A_(X, m, i, cp) = c * xp + s * xj;
                A_(X, m, i, cj) = c * xj - s * xp;
            }
            double dp = dv[p] * c * c + dv[j] * s * s;
            double dj = dv[p] * s * s + dv[j] * c * c;
            dv[p] = dp;
            dv[j] = dj;
            zv[j] = tau;
            zv[p] = 0.0;
            if (part[p] != part[j]) part[j] = 2;
            defl[p] = 2;
            ++ntype2;
        }
        p = j;
    }
    int K = m - ntype1 - ntype2;

    /* survivors (ascending d) and removed poles */
    double *ds = malloc(sizeof(double) * (K ? K : 1)), *zs = malloc(sizeof(double) * (K ? K : 1));
    int *cs = malloc(sizeof(int) * (K ? K : 1));
    int k1 = 0, k2 = 0, k3 = 0;
    {
        int k = 0;
        for (int i = 0; i < m; ++i)
            if (!defl[i]) {
                ds[k] = dv[i];
                zs[k] = zv[i];
                cs[k] = col[i];
                if (part[i] == 1) ++k1;
                else if (part[i] == 2) ++k2;
                else ++k3;
                ++k;
            }
    }

    /* 4.-5. secular roots, Loewner zhat, Uhat */
    int *o = malloc(sizeof(int) * (K ? K : 1));
    double *tau = malloc(sizeof(double) * (K ? K : 1));
    double *zh = malloc(sizeof(double) * (K ? K : 1));
    double *U = malloc(sizeof(double) * ((size_t)K * K ? (size_t)K * K : 1));
    if (K > 0) {
        or_secular(K, ds, zs, r, o, tau);
        or_lowner(K, ds, r, o, tau, zs, zh);
        or_uhat(K, ds, o, tau, zh, U, K);
    }

    /* 6. eigenvectors: Y(:, 0:K) = X(:, survivors) * Uhat; Y(:, K:m) removed columns */
    double *Y = malloc(sizeof(double) * (size_t)m * m);
    double *ly = malloc(sizeof(double) * m);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < K; ++j) {
        for (int i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int l = 0; l < K; ++l) acc += A_(X, m, i, cs[l]) * A_(U, K, l, j);
            A_(Y, m, i, j) = acc;
        }
        ly[j] = ds[o[j]] + tau[j];
    }
    {
        int k = K;
        for (int i = 0; i < m; ++i)
            if (defl[i]) {
                for (int r2 = 0; r2 < m; ++r2) A_(Y, m, r2, k) = A_(X, m, r2, col[i]);
                ly[k] = dv[i];
                ++k;
            }
    }

    /* 7. stable sort of all m eigenvalues with their columns */
    int *ord = malloc(sizeof(int) * m);
    for (int i = 0; i < m; ++i) ord[i] = i;
    for (int i = 1; i < m; ++i) { /* insertion sort keeps equal keys in order */
        int v = ord[i], k = i - 1;
        while (k >= 0 && ly[ord[k]] > ly[v]) {
            ord[k + 1] = ord[k];
            --k;
        }
        ord[k + 1] = v;
    }
    for (int j = 0; j < m; ++j) {
        lam[j] = ly[ord[j]];
        for (int i = 0; i < m; ++i) A_(Q, ldq, i, j) = A_(Y, m, i, ord[j]);
    }
    if (stats) {
        stats[0] = K;
        stats[1] = k1;
        stats[2] = k2;
        stats[3] = k3;
        stats[4] = ntype1;
        stats[5] = ntype2;
        stats[6] = 0;
        stats[7] = 0;
    }
    free(X); free(dv); free(zv); free(col); free(part); free(defl);
    free(ds); free(zs); free(cs); free(o); free(tau); free(zh); free(U);
    free(Y); free(ly); free(ord);
    return K;
}

/* ------------------------------------------------------------------------- */
/* Divide and conquer over the tridiagonal T of Eq. (1) (diagonal d[0:m],      */
/* off-diagonal e[0:m-1]).                                                    */
/* Split (Eq. (2)): at k = floor(m/2), T = diag(T1, T2) + rho v v^T with       */
/* rho = |e_{k-1}| and v = e_{k-1} + sign(e_{k-1}) e_k (unit vectors), so the  */
/* last diagonal entry of T1 and the first of T2 each lose rho.  Recursion    */
/* stops at blocks of at most `leaf` rows, solved by or_jacobi.  Merge        */
/* (Eq. (3)): z = [last row of Q1, sign(e_{k-1}) * first row of Q2].          */
/* d is modified in place (corner updates).  stats_top (may be NULL) gets the */
/* or_merge statistics of the top-level merge.                                */
/* ------------------------------------------------------------------------- */
static int stedc_rec(int m, double *d, const double *e, double *lam, double *Q, int ldq, int leaf,
                     int *stats_top, int depth)
{
    if (m <= 0) return 0;
    if (m <= leaf) {
        double *A = calloc((size_t)m * m, sizeof(double));
        double *V = malloc(sizeof(double) * (size_t)m * m);
        for (int i = 0; i < m; ++i) A_(A, m, i, i) = d[i];
        for (int i = 0; i + 1 < m; ++i) {
            A_(A, m, i + 1, i) = e[i];
            A_(A, m, i, i + 1) = e[i];
        }
        int rc = or_jacobi(m, A, m, lam, V, m);
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) A_(Q, ldq, i, j) = A_(V, m, i, j);
        free(A);
        free(V);
        return rc < 0 ? 1 : 0;
    }
    int k = m / 2;
    double b = e[k - 1];
    double rho = fabs(b);
    double sg = (b < 0.0) ? -1.0 : 1.0;
    d[k - 1] -= rho;
    d[k] -= rho;
    int n1 = k, n2 = m - k;
    double *Q1 = malloc(sizeof(double) * (size_t)n1 * n1);
    double *Q2 = malloc(sizeof(double) * (size_t)n2 * n2);
    double *D = malloc(sizeof(double) * m);
    int info = stedc_rec(n1, d, e, D, Q1, n1, leaf, NULL, depth + 1);
    info |= stedc_rec(n2, d + k, e + k, D + k, Q2, n2, leaf, NULL, depth + 1);
    double *z = malloc(sizeof(double) * m);
    for (int i = 0; i < n1; ++i) z[i] = A_(Q1, n1, n1 - 1, i);
    for (int i = 0; i < n2; ++i) z[n1 + i] = sg * A_(Q2, n2, 0, i);
    or_merge(n1, n2, D, z, rho, Q1, n1, Q2, n2, lam, Q, ldq, depth == 0 ? stats_top : NULL);
    free(Q1);
    free(Q2);
    free(D);
    free(z);
    return info;
}

/* All eigenvalues (ascending, lam[0:n]) and eigenvectors (Q, n x n) of the
 * symmetric tridiagonal matrix with diagonal d[0:n] and off-diagonal e[0:n-1].
 * d and e are not modified.  Returns 0, or 1 if a leaf failed to converge. */
int or_stedc(int n, const double *d, const double *e, double *lam, double *Q, int ldq, int leaf,
             int *stats_top)
{
    if (n <= 0) return 0;
    if (leaf < 1) leaf = 1;
    double *dw = malloc(sizeof(double) * n);
    memcpy(dw, d, sizeof(double) * n);
    int info = stedc_rec(n, dw, e, lam, Q, ldq, leaf, stats_top, 0);
    free(dw);
    return info;
}

/* ------------------------------------------------------------------------- */
/* Adjoint of the eigen-decomposition T = Q diag(lambda) Q^T with respect to   */
/* the tridiagonal entries.  For a loss L(lambda, Q) with gradients lbar and   */
/* Qbar, first-order perturbation theory of a symmetric eigenproblem with     */
/* simple eigenvalues gives                                                   */
/*   Tbar = Q (diag(lbar) + F o (Q^T Qbar)) Q^T,  F_ij = 1/(lambda_j - lambda_i) */
/* for i != j and 0 on the diagonal.  d_i enters T at (i,i) and e_i at        */
/* (i,i+1) and (i+1,i), so dbar_i = Tbar_ii and ebar_i = Tbar_{i,i+1} +       */
/* Tbar_{i+1,i}.                                                              */
/* ------------------------------------------------------------------------- */
void or_adjoint(int n, const double *lam, const double *Q, int ldq, const double *lbar,
                const double *Qbar, int ldqb, double *dbar, double *ebar)
{
    double *M = malloc(sizeof(double) * (size_t)n * n); /* Q^T Qbar, then diag(lbar) + F o . */
    double *W = malloc(sizeof(double) * (size_t)n * n); /* Q M */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += A_(Q, ldq, k, i) * A_(Qbar, ldqb, k, j);
            A_(M, n, i, j) = (i == j) ? lbar[i] : acc / (lam[j] - lam[i]);
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += A_(Q, ldq, i, k) * A_(M, n, k, j);
            A_(W, n, i, j) = acc;
        }
    /* Tbar(a,b) = sum_j W(a,j) Q(b,j) on the band only. */
    for (int a = 0; a < n; ++a) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += A_(W, n, a, j) * A_(Q, ldq, a, j);
        dbar[a] = acc;
    }
    for (int a = 0; a + 1 < n; ++a) {
        double up = 0.0, lo = 0.0;
        for (int j = 0; j < n; ++j) {
            up += A_(W, n, a, j) * A_(Q, ldq, a + 1, j);
            lo += A_(W, n, a + 1, j) * A_(Q, ldq, a, j);
        }
        ebar[a] = up + lo;
    }
    free(M);
    free(W);
}

/* Plain matrix product C = A * B (A: m x k, B: k x n, all column-major). */
void or_gemm(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int l = 0; l < k; ++l) acc += A_(A, lda, i, l) * A_(B, ldb, l, j);
            A_(C, ldc, i, j) = acc;
        }
}
