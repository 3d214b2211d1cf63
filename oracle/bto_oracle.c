/*
 * Reference oracle for the nine BLAS-1/2 kernels of Table I (and BATAX's
 * building block, ATAX) of Belter, Jessup,
 * Nelson, Norris and Siek, "Reliable Generation of High-Performance Matrix
 * Algebra" (the Build to Order BLAS).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or helper with the
 * GPU library.
 *
 * What it computes is the plain definition of each kernel from Table I
 * (Section V-A), written as the unfused loop nests of Fig. 5 (Section III-D):
 * one loop nest per statement, statements in the order the table lists them,
 * every reduction accumulated in increasing index order, every scale factor
 * applied after its reduction.  Loop fusion, contraction and partitioning,
 * which the paper shows preserve these semantics (Section III-D), are the
 * GPU library's business, not this file's.
 *
 * Conventions (shared with the C entry points only by specification):
 *   - A is m x n, row-major, element (i, j) at A[i*lda + j], lda >= n.
 *   - All arithmetic is binary64; the file is compiled with
 *     -ffp-contract=off so that no multiply-add is fused.
 *   - The long dot product of AXPYDOT uses pairwise summation (sequential
 *     below 128 terms, otherwise split at floor(L/2)); every matrix
 *     reduction is sequential.
 *   - OpenMP, when enabled, only splits loops whose iterations own disjoint
 *     outputs and keeps each output's summation order, so results are
 *     bitwise identical for any thread count.
 *
 * Parity pins: every function here is checked by the test suite against
 * exact rational arithmetic on tiny inputs, exact integer arithmetic at
 * larger sizes, closed forms (identity, permutation, diagonal and rank-1
 * matrices) and algebraic invariants.  None is left unpinned.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
static int g_threads = 1;

void oracle_set_threads(int t)
{
    g_threads = t < 1 ? 1 : t;
#ifdef _OPENMP
    omp_set_num_threads(g_threads);
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return g_threads;
#else
    return 1;
#endif
}

/* Column block used to split a column-sum loop over threads: each thread
 * owns a contiguous set of output columns and walks all rows for them. */
#define COLBLK 256

/* out[i] = sum_{j=0..n-1} A[i,j] * v[j], j ascending (a row dot per row). */
static void rowdots(int64_t m, int64_t n, const double *A, int64_t lda,
                    const double *v, double *out)
{
    int64_t i;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (i = 0; i < m; ++i) {
        const double *a = A + i * lda;
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j)
            acc += a[j] * v[j];
        out[i] = acc;
    }
}

/* out[j] = sum_{i=0..m-1} A[i,j] * v[i], i ascending (a column sum per
 * column), the loop order of the second nest of Fig. 5: i outer, j inner. */
static void colsums(int64_t m, int64_t n, const double *A, int64_t lda,
                    const double *v, double *out)
{
    int64_t nblk = (n + COLBLK - 1) / COLBLK, b;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (b = 0; b < nblk; ++b) {
        int64_t j0 = b * COLBLK, j1 = j0 + COLBLK < n ? j0 + COLBLK : n;
        for (int64_t j = j0; j < j1; ++j)
            out[j] = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const double *a = A + i * lda;
            double vi = v[i];
            for (int64_t j = j0; j < j1; ++j)
                out[j] += a[j] * vi;
        }
    }
}

/* Pairwise (cascade) summation of x[k]*y[k], k in [0, len). */
static double pairwise_dot(const double *x, const double *y, int64_t len)
{
    if (len < 128) {
        double acc = 0.0;
        for (int64_t k = 0; k < len; ++k)
            acc += x[k] * y[k];
        return acc;
    }
    int64_t h = len / 2;
    return pairwise_dot(x, y, h) + pairwise_dot(x + h, y + h, len - h);
}

/* BICGK, Table I:  q <- A p ;  s <- A^T r.
 * The BLAS form of Section V-A: two dgemv calls, 'N' then 'T'. */
void oracle_bicgk(int64_t m, int64_t n, const double *A, int64_t lda,
                  const double *p, const double *r, double *q, double *s)
{
    rowdots(m, n, A, lda, p, q);
    colsums(m, n, A, lda, r, s);
}

/* GEMVER, Table I:
 *   B <- A + u1 v1^T + u2 v2^T      B[i,j] = (A[i,j] + u1[i]*v1[j]) + u2[i]*v2[j]
 *   x <- beta B^T y + z             x[j] = beta * (sum_i B[i,j]*y[i]) + z[j]
 *   w <- alpha B x                  w[i] = alpha * (sum_j B[i,j]*x[j])
 * The statements run in order, so w uses the x just computed.  B may be the
 * same array as A (ldb == lda): the update is elementwise. */
void oracle_gemver(int64_t m, int64_t n, double alpha, double beta,
                   const double *A, int64_t lda,
                   const double *u1, const double *v1,
                   const double *u2, const double *v2,
                   const double *y, const double *z,
                   double *B, int64_t ldb, double *x, double *w)
{
    int64_t i;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (i = 0; i < m; ++i) {
        const double *a = A + i * lda;
        double *b = B + i * ldb;
        for (int64_t j = 0; j < n; ++j) {
            double t = a[j] + u1[i] * v1[j];
            b[j] = t + u2[i] * v2[j];
        }
    }
    colsums(m, n, B, ldb, y, x);
    for (int64_t j = 0; j < n; ++j)
        x[j] = beta * x[j] + z[j];
    rowdots(m, n, B, ldb, x, w);
    for (i = 0; i < m; ++i)
        w[i] = alpha * w[i];
}

/* ATAX, Table I:  y <- A^T A x, i.e. the loops of Fig. 5 without the beta
 * scale:  t[i] = sum_j A[i,j]*x[j];  y[j] = sum_i A[i,j]*t[i]. */
void oracle_atax(int64_t m, int64_t n, const double *A, int64_t lda,
                 const double *x, double *y)
{
    double *t = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    if (!t)
        abort();
    rowdots(m, n, A, lda, x, t);
    colsums(m, n, A, lda, t, y);
    free(t);
}

/* DGEMVT, Table I:
 *   x <- beta A^T y + z       x[j] = beta * (sum_i A[i,j]*y[i]) + z[j]
 *   w <- alpha A x            w[i] = alpha * (sum_j A[i,j]*x[j]), new x. */
void oracle_dgemvt(int64_t m, int64_t n, double alpha, double beta,
                   const double *A, int64_t lda,
                   const double *y, const double *z, double *x, double *w)
{
    colsums(m, n, A, lda, y, x);
    for (int64_t j = 0; j < n; ++j)
        x[j] = beta * x[j] + z[j];
    rowdots(m, n, A, lda, x, w);
    for (int64_t i = 0; i < m; ++i)
        w[i] = alpha * w[i];
}

/* DGEMV, Table I:  z <- alpha A x + beta y,
 *   z[i] = alpha * (sum_j A[i,j]*x[j]) + beta * y[i].
 * One BLAS call (Section V-A).  z may be the same array as y: the row dots
 * go to a temporary first. */
void oracle_dgemv(int64_t m, int64_t n, double alpha, double beta,
                  const double *A, int64_t lda, const double *x,
                  const double *y, double *z)
{
    double *t = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    if (!t)
        abort();
    rowdots(m, n, A, lda, x, t);
    for (int64_t i = 0; i < m; ++i) {
        double a = alpha * t[i];
        double b = beta * y[i];
        z[i] = a + b;
    }
    free(t);
}

/* GESUMMV, Table I:  y <- alpha A x + beta B x,
 *   y[i] = alpha * (sum_j A[i,j]*x[j]) + beta * (sum_j B[i,j]*x[j]).
 * A and B are both m x n, row-major, with their own leading dimensions. */
void oracle_gesummv(int64_t m, int64_t n, double alpha, double beta,
                    const double *A, int64_t lda, const double *B, int64_t ldb,
                    const double *x, double *y)
{
    double *t = (double *)malloc((size_t)(m > 0 ? 2 * m : 2) * sizeof(double));
    if (!t)
        abort();
    rowdots(m, n, A, lda, x, t);
    rowdots(m, n, B, ldb, x, t + m);
    for (int64_t i = 0; i < m; ++i) {
        double a = alpha * t[i];
        double b = beta * t[m + i];
        y[i] = a + b;
    }
    free(t);
}

/* AXPYDOT, Table I (its scalar result is named beta there, r here):
 *   z <- w - alpha v ;  r <- z^T u   (pairwise sum).
 * z may be the same array as w. */
void oracle_axpydot(int64_t n, double alpha, const double *w, const double *v,
                    const double *u, double *z, double *r)
{
    for (int64_t k = 0; k < n; ++k)
        z[k] = w[k] - alpha * v[k];
    *r = pairwise_dot(z, u, n);
}

/* WAXPBY, Table I:  w <- alpha x + beta y,  w[k] = alpha*x[k] + beta*y[k]. */
void oracle_waxpby(int64_t n, double alpha, const double *x, double beta,
                   const double *y, double *w)
{
    for (int64_t k = 0; k < n; ++k) {
        double a = alpha * x[k];
        double b = beta * y[k];
        w[k] = a + b;
    }
}

/* VADD, Table I:  x <- w + y + z,  x[k] = (w[k] + y[k]) + z[k]. */
void oracle_vadd(int64_t n, const double *w, const double *y, const double *z,
                 double *x)
{
    for (int64_t k = 0; k < n; ++k) {
        double t = w[k] + y[k];
        x[k] = t + z[k];
    }
}
