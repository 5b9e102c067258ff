/*
 * dm_oracle.c - CPU oracle for the distance-matrix matrix-vector product.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the HIP library.
 *
 * What it computes is the plain definition of the query (Section 1, the
 * matrix-vector query model; Theorem for p = 1 in Section 2):
 *
 *     (A z)_i = sum_j z_j * f(x_i, x_j)
 *
 * with f(x, y) = sum_k |x(k) - y(k)|          (l1, Section 2),
 *      f(x, y) = sum_k (x(k) - y(k))^2        (l2 squared, Appendix A, p = 2)
 *      f(x, y) = (1/2) sum_k |x(k) - y(k)|    (total variation of two
 *      distributions given as probability vectors, Appendix A.3; FP64 only)
 *      f(x, y) = sum_k |x(k) - y(k)|^p, p = 3 or 5   (l_p^p for odd p,
 *      Appendix A.1; the power by repeated multiplication)
 *      f(x, y) = sum_k (x(k) - y(k))^p, p = 4 or 6    (l_p^p for even p,
 *      the even-p theorem of Appendix A.1)
 * and, FP64 only, with a d x d matrix M where one is named:
 *      f(x, y) = sum_k x(k) log(x(k) / y(k))     (KL divergence D(x || y),
 *                the KL theorem of Appendix A; 0 log 0 = 0)
 *      f(x, y) = -sum_k x(k) log y(k)           (cross entropy, Appendix A.3)
 *      f(x, y) = (x - y)^T M (x - y)            (squared Mahalanobis distance)
 *      f(x, y) = x^T M y                        (the bilinear form that the
 *                Mahalanobis paragraph of Appendix A.2 writes down)
 *
 * Each requested row of A is formed explicitly, entry by entry (a difference
 * then an absolute value or a power, a logarithm of a ratio, or a quadratic
 * form, summed over the coordinates), and then multiplied by Z with j
 * ascending.  No prefix sums, no sorting, no moment or norm expansion are
 * used, so the oracle shares neither the l1 method's scan nor the
 * cancellation of the expanded forms.
 *
 * Floating point: every quantity is FP64, compiled with -ffp-contract=off.
 * Integer variant: int64 inputs, entries and products in __int128, so the
 * result is exact; a flag reports any output that does not fit in int64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

#define DM_ORACLE_L1 1
#define DM_ORACLE_L2SQ 2
#define DM_ORACLE_TV 3
#define DM_ORACLE_L3 4
#define DM_ORACLE_L5 5
#define DM_ORACLE_L4 6
#define DM_ORACLE_L6 7
#define DM_ORACLE_KL 8
#define DM_ORACLE_CE 9
#define DM_ORACLE_MAHA2 10
#define DM_ORACLE_BILINEAR 11

/* The distances that need a logarithm or the matrix M, entry by entry as
 * written in their definitions above. */
static double entry_form_f64(const double* xi, const double* xj, int32_t d, int metric, const double* M)
{
    double a = 0.0;
    if (metric == DM_ORACLE_KL) {
        for (int32_t k = 0; k < d; ++k)
            if (xi[k] != 0.0) a += xi[k] * log(xi[k] / xj[k]);
    } else if (metric == DM_ORACLE_CE) {
        for (int32_t k = 0; k < d; ++k)
            if (xi[k] != 0.0) a -= xi[k] * log(xj[k]);
    } else if (metric == DM_ORACLE_MAHA2) {
        for (int32_t k = 0; k < d; ++k)
            for (int32_t l = 0; l < d; ++l)
                a += (xi[k] - xj[k]) * M[(int64_t)k * d + l] * (xi[l] - xj[l]);
    } else {
        for (int32_t k = 0; k < d; ++k)
            for (int32_t l = 0; l < d; ++l)
                a += xi[k] * M[(int64_t)k * d + l] * xj[l];
    }
    return a;
}

/* One entry of A in FP64: f(x_i, x_j). */
static double entry_f64(const double* xi, const double* xj, int32_t d, int metric, const double* M)
{
    if (metric >= DM_ORACLE_KL) return entry_form_f64(xi, xj, d, metric, M);
    double a = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double diff = xi[k] - xj[k];
        if (metric == DM_ORACLE_L1 || metric == DM_ORACLE_TV) {
            a += fabs(diff);
        } else if (metric == DM_ORACLE_L3 || metric == DM_ORACLE_L5) {
            double ad = fabs(diff), pw = ad;
            for (int e = 1; e < (metric == DM_ORACLE_L3 ? 3 : 5); ++e) pw *= ad;
            a += pw;
        } else if (metric == DM_ORACLE_L4 || metric == DM_ORACLE_L6) {
            double pw = diff;
            for (int e = 1; e < (metric == DM_ORACLE_L4 ? 4 : 6); ++e) pw *= diff;
            a += pw;
        } else {
            a += diff * diff;
        }
    }
    return metric == DM_ORACLE_TV ? 0.5 * a : a;
}

/* One entry of A exactly, from int64 coordinates. */
static __int128 entry_i128(const int64_t* xi, const int64_t* xj, int32_t d, int metric)
{
    __int128 a = 0;
    for (int32_t k = 0; k < d; ++k) {
        __int128 diff = (__int128)xi[k] - (__int128)xj[k];
        __int128 ad = diff < 0 ? -diff : diff;
        if (metric == DM_ORACLE_L1) {
            a += ad;
        } else if (metric == DM_ORACLE_L3 || metric == DM_ORACLE_L5) {
            /* exact while |diff|^p fits: |diff| < 2^25 for p = 5 */
            __int128 pw = ad;
            for (int e = 1; e < (metric == DM_ORACLE_L3 ? 3 : 5); ++e) pw *= ad;
            a += pw;
        } else if (metric == DM_ORACLE_L4 || metric == DM_ORACLE_L6) {
            /* exact while d |diff|^p < 2^127: |diff| < 2^21 for p = 6 */
            __int128 pw = diff;
            for (int e = 1; e < (metric == DM_ORACLE_L4 ? 4 : 6); ++e) pw *= diff;
            a += pw;
        } else {
            a += diff * diff;
        }
    }
    return a;
}

/*
 * Rows `rows[0..m)` of the explicit distance matrix, A_out is m x n row-major.
 * X is n x d row-major; M is d x d row-major (NULL unless the metric uses it).
 */
void oracle_rows_f64(const double* X, int64_t n, int32_t d, int metric, const double* M,
                     const int64_t* rows, int64_t m, double* A_out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < m; ++t) {
        const double* xi = X + rows[t] * (int64_t)d;
        for (int64_t j = 0; j < n; ++j)
            A_out[t * n + j] = entry_f64(xi, X + j * (int64_t)d, d, metric, M);
    }
}

/*
 * Y[t, c] = sum_j A[rows[t], j] * Z[j, c]   (Z is n x b row-major, Y is m x b)
 * rownorm2[t]  = sum_j A[rows[t], j]^2                 (may be NULL)
 * absdot[t, c] = sum_j |A[rows[t], j]| * |Z[j, c]|     (may be NULL)
 */
void oracle_matvec_f64(const double* X, int64_t n, int32_t d, int metric, const double* M,
                       const double* Z, int32_t b, const int64_t* rows, int64_t m,
                       double* Y, double* rownorm2, double* absdot)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < m; ++t) {
        const double* xi = X + rows[t] * (int64_t)d;
        double* y = Y + t * (int64_t)b;
        double* ad = absdot ? absdot + t * (int64_t)b : NULL;
        double rn = 0.0;
        for (int32_t c = 0; c < b; ++c) {
            y[c] = 0.0;
            if (ad) ad[c] = 0.0;
        }
        for (int64_t j = 0; j < n; ++j) {
            double a = entry_f64(xi, X + j * (int64_t)d, d, metric, M);
            const double* zj = Z + j * (int64_t)b;
            for (int32_t c = 0; c < b; ++c) {
                y[c] += a * zj[c];
                if (ad) ad[c] += fabs(a) * fabs(zj[c]);
            }
            rn += a * a;
        }
        if (rownorm2) rownorm2[t] = rn;
    }
}

/*
 * Exact integer variant.  Returns the number of outputs whose exact value does
 * not fit in int64 (those outputs hold the low 64 bits of the exact value).
 */
int64_t oracle_matvec_i64(const int64_t* X, int64_t n, int32_t d, int metric,
                          const int64_t* Z, int32_t b, const int64_t* rows, int64_t m,
                          int64_t* Y)
{
    int64_t overflow = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : overflow)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t* xi = X + rows[t] * (int64_t)d;
        __int128* acc = (__int128*)calloc((size_t)b, sizeof(__int128));
        for (int64_t j = 0; j < n; ++j) {
            __int128 a = entry_i128(xi, X + j * (int64_t)d, d, metric);
            const int64_t* zj = Z + j * (int64_t)b;
            for (int32_t c = 0; c < b; ++c)
                acc[c] += a * (__int128)zj[c];
        }
        for (int32_t c = 0; c < b; ++c) {
            if (acc[c] > (__int128)INT64_MAX || acc[c] < (__int128)INT64_MIN) overflow += 1;
            Y[t * (int64_t)b + c] = (int64_t)(uint64_t)(unsigned __int128)acc[c];
        }
        free(acc);
    }
    return overflow;
}

/* Number of OpenMP threads the oracle runs on (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
