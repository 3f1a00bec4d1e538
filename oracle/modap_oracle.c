/*
 * CPU oracle for the pseudo-projection method on a system  A x <= b.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the method computes.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it.  It shares no code, header
 * or constant with the GPU library, and the GPU library never calls it.
 *
 * Definitions followed (Sokolinsky & Sokolinskaya, "Scalable Parallel
 * Algorithm for Solving Non-stationary Systems of Linear Inequalities"):
 *   - section 2: half-space P_i = { x : <a_i,x> <= b_i }, a_i != 0;
 *     reflection vector rho_i(x) = (<a_i,x> - b_i) / ||a_i||^2 * a_i;
 *   - eq. (7): positive slice rho+_i(x) = max(<a_i,x> - b_i, 0)/||a_i||^2 * a_i;
 *   - eq. (8): phi(x) = (1/h) * sum_i rho+_i(x), h = number of non-zero terms;
 *   - eq. (10): x is eps-feasible iff for every i either <a_i,x> <= b_i or
 *     |<a_i,x> - b_i| / ||a_i|| < eps.  This oracle compares with "<=": a row
 *     whose distance equals eps_abs counts as satisfied, which changes nothing
 *     but the case of exact equality;
 *   - eq. (12): psi(x) = lambda * phi(x)/||phi(x)||, which equals
 *     lambda * y/||y|| with y = sum_i rho+_i(x) (section 3, list form);
 *   - section 3, ModAP on lists: Map computes the list of positive slices,
 *     Reduce(+) sums them to y, the next approximation is x - psi, then the
 *     data are updated and the approximation is checked for eps-feasibility.
 *
 * Arithmetic: every stored element is widened exactly to double; every sum
 * (dot products, norms, the Reduce) is accumulated in x86 extended precision
 * (long double, 64-bit significand) in plain row order and rounded to double
 * once at the end.  No blocking, no reordering, no threads.
 *
 * Storage type codes: 0 = IEEE binary64, 1 = IEEE binary32, 2 = bfloat16
 * (the upper 16 bits of a binary32).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ext;

/* Exact widening of element idx of a stored matrix to double. */
static double elem(const void *A, int dtype, int64_t idx)
{
    if (dtype == 0) {
        return ((const double *)A)[idx];
    } else if (dtype == 1) {
        return (double)((const float *)A)[idx];
    } else {
        uint32_t bits = ((uint32_t)((const uint16_t *)A)[idx]) << 16;
        float f;
        memcpy(&f, &bits, sizeof f);
        return (double)f;
    }
}

/* <a_i, u> accumulated in extended precision. */
static ext row_dot(const void *A, int dtype, int64_t lda, int64_t i, int64_t n,
                   const double *u)
{
    ext s = 0.0L;
    for (int64_t j = 0; j < n; ++j)
        s += (ext)elem(A, dtype, i * lda + j) * (ext)u[j];
    return s;
}

/* ||a_i||^2 (the denominator of the reflection vector, section 2). */
static ext row_norm2(const void *A, int dtype, int64_t lda, int64_t i, int64_t n)
{
    ext s = 0.0L;
    for (int64_t j = 0; j < n; ++j) {
        ext a = (ext)elem(A, dtype, i * lda + j);
        s += a * a;
    }
    return s;
}

/*
 * Row norms nu_i = ||a_i||^2.  Returns -1 when every row is non-zero and
 * finite, else the index of the first zero or non-finite row (section 2
 * assumes a_i != 0 for all i).
 */
int64_t oracle_norms(int64_t m, int64_t n, int dtype, const void *A, int64_t lda,
                     double *nu)
{
    int64_t bad = -1;
    for (int64_t i = 0; i < m; ++i) {
        ext s = row_norm2(A, dtype, lda, i, n);
        nu[i] = (double)s;
        if (bad < 0 && (!(s > 0.0L) || !isfinite(nu[i])))
            bad = i;
    }
    return bad;
}

/*
 * Data update by translation of the feasible set by +v: each half-space
 * <a_i, x> <= b_i becomes <a_i, x - v> <= b_i, i.e. b_i <- b_i + <a_i, v>.
 * (Non-stationarity as a translation of the polytope, sections 2 and 5.)
 */
void oracle_translate(int64_t m, int64_t n, int dtype, const void *A, int64_t lda,
                      const double *v, double *b)
{
    for (int64_t i = 0; i < m; ++i)
        b[i] = (double)((ext)b[i] + row_dot(A, dtype, lda, i, n, v));
}

/*
 * One sweep at the point x on the data (A, b).  Outputs (any may be NULL
 * except y):
 *   r[i]   = <a_i, x> - b_i                          (residual)
 *   t[i]   = sum_j |a_ij x_j| + |b_i|                 (rounding-error scale of r[i])
 *   y[j]   = sum over i with r_i > 0 of (r_i/||a_i||^2) a_ij   (Map then Reduce(+))
 *   *h     = number of rows with r_i > 0              (non-zero terms of eq. (8))
 *   *dmax  = max over violated rows of r_i/||a_i||    (distance to P_i, eq. (10)); 0 if none
 *   *binf  = max_i |b_i|
 * nu may be NULL, in which case ||a_i||^2 is recomputed for every row, as
 * the Map of section 3 does.
 */
void oracle_sweep(int64_t m, int64_t n, int dtype, const void *A, int64_t lda,
                  const double *b, const double *nu, const double *x,
                  double *r, double *t, double *y, int64_t *h, double *dmax,
                  double *binf)
{
    ext *yy = (ext *)calloc((size_t)(n > 0 ? n : 1), sizeof(ext));
    int64_t count = 0;
    double worst = 0.0, bmax = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        ext res = row_dot(A, dtype, lda, i, n, x) - (ext)b[i];
        if (r)
            r[i] = (double)res;
        if (t) {
            ext sc = fabsl((ext)b[i]);
            for (int64_t j = 0; j < n; ++j)
                sc += fabsl((ext)elem(A, dtype, i * lda + j) * (ext)x[j]);
            t[i] = (double)sc;
        }
        if (fabs(b[i]) > bmax)
            bmax = fabs(b[i]);
        /* positive slice, eq. (7): non-zero iff row i is violated */
        if (res > 0.0L) {
            ext norm2 = nu ? (ext)nu[i] : row_norm2(A, dtype, lda, i, n);
            ext w = res / norm2;
            for (int64_t j = 0; j < n; ++j)
                yy[j] += w * (ext)elem(A, dtype, i * lda + j);
            count += 1;
            double d = (double)(res / sqrtl(norm2));
            if (d > worst)
                worst = d;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        y[j] = (double)yy[j];
    if (h)
        *h = count;
    if (dmax)
        *dmax = worst;
    if (binf)
        *binf = bmax;
    free(yy);
}

/*
 * The step of the iteration.
 *   rule 0 (ModAP, eq. (12)):  x <- x - lambda * y/||y||
 *   rule 1 (Algorithm 1 with relaxation lambda; lambda = 1 is Algorithm 1):
 *                              x <- x - (lambda/h) * y     (phi = y/h, eq. (8))
 * Returns 0 on success, 2 when ||y|| = 0 (no direction: no step possible).
 */
int oracle_step(int64_t n, const double *y, int64_t h, int rule, double lambda,
                double *x)
{
    ext nrm2 = 0.0L;
    for (int64_t j = 0; j < n; ++j)
        nrm2 += (ext)y[j] * (ext)y[j];
    if (!(nrm2 > 0.0L) || h <= 0)
        return 2;
    ext scale = (rule == 0) ? (ext)lambda / sqrtl(nrm2) : (ext)lambda / (ext)h;
    for (int64_t j = 0; j < n; ++j)
        x[j] = (double)((ext)x[j] - scale * (ext)y[j]);
    return 0;
}

/*
 * ModAP on lists, run to eps-feasibility (section 3), with the data updated
 * between steps by the translation schedule V (may be NULL): after step k
 * (k < T) the system is translated by V[k] (row k of a [T x ldv] array).
 *
 * Order of one iteration (readings of the listing, which is an image in the
 * text): check x_k against the current data (eq. (10)); if eps-feasible, stop
 * and output x_k; otherwise Map/Reduce at x_k to y, step to x_{k+1}, then
 * update the data.  The paper's check of x_{k+1} on the updated data, which
 * follows the data update, is the next iteration's check here; the only
 * addition is the check of x_0.
 *
 * eps_abs = eps * max_i |b_i| (current b) when eps_relative != 0, else eps.
 * Returns 0 converged, 1 step limit reached, 2 no direction (||y|| = 0 while
 * a row is violated), 3 zero or non-finite row.
 * Outputs: *iters = steps taken; *dmax_out, *h_out at the last check.
 * Optional traces (NULL to skip): dmax_trace[k] for k = 0..iters,
 * x_trace[k*n + j] for k = 0..iters.
 */
int oracle_solve(int64_t m, int64_t n, int dtype, const void *A, int64_t lda,
                 double *b, double *x, double lambda, double eps, int eps_relative,
                 int rule, int64_t max_steps, const double *V, int64_t T,
                 int64_t ldv, int64_t *iters, double *dmax_out, int64_t *h_out,
                 double *dmax_trace, double *x_trace)
{
    double *nu = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int status = 1;
    int64_t k = 0;
    if (oracle_norms(m, n, dtype, A, lda, nu) >= 0) {
        status = 3;
        goto done;
    }
    for (k = 0;; ++k) {
        int64_t h = 0;
        double dmax = 0.0, binf = 0.0;
        oracle_sweep(m, n, dtype, A, lda, b, nu, x, NULL, NULL, y, &h, &dmax, &binf);
        if (dmax_trace)
            dmax_trace[k] = dmax;
        if (x_trace)
            memcpy(x_trace + k * n, x, (size_t)n * sizeof(double));
        if (dmax_out)
            *dmax_out = dmax;
        if (h_out)
            *h_out = h;
        double eps_abs = eps_relative ? eps * binf : eps;
        if (dmax <= eps_abs) {
            status = 0;
            break;
        }
        if (k >= max_steps) {
            status = 1;
            break;
        }
        if (oracle_step(n, y, h, rule, lambda, x) != 0) {
            status = 2;
            break;
        }
        if (V && k < T)
            oracle_translate(m, n, dtype, A, lda, V + k * ldv, b);
    }
done:
    if (iters)
        *iters = k;
    free(nu);
    free(y);
    return status;
}

/*
 * Data update by replacement of rows (coefficients and right-hand side change
 * during the computation, section 1): row rows[q] of A becomes new_rows[q]
 * (stored type, [k x n]) and b[rows[q]] becomes new_b[q].
 */
void oracle_replace_rows(int64_t n, int dtype, void *A, int64_t lda, double *b,
                         int64_t k, const int64_t *rows, const void *new_rows,
                         const double *new_b)
{
    size_t es = dtype == 0 ? 8 : dtype == 1 ? 4 : 2;
    for (int64_t q = 0; q < k; ++q) {
        memcpy((char *)A + (size_t)(rows[q] * lda) * es,
               (const char *)new_rows + (size_t)(q * n) * es, (size_t)n * es);
        b[rows[q]] = new_b[q];
    }
}
