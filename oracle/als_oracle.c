/*
 * Plain FP64 CPU oracle for the ALS / ALS-NCG hot path.
 *
 * TEST INFRASTRUCTURE ONLY: this file exists to check the GPU library.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it; the product path never links or calls it, and it shares no code,
 * header or constant with the GPU library.
 *
 * Everything is double precision, written for readability, not speed: one
 * row of the ratings matrix at a time, textbook Cholesky, plain loops.  Rows
 * are independent inside a half-sweep (Section III-A), so the row loops are
 * shared out over OpenMP threads; every reduction first stores one partial
 * per row and then sums the partials in row order, so results do not depend
 * on the thread count.
 *
 * Notation follows the paper: user factors u_i and item factors m_j are rows
 * of U [n_u, n_f] and M [n_m, n_f] (row-major); I_i is the set of items rated
 * by user i, n_ui = |I_i|, and similarly n_mj for item j.
 *
 * The ratings come as a compressed sparse row structure (indptr int64
 * [n_rows+1], indices int32 [nnz], values double [nnz]).  For the item
 * orientation the same routine is called with the CSR of R^T.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Textbook Cholesky A = L L^T (lower triangle of the row-major n x n matrix A
 * is overwritten by L).  Returns 0, or k+1 when the k-th pivot is not
 * positive (A not numerically SPD). */
static int cholesky(double *A, int n)
{
    for (int k = 0; k < n; ++k) {
        double d = A[k * n + k];
        for (int p = 0; p < k; ++p) d -= A[k * n + p] * A[k * n + p];
        if (!(d > 0.0)) return k + 1;
        double lkk = sqrt(d);
        A[k * n + k] = lkk;
        for (int i = k + 1; i < n; ++i) {
            double s = A[i * n + k];
            for (int p = 0; p < k; ++p) s -= A[i * n + p] * A[k * n + p];
            A[i * n + k] = s / lkk;
        }
    }
    return 0;
}

/* Solve L L^T x = b in place (b becomes x). */
static void cholesky_solve(const double *L, int n, double *b)
{
    for (int i = 0; i < n; ++i) {          /* L y = b */
        double s = b[i];
        for (int p = 0; p < i; ++p) s -= L[i * n + p] * b[p];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {     /* L^T x = y */
        double s = b[i];
        for (int p = i + 1; p < n; ++p) s -= L[p * n + i] * b[p];
        b[i] = s / L[i * n + i];
    }
}

static double dot(const double *a, const double *b, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += a[k] * b[k];
    return s;
}

/*
 * One ALS half-sweep, Eq. (3) (or Eq. (4) when called with the CSR of R^T):
 * for every row i with n_i > 0,
 *     A_i = sum_{j in I_i} y_j y_j^T + lambda * n_i * I,
 *     v_i = sum_{j in I_i} r_ij y_j,
 *     x_i = A_i^{-1} v_i            (Cholesky, as in Section V-B),
 * where y_j are rows of the fixed factor Y.  Rows with n_i = 0 get x_i = 0
 * (the loss does not depend on them).  Returns 0, or -1 when some A_i is not
 * SPD; *bad_row then holds the smallest such row index.
 */
int orc_half_sweep(int64_t n_rows, const int64_t *indptr, const int32_t *indices,
                   const double *vals, const double *Y, int n_f, double lambda,
                   double *X, int64_t *bad_row)
{
    int64_t first_bad = -1;
#pragma omp parallel
    {
        double *A = (double *)malloc(sizeof(double) * (size_t)n_f * n_f);
        double *v = (double *)malloc(sizeof(double) * (size_t)n_f);
        int64_t my_bad = -1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n_rows; ++i) {
            int64_t b = indptr[i], e = indptr[i + 1];
            double *xi = X + i * n_f;
            if (e == b) {
                for (int k = 0; k < n_f; ++k) xi[k] = 0.0;
                continue;
            }
            memset(A, 0, sizeof(double) * (size_t)n_f * n_f);
            memset(v, 0, sizeof(double) * (size_t)n_f);
            for (int64_t t = b; t < e; ++t) {
                const double *y = Y + (int64_t)indices[t] * n_f;
                double r = vals[t];
                for (int p = 0; p < n_f; ++p) {
                    for (int q = p; q < n_f; ++q) A[p * n_f + q] += y[p] * y[q];
                    v[p] += r * y[p];
                }
            }
            for (int p = 0; p < n_f; ++p)       /* A is symmetric: mirror the upper triangle */
                for (int q = 0; q < p; ++q) A[p * n_f + q] = A[q * n_f + p];
            double reg = lambda * (double)(e - b);
            for (int p = 0; p < n_f; ++p) A[p * n_f + p] += reg;
            if (cholesky(A, n_f) != 0) {
                if (my_bad < 0 || i < my_bad) my_bad = i;
                for (int k = 0; k < n_f; ++k) xi[k] = NAN;
                continue;
            }
            cholesky_solve(A, n_f, v);
            for (int k = 0; k < n_f; ++k) xi[k] = v[k];
        }
#pragma omp critical
        {
            if (my_bad >= 0 && (first_bad < 0 || my_bad < first_bad)) first_bad = my_bad;
        }
        free(A);
        free(v);
    }
    if (bad_row) *bad_row = first_bad;
    return first_bad >= 0 ? -1 : 0;
}

/* n_mj: number of ratings of every column, counted from the CSR itself. */
static int64_t *column_counts(int64_t nnz, const int32_t *indices, int64_t n_cols)
{
    int64_t *c = (int64_t *)calloc((size_t)n_cols, sizeof(int64_t));
    for (int64_t t = 0; t < nnz; ++t) c[indices[t]]++;
    return c;
}

/*
 * Loss of Eq. (1):
 *   f = sum_{(i,j) in I} (r_ij - u_i^T m_j)^2
 *       + lambda (sum_i n_ui ||u_i||^2 + sum_j n_mj ||m_j||^2).
 * Only the user-major CSR is used; n_mj is counted from its column ids.
 */
double orc_loss(int64_t n_u, int64_t n_m, const int64_t *indptr, const int32_t *indices,
                const double *vals, const double *U, const double *M, int n_f, double lambda)
{
    double *part = (double *)malloc(sizeof(double) * (size_t)(n_u > 0 ? n_u : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_u; ++i) {
        const double *u = U + i * n_f;
        double s = 0.0;
        for (int64_t t = indptr[i]; t < indptr[i + 1]; ++t) {
            double e = vals[t] - dot(u, M + (int64_t)indices[t] * n_f, n_f);
            s += e * e;
        }
        part[i] = s + lambda * (double)(indptr[i + 1] - indptr[i]) * dot(u, u, n_f);
    }
    double f = 0.0;
    for (int64_t i = 0; i < n_u; ++i) f += part[i];
    int64_t *cm = column_counts(indptr[n_u], indices, n_m);
    double rm = 0.0;
    for (int64_t j = 0; j < n_m; ++j) {
        const double *m = M + j * n_f;
        rm += (double)cm[j] * dot(m, m, n_f);
    }
    free(cm);
    free(part);
    return f + lambda * rm;
}

/*
 * Gradient of Eq. (1) (Section III-A, and the form used in Section V-C):
 *   g_ui = 2 lambda n_ui u_i + 2 sum_{j in I_i} m_j (u_i^T m_j - r_ij)
 *   g_mj = 2 lambda n_mj m_j + 2 sum_{i in I_j} u_i (u_i^T m_j - r_ij)
 * The U block walks the CSR of R, the M block the CSR of R^T.
 */
void orc_gradient(int64_t n_u, const int64_t *indptr, const int32_t *indices, const double *vals,
                  int64_t n_m, const int64_t *indptr_t, const int32_t *indices_t,
                  const double *vals_t, const double *U, const double *M, int n_f,
                  double lambda, double *gU, double *gM)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_u; ++i) {
        const double *u = U + i * n_f;
        double *g = gU + i * n_f;
        double reg = 2.0 * lambda * (double)(indptr[i + 1] - indptr[i]);
        for (int k = 0; k < n_f; ++k) g[k] = reg * u[k];
        for (int64_t t = indptr[i]; t < indptr[i + 1]; ++t) {
            const double *m = M + (int64_t)indices[t] * n_f;
            double e = dot(u, m, n_f) - vals[t];
            for (int k = 0; k < n_f; ++k) g[k] += 2.0 * e * m[k];
        }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < n_m; ++j) {
        const double *m = M + j * n_f;
        double *g = gM + j * n_f;
        double reg = 2.0 * lambda * (double)(indptr_t[j + 1] - indptr_t[j]);
        for (int k = 0; k < n_f; ++k) g[k] = reg * m[k];
        for (int64_t t = indptr_t[j]; t < indptr_t[j + 1]; ++t) {
            const double *u = U + (int64_t)indices_t[t] * n_f;
            double e = dot(u, m, n_f) - vals_t[t];
            for (int k = 0; k < n_f; ++k) g[k] += 2.0 * e * u[k];
        }
    }
}

/*
 * Coefficients of the quartic Q(alpha) = f(x + alpha p) (Section V-C, line
 * search): f is expanded with u_i = xu_i + alpha pu_i and m_j = xm_j + alpha pm_j.
 * Per rating, with a0 = xu.xm, a1 = xu.pm + pu.xm, a2 = pu.pm and d = r - a0,
 *   (r - u.m)^2 = d^2 - 2 d a1 alpha + (a1^2 - 2 d a2) alpha^2
 *                 + 2 a1 a2 alpha^3 + a2^2 alpha^4,
 * and every regulariser term n ||x + alpha p||^2 contributes
 *   n (||x||^2 + 2 x.p alpha + ||p||^2 alpha^2).
 * C[n] is the coefficient of alpha^n.  Uses the user-major CSR only.
 */
void orc_quartic(int64_t n_u, int64_t n_m, const int64_t *indptr, const int32_t *indices,
                 const double *vals, const double *XU, const double *XM, const double *PU,
                 const double *PM, int n_f, double lambda, double *C)
{
    double *part = (double *)malloc(sizeof(double) * 5 * (size_t)(n_u > 0 ? n_u : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_u; ++i) {
        const double *xu = XU + i * n_f, *pu = PU + i * n_f;
        double c[5] = {0, 0, 0, 0, 0};
        for (int64_t t = indptr[i]; t < indptr[i + 1]; ++t) {
            const double *xm = XM + (int64_t)indices[t] * n_f;
            const double *pm = PM + (int64_t)indices[t] * n_f;
            double a0 = dot(xu, xm, n_f);
            double a1 = dot(xu, pm, n_f) + dot(pu, xm, n_f);
            double a2 = dot(pu, pm, n_f);
            double d = vals[t] - a0;
            c[0] += d * d;
            c[1] += -2.0 * d * a1;
            c[2] += a1 * a1 - 2.0 * d * a2;
            c[3] += 2.0 * a1 * a2;
            c[4] += a2 * a2;
        }
        double n = (double)(indptr[i + 1] - indptr[i]);
        c[0] += lambda * n * dot(xu, xu, n_f);
        c[1] += 2.0 * lambda * n * dot(xu, pu, n_f);
        c[2] += lambda * n * dot(pu, pu, n_f);
        for (int k = 0; k < 5; ++k) part[5 * i + k] = c[k];
    }
    for (int k = 0; k < 5; ++k) C[k] = 0.0;
    for (int64_t i = 0; i < n_u; ++i)
        for (int k = 0; k < 5; ++k) C[k] += part[5 * i + k];
    int64_t *cm = column_counts(indptr[n_u], indices, n_m);
    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
    for (int64_t j = 0; j < n_m; ++j) {
        const double *xm = XM + j * n_f, *pm = PM + j * n_f;
        double n = (double)cm[j];
        r0 += n * dot(xm, xm, n_f);
        r1 += n * dot(xm, pm, n_f);
        r2 += n * dot(pm, pm, n_f);
    }
    C[0] += lambda * r0;
    C[1] += 2.0 * lambda * r1;
    C[2] += lambda * r2;
    free(cm);
    free(part);
}
