/*
 * CPU oracle for the Hierarchical SUMMA local update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the GPU path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no BLAS; -ffp-contract=off so that every a*b and every + is one IEEE
 * binary64 rounding, in the order written here).
 *
 * What it computes (all double precision, row-major with leading dims):
 *
 *   oracle_gemm       the plain definition of the result that SUMMA and
 *                     HSUMMA reach after all n/b steps (Sec. II-A and
 *                     Sec. III: c_ij = sum over k of a_ik * b_kj), summed
 *                     in increasing k, one rounding per multiply and per add.
 *                     With accumulate != 0 it adds into C (the local update
 *                     c_ij = c_ij + a_ik * b_kj of one step, Sec. II-A).
 *   oracle_dot2       compensated dot product (Ogita, Rump, Oishi, "Accurate
 *                     sum and dot product", SIAM J. Sci. Comput. 26(6), 2005,
 *                     Algorithm Dot2): result as if computed in twice the
 *                     working precision, then rounded.  Also returns
 *                     s = sum |a_ik| |b_kj| (the scale of the error bounds).
 *   oracle_sampled    oracle_dot2 for a list of (i, j) entries of A*B.
 *   oracle_matvec2    y = M x with every row done by Dot2 (for Freivalds'
 *                     check), plus |M| |x|.
 *
 * Parity status: oracle_gemm is pinned against exact rational brute force
 * (bit-exact after rounding, tests/test_oracle.py); oracle_dot2 against the
 * same brute force and against hand-made cancellation cases.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* C[m x n] (+)= A[m x k] * B[k x n]; loop order i, kk, j so that each c_ij
 * receives its k products strictly in increasing kk, starting from 0 (or
 * from the loaded value when accumulating). */
void oracle_gemm(int64_t m, int64_t n, int64_t k,
                 const double *A, int64_t lda,
                 const double *B, int64_t ldb,
                 double *C, int64_t ldc, int accumulate)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        double *c = C + i * ldc;
        if (!accumulate)
            for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t kk = 0; kk < k; ++kk) {
            const double aik = A[i * lda + kk];
            const double *b = B + kk * ldb;
            for (int64_t j = 0; j < n; ++j) {
                double prod = aik * b[j];
                c[j] = c[j] + prod;
            }
        }
    }
}

/* Error-free transformations (Knuth TwoSum; TwoProduct by fused multiply-add). */
static inline void two_sum(double a, double b, double *x, double *y)
{
    double s = a + b;
    double z = s - a;
    *x = s;
    *y = (a - (s - z)) + (b - z);
}

static inline void two_prod(double a, double b, double *x, double *y)
{
    double p = a * b;
    *x = p;
    *y = fma(a, b, -p);
}

/* Dot2 over x[0..len) with stride incx and y[0..len) with stride incy.
 * Returns the compensated result; *abs_sum = sum |x_i| |y_i| (plain sum,
 * only used as a scale, so its own rounding is irrelevant). */
double oracle_dot2(int64_t len, const double *x, int64_t incx,
                   const double *y, int64_t incy, double *abs_sum)
{
    double p = 0.0, s = 0.0, as = 0.0;
    for (int64_t t = 0; t < len; ++t) {
        double xv = x[t * incx], yv = y[t * incy];
        double h, r, q;
        two_prod(xv, yv, &h, &r);
        two_sum(p, h, &p, &q);
        s = s + (q + r);
        as = as + fabs(xv) * fabs(yv);
    }
    if (abs_sum) *abs_sum = as;
    return p + s;
}

/* Entries (rows[t], cols[t]) of A*B by Dot2, and their scales. */
void oracle_sampled(int64_t k, const double *A, int64_t lda,
                    const double *B, int64_t ldb,
                    int64_t count, const int64_t *rows, const int64_t *cols,
                    double *out_c, double *out_s)
{
    int64_t t;
#pragma omp parallel for schedule(dynamic, 16)
    for (t = 0; t < count; ++t) {
        double s;
        out_c[t] = oracle_dot2(k, A + rows[t] * lda, 1, B + cols[t], ldb, &s);
        out_s[t] = s;
    }
}

/* y = M x (M is r x c, row-major, ld), each row by Dot2; sy = |M| |x|. */
void oracle_matvec2(int64_t r, int64_t c, const double *Mtx, int64_t ld,
                    const double *x, double *y, double *sy)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < r; ++i) {
        double s;
        y[i] = oracle_dot2(c, Mtx + i * ld, 1, x, 1, &s);
        sy[i] = s;
    }
}

/* Number of OpenMP threads the oracle runs with (reported beside timings). */
int oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
