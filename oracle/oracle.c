/*
 * oracle.c -- plain CPU oracle for mixed-precision iterative refinement.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * used by the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark.  The GPU library never links, loads or calls it, and it shares
 * no code with the GPU library.
 *
 * Paper: Baboulin, Buttari, Dongarra, Kurzak, Langou, Langou, Luszczek,
 * Tomov, "Accelerating Scientific Computations with Mixed Precision
 * Algorithms" (arXiv:0808.2794).
 *
 * Everything here is the textbook algorithm, unblocked and unfused, so that
 * it can be checked by eye against the paper:
 *   - Gaussian elimination with partial row pivoting, PA = LU, then
 *     Ly = Pb and Ux = y (Section 2.1, "Direct Methods").
 *   - Iterative refinement, Algorithm 1 (Section 2.1): factor and solve in
 *     the working precision eps_s, residual r = b - A x and update x += z in
 *     eps_d, using the original double-precision A.  The fixed-precision
 *     variant (eps_s = eps_d, the double/double refinement the paper cites
 *     to Wilkinson, Moler and Stewart) is the reference solver; the
 *     FP32/FP64 variant is Algorithm 1 exactly as printed.
 *   - The Cholesky variant (SPOTRF/SPOTRS + DSYMM residual, Section 3.1.1).
 *   - The stopping test of Section 3: ||b - A x|| <= ||x|| ||A|| eps sqrt(n),
 *     taken in the infinity norm with eps = 2^-53 (see the readings listed
 *     with the design notes: the 2-norm of the paper is not computable in
 *     O(n^2)).  The test is made at the top of each iteration on the
 *     residual of the current x, so the returned x is the one certified.
 *   - 30 iterations means failure (Section 4, "Numerical Remarks").
 *
 * Storage: all matrices are row-major; element (i, j) of a matrix with
 * leading dimension ld is M[i*ld + j].  Right-hand sides and solutions are
 * n x nrhs row-major (column c of B is B[i*ldb + c]).  Pivots are a 0-based
 * LAPACK-style swap sequence: at step k rows k and ipiv[k] were exchanged.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EPS_D 0x1p-53 /* unit roundoff of IEEE double */

/* ---------------------------------------------------------------- norms */

/* ||A||_inf = max_i sum_j |a_ij|  (the DLANGE quantity of Table 7). */
double orc_norm_inf(int n, const double *A, int lda)
{
    double best = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            s += fabs(A[(size_t)i * lda + j]);
        if (s > best || isnan(s))
            best = s;
    }
    return best;
}

/* ---------------------------------------------- LU with partial pivoting */

/*
 * Unblocked right-looking Gaussian elimination with partial row pivoting on
 * the first `steps` columns (steps = n for a full factorization).  At step k
 * the pivot is the entry of largest magnitude in column k on or below the
 * diagonal; on ties the smallest row index wins.  Whole rows are exchanged,
 * so on return PA = LU with the unit lower L stored below the diagonal and U
 * on and above it.  Returns 0, or k+1 if the pivot of step k is exactly zero
 * (the factorization stops there; A is singular).
 */
int orc_dgetrf_steps(int n, double *A, int lda, int *ipiv, int steps)
{
    if (steps > n)
        steps = n;
    for (int k = 0; k < steps; ++k) {
        int p = k;
        double best = fabs(A[(size_t)k * lda + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(A[(size_t)i * lda + k]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        ipiv[k] = p;
        if (A[(size_t)p * lda + k] == 0.0)
            return k + 1;
        if (p != k) {
            double *rk = A + (size_t)k * lda, *rp = A + (size_t)p * lda;
            for (int j = 0; j < n; ++j) {
                double t = rk[j];
                rk[j] = rp[j];
                rp[j] = t;
            }
        }
        const double *rowk = A + (size_t)k * lda;
        const double piv = rowk[k];
#pragma omp parallel for schedule(static) if ((n - k) > 256)
        for (int i = k + 1; i < n; ++i) {
            double *ri = A + (size_t)i * lda;
            double l = ri[k] / piv;
            ri[k] = l;
            for (int j = k + 1; j < n; ++j)
                ri[j] -= l * rowk[j];
        }
    }
    return 0;
}

int orc_dgetrf(int n, double *A, int lda, int *ipiv)
{
    return orc_dgetrf_steps(n, A, lda, ipiv, n);
}

/* Same elimination carried out entirely in single precision (Algorithm 1,
   step 1, in eps_s).  */
int orc_sgetrf(int n, float *A, int lda, int *ipiv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        float best = fabsf(A[(size_t)k * lda + k]);
        for (int i = k + 1; i < n; ++i) {
            float v = fabsf(A[(size_t)i * lda + k]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        ipiv[k] = p;
        if (A[(size_t)p * lda + k] == 0.0f)
            return k + 1;
        if (p != k) {
            float *rk = A + (size_t)k * lda, *rp = A + (size_t)p * lda;
            for (int j = 0; j < n; ++j) {
                float t = rk[j];
                rk[j] = rp[j];
                rp[j] = t;
            }
        }
        const float *rowk = A + (size_t)k * lda;
        const float piv = rowk[k];
#pragma omp parallel for schedule(static) if ((n - k) > 256)
        for (int i = k + 1; i < n; ++i) {
            float *ri = A + (size_t)i * lda;
            float l = ri[k] / piv;
            ri[k] = l;
            for (int j = k + 1; j < n; ++j)
                ri[j] = ri[j] - l * rowk[j];
        }
    }
    return 0;
}

/*
 * Solve A X = B (trans = 0) or A^T X = B (trans = 1) in place in B with the
 * factors of orc_dgetrf.  trans = 0: apply the swaps to B (P B), forward
 * substitution with the unit lower L, back substitution with U.
 * trans = 1: since PA = LU, A^T = U^T L^T P, so solve U^T y = b (forward),
 * L^T v = y (backward), then x = P^T v (swaps applied in reverse order).
 */
void orc_dgetrs(int n, int nrhs, const double *LU, int lda, const int *ipiv,
                double *B, int ldb, int trans)
{
    if (!trans) {
        for (int k = 0; k < n; ++k) {
            int p = ipiv[k];
            if (p != k)
                for (int c = 0; c < nrhs; ++c) {
                    double t = B[(size_t)k * ldb + c];
                    B[(size_t)k * ldb + c] = B[(size_t)p * ldb + c];
                    B[(size_t)p * ldb + c] = t;
                }
        }
        for (int c = 0; c < nrhs; ++c) {
            for (int i = 0; i < n; ++i) {
                double s = B[(size_t)i * ldb + c];
                for (int j = 0; j < i; ++j)
                    s -= LU[(size_t)i * lda + j] * B[(size_t)j * ldb + c];
                B[(size_t)i * ldb + c] = s;
            }
            for (int i = n - 1; i >= 0; --i) {
                double s = B[(size_t)i * ldb + c];
                for (int j = i + 1; j < n; ++j)
                    s -= LU[(size_t)i * lda + j] * B[(size_t)j * ldb + c];
                B[(size_t)i * ldb + c] = s / LU[(size_t)i * lda + i];
            }
        }
    } else {
        for (int c = 0; c < nrhs; ++c) {
            /* U^T y = b: row i of U^T is column i of U. */
            for (int i = 0; i < n; ++i) {
                double s = B[(size_t)i * ldb + c];
                for (int j = 0; j < i; ++j)
                    s -= LU[(size_t)j * lda + i] * B[(size_t)j * ldb + c];
                B[(size_t)i * ldb + c] = s / LU[(size_t)i * lda + i];
            }
            /* L^T v = y, unit diagonal. */
            for (int i = n - 1; i >= 0; --i) {
                double s = B[(size_t)i * ldb + c];
                for (int j = i + 1; j < n; ++j)
                    s -= LU[(size_t)j * lda + i] * B[(size_t)j * ldb + c];
                B[(size_t)i * ldb + c] = s;
            }
        }
        for (int k = n - 1; k >= 0; --k) {
            int p = ipiv[k];
            if (p != k)
                for (int c = 0; c < nrhs; ++c) {
                    double t = B[(size_t)k * ldb + c];
                    B[(size_t)k * ldb + c] = B[(size_t)p * ldb + c];
                    B[(size_t)p * ldb + c] = t;
                }
        }
    }
}

/* Single-precision solve with single-precision factors (Algorithm 1,
   steps 2-3 and 5-6), no transposition. */
void orc_sgetrs(int n, int nrhs, const float *LU, int lda, const int *ipiv,
                float *B, int ldb)
{
    for (int k = 0; k < n; ++k) {
        int p = ipiv[k];
        if (p != k)
            for (int c = 0; c < nrhs; ++c) {
                float t = B[(size_t)k * ldb + c];
                B[(size_t)k * ldb + c] = B[(size_t)p * ldb + c];
                B[(size_t)p * ldb + c] = t;
            }
    }
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < n; ++i) {
            float s = B[(size_t)i * ldb + c];
            for (int j = 0; j < i; ++j)
                s = s - LU[(size_t)i * lda + j] * B[(size_t)j * ldb + c];
            B[(size_t)i * ldb + c] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            float s = B[(size_t)i * ldb + c];
            for (int j = i + 1; j < n; ++j)
                s = s - LU[(size_t)i * lda + j] * B[(size_t)j * ldb + c];
            B[(size_t)i * ldb + c] = s / LU[(size_t)i * lda + i];
        }
    }
}

/* ------------------------------------------------------------- Cholesky */

/*
 * A = L L^T for symmetric positive definite A (the SPOTRF/DPOTRF step of the
 * symmetric variant, Section 3.1.1), reading only the lower triangle and
 * writing L there.  Column by column:
 *   l_jj = sqrt(a_jj - sum_{k<j} l_jk^2),
 *   l_ij = (a_ij - sum_{k<j} l_ik l_jk) / l_jj   for i > j.
 * Returns 0, or j+1 if the quantity under the square root is not positive.
 */
int orc_dpotrf(int n, double *A, int lda)
{
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * lda + j];
        for (int k = 0; k < j; ++k)
            d -= A[(size_t)j * lda + k] * A[(size_t)j * lda + k];
        if (!(d > 0.0))
            return j + 1;
        double ljj = sqrt(d);
        A[(size_t)j * lda + j] = ljj;
#pragma omp parallel for schedule(static) if ((n - j) > 256)
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * lda + j];
            for (int k = 0; k < j; ++k)
                s -= A[(size_t)i * lda + k] * A[(size_t)j * lda + k];
            A[(size_t)i * lda + j] = s / ljj;
        }
    }
    return 0;
}

int orc_spotrf(int n, float *A, int lda)
{
    for (int j = 0; j < n; ++j) {
        float d = A[(size_t)j * lda + j];
        for (int k = 0; k < j; ++k)
            d = d - A[(size_t)j * lda + k] * A[(size_t)j * lda + k];
        if (!(d > 0.0f))
            return j + 1;
        float ljj = sqrtf(d);
        A[(size_t)j * lda + j] = ljj;
#pragma omp parallel for schedule(static) if ((n - j) > 256)
        for (int i = j + 1; i < n; ++i) {
            float s = A[(size_t)i * lda + j];
            for (int k = 0; k < j; ++k)
                s = s - A[(size_t)i * lda + k] * A[(size_t)j * lda + k];
            A[(size_t)i * lda + j] = s / ljj;
        }
    }
    return 0;
}

/* Solve L L^T X = B in place: L y = b, then L^T x = y. */
void orc_dpotrs(int n, int nrhs, const double *L, int lda, double *B, int ldb)
{
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = B[(size_t)i * ldb + c];
            for (int k = 0; k < i; ++k)
                s -= L[(size_t)i * lda + k] * B[(size_t)k * ldb + c];
            B[(size_t)i * ldb + c] = s / L[(size_t)i * lda + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = B[(size_t)i * ldb + c];
            for (int k = i + 1; k < n; ++k)
                s -= L[(size_t)k * lda + i] * B[(size_t)k * ldb + c];
            B[(size_t)i * ldb + c] = s / L[(size_t)i * lda + i];
        }
    }
}

void orc_spotrs(int n, int nrhs, const float *L, int lda, float *B, int ldb)
{
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < n; ++i) {
            float s = B[(size_t)i * ldb + c];
            for (int k = 0; k < i; ++k)
                s = s - L[(size_t)i * lda + k] * B[(size_t)k * ldb + c];
            B[(size_t)i * ldb + c] = s / L[(size_t)i * lda + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            float s = B[(size_t)i * ldb + c];
            for (int k = i + 1; k < n; ++k)
                s = s - L[(size_t)k * lda + i] * B[(size_t)k * ldb + c];
            B[(size_t)i * ldb + c] = s / L[(size_t)i * lda + i];
        }
    }
}

/* ------------------------------------------------------------ residuals */

/*
 * R = B - op(A) X in double precision (Algorithm 1, step 4), plain
 * sequential dot products.  op(A) = A (trans = 0) or A^T (trans = 1).
 */
void orc_residual(int n, int nrhs, const double *A, int lda, const double *X,
                  int ldx, const double *B, int ldb, double *R, int ldr,
                  int trans)
{
#pragma omp parallel for schedule(static) if (n > 256)
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < nrhs; ++c) {
            double s = B[(size_t)i * ldb + c];
            for (int j = 0; j < n; ++j) {
                double a = trans ? A[(size_t)j * lda + i] : A[(size_t)i * lda + j];
                s -= a * X[(size_t)j * ldx + c];
            }
            R[(size_t)i * ldr + c] = s;
        }
}

/*
 * Extended-precision residual for checking results: for each column c,
 * rnorm[c] = ||b - A x||_inf and, per row, the componentwise denominator
 * (|A||x| + |b|)_i, all accumulated in long double (x86 80-bit, 64-bit
 * significand), then rounded to double.  comp[c] receives
 * max_i |r_i| / (|A||x| + |b|)_i (Oettli-Prager componentwise backward
 * error, cited in Section 2.1); 0/0 counts as 0.
 */
void orc_residual_ld(int n, int nrhs, const double *A, int lda, const double *X,
                     int ldx, const double *B, int ldb, double *rnorm,
                     double *comp)
{
    for (int c = 0; c < nrhs; ++c) {
        long double rmax = 0.0L, cmax = 0.0L;
        for (int i = 0; i < n; ++i) {
            long double s = (long double)B[(size_t)i * ldb + c];
            long double d = fabsl(s);
            for (int j = 0; j < n; ++j) {
                long double t = (long double)A[(size_t)i * lda + j] *
                                (long double)X[(size_t)j * ldx + c];
                s -= t;
                d += fabsl(t);
            }
            long double a = fabsl(s);
            if (a > rmax || isnan((double)a))
                rmax = a;
            long double q = (d > 0.0L) ? a / d : (a > 0.0L ? INFINITY : 0.0L);
            if (q > cmax || isnan((double)q))
                cmax = q;
        }
        rnorm[c] = (double)rmax;
        comp[c] = (double)cmax;
    }
}

/* ------------------------------------------------- stopping rule helper */

/* Column c passes when ||r||_inf <= sqrt(n) * eps_d * ||A||_inf * ||x||_inf
   (Section 3, infinity-norm reading). */
static int orc_converged(int n, int nrhs, const double *R, int ldr,
                         const double *X, int ldx, double anorm)
{
    const double thr = sqrt((double)n) * ORC_EPS_D * anorm;
    for (int c = 0; c < nrhs; ++c) {
        double rn = 0.0, xn = 0.0;
        for (int i = 0; i < n; ++i) {
            double r = fabs(R[(size_t)i * ldr + c]);
            double x = fabs(X[(size_t)i * ldx + c]);
            if (r > rn || isnan(r))
                rn = r;
            if (x > xn || isnan(x))
                xn = x;
        }
        if (!(rn <= thr * xn))
            return 0;
    }
    return 1;
}

/* ----------------------------------------------- refinement drivers */

/*
 * Iterative refinement with the structure of Algorithm 1.
 *   lowp = 0: factor and correction solves in double (fixed precision
 *             refinement: the reference solver of the test-suite);
 *   lowp = 1: factor and correction solves in single precision, residual
 *             and update in double: Algorithm 1 with eps_s = FP32.
 *   trans = 1 solves A^T X = B (lowp = 0 only).
 * On entry X is ignored; on return X holds the solution and *iters the
 * number of corrections applied (x_0 counts as zero), or -(itermax+1) if the
 * stopping rule was never met, or -1 if the factorization found a zero pivot.
 * The return value is the factorization info (0 on success).
 */
int orc_gesv_ir(int n, int nrhs, const double *A, int lda, const double *B,
                int ldb, double *X, int ldx, int itermax, int lowp, int trans,
                int *iters)
{
    const double anorm = orc_norm_inf(n, A, lda);
    int *ipiv = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double *R = (double *)malloc(sizeof(double) * (size_t)n * nrhs + 1);
    int info;
    *iters = 0;
    if (n == 0) {
        free(ipiv);
        free(R);
        return 0;
    }
    if (!lowp) {
        double *F = (double *)malloc(sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; ++i)
            memcpy(F + (size_t)i * n, A + (size_t)i * lda, sizeof(double) * n);
        info = orc_dgetrf(n, F, n, ipiv);
        if (info) {
            *iters = -1;
            free(F); free(ipiv); free(R);
            return info;
        }
        /* x_0 (steps 2-3) */
        {
            double *T = (double *)malloc(sizeof(double) * (size_t)n * nrhs);
            for (int i = 0; i < n; ++i)
                for (int c = 0; c < nrhs; ++c)
                    T[(size_t)i * nrhs + c] = B[(size_t)i * ldb + c];
            orc_dgetrs(n, nrhs, F, n, ipiv, T, nrhs, trans);
            for (int i = 0; i < n; ++i)
                for (int c = 0; c < nrhs; ++c)
                    X[(size_t)i * ldx + c] = T[(size_t)i * nrhs + c];
            free(T);
        }
        int k = 0;
        for (;;) {
            orc_residual(n, nrhs, A, lda, X, ldx, B, ldb, R, nrhs, trans); /* step 4 */
            if (orc_converged(n, nrhs, R, nrhs, X, ldx, anorm))
                break;
            if (k == itermax) {
                k = -(itermax + 1);
                break;
            }
            orc_dgetrs(n, nrhs, F, n, ipiv, R, nrhs, trans); /* steps 5-6 */
            for (int i = 0; i < n; ++i)                     /* step 7 */
                for (int c = 0; c < nrhs; ++c)
                    X[(size_t)i * ldx + c] += R[(size_t)i * nrhs + c];
            ++k;
        }
        *iters = k;
        free(F);
    } else {
        float *F = (float *)malloc(sizeof(float) * (size_t)n * n);
        float *Z = (float *)malloc(sizeof(float) * (size_t)n * nrhs);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                F[(size_t)i * n + j] = (float)A[(size_t)i * lda + j];
        info = orc_sgetrf(n, F, n, ipiv); /* step 1 */
        if (info) {
            *iters = -1;
            free(F); free(Z); free(ipiv); free(R);
            return info;
        }
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < nrhs; ++c)
                Z[(size_t)i * nrhs + c] = (float)B[(size_t)i * ldb + c];
        orc_sgetrs(n, nrhs, F, n, ipiv, Z, nrhs); /* steps 2-3 */
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < nrhs; ++c)
                X[(size_t)i * ldx + c] = (double)Z[(size_t)i * nrhs + c];
        int k = 0;
        for (;;) {
            orc_residual(n, nrhs, A, lda, X, ldx, B, ldb, R, nrhs, 0); /* step 4 */
            if (orc_converged(n, nrhs, R, nrhs, X, ldx, anorm))
                break;
            if (k == itermax) {
                k = -(itermax + 1);
                break;
            }
            for (int i = 0; i < n; ++i)
                for (int c = 0; c < nrhs; ++c)
                    Z[(size_t)i * nrhs + c] = (float)R[(size_t)i * nrhs + c];
            orc_sgetrs(n, nrhs, F, n, ipiv, Z, nrhs); /* steps 5-6 */
            for (int i = 0; i < n; ++i)                /* step 7 */
                for (int c = 0; c < nrhs; ++c)
                    X[(size_t)i * ldx + c] += (double)Z[(size_t)i * nrhs + c];
            ++k;
        }
        *iters = k;
        free(F);
        free(Z);
    }
    free(ipiv);
    free(R);
    return 0;
}

/*
 * Symmetric positive definite variant (Section 3.1.1: SPOTRF, SPOTRS and a
 * DSYMM residual with the full stored symmetric A).  lowp as above.
 * Returns the Cholesky info; *iters as in orc_gesv_ir.
 */
int orc_posv_ir(int n, int nrhs, const double *A, int lda, const double *B,
                int ldb, double *X, int ldx, int itermax, int lowp, int *iters)
{
    const double anorm = orc_norm_inf(n, A, lda);
    double *R = (double *)malloc(sizeof(double) * (size_t)n * nrhs + 1);
    int info, k = 0;
    *iters = 0;
    if (n == 0) {
        free(R);
        return 0;
    }
    if (!lowp) {
        double *F = (double *)malloc(sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; ++i)
            memcpy(F + (size_t)i * n, A + (size_t)i * lda, sizeof(double) * n);
        info = orc_dpotrf(n, F, n);
        if (info) {
            *iters = -1;
            free(F); free(R);
            return info;
        }
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < nrhs; ++c)
                R[(size_t)i * nrhs + c] = B[(size_t)i * ldb + c];
        orc_dpotrs(n, nrhs, F, n, R, nrhs);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < nrhs; ++c)
                X[(size_t)i * ldx + c] = R[(size_t)i * nrhs + c];
        for (;;) {
            orc_residual(n, nrhs, A, lda, X, ldx, B, ldb, R, nrhs, 0);
            if (orc_converged(n, nrhs, R, nrhs, X, ldx, anorm))
                break;
            if (k == itermax) {
                k = -(itermax + 1);
                break;
            }
            orc_dpotrs(n, nrhs, F, n, R, nrhs);
            for (int i = 0; i < n; ++i)
                for (int c = 0; c < nrhs; ++c)
                    X[(size_t)i * ldx + c] += R[(size_t)i * nrhs + c];
            ++k;
        }
        free(F);
    } else {
        float *F = (float *)malloc(sizeof(float) * (size_t)n * n);
        float *Z = (float *)malloc(sizeof(float) * (size_t)n * nrhs);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                F[(size_t)i * n + j] = (float)A[(size_t)i * lda + j];
        info = orc_spotrf(n, F, n);
        if (info) {
            *iters = -1;
            free(F); free(Z); free(R);
            return info;
        }
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < nrhs; ++c)
                Z[(size_t)i * nrhs + c] = (float)B[(size_t)i * ldb + c];
        orc_spotrs(n, nrhs, F, n, Z, nrhs);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < nrhs; ++c)
                X[(size_t)i * ldx + c] = (double)Z[(size_t)i * nrhs + c];
        for (;;) {
            orc_residual(n, nrhs, A, lda, X, ldx, B, ldb, R, nrhs, 0);
            if (orc_converged(n, nrhs, R, nrhs, X, ldx, anorm))
                break;
            if (k == itermax) {
                k = -(itermax + 1);
                break;
            }
            for (int i = 0; i < n; ++i)
                for (int c = 0; c < nrhs; ++c)
                    Z[(size_t)i * nrhs + c] = (float)R[(size_t)i * nrhs + c];
            orc_spotrs(n, nrhs, F, n, Z, nrhs);
            for (int i = 0; i < n; ++i)
                for (int c = 0; c < nrhs; ++c)
                    X[(size_t)i * ldx + c] += (double)Z[(size_t)i * nrhs + c];
            ++k;
        }
        free(F);
        free(Z);
    }
    *iters = k;
    free(R);
    return 0;
}
