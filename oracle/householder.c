/*
 * Plain FP64 Householder QR -- the oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct CPU
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header or constant with the HIP library and includes nothing from it.
 *
 * What it computes (Buttari, Langou, Kurzak, Dongarra, "Parallel Tiled QR
 * Factorization for Multicore Architectures", Sec. 2.1): A = QR by
 * min(m,n) Householder reflections applied one column at a time -- the
 * unblocked, level-2 panel algorithm that the paper calls DGEQR2.  The tiled
 * algorithm of Sec. 3 reaches the same factorization through a different
 * sequence of orthogonal transformations, so for full column rank the
 * sign-normalised R of both must agree.
 *
 * Conventions (all column-major, 0-based indices, leading dimensions >= rows):
 *   reflector j:  H_j = I - tau_j v_j v_j^T,  v_j = [0..0, 1, A[j+1:m, j]]
 *   beta = -sgn(alpha) * sqrt(alpha^2 + sigma^2), sgn(0) = +1
 *   sigma^2 == 0  ->  tau_j = 0, H_j = I, column left as it is (even if
 *                     alpha < 0), so an upper-triangular input is returned
 *                     unchanged.
 *   Q = H_0 H_1 ... H_{k-1},  Q^T A = R.
 * No scaling is applied before the square root: the inputs this oracle sees
 * (entries of order 1e-8 .. 1e2) are far from FP64 overflow and underflow.
 *
 * Built twice from this one source: once plain (-O2, single thread) and once
 * with OpenMP, where the trailing-column loop of the update runs across all
 * host cores -- the fork-join style of Sec. 2.2.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Householder QR in place.  On exit the upper triangle of the leading
 * min(m,n) rows holds R, the strict lower part holds the reflector tails
 * (the unit leading entry is implicit) and tau[0:min(m,n)] the scalars.
 * Returns 0, or -1 for an illegal argument. */
int orc_geqr2(int64_t m, int64_t n, double *A, int64_t lda, double *tau)
{
    if (m < 0 || n < 0 || lda < (m > 1 ? m : 1))
        return -1;
    int64_t kmax = m < n ? m : n;
    for (int64_t j = 0; j < kmax; ++j) {
        double *colj = A + j * lda;
        double alpha = colj[j];
        double sigma2 = 0.0;
        for (int64_t i = j + 1; i < m; ++i)
            sigma2 += colj[i] * colj[i];
        if (sigma2 == 0.0) {
            tau[j] = 0.0;
            continue;
        }
        double norm = sqrt(alpha * alpha + sigma2);
        double beta = (alpha >= 0.0) ? -norm : norm;
        double t = (beta - alpha) / beta;
        double denom = alpha - beta;
        for (int64_t i = j + 1; i < m; ++i)
            colj[i] = colj[i] / denom;
        colj[j] = beta;
        tau[j] = t;
        /* apply H_j to the trailing columns: w = v^T A[j:m,c]; A[j:m,c] -= tau v w */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t c = j + 1; c < n; ++c) {
            double *colc = A + c * lda;
            double w = colc[j];
            for (int64_t i = j + 1; i < m; ++i)
                w += colj[i] * colc[i];
            w *= t;
            colc[j] -= w;
            for (int64_t i = j + 1; i < m; ++i)
                colc[i] -= w * colj[i];
        }
    }
    return 0;
}

/* B <- Q^T B with Q from orc_geqr2 (H_0 applied first).  B is m x nrhs. */
int orc_apply_qt(int64_t m, int64_t n, const double *A, int64_t lda,
                 const double *tau, int64_t nrhs, double *B, int64_t ldb)
{
    if (m < 0 || n < 0 || nrhs < 0 || lda < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1))
        return -1;
    int64_t kmax = m < n ? m : n;
    for (int64_t j = 0; j < kmax; ++j) {
        const double *v = A + j * lda;
        double t = tau[j];
        if (t == 0.0)
            continue;
        for (int64_t c = 0; c < nrhs; ++c) {
            double *b = B + c * ldb;
            double w = b[j];
            for (int64_t i = j + 1; i < m; ++i)
                w += v[i] * b[i];
            w *= t;
            b[j] -= w;
            for (int64_t i = j + 1; i < m; ++i)
                b[i] -= w * v[i];
        }
    }
    return 0;
}

/* B <- Q B (H_{k-1} applied first). */
int orc_apply_q(int64_t m, int64_t n, const double *A, int64_t lda,
                const double *tau, int64_t nrhs, double *B, int64_t ldb)
{
    if (m < 0 || n < 0 || nrhs < 0 || lda < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1))
        return -1;
    int64_t kmax = m < n ? m : n;
    for (int64_t j = kmax - 1; j >= 0; --j) {
        const double *v = A + j * lda;
        double t = tau[j];
        if (t == 0.0)
            continue;
        for (int64_t c = 0; c < nrhs; ++c) {
            double *b = B + c * ldb;
            double w = b[j];
            for (int64_t i = j + 1; i < m; ++i)
                w += v[i] * b[i];
            w *= t;
            b[j] -= w;
            for (int64_t i = j + 1; i < m; ++i)
                b[i] -= w * v[i];
        }
    }
    return 0;
}

/* Thin Q (m x min(m,n)) = H_0 ... H_{k-1} [I; 0]. */
int orc_form_q(int64_t m, int64_t n, const double *A, int64_t lda,
               const double *tau, double *Q, int64_t ldq)
{
    if (m < 0 || n < 0 || ldq < (m > 1 ? m : 1))
        return -1;
    int64_t kmax = m < n ? m : n;
    for (int64_t c = 0; c < kmax; ++c) {
        memset(Q + c * ldq, 0, (size_t)m * sizeof(double));
        Q[c * ldq + c] = 1.0;
    }
    return orc_apply_q(m, n, A, lda, tau, kmax, Q, ldq);
}

/* Back substitution X <- R^{-1} X for the n x n upper triangle of R.
 * Returns 0, the 1-based index of the first exactly-zero diagonal entry
 * (nothing is written then), or -1 for an illegal argument. */
int orc_trsv_upper(int64_t n, const double *R, int64_t ldr, int64_t nrhs,
                   double *X, int64_t ldx)
{
    if (n < 0 || nrhs < 0 || ldr < (n > 1 ? n : 1) || ldx < (n > 1 ? n : 1))
        return -1;
    for (int64_t i = 0; i < n; ++i)
        if (R[i * ldr + i] == 0.0)
            return (int)(i + 1);
    for (int64_t c = 0; c < nrhs; ++c) {
        double *x = X + c * ldx;
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int64_t j = i + 1; j < n; ++j)
                s -= R[j * ldr + i] * x[j];
            x[i] = s / R[i * ldr + i];
        }
    }
    return 0;
}
