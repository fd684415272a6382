/*
 * Band-bidiagonalization oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU library never links or calls it,
 * and the two share no code, headers or tables.
 *
 * What it computes (Section 3.4, the BiDiag sequence QR(1);LQ(1);...;QR(q),
 * written at element granularity): for an m x n matrix A with m >= n and a
 * bandwidth nb >= 1, orthogonal Q (m x m) and P (n x n) with
 *     B = Q^T A P,   B(i,j) = 0 unless 0 <= j - i <= nb,   rows >= n zero.
 * The tiled step QR(k) leaves tile column k upper triangular; in scalar form
 * that is a Householder QR of the columns k*nb .. k*nb+nb-1 over all rows at
 * or below the diagonal.  The tiled step LQ(k) leaves tile (k,k+1) lower
 * triangular and zeroes the rest of tile row k; in scalar form that is one
 * row Householder per row r of the block, acting on columns r+nb .. n-1.
 * With nb = 1 this is the classical Golub-Kahan Householder bidiagonalization
 * (Section 2, xGEBD2), whose cost is 4mn^2 - 4n^3/3.
 *
 * Reflector convention (the paper uses the PLASMA/LAPACK kernels and states no
 * other): for x = (alpha, x_tail),
 *     beta = -sign(alpha) * ||x||,  tau = (beta - alpha)/beta,
 *     v = (1, x_tail / (alpha - beta)),  H = I - tau v v^T,  H x = beta e_1,
 * with sign(0) = +1, and tau = 0 (H = I, beta = alpha) when x_tail == 0.
 *
 * Everything is plain FP64, unblocked, one dot and one axpy per column (or
 * row) touched.  OpenMP splits only the independent columns (rows) of one
 * reflector application; every output element is computed by one thread in a
 * fixed order, so results do not depend on the thread count.
 *
 * Storage of the reflectors (column-major, all caller-owned):
 *   VQ   m x n, ldvq >= m : column reflector c stored in VQ(c:m-1, c), VQ(c,c)=1,
 *                           zero above.          tauq[c] its tau.
 *   WP   n x n, ldwp >= n : row reflector r stored in WP(r, r+nb : n-1),
 *                           WP(r, r+nb) = 1, zero elsewhere in that row.
 *                           taup[r] its tau (0 when r+nb >= n-1).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define AT(M, ld, i, j) (M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)]

/* Householder generation for a vector x of length len with stride inc.
 * On return x[0] holds beta and x[1..] holds v[1..] (v[0] = 1 implicit).
 * Returns tau. */
static double make_reflector(double *x, int64_t len, int64_t inc) {
    double alpha = x[0];
    double ss = 0.0;
    for (int64_t t = 1; t < len; ++t) ss += x[t * inc] * x[t * inc];
    if (len <= 1 || ss == 0.0) return 0.0;
    double norm = hypot(alpha, sqrt(ss));
    double beta = (alpha >= 0.0) ? -norm : norm;
    double tau = (beta - alpha) / beta;
    double scale = 1.0 / (alpha - beta);
    for (int64_t t = 1; t < len; ++t) x[t * inc] *= scale;
    x[0] = beta;
    return tau;
}

/* Flop counter for the last call, for the cost pin at nb = 1. */
static double g_flops = 0.0;
double oracle_last_flops(void) { return g_flops; }

/*
 * Reduce A (m x n, column-major, lda >= m) in place to the band form B.
 * Returns 0 on success, -k when argument k is invalid.
 */
int oracle_band_reduce(int64_t m, int64_t n, int64_t nb, double *A, int64_t lda,
                       double *VQ, int64_t ldvq, double *tauq,
                       double *WP, int64_t ldwp, double *taup) {
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nb < 1) return -3;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (ldvq < (m > 1 ? m : 1)) return -7;
    if (ldwp < (n > 1 ? n : 1)) return -10;
    g_flops = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) AT(VQ, ldvq, i, j) = 0.0;
        for (int64_t i = 0; i < n; ++i) AT(WP, ldwp, i, j) = 0.0;
        tauq[j] = 0.0;
        taup[j] = 0.0;
    }

    for (int64_t k0 = 0; k0 < n; k0 += nb) {
        int64_t kend = (k0 + nb < n) ? k0 + nb : n;

        /* Step QR(k): one column Householder per column of the block. */
        for (int64_t c = k0; c < kend; ++c) {
            int64_t len = m - c;
            double *x = &AT(A, lda, c, c);
            double tau = make_reflector(x, len, 1);
            g_flops += 3.0 * (double)len;
            tauq[c] = tau;
            AT(VQ, ldvq, c, c) = 1.0;
            for (int64_t t = 1; t < len; ++t) AT(VQ, ldvq, c + t, c) = x[t];
            for (int64_t t = 1; t < len; ++t) x[t] = 0.0;
            if (tau != 0.0) {
                const double *v = &AT(VQ, ldvq, c, c);
#pragma omp parallel for schedule(static)
                for (int64_t j = c + 1; j < n; ++j) {
                    double *col = &AT(A, lda, c, j);
                    double w = 0.0;
                    for (int64_t t = 0; t < len; ++t) w += v[t] * col[t];
                    w *= tau;
                    for (int64_t t = 0; t < len; ++t) col[t] -= w * v[t];
                }
                g_flops += 4.0 * (double)len * (double)(n - c - 1);
            }
        }

        /* Step LQ(k): one row Householder per row of the block, pivot at the
         * band edge d = r + nb, zeroing B(r, d+1 : n-1). */
        for (int64_t r = k0; r < kend; ++r) {
            int64_t d = r + nb;
            if (d >= n - 1) continue;
            int64_t len = n - d;
            double *y = &AT(A, lda, r, d);
            double tau = make_reflector(y, len, lda);
            g_flops += 3.0 * (double)len;
            taup[r] = tau;
            AT(WP, ldwp, r, d) = 1.0;
            for (int64_t t = 1; t < len; ++t) AT(WP, ldwp, r, d + t) = y[t * lda];
            for (int64_t t = 1; t < len; ++t) y[t * lda] = 0.0;
            if (tau != 0.0) {
#pragma omp parallel for schedule(static)
                for (int64_t i = r + 1; i < m; ++i) {
                    double z = 0.0;
                    for (int64_t t = 0; t < len; ++t)
                        z += AT(A, lda, i, d + t) * AT(WP, ldwp, r, d + t);
                    z *= tau;
                    for (int64_t t = 0; t < len; ++t)
                        AT(A, lda, i, d + t) -= z * AT(WP, ldwp, r, d + t);
                }
                g_flops += 4.0 * (double)len * (double)(m - r - 1);
            }
        }
    }
    return 0;
}

/* Q(:, 0:ncols-1) = H_0 H_1 ... H_{n-1} I(:, 0:ncols-1), Q m x ncols. */
int oracle_form_q(int64_t m, int64_t n, const double *VQ, int64_t ldvq,
                  const double *tauq, int64_t ncols, double *Q, int64_t ldq) {
    if (ncols < 0 || ncols > m) return -6;
    for (int64_t j = 0; j < ncols; ++j)
        for (int64_t i = 0; i < m; ++i) AT(Q, ldq, i, j) = (i == j) ? 1.0 : 0.0;
    for (int64_t c = n - 1; c >= 0; --c) {
        double tau = tauq[c];
        if (tau == 0.0) continue;
        int64_t len = m - c;
        const double *v = &AT(VQ, ldvq, c, c);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < ncols; ++j) {
            double *col = &AT(Q, ldq, c, j);
            double w = 0.0;
            for (int64_t t = 0; t < len; ++t) w += v[t] * col[t];
            w *= tau;
            for (int64_t t = 0; t < len; ++t) col[t] -= w * v[t];
        }
    }
    return 0;
}

/* P = G_0 G_1 ... G_{n-1} (n x n), G_r = I - taup[r] w_r w_r^T. */
int oracle_form_p(int64_t n, const double *WP, int64_t ldwp, const double *taup,
                  double *P, int64_t ldp) {
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) AT(P, ldp, i, j) = (i == j) ? 1.0 : 0.0;
    /* P = G_0 (G_1 (... (G_{n-1} I))): apply from the last reflector. */
    for (int64_t r = n - 1; r >= 0; --r) {
        double tau = taup[r];
        if (tau == 0.0) continue;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            double w = 0.0;
            for (int64_t t = 0; t < n; ++t) w += AT(WP, ldwp, r, t) * AT(P, ldp, t, j);
            w *= tau;
            for (int64_t t = 0; t < n; ++t) AT(P, ldp, t, j) -= w * AT(WP, ldwp, r, t);
        }
    }
    return 0;
}

/*
 * R-BiDiag in scalar form (Section 3.5): a full column-Householder QR of A
 * first, then the band reduction of the leading n x n triangle R.  Produces
 * only B (A overwritten, rows >= n zero); used as a cross-check that both
 * variants reach the same band matrix.
 */
int oracle_rbidiag_reduce(int64_t m, int64_t n, int64_t nb, double *A, int64_t lda,
                          double *VQ, int64_t ldvq, double *tauq,
                          double *WP, int64_t ldwp, double *taup,
                          double *R, int64_t ldr) {
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nb < 1) return -3;
    for (int64_t c = 0; c < n; ++c) {
        int64_t len = m - c;
        double *x = &AT(A, lda, c, c);
        double tau = make_reflector(x, len, 1);
        if (tau != 0.0) {
#pragma omp parallel for schedule(static)
            for (int64_t j = c + 1; j < n; ++j) {
                double *col = &AT(A, lda, c, j);
                double w = col[0];
                for (int64_t t = 1; t < len; ++t) w += x[t] * col[t];
                w *= tau;
                col[0] -= w;
                for (int64_t t = 1; t < len; ++t) col[t] -= w * x[t];
            }
        }
        for (int64_t t = 1; t < len; ++t) x[t] = 0.0;
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) AT(R, ldr, i, j) = AT(A, lda, i, j);
    int rc = oracle_band_reduce(n, n, nb, R, ldr, VQ, ldvq, tauq, WP, ldwp, taup);
    if (rc != 0) return rc;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i) AT(A, lda, i, j) = AT(R, ldr, i, j);
        for (int64_t i = n; i < m; ++i) AT(A, lda, i, j) = 0.0;
    }
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
