/*
 * mhar_ref.c -- plain FP64 CPU oracle for Matrix Hit-and-Run.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU-baseline leg.  The product (HIP library + binding) never
 * includes, links or calls this file.  It shares no code with the GPU path;
 * the only common ground is the published definition of the random streams
 * (Philox4x32-10 counters, 52-bit uniforms, Box-Muller pairs), written out
 * independently on each side.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 * Every dot product is a sequential sum over j = 0 .. n-1.
 *
 * Parity pins (what checks this file against something other than itself)
 * are listed in the test suite; see tests/test_oracle_*.py.
 */
#include "mhar_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Random streams                                                            */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): ten rounds of two 32x32->64 multiplies with the published
 * multipliers, Weyl key schedule with the published increments. */
void mhar_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mul_a = 0xD2511F53u, mul_b = 0xCD9E8D57u;
    const uint32_t weyl_a = 0x9E3779B9u, weyl_b = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)mul_a * (uint64_t)x0;
        uint64_t pb = (uint64_t)mul_b * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)pb;
        uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)pa;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += weyl_a;
        k1 += weyl_b;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter layout: (block, chain, step low 32 bits, tag | (step >> 32) << 4);
 * key = (seed low 32 bits, seed high 32 bits). */
static void stream_block(uint64_t seed, uint32_t tag, uint64_t chain, uint64_t step,
                         uint32_t block, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = block;
    ctr[1] = (uint32_t)chain;
    ctr[2] = (uint32_t)step;
    ctr[3] = tag | (uint32_t)((step >> 32) << 4);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    mhar_ref_philox4x32_10(ctr, key, out);
}

/* 52 bits (hi word then lo word, top 52 of the 64) -> (k + 1/2) 2^-52,
 * exact in binary64 and strictly inside (0,1). */
static double open_uniform(uint32_t hi, uint32_t lo)
{
    uint64_t bits = (((uint64_t)hi << 32) | (uint64_t)lo) >> 12;
    return ((double)bits + 0.5) * 0x1.0p-52;
}

double mhar_ref_uniform(uint64_t seed, uint32_t tag, uint64_t chain, uint64_t step,
                        uint32_t block, int which)
{
    uint32_t w[4];
    stream_block(seed, tag, chain, step, block, w);
    return which ? open_uniform(w[2], w[3]) : open_uniform(w[0], w[1]);
}

/* Box-Muller (S4.3 draws each entry of H as an independent N(0,1) variate
 * by this method): block j/2 gives u_a, u_b; radius sqrt(-2 ln u_a), angle
 * 2 pi u_b; even j takes the cosine, odd j the sine. */
double mhar_ref_gauss(uint64_t seed, uint32_t tag, uint64_t chain, uint64_t step, int64_t j)
{
    uint32_t w[4];
    stream_block(seed, tag, chain, step, (uint32_t)(j >> 1), w);
    double ua = open_uniform(w[0], w[1]);
    double ub = open_uniform(w[2], w[3]);
    double radius = sqrt(-2.0 * log(ua));
    double angle = 6.283185307179586 * ub;
    return (j & 1) ? radius * sin(angle) : radius * cos(angle);
}

/* ------------------------------------------------------------------------ */
/* Projection onto null(A_E)  (S3.2, Lemma 3.1)                              */
/* ------------------------------------------------------------------------ */

/* Cholesky factor of the m x m SPD matrix G (lower, row-major, in place of L).
 * A pivot at or below 1e-12 * max diag(G) means linearly dependent rows. */
static int cholesky_lower(int64_t m, const double* G, double* L)
{
    double max_diag = 0.0;
    for (int64_t i = 0; i < m; ++i)
        if (G[i * m + i] > max_diag) max_diag = G[i * m + i];
    memset(L, 0, sizeof(double) * (size_t)(m * m));
    for (int64_t j = 0; j < m; ++j) {
        double pivot = G[j * m + j];
        for (int64_t k = 0; k < j; ++k) pivot -= L[j * m + k] * L[j * m + k];
        if (!(pivot > 1e-12 * max_diag)) return MHAR_REF_E_RANK_DEFICIENT;
        double ljj = sqrt(pivot);
        L[j * m + j] = ljj;
        for (int64_t i = j + 1; i < m; ++i) {
            double v = G[i * m + j];
            for (int64_t k = 0; k < j; ++k) v -= L[i * m + k] * L[j * m + k];
            L[i * m + j] = v / ljj;
        }
    }
    return MHAR_REF_OK;
}

/* Solve L L^T y = rhs in place (L lower, m x m). */
static void cholesky_solve(int64_t m, const double* L, double* y)
{
    for (int64_t i = 0; i < m; ++i) {
        double v = y[i];
        for (int64_t k = 0; k < i; ++k) v -= L[i * m + k] * y[k];
        y[i] = v / L[i * m + i];
    }
    for (int64_t i = m - 1; i >= 0; --i) {
        double v = y[i];
        for (int64_t k = i + 1; k < m; ++k) v -= L[k * m + i] * y[k];
        y[i] = v / L[i * m + i];
    }
}

/* P = I - A_E^T (A_E A_E^T)^{-1} A_E, with the inverse applied through a
 * Cholesky factorisation of A_E A_E^T instead of an explicit inverse. */
int mhar_ref_projection(int64_t n, int64_t m_eq, const double* A_eq, double* P)
{
    if (n <= 0 || m_eq < 0 || (m_eq > 0 && !A_eq) || !P) return MHAR_REF_E_INVALID_ARG;
    if (m_eq >= n) return MHAR_REF_E_RANK_DEFICIENT;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) P[i * n + j] = (i == j) ? 1.0 : 0.0;
    if (m_eq == 0) return MHAR_REF_OK;

    double* G = (double*)malloc(sizeof(double) * (size_t)(m_eq * m_eq));
    double* L = (double*)malloc(sizeof(double) * (size_t)(m_eq * m_eq));
    double* Y = (double*)malloc(sizeof(double) * (size_t)(m_eq * n)); /* G^{-1} A_E */
    double* col = (double*)malloc(sizeof(double) * (size_t)m_eq);
    int rc = MHAR_REF_OK;
    for (int64_t p = 0; p < m_eq; ++p)
        for (int64_t q = 0; q < m_eq; ++q) {
            double v = 0.0;
            for (int64_t j = 0; j < n; ++j) v += A_eq[p * n + j] * A_eq[q * n + j];
            G[p * m_eq + q] = v;
        }
    rc = cholesky_lower(m_eq, G, L);
    if (rc == MHAR_REF_OK) {
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t p = 0; p < m_eq; ++p) col[p] = A_eq[p * n + j];
            cholesky_solve(m_eq, L, col);
            for (int64_t p = 0; p < m_eq; ++p) Y[p * n + j] = col[p];
        }
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double v = 0.0;
                for (int64_t p = 0; p < m_eq; ++p) v += A_eq[p * n + i] * Y[p * n + j];
                P[i * n + j] -= v;
            }
    }
    free(G); free(L); free(Y); free(col);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Start points (Alg. 2 needs a strictly inner point of Delta)               */
/* ------------------------------------------------------------------------ */

int mhar_ref_check_interior(int64_t n, int64_t m, const double* A, const double* b,
                            int64_t m_eq, const double* A_eq, const double* b_eq,
                            int64_t z, const double* X)
{
    if (n <= 0 || m <= 0 || z <= 0 || !A || !b || !X) return MHAR_REF_E_INVALID_ARG;
    if (m_eq > 0 && (!A_eq || !b_eq)) return MHAR_REF_E_INVALID_ARG;
    for (int64_t k = 0; k < z; ++k) {
        const double* x = X + k * n;
        for (int64_t i = 0; i < m; ++i) {
            double s = b[i];
            for (int64_t j = 0; j < n; ++j) s -= A[i * n + j] * x[j];
            if (!(s > 0.0)) return MHAR_REF_E_NOT_INTERIOR;
        }
        for (int64_t p = 0; p < m_eq; ++p) {
            double r = 0.0;
            for (int64_t j = 0; j < n; ++j) r += A_eq[p * n + j] * x[j];
            r -= b_eq[p];
            if (!(fabs(r) <= 1e-9)) return MHAR_REF_E_NOT_INTERIOR;
        }
    }
    return MHAR_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Line set of one walk  (S4.4, Lemma 4.2)                                   */
/* ------------------------------------------------------------------------ */

/* For each inequality row: slack s_i = b_i - a_i x (clamped at 0 against
 * rounding), directional derivative g_i = a_i d, ratio s_i / g_i.  The
 * upper end is the least ratio over rows with g_i > 0, the lower end the
 * greatest ratio over rows with g_i < 0; rows with g_i = 0 never bind. */
void mhar_ref_chord(int64_t n, int64_t m, const double* A, const double* b,
                    const double* x, const double* d,
                    double* lambda_min, double* lambda_max, int32_t* flags)
{
    double lo = -INFINITY, hi = INFINITY;
    int32_t f = 0;
    for (int64_t i = 0; i < m; ++i) {
        const double* a = A + i * n;
        double s = b[i];
        for (int64_t j = 0; j < n; ++j) s -= a[j] * x[j];
        double tol = 1e-12 * (fabs(b[i]) > 1.0 ? fabs(b[i]) : 1.0);
        if (s < -tol) f |= MHAR_REF_CHAIN_INFEASIBLE;
        if (s < 0.0) s = 0.0;
        double g = 0.0;
        for (int64_t j = 0; j < n; ++j) g += a[j] * d[j];
        if (g > 0.0) {
            double r = s / g;
            if (r < hi) hi = r;
        } else if (g < 0.0) {
            double r = s / g;
            if (r > lo) lo = r;
        }
    }
    if (hi == INFINITY || lo == -INFINITY) f |= MHAR_REF_CHAIN_UNBOUNDED;
    *lambda_min = lo;
    *lambda_max = hi;
    *flags = f;
}

/* ------------------------------------------------------------------------ */
/* Directions  (S4.3; projection S3.2)                                       */
/* ------------------------------------------------------------------------ */

static void direction_into(int64_t n, const double* P, int64_t r, const double* U,
                           const double* log_sigma, uint64_t seed, uint64_t chain,
                           uint64_t step, double* h, double* eps, double* d)
{
    for (int64_t j = 0; j < n; ++j) h[j] = mhar_ref_gauss(seed, MHAR_REF_TAG_DIR, chain, step, j);
    if (r > 0) {
        for (int64_t a = 0; a < r; ++a)
            eps[a] = mhar_ref_gauss(seed, MHAR_REF_TAG_LOWRANK, chain, step, a);
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            for (int64_t a = 0; a < r; ++a) v += U[j * r + a] * eps[a];
            h[j] = v + exp(log_sigma[j]) * h[j];
        }
    }
    if (P) {
        for (int64_t i = 0; i < n; ++i) {
            double v = 0.0;
            for (int64_t j = 0; j < n; ++j) v += P[i * n + j] * h[j];
            d[i] = v;
        }
    } else {
        for (int64_t j = 0; j < n; ++j) d[j] = h[j];
    }
}

void mhar_ref_direction(int64_t n, const double* P, int64_t r, const double* U,
                        const double* log_sigma, uint64_t seed, uint64_t chain,
                        uint64_t step, double* d)
{
    double* h = (double*)malloc(sizeof(double) * (size_t)n);
    double* eps = (double*)malloc(sizeof(double) * (size_t)(r > 0 ? r : 1));
    direction_into(n, P, r, U, log_sigma, seed, chain, step, h, eps, d);
    free(h);
    free(eps);
}

/* ------------------------------------------------------------------------ */
/* MHAR iterations  (Alg. 2; S4.3-S4.5)                                      */
/* ------------------------------------------------------------------------ */

int mhar_ref_run(int64_t n, int64_t m, const double* A, const double* b,
                 const double* P, int64_t r, const double* U, const double* log_sigma,
                 int64_t z, double* X, uint64_t seed, uint64_t chain_offset,
                 uint64_t step0, int64_t steps, int32_t* status,
                 int64_t rec_stride, int64_t rec_chains, double* rec_out, int threads)
{
    if (n <= 0 || m <= 0 || z <= 0 || steps < 0 || !A || !b || !X || !status)
        return MHAR_REF_E_INVALID_ARG;
    if (r > 0 && (!U || !log_sigma)) return MHAR_REF_E_INVALID_ARG;
    if (rec_stride > 0 && (!rec_out || rec_chains < 0 || rec_chains > z))
        return MHAR_REF_E_INVALID_ARG;
#ifdef _OPENMP
    int nthreads = threads > 0 ? threads : omp_get_max_threads();
#else
    int nthreads = 1;
    (void)threads;
#endif

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t k = 0; k < z; ++k) {
        double* x = X + k * n;
        double* h = (double*)malloc(sizeof(double) * (size_t)n);
        double* d = (double*)malloc(sizeof(double) * (size_t)n);
        double* eps = (double*)malloc(sizeof(double) * (size_t)(r > 0 ? r : 1));
        uint64_t chain = chain_offset + (uint64_t)k;
        int32_t flags = 0;
        for (int64_t t = 0; t < steps; ++t) {
            uint64_t step = step0 + (uint64_t)t;
            direction_into(n, P, r, U, log_sigma, seed, chain, step, h, eps, d);
            double lo, hi;
            int32_t f;
            mhar_ref_chord(n, m, A, b, x, d, &lo, &hi, &f);
            flags |= f;
            double theta = 0.0;
            if (f & MHAR_REF_CHAIN_UNBOUNDED) {
                theta = 0.0;
            } else if (!(hi > lo)) {
                flags |= MHAR_REF_CHAIN_DEGENERATE;
                theta = 0.0;
            } else {
                double u = mhar_ref_uniform(seed, MHAR_REF_TAG_THETA, chain, step, 0, 0);
                theta = lo + u * (hi - lo);
            }
            int finite = isfinite(theta);
            for (int64_t j = 0; j < n; ++j) {
                x[j] = x[j] + theta * d[j];
                if (!isfinite(x[j])) finite = 0;
            }
            if (!finite) flags |= MHAR_REF_CHAIN_NONFINITE;
            if (rec_stride > 0 && k < rec_chains && (t + 1) % rec_stride == 0) {
                int64_t slot = (t + 1) / rec_stride - 1;
                memcpy(rec_out + (slot * rec_chains + k) * n, x, sizeof(double) * (size_t)n);
            }
        }
        status[k] = flags;
        free(h);
        free(d);
        free(eps);
    }
    return MHAR_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Direction covariance fit (learned preconditioner; not in the paper)       */
/* ------------------------------------------------------------------------ */

/* NLL = 1/2 log det Sigma + 1/2 tr(Sigma^{-1} S), S the (1/z) sample
 * covariance of the states about their mean.  With M = Sigma^{-1} -
 * Sigma^{-1} S Sigma^{-1}: dNLL/dU = M U, dNLL/dl_i = M_ii exp(2 l_i). */
int mhar_ref_precond_nll(int64_t n, int64_t r, const double* U, const double* log_sigma,
                         int64_t z, const double* X, double* nll, double* grad_U,
                         double* grad_log_sigma)
{
    if (n <= 0 || r < 0 || z <= 0 || !log_sigma || !X || !nll) return MHAR_REF_E_INVALID_ARG;
    size_t nn = (size_t)(n * n);
    double* Sig = (double*)malloc(sizeof(double) * nn);
    double* L = (double*)malloc(sizeof(double) * nn);
    double* Sinv = (double*)malloc(sizeof(double) * nn);
    double* S = (double*)calloc(nn, sizeof(double));
    double* mean = (double*)calloc((size_t)n, sizeof(double));
    double* col = (double*)malloc(sizeof(double) * (size_t)n);
    double* T = (double*)malloc(sizeof(double) * nn);
    double* M = (double*)malloc(sizeof(double) * nn);
    int rc = MHAR_REF_OK;

    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            for (int64_t a = 0; a < r; ++a) v += U[i * r + a] * U[j * r + a];
            if (i == j) v += exp(2.0 * log_sigma[i]);
            Sig[i * n + j] = v;
        }
    for (int64_t k = 0; k < z; ++k)
        for (int64_t j = 0; j < n; ++j) mean[j] += X[k * n + j];
    for (int64_t j = 0; j < n; ++j) mean[j] /= (double)z;
    for (int64_t k = 0; k < z; ++k)
        for (int64_t i = 0; i < n; ++i) {
            double ci = X[k * n + i] - mean[i];
            for (int64_t j = 0; j < n; ++j) S[i * n + j] += ci * (X[k * n + j] - mean[j]);
        }
    for (size_t e = 0; e < nn; ++e) S[e] /= (double)z;

    rc = cholesky_lower(n, Sig, L);
    if (rc != MHAR_REF_OK) goto done;
    double logdet = 0.0;
    for (int64_t i = 0; i < n; ++i) logdet += 2.0 * log(L[i * n + i]);
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i) col[i] = (i == j) ? 1.0 : 0.0;
        cholesky_solve(n, L, col);
        for (int64_t i = 0; i < n; ++i) Sinv[i * n + j] = col[i];
    }
    double tr = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) tr += Sinv[i * n + j] * S[j * n + i];
    *nll = 0.5 * logdet + 0.5 * tr;

    /* T = Sinv S;  M = Sinv - T Sinv */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            for (int64_t k = 0; k < n; ++k) v += Sinv[i * n + k] * S[k * n + j];
            T[i * n + j] = v;
        }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            for (int64_t k = 0; k < n; ++k) v += T[i * n + k] * Sinv[k * n + j];
            M[i * n + j] = Sinv[i * n + j] - v;
        }
    if (grad_U)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t a = 0; a < r; ++a) {
                double v = 0.0;
                for (int64_t k = 0; k < n; ++k) v += M[i * n + k] * U[k * r + a];
                grad_U[i * r + a] = v;
            }
    if (grad_log_sigma)
        for (int64_t i = 0; i < n; ++i) grad_log_sigma[i] = M[i * n + i] * exp(2.0 * log_sigma[i]);
done:
    free(Sig); free(L); free(Sinv); free(S); free(mean); free(col); free(T); free(M);
    return rc;
}

void mhar_ref_adam(int64_t count, double* param, const double* grad, double* m1,
                   double* m2, int64_t t, double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < count; ++i) {
        m1[i] = beta1 * m1[i] + (1.0 - beta1) * grad[i];
        m2[i] = beta2 * m2[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = m1[i] / c1;
        double vh = m2[i] / c2;
        param[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

int mhar_ref_precond_train_step(int64_t n, int64_t r, double* V, double* log_sigma,
                                double* m1V, double* m2V, double* m1l, double* m2l, int64_t z,
                                const double* X, int64_t t, double lr, double beta1,
                                double beta2, double eps, double* U_out)
{
    if (n <= 0 || r <= 0 || z <= 0 || !V || !log_sigma || !X || !U_out) return MHAR_REF_E_INVALID_ARG;
    size_t nr = (size_t)(n * r);
    double* U = (double*)malloc(sizeof(double) * nr);
    double* gU = (double*)malloc(sizeof(double) * nr);
    double* gV = (double*)malloc(sizeof(double) * nr);
    double* gl = (double*)malloc(sizeof(double) * (size_t)n);
    double nll = 0.0;
    int rc = MHAR_REF_OK;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t a = 0; a < r; ++a) U[i * r + a] = exp(log_sigma[i]) * V[i * r + a];
    rc = mhar_ref_precond_nll(n, r, U, log_sigma, z, X, &nll, gU, gl);
    if (rc == MHAR_REF_OK) {
        /* d/dV_ia = exp(l_i) dNLL/dU_ia;  d/dl_i = dNLL/dl_i + sum_a dNLL/dU_ia * U_ia */
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t a = 0; a < r; ++a) {
                gV[i * r + a] = gU[i * r + a] * exp(log_sigma[i]);
                gl[i] += gU[i * r + a] * U[i * r + a];
            }
        }
        mhar_ref_adam((int64_t)nr, V, gV, m1V, m2V, t, lr, beta1, beta2, eps);
        mhar_ref_adam(n, log_sigma, gl, m1l, m2l, t, lr, beta1, beta2, eps);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t a = 0; a < r; ++a) U_out[i * r + a] = exp(log_sigma[i]) * V[i * r + a];
    }
    free(U);
    free(gU);
    free(gV);
    free(gl);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Direction covariance fitted to the Dikin ellipsoid (not in the paper)     */
/* ------------------------------------------------------------------------ */

/* The log-barrier phi(x) = -sum_i log(b_i - a_i x) of the inequality rows
 * has Hessian sum_i a_i a_i^T / s_i(x)^2; its unit ellipsoid at x (the
 * Dikin ellipsoid) lies inside the polytope.  Evaluated at the mean of the
 * walk states. */
int mhar_ref_dikin_hessian(int64_t n, int64_t m, const double* A, const double* b,
                           int64_t z, const double* X, double* xbar, double* H)
{
    if (n <= 0 || m <= 0 || z <= 0 || !A || !b || !X || !H) return MHAR_REF_E_INVALID_ARG;
    double* mean = (double*)calloc((size_t)n, sizeof(double));
    double* w = (double*)malloc(sizeof(double) * (size_t)m);
    int rc = MHAR_REF_OK;
    for (int64_t k = 0; k < z; ++k)
        for (int64_t j = 0; j < n; ++j) mean[j] += X[k * n + j];
    for (int64_t j = 0; j < n; ++j) mean[j] /= (double)z;
    for (int64_t i = 0; i < m; ++i) {
        double s = b[i];
        for (int64_t j = 0; j < n; ++j) s -= A[i * n + j] * mean[j];
        if (!(s > 0.0)) rc = MHAR_REF_E_NOT_INTERIOR;
        w[i] = 1.0 / (s * s);
    }
    for (int64_t p = 0; p < n; ++p)
        for (int64_t q = 0; q < n; ++q) {
            double v = 0.0;
            for (int64_t i = 0; i < m; ++i) v += w[i] * A[i * n + p] * A[i * n + q];
            H[p * n + q] = v;
        }
    if (xbar) memcpy(xbar, mean, sizeof(double) * (size_t)n);
    free(mean);
    free(w);
    return rc;
}

/* K(Sigma) = 1/2 tr(H Sigma) - 1/2 log det Sigma, Sigma = U U^T + diag(exp(2 l)):
 * the Kullback-Leibler divergence of N(0, Sigma) from N(0, H^{-1}) up to a
 * constant.  dK/dU = (H - Sigma^{-1}) U, dK/dl_i = (H - Sigma^{-1})_ii exp(2 l_i).
 * Dense n x n algebra. */
int mhar_ref_dikin_objective(int64_t n, int64_t r, const double* U, const double* log_sigma,
                             const double* H, double* K, double* grad_U, double* grad_log_sigma)
{
    if (n <= 0 || r < 0 || !log_sigma || !H || !K || (r > 0 && !U)) return MHAR_REF_E_INVALID_ARG;
    size_t nn = (size_t)(n * n);
    double* Sig = (double*)malloc(sizeof(double) * nn);
    double* L = (double*)malloc(sizeof(double) * nn);
    double* Sinv = (double*)malloc(sizeof(double) * nn);
    double* col = (double*)malloc(sizeof(double) * (size_t)n);
    int rc;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            for (int64_t a = 0; a < r; ++a) v += U[i * r + a] * U[j * r + a];
            if (i == j) v += exp(2.0 * log_sigma[i]);
            Sig[i * n + j] = v;
        }
    rc = cholesky_lower(n, Sig, L);
    if (rc == MHAR_REF_OK) {
        double logdet = 0.0;
        for (int64_t i = 0; i < n; ++i) logdet += 2.0 * log(L[i * n + i]);
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t i = 0; i < n; ++i) col[i] = (i == j) ? 1.0 : 0.0;
            cholesky_solve(n, L, col);
            for (int64_t i = 0; i < n; ++i) Sinv[i * n + j] = col[i];
        }
        double tr = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) tr += H[i * n + j] * Sig[j * n + i];
        *K = 0.5 * tr - 0.5 * logdet;
        if (grad_U)
            for (int64_t i = 0; i < n; ++i)
                for (int64_t a = 0; a < r; ++a) {
                    double v = 0.0;
                    for (int64_t k = 0; k < n; ++k) v += (H[i * n + k] - Sinv[i * n + k]) * U[k * r + a];
                    grad_U[i * r + a] = v;
                }
        if (grad_log_sigma)
            for (int64_t i = 0; i < n; ++i)
                grad_log_sigma[i] = (H[i * n + i] - Sinv[i * n + i]) * exp(2.0 * log_sigma[i]);
    }
    free(Sig); free(L); free(Sinv); free(col);
    return rc;
}

/* One burn-in update of the covariance toward the Dikin ellipsoid at the
 * mean of the walk states X (z x n):
 *   1. H = the log-barrier Hessian at mean(X);
 *   2. J = diag(H)^{-1/2} H diag(H)^{-1/2}; k_pow power iterations
 *      v <- J v / |J v| from v (in/out), lam = v^T J v (an estimate of
 *      lambda_max(J) from below);
 *   3. log_sigma_i = log(kappa) - 1/2 log(lam H_ii): at kappa = 1 the
 *      diagonal D = diag(1/(lam H_ii)) has D^{1/2} H D^{1/2} = J / lam, so
 *      N(0, D) is (up to the estimate) the largest Gaussian of this diagonal
 *      shape inside the Dikin ellipsoid; kappa in (0, 1] shrinks it;
 *   4. with that diagonal, U <- U - eta H^{-1} dK/dU (a Newton-type step on
 *      K: the H^{-1} factor is the inverse of the curvature of the
 *      tr(H Sigma) term).  With eta = 1/2 the column norms follow the
 *      Babylonian iteration towards their optimum.
 * lam_out (may be NULL) receives lam. */
int mhar_ref_dikin_train_step(int64_t n, int64_t m, const double* A, const double* b,
                              int64_t z, const double* X, int64_t r, double* U,
                              double* log_sigma, double* v, int k_pow, double eta,
                              double kappa, double* lam_out)
{
    if (n <= 0 || m <= 0 || z <= 0 || r <= 0 || !A || !b || !X || !U || !log_sigma || !v ||
        k_pow < 1 || !(kappa > 0.0 && kappa <= 1.0))
        return MHAR_REF_E_INVALID_ARG;
    size_t nn = (size_t)(n * n), nr = (size_t)(n * r);
    double* H = (double*)malloc(sizeof(double) * nn);
    double* L = (double*)malloc(sizeof(double) * nn);
    double* dsq = (double*)malloc(sizeof(double) * (size_t)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    double* gU = (double*)malloc(sizeof(double) * nr);
    double* col = (double*)malloc(sizeof(double) * (size_t)n);
    double K = 0.0, lam = 0.0;
    int rc = mhar_ref_dikin_hessian(n, m, A, b, z, X, NULL, H);
    if (rc != MHAR_REF_OK) goto done;
    for (int64_t i = 0; i < n; ++i) dsq[i] = sqrt(H[i * n + i]);
    for (int it = 0; it < k_pow; ++it) {
        double norm2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double t = 0.0;
            for (int64_t j = 0; j < n; ++j) t += H[i * n + j] / (dsq[i] * dsq[j]) * v[j];
            y[i] = t;
            norm2 += t * t;
        }
        double norm = sqrt(norm2);
        for (int64_t i = 0; i < n; ++i) v[i] = y[i] / norm;
    }
    for (int64_t i = 0; i < n; ++i) {
        double t = 0.0;
        for (int64_t j = 0; j < n; ++j) t += H[i * n + j] / (dsq[i] * dsq[j]) * v[j];
        lam += v[i] * t;
    }
    for (int64_t i = 0; i < n; ++i) log_sigma[i] = log(kappa) - 0.5 * log(lam * H[i * n + i]);
    rc = mhar_ref_dikin_objective(n, r, U, log_sigma, H, &K, gU, NULL);
    if (rc != MHAR_REF_OK) goto done;
    rc = cholesky_lower(n, H, L);
    if (rc != MHAR_REF_OK) goto done;
    for (int64_t a = 0; a < r; ++a) {
        for (int64_t i = 0; i < n; ++i) col[i] = gU[i * r + a];
        cholesky_solve(n, L, col);
        for (int64_t i = 0; i < n; ++i) U[i * r + a] -= eta * col[i];
    }
    if (lam_out) *lam_out = lam;
done:
    free(H); free(L); free(dsq); free(y); free(gU); free(col);
    return rc;
}
