/*
 * mhar_ref.h -- plain FP64 CPU oracle for Matrix Hit-and-Run (MHAR).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library,
 * its Python binding) may include, link or call this code.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * The oracle is written from the paper (Vazquez Corte & Montiel, "Novel
 * Matrix Hit and Run for Sampling Polytopes and Its GPU Implementation"):
 *   - problem statement Delta = {A^I x <= b^I} cap {A^E x = b^E}  (S2.1)
 *   - projection P = I - A_E^T (A_E A_E^T)^{-1} A_E               (S3.2)
 *   - MHAR loop, z walks as matrix columns                        (S4.1, Alg. 2)
 *   - directions from i.i.d. N(0,1) variates (Box-Muller)        (S4.3, Lemma 4.1)
 *   - line sets lambda_i = (b_i - a_i x)/(a_i d), min/max        (S4.4, Lemma 4.2)
 *   - theta uniform in (lambda_min, lambda_max), x += theta d     (S4.5, Lemma 4.3)
 * plus the counter-based random streams that the GPU path also implements
 * (independently) so that both sides walk the same trajectories.
 *
 * Everything is FP64, sequential left-to-right sums, built without FMA
 * contraction.  The slack b - A x is recomputed from scratch at every step,
 * exactly as the paper's line-set procedure does.
 */
#ifndef MHAR_REF_H
#define MHAR_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes (same numbering as the product library) */
#define MHAR_REF_OK               0
#define MHAR_REF_E_INVALID_ARG   (-1)
#define MHAR_REF_E_RANK_DEFICIENT (-3)
#define MHAR_REF_E_NOT_INTERIOR  (-4)

/* per-chain status bits */
#define MHAR_REF_CHAIN_UNBOUNDED  1
#define MHAR_REF_CHAIN_DEGENERATE 2
#define MHAR_REF_CHAIN_NONFINITE  4
#define MHAR_REF_CHAIN_INFEASIBLE 8

/* random stream tags (counter word 3, low 4 bits) */
#define MHAR_REF_TAG_DIR     0
#define MHAR_REF_TAG_THETA   1
#define MHAR_REF_TAG_LOWRANK 2
#define MHAR_REF_TAG_TRAIN   4

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void mhar_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Uniform in the open interval (0,1) from 52 random bits of block `block`
 * of stream (seed, tag, chain, step); which = 0 uses words (0,1), 1 uses (2,3). */
double mhar_ref_uniform(uint64_t seed, uint32_t tag, uint64_t chain, uint64_t step,
                        uint32_t block, int which);

/* j-th standard normal of stream (seed, tag, chain, step) via Box-Muller. */
double mhar_ref_gauss(uint64_t seed, uint32_t tag, uint64_t chain, uint64_t step, int64_t j);

/* Dense projection P (n x n, row-major) onto null(A_eq); A_eq is m_eq x n. */
int mhar_ref_projection(int64_t n, int64_t m_eq, const double* A_eq, double* P);

/* Interior test of the start points X (z x n row-major): b - A x > 0 and
 * |A_eq x - b_eq|_inf <= 1e-9 for every chain. */
int mhar_ref_check_interior(int64_t n, int64_t m, const double* A, const double* b,
                            int64_t m_eq, const double* A_eq, const double* b_eq,
                            int64_t z, const double* X);

/* Line set of one walk: lambda bounds along d from x (S4.4). flags gets
 * UNBOUNDED when one side has no bounding row. */
void mhar_ref_chord(int64_t n, int64_t m, const double* A, const double* b,
                    const double* x, const double* d,
                    double* lambda_min, double* lambda_max, int32_t* flags);

/* Direction of chain `chain` at step `step`: h ~ N(0,I) (DIR stream),
 * optional preconditioner h <- U eps + exp(log_sigma) o h (eps from the
 * LOWRANK stream, r = 0 disables), then d = P h when P != NULL. */
void mhar_ref_direction(int64_t n, const double* P, int64_t r, const double* U,
                        const double* log_sigma, uint64_t seed, uint64_t chain,
                        uint64_t step, double* d);

/* Run `steps` MHAR iterations on z chains.  X (z x n row-major, chain k is
 * row k) is advanced in place; global chain id = chain_offset + k; global
 * step id = step0 + t.  status (z) receives the OR of per-chain flags.
 * If rec_stride > 0, the states of chains [0, rec_chains) after every
 * step t with (t+1) % rec_stride == 0 go to rec_out
 * ((steps/rec_stride) x rec_chains x n).  threads <= 0 uses all cores. */
int mhar_ref_run(int64_t n, int64_t m, const double* A, const double* b,
                 const double* P, int64_t r, const double* U, const double* log_sigma,
                 int64_t z, double* X, uint64_t seed, uint64_t chain_offset,
                 uint64_t step0, int64_t steps, int32_t* status,
                 int64_t rec_stride, int64_t rec_chains, double* rec_out, int threads);

/* Gaussian negative log-likelihood of the chain states X (z x n) under
 * N(mean(X), Sigma), Sigma = U U^T + diag(exp(2 log_sigma)) (U is n x r),
 * and its gradient with respect to U and log_sigma.  Dense n x n algebra. */
int mhar_ref_precond_nll(int64_t n, int64_t r, const double* U, const double* log_sigma,
                         int64_t z, const double* X, double* nll, double* grad_U,
                         double* grad_log_sigma);

/* One Adam update (Kingma & Ba) of `count` parameters; t is the 1-based step. */
void mhar_ref_adam(int64_t count, double* param, const double* grad, double* m1,
                   double* m2, int64_t t, double lr, double beta1, double beta2, double eps);

/* One burn-in update of the covariance in the scale-free coordinates
 * V = diag(exp(-log_sigma)) U.  U is formed as diag(exp(log_sigma)) V, the
 * NLL gradient (grad_U, grad_l) is taken at the states X (z x n); the chain
 * rule gives grad_V = diag(exp(log_sigma)) grad_U and grad_l + rowsum(grad_U o U)
 * for log_sigma; one Adam step moves V (moments m1V, m2V) and log_sigma
 * (moments m1l, m2l); U_out (n x r) receives diag(exp(log_sigma_new)) V_new. */
int mhar_ref_precond_train_step(int64_t n, int64_t r, double* V, double* log_sigma,
                                double* m1V, double* m2V, double* m1l, double* m2l, int64_t z,
                                const double* X, int64_t t, double lr, double beta1,
                                double beta2, double eps, double* U_out);

/* Log-barrier Hessian sum_i a_i a_i^T / s_i^2, s = b - A xbar, at the mean
 * xbar of the walk states X (z x n); H is n x n, xbar (n, may be NULL).
 * MHAR_REF_E_NOT_INTERIOR if some s_i <= 0. */
int mhar_ref_dikin_hessian(int64_t n, int64_t m, const double* A, const double* b,
                           int64_t z, const double* X, double* xbar, double* H);

/* K = 1/2 tr(H Sigma) - 1/2 log det Sigma for Sigma = U U^T + diag(exp(2 log_sigma))
 * and its gradient with respect to U and log_sigma (either may be NULL). */
int mhar_ref_dikin_objective(int64_t n, int64_t r, const double* U, const double* log_sigma,
                             const double* H, double* K, double* grad_U, double* grad_log_sigma);

/* One burn-in update towards the Dikin ellipsoid at the mean state: Hessian,
 * k_pow power iterations on the Jacobi-scaled Hessian (v in/out), the
 * inscribed diagonal scaled by kappa in (0, 1] (log_sigma, out), then
 * U <- U - eta H^{-1} dK/dU. */
int mhar_ref_dikin_train_step(int64_t n, int64_t m, const double* A, const double* b,
                              int64_t z, const double* X, int64_t r, double* U,
                              double* log_sigma, double* v, int k_pow, double eta,
                              double kappa, double* lam_out);

#ifdef __cplusplus
}
#endif
#endif
