/* Host sanitizer run of the oracle (built with -fsanitize=address,undefined):
 * every entry point on small inputs, including the boundary branches (a
 * walk on a facet, past a facet, at a vertex, a NaN coordinate), the
 * projection, both covariance fits and the rank-deficiency error.
 * Exit status 0 when every call returned the expected code. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/mhar_ref.h"

static int fails = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++fails;                                                   \
        }                                                              \
    } while (0)

int main(void)
{
    enum { n = 3, m = 6, z = 8, r = 2 };
    double A[m * n] = {0}, b[m];
    for (int i = 0; i < n; ++i) {
        A[i * n + i] = 1.0;
        A[(n + i) * n + i] = -1.0;
    }
    for (int i = 0; i < m; ++i) b[i] = 1.0;

    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    mhar_ref_philox4x32_10(ctr, key, out);
    const double u = mhar_ref_uniform(7, 1, 3, 11, 0, 0);
    EXPECT(u > 0.0 && u < 1.0);
    EXPECT(isfinite(mhar_ref_gauss(7, 1, 3, 11, 5)));

    /* walks: interior, facet, just past a facet, vertex, NaN, interior */
    double X[z * n] = {0.1, -0.2, 0.3, 1.0, 0.2, -0.3, 1.0 + 1e-9, 0.0, 0.0, 1.0, 1.0, 1.0,
                       NAN, 0.0, 0.0, -0.4, 0.5, 0.0, 0.0, 0.0, 0.0, 0.2, 0.2, 0.2};
    int32_t status[z];
    EXPECT(mhar_ref_run(n, m, A, b, NULL, 0, NULL, NULL, z, X, 3, 0, 0, 5, status, 0, 0, NULL, 1) == 0);
    double lo, hi;
    int32_t fl;
    const double x0[n] = {0, 0, 0}, d0[n] = {0.3, -0.2, 0.1};
    mhar_ref_chord(n, m, A, b, x0, d0, &lo, &hi, &fl);
    EXPECT(fl == 0 && lo < 0.0 && hi > 0.0);

    /* recording */
    double Xs[z * n] = {0}, rec[4 * 2 * n];
    EXPECT(mhar_ref_run(n, m, A, b, NULL, 0, NULL, NULL, z, Xs, 3, 0, 0, 8, status, 2, 2, rec, 1) == 0);
    EXPECT(mhar_ref_check_interior(n, m, A, b, 0, NULL, NULL, z, Xs) == 0);

    /* projection and the rank-deficiency error */
    double Aeq[2 * n] = {1, 1, 1, 2, 2, 2}, P[n * n];
    EXPECT(mhar_ref_projection(n, 1, Aeq, P) == 0);
    EXPECT(mhar_ref_projection(n, 2, Aeq, P) != 0);

    /* learned covariance: direction, NLL fit, Adam */
    double U[n * r] = {0.01, 0.02, -0.01, 0.03, 0.0, 0.01}, ls[n] = {0, 0.1, -0.1}, dvec[n];
    mhar_ref_direction(n, P, r, U, ls, 3, 1, 2, dvec);
    double nll, gU[n * r], gl[n];
    EXPECT(mhar_ref_precond_nll(n, r, U, ls, z, Xs, &nll, gU, gl) == 0);
    double V[n * r], m1V[n * r] = {0}, m2V[n * r] = {0}, m1l[n] = {0}, m2l[n] = {0}, Uo[n * r];
    for (int e = 0; e < n * r; ++e) V[e] = U[e] / exp(ls[e / r]);
    EXPECT(mhar_ref_precond_train_step(n, r, V, ls, m1V, m2V, m1l, m2l, z, Xs, 1, 0.01, 0.9, 0.999,
                                       1e-8, Uo) == 0);
    double p1[4] = {1, 2, 3, 4}, g1[4] = {0.1, -0.1, 0.2, 0}, a1[4] = {0}, a2[4] = {0};
    mhar_ref_adam(4, p1, g1, a1, a2, 1, 0.01, 0.9, 0.999, 1e-8);

    /* Dikin fit: Hessian, objective, one training step; a mean outside fails */
    double H[n * n], xbar[n], K;
    EXPECT(mhar_ref_dikin_hessian(n, m, A, b, z, Xs, xbar, H) == 0);
    EXPECT(mhar_ref_dikin_objective(n, r, U, ls, H, &K, gU, gl) == 0);
    double v[n] = {1, 0.5, 0.25}, lam;
    EXPECT(mhar_ref_dikin_train_step(n, m, A, b, z, Xs, r, U, ls, v, 4, 0.5, 0.3, &lam) == 0);
    double Xout[z * n];
    for (int e = 0; e < z * n; ++e) Xout[e] = 2.0;
    EXPECT(mhar_ref_dikin_hessian(n, m, A, b, z, Xout, xbar, H) != 0);

    printf("oracle driver: %d failed expectations\n", fails);
    return fails != 0;
}
