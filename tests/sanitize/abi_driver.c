/* Host sanitizer run of the C ABI's host logic (the library built with the
 * host code under -fsanitize=address,undefined): option defaults, status
 * strings, workspace sizes of problems, packed batches and covariances
 * over valid and invalid shapes, and the argument checks that return
 * before any device call.  No GPU is touched. */
#include <stdio.h>
#include <string.h>

#include "../../include/mhar.h"

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
    mhar_options_t o;
    EXPECT(mhar_options_default(&o) == MHAR_OK);
    EXPECT(mhar_version() >= 100);
    for (int s = -9; s <= 1; ++s) EXPECT(strlen(mhar_status_string(s)) > 0);
    size_t bytes = 0;
    for (int p = 0; p <= 2; ++p) {
        o.precision = p;
        EXPECT(mhar_problem_workspace_size(100, 2000, 0, &o, &bytes) == MHAR_OK && bytes > 0);
        EXPECT(mhar_problem_workspace_size(500, 5500, 5, &o, &bytes) == MHAR_OK);
        EXPECT(mhar_problem_workspace_size(0, 10, 0, &o, &bytes) != MHAR_OK);
        EXPECT(mhar_problem_workspace_size(10, 0, 0, &o, &bytes) != MHAR_OK);
        EXPECT(mhar_problem_workspace_size(10, 20, 10, &o, &bytes) != MHAR_OK);
    }
    EXPECT(strlen(mhar_last_error()) > 0);
    o.precision = 1;
    const int64_t n[3] = {20, 64, 400}, m[3] = {100, 600, 8000}, z[3] = {16, 130, 256};
    EXPECT(mhar_batch_packed_workspace_size(3, n, m, z, &o, &bytes) == MHAR_OK && bytes > 0);
    const int64_t bad_n[1] = {5000};
    EXPECT(mhar_batch_packed_workspace_size(1, bad_n, m, z, &o, &bytes) != MHAR_OK);
    EXPECT(mhar_batch_packed_workspace_size(0, n, m, z, &o, &bytes) != MHAR_OK);
    mhar_problem_t prob = NULL;
    EXPECT(mhar_problem_create(10, 20, NULL, NULL, 0, NULL, NULL, &o, NULL, 0, NULL, &prob) != MHAR_OK);
    mhar_chains_t ch = NULL;
    EXPECT(mhar_chains_create(NULL, 16, NULL, 0, 0, NULL, 0, NULL, &ch) != MHAR_OK);
    EXPECT(mhar_step(NULL, 1, NULL) != MHAR_OK);
    EXPECT(mhar_chains_set_graph(NULL, 50) != MHAR_OK);
    mhar_tune_t t;
    EXPECT(mhar_chains_autotune(NULL, 10, NULL, &t) != MHAR_OK);
    EXPECT(mhar_batch_get_chains(NULL, 0, &ch) != MHAR_OK);
    EXPECT(mhar_chains_destroy(NULL) == MHAR_OK && mhar_problem_destroy(NULL) == MHAR_OK);
    printf("abi driver: %d failed expectations\n", fails);
    return fails != 0;
}
