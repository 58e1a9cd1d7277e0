/*
 * A plain C99 client of include/pprviz.h: compiles the header as C, links
 * libpprviz.so and calls the entry points whose work is host-only (version,
 * status strings, the push count, workspace queries, argument validation).
 * Built and run by tests/test_abi.py; no GPU work is launched.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "pprviz.h"

static int failures = 0;

#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                               \
        }                                                             \
    } while (0)

int main(void) {
    const char* v = pprviz_version();
    CHECK(v != NULL && strlen(v) > 0);
    CHECK(strcmp(pprviz_status_string(PPR_EINVAL), "invalid argument") == 0);

    int32_t T = 0, conv = 0;
    CHECK(pprviz_pushes_for_tolerance(0.15f, 1e-6, 1000, &T, &conv) == PPR_OK);
    CHECK(T == 86 && conv == 1);
    CHECK(pprviz_pushes_for_tolerance(0.15f, 1e-10, 100, &T, &conv) == PPR_OK);
    CHECK(T == 100 && conv == 0);
    CHECK(pprviz_pushes_for_tolerance(1.5f, 1e-6, 100, &T, &conv) == PPR_EINVAL);

    /* fake device pointers: every call below returns before touching them */
    int32_t dummy_i[4];
    float dummy_f[4];
    ppr_csr g;
    g.n = 100;
    g.nnz = 400;
    g.row_ptr = dummy_i;
    g.col_idx = dummy_i;
    g.weight = NULL;
    CHECK(ppr_matrix_workspace(&g, 100, 100) > 0);
    CHECK(ppr_matrix(NULL, NULL, 0, NULL, 0, 0.15f, 1e-6, 10, NULL, NULL, NULL, NULL, NULL, 0, NULL) ==
          PPR_EINVAL);
    CHECK(gfp_workspace(&g, 25, 100) > 0);
    CHECK(gfp_level_dppr(&g, NULL, dummy_i, 3, 10, 0.15f, 1e-6, 100, dummy_f, NULL, NULL, NULL, dummy_f, 1 << 20,
                         NULL) == PPR_EINVAL);
    CHECK(tau_push_level_dppr(&g, dummy_i, dummy_i, 3, 10, 0.15f, 0.0, 0.1, 0.0, 100, dummy_f, NULL, NULL,
                              dummy_f, 1 << 20, NULL) == PPR_EINVAL);
    CHECK(layout_exact_workspace(4096) > 0);
    CHECK(layout_step_exact(dummy_f, 4, dummy_f, dummy_f, 1e-6, 10, NULL, dummy_f, 1 << 20, NULL) == PPR_EINVAL);
    CHECK(layout_metrics(dummy_f, 4, NULL, NULL, NULL, dummy_f, 1 << 20, NULL) == PPR_EINVAL);
    CHECK(pprviz_batch_max_n() == 2304);

    if (failures == 0) printf("c abi ok: %s\n", v);
    return failures == 0 ? 0 : 1;
}
