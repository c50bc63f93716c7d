/*
 * Host-side run of the C ABI under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (built by tests/test_sanitizers.py): every path that runs before
 * a HIP call -- workspace planning for many shapes (2D, 3D, deep halos,
 * batches), argument and handle checks, status strings, the depth query and
 * the allocation-free entry point's checks.  No GPU is touched.  Exits 0 if
 * every result is as documented in include/jacobi.h.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "jacobi.h"

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);    \
            return 1;                                                          \
        }                                                                      \
    } while (0)

static int plan_many(void) {
    static const int64_t sides[] = {1, 2, 7, 8, 9, 31, 33, 37, 100, 513, 1000};
    const int ns = (int)(sizeof(sides) / sizeof(sides[0]));
    for (int dt = 0; dt < 2; ++dt)
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; j += 2)
                for (int64_t bx = 1; bx <= 4; ++bx)
                    for (int64_t by = 1; by <= 3; ++by) {
                        int64_t g[3] = {sides[i], sides[j], sides[(i + j) % ns]};
                        int64_t b[3] = {bx, by, 2};
                        size_t bytes = 0;
                        int rc = jacobi_workspace_bytes(2, g, b, dt, &bytes);
                        CHECK(rc == JACOBI_OK || rc == JACOBI_E_INVAL);
                        CHECK(rc != JACOBI_OK || bytes > 0);
                        rc = jacobi_workspace_bytes(3, g, b, dt, &bytes);
                        CHECK(rc == JACOBI_OK || rc == JACOBI_E_INVAL);
                        for (int halo = 1; halo <= 14; halo += 3) {
                            rc = jacobi_deep_workspace_bytes(2, g, b, dt, halo, &bytes);
                            CHECK(rc == JACOBI_OK || rc == JACOBI_E_INVAL);
                            rc = jacobi_deep_workspace_bytes(3, g, b, dt, halo, &bytes);
                            CHECK(rc == JACOBI_OK || rc == JACOBI_E_INVAL);
                        }
                        if (rc != JACOBI_OK) (void)jacobi_last_error();
                    }
    return 0;
}

int main(void) {
    size_t bytes = 0;
    int64_t g2[2] = {8192, 8192}, b2[2] = {16, 16};
    CHECK(jacobi_workspace_bytes(2, g2, b2, JACOBI_F32, &bytes) == JACOBI_OK);
    CHECK(bytes >= (size_t)3 * 8192 * 8192 * 4);
    int64_t g3[3] = {512, 512, 512}, b3[3] = {8, 8, 8};
    CHECK(jacobi_workspace_bytes(3, g3, b3, JACOBI_F64, &bytes) == JACOBI_OK);
    CHECK(jacobi_deep_workspace_bytes(2, g2, b2, JACOBI_F32, 13, &bytes) == JACOBI_OK);
    CHECK(jacobi_deep_workspace_bytes(3, g3, b3, JACOBI_F32, 4, &bytes) == JACOBI_OK);

    /* rejected arguments */
    int64_t bad[2] = {0, 8}, one[2] = {1, 1};
    CHECK(jacobi_workspace_bytes(1, g2, b2, JACOBI_F32, &bytes) == JACOBI_E_INVAL);
    CHECK(jacobi_workspace_bytes(4, g2, b2, JACOBI_F32, &bytes) == JACOBI_E_INVAL);
    CHECK(jacobi_workspace_bytes(2, bad, one, JACOBI_F32, &bytes) == JACOBI_E_INVAL);
    CHECK(jacobi_workspace_bytes(2, g2, b2, 7, &bytes) == JACOBI_E_INVAL);
    CHECK(jacobi_workspace_bytes(2, NULL, NULL, JACOBI_F32, NULL) == JACOBI_E_INVAL);
    CHECK(strlen(jacobi_last_error()) > 0);
    int64_t huge[2] = {INT64_C(1) << 40, INT64_C(1) << 40};
    CHECK(jacobi_workspace_bytes(2, huge, one, JACOBI_F64, &bytes) == JACOBI_E_INVAL);
    int64_t small[2] = {37, 29}, sb[2] = {3, 4};
    CHECK(jacobi_deep_workspace_bytes(2, small, sb, JACOBI_F32, 13, &bytes) == JACOBI_E_INVAL);
    CHECK(jacobi_deep_workspace_bytes(2, g2, b2, JACOBI_F32, 0, &bytes) == JACOBI_E_INVAL);
    if (plan_many()) return 1;

    /* handles: NULL workspace, misaligned or too small workspace, NULL handle */
    jacobi_t h = NULL;
    int64_t g8[2] = {8, 8};
    CHECK(jacobi_create(2, g8, one, JACOBI_F32, NULL, 1 << 20, NULL, &h) == JACOBI_E_INVAL);
    CHECK(h == NULL);
    CHECK(jacobi_create(2, g8, one, JACOBI_F32, (void *)16, (size_t)1 << 30, NULL, &h) ==
          JACOBI_E_INVAL);
    CHECK(jacobi_create(2, g8, one, JACOBI_F32, (void *)256, 16, NULL, &h) == JACOBI_E_NOMEM);
    CHECK(jacobi_deep_create(2, g8, one, JACOBI_F32, 3, NULL, 1 << 20, NULL, &h) ==
          JACOBI_E_INVAL);
    CHECK(jacobi_sweep(NULL, 1) == JACOBI_E_INVAL);
    CHECK(jacobi_halo_exchange(NULL) == JACOBI_E_INVAL);
    CHECK(jacobi_solve(NULL, 1, 1, NULL) == JACOBI_E_INVAL);
    CHECK(jacobi_set_tuning(NULL, 1, 1, 0) == JACOBI_E_INVAL);
    int halo = -1;
    CHECK(jacobi_get_halo(NULL, &halo) == JACOBI_E_INVAL);
    CHECK(jacobi_destroy(NULL) == JACOBI_OK);

    /* batches */
    int64_t grids[6] = {300, 200, 17, 9, 1000, 1000};
    CHECK(jacobi_batch_workspace_bytes(3, grids, 64, JACOBI_F32, &bytes) == JACOBI_OK);
    CHECK(bytes > 0);
    CHECK(jacobi_batch_workspace_bytes(0, grids, 64, JACOBI_F32, &bytes) == JACOBI_E_INVAL);
    CHECK(jacobi_batch_workspace_bytes(3, NULL, 64, JACOBI_F32, &bytes) == JACOBI_E_INVAL);
    CHECK(jacobi_batch_workspace_bytes(3, grids, 2, JACOBI_F32, &bytes) == JACOBI_E_INVAL);
    jacobi_batch_t bt = NULL;
    CHECK(jacobi_batch_create(3, grids, 64, JACOBI_F32, NULL, 1 << 20, NULL, &bt) ==
          JACOBI_E_INVAL);
    CHECK(jacobi_batch_destroy(NULL) == JACOBI_OK);

    /* the allocation-free entry point checks its arguments first */
    const void *p = (const void *)256;
    int64_t g64[2] = {64, 64}, b22[2] = {2, 2};
    CHECK(jacobi_solve_noalloc(2, g64, b22, 0, NULL, p, 1e-4, 10, 5, (void *)p, (double *)p,
                               NULL) == JACOBI_E_INVAL);
    CHECK(jacobi_solve_noalloc(2, g64, b22, 0, p, p, 1e-4, -1, 5, (void *)p, (double *)p,
                               NULL) == JACOBI_E_INVAL);
    int64_t g4k[2] = {4096, 4096}, b88[2] = {8, 8};
    CHECK(jacobi_solve_noalloc(2, g4k, b88, 0, p, p, 1e-4, 10, 5, (void *)p, (double *)p,
                               NULL) == JACOBI_E_NOMEM);

    /* status strings and the depth query */
    for (int s = -8; s <= 2; ++s) CHECK(jacobi_strerror(s) != NULL);
    CHECK(jacobi_max_depth(2, JACOBI_F32) >= 13);
    CHECK(jacobi_max_depth(3, JACOBI_F64) >= 1);
    CHECK(jacobi_max_depth(5, JACOBI_F32) == JACOBI_E_INVAL);
    printf("abi sanitize check: ok\n");
    return 0;
}
