/*
 * The oracle (oracle/jacobi_oracle.c, test infrastructure) run under
 * AddressSanitizer and UndefinedBehaviorSanitizer (built by
 * tests/test_sanitizers.py): every entry point on small ragged grids, in FP64
 * and FP32, with and without a source, with block partitions that include
 * one-node blocks.  Exits 0 if every call succeeds and the block-decomposed
 * and windowed sweeps equal the monolithic one bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define DECL(R, S)                                                                          \
    void orc_scale_source_##S(int64_t, double, const R *, R *);                             \
    int orc_sweep2d_##S(int64_t, int64_t, const R *, R *, int64_t);                         \
    int orc_sweep3d_##S(int64_t, int64_t, int64_t, const R *, R *, int64_t);                \
    int orc_blocked_sweep2d_##S(int64_t, int64_t, int64_t, const int64_t *, int64_t,        \
                                const int64_t *, const R *, R *, int64_t);                  \
    int orc_blocked_sweep3d_##S(int64_t, int64_t, int64_t, int64_t, const int64_t *,        \
                                int64_t, const int64_t *, int64_t, const int64_t *,         \
                                const R *, R *, int64_t);                                   \
    double orc_residual2d_##S(int64_t, int64_t, const R *, const R *);                      \
    double orc_residual3d_##S(int64_t, int64_t, int64_t, const R *, const R *);             \
    int orc_window2d_##S(int64_t, int64_t, const R *, const R *, int64_t, int64_t, int64_t, \
                         int64_t, int64_t, R *);                                            \
    int orc_window3d_##S(int64_t, int64_t, int64_t, const R *, const R *, int64_t, int64_t, \
                         int64_t, int64_t, int64_t, int64_t, int64_t, R *);
DECL(double, f64)
DECL(float, f32)
int orc_adjoint2d_f64(int64_t, int64_t, int64_t, const double *, double *, double *, double *);
void orc_set_num_threads(int);

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

static uint64_t rng = 88172645463325252ull;
static double urand(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0;
}

#define BODY(R, S)                                                                         \
    static int check_##S(int64_t nx, int64_t ny, int64_t nz, int64_t K, int src) {         \
        const size_t n2 = (size_t)(nx + 2) * (ny + 2), n3 = n2 * (nz + 2);                 \
        R *u = malloc(n3 * sizeof(R)), *v = malloc(n3 * sizeof(R)),                        \
          *f = malloc((size_t)nx * ny * nz * sizeof(R)), *b = malloc((size_t)nx * ny * nz * sizeof(R)); \
        CHECK(u && v && f && b);                                                           \
        for (size_t i = 0; i < n3; ++i) u[i] = (R)urand();                                 \
        for (int64_t i = 0; i < nx * ny * nz; ++i) f[i] = (R)(urand() - 0.5);              \
        orc_scale_source_##S(nx * ny * nz, 1e-3, f, b);                                    \
        const R *bb = src ? b : NULL;                                                      \
        int64_t xs[4] = {0, nx / 3, (2 * nx) / 3, nx}, ys[3] = {0, ny / 2, ny},            \
                zs[3] = {0, nz - 1 > 0 ? nz - 1 : 0, nz};                                  \
        int nbx = nx >= 3 ? 3 : 1, nby = ny >= 2 ? 2 : 1, nbz = nz >= 2 ? 2 : 1;           \
        if (nbx == 1) xs[1] = nx;                                                          \
        if (nby == 1) ys[1] = ny;                                                          \
        if (nbz == 1) zs[1] = nz;                                                          \
        /* 2D on the first plane layout */                                                 \
        memcpy(v, u, n2 * sizeof(R));                                                      \
        CHECK(orc_sweep2d_##S(nx, ny, bb, v, K) == 0);                                     \
        R *w = malloc(n2 * sizeof(R));                                                     \
        CHECK(w != NULL);                                                                  \
        memcpy(w, u, n2 * sizeof(R));                                                      \
        CHECK(orc_blocked_sweep2d_##S(nx, ny, nbx, xs, nby, ys, bb, w, K) == 0);           \
        CHECK(memcmp(v, w, n2 * sizeof(R)) == 0);                                          \
        R *win = malloc((size_t)nx * ny * sizeof(R));                                      \
        CHECK(win != NULL);                                                                \
        CHECK(orc_window2d_##S(nx, ny, bb, u, K, 0, nx, 0, ny, win) == 0);                 \
        for (int64_t j = 0; j < ny; ++j)                                                   \
            CHECK(memcmp(&win[j * nx], &v[(j + 1) * (nx + 2) + 1], nx * sizeof(R)) == 0); \
        CHECK(isfinite(orc_residual2d_##S(nx, ny, bb, v)));                                \
        /* 3D */                                                                           \
        memcpy(v, u, n3 * sizeof(R));                                                      \
        CHECK(orc_sweep3d_##S(nx, ny, nz, bb, v, K) == 0);                                 \
        R *w3 = malloc(n3 * sizeof(R));                                                    \
        CHECK(w3 != NULL);                                                                 \
        memcpy(w3, u, n3 * sizeof(R));                                                     \
        CHECK(orc_blocked_sweep3d_##S(nx, ny, nz, nbx, xs, nby, ys, nbz, zs, bb, w3, K) == 0); \
        CHECK(memcmp(v, w3, n3 * sizeof(R)) == 0);                                         \
        R *win3 = malloc((size_t)nx * ny * nz * sizeof(R));                                \
        CHECK(win3 != NULL);                                                               \
        CHECK(orc_window3d_##S(nx, ny, nz, bb, u, K, 0, nx, 0, ny, 0, nz, win3) == 0);     \
        for (int64_t k = 0; k < nz; ++k)                                                   \
            for (int64_t j = 0; j < ny; ++j)                                               \
                CHECK(memcmp(&win3[(k * ny + j) * nx],                                     \
                             &v[((k + 1) * (ny + 2) + j + 1) * (nx + 2) + 1], nx * sizeof(R)) == 0); \
        CHECK(isfinite(orc_residual3d_##S(nx, ny, nz, bb, v)));                            \
        free(u); free(v); free(f); free(b); free(w); free(win); free(w3); free(win3);      \
        return 0;                                                                          \
    }
BODY(double, f64)
BODY(float, f32)

int main(void) {
    static const int64_t shapes[][4] = {{1, 1, 1, 3}, {2, 5, 3, 4}, {7, 3, 2, 5}, {13, 9, 11, 6},
                                        {31, 17, 4, 2}, {64, 33, 5, 9}};
    for (int t = 1; t <= 2; ++t) {
        orc_set_num_threads(t);
        for (size_t i = 0; i < sizeof(shapes) / sizeof(shapes[0]); ++i)
            for (int src = 0; src <= 1; ++src) {
                const int64_t *s = shapes[i];
                if (check_f64(s[0], s[1], s[2], s[3], src)) return 1;
                if (check_f32(s[0], s[1], s[2], s[3], src)) return 1;
            }
    }
    /* the adjoint on a ragged grid */
    const int64_t nx = 11, ny = 7;
    double lam[77], Gb[77], lam0[77], Gring[13 * 9];
    for (int i = 0; i < 77; ++i) lam[i] = urand() - 0.5;
    CHECK(orc_adjoint2d_f64(nx, ny, 9, lam, Gb, Gring, lam0) == 0);
    for (int i = 0; i < 77; ++i) CHECK(isfinite(Gb[i]) && isfinite(lam0[i]));
    printf("oracle sanitize check: ok\n");
    return 0;
}
