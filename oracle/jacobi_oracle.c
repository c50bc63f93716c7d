/*
 * CPU oracle for the over-decomposed Jacobi sweep of the paper's Jacobi3D
 * proxy application (Section 4.3, Proxy Application: Jacobi3D; Section 4.4,
 * Over-decomposition).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is what the device path is checked
 * against; only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, table or helper with the
 * device library, and the device library never calls it.
 *
 * Plain and slow on purpose: FP64 loops written straight from the definitions
 * (an FP32 twin of the sweep exists only so FP32 device runs can be compared
 * bit for bit).  Build flags: -O2 -ffp-contract=off, no fast-math, so every
 * operation is one IEEE round-to-nearest step in the order written.  OpenMP
 * parallelises only loops whose iterations are independent; reductions are
 * summed serially in index order, so results do not depend on thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REAL double
#define SUF f64
#include "jacobi_oracle_body.h"
#undef REAL
#undef SUF

#define REAL float
#define SUF f32
#include "jacobi_oracle_body.h"
#undef REAL
#undef SUF

/* Threads an OpenMP region of the oracle uses. */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* Set the threads of later OpenMP regions (results never depend on it). */
void orc_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/*
 * Reverse-mode derivative of L = 1/2 * sum_interior (u_K - t)^2 through K
 * sweeps of the 2D iteration (not in the paper; the differentiable form of the
 * sweep).  In exact arithmetic one sweep is the affine map
 *     u_k = w * (S u_{k-1} + B g + b),   w = 1/4,
 * where S sums the four neighbours with a zero ring (a symmetric operator) and
 * B moves each ring value g_q into the single interior node p(q) next to it
 * (the four corner nodes touch no interior node).  With lam_K = u_K - t the
 * adjoint recurrence, for k = K down to 1, is
 *     Gb    += w * lam_k                  (dL/db; dL/df = h^2 dL/db)
 *     Gg[q] += w * lam_k[p(q)]            for every non-corner ring node q
 *     lam_{k-1} = w * S lam_k             (zero ring, no source),
 * and dL/du_0 = lam_0.  The recurrence needs no forward state but u_K, which
 * the caller folds into lamK.
 *
 *   lamK   nx*ny interior values of u_K - t (x fastest)
 *   Gb     nx*ny out, dL/db
 *   Gring  (nx+2)*(ny+2) out: dL/dg on non-corner ring nodes, zero elsewhere
 *   lam0   nx*ny out, dL/du_0 on the interior
 * Every operation is FP64, accumulated in the order k = K, ..., 1.
 */
int orc_adjoint2d_f64(int64_t nx, int64_t ny, int64_t K, const double *lamK,
                      double *Gb, double *Gring, double *lam0)
{
    const int64_t ld = nx + 2;
    const size_t cnt = (size_t)(nx + 2) * (size_t)(ny + 2);
    double *lam = (double *)calloc(cnt, sizeof(double)); /* zero ring */
    double *nxt = (double *)calloc(cnt, sizeof(double));
    if (!lam || !nxt) { free(lam); free(nxt); return -1; }
    for (int64_t j = 1; j <= ny; ++j)
        for (int64_t i = 1; i <= nx; ++i) lam[j * ld + i] = lamK[(j - 1) * nx + (i - 1)];
    memset(Gb, 0, (size_t)(nx * ny) * sizeof(double));
    memset(Gring, 0, cnt * sizeof(double));
    const double w = 0.25;
    for (int64_t k = K; k >= 1; --k) {
        /* cells are independent; each cell still adds its terms in k order */
#pragma omp parallel for schedule(static)
        for (int64_t j = 1; j <= ny; ++j)
            for (int64_t i = 1; i <= nx; ++i) Gb[(j - 1) * nx + (i - 1)] += w * lam[j * ld + i];
        for (int64_t i = 1; i <= nx; ++i) {
            Gring[0 * ld + i] += w * lam[1 * ld + i];                 /* south edge */
            Gring[(ny + 1) * ld + i] += w * lam[ny * ld + i];         /* north edge */
        }
        for (int64_t j = 1; j <= ny; ++j) {
            Gring[j * ld + 0] += w * lam[j * ld + 1];                 /* west edge  */
            Gring[j * ld + nx + 1] += w * lam[j * ld + nx];           /* east edge  */
        }
#pragma omp parallel for schedule(static)
        for (int64_t j = 1; j <= ny; ++j)
            for (int64_t i = 1; i <= nx; ++i) {
                const int64_t c = j * ld + i;
                nxt[c] = ((lam[c - 1] + lam[c + 1]) + (lam[c - ld] + lam[c + ld])) * w;
            }
        double *t = lam; lam = nxt; nxt = t;
    }
    for (int64_t j = 1; j <= ny; ++j)
        for (int64_t i = 1; i <= nx; ++i) lam0[(j - 1) * nx + (i - 1)] = lam[j * ld + i];
    free(lam); free(nxt);
    return 0;
}
