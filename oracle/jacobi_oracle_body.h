/*
 * Precision-generic body of the CPU oracle for the over-decomposed Jacobi
 * sweep.  jacobi_oracle.c includes this file twice: once with REAL = double
 * (suffix f64, the oracle proper) and once with REAL = float (suffix f32, used
 * only to check FP32 device runs bit for bit, since every cell update is a
 * fixed sequence of IEEE operations).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call it.
 *
 * Notation (shared with the Python wrapper in oracle/__init__.py):
 *   nx, ny, nz   interior nodes per axis; node indices run 0 .. n+1 and the
 *                outer ring (index 0 or n+1 on any axis) holds the Dirichlet
 *                boundary values, which no sweep ever changes.
 *   u            state array over all nodes, x fastest: 2D u[j][i], 3D u[k][j][i].
 *   b            scaled source h^2 f over interior nodes only (n^d values,
 *                x fastest), or NULL for the Laplace equation (b = 0).
 *
 * The method is the Jacobi iteration of the proxy application in Section 4.3
 * (Proxy Application: Jacobi3D) of the paper: a fixed number of synchronous
 * Jacobi updates of a 3D (here also 2D) domain.  The paper states no stencil,
 * weights or arithmetic order, so the textbook 5-point / 7-point Jacobi update
 * for -Laplace(u) = f on the unit square / cube is used, with this fixed
 * operation order and no fused multiply-add:
 *   2D  s = (u[W] + u[E]) + (u[S] + u[N]);             u'[c] = (s + b[c]) * 1/4
 *   3D  s = ((u[W] + u[E]) + (u[S] + u[N])) + (u[B] + u[F]);
 *                                                       u'[c] = (s + b[c]) * fl(1/6)
 * (Laplace: u'[c] = s * w.)
 */

#define ORC_CAT_(a, b) a##_##b
#define ORC_CAT(a, b) ORC_CAT_(a, b)
#define FN(name) ORC_CAT(name, SUF)

/* Source scaling: b[c] = fl_REAL(fl64(h^2) * f[c]), product in FP64 and one
 * rounding to the run type. */
void FN(orc_scale_source)(int64_t count, double h2, const REAL *f, REAL *b)
{
    for (int64_t c = 0; c < count; ++c)
        b[c] = (REAL)(h2 * (double)f[c]);
}

/* One synchronous 5-point sweep over an ex x ey rectangle of interior nodes.
 * u, v point at node (0, 0) of an array whose rows are ldu apart; the nodes of
 * the rectangle are (1..ex, 1..ey).  b points at the source of node (1, 1)
 * with rows ldb apart (or NULL).  v receives the new interior; nothing else in
 * v is touched. */
static void FN(sweep2d_rect)(int64_t ex, int64_t ey, const REAL *b, int64_t ldb,
                             const REAL *u, REAL *v, int64_t ldu)
{
    const REAL w = (REAL)0.25;
#pragma omp parallel for schedule(static)
    for (int64_t j = 1; j <= ey; ++j) {
        for (int64_t i = 1; i <= ex; ++i) {
            const int64_t c = j * ldu + i;
            const REAL s = (u[c - 1] + u[c + 1]) + (u[c - ldu] + u[c + ldu]);
            v[c] = b ? (s + b[(j - 1) * ldb + (i - 1)]) * w : s * w;
        }
    }
}

/* Same for the 7-point stencil over ex x ey x ez nodes; planes are ldp apart. */
static void FN(sweep3d_rect)(int64_t ex, int64_t ey, int64_t ez, const REAL *b,
                             int64_t ldb, int64_t ldbp, const REAL *u, REAL *v,
                             int64_t ldu, int64_t ldp)
{
    const REAL w = (REAL)1 / (REAL)6;
#pragma omp parallel for schedule(static) collapse(2)
    for (int64_t k = 1; k <= ez; ++k) {
        for (int64_t j = 1; j <= ey; ++j) {
            for (int64_t i = 1; i <= ex; ++i) {
                const int64_t c = k * ldp + j * ldu + i;
                const REAL s = ((u[c - 1] + u[c + 1]) + (u[c - ldu] + u[c + ldu])) +
                               (u[c - ldp] + u[c + ldp]);
                v[c] = b ? (s + b[(k - 1) * ldbp + (j - 1) * ldb + (i - 1)]) * w : s * w;
            }
        }
    }
}

/* K synchronous sweeps of the monolithic 2D grid; the result replaces u. */
int FN(orc_sweep2d)(int64_t nx, int64_t ny, const REAL *b, REAL *u, int64_t K)
{
    const size_t count = (size_t)(nx + 2) * (size_t)(ny + 2);
    REAL *v = (REAL *)malloc(count * sizeof(REAL));
    if (!v) return -1;
    memcpy(v, u, count * sizeof(REAL)); /* the ring of v equals that of u */
    REAL *cur = u, *nxt = v;
    for (int64_t k = 0; k < K; ++k) {
        FN(sweep2d_rect)(nx, ny, b, nx, cur, nxt, nx + 2);
        REAL *t = cur; cur = nxt; nxt = t;
    }
    if (cur != u) memcpy(u, cur, count * sizeof(REAL));
    free(v);
    return 0;
}

/* K synchronous sweeps of the monolithic 3D grid; the result replaces u. */
int FN(orc_sweep3d)(int64_t nx, int64_t ny, int64_t nz, const REAL *b, REAL *u, int64_t K)
{
    const size_t count = (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(nz + 2);
    REAL *v = (REAL *)malloc(count * sizeof(REAL));
    if (!v) return -1;
    memcpy(v, u, count * sizeof(REAL));
    REAL *cur = u, *nxt = v;
    for (int64_t k = 0; k < K; ++k) {
        FN(sweep3d_rect)(nx, ny, nz, b, nx, nx * ny, cur, nxt, nx + 2, (nx + 2) * (ny + 2));
        REAL *t = cur; cur = nxt; nxt = t;
    }
    if (cur != u) memcpy(u, cur, count * sizeof(REAL));
    free(v);
    return 0;
}

/*
 * Block-decomposed form (Section 4.3: the domain is cut into cuboids; every
 * iteration each block receives the edge cells of its face neighbours into a
 * one-cell halo, and the update runs once all halos are in; Section 4.4 and
 * the caption of the over-decomposition timeline figure: one halo buffer per
 * face).  Block (p, q) owns interior nodes xs[p] .. xs[p+1]-1 by
 * ys[q] .. ys[q+1]-1 (0-based interior coordinates; xs[0] = 0, xs[nbx] = nx,
 * strictly increasing) and stores (ex+2) x (ey+2) values: its interior plus a
 * one-cell halo ring.  Halo cells on the domain boundary hold the Dirichlet
 * values; the others are refreshed from the neighbour before every sweep.
 * Corner halo cells are never read by the 5-point stencil.  The result
 * replaces u and must equal orc_sweep2d bit for bit.
 */
int FN(orc_blocked_sweep2d)(int64_t nx, int64_t ny, int64_t nbx, const int64_t *xs,
                            int64_t nby, const int64_t *ys, const REAL *b, REAL *u,
                            int64_t K)
{
    const int64_t nb = nbx * nby;
    REAL **cur = (REAL **)calloc((size_t)nb, sizeof(REAL *));
    REAL **nxt = (REAL **)calloc((size_t)nb, sizeof(REAL *));
    int rc = 0;
    if (!cur || !nxt) { rc = -1; goto done; }
    for (int64_t q = 0; q < nby; ++q) {
        for (int64_t p = 0; p < nbx; ++p) {
            const int64_t ex = xs[p + 1] - xs[p], ey = ys[q + 1] - ys[q];
            const size_t cnt = (size_t)(ex + 2) * (size_t)(ey + 2);
            REAL *a = (REAL *)malloc(cnt * sizeof(REAL));
            REAL *c = (REAL *)malloc(cnt * sizeof(REAL));
            cur[q * nbx + p] = a; nxt[q * nbx + p] = c;
            if (!a || !c) { rc = -1; goto done; }
            /* scatter: block node (li, lj) is global node (xs[p]+li, ys[q]+lj),
             * halo included (domain-edge halos take the ring values) */
            for (int64_t lj = 0; lj < ey + 2; ++lj)
                for (int64_t li = 0; li < ex + 2; ++li)
                    a[lj * (ex + 2) + li] = u[(ys[q] + lj) * (nx + 2) + (xs[p] + li)];
            memcpy(c, a, cnt * sizeof(REAL));
        }
    }
    for (int64_t k = 0; k < K; ++k) {
        /* halo exchange: each internal face halo <- neighbour's edge interior */
        for (int64_t q = 0; q < nby; ++q) {
            for (int64_t p = 0; p < nbx; ++p) {
                const int64_t ex = xs[p + 1] - xs[p], ey = ys[q + 1] - ys[q];
                const int64_t ld = ex + 2;
                REAL *me = cur[q * nbx + p];
                if (p > 0) { /* west halo column <- east edge column of (p-1, q) */
                    const REAL *nb_ = cur[q * nbx + p - 1];
                    const int64_t nex = xs[p] - xs[p - 1], nld = nex + 2;
                    for (int64_t lj = 1; lj <= ey; ++lj) me[lj * ld + 0] = nb_[lj * nld + nex];
                }
                if (p + 1 < nbx) { /* east halo column <- west edge column of (p+1, q) */
                    const REAL *nb_ = cur[q * nbx + p + 1];
                    const int64_t nld = (xs[p + 2] - xs[p + 1]) + 2;
                    for (int64_t lj = 1; lj <= ey; ++lj) me[lj * ld + ex + 1] = nb_[lj * nld + 1];
                }
                if (q > 0) { /* south halo row <- north edge row of (p, q-1) */
                    const REAL *nb_ = cur[(q - 1) * nbx + p];
                    const int64_t ney = ys[q] - ys[q - 1];
                    for (int64_t li = 1; li <= ex; ++li) me[0 * ld + li] = nb_[ney * ld + li];
                }
                if (q + 1 < nby) { /* north halo row <- south edge row of (p, q+1) */
                    const REAL *nb_ = cur[(q + 1) * nbx + p];
                    for (int64_t li = 1; li <= ex; ++li) me[(ey + 1) * ld + li] = nb_[1 * ld + li];
                }
            }
        }
        /* update every block from its own storage only */
        for (int64_t q = 0; q < nby; ++q) {
            for (int64_t p = 0; p < nbx; ++p) {
                const int64_t ex = xs[p + 1] - xs[p], ey = ys[q + 1] - ys[q];
                const REAL *bb = b ? b + ys[q] * nx + xs[p] : NULL;
                FN(sweep2d_rect)(ex, ey, bb, nx, cur[q * nbx + p], nxt[q * nbx + p], ex + 2);
            }
        }
        REAL **t = cur; cur = nxt; nxt = t;
    }
    /* gather the interiors; the ring of u is unchanged */
    for (int64_t q = 0; q < nby; ++q) {
        for (int64_t p = 0; p < nbx; ++p) {
            const int64_t ex = xs[p + 1] - xs[p], ey = ys[q + 1] - ys[q];
            const REAL *a = cur[q * nbx + p];
            for (int64_t lj = 1; lj <= ey; ++lj)
                for (int64_t li = 1; li <= ex; ++li)
                    u[(ys[q] + lj) * (nx + 2) + (xs[p] + li)] = a[lj * (ex + 2) + li];
        }
    }
done:
    if (cur) for (int64_t i = 0; i < nb; ++i) free(cur[i]);
    if (nxt) for (int64_t i = 0; i < nb; ++i) free(nxt[i]);
    free(cur); free(nxt);
    return rc;
}

/* 3D block-decomposed form: six face halos per cuboid (left, right, bottom,
 * top, back, front), otherwise as orc_blocked_sweep2d.  Edge and corner halo
 * cells are never read by the 7-point stencil. */
int FN(orc_blocked_sweep3d)(int64_t nx, int64_t ny, int64_t nz, int64_t nbx, const int64_t *xs,
                            int64_t nby, const int64_t *ys, int64_t nbz, const int64_t *zs,
                            const REAL *b, REAL *u, int64_t K)
{
    const int64_t nb = nbx * nby * nbz;
    const int64_t gx = nx + 2, gp = (nx + 2) * (ny + 2);
    REAL **cur = (REAL **)calloc((size_t)nb, sizeof(REAL *));
    REAL **nxt = (REAL **)calloc((size_t)nb, sizeof(REAL *));
    int rc = 0;
#define BID(p, q, r) (((r) * nby + (q)) * nbx + (p))
    if (!cur || !nxt) { rc = -1; goto done3; }
    for (int64_t r = 0; r < nbz; ++r)
        for (int64_t q = 0; q < nby; ++q)
            for (int64_t p = 0; p < nbx; ++p) {
                const int64_t ex = xs[p + 1] - xs[p], ey = ys[q + 1] - ys[q], ez = zs[r + 1] - zs[r];
                const int64_t ld = ex + 2, lp = (ex + 2) * (ey + 2);
                const size_t cnt = (size_t)lp * (size_t)(ez + 2);
                REAL *a = (REAL *)malloc(cnt * sizeof(REAL));
                REAL *c = (REAL *)malloc(cnt * sizeof(REAL));
                cur[BID(p, q, r)] = a; nxt[BID(p, q, r)] = c;
                if (!a || !c) { rc = -1; goto done3; }
                for (int64_t lk = 0; lk < ez + 2; ++lk)
                    for (int64_t lj = 0; lj < ey + 2; ++lj)
                        for (int64_t li = 0; li < ex + 2; ++li)
                            a[lk * lp + lj * ld + li] =
                                u[(zs[r] + lk) * gp + (ys[q] + lj) * gx + (xs[p] + li)];
                memcpy(c, a, cnt * sizeof(REAL));
            }
    for (int64_t k = 0; k < K; ++k) {
        for (int64_t r = 0; r < nbz; ++r)
            for (int64_t q = 0; q < nby; ++q)
                for (int64_t p = 0; p < nbx; ++p) {
                    const int64_t ex = xs[p + 1] - xs[p], ey = ys[q + 1] - ys[q], ez = zs[r + 1] - zs[r];
                    const int64_t ld = ex + 2, lp = (ex + 2) * (ey + 2);
                    REAL *me = cur[BID(p, q, r)];
                    if (p > 0) { /* left face <- right edge of (p-1) */
                        const REAL *o = cur[BID(p - 1, q, r)];
                        const int64_t oex = xs[p] - xs[p - 1], old_ = oex + 2, olp = old_ * (ey + 2);
                        for (int64_t lk = 1; lk <= ez; ++lk)
                            for (int64_t lj = 1; lj <= ey; ++lj)
                                me[lk * lp + lj * ld + 0] = o[lk * olp + lj * old_ + oex];
                    }
                    if (p + 1 < nbx) { /* right face <- left edge of (p+1) */
                        const REAL *o = cur[BID(p + 1, q, r)];
                        const int64_t oex = xs[p + 2] - xs[p + 1], old_ = oex + 2, olp = old_ * (ey + 2);
                        for (int64_t lk = 1; lk <= ez; ++lk)
                            for (int64_t lj = 1; lj <= ey; ++lj)
                                me[lk * lp + lj * ld + ex + 1] = o[lk * olp + lj * old_ + 1];
                    }
                    if (q > 0) { /* bottom face <- top edge of (q-1) */
                        const REAL *o = cur[BID(p, q - 1, r)];
                        const int64_t oey = ys[q] - ys[q - 1], olp = ld * (oey + 2);
                        for (int64_t lk = 1; lk <= ez; ++lk)
                            for (int64_t li = 1; li <= ex; ++li)
                                me[lk * lp + 0 * ld + li] = o[lk * olp + oey * ld + li];
                    }
                    if (q + 1 < nby) { /* top face <- bottom edge of (q+1) */
                        const REAL *o = cur[BID(p, q + 1, r)];
                        const int64_t oey = ys[q + 2] - ys[q + 1], olp = ld * (oey + 2);
                        for (int64_t lk = 1; lk <= ez; ++lk)
                            for (int64_t li = 1; li <= ex; ++li)
                                me[lk * lp + (ey + 1) * ld + li] = o[lk * olp + 1 * ld + li];
                    }
                    if (r > 0) { /* back face <- front edge of (r-1) */
                        const REAL *o = cur[BID(p, q, r - 1)];
                        const int64_t oez = zs[r] - zs[r - 1];
                        for (int64_t lj = 1; lj <= ey; ++lj)
                            for (int64_t li = 1; li <= ex; ++li)
                                me[0 * lp + lj * ld + li] = o[oez * lp + lj * ld + li];
                    }
                    if (r + 1 < nbz) { /* front face <- back edge of (r+1) */
                        const REAL *o = cur[BID(p, q, r + 1)];
                        for (int64_t lj = 1; lj <= ey; ++lj)
                            for (int64_t li = 1; li <= ex; ++li)
                                me[(ez + 1) * lp + lj * ld + li] = o[1 * lp + lj * ld + li];
                    }
                }
        for (int64_t r = 0; r < nbz; ++r)
            for (int64_t q = 0; q < nby; ++q)
                for (int64_t p = 0; p < nbx; ++p) {
                    const int64_t ex = xs[p + 1] - xs[p], ey = ys[q + 1] - ys[q], ez = zs[r + 1] - zs[r];
                    const REAL *bb = b ? b + (zs[r] * ny + ys[q]) * nx + xs[p] : NULL;
                    FN(sweep3d_rect)(ex, ey, ez, bb, nx, nx * ny, cur[BID(p, q, r)],
                                     nxt[BID(p, q, r)], ex + 2, (ex + 2) * (ey + 2));
                }
        REAL **t = cur; cur = nxt; nxt = t;
    }
    for (int64_t r = 0; r < nbz; ++r)
        for (int64_t q = 0; q < nby; ++q)
            for (int64_t p = 0; p < nbx; ++p) {
                const int64_t ex = xs[p + 1] - xs[p], ey = ys[q + 1] - ys[q], ez = zs[r + 1] - zs[r];
                const int64_t ld = ex + 2, lp = (ex + 2) * (ey + 2);
                const REAL *a = cur[BID(p, q, r)];
                for (int64_t lk = 1; lk <= ez; ++lk)
                    for (int64_t lj = 1; lj <= ey; ++lj)
                        for (int64_t li = 1; li <= ex; ++li)
                            u[(zs[r] + lk) * gp + (ys[q] + lj) * gx + (xs[p] + li)] =
                                a[lk * lp + lj * ld + li];
            }
#undef BID
done3:
    if (cur) for (int64_t i = 0; i < nb; ++i) free(cur[i]);
    if (nxt) for (int64_t i = 0; i < nb; ++i) free(nxt[i]);
    free(cur); free(nxt);
    return rc;
}

/*
 * L2 residual of a state (not stated by the paper; the h^2-scaled algebraic
 * residual of the discrete Poisson system A_h u = b, A_h = 2d I - S):
 *   r[c] = b[c] - (2d * u[c] - s[c]),   res = sqrt(sum_c r[c]^2),
 * every value widened to FP64 first and every operation in FP64, s summed in
 * the sweep's order.  Each x-row is summed in index order, then the row sums
 * in index order, so the value does not depend on the thread count.
 */
double FN(orc_residual2d)(int64_t nx, int64_t ny, const REAL *b, const REAL *u)
{
    double *rows = (double *)malloc((size_t)ny * sizeof(double));
    if (!rows) return NAN;
    const int64_t ld = nx + 2;
#pragma omp parallel for schedule(static)
    for (int64_t j = 1; j <= ny; ++j) {
        double acc = 0.0;
        for (int64_t i = 1; i <= nx; ++i) {
            const int64_t c = j * ld + i;
            const double s = ((double)u[c - 1] + (double)u[c + 1]) +
                             ((double)u[c - ld] + (double)u[c + ld]);
            const double bc = b ? (double)b[(j - 1) * nx + (i - 1)] : 0.0;
            const double r = bc - (4.0 * (double)u[c] - s);
            acc += r * r;
        }
        rows[j - 1] = acc;
    }
    double total = 0.0;
    for (int64_t j = 0; j < ny; ++j) total += rows[j];
    free(rows);
    return sqrt(total);
}

double FN(orc_residual3d)(int64_t nx, int64_t ny, int64_t nz, const REAL *b, const REAL *u)
{
    double *rows = (double *)malloc((size_t)(ny * nz) * sizeof(double));
    if (!rows) return NAN;
    const int64_t ld = nx + 2, lp = (nx + 2) * (ny + 2);
#pragma omp parallel for schedule(static) collapse(2)
    for (int64_t k = 1; k <= nz; ++k) {
        for (int64_t j = 1; j <= ny; ++j) {
            double acc = 0.0;
            for (int64_t i = 1; i <= nx; ++i) {
                const int64_t c = k * lp + j * ld + i;
                const double s = (((double)u[c - 1] + (double)u[c + 1]) +
                                  ((double)u[c - ld] + (double)u[c + ld])) +
                                 ((double)u[c - lp] + (double)u[c + lp]);
                const double bc = b ? (double)b[((k - 1) * ny + (j - 1)) * nx + (i - 1)] : 0.0;
                const double r = bc - (6.0 * (double)u[c] - s);
                acc += r * r;
            }
            rows[(k - 1) * ny + (j - 1)] = acc;
        }
    }
    double total = 0.0;
    for (int64_t t = 0; t < ny * nz; ++t) total += rows[t];
    free(rows);
    return sqrt(total);
}

/*
 * State after K sweeps on a sub-rectangle only, for checking single outputs of
 * very large runs.  The value of a node after K sweeps depends only on nodes
 * within K steps of it, so the plain sweep is applied to a copy of the
 * rectangle grown by K+1 nodes per side (clipped at the ring); nodes on the
 * copy's cut border are never updated, and their staleness reaches at most K
 * nodes inward.  Output: interior nodes x0..x1-1, y0..y1-1 (0-based interior
 * coordinates), x fastest.
 */
int FN(orc_window2d)(int64_t nx, int64_t ny, const REAL *b, const REAL *u, int64_t K,
                     int64_t x0, int64_t x1, int64_t y0, int64_t y1, REAL *out)
{
    /* node range of the copy, inclusive */
    const int64_t I0 = (x0 + 1 - K - 1 > 0) ? x0 + 1 - K - 1 : 0;
    const int64_t I1 = (x1 + K + 1 < nx + 1) ? x1 + K + 1 : nx + 1;
    const int64_t J0 = (y0 + 1 - K - 1 > 0) ? y0 + 1 - K - 1 : 0;
    const int64_t J1 = (y1 + K + 1 < ny + 1) ? y1 + K + 1 : ny + 1;
    const int64_t w = I1 - I0 + 1, h = J1 - J0 + 1;
    REAL *a = (REAL *)malloc((size_t)(w * h) * sizeof(REAL));
    REAL *c = (REAL *)malloc((size_t)(w * h) * sizeof(REAL));
    if (!a || !c) { free(a); free(c); return -1; }
    for (int64_t j = 0; j < h; ++j)
        for (int64_t i = 0; i < w; ++i)
            a[j * w + i] = u[(J0 + j) * (nx + 2) + (I0 + i)];
    memcpy(c, a, (size_t)(w * h) * sizeof(REAL));
    const REAL wt = (REAL)0.25;
    for (int64_t k = 0; k < K; ++k) {
#pragma omp parallel for schedule(static)
        for (int64_t j = 1; j < h - 1; ++j) {
            const int64_t gj = J0 + j;
            if (gj < 1 || gj > ny) continue;
            for (int64_t i = 1; i < w - 1; ++i) {
                const int64_t gi = I0 + i;
                if (gi < 1 || gi > nx) continue;
                const int64_t p = j * w + i;
                const REAL s = (a[p - 1] + a[p + 1]) + (a[p - w] + a[p + w]);
                c[p] = b ? (s + b[(gj - 1) * nx + (gi - 1)]) * wt : s * wt;
            }
        }
        REAL *t = a; a = c; c = t;
    }
    for (int64_t j = y0; j < y1; ++j)
        for (int64_t i = x0; i < x1; ++i)
            out[(j - y0) * (x1 - x0) + (i - x0)] = a[(j + 1 - J0) * w + (i + 1 - I0)];
    free(a); free(c);
    return 0;
}

/* 3D counterpart of orc_window2d: output nodes x0..x1-1, y0..y1-1, z0..z1-1. */
int FN(orc_window3d)(int64_t nx, int64_t ny, int64_t nz, const REAL *b, const REAL *u,
                     int64_t K, int64_t x0, int64_t x1, int64_t y0, int64_t y1, int64_t z0,
                     int64_t z1, REAL *out)
{
    const int64_t I0 = (x0 - K > 0) ? x0 - K : 0, I1 = (x1 + K + 1 < nx + 1) ? x1 + K + 1 : nx + 1;
    const int64_t J0 = (y0 - K > 0) ? y0 - K : 0, J1 = (y1 + K + 1 < ny + 1) ? y1 + K + 1 : ny + 1;
    const int64_t L0 = (z0 - K > 0) ? z0 - K : 0, L1 = (z1 + K + 1 < nz + 1) ? z1 + K + 1 : nz + 1;
    const int64_t w = I1 - I0 + 1, h = J1 - J0 + 1, d = L1 - L0 + 1;
    const int64_t gx = nx + 2, gp = (nx + 2) * (ny + 2);
    REAL *a = (REAL *)malloc((size_t)(w * h * d) * sizeof(REAL));
    REAL *c = (REAL *)malloc((size_t)(w * h * d) * sizeof(REAL));
    if (!a || !c) { free(a); free(c); return -1; }
    for (int64_t k = 0; k < d; ++k)
        for (int64_t j = 0; j < h; ++j)
            for (int64_t i = 0; i < w; ++i)
                a[(k * h + j) * w + i] = u[(L0 + k) * gp + (J0 + j) * gx + (I0 + i)];
    memcpy(c, a, (size_t)(w * h * d) * sizeof(REAL));
    const REAL wt = (REAL)1 / (REAL)6;
    const int64_t pw = w * h;
    for (int64_t t = 0; t < K; ++t) {
#pragma omp parallel for schedule(static) collapse(2)
        for (int64_t k = 1; k < d - 1; ++k) {
            for (int64_t j = 1; j < h - 1; ++j) {
                const int64_t gk = L0 + k, gj = J0 + j;
                if (gk < 1 || gk > nz || gj < 1 || gj > ny) continue;
                for (int64_t i = 1; i < w - 1; ++i) {
                    const int64_t gi = I0 + i;
                    if (gi < 1 || gi > nx) continue;
                    const int64_t p = (k * h + j) * w + i;
                    const REAL s = ((a[p - 1] + a[p + 1]) + (a[p - w] + a[p + w])) +
                                   (a[p - pw] + a[p + pw]);
                    c[p] = b ? (s + b[((gk - 1) * ny + (gj - 1)) * nx + (gi - 1)]) * wt : s * wt;
                }
            }
        }
        REAL *tt = a; a = c; c = tt;
    }
    for (int64_t k = z0; k < z1; ++k)
        for (int64_t j = y0; j < y1; ++j)
            for (int64_t i = x0; i < x1; ++i)
                out[((k - z0) * (y1 - y0) + (j - y0)) * (x1 - x0) + (i - x0)] =
                    a[((k + 1 - L0) * h + (j + 1 - J0)) * w + (i + 1 - I0)];
    free(a); free(c);
    return 0;
}

#undef FN
#undef ORC_CAT
#undef ORC_CAT_
