// C ABI of the over-decomposed Jacobi library (declared in include/jacobi.h).
//
// Host side: argument validation (always before any HIP call), the block
// layout planner, the workspace carve-up, and the pass planner that turns
// jacobi_sweep(n) into kernel launches on the handle's stream.  The library
// allocates no device memory: the caller's workspace holds everything.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/jacobi.h"
#include "jacobi_internal.h"
#include "kernels.h"

using jac::Geom;

namespace {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(JACOBI_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxCoord = 1 << 30;  // interior nodes per axis (coordinates are int32)

bool mul_ok(size_t a, size_t b, size_t *out) { return !__builtin_mul_overflow(a, b, out); }
bool add_ok(size_t a, size_t b, size_t *out) { return !__builtin_add_overflow(a, b, out); }
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    size_t off_u0, off_u1, off_b, off_part, off_scratch, bytes;
    size_t part_cap;  // doubles available for residual partial sums
};

constexpr int kMinRows = 8;  // smallest tile height of the pass kernels

// Block geometry and workspace carve-up.  All checks, no HIP.
int plan(int ndim, const int64_t *grid, const int64_t *blocks, int dtype, Geom *g, Layout *l) {
    if (ndim != 2 && ndim != 3) return fail(JACOBI_E_INVAL, "ndim must be 2 or 3 (got %d)", ndim);
    if (!grid || !blocks) return fail(JACOBI_E_INVAL, "grid and blocks must not be NULL");
    if (dtype != JACOBI_F32 && dtype != JACOBI_F64)
        return fail(JACOBI_E_INVAL, "dtype must be JACOBI_F32 or JACOBI_F64 (got %d)", dtype);
    const size_t es = dtype == JACOBI_F32 ? 4 : 8;
    std::memset(g, 0, sizeof *g);
    g->ndim = ndim;
    g->ax = (int)(32 / es);
    for (int a = 0; a < 3; ++a) {
        int64_t n = 1, b = 1;
        if (a < ndim) {
            n = grid[a];
            b = blocks[a];
            if (n < 1 || n > kMaxCoord)
                return fail(JACOBI_E_INVAL, "grid[%d] = %lld out of range [1, 2^30]", a, (long long)n);
            if (b < 1 || b > n)
                return fail(JACOBI_E_INVAL, "blocks[%d] = %lld must be in [1, grid[%d] = %lld]", a,
                            (long long)b, a, (long long)n);
        }
        int64_t e = (n + b - 1) / b;
        if (a == 0) e = (e + g->ax - 1) / g->ax * g->ax;
        if ((b - 1) * e >= n)
            return fail(JACOBI_E_INVAL,
                        "blocks[%d] = %lld leaves the last block empty (block extent %lld, n = %lld)",
                        a, (long long)b, (long long)e, (long long)n);
        g->n[a] = (int)n;
        g->nb[a] = (int)b;
        g->e[a] = (int)e;
    }
    size_t pitch = (size_t)g->e[0] + 2 * (size_t)g->ax, plane, bstride, sstride, nblk, t;
    if (!mul_ok(pitch, (size_t)g->e[1] + 2, &plane)) return fail(JACOBI_E_INVAL, "size overflow");
    bstride = plane;
    if (ndim == 3 && !mul_ok(plane, (size_t)g->e[2] + 2, &bstride))
        return fail(JACOBI_E_INVAL, "size overflow");
    bstride = round_up(bstride, 64);
    if (!mul_ok((size_t)g->e[0], (size_t)g->e[1], &sstride) ||
        !mul_ok(sstride, (size_t)g->e[2], &sstride))
        return fail(JACOBI_E_INVAL, "size overflow");
    sstride = round_up(sstride, 64);
    if (!mul_ok((size_t)g->nb[0], (size_t)g->nb[1], &nblk) || !mul_ok(nblk, (size_t)g->nb[2], &nblk))
        return fail(JACOBI_E_INVAL, "size overflow");
    g->pitch = (int64_t)pitch;
    g->plane = (int64_t)plane;
    g->bstride = (int64_t)bstride;
    g->sstride = (int64_t)sstride;
    g->nblocks = (int64_t)nblk;
    size_t sbytes, bbytes, off = 0;
    if (!mul_ok(nblk, bstride, &sbytes) || !mul_ok(sbytes, es, &sbytes) ||
        !mul_ok(nblk, sstride, &bbytes) || !mul_ok(bbytes, es, &bbytes))
        return fail(JACOBI_E_INVAL, "size overflow");
    if (sbytes > ((size_t)1 << 62) || bbytes > ((size_t)1 << 62))
        return fail(JACOBI_E_INVAL, "size overflow");
    l->off_u0 = off;
    off = round_up(off + sbytes, kAlign);
    l->off_u1 = off;
    off = round_up(off + sbytes, kAlign);
    l->off_b = off;
    off = round_up(off + bbytes, kAlign);
    // residual partials: one per work item of a pass kernel (strips of at
    // least 32 columns, tiles of at least kMinRows rows), or one per
    // workgroup of the standalone residual kernel
    size_t cap = ((size_t)g->n[0] / 32 + 2) * ((size_t)g->n[1] * g->n[2] / kMinRows + 2);
    if (cap < (size_t)jac::kResidualGroups) cap = jac::kResidualGroups;
    l->part_cap = cap;
    l->off_part = off;
    off = round_up(off + sizeof(double) * cap, kAlign);
    l->off_scratch = off;
    if (!add_ok(off, kAlign, &t)) return fail(JACOBI_E_INVAL, "size overflow");
    l->bytes = t;
    return JACOBI_OK;
}

}  // namespace

struct jacobi_s {
    Geom g;
    Layout lay;
    int dtype;
    char *ws;
    void *u[2];
    void *b;
    double *partials;
    double *scratch;
    int cur;
    bool has_state, has_source;
    hipStream_t stream;
    int depth, rows, flags;
    int adj_depth, adj_rows;  // schedule of adjoint passes (0 = default)
    double *gacc;             // adjoint: caller's FP64 dL/db accumulator (NULL = none)
    // profiling: event pairs around sweep-kernel launches
    bool profiling;
    std::vector<hipEvent_t> ev_pool;
    struct Rec {
        int depth;
        double updates, bytes;
    };
    std::vector<Rec> recs;  // one per recorded launch; events 2i, 2i+1
};

namespace {

int check_handle(jacobi_t h) {
    if (!h) return fail(JACOBI_E_INVAL, "handle is NULL");
    return JACOBI_OK;
}

// Tile height that makes one march launch fill the GPU in `rounds` whole
// rounds of resident waves: strips x tiles ~= rounds x (waves per CU x CUs).
int balanced_rows(const jacobi_s *h, int depth, int mode, int rounds) {
    if (h->g.ndim != 2) return 64;
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 64;
    const int wpc = h->dtype == JACOBI_F32 ? jac::march2d_waves_per_cu<float>(depth, mode)
                                           : jac::march2d_waves_per_cu<double>(depth, mode);
    const int64_t strips = h->dtype == JACOBI_F32 ? jac::march2d_strips<float>(h->g, depth)
                                                  : jac::march2d_strips<double>(h->g, depth);
    if (wpc <= 0 || strips <= 0) return 64;
    int64_t tiles = (int64_t)rounds * wpc * cus / strips;
    if (tiles < 1) tiles = 1;
    int64_t rows = (h->g.n[1] + tiles - 1) / tiles;
    if (rows < kMinRows) rows = kMinRows;
    if (rows > (1 << 20)) rows = 1 << 20;
    return (int)rows;
}

// Defaults before any tuning: the fastest depth measured on MI355X for a 2D
// FP32 8192^2 grid, with a tile height that fills the GPU in one round;
// explicit halos (depth 1) for 3D.
int default_depth(const jacobi_s *h) {
    if (h->g.ndim == 3) return 1;
    return h->dtype == JACOBI_F32 ? 7 : 4;
}

int default_rows(const jacobi_s *h) {
    const int d = h->depth > 0 ? h->depth : default_depth(h);
    return balanced_rows(h, d, h->has_source ? 1 : 0, 1);
}

int max_depth(int ndim, int dtype) {
    if (ndim == 3) return 1;
    const int *list;
    const int n = jac::march2d_depths(dtype, &list);
    return list[n - 1];
}

// Largest compiled march depth <= want.
int pick_depth(int dtype, int want) {
    const int *list;
    const int n = jac::march2d_depths(dtype, &list);
    int best = 1;
    for (int i = 0; i < n; ++i)
        if (list[i] <= want) best = list[i];
    return best;
}

// Event pair around one sweep-kernel launch when profiling is on.
int prof_begin(jacobi_t h) {
    if (!h->profiling) return JACOBI_OK;
    const size_t used = 2 * h->recs.size();
    while (h->ev_pool.size() < used + 2) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e), "event create");
        h->ev_pool.push_back(e);
    }
    HIP_TRY(hipEventRecord(h->ev_pool[used], h->stream), "event record");
    return JACOBI_OK;
}

int prof_end(jacobi_t h, int sweeps) {
    if (!h->profiling) return JACOBI_OK;
    HIP_TRY(hipEventRecord(h->ev_pool[2 * h->recs.size() + 1], h->stream), "event record");
    const double cells = (double)h->g.n[0] * h->g.n[1] * (h->g.ndim == 3 ? h->g.n[2] : 1);
    const double es = h->dtype == JACOBI_F32 ? 4.0 : 8.0;
    h->recs.push_back({sweeps, cells * sweeps, cells * es * (h->has_source ? 3.0 : 2.0)});
    return JACOBI_OK;
}

template <typename R>
int do_halo(jacobi_t h) {
    HIP_TRY(jac::launch_halo_exchange<R>(h->g, h->u[h->cur], h->stream), "halo exchange launch");
    return JACOBI_OK;
}

template <typename R>
int do_residual(jacobi_t h, double *out) {
    const void *b = h->has_source ? h->b : nullptr;
    if (h->g.ndim == 2) {
        // one residual-only pass of the march kernel (no stores)
        const int rows = balanced_rows(h, 1, h->has_source ? 1 : 0, 1);
        const int64_t nw = jac::march2d_work_items<R>(h->g, 1, rows);
        if (nw < 0 || (size_t)nw > h->lay.part_cap) return fail(JACOBI_E_INVAL, "partials overflow");
        int64_t nwork = 0;
        HIP_TRY(jac::launch_sweep2d_march<R>(h->g, h->u[h->cur], nullptr, b, h->partials, nullptr, 1, rows,
                                             h->stream, &nwork),
                "residual launch");
        HIP_TRY(jac::launch_residual_final(h->partials, (int)nwork, out, h->stream),
                "residual launch");
        return JACOBI_OK;
    }
    HIP_TRY(jac::launch_residual<R>(h->g, h->u[h->cur], b, h->partials, out, h->stream),
            "residual launch");
    return JACOBI_OK;
}

// n sweeps; if res_first is not NULL, the FP64 residual of the state the call
// starts from is written there (folded into the first pass when possible).
template <typename R>
int do_sweep(jacobi_t h, int64_t n, double *res_first) {
    const void *b = h->has_source ? h->b : nullptr;
    const bool explicit_halo = (h->flags & JACOBI_FLAG_EXPLICIT_HALO) || h->g.ndim == 3;
    if (explicit_halo || n == 0) {
        if (res_first) {
            int rc = do_residual<R>(h, res_first);
            if (rc) return rc;
        }
        for (int64_t k = 0; k < n; ++k) {
            int rc = prof_begin(h);
            if (rc) return rc;
            HIP_TRY(jac::launch_sweep_local<R>(h->g, h->u[h->cur], h->u[h->cur ^ 1], b, h->stream),
                    "sweep launch");
            rc = prof_end(h, 1);
            if (rc) return rc;
            h->cur ^= 1;
            HIP_TRY(jac::launch_halo_exchange<R>(h->g, h->u[h->cur], h->stream),
                    "halo exchange launch");
        }
        return JACOBI_OK;
    }
    const int depth = h->depth > 0 ? h->depth : default_depth(h);
    const int rows = h->rows > 0 ? h->rows : default_rows(h);
    int64_t left = n;
    bool first = true;
    while (left > 0) {
        // split what is left into the fewest passes of at most `depth`
        // sweeps, as evenly as possible (50 at depth 6: 6,6,6,6,6,5,5,5,5)
        const int64_t passes = (left + depth - 1) / depth;
        const int t = pick_depth(h->dtype, (int)((left + passes - 1) / passes));
        double *part = nullptr;
        if (first && res_first) {
            const int64_t nw = jac::march2d_work_items<R>(h->g, t, rows);
            if (nw < 0 || (size_t)nw > h->lay.part_cap)
                return fail(JACOBI_E_INVAL, "partials overflow");
            part = h->partials;
        }
        int rc = prof_begin(h);
        if (rc) return rc;
        int64_t nwork = 0;
        HIP_TRY(jac::launch_sweep2d_march<R>(h->g, h->u[h->cur], h->u[h->cur ^ 1], b, part, nullptr, t,
                                             rows, h->stream, &nwork),
                "sweep launch");
        rc = prof_end(h, t);
        if (rc) return rc;
        if (part)
            HIP_TRY(jac::launch_residual_final(part, (int)nwork, res_first, h->stream),
                    "residual launch");
        first = false;
        h->cur ^= 1;
        left -= t;
    }
    HIP_TRY(jac::launch_halo_exchange<R>(h->g, h->u[h->cur], h->stream), "halo exchange launch");
    return JACOBI_OK;
}

// Adjoint passes: n sweeps of the zero-ring state with the FP64 accumulation.
template <typename R>
int do_adjoint(jacobi_t h, int64_t n) {
    int depth = h->adj_depth > 0 ? h->adj_depth : (h->dtype == JACOBI_F32 ? 4 : 3);
    const int rows = h->adj_rows > 0 ? h->adj_rows : balanced_rows(h, depth, 2, 1);
    int64_t left = n;
    while (left > 0) {
        const int64_t passes = (left + depth - 1) / depth;
        const int t = pick_depth(h->dtype, (int)((left + passes - 1) / passes));
        int rc = prof_begin(h);
        if (rc) return rc;
        HIP_TRY(jac::launch_sweep2d_march<R>(h->g, h->u[h->cur], h->u[h->cur ^ 1], nullptr, nullptr,
                                             h->gacc, t, rows, h->stream, nullptr),
                "adjoint launch");
        rc = prof_end(h, t);
        if (rc) return rc;
        h->cur ^= 1;
        left -= t;
    }
    if (n > 0)
        HIP_TRY(jac::launch_halo_exchange<R>(h->g, h->u[h->cur], h->stream), "halo exchange launch");
    return JACOBI_OK;
}

}  // namespace

extern "C" {

int jacobi_workspace_bytes(int ndim, const int64_t *grid, const int64_t *blocks, int dtype,
                           size_t *bytes) {
    if (!bytes) return fail(JACOBI_E_INVAL, "bytes must not be NULL");
    Geom g;
    Layout l;
    const int rc = plan(ndim, grid, blocks, dtype, &g, &l);
    if (rc != JACOBI_OK) return rc;
    *bytes = l.bytes;
    return JACOBI_OK;
}

int jacobi_create(int ndim, const int64_t *grid, const int64_t *blocks, int dtype, void *workspace,
                  size_t workspace_bytes, void *stream, jacobi_t *out) {
    if (!out) return fail(JACOBI_E_INVAL, "out must not be NULL");
    *out = nullptr;
    Geom g;
    Layout l;
    int rc = plan(ndim, grid, blocks, dtype, &g, &l);
    if (rc != JACOBI_OK) return rc;
    if (!workspace) return fail(JACOBI_E_INVAL, "workspace must not be NULL");
    if ((uintptr_t)workspace % kAlign)
        return fail(JACOBI_E_INVAL, "workspace must be %zu-byte aligned", kAlign);
    if (workspace_bytes < l.bytes)
        return fail(JACOBI_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, l.bytes);
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, workspace);
    if (e != hipSuccess) return hip_fail(e, "workspace pointer query");
    if (attr.type != hipMemoryTypeDevice)
        return fail(JACOBI_E_INVAL, "workspace is not device memory");
    jacobi_s *h = new (std::nothrow) jacobi_s();
    if (!h) return fail(JACOBI_E_NOMEM, "host allocation failed");
    h->g = g;
    h->lay = l;
    h->dtype = dtype;
    h->ws = (char *)workspace;
    h->u[0] = h->ws + l.off_u0;
    h->u[1] = h->ws + l.off_u1;
    h->b = h->ws + l.off_b;
    h->partials = (double *)(h->ws + l.off_part);
    h->scratch = (double *)(h->ws + l.off_scratch);
    h->cur = 0;
    h->has_state = false;
    h->has_source = false;
    h->stream = (hipStream_t)stream;
    h->depth = 0;
    h->rows = 0;
    h->flags = 0;
    h->profiling = false;
    h->adj_depth = 0;
    h->adj_rows = 0;
    h->gacc = nullptr;
    *out = h;
    return JACOBI_OK;
}

int jacobi_destroy(jacobi_t h) {
    if (!h) return JACOBI_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    for (hipEvent_t ev : h->ev_pool) hipEventDestroy(ev);
    delete h;
    if (e != hipSuccess) return hip_fail(e, "stream synchronize in destroy");
    return JACOBI_OK;
}

int jacobi_set_stream(jacobi_t h, void *stream) {
    int rc = check_handle(h);
    if (rc) return rc;
    h->stream = (hipStream_t)stream;
    return JACOBI_OK;
}

int jacobi_get_layout(jacobi_t h, int64_t *blocks3, int64_t *extent3) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!blocks3 || !extent3) return fail(JACOBI_E_INVAL, "output pointers must not be NULL");
    for (int a = 0; a < 3; ++a) {
        blocks3[a] = h->g.nb[a];
        extent3[a] = h->g.e[a];
    }
    return JACOBI_OK;
}

int jacobi_set_state(jacobi_t h, const void *u) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!u) return fail(JACOBI_E_INVAL, "u must not be NULL");
    if (h->dtype == JACOBI_F32) {
        HIP_TRY(jac::launch_scatter<float>(h->g, u, h->u[0], h->u[1], false, h->stream), "scatter launch");
        HIP_TRY(jac::launch_halo_exchange<float>(h->g, h->u[0], h->stream), "halo exchange launch");
        HIP_TRY(jac::launch_halo_exchange<float>(h->g, h->u[1], h->stream), "halo exchange launch");
    } else {
        HIP_TRY(jac::launch_scatter<double>(h->g, u, h->u[0], h->u[1], false, h->stream), "scatter launch");
        HIP_TRY(jac::launch_halo_exchange<double>(h->g, h->u[0], h->stream), "halo exchange launch");
        HIP_TRY(jac::launch_halo_exchange<double>(h->g, h->u[1], h->stream), "halo exchange launch");
    }
    h->cur = 0;
    h->has_state = true;
    return JACOBI_OK;
}

int jacobi_get_state(jacobi_t h, void *u) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!u) return fail(JACOBI_E_INVAL, "u must not be NULL");
    if (!h->has_state) return fail(JACOBI_E_STATE, "no state set (call jacobi_set_state first)");
    if (h->dtype == JACOBI_F32)
        HIP_TRY(jac::launch_gather<float>(h->g, h->u[h->cur], u, h->stream), "gather launch");
    else
        HIP_TRY(jac::launch_gather<double>(h->g, h->u[h->cur], u, h->stream), "gather launch");
    return JACOBI_OK;
}

int jacobi_set_source(jacobi_t h, const void *f, double h2) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!f) {
        h->has_source = false;
        return JACOBI_OK;
    }
    if (!(h2 > 0.0) || !std::isfinite(h2))
        return fail(JACOBI_E_INVAL, "h2 must be positive and finite (got %g)", h2);
    if (h->dtype == JACOBI_F32)
        HIP_TRY(jac::launch_scale_source<float>(h->g, f, h->b, h2, h->stream), "source launch");
    else
        HIP_TRY(jac::launch_scale_source<double>(h->g, f, h->b, h2, h->stream), "source launch");
    h->has_source = true;
    return JACOBI_OK;
}

int jacobi_halo_exchange(jacobi_t h) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!h->has_state) return fail(JACOBI_E_STATE, "no state set (call jacobi_set_state first)");
    return h->dtype == JACOBI_F32 ? do_halo<float>(h) : do_halo<double>(h);
}

int jacobi_sweep(jacobi_t h, int64_t n_iter) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (n_iter < 0) return fail(JACOBI_E_INVAL, "n_iter must be >= 0 (got %lld)", (long long)n_iter);
    if (!h->has_state) return fail(JACOBI_E_STATE, "no state set (call jacobi_set_state first)");
    if (n_iter == 0) return JACOBI_OK;
    return h->dtype == JACOBI_F32 ? do_sweep<float>(h, n_iter, nullptr)
                                   : do_sweep<double>(h, n_iter, nullptr);
}

int jacobi_residual_async(jacobi_t h, double *res_dev) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!res_dev) return fail(JACOBI_E_INVAL, "res_dev must not be NULL");
    if (!h->has_state) return fail(JACOBI_E_STATE, "no state set (call jacobi_set_state first)");
    return h->dtype == JACOBI_F32 ? do_residual<float>(h, res_dev) : do_residual<double>(h, res_dev);
}

int jacobi_residual(jacobi_t h, double *res_host) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!res_host) return fail(JACOBI_E_INVAL, "res_host must not be NULL");
    if (!h->has_state) return fail(JACOBI_E_STATE, "no state set (call jacobi_set_state first)");
    rc = h->dtype == JACOBI_F32 ? do_residual<float>(h, h->scratch)
                                : do_residual<double>(h, h->scratch);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(res_host, h->scratch, sizeof(double), hipMemcpyDeviceToHost, h->stream),
            "residual copy");
    HIP_TRY(hipStreamSynchronize(h->stream), "stream synchronize");
    return JACOBI_OK;
}

int jacobi_solve(jacobi_t h, int64_t n_iter, int64_t check_every, double *res_dev) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (n_iter < 0) return fail(JACOBI_E_INVAL, "n_iter must be >= 0");
    if (check_every < 1) return fail(JACOBI_E_INVAL, "check_every must be >= 1");
    if (!res_dev) return fail(JACOBI_E_INVAL, "res_dev must not be NULL");
    if (!h->has_state) return fail(JACOBI_E_STATE, "no state set (call jacobi_set_state first)");
    // the residual of the state at the start of each interval rides on the
    // interval's first pass; the final state's residual needs its own pass
    int64_t k = 0, i = 0;
    while (k < n_iter) {
        const int64_t step = n_iter - k < check_every ? n_iter - k : check_every;
        rc = h->dtype == JACOBI_F32 ? do_sweep<float>(h, step, res_dev + i)
                                    : do_sweep<double>(h, step, res_dev + i);
        if (rc) return rc;
        k += step;
        ++i;
    }
    return jacobi_residual_async(h, res_dev + i);
}

int jacobi_adjoint_begin(jacobi_t h, const void *lam, double *grad_b) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!lam || !grad_b) return fail(JACOBI_E_INVAL, "lam and grad_b must not be NULL");
    if (h->g.ndim != 2) return fail(JACOBI_E_UNSUPPORTED, "the adjoint is implemented for 2D grids");
    if (h->dtype == JACOBI_F32) {
        HIP_TRY(jac::launch_scatter<float>(h->g, lam, h->u[0], h->u[1], true, h->stream),
                "scatter launch");
        HIP_TRY(jac::launch_halo_exchange<float>(h->g, h->u[0], h->stream), "halo exchange launch");
        HIP_TRY(jac::launch_halo_exchange<float>(h->g, h->u[1], h->stream), "halo exchange launch");
    } else {
        HIP_TRY(jac::launch_scatter<double>(h->g, lam, h->u[0], h->u[1], true, h->stream),
                "scatter launch");
        HIP_TRY(jac::launch_halo_exchange<double>(h->g, h->u[0], h->stream), "halo exchange launch");
        HIP_TRY(jac::launch_halo_exchange<double>(h->g, h->u[1], h->stream), "halo exchange launch");
    }
    HIP_TRY(jac::launch_fill_f64(grad_b, 0.0, (int64_t)h->g.n[0] * h->g.n[1], h->stream),
            "fill launch");
    h->cur = 0;
    h->has_state = true;
    h->gacc = grad_b;
    return JACOBI_OK;
}

int jacobi_adjoint_sweep(jacobi_t h, int64_t n_iter) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (n_iter < 0) return fail(JACOBI_E_INVAL, "n_iter must be >= 0");
    if (!h->gacc) return fail(JACOBI_E_STATE, "no adjoint in progress (call jacobi_adjoint_begin)");
    if (n_iter == 0) return JACOBI_OK;
    return h->dtype == JACOBI_F32 ? do_adjoint<float>(h, n_iter) : do_adjoint<double>(h, n_iter);
}

int jacobi_adjoint_end(jacobi_t h, double h2, double *grad_f, double *grad_ring) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!h->gacc) return fail(JACOBI_E_STATE, "no adjoint in progress (call jacobi_adjoint_begin)");
    if (!(h2 > 0.0) || !std::isfinite(h2))
        return fail(JACOBI_E_INVAL, "h2 must be positive and finite (got %g)", h2);
    HIP_TRY(jac::launch_adjoint_finish(h->g, h->gacc, h2, grad_f, grad_ring, h->stream),
            "adjoint finish launch");
    h->gacc = nullptr;
    return JACOBI_OK;
}

int jacobi_set_tuning(jacobi_t h, int t_depth, int rows, int flags) {
    int rc = check_handle(h);
    if (rc) return rc;
    const int md = max_depth(h->g.ndim, h->dtype);
    if (t_depth < 0 || t_depth > md)
        return fail(JACOBI_E_INVAL, "t_depth must be in [0, %d] (got %d)", md, t_depth);
    if (rows < 0 || (rows > 0 && rows < kMinRows) || rows > (1 << 20))
        return fail(JACOBI_E_INVAL, "rows must be 0 or in [%d, 2^20] (got %d)", kMinRows, rows);
    if (flags & ~JACOBI_FLAG_EXPLICIT_HALO) return fail(JACOBI_E_INVAL, "unknown flags 0x%x", flags);
    h->depth = t_depth;
    h->rows = rows;
    h->flags = flags;
    return JACOBI_OK;
}

int jacobi_get_tuning(jacobi_t h, int *t_depth, int *rows, int *flags) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!t_depth || !rows || !flags) return fail(JACOBI_E_INVAL, "output pointers must not be NULL");
    *t_depth = h->depth > 0 ? h->depth : default_depth(h);
    *rows = h->rows > 0 ? h->rows : default_rows(h);
    *flags = h->flags;
    return JACOBI_OK;
}

int jacobi_max_depth(int ndim, int dtype) {
    if ((ndim != 2 && ndim != 3) || (dtype != JACOBI_F32 && dtype != JACOBI_F64)) {
        fail(JACOBI_E_INVAL, "bad ndim/dtype");
        return JACOBI_E_INVAL;
    }
    return max_depth(ndim, dtype);
}

int jacobi_profile(jacobi_t h, int enable) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (enable) {
        HIP_TRY(hipStreamSynchronize(h->stream), "stream synchronize");
        h->recs.clear();
    }
    h->profiling = enable != 0;
    return JACOBI_OK;
}

int jacobi_profile_read(jacobi_t h, int depth, double *ms, int64_t *launches, double *cell_updates,
                        double *alg_bytes) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (depth < 0) return fail(JACOBI_E_INVAL, "depth must be >= 0");
    HIP_TRY(hipStreamSynchronize(h->stream), "stream synchronize");
    double total = 0.0, up = 0.0, by = 0.0;
    int64_t cnt = 0;
    for (size_t i = 0; i < h->recs.size(); ++i) {
        if (depth && h->recs[i].depth != depth) continue;
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, h->ev_pool[2 * i], h->ev_pool[2 * i + 1]),
                "event elapsed time");
        total += t;
        up += h->recs[i].updates;
        by += h->recs[i].bytes;
        ++cnt;
    }
    if (ms) *ms = total;
    if (launches) *launches = cnt;
    if (cell_updates) *cell_updates = up;
    if (alg_bytes) *alg_bytes = by;
    return JACOBI_OK;
}

namespace {

std::string tune_key(const jacobi_s *h, int64_t n, int src) {
    char buf[256];
    snprintf(buf, sizeof buf, "jacobi-v1 nd=%d n=%d,%d,%d b=%d,%d,%d dt=%d src=%d sweeps=%lld",
             h->g.ndim, h->g.n[0], h->g.n[1], h->g.n[2], h->g.nb[0], h->g.nb[1], h->g.nb[2],
             h->dtype, src, (long long)n);
    return buf;
}

bool cache_lookup(const std::string &key, int *d, int *r, int *f) {
    const char *path = getenv("JACOBI_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *fp = fopen(path, "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, fp)) {
        const size_t kl = key.size();
        if (strncmp(line, key.c_str(), kl) == 0 && line[kl] == ' ') {
            if (sscanf(line + kl, " -> %d %d %d", d, r, f) == 3) found = true;
        }
    }
    fclose(fp);
    return found;
}

void cache_store(const std::string &key, int d, int r, int f) {
    const char *path = getenv("JACOBI_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *fp = fopen(path, "a");
    if (!fp) return;
    fprintf(fp, "%s -> %d %d %d\n", key.c_str(), d, r, f);
    fclose(fp);
}

}  // namespace

int jacobi_autotune(jacobi_t h, int64_t n_sweeps, int with_source, int *t_depth, int *rows,
                    int *flags) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (n_sweeps < 1 || n_sweeps > (1 << 20))
        return fail(JACOBI_E_INVAL, "n_sweeps must be in [1, 2^20] (got %lld)", (long long)n_sweeps);
    const int src = with_source ? 1 : 0;
    const std::string key = tune_key(h, n_sweeps, src);
    int bd = 0, br = 0, bf = 0;
    if (!cache_lookup(key, &bd, &br, &bf) || jacobi_set_tuning(h, bd, br, bf) != JACOBI_OK) {
        struct Cand {
            int d, r, f;
        };
        std::vector<Cand> cands;
        cands.push_back({1, 0, JACOBI_FLAG_EXPLICIT_HALO});
        if (h->g.ndim == 2) {
            const int *list;
            const int nd = jac::march2d_depths(h->dtype, &list);
            static const int kRows[] = {16, 32, 64, 96, 128, 192, 256};
            for (int i = 0; i < nd; ++i) {
                std::vector<int> rs(kRows, kRows + sizeof(kRows) / sizeof(int));
                for (int k = 1; k <= 3; ++k) rs.push_back(balanced_rows(h, list[i], src, k));
                std::vector<int> seen;
                for (int r : rs) {
                    bool dup = false;
                    for (int q : seen) dup = dup || q == r;
                    if (dup) continue;
                    seen.push_back(r);
                    cands.push_back({list[i], r, 0});
                }
            }
        }
        const bool saved_src = h->has_source;
        const bool saved_prof = h->profiling;
        h->has_source = src;
        h->has_state = true;  // the buffers serve as scratch
        h->profiling = false;
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0), "event create");
        HIP_TRY(hipEventCreate(&e1), "event create");
        float best = 1e30f;
        for (const Cand &c : cands) {
            h->depth = c.d;
            h->rows = c.r;
            h->flags = c.f;
            rc = jacobi_sweep(h, n_sweeps);  // warm-up
            if (!rc && hipEventRecord(e0, h->stream) != hipSuccess) rc = JACOBI_E_HIP;
            if (!rc) rc = jacobi_sweep(h, n_sweeps);
            if (!rc) rc = jacobi_sweep(h, n_sweeps);
            if (!rc && hipEventRecord(e1, h->stream) != hipSuccess) rc = JACOBI_E_HIP;
            float t = 0.0f;
            if (!rc && (hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                rc = fail(JACOBI_E_HIP, "autotune timing failed");
            if (rc) break;
            if (t < best) {
                best = t;
                bd = c.d;
                br = c.r;
                bf = c.f;
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        h->has_source = saved_src;
        h->profiling = saved_prof;
        if (rc) {
            h->has_state = false;
            return rc;
        }
        cache_store(key, bd, br, bf);
    }
    h->has_state = false;
    h->depth = bd;
    h->rows = br;
    h->flags = bf;
    if (t_depth) *t_depth = bd;
    if (rows) *rows = br;
    if (flags) *flags = bf;
    return JACOBI_OK;
}

const char *jacobi_strerror(int status) {
    switch (status) {
    case JACOBI_OK: return "success";
    case JACOBI_E_INVAL: return "invalid argument";
    case JACOBI_E_NOMEM: return "insufficient memory";
    case JACOBI_E_HIP: return "HIP runtime error";
    case JACOBI_E_STATE: return "invalid call for the handle's state";
    case JACOBI_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *jacobi_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
