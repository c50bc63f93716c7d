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
#include <mutex>
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
    // x extents are multiples of 32 bytes (every 16-byte lane chunk of a row
    // lies in one block); interior rows start 128 bytes into their row
    const int xgran = (int)(32 / es);
    g->ax = (int)(128 / es);
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
        if (a == 0) e = (e + xgran - 1) / xgran * xgran;
        if ((b - 1) * e >= n)
            return fail(JACOBI_E_INVAL,
                        "blocks[%d] = %lld leaves the last block empty (block extent %lld, n = %lld)",
                        a, (long long)b, (long long)e, (long long)n);
        g->n[a] = (int)n;
        g->nb[a] = (int)b;
        g->e[a] = (int)e;
    }
    // pitch: a multiple of 128 bytes, so every interior row is 128-byte
    // aligned; the east ring cell of a full-width row may be element 0 of the
    // next row, which no row uses (west rings sit at ax - 1)
    size_t pitch = (size_t)g->ax + round_up((size_t)g->e[0], (size_t)g->ax), plane, bstride,
           sstride, nblk, t;
    if (!mul_ok(pitch, (size_t)g->e[1] + 2, &plane)) return fail(JACOBI_E_INVAL, "size overflow");
    bstride = plane;
    if (ndim == 3 && !mul_ok(plane, (size_t)g->e[2] + 2, &bstride))
        return fail(JACOBI_E_INVAL, "size overflow");
    // slack after the last row: its east ring and a 16-byte chunk loaded
    // from there stay inside the block
    bstride = round_up(bstride + (size_t)g->ax, 64);
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
    if (ndim == 3) {
        // 3D pass: 8 partials (one per wave) per work item of (strip of
        // >= 24 output columns, >= 26 output rows, z segment of >= kMinRows
        // planes), the smallest tiles of any depth; 4 per 10 rows bounds it
        const size_t c3 = ((size_t)g->n[0] / 24 + 2) * 4 * ((size_t)g->n[1] / 10 + 2) *
                          ((size_t)g->n[2] / kMinRows + 2);
        if (c3 > cap) cap = c3;
    }
    if (ndim == 2) {
        // 2D tile sweep at depth 1: one partial per wave, 4 per work item of
        // (block, 64 x 16-byte column chunk, 4-row tile)
        const size_t chunk = 64 * (16 / es);
        const size_t ct = 4 * nblk * (((size_t)g->e[0] + chunk - 1) / chunk) *
                          (((size_t)g->e[1] + 3) / 4);
        if (ct > cap) cap = ct;
    }
    if (cap < (size_t)jac::kResidualGroups) cap = jac::kResidualGroups;
    l->part_cap = cap;
    l->off_part = off;
    off = round_up(off + sizeof(double) * cap, kAlign);
    l->off_scratch = off;
    if (!add_ok(off, kAlign, &t)) return fail(JACOBI_E_INVAL, "size overflow");
    l->bytes = t;
    return JACOBI_OK;
}

constexpr int kDeepMaxDepth = 16;  // prefix tables per pass depth 1 .. 16

// Deep-halo layout on top of plan(): every block stores local nodes -Hs ..
// e+Hs-1 on each axis (Hs = the requested halo rounded up so that a small
// grid's first interior column is 16-byte aligned whether or not it extends
// into a neighbour), in rows of pitch_d elements whose column Hs-1 past
// 128 bytes holds local x = 0.  g is rewritten to a view of that storage
// (pitch, plane, bstride and ax), so local_offset addresses it; the blocked
// source keeps plan()'s layout.  Workspace: two state buffers, the blocked
// source, the deep source, residual partials, scratch, two descriptor tables,
// prefix tables, activity flags and a pass counter.
struct DeepLayout {
    int hs;
    size_t off_bd, off_tab, off_prefix, off_active, off_pc;
};

int plan_deep(int ndim, const int64_t *grid, const int64_t *blocks, int dtype, int halo, Geom *g,
              Layout *l, DeepLayout *dl) {
    int rc = plan(ndim, grid, blocks, dtype, g, l);
    if (rc != JACOBI_OK) return rc;
    if (halo < 1 || halo > 64) return fail(JACOBI_E_INVAL, "halo must be in [1, 64] (got %d)", halo);
    const size_t es = dtype == JACOBI_F32 ? 4 : 8;
    const int V = (int)(16 / es);
    const int hs = 1 + (halo - 1 + V - 1) / V * V;
    // a small grid reaching into a neighbour must stay inside the domain
    for (int a = 0; a < ndim; ++a) {
        if (g->nb[a] < 2) continue;
        const int last = g->n[a] - (g->nb[a] - 1) * g->e[a];
        const int lim = last < g->e[a] ? last : g->e[a];
        if (hs > lim)
            return fail(JACOBI_E_INVAL,
                        "halo %d (stored %d) exceeds the block extent %d on axis %d", halo, hs, lim,
                        a);
    }
    const size_t axc = 128 / es;
    const size_t co = axc + hs - 1;  // storage column of local x = 0
    const size_t pitch = round_up(co + (size_t)g->e[0] + hs + V, axc);
    const size_t rows = (size_t)g->e[1] + 2 * hs;
    const size_t plane = rows * pitch;
    size_t bstride = ndim == 3 ? plane * ((size_t)g->e[2] + 2 * hs) : plane;
    bstride = round_up(bstride + axc, 64);
    size_t ax = co + (size_t)(hs - 1) * pitch + (ndim == 3 ? (size_t)(hs - 1) * plane : 0);
    if (ax > ((size_t)1 << 30)) return fail(JACOBI_E_INVAL, "size overflow");
    g->pitch = (int64_t)pitch;
    g->plane = (int64_t)plane;
    g->bstride = (int64_t)bstride;
    g->ax = (int)ax;
    size_t sbytes, t;
    if (!mul_ok((size_t)g->nblocks, bstride, &sbytes) || !mul_ok(sbytes, es, &sbytes) ||
        sbytes > ((size_t)1 << 62))
        return fail(JACOBI_E_INVAL, "size overflow");
    const size_t bbytes = l->off_part - l->off_b;  // the blocked source (plan's layout)
    const size_t part_bytes = l->off_scratch - l->off_part;
    size_t off = 0;
    l->off_u0 = off;
    off = round_up(off + sbytes, kAlign);
    l->off_u1 = off;
    off = round_up(off + sbytes, kAlign);
    l->off_b = off;
    off = round_up(off + bbytes, kAlign);
    dl->off_bd = off;
    off = round_up(off + sbytes, kAlign);
    l->off_part = off;
    off = round_up(off + part_bytes, kAlign);
    l->off_scratch = off;
    off = round_up(off + kAlign, kAlign);
    const size_t nb = (size_t)g->nblocks;
    dl->off_tab = off;
    off = round_up(off + 2 * nb * sizeof(jac::BatchGrid), kAlign);
    dl->off_prefix = off;
    off = round_up(off + (kDeepMaxDepth + 1) * (nb + 1) * sizeof(int), kAlign);
    dl->off_active = off;
    off = round_up(off + nb * sizeof(int), kAlign);
    dl->off_pc = off;
    if (!add_ok(off, kAlign, &t)) return fail(JACOBI_E_INVAL, "size overflow");
    l->bytes = t;
    dl->hs = hs;
    return JACOBI_OK;
}

// The small grid of block blk in the deep layout: the block's interior
// extended by hs-1 nodes into every neighbour, with its ring on the layer
// beyond (a neighbour's nodes, refreshed by the exchange before each pass)
// or on the domain's Dirichlet ring.  Geometry of one unblocked grid whose
// state rows / planes are those of the deep storage and whose source rows
// are those of the deep source; u[k] from buffer bufk, b from bd.
jac::BatchGrid small_grid(const Geom &g, int hs, int64_t blk, int dtype, char *buf0, char *buf1,
                          char *bd) {
    const size_t es = dtype == JACOBI_F32 ? 4 : 8;
    const int bi[3] = {(int)(blk % g.nb[0]), (int)((blk / g.nb[0]) % g.nb[1]),
                       g.ndim == 3 ? (int)(blk / ((int64_t)g.nb[0] * g.nb[1])) : 0};
    int lo[3] = {0, 0, 0}, n[3] = {1, 1, 1};
    for (int a = 0; a < g.ndim; ++a) {
        const int ext = jac::extent(g.n[a], g.e[a], bi[a]);
        lo[a] = bi[a] > 0 ? -(hs - 1) : 0;
        const int hi = bi[a] < g.nb[a] - 1 ? ext + hs - 1 : ext;
        n[a] = hi - lo[a];
    }
    jac::BatchGrid d;
    std::memset(&d, 0, sizeof d);
    Geom &s = d.g;
    s.ndim = g.ndim;
    const int64_t co = (int64_t)(128 / es) + hs - 1;
    s.ax = (int)(co + lo[0]);
    for (int a = 0; a < 3; ++a) {
        s.n[a] = n[a];
        s.nb[a] = 1;
    }
    // e: source row stride (the deep pitch), rows per source plane, and a
    // z extent no plane reaches (one block per axis)
    s.e[0] = (int)g.pitch;
    s.e[1] = g.ndim == 3 ? (int)(g.plane / g.pitch) : (1 << 30);
    s.e[2] = 1 << 30;
    s.pitch = g.pitch;
    s.plane = g.plane;
    s.bstride = g.bstride;
    s.sstride = 0;
    s.nblocks = 1;
    const int64_t zpart = g.ndim == 3 ? (int64_t)(lo[2] + hs - 1) * g.plane : 0;
    const int64_t ring = blk * g.bstride + zpart + (int64_t)(lo[1] + hs - 1) * g.pitch;
    d.u[0] = buf0 + ring * es;
    d.u[1] = buf1 + ring * es;
    const int64_t bz = g.ndim == 3 ? (int64_t)(lo[2] + hs) * g.plane : 0;
    d.b = bd + (blk * g.bstride + bz + (int64_t)(lo[1] + hs) * g.pitch + co + lo[0]) * es;
    return d;
}

}  // namespace

// Device scratch of jacobi_solve_noalloc: a file-scope array of fixed size,
// one copy on every GPU the library runs on, held until the process ends.
// In host code `scratch` names a host-side stand-in, never the device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[JACOBI_NOALLOC_MAX_BYTES];

// Pieces of an overlapped explicit-halo sweep (slabs of block layers).
constexpr int kPieces = 4;

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
    // overlapped explicit-halo sweeps: the stream that sends faces, and
    // events handing each piece over to it and joining it back
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_piece[kPieces] = {};
    hipEvent_t ev_join = nullptr;
    // deep-halo block storage (halo > 0): the state buffers hold an H-deep
    // frame around every block; bdeep is the source in the same layout, and
    // each pass runs every block as its own small grid from a descriptor
    // table (one per buffer parity) and work-prefix tables per depth
    int halo = 0;
    void *bdeep = nullptr;
    jac::BatchGrid *d_tab[2] = {nullptr, nullptr};
    int *d_prefix = nullptr;
    int *d_active = nullptr;
    int *d_pc = nullptr;
    int tab_rows = 0;  // tile height / z segment the prefix tables hold (0: none)
    std::vector<int> h_prefix;
};

namespace {

int check_handle(jacobi_t h) {
    if (!h) return fail(JACOBI_E_INVAL, "handle is NULL");
    return JACOBI_OK;
}

// Tile height that makes one march launch fill the GPU in `rounds` whole
// rounds of resident waves: the smallest height whose tiles (edge bands and
// outer strips included) number at most rounds x (waves per CU x CUs).
int balanced_rows(const jacobi_s *h, int depth, int mode, int rounds) {
    if (h->g.ndim != 2) return 64;
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 64;
    const int wpc = h->dtype == JACOBI_F32 ? jac::march2d_waves_per_cu<float>(depth, mode)
                                           : jac::march2d_waves_per_cu<double>(depth, mode);
    if (wpc <= 0) return 64;
    const int64_t slots = (int64_t)rounds * wpc * cus;
    auto tiles = [&](int rows) {
        return h->dtype == JACOBI_F32 ? jac::march2d_work_items<float>(h->g, depth, rows)
                                      : jac::march2d_work_items<double>(h->g, depth, rows);
    };
    int lo = kMinRows, hi = h->g.n[1] > kMinRows ? h->g.n[1] : kMinRows;
    if (hi > (1 << 20)) hi = 1 << 20;
    const int64_t most = tiles(hi);
    if (most < 0 || most > slots) return hi;  // more strips than one round holds
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        const int64_t n = tiles(mid);
        if (n >= 0 && n <= slots)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Defaults before any tuning: the fastest schedules measured on MI355X for
// a 2D FP32 8192^2 grid with a residual every 50 sweeps (depth 13: passes of
// 13, 13, 12, 12), with a tile height that fills the GPU in one round of
// resident waves, and for a 512^3 grid in 64^3 blocks (depth 4, the deepest
// 3D pass: 836 / 475 GLUP/s in FP32 / FP64 against 381 / 190 at depth 1).
int default_depth(const jacobi_s *h) {
    if (h->g.ndim == 3) return 4;
    return h->dtype == JACOBI_F32 ? 13 : 4;
}

// The 2D pass kernels address a lane's chunk as a 32-bit byte offset from a
// row of block column 0; grids whose block columns span 4 GiB or more use
// the explicit-halo sweep and the standalone residual kernel instead.
bool march_fits(const Geom &g, int dtype) {
    const double es = dtype == JACOBI_F32 ? 4.0 : 8.0;
    const double span = (double)g.nb[0] * (double)(g.bstride > g.sstride ? g.bstride : g.sstride);
    return span * es < 4294967296.0 - 4096.0;
}


int default_rows(const jacobi_s *h) {
    const int d = h->depth > 0 ? h->depth : default_depth(h);
    return balanced_rows(h, d, h->has_source ? 1 : 0, 1);
}

int max_depth(int ndim, int dtype) {
    if (ndim == 3) return jac::march3d_max_depth();
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

// z planes per work item of the 3D pass: 32 (FP32) / 64 (FP64) measured
// fastest at depth 4 on 512^3 (16 .. 128 tried; shorter segments repeat the
// 2(T-1) warm-up planes more often, longer ones leave too few work items).
int zseg_of(const jacobi_s *h) {
    return h->rows > 0 ? h->rows : h->dtype == JACOBI_F32 ? 32 : 64;
}

template <typename R>
int do_residual(jacobi_t h, double *out) {
    const void *b = h->has_source ? h->b : nullptr;
    if (h->g.ndim == 3) {
        const int64_t nw = jac::march3d_work_items<R>(h->g, zseg_of(h));
        if ((size_t)nw > h->lay.part_cap) return fail(JACOBI_E_INVAL, "partials overflow");
        int64_t nwork = 0;
        HIP_TRY(jac::launch_march3d<R>(h->g, h->u[h->cur], nullptr, b, h->partials, zseg_of(h),
                                       h->stream, &nwork),
                "residual launch");
        HIP_TRY(jac::launch_residual_final(h->partials, (int)nwork, out, h->stream),
                "residual launch");
        return JACOBI_OK;
    }
    if (h->g.ndim == 2 && march_fits(h->g, h->dtype)) {
        // one residual-only pass of the march kernel (no stores)
        const int rows = balanced_rows(h, 1, h->has_source ? 1 : 0, 1);
        const int64_t nw = jac::march2d_work_items<R>(h->g, 1, rows);
        if (nw < 0 || (size_t)nw > h->lay.part_cap) return fail(JACOBI_E_INVAL, "partials overflow");
        int64_t nwork = 0;
        HIP_TRY(jac::launch_sweep2d_march<R>(h->g, h->u[h->cur], nullptr, b, h->partials, nullptr, 1, rows,
                                             h->stream, &nwork, 0),
                "residual launch");
        HIP_TRY(jac::launch_residual_final(h->partials, (int)nwork, out, h->stream),
                "residual launch");
        return JACOBI_OK;
    }
    HIP_TRY(jac::launch_residual<R>(h->g, h->u[h->cur], b, h->partials, out, h->stream),
            "residual launch");
    return JACOBI_OK;
}

// Explicit-halo sweeps with the exchange overlapped: the blocks are cut into
// up to kPieces slabs of whole block layers along the slowest axis; each
// slab is swept on the handle's stream, then its faces are sent into its
// neighbours' halos of the new state on a second stream while the next slab
// is swept (the over-decomposition of Section 4.4: one piece's transfer
// hidden under another piece's kernel).  The sweeps read the old state and
// write only interiors of the new one, the sends write only halos of the new
// state, so the two streams never touch the same elements; the handle's
// stream waits for all sends before the next sweep.
template <typename R>
int do_sweep_overlap(jacobi_t h, int64_t n, double *res_first) {
    const void *b = h->has_source ? h->b : nullptr;
    if (res_first) {
        int rc = do_residual<R>(h, res_first);
        if (rc) return rc;
    }
    if (n == 0) return JACOBI_OK;
    if (!h->stream2) {
        HIP_TRY(hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking), "stream create");
        for (hipEvent_t &ev : h->ev_piece)
            HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event create");
        HIP_TRY(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming), "event create");
    }
    const int slow = h->g.ndim - 1;
    const int64_t layers = h->g.nb[slow];
    const int64_t per_layer = h->g.nblocks / layers;
    const int pieces = layers < kPieces ? (int)layers : kPieces;
    for (int64_t k = 0; k < n; ++k) {
        int rc = prof_begin(h);
        if (rc) return rc;
        for (int p = 0; p < pieces; ++p) {
            const int64_t b0 = layers * p / pieces * per_layer;
            const int64_t b1 = layers * (p + 1) / pieces * per_layer;
            HIP_TRY(jac::launch_sweep_local<R>(h->g, h->u[h->cur], h->u[h->cur ^ 1], b, h->stream,
                                               h->rows, b0, b1),
                    "sweep launch");
            HIP_TRY(hipEventRecord(h->ev_piece[p], h->stream), "event record");
            HIP_TRY(hipStreamWaitEvent(h->stream2, h->ev_piece[p], 0), "stream wait");
            HIP_TRY(jac::launch_halo_send<R>(h->g, h->u[h->cur ^ 1], b0, b1, h->stream2),
                    "halo send launch");
        }
        HIP_TRY(hipEventRecord(h->ev_join, h->stream2), "event record");
        HIP_TRY(hipStreamWaitEvent(h->stream, h->ev_join, 0), "stream wait");
        rc = prof_end(h, 1);
        if (rc) return rc;
        h->cur ^= 1;
    }
    return JACOBI_OK;
}

// n sweeps; if res_first is not NULL, the FP64 residual of the state the call
// starts from is written there (folded into the first pass when possible).
// The fused passes read a block-edge neighbour from the block that owns it
// and never the stored halos, so they refresh the halos (for the API's
// other paths) only once, after their last pass, and only when
// sync_halos is set; the explicit-halo sweep keeps them valid after every
// sweep, as it must.
template <typename R>
int do_deep_sweep(jacobi_t h, int64_t n, double *res_first, bool sync_halos);

template <typename R>
int do_sweep(jacobi_t h, int64_t n, double *res_first, bool sync_halos = true) {
    const void *b = h->has_source ? h->b : nullptr;
    const bool explicit_halo = (h->flags & JACOBI_FLAG_EXPLICIT_HALO) != 0 ||
                               (h->g.ndim == 2 && !march_fits(h->g, h->dtype));
    if (h->halo > 0 && !explicit_halo) return do_deep_sweep<R>(h, n, res_first, sync_halos);
    if (h->g.ndim == 3 && !explicit_halo && n > 0) {
        // fused 3D passes of up to `depth` sweeps each, split as evenly as
        // possible; the first also sums the residual of its input
        const int zseg = zseg_of(h);
        const int depth = h->depth > 0 ? h->depth : default_depth(h);
        int64_t left = n;
        bool first = true;
        while (left > 0) {
            const int64_t passes = (left + depth - 1) / depth;
            const int t = (int)((left + passes - 1) / passes);
            double *part = (first && res_first) ? h->partials : nullptr;
            if (part && (size_t)jac::march3d_work_items<R>(h->g, zseg, t) > h->lay.part_cap)
                return fail(JACOBI_E_INVAL, "partials overflow");
            int rc = prof_begin(h);
            if (rc) return rc;
            int64_t nwork = 0;
            HIP_TRY(jac::launch_march3d<R>(h->g, h->u[h->cur], h->u[h->cur ^ 1], b, part, zseg,
                                           h->stream, &nwork, h->flags & JACOBI_FLAG_NT_STORES, t),
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
        if (sync_halos)
            HIP_TRY(jac::launch_halo_exchange<R>(h->g, h->u[h->cur], h->stream),
                    "halo exchange launch");
        return JACOBI_OK;
    }
    if ((h->flags & JACOBI_FLAG_OVERLAP) && explicit_halo) return do_sweep_overlap<R>(h, n, res_first);
    if (explicit_halo || n == 0) {
        if (res_first) {
            int rc = do_residual<R>(h, res_first);
            if (rc) return rc;
        }
        for (int64_t k = 0; k < n; ++k) {
            int rc = prof_begin(h);
            if (rc) return rc;
            HIP_TRY(jac::launch_sweep_local<R>(h->g, h->u[h->cur], h->u[h->cur ^ 1], b, h->stream,
                                               h->rows, 0, -1, h->flags & JACOBI_FLAG_NT_STORES),
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
        if (t == 1) {
            // one sweep per pass: the tile kernel, reading block-edge
            // neighbours from their owning blocks
            if (first && res_first) {
                const int64_t nw = jac::sweep_tile_partials<R>(h->g, 0);
                if (nw < 0 || (size_t)nw > h->lay.part_cap)
                    return fail(JACOBI_E_INVAL, "partials overflow");
                part = h->partials;
            }
            int rc = prof_begin(h);
            if (rc) return rc;
            int64_t nwork = 0;
            HIP_TRY(jac::launch_sweep2d_tile_fused<R>(h->g, h->u[h->cur], h->u[h->cur ^ 1], b, part,
                                                      0, h->stream, &nwork,
                                                      h->flags & JACOBI_FLAG_NT_STORES),
                    "sweep launch");
            rc = prof_end(h, 1);
            if (rc) return rc;
            if (part)
                HIP_TRY(jac::launch_residual_final(part, (int)nwork, res_first, h->stream),
                        "residual launch");
            first = false;
            h->cur ^= 1;
            left -= 1;
            continue;
        }
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
                                             rows, h->stream, &nwork,
                                             h->flags & JACOBI_FLAG_NT_STORES),
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
    if (sync_halos)
        HIP_TRY(jac::launch_halo_exchange<R>(h->g, h->u[h->cur], h->stream),
                "halo exchange launch");
    return JACOBI_OK;
}

// Deep-halo passes ------------------------------------------------------

// Descriptor and work-prefix tables of the small grids for tile height (2D)
// or z segment (3D) `rows`; uploaded when it changes.
template <typename R>
int deep_tables(jacobi_t h, int rows) {
    if (h->tab_rows == rows) return JACOBI_OK;
    const int64_t nb = h->g.nblocks;
    std::vector<jac::BatchGrid> t[2];
    for (int p = 0; p < 2; ++p) {
        t[p].resize(nb);
        for (int64_t k = 0; k < nb; ++k)
            t[p][k] = small_grid(h->g, h->halo, k, h->dtype, (char *)h->u[p], (char *)h->u[p ^ 1],
                                 (char *)h->bdeep);
    }
    h->h_prefix.assign((size_t)(kDeepMaxDepth + 1) * (nb + 1), -1);
    for (int d = 1; d <= kDeepMaxDepth; ++d) {
        int *pre = &h->h_prefix[(size_t)d * (nb + 1)];
        int64_t acc = 0;
        for (int64_t k = 0; k < nb && acc >= 0; ++k) {
            pre[k] = (int)acc;
            const int64_t w = h->g.ndim == 2 ? jac::march2d_batch_work<R>(t[0][k].g, d, rows)
                                             : jac::march3d_batch_items<R>(t[0][k].g, rows, d);
            if (w < 0) {
                acc = -1;
                break;
            }
            acc += w;
            if (acc > 0x3fffffff) return fail(JACOBI_E_INVAL, "deep-halo pass exceeds 2^30 work items");
        }
        pre[nb] = (int)acc;
    }
    std::vector<int> ones((size_t)nb, 1);
    const int zero = 0;
    for (int p = 0; p < 2; ++p)
        HIP_TRY(hipMemcpyAsync(h->d_tab[p], t[p].data(), sizeof(jac::BatchGrid) * nb,
                               hipMemcpyHostToDevice, h->stream),
                "deep table upload");
    HIP_TRY(hipMemcpyAsync(h->d_prefix, h->h_prefix.data(), sizeof(int) * h->h_prefix.size(),
                           hipMemcpyHostToDevice, h->stream),
            "deep table upload");
    HIP_TRY(hipMemcpyAsync(h->d_active, ones.data(), sizeof(int) * nb, hipMemcpyHostToDevice,
                           h->stream),
            "deep table upload");
    HIP_TRY(hipMemcpyAsync(h->d_pc, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream),
            "deep table upload");
    HIP_TRY(hipStreamSynchronize(h->stream), "stream synchronize");
    h->tab_rows = rows;
    return JACOBI_OK;
}

// Tile height of the 2D small-grid passes at `depth`: the smallest whose
// work items over all blocks fit one round of resident waves.
template <typename R>
int deep_rows(jacobi_t h, int depth) {
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 64;
    const int wpc = jac::march2d_waves_per_cu<R>(depth, h->has_source ? 1 : 0);
    if (wpc <= 0) return 64;
    const int64_t slots = (int64_t)wpc * cus;
    std::vector<jac::BatchGrid> t((size_t)h->g.nblocks);
    int maxn = kMinRows;
    for (int64_t k = 0; k < h->g.nblocks; ++k) {
        t[k] = small_grid(h->g, h->halo, k, h->dtype, nullptr, nullptr, nullptr);
        if (t[k].g.n[1] > maxn) maxn = t[k].g.n[1];
    }
    auto work = [&](int rows) {
        int64_t acc = 0;
        for (const auto &d : t) acc += jac::march2d_batch_work<R>(d.g, depth, rows);
        return acc;
    };
    int lo = kMinRows, hi = maxn;
    if (work(hi) > slots) return hi;
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (work(mid) <= slots) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// n sweeps of a deep-halo handle: passes of up to min(depth, halo) sweeps,
// each an H-deep frame exchange followed by one launch over every block's
// small grid (each reads only its own block's storage).
template <typename R>
int do_deep_sweep(jacobi_t h, int64_t n, double *res_first, bool sync_halos) {
    if (res_first) {
        int rc = do_residual<R>(h, res_first);
        if (rc) return rc;
    }
    if (n == 0) return JACOBI_OK;
    const int nd = h->g.ndim;
    int depth = h->depth > 0 ? h->depth : default_depth(h);
    if (depth > h->halo) depth = h->halo;
    if (nd == 2) depth = pick_depth(h->dtype, depth);
    // 3D: one z segment per small grid unless set (its 2(T-1) warm-up planes
    // are paid once; measured fastest on 64^3 blocks)
    const int rows = nd == 2 ? (h->rows > 0 ? h->rows : deep_rows<R>(h, depth))
                             : (h->rows > 0 ? h->rows : h->g.e[2] + 2 * (h->halo - 1));
    int rc = deep_tables<R>(h, rows);
    if (rc) return rc;
    const int64_t nb = h->g.nblocks;
    int64_t left = n;
    while (left > 0) {
        const int64_t passes = (left + depth - 1) / depth;
        int t = (int)((left + passes - 1) / passes);
        if (nd == 2) t = pick_depth(h->dtype, t);
        const int nwork = h->h_prefix[(size_t)t * (nb + 1) + nb];
        if (nwork < 0) return fail(JACOBI_E_INVAL, "no deep-halo pass of depth %d", t);
        HIP_TRY(jac::launch_deep_exchange<R>(h->g, h->u[h->cur], h->halo, h->stream),
                "deep exchange launch");
        rc = prof_begin(h);
        if (rc) return rc;
        const int *pre = h->d_prefix + (size_t)t * (nb + 1);
        if (nd == 2)
            HIP_TRY(jac::launch_march2d_batch<R>(h->d_tab[h->cur], pre, (int)nb, h->d_active, h->d_pc,
                                                 nullptr, true, t, rows, nwork, h->stream,
                                                 h->has_source ? 1 : 0),
                    "deep pass launch");
        else
            HIP_TRY(jac::launch_march3d_batch<R>(h->d_tab[h->cur], pre, (int)nb, h->has_source, t,
                                                 rows, nwork, h->stream),
                    "deep pass launch");
        rc = prof_end(h, t);
        if (rc) return rc;
        h->cur ^= 1;
        left -= t;
    }
    if (sync_halos)
        HIP_TRY(jac::launch_halo_exchange<R>(h->g, h->u[h->cur], h->stream), "halo exchange launch");
    return JACOBI_OK;
}

// Adjoint passes: n sweeps of the zero-ring state with the FP64 accumulation.
template <typename R>
int do_adjoint(jacobi_t h, int64_t n) {
    // adjoint passes: depth 7 measured fastest for FP32 on MI355X (4096^2:
    // 820 GLUP/s vs 586 at depth 4; depth 8 runs out of registers for the
    // FP64 accumulator ring)
    int depth = h->adj_depth > 0 ? h->adj_depth : (h->dtype == JACOBI_F32 ? 7 : 3);
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

// A fresh handle's fields over workspace ws (no state, no source, default
// schedule, no profiling).
void init_handle(jacobi_s *h, const Geom &g, const Layout &l, int dtype, void *ws, void *stream) {
    h->g = g;
    h->lay = l;
    h->dtype = dtype;
    h->ws = (char *)ws;
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
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_address(void **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "get device");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(JACOBI_E_UNSUPPORTED, "device index %d beyond the %d the library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (!p) return fail(JACOBI_E_HIP, "scratch symbol address is NULL");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
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
    init_handle(h, g, l, dtype, workspace, stream);
    *out = h;
    return JACOBI_OK;
}

int jacobi_deep_workspace_bytes(int ndim, const int64_t *grid, const int64_t *blocks, int dtype,
                                int halo, size_t *bytes) {
    if (!bytes) return fail(JACOBI_E_INVAL, "bytes must not be NULL");
    Geom g;
    Layout l;
    DeepLayout dl;
    const int rc = plan_deep(ndim, grid, blocks, dtype, halo, &g, &l, &dl);
    if (rc != JACOBI_OK) return rc;
    *bytes = l.bytes;
    return JACOBI_OK;
}

int jacobi_deep_create(int ndim, const int64_t *grid, const int64_t *blocks, int dtype, int halo,
                       void *workspace, size_t workspace_bytes, void *stream, jacobi_t *out) {
    if (!out) return fail(JACOBI_E_INVAL, "out must not be NULL");
    *out = nullptr;
    Geom g;
    Layout l;
    DeepLayout dl;
    int rc = plan_deep(ndim, grid, blocks, dtype, halo, &g, &l, &dl);
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
    init_handle(h, g, l, dtype, workspace, stream);
    char *ws = (char *)workspace;
    h->halo = dl.hs;
    h->bdeep = ws + dl.off_bd;
    h->d_tab[0] = (jac::BatchGrid *)(ws + dl.off_tab);
    h->d_tab[1] = h->d_tab[0] + g.nblocks;
    h->d_prefix = (int *)(ws + dl.off_prefix);
    h->d_active = (int *)(ws + dl.off_active);
    h->d_pc = (int *)(ws + dl.off_pc);
    *out = h;
    return JACOBI_OK;
}

int jacobi_get_halo(jacobi_t h, int *halo) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!halo) return fail(JACOBI_E_INVAL, "halo must not be NULL");
    *halo = h->halo;
    return JACOBI_OK;
}

int jacobi_destroy(jacobi_t h) {
    if (!h) return JACOBI_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (h->stream2) {
        const hipError_t e2 = hipStreamSynchronize(h->stream2);
        if (e == hipSuccess) e = e2;
        hipStreamDestroy(h->stream2);
    }
    for (hipEvent_t ev : h->ev_piece)
        if (ev) hipEventDestroy(ev);
    if (h->ev_join) hipEventDestroy(h->ev_join);
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
    if (h->halo > 0) {
        // every block's whole frame, ring nodes beyond its own ring included
        for (int k = 0; k < 2; ++k)
            HIP_TRY(h->dtype == JACOBI_F32
                        ? jac::launch_deep_exchange<float>(h->g, h->u[k], h->halo, h->stream)
                        : jac::launch_deep_exchange<double>(h->g, h->u[k], h->halo, h->stream),
                    "deep exchange launch");
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
    if (h->halo > 0)
        HIP_TRY(h->dtype == JACOBI_F32
                    ? jac::launch_deep_source<float>(h->g, h->b, h->bdeep, h->halo, h->stream)
                    : jac::launch_deep_source<double>(h->g, h->b, h->bdeep, h->halo, h->stream),
                "deep source launch");
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
    // interval's first pass; the final state's residual needs its own pass.
    // Halos are refreshed after the last interval only (the fused passes
    // and their residuals do not read them).
    int64_t k = 0, i = 0;
    while (k < n_iter) {
        const int64_t step = n_iter - k < check_every ? n_iter - k : check_every;
        const bool last = k + step >= n_iter;
        rc = h->dtype == JACOBI_F32 ? do_sweep<float>(h, step, res_dev + i, last)
                                    : do_sweep<double>(h, step, res_dev + i, last);
        if (rc) return rc;
        k += step;
        ++i;
    }
    return jacobi_residual_async(h, res_dev + i);
}

int jacobi_solve_noalloc(int ndim, const int64_t *grid, const int64_t *blocks, int dtype,
                         const void *u0, const void *f, double h2, int64_t n_iter,
                         int64_t check_every, void *u_out, double *res_dev, void *stream) {
    // every argument check before any HIP call
    Geom g;
    Layout l;
    int rc = plan(ndim, grid, blocks, dtype, &g, &l);
    if (rc != JACOBI_OK) return rc;
    if (!u0 || !u_out || !res_dev) return fail(JACOBI_E_INVAL, "u0, u_out and res_dev must not be NULL");
    if (n_iter < 0) return fail(JACOBI_E_INVAL, "n_iter must be >= 0");
    if (check_every < 1) return fail(JACOBI_E_INVAL, "check_every must be >= 1");
    if (f && (!(h2 > 0.0) || !std::isfinite(h2)))
        return fail(JACOBI_E_INVAL, "h2 must be positive and finite (got %g)", h2);
    if (l.bytes > (size_t)JACOBI_NOALLOC_MAX_BYTES)
        return fail(JACOBI_E_NOMEM,
                    "problem needs %zu bytes of device scratch; jacobi_solve_noalloc holds %zu "
                    "(use jacobi_create with a workspace)",
                    l.bytes, (size_t)JACOBI_NOALLOC_MAX_BYTES);
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != JACOBI_OK) return rc;
    // a handle on the stack over the scratch: host metadata only, nothing to
    // free afterwards (no profiling events, no second stream)
    jacobi_s h;
    init_handle(&h, g, l, dtype, ws, stream);
    if ((rc = jacobi_set_source(&h, f, h2)) != JACOBI_OK) return rc;
    if ((rc = jacobi_set_state(&h, u0)) != JACOBI_OK) return rc;
    if ((rc = jacobi_solve(&h, n_iter, check_every, res_dev)) != JACOBI_OK) return rc;
    return jacobi_get_state(&h, u_out);
}

int jacobi_adjoint_begin(jacobi_t h, const void *lam, double *grad_b) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!lam || !grad_b) return fail(JACOBI_E_INVAL, "lam and grad_b must not be NULL");
    if (h->g.ndim != 2) return fail(JACOBI_E_UNSUPPORTED, "the adjoint is implemented for 2D grids");
    if (!march_fits(h->g, h->dtype))
        return fail(JACOBI_E_UNSUPPORTED,
                    "the adjoint pass needs the grid's block columns to span less than 4 GiB");
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

int jacobi_forward_ckpt(jacobi_t h, int64_t K, int64_t C, void *ckpt) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (K < 0) return fail(JACOBI_E_INVAL, "K must be >= 0 (got %lld)", (long long)K);
    if (C < 1) return fail(JACOBI_E_INVAL, "C must be >= 1 (got %lld)", (long long)C);
    if (!h->has_state) return fail(JACOBI_E_STATE, "no state set (call jacobi_set_state first)");
    const size_t es = h->dtype == JACOBI_F32 ? 4 : 8;
    const size_t state_bytes =
        (size_t)(h->g.n[0] + 2) * (h->g.n[1] + 2) * (h->g.ndim == 3 ? h->g.n[2] + 2 : 1) * es;
    int64_t k = 0, j = 0;
    while (k < K) {
        const int64_t step = K - k < C ? K - k : C;
        if (ckpt) {
            void *dst = (char *)ckpt + (size_t)j * state_bytes;
            if (h->dtype == JACOBI_F32)
                HIP_TRY(jac::launch_gather<float>(h->g, h->u[h->cur], dst, h->stream), "gather launch");
            else
                HIP_TRY(jac::launch_gather<double>(h->g, h->u[h->cur], dst, h->stream), "gather launch");
        }
        // the gather reads block interiors and the domain-edge halos only, so
        // the internal halos are refreshed once, after the last segment
        const bool last = k + step >= K;
        rc = h->dtype == JACOBI_F32 ? do_sweep<float>(h, step, nullptr, last)
                                    : do_sweep<double>(h, step, nullptr, last);
        if (rc) return rc;
        k += step;
        ++j;
    }
    return JACOBI_OK;
}

int jacobi_adjoint(jacobi_t h, int64_t K, int64_t C, const void *dL_duK, double h2, double *dL_df,
                   double *dL_dU0) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (K < 0) return fail(JACOBI_E_INVAL, "K must be >= 0 (got %lld)", (long long)K);
    if (C < 1) return fail(JACOBI_E_INVAL, "C must be >= 1 (got %lld)", (long long)C);
    if (!dL_duK || !dL_df || !dL_dU0)
        return fail(JACOBI_E_INVAL, "dL_duK, dL_df and dL_dU0 must not be NULL");
    if (!(h2 > 0.0) || !std::isfinite(h2))
        return fail(JACOBI_E_INVAL, "h2 must be positive and finite (got %g)", h2);
    if ((void *)dL_df == (void *)dL_dU0) return fail(JACOBI_E_INVAL, "dL_df and dL_dU0 must differ");
    rc = jacobi_adjoint_begin(h, dL_duK, dL_df);
    if (rc) return rc;
    for (int64_t k = 0; k < K && !rc; k += C) rc = jacobi_adjoint_sweep(h, K - k < C ? K - k : C);
    if (rc) {
        h->gacc = nullptr;
        return rc;
    }
    // dL/dU0 reads the accumulator before it is scaled in place into dL/df
    if (h->dtype == JACOBI_F32)
        HIP_TRY(jac::launch_adjoint_full<float>(h->g, dL_df, dL_duK, h->u[h->cur], dL_dU0, h->stream),
                "adjoint finish launch");
    else
        HIP_TRY(jac::launch_adjoint_full<double>(h->g, dL_df, dL_duK, h->u[h->cur], dL_dU0, h->stream),
                "adjoint finish launch");
    return jacobi_adjoint_end(h, h2, dL_df, nullptr);
}

int jacobi_set_tuning(jacobi_t h, int t_depth, int rows, int flags) {
    int rc = check_handle(h);
    if (rc) return rc;
    const int md = max_depth(h->g.ndim, h->dtype);
    if (t_depth < 0 || t_depth > md)
        return fail(JACOBI_E_INVAL, "t_depth must be in [0, %d] (got %d)", md, t_depth);
    // rows: tile height of the 2D pass kernels and z segment of the 3D ones
    // (>= kMinRows, which sizes the residual partials); rows per work item of
    // the explicit 2D sweep (>= 1)
    const int min_rows =
        ((flags & JACOBI_FLAG_EXPLICIT_HALO) && h->g.ndim == 2) ? 1 : kMinRows;
    if (rows < 0 || (rows > 0 && rows < min_rows) || rows > (1 << 20))
        return fail(JACOBI_E_INVAL, "rows must be 0 or in [%d, 2^20] (got %d)", min_rows, rows);
    if (flags & ~(JACOBI_FLAG_EXPLICIT_HALO | JACOBI_FLAG_NT_STORES | JACOBI_FLAG_DEEP_PREFETCH |
                  JACOBI_FLAG_OVERLAP))
        return fail(JACOBI_E_INVAL, "unknown flags 0x%x", flags);
    if ((flags & JACOBI_FLAG_OVERLAP) && !(flags & JACOBI_FLAG_EXPLICIT_HALO))
        return fail(JACOBI_E_INVAL, "JACOBI_FLAG_OVERLAP needs JACOBI_FLAG_EXPLICIT_HALO");
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
    if (h->rows > 0)
        *rows = h->rows;
    else if (h->halo > 0 && h->g.ndim == 3)
        *rows = h->g.e[2] + 2 * (h->halo - 1);  // deep-halo passes: one z segment per block
    else
        *rows = h->g.ndim == 3 ? zseg_of(h) : default_rows(h);
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
        if (h->g.ndim == 2)
            for (int rg : {2, 4, 8, 16}) cands.push_back({1, rg, JACOBI_FLAG_EXPLICIT_HALO});
        cands.push_back({1, 0, JACOBI_FLAG_EXPLICIT_HALO | JACOBI_FLAG_OVERLAP});
        if (h->g.ndim == 3) {
            static const int kZseg[] = {16, 32, 64, 128};
            for (int d = 1; d <= jac::march3d_max_depth(); ++d)
                for (int z : kZseg)
                    for (int f : {0, (int)JACOBI_FLAG_NT_STORES}) cands.push_back({d, z, f});
        }
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
                    cands.push_back({list[i], r, (int)JACOBI_FLAG_NT_STORES});
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

// ====================================================================== batch
namespace {

constexpr int kMaxDepth = 16;  // deepest pass kernel (FP32)

struct BatchLayout {
    std::vector<Geom> geoms;
    std::vector<Layout> lays;
    std::vector<size_t> base;  // workspace offset of each grid's buffers
    size_t off_grids, off_prefix, off_state, off_part, part_cap, bytes;
};

// Pick blocks per axis so that blocks have about `block` interior nodes per side.
int batch_plan(int count, const int64_t *grids, int64_t block, int dtype, BatchLayout *bl) {
    if (count < 1 || count > (1 << 20)) return fail(JACOBI_E_INVAL, "count must be in [1, 2^20]");
    if (!grids) return fail(JACOBI_E_INVAL, "grids must not be NULL");
    if (block < 8 || block > (1 << 30)) return fail(JACOBI_E_INVAL, "block must be in [8, 2^30]");
    bl->geoms.resize(count);
    bl->lays.resize(count);
    bl->base.resize(count);
    size_t off = 0, cap = 0, t;
    for (int i = 0; i < count; ++i) {
        const int64_t g2[2] = {grids[2 * i], grids[2 * i + 1]};
        if (g2[0] < 1 || g2[1] < 1 || g2[0] > (1 << 30) || g2[1] > (1 << 30))
            return fail(JACOBI_E_INVAL, "grid %d has a side out of [1, 2^30]", i);
        int64_t b2[2];
        int rc = JACOBI_E_INVAL;
        for (int a = 0; a < 2; ++a) b2[a] = (g2[a] + block - 1) / block;
        // the x extent is rounded up to 32 bytes of elements, which can leave
        // the last block empty: use fewer blocks until the split is valid
        for (int tries = 0; tries < 64 && rc != JACOBI_OK; ++tries) {
            rc = plan(2, g2, b2, dtype, &bl->geoms[i], &bl->lays[i]);
            if (rc != JACOBI_OK) {
                if (b2[0] > 1) --b2[0];
                else if (b2[1] > 1) --b2[1];
                else break;
            }
        }
        if (rc != JACOBI_OK) return rc;
        if (!march_fits(bl->geoms[i], dtype))
            return fail(JACOBI_E_INVAL, "grid %d: block columns span 4 GiB or more", i);
        bl->base[i] = off;
        // a grid needs its two state buffers and its source (not the
        // single-grid partials/scratch area)
        if (!add_ok(off, bl->lays[i].off_part, &t)) return fail(JACOBI_E_INVAL, "size overflow");
        off = round_up(t, kAlign);
        cap += ((size_t)g2[0] / 32 + 2) * ((size_t)g2[1] / kMinRows + 2);
    }
    bl->off_grids = off;
    off = round_up(off + sizeof(jac::BatchGrid) * count, kAlign);
    bl->off_prefix = off;
    off = round_up(off + sizeof(int) * (size_t)(count + 1) * (kMaxDepth + 1), kAlign);
    bl->off_state = off;
    // active, status, final_buf (int); sweeps (int64); rel, res0, res (double); 2 counters
    off = round_up(off + (size_t)count * (3 * sizeof(int) + sizeof(long long) + 3 * sizeof(double)) +
                       64,
                   kAlign);
    bl->off_part = off;
    bl->part_cap = cap;
    if (!add_ok(off, sizeof(double) * cap, &t)) return fail(JACOBI_E_INVAL, "size overflow");
    bl->bytes = round_up(t, kAlign);
    return JACOBI_OK;
}

}  // namespace

struct jacobi_batch_s {
    int count, dtype;
    BatchLayout bl;
    char *ws;
    hipStream_t stream;
    jac::BatchGrid *d_grids;
    int *d_prefix;  // (kMaxDepth + 1) arrays of count + 1 work offsets, indexed by depth
    jac::BatchState st;
    double *partials;
    std::vector<jac::BatchGrid> h_grids;
    std::vector<int> h_prefix;
    std::vector<int> h_final_buf;
    std::vector<char> grid_set;
    int depth, rows, use_graph;
    int table_rows;  // tile height the uploaded tables were built for (0: none)
    int *h_active;   // pinned host copy of the activity flags
    // captured interval
    hipGraphExec_t graph;
    int64_t graph_R;
    int graph_depth, graph_rows;
    double graph_tol;
};

namespace {

int batch_check(jacobi_batch_t b) {
    if (!b) return fail(JACOBI_E_INVAL, "batch handle is NULL");
    return JACOBI_OK;
}

void batch_drop_graph(jacobi_batch_t b) {
    if (b->graph) hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_R = 0;
}

int batch_rows(const jacobi_batch_t b) { return b->rows > 0 ? b->rows : 64; }
int batch_depth(const jacobi_batch_t b) {
    return b->depth > 0 ? b->depth : (b->dtype == JACOBI_F32 ? 7 : 4);
}

// Work tables for the current tile height: per grid its tiles per strip, and
// per depth the prefix sums of work items.  Uploaded when the height changes.
template <typename R>
int batch_tables(jacobi_batch_t b) {
    const int rows = batch_rows(b);
    if (b->table_rows == rows) return JACOBI_OK;
    const int n = b->count;
    b->h_prefix.assign((size_t)(kMaxDepth + 1) * (n + 1), 0);
    for (int d = 1; d <= kMaxDepth; ++d) {
        int *pre = &b->h_prefix[(size_t)d * (n + 1)];
        int64_t acc = 0;
        for (int i = 0; i < n; ++i) {
            pre[i] = (int)acc;
            const int64_t w = jac::march2d_batch_work<R>(b->bl.geoms[i], d, rows);
            if (w < 0) { acc = -1; break; }
            acc += w;
            if (acc > 0x3fffffff) return fail(JACOBI_E_INVAL, "batch work exceeds 2^30 items");
        }
        if (acc >= 0) {
            pre[n] = (int)acc;
            if ((size_t)acc > b->bl.part_cap) return fail(JACOBI_E_INVAL, "partials overflow");
        }
    }
    HIP_TRY(hipMemcpyAsync(b->d_grids, b->h_grids.data(), sizeof(jac::BatchGrid) * n,
                           hipMemcpyHostToDevice, b->stream),
            "batch table upload");
    HIP_TRY(hipMemcpyAsync(b->d_prefix, b->h_prefix.data(), sizeof(int) * b->h_prefix.size(),
                           hipMemcpyHostToDevice, b->stream),
            "batch table upload");
    HIP_TRY(hipStreamSynchronize(b->stream), "stream synchronize");
    b->table_rows = rows;
    batch_drop_graph(b);
    return JACOBI_OK;
}

// Depths of the passes of an interval of n sweeps (even split, at most `depth`).
std::vector<int> batch_passes(int dtype, int depth, int64_t n) {
    std::vector<int> out;
    int64_t left = n;
    while (left > 0) {
        const int64_t passes = (left + depth - 1) / depth;
        const int t = pick_depth(dtype, (int)((left + passes - 1) / passes));
        out.push_back(t);
        left -= t;
    }
    return out;
}

// One check interval: passes of n sweeps in total, the first also summing the
// residual of the interval's starting state, which the stop test then checks.
// check = false (autotuning): no residual and no stop test, so scratch
// contents cannot deactivate grids and every candidate does the full work.
template <typename R>
int batch_interval(jacobi_batch_t b, int64_t n, double tol, bool check = true) {
    const std::vector<int> ds = batch_passes(b->dtype, batch_depth(b), n);
    const int rows = batch_rows(b);
    const int cnt = b->count;
    for (size_t p = 0; p < ds.size(); ++p) {
        const int t = ds[p];
        const int *pre = b->d_prefix + (size_t)t * (cnt + 1);
        const int nwork = b->h_prefix[(size_t)t * (cnt + 1) + cnt];
        HIP_TRY(jac::launch_march2d_batch<R>(b->d_grids, pre, cnt, b->st.active, b->st.pass_count,
                                             (p == 0 && check) ? b->partials : nullptr, true, t,
                                             rows, nwork, b->stream),
                "batch pass launch");
        if (p == 0 && check)
            HIP_TRY(jac::launch_batch_check(pre, b->partials, cnt, b->st, tol, false, b->stream),
                    "batch check launch");
        HIP_TRY(jac::launch_batch_advance(b->st, t, b->stream), "batch advance launch");
    }
    return JACOBI_OK;
}

// Residual of the current states of the active grids and the final test.
template <typename R>
int batch_final(jacobi_batch_t b, double tol) {
    const int cnt = b->count;
    const int *pre = b->d_prefix + (size_t)1 * (cnt + 1);
    const int nwork = b->h_prefix[(size_t)1 * (cnt + 1) + cnt];
    HIP_TRY(jac::launch_march2d_batch<R>(b->d_grids, pre, cnt, b->st.active, b->st.pass_count,
                                         b->partials, false, 1, batch_rows(b), nwork, b->stream),
            "batch residual launch");
    HIP_TRY(jac::launch_batch_check(pre, b->partials, cnt, b->st, tol, true, b->stream),
            "batch check launch");
    return JACOBI_OK;
}

template <typename R>
int batch_capture(jacobi_batch_t b, int64_t n, double tol) {
    if (b->graph && b->graph_R == n && b->graph_depth == batch_depth(b) &&
        b->graph_rows == batch_rows(b) && b->graph_tol == tol)
        return JACOBI_OK;
    batch_drop_graph(b);
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    const int rc = batch_interval<R>(b, n, tol);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (rc) {
        if (graph) hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e2 != hipSuccess) return hip_fail(e2, "graph instantiate");
    b->graph = exec;
    b->graph_R = n;
    b->graph_depth = batch_depth(b);
    b->graph_rows = batch_rows(b);
    b->graph_tol = tol;
    return JACOBI_OK;
}

template <typename R>
int batch_solve(jacobi_batch_t b, double tol, int64_t max_sweeps, int64_t R_, int64_t *sweeps,
                double *rel, int *status) {
    int rc = batch_tables<R>(b);
    if (rc) return rc;
    const int cnt = b->count;
    HIP_TRY(jac::launch_batch_init(cnt, b->st, b->stream), "batch init launch");
    const int64_t full = max_sweeps / R_, rem = max_sweeps % R_;
    const bool graphs = b->use_graph && b->stream != nullptr && full > 0;
    if (graphs) {
        rc = batch_capture<R>(b, R_, tol);
        if (rc) return rc;
    }
    for (int64_t i = 0; i < full; ++i) {
        if (graphs)
            HIP_TRY(hipGraphLaunch(b->graph, b->stream), "graph launch");
        else if ((rc = batch_interval<R>(b, R_, tol)))
            return rc;
        if ((i + 1) % 4 == 0 && i + 1 < full) {
            // stop early once every grid has stopped
            HIP_TRY(hipMemcpyAsync(b->h_active, b->st.active, sizeof(int) * cnt,
                                   hipMemcpyDeviceToHost, b->stream),
                    "activity copy");
            HIP_TRY(hipStreamSynchronize(b->stream), "stream synchronize");
            int any = 0;
            for (int g = 0; g < cnt; ++g) any |= b->h_active[g];
            if (!any) break;
        }
    }
    if (rem > 0 && (rc = batch_interval<R>(b, rem, tol))) return rc;
    if ((rc = batch_final<R>(b, tol))) return rc;
    std::vector<long long> sw(cnt);
    std::vector<double> rl(cnt);
    std::vector<int> stt(cnt);
    HIP_TRY(hipMemcpyAsync(sw.data(), b->st.sweeps, sizeof(long long) * cnt, hipMemcpyDeviceToHost,
                           b->stream),
            "result copy");
    HIP_TRY(hipMemcpyAsync(rl.data(), b->st.rel, sizeof(double) * cnt, hipMemcpyDeviceToHost,
                           b->stream),
            "result copy");
    HIP_TRY(hipMemcpyAsync(stt.data(), b->st.status, sizeof(int) * cnt, hipMemcpyDeviceToHost,
                           b->stream),
            "result copy");
    HIP_TRY(hipMemcpyAsync(b->h_final_buf.data(), b->st.final_buf, sizeof(int) * cnt,
                           hipMemcpyDeviceToHost, b->stream),
            "result copy");
    HIP_TRY(hipStreamSynchronize(b->stream), "stream synchronize");
    for (int g = 0; g < cnt; ++g) {
        if (sweeps) sweeps[g] = sw[g];
        if (rel) rel[g] = rl[g];
        if (status) status[g] = stt[g];
    }
    return JACOBI_OK;
}

}  // namespace

extern "C" {

int jacobi_batch_workspace_bytes(int count, const int64_t *grids, int64_t block, int dtype,
                                 size_t *bytes) {
    if (!bytes) return fail(JACOBI_E_INVAL, "bytes must not be NULL");
    BatchLayout bl;
    const int rc = batch_plan(count, grids, block, dtype, &bl);
    if (rc) return rc;
    *bytes = bl.bytes;
    return JACOBI_OK;
}

int jacobi_batch_create(int count, const int64_t *grids, int64_t block, int dtype,
                        void *workspace, size_t workspace_bytes, void *stream,
                        jacobi_batch_t *out) {
    if (!out) return fail(JACOBI_E_INVAL, "out must not be NULL");
    *out = nullptr;
    BatchLayout bl;
    int rc = batch_plan(count, grids, block, dtype, &bl);
    if (rc) return rc;
    if (!workspace) return fail(JACOBI_E_INVAL, "workspace must not be NULL");
    if ((uintptr_t)workspace % kAlign)
        return fail(JACOBI_E_INVAL, "workspace must be %zu-byte aligned", kAlign);
    if (workspace_bytes < bl.bytes)
        return fail(JACOBI_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, bl.bytes);
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, workspace);
    if (e != hipSuccess) return hip_fail(e, "workspace pointer query");
    if (attr.type != hipMemoryTypeDevice) return fail(JACOBI_E_INVAL, "workspace is not device memory");
    jacobi_batch_s *b = new (std::nothrow) jacobi_batch_s();
    if (!b) return fail(JACOBI_E_NOMEM, "host allocation failed");
    b->count = count;
    b->dtype = dtype;
    b->bl = bl;
    b->ws = (char *)workspace;
    b->stream = (hipStream_t)stream;
    b->d_grids = (jac::BatchGrid *)(b->ws + bl.off_grids);
    b->d_prefix = (int *)(b->ws + bl.off_prefix);
    char *sp = b->ws + bl.off_state;
    b->st.active = (int *)sp;
    b->st.status = b->st.active + count;
    b->st.final_buf = b->st.status + count;
    sp = (char *)round_up((uintptr_t)(b->st.final_buf + count), 8);
    b->st.sweeps = (long long *)sp;
    b->st.rel = (double *)(b->st.sweeps + count);
    b->st.res0 = b->st.rel + count;
    b->st.res = b->st.res0 + count;
    b->st.k_now = (long long *)(b->st.res + count);
    b->st.pass_count = (int *)(b->st.k_now + 1);
    b->partials = (double *)(b->ws + bl.off_part);
    b->h_grids.resize(count);
    for (int i = 0; i < count; ++i) {
        jac::BatchGrid &g = b->h_grids[i];
        std::memset(&g, 0, sizeof g);
        g.g = bl.geoms[i];
        g.u[0] = b->ws + bl.base[i] + bl.lays[i].off_u0;
        g.u[1] = b->ws + bl.base[i] + bl.lays[i].off_u1;
        g.b = b->ws + bl.base[i] + bl.lays[i].off_b;
    }
    b->h_final_buf.assign(count, 0);
    b->grid_set.assign(count, 0);
    b->depth = 0;
    b->rows = 0;
    b->use_graph = 1;
    b->table_rows = 0;
    b->graph = nullptr;
    b->graph_R = 0;
    if (hipHostMalloc((void **)&b->h_active, sizeof(int) * count, hipHostMallocDefault) != hipSuccess) {
        delete b;
        return fail(JACOBI_E_NOMEM, "pinned host allocation failed");
    }
    *out = b;
    return JACOBI_OK;
}

int jacobi_batch_destroy(jacobi_batch_t b) {
    if (!b) return JACOBI_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    hipHostFree(b->h_active);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "stream synchronize in destroy");
    return JACOBI_OK;
}

int jacobi_batch_set_grid(jacobi_batch_t b, int i, const void *u, const void *f, double h2) {
    int rc = batch_check(b);
    if (rc) return rc;
    if (i < 0 || i >= b->count) return fail(JACOBI_E_INVAL, "grid index %d out of range", i);
    if (!u || !f) return fail(JACOBI_E_INVAL, "u and f must not be NULL");
    if (!(h2 > 0.0) || !std::isfinite(h2))
        return fail(JACOBI_E_INVAL, "h2 must be positive and finite (got %g)", h2);
    const jac::BatchGrid &g = b->h_grids[i];
    if (b->dtype == JACOBI_F32) {
        HIP_TRY(jac::launch_scatter<float>(g.g, u, g.u[0], g.u[1], false, b->stream), "scatter launch");
        HIP_TRY(jac::launch_halo_exchange<float>(g.g, g.u[0], b->stream), "halo launch");
        HIP_TRY(jac::launch_halo_exchange<float>(g.g, g.u[1], b->stream), "halo launch");
        HIP_TRY(jac::launch_scale_source<float>(g.g, f, (void *)g.b, h2, b->stream), "source launch");
    } else {
        HIP_TRY(jac::launch_scatter<double>(g.g, u, g.u[0], g.u[1], false, b->stream), "scatter launch");
        HIP_TRY(jac::launch_halo_exchange<double>(g.g, g.u[0], b->stream), "halo launch");
        HIP_TRY(jac::launch_halo_exchange<double>(g.g, g.u[1], b->stream), "halo launch");
        HIP_TRY(jac::launch_scale_source<double>(g.g, f, (void *)g.b, h2, b->stream), "source launch");
    }
    b->h_final_buf[i] = 0;
    b->grid_set[i] = 1;
    return JACOBI_OK;
}

int jacobi_batch_get_grid(jacobi_batch_t b, int i, void *u) {
    int rc = batch_check(b);
    if (rc) return rc;
    if (i < 0 || i >= b->count) return fail(JACOBI_E_INVAL, "grid index %d out of range", i);
    if (!u) return fail(JACOBI_E_INVAL, "u must not be NULL");
    if (!b->grid_set[i]) return fail(JACOBI_E_STATE, "grid %d has no state", i);
    const jac::BatchGrid &g = b->h_grids[i];
    const void *src = g.u[b->h_final_buf[i] & 1];
    if (b->dtype == JACOBI_F32)
        HIP_TRY(jac::launch_gather<float>(g.g, src, u, b->stream), "gather launch");
    else
        HIP_TRY(jac::launch_gather<double>(g.g, src, u, b->stream), "gather launch");
    return JACOBI_OK;
}

int jacobi_batch_set_tuning(jacobi_batch_t b, int t_depth, int rows, int use_graph) {
    int rc = batch_check(b);
    if (rc) return rc;
    const int md = max_depth(2, b->dtype);
    if (t_depth < 0 || t_depth > md)
        return fail(JACOBI_E_INVAL, "t_depth must be in [0, %d] (got %d)", md, t_depth);
    if (rows < 0 || (rows > 0 && rows < kMinRows) || rows > (1 << 20))
        return fail(JACOBI_E_INVAL, "rows must be 0 or in [%d, 2^20] (got %d)", kMinRows, rows);
    b->depth = t_depth;
    b->rows = rows;
    b->use_graph = use_graph ? 1 : 0;
    batch_drop_graph(b);
    return JACOBI_OK;
}

int jacobi_batch_get_tuning(jacobi_batch_t b, int *t_depth, int *rows, int *use_graph) {
    int rc = batch_check(b);
    if (rc) return rc;
    if (t_depth) *t_depth = batch_depth(b);
    if (rows) *rows = batch_rows(b);
    if (use_graph) *use_graph = b->use_graph;
    return JACOBI_OK;
}

int jacobi_batch_solve(jacobi_batch_t b, double rel_tol, int64_t max_sweeps, int64_t check_every,
                       int64_t *sweeps, double *rel, int *status) {
    int rc = batch_check(b);
    if (rc) return rc;
    if (max_sweeps < 0) return fail(JACOBI_E_INVAL, "max_sweeps must be >= 0");
    if (check_every < 1) return fail(JACOBI_E_INVAL, "check_every must be >= 1");
    if (!(rel_tol >= 0.0)) return fail(JACOBI_E_INVAL, "rel_tol must be >= 0");
    for (int i = 0; i < b->count; ++i)
        if (!b->grid_set[i]) return fail(JACOBI_E_STATE, "grid %d has no state", i);
    return b->dtype == JACOBI_F32 ? batch_solve<float>(b, rel_tol, max_sweeps, check_every, sweeps, rel, status)
                                  : batch_solve<double>(b, rel_tol, max_sweeps, check_every, sweeps, rel, status);
}

int jacobi_batch_autotune(jacobi_batch_t b, int64_t check_every, int *t_depth, int *rows) {
    int rc = batch_check(b);
    if (rc) return rc;
    if (check_every < 1 || check_every > (1 << 20)) return fail(JACOBI_E_INVAL, "check_every out of range");
    static const int kRows[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 320, 384};
    const int *list;
    const int nd = jac::march2d_depths(b->dtype, &list);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event create");
    HIP_TRY(hipEventCreate(&e1), "event create");
    const int saved_graph = b->use_graph;
    float best = 1e30f;
    int bd = 0, br = 0;
    for (int i = 0; i < nd && !rc; ++i) {
        for (int r : kRows) {
            b->depth = list[i];
            b->rows = r;
            b->use_graph = 0;
            rc = b->dtype == JACOBI_F32 ? batch_tables<float>(b) : batch_tables<double>(b);
            if (rc) break;
            HIP_TRY(jac::launch_batch_init(b->count, b->st, b->stream), "batch init launch");
            rc = b->dtype == JACOBI_F32 ? batch_interval<float>(b, check_every, 0.0, false)
                                        : batch_interval<double>(b, check_every, 0.0, false);
            if (rc) break;
            if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = JACOBI_E_HIP; break; }
            rc = b->dtype == JACOBI_F32 ? batch_interval<float>(b, check_every, 0.0, false)
                                        : batch_interval<double>(b, check_every, 0.0, false);
            if (rc) break;
            float t = 0.0f;
            if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                rc = fail(JACOBI_E_HIP, "batch autotune timing failed");
                break;
            }
            if (t < best) {
                best = t;
                bd = list[i];
                br = r;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->use_graph = saved_graph;
    // the grids' buffers served as scratch
    for (int i = 0; i < b->count; ++i) b->grid_set[i] = 0;
    if (rc) return rc;
    b->depth = bd;
    b->rows = br;
    batch_drop_graph(b);
    if (t_depth) *t_depth = bd;
    if (rows) *rows = br;
    return JACOBI_OK;
}

}  // extern "C"
