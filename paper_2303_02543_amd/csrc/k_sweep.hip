// Jacobi sweep kernels for gfx950.
//
// The update is the synchronous 5-point (2D) / 7-point (3D) Jacobi step of
// the proxy application in Section 4.3 of the paper, evaluated in the fixed
// order
//   2D  s = (W + E) + (S + N);            u' = (s + b) * 1/4
//   3D  s = ((W + E) + (S + N)) + (B + F); u' = (s + b) * fl(1/6)
// with no contraction into FMA (the library is built with -ffp-contract=off)
// and IEEE denormals, so results are identical whatever the schedule.
//
// This file holds the one-sweep kernels: the block-local sweep (every block
// from its own storage, its interior plus the one-cell halo a preceding halo
// exchange filled -- the step order of the paper's proxy: exchange, then
// update) and the fused 2D tile sweep, which reads the cells just outside a
// block from the neighbouring blocks that own them.  The multi-sweep pass
// kernels live in k_march2d.hip and k_march3d.hip.
//
// 2D blocks use k_sweep_tile (a workgroup walks a tile of rows 4 at a time,
// sharing rows through LDS) or, for 1-3 rows per work item, k_sweep_rows (a
// wave walks a short group of rows, keeping the rows above and below in
// registers).  Both take west/east neighbours from the adjacent lanes (DPP)
// and number work items in memory order (column chunk, then rows, then
// block), so the waves resident at any time stream one compact window of the
// arrays, the access pattern HBM serves best.  3D blocks use k_sweep_local.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

template <typename R> __device__ __forceinline__ R weight2d() { return (R)0.25; }

// ------------------------------------------------------------ local sweep
// One thread per V-element chunk of a block row; everything read from the
// block's own storage.  Work items cover max-extent blocks; chunks outside a
// smaller block's extent exit.
template <typename R, bool SRC>
__global__ __launch_bounds__(256) void k_sweep_local(Geom g, const R *__restrict__ uin,
                                                     R *__restrict__ uout,
                                                     const R *__restrict__ b, int64_t blk0,
                                                     int64_t total) {
    constexpr int V = 16 / sizeof(R);
    const int cpr = (g.e[0] + V - 1) / V;           // chunks per row
    const int64_t rows = (int64_t)g.e[1] * (g.ndim == 3 ? g.e[2] : 1);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int cx = (int)(i % cpr);
    const int64_t rest = i / cpr;
    const int64_t rr = rest % rows;
    const int64_t blk = blk0 + rest / rows;
    const int ly = (int)(rr % g.e[1]);
    const int lz = (int)(rr / g.e[1]);
    const int bx = (int)(blk % g.nb[0]);
    const int by = (int)((blk / g.nb[0]) % g.nb[1]);
    const int bz = (int)(blk / ((int64_t)g.nb[0] * g.nb[1]));
    const int ex = extent(g.n[0], g.e[0], bx);
    const int ey = extent(g.n[1], g.e[1], by);
    const int ez = g.ndim == 3 ? extent(g.n[2], g.e[2], bz) : 1;
    const int c = cx * V;
    if (c >= ex || ly >= ey || lz >= ez) return;
    const int64_t o = local_offset(g, blk, c, ly, lz);
    const Chunk<R, V> cen = *reinterpret_cast<const Chunk<R, V> *>(uin + o);
    const Chunk<R, V> dn = *reinterpret_cast<const Chunk<R, V> *>(uin + o - g.pitch);
    const Chunk<R, V> up = *reinterpret_cast<const Chunk<R, V> *>(uin + o + g.pitch);
    const R west = uin[o - 1];
    const R east = (c + V <= ex) ? uin[o + V] : (R)0;
    Chunk<R, V> bb;
    if (SRC) bb = *reinterpret_cast<const Chunk<R, V> *>(
                 b + blk * g.sstride + ((int64_t)lz * g.e[1] + ly) * g.e[0] + c);
    Chunk<R, V> out;
    if (g.ndim == 2) {
        const R w = weight2d<R>();
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R W = v > 0 ? cen.v[v - 1] : west;
            const R E = v < V - 1 ? cen.v[v + 1] : east;
            const R s = (W + E) + (dn.v[v] + up.v[v]);
            out.v[v] = SRC ? (s + bb.v[v]) * w : s * w;
        }
    } else {
        const R w = (R)1 / (R)6;
        const Chunk<R, V> bk = *reinterpret_cast<const Chunk<R, V> *>(uin + o - g.plane);
        const Chunk<R, V> fr = *reinterpret_cast<const Chunk<R, V> *>(uin + o + g.plane);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R W = v > 0 ? cen.v[v - 1] : west;
            const R E = v < V - 1 ? cen.v[v + 1] : east;
            const R s = ((W + E) + (dn.v[v] + up.v[v])) + (bk.v[v] + fr.v[v]);
            out.v[v] = SRC ? (s + bb.v[v]) * w : s * w;
        }
    }
    if (c + V <= ex) {
        *reinterpret_cast<Chunk<R, V> *>(uout + o) = out;
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (c + v < ex) uout[o + v] = out.v[v];
    }
}

// ------------------------------------------------------------ row sweep (2D)
template <typename R, bool SRC>
__global__ __launch_bounds__(256) void k_sweep_rows(Geom g, const R *__restrict__ uin,
                                                    R *__restrict__ uout,
                                                    const R *__restrict__ b, int rg, int ngroups,
                                                    int nchunks, int blk0, int nwork) {
    constexpr int V = 16 / sizeof(R);
    constexpr int W = 64 * V;
    using C = Chunk<R, V>;
    // plain workgroup order: consecutive workgroups, dealt round-robin over
    // the XCDs, cover consecutive memory, so the whole chip streams one
    // window (measured faster here than giving each XCD its own range)
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wid >= nwork) return;
    const int chunk = wid % nchunks;
    const int rest = wid / nchunks;
    const int grp = rest % ngroups;
    const int blk = blk0 + rest / ngroups;
    const int bx = blk % g.nb[0], by = blk / g.nb[0];
    const int ex = extent(g.n[0], g.e[0], bx);
    const int ey = extent(g.n[1], g.e[1], by);
    const int ly0 = grp * rg;
    if (ly0 >= ey) return;  // row group beyond a short block (wave-uniform)
    const int ly1 = ly0 + rg < ey ? ly0 + rg : ey;
    const int lane = threadIdx.x & 63;
    const int c = chunk * W + lane * V;
    // lanes whose chunk holds interior cells or the east ring cell load it;
    // lane 0 also needs the cell west of the wave, lane 63 the one east of it
    const bool ld = c <= ex;
    const int xe = lane == 0 ? c - 1 : lane == 63 ? c + V : c;
    const bool lde = xe <= ex && (lane == 0 || lane == 63 || ld);
    // byte offsets from the start of a stored row (column -1 is at ax - 1,
    // so every offset is non-negative)
    const R *base = uin + (int64_t)blk * g.bstride;
    const uint32_t lane_b = (uint32_t)((g.ax + (ld ? c : 0)) * (int)sizeof(R));
    const uint32_t edge_b = (uint32_t)((g.ax + (lde ? xe : 0)) * (int)sizeof(R));
    bool upd[V];
#pragma unroll
    for (int v = 0; v < V; ++v) upd[v] = c + v < ex;
    const bool full = c + V <= ex;
    auto row_of = [&](int ly) { return base + (int64_t)(ly + 1) * g.pitch; };
    auto load = [&](int ly) {
        C r = at<C>(row_of(ly), lane_b);
        if (!ld) {
#pragma unroll
            for (int v = 0; v < V; ++v) r.v[v] = (R)0;
        }
        return r;
    };
    const R *bsrc = SRC ? b + (int64_t)blk * g.sstride : nullptr;
    C up = load(ly0 - 1), cen = load(ly0);
    R e = at<R>(row_of(ly0), edge_b);
    const R w = (R)0.25;
    for (int ly = ly0; ly < ly1; ++ly) {
        // next row and the next edge cell first, so their loads overlap this row
        const C dn = load(ly + 1);
        const R e_next = at<R>(row_of(ly + 1), edge_b);
        C bb;
        if constexpr (SRC) {
            bb = at<C>(bsrc + (int64_t)ly * g.e[0],
                       (uint32_t)((ld && c < ex ? c : 0) * (int)sizeof(R)));
        }
        const R eo = lde ? e : (R)0;
        const R left = shift_up(eo, cen.v[V - 1]);
        const R right = shift_down(eo, cen.v[0]);
        C out;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R Wv = v > 0 ? cen.v[v - 1] : left;
            const R Ev = v < V - 1 ? cen.v[v + 1] : right;
            const R sum = (Wv + Ev) + (up.v[v] + dn.v[v]);
            out.v[v] = SRC ? (sum + bb.v[v]) * w : sum * w;
        }
        R *orow = uout + (int64_t)blk * g.bstride + (int64_t)(ly + 1) * g.pitch;
        if (full) {
            at_mut<C>(orow, lane_b) = out;
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (upd[v]) orow[g.ax + c + v] = out.v[v];
        }
        up = cen;
        cen = dn;
        e = e_next;
    }
}

// ------------------------------------------------------- tile sweep (2D)
// A workgroup of 4 waves owns one 64 x V column chunk of a block and a tile
// of 4 * steps rows, and walks down it 4 rows per step (wave q takes row
// Y + q).  Each row is loaded from memory once: the waves put their rows in
// LDS and take the rows above and below from there; wave 3 also loads the
// row after the step's 4 rows, and wave 0 takes the row before them from the
// previous step's buffer.  Three LDS buffers by step make one barrier per
// step enough: a wave is at most one step ahead of the others, so a buffer
// being written is never one still being read.
//
// FUSED: the cells just outside the block (the row above and below it, the
// column left and right of it) are read from the neighbouring blocks that
// own them instead of from the block's stored halo, so no halo exchange has
// to run before the sweep (the exchange fused into the loads); on the
// domain's boundary the stored halo is the Dirichlet ring and is read as it
// is.  RES: each wave also sums the FP64 residual of its input rows into
// res[4 * item + wave].
//
// Work items are numbered in memory order (column chunk fastest, then tile,
// then block).  Workgroups are dealt round-robin over the 8 XCDs; runs of
// `group` consecutive items go to one XCD (see tile_item), so the row a tile
// shares with the tile below it is fetched into that XCD's L2 once while the
// whole chip still streams one compact window of memory.

// Logical item of physical workgroup p out of np: XCD x = p % 8 takes its
// k-th workgroup (k = p / 8) from run k / group of its own runs, which
// interleave with the other XCDs' runs in memory order.  Workgroups past
// the last whole round of 8 runs keep their own number.
__device__ __forceinline__ int tile_item(int p, int np, int group) {
    const int round = 8 * group;
    const int full = np / round * round;
    if (group <= 1 || p >= full) return p;
    const int x = p & 7, k = p >> 3;
    return (k / group) * round + x * group + (k % group);
}

template <typename R, bool SRC, bool FUSED, bool RES>
__global__ __launch_bounds__(256) void k_sweep_tile(Geom g, const R *__restrict__ uin,
                                                    R *__restrict__ uout,
                                                    const R *__restrict__ b,
                                                    double *__restrict__ res, int steps,
                                                    int ntiles, int nchunks, int blk0,
                                                    int nitems, int group, int nt) {
    constexpr int V = 16 / sizeof(R);
    constexpr int W = 64 * V;
    using C = Chunk<R, V>;
    __shared__ C sh[3][6][64];  // slots 1..4: the step's rows, 5: the row after
    const int item = tile_item(blockIdx.x, gridDim.x, group);
    if (item >= nitems) return;   // whole workgroup
    const int chunk = item % nchunks;
    const int rest = item / nchunks;
    const int tile = rest % ntiles;
    const int blk = blk0 + rest / ntiles;
    const int bx = blk % g.nb[0], by = blk / g.nb[0];
    const int ex = extent(g.n[0], g.e[0], bx);
    const int ey = extent(g.n[1], g.e[1], by);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int y0 = tile * 4 * steps;
    if (y0 >= ey) {  // tile beyond a short block (whole workgroup)
        if (RES && lane == 0) res[4 * (int64_t)item + wv] = 0.0;
        return;
    }
    const int nst = ((ey - y0 < 4 * steps ? ey - y0 : 4 * steps) + 3) / 4;
    const int c = chunk * W + lane * V;
    const bool ld = c <= ex;
    // byte offsets from the start of a stored row (non-negative)
    const R *base = uin + (int64_t)blk * g.bstride;
    const uint32_t lane_b = (uint32_t)((g.ax + (ld ? c : 0)) * (int)sizeof(R));
    // the cell just west of the wave (lane 0), east of it (lane 63); with
    // FUSED the lane whose chunk starts on the east halo column replaces that
    // element with the east neighbour's first column
    int xe = lane == 0 ? c - 1 : lane == 63 ? c + V : c;
    bool lde = xe <= ex && (lane == 0 || lane == 63 || ld);
    const R *ebase = base;
    bool east_sub = false;
    if (FUSED) {
        if (xe == -1 && bx > 0) {
            ebase = uin + (int64_t)(blk - 1) * g.bstride;
            xe = g.e[0] - 1;
        } else if (xe == ex && bx < g.nb[0] - 1 && lde) {
            ebase = uin + (int64_t)(blk + 1) * g.bstride;
            xe = 0;
            east_sub = lane != 63;  // lane 63: xe is its east cell already
        }
    }
    const uint32_t edge_b = (uint32_t)((g.ax + (lde ? xe : 0)) * (int)sizeof(R));
    bool upd[V];
#pragma unroll
    for (int v = 0; v < V; ++v) upd[v] = c + v < ex;
    const bool full = c + V <= ex;
    // rows -1 and ey: the stored halo, or with FUSED the neighbour block's
    // edge row
    const R *above = base, *below = base;
    int64_t above_row = 0, below_row = (int64_t)(ey + 1) * g.pitch;
    if (FUSED && by > 0) {
        above = uin + (int64_t)(blk - g.nb[0]) * g.bstride;
        above_row = (int64_t)g.e[1] * g.pitch;  // its last row, e[1] - 1
    }
    if (FUSED && by < g.nb[1] - 1) {
        below = uin + (int64_t)(blk + g.nb[0]) * g.bstride;
        below_row = g.pitch;  // its row 0
    }
    auto row_of = [&](int ly) {
        if (ly < 0) return above + above_row;
        if (ly >= ey) return below + below_row;
        return base + (int64_t)(ly + 1) * g.pitch;
    };
    auto load = [&](int ly) {
        C r = at<C>(row_of(ly), lane_b);
        if (!ld) {
#pragma unroll
            for (int v = 0; v < V; ++v) r.v[v] = (R)0;
        }
        return r;
    };
    const R *bsrc = SRC ? b + (int64_t)blk * g.sstride : nullptr;
    const R w = (R)0.25;
    double acc = 0.0;
    // the rows of step s: own row (cen), its edge cell (e), its source row
    // (bb) and, for wave 3, the row after the step (nx); loaded one step
    // ahead of their use, so each wave has the next step's loads in flight
    // while it computes
    struct Rows {
        C cen, nx, bb;
        R e;
    };
    auto fetch = [&](int s) {
        Rows r;
        const int y = y0 + 4 * s + wv;
        const bool valid = y < ey;
        r.cen = load(valid ? y : ey);  // rows past the block read the row after it
        if (wv == 3) r.nx = load(y + 1 < ey ? y + 1 : ey);
        r.e = at<R>((FUSED ? ebase : base) + (int64_t)((valid ? y : 0) + 1) * g.pitch, edge_b);
        if constexpr (SRC)
            r.bb = at<C>(bsrc + (int64_t)(valid ? y : 0) * g.e[0],
                         (uint32_t)((ld && c < ex ? c : 0) * (int)sizeof(R)));
        return r;
    };
    auto step = [&](int s, Rows &r) {
        const int buf = s % 3, prev = (s + 2) % 3;
        const int y = y0 + 4 * s + wv;
        const bool valid = y < ey;  // wave-uniform
        C cen = r.cen;
        if (FUSED && east_sub && valid) cen.v[0] = r.e;
        sh[buf][wv + 1][lane] = cen;
        if (wv == 3) sh[buf][5][lane] = r.nx;
        __syncthreads();
        const C up = wv == 0 ? sh[prev][4][lane] : sh[buf][wv][lane];
        const C dn = sh[buf][wv + 2][lane];
        const R eo = lde ? r.e : (R)0;
        const R left = shift_up(eo, cen.v[V - 1]);
        const R right = shift_down(eo, cen.v[0]);
        C out;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R Wv = v > 0 ? cen.v[v - 1] : left;
            const R Ev = v < V - 1 ? cen.v[v + 1] : right;
            const R sum = (Wv + Ev) + (up.v[v] + dn.v[v]);
            out.v[v] = SRC ? (sum + r.bb.v[v]) * w : sum * w;
            if (RES && valid && upd[v]) {
                // residual of the input state, FP64 from widened values
                const double sd = ((double)Wv + (double)Ev) + ((double)up.v[v] + (double)dn.v[v]);
                const double bd = SRC ? (double)r.bb.v[v] : 0.0;
                const double rr = bd - (4.0 * (double)cen.v[v] - sd);
                acc += rr * rr;
            }
        }
        if (valid) {
            R *orow = uout + (int64_t)blk * g.bstride + (int64_t)(y + 1) * g.pitch;
            if (full) {
                if (nt)
                    store_nt16(&at_mut<C>(orow, lane_b), out);
                else
                    at_mut<C>(orow, lane_b) = out;
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (upd[v]) orow[g.ax + c + v] = out.v[v];
            }
        }
    };
    if (wv == 0) sh[2][4][lane] = load(y0 - 1);  // "previous step's last row"
    Rows cur = fetch(0);
    for (int s = 0; s + 1 < nst; ++s) {
        Rows nxt = fetch(s + 1);
        step(s, cur);
        cur = nxt;
    }
    step(nst - 1, cur);
    if (RES) {
        const double a = wave_sum(acc);
        if (lane == 0) res[4 * (int64_t)item + wv] = a;
    }
}

// Rows per work item of the 2D block-local sweep when none is given.  Below
// 4, k_sweep_rows runs that many rows per wave; from 4 on, k_sweep_tile runs
// tiles of that many rows (rounded up to a multiple of 4).  8 (two 4-row
// steps, the second step's loads in flight during the first) measured
// fastest on MI355X for 8192^2 FP32 and FP64, explicit and fused, against
// 4, 12, 16, 24, 32 and 64: a 4-row tile reads 6 rows of state per 4 it
// writes, an 8-row tile 10 per 8; taller tiles spend longer on their
// one-barrier-per-step walk than they save in rows.
template <typename R> constexpr int sweep_rows_default() { return 8; }

// Consecutive tiles of one block's column chunks that go to one XCD
// (tile_item): 8 measured fastest with 8-row tiles (+2-3% over the plain
// round-robin order, the same at 32 tiles, less at 4).
constexpr int kTileRun = 8;

template <typename R, bool FUSED>
static hipError_t launch_tile(const Geom &g, const void *uin, void *uout, const void *b,
                              double *res, int rg, int64_t b0, int64_t b1, hipStream_t st,
                              int64_t *nwork, int nt) {
    constexpr int W = 64 * (16 / (int)sizeof(R));
    const int nchunks = (g.e[0] + W - 1) / W;
    const int steps = (rg + 3) / 4;
    const int ntiles = (g.e[1] + 4 * steps - 1) / (4 * steps);
    const int64_t items = (b1 - b0) * ntiles * nchunks;
    if (nwork) *nwork = 4 * items;
    if (items > 0x7fffffff / 4) return hipErrorInvalidValue;
    const int grp = kTileRun * nchunks;
    const R *bb = (const R *)b;
#define JAC_TILE(SRCV, RESV)                                                                    \
    hipLaunchKernelGGL((k_sweep_tile<R, SRCV, FUSED, RESV>), dim3((unsigned)items), dim3(256),  \
                       0, st, g, (const R *)uin, (R *)uout, bb, res, steps, ntiles, nchunks,    \
                       (int)b0, (int)items, grp, nt)
    if (b && res)
        JAC_TILE(true, true);
    else if (b)
        JAC_TILE(true, false);
    else if (res)
        JAC_TILE(false, true);
    else
        JAC_TILE(false, false);
#undef JAC_TILE
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_sweep_rows(const Geom &g, const void *uin, void *uout, const void *b,
                                    int rg, int64_t b0, int64_t b1, hipStream_t st, int nt) {
    constexpr int W = 64 * (16 / (int)sizeof(R));
    if (rg <= 0) rg = sweep_rows_default<R>();
    const int nchunks = (g.e[0] + W - 1) / W;
    if (rg >= 4)
        return launch_tile<R, false>(g, uin, uout, b, nullptr, rg, b0, b1, st, nullptr, nt);
    const int ngroups = (g.e[1] + rg - 1) / rg;
    const int64_t nwork = (b1 - b0) * ngroups * nchunks;
    if (nwork > 0x7fffffff - 3) return hipErrorInvalidValue;
    const int grid = (int)((nwork + 3) / 4);
    if (b)
        hipLaunchKernelGGL((k_sweep_rows<R, true>), dim3(grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)b, rg, ngroups, nchunks,
                           (int)b0, (int)nwork);
    else
        hipLaunchKernelGGL((k_sweep_rows<R, false>), dim3(grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)nullptr, rg, ngroups, nchunks,
                           (int)b0, (int)nwork);
    return hipGetLastError();
}

template <typename R>
int64_t sweep_tile_partials(const Geom &g, int rg) {
    constexpr int W = 64 * (16 / (int)sizeof(R));
    if (rg <= 0) rg = sweep_rows_default<R>();
    if (rg < 4) rg = 4;
    const int64_t nchunks = (g.e[0] + W - 1) / W;
    const int64_t steps = (rg + 3) / 4;
    const int64_t ntiles = (g.e[1] + 4 * steps - 1) / (4 * steps);
    return 4 * g.nblocks * ntiles * nchunks;
}

template <typename R>
hipError_t launch_sweep2d_tile_fused(const Geom &g, const void *uin, void *uout, const void *b,
                                     double *res, int rg, hipStream_t st, int64_t *nwork, int nt) {
    if (g.ndim != 2) return hipErrorInvalidValue;
    if (rg <= 0) rg = sweep_rows_default<R>();
    if (rg < 4) rg = 4;
    return launch_tile<R, true>(g, uin, uout, b, res, rg, 0, g.nblocks, st, nwork, nt);
}

template <typename R>
hipError_t launch_sweep_local(const Geom &g, const void *uin, void *uout, const void *b,
                              hipStream_t st, int rg, int64_t b0, int64_t b1, int nt) {
    if (b1 < 0) b1 = g.nblocks;
    if (b0 < 0 || b1 > g.nblocks || b0 >= b1) return b0 == b1 ? hipSuccess : hipErrorInvalidValue;
    if (g.ndim == 2) return launch_sweep_rows<R>(g, uin, uout, b, rg, b0, b1, st, nt);
    constexpr int V = 16 / sizeof(R);
    const int64_t cpr = (g.e[0] + V - 1) / V;
    const int64_t total = (b1 - b0) * (int64_t)g.e[1] * (g.ndim == 3 ? g.e[2] : 1) * cpr;
    const int64_t grid = (total + 255) / 256;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    if (b)
        hipLaunchKernelGGL((k_sweep_local<R, true>), dim3((unsigned)grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)b, b0, total);
    else
        hipLaunchKernelGGL((k_sweep_local<R, false>), dim3((unsigned)grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)nullptr, b0, total);
    return hipGetLastError();
}

template hipError_t launch_sweep_local<float>(const Geom &, const void *, void *, const void *,
                                              hipStream_t, int, int64_t, int64_t, int);
template int64_t sweep_tile_partials<float>(const Geom &, int);
template int64_t sweep_tile_partials<double>(const Geom &, int);
template hipError_t launch_sweep2d_tile_fused<float>(const Geom &, const void *, void *,
                                                     const void *, double *, int, hipStream_t,
                                                     int64_t *, int);
template hipError_t launch_sweep2d_tile_fused<double>(const Geom &, const void *, void *,
                                                      const void *, double *, int, hipStream_t,
                                                      int64_t *, int);
template hipError_t launch_sweep_local<double>(const Geom &, const void *, void *, const void *,
                                               hipStream_t, int, int64_t, int64_t, int);

}  // namespace jac
