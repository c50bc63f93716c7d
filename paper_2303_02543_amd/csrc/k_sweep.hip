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
// This file holds the block-local sweep: one sweep of every block from its
// own storage (its interior plus the one-cell halo a preceding halo exchange
// filled), the step order of the paper's proxy -- exchange, then update.  The
// fused multi-sweep pass kernel lives in k_march2d.hip.
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
template <typename R, bool SRC>
__global__ __launch_bounds__(256) void k_sweep_tile(Geom g, const R *__restrict__ uin,
                                                    R *__restrict__ uout,
                                                    const R *__restrict__ b, int steps,
                                                    int ntiles, int nchunks, int blk0,
                                                    int nitems) {
    constexpr int V = 16 / sizeof(R);
    constexpr int W = 64 * V;
    using C = Chunk<R, V>;
    __shared__ C sh[3][6][64];  // slots 1..4: the step's rows, 5: the row after
    const int item = blockIdx.x;  // memory order, as in k_sweep_rows
    if (item >= nitems) return;   // whole workgroup
    const int chunk = item % nchunks;
    const int rest = item / nchunks;
    const int tile = rest % ntiles;
    const int blk = blk0 + rest / ntiles;
    const int bx = blk % g.nb[0], by = blk / g.nb[0];
    const int ex = extent(g.n[0], g.e[0], bx);
    const int ey = extent(g.n[1], g.e[1], by);
    const int y0 = tile * 4 * steps;
    if (y0 >= ey) return;  // tile beyond a short block (whole workgroup)
    const int nst = ((ey - y0 < 4 * steps ? ey - y0 : 4 * steps) + 3) / 4;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = chunk * W + lane * V;
    const bool ld = c <= ex;
    const int xe = lane == 0 ? c - 1 : lane == 63 ? c + V : c;
    const bool lde = xe <= ex && (lane == 0 || lane == 63 || ld);
    // byte offsets from the start of a stored row (non-negative)
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
    const R w = (R)0.25;
    if (wv == 0) sh[2][4][lane] = load(y0 - 1);  // "previous step's last row"
    for (int s = 0; s < nst; ++s) {
        const int buf = s % 3, prev = (s + 2) % 3;
        const int y = y0 + 4 * s + wv;
        const bool valid = y < ey;      // wave-uniform
        const int yl = valid ? y : ey;  // rows past the block read the ring row
        const C cen = load(yl);
        sh[buf][wv + 1][lane] = cen;
        if (wv == 3) sh[buf][5][lane] = load(y + 1 < ey ? y + 1 : ey);
        const R e = at<R>(row_of(yl), edge_b);
        C bb;
        if constexpr (SRC) {
            bb = at<C>(bsrc + (int64_t)(valid ? y : 0) * g.e[0],
                       (uint32_t)((ld && c < ex ? c : 0) * (int)sizeof(R)));
        }
        __syncthreads();
        const C up = wv == 0 ? sh[prev][4][lane] : sh[buf][wv][lane];
        const C dn = sh[buf][wv + 2][lane];
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
        if (valid) {
            R *orow = uout + (int64_t)blk * g.bstride + (int64_t)(y + 1) * g.pitch;
            if (full) {
                at_mut<C>(orow, lane_b) = out;
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (upd[v]) orow[g.ax + c + v] = out.v[v];
            }
        }
    }
}

// Rows per work item of the 2D block-local sweep when none is given (fastest
// measured on MI355X for 8192^2 FP32 / FP64).  Below 4, k_sweep_rows runs
// that many rows per wave; from 4 on, k_sweep_tile runs tiles of that many
// rows (rounded up to a multiple of 4).
// (4: one 4-row step per workgroup; taller tiles read fewer boundary rows but
// stream worse).
template <typename R> constexpr int sweep_rows_default() { return 4; }

template <typename R>
static hipError_t launch_sweep_rows(const Geom &g, const void *uin, void *uout, const void *b,
                                    int rg, int64_t b0, int64_t b1, hipStream_t st) {
    constexpr int W = 64 * (16 / (int)sizeof(R));
    if (rg <= 0) rg = sweep_rows_default<R>();
    const int nchunks = (g.e[0] + W - 1) / W;
    if (rg >= 4) {
        const int steps = (rg + 3) / 4;
        const int ntiles = (g.e[1] + 4 * steps - 1) / (4 * steps);
        const int64_t items = (b1 - b0) * ntiles * nchunks;
        if (items > 0x7fffffff) return hipErrorInvalidValue;
        if (b)
            hipLaunchKernelGGL((k_sweep_tile<R, true>), dim3((unsigned)items), dim3(256), 0, st, g,
                               (const R *)uin, (R *)uout, (const R *)b, steps, ntiles, nchunks,
                               (int)b0, (int)items);
        else
            hipLaunchKernelGGL((k_sweep_tile<R, false>), dim3((unsigned)items), dim3(256), 0, st,
                               g, (const R *)uin, (R *)uout, (const R *)nullptr, steps, ntiles,
                               nchunks, (int)b0, (int)items);
        return hipGetLastError();
    }
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
hipError_t launch_sweep_local(const Geom &g, const void *uin, void *uout, const void *b,
                              hipStream_t st, int rg, int64_t b0, int64_t b1) {
    if (b1 < 0) b1 = g.nblocks;
    if (b0 < 0 || b1 > g.nblocks || b0 >= b1) return b0 == b1 ? hipSuccess : hipErrorInvalidValue;
    if (g.ndim == 2) return launch_sweep_rows<R>(g, uin, uout, b, rg, b0, b1, st);
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
                                              hipStream_t, int, int64_t, int64_t);
template hipError_t launch_sweep_local<double>(const Geom &, const void *, void *, const void *,
                                               hipStream_t, int, int64_t, int64_t);

}  // namespace jac
