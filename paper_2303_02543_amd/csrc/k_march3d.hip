// Fused 3D Jacobi pass kernel for gfx950 (one sweep per pass).
//
// The update is the 7-point Jacobi step of the proxy application in
// Section 4.3 of the paper, evaluated as
//   s = ((W + E) + (S + N)) + (B + F);  u' = (s + b) * fl(1/6)
// with no FMA contraction.
//
// A workgroup of 4 waves owns 16 rows by 16 lanes x V elements along x (one
// 16-lane row of a wave per grid row; 64 columns in FP32, 32 in FP64) and
// marches along z through a segment of planes, each lane keeping the planes
// z-1, z, z+1 of its cells in registers.  For the 64^3 blocks of the
// workloads a wave's 4 rows lie in one block, so every load instruction reads
// neighbouring rows of one block (about 1.5 KiB of consecutive addresses).
// The rows y-1 and y+1 of plane z come from the workgroup's LDS copy of that
// plane (only its two halo rows are read from memory), x neighbours from DPP
// shifts within each 16-lane row plus one scalar load per row end.  Every load goes to the block that owns the cell,
// so the face-halo exchange between blocks happens inside the loads.  The
// FP64 residual of the input state can be accumulated in the same pass.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

// Element offset of the z part (block layer and plane) of a global plane z.
__device__ __forceinline__ int64_t plane_part(const Geom &g, int zblk, int zloc) {
    return (int64_t)zblk * g.nb[1] * g.nb[0] * g.bstride + (int64_t)(zloc + 1) * g.plane;
}
__device__ __forceinline__ int64_t src_plane_part(const Geom &g, int zblk, int zloc) {
    return (int64_t)zblk * g.nb[1] * g.nb[0] * g.sstride + (int64_t)zloc * g.e[1] * g.e[0];
}
// Element offset of the x/y part of node (x, y) inside its z layer: its
// block column / row and its place in the block's plane (state buffers).
__device__ __forceinline__ int64_t xy_part(const Geom &g, int x, int y) {
    int bx, lx, by, ly;
    owner(x, g.e[0], g.nb[0], bx, lx);
    owner(y, g.e[1], g.nb[1], by, ly);
    return ((int64_t)by * g.nb[0] + bx) * g.bstride + (int64_t)(ly + 1) * g.pitch + g.ax + lx;
}
__device__ __forceinline__ int64_t src_xy_part(const Geom &g, int x, int y) {
    int bx, lx, by, ly;
    owner(x, g.e[0], g.nb[0], bx, lx);
    owner(y, g.e[1], g.nb[1], by, ly);
    return ((int64_t)by * g.nb[0] + bx) * g.sstride + (int64_t)ly * g.e[0] + lx;
}

// Block layer and local index of a plane, advanced one plane at a time.
struct ZPos {
    int blk, loc;
};

__device__ __forceinline__ void z_next(ZPos &p, int e, int nb) {
    ++p.loc;
    if (p.loc >= e && p.blk < nb - 1) {
        ++p.blk;
        p.loc = 0;
    }
}

// Per-lane constants of a work item.
struct M3Lane {
    int64_t c_off, h_off, e_off, b_off;  // own row, halo row (loaders), edge cell, source
    int k;                               // LDS row slot of the lane's own row (1 .. 16)
    int hk;                              // LDS slot the lane's halo load fills (0, 17; -1: none)
    bool ld, lde, ldb;                   // lane loads interior/east-ring, edge, source
    bool upd[8];                         // element is an interior cell of a valid row
};

constexpr int kM3Rows = 16;  // rows per work item (4 waves x 4 rows)

// Rows y-1 and y+1 of plane z come from the workgroup's LDS copy of the
// plane's rows y0-1 .. y0+16 (double-buffered by plane parity, so one barrier
// per step suffices); only the two halo rows are read from memory, one step
// ahead of use, by the first row of wave 0 and the last row of wave 3.
template <typename R, int MODE, bool EDGE>
__device__ __forceinline__ void m3_body(const Geom &g, const R *__restrict__ uin,
                                        R *__restrict__ uout, const R *__restrict__ bsrc,
                                        double *__restrict__ res_slot, const M3Lane &L, int oz0,
                                        int oz1, bool nt,
                                        Chunk<R, 16 / sizeof(R)> (*sh)[kM3Rows + 2][16]) {
    constexpr int V = 16 / (int)sizeof(R);
    constexpr bool SRC = MODE == 1;
    using C = Chunk<R, V>;
    const int cx = threadIdx.x & 15;
    auto load = [&](int64_t off) -> C {
        C r = *reinterpret_cast<const C *>(uin + off);
        if (EDGE && !L.ld) {
#pragma unroll
            for (int v = 0; v < V; ++v) r.v[v] = (R)0;
        }
        return r;
    };
    ZPos pz;
    owner(oz0 - 1, g.e[2], g.nb[2], pz.blk, pz.loc);
    C zm = load(plane_part(g, pz.blk, pz.loc) + L.c_off);
    z_next(pz, g.e[2], g.nb[2]);
    C zc = load(plane_part(g, pz.blk, pz.loc) + L.c_off);
    C halo;  // halo row of the current plane (loader lanes)
    if (L.hk >= 0) halo = load(plane_part(g, pz.blk, pz.loc) + L.h_off);
    ZPos pzn = pz;
    z_next(pzn, g.e[2], g.nb[2]);
    const R w = (R)1 / (R)6;
    double acc = 0.0;
    for (int z = oz0; z < oz1; ++z) {
        const int buf = z & 1;
        const int64_t pc = plane_part(g, pz.blk, pz.loc), pp = plane_part(g, pzn.blk, pzn.loc);
        sh[buf][L.k][cx] = zc;
        if (L.hk >= 0) sh[buf][L.hk][cx] = halo;
        const C zp = load(pp + L.c_off);
        if (L.hk >= 0) halo = load(pp + L.h_off);  // next plane's halo row
        R eo = uin[pc + L.e_off];
        if (EDGE && !L.lde) eo = (R)0;
        C bb;
        if constexpr (SRC) {
            bb = *reinterpret_cast<const C *>(bsrc + src_plane_part(g, pz.blk, pz.loc) + L.b_off);
            if (EDGE && !L.ldb) {
#pragma unroll
                for (int v = 0; v < V; ++v) bb.v[v] = (R)0;
            }
        }
        __syncthreads();
        const C so = sh[buf][L.k - 1][cx];
        const C no = sh[buf][L.k + 1][cx];
        const R left = row_shift_up(eo, zc.v[V - 1]);
        const R right = row_shift_down(eo, zc.v[0]);
        C out;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R Wv = v > 0 ? zc.v[v - 1] : left;
            const R Ev = v < V - 1 ? zc.v[v + 1] : right;
            const R s = ((Wv + Ev) + (so.v[v] + no.v[v])) + (zm.v[v] + zp.v[v]);
            out.v[v] = SRC ? (s + bb.v[v]) * w : s * w;
            if (res_slot) {
                const double sd = (((double)Wv + (double)Ev) + ((double)so.v[v] + (double)no.v[v])) +
                                  ((double)zm.v[v] + (double)zp.v[v]);
                const double bd = SRC ? (double)bb.v[v] : 0.0;
                const double r = bd - (6.0 * (double)zc.v[v] - sd);
                acc += (!EDGE || L.upd[v]) ? r * r : 0.0;
            }
        }
        if (uout) {
            R *p = uout + pc + L.c_off;
            if (!EDGE) {
                if (nt)
                    store_nt16(reinterpret_cast<C *>(p), out);
                else
                    *reinterpret_cast<C *>(p) = out;
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (L.upd[v]) p[v] = out.v[v];
            }
        }
        zm = zc;
        zc = zp;
        pz = pzn;
        z_next(pzn, g.e[2], g.nb[2]);
    }
    if (res_slot) {
        const double a = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) *res_slot = a;
    }
}

// Work item (one workgroup of 4 waves): 16 rows (fastest), column strip, z
// segment of `zseg` planes; wave q takes rows y0+4q .. y0+4q+3.  The residual
// partials are per wave: work item i owns partials 4i .. 4i+3.
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_march3d(Geom g, const R *__restrict__ uin,
                                                 R *__restrict__ uout,
                                                 const R *__restrict__ bsrc,
                                                 double *__restrict__ res, int nstrips, int ngrp,
                                                 int zseg, int nitems, int nt) {
    constexpr int V = 16 / (int)sizeof(R);
    constexpr int W = 16 * V;  // columns per tile
    __shared__ Chunk<R, V> sh[2][kM3Rows + 2][16];
    const int item = xcd_logical_block(blockIdx.x, gridDim.x);
    if (item >= nitems) return;  // whole workgroup
    const int grp = item % ngrp;
    const int rest = item / ngrp;
    const int strip = rest % nstrips;
    const int zs = rest / nstrips;
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int ry = lane >> 4, cx = lane & 15;
    const int nx = g.n[0], ny = g.n[1];
    const int a = strip * W;
    const int c = a + cx * V;
    const int y0 = grp * kM3Rows;
    const int yy = y0 + 4 * wv + ry;
    const bool row_ok = yy < ny;
    // rows past the grid read the ring row ny (the north neighbour of row
    // ny-1) or, further out, that row again (values not used)
    const int yc = yy < ny ? yy : ny;
    M3Lane L;
    L.k = 1 + 4 * wv + ry;
    // chunk holds interior cells or the east ring cell
    L.ld = c <= nx;
    const int cl = L.ld ? c : 0;
    L.c_off = xy_part(g, cl, yc);
    L.hk = -1;
    if (wv == 0 && ry == 0) {
        L.hk = 0;
        L.h_off = xy_part(g, cl, y0 - 1);
    } else if (wv == 3 && ry == 3) {
        L.hk = kM3Rows + 1;
        L.h_off = xy_part(g, cl, y0 + kM3Rows < ny ? y0 + kM3Rows : ny);
    } else {
        L.h_off = L.c_off;
    }
    // the first / last lane of each 16-lane row fetch the cells just west /
    // east of the tile; the others re-read their own first cell
    const int xe = cx == 0 ? a - 1 : cx == 15 ? a + W : c;
    L.lde = xe >= -1 && xe <= nx && (cx == 0 || cx == 15 || L.ld);
    L.e_off = xy_part(g, L.lde ? xe : 0, yc);
    L.ldb = c < nx && row_ok;
    L.b_off = src_xy_part(g, L.ldb ? c : 0, L.ldb ? yc : 0);
#pragma unroll
    for (int v = 0; v < 8; ++v) L.upd[v] = v < V && row_ok && c + v < nx;
    const int oz0 = zs * zseg;
    const int oz1 = oz0 + zseg < g.n[2] ? oz0 + zseg : g.n[2];
    double *slot = res ? res + (int64_t)item * 4 + wv : nullptr;
    const bool edge = a + W > nx || y0 + kM3Rows > ny;
    if (edge)
        m3_body<R, MODE, true>(g, uin, uout, bsrc, slot, L, oz0, oz1, nt != 0, sh);
    else
        m3_body<R, MODE, false>(g, uin, uout, bsrc, slot, L, oz0, oz1, nt != 0, sh);
}

// Residual partials of one pass (one per wave, 4 per work item).
template <typename R>
int64_t march3d_work_items(const Geom &g, int zseg) {
    constexpr int W = 16 * (16 / (int)sizeof(R));
    const int64_t nstrips = (g.n[0] + W - 1) / W;
    const int64_t ngrp = (g.n[1] + kM3Rows - 1) / kM3Rows;
    const int64_t nzs = (g.n[2] + zseg - 1) / zseg;
    return 4 * nstrips * ngrp * nzs;
}

template <typename R>
hipError_t launch_march3d(const Geom &g, const void *uin, void *uout, const void *b, double *res,
                          int zseg, hipStream_t st, int64_t *nwork_out, int nt) {
    constexpr int W = 16 * (16 / (int)sizeof(R));
    const int nstrips = (g.n[0] + W - 1) / W;
    const int ngrp = (g.n[1] + kM3Rows - 1) / kM3Rows;
    const int64_t nwaves = march3d_work_items<R>(g, zseg);
    if (nwork_out) *nwork_out = nwaves;
    if (nwaves > 0x7fffffff - 3) return hipErrorInvalidValue;
    const int items = (int)(nwaves / 4);
    if (b)
        hipLaunchKernelGGL((k_march3d<R, 1>), dim3(items), dim3(256), 0, st, g, (const R *)uin,
                           (R *)uout, (const R *)b, res, nstrips, ngrp, zseg, items, nt);
    else
        hipLaunchKernelGGL((k_march3d<R, 0>), dim3(items), dim3(256), 0, st, g, (const R *)uin,
                           (R *)uout, (const R *)nullptr, res, nstrips, ngrp, zseg, items, nt);
    return hipGetLastError();
}

template int64_t march3d_work_items<float>(const Geom &, int);
template int64_t march3d_work_items<double>(const Geom &, int);
template hipError_t launch_march3d<float>(const Geom &, const void *, void *, const void *,
                                          double *, int, hipStream_t, int64_t *, int);
template hipError_t launch_march3d<double>(const Geom &, const void *, void *, const void *,
                                           double *, int, hipStream_t, int64_t *, int);

}  // namespace jac
