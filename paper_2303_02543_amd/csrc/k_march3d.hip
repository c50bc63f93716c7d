// Fused 3D Jacobi pass kernel for gfx950 (one sweep per pass).
//
// The update is the 7-point Jacobi step of the proxy application in
// Section 4.3 of the paper, evaluated as
//   s = ((W + E) + (S + N)) + (B + F);  u' = (s + b) * fl(1/6)
// with no FMA contraction.
//
// A wave owns one row y of a strip of 64 lanes x V elements along x and
// marches along z through a segment of planes, keeping the planes z-1, z,
// z+1 of its row in registers.  The rows y-1 and y+1 of plane z are loaded
// each step (they are the centre rows of the neighbouring waves, so they come
// mostly from L2); x neighbours come from DPP lane shifts plus two scalar
// loads per plane.  Every load goes to the block that owns the cell, so the
// face-halo exchange between blocks happens inside the loads.  The FP64
// residual of the input state can be accumulated in the same pass.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

// Offset bookkeeping along one axis: block index, local coordinate, and the
// element offset contributed by that axis.
struct AxisPos {
    int blk, loc;
};

__device__ __forceinline__ AxisPos axis_pos(int v, int e, int nb) {
    AxisPos p;
    owner(v, e, nb, p.blk, p.loc);
    return p;
}

// Element offset of (lane part) + row (y) + plane (z) for a 3D block layout.
__device__ __forceinline__ int64_t row_part(const Geom &g, AxisPos y) {
    return (int64_t)y.blk * g.nb[0] * g.bstride + (int64_t)(y.loc + 1) * g.pitch;
}
__device__ __forceinline__ int64_t plane_part(const Geom &g, AxisPos z) {
    return (int64_t)z.blk * g.nb[1] * g.nb[0] * g.bstride + (int64_t)(z.loc + 1) * g.plane;
}
__device__ __forceinline__ int64_t src_row_part(const Geom &g, AxisPos y) {
    return (int64_t)y.blk * g.nb[0] * g.sstride + (int64_t)y.loc * g.e[0];
}
__device__ __forceinline__ int64_t src_plane_part(const Geom &g, AxisPos z) {
    return (int64_t)z.blk * g.nb[1] * g.nb[0] * g.sstride + (int64_t)z.loc * g.e[1] * g.e[0];
}

__device__ __forceinline__ void axis_next(AxisPos &p, int e, int nb) {
    ++p.loc;
    if (p.loc >= e && p.blk < nb - 1) {
        ++p.blk;
        p.loc = 0;
    }
}

template <typename R, int MODE, bool RINGX>
__device__ __forceinline__ void m3_body(const Geom &g, const R *__restrict__ uin,
                                        R *__restrict__ uout, const R *__restrict__ bsrc,
                                        double *__restrict__ res_slot, int c, int64_t lane_off,
                                        int64_t edge_off, int64_t lane_soff, bool ld, bool lde,
                                        int y, int oz0, int oz1, bool nt) {
    constexpr int V = 16 / (int)sizeof(R);
    constexpr bool SRC = MODE == 1;
    using C = Chunk<R, V>;
    const int nx = g.n[0];
    bool upd[V];
#pragma unroll
    for (int v = 0; v < V; ++v) upd[v] = c + v >= 0 && c + v < nx;
    const AxisPos py = axis_pos(y, g.e[1], g.nb[1]);
    const AxisPos ps = axis_pos(y - 1, g.e[1], g.nb[1]);
    const AxisPos pn = axis_pos(y + 1, g.e[1], g.nb[1]);
    const int64_t ry = row_part(g, py), rs = row_part(g, ps), rn = row_part(g, pn);
    const int64_t sry = src_row_part(g, py);
    auto load = [&](int64_t off) -> C {
        C r;
        if (!RINGX || ld) {
            r = *reinterpret_cast<const C *>(uin + off + lane_off);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) r.v[v] = (R)0;
        }
        return r;
    };
    AxisPos pz = axis_pos(oz0 - 1, g.e[2], g.nb[2]);
    C zm = load(plane_part(g, pz) + ry);
    axis_next(pz, g.e[2], g.nb[2]);
    C zc = load(plane_part(g, pz) + ry);
    AxisPos pzn = pz;
    axis_next(pzn, g.e[2], g.nb[2]);
    const R w = (R)1 / (R)6;
    double acc = 0.0;
    for (int z = oz0; z < oz1; ++z) {
        const int64_t pc = plane_part(g, pz), pp = plane_part(g, pzn);
        const C zp = load(pp + ry);
        const C so = load(pc + rs);
        const C no = load(pc + rn);
        const R eo = (!RINGX || lde) ? uin[pc + ry + edge_off] : (R)0;
        C bb;
        if constexpr (SRC) {
            if (!RINGX || (c >= 0 && c < nx)) {
                bb = *reinterpret_cast<const C *>(bsrc + src_plane_part(g, pz) + sry + lane_soff);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) bb.v[v] = (R)0;
            }
        }
        const R left = shift_up(eo, zc.v[V - 1]);
        const R right = shift_down(eo, zc.v[0]);
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
                acc += (!RINGX || upd[v]) ? r * r : 0.0;
            }
        }
        if (uout) {
            R *p = uout + pc + ry + lane_off;
            if (!RINGX) {
                if (nt)
                    store_nt16(reinterpret_cast<C *>(p), out);
                else
                    *reinterpret_cast<C *>(p) = out;
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (upd[v]) p[v] = out.v[v];
            }
        }
        zm = zc;
        zc = zp;
        pz = pzn;
        axis_next(pzn, g.e[2], g.nb[2]);
    }
    if (res_slot) {
        const double a = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) *res_slot = a;
    }
}

// Work item wid: strip (x), row y, z segment of `zseg` planes.
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_march3d(Geom g, const R *__restrict__ uin,
                                                 R *__restrict__ uout,
                                                 const R *__restrict__ bsrc,
                                                 double *__restrict__ res, int nstrips, int nzs,
                                                 int zseg, int nwork, int nt) {
    constexpr int V = 16 / (int)sizeof(R);
    constexpr int W = 64 * V;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int wid = __builtin_amdgcn_readfirstlane(lb * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wid >= nwork) return;
    // order: z segment slowest, then strip, then row (adjacent rows in one
    // workgroup share their neighbour rows through L1/L2)
    const int y = wid % g.n[1];
    const int rest = wid / g.n[1];
    const int strip = rest % nstrips;
    const int zs = rest / nstrips;
    const int lane = threadIdx.x & 63;
    const int nx = g.n[0];
    const int a = strip * W;
    const int c = a + lane * V;
    const bool ld = c <= nx;  // chunk holds interior cells or the east ring cell
    int bx, lx;
    owner(ld ? c : 0, g.e[0], g.nb[0], bx, lx);
    const int64_t lane_off = (int64_t)bx * g.bstride + g.ax + lx;
    const int64_t lane_soff = (int64_t)bx * g.sstride + lx;
    const int xe = lane == 0 ? a - 1 : lane == 63 ? a + W : c;
    const bool lde = (xe >= -1 && xe <= nx) && (lane == 0 || lane == 63 || ld);
    int bxe, lxe;
    owner(lde ? xe : 0, g.e[0], g.nb[0], bxe, lxe);
    const int64_t edge_off = (int64_t)bxe * g.bstride + g.ax + lxe;
    const int oz0 = zs * zseg;
    const int oz1 = oz0 + zseg < g.n[2] ? oz0 + zseg : g.n[2];
    double *slot = res ? res + wid : nullptr;
    const bool ringx = a + W > nx;
    if (ringx)
        m3_body<R, MODE, true>(g, uin, uout, bsrc, slot, c, lane_off, edge_off, lane_soff, ld, lde,
                               y, oz0, oz1, nt != 0);
    else
        m3_body<R, MODE, false>(g, uin, uout, bsrc, slot, c, lane_off, edge_off, lane_soff, ld,
                                lde, y, oz0, oz1, nt != 0);
}

template <typename R>
int64_t march3d_work_items(const Geom &g, int zseg) {
    constexpr int W = 64 * (16 / (int)sizeof(R));
    const int64_t nstrips = (g.n[0] + W - 1) / W;
    const int64_t nzs = (g.n[2] + zseg - 1) / zseg;
    return nstrips * g.n[1] * nzs;
}

template <typename R>
hipError_t launch_march3d(const Geom &g, const void *uin, void *uout, const void *b, double *res,
                          int zseg, hipStream_t st, int64_t *nwork_out, int nt) {
    constexpr int W = 64 * (16 / (int)sizeof(R));
    const int nstrips = (g.n[0] + W - 1) / W;
    const int nzs = (g.n[2] + zseg - 1) / zseg;
    const int64_t nwork = (int64_t)nstrips * g.n[1] * nzs;
    if (nwork_out) *nwork_out = nwork;
    if (nwork > 0x7fffffff) return hipErrorInvalidValue;
    const int grid = (int)((nwork + 3) / 4);
    if (b)
        hipLaunchKernelGGL((k_march3d<R, 1>), dim3(grid), dim3(256), 0, st, g, (const R *)uin,
                           (R *)uout, (const R *)b, res, nstrips, nzs, zseg, (int)nwork, nt);
    else
        hipLaunchKernelGGL((k_march3d<R, 0>), dim3(grid), dim3(256), 0, st, g, (const R *)uin,
                           (R *)uout, (const R *)nullptr, res, nstrips, nzs, zseg, (int)nwork, nt);
    return hipGetLastError();
}

template int64_t march3d_work_items<float>(const Geom &, int);
template int64_t march3d_work_items<double>(const Geom &, int);
template hipError_t launch_march3d<float>(const Geom &, const void *, void *, const void *,
                                          double *, int, hipStream_t, int64_t *, int);
template hipError_t launch_march3d<double>(const Geom &, const void *, void *, const void *,
                                           double *, int, hipStream_t, int64_t *, int);

}  // namespace jac
