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
                                                     const R *__restrict__ b, int64_t total) {
    constexpr int V = 16 / sizeof(R);
    const int cpr = (g.e[0] + V - 1) / V;           // chunks per row
    const int64_t rows = (int64_t)g.e[1] * (g.ndim == 3 ? g.e[2] : 1);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int cx = (int)(i % cpr);
    const int64_t rest = i / cpr;
    const int64_t rr = rest % rows;
    const int64_t blk = rest / rows;
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

template <typename R>
hipError_t launch_sweep_local(const Geom &g, const void *uin, void *uout, const void *b,
                              hipStream_t st) {
    constexpr int V = 16 / sizeof(R);
    const int64_t cpr = (g.e[0] + V - 1) / V;
    const int64_t total = g.nblocks * (int64_t)g.e[1] * (g.ndim == 3 ? g.e[2] : 1) * cpr;
    const int64_t grid = (total + 255) / 256;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    if (b)
        hipLaunchKernelGGL((k_sweep_local<R, true>), dim3((unsigned)grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)b, total);
    else
        hipLaunchKernelGGL((k_sweep_local<R, false>), dim3((unsigned)grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)nullptr, total);
    return hipGetLastError();
}

template hipError_t launch_sweep_local<float>(const Geom &, const void *, void *, const void *,
                                              hipStream_t);
template hipError_t launch_sweep_local<double>(const Geom &, const void *, void *, const void *,
                                               hipStream_t);

}  // namespace jac
