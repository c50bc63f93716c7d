// Layout kernels: scatter a full state into blocks, gather it back, scale the
// source into blocks, and the face-halo exchange between blocks.
//
// The paper's proxy cuts the domain into cuboids and, every iteration, packs
// each block's edge cells, moves them to the face neighbours and unpacks them
// into their halos (Section 4.3; the over-decomposition timeline figure of
// Section 4.4 names the six per-face halo buffers).  On one GPU every block
// lives in the same HBM, so pack, copy and unpack collapse into one gather
// per halo cell: read the neighbour's edge cell, write the halo slot.
#include <hip/hip_runtime.h>

#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

// The element maps below run over rows of the full array (or of the source
// for k_scale_source): one workgroup per row (rows strided over the grid),
// its threads walking the row block by block, so no element needs a
// division to find its owner and every access is coalesced.  (A flat
// grid-stride form, which split a 64-bit element index per element, ran at
// ~2 TB/s; one element per thread with one workgroup per 256 columns was
// slower still, bound by workgroup dispatch.)

// Element offset of row y / plane z (ring-extended) in block (0, by, bz) at
// local x = 0, and whether the row is on the Dirichlet ring (uniform).
struct RowYZ {
    int64_t base;
    bool ring;
};
__device__ __forceinline__ RowYZ row_yz(const Geom &g, int y, int z) {
    int by, ly, bz = 0, lz = 0;
    owner(y, g.e[1], g.nb[1], by, ly);
    if (g.ndim == 3) owner(z, g.e[2], g.nb[2], bz, lz);
    RowYZ r;
    r.base = local_offset(g, ((int64_t)bz * g.nb[1] + by) * g.nb[0], 0, ly, lz);
    r.ring = y < 0 || y >= g.n[1] || (g.ndim == 3 && (z < 0 || z >= g.n[2]));
    return r;
}

// Every node of the full (n+2)^d array goes to the block that owns it (ring
// nodes to the domain-edge halo slots), in both state buffers.  Internal
// halos are filled afterwards by the halo exchange.
template <typename R>
__global__ __launch_bounds__(256) void k_scatter(Geom g, const R *__restrict__ u,
                                                 R *__restrict__ s0, R *__restrict__ s1,
                                                 int64_t rows, int zero_ring) {
    const int nx2 = g.n[0] + 2, ny2 = g.n[1] + 2;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const RowYZ yz = row_yz(g, (int)(r % ny2) - 1, (int)(r / ny2) - 1);
        const R *urow = u + r * nx2 + 1;  // urow[x], x in [-1, n]
        for (int bx = 0; bx < g.nb[0]; ++bx) {
            const int ext = extent(g.n[0], g.e[0], bx);
            const int lo = bx == 0 ? -1 : 0, hi = bx == g.nb[0] - 1 ? ext + 1 : ext;
            const int x0 = bx * g.e[0];
            const int64_t boff = yz.base + (int64_t)bx * g.bstride;
            for (int lx = lo + (int)threadIdx.x; lx < hi; lx += blockDim.x) {
                const int x = x0 + lx;
                const bool ring = yz.ring || x < 0 || x >= g.n[0];
                const R v = (zero_ring && ring) ? (R)0 : urow[x];
                s0[boff + lx] = v;
                s1[boff + lx] = v;
            }
        }
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_gather(Geom g, const R *__restrict__ s,
                                                R *__restrict__ u, int64_t rows) {
    const int nx2 = g.n[0] + 2, ny2 = g.n[1] + 2;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const RowYZ yz = row_yz(g, (int)(r % ny2) - 1, (int)(r / ny2) - 1);
        R *urow = u + r * nx2 + 1;
        for (int bx = 0; bx < g.nb[0]; ++bx) {
            const int ext = extent(g.n[0], g.e[0], bx);
            const int lo = bx == 0 ? -1 : 0, hi = bx == g.nb[0] - 1 ? ext + 1 : ext;
            const int x0 = bx * g.e[0];
            const int64_t boff = yz.base + (int64_t)bx * g.bstride;
            for (int lx = lo + (int)threadIdx.x; lx < hi; lx += blockDim.x)
                urow[x0 + lx] = s[boff + lx];
        }
    }
}

// b = fl_R(h2 * f): the product in FP64, one rounding to R.
template <typename R>
__global__ __launch_bounds__(256) void k_scale_source(Geom g, const R *__restrict__ f,
                                                      R *__restrict__ b, double h2,
                                                      int64_t rows) {
    const int nx = g.n[0], ny = g.n[1];
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = (int)(r % ny), z = (int)(r / ny);
        int by, ly, bz = 0, lz = 0;
        owner(y, g.e[1], g.nb[1], by, ly);
        if (g.ndim == 3) owner(z, g.e[2], g.nb[2], bz, lz);
        const int64_t base = ((int64_t)bz * g.nb[1] + by) * g.nb[0] * g.sstride +
                             ((int64_t)lz * g.e[1] + ly) * g.e[0];
        const R *frow = f + r * nx;
        for (int bx = 0; bx < g.nb[0]; ++bx) {
            const int ext = extent(g.n[0], g.e[0], bx);
            const int x0 = bx * g.e[0];
            const int64_t boff = base + (int64_t)bx * g.sstride;
            for (int lx = (int)threadIdx.x; lx < ext; lx += blockDim.x)
                b[boff + lx] = (R)(h2 * (double)frow[x0 + lx]);
        }
    }
}

// Halo exchange.  Work item (block, face, t): face = 2*axis + side (side 0 =
// low, 1 = high), t enumerates the face's cells over the block's extents in
// the other axes (first of them fastest, so y- and z-faces are contiguous
// rows).  Faces on the domain boundary keep the Dirichlet values.
template <typename R>
__global__ __launch_bounds__(256) void k_halo_exchange(Geom g, R *__restrict__ s,
                                                       int64_t maxface, int64_t total) {
    const int nf = 2 * g.ndim;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i % maxface;
        const int64_t rest = i / maxface;
        const int face = (int)(rest % nf);
        const int64_t blk = rest / nf;
        const int axis = face >> 1, side = face & 1;
        int bc[3];
        bc[0] = (int)(blk % g.nb[0]);
        bc[1] = (int)((blk / g.nb[0]) % g.nb[1]);
        bc[2] = (int)(blk / ((int64_t)g.nb[0] * g.nb[1]));
        if (side == 0 && bc[axis] == 0) continue;
        if (side == 1 && bc[axis] == g.nb[axis] - 1) continue;
        int ext[3];
        for (int a = 0; a < 3; ++a) ext[a] = a < g.ndim ? extent(g.n[a], g.e[a], bc[a]) : 1;
        // the two tangential axes, lower one first
        const int ta = axis == 0 ? 1 : 0;
        const int tb = axis == 2 ? 1 : 2;
        const int64_t fa = ext[ta];
        const int64_t fb = (g.ndim == 3) ? ext[tb] : 1;
        if (t >= fa * fb) continue;
        int loc[3] = {0, 0, 0};
        loc[ta] = (int)(t % fa);
        if (g.ndim == 3) loc[tb] = (int)(t / fa);
        loc[axis] = side == 0 ? -1 : ext[axis];
        const int64_t dst = local_offset(g, blk, loc[0], loc[1], loc[2]);
        // the halo cell's global coordinates; its owner is the face neighbour
        const int gx = bc[0] * g.e[0] + loc[0];
        const int gy = bc[1] * g.e[1] + loc[1];
        const int gz = g.ndim == 3 ? bc[2] * g.e[2] + loc[2] : 0;
        s[dst] = s[state_offset(g, gx, gy, gz)];
    }
}

// Face sends of the source blocks b0 .. b1-1: work item (block, face, t) as
// in k_halo_exchange, but the block is the sender: its edge cells go into
// the halo of its face neighbour.  Sending the faces of every block fills
// the same halo cells, with the same values, as k_halo_exchange.
template <typename R>
__global__ __launch_bounds__(256) void k_halo_send(Geom g, R *__restrict__ s, int64_t b0,
                                                   int64_t maxface, int64_t total) {
    const int nf = 2 * g.ndim;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i % maxface;
        const int64_t rest = i / maxface;
        const int face = (int)(rest % nf);
        const int64_t blk = b0 + rest / nf;
        const int axis = face >> 1, side = face & 1;
        int bc[3];
        bc[0] = (int)(blk % g.nb[0]);
        bc[1] = (int)((blk / g.nb[0]) % g.nb[1]);
        bc[2] = (int)(blk / ((int64_t)g.nb[0] * g.nb[1]));
        if (side == 0 && bc[axis] == 0) continue;
        if (side == 1 && bc[axis] == g.nb[axis] - 1) continue;
        int ext[3];
        for (int a = 0; a < 3; ++a) ext[a] = a < g.ndim ? extent(g.n[a], g.e[a], bc[a]) : 1;
        const int ta = axis == 0 ? 1 : 0;
        const int tb = axis == 2 ? 1 : 2;
        const int64_t fa = ext[ta];
        const int64_t fb = (g.ndim == 3) ? ext[tb] : 1;
        if (t >= fa * fb) continue;
        int loc[3] = {0, 0, 0};
        loc[ta] = (int)(t % fa);
        if (g.ndim == 3) loc[tb] = (int)(t / fa);
        loc[axis] = side == 0 ? 0 : ext[axis] - 1;  // the block's edge cell
        const int64_t src = local_offset(g, blk, loc[0], loc[1], loc[2]);
        // the neighbour across the face and the halo slot facing this block
        int64_t step = 1;
        for (int a = 0; a < axis; ++a) step *= g.nb[a];
        const int64_t nbr = side == 0 ? blk - step : blk + step;
        int nloc[3] = {loc[0], loc[1], loc[2]};
        nloc[axis] = side == 0 ? g.e[axis] : -1;  // a low neighbour is a full block
        s[local_offset(g, nbr, nloc[0], nloc[1], nloc[2])] = s[src];
    }
}

// Grid of the row maps: one workgroup per row, rows strided beyond 2^20.
static inline dim3 row_grid(int64_t rows) {
    const int64_t gx = rows < 1 ? 1 : rows > (1 << 20) ? (1 << 20) : rows;
    return dim3((unsigned)gx);
}

static inline int grid_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename R>
hipError_t launch_scatter(const Geom &g, const void *u, void *s0, void *s1, bool zero_ring,
                          hipStream_t st) {
    const int64_t rows = (int64_t)(g.n[1] + 2) * (g.ndim == 3 ? g.n[2] + 2 : 1);
    hipLaunchKernelGGL(k_scatter<R>, row_grid(rows), dim3(256), 0, st, g,
                       (const R *)u, (R *)s0, (R *)s1, rows, zero_ring ? 1 : 0);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_f64(double *__restrict__ p, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// End of a 2D adjoint run.  gb: FP64 interior accumulator dL/db (n_y x n_x).
// Two stream-ordered kernels so that grad_f may alias gb:
//  1. grad_ring (full (n_y+2) x (n_x+2) array): each non-corner ring node gets
//     gb at the one interior node next to it (dL/dg_q = sum_k w lam_k[p(q)]
//     = gb[p(q)]); corners and interior nodes get 0;
//  2. grad_f (interior) = h2 * gb.
__global__ __launch_bounds__(256) void k_adjoint_ring(int nx, int ny, const double *__restrict__ gb,
                                                      double *__restrict__ grad_ring,
                                                      int64_t total) {
    const int64_t nx2 = nx + 2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx2) - 1;
        const int y = (int)(i / nx2) - 1;
        const bool inx = x >= 0 && x < nx, iny = y >= 0 && y < ny;
        double v = 0.0;
        if (inx && !iny) v = gb[(int64_t)(y < 0 ? 0 : ny - 1) * nx + x];
        if (iny && !inx) v = gb[(int64_t)y * nx + (x < 0 ? 0 : nx - 1)];
        grad_ring[i] = v;
    }
}

// Full dL/dU0 of a 2D adjoint run whose loss reads all of u_K (ring
// included).  A sweep copies the ring, so the ring of u_K is g itself and
// each ring node gets dL/du_K there plus, for non-corner nodes, what flowed
// through the sweeps (gb at its interior neighbour); corners get only
// dL/du_K.  Interior nodes get lam_0, read from the blocked state s.
template <typename R>
__global__ __launch_bounds__(256) void k_adjoint_full(Geom g, const double *__restrict__ gb,
                                                      const R *__restrict__ lamK,
                                                      const R *__restrict__ s,
                                                      double *__restrict__ out, int64_t total) {
    const int nx = g.n[0], ny = g.n[1];
    const int64_t nx2 = nx + 2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx2) - 1;
        const int y = (int)(i / nx2) - 1;
        const bool inx = x >= 0 && x < nx, iny = y >= 0 && y < ny;
        double v;
        if (inx && iny) {
            v = (double)s[state_offset(g, x, y, 0)];
        } else {
            v = (double)lamK[i];
            if (inx) v = v + gb[(int64_t)(y < 0 ? 0 : ny - 1) * nx + x];
            if (iny) v = v + gb[(int64_t)y * nx + (x < 0 ? 0 : nx - 1)];
        }
        out[i] = v;
    }
}

template <typename R>
hipError_t launch_adjoint_full(const Geom &g, const double *gb, const void *lamK, const void *s,
                               double *out, hipStream_t st) {
    const int64_t total = (int64_t)(g.n[0] + 2) * (g.n[1] + 2);
    hipLaunchKernelGGL(k_adjoint_full<R>, dim3(grid_for(total)), dim3(256), 0, st, g, gb,
                       (const R *)lamK, (const R *)s, out, total);
    return hipGetLastError();
}
template hipError_t launch_adjoint_full<float>(const Geom &, const double *, const void *,
                                               const void *, double *, hipStream_t);
template hipError_t launch_adjoint_full<double>(const Geom &, const double *, const void *,
                                                const void *, double *, hipStream_t);

__global__ __launch_bounds__(256) void k_scale_f64(const double *gb, double h2, double *out,
                                                   int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = h2 * gb[i];
}

hipError_t launch_adjoint_finish(const Geom &g, const double *gb, double h2, double *grad_f,
                                 double *grad_ring, hipStream_t st) {
    if (grad_ring) {
        const int64_t total = (int64_t)(g.n[0] + 2) * (g.n[1] + 2);
        hipLaunchKernelGGL(k_adjoint_ring, dim3(grid_for(total)), dim3(256), 0, st, g.n[0],
                           g.n[1], gb, grad_ring, total);
    }
    if (grad_f) {
        const int64_t n = (int64_t)g.n[0] * g.n[1];
        hipLaunchKernelGGL(k_scale_f64, dim3(grid_for(n)), dim3(256), 0, st, gb, h2, grad_f, n);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gather(const Geom &g, const void *s, void *u, hipStream_t st) {
    const int64_t rows = (int64_t)(g.n[1] + 2) * (g.ndim == 3 ? g.n[2] + 2 : 1);
    hipLaunchKernelGGL(k_gather<R>, row_grid(rows), dim3(256), 0, st, g,
                       (const R *)s, (R *)u, rows);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_scale_source(const Geom &g, const void *f, void *b, double h2, hipStream_t st) {
    const int64_t rows = (int64_t)g.n[1] * (g.ndim == 3 ? g.n[2] : 1);
    hipLaunchKernelGGL(k_scale_source<R>, row_grid(rows), dim3(256), 0, st, g,
                       (const R *)f, (R *)b, h2, rows);
    return hipGetLastError();
}

int64_t halo_maxface(const Geom &g) {
    if (g.ndim == 2) return g.e[0] > g.e[1] ? g.e[0] : g.e[1];
    int64_t a = (int64_t)g.e[1] * g.e[2], b = (int64_t)g.e[0] * g.e[2], c = (int64_t)g.e[0] * g.e[1];
    int64_t m = a > b ? a : b;
    return m > c ? m : c;
}

template <typename R>
hipError_t launch_halo_exchange(const Geom &g, void *s, hipStream_t st) {
    const int64_t maxface = halo_maxface(g);
    const int64_t total = g.nblocks * 2 * g.ndim * maxface;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_halo_exchange<R>, dim3(grid_for(total)), dim3(256), 0, st, g, (R *)s,
                       maxface, total);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_halo_send(const Geom &g, void *s, int64_t b0, int64_t b1, hipStream_t st) {
    const int64_t maxface = halo_maxface(g);
    const int64_t total = (b1 - b0) * 2 * g.ndim * maxface;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_halo_send<R>, dim3(grid_for(total)), dim3(256), 0, st, g, (R *)s, b0,
                       maxface, total);
    return hipGetLastError();
}

template hipError_t launch_halo_send<float>(const Geom &, void *, int64_t, int64_t, hipStream_t);
template hipError_t launch_halo_send<double>(const Geom &, void *, int64_t, int64_t, hipStream_t);
template hipError_t launch_scatter<float>(const Geom &, const void *, void *, void *, bool,
                                          hipStream_t);
template hipError_t launch_scatter<double>(const Geom &, const void *, void *, void *, bool,
                                           hipStream_t);
template hipError_t launch_gather<float>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_gather<double>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_scale_source<float>(const Geom &, const void *, void *, double, hipStream_t);
template hipError_t launch_scale_source<double>(const Geom &, const void *, void *, double, hipStream_t);
template hipError_t launch_halo_exchange<float>(const Geom &, void *, hipStream_t);
template hipError_t launch_halo_exchange<double>(const Geom &, void *, hipStream_t);

}  // namespace jac
