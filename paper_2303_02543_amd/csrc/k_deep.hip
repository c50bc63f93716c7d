// Deep-halo block storage: every block keeps a frame of H cells around its
// interior (faces, edges and corners), refreshed by one exchange every H
// sweeps, after which each block can run up to H sweeps from its own storage
// alone -- the communication-avoiding form of the over-decomposed Jacobi
// proxy (Section 4.3's per-iteration face exchange, Section 4.4's
// over-decomposition), where a piece talks to its neighbours once per H
// sweeps instead of once per sweep.
//
// The state buffers use the block layout of jacobi_internal.h with a larger
// row pitch, more rows and planes per block and a larger ax, so local_offset
// addresses local nodes -H .. e+H-1 on every axis: the standard kernels see
// the interior and the one-cell ring of each block as usual.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

// Frame cell f of a block with extents (ex, ey, ez) and frame width H:
// local coordinates, or false if f lies outside this block's frame (the
// enumeration covers the largest block, W = e0 + 2H wide, Y = e1 + 2H rows).
// 2D: the H rows above and below the block over the full frame width, then
// the H columns left and right of each interior row.  3D: the H planes below
// and above the block (full W x Y), then in each interior plane the H rows
// below and above (full W), then in each interior row the H columns on
// either side.
__device__ __forceinline__ bool frame_cell(const Geom &g, int H, int ex, int ey, int ez, int f,
                                           int &lx, int &ly, int &lz) {
    const int W = g.e[0] + 2 * H;
    if (g.ndim == 2) {
        lz = 0;
        const int band = 2 * H * W;
        if (f < band) {
            const int r = f / W;
            lx = f - r * W - H;
            ly = r < H ? r - H : ey + (r - H);
        } else {
            const int q = f - band;
            ly = q / (2 * H);
            const int c = q - ly * 2 * H;
            lx = c < H ? c - H : ex + (c - H);
            if (ly >= ey) return false;
        }
        return lx < ex + H;
    }
    const int Y = g.e[1] + 2 * H;
    const int zb = 2 * H * W * Y;           // plane slabs
    const int yb = g.e[2] * 2 * H * W;      // row slabs of the interior planes
    if (f < zb) {
        const int pl = f / (W * Y);
        const int r = f - pl * W * Y;
        lz = pl < H ? pl - H : ez + (pl - H);
        ly = r / W - H;
        lx = r % W - H;
    } else if (f < zb + yb) {
        const int q = f - zb;
        lz = q / (2 * H * W);
        const int r = q - lz * 2 * H * W;
        const int row = r / W;
        ly = row < H ? row - H : ey + (row - H);
        lx = r - row * W - H;
        if (lz >= ez) return false;
    } else {
        const int q = f - zb - yb;
        const int per_plane = g.e[1] * 2 * H;
        lz = q / per_plane;
        const int r = q - lz * per_plane;
        ly = r / (2 * H);
        const int c = r - ly * 2 * H;
        lx = c < H ? c - H : ex + (c - H);
        if (lz >= ez || ly >= ey) return false;
    }
    return lx < ex + H && ly < ey + H && lz < ez + H;
}

__host__ __device__ inline int64_t frame_cells(const Geom &g, int H) {
    const int64_t W = g.e[0] + 2 * H;
    if (g.ndim == 2) return 2 * (int64_t)H * W + (int64_t)g.e[1] * 2 * H;
    const int64_t Y = g.e[1] + 2 * H;
    return 2 * (int64_t)H * W * Y + (int64_t)g.e[2] * 2 * H * W +
           (int64_t)g.e[2] * g.e[1] * 2 * H;
}

// Refresh every block's frame: a frame cell whose node belongs to a
// neighbouring block takes that block's value (an interior cell, or a ring
// node the neighbour holds in its own one-cell ring: a corner region along
// the domain's side); on the domain's own sides the frame holds the block's
// ring, which never changes, and cells beyond it, which no pass reads.
// Grid: x over the frame cells of one block, kDeepCells per thread (few
// large workgroups: one cell per thread made the 3D exchange bound by
// workgroup dispatch), y over blocks (strided).
constexpr int kDeepCells = 16;

template <typename R>
__global__ __launch_bounds__(256) void k_deep_exchange(Geom g, R *__restrict__ s, int H,
                                                       int per_block) {
    for (int64_t blk = blockIdx.y; blk < g.nblocks; blk += gridDim.y) {
        const int bx = (int)(blk % g.nb[0]);
        const int by = (int)((blk / g.nb[0]) % g.nb[1]);
        const int bz = g.ndim == 3 ? (int)(blk / ((int64_t)g.nb[0] * g.nb[1])) : 0;
        const int ex = extent(g.n[0], g.e[0], bx);
        const int ey = extent(g.n[1], g.e[1], by);
        const int ez = g.ndim == 3 ? extent(g.n[2], g.e[2], bz) : 1;
        for (int k = 0; k < kDeepCells; ++k) {
        const int f = (blockIdx.x * kDeepCells + k) * blockDim.x + threadIdx.x;
        if (f >= per_block) break;
        int lx, ly, lz;
        if (!frame_cell(g, H, ex, ey, ez, f, lx, ly, lz)) continue;
        // the owner along each axis is the adjacent block or this one (the
        // frame is no deeper than any block); on a domain side the ring layer
        // (-1 or the extent) is held by this axis's own block in its one-cell
        // ring, and cells beyond it are never read
        int o[3] = {bx, by, bz}, l[3] = {lx, ly, lz};
        const int ext[3] = {ex, ey, ez};
        bool skip = false;
        for (int a = 0; a < g.ndim; ++a) {
            if (l[a] < 0) {
                if (o[a] > 0) {
                    --o[a];
                    l[a] += g.e[a];
                } else if (l[a] < -1) {
                    skip = true;
                }
            } else if (l[a] >= ext[a]) {
                if (o[a] < g.nb[a] - 1) {
                    ++o[a];
                    l[a] -= ext[a];
                } else if (l[a] > ext[a]) {
                    skip = true;
                }
            }
        }
        const int64_t ob = ((int64_t)o[2] * g.nb[1] + o[1]) * g.nb[0] + o[0];
        if (skip || ob == blk) continue;  // beyond the ring, or the block's own ring
        s[local_offset(g, blk, lx, ly, lz)] = s[local_offset(g, ob, l[0], l[1], l[2])];
        }
    }
}

// Fill the deep source buffer (the state layout) from the blocked source:
// every cell of a block's interior and frame whose global node is interior
// gets b there, every other cell 0.
template <typename R>
__global__ __launch_bounds__(256) void k_deep_source(Geom g, const R *__restrict__ b,
                                                     R *__restrict__ bd, int H, int64_t total) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t W = g.e[0] + 2 * H, Y = g.e[1] + 2 * H;
    const int64_t Zn = g.ndim == 3 ? g.e[2] + 2 * H : 1;
    const int64_t per = W * Y * Zn;
    const int64_t blk = i / per;
    const int64_t r = i % per;
    const int lx = (int)(r % W) - H;
    const int ly = (int)((r / W) % Y) - H;
    const int lz = g.ndim == 3 ? (int)(r / (W * Y)) - H : 0;
    const int bx = (int)(blk % g.nb[0]);
    const int by = (int)((blk / g.nb[0]) % g.nb[1]);
    const int bz = g.ndim == 3 ? (int)(blk / ((int64_t)g.nb[0] * g.nb[1])) : 0;
    const int X = bx * g.e[0] + lx, Y2 = by * g.e[1] + ly, Z = bz * g.e[2] + lz;
    const bool in = X >= 0 && X < g.n[0] && Y2 >= 0 && Y2 < g.n[1] &&
                    (g.ndim == 2 || (Z >= 0 && Z < g.n[2]));
    bd[local_offset(g, blk, lx, ly, lz)] = in && b ? b[source_offset(g, X, Y2, Z)] : (R)0;
}

template <typename R>
hipError_t launch_deep_exchange(const Geom &g, void *s, int H, hipStream_t st) {
    const int64_t per = frame_cells(g, H);
    if (per > 0x7fffffff - 255) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)((per + 256 * kDeepCells - 1) / (256 * kDeepCells));
    const unsigned gy = (unsigned)(g.nblocks < 65535 ? g.nblocks : 65535);
    hipLaunchKernelGGL(k_deep_exchange<R>, dim3(gx, gy), dim3(256), 0, st, g, (R *)s, H, (int)per);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_deep_source(const Geom &g, const void *b, void *bd, int H, hipStream_t st) {
    const int64_t per = (int64_t)(g.e[0] + 2 * H) * (g.e[1] + 2 * H) *
                        (g.ndim == 3 ? g.e[2] + 2 * H : 1);
    const int64_t total = per * g.nblocks;
    const int64_t grid = (total + 255) / 256;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_deep_source<R>, dim3((unsigned)grid), dim3(256), 0, st, g,
                       (const R *)b, (R *)bd, H, total);
    return hipGetLastError();
}

template hipError_t launch_deep_exchange<float>(const Geom &, void *, int, hipStream_t);
template hipError_t launch_deep_exchange<double>(const Geom &, void *, int, hipStream_t);
template hipError_t launch_deep_source<float>(const Geom &, const void *, void *, int, hipStream_t);
template hipError_t launch_deep_source<double>(const Geom &, const void *, void *, int,
                                               hipStream_t);

}  // namespace jac
