// Internal definitions shared by the host library and the gfx950 kernels.
//
// Block storage (one layout for every state buffer):
//   The interior is cut into nb[0] x nb[1] (x nb[2]) blocks with maximum
//   extents e[0], e[1] (, e[2]); block (p, q, r) owns interior nodes
//   p*e[0] ... min((p+1)*e[0], n[0]) - 1 along x, and likewise on y and z.
//   e[0] is a multiple of 32 bytes of elements, so every 16-byte lane chunk
//   of a row lies inside one block.
//   Each block stores its interior plus a one-cell halo ring as rows of
//   `pitch` = AX + e[0] rounded up to AX elements, AX = 128 bytes of
//   elements: local node (lx, ly, lz) with lx in [-1, ex], ly in [-1, ey],
//   lz in [-1, ez] lives at element
//       blk * bstride + (lz+1) * plane + (ly+1) * pitch + AX + lx
//   with plane = (e[1]+2) * pitch (the plane term is absent in 2D), so every
//   interior row starts 128-byte aligned (an interior row of 2^k cache lines
//   is fetched as exactly those lines) and a whole block is one contiguous
//   stream of rows.  The east ring cell (lx = ex) of a full-width row is
//   element 0 of the next row, a slot no row uses; bstride leaves AX
//   elements of slack after the last row.  Halo cells on the domain boundary hold the
//   Dirichlet ring; the others mirror the face neighbour's edge cells.
//   Source b is stored per block without halo: element
//       blk * sstride + (lz * e[1] + ly) * e[0] + lx.
#pragma once

#include <stdint.h>

namespace jac {

constexpr int kMaxDim = 3;

struct Geom {
    int ndim;
    int ax;              // offset of interior column 0 in a row, elements (128 bytes)
    int n[3];            // interior nodes per axis (x, y, z); 1 for unused axes
    int nb[3];           // blocks per axis
    int e[3];            // maximum block extent per axis
    int64_t pitch;       // row pitch of a stored block, elements
    int64_t plane;       // (e[1] + 2) * pitch
    int64_t bstride;     // elements between consecutive blocks (state)
    int64_t sstride;     // elements between consecutive blocks (source)
    int64_t nblocks;
};

// One grid of a batch, as the batched pass kernel sees it.
struct BatchGrid {
    Geom g;
    void *u[2];     // the two state buffers
    const void *b;  // blocked source
};

// Device-side state of a batched solve (arrays of one entry per grid).
struct BatchState {
    int *active;          // 1 while the grid still sweeps
    int *status;          // 0 running, 1 converged, 2 max sweeps, 3 diverged
    int *final_buf;       // state buffer holding the grid's final state
    long long *sweeps;    // sweeps of the final state
    double *rel;          // last relative residual
    double *res0;         // residual of the initial state
    double *res;          // last residual
    int *pass_count;      // passes done (parity of the current buffer)
    long long *k_now;     // sweeps done by the active grids
};

// Block index and local coordinate of global coordinate v in [-1, n] along an
// axis with extent e and nb blocks: -1 belongs to block 0 (its low halo),
// n to the last block (its high halo).
__host__ __device__ inline void owner(int v, int e, int nb, int &blk, int &loc) {
    int b = v < 0 ? 0 : v / e;
    b = b < nb - 1 ? b : nb - 1;
    blk = b;
    loc = v - b * e;
}

__host__ __device__ inline int extent(int n, int e, int blk) {
    const int rest = n - blk * e;
    return rest < e ? rest : e;
}

// Element offset of local node (lx, ly, lz) of block blk (lz ignored in 2D).
__host__ __device__ inline int64_t local_offset(const Geom &g, int64_t blk, int lx, int ly, int lz) {
    const int64_t planes = g.ndim == 3 ? (int64_t)(lz + 1) * g.plane : 0;
    return blk * g.bstride + planes + (int64_t)(ly + 1) * g.pitch + g.ax + lx;
}

// Element offset of global node (x, y, z), each in [-1, n], inside the block
// that owns it (halo slot for ring nodes).
__host__ __device__ inline int64_t state_offset(const Geom &g, int x, int y, int z) {
    int bx, lx, by, ly, bz = 0, lz = 0;
    owner(x, g.e[0], g.nb[0], bx, lx);
    owner(y, g.e[1], g.nb[1], by, ly);
    if (g.ndim == 3) owner(z, g.e[2], g.nb[2], bz, lz);
    const int64_t blk = ((int64_t)bz * g.nb[1] + by) * g.nb[0] + bx;
    return local_offset(g, blk, lx, ly, lz);
}

// Element offset of the source value of interior node (x, y, z).
__host__ __device__ inline int64_t source_offset(const Geom &g, int x, int y, int z) {
    int bx, lx, by, ly, bz = 0, lz = 0;
    owner(x, g.e[0], g.nb[0], bx, lx);
    owner(y, g.e[1], g.nb[1], by, ly);
    if (g.ndim == 3) owner(z, g.e[2], g.nb[2], bz, lz);
    const int64_t blk = ((int64_t)bz * g.nb[1] + by) * g.nb[0] + bx;
    return blk * g.sstride + ((int64_t)lz * g.e[1] + ly) * g.e[0] + lx;
}

}  // namespace jac
