// Fused 3D Jacobi pass kernel for gfx950: T sweeps per pass (temporal
// blocking along z), halo cells read straight from the neighbouring blocks,
// and the FP64 residual of the pass's input state folded into the first
// level.
//
// The update is the 7-point Jacobi step of the proxy application in
// Section 4.3 of the paper, evaluated as
//   s = ((W + E) + (S + N)) + (B + F);  u' = (s + b) * fl(1/6)
// with no FMA contraction, so every schedule gives the same bits.
//
// A workgroup of 8 waves holds 32 rows by 16 lanes x V elements along x (one
// 16-lane row of a wave per grid row; 64 columns in FP32, 32 in FP64) and
// marches along z through a segment of planes.  For the 64^3 blocks of the
// workloads a wave's 4 rows lie in one block, so every load instruction reads
// neighbouring rows of one block.  Each plane of the state and the source is
// loaded once, from whichever block owns it -- the exchange of halo cells
// between blocks happens inside these loads -- and pushed through T levels:
// at the step that loads plane z + 1, level s computes plane z - s + 1 from
// the planes z - s .. z - s + 2 of level s - 1, each lane keeping three planes
// of every level in registers.  The rows y - 1 and y + 1 come from the
// workgroup's LDS copy of level s - 1's plane, which that level computed one
// step earlier, so one barrier per step serves every level (two LDS buffers
// alternate by step).  x neighbours come from DPP shifts within each 16-lane
// row; level 1 also reads the cells just outside the tile (one scalar load
// per row end) and the two rows just outside it (one load each), so it is
// valid on the whole tile, and level s on the tile less s - 1 cells on every
// side in x and y.  Level T is the pass's output on the inner tile: rows
// T-1 .. 32-T, columns A0 .. A0+OW-1 (chunk-aligned).  A z segment costs
// 2(T-1) extra planes of warm-up.
//
// The Dirichlet ring keeps its values at every level: a level on a ring
// plane (z = -1 or n_z) copies its input; tiles that reach the ring in x or
// y copy the input on every ring cell.  Rows, columns and planes beyond the
// ring are read from clamped in-bounds addresses and never reach an output.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

constexpr int kM3Waves = 8;              // waves per work item (workgroup)
constexpr int kM3Threads = 64 * kM3Waves;
constexpr int kM3Rows = 4 * kM3Waves;    // rows held per work item (4 per wave)

template <typename R, int T>
struct M3 {
    static constexpr int V = 16 / (int)sizeof(R);
    static constexpr int W = 16 * V;                         // columns held per work item
    static constexpr int A0 = V * ((T - 1 + V - 1) / V);     // first output column (chunk-aligned)
    static constexpr int OW = V * ((W - (T - 1) - A0) / V);  // output columns per work item
    static constexpr int OY = kM3Rows - 2 * (T - 1);         // output rows per work item
    static constexpr int U = 6;   // steps per unrolled group: ring slots mod 3, LDS buffers mod 2
    static constexpr int NL = T > 1 ? T - 1 : 1;             // levels 1 .. T-1 held in registers
    static_assert(T >= 1 && T + 1 <= U, "source ring holds T + 1 planes");
    static_assert(OW > 0 && OY > 0, "tile too small for this depth");
};

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

// Plane cursor: global plane q (any integer), advanced one plane at a time;
// off / soff are the element offsets of plane q clamped to [-1, n_z] in the
// state buffers and (0 for the ring planes) in the source (the ring planes
// stand in for the planes beyond them).
struct ZCur {
    int q, blk, loc;
    int64_t off, soff;
    __device__ __forceinline__ void set(const Geom &g) {
        off = plane_part(g, blk, loc);
        soff = q >= 0 && q < g.n[2] ? src_plane_part(g, blk, loc) : 0;
    }
    __device__ __forceinline__ void init(const Geom &g, int q0) {
        q = q0;
        owner(q0 < -1 ? -1 : q0 > g.n[2] ? g.n[2] : q0, g.e[2], g.nb[2], blk, loc);
        set(g);
    }
    __device__ __forceinline__ void advance(const Geom &g) {
        const bool moves = q >= -1 && q < g.n[2];
        ++q;
        if (moves) {
            ++loc;
            if (loc >= g.e[2] && blk < g.nb[2] - 1) {
                ++blk;
                loc = 0;
                set(g);
            } else {
                off += g.plane;
                soff = q >= 0 && q < g.n[2] ? (q == 0 ? src_plane_part(g, blk, loc)
                                                      : soff + (int64_t)g.e[1] * g.e[0])
                                            : 0;
            }
        }
    }
};

// Per-lane constants of a work item.
struct M3Lane {
    int64_t c_off, h_off, e_off, b_off;  // own row, halo row (loaders), edge cell, source
    int k;                               // LDS row slot of the lane's own row (1 .. 16)
    int hk;                              // LDS slot of the lane's halo load (0, 17; own slot: none)
    bool ld, lde, ldb;                   // lane loads interior/east-ring, edge, source
    bool upd[8];                         // element is an interior cell
    bool mine[8];                        // element is an output cell of this work item
    bool out_lane;                       // the whole chunk is output (interior tiles)
};

template <typename R, int T>
struct M3Regs {
    using S = M3<R, T>;
    Chunk<R, S::V> l0[3];       // level 0: planes by plane index mod 3
    Chunk<R, S::V> halo[3];     // level-0 halo row (loader lanes)
    R edge[3];                  // level-0 cell just outside the tile (row ends)
    Chunk<R, S::V> bq[S::U];    // source planes by plane index mod U
    Chunk<R, S::V> lv[S::NL][3];  // levels 1 .. T-1: planes by step mod 3
    double acc;                 // residual partial (level 1)
};

template <typename R, int T>
using M3Sh = Chunk<R, 16 / sizeof(R)> (*)[2][kM3Rows + 2][16];

// Store a register chunk into LDS element by element (one 16-byte write).
template <typename R, int V>
__device__ __forceinline__ void lds_put(Chunk<R, V> &dst, const Chunk<R, V> &src) {
    Chunk<R, V> t;
#pragma unroll
    for (int v = 0; v < V; ++v) t.v[v] = src.v[v];
    dst = t;
}

// Issue the loads of plane lc.q into slot J1 (level 0, halo, edge) and
// source slot JB, then advance the cursor.
template <typename R, int T, bool EDGE, bool SRC, int J1, int JB>
__device__ __forceinline__ void m3_load(const Geom &g, const R *__restrict__ uin,
                                        const R *__restrict__ bsrc, const M3Lane &L,
                                        M3Regs<R, T> &m, ZCur &lc) {
    constexpr int V = M3<R, T>::V;
    using C = Chunk<R, V>;
    const int64_t pp = lc.off;
    // element-wise copies keep every ring slot in registers
    const C c = *reinterpret_cast<const C *>(uin + pp + L.c_off);
    // every lane loads (non-loader lanes their own row again), so no load
    // sits under a per-lane branch
    const C h = *reinterpret_cast<const C *>(uin + pp + L.h_off);
    const R e = uin[pp + L.e_off];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        m.l0[J1].v[v] = (EDGE && !L.ld) ? (R)0 : c.v[v];
        m.halo[J1].v[v] = (EDGE && !L.ld) ? (R)0 : h.v[v];
    }
    m.edge[J1] = (EDGE && !L.lde) ? (R)0 : e;
    if constexpr (SRC) {
        const C b = *reinterpret_cast<const C *>(bsrc + lc.soff + L.b_off);
#pragma unroll
        for (int v = 0; v < V; ++v) m.bq[JB].v[v] = (EDGE && !L.ldb) ? (R)0 : b.v[v];
    }
    lc.advance(g);
}

// Level S of step J (z = base + J): plane p = z - S + 1 of level S from the
// planes p-1, p, p+1 of level S-1 (registers) and the rows y-1, y+1 of plane
// p of level S-1 (LDS buffer J & 1).
template <typename R, int T, int MODE, bool EDGE, bool RES, int J, int S>
__device__ __forceinline__ void m3_level(const Geom &g, R *__restrict__ uout, const M3Lane &L,
                                         M3Regs<R, T> &m, M3Sh<R, T> sh, const int z,
                                         const int oz0, const int oz1, ZCur &sc, bool nt) {
    using M = M3<R, T>;
    constexpr int V = M::V;
    constexpr bool SRC = MODE == 1;
    using C = Chunk<R, V>;
    if constexpr (S <= T) {
        const int p = z - S + 1;
        const int cx = threadIdx.x & 15;
        C zm, zc, zp;
        R eo = (R)0;
        if constexpr (S == 1) {
            zm = m.l0[(J + 2) % 3];
            zc = m.l0[J % 3];
            zp = m.l0[(J + 1) % 3];
            eo = m.edge[J % 3];
        } else {
            zm = m.lv[S - 2][(J + 1) % 3];  // step J - 2
            zc = m.lv[S - 2][(J + 2) % 3];  // step J - 1
            zp = m.lv[S - 2][J % 3];        // this step
        }
        const C so = sh[S - 1][J & 1][L.k - 1][cx];
        const C no = sh[S - 1][J & 1][L.k + 1][cx];
        C bb;
        if constexpr (SRC) bb = m.bq[(J - S + 1 + M::U) % M::U];
        const R left = row_shift_up(eo, zc.v[V - 1]);
        const R right = row_shift_down(eo, zc.v[0]);
        const R w = (R)1 / (R)6;
        const bool pin = p >= 0 && p < g.n[2];
        const bool res_plane = RES && S == 1 && p >= oz0 && p < oz1;
        C out;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R Wv = v > 0 ? zc.v[v - 1] : left;
            const R Ev = v < V - 1 ? zc.v[v + 1] : right;
            const R s = ((Wv + Ev) + (so.v[v] + no.v[v])) + (zm.v[v] + zp.v[v]);
            R o = SRC ? (s + bb.v[v]) * w : s * w;
            if (res_plane) {
                // residual of the input state, FP64 from widened values
                const double sd = (((double)Wv + (double)Ev) + ((double)so.v[v] + (double)no.v[v])) +
                                  ((double)zm.v[v] + (double)zp.v[v]);
                const double bd = SRC ? (double)bb.v[v] : 0.0;
                const double r = bd - (6.0 * (double)zc.v[v] - sd);
                m.acc += L.mine[v] ? r * r : 0.0;
            }
            // ring cells and cells beyond the ring keep their values
            if constexpr (EDGE) o = L.upd[v] ? o : zc.v[v];
            out.v[v] = o;
        }
        if (!pin) out = zc;  // a ring plane (or beyond) keeps its values
        if constexpr (S < T) {
            m.lv[S - 1][J % 3] = out;
        } else {
            if (uout && p >= oz0 && p < oz1) {
                R *q = uout + sc.off + L.c_off;
                if (!EDGE) {
                    if (L.out_lane) {
                        if (nt)
                            store_nt16(reinterpret_cast<C *>(q), out);
                        else
                            *reinterpret_cast<C *>(q) = out;
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        if (L.mine[v]) q[v] = out.v[v];
                }
            }
        }
        m3_level<R, T, MODE, EDGE, RES, J, S + 1>(g, uout, L, m, sh, z, oz0, oz1, sc, nt);
    }
}

template <typename R, int T, int MODE, bool EDGE, bool RES, int J>
__device__ __forceinline__ void m3_steps(const Geom &g, const R *__restrict__ uin,
                                         R *__restrict__ uout, const R *__restrict__ bsrc,
                                         const M3Lane &L, M3Regs<R, T> &m, M3Sh<R, T> sh,
                                         const int base, const int zend, const int oz0,
                                         const int oz1, ZCur &lc, ZCur &sc, bool nt) {
    using M = M3<R, T>;
    constexpr bool SRC = MODE == 1;
    if constexpr (J < M::U) {
        const int z = base + J;
        if (z > zend) return;
        const int cx = threadIdx.x & 15;
        // plane z + 1 of level 0, its halo row, edge cell and source
        m3_load<R, T, EDGE, SRC, (J + 1) % 3, (J + 1) % M::U>(g, uin, bsrc, L, m, lc);
        // level 0's plane z and levels 1 .. T-1's planes of the previous step
        // go to LDS buffer J & 1 for their y neighbours
        lds_put(sh[0][J & 1][L.k][cx], m.l0[J % 3]);
        lds_put(sh[0][J & 1][L.hk][cx], m.halo[J % 3]);  // non-loaders: their own row again
#pragma unroll
        for (int s = 1; s < T; ++s) lds_put(sh[s][J & 1][L.k][cx], m.lv[s - 1][(J + 2) % 3]);
        __syncthreads();
        m3_level<R, T, MODE, EDGE, RES, J, 1>(g, uout, L, m, sh, z, oz0, oz1, sc, nt);
        sc.advance(g);
        m3_steps<R, T, MODE, EDGE, RES, J + 1>(g, uin, uout, bsrc, L, m, sh, base, zend, oz0, oz1,
                                               lc, sc, nt);
    }
}

template <typename R, int T, int MODE, bool EDGE, bool RES>
__device__ __forceinline__ void m3_body(const Geom &g, const R *__restrict__ uin,
                                        R *__restrict__ uout, const R *__restrict__ bsrc,
                                        double *__restrict__ res_slot, const M3Lane &L, int oz0,
                                        int oz1, bool nt, M3Sh<R, T> sh) {
    using M = M3<R, T>;
    constexpr int V = M::V;
    constexpr bool SRC = MODE == 1;
    M3Regs<R, T> m;
#pragma unroll
    for (int s = 0; s < M::NL; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) m.lv[s][k].v[v] = (R)0;
    m.acc = 0.0;
    // steps zs .. zend: level T computes planes oz0 .. oz1-1; planes zs-1 and
    // zs are loaded before the first step
    const int zs = oz0 - T + 1;
    const int zend = oz1 + T - 2;
    ZCur lc, sc;
    lc.init(g, zs - 1);
    m3_load<R, T, EDGE, SRC, 2, M::U - 1>(g, uin, bsrc, L, m, lc);
    m3_load<R, T, EDGE, SRC, 0, 0>(g, uin, bsrc, L, m, lc);
    sc.init(g, zs - T + 1);  // the plane level T computes at the first step
    for (int base = zs; base <= zend; base += M::U)
        m3_steps<R, T, MODE, EDGE, RES, 0>(g, uin, uout, bsrc, L, m, sh, base, zend, oz0, oz1, lc,
                                           sc, nt);
    if (RES) {
        const double a = wave_sum(m.acc);
        if ((threadIdx.x & 63) == 0) *res_slot = a;
    }
}

// Work item (one workgroup of 8 waves) number `item` of a grid cut into
// ngrp row groups (fastest), nstrips column strips and z segments of `zseg`
// output planes; wave q takes rows y0+4q .. y0+4q+3.  The residual partials
// are per wave: work item i owns partials 8i .. 8i+7 (res points at them).
template <typename R, int T, int MODE, bool RES>
__device__ __forceinline__ void m3_item(const Geom &g, const R *__restrict__ uin,
                                        R *__restrict__ uout, const R *__restrict__ bsrc,
                                        double *__restrict__ res, int item, int nstrips, int ngrp,
                                        int zseg, int nt, M3Sh<R, T> sh) {
    using M = M3<R, T>;
    constexpr int V = M::V;
    constexpr int W = M::W;
    const int grp = item % ngrp;
    const int rest = item / ngrp;
    const int strip = rest % nstrips;
    const int zs = rest / nstrips;
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int ry = lane >> 4, cx = lane & 15;
    const int nx = g.n[0], ny = g.n[1];
    const int a = strip * M::OW - M::A0;  // first column held
    const int c = a + cx * V;
    const int y0 = grp * M::OY - (T - 1);  // first row held
    const int kk = 4 * wv + ry;            // row within the tile
    const int yy = y0 + kk;
    auto clampy = [&](int y) { return y < -1 ? -1 : y > ny ? ny : y; };
    M3Lane L;
    L.k = 1 + kk;
    // chunk holds interior cells or ring / outside cells at in-bounds addresses
    L.ld = c <= nx;
    const int cl = L.ld ? c : 0;
    L.c_off = xy_part(g, cl, clampy(yy));
    L.hk = L.k;
    L.h_off = L.c_off;
    if (wv == 0 && ry == 0) {
        L.hk = 0;
        L.h_off = xy_part(g, cl, clampy(y0 - 1));
    } else if (wv == kM3Waves - 1 && ry == 3) {
        L.hk = kM3Rows + 1;
        L.h_off = xy_part(g, cl, clampy(y0 + kM3Rows));
    }
    // the first / last lane of each 16-lane row fetch the cells just west /
    // east of the tile; the others re-read their own first cell
    const int xe = cx == 0 ? a - 1 : cx == 15 ? a + W : c;
    L.lde = xe >= -1 && xe <= nx && (cx == 0 || cx == 15 || L.ld);
    L.e_off = xy_part(g, L.lde ? xe : 0, clampy(yy));
    const bool row_in = yy >= 0 && yy < ny;
    L.ldb = c >= 0 && c < nx && row_in;
    L.b_off = src_xy_part(g, L.ldb ? c : 0, L.ldb ? yy : 0);
    const bool out_row = kk >= T - 1 && kk < T - 1 + M::OY;
    L.out_lane = out_row && cx * V >= M::A0 && cx * V < M::A0 + M::OW;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        L.upd[v] = v < V && row_in && c + v >= 0 && c + v < nx;
        L.mine[v] = L.upd[v] && L.out_lane;
    }
    const int oz0 = zs * zseg;
    const int oz1 = oz0 + zseg < g.n[2] ? oz0 + zseg : g.n[2];
    double *slot = RES ? res + (int64_t)item * kM3Waves + wv : nullptr;
    const bool edge = a < 0 || a + W > nx || y0 < 0 || y0 + kM3Rows > ny;
    const bool ntb = nt != 0;
    if (edge)
        m3_body<R, T, MODE, true, RES>(g, uin, uout, bsrc, slot, L, oz0, oz1, ntb, sh);
    else
        m3_body<R, T, MODE, false, RES>(g, uin, uout, bsrc, slot, L, oz0, oz1, ntb, sh);
}

// Waves per SIMD the pass kernels are compiled for.  FP32 at depths up to 4:
// four (two workgroups per CU; their planes take at most 68 KiB of LDS), so
// that one workgroup's waves compute while the other's wait at the per-step
// barrier.  This caps the kernels at 128 VGPRs, which the FP32 Poisson pass
// with the folded residual (131 otherwise, one workgroup per CU) meets
// without spilling: 512^3 FP32 went from 0.672 to 0.627 ms per depth-4 pass.
// In FP64 the cap spilled registers and was 1% slower, so FP64 and depth 5
// keep two (the least an eight-wave workgroup implies).
template <typename R, int T>
constexpr int m3_waves_per_simd() {
    return sizeof(R) == 4 && T <= 4 ? 4 : 2;
}

template <typename R, int T, int MODE, bool RES>
__global__ __launch_bounds__(kM3Threads) __attribute__((amdgpu_waves_per_eu(m3_waves_per_simd<R, T>()))) void k_march3d(Geom g, const R *__restrict__ uin,
                                                 R *__restrict__ uout,
                                                 const R *__restrict__ bsrc,
                                                 double *__restrict__ res, int nstrips, int ngrp,
                                                 int zseg, int nitems, int nt) {
    // per level 0 .. T-1: two plane buffers of rows y0-1 .. y0+kM3Rows
    __shared__ Chunk<R, M3<R, T>::V> sh[T][2][kM3Rows + 2][16];
    const int item = xcd_logical_block(blockIdx.x, gridDim.x);
    if (item >= nitems) return;  // whole workgroup
    m3_item<R, T, MODE, RES>(g, uin, uout, bsrc, res, item, nstrips, ngrp, zseg, nt, sh);
}

// Batched pass: the work items of many grids in one launch (one descriptor
// each; the deep-halo form runs every block as its own grid).  Work item w
// belongs to grid gi with prefix[gi] <= w < prefix[gi+1]; every grid's input
// is u[0] and its output u[1].
template <typename R, int T, int MODE>
__global__ __launch_bounds__(kM3Threads) __attribute__((amdgpu_waves_per_eu(m3_waves_per_simd<R, T>()))) void k_march3d_batch(const BatchGrid *__restrict__ grids,
                                                       const int *__restrict__ prefix,
                                                       int ngrids, int zseg, int nitems) {
    using M = M3<R, T>;
    __shared__ Chunk<R, M::V> sh[T][2][kM3Rows + 2][16];
    const int w = xcd_logical_block(blockIdx.x, gridDim.x);
    if (w >= nitems) return;  // whole workgroup
    int lo = 0, hi = ngrids;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= w) lo = mid; else hi = mid;
    }
    const int gi = lo;
    const Geom g = grids[gi].g;
    const int nstrips = (g.n[0] + M::OW - 1) / M::OW;
    const int ngrp = (g.n[1] + M::OY - 1) / M::OY;
    m3_item<R, T, MODE, false>(g, (const R *)grids[gi].u[0], (R *)grids[gi].u[1],
                               (const R *)grids[gi].b, nullptr, w - prefix[gi], nstrips, ngrp, zseg,
                               0, sh);
}

template <typename R, int T>
static void m3_shape(const Geom &g, int zseg, int &nstrips, int &ngrp, int &nzs) {
    using M = M3<R, T>;
    nstrips = (g.n[0] + M::OW - 1) / M::OW;
    ngrp = (g.n[1] + M::OY - 1) / M::OY;
    nzs = (g.n[2] + zseg - 1) / zseg;
}

template <typename R, int T>
static int64_t m3_work_items(const Geom &g, int zseg) {
    int ns, ng, nz;
    m3_shape<R, T>(g, zseg, ns, ng, nz);
    return kM3Waves * (int64_t)ns * ng * nz;
}

template <typename R, int T>
static hipError_t m3_launch(const Geom &g, const void *uin, void *uout, const void *b,
                            double *res, int zseg, hipStream_t st, int64_t *nwork_out, int nt) {
    int ns, ng, nz;
    m3_shape<R, T>(g, zseg, ns, ng, nz);
    const int64_t nwaves = kM3Waves * (int64_t)ns * ng * nz;
    if (nwork_out) *nwork_out = nwaves;
    if (nwaves > 0x7fffffff - 3) return hipErrorInvalidValue;
    const int items = (int)(nwaves / kM3Waves);
    const R *bb = (const R *)b;
#define JAC_M3(MODEV, RESV)                                                                   \
    hipLaunchKernelGGL((k_march3d<R, T, MODEV, RESV>), dim3(items), dim3(kM3Threads), 0, st, g,      \
                       (const R *)uin, (R *)uout, bb, res, ns, ng, zseg, items, nt)
    if (b && res)
        JAC_M3(1, true);
    else if (b)
        JAC_M3(1, false);
    else if (res)
        JAC_M3(0, true);
    else
        JAC_M3(0, false);
#undef JAC_M3
    return hipGetLastError();
}

template <typename R, int T>
static hipError_t m3b_launch(const BatchGrid *grids, const int *prefix, int ngrids, bool src,
                             int zseg, int nitems, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (src)
        hipLaunchKernelGGL((k_march3d_batch<R, T, 1>), dim3(nitems), dim3(kM3Threads), 0, st, grids,
                           prefix, ngrids, zseg, nitems);
    else
        hipLaunchKernelGGL((k_march3d_batch<R, T, 0>), dim3(nitems), dim3(kM3Threads), 0, st, grids,
                           prefix, ngrids, zseg, nitems);
    return hipGetLastError();
}

int march3d_max_depth() { return 5; }

template <typename R>
int64_t march3d_batch_items(const Geom &g, int zseg, int depth) {
    const int64_t w = march3d_work_items<R>(g, zseg, depth);
    return w < 0 ? w : w / kM3Waves;
}

template <typename R>
hipError_t launch_march3d_batch(const BatchGrid *grids, const int *prefix, int ngrids, bool src,
                                int depth, int zseg, int nitems, hipStream_t st) {
    switch (depth) {
    case 1: return m3b_launch<R, 1>(grids, prefix, ngrids, src, zseg, nitems, st);
    case 2: return m3b_launch<R, 2>(grids, prefix, ngrids, src, zseg, nitems, st);
    case 3: return m3b_launch<R, 3>(grids, prefix, ngrids, src, zseg, nitems, st);
    case 4: return m3b_launch<R, 4>(grids, prefix, ngrids, src, zseg, nitems, st);
    case 5: return m3b_launch<R, 5>(grids, prefix, ngrids, src, zseg, nitems, st);
    default: return hipErrorInvalidValue;
    }
}

// Residual partials of one pass (one per wave, 4 per work item).
template <typename R>
int64_t march3d_work_items(const Geom &g, int zseg, int depth) {
    switch (depth) {
    case 1: return m3_work_items<R, 1>(g, zseg);
    case 2: return m3_work_items<R, 2>(g, zseg);
    case 3: return m3_work_items<R, 3>(g, zseg);
    case 4: return m3_work_items<R, 4>(g, zseg);
    case 5: return m3_work_items<R, 5>(g, zseg);
    default: return -1;
    }
}

template <typename R>
hipError_t launch_march3d(const Geom &g, const void *uin, void *uout, const void *b, double *res,
                          int zseg, hipStream_t st, int64_t *nwork_out, int nt, int depth) {
    switch (depth) {
    case 1: return m3_launch<R, 1>(g, uin, uout, b, res, zseg, st, nwork_out, nt);
    case 2: return m3_launch<R, 2>(g, uin, uout, b, res, zseg, st, nwork_out, nt);
    case 3: return m3_launch<R, 3>(g, uin, uout, b, res, zseg, st, nwork_out, nt);
    case 4: return m3_launch<R, 4>(g, uin, uout, b, res, zseg, st, nwork_out, nt);
    case 5: return m3_launch<R, 5>(g, uin, uout, b, res, zseg, st, nwork_out, nt);
    default: return hipErrorInvalidValue;
    }
}

template int64_t march3d_batch_items<float>(const Geom &, int, int);
template int64_t march3d_batch_items<double>(const Geom &, int, int);
template hipError_t launch_march3d_batch<float>(const BatchGrid *, const int *, int, bool, int, int,
                                                int, hipStream_t);
template hipError_t launch_march3d_batch<double>(const BatchGrid *, const int *, int, bool, int,
                                                 int, int, hipStream_t);
template int64_t march3d_work_items<float>(const Geom &, int, int);
template int64_t march3d_work_items<double>(const Geom &, int, int);
template hipError_t launch_march3d<float>(const Geom &, const void *, void *, const void *,
                                          double *, int, hipStream_t, int64_t *, int, int);
template hipError_t launch_march3d<double>(const Geom &, const void *, void *, const void *,
                                           double *, int, hipStream_t, int64_t *, int, int);

}  // namespace jac
