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
// Two kernel families:
//  * k_sweep_local   -- one sweep of every block from its own storage (its
//    interior plus the one-cell halo a preceding halo exchange filled), the
//    step order of the paper's proxy: exchange, then update.
//  * k_sweep2d_march -- the fused form used for speed.  A wave owns a strip
//    of 64 lanes x V elements (16 bytes per lane) along x and walks down a
//    segment of rows.  Every row is loaded once with one 16-byte load per
//    lane, from whichever block owns it (so the halo exchange happens inside
//    the loads), and pushed through T pipelined levels held in registers:
//    level s computes row r-s from the three newest rows of level s-1.  West
//    and east neighbours come from the adjacent lanes by DPP wave shifts; the
//    two cells just outside the strip come from two scalar loads at level 0.
//    Each pass therefore performs T sweeps while reading the state and the
//    source once and writing the state once (temporal blocking), at the price
//    of recomputing 2(T-1) columns per strip and 2T rows per segment.
#include <hip/hip_runtime.h>

#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

template <typename R, int V>
struct alignas(16) Chunk {
    R v[V];
};

// lane i receives src of lane i-1; lane 0 keeps `old`
__device__ __forceinline__ float shift_up(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}
// lane i receives src of lane i+1; lane 63 keeps `old`
__device__ __forceinline__ float shift_down(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}
__device__ __forceinline__ double shift_up(double old, double src) {
    const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double shift_down(double old, double src) {
    const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

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

// ------------------------------------------------------------ 2D march
template <typename R, int T>
struct MarchShape {
    static constexpr int V = 16 / (int)sizeof(R);          // elements per lane
    static constexpr int W = 64 * V;                        // strip width
    static constexpr int A0 = V * ((T - 1 + V - 1) / V);    // strip origin shift
    static constexpr int OW = V * ((W - 2 * (T - 1)) / V);  // output columns per strip
    static constexpr int RB = 3 * ((T + 3) / 3);            // source ring (mult. of 3, > T)
    static constexpr int U = RB;                            // rows per unrolled group
};

// Row cursor: block row `by` and local row `ly` of global row y, and the
// uniform parts of the state / source offsets of that row.
struct RowCursor {
    int y, by, ly;
    __device__ __forceinline__ void init(const Geom &g, int y0) {
        y = y0;
        if (y0 < 0) {
            by = 0;
            ly = y0;
        } else {
            by = y0 / g.e[1];
            if (by > g.nb[1] - 1) by = g.nb[1] - 1;
            ly = y0 - by * g.e[1];
        }
    }
    __device__ __forceinline__ void advance(const Geom &g) {
        ++y;
        ++ly;
        if (ly >= g.e[1] && by < g.nb[1] - 1) {
            ++by;
            ly = 0;
        }
    }
    __device__ __forceinline__ int64_t state_row(const Geom &g) const {
        return (int64_t)by * g.nb[0] * g.bstride + (int64_t)(ly + 1) * g.pitch;
    }
    __device__ __forceinline__ int64_t source_row(const Geom &g) const {
        return (int64_t)by * g.nb[0] * g.sstride + (int64_t)ly * g.e[0];
    }
};

template <typename R, int T>
struct MarchRegs {
    using S = MarchShape<R, T>;
    R lv[T][3][S::V];   // level s rows, ring of 3 (level 0 = loaded rows)
    R edge[3];          // level-0 cells just outside the strip (lanes 0 and 63)
    R bq[S::RB][S::V];  // source rows, ring
};

struct MarchLane {
    int64_t lane_off, lane_boff, edge_off;
    bool ld, ldb, lde, st_all;
    bool upd[8], st[8];
    int ox0, ox1, oy0, oy1, r1;
};

template <typename R, int T, bool SRC, bool RINGX, int J>
__device__ __forceinline__ void march_steps(const Geom &g, const R *__restrict__ uin,
                                            R *__restrict__ uout, const R *__restrict__ bsrc,
                                            const MarchLane &L, MarchRegs<R, T> &m, int base,
                                            RowCursor &lc, RowCursor &sc) {
    using S = MarchShape<R, T>;
    constexpr int V = S::V;
    if constexpr (J < S::U) {
        const int r = base + J;
        if (r > L.r1) return;
        const int ny = g.n[1];
        // level 0: load row r
        {
            Chunk<R, V> nv;
#pragma unroll
            for (int v = 0; v < V; ++v) nv.v[v] = (R)0;
            R ne = (R)0;
            if (r >= -1 && r <= ny) {
                const int64_t ro = lc.state_row(g);
                if (L.ld) nv = *reinterpret_cast<const Chunk<R, V> *>(uin + ro + L.lane_off);
                if (L.lde) ne = uin[ro + L.edge_off];
                if (SRC && r >= 0 && r < ny && L.ldb) {
                    const Chunk<R, V> bv =
                        *reinterpret_cast<const Chunk<R, V> *>(bsrc + lc.source_row(g) + L.lane_boff);
#pragma unroll
                    for (int v = 0; v < V; ++v) m.bq[J % S::RB][v] = bv.v[v];
                }
            }
#pragma unroll
            for (int v = 0; v < V; ++v) m.lv[0][J % 3][v] = nv.v[v];
            m.edge[J % 3] = ne;
            lc.advance(g);
        }
        // levels 1..T: level s computes row r - s from level s-1 rows
        // r-s-1 (slot J-2), r-s (slot J-1), r-s+1 (slot J)
#pragma unroll
        for (int s = 1; s <= T; ++s) {
            const int y = r - s;
            const R *up = m.lv[s - 1][(J + 1) % 3];  // row y - 1 (south)
            const R *cen = m.lv[s - 1][(J + 2) % 3]; // row y
            const R *dn = m.lv[s - 1][J % 3];        // row y + 1 (north)
            R out[V];
            if (y >= 0 && y < ny) {
                const R eo = (s == 1) ? m.edge[(J + 2) % 3] : (R)0;
                const R left = shift_up(eo, cen[V - 1]);
                const R right = shift_down(eo, cen[0]);
                const R w = weight2d<R>();
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const R Wv = v > 0 ? cen[v - 1] : left;
                    const R Ev = v < V - 1 ? cen[v + 1] : right;
                    const R sum = (Wv + Ev) + (up[v] + dn[v]);
                    R o;
                    if constexpr (SRC)
                        o = (sum + m.bq[(J - s + S::RB) % S::RB][v]) * w;
                    else
                        o = sum * w;
                    if constexpr (RINGX) o = L.upd[v] ? o : cen[v];
                    out[v] = o;
                }
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) out[v] = cen[v];
            }
            if (s < T) {
#pragma unroll
                for (int v = 0; v < V; ++v) m.lv[s][J % 3][v] = out[v];
            } else if (y >= L.oy0 && y < L.oy1) {
                R *p = uout + sc.state_row(g) + L.lane_off;
                if (L.st_all) {
                    Chunk<R, V> o;
#pragma unroll
                    for (int v = 0; v < V; ++v) o.v[v] = out[v];
                    *reinterpret_cast<Chunk<R, V> *>(p) = o;
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        if (L.st[v]) p[v] = out[v];
                }
            }
        }
        sc.advance(g);
        march_steps<R, T, SRC, RINGX, J + 1>(g, uin, uout, bsrc, L, m, base, lc, sc);
    }
}

template <typename R, int T, bool SRC, bool RINGX>
__device__ __forceinline__ void march_body(const Geom &g, const R *__restrict__ uin,
                                           R *__restrict__ uout, const R *__restrict__ bsrc,
                                           const MarchLane &L, int r0) {
    using S = MarchShape<R, T>;
    MarchRegs<R, T> m;
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < S::V; ++v) m.lv[s][k][v] = (R)0;
#pragma unroll
    for (int k = 0; k < 3; ++k) m.edge[k] = (R)0;
#pragma unroll
    for (int k = 0; k < S::RB; ++k)
#pragma unroll
        for (int v = 0; v < S::V; ++v) m.bq[k][v] = (R)0;
    RowCursor lc, sc;
    lc.init(g, r0);
    sc.init(g, r0 - T);
    for (int base = r0; base <= L.r1; base += S::U)
        march_steps<R, T, SRC, RINGX, 0>(g, uin, uout, bsrc, L, m, base, lc, sc);
}

template <typename R, int T, bool SRC>
__global__ __launch_bounds__(256) void k_sweep2d_march(Geom g, const R *__restrict__ uin,
                                                       R *__restrict__ uout,
                                                       const R *__restrict__ bsrc, int nstrips,
                                                       int rows, int nwork) {
    using S = MarchShape<R, T>;
    constexpr int V = S::V;
    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wid >= nwork) return;
    const int strip = wid % nstrips, seg = wid / nstrips;
    const int nx = g.n[0], ny = g.n[1];
    const int a = strip * S::OW - S::A0;
    MarchLane L;
    L.ox0 = a + T - 1;
    L.ox1 = L.ox0 + S::OW;
    L.oy0 = seg * rows;
    L.oy1 = L.oy0 + rows < ny ? L.oy0 + rows : ny;
    L.r1 = L.oy1 - 1 + T;
    const int c = a + lane * V;
    L.ld = (c >= -V) && (c <= nx);
    {
        int bx, lx;
        owner(L.ld ? c : 0, g.e[0], g.nb[0], bx, lx);
        L.lane_off = (int64_t)bx * g.bstride + g.ax + lx;
        L.ldb = SRC && c >= 0 && c < nx;
        L.lane_boff = (int64_t)bx * g.sstride + lx;
    }
    {
        const int xe = lane == 0 ? a - 1 : a + S::W;
        L.lde = (lane == 0 || lane == 63) && xe >= -1 && xe <= nx;
        int bx, lx;
        owner(L.lde ? xe : 0, g.e[0], g.nb[0], bx, lx);
        L.edge_off = (int64_t)bx * g.bstride + g.ax + lx;
    }
    L.st_all = true;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int x = c + v;
        L.upd[v] = x >= 0 && x < nx;
        L.st[v] = v < V && L.upd[v] && x >= L.ox0 && x < L.ox1;
        if (v < V) L.st_all = L.st_all && L.st[v];
    }
    const bool ringx = (a < 0) || (a + S::W > nx);
    const int r0 = L.oy0 - T;
    if (ringx)
        march_body<R, T, SRC, true>(g, uin, uout, bsrc, L, r0);
    else
        march_body<R, T, SRC, false>(g, uin, uout, bsrc, L, r0);
}

template <typename R, int T>
static hipError_t launch_march_t(const Geom &g, const void *uin, void *uout, const void *b,
                                 int rows, hipStream_t st) {
    using S = MarchShape<R, T>;
    // strips: output columns start at T-1-A0 <= 0, OW per strip
    const int first = T - 1 - S::A0;
    const int nstrips = (g.n[0] - first + S::OW - 1) / S::OW;
    const int nseg = (g.n[1] + rows - 1) / rows;
    const int64_t nwork = (int64_t)nstrips * nseg;
    if (nwork > 0x7fffffff) return hipErrorInvalidValue;
    const int grid = (int)((nwork + 3) / 4);
    if (b)
        hipLaunchKernelGGL((k_sweep2d_march<R, T, true>), dim3(grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)b, nstrips, rows, (int)nwork);
    else
        hipLaunchKernelGGL((k_sweep2d_march<R, T, false>), dim3(grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)nullptr, nstrips, rows,
                           (int)nwork);
    return hipGetLastError();
}

static const int kDepthsF32[] = {1, 2, 3, 4, 5, 6, 8};
static const int kDepthsF64[] = {1, 2, 3, 4};

int march2d_depths(int dtype, const int **list) {
    if (dtype == 0) {
        *list = kDepthsF32;
        return (int)(sizeof(kDepthsF32) / sizeof(int));
    }
    *list = kDepthsF64;
    return (int)(sizeof(kDepthsF64) / sizeof(int));
}

template <>
hipError_t launch_sweep2d_march<float>(const Geom &g, const void *uin, void *uout, const void *b,
                                       int depth, int rows, hipStream_t st) {
    switch (depth) {
    case 1: return launch_march_t<float, 1>(g, uin, uout, b, rows, st);
    case 2: return launch_march_t<float, 2>(g, uin, uout, b, rows, st);
    case 3: return launch_march_t<float, 3>(g, uin, uout, b, rows, st);
    case 4: return launch_march_t<float, 4>(g, uin, uout, b, rows, st);
    case 5: return launch_march_t<float, 5>(g, uin, uout, b, rows, st);
    case 6: return launch_march_t<float, 6>(g, uin, uout, b, rows, st);
    case 8: return launch_march_t<float, 8>(g, uin, uout, b, rows, st);
    default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t launch_sweep2d_march<double>(const Geom &g, const void *uin, void *uout, const void *b,
                                        int depth, int rows, hipStream_t st) {
    switch (depth) {
    case 1: return launch_march_t<double, 1>(g, uin, uout, b, rows, st);
    case 2: return launch_march_t<double, 2>(g, uin, uout, b, rows, st);
    case 3: return launch_march_t<double, 3>(g, uin, uout, b, rows, st);
    case 4: return launch_march_t<double, 4>(g, uin, uout, b, rows, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_sweep_local<float>(const Geom &, const void *, void *, const void *,
                                              hipStream_t);
template hipError_t launch_sweep_local<double>(const Geom &, const void *, void *, const void *,
                                               hipStream_t);

}  // namespace jac
