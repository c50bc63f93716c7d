// Fused 2D Jacobi pass kernel for gfx950: T sweeps per pass (temporal
// blocking), halo cells read straight from the neighbouring blocks, and the
// FP64 residual of the pass's input state folded into the first level.
//
// The update is the 5-point Jacobi step of the proxy application in Section
// 4.3 of the paper, evaluated as s = (W + E) + (S + N); u' = (s + b) * 1/4
// with no FMA contraction, so every schedule gives the same bits.
//
// Work decomposition.  A wave owns a strip of 64 lanes x V elements
// (16 bytes per lane) along x and marches down a segment of rows.  Each row
// of the state and the source is loaded once, with one 16-byte load per
// lane, from whichever block owns it -- the exchange of halo cells between
// blocks happens inside these loads -- and pushed through T levels held in
// registers: at the step that loads row r, level s computes row r - s from
// the three newest rows of level s - 1.  West/east neighbours come from the
// adjacent lanes through DPP wave shifts; the two cells just outside the
// strip arrive by one scalar load per row.  Level T is the pass's output.
// A strip recomputes T - 1 columns on each side and a segment T rows on each
// side; only the strip's output lanes [L0, L1) and the segment's own rows
// are stored.  Rows are loaded one step ahead of use, straight into their
// ring slot, so no register copies are needed.
//
// Strips that touch the Dirichlet ring (first/last strip) run a second copy
// of the body with per-element masks; every other strip is branch-free.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

// Pass modes: Laplace (no source), Poisson (source b), and the adjoint pass,
// which sweeps a zero-ring Laplace state and adds w * (every level it holds)
// into an FP64 accumulator.
enum { MODE_LAPLACE = 0, MODE_POISSON = 1, MODE_ADJOINT = 2 };

template <typename R, int T>
struct M2 {
    static constexpr int V = 16 / (int)sizeof(R);            // elements per lane
    static constexpr int W = 64 * V;                          // strip width
    static constexpr int A0 = V * ((T - 1 + V - 1) / V);      // first output column in strip
    static constexpr int OW = V * ((W - (T - 1) - A0) / V);   // output columns per strip
    static constexpr int L0 = A0 / V;                         // first output lane
    static constexpr int L1 = (A0 + OW) / V;                  // one past the last output lane
    static constexpr int U = 12;                              // steps per unrolled group
    static constexpr int RB = T + 2;                          // source rows r-T .. r+1 (LDS)
    static constexpr int NL = T > 1 ? T - 1 : 1;              // stored levels 1..T-1
    // adjoint accumulator rows r-T+1 .. r+1
    static constexpr int RA = T + 1 <= 2 ? 2 : T + 1 <= 3 ? 3 : T + 1 <= 4 ? 4 : T + 1 <= 6 ? 6 : 12;
};

// Row cursor: global row y, its block row / local row, and the element
// offsets of that row's start in the state and source buffers (all uniform).
struct Cur {
    int y, by, ly;
    int64_t su, sb;
    __device__ __forceinline__ void set(const Geom &g) {
        su = (int64_t)by * g.nb[0] * g.bstride + (int64_t)(ly + 1) * g.pitch;
        sb = (int64_t)by * g.nb[0] * g.sstride + (int64_t)ly * g.e[0];
    }
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
        set(g);
    }
    __device__ __forceinline__ void advance(const Geom &g) {
        ++y;
        ++ly;
        if (ly >= g.e[1] && by < g.nb[1] - 1) {
            ++by;
            ly = 0;
            set(g);
        } else {
            su += g.pitch;
            sb += g.e[0];
        }
    }
};

template <typename R, int T>
struct MRegs {
    using S = M2<R, T>;
    R l0[4][S::V];           // level-0 rows, slot = row mod 4 (r-2 .. r+1)
    R e0[4];                 // level-0 cell just outside the strip (lanes 0, 63)
    R lv[S::NL][3][S::V];    // levels 1..T-1, slot = step mod 3
    double ga[S::RA][S::V];  // adjoint: FP64 accumulator rows r-T+1 .. r+1
    double acc;              // residual partial sum (level 1)
};

struct MLane {
    uint32_t lane_b, edge_b, src_b;  // byte offsets of the lane's chunk / edge / source
    bool ld, ldb, lde;
    bool upd[8];                     // per-element: interior column (ring strips)
    bool st[8];                      // per-element: interior output column (ring strips)
    bool out_lane;                   // lane holds output columns
    bool nt;                         // non-temporal output stores
    int c;                           // global column of the lane's first element
    void *bs;                        // this lane's slot 0 of the wave's LDS source ring
    int oy0, oy1, r1;
};

// Issue the loads of row lc.y into level-0 slot SL, source slot SB and (adjoint
// pass) accumulator slot SA, then advance the cursor.
template <typename R, int T, int MODE, bool RINGX, int SL, int SA>
__device__ __forceinline__ void m2_load(const Geom &g, const R *__restrict__ uin,
                                        const R *__restrict__ bsrc,
                                        const double *__restrict__ gacc, const MLane &L,
                                        MRegs<R, T> &m, Cur &lc, const int bslot) {
    constexpr int V = M2<R, T>::V;
    constexpr bool SRC = MODE == MODE_POISSON;
    using C = Chunk<R, V>;
    const int y = lc.y, ny = g.n[1];
    if constexpr (MODE == MODE_ADJOINT) {
        // the row's accumulator starts from what earlier passes summed
        const int nx = g.n[0];
        const bool row_in = y >= 0 && y < ny;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool in = row_in && L.c + v >= 0 && L.c + v < nx;
            m.ga[SA][v] = in ? gacc[(int64_t)y * nx + (L.c + v)] : 0.0;
        }
    }
    if (y >= -1 && y <= ny) {
        const R *row = uin + lc.su;
        if (!RINGX || L.ld) {
            const C c = at<C>(row, L.lane_b);
#pragma unroll
            for (int v = 0; v < V; ++v) m.l0[SL][v] = c.v[v];
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) m.l0[SL][v] = (R)0;
        }
        m.e0[SL] = (!RINGX || L.lde) ? at<R>(row, L.edge_b) : (R)0;
        if constexpr (SRC) {
            C c;
            if (y >= 0 && y < ny && (!RINGX || L.ldb)) {
                c = at<C>(bsrc + lc.sb, L.src_b);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) c.v[v] = (R)0;
            }
            static_cast<C *>(L.bs)[bslot * 64] = c;
        }
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) m.l0[SL][v] = (R)0;
        m.e0[SL] = (R)0;
    }
    lc.advance(g);
}

// Adjoint pass: add w * (level values of row y) into the row's accumulator,
// in the order of decreasing sweep index; store the accumulator when its last
// level (T - 1) has been added.
template <typename R, int T, int MODE, bool RINGX, int SA, bool LAST>
__device__ __forceinline__ void m2_accumulate(const Geom &g, double *__restrict__ gacc,
                                              const MLane &L, MRegs<R, T> &m, const int y,
                                              const R (&val)[M2<R, T>::V]) {
    constexpr int V = M2<R, T>::V;
    if constexpr (MODE == MODE_ADJOINT) {
        if (y >= 0 && y < g.n[1]) {
            const R w = (R)0.25;
#pragma unroll
            for (int v = 0; v < V; ++v) m.ga[SA][v] += (double)(w * val[v]);
            if (LAST && y >= L.oy0 && y < L.oy1) {
                double *row = gacc + (int64_t)y * g.n[0] + L.c;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const bool mine = RINGX ? L.st[v] : L.out_lane;
                    if (mine) row[v] = m.ga[SA][v];
                }
            }
        }
    }
}

// Level S of step J (row r = base + J): computes row r - S from the three
// newest rows of level S - 1 (level 0 = the loaded rows).  All ring slots are
// compile-time constants so the rings live in registers.
template <typename R, int T, int MODE, bool RINGX, int J, int S>
__device__ __forceinline__ void m2_level(const Geom &g, R *__restrict__ uout,
                                         double *__restrict__ gacc, const bool res,
                                         const MLane &L, MRegs<R, T> &m, const int r,
                                         const Cur &sc, const int sr) {
    using M = M2<R, T>;
    constexpr int V = M::V;
    constexpr bool SRC = MODE == MODE_POISSON;
    if constexpr (S <= T) {
        const int y = r - S;
        const int ny = g.n[1];
        // value copies (register renames): pointers into the rings would
        // keep them out of registers
        R up[V], cen[V], dn[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if constexpr (S == 1) {
                up[v] = m.l0[(J + 2) % 4][v];   // row r-2
                cen[v] = m.l0[(J + 3) % 4][v];  // row r-1
                dn[v] = m.l0[J % 4][v];         // row r
            } else {
                up[v] = m.lv[S - 2][(J + 1) % 3][v];
                cen[v] = m.lv[S - 2][(J + 2) % 3][v];
                dn[v] = m.lv[S - 2][J % 3][v];
            }
        }
        R bv[V];  // source row r - S from the wave's LDS ring
        if constexpr (SRC) {
            const int slot = sr - S < 0 ? sr - S + M::RB : sr - S;
            const Chunk<R, V> c = static_cast<const Chunk<R, V> *>(L.bs)[slot * 64];
#pragma unroll
            for (int v = 0; v < V; ++v) bv[v] = c.v[v];
        }
        R out[V];
        if (y >= 0 && y < ny) {
            R eo = (R)0;
            if constexpr (S == 1) eo = m.e0[(J + 3) % 4];
            const R left = shift_up(eo, cen[V - 1]);
            const R right = shift_down(eo, cen[0]);
            const R w = (R)0.25;
            const bool acc_row = (S == 1) && res && y >= L.oy0 && y < L.oy1;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const R Wv = v > 0 ? cen[v - 1] : left;
                const R Ev = v < V - 1 ? cen[v + 1] : right;
                const R sum = (Wv + Ev) + (up[v] + dn[v]);
                R o;
                if constexpr (SRC)
                    o = (sum + bv[v]) * w;
                else
                    o = sum * w;
                if constexpr (S == 1) {
                    if (acc_row) {
                        // residual of the input state, FP64 from widened values
                        const double sd =
                            ((double)Wv + (double)Ev) + ((double)up[v] + (double)dn[v]);
                        const double bd = SRC ? (double)bv[v] : 0.0;
                        const double rr = bd - (4.0 * (double)cen[v] - sd);
                        const bool mine = RINGX ? L.st[v] : L.out_lane;
                        m.acc += mine ? rr * rr : 0.0;
                    }
                }
                // ring cells (and cells beyond the ring) keep their values
                if constexpr (RINGX) o = L.upd[v] ? o : cen[v];
                out[v] = o;
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) out[v] = cen[v];
        }
        if constexpr (S < T) {
#pragma unroll
            for (int v = 0; v < V; ++v) m.lv[S - 1][J % 3][v] = out[v];
            m2_accumulate<R, T, MODE, RINGX, (J - S + 2 * M::RA) % M::RA, S == T - 1>(g, gacc, L,
                                                                                     m, y, out);
        } else {
            if (uout && y >= L.oy0 && y < L.oy1) {
                R *row = uout + sc.su;
                if constexpr (!RINGX) {
                    if (L.out_lane) {
                        Chunk<R, V> o;
#pragma unroll
                        for (int v = 0; v < V; ++v) o.v[v] = out[v];
                        if (L.nt)
                            store_nt16(&at_mut<Chunk<R, V>>(row, L.lane_b), o);
                        else
                            at_mut<Chunk<R, V>>(row, L.lane_b) = o;
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        if (L.st[v]) at_mut<R>(row, L.lane_b + v * (uint32_t)sizeof(R)) = out[v];
                }
            }
        }
        m2_level<R, T, MODE, RINGX, J, S + 1>(g, uout, gacc, res, L, m, r, sc, sr);
    }
}

template <typename R, int T, int MODE, bool RINGX, int J>
__device__ __forceinline__ void m2_steps(const Geom &g, const R *__restrict__ uin,
                                         R *__restrict__ uout, const R *__restrict__ bsrc,
                                         double *__restrict__ gacc, const bool res,
                                         const MLane &L, MRegs<R, T> &m, const int base, Cur &lc,
                                         Cur &sc, int &sr) {
    using M = M2<R, T>;
    constexpr int V = M::V;
    if constexpr (J < M::U) {
        const int r = base + J;
        if (r > L.r1) return;
        // row r+1 goes into the slots rows r-3 (state), r+1-RB (source) and
        // r+1-RA (accumulator) held
        const int sr1 = sr + 1 == M::RB ? 0 : sr + 1;  // LDS source slot of row r+1
        if (r + 1 <= L.r1)
            m2_load<R, T, MODE, RINGX, (J + 1) % 4, (J + 1) % M::RA>(g, uin, bsrc, gacc, L, m, lc,
                                                                     sr1);
        if constexpr (MODE == MODE_ADJOINT) {
            // level 0 of row r (the pass's input) is the first term added
            R v0[V];
#pragma unroll
            for (int v = 0; v < V; ++v) v0[v] = m.l0[J % 4][v];
            m2_accumulate<R, T, MODE, RINGX, J % M::RA, T == 1>(g, gacc, L, m, r, v0);
        }
        m2_level<R, T, MODE, RINGX, J, 1>(g, uout, gacc, res, L, m, r, sc, sr);
        sc.advance(g);
        sr = sr1;
        m2_steps<R, T, MODE, RINGX, J + 1>(g, uin, uout, bsrc, gacc, res, L, m, base, lc, sc, sr);
    }
}

template <typename R, int T, int MODE, bool RINGX>
__device__ __forceinline__ void m2_body(const Geom &g, const R *__restrict__ uin,
                                        R *__restrict__ uout, const R *__restrict__ bsrc,
                                        double *__restrict__ res_slot,
                                        double *__restrict__ gacc, const MLane &L, int r0) {
    using S = M2<R, T>;
    MRegs<R, T> m;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        m.e0[k] = (R)0;
#pragma unroll
        for (int v = 0; v < S::V; ++v) m.l0[k][v] = (R)0;
    }
#pragma unroll
    for (int s = 0; s < S::NL; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < S::V; ++v) m.lv[s][k][v] = (R)0;
#pragma unroll
    for (int k = 0; k < S::RA; ++k)
#pragma unroll
        for (int v = 0; v < S::V; ++v) m.ga[k][v] = 0.0;
    m.acc = 0.0;
    Cur lc, sc;
    lc.init(g, r0);
    sc.init(g, r0 - T);
    m2_load<R, T, MODE, RINGX, 0, 0>(g, uin, bsrc, gacc, L, m, lc, 0);  // row r0 -> slot 0
    const bool want_res = res_slot != nullptr;
    int sr = 0;  // LDS source slot of the current row
    for (int base = r0; base <= L.r1; base += S::U)
        m2_steps<R, T, MODE, RINGX, 0>(g, uin, uout, bsrc, gacc, want_res, L, m, base, lc, sc, sr);
    if (want_res) {
        const double a = wave_sum(m.acc);
        if ((threadIdx.x & 63) == 0) *res_slot = a;
    }
}

// One work item (wave): strip/tile number `wid` of a grid with `nseg` tiles
// per strip.  wid is wave-uniform.  res_slot: where the wave's residual
// partial goes (NULL: none).  bs_wave: the wave's LDS source ring.
template <typename R, int T, int MODE>
__device__ __forceinline__ void m2_run(const Geom &g, const R *__restrict__ uin,
                                       R *__restrict__ uout, const R *__restrict__ bsrc,
                                       double *__restrict__ res_slot, double *__restrict__ gacc,
                                       int wid, int nseg, int rows, Chunk<R, M2<R, T>::V> *bs_wave,
                                       bool nt) {
    using S = M2<R, T>;
    constexpr bool SRC = MODE == MODE_POISSON;
    constexpr int V = S::V;
    const int lane = threadIdx.x & 63;
    const int strip = wid / nseg, seg = wid % nseg;
    const int nx = g.n[0], ny = g.n[1];
    const int a = strip * S::OW - S::A0;  // first column held by the strip
    MLane L;
    L.bs = SRC ? (void *)(bs_wave + lane) : nullptr;
    L.oy0 = seg * rows;
    L.oy1 = L.oy0 + rows < ny ? L.oy0 + rows : ny;
    L.r1 = L.oy1 - 1 + T;
    const int c = a + lane * V;
    L.c = c;
    L.ld = c >= -V && c <= nx;
    {
        int bx, lx;
        owner(L.ld ? c : 0, g.e[0], g.nb[0], bx, lx);
        L.lane_b = (uint32_t)(((int64_t)bx * g.bstride + g.ax + lx) * (int64_t)sizeof(R));
        L.ldb = SRC && c >= 0 && c < nx;
        L.src_b = (uint32_t)(((int64_t)bx * g.sstride + (L.ldb ? lx : 0)) * (int64_t)sizeof(R));
    }
    {
        // lanes 0 and 63 fetch the cells just outside the strip; the others
        // re-read their own first cell (a harmless in-bounds load)
        const int xe = lane == 0 ? a - 1 : lane == 63 ? a + S::W : c;
        L.lde = xe >= -1 && xe <= nx && (lane == 0 || lane == 63 || L.ld);
        int bx, lx;
        owner(L.lde ? xe : 0, g.e[0], g.nb[0], bx, lx);
        L.edge_b = (uint32_t)(((int64_t)bx * g.bstride + g.ax + lx) * (int64_t)sizeof(R));
    }
    L.out_lane = lane >= S::L0 && lane < S::L1;
    L.nt = nt;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int x = c + v;
        L.upd[v] = x >= 0 && x < nx;
        L.st[v] = v < V && L.upd[v] && L.out_lane;
    }
    const bool ringx = a < 0 || a + S::W > nx;
    const int r0 = L.oy0 - T;
    if (ringx)
        m2_body<R, T, MODE, true>(g, uin, uout, bsrc, res_slot, gacc, L, r0);
    else
        m2_body<R, T, MODE, false>(g, uin, uout, bsrc, res_slot, gacc, L, r0);
}

// uout may be NULL (no stores: residual only); res may be NULL (no residual);
// gacc is the FP64 accumulator of the adjoint pass (MODE_ADJOINT only).
template <typename R, int T, int MODE>
__global__ __launch_bounds__(256) void k_march2d(Geom g, const R *__restrict__ uin,
                                                 R *__restrict__ uout,
                                                 const R *__restrict__ bsrc,
                                                 double *__restrict__ res,
                                                 double *__restrict__ gacc, int nseg, int rows,
                                                 int nwork, int nt) {
    using S = M2<R, T>;
    constexpr bool SRC = MODE == MODE_POISSON;
    // per wave: a ring of RB source rows, one 16-byte chunk per lane each
    __shared__ Chunk<R, S::V> bsm[SRC ? 4 * S::RB * 64 : 1];
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int wid = __builtin_amdgcn_readfirstlane(lb * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wid >= nwork) return;
    m2_run<R, T, MODE>(g, uin, uout, bsrc, res ? res + wid : nullptr, gacc, wid, nseg, rows,
                       &bsm[SRC ? (threadIdx.x >> 6) * S::RB * 64 : 0], nt != 0);
}

// Batched pass: the work items of all grids of a batch in one launch.  Work
// item w belongs to grid gi with prefix[gi] <= w < prefix[gi+1]; inactive
// grids (stopped by the convergence test) skip their items.  All active
// grids advance together, so the input buffer is u[pass_count & 1].
template <typename R, int T>
__global__ __launch_bounds__(256) void k_march2d_batch(const BatchGrid *__restrict__ grids,
                                                       const int *__restrict__ prefix, int ngrids,
                                                       const int *__restrict__ active,
                                                       const int *__restrict__ pass_count,
                                                       double *__restrict__ res, int store,
                                                       int rows, int nwork) {
    using S = M2<R, T>;
    __shared__ Chunk<R, S::V> bsm[4 * S::RB * 64];
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int wid = __builtin_amdgcn_readfirstlane(lb * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wid >= nwork) return;
    int lo = 0, hi = ngrids;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= wid) lo = mid; else hi = mid;
    }
    const int gi = __builtin_amdgcn_readfirstlane(lo);
    if (!active[gi]) return;
    const Geom g = grids[gi].g;
    const int par = *pass_count & 1;
    const R *uin = (const R *)grids[gi].u[par];
    R *uout = store ? (R *)grids[gi].u[par ^ 1] : nullptr;
    m2_run<R, T, MODE_POISSON>(g, uin, uout, (const R *)grids[gi].b, res ? res + wid : nullptr,
                               nullptr, wid - prefix[gi], grids[gi].nseg, rows,
                               &bsm[(threadIdx.x >> 6) * S::RB * 64], false);
}

template <typename R, int T>
static int64_t m2_nwork(const Geom &g, int rows, int *nseg_out) {
    using S = M2<R, T>;
    const int64_t nstrips = (g.n[0] + S::OW - 1) / S::OW;
    const int64_t nseg = (g.n[1] + rows - 1) / rows;
    if (nseg_out) *nseg_out = (int)nseg;
    return nstrips * nseg;
}

template <typename R, int T>
static hipError_t m2_launch_t(const Geom &g, const void *uin, void *uout, const void *b,
                              double *res, double *gacc, int rows, hipStream_t st,
                              int64_t *nwork_out, int nt) {
    int nseg = 0;
    const int64_t nwork = m2_nwork<R, T>(g, rows, &nseg);
    if (nwork_out) *nwork_out = nwork;
    if (nwork > 0x7fffffff) return hipErrorInvalidValue;
    const int grid = (int)((nwork + 3) / 4);
    if (gacc)
        hipLaunchKernelGGL((k_march2d<R, T, MODE_ADJOINT>), dim3(grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)nullptr, (double *)nullptr,
                           gacc, nseg, rows, (int)nwork, nt);
    else if (b)
        hipLaunchKernelGGL((k_march2d<R, T, MODE_POISSON>), dim3(grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)b, res, (double *)nullptr, nseg,
                           rows, (int)nwork, nt);
    else
        hipLaunchKernelGGL((k_march2d<R, T, MODE_LAPLACE>), dim3(grid), dim3(256), 0, st, g,
                           (const R *)uin, (R *)uout, (const R *)nullptr, res, (double *)nullptr,
                           nseg, rows, (int)nwork, nt);
    return hipGetLastError();
}

static const int kDepthsF32[] = {1, 2, 3, 4, 5, 6, 7, 8};
static const int kDepthsF64[] = {1, 2, 3, 4};

int march2d_depths(int dtype, const int **list) {
    if (dtype == 0) {
        *list = kDepthsF32;
        return (int)(sizeof(kDepthsF32) / sizeof(int));
    }
    *list = kDepthsF64;
    return (int)(sizeof(kDepthsF64) / sizeof(int));
}

template <typename R>
int64_t march2d_work_items(const Geom &g, int depth, int rows);

template <typename R, int T>
static int m2_waves_per_cu_t(int mode) {
    int blocks = 0;
    hipError_t e;
    if (mode == MODE_ADJOINT)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_march2d<R, T, MODE_ADJOINT>, 256, 0);
    else if (mode == MODE_POISSON)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_march2d<R, T, MODE_POISSON>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_march2d<R, T, MODE_LAPLACE>, 256, 0);
    return e == hipSuccess ? blocks * 4 : 0;
}

template <typename R>
int march2d_waves_per_cu(int depth, int mode) {
    switch (depth) {
    case 1: return m2_waves_per_cu_t<R, 1>(mode);
    case 2: return m2_waves_per_cu_t<R, 2>(mode);
    case 3: return m2_waves_per_cu_t<R, 3>(mode);
    case 4: return m2_waves_per_cu_t<R, 4>(mode);
    case 5: return m2_waves_per_cu_t<R, 5>(mode);
    case 6: return m2_waves_per_cu_t<R, 6>(mode);
    case 7: return m2_waves_per_cu_t<R, 7>(mode);
    case 8: return m2_waves_per_cu_t<R, 8>(mode);
    default: return 0;
    }
}

template <typename R>
int64_t march2d_strips(const Geom &g, int depth) {
    const int64_t nw = march2d_work_items<R>(g, depth, g.n[1]);  // one tile per strip
    return nw;
}

template <typename R>
int64_t march2d_work_items(const Geom &g, int depth, int rows) {
    switch (depth) {
    case 1: return m2_nwork<R, 1>(g, rows, nullptr);
    case 2: return m2_nwork<R, 2>(g, rows, nullptr);
    case 3: return m2_nwork<R, 3>(g, rows, nullptr);
    case 4: return m2_nwork<R, 4>(g, rows, nullptr);
    case 5: return m2_nwork<R, 5>(g, rows, nullptr);
    case 6: return m2_nwork<R, 6>(g, rows, nullptr);
    case 7: return m2_nwork<R, 7>(g, rows, nullptr);
    case 8: return m2_nwork<R, 8>(g, rows, nullptr);
    default: return -1;
    }
}

template <>
hipError_t launch_sweep2d_march<float>(const Geom &g, const void *uin, void *uout, const void *b,
                                       double *res, double *gacc, int depth, int rows,
                                       hipStream_t st, int64_t *nwork, int nt) {
    switch (depth) {
    case 1: return m2_launch_t<float, 1>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 2: return m2_launch_t<float, 2>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 3: return m2_launch_t<float, 3>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 4: return m2_launch_t<float, 4>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 5: return m2_launch_t<float, 5>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 6: return m2_launch_t<float, 6>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 7: return m2_launch_t<float, 7>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 8: return m2_launch_t<float, 8>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t launch_sweep2d_march<double>(const Geom &g, const void *uin, void *uout, const void *b,
                                        double *res, double *gacc, int depth, int rows,
                                        hipStream_t st, int64_t *nwork, int nt) {
    switch (depth) {
    case 1: return m2_launch_t<double, 1>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 2: return m2_launch_t<double, 2>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 3: return m2_launch_t<double, 3>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    case 4: return m2_launch_t<double, 4>(g, uin, uout, b, res, gacc, rows, st, nwork, nt);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
int64_t march2d_batch_work(const Geom &g, int depth, int rows, int *nseg) {
    switch (depth) {
    case 1: return m2_nwork<R, 1>(g, rows, nseg);
    case 2: return m2_nwork<R, 2>(g, rows, nseg);
    case 3: return m2_nwork<R, 3>(g, rows, nseg);
    case 4: return m2_nwork<R, 4>(g, rows, nseg);
    case 5: return m2_nwork<R, 5>(g, rows, nseg);
    case 6: return m2_nwork<R, 6>(g, rows, nseg);
    case 7: return m2_nwork<R, 7>(g, rows, nseg);
    case 8: return m2_nwork<R, 8>(g, rows, nseg);
    default: return -1;
    }
}

template <typename R, int T>
static hipError_t m2b_launch_t(const BatchGrid *grids, const int *prefix, int ngrids,
                               const int *active, const int *pass_count, double *res, bool store,
                               int rows, int nwork, hipStream_t st) {
    const int grid = (nwork + 3) / 4;
    hipLaunchKernelGGL((k_march2d_batch<R, T>), dim3(grid), dim3(256), 0, st, grids, prefix,
                       ngrids, active, pass_count, res, store ? 1 : 0, rows, nwork);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_march2d_batch(const BatchGrid *grids, const int *prefix, int ngrids,
                                const int *active, const int *pass_count, double *res, bool store,
                                int depth, int rows, int nwork, hipStream_t st) {
    if (nwork <= 0) return hipSuccess;
    switch (depth) {
    case 1: return m2b_launch_t<R, 1>(grids, prefix, ngrids, active, pass_count, res, store, rows, nwork, st);
    case 2: return m2b_launch_t<R, 2>(grids, prefix, ngrids, active, pass_count, res, store, rows, nwork, st);
    case 3: return m2b_launch_t<R, 3>(grids, prefix, ngrids, active, pass_count, res, store, rows, nwork, st);
    case 4: return m2b_launch_t<R, 4>(grids, prefix, ngrids, active, pass_count, res, store, rows, nwork, st);
    case 5: return m2b_launch_t<R, 5>(grids, prefix, ngrids, active, pass_count, res, store, rows, nwork, st);
    case 6: return m2b_launch_t<R, 6>(grids, prefix, ngrids, active, pass_count, res, store, rows, nwork, st);
    case 7: return m2b_launch_t<R, 7>(grids, prefix, ngrids, active, pass_count, res, store, rows, nwork, st);
    case 8: return m2b_launch_t<R, 8>(grids, prefix, ngrids, active, pass_count, res, store, rows, nwork, st);
    default: return hipErrorInvalidValue;
    }
}

template int64_t march2d_batch_work<float>(const Geom &, int, int, int *);
template int64_t march2d_batch_work<double>(const Geom &, int, int, int *);
template hipError_t launch_march2d_batch<float>(const BatchGrid *, const int *, int, const int *,
                                                const int *, double *, bool, int, int, int,
                                                hipStream_t);
template hipError_t launch_march2d_batch<double>(const BatchGrid *, const int *, int, const int *,
                                                 const int *, double *, bool, int, int, int,
                                                 hipStream_t);
template int64_t march2d_work_items<float>(const Geom &, int, int);
template int64_t march2d_work_items<double>(const Geom &, int, int);
template int march2d_waves_per_cu<float>(int, int);
template int march2d_waves_per_cu<double>(int, int);
template int64_t march2d_strips<float>(const Geom &, int);
template int64_t march2d_strips<double>(const Geom &, int);

}  // namespace jac
