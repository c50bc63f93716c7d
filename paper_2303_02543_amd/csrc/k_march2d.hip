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
// are stored.  Rows are loaded P steps ahead of use (P = 2 at most depths,
// see m2_pf), straight into their ring slot, so no register
// copies are needed.  A source row waits in
// registers for one step before it is written to the wave's LDS ring (it is
// first read one step after that), so the wait for its load overlaps a whole
// step of arithmetic instead of stalling the step that issued it.
//
// Every load is unconditional: a load issued on only some paths would turn
// the next step's wait for its data into a wait for every load in flight.
// Tiles that reach the Dirichlet ring or the rows beyond it run an edge copy
// of the body, which reads an in-bounds stand-in address where a row or
// column lies beyond the ring and keeps ring cells at their values at every
// level; what lies beyond the ring only ever feeds ring cells, so it is
// never cleared.  There are three copies: row and column tests (tiles of a
// strip that reaches the ring in x), row tests only (the other tiles that
// reach it in y), and none (interior tiles).
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

// Waves per workgroup of the pass kernels.  The waves of a workgroup share
// nothing (each has its own LDS ring); one wave per workgroup (a finished
// wave freeing its slot at once) measured the same as four on the 8192^2
// pass and the 64-grid batch.
constexpr int kM2Waves = 4;

// Pass modes: Laplace (no source), Poisson (source b), and the adjoint pass,
// which sweeps a zero-ring Laplace state and adds w * (every level it holds)
// into an FP64 accumulator.
enum { MODE_LAPLACE = 0, MODE_POISSON = 1, MODE_ADJOINT = 2 };

template <typename R, int T, int P>
struct M2 {
    static constexpr int V = 16 / (int)sizeof(R);            // elements per lane
    static constexpr int W = 64 * V;                          // strip width
    static constexpr int A0 = V * ((T - 1 + V - 1) / V);      // first output column in strip
    static constexpr int OW = V * ((W - (T - 1) - A0) / V);   // output columns per strip
    static constexpr int L0 = A0 / V;                         // first output lane
    static constexpr int L1 = (A0 + OW) / V;                  // one past the last output lane
    // rows loaded ahead (prefetch distance): row r + P is loaded at step r
    static_assert(P >= 1 && P <= 3, "prefetch distance 1..3");
    static constexpr int LR = P == 1 ? 4 : 6;                 // level-0 ring: rows r-2 .. r+P
    static constexpr int BQ = P == 1 ? 2 : P;                 // source registers: rows r .. r+P
    // BQ == P: the slot of row r is reused for row r + P, so row r goes to
    // LDS before that load is issued; otherwise after it
    static constexpr bool WRITE_FIRST = BQ == P;
    static constexpr int U = 12;                              // steps per unrolled group
    // ring slots are compile-time step indices mod 4, 3 and 2
    static_assert(U % LR == 0 && U % 3 == 0 && U % BQ == 0, "ring sizes must divide U");
    static constexpr int RB = T + 1;                          // source rows r-T .. r (LDS)
    static constexpr int NL = T > 1 ? T - 1 : 1;              // stored levels 1..T-1
    // adjoint accumulator rows r-T+1 .. r+1
    static constexpr int RA = T + 1 <= 2 ? 2 : T + 1 <= 3 ? 3 : T + 1 <= 4 ? 4 : T + 1 <= 6 ? 6 : 12;
};

// Tiling of a pass over an nx x ny grid.  Strips of OW output columns;
// the inner strips 1 .. ns-2 are cut into a band of hb rows at the top, one
// at the bottom, and tiles of `rows` rows between them; the outer strips 0
// and ns-1 into tiles of ho rows throughout.  A tile of h rows takes h + 2T
// steps.  Tiles that reach the Dirichlet ring run an edge copy of the step:
// the bands one with row tests (~1.2x the VALU instructions of the interior
// step), the outer strips one with row and column tests (~1.4x).  Their
// heights follow from (h + 2T) = (rows + 2T) * F / 16, with F = kBand16 for
// the bands and kOuter16 for the outer strips, so edge tiles take about as
// long as interior ones and a pass, whose tiles all run as one generation
// of waves, is not held up by its edges.  F was measured on MI355X (8192^2
// FP32, depth 13): 15/13 0.232 ms per pass, 14/12 0.225, 13/11 0.215,
// 12/10 0.215.
constexpr int kBand16 = 13, kOuter16 = 11;
struct M2Tiles {
    int ns, hb, ho, sa, sb, na, nb;  // strips, band / outer tile height, tiles per inner / outer strip, inner / outer strips
    int64_t ninner, nwork;           // tiles of the inner strips, all tiles
};
__host__ __device__ inline int m2_edge_rows(int rows, int T, int f16, int ny) {
    const int lo = rows < 8 ? rows : 8;
    int h = (rows + 2 * T) * f16 / 16 - 2 * T;
    h = h > lo ? h : lo;
    return h < ny ? h : ny;
}
__host__ __device__ inline M2Tiles m2_tiles(int nx, int ny, int ow, int rows, int T) {
    M2Tiles t;
    t.ns = (nx + ow - 1) / ow;
    t.hb = m2_edge_rows(rows, T, kBand16, ny);
    t.ho = m2_edge_rows(rows, T, kOuter16, ny);
    const int mid = ny - 2 * t.hb;
    t.sa = ny <= t.hb ? 1 : 2 + (mid > 0 ? (mid + rows - 1) / rows : 0);
    t.sb = (ny + t.ho - 1) / t.ho;
    t.na = t.ns > 2 ? t.ns - 2 : 0;
    t.nb = t.ns < 2 ? t.ns : 2;
    t.ninner = (int64_t)t.na * t.sa;
    t.nwork = t.ninner + (int64_t)t.nb * t.sb;
    return t;
}
// Strip and output rows [oy0, oy1) of tile w (0 <= w < nwork).  Adjacent
// tiles of the inner strips are adjacent strips of one row segment.
__host__ __device__ inline void m2_tile(const M2Tiles &t, int ny, int rows, int64_t w,
                                        int &strip, int &oy0, int &oy1) {
    if (w < t.ninner) {
        strip = 1 + (int)(w % t.na);
        const int seg = (int)(w / t.na);
        if (seg == 0) {
            oy0 = 0;
            oy1 = t.hb;
        } else if (seg == t.sa - 1) {
            oy0 = ny - t.hb > t.hb ? ny - t.hb : t.hb;
            oy1 = ny;
        } else {
            oy0 = t.hb + (seg - 1) * rows;
            oy1 = oy0 + rows < ny - t.hb ? oy0 + rows : ny - t.hb;
        }
    } else {
        const int64_t v = w - t.ninner;
        strip = t.nb == 2 && (v & 1) ? t.ns - 1 : 0;
        const int seg = (int)(t.nb == 2 ? v >> 1 : v);
        oy0 = seg * t.ho;
        oy1 = oy0 + t.ho < ny ? oy0 + t.ho : ny;
    }
}

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

template <typename R, int T, int P>
struct MRegs {
    using S = M2<R, T, P>;
    R l0[S::LR][S::V];       // level-0 rows, slot = row mod LR (r-2 .. r+P)
    R e0[S::LR];             // level-0 cell just outside the strip (lanes 0, 63)
    R bq[S::BQ][S::V];       // source rows in flight, slot = row mod BQ
    R bn[2][S::V];           // source rows read ahead from LDS, slot = level mod 2
    R lv[S::NL][3][S::V];    // levels 1..T-1, slot = step mod 3
    double ga[S::RA][S::V];  // adjoint: FP64 accumulator rows r-T+1 .. r+1
    double acc;              // residual partial sum (level 1)
};

struct MLane {
    uint32_t lane_b, edge_b, src_b;  // byte offsets of the lane's chunk / edge / source
    bool upd[8];                     // per element: interior column (column-edge tiles)
    bool st[8];                      // per element: interior output column (column-edge tiles)
    bool out_lane;                   // lane holds output columns
    bool st_all;                     // every column of the lane is an interior output
    bool st_part;                    // some but not all are (the east ring's lane)
    bool nt;                         // non-temporal output stores
    int c;                           // global column of the lane's first element
    void *bs;                        // this lane's slot 0 of the wave's LDS source ring
    int oy0, oy1, r1;
};

// Issue the loads of row lc.y into level-0 slot SL, source register slot SQ
// and (adjoint pass) accumulator slot SA, then advance the cursor.
template <typename R, int T, int P, int MODE, int EK, int SL, int SQ, int SA>
__device__ __forceinline__ void m2_load(const Geom &g, const R *__restrict__ uin,
                                        const R *__restrict__ bsrc,
                                        const double *__restrict__ gacc, const MLane &L,
                                        MRegs<R, T, P> &m, Cur &lc) {
    constexpr int V = M2<R, T, P>::V;
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
    // rows and columns beyond the ring are read from in-bounds stand-ins and
    // kept as they come: they only ever feed ring cells, which every level
    // keeps at their values
    const bool row_ok = !(EK & 1) || (y >= -1 && y <= ny);
    const R *row = uin + (row_ok ? lc.su : (int64_t)g.pitch);
    const C c = at<C>(row, L.lane_b);
#pragma unroll
    for (int v = 0; v < V; ++v) m.l0[SL][v] = c.v[v];
    m.e0[SL] = at<R>(row, L.edge_b);
    if constexpr (SRC) {
        const bool brow = !(EK & 1) || (y >= 0 && y < ny);
        const C cb = at<C>(bsrc + (brow ? lc.sb : (int64_t)0), L.src_b);
#pragma unroll
        for (int v = 0; v < V; ++v) m.bq[SQ][v] = cb.v[v];
    }
    lc.advance(g);
}

// Adjoint pass: add w * (level values of row y) into the row's accumulator,
// in the order of decreasing sweep index; store the accumulator when its last
// level (T - 1) has been added.
template <typename R, int T, int P, int MODE, int EK, int SA, bool LAST>
__device__ __forceinline__ void m2_accumulate(const Geom &g, double *__restrict__ gacc,
                                              const MLane &L, MRegs<R, T, P> &m, const int y,
                                              const R (&val)[M2<R, T, P>::V]) {
    constexpr int V = M2<R, T, P>::V;
    if constexpr (MODE == MODE_ADJOINT) {
        if (!(EK & 1) || (y >= 0 && y < g.n[1])) {
            const R w = (R)0.25;
#pragma unroll
            for (int v = 0; v < V; ++v) m.ga[SA][v] += (double)(w * val[v]);
            if (LAST && y >= L.oy0 && y < L.oy1) {
                double *row = gacc + (int64_t)y * g.n[0] + L.c;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const bool mine = (EK & 2) ? L.st[v] : L.out_lane;
                    if (mine) row[v] = m.ga[SA][v];
                }
            }
        }
    }
}

// Read the source row of level S from the wave's LDS ring into bn[S & 1]:
// the row K steps back (K = S: row r - S, for level S of this step; K = 0:
// row r, for level 1 of the next step).  Issued one level before its use, so
// the LDS latency overlaps the arithmetic of the level in between.
template <typename R, int T, int P, int S, int K = S>
__device__ __forceinline__ void m2_read_src(const MLane &L, MRegs<R, T, P> &m, const int sr) {
    using M = M2<R, T, P>;
    const int slot = sr - K < 0 ? sr - K + M::RB : sr - K;
    const Chunk<R, M::V> c = static_cast<const Chunk<R, M::V> *>(L.bs)[slot * 64];
#pragma unroll
    for (int v = 0; v < M::V; ++v) m.bn[S & 1][v] = c.v[v];
}

// Level S of step J (row r = base + J): computes row r - S from the three
// newest rows of level S - 1 (level 0 = the loaded rows).  All ring slots are
// compile-time constants so the rings live in registers.
// Deepest level worth computing at step J of unrolled group G of a tile
// (G < 0: past the tile's first two groups).  Level S of the tile's step j
// reads level-0 rows back to r0 + j - 2S, so it holds a row of the output's
// dependence cone only from j = 2S on; earlier levels are skipped.
template <int T, int U, int G, int J>
constexpr int m2_lmax() {
    return G < 0 ? T : ((G * U + J) / 2 < T ? (G * U + J) / 2 : T);
}

// Whether the step after step J of group G computes level 1.
template <int T, int U, int G, int J>
constexpr bool m2_next_l1() {
    return J + 1 == U || m2_lmax<T, U, G, J + 1>() >= 1;
}

template <typename R, int T, int P, int MODE, int EK, bool RES, int J, int S, int G = -1>
__device__ __forceinline__ void m2_level(const Geom &g, R *__restrict__ uout,
                                         double *__restrict__ gacc, const MLane &L, MRegs<R, T, P> &m, const int r,
                                         const Cur &sc, const int sr) {
    using M = M2<R, T, P>;
    constexpr int V = M::V;
    constexpr bool SRC = MODE == MODE_POISSON;
    constexpr int LMAX = m2_lmax<T, M::U, G, J>();
    if constexpr (S <= LMAX) {
        const int y = r - S;
        const int ny = g.n[1];
        // value copies (register renames): pointers into the rings would
        // keep them out of registers
        R up[V], cen[V], dn[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if constexpr (S == 1) {
                up[v] = m.l0[(J + M::LR - 2) % M::LR][v];   // row r-2
                cen[v] = m.l0[(J + M::LR - 1) % M::LR][v];  // row r-1
                dn[v] = m.l0[J % M::LR][v];                 // row r
            } else {
                up[v] = m.lv[S - 2][(J + 1) % 3][v];
                cen[v] = m.lv[S - 2][(J + 2) % 3][v];
                dn[v] = m.lv[S - 2][J % 3][v];
            }
        }
        R bv[V];  // source row r - S, read from the wave's LDS ring one level ahead
        if constexpr (SRC) {
#pragma unroll
            for (int v = 0; v < V; ++v) bv[v] = m.bn[S & 1][v];
            if constexpr (S < LMAX)
                m2_read_src<R, T, P, S + 1>(L, m, sr);
            else if constexpr (m2_next_l1<T, M::U, G, J>())
                m2_read_src<R, T, P, 1, 0>(L, m, sr);  // the next step's level 1: this row
            // keep the read ahead of this level's arithmetic: left to itself
            // the scheduler sinks it to just before its use, a few
            // instructions on, and every level then waits for LDS
            __builtin_amdgcn_sched_barrier(0);
        }
        R out[V];
        {
            R eo = (R)0;
            if constexpr (S == 1) eo = m.e0[(J + M::LR - 1) % M::LR];
            const R left = shift_up(eo, cen[V - 1]);
            const R right = shift_down(eo, cen[0]);
            const R w = (R)0.25;
            const bool acc_row = (S == 1) && RES && y >= L.oy0 && y < L.oy1;
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
                        const bool mine = (EK & 2) ? L.st[v] : L.out_lane;
                        m.acc += mine ? rr * rr : 0.0;
                    }
                }
                // ring columns (and columns beyond them) keep their values
                if constexpr ((EK & 2) != 0) o = L.upd[v] ? o : cen[v];
                out[v] = o;
            }
        }
        // ring rows (and rows beyond them) keep their values
        if constexpr ((EK & 1) != 0) {
            if (y < 0 || y >= ny) {
#pragma unroll
                for (int v = 0; v < V; ++v) out[v] = cen[v];
            }
        }
        if constexpr (S < T) {
#pragma unroll
            for (int v = 0; v < V; ++v) m.lv[S - 1][J % 3][v] = out[v];
            m2_accumulate<R, T, P, MODE, EK, (J - S + 2 * M::RA) % M::RA, S == T - 1>(g, gacc, L,
                                                                                     m, y, out);
        } else {
            if (uout && y >= L.oy0 && y < L.oy1) {
                R *row = uout + sc.su;
                Chunk<R, V> o;
#pragma unroll
                for (int v = 0; v < V; ++v) o.v[v] = out[v];
                if (L.st_all) {
                    if (L.nt)
                        store_nt16(&at_mut<Chunk<R, V>>(row, L.lane_b), o);
                    else
                        at_mut<Chunk<R, V>>(row, L.lane_b) = o;
                } else if constexpr ((EK & 2) != 0) {
                    // the lane holding the east ring column and interior
                    // columns before it stores element by element
                    if (L.st_part) {
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            if (L.st[v]) at_mut<R>(row, L.lane_b + v * (uint32_t)sizeof(R)) = out[v];
                    }
                }
            }
        }
        m2_level<R, T, P, MODE, EK, RES, J, S + 1, G>(g, uout, gacc, L, m, r, sc, sr);
    }
}

template <typename R, int T, int P, int MODE, int EK, bool RES, int J, int G = -1>
__device__ __forceinline__ void m2_steps(const Geom &g, const R *__restrict__ uin,
                                         R *__restrict__ uout, const R *__restrict__ bsrc,
                                         double *__restrict__ gacc, const MLane &L, MRegs<R, T, P> &m, const int base, Cur &lc,
                                         Cur &sc, int &sr) {
    using M = M2<R, T, P>;
    constexpr int V = M::V;
    if constexpr (J < M::U) {
        const int r = base + J;
        if (r > L.r1) return;
        // the source row r, loaded P steps ago, moves to the LDS slot that
        // row r - RB held; levels read it from the next step on
        auto to_lds = [&]() {
            if constexpr (MODE == MODE_POISSON) {
                Chunk<R, V> c;
#pragma unroll
                for (int v = 0; v < V; ++v) c.v[v] = m.bq[J % M::BQ][v];
                static_cast<Chunk<R, V> *>(L.bs)[sr * 64] = c;
            }
        };
        if constexpr (M::WRITE_FIRST) to_lds();
        // row r+P goes into the slots rows r+P-LR (state), r+P-BQ (source
        // registers) and r+1-RA (accumulator, P = 1) held; at the last P
        // steps this reads rows no level uses, which keeps the loads
        // unconditional
        m2_load<R, T, P, MODE, EK, (J + P) % M::LR, (J + P) % M::BQ, (J + 1) % M::RA>(
            g, uin, bsrc, gacc, L, m, lc);
        if constexpr (!M::WRITE_FIRST) to_lds();
        if constexpr (MODE == MODE_ADJOINT) {
            // level 0 of row r (the pass's input) is the first term added
            R v0[V];
#pragma unroll
            for (int v = 0; v < V; ++v) v0[v] = m.l0[J % M::LR][v];
            m2_accumulate<R, T, P, MODE, EK, J % M::RA, T == 1>(g, gacc, L, m, r, v0);
        }
        // level 1's source row was read by the last level of the step before;
        // a step that computes no level reads the next step's row itself
        if constexpr (MODE == MODE_POISSON && m2_lmax<T, M::U, G, J>() == 0 &&
                      m2_next_l1<T, M::U, G, J>())
            m2_read_src<R, T, P, 1, 0>(L, m, sr);
        m2_level<R, T, P, MODE, EK, RES, J, 1, G>(g, uout, gacc, L, m, r, sc, sr);
        sc.advance(g);
        sr = sr + 1 == M::RB ? 0 : sr + 1;
        m2_steps<R, T, P, MODE, EK, RES, J + 1, G>(g, uin, uout, bsrc, gacc, L, m, base, lc, sc,
                                                     sr);
    }
}

template <typename R, int T, int P, int MODE, int EK, bool RES>
__device__ __forceinline__ void m2_body(const Geom &g, const R *__restrict__ uin,
                                        R *__restrict__ uout, const R *__restrict__ bsrc,
                                        double *__restrict__ res_slot,
                                        double *__restrict__ gacc, const MLane &L, int r0) {
    using S = M2<R, T, P>;
    MRegs<R, T, P> m;
#pragma unroll
    for (int k = 0; k < S::LR; ++k) {
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
    // rows r0 .. r0+P-1 -> slots 0 .. P-1
    m2_load<R, T, P, MODE, EK, 0, 0, 0>(g, uin, bsrc, gacc, L, m, lc);
    if constexpr (P > 1) m2_load<R, T, P, MODE, EK, 1, 1 % S::BQ, 1 % S::RA>(g, uin, bsrc, gacc, L, m, lc);
    if constexpr (P > 2) m2_load<R, T, P, MODE, EK, 2, 2 % S::BQ, 2 % S::RA>(g, uin, bsrc, gacc, L, m, lc);
    int sr = 0;  // LDS source slot of the current row
    int base = r0;
    if constexpr (MODE != MODE_ADJOINT && T > 1) {
        // the tile's first group (and, from depth 7 on, its second) skip the
        // levels still outside the output's dependence cone (the adjoint
        // pass accumulates every level it holds, so it runs them all)
        m2_steps<R, T, P, MODE, EK, RES, 0, 0>(g, uin, uout, bsrc, gacc, L, m, base, lc, sc, sr);
        base += S::U;
        if constexpr (T > S::U / 2) {
            if (base <= L.r1) {
                m2_steps<R, T, P, MODE, EK, RES, 0, 1>(g, uin, uout, bsrc, gacc, L, m, base, lc,
                                                         sc, sr);
                base += S::U;
            }
        }
    }
    // without the warm-up groups the first step computes level 1 (its row
    // lies before the tile and is not an output)
    if constexpr (MODE == MODE_POISSON && T == 1) m2_read_src<R, T, P, 1>(L, m, sr);
    for (; base <= L.r1; base += S::U)
        m2_steps<R, T, P, MODE, EK, RES, 0>(g, uin, uout, bsrc, gacc, L, m, base, lc, sc, sr);
    if constexpr (RES) {
        const double a = wave_sum(m.acc);
        if ((threadIdx.x & 63) == 0) *res_slot = a;
    }
}

// One work item (wave): tile number `wid` of a grid cut into tiles of
// `rows` rows.  wid is wave-uniform.  RES: accumulate the residual partial into
// *res_slot.  bs_wave: the wave's LDS source ring.
template <typename R, int T, int P, int MODE, bool RES>
__device__ __forceinline__ void m2_run(const Geom &g, const R *__restrict__ uin,
                                       R *__restrict__ uout, const R *__restrict__ bsrc,
                                       double *__restrict__ res_slot, double *__restrict__ gacc,
                                       int wid, int rows, Chunk<R, M2<R, T, P>::V> *bs_wave,
                                       bool nt) {
    using S = M2<R, T, P>;
    constexpr bool SRC = MODE == MODE_POISSON;
    constexpr int V = S::V;
    const int lane = threadIdx.x & 63;
    const int nx = g.n[0], ny = g.n[1];
    const M2Tiles tl = m2_tiles(nx, ny, S::OW, rows, T);
    int strip, oy0, oy1;
    m2_tile(tl, ny, rows, wid, strip, oy0, oy1);
    const int a = strip * S::OW - S::A0;  // first column held by the strip
    MLane L;
    L.bs = SRC ? (void *)(bs_wave + lane) : nullptr;
    L.oy0 = oy0;
    L.oy1 = oy1;
    L.r1 = L.oy1 - 1 + T;
    const int c = a + lane * V;
    L.c = c;
    // lanes whose chunk lies beyond the ring read column 0's chunk instead
    const bool ld = c >= -V && c <= nx;
    {
        int bx, lx;
        owner(ld ? c : 0, g.e[0], g.nb[0], bx, lx);
        L.lane_b = (uint32_t)(((int64_t)bx * g.bstride + g.ax + lx) * (int64_t)sizeof(R));
        const bool ldb = SRC && c >= 0 && c < nx;
        L.src_b = (uint32_t)(((int64_t)bx * g.sstride + (ldb ? lx : 0)) * (int64_t)sizeof(R));
    }
    {
        // lanes 0 and 63 fetch the cells just outside the strip; the others
        // re-read their own first cell (a harmless in-bounds load)
        const int xe = lane == 0 ? a - 1 : lane == 63 ? a + S::W : c;
        const bool lde = xe >= -1 && xe <= nx && (lane == 0 || lane == 63 || ld);
        int bx, lx;
        owner(lde ? xe : 0, g.e[0], g.nb[0], bx, lx);
        L.edge_b = (uint32_t)(((int64_t)bx * g.bstride + g.ax + lx) * (int64_t)sizeof(R));
    }
    L.out_lane = lane >= S::L0 && lane < S::L1;
    L.nt = nt;
    bool all = L.out_lane, any = false;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int x = c + v;
        L.upd[v] = x >= 0 && x < nx;
        L.st[v] = v < V && L.upd[v] && L.out_lane;
        if (v < V) {
            all = all && L.upd[v];
            any = any || L.st[v];
        }
    }
    L.st_all = all;
    L.st_part = any && !all;
    // rows r0 .. r1 + P are read; an interior tile reads only grid rows and
    // columns, none of them on the ring
    static_assert(MODE != MODE_ADJOINT || P == 1, "the adjoint pass prefetches one row");
    static_assert(MODE != MODE_ADJOINT || T + 1 <= S::RA, "adjoint accumulator ring too small");
    // edge kinds: bit 0 = the tile reads rows on or beyond the ring (row
    // tests), bit 1 = the strip holds columns on or beyond it (column tests)
    const int r0 = L.oy0 - T;
    const bool ex = a < 0 || a + S::W > nx;
    const bool ey = r0 < 0 || L.r1 + P > ny - 1;
    // (the middle tiles of the outer strips run the copy with both tests: a
    // fourth copy pushes the kernel past the registers of two waves per SIMD)
    if (ex)
        m2_body<R, T, P, MODE, 3, RES>(g, uin, uout, bsrc, res_slot, gacc, L, r0);
    else if (ey)
        m2_body<R, T, P, MODE, 1, RES>(g, uin, uout, bsrc, res_slot, gacc, L, r0);
    else
        m2_body<R, T, P, MODE, 0, RES>(g, uin, uout, bsrc, res_slot, gacc, L, r0);
}

// uout may be NULL (no stores: residual only); res (used when RES) receives
// one residual partial per work item; gacc is the FP64 accumulator of the
// adjoint pass (MODE_ADJOINT only).
template <typename R, int T, int P, int MODE, bool RES>
__global__ __launch_bounds__(64 * kM2Waves) void k_march2d(Geom g, const R *__restrict__ uin,
                                                 R *__restrict__ uout,
                                                 const R *__restrict__ bsrc,
                                                 double *__restrict__ res,
                                                 double *__restrict__ gacc, int rows, int nwork,
                                                 int nt) {
    using S = M2<R, T, P>;
    constexpr bool SRC = MODE == MODE_POISSON;
    // per wave: a ring of RB source rows, one 16-byte chunk per lane each
    __shared__ Chunk<R, S::V> bsm[SRC ? kM2Waves * S::RB * 64 : 1];
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int wid = __builtin_amdgcn_readfirstlane(lb * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wid >= nwork) return;
    m2_run<R, T, P, MODE, RES>(g, uin, uout, bsrc, RES ? res + wid : nullptr, gacc, wid, rows,
                               &bsm[SRC ? (threadIdx.x >> 6) * S::RB * 64 : 0], nt != 0);
}

// Batched pass: the work items of all grids of a batch in one launch.  Work
// item w belongs to grid gi with prefix[gi] <= w < prefix[gi+1]; inactive
// grids (stopped by the convergence test) skip their items.  All active
// grids advance together, so the input buffer is u[pass_count & 1].
// MODE: Poisson (the batched solver; the deep-halo form with a source) or
// Laplace (the deep-halo form without one).
template <typename R, int T, int P, bool RES, int MODE>
__global__ __launch_bounds__(64 * kM2Waves) void k_march2d_batch(const BatchGrid *__restrict__ grids,
                                                       const int *__restrict__ prefix, int ngrids,
                                                       const int *__restrict__ active,
                                                       const int *__restrict__ pass_count,
                                                       double *__restrict__ res, int store,
                                                       int rows, int nwork) {
    using S = M2<R, T, P>;
    constexpr bool SRC = MODE == MODE_POISSON;
    __shared__ Chunk<R, S::V> bsm[SRC ? kM2Waves * S::RB * 64 : 1];
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
    m2_run<R, T, P, MODE, RES>(g, uin, uout, SRC ? (const R *)grids[gi].b : nullptr,
                               RES ? res + wid : nullptr, nullptr, wid - prefix[gi], rows,
                               &bsm[SRC ? (threadIdx.x >> 6) * S::RB * 64 : 0], false);
}

// ---- host side -------------------------------------------------------------
// The kernels of each temporal depth T are compiled in an object of their
// own (this file built with JAC_MARCH2D_DEPTH=T), so the depths compile in
// parallel; the object built without it holds the depth dispatch only, which
// sees the per-depth launchers as declarations and instantiates no kernel.

template <typename R, int T>
static int64_t m2_nwork(const Geom &g, int rows) {
    using S = M2<R, T, 1>;  // the tiling does not depend on the prefetch distance
    return m2_tiles(g.n[0], g.n[1], S::OW, rows, T).nwork;
}

// Prefetch distance of the Laplace and Poisson passes of depth T: two rows
// ahead (one step of arithmetic did not always cover the memory latency;
// measured at 8192^2 FP32, depth 13: 0.239 -> 0.222 ms per pass, depth 8:
// -3%, depth 4: equal), except at the depths whose levels leave no registers
// for the two extra rows (14 and 16).  The adjoint pass loads one row ahead.
template <int T>
constexpr int m2_pf() {
    return T <= 13 ? 2 : 1;
}

template <typename R, int T>
hipError_t m2_launch_t(const Geom &g, const void *uin, void *uout, const void *b, double *res,
                       double *gacc, int rows, hipStream_t st, int64_t *nwork_out, int nt);
template <typename R, int T>
hipError_t m2b_launch_t(const BatchGrid *grids, const int *prefix, int ngrids, const int *active,
                        const int *pass_count, double *res, bool store, int rows, int nwork,
                        hipStream_t st, int mode);
template <typename R, int T>
int m2_waves_per_cu_t(int mode);

#ifdef JAC_MARCH2D_DEPTH

template <typename R, int T, int P>
static hipError_t m2_launch_p(const Geom &g, const void *uin, void *uout, const void *b,
                              double *res, double *gacc, int rows, int nwork, hipStream_t st,
                              int nt) {
    const int grid = (nwork + kM2Waves - 1) / kM2Waves;
    const R *bb = (const R *)b;
    if (gacc) {
        // adjoint passes go to depth 8 (the accumulator ring holds T + 1 rows)
        if constexpr (T > 8) {
            return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((k_march2d<R, T, 1, MODE_ADJOINT, false>), dim3(grid), dim3(64 * kM2Waves), 0,
                               st, g, (const R *)uin, (R *)uout, (const R *)nullptr,
                               (double *)nullptr, gacc, rows, nwork, nt);
            return hipGetLastError();
        }
    }
    if (b && res)
        hipLaunchKernelGGL((k_march2d<R, T, P, MODE_POISSON, true>), dim3(grid), dim3(64 * kM2Waves), 0, st,
                           g, (const R *)uin, (R *)uout, bb, res, (double *)nullptr, rows, nwork,
                           nt);
    else if (b)
        hipLaunchKernelGGL((k_march2d<R, T, P, MODE_POISSON, false>), dim3(grid), dim3(64 * kM2Waves), 0, st,
                           g, (const R *)uin, (R *)uout, bb, (double *)nullptr, (double *)nullptr,
                           rows, nwork, nt);
    else if (res)
        hipLaunchKernelGGL((k_march2d<R, T, P, MODE_LAPLACE, true>), dim3(grid), dim3(64 * kM2Waves), 0, st,
                           g, (const R *)uin, (R *)uout, (const R *)nullptr, res,
                           (double *)nullptr, rows, nwork, nt);
    else
        hipLaunchKernelGGL((k_march2d<R, T, P, MODE_LAPLACE, false>), dim3(grid), dim3(64 * kM2Waves), 0, st,
                           g, (const R *)uin, (R *)uout, (const R *)nullptr, (double *)nullptr,
                           (double *)nullptr, rows, nwork, nt);
    return hipGetLastError();
}

template <typename R, int T>
hipError_t m2_launch_t(const Geom &g, const void *uin, void *uout, const void *b, double *res,
                       double *gacc, int rows, hipStream_t st, int64_t *nwork_out, int nt) {
    const int64_t nwork = m2_nwork<R, T>(g, rows);
    if (nwork_out) *nwork_out = nwork;
    if (nwork > 0x7fffffff - 3) return hipErrorInvalidValue;
    return m2_launch_p<R, T, m2_pf<T>()>(g, uin, uout, b, res, gacc, rows, (int)nwork, st, nt);
}

template <typename R, int T, int P>
static hipError_t m2b_launch_p(const BatchGrid *grids, const int *prefix, int ngrids,
                               const int *active, const int *pass_count, double *res, bool store,
                               int rows, int nwork, hipStream_t st, int mode) {
    const int grid = (nwork + kM2Waves - 1) / kM2Waves;
    if (mode == MODE_LAPLACE) {
        // the deep-halo form without a source: no residual
        if (res) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_march2d_batch<R, T, P, false, MODE_LAPLACE>), dim3(grid), dim3(64 * kM2Waves),
                           0, st, grids, prefix, ngrids, active, pass_count, res, store ? 1 : 0,
                           rows, nwork);
    } else if (res)
        hipLaunchKernelGGL((k_march2d_batch<R, T, P, true, MODE_POISSON>), dim3(grid), dim3(64 * kM2Waves),
                           0, st, grids, prefix, ngrids, active, pass_count, res, store ? 1 : 0,
                           rows, nwork);
    else
        hipLaunchKernelGGL((k_march2d_batch<R, T, P, false, MODE_POISSON>), dim3(grid), dim3(64 * kM2Waves),
                           0, st, grids, prefix, ngrids, active, pass_count, res, store ? 1 : 0,
                           rows, nwork);
    return hipGetLastError();
}

template <typename R, int T>
hipError_t m2b_launch_t(const BatchGrid *grids, const int *prefix, int ngrids, const int *active,
                        const int *pass_count, double *res, bool store, int rows, int nwork,
                        hipStream_t st, int mode) {
    return m2b_launch_p<R, T, m2_pf<T>()>(grids, prefix, ngrids, active, pass_count, res, store,
                                          rows, nwork, st, mode);
}

template <typename R, int T>
int m2_waves_per_cu_t(int mode) {
    constexpr int P = m2_pf<T>();
    int blocks = 0;
    hipError_t e;
    if (mode == MODE_ADJOINT) {
        if constexpr (T > 8)
            return 0;
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_march2d<R, T, 1, MODE_ADJOINT, false>, 64 * kM2Waves, 0);
    } else if (mode == MODE_POISSON)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_march2d<R, T, P, MODE_POISSON, false>, 64 * kM2Waves, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_march2d<R, T, P, MODE_LAPLACE, false>, 64 * kM2Waves, 0);
    return e == hipSuccess ? blocks * kM2Waves : 0;
}

#define JAC_M2_INSTANTIATE(R, T)                                                              \
    template hipError_t m2_launch_t<R, T>(const Geom &, const void *, void *, const void *,    \
                                          double *, double *, int, hipStream_t, int64_t *,     \
                                          int);                                                \
    template hipError_t m2b_launch_t<R, T>(const BatchGrid *, const int *, int, const int *,   \
                                           const int *, double *, bool, int, int,              \
                                           hipStream_t, int);                                  \
    template int m2_waves_per_cu_t<R, T>(int);

JAC_M2_INSTANTIATE(float, JAC_MARCH2D_DEPTH)
#if JAC_MARCH2D_DEPTH <= 4
JAC_M2_INSTANTIATE(double, JAC_MARCH2D_DEPTH)
#endif

#else  // dispatch object

static const int kDepthsF32[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 11, 12, 13, 14, 16};
static const int kDepthsF64[] = {1, 2, 3, 4};

int march2d_depths(int dtype, const int **list) {
    if (dtype == 0) {
        *list = kDepthsF32;
        return (int)(sizeof(kDepthsF32) / sizeof(int));
    }
    *list = kDepthsF64;
    return (int)(sizeof(kDepthsF64) / sizeof(int));
}

// Calls F<R, depth>(args...) for a compiled depth (1..8, 10..14, 16 in FP32,
// 1..4 in FP64); `bad` otherwise.
#define JAC_M2_CASE(F, R, D, BAD, ...)                                  \
    case D:                                                             \
        if constexpr (sizeof(R) == 8 && D > 4)                          \
            return BAD;                                                 \
        else                                                            \
            return F<R, D>(__VA_ARGS__);
#define JAC_M2_SWITCH(depth, F, R, BAD, ...)                            \
    switch (depth) {                                                    \
        JAC_M2_CASE(F, R, 1, BAD, __VA_ARGS__)                          \
        JAC_M2_CASE(F, R, 2, BAD, __VA_ARGS__)                          \
        JAC_M2_CASE(F, R, 3, BAD, __VA_ARGS__)                          \
        JAC_M2_CASE(F, R, 4, BAD, __VA_ARGS__)                          \
        JAC_M2_CASE(F, R, 5, BAD, __VA_ARGS__)                          \
        JAC_M2_CASE(F, R, 6, BAD, __VA_ARGS__)                          \
        JAC_M2_CASE(F, R, 7, BAD, __VA_ARGS__)                          \
        JAC_M2_CASE(F, R, 8, BAD, __VA_ARGS__)                          \
        JAC_M2_CASE(F, R, 10, BAD, __VA_ARGS__)                         \
        JAC_M2_CASE(F, R, 11, BAD, __VA_ARGS__)                         \
        JAC_M2_CASE(F, R, 12, BAD, __VA_ARGS__)                         \
        JAC_M2_CASE(F, R, 13, BAD, __VA_ARGS__)                         \
        JAC_M2_CASE(F, R, 14, BAD, __VA_ARGS__)                         \
        JAC_M2_CASE(F, R, 16, BAD, __VA_ARGS__)                         \
    default:                                                            \
        return BAD;                                                     \
    }

template <typename R>
int march2d_waves_per_cu(int depth, int mode) {
    JAC_M2_SWITCH(depth, m2_waves_per_cu_t, R, 0, mode)
}

template <typename R>
int64_t march2d_work_items(const Geom &g, int depth, int rows) {
    JAC_M2_SWITCH(depth, m2_nwork, R, (int64_t)-1, g, rows)
}


template <typename R>
hipError_t launch_sweep2d_march(const Geom &g, const void *uin, void *uout, const void *b,
                                double *res, double *gacc, int depth, int rows, hipStream_t st,
                                int64_t *nwork, int nt) {
    JAC_M2_SWITCH(depth, m2_launch_t, R, hipErrorInvalidValue, g, uin, uout, b, res, gacc, rows,
                  st, nwork, nt)
}

template <typename R>
int64_t march2d_batch_work(const Geom &g, int depth, int rows) {
    JAC_M2_SWITCH(depth, m2_nwork, R, (int64_t)-1, g, rows)
}

template <typename R>
hipError_t launch_march2d_batch(const BatchGrid *grids, const int *prefix, int ngrids,
                                const int *active, const int *pass_count, double *res, bool store,
                                int depth, int rows, int nwork, hipStream_t st, int mode) {
    if (nwork <= 0) return hipSuccess;
    JAC_M2_SWITCH(depth, m2b_launch_t, R, hipErrorInvalidValue, grids, prefix, ngrids, active,
                  pass_count, res, store, rows, nwork, st, mode)
}

template hipError_t launch_sweep2d_march<float>(const Geom &, const void *, void *, const void *,
                                                double *, double *, int, int, hipStream_t,
                                                int64_t *, int);
template hipError_t launch_sweep2d_march<double>(const Geom &, const void *, void *, const void *,
                                                 double *, double *, int, int, hipStream_t,
                                                 int64_t *, int);
template int64_t march2d_batch_work<float>(const Geom &, int, int);
template int64_t march2d_batch_work<double>(const Geom &, int, int);
template hipError_t launch_march2d_batch<float>(const BatchGrid *, const int *, int, const int *,
                                                const int *, double *, bool, int, int, int,
                                                hipStream_t, int);
template hipError_t launch_march2d_batch<double>(const BatchGrid *, const int *, int, const int *,
                                                 const int *, double *, bool, int, int, int,
                                                 hipStream_t, int);
template int64_t march2d_work_items<float>(const Geom &, int, int);
template int64_t march2d_work_items<double>(const Geom &, int, int);
template int march2d_waves_per_cu<float>(int, int);
template int march2d_waves_per_cu<double>(int, int);

#endif  // JAC_MARCH2D_DEPTH

}  // namespace jac
