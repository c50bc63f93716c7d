// Launch functions of the gfx950 kernels (host side, internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "jacobi_internal.h"

namespace jac {

// zero_ring: write 0 instead of the ring values (the adjoint state's ring).
template <typename R>
hipError_t launch_scatter(const Geom &g, const void *u, void *s0, void *s1, bool zero_ring,
                          hipStream_t st);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t st);
hipError_t launch_adjoint_finish(const Geom &g, const double *gb, double h2, double *grad_f,
                                 double *grad_ring, hipStream_t st);
// Full FP64 dL/dU0 ((n_y+2) x (n_x+2)) of a 2D adjoint run: interior =
// lam_0 from the blocked state s; ring = lamK's ring (the loss's gradient on
// the ring of u_K) plus, off the corners, gb at the adjacent interior node.
template <typename R>
hipError_t launch_adjoint_full(const Geom &g, const double *gb, const void *lamK, const void *s,
                               double *out, hipStream_t st);
template <typename R>
hipError_t launch_gather(const Geom &g, const void *s, void *u, hipStream_t st);
template <typename R>
hipError_t launch_scale_source(const Geom &g, const void *f, void *b, double h2, hipStream_t st);
template <typename R>
hipError_t launch_halo_exchange(const Geom &g, void *s, hipStream_t st);

// One sweep of blocks b0 .. b1-1 (b1 < 0: to the last block) from their own
// storage (halos must be current).  2D: rg rows per work item (0: a default);
// nt != 0: non-temporal output stores (2D tiles).
template <typename R>
hipError_t launch_sweep_local(const Geom &g, const void *uin, void *uout, const void *b,
                              hipStream_t st, int rg = 0, int64_t b0 = 0, int64_t b1 = -1,
                              int nt = 0);
// One 2D sweep of the whole grid by the tile kernel, reading the cells just
// outside each block from the neighbouring blocks that own them (no halo
// exchange needed; the stored halos are not refreshed).  rg: rows per tile
// (0: the default).  If res is not NULL, the FP64 residual of the input
// state is summed into one partial per wave, res[0 .. *nwork).
template <typename R>
hipError_t launch_sweep2d_tile_fused(const Geom &g, const void *uin, void *uout, const void *b,
                                     double *res, int rg, hipStream_t st, int64_t *nwork,
                                     int nt = 0);
// Residual partials of one launch_sweep2d_tile_fused launch.
template <typename R>
int64_t sweep_tile_partials(const Geom &g, int rg);
// Face sends of blocks b0 .. b1-1: each block's edge cells into the halos of
// its face neighbours (all blocks together: the same as launch_halo_exchange).
template <typename R>
hipError_t launch_halo_send(const Geom &g, void *s, int64_t b0, int64_t b1, hipStream_t st);

// `depth` sweeps in one pass over the whole 2D grid, reading face neighbours'
// cells from their owning blocks.  uout may be NULL (no output: residual
// only).  If res is not NULL, the FP64 residual of the input state is
// accumulated and one partial per work item is written to res[0 .. nwork);
// k_residual_final then sums them.  If gacc is not NULL the pass is an
// adjoint pass: b and res must be NULL, the state's ring must be zero, and
// w * (the pass's input and its first depth-1 levels) is added, in that
// order, to the FP64 interior array gacc (n_y x n_x).  depth must be one of
// march2d_depths().  nt != 0: non-temporal output stores.
template <typename R>
hipError_t launch_sweep2d_march(const Geom &g, const void *uin, void *uout, const void *b,
                                double *res, double *gacc, int depth, int rows, hipStream_t st,
                                int64_t *nwork, int nt = 0);
// Work items (waves) of one march launch; -1 for an unknown depth.
template <typename R>
int64_t march2d_work_items(const Geom &g, int depth, int rows);
// Resident waves per CU of the depth-`depth` march kernel in `mode`
// (0 Laplace, 1 Poisson, 2 adjoint); 0 if unknown.
template <typename R>
int march2d_waves_per_cu(int depth, int mode);
// Depths compiled for the 2D march kernel, ascending; returns the count.
int march2d_depths(int dtype, const int **list);

// Batched pass over the grids of a batch (Poisson kernels; see
// k_march2d_batch).  nwork = prefix[ngrids]; res: one partial per work item
// (NULL: no residual); store = false: residual only.
// mode: 1 Poisson (the grids' sources), 0 Laplace (no residual).
template <typename R>
hipError_t launch_march2d_batch(const BatchGrid *grids, const int *prefix, int ngrids,
                                const int *active, const int *pass_count, double *res, bool store,
                                int depth, int rows, int nwork, hipStream_t st, int mode = 1);
// Work items of one grid at this depth / tile height.
template <typename R>
int64_t march2d_batch_work(const Geom &g, int depth, int rows);

// `depth` 3D sweeps in one pass over the whole grid (k_march3d.hip), reading
// face neighbours' cells from their owning blocks; zseg output planes per
// work item.  uout may be NULL (residual only); res: one partial per wave
// (8 per work item) or NULL.  depth in 1 .. march3d_max_depth().
template <typename R>
hipError_t launch_march3d(const Geom &g, const void *uin, void *uout, const void *b, double *res,
                          int zseg, hipStream_t st, int64_t *nwork, int nt = 0, int depth = 1);
template <typename R>
int64_t march3d_work_items(const Geom &g, int zseg, int depth = 1);
int march3d_max_depth();

// Batched 3D pass (k_march3d.hip): the work items of every grid of a
// descriptor table in one launch, each grid read from u[0] and written to
// u[1]; src: Poisson (the grids' sources) or Laplace.  prefix[i]: first work
// item of grid i, prefix[ngrids] = nitems.  march3d_batch_items: work items
// of one grid.
template <typename R>
hipError_t launch_march3d_batch(const BatchGrid *grids, const int *prefix, int ngrids, bool src,
                                int depth, int zseg, int nitems, hipStream_t st);
template <typename R>
int64_t march3d_batch_items(const Geom &g, int zseg, int depth);

// Deep-halo block storage (k_deep.hip): refresh every block's H-deep frame
// of state buffer s from the cells' owning blocks; fill the deep source
// buffer bd (state layout) from the blocked source b (NULL: zeros).
template <typename R>
hipError_t launch_deep_exchange(const Geom &g, void *s, int H, hipStream_t st);
template <typename R>
hipError_t launch_deep_source(const Geom &g, const void *b, void *bd, int H, hipStream_t st);

// Batched-solver bookkeeping (k_batch.hip).
hipError_t launch_batch_init(int count, const BatchState &st, hipStream_t s);
hipError_t launch_batch_advance(const BatchState &st, int sweeps, hipStream_t s);
hipError_t launch_batch_check(const int *prefix, const double *partials, int count,
                              const BatchState &st, double tol, bool final_check, hipStream_t s);

// Sum n partials in a fixed order and write sqrt(total) to *out.
hipError_t launch_residual_final(const double *partials, int n, double *out, hipStream_t st);

// FP64 residual: per-workgroup partial sums into `partials` (kResidualGroups
// doubles), then one workgroup sums them in a fixed order and writes
// sqrt(total) to *out.
constexpr int kResidualGroups = 1024;
template <typename R>
hipError_t launch_residual(const Geom &g, const void *u, const void *b, double *partials,
                           double *out, hipStream_t st);

}  // namespace jac
