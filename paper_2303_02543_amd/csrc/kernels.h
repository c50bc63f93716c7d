// Launch functions of the gfx950 kernels (host side, internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "jacobi_internal.h"

namespace jac {

template <typename R>
hipError_t launch_scatter(const Geom &g, const void *u, void *s0, void *s1, hipStream_t st);
template <typename R>
hipError_t launch_gather(const Geom &g, const void *s, void *u, hipStream_t st);
template <typename R>
hipError_t launch_scale_source(const Geom &g, const void *f, void *b, double h2, hipStream_t st);
template <typename R>
hipError_t launch_halo_exchange(const Geom &g, void *s, hipStream_t st);

// One sweep of every block from its own storage (halos must be current).
template <typename R>
hipError_t launch_sweep_local(const Geom &g, const void *uin, void *uout, const void *b,
                              hipStream_t st);

// `depth` sweeps in one pass over the whole 2D grid, reading face neighbours'
// cells from their owning blocks.  depth must be one of march2d_depths().
template <typename R>
hipError_t launch_sweep2d_march(const Geom &g, const void *uin, void *uout, const void *b,
                                int depth, int rows, hipStream_t st);
// Depths compiled for the 2D march kernel, ascending; returns the count.
int march2d_depths(int dtype, const int **list);

// FP64 residual: per-workgroup partial sums into `partials` (kResidualGroups
// doubles), then one workgroup sums them in a fixed order and writes
// sqrt(total) to *out.
constexpr int kResidualGroups = 1024;
template <typename R>
hipError_t launch_residual(const Geom &g, const void *u, const void *b, double *partials,
                           double *out, hipStream_t st);

}  // namespace jac
