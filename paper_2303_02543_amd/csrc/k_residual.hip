// FP64 residual of the blocked state.
//
// The paper's proxy runs a fixed number of iterations and states no residual;
// the library reports the L2 norm of the h^2-scaled residual of the discrete
// Poisson system, r = b - (2d u - s) with s the sweep's neighbour sum, every
// value widened to FP64 and every operation done in FP64 (the cancellation in
// 2d u - s is what makes FP32 unusable there).
//
// Deterministic two-stage sum: a fixed grid of kResidualGroups workgroups
// walks the chunks with a fixed stride, reduces within each wave by xor
// shuffles and across the four waves through LDS, and writes one partial per
// workgroup; a single workgroup then adds the partials in a fixed tree.  The
// order never depends on scheduling, so repeated calls give identical bits.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

template <typename R, bool SRC>
__global__ __launch_bounds__(256) void k_residual(Geom g, const R *__restrict__ u,
                                                  const R *__restrict__ b,
                                                  double *__restrict__ partials, int64_t total,
                                                  int cpr) {
    constexpr int V = 16 / sizeof(R);
    using C = Chunk<R, V>;
    const int nx = g.n[0], ny = g.n[1];
    const double c2d = 2.0 * g.ndim;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % cpr) * V;
        const int64_t row = i / cpr;
        const int y = (int)(row % ny);
        const int z = (int)(row / ny);
        const C cen = *reinterpret_cast<const C *>(u + state_offset(g, c, y, z));
        const C so = *reinterpret_cast<const C *>(u + state_offset(g, c, y - 1, z));
        const C no = *reinterpret_cast<const C *>(u + state_offset(g, c, y + 1, z));
        C ba, fr;
        if (g.ndim == 3) {
            ba = *reinterpret_cast<const C *>(u + state_offset(g, c, y, z - 1));
            fr = *reinterpret_cast<const C *>(u + state_offset(g, c, y, z + 1));
        }
        const double west = (double)u[state_offset(g, c - 1, y, z)];
        const double east = (c + V <= nx) ? (double)u[state_offset(g, c + V, y, z)] : 0.0;
        C bb;
        if (SRC) bb = *reinterpret_cast<const C *>(b + source_offset(g, c, y, z));
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (c + v < nx) {
                const double W = v > 0 ? (double)cen.v[v - 1] : west;
                const double E = v < V - 1 ? (double)cen.v[v + 1] : east;
                double s = (W + E) + ((double)so.v[v] + (double)no.v[v]);
                if (g.ndim == 3) s = s + ((double)ba.v[v] + (double)fr.v[v]);
                const double bv = SRC ? (double)bb.v[v] : 0.0;
                const double r = bv - (c2d * (double)cen.v[v] - s);
                acc += r * r;
            }
        }
    }
    __shared__ double part[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ __launch_bounds__(256) void k_residual_final(const double *__restrict__ partials,
                                                        int n, double *__restrict__ out) {
    __shared__ double sh[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += partials[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(sh[0]);
}

hipError_t launch_residual_final(const double *partials, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, st, partials, n, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_residual(const Geom &g, const void *u, const void *b, double *partials,
                           double *out, hipStream_t st) {
    constexpr int V = 16 / sizeof(R);
    const int cpr = (g.n[0] + V - 1) / V;
    const int64_t total = (int64_t)cpr * g.n[1] * (g.ndim == 3 ? g.n[2] : 1);
    if (b)
        hipLaunchKernelGGL((k_residual<R, true>), dim3(kResidualGroups), dim3(256), 0, st, g,
                           (const R *)u, (const R *)b, partials, total, cpr);
    else
        hipLaunchKernelGGL((k_residual<R, false>), dim3(kResidualGroups), dim3(256), 0, st, g,
                           (const R *)u, (const R *)nullptr, partials, total, cpr);
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, st, partials, kResidualGroups,
                       out);
    return hipGetLastError();
}

template hipError_t launch_residual<float>(const Geom &, const void *, const void *, double *,
                                           double *, hipStream_t);
template hipError_t launch_residual<double>(const Geom &, const void *, const void *, double *,
                                            double *, hipStream_t);

}  // namespace jac
