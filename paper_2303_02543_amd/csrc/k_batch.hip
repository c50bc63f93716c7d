// Device-side bookkeeping of the batched solver: per-grid activity, the
// relative-residual stop rule in FP64, and the pass / sweep counters.  Every
// decision is taken on the GPU, so a whole check interval (its passes, the
// counter updates and the convergence test) can be captured in one hipGraph
// and replayed without the host looking at any result in between.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "jacobi_internal.h"
#include "kernels.h"

namespace jac {

// Stop rule (reading of the relative-residual test; not in the paper): the
// residual of grid g's state after k sweeps is checked at k = 0, R, 2R, ...
// and at the cap.  res_0 == 0: converged at 0 sweeps.  Non-finite: diverged.
// Otherwise rel = res_k / res_0 and the grid stops, converged, at the first
// checked k > 0 with rel <= tol; at the final check (the cap) it stops with
// status "max sweeps".  A stopped grid keeps the state it was checked on.
__global__ void k_batch_init(int count, BatchState st) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        *st.pass_count = 0;
        *st.k_now = 0;
    }
    if (g < count) {
        st.active[g] = 1;
        st.status[g] = 0;
        st.sweeps[g] = 0;
        st.rel[g] = 0.0;
        st.res0[g] = 0.0;
        st.res[g] = 0.0;
        st.final_buf[g] = 0;
    }
}

__global__ void k_batch_advance(BatchState st, int sweeps) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *st.pass_count += 1;
        *st.k_now += sweeps;
    }
}

// One workgroup per grid: sum the grid's residual partials in a fixed order
// (per-thread strided sums, then a fixed LDS tree), then apply the stop rule.
__global__ __launch_bounds__(256) void k_batch_check(const int *__restrict__ prefix,
                                                     const double *__restrict__ partials,
                                                     BatchState st, double tol, int final_check) {
    __shared__ double sh[256];
    const int g = blockIdx.x;
    if (!st.active[g]) return;
    double a = 0.0;
    for (int i = prefix[g] + (int)threadIdx.x; i < prefix[g + 1]; i += 256) a += partials[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double res = sqrt(sh[0]);
    const long long k = *st.k_now;
    const int par = *st.pass_count & 1;  // buffer holding the checked state
    st.res[g] = res;
    if (k == 0) st.res0[g] = res;
    const double r0 = st.res0[g];
    int stop = 0;
    if (!isfinite(res)) {
        st.status[g] = 3;  // diverged
        st.rel[g] = res;
        stop = 1;
    } else if (r0 == 0.0) {
        st.status[g] = 1;  // converged (zero residual)
        st.rel[g] = 0.0;
        stop = 1;
    } else {
        const double rel = res / r0;
        st.rel[g] = rel;
        if (k > 0 && rel <= tol) {
            st.status[g] = 1;
            stop = 1;
        } else if (final_check) {
            st.status[g] = 2;  // max sweeps
            stop = 1;
        }
    }
    if (stop) {
        st.active[g] = 0;
        st.sweeps[g] = k;
        st.final_buf[g] = par;
    }
}

hipError_t launch_batch_init(int count, const BatchState &st, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_init, dim3((count + 255) / 256), dim3(256), 0, s, count, st);
    return hipGetLastError();
}

hipError_t launch_batch_advance(const BatchState &st, int sweeps, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, st, sweeps);
    return hipGetLastError();
}

hipError_t launch_batch_check(const int *prefix, const double *partials, int count,
                              const BatchState &st, double tol, bool final_check, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_check, dim3(count), dim3(256), 0, s, prefix, partials, st, tol,
                       final_check ? 1 : 0);
    return hipGetLastError();
}

}  // namespace jac
