// FP64 reductions on the device: the sum of sliced amplitudes (Sec. 5.3) and
// the terms of the fidelity between two amplitude vectors.  These are the
// only FP64 arithmetic on the GPU path.  The fidelity sums are deterministic:
// per-block partial sums in a fixed order, then one block adds the partials
// in block order.
#include "common.hpp"

namespace qce {

namespace {

constexpr int kThreads = 256;

__global__ void accumulate_kernel(const float2 *src, double *acc2) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const float2 v = *src;
        acc2[0] += (double)v.x;
        acc2[1] += (double)v.y;
    }
}

__device__ inline double block_sum_d(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; ++i) r += sh[i];
    return r;
}

__global__ __launch_bounds__(kThreads) void fidelity_partial_kernel(const float2 *a,
                                                                    const float2 *b, int64_t n,
                                                                    double *partials) {
    __shared__ double sh[kThreads / 64];
    double ore = 0.0, oim = 0.0, na = 0.0, nb = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const float2 x = a[i], y = b[i];
        const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
        // conj(b) * a
        ore += yr * xr + yi * xi;
        oim += yr * xi - yi * xr;
        na += xr * xr + xi * xi;
        nb += yr * yr + yi * yi;
    }
    ore = block_sum_d(ore, sh);
    oim = block_sum_d(oim, sh);
    na = block_sum_d(na, sh);
    nb = block_sum_d(nb, sh);
    if (threadIdx.x == 0) {
        double *p = partials + 4 * blockIdx.x;
        p[0] = ore;
        p[1] = oim;
        p[2] = na;
        p[3] = nb;
    }
}

__global__ void fidelity_final_kernel(const double *partials, int nblocks, double *out4) {
    if (threadIdx.x < 4 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nblocks; ++i) s += partials[4 * i + threadIdx.x];
        out4[threadIdx.x] = s;
    }
}

// Sum of n complex64 values in FP64 (the slice amplitudes of a batched
// pass): per-block partial sums in a fixed order, then one block adds them
// in block order to the accumulator.
__global__ __launch_bounds__(kThreads) void sum_partial_kernel(const float2 *src, int64_t n,
                                                               double *partials) {
    __shared__ double sh[kThreads / 64];
    double re = 0.0, im = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const float2 v = src[i];
        re += (double)v.x;
        im += (double)v.y;
    }
    re = block_sum_d(re, sh);
    im = block_sum_d(im, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = re;
        partials[2 * blockIdx.x + 1] = im;
    }
}

__global__ void sum_final_kernel(const double *partials, int nblocks, double *acc2) {
    if (threadIdx.x < 2 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nblocks; ++i) s += partials[2 * i + threadIdx.x];
        acc2[threadIdx.x] += s;
    }
}

}  // namespace

hipError_t launch_accumulate_n_f64(const float2 *src, int64_t n, double *partials, int nblocks,
                                   double *acc2, hipStream_t s) {
    hipLaunchKernelGGL(sum_partial_kernel, dim3(nblocks), dim3(kThreads), 0, s, src, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(64), 0, s, partials, nblocks, acc2);
    return hipGetLastError();
}

hipError_t launch_accumulate_f64(const float2 *src, double *acc2, hipStream_t s) {
    hipLaunchKernelGGL(accumulate_kernel, dim3(1), dim3(64), 0, s, src, acc2);
    return hipGetLastError();
}

hipError_t launch_fidelity_f64(const float2 *a, const float2 *b, int64_t n, double *partials,
                               int nblocks, double *out4, hipStream_t s) {
    hipLaunchKernelGGL(fidelity_partial_kernel, dim3(nblocks), dim3(kThreads), 0, s, a, b, n,
                       partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fidelity_final_kernel, dim3(1), dim3(64), 0, s, partials, nblocks, out4);
    return hipGetLastError();
}

}  // namespace qce
