// Axis permutation of a dense row-major complex64 tensor: the transposes of
// transpose-transpose-GEMM-transpose (Sec. 1).  Output axes that stay
// adjacent and in order in the input are merged on the host, so a typical
// circuit tensor (all extents 2) becomes a permutation of a few wide axes.
// One thread per output element (coalesced writes); the input offset is the
// dot product of the output coordinates with the input strides.  When every
// merged extent is a power of two the coordinates come from shifts and masks.
#include "common.hpp"

namespace qce {

namespace {

constexpr int kThreads = 256;

template <bool POW2>
__global__ __launch_bounds__(kThreads) void permute_kernel(const float2 *__restrict__ x,
                                                           float2 *__restrict__ y, int64_t total,
                                                           PermDesc d) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < total; o += stride) {
        int64_t rem = o, off = 0;
        for (int a = d.rank - 1; a >= 0; --a) {
            int64_t c;
            if (POW2) {
                c = rem & (d.ext[a] - 1);
                rem >>= d.log2ext[a];
            } else {
                c = rem % d.ext[a];
                rem /= d.ext[a];
            }
            off += c * d.istride[a];
        }
        y[o] = x[off];
    }
}

}  // namespace

hipError_t launch_permute(const float2 *x, float2 *y, int64_t total, const PermDesc &d,
                          hipStream_t s) {
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + kThreads - 1) / kThreads;
    if (blocks > 65536) blocks = 65536;
    if (d.pow2)
        hipLaunchKernelGGL(permute_kernel<true>, dim3((unsigned)blocks), dim3(kThreads), 0, s, x, y,
                           total, d);
    else
        hipLaunchKernelGGL(permute_kernel<false>, dim3((unsigned)blocks), dim3(kThreads), 0, s, x, y,
                           total, d);
    return hipGetLastError();
}

}  // namespace qce
