// Grouped small contractions: many independent small pairwise contractions
// (the irregular shapes a sliced or batched circuit network is full of: a
// gate absorbed into a tensor of a few labels, outer products of vectors)
// in one launch instead of one (or three, with the TTGT transposes) each.
//
// Each item is C[o] = sum_s A[offA(o) + offA(s)] * B[offB(o) + offB(s)],
// o over the output elements of C (row-major in its labels), s over the
// summed labels; a label of C carries strides into A and / or B (both for a
// batch label), so no operand is permuted.  Workgroups are assigned to items
// by a prefix sum of their block counts; a thread owns one output element
// and sums in a fixed order (FP32 fused multiply-add, as the irregular-shape
// GEMM kernels).
#include "common.hpp"

namespace qce {

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void group_kernel(const SmallItem *__restrict__ items,
                                                         const int64_t *__restrict__ block_start,
                                                         int count) {
    // the item of this block: the last one whose first block is <= blockIdx.x
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block_start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const SmallItem &it = items[lo];
    const int64_t o = (b - block_start[lo]) * kThreads + threadIdx.x;
    if (o >= it.n_out) return;
    int64_t a = 0, c = 0, rem = o;
    for (int d = it.nd_out - 1; d >= 0; --d) {  // last output dimension fastest
        const int64_t e = it.out_ext[d];
        const int64_t v = rem % e;
        rem /= e;
        a += v * it.out_sa[d];
        c += v * it.out_sb[d];
    }
    // odometer over the summed dimensions (sum_* are stored fastest first)
    int64_t cnt[kSmallSum];
#pragma unroll
    for (int t = 0; t < kSmallSum; ++t) cnt[t] = 0;
    float re = 0.f, im = 0.f;
    for (int64_t s = 0; s < it.n_sum; ++s) {
        const float2 x = it.A[a], y = it.B[c];
        re = fmaf(x.x, y.x, re);
        re = fmaf(-x.y, y.y, re);
        im = fmaf(x.x, y.y, im);
        im = fmaf(x.y, y.x, im);
#pragma unroll
        for (int t = 0; t < kSmallSum; ++t) {
            if (t >= it.nd_sum) break;
            a += it.sum_sa[t];
            c += it.sum_sb[t];
            if (++cnt[t] < it.sum_ext[t]) break;
            cnt[t] = 0;
            a -= it.sum_ext[t] * it.sum_sa[t];
            c -= it.sum_ext[t] * it.sum_sb[t];
        }
    }
    it.C[o] = make_float2(re, im);
}

}  // namespace

hipError_t launch_group(const SmallItem *items, const int64_t *block_start, int count,
                        int64_t total_blocks, hipStream_t s) {
    if (count == 0 || total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(group_kernel, dim3((unsigned)total_blocks), dim3(kThreads), 0, s, items,
                       block_start, count);
    return hipGetLastError();
}

}  // namespace qce
