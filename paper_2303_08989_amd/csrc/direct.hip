// Irregular-shape complex GEMM: a bandwidth-bound FP32 kernel for shapes
// the tiled matrix-core kernels would pad heavily (a thin side, a tiny k, or
// a small output with a long k).  The paper runs a specialised kernel for
// such shapes in every computing mode (Sec. 5.1.2 and its appendix); so does
// this library.
//
// Operand views are those of the split kernel: PA[i][l] (i < m) and PB[j][l]
// (j < n) read straight from the stored matrices.  A block owns an output
// tile of TI x TJ elements and a range of k; each output is shared by KL
// threads that take every KL-th k-value of the range and are then summed in
// LDS in a fixed order.  With several k-ranges the partial tiles go to a
// workspace and a second kernel adds them in k order, so results are
// deterministic.  Arithmetic: FP32 products with FP32 fused accumulation.
//
// Short k (k <= 16, e.g. a gate absorbed into a large tensor, or an outer
// product over a few labels) needs no reduction across threads; there the
// cost is streaming the large operand and C, so a thread keeps a register
// tile along the short side: direct_rows_kernel gives a thread one row and
// up to 8 columns (its A values are read once for all of them; the B values
// are the same for the whole block), direct_cols_kernel gives a thread one
// column and every row of a short m (it writes m contiguous outputs).
#include "common.hpp"

#include <algorithm>

namespace qce {

namespace {

constexpr int kThreads = 256;

__device__ inline float2 load_view(const float2 *p, int64_t ld, int kcontig, int conj, int64_t r,
                                   int64_t l) {
    float2 v = kcontig ? p[l + r * ld] : p[r + l * ld];
    if (conj) v.y = -v.y;
    return v;
}

// Batched launches: entry blockIdx.z works on its own operands, C and
// partial tiles.
__device__ inline void select_entry(DirectArgs &d) {
    const int64_t z = blockIdx.z;
    d.A += z * d.bsA;
    d.B += z * d.bsB;
    d.C += z * d.bsC;
    if (d.partial) d.partial += z * d.bsPartial;
}

__global__ __launch_bounds__(kThreads) void direct_kernel(DirectArgs d) {
    __shared__ float2 red[kThreads];
    select_entry(d);
    const int t = threadIdx.x;
    const int kl = t % d.kl;
    const int o = t / d.kl;           // output within the tile
    const int ti = o % d.ti, tj = o / d.ti;
    const int64_t tiles_i = (d.m + d.ti - 1) / d.ti;
    const int64_t tile = blockIdx.x;
    const int64_t i = (tile % tiles_i) * d.ti + ti;
    const int64_t j = (tile / tiles_i) * d.tj + tj;
    const int64_t k0 = (int64_t)blockIdx.y * d.kchunk;
    const int64_t k1 = min(d.k, k0 + d.kchunk);
    float re = 0.f, im = 0.f;
    if (i < d.m && j < d.n) {
        for (int64_t l = k0 + kl; l < k1; l += d.kl) {
            const float2 a = load_view(d.A, d.lda, d.a_kcontig, d.a_conj, i, l);
            const float2 b = load_view(d.B, d.ldb, d.b_kcontig, d.b_conj, j, l);
            re = fmaf(a.x, b.x, re);
            re = fmaf(-a.y, b.y, re);
            im = fmaf(a.x, b.y, im);
            im = fmaf(a.y, b.x, im);
        }
    }
    if (d.kl > 1) {
        red[t] = make_float2(re, im);
        __syncthreads();
        for (int s = d.kl >> 1; s > 0; s >>= 1) {
            if (kl < s) {
                const float2 u = red[t + s];
                red[t].x += u.x;
                red[t].y += u.y;
            }
            __syncthreads();
        }
        re = red[t].x;
        im = red[t].y;
    }
    if (kl != 0 || i >= d.m || j >= d.n) return;
    if (gridDim.y > 1) {
        d.partial[(int64_t)blockIdx.y * d.m * d.n + i + j * d.m] = make_float2(re, im);
        return;
    }
    float2 out = make_float2(d.alpha.x * re - d.alpha.y * im, d.alpha.x * im + d.alpha.y * re);
    if (d.alpha.x == 1.f && d.alpha.y == 0.f) out = make_float2(re, im);
    float2 *cp = d.C + i + j * d.ldc;
    if (!d.beta_zero) {
        const float2 c = *cp;
        out.x += d.beta.x * c.x - d.beta.y * c.y;
        out.y += d.beta.x * c.y + d.beta.y * c.x;
    }
    *cp = out;
}

__global__ __launch_bounds__(kThreads) void direct_reduce_kernel(DirectArgs d, int splits) {
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o >= d.m * d.n) return;
    select_entry(d);
    float re = 0.f, im = 0.f;
    for (int s = 0; s < splits; ++s) {
        const float2 p = d.partial[(int64_t)s * d.m * d.n + o];
        re += p.x;
        im += p.y;
    }
    const int64_t i = o % d.m, j = o / d.m;
    float2 out = make_float2(d.alpha.x * re - d.alpha.y * im, d.alpha.x * im + d.alpha.y * re);
    if (d.alpha.x == 1.f && d.alpha.y == 0.f) out = make_float2(re, im);
    float2 *cp = d.C + i + j * d.ldc;
    if (!d.beta_zero) {
        const float2 c = *cp;
        out.x += d.beta.x * c.x - d.beta.y * c.y;
        out.y += d.beta.x * c.y + d.beta.y * c.x;
    }
    *cp = out;
}

__device__ inline float2 scale_out(const DirectArgs &d, float re, float im, float2 *cp) {
    float2 out = make_float2(d.alpha.x * re - d.alpha.y * im, d.alpha.x * im + d.alpha.y * re);
    if (d.alpha.x == 1.f && d.alpha.y == 0.f) out = make_float2(re, im);
    if (!d.beta_zero) {
        const float2 c = *cp;
        out.x += d.beta.x * c.x - d.beta.y * c.y;
        out.y += d.beta.x * c.y + d.beta.y * c.x;
    }
    return out;
}

// VEC: A's columns hold its rows contiguously (op(A) = A) and C's rows are
// contiguous too, both 16-byte aligned with m even: a thread takes two
// consecutive rows, one 16-byte load per k-value and one 16-byte store per
// column (each row's products are added in the same order as one row per
// thread).
template <int JT, bool VEC>
__global__ __launch_bounds__(kThreads) void direct_rows_kernel(DirectArgs d) {
    constexpr int RT = VEC ? 2 : 1;  // rows per thread
    select_entry(d);
    const int64_t mt = (d.m + RT - 1) / RT;
    const int64_t row_blocks = (mt + kThreads - 1) / kThreads;
    const int64_t b = blockIdx.x;
    const int64_t i = ((b % row_blocks) * kThreads + threadIdx.x) * RT;
    const int64_t j0 = (b / row_blocks) * JT;
    if (i >= d.m) return;
    float re[RT][JT], im[RT][JT];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) re[rr][jj] = im[rr][jj] = 0.f;
    for (int64_t l = 0; l < d.k; ++l) {
        float2 a[RT];
        if constexpr (VEC) {
            const float4 v = *reinterpret_cast<const float4 *>(d.A + i + l * d.lda);
            a[0] = make_float2(v.x, d.a_conj ? -v.y : v.y);
            a[1] = make_float2(v.z, d.a_conj ? -v.w : v.w);
        } else {
            a[0] = load_view(d.A, d.lda, d.a_kcontig, d.a_conj, i, l);
        }
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
            if (j0 + jj >= d.n) break;
            const float2 bv = load_view(d.B, d.ldb, d.b_kcontig, d.b_conj, j0 + jj, l);
#pragma unroll
            for (int rr = 0; rr < RT; ++rr) {
                re[rr][jj] = fmaf(a[rr].x, bv.x, re[rr][jj]);
                re[rr][jj] = fmaf(-a[rr].y, bv.y, re[rr][jj]);
                im[rr][jj] = fmaf(a[rr].x, bv.y, im[rr][jj]);
                im[rr][jj] = fmaf(a[rr].y, bv.x, im[rr][jj]);
            }
        }
    }
#pragma unroll
    for (int jj = 0; jj < JT; ++jj) {
        if (j0 + jj >= d.n) break;
        float2 *cp = d.C + i + (j0 + jj) * d.ldc;
        if constexpr (VEC) {
            const float2 o0 = scale_out(d, re[0][jj], im[0][jj], cp);
            const float2 o1 = scale_out(d, re[1][jj], im[1][jj], cp + 1);
            *reinterpret_cast<float4 *>(cp) = make_float4(o0.x, o0.y, o1.x, o1.y);
        } else {
            *cp = scale_out(d, re[0][jj], im[0][jj], cp);
        }
    }
}

// VEC: column j of B holds its k values contiguously and column j of C its
// m values, both 16-byte aligned with k and m even: two complex values per
// load and per store (the products are added in the same order).
template <int MT, bool VEC>
__global__ __launch_bounds__(kThreads) void direct_cols_kernel(DirectArgs d) {
    select_entry(d);
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= d.n) return;
    float re[MT], im[MT];
#pragma unroll
    for (int ii = 0; ii < MT; ++ii) re[ii] = im[ii] = 0.f;
    auto add = [&](int64_t l, float2 bv) {
#pragma unroll
        for (int ii = 0; ii < MT; ++ii) {
            if (ii >= d.m) break;
            const float2 a = load_view(d.A, d.lda, d.a_kcontig, d.a_conj, ii, l);
            re[ii] = fmaf(a.x, bv.x, re[ii]);
            re[ii] = fmaf(-a.y, bv.y, re[ii]);
            im[ii] = fmaf(a.x, bv.y, im[ii]);
            im[ii] = fmaf(a.y, bv.x, im[ii]);
        }
    };
    if constexpr (VEC) {
        const float4 *bp = reinterpret_cast<const float4 *>(d.B + j * d.ldb);
        for (int64_t l2 = 0; l2 < d.k / 2; ++l2) {
            const float4 v = bp[l2];
            add(2 * l2, make_float2(v.x, d.b_conj ? -v.y : v.y));
            add(2 * l2 + 1, make_float2(v.z, d.b_conj ? -v.w : v.w));
        }
#pragma unroll
        for (int ii = 0; ii < MT; ii += 2) {
            if (ii >= d.m) break;
            float2 *cp = d.C + ii + j * d.ldc;
            const float2 o0 = scale_out(d, re[ii], im[ii], cp);
            const float2 o1 = scale_out(d, re[ii + 1], im[ii + 1], cp + 1);
            *reinterpret_cast<float4 *>(cp) = make_float4(o0.x, o0.y, o1.x, o1.y);
        }
    } else {
        for (int64_t l = 0; l < d.k; ++l) add(l, load_view(d.B, d.ldb, d.b_kcontig, d.b_conj, j, l));
#pragma unroll
        for (int ii = 0; ii < MT; ++ii) {
            if (ii >= d.m) break;
            float2 *cp = d.C + ii + j * d.ldc;
            *cp = scale_out(d, re[ii], im[ii], cp);
        }
    }
}

constexpr int64_t kShortK = 16;

int pow2_at_least(int64_t x) {
    int p = 1;
    while (p < x) p *= 2;
    return p;
}

}  // namespace

void direct_plan(DirectArgs &d, int64_t &splits) {
    // threads per output: enough to fill the block when the output is small,
    // and to spread a long k
    const int64_t mn = d.m * d.n;
    int kl = 1;
    while (kl < kThreads && mn * kl < kThreads && d.k >= 8 * (int64_t)kl) kl *= 2;
    d.kl = kl;
    const int outs = kThreads / kl;  // outputs per block
    // tile shape: rows first (coalesced column-major access)
    int ti = 1;
    while (ti < outs && ti < d.m) ti *= 2;
    if (ti > outs) ti = outs;
    d.ti = ti;
    d.tj = outs / ti;
    const int64_t tiles = ((d.m + d.ti - 1) / d.ti) * ((d.n + d.tj - 1) / d.tj);
    // split k while the grid is small and k is long
    splits = 1;
    while (tiles * splits < 1024 && d.k / (splits * 2) >= 256 * (int64_t)kl / 4 && splits < 4096)
        splits *= 2;
    d.kchunk = (d.k + splits - 1) / splits;
    splits = (d.k + d.kchunk - 1) / d.kchunk;
    if (splits < 1) splits = 1;
}

size_t direct_ws_bytes(int64_t m, int64_t n, int64_t k, int batch) {
    if (k <= kShortK) return 0;
    DirectArgs d{};
    d.m = m;
    d.n = n;
    d.k = k;
    int64_t splits = 1;
    direct_plan(d, splits);
    return splits > 1 ? (size_t)std::max(1, batch) * (size_t)splits * (size_t)(m * n) * sizeof(float2) : 0;
}

hipError_t launch_direct(DirectArgs d, hipStream_t s) {
    const unsigned nz = (unsigned)std::max(1, d.batch);
    if (d.k <= kShortK) {
        if (d.m >= 32) {
            auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
            const bool vec = !d.a_kcontig && d.lda % 2 == 0 && al16(d.A) && (nz == 1 || d.bsA % 2 == 0) &&
                             d.m % 2 == 0 && d.ldc % 2 == 0 && al16(d.C) && (nz == 1 || d.bsC % 2 == 0);
            const int jt = std::min(8, pow2_at_least(d.n));
            const int64_t mt = vec ? d.m / 2 : d.m;
            const int64_t blocks = ((mt + kThreads - 1) / kThreads) * ((d.n + jt - 1) / jt);
            const dim3 g((unsigned)blocks, 1, nz), t(kThreads);
            switch (jt * (vec ? -1 : 1)) {
            case 1: hipLaunchKernelGGL((direct_rows_kernel<1, false>), g, t, 0, s, d); break;
            case 2: hipLaunchKernelGGL((direct_rows_kernel<2, false>), g, t, 0, s, d); break;
            case 4: hipLaunchKernelGGL((direct_rows_kernel<4, false>), g, t, 0, s, d); break;
            case 8: hipLaunchKernelGGL((direct_rows_kernel<8, false>), g, t, 0, s, d); break;
            case -1: hipLaunchKernelGGL((direct_rows_kernel<1, true>), g, t, 0, s, d); break;
            case -2: hipLaunchKernelGGL((direct_rows_kernel<2, true>), g, t, 0, s, d); break;
            case -4: hipLaunchKernelGGL((direct_rows_kernel<4, true>), g, t, 0, s, d); break;
            default: hipLaunchKernelGGL((direct_rows_kernel<8, true>), g, t, 0, s, d); break;
            }
        } else {
            const dim3 g((unsigned)((d.n + kThreads - 1) / kThreads), 1, nz), t(kThreads);
            auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
            const bool vec = d.b_kcontig && d.k % 2 == 0 && d.ldb % 2 == 0 && al16(d.B) &&
                             (nz == 1 || d.bsB % 2 == 0) && d.m % 2 == 0 && d.ldc % 2 == 0 && al16(d.C) &&
                             (nz == 1 || d.bsC % 2 == 0);
            switch (pow2_at_least(d.m) * (vec ? -1 : 1)) {
            case 1: hipLaunchKernelGGL((direct_cols_kernel<1, false>), g, t, 0, s, d); break;
            case 2: hipLaunchKernelGGL((direct_cols_kernel<2, false>), g, t, 0, s, d); break;
            case 4: hipLaunchKernelGGL((direct_cols_kernel<4, false>), g, t, 0, s, d); break;
            case 8: hipLaunchKernelGGL((direct_cols_kernel<8, false>), g, t, 0, s, d); break;
            case 16: hipLaunchKernelGGL((direct_cols_kernel<16, false>), g, t, 0, s, d); break;
            case 32: hipLaunchKernelGGL((direct_cols_kernel<32, false>), g, t, 0, s, d); break;
            case -2: hipLaunchKernelGGL((direct_cols_kernel<2, true>), g, t, 0, s, d); break;
            case -4: hipLaunchKernelGGL((direct_cols_kernel<4, true>), g, t, 0, s, d); break;
            case -8: hipLaunchKernelGGL((direct_cols_kernel<8, true>), g, t, 0, s, d); break;
            case -16: hipLaunchKernelGGL((direct_cols_kernel<16, true>), g, t, 0, s, d); break;
            default: hipLaunchKernelGGL((direct_cols_kernel<32, true>), g, t, 0, s, d); break;
            }
        }
        return hipGetLastError();
    }
    int64_t splits = 1;
    direct_plan(d, splits);
    const int64_t tiles = ((d.m + d.ti - 1) / d.ti) * ((d.n + d.tj - 1) / d.tj);
    d.bsPartial = splits * d.m * d.n;
    hipLaunchKernelGGL(direct_kernel, dim3((unsigned)tiles, (unsigned)splits, nz), dim3(kThreads), 0, s, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    const int64_t mn = d.m * d.n;
    hipLaunchKernelGGL(direct_reduce_kernel, dim3((unsigned)((mn + kThreads - 1) / kThreads), 1, nz),
                       dim3(kThreads), 0, s, d, (int)splits);
    return hipGetLastError();
}

}  // namespace qce
