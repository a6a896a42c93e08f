// Axis permutation of a dense row-major complex64 tensor: the transposes of
// transpose-transpose-GEMM-transpose (Sec. 1).  Output axes that stay
// adjacent and in order in the input are merged on the host, so a typical
// circuit tensor (all extents 2) becomes a permutation of a few wide axes.
// When every merged extent is a power of two (circuit tensors: every extent
// is 2) the permutation is a permutation of index bits and runs tiled: a
// block owns the elements whose index bits outside a small tile set are
// fixed, where the tile set holds the lowest input bits and the lowest output
// bits.  It reads them in input order (runs of >= 32 contiguous elements),
// stages them in LDS, and writes them in output order (runs of >= 32), so
// both sides of the HBM traffic are coalesced.  Otherwise, or for tensors
// too small to tile, one thread per output element gathers its input (the
// input offset is the dot product of the output coordinates with the input
// strides).
#include "common.hpp"
#include "gather.hpp"

#include <algorithm>
#include <cstring>

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

// Bit-permutation tile: u indexes the tile in input order (bit i of u is
// input bit tin[i], ascending), v in output order (bit i of v is output bit
// tout[i], ascending); the lowest tile bits are the lowest input / output
// bits.  Offsets are sums of per-bit terms, split into the thread's part
// (bits 0-7) and the uniform part of element e (bits 8 and up).
// The LDS slot of element u is linear over GF(2): slot = XOR of su[i] over
// the set bits i of u, where su[i] = 2^i, plus, for a tile bit that the
// output order puts among the lowest five, a low bit that the input order
// leaves free.  Then the 32 lanes of a half-wave hit 32 distinct 8-byte
// bank pairs both when they vary u's lowest five bits (reads from HBM) and
// when they vary v's lowest five bits (writes to HBM); sv[i] is the slot
// term of v bit i.
struct BitTile {
    int t;                 // tile bits, 8..12
    int nrest;             // bits enumerated by the block index
    int64_t in_u[12];      // input offset of u bit i
    int64_t out_v[12];     // output offset of v bit i
    int su[12];            // LDS slot term of u bit i
    int sv[12];            // LDS slot term of v bit i
    int64_t rest_in[48];   // input offset of block-index bit i
    int64_t rest_out[48];  // output offset of block-index bit i
};

constexpr int kTileMaxBits = 12;

template <int E>
__global__ __launch_bounds__(kThreads) void permute_tiled_kernel(const float2 *__restrict__ x,
                                                                 float2 *__restrict__ y, BitTile d) {
    __shared__ float2 lds[1 << kTileMaxBits];
    const int64_t bid = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    int64_t bin = 0, bout = 0;
    for (int i = 0; i < d.nrest; ++i)
        if ((bid >> i) & 1) {
            bin += d.rest_in[i];
            bout += d.rest_out[i];
        }
    const int tid = threadIdx.x;
    // reads: u = tid + 256 e
    int64_t tin = bin;
    int tsl = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if ((tid >> i) & 1) {
            tin += d.in_u[i];
            tsl ^= d.su[i];
        }
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int64_t off = tin;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (((e >> i) & 1) && 8 + i < d.t) off += d.in_u[8 + i];
        v[e] = x[off];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int sl = tsl;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (((e >> i) & 1) && 8 + i < d.t) sl ^= d.su[8 + i];
        lds[sl] = v[e];
    }
    __syncthreads();
    // writes: v = tid + 256 e
    int64_t tout = bout;
    tsl = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if ((tid >> i) & 1) {
            tout += d.out_v[i];
            tsl ^= d.sv[i];
        }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int64_t off = tout;
        int sl = tsl;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (((e >> i) & 1) && 8 + i < d.t) {
                off += d.out_v[8 + i];
                sl ^= d.sv[8 + i];
            }
        y[off] = lds[sl];
    }
}

// Full contraction sum_i x[i] * y[i] of two tensors over every label, x in
// y's index order only after a bit permutation: the tile of that
// permutation (x the input, y's order the output) is read from x in x's
// order into LDS, as the permute does, and each thread multiplies the
// elements it takes in y's order with y's (read in y's order) instead of
// writing them.  FP32 products and sums, one partial per block, reduced in
// a fixed order (deterministic).
template <int E>
__global__ __launch_bounds__(kThreads) void permuted_dot_kernel(const float2 *__restrict__ x,
                                                                const float2 *__restrict__ y,
                                                                float2 *__restrict__ partial, BitTile d) {
    __shared__ float2 lds[1 << kTileMaxBits];
    __shared__ float2 red[kThreads / 64];
    const int64_t bid = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    int64_t bin = 0, bout = 0;
    for (int i = 0; i < d.nrest; ++i)
        if ((bid >> i) & 1) {
            bin += d.rest_in[i];
            bout += d.rest_out[i];
        }
    const int tid = threadIdx.x;
    int64_t tin = bin;
    int tsl = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if ((tid >> i) & 1) {
            tin += d.in_u[i];
            tsl ^= d.su[i];
        }
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int64_t off = tin;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (((e >> i) & 1) && 8 + i < d.t) off += d.in_u[8 + i];
        v[e] = x[off];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int sl = tsl;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (((e >> i) & 1) && 8 + i < d.t) sl ^= d.su[8 + i];
        lds[sl] = v[e];
    }
    __syncthreads();
    int64_t tout = bout;
    tsl = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if ((tid >> i) & 1) {
            tout += d.out_v[i];
            tsl ^= d.sv[i];
        }
    float2 w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int64_t off = tout;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (((e >> i) & 1) && 8 + i < d.t) off += d.out_v[8 + i];
        w[e] = y[off];
    }
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int sl = tsl;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (((e >> i) & 1) && 8 + i < d.t) sl ^= d.sv[8 + i];
        const float2 a = lds[sl], b = w[e];
        re = fmaf(a.x, b.x, re);
        re = fmaf(-a.y, b.y, re);
        im = fmaf(a.x, b.y, im);
        im = fmaf(a.y, b.x, im);
    }
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
    }
    if ((tid & 63) == 0) red[tid >> 6] = make_float2(re, im);
    __syncthreads();
    if (tid == 0) {
        float2 acc = red[0];
        for (int w2 = 1; w2 < kThreads / 64; ++w2) {
            acc.x += red[w2].x;
            acc.y += red[w2].y;
        }
        partial[bid] = acc;
    }
}

// c[0] = sum of n partials: thread t adds partials t, t + 1024, ... in
// order (loads unrolled so that several are in flight), then a fixed tree.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void dot_reduce_kernel(const float2 *__restrict__ partial,
                                                                    int64_t n, float2 *__restrict__ c) {
    __shared__ float2 red[kReduceThreads / 64];
    const int tid = threadIdx.x;
    float re = 0.f, im = 0.f;
#pragma unroll 8
    for (int64_t i = tid; i < n; i += kReduceThreads) {
        const float2 p = partial[i];
        re += p.x;
        im += p.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
    }
    if ((tid & 63) == 0) red[tid >> 6] = make_float2(re, im);
    __syncthreads();
    if (tid == 0) {
        float2 acc = red[0];
        for (int w2 = 1; w2 < kReduceThreads / 64; ++w2) {
            acc.x += red[w2].x;
            acc.y += red[w2].y;
        }
        c[0] = acc;
    }
}

// Tile for a power-of-two permutation, or false when the tensor is too
// small to tile (fewer than 2^8 elements).
bool plan_bit_tile(const PermDesc &d, BitTile &b) {
    // output bit -> input bit (output axis rank-1 holds the lowest bits)
    int sigma[64], n = 0;
    for (int a = d.rank - 1; a >= 0; --a) {
        int s = 0;
        while ((int64_t(1) << s) < d.istride[a]) ++s;
        for (int j = 0; j < d.log2ext[a]; ++j) sigma[n++] = s + j;
    }
    if (n < 8) return false;
    int sinv[64];
    for (int o = 0; o < n; ++o) sinv[sigma[o]] = o;
    auto tile_bits = [&](int a, int c) {
        uint64_t m = 0;
        for (int i = 0; i < a; ++i) m |= uint64_t(1) << i;
        for (int i = 0; i < c; ++i) m |= uint64_t(1) << sigma[i];
        return m;
    };
    // grow the lowest input bits (a) and output bits (c) alternately while
    // the tile stays within 2^12 elements (a, c >= 6: 512-byte runs)
    int a = 0, c = 0;
    bool grew = true;
    while (grew && __builtin_popcountll(tile_bits(a, c)) < kTileMaxBits) {
        grew = false;
        if (a < n && __builtin_popcountll(tile_bits(a + 1, c)) <= kTileMaxBits) {
            ++a;
            grew = true;
        }
        if (c < n && __builtin_popcountll(tile_bits(a, c + 1)) <= kTileMaxBits) {
            ++c;
            grew = true;
        }
    }
    const uint64_t tm = tile_bits(a, c);
    const int t = __builtin_popcountll(tm);
    if (t < 8 || n - t > 46) return false;  // grid: 2^30 x 2^16 blocks at most
    memset(&b, 0, sizeof(b));
    b.t = t;
    int tin[kTileMaxBits], nt = 0;
    for (int p = 0; p < n; ++p)
        if ((tm >> p) & 1) tin[nt++] = p;
    int tout[kTileMaxBits];
    for (int i = 0; i < t; ++i) tout[i] = sinv[tin[i]];
    std::sort(tout, tout + t);
    int u_of_v[kTileMaxBits];
    for (int i = 0; i < t; ++i) {
        b.in_u[i] = int64_t(1) << tin[i];
        b.out_v[i] = int64_t(1) << tout[i];
        u_of_v[i] = (int)(std::find(tin, tin + t, sigma[tout[i]]) - tin);
    }
    // slot terms: u bits 0-4 are their own slot bits; each u bit >= 5 that is
    // one of v's lowest five bits also flips a slot bit among 0-4 that none
    // of v's lowest five bits uses
    for (int i = 0; i < t; ++i) b.su[i] = 1 << i;
    int used = 0;
    for (int i = 0; i < 5 && i < t; ++i)
        if (u_of_v[i] < 5) used |= 1 << u_of_v[i];
    for (int i = 0; i < 5 && i < t; ++i) {
        const int ub = u_of_v[i];
        if (ub < 5) continue;
        int f = 0;
        while (f < 5 && ((used >> f) & 1)) ++f;
        if (f < 5) {
            b.su[ub] |= 1 << f;
            used |= 1 << f;
        }
    }
    for (int i = 0; i < t; ++i) b.sv[i] = b.su[u_of_v[i]];
    b.nrest = 0;
    for (int p = 0; p < n; ++p)
        if (!((tm >> p) & 1)) {
            b.rest_in[b.nrest] = int64_t(1) << p;
            b.rest_out[b.nrest] = int64_t(1) << sinv[p];
            ++b.nrest;
        }
    return true;
}

}  // namespace

int64_t permuted_dot_partials(const PermDesc &d) {
    BitTile bt;
    if (!d.pow2 || !plan_bit_tile(d, bt)) return 0;
    return int64_t(1) << bt.nrest;
}

hipError_t launch_permuted_dot(const float2 *x, const float2 *y, const PermDesc &d, float2 *partial,
                               float2 *c, hipStream_t s) {
    BitTile bt;
    if (!d.pow2 || !plan_bit_tile(d, bt)) return hipErrorInvalidValue;
    const int64_t nblocks = int64_t(1) << bt.nrest;
    const unsigned gx = (unsigned)std::min<int64_t>(nblocks, int64_t(1) << 30);
    const unsigned gy = (unsigned)(nblocks / gx);
    const dim3 grid(gx, gy);
    switch (bt.t - 8) {
    case 0: hipLaunchKernelGGL(permuted_dot_kernel<1>, grid, dim3(kThreads), 0, s, x, y, partial, bt); break;
    case 1: hipLaunchKernelGGL(permuted_dot_kernel<2>, grid, dim3(kThreads), 0, s, x, y, partial, bt); break;
    case 2: hipLaunchKernelGGL(permuted_dot_kernel<4>, grid, dim3(kThreads), 0, s, x, y, partial, bt); break;
    case 3: hipLaunchKernelGGL(permuted_dot_kernel<8>, grid, dim3(kThreads), 0, s, x, y, partial, bt); break;
    default: hipLaunchKernelGGL(permuted_dot_kernel<16>, grid, dim3(kThreads), 0, s, x, y, partial, bt); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dot_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, partial, nblocks, c);
    return hipGetLastError();
}

hipError_t launch_permute(const float2 *x, float2 *y, int64_t total, const PermDesc &d,
                          hipStream_t s) {
    if (total == 0) return hipSuccess;
    BitTile bt;
    if (d.pow2 && plan_bit_tile(d, bt)) {
        const int64_t nblocks = int64_t(1) << bt.nrest;
        const unsigned gx = (unsigned)std::min<int64_t>(nblocks, int64_t(1) << 30);
        const unsigned gy = (unsigned)(nblocks / gx);
        const dim3 grid(gx, gy);
        switch (bt.t - 8) {
        case 0: hipLaunchKernelGGL(permute_tiled_kernel<1>, grid, dim3(kThreads), 0, s, x, y, bt); break;
        case 1: hipLaunchKernelGGL(permute_tiled_kernel<2>, grid, dim3(kThreads), 0, s, x, y, bt); break;
        case 2: hipLaunchKernelGGL(permute_tiled_kernel<4>, grid, dim3(kThreads), 0, s, x, y, bt); break;
        case 3: hipLaunchKernelGGL(permute_tiled_kernel<8>, grid, dim3(kThreads), 0, s, x, y, bt); break;
        default: hipLaunchKernelGGL(permute_tiled_kernel<16>, grid, dim3(kThreads), 0, s, x, y, bt); break;
        }
        return hipGetLastError();
    }
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
