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
//
// A small output with a long k (the adjoint of a gate against a large
// tensor, the last thin contraction of a slice) takes direct_outer_kernel:
// every thread accumulates a whole output tile over its own k-values, so
// each operand element is read once.
#include "common.hpp"

#include <algorithm>

namespace qce {

namespace {

constexpr int kThreads = 256;
// k-values (direct_kernel) or k-ranges (direct_reduce_kernel) a thread has
// in flight at once
constexpr int kUnroll = 8;
// longest k of the short-k kernels (direct_rows_kernel, direct_cols_kernel)
constexpr int kShortK = 16;

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
        // kUnroll k-values per round: every load of a round is issued before
        // its products, which then run in k order (the same sequence of
        // fused multiply-adds as one k-value at a time)
        const int64_t step = d.kl;
        int64_t l = k0 + kl;
        for (; l + (kUnroll - 1) * step < k1; l += kUnroll * step) {
            float2 a[kUnroll], b[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                a[u] = load_view(d.A, d.lda, d.a_kcontig, d.a_conj, i, l + u * step);
                b[u] = load_view(d.B, d.ldb, d.b_kcontig, d.b_conj, j, l + u * step);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                re = fmaf(a[u].x, b[u].x, re);
                re = fmaf(-a[u].y, b[u].y, re);
                im = fmaf(a[u].x, b[u].y, im);
                im = fmaf(a[u].y, b[u].x, im);
            }
        }
        for (; l < k1; l += step) {
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

// The partial tiles of the k-ranges added up: `ways` threads per output
// (a power of two), thread w adding ranges w, w + ways, ... in order
// (kUnroll loads in flight), then the ways sums pairwise in LDS in a fixed
// order, so the result does not depend on timing.
__global__ __launch_bounds__(kThreads) void direct_reduce_kernel(DirectArgs d, int splits, int ways) {
    __shared__ float2 red[kThreads];
    select_entry(d);
    const int t = threadIdx.x;
    const int w = t & (ways - 1);
    const int64_t mn = d.m * d.n;
    const int64_t o = (int64_t)blockIdx.x * (kThreads / ways) + t / ways;
    float re = 0.f, im = 0.f;
    if (o < mn) {
        const float2 *p = d.partial + o;
        int s = w;
        for (; s + (kUnroll - 1) * ways < splits; s += kUnroll * ways) {
            float2 v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) v[u] = p[(int64_t)(s + u * ways) * mn];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                re += v[u].x;
                im += v[u].y;
            }
        }
        for (; s < splits; s += ways) {
            const float2 v = p[(int64_t)s * mn];
            re += v.x;
            im += v.y;
        }
    }
    if (ways > 1) {
        red[t] = make_float2(re, im);
        __syncthreads();
        for (int h = ways >> 1; h > 0; h >>= 1) {
            if (w < h) {
                const float2 u = red[t + h];
                red[t].x += u.x;
                red[t].y += u.y;
            }
            __syncthreads();
        }
        re = red[t].x;
        im = red[t].y;
    }
    if (w != 0 || o >= mn) return;
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

// Sum over the 64 lanes of a wave in a fixed order (an inclusive scan by DPP
// row shifts and row broadcasts; lanes without a source add +0), the total
// in lane 63.
__device__ inline float lane_scan_f(float v) {
    auto add = [](float x, int y) { return x + __int_as_float(y); };
    v = add(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));  // row_shr:1
    v = add(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, false));  // row_shr:2
    v = add(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, false));  // row_shr:4
    v = add(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));  // row_shr:8
    v = add(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = add(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// A small output (one tile of kOuterTiles, or up to four 8 x 8, 4 x 16 or
// 16 x 4 tiles) with a long k: every thread of a group accumulates the
// group's whole TM x TN output tile over its own k-values (for each, TM
// values of op(A) and TN of op(B), every element read once), two k-values
// in flight; the k-values of a block are split over the group's d.kl
// threads (whole waves).  The tile is then added up over each wave's lanes
// (lane_scan_f) and over the group's waves in LDS, in a fixed order.
// d.ti x d.tj groups of tiles cover the output (groups along m first).
// VEC: both operand views hold a k-value's rows contiguously
// (P[r][l] = x[r + l ld]), 16-byte aligned with even leading dimensions:
// the values are read two at a time.
template <int TM, int TN, bool VEC>
__global__ __launch_bounds__(kThreads) void direct_outer_kernel(DirectArgs d) {
    __shared__ float red[kThreads / 64][2 * TM * TN];
    select_entry(d);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int kl = d.kl, gi = d.ti;
    const int g = t / kl, q = t % kl;
    const int64_t i0 = (int64_t)(g % gi) * TM, j0 = (int64_t)(g / gi) * TN;
    const int64_t k0 = (int64_t)blockIdx.y * d.kchunk;
    const int64_t k1 = min(d.k, k0 + d.kchunk);
    float re[TM][TN], im[TM][TN];
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) re[r][c] = im[r][c] = 0.f;
    auto fma_tile = [&](const float2 (&a)[TM], const float2 (&b)[TN]) {
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int c = 0; c < TN; ++c) {
                re[r][c] = fmaf(a[r].x, b[c].x, re[r][c]);
                re[r][c] = fmaf(-a[r].y, b[c].y, re[r][c]);
                im[r][c] = fmaf(a[r].x, b[c].y, im[r][c]);
                im[r][c] = fmaf(a[r].y, b[c].x, im[r][c]);
            }
    };
    // rows i0 + r >= m and columns j0 + c >= n read nothing (the bounds are
    // uniform over a group, hence over a wave)
    auto load = [&](float2 (&a)[TM], float2 (&b)[TN], int64_t l) {
        if constexpr (VEC) {
            // rows r, r + 1 of column l: one 16-byte load (i0 and the
            // leading dimensions are even, the operands 16-byte aligned)
            auto pair = [](const float2 *p, int64_t ld, int conj, int64_t rows, int64_t r, int64_t l,
                           float2 &x, float2 &y) {
                const float2 *q = p + r + l * ld;
                if (r + 1 < rows) {
                    const float4 v = *reinterpret_cast<const float4 *>(q);
                    x = make_float2(v.x, conj ? -v.y : v.y);
                    y = make_float2(v.z, conj ? -v.w : v.w);
                } else {
                    x = r < rows ? *q : make_float2(0.f, 0.f);
                    if (conj) x.y = -x.y;
                    y = make_float2(0.f, 0.f);
                }
            };
#pragma unroll
            for (int r = 0; r < TM; r += 2) pair(d.A, d.lda, d.a_conj, d.m, i0 + r, l, a[r], a[r + 1]);
#pragma unroll
            for (int c = 0; c < TN; c += 2) pair(d.B, d.ldb, d.b_conj, d.n, j0 + c, l, b[c], b[c + 1]);
        } else {
#pragma unroll
            for (int r = 0; r < TM; ++r)
                a[r] = i0 + r < d.m ? load_view(d.A, d.lda, d.a_kcontig, d.a_conj, i0 + r, l)
                                    : make_float2(0.f, 0.f);
#pragma unroll
            for (int c = 0; c < TN; ++c)
                b[c] = j0 + c < d.n ? load_view(d.B, d.ldb, d.b_kcontig, d.b_conj, j0 + c, l)
                                    : make_float2(0.f, 0.f);
        }
    };
    int64_t l = k0 + q;
    for (; l + kl < k1; l += 2 * (int64_t)kl) {
        float2 a0[TM], b0[TN], a1[TM], b1[TN];
        load(a0, b0, l);
        load(a1, b1, l + kl);
        fma_tile(a0, b0);
        fma_tile(a1, b1);
    }
    if (l < k1) {
        float2 a0[TM], b0[TN];
        load(a0, b0, l);
        fma_tile(a0, b0);
    }
    // each wave's sums (lane 63 holds them after the scan)
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) {
            const float sr = lane_scan_f(re[r][c]), si = lane_scan_f(im[r][c]);
            if (lane == 63) {
                red[wv][2 * (r + c * TM)] = sr;
                red[wv][2 * (r + c * TM) + 1] = si;
            }
        }
    __syncthreads();
    // thread t: output (r, c) of group t / (TM TN), its waves added in order
    const int groups = kThreads / kl;
    if (t >= groups * TM * TN) return;
    const int g2 = t / (TM * TN), o2 = t % (TM * TN);
    const int r = o2 % TM, c = o2 / TM;
    const int64_t i = (int64_t)(g2 % gi) * TM + r, j = (int64_t)(g2 / gi) * TN + c;
    if (i >= d.m || j >= d.n) return;
    const int w0 = g2 * (kl / 64);
    float sr = 0.f, si = 0.f;
    for (int x = 0; x < kl / 64; ++x) {
        sr += red[w0 + x][2 * o2];
        si += red[w0 + x][2 * o2 + 1];
    }
    if (gridDim.y > 1) {
        d.partial[(int64_t)blockIdx.y * d.m * d.n + i + j * d.m] = make_float2(sr, si);
        return;
    }
    float2 *cp = d.C + i + j * d.ldc;
    *cp = scale_out(d, sr, si, cp);
}

// The 8 x 8 tile of direct_outer_kernel with VEC operands, four lanes per
// k-value: lane p of a quad loads rows 2p, 2p + 1 of the k-value's op(A)
// and op(B) values (one 16-byte load each; consecutive quads take
// consecutive k-values, so a wave's load covers 16 whole 64-byte runs),
// takes the quad's other op(B) values by DPP and accumulates rows 2p, 2p + 1
// of the tile.  The quads' tiles are then added over the wave (lanes p,
// p + 4, ...) and over the group's waves in LDS, in a fixed order.
__device__ inline float quad_bcast(float x, int src) {
    // quad_perm [src, src, src, src]
    switch (src) {
    case 0: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x00, 0xf, 0xf, false));
    case 1: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x55, 0xf, 0xf, false));
    case 2: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xaa, 0xf, 0xf, false));
    default: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xff, 0xf, 0xf, false));
    }
}

__global__ __launch_bounds__(kThreads) void direct_outer_quad_kernel(DirectArgs d) {
    __shared__ float red[kThreads / 64][2 * 64];
    select_entry(d);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, p = lane & 3;
    const int kl = d.kl, gi = d.ti;
    const int g = t / kl, q = (t % kl) >> 2;
    const int64_t nq = kl >> 2;  // k-values a group takes per round
    const int64_t ia = (int64_t)(g % gi) * 8 + 2 * p, jb = (int64_t)(g / gi) * 8 + 2 * p;
    const int64_t k0 = (int64_t)blockIdx.y * d.kchunk;
    const int64_t k1 = min(d.k, k0 + d.kchunk);
    float re[2][8], im[2][8];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) re[r][c] = im[r][c] = 0.f;
    // rows r, r + 1 of column l (zeros past rows)
    auto pair = [](const float2 *x, int64_t ld, int conj, int64_t rows, int64_t r, int64_t l, float2 &u,
                   float2 &v) {
        const float2 *ptr = x + r + l * ld;
        if (r + 1 < rows) {
            const float4 w = *reinterpret_cast<const float4 *>(ptr);
            u = make_float2(w.x, conj ? -w.y : w.y);
            v = make_float2(w.z, conj ? -w.w : w.w);
        } else {
            u = r < rows ? *ptr : make_float2(0.f, 0.f);
            if (conj) u.y = -u.y;
            v = make_float2(0.f, 0.f);
        }
    };
    auto step = [&](const float2 (&a)[2], const float2 (&bp)[2]) {
        float2 b[8];
#pragma unroll
        for (int src = 0; src < 4; ++src)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                b[2 * src + h] = make_float2(quad_bcast(bp[h].x, src), quad_bcast(bp[h].y, src));
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                re[r][c] = fmaf(a[r].x, b[c].x, re[r][c]);
                re[r][c] = fmaf(-a[r].y, b[c].y, re[r][c]);
                im[r][c] = fmaf(a[r].x, b[c].y, im[r][c]);
                im[r][c] = fmaf(a[r].y, b[c].x, im[r][c]);
            }
    };
    // a quad's lanes share l, so a quad is active or idle as a whole
    int64_t l = k0 + q;
    for (; l + nq < k1; l += 2 * nq) {
        float2 a0[2], b0[2], a1[2], b1[2];
        pair(d.A, d.lda, d.a_conj, d.m, ia, l, a0[0], a0[1]);
        pair(d.B, d.ldb, d.b_conj, d.n, jb, l, b0[0], b0[1]);
        pair(d.A, d.lda, d.a_conj, d.m, ia, l + nq, a1[0], a1[1]);
        pair(d.B, d.ldb, d.b_conj, d.n, jb, l + nq, b1[0], b1[1]);
        step(a0, b0);
        step(a1, b1);
    }
    if (l < k1) {
        float2 a0[2], b0[2];
        pair(d.A, d.lda, d.a_conj, d.m, ia, l, a0[0], a0[1]);
        pair(d.B, d.ldb, d.b_conj, d.n, jb, l, b0[0], b0[1]);
        step(a0, b0);
    }
    // over the wave's quads: lanes 12 + p of each row of 16 add up their
    // row (shifts by 4 and 8), then the rows are added pairwise
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float v[2] = {re[r][c], im[r][c]};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float x = v[h];
                x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xf, 0xf, false));
                x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xf, 0xf, false));
                x += __shfl_xor(x, 16);
                x += __shfl_xor(x, 32);
                v[h] = x;
            }
            if (lane >= 12 && lane < 16) {
                const int o = 2 * p + r + 8 * c;
                red[wv][2 * o] = v[0];
                red[wv][2 * o + 1] = v[1];
            }
        }
    __syncthreads();
    const int groups = kThreads / kl;
    if (t >= groups * 64) return;
    const int g2 = t / 64, o2 = t % 64;
    const int64_t i = (int64_t)(g2 % gi) * 8 + o2 % 8, j = (int64_t)(g2 / gi) * 8 + o2 / 8;
    if (i >= d.m || j >= d.n) return;
    const int w0 = g2 * (kl / 64);
    float sr = 0.f, si = 0.f;
    for (int x = 0; x < kl / 64; ++x) {
        sr += red[w0 + x][2 * o2];
        si += red[w0 + x][2 * o2 + 1];
    }
    if (gridDim.y > 1) {
        d.partial[(int64_t)blockIdx.y * d.m * d.n + i + j * d.m] = make_float2(sr, si);
        return;
    }
    float2 *cp = d.C + i + j * d.ldc;
    *cp = scale_out(d, sr, si, cp);
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
// load and per store (the products are added in the same order).  Without
// it the column's B values are all loaded before the products, and where
// C's columns are adjacent (ldc = m, C = alpha A B, 2 <= m <= 8, C 16-byte
// aligned) the block's 256 columns, one contiguous run of C, are staged in
// LDS and written by consecutive lanes, 16 bytes each.
template <int MT, bool VEC>
__global__ __launch_bounds__(kThreads) void direct_cols_kernel(DirectArgs d) {
    constexpr bool kCanStage = !VEC && MT >= 2 && MT <= 8;
    __shared__ __attribute__((aligned(16))) float2 stage[kThreads * (kCanStage ? MT : 1)];
    select_entry(d);
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool active = j < d.n;
    const bool staged = kCanStage && d.m >= 2 && d.beta_zero && d.ldc == d.m &&
                        (reinterpret_cast<uintptr_t>(d.C) & 15) == 0;
    if (!staged && !active) return;
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
    if (active) {
        if constexpr (VEC) {
            const float4 *bp = reinterpret_cast<const float4 *>(d.B + j * d.ldb);
            for (int64_t l2 = 0; l2 < d.k / 2; ++l2) {
                const float4 v = bp[l2];
                add(2 * l2, make_float2(v.x, d.b_conj ? -v.y : v.y));
                add(2 * l2 + 1, make_float2(v.z, d.b_conj ? -v.w : v.w));
            }
        } else {
            float2 bv[kShortK];
#pragma unroll
            for (int l = 0; l < kShortK; ++l) {
                if (l >= d.k) break;
                bv[l] = load_view(d.B, d.ldb, d.b_kcontig, d.b_conj, j, l);
            }
#pragma unroll
            for (int l = 0; l < kShortK; ++l) {
                if (l >= d.k) break;
                add(l, bv[l]);
            }
        }
    }
    if (staged) {
        // beta = 0: scale_out does not read C
        if (active) {
#pragma unroll
            for (int ii = 0; ii < MT; ++ii) {
                if (ii >= d.m) break;
                stage[threadIdx.x * d.m + ii] = scale_out(d, re[ii], im[ii], nullptr);
            }
        }
        __syncthreads();
        const int64_t j0 = (int64_t)blockIdx.x * kThreads;
        const int64_t len = min((int64_t)kThreads, d.n - j0) * d.m;
        float2 *base = d.C + j0 * d.m;  // 16-byte aligned: j0 is a multiple of 256
        for (int64_t e = 2 * (int64_t)threadIdx.x; e < len; e += 2 * kThreads) {
            if (e + 1 < len) {
                const float2 u = stage[e], v = stage[e + 1];
                *reinterpret_cast<float4 *>(base + e) = make_float4(u.x, u.y, v.x, v.y);
            } else {
                base[e] = stage[e];
            }
        }
        return;
    }
#pragma unroll
    for (int ii = 0; ii < MT; ii += (VEC ? 2 : 1)) {
        if (ii >= d.m) break;
        float2 *cp = d.C + ii + j * d.ldc;
        if constexpr (VEC) {
            const float2 o0 = scale_out(d, re[ii], im[ii], cp);
            const float2 o1 = scale_out(d, re[ii + 1], im[ii + 1], cp + 1);
            *reinterpret_cast<float4 *>(cp) = make_float4(o0.x, o0.y, o1.x, o1.y);
        } else {
            *cp = scale_out(d, re[ii], im[ii], cp);
        }
    }
}

// threads a split-k reduction aims for (below this, outputs share their
// k-ranges among several threads)
constexpr int64_t kReduceThreads = 32768;
// direct_outer_kernel: shortest k it takes, and the fewest k-values a
// thread keeps when the k range is split over blocks
constexpr int64_t kOuterMinK = 1024;
constexpr int64_t kOuterPerThread = 8;
// direct_outer_quad_kernel: shortest k it takes
constexpr int64_t kQuadMinK = int64_t(1) << 20;

int pow2_at_least(int64_t x) {
    int p = 1;
    while (p < x) p *= 2;
    return p;
}

// The tile of direct_outer_kernel for an m x n output with this k (1 + its
// index in kOuterTiles), or 0; the groups of tiles are a power of two
// along each side, and k is long enough that every thread has several
// k-values.
struct OuterTile {
    int tm, tn;
};
constexpr OuterTile kOuterTiles[] = {{2, 2}, {4, 4}, {8, 2}, {2, 8}, {8, 8}, {4, 16}, {16, 4}};
constexpr int kOuterTileCount = sizeof(kOuterTiles) / sizeof(kOuterTiles[0]);
int outer_tile(int64_t m, int64_t n, int64_t k) {
    // a single row or column (a GEMV) is left to direct_kernel, measured
    // faster there (8 x 1 over k = 2^16, 128 entries: 168 against 205 us)
    if (k < kOuterMinK || m == 1 || n == 1) return 0;
    auto groups = [&](int q) {
        const int tm = kOuterTiles[q].tm, tn = kOuterTiles[q].tn;
        return pow2_at_least((m + tm - 1) / tm) * pow2_at_least((n + tn - 1) / tn);
    };
    // the smallest tile that holds the whole output (each operand element
    // read by one group), else a 64-output tile in up to four groups
    for (int q = 0; q < kOuterTileCount; ++q)
        if (groups(q) == 1) return q + 1;
    for (int q = 0; q < kOuterTileCount; ++q)
        if (kOuterTiles[q].tm * kOuterTiles[q].tn == 64 && groups(q) <= 4) return q + 1;
    return 0;
}

}  // namespace

// Returns outer_tile's choice for direct_outer_kernel, or 0 for direct_kernel.
int direct_plan(DirectArgs &d, int64_t &splits) {
    if (const int q = outer_tile(d.m, d.n, d.k)) {
        const OuterTile &tt = kOuterTiles[q - 1];
        d.ti = pow2_at_least((d.m + tt.tm - 1) / tt.tm);
        d.tj = pow2_at_least((d.n + tt.tn - 1) / tt.tn);
        d.kl = kThreads / (d.ti * d.tj);
        // blocks over k while each thread keeps at least kOuterPerThread
        // k-values, up to 1024 blocks
        splits = 1;
        while (splits < 1024 && d.k / (splits * 2) >= (int64_t)d.kl * kOuterPerThread) splits *= 2;
        d.kchunk = (d.k + splits - 1) / splits;
        splits = (d.k + d.kchunk - 1) / d.kchunk;
        return q;
    }
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
    return 0;
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
    const int outer = direct_plan(d, splits);
    d.bsPartial = splits * d.m * d.n;
    if (outer) {
        const dim3 g(1, (unsigned)splits, nz), t(kThreads);
        auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
        const bool vec = !d.a_kcontig && !d.b_kcontig && d.lda % 2 == 0 && d.ldb % 2 == 0 && al16(d.A) &&
                         al16(d.B) && (nz == 1 || (d.bsA % 2 == 0 && d.bsB % 2 == 0));
        switch (outer * (vec ? -1 : 1)) {
        case 1: hipLaunchKernelGGL((direct_outer_kernel<2, 2, false>), g, t, 0, s, d); break;
        case 2: hipLaunchKernelGGL((direct_outer_kernel<4, 4, false>), g, t, 0, s, d); break;
        case 3: hipLaunchKernelGGL((direct_outer_kernel<8, 2, false>), g, t, 0, s, d); break;
        case 4: hipLaunchKernelGGL((direct_outer_kernel<2, 8, false>), g, t, 0, s, d); break;
        case 5: hipLaunchKernelGGL((direct_outer_kernel<8, 8, false>), g, t, 0, s, d); break;
        case 6: hipLaunchKernelGGL((direct_outer_kernel<4, 16, false>), g, t, 0, s, d); break;
        case 7: hipLaunchKernelGGL((direct_outer_kernel<16, 4, false>), g, t, 0, s, d); break;
        case -1: hipLaunchKernelGGL((direct_outer_kernel<2, 2, true>), g, t, 0, s, d); break;
        case -2: hipLaunchKernelGGL((direct_outer_kernel<4, 4, true>), g, t, 0, s, d); break;
        case -3: hipLaunchKernelGGL((direct_outer_kernel<8, 2, true>), g, t, 0, s, d); break;
        case -4: hipLaunchKernelGGL((direct_outer_kernel<2, 8, true>), g, t, 0, s, d); break;
        case -5:
            // four lanes per k-value from k = 2^20 (8 x 8 x 2^22: 148 against 166
            // us); below that the one-lane kernel measured faster (20 against 27 us)
            if (d.k >= kQuadMinK) hipLaunchKernelGGL(direct_outer_quad_kernel, g, t, 0, s, d);
            else hipLaunchKernelGGL((direct_outer_kernel<8, 8, true>), g, t, 0, s, d);
            break;
        case -6: hipLaunchKernelGGL((direct_outer_kernel<4, 16, true>), g, t, 0, s, d); break;
        default: hipLaunchKernelGGL((direct_outer_kernel<16, 4, true>), g, t, 0, s, d); break;
        }
    } else {
        const int64_t tiles = ((d.m + d.ti - 1) / d.ti) * ((d.n + d.tj - 1) / d.tj);
        hipLaunchKernelGGL(direct_kernel, dim3((unsigned)tiles, (unsigned)splits, nz), dim3(kThreads), 0, s, d);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    // threads per output: a few outputs with many k-ranges would otherwise
    // leave one thread per output walking every range
    const int64_t mn = d.m * d.n;
    int ways = 1;
    while (ways < kThreads && ways < splits && mn * ways < kReduceThreads) ways *= 2;
    const int64_t per_block = kThreads / ways;
    hipLaunchKernelGGL(direct_reduce_kernel, dim3((unsigned)((mn + per_block - 1) / per_block), 1, nz),
                       dim3(kThreads), 0, s, d, (int)splits, ways);
    return hipGetLastError();
}

}  // namespace qce
