// Split and scale (Sec. 2.1, Eq. 2; scaling of Sec. 4.2).
//
// Each GEMM operand op(X) (rows x k) is read once and rewritten into panels
// in the format of the selected mode (see PanelGeom in common.hpp):
//   FP16X2 / FP16X2_SCALED: x' = x * 2^s, hi = fp16(x'), lo = fp16((x' - hi) * 2^11)
//   BF16X3:                 b0 = bf16(x), b1 = bf16(x - b0), b2 = bf16(x - b0 - b1)
//   FP32:                   re and im de-interleaved into two FP32 planes
// All conversions round to nearest even; the subtractions are exact in FP32
// and the power-of-two scalings are exact (ldexp).  The mode and shift come
// from the device decision when statistics ran, so no host round trip is
// needed (Sec. 4.2).  Inputs are never modified.
#include <algorithm>

#include "gather.hpp"
#include "split_math.hpp"

namespace qce {

namespace {

constexpr int kThreads = 256;

// Operand layouts of the split
constexpr int kRowsContig = 0, kKContig = 1, kGather = 2;

// LDS slot of tile element (row tr, k-value tq) of a 64 x 64 staging tile:
// the k index is XORed with the row's low five bits, so that 32 lanes on
// consecutive rows (the conversion reads) and 32 lanes on consecutive k
// (the row-run loads) hit distinct 8-byte bank pairs, without padding:
// 32 KB per block, five blocks per CU.
__device__ inline int tile_slot(int tr, int tq) { return tr * 64 + (tq ^ (tr & 31)); }

// Panel row r holds P[r][l], l = 0..k-1.  kRowsContig: P[r][l] =
// x[r + l * ldx] (rows contiguous: op(A) = A, or op(B) = B^T / B^H);
// kKContig: P[r][l] = x[l + r * ldx] (k contiguous: op(A) = A^T / A^H, or
// op(B) = B); kGather: P[r][l] read through the bit map gm.  conj negates
// the imaginary part.
//
// A thread converts one chunk row: 16 k-values of one row, written as the
// row's whole slot in every plane (32 bytes per plane, 64 for FP32).
// kRowsContig: a wave takes 64 consecutive rows of one chunk, so each of
// its 16 loads reads 512 contiguous bytes and each plane's stores cover
// 2 KB.  kKContig and kGather: a block stages 64 rows x 64 k-values
// through LDS (read in runs of consecutive addresses), then converts like
// the first layout (64 consecutive rows of one chunk per wave, 2 KB stores
// per plane).
//
// Block bx of one operand's split (one batch entry); `tile` is the block's
// 32 KB LDS staging tile (unused by kRowsContig).
template <int LAYOUT>
__device__ __attribute__((always_inline)) inline void split_body(
    const float2 *__restrict__ x, int64_t ldx, int conj, int64_t rows, int64_t k,
    int64_t rows_pad, int64_t nchunks, char *__restrict__ panels, const DevState *st, int which,
    int forced_mode, int forced_shift, const GatherMap &gm, int64_t bx, float2 *tile) {
    constexpr int kK = 16;  // k-values per chunk row
    float re[kK], im[kK];
    int64_t r, c;  // row and chunk
    if constexpr (LAYOUT == kGather) {
        // A block takes 64 rows x 4 chunks (64 k-values) as in kKContig.
        // Thread t loads the tile elements e = t + 256 i, whose bits are
        // the tile's index bits by increasing stride in x: the low bits of
        // e walk x's lowest bits wherever the tile holds them.
        const int64_t row_blocks = rows_pad / 64;
        const int64_t r0 = (int64_t)(bx % row_blocks) * 64;
        const int64_t c0 = (int64_t)(bx / row_blocks) * 4;
        const int64_t l0 = c0 * kK;
        if (r0 < rows && l0 < k) {
            int64_t base = 0;
            for (int i = 6; i < gm.nr; ++i)
                if ((r0 >> i) & 1) base += (int64_t)1 << gm.rsh[i];
            for (int j = 6; j < gm.nk; ++j)
                if ((l0 >> j) & 1) base += (int64_t)1 << gm.ksh[j];
            // e's bits 0-7 come from the thread, bits 8-11 from the unrolled
            // load index: every per-bit term is uniform or per thread
            int tr0 = 0, tq0 = 0;
            int64_t off0 = base;
            for (int b = 0; b < 8 && b < gm.nt; ++b) {
                if ((threadIdx.x >> b) & 1) {
                    if (gm.tpos[b] < 6) tr0 += 1 << gm.tpos[b];
                    else tq0 += 1 << (gm.tpos[b] - 6);
                    off0 += (int64_t)1 << gm.tsh[b];
                }
            }
            int hi_tr[4], hi_tq[4];
            int64_t hi_off[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int b = 8 + j;
                hi_tr[j] = b < gm.nt && gm.tpos[b] < 6 ? 1 << gm.tpos[b] : 0;
                hi_tq[j] = b < gm.nt && gm.tpos[b] >= 6 ? 1 << (gm.tpos[b] - 6) : 0;
                hi_off[j] = b < gm.nt ? (int64_t)1 << gm.tsh[b] : 0;
            }
            const int ne = 1 << gm.nt;
            constexpr int kE = 64 * 64 / kThreads;
            float2 v[kE];
            // all loads first, then the LDS stores
#pragma unroll
            for (int i = 0; i < kE; ++i) {
                int64_t off = off0;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if ((i >> j) & 1) off += hi_off[j];
                if (i * kThreads + (int)threadIdx.x < ne) v[i] = x[off];
            }
#pragma unroll
            for (int i = 0; i < kE; ++i) {
                int tr = tr0, tq = tq0;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if ((i >> j) & 1) {
                        tr += hi_tr[j];
                        tq += hi_tq[j];
                    }
                if (i * kThreads + (int)threadIdx.x < ne) tile[tile_slot(tr, tq)] = v[i];
            }
        }
        __syncthreads();
        const int tr = threadIdx.x & 63, tc = threadIdx.x >> 6;
        r = r0 + tr;
        c = c0 + tc;
        if (c >= nchunks) return;
#pragma unroll
        for (int j = 0; j < kK; ++j) {
            const int64_t l = c * kK + j;
            const float2 v = r < rows && l < k ? tile[tile_slot(tr, tc * kK + j)] : make_float2(0.f, 0.f);
            re[j] = v.x;
            im[j] = v.y;
        }
    } else if constexpr (LAYOUT == kKContig) {
        // A block takes 64 rows x 4 chunks (64 k-values).  The tile is read
        // in 512-byte row runs (a wave reads one row per load) into LDS,
        // in the swizzled layout of tile_slot (all 16 loads of a thread are
        // issued before its LDS stores); each thread then takes one chunk
        // row, with waves on consecutive rows as in the other layout (whose
        // panel stores are contiguous).
        const int64_t row_blocks = rows_pad / 64;
        const int64_t r0 = (int64_t)(bx % row_blocks) * 64;
        const int64_t c0 = (int64_t)(bx / row_blocks) * 4;
        constexpr int kE = 64 * 64 / kThreads;
        float2 v[kE];
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            const int e = i * kThreads + threadIdx.x;
            const int tr = e >> 6, tq = e & 63;
            const int64_t rr = r0 + tr, l = c0 * kK + tq;
            v[i] = make_float2(0.f, 0.f);
            if (rr < rows && l < k) {
                v[i] = x[l + rr * ldx];
                if (conj) v[i].y = -v[i].y;  // (padding stays +0)
            }
        }
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            const int e = i * kThreads + threadIdx.x;
            tile[tile_slot(e >> 6, e & 63)] = v[i];
        }
        __syncthreads();
        const int tr = threadIdx.x & 63, tc = threadIdx.x >> 6;
        r = r0 + tr;
        c = c0 + tc;
        if (c >= nchunks) return;
#pragma unroll
        for (int j = 0; j < kK; ++j) {
            const float2 v = tile[tile_slot(tr, tc * kK + j)];
            re[j] = v.x;
            im[j] = v.y;
        }
    } else {
        const int64_t t = bx * kThreads + threadIdx.x;
        if (t >= rows_pad * nchunks) return;
        r = t % rows_pad;
        c = t / rows_pad;
        const int64_t l0 = c * kK;
#pragma unroll
        for (int j = 0; j < kK; ++j) {
            const int64_t l = l0 + j;
            float2 v = make_float2(0.f, 0.f);
            if (r < rows && l < k) {
                v = x[r + l * ldx];
                if (conj) v.y = -v.y;  // (padding stays +0)
            }
            re[j] = v.x;
            im[j] = v.y;
        }
    }
    const int mode = st ? st->mode : forced_mode;
    const int shift = st ? st->shift[which] : forced_shift;
    const int64_t rb = r / kPanelRows;
    const int rin = (int)(r % kPanelRows);
    if (mode == QCE_MODE_FP16X2 || mode == QCE_MODE_FP16X2_SCALED) {
        using G = PanelGeom<QCE_MODE_FP16X2>;
        static_assert(PanelFmt<QCE_MODE_FP16X2>::kBK == kK, "one chunk row per thread");
        char *chunk = panels + (rb * nchunks + c) * (int64_t)G::kChunkBytes;
        const int sh = mode == QCE_MODE_FP16X2_SCALED ? shift : 0;
        uint16_t h[4][kK];
#pragma unroll
        for (int j = 0; j < kK; ++j) {
            split_fp16x2(re[j], sh, h[0][j], h[1][j]);
            split_fp16x2(im[j], sh, h[2][j], h[3][j]);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int g = 0; g < 2; ++g)
                *reinterpret_cast<uint4 *>(chunk + G::offset(p, rin, g)) = pack8(h[p] + 8 * g);
    } else if (mode == QCE_MODE_BF16X3) {
        using G = PanelGeom<QCE_MODE_BF16X3>;
        static_assert(PanelFmt<QCE_MODE_BF16X3>::kBK == kK, "one chunk row per thread");
        char *chunk = panels + (rb * nchunks + c) * (int64_t)G::kChunkBytes;
        uint16_t b[6][kK];
#pragma unroll
        for (int j = 0; j < kK; ++j) {
            split_bf16x3(re[j], b[0][j], b[1][j], b[2][j]);
            split_bf16x3(im[j], b[3][j], b[4][j], b[5][j]);
        }
#pragma unroll
        for (int p = 0; p < 6; ++p)
#pragma unroll
            for (int g = 0; g < 2; ++g)
                *reinterpret_cast<uint4 *>(chunk + G::offset(p, rin, g)) = pack8(b[p] + 8 * g);
    } else {
        using G = PanelGeom<QCE_MODE_FP32>;
        static_assert(PanelFmt<QCE_MODE_FP32>::kBK == kK, "one chunk row per thread");
        char *chunk = panels + (rb * nchunks + c) * (int64_t)G::kChunkBytes;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            *reinterpret_cast<float4 *>(chunk + G::offset(0, rin, g)) =
                make_float4(re[4 * g], re[4 * g + 1], re[4 * g + 2], re[4 * g + 3]);
            *reinterpret_cast<float4 *>(chunk + G::offset(1, rin, g)) =
                make_float4(im[4 * g], im[4 * g + 1], im[4 * g + 2], im[4 * g + 3]);
        }
    }
}

template <int LAYOUT>
__global__ __launch_bounds__(kThreads) void split_panels_kernel(
    const float2 *__restrict__ x, int64_t ldx, int conj, int64_t rows, int64_t k,
    int64_t rows_pad, int64_t nchunks, char *__restrict__ panels, const DevState *st, int which,
    int forced_mode, int forced_shift, int64_t xstride, int64_t pstride, const GatherMap gm) {
    __shared__ float2 tile[LAYOUT == kRowsContig ? 1 : 64 * 64];
    // batch entry
    x += (int64_t)blockIdx.z * xstride;
    panels += (int64_t)blockIdx.z * pstride;
    if (st) st += blockIdx.z;
    split_body<LAYOUT>(x, ldx, conj, rows, k, rows_pad, nchunks, panels, st, which, forced_mode, forced_shift,
                       gm, blockIdx.x, tile);
}

__device__ __attribute__((always_inline)) inline void split_job_block(const SplitJob &q, int64_t j, float2 *tile) {
    const int64_t z = j / q.blocks, bx = j % q.blocks;
    const int64_t rows_pad = round_up(q.rows, kPanelRows), nchunks = round_up(q.k, kKPad) / kKPad;
    const DevState *st = q.st ? q.st + z : nullptr;
    const GatherMap gm{};
    if (q.kcontig)
        split_body<kKContig>(q.x + z * q.xstride, q.ldx, q.conj, q.rows, q.k, rows_pad, nchunks,
                             q.panels + z * q.pstride, st, q.which, q.forced_mode, q.shift, gm, bx, tile);
    else
        split_body<kRowsContig>(q.x + z * q.xstride, q.ldx, q.conj, q.rows, q.k, rows_pad, nchunks,
                                q.panels + z * q.pstride, st, q.which, q.forced_mode, q.shift, gm, bx, tile);
}

// Grouped launch: the blocks of every job (one operand of one GEMM, each a
// batch) in one grid; block b belongs to the last job whose block_start <= b.
__global__ __launch_bounds__(kThreads) void split_grouped_kernel(const SplitJob *__restrict__ jobs, int count) {
    __shared__ float2 tile[64 * 64];
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_start <= b) lo = mid;
        else hi = mid - 1;
    }
    const SplitJob &q = jobs[lo];
    const int64_t j = b - q.block_start;
    if (q.blocks <= 0 || j >= q.blocks * q.batch) return;
    split_job_block(q, j, tile);
}

// Both operands of one GEMM (or batch) in one launch, the jobs passed by
// value: blocks [0, a.blocks * a.batch) split op(A), the rest op(B).
__global__ __launch_bounds__(kThreads) void split_pair_kernel(const SplitJob a, const SplitJob b) {
    __shared__ float2 tile[64 * 64];
    const int64_t blk = blockIdx.x, na = a.blocks * a.batch;
    if (blk < na) split_job_block(a, blk, tile);
    else split_job_block(b, blk - na, tile);
}

__global__ __launch_bounds__(kThreads) void split_planar_kernel(int mode, int shift,
                                                                const float2 *__restrict__ x,
                                                                int64_t n, uint16_t *planes) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    float2 v = x[i];
    if (mode == QCE_MODE_BF16X3) {
        uint16_t b[6];
        split_bf16x3(v.x, b[0], b[1], b[2]);
        split_bf16x3(v.y, b[3], b[4], b[5]);
        for (int p = 0; p < 6; ++p) planes[p * n + i] = b[p];
    } else {
        uint16_t h[4];
        split_fp16x2(v.x, shift, h[0], h[1]);
        split_fp16x2(v.y, shift, h[2], h[3]);
        for (int p = 0; p < 4; ++p) planes[p * n + i] = h[p];
    }
}

}  // namespace

int64_t split_job_blocks(int64_t rows, int64_t k, int kcontig) {
    const int64_t rows_pad = round_up(rows, kPanelRows);
    const int64_t nchunks = round_up(k, kKPad) / kKPad;
    if (rows_pad * nchunks == 0) return 0;
    return kcontig ? (rows_pad / 64) * ((nchunks + 3) / 4) : (rows_pad * nchunks + kThreads - 1) / kThreads;
}

hipError_t launch_split_pair(const SplitJob &a, const SplitJob &b, hipStream_t s) {
    const int64_t total = a.blocks * a.batch + b.blocks * b.batch;
    if (total <= 0) return hipSuccess;
    if (total > INT32_MAX || a.blocks <= 0 || b.blocks <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(split_pair_kernel, dim3((unsigned)total), dim3(kThreads), 0, s, a, b);
    return hipGetLastError();
}

hipError_t launch_split_grouped(const SplitJob *dev_jobs, int count, int64_t total_blocks, hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    if (total_blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(split_grouped_kernel, dim3((unsigned)total_blocks), dim3(kThreads), 0, s, dev_jobs, count);
    return hipGetLastError();
}

hipError_t launch_split_panels(const float2 *x, int64_t ldx, int kcontig, int conj, int64_t rows,
                               int64_t k, void *panels, const DevState *st, int which,
                               int forced_mode, int shift, hipStream_t s, int batch,
                               int64_t xstride, int64_t pstride) {
    const int64_t rows_pad = round_up(rows, kPanelRows);
    const int64_t nchunks = round_up(k, kKPad) / kKPad;
    const int64_t total = rows_pad * nchunks;
    if (total == 0) return hipSuccess;
    char *p = static_cast<char *>(panels);
    if (!kcontig) {
        const int64_t blocks = (total + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(split_panels_kernel<kRowsContig>, dim3((unsigned)blocks, 1, batch), dim3(kThreads),
                           0, s, x, ldx, conj, rows, k, rows_pad, nchunks, p, st, which, forced_mode, shift,
                           xstride, pstride, GatherMap{});
    } else {
        const int64_t blocks = (rows_pad / 64) * ((nchunks + 3) / 4);
        hipLaunchKernelGGL(split_panels_kernel<kKContig>, dim3((unsigned)blocks, 1, batch), dim3(kThreads), 0,
                           s, x, ldx, conj, rows, k, rows_pad, nchunks, p, st, which, forced_mode, shift,
                           xstride, pstride, GatherMap{});
    }
    return hipGetLastError();
}

bool gather_map_valid(const GatherMap &gm) {
    if (gm.nr < 0 || gm.nk < 0 || gm.nr > 31 || gm.nk > 31 || gm.nr + gm.nk > 62) return false;
    const int nb = gm.nr + gm.nk;
    uint64_t seen = 0;
    for (int i = 0; i < nb; ++i) {
        const int sh = i < gm.nr ? gm.rsh[i] : gm.ksh[i - gm.nr];
        if (sh < 0 || sh >= nb || ((seen >> sh) & 1)) return false;
        seen |= uint64_t(1) << sh;
    }
    // the tile: the low min(6, nr) bits of r and min(6, nk) of l, each once,
    // by increasing stride
    const int tr = std::min(6, gm.nr), tk = std::min(6, gm.nk);
    if (gm.nt != tr + tk) return false;
    unsigned used = 0;
    for (int b = 0; b < gm.nt; ++b) {
        const int p = gm.tpos[b];
        const bool is_r = p >= 0 && p < tr, is_k = p >= 6 && p < 6 + tk;
        if (!(is_r || is_k) || ((used >> p) & 1)) return false;
        used |= 1u << p;
        if (gm.tsh[b] != (is_r ? gm.rsh[p] : gm.ksh[p - 6])) return false;
        if (b > 0 && gm.tsh[b] <= gm.tsh[b - 1]) return false;
    }
    return true;
}

hipError_t launch_split_gather(const float2 *x, const GatherMap &gm, void *panels, const DevState *st,
                               int which, int forced_mode, int shift, hipStream_t s) {
    if (!gather_map_valid(gm)) return hipErrorInvalidValue;
    const int64_t rows = int64_t(1) << gm.nr, k = int64_t(1) << gm.nk;
    const int64_t rows_pad = round_up(rows, kPanelRows);
    const int64_t nchunks = round_up(k, kKPad) / kKPad;
    const int64_t blocks = (rows_pad / 64) * ((nchunks + 3) / 4);
    hipLaunchKernelGGL(split_panels_kernel<kGather>, dim3((unsigned)blocks, 1, 1), dim3(kThreads), 0, s, x,
                       int64_t(0), 0, rows, k, rows_pad, nchunks, static_cast<char *>(panels), st, which,
                       forced_mode, shift, int64_t(0), int64_t(0), gm);
    return hipGetLastError();
}

hipError_t launch_split_planar(int mode, int shift, const float2 *x, int64_t n, uint16_t *planes,
                               hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(split_planar_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, mode,
                       shift, x, n, planes);
    return hipGetLastError();
}

}  // namespace qce
