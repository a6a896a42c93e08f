// Exponent statistics and mode selection (Sec. 4.1 and 4.2).
//
// Every FP32 component of both operands is read once (Sec. 4: all elements
// are checked, no sampling) and binned by its exact exponent
// e = floor(log2|v|) (bin = e + 149, FP32 subnormals included; zeros and
// Inf/NaN in bins of their own).  One pass gives both stages of the rule:
// stage 1 needs the counts above 2^-14 and 2^-110 and e_max, stage 2 the
// count inside [e_max - 28, e_max], which only a histogram can give before
// e_max is known.
//
// stats_kernel: a block bins its share of one operand into a histogram in
// LDS (lane l of every wave adds into column l % 32 of 16-bit counters, so
// the LDS adds of a half wave hit distinct banks), then writes a record: its nonzero,
// stage-1, BF16X3-floor and non-finite counts, its largest exponent bin and
// the cumulative counts of the 32 bins below it.  select_kernel (the next
// launch, one block per GEMM) adds up the records -- the stage-2 count of a
// block is one cumulative entry -- and turns both operands' statistics
// into the device mode flag and shifts, with a record for the host.  The
// kernel boundary publishes the records; a last-block-arrives scheme would
// need a device-scope fence in every block, which on this part writes back
// and invalidates the XCD's L2.  Counts are exact integers (the result does
// not depend on block order), and nothing is copied to the host (Sec. 4.2).
#include <algorithm>

#include "common.hpp"
#include "select.hpp"

namespace qce {

namespace {

constexpr int kThreads = 256;
constexpr int kBinZero = 277, kBinNonfinite = 278;
constexpr int kBins = 279;                 // exponent bins 0..276, zero, non-finite
constexpr int kWords = (kBins + 1) / 2;    // two 16-bit counters per word
constexpr int kCols = 32;                  // lanes l and l + 32 of every wave share a column
constexpr int kBin1 = kFp16Emin + 149;     // stage 1: e >= -14
constexpr int kBin3 = kBf16x3Emin + 149;   // BF16X3 floor: e >= -110
// elements one lane may bin before a 16-bit counter of its column could
// overflow
constexpr int64_t kMaxPerLane = 8000;  // eight lanes per column, 16-bit counters

// exact exponent bin of one FP32 component
__device__ inline int bin_of(float v) {
    const unsigned int b = __float_as_uint(v) & 0x7fffffffu;
    const unsigned int e8 = b >> 23;
    int bin = e8 ? (int)e8 + 22 : 31 - (int)__clz(b);  // subnormal: -118 - clz(mantissa) + 149
    bin = b == 0u ? kBinZero : bin;
    bin = e8 == 255u ? kBinNonfinite : bin;
    return bin;
}

// The block's LDS histogram: word t (bins 2t, 2t + 1 as 16-bit halves) has
// kCols counters side by side, lane l of every wave in column l % 32 (the
// 32 lanes of a half wave hit distinct banks; the waves share the columns,
// which keeps the histogram at 18 KB to clear and add up).
constexpr int kRow = kCols;  // counters per word
struct HistCounter {
    unsigned int *col;  // this lane's column (LDS)
    // on = 0 adds nothing (the masked end of a batch: no branch, so the
    // compiler cannot sink the batch's loads into one)
    __device__ inline void operator()(float v, unsigned int on = 1u) {
        const int bin = bin_of(v);
        __hip_atomic_fetch_add(col + (bin >> 1) * kRow, on << ((bin & 1) << 4), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
};

// Visit every FP32 component of a stored column-major complex matrix; the
// work is split over `nblk` blocks starting at block index `blk`.  Every
// loop issues a batch of loads (from clamped, valid addresses where a
// batch runs past the end) before binning any of them, so a lane never
// waits for one load at a time.
template <class F>
__device__ inline void scan_matrix(const MatDesc &d, int64_t blk, int64_t nblk, F &f) {
    if (d.rows <= 0 || d.cols <= 0) return;
    const int64_t tid = blk * kThreads + threadIdx.x;
    const int64_t nthr = nblk * kThreads;
    if (d.ld == d.rows || d.cols == 1) {
        const float *p = reinterpret_cast<const float *>(d.ptr);
        const int64_t nf = 2 * d.rows * d.cols;
        if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
            // kBatch 16-byte loads in flight per lane before any is binned;
            // the rest in masked batches of kRest
            constexpr int kBatch = 16, kRest = 8;
            const int64_t n4 = nf >> 2;
            const float4 *p4 = reinterpret_cast<const float4 *>(p);
            int64_t i = tid;
            for (; i + (kBatch - 1) * nthr < n4; i += kBatch * nthr) {
                float4 v[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) v[u] = p4[i + u * nthr];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    f(v[u].x); f(v[u].y); f(v[u].z); f(v[u].w);
                }
            }
            for (; i < n4; i += kRest * nthr) {
                float4 v[kRest];
#pragma unroll
                for (int u = 0; u < kRest; ++u) v[u] = p4[min(i + u * nthr, n4 - 1)];
#pragma unroll
                for (int u = 0; u < kRest; ++u) {
                    const unsigned int on = i + u * nthr < n4;
                    f(v[u].x, on); f(v[u].y, on); f(v[u].z, on); f(v[u].w, on);
                }
            }
            for (int64_t j = (n4 << 2) + tid; j < nf; j += nthr) f(p[j]);
        } else {
            constexpr int kBatch = 16, kRest = 8;
            const int64_t n2 = nf >> 1;
            const float2 *p2 = reinterpret_cast<const float2 *>(p);
            int64_t i = tid;
            for (; i + (kBatch - 1) * nthr < n2; i += kBatch * nthr) {
                float2 v[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) v[u] = p2[i + u * nthr];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    f(v[u].x); f(v[u].y);
                }
            }
            for (; i < n2; i += kRest * nthr) {
                float2 v[kRest];
#pragma unroll
                for (int u = 0; u < kRest; ++u) v[u] = p2[min(i + u * nthr, n2 - 1)];
#pragma unroll
                for (int u = 0; u < kRest; ++u) {
                    const unsigned int on = i + u * nthr < n2;
                    f(v[u].x, on); f(v[u].y, on);
                }
            }
        }
    } else {
        // strided: the block's columns blk, blk + nblk, ... one after the
        // other as a flat index e = (column number) * rows + row, threads
        // over e; a thread's (column, row) advances by counting
        constexpr int kBatch = 8;
        const int64_t mycols = blk < d.cols ? (d.cols - 1 - blk) / nblk + 1 : 0;
        const int64_t total = mycols * d.rows;
        const int64_t dc = kThreads / d.rows, dr = kThreads % d.rows;
        int64_t cl = threadIdx.x / d.rows, r = threadIdx.x % d.rows;
        for (int64_t e = threadIdx.x; e < total; e += kBatch * kThreads) {
            float2 v[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const bool ok = e + u * kThreads < total;
                v[u] = d.ptr[ok ? (blk + cl * nblk) * d.ld + r : blk * d.ld];
                cl += dc;
                r += dr;
                const bool wrap = r >= d.rows;
                r -= wrap ? d.rows : 0;
                cl += wrap ? 1 : 0;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const unsigned int on = e + u * kThreads < total;
                f(v[u].x, on); f(v[u].y, on);
            }
        }
    }
}

// Block bx of batch entry z of one statistics launch.
__device__ inline void stats_body(const StatsArgs &g, int z, int bx) {
    __shared__ __attribute__((aligned(16))) unsigned int hist[kWords * kCols];
    __shared__ unsigned int bins[kWords * 2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    MatDesc a = g.a, b = g.b;
    a.ptr += (int64_t)z * a.bstride;
    b.ptr += (int64_t)z * b.bstride;
    const int total = g.blocks_a + g.blocks_b;
    StatsRecord *rec = g.rec + (int64_t)z * total;
    const bool is_a = bx < g.blocks_a;
    const int blk = is_a ? bx : bx - g.blocks_a;
    const int nblk = is_a ? g.blocks_a : g.blocks_b;

    {
        uint4 *h4 = reinterpret_cast<uint4 *>(hist);
        for (int i = threadIdx.x; i < kWords * kCols / 4; i += kThreads) h4[i] = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    HistCounter c;
    c.col = hist + (lane & 31);
    scan_matrix(is_a ? a : b, blk, nblk, c);
    __syncthreads();
    // the block's histogram: two threads per word, each adding half of its
    // kRow counters with 16-byte reads (a thread starts at a different
    // 16-byte slot than its neighbour)
    for (int p = threadIdx.x; p < 2 * kWords; p += kThreads) {
        const int t = p >> 1, half = p & 1;
        const uint4 *row = reinterpret_cast<const uint4 *>(hist + t * kRow + half * (kRow / 2));
        unsigned int lo = 0, hi = 0;
#pragma unroll
        for (int j = 0; j < kRow / 8; ++j) {
            const uint4 v = row[(j + p) & (kRow / 8 - 1)];
            lo += (v.x & 0xffffu) + (v.y & 0xffffu) + (v.z & 0xffffu) + (v.w & 0xffffu);
            hi += (v.x >> 16) + (v.y >> 16) + (v.z >> 16) + (v.w >> 16);
        }
        // the other half's sums (the partner thread is the neighbouring lane)
        lo += (unsigned int)__builtin_amdgcn_mov_dpp((int)lo, kDppQuadSwap1, 0xf, 0xf, false);
        hi += (unsigned int)__builtin_amdgcn_mov_dpp((int)hi, kDppQuadSwap1, 0xf, 0xf, false);
        if (!half) {
            bins[2 * t] = lo;
            bins[2 * t + 1] = hi;
        }
    }
    __syncthreads();
    // the block's record (wave 0)
    if (w == 0) {
        unsigned int nnz = 0, n1 = 0, n3 = 0;
        int mb = -1;
        for (int bI = lane; bI < kBinZero; bI += 64) {
            const unsigned int v = bins[bI];
            nnz += v;
            n1 += bI >= kBin1 ? v : 0u;
            n3 += bI >= kBin3 ? v : 0u;
            if (v) mb = bI;
        }
        nnz = lane_total(nnz);
        n1 = lane_total(n1);
        n3 = lane_total(n3);
        mb = lane_max(mb);
        StatsRecord &r = rec[bx];
        if (lane == 0) {
            r.nnz = nnz;
            r.n1 = n1;
            r.n3 = n3;
            r.nonfinite = bins[kBinNonfinite];
            r.maxbin = mb;
        }
        // cumulative count of bins mb - d .. mb for d = lane < 32: lane d
        // holds bin mb - d, then an inclusive scan over the 32 lanes
        static_assert(kRelBins == 32, "one lane per cumulative entry in the low half of the wave");
        unsigned int c = (lane < kRelBins && mb - lane >= 0) ? bins[mb - lane] : 0u;
        c = lane_scan_add<2>(c);
        if (lane < kRelBins) r.cum[lane] = c;
    }
}

__global__ __launch_bounds__(kThreads) void stats_kernel(StatsArgs g) {
    stats_body(g, blockIdx.z, blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void select_kernel(StatsArgs g) { select_block(g, blockIdx.z, true); }

// Grouped launch: the blocks of every entry (each a batch) in one grid;
// block b belongs to the last entry whose block_start <= b.
__global__ __launch_bounds__(kThreads) void stats_grouped_kernel(const GroupStatsEntry *__restrict__ ents,
                                                                 int count) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ents[mid].block_start <= b) lo = mid;
        else hi = mid - 1;
    }
    const GroupStatsEntry &e = ents[lo];
    const int per_z = e.args.blocks_a + e.args.blocks_b;
    const int64_t j = b - e.block_start;
    if (per_z <= 0 || j >= (int64_t)per_z * e.batch) return;
    stats_body(e.args, (int)(j / per_z), (int)(j % per_z));
}

// Grouped decisions: block b takes batch entry z of the last entry whose
// select_start <= b.
__global__ __launch_bounds__(kThreads) void select_grouped_kernel(const GroupStatsEntry *__restrict__ ents,
                                                                  int count) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ents[mid].select_start <= b) lo = mid;
        else hi = mid - 1;
    }
    const GroupStatsEntry &e = ents[lo];
    const int64_t z = b - e.select_start;
    if (z >= e.batch) return;
    select_block(e.args, (int)z, true);
}

}  // namespace

namespace {
// blocks of the contiguous and of the strided scan of a rows x cols operand
int64_t blocks_base(int64_t nf) {
    // enough blocks to cover the device several times, not more than needed
    const int64_t b = (nf + (int64_t)kThreads * 64 - 1) / ((int64_t)kThreads * 64);
    return std::max<int64_t>(1, std::min<int64_t>(b, 512));
}
// ... and enough that no lane bins more than kMaxPerLane components
int64_t blocks_contig(int64_t rows, int64_t cols) {
    const int64_t nf = 2 * rows * cols;
    const int64_t need = (nf + kThreads * (kMaxPerLane - 8) - 1) / (kThreads * (kMaxPerLane - 8));
    return std::max(blocks_base(nf), need);
}
int64_t blocks_strided(int64_t rows, int64_t cols) {
    const int64_t per_col = 2 * ((rows + kThreads - 1) / kThreads);  // per lane per column
    const int64_t cols_per_block = std::max<int64_t>(1, kMaxPerLane / per_col);
    return std::max(blocks_base(2 * rows * cols), (cols + cols_per_block - 1) / cols_per_block);
}
// the fewest blocks that keep every lane's count of d below kMaxPerLane
int64_t blocks_min(const MatDesc &d) {
    if (d.rows <= 0 || d.cols <= 0) return 0;
    if (d.ld == d.rows || d.cols == 1) {
        const int64_t nf = 2 * d.rows * d.cols;
        return std::max<int64_t>(1, (nf + kThreads * (kMaxPerLane - 8) - 1) / (kThreads * (kMaxPerLane - 8)));
    }
    const int64_t per_col = 2 * ((d.rows + kThreads - 1) / kThreads);
    const int64_t cols_per_block = std::max<int64_t>(1, kMaxPerLane / per_col);
    return (d.cols + cols_per_block - 1) / cols_per_block;
}

// statistics blocks the device holds at once (0 if it cannot be queried)
int stats_slots() {
    static int slots = -1;
    if (slots < 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, stats_kernel, kThreads, 0) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        slots = cus * std::max(per, 1);
    }
    return slots;
}

// A GEMM's pair of operands whose blocks exceed a whole number of rounds of
// resident blocks by a few would leave those few to run alone after the
// rest (e.g. 512 blocks of a 65536 x 64 operand and 1 of its 64 x 64
// partner on 512 slots): trim both counts in proportion, never below what
// the 16-bit counters need, so that the pair fills whole rounds.
void fit_pair(const MatDesc &a, const MatDesc &b, int &ba, int &bb) {
    const int slots = stats_slots();
    const int total = ba + bb;
    if (slots <= 0 || total <= slots || total % slots == 0) return;
    const int target = total / slots * slots;
    const int na = (int)blocks_min(a), nb = (int)blocks_min(b);
    int fa = ba ? std::max<int>(na, (int)((int64_t)ba * target / total)) : 0;
    fa = std::min(fa, ba);
    int fb = bb ? std::max<int>(nb, std::min(bb, target - fa)) : 0;
    fb = std::min(fb, bb);
    ba = fa;
    bb = fb;
}
}  // namespace

int stats_blocks(const MatDesc &d) {
    if (d.rows <= 0 || d.cols <= 0) return 0;
    const bool contig = d.ld == d.rows || d.cols == 1;
    const int64_t b = contig ? blocks_contig(d.rows, d.cols) : blocks_strided(d.rows, d.cols);
    return (int)std::min<int64_t>(b, kMaxStatsBlocks);
}

int stats_blocks_bound(int64_t rows, int64_t cols) {
    if (rows <= 0 || cols <= 0) return 0;
    // either orientation (the stored matrix of op(X) may be X or X^T)
    const int64_t b = std::max({blocks_contig(rows, cols), blocks_strided(rows, cols), blocks_strided(cols, rows)});
    return (int)std::min<int64_t>(b, kMaxStatsBlocks);
}

bool stats_supported(const MatDesc &d) {
    if (d.rows <= 0 || d.cols <= 0) return true;
    const int b = stats_blocks(d);
    if (d.ld == d.rows || d.cols == 1) return 2 * d.rows * d.cols <= (int64_t)b * kThreads * (kMaxPerLane - 8);
    const int64_t per_col = 2 * ((d.rows + kThreads - 1) / kThreads);
    return per_col <= kMaxPerLane && ((d.cols + b - 1) / b) * per_col <= kMaxPerLane;
}

size_t stats_record_bytes(const MatDesc &a, const MatDesc &b, int batch) {
    return sizeof(StatsRecord) * (size_t)(stats_blocks(a) + stats_blocks(b)) * (size_t)std::max(1, batch);
}

hipError_t stats_group_entry(const MatDesc &a, const MatDesc &b, DevState *st, StatsRecord *rec, double t,
                             double t3, int forced_mode, int batch, GroupStatsEntry &out) {
    if (!stats_supported(a) || !stats_supported(b)) return hipErrorInvalidValue;
    StatsArgs &g = out.args;
    g.a = a;
    g.b = b;
    g.blocks_a = stats_blocks(a);
    g.blocks_b = stats_blocks(b);
    g.st = st;
    g.rec = rec;
    g.t = t;
    g.t3 = t3;
    g.forced = forced_mode;
    g.mode_log = nullptr;
    g.slot = 0;
    out.batch = std::max(1, batch);
    out.block_start = 0;
    out.select_start = 0;
    return g.blocks_a + g.blocks_b > 0 ? hipSuccess : hipErrorInvalidValue;
}

hipError_t launch_stats_grouped(const GroupStatsEntry *dev_entries, int count, int64_t total_blocks,
                                int64_t total_selects, hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    if (total_blocks > INT32_MAX || total_selects > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stats_grouped_kernel, dim3((unsigned)total_blocks), dim3(kThreads), 0, s, dev_entries, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(select_grouped_kernel, dim3((unsigned)total_selects), dim3(kThreads), 0, s, dev_entries,
                       count);
    return hipGetLastError();
}

hipError_t launch_stats(const MatDesc &a, const MatDesc &b, DevState *st, StatsRecord *rec, double t, double t3,
                        int forced_mode, int *mode_log, int slot, hipStream_t s, int batch, bool with_select,
                        StatsArgs *args_out) {
    if (!stats_supported(a) || !stats_supported(b)) return hipErrorInvalidValue;
    StatsArgs g;
    g.a = a;
    g.b = b;
    g.blocks_a = stats_blocks(a);
    g.blocks_b = stats_blocks(b);
    if (batch <= 1) fit_pair(a, b, g.blocks_a, g.blocks_b);
    g.st = st;
    g.rec = rec;
    g.t = t;
    g.t3 = t3;
    g.forced = forced_mode;
    g.mode_log = mode_log;
    g.slot = slot;
    const int total = g.blocks_a + g.blocks_b;
    if (total == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stats_kernel, dim3(total, 1, std::max(1, batch)), dim3(kThreads), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (args_out) *args_out = g;
    if (!with_select) return hipSuccess;
    hipLaunchKernelGGL(select_kernel, dim3(1, 1, std::max(1, batch)), dim3(kThreads), 0, s, g);
    return hipGetLastError();
}

}  // namespace qce
