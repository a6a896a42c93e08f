// Internal definitions shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qcemu.h"

namespace qce {

// ---------------------------------------------------------------------------
// Device-side statistics and decision (the paper's "exp stats buffer" and
// "mode flag buffer", Sec. 4.2).
// ---------------------------------------------------------------------------
struct OperandStats {
    unsigned long long nnz;        // nonzero finite components
    unsigned long long n1;         // floor(log2|v|) >= -14
    unsigned long long n2;         // floor(log2|v|) >= emax - 28 (stage 2)
    unsigned long long n3;         // floor(log2|v|) >= -110
    unsigned long long nonfinite;  // Inf / NaN
    unsigned int maxbits;          // largest |v| bit pattern among finite v
    unsigned int pad;
};

constexpr int kMaxStatsBlocks = 16384;  // per operand
constexpr int kRelBins = 32;            // exponent bins a block record keeps below its maximum

// One statistics block's summary of its share of one operand (exact counts
// of its FP32 components): nonzero finite, floor(log2|v|) >= -14 and
// >= -110, non-finite, its largest exponent bin (e + 149; -1 if none) and
// the cumulative counts of the kRelBins bins from there down (cum[d]: bins
// maxbin - d .. maxbin), so that the count of a window [x, maxbin] is one
// entry.  160 bytes, 16-byte aligned (vector loads).
struct __attribute__((aligned(16))) StatsRecord {
    unsigned int nnz, n1, n3, nonfinite;
    int maxbin;
    unsigned int pad[3];
    unsigned int cum[kRelBins];
};

struct DevState {
    int mode;             // selected qce_mode (never AUTO)
    int shift[2];         // power-of-two shifts sA, sB
    int pad;
    OperandStats acc[2];  // statistics of both operands (kept for the record)
    qce_decision last;    // record of the last decision
};

constexpr int kFp16Emax = 14;
constexpr int kFp16Emin = -14;
constexpr int kBf16x3Emin = -110;
constexpr int kBf16x3Emax = 126;
constexpr int kWindowSpan = kFp16Emax - kFp16Emin;  // 28: FP16 window [-14, 14]

// ---------------------------------------------------------------------------
// Panel geometry.  Each GEMM operand is rewritten by the split kernel into
// "panels": for a block of kPanelRows rows (rows of op(A) or columns of
// op(B)) and a block of BK k-values, one contiguous chunk laid out as
// [plane][row][k] with the k-values of a row in 16-byte granules whose
// position is XOR-swizzled by row (bank-conflict-free fragment reads).
// Rows and k beyond the matrix are zero.
// ---------------------------------------------------------------------------
constexpr int kPanelRows = 128;

template <int MODE> struct PanelFmt;
// FP16X2: planes hi(re), lo(re), hi(im), lo(im); FP16; 16 k per chunk.
template <> struct PanelFmt<QCE_MODE_FP16X2> {
    static constexpr int kPlanes = 4, kBK = 16, kElemBytes = 2;
};
// BF16X3: planes b0(re), b1(re), b2(re), b0(im), b1(im), b2(im); 16 k per chunk.
template <> struct PanelFmt<QCE_MODE_BF16X3> {
    static constexpr int kPlanes = 6, kBK = 16, kElemBytes = 2;
};
// FP32: planes re, im; 16 k per chunk.
template <> struct PanelFmt<QCE_MODE_FP32> {
    static constexpr int kPlanes = 2, kBK = 16, kElemBytes = 4;
};

template <int MODE> struct PanelGeom {
    using F = PanelFmt<MODE>;
    static constexpr int kRowBytes = F::kBK * F::kElemBytes;          // 32 (fp16/bf16) or 64 (fp32)
    static constexpr int kGranules = kRowBytes / 16;                  // 2 or 4
    static constexpr int kPlaneBytes = kPanelRows * kRowBytes;
    static constexpr int kChunkBytes = F::kPlanes * kPlaneBytes;
    static constexpr int kKPerGranule = 16 / F::kElemBytes;           // 8 or 4
    // Granule XOR swizzle: for the MFMA fragment reads (32 consecutive rows,
    // one granule) every group of 8 or 16 consecutive lanes hits distinct
    // 16-byte bank slots, i.e. conflict-free for 128- or 256-byte LDS
    // bank rows.
    __host__ __device__ static constexpr int swz(int row) {
        return kGranules == 4 ? (((row >> 2) & 1) | ((((row >> 1) ^ (row >> 3)) & 1) << 1))
                              : (((row >> 2) ^ (row >> 3)) & 1);
    }
    // byte offset of (plane, row, granule) inside a chunk
    __host__ __device__ static constexpr int offset(int plane, int row, int granule) {
        return plane * kPlaneBytes + row * kRowBytes + ((granule ^ swz(row)) << 4);
    }
};

// k is padded to a multiple of this for every mode (the chunk depth).
constexpr int kKPad = 16;

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Bytes of the panel buffer of one operand with `rows` rows and k values,
// large enough for every mode.
inline size_t panel_bytes(int64_t rows, int64_t k) {
    int64_t r = round_up(rows, kPanelRows), kk = round_up(k, kKPad);
    return (size_t)r * (size_t)kk * 12u;  // BF16X3: 6 planes x 2 bytes
}
static_assert(PanelFmt<QCE_MODE_FP16X2>::kBK == kKPad && PanelFmt<QCE_MODE_BF16X3>::kBK == kKPad &&
                  PanelFmt<QCE_MODE_FP32>::kBK == kKPad, "one chunk depth for every mode");

// ---------------------------------------------------------------------------
// Launch wrappers implemented in the .hip files.
// ---------------------------------------------------------------------------
struct MatDesc {  // a stored column-major complex64 matrix
    const float2 *ptr;
    int64_t rows, cols, ld;
    int64_t bstride;  // elements between batch entries (entry z at ptr + z * bstride)
};

// Batched launches put the batch entry in blockIdx.z; entry z uses the
// device state st + z (its own statistics, decision and record).
constexpr int kMaxBatch = 65535;

// Exponent statistics of both operands (one read, per-block records) and
// the mode selection of Sec. 4.1 (one block per GEMM, next launch)
// (stats.hip).  rec: stats_record_bytes of device scratch.  forced_mode:
// -1 = the rule; >= 0 = that mode (statistics taken for its shifts and the
// record).  mode_log (nullable) receives entry 0's mode at slot.  Batched:
// entry z reads a / b shifted by z * bstride and writes st + z.
struct StatsArgs {
    MatDesc a, b;
    int blocks_a, blocks_b;
    DevState *st;           // entry z: st + z
    StatsRecord *rec;       // entry z: rec + z * (blocks_a + blocks_b)
    double t, t3;
    int forced;             // -1: rule; >= 0: that mode (statistics for its shifts)
    int *mode_log;          // nullable: mode of entry 0 at mode_log[slot]
    int slot;
};
// One GEMM (or batch) of a grouped statistics launch: its blocks are
// [block_start, block_start + (blocks_a + blocks_b) * batch) of the grid.
struct GroupStatsEntry {
    StatsArgs args;
    int batch, pad;
    int64_t block_start;   // first statistics block
    int64_t select_start;  // first block of the selection launch (one per batch entry)
};
// fills `out` for launch_stats's arguments (block_start left 0)
hipError_t stats_group_entry(const MatDesc &a, const MatDesc &b, DevState *st, StatsRecord *rec, double t,
                             double t3, int forced_mode, int batch, GroupStatsEntry &out);
// total_selects: sum of the entries' batch counts
hipError_t launch_stats_grouped(const GroupStatsEntry *dev_entries, int count, int64_t total_blocks,
                                int64_t total_selects, hipStream_t s);
int stats_blocks(const MatDesc &d);
// upper bound of stats_blocks over every leading dimension of a rows x cols
// operand stored either way (rows x cols or cols x rows)
int stats_blocks_bound(int64_t rows, int64_t cols);
size_t stats_record_bytes(const MatDesc &a, const MatDesc &b, int batch = 1);
// with_select = false: the statistics launch only, its arguments in
// *args_out (nullable) for a consumer that selects in its own prologue
hipError_t launch_stats(const MatDesc &a, const MatDesc &b, DevState *st, StatsRecord *rec, double t, double t3,
                        int forced_mode, int *mode_log, int slot, hipStream_t s, int batch = 1,
                        bool with_select = true, StatsArgs *args_out = nullptr);

// Split a rows x k operand view into panels: P[r][l] = x[l + r*ldx] if
// kcontig else x[r + l*ldx], imaginary part negated if conj.  st != nullptr:
// mode and shift come from the device decision (operand index `which`);
// otherwise forced_mode / shift.
// Batched: entry z reads x + z * xstride, writes panels + z * pstride bytes
// and takes its decision from st + z.
hipError_t launch_split_panels(const float2 *x, int64_t ldx, int kcontig, int conj, int64_t rows,
                               int64_t k, void *panels, const DevState *st, int which,
                               int forced_mode, int shift, hipStream_t s, int batch = 1,
                               int64_t xstride = 0, int64_t pstride = 0);

// One operand of a grouped split launch (split.hip): the arguments of
// launch_split_panels for a rows-contiguous or k-contiguous operand, with
// its blocks [block_start, block_start + blocks * batch) of the grid.
struct SplitJob {
    const float2 *x;
    int64_t ldx;
    int kcontig, conj;
    int64_t rows, k;
    char *panels;
    const DevState *st;  // nullable: forced_mode / shift
    int which, forced_mode, shift, batch;
    int64_t xstride, pstride;  // elements / panel bytes between batch entries
    int64_t blocks;            // per batch entry: split_job_blocks
    int64_t block_start;
};
int64_t split_job_blocks(int64_t rows, int64_t k, int kcontig);
hipError_t launch_split_grouped(const SplitJob *dev_jobs, int count, int64_t total_blocks, hipStream_t s);
// both operands of one GEMM (or batch) in one launch (jobs by value;
// block_start ignored)
hipError_t launch_split_pair(const SplitJob &a, const SplitJob &b, hipStream_t s);

struct GemmArgs {
    const void *panelsA;  // rows = m
    const void *panelsB;  // rows = n
    int64_t m, n, k;
    float2 *C;
    int64_t ldc;
    float2 alpha, beta;
    int beta_zero;
    const DevState *st;  // nullable: forced mode
    int forced_mode;
    float2 *partial;         // split-k partial tiles (workspace), may be null if no split
    int64_t kpad_per_split;  // set by launch_gemm
    int batch;               // entries (blockIdx.z); 0 or 1: one GEMM
    int64_t bsA, bsB;        // panel bytes between entries
    int64_t bsC;             // C elements between entries
    int64_t bsPartial;       // partial elements between entries
    int tile;                // 64 or 128: that tile; else the tile table's choice
};
// which_kernel: a mode (forced) or -1 (AUTO: read the device flag)
hipError_t launch_gemm(const GemmArgs &g, int which_kernel, hipStream_t s);
size_t gemm_partial_bytes(int64_t m, int64_t n, int64_t k, int batch = 1);  // per entry, either tile
// tile of the panel GEMM for this output size (the tuned table)
int gemm_tile(int64_t m, int64_t n, int64_t k, int batch = 1);

// One entry of a grouped GEMM launch (gemm.hip): a GEMM (or a batch of
// equally shaped ones, g.batch) over its own split panels, with its own
// shape, alpha / beta, mode source (g.st per batch entry, or
// g.forced_mode) and k splits.  The host fills g (partial set once the
// split count is known); gemm_group_shape and gemm_group_schedule fill the
// rest.
struct GroupGemmEntry {
    GemmArgs g;
    int nbm, nbn, nsplit, pad;
    int64_t tiles;       // nbm * nbn * nsplit * batch
    int64_t tile_start;  // first tile id in the launch (a multiple of 8)
    int64_t red_start, red_blocks;  // blocks of the split-k sum (0 if nsplit == 1)
};
// tile of a grouped launch (64 or 128): forced_tile if 64 or 128, else the
// tuned table applied to the whole launch's output
int gemm_group_tile(const GroupGemmEntry *e, int count, int forced_tile);
// per-entry tile grid, k splits (counting every entry's tiles), partial
// sizes (g.bsPartial elements per batch entry) and reduction blocks
void gemm_group_shape(GroupGemmEntry *e, int count, int tile);
// orders the entries by tile cost (heaviest first) and assigns the starts
void gemm_group_schedule(GroupGemmEntry *e, int count, int64_t &total_tiles, int64_t &total_red);
// queue: kGroupQueueWords zeroed device counters (left zeroed)
constexpr int kGroupQueueWords = 9;
hipError_t launch_gemm_grouped(const GroupGemmEntry *dev_entries, int count, int64_t total_tiles,
                               int64_t total_red, int tile, unsigned int *queue, hipStream_t s);

// Short-k, narrow-output GEMM with the split done on load (gemm.hip):
// C (m x n, n <= 64) = alpha op(A) op(B) + beta C for k <= 128, reading the
// stored operands directly (op(A)[i][l] = a_kcontig ? A[l + i lda] :
// A[i + l lda]; op(B)[l][j] = b_kcontig ? B[l + j ldb] : B[j + l ldb];
// conj negates the imaginary part).  Mode and shifts from st (AUTO,
// forced_mode < 0, or FP16X2_SCALED) or forced_mode.  Batched: entry
// blockIdx.z at A + z bsA, B + z bsB, C + z bsC (elements), st + z.
struct SmallKArgs {
    const float2 *A, *B;
    int64_t lda, ldb;
    int a_kcontig, a_conj, b_kcontig, b_conj;
    int64_t m, n, k;
    float2 *C;
    int64_t ldc;
    float2 alpha, beta;
    int beta_zero;
    const DevState *st;
    int forced_mode;
    int batch;
    int64_t bsA, bsB, bsC;
    int a_stage;  // set by launch_smallk: full row tiles of op(A) copied to LDS directly
    // select_here: every workgroup takes the mode decision from the
    // statistics records of `sel` itself (workgroup 0 of each batch entry
    // publishes it to sel.st), in place of a selection launch
    int select_here;
    StatsArgs sel;
};
bool smallk_shape(int64_t m, int64_t n, int64_t k);
hipError_t launch_smallk(const SmallKArgs &g, hipStream_t s);

// Irregular-shape CGEMM (direct.hip): PA[i][l], PB[j][l] read from the
// stored matrices as in the split kernel; FP32 arithmetic.
struct DirectArgs {
    const float2 *A, *B;
    int64_t lda, ldb;
    int a_kcontig, a_conj, b_kcontig, b_conj;
    int64_t m, n, k;
    float2 *C;
    int64_t ldc;
    float2 alpha, beta;
    int beta_zero;
    float2 *partial;  // split-k partial tiles (workspace)
    int kl, ti, tj;   // set by the planner
    int64_t kchunk;
    int batch;                  // entries (blockIdx.z); 0 or 1: one GEMM
    int64_t bsA, bsB, bsC;      // elements between entries
    int64_t bsPartial;          // set by launch_direct
};
hipError_t launch_direct(DirectArgs d, hipStream_t s);
size_t direct_ws_bytes(int64_t m, int64_t n, int64_t k, int batch = 1);
// shapes sent to the irregular kernel in every mode
inline bool irregular_shape(int64_t m, int64_t n, int64_t k) { return m < 32 || n < 32 || k < 16; }

hipError_t launch_scale_c(float2 *C, int64_t m, int64_t n, int64_t ldc, float2 beta, int beta_zero,
                          hipStream_t s, int batch = 1, int64_t bsC = 0);

struct PermDesc {
    int rank;            // merged rank, <= kMaxRank
    int pow2;            // all extents powers of two
    int64_t ext[32];     // output extents (merged)
    int64_t istride[32]; // input stride of each output axis
    int log2ext[32];
};
constexpr int kMaxRank = 32;
hipError_t launch_permute(const float2 *x, float2 *y, int64_t total, const PermDesc &d,
                          hipStream_t s);

// One small contraction of a grouped launch (group.hip): output dimensions
// in C's row-major order (last fastest) with strides into A and B (0 where
// the operand lacks the label), summed dimensions stored fastest first.
constexpr int kSmallOut = 16, kSmallSum = 8;
struct SmallItem {
    const float2 *A, *B;
    float2 *C;
    int64_t n_out, n_sum;
    int nd_out, nd_sum;
    int64_t out_ext[kSmallOut], out_sa[kSmallOut], out_sb[kSmallOut];
    int64_t sum_ext[kSmallSum], sum_sa[kSmallSum], sum_sb[kSmallSum];
};
// block_start[i]: first block of item i (block_start[0] = 0), items and
// block_start in device memory.
hipError_t launch_group(const SmallItem *items, const int64_t *block_start, int count,
                        int64_t total_blocks, hipStream_t s);

hipError_t launch_accumulate_f64(const float2 *src, double *acc2, hipStream_t s);
hipError_t launch_accumulate_n_f64(const float2 *src, int64_t n, double *partials, int nblocks,
                                   double *acc2, hipStream_t s);
hipError_t launch_fidelity_f64(const float2 *a, const float2 *b, int64_t n, double *partials,
                               int nblocks, double *out4, hipStream_t s);
hipError_t launch_split_planar(int mode, int shift, const float2 *x, int64_t n, uint16_t *planes,
                               hipStream_t s);

}  // namespace qce
