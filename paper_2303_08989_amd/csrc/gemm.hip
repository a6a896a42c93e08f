// Complex GEMM on gfx950 matrix cores over split panels.
//
// C = alpha * op(A) op(B) + beta * C with the complex product written as four
// real products (Sec. 3): Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br.  Each real
// product is emulated from the split parts (Sec. 2.1, Eq. 2):
//   FP16X2:  hi*hi + (lo*hi + hi*lo) / 2^11        (3 MFMA products)
//   BF16X3:  b0*c0 + (b0*c1 + b1*c0 + b0*c2 + b1*c1 + b2*c0)   (6 products)
//   FP32:    x*y on the FP32 matrix instruction (the plain baseline)
// The leading product and the correction products go to separate FP32
// accumulators and are combined in the epilogue.  gfx950's f16/bf16 MFMA
// sums each instruction's products exactly and rounds once to nearest even
// (measured), so the leading term needs no separate round-to-nearest
// accumulation step (the paper's workaround for round-toward-zero inside the
// Tensor Core, Sec. 2.1).
//
// Mapping: the MFMA "A" operand is read from the op(B) panels (rows j) and
// the MFMA "B" operand from the op(A) panels (rows i), so D[j][i] = C[i][j]
// and the 32 lanes of an output row of a 32x32 MFMA block hold 32 consecutive
// rows i of column-major C: coalesced stores.
//
// One workgroup = 4 waves = a 128 x 128 complex tile; each wave owns 64 x 64
// (2 x 2 blocks of 32 x 32).  K advances one panel chunk per iteration with
// two LDS stages: global loads of chunk k+1 are issued before the MFMAs of
// chunk k and written to the other stage afterwards.
//
// Device-side dispatch (Sec. 4.2): in AUTO mode a single launch reads the
// mode flag written by the selection kernel and runs that mode's tile, so no
// host round trip and no launch of unselected kernels is needed.
//
// Split-k: when the output has fewer tiles than the device has CUs and k is
// long, blockIdx.y splits the k range; partial tiles are added in split order
// by gemm_reduce_kernel, which also applies the shift, alpha and beta.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "select.hpp"
#include "split_math.hpp"

namespace qce {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;

__device__ inline u32x4 neg_halves(u32x4 v) { return v ^ 0x80008000u; }

__device__ inline floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a),
                                                  __builtin_bit_cast(half8, b), c, 0, 0, 0);
}
__device__ inline floatx16 mfmab(u32x4 a, u32x4 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ inline floatx16 mfma32(float a, float b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Tile order: consecutive workgroup ids are dispatched round-robin over the
// 8 XCDs (each with its own L2).  Remap so that each XCD receives a
// contiguous range of tile ids, and walk tiles in groups of kGroupM tile-rows
// so that concurrently running tiles share A and B panels.
constexpr int kXcds = 8;
constexpr int kGroupM = 8;

__device__ inline void tile_of(int bid, int nbm, int nbn, int &mb, int &nb) {
    const int total = nbm * nbn;
    const int q = total / kXcds, rem = total % kXcds;
    const int x = bid % kXcds, local = bid / kXcds;
    const int id = (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + local;
    const int group = kGroupM * nbn;
    const int g = id / group;
    const int first = g * kGroupM;
    const int gm = min(nbm - first, kGroupM);
    const int in = id % group;
    mb = first + in % gm;
    nb = in / gm;
}

#define LDS_PTR(p) ((__attribute__((address_space(3))) void *)(p))

// Word 3 of a raw buffer descriptor on gfx9-family parts (32-bit data
// format; no swizzle, no index stride).
constexpr int kRsrcWord3 = 0x00020000;

// Wait until at most N vector-memory operations of this wave are
// outstanding (gfx9 s_waitcnt encoding: vmcnt in bits 3:0 and 15:14, expcnt
// and lgkmcnt left at their "no wait" maxima).
template <int N>
__device__ __attribute__((always_inline)) inline void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup barrier entered once at most N vector-memory operations and no
// LDS operation of this wave are outstanding.  The scheduling fences keep
// every instruction on its side, so no LDS read slips between the wait and
// the barrier; the wait is an ordinary instruction the compiler's own wait
// insertion takes into account.
template <int N>
__device__ __attribute__((always_inline)) inline void wait_barrier() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
    asm volatile("s_barrier" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// A chunk of zeros in global memory: the source of the padding chunk that
// makes a block's chunk count even (it adds exact zeros to the products).
__device__ __attribute__((aligned(256))) uint4 g_zero_chunk[PanelGeom<QCE_MODE_BF16X3>::kChunkBytes / 16];

// c < n ? p : z for wave-uniform operands, as one scalar compare and select
// (the compiler would otherwise turn it into branches, which split the
// scheduling region of the k-loop).
__device__ __attribute__((always_inline)) inline const char *chunk_src(int c, int n, const char *p,
                                                                      const char *z) {
    const char *r;
    asm("s_cmp_lt_i32 %1, %2\n\ts_cselect_b64 %0, %3, %4" : "=s"(r) : "s"(c), "s"(n), "s"(p), "s"(z) : "scc");
    return r;
}

// Hides a value's origin from the optimizer (no instruction is emitted).
__device__ __attribute__((always_inline)) inline void opaque(u32x4 &v) { asm volatile("" : "+v"(v)); }

// LDS stages of the chunk ring per mode (stage = one chunk of each operand)
template <int MODE> struct Stages { static constexpr int kNS = 4; };
template <> struct Stages<QCE_MODE_BF16X3> { static constexpr int kNS = 3; };

template <int MODE> struct Acc;
template <> struct Acc<QCE_MODE_FP16X2> { floatx16 re_m[2][2], im_m[2][2], re_c[2][2], im_c[2][2]; };
template <> struct Acc<QCE_MODE_BF16X3> { floatx16 re_m[2][2], im_m[2][2], re_c[2][2], im_c[2][2]; };
// FP32: Re = sum Ar Br - sum Ai Bi with the subtracted sum in re_n (no
// sign flip of a fragment: a vector instruction between two FP32 MFMAs does
// not overlap them, it adds its own latency)
template <> struct Acc<QCE_MODE_FP32> { floatx16 re_m[2][2], im_m[2][2], re_n[2][2]; };

// 12 MFMAs of one 32x32 block for one k16 step (planes: 0 = hi(re),
// 1 = lo(re), 2 = hi(im), 3 = lo(im); nx = -hi(im), -lo(im) of x)
__device__ __attribute__((always_inline)) inline void fp16x2_block(const u32x4 *x, const u32x4 *nx,
                                                                   const u32x4 *y, floatx16 &re_m,
                                                                   floatx16 &im_m, floatx16 &re_c,
                                                                   floatx16 &im_c) {
    re_c = mfma16(x[1], y[0], re_c);
    re_c = mfma16(x[0], y[1], re_c);
    re_c = mfma16(nx[1], y[2], re_c);
    re_c = mfma16(nx[0], y[3], re_c);
    im_c = mfma16(x[1], y[2], im_c);
    im_c = mfma16(x[0], y[3], im_c);
    im_c = mfma16(x[3], y[0], im_c);
    im_c = mfma16(x[2], y[1], im_c);
    re_m = mfma16(x[0], y[0], re_m);
    re_m = mfma16(nx[0], y[2], re_m);
    im_m = mfma16(x[0], y[2], im_m);
    im_m = mfma16(x[2], y[0], im_m);
}

// 24 MFMAs of one 32x32 block for one k16 step (planes: b0, b1, b2 of re,
// then of im; x from op(B), y from op(A))
__device__ __attribute__((always_inline)) inline void bf16x3_block(const u32x4 *x, const u32x4 *y, floatx16 &re_m,
                                                                   floatx16 &im_m, floatx16 &re_c, floatx16 &im_c) {
    const u32x4 nx[3] = {neg_halves(x[3]), neg_halves(x[4]), neg_halves(x[5])};
    // corrections, smallest first: (2,0) (1,1) (0,2) (1,0) (0,1)
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const int i = t == 0 ? 2 : t == 1 ? 1 : t == 2 ? 0 : t == 3 ? 1 : 0;
        const int j = t == 0 ? 0 : t == 1 ? 1 : t == 2 ? 2 : t == 3 ? 0 : 1;
        re_c = mfmab(x[i], y[j], re_c);
        re_c = mfmab(nx[i], y[3 + j], re_c);
        im_c = mfmab(x[i], y[3 + j], im_c);
        im_c = mfmab(x[3 + i], y[j], im_c);
    }
    re_m = mfmab(x[0], y[0], re_m);
    re_m = mfmab(nx[0], y[3], re_m);
    im_m = mfmab(x[0], y[3], im_m);
    im_m = mfmab(x[3], y[0], im_m);
}

// ---------------------------------------------------------------------------
// Fragments of one chunk in registers (all rows of the wave's 64 x 64 tile,
// 16 k-values) and the MFMAs of one chunk.  The k-loop keeps two such sets:
// chunk i's MFMAs run from one while chunk i+1's fragments are read into the
// other.
// ---------------------------------------------------------------------------
template <int MODE> struct Frag;
template <> struct Frag<QCE_MODE_FP16X2> {
    static constexpr int kP = 4;  // planes: hi(re), lo(re), hi(im), lo(im)
    static constexpr int kReads = 16, kMfma = 48, kMfmaPerRead = 2;
    u32x4 x[2][4], y[2][4];
};
template <> struct Frag<QCE_MODE_BF16X3> {
    static constexpr int kP = 6;  // planes: b0, b1, b2 of re; b0, b1, b2 of im
    static constexpr int kReads = 24, kMfma = 96, kMfmaPerRead = 3;
    u32x4 x[2][6], y[2][6];
};
// FP32: per k8 half s and 32-row block, four consecutive k-values of re and
// of im; MFMA step j takes value j, so lanes 0-31 and 32-63 supply
// k = 8s + j and 8s + 4 + j (the same pairing for both operands, so every k
// is summed once).
template <> struct Frag<QCE_MODE_FP32> {
    static constexpr int kReads = 16, kMfma = 128, kMfmaPerRead = 4;
    f32x4 xr[2][2], xi[2][2], yr[2][2], yi[2][2];  // [s][block]
};

// Per-chunk counts of a wave with WB x WB blocks of 32 x 32 (WB = 2: the
// 128 x 128 tile, WB = 1: the 64 x 64 tile): fragment reads and MFMAs.
template <int MODE, int WB> struct ChunkWork {
    static constexpr int kReads = Frag<MODE>::kReads * WB / 2;
    static constexpr int kMfma = Frag<MODE>::kMfma * WB * WB / 4;
};

// LDS offset of (plane, row, granule) in a stage holding ROWS rows of each
// plane (the panel chunk, or the half of it a 64-row tile copies); the
// granule swizzle depends on the row's low bits only, so either half of a
// chunk keeps the panel's swizzle.
template <int MODE, int ROWS>
__device__ __host__ constexpr int lds_offset(int plane, int row, int granule) {
    using G = PanelGeom<MODE>;
    return plane * ROWS * G::kRowBytes + row * G::kRowBytes + ((granule ^ G::swz(row)) << 4);
}

template <int MODE, int ROWS>
__device__ __attribute__((always_inline)) inline void load_part(u32x4 *dst, const char *s, int row, int gr) {
#pragma unroll
    for (int p = 0; p < Frag<MODE>::kP; ++p)
        dst[p] = *reinterpret_cast<const u32x4 *>(s + lds_offset<MODE, ROWS>(p, row, gr));
}

// Every fragment of one chunk: x rows from the B panel (sx), y rows from
// the A panel (sy); r0 = wave's first x row + lane%32, q0 likewise for y.
template <int MODE, int WB>
__device__ __attribute__((always_inline)) inline void load_chunk(Frag<MODE> &f, const char *sx, const char *sy,
                                                                 int rx0, int ry0, int lane) {
    constexpr int kRows = 64 * WB;  // rows of each plane in the stage
    const int hi = lane >> 5;
    if constexpr (MODE == QCE_MODE_FP32) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int b = 0; b < WB; ++b) {
                f.xr[s][b] = *reinterpret_cast<const f32x4 *>(sx + lds_offset<MODE, kRows>(0, rx0 + 32 * b, 2 * s + hi));
                f.xi[s][b] = *reinterpret_cast<const f32x4 *>(sx + lds_offset<MODE, kRows>(1, rx0 + 32 * b, 2 * s + hi));
                f.yr[s][b] = *reinterpret_cast<const f32x4 *>(sy + lds_offset<MODE, kRows>(0, ry0 + 32 * b, 2 * s + hi));
                f.yi[s][b] = *reinterpret_cast<const f32x4 *>(sy + lds_offset<MODE, kRows>(1, ry0 + 32 * b, 2 * s + hi));
            }
    } else {
        load_part<MODE, kRows>(f.x[0], sx, rx0, hi);
        load_part<MODE, kRows>(f.y[0], sy, ry0, hi);
        if constexpr (WB == 2) {
            load_part<MODE, kRows>(f.y[1], sy, ry0 + 32, hi);
            load_part<MODE, kRows>(f.x[1], sx, rx0 + 32, hi);
        }
    }
}

template <int MODE>
__device__ __attribute__((always_inline)) inline void mma_block(const Frag<MODE> &f, int ub, int vb, Acc<MODE> &acc) {
    if constexpr (MODE == QCE_MODE_FP16X2) {
        const u32x4 nx[2] = {neg_halves(f.x[ub][2]), neg_halves(f.x[ub][3])};
        fp16x2_block(f.x[ub], nx, f.y[vb], acc.re_m[ub][vb], acc.im_m[ub][vb], acc.re_c[ub][vb], acc.im_c[ub][vb]);
    } else if constexpr (MODE == QCE_MODE_BF16X3) {
        bf16x3_block(f.x[ub], f.y[vb], acc.re_m[ub][vb], acc.im_m[ub][vb], acc.re_c[ub][vb], acc.im_c[ub][vb]);
    } else {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float a_r = f.xr[s][ub][j], a_i = f.xi[s][ub][j];
                const float b_r = f.yr[s][vb][j], b_i = f.yi[s][vb][j];
                acc.re_m[ub][vb] = mfma32(a_r, b_r, acc.re_m[ub][vb]);
                acc.re_n[ub][vb] = mfma32(a_i, b_i, acc.re_n[ub][vb]);
                acc.im_m[ub][vb] = mfma32(a_r, b_i, acc.im_m[ub][vb]);
                acc.im_m[ub][vb] = mfma32(a_i, b_r, acc.im_m[ub][vb]);
            }
    }
}

__device__ __attribute__((always_inline)) inline void opaque(f32x4 &v) { asm volatile("" : "+v"(v)); }

template <int MODE, int WB>
__device__ __attribute__((always_inline)) inline void opaque_frag(Frag<MODE> &f) {
    if constexpr (MODE == QCE_MODE_FP32) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int b = 0; b < WB; ++b) {
                opaque(f.xr[s][b]);
                opaque(f.xi[s][b]);
                opaque(f.yr[s][b]);
                opaque(f.yi[s][b]);
            }
    } else {
#pragma unroll
        for (int p = 0; p < Frag<MODE>::kP; ++p)
#pragma unroll
            for (int b = 0; b < WB; ++b) {
                opaque(f.x[b][p]);
                opaque(f.y[b][p]);
            }
    }
}

template <int MODE, int WB>
__device__ __attribute__((always_inline)) inline void mma_chunk(const Frag<MODE> &f, Acc<MODE> &acc) {
    mma_block<MODE>(f, 0, 0, acc);
    if constexpr (WB == 2) {
        mma_block<MODE>(f, 0, 1, acc);
        mma_block<MODE>(f, 1, 0, acc);
        mma_block<MODE>(f, 1, 1, acc);
    }
}

template <int MODE> constexpr int smem_bytes() {
    return Stages<MODE>::kNS * 2 * PanelGeom<MODE>::kChunkBytes;
}
constexpr int kSmemBytes = smem_bytes<QCE_MODE_BF16X3>();  // largest mode
static_assert(smem_bytes<QCE_MODE_FP16X2>() <= kSmemBytes && smem_bytes<QCE_MODE_FP32>() <= kSmemBytes,
              "LDS budget");
static_assert(kSmemBytes <= 160 * 1024, "gfx950 LDS");

// The tile of one workgroup for one mode: TILE x TILE outputs (128: four
// waves of 64 x 64; 64: four waves of 32 x 32, reading half of each panel
// chunk).  blockIdx.y selects a range of k (split-k): with several ranges
// the unscaled partial tile goes to g.partial and gemm_reduce_kernel
// finishes the sum and the epilogue.
// bid: the tile's index (mapped to a tile by tile_of), ks: its k range,
// split: the k range is one of several (the partial tile is written).
template <int MODE, int TILE>
__device__ __attribute__((always_inline)) inline void gemm_body(const GemmArgs &g, int nbm, int nbn,
                                                                int mode, char *smem_raw, int bid, int ks,
                                                                bool split) {
    int shift_total = 0;
    if (MODE == QCE_MODE_FP16X2 && mode == QCE_MODE_FP16X2_SCALED && g.st)
        shift_total = g.st->shift[0] + g.st->shift[1];

    using G = PanelGeom<MODE>;
    static_assert(TILE == 128 || TILE == 64, "tile shapes");
    constexpr int kWB = TILE / 64;                  // 32 x 32 blocks per wave and dimension
    constexpr int kCB = G::kChunkBytes;             // one panel chunk (128 rows) in HBM
    constexpr int kOB = kCB * TILE / kPanelRows;    // the rows of it one operand copies
    constexpr int kHalf = G::kPlaneBytes / 2;       // a 64-row half of one plane
    constexpr int kNS = Stages<MODE>::kNS;          // LDS stages in the ring
    constexpr int kL1 = kOB / (16 * kThreads);      // 16-byte copies per thread per operand chunk
    constexpr int kL = 2 * kL1;                      // per stage (both operands)
    static_assert(kOB % (16 * kThreads) == 0, "whole copies");
    typedef char Stage[2][kOB];
    Stage *smem = reinterpret_cast<Stage *>(smem_raw);

    int mb, nb;
    tile_of(bid, nbm, nbn, mb, nb);
    const int64_t kpad = round_up(g.k, kKPad);
    const int nkb = (int)(kpad / PanelFmt<MODE>::kBK);
    // this split's chunk range (split boundaries are multiples of the chunk depth)
    const int kb0 = (int)((int64_t)ks * g.kpad_per_split / PanelFmt<MODE>::kBK);
    const int kb1 = min(nkb, kb0 + (int)(g.kpad_per_split / PanelFmt<MODE>::kBK));
    const int nk = max(0, kb1 - kb0);
    // panel row block of the tile and, for 64-row tiles, its half
    const int64_t pnb = (int64_t)nb * TILE / kPanelRows, pmb = (int64_t)mb * TILE / kPanelRows;
    const int hnb = TILE == 64 ? (nb & 1) : 0, hmb = TILE == 64 ? (mb & 1) : 0;
    const char *px = static_cast<const char *>(g.panelsB) + (pnb * nkb + kb0) * kCB;
    const char *py = static_cast<const char *>(g.panelsA) + (pmb * nkb + kb0) * kCB;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wu = w >> 1, wv = w & 1;

    Acc<MODE> acc;
    {
        floatx16 z;
#pragma unroll
        for (int r = 0; r < 16; ++r) z[r] = 0.f;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc.re_m[a][b] = z;
                acc.im_m[a][b] = z;
                if constexpr (MODE != QCE_MODE_FP32) {
                    acc.re_c[a][b] = z;
                    acc.im_c[a][b] = z;
                } else {
                    acc.re_n[a][b] = z;
                }
            }
    }

    // Chunk c of both operands goes straight from global memory into LDS
    // (global_load_lds: lane l of a wave writes 16 bytes at the wave's LDS
    // address + 16 l), kNS - 1 chunks ahead of the MFMAs.
    //
    // The k-steps run in pairs (two register sets, no dynamic indexing); an
    // odd count gets one chunk of zeros, whose products add exact zeros.
    // Every k-step issues one chunk, and chunks past the end come from the
    // zero chunk, so the number of copies outstanding after a chunk is a
    // constant and the loop body has no branches to split the schedule.
    if (nk > 0) {
        const int nk2 = nk + (nk & 1);
        const char *zero = reinterpret_cast<const char *>(g_zero_chunk);
        asm volatile("" : "+s"(zero));   // computed once, kept in scalar registers
        // Copies are buffer loads into LDS: the chunk's address lives in a
        // scalar buffer descriptor (one chunk long, so no access can leave
        // it), the lane's byte offset in one loop-invariant vector register,
        // the copy's offset within the chunk and the LDS destination (M0) in
        // scalar registers (the wave index read once).  Issuing a copy then
        // takes no vector instruction, which matters because a vector
        // instruction between two FP32 MFMAs adds its full latency.
        const int wsc = __builtin_amdgcn_readfirstlane(w);
        // source byte of this lane's first copy: the whole chunk is copied
        // in order for 128-row tiles; a 64-row tile copies, plane by plane,
        // the half holding its rows (LDS byte b of the stage comes from
        // plane b / kHalf, byte kHalf * half + b % kHalf of that plane)
        const unsigned off_x = TILE == kPanelRows ? (unsigned)tid * 16u
                             : (unsigned)((tid * 16 / kHalf) * G::kPlaneBytes + (tid * 16) % kHalf + hnb * kHalf);
        const unsigned off_y = TILE == kPanelRows ? (unsigned)tid * 16u
                             : (unsigned)((tid * 16 / kHalf) * G::kPlaneBytes + (tid * 16) % kHalf + hmb * kHalf);
        // source distance between a thread's consecutive copies
        constexpr int kSrcStep = TILE == kPanelRows ? kThreads * 16 : 2 * kThreads * 16;
        static_assert(TILE == kPanelRows || kHalf % (kThreads * 16) == 0 || (kThreads * 16) % kHalf == 0,
                      "copy rows align with half planes");
        auto issue_to = [&](int c, int stage) {
            const char *gx = chunk_src(c, nk, px + (int64_t)c * kCB, zero);
            const char *gy = chunk_src(c, nk, py + (int64_t)c * kCB, zero);
            const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void *)gx, (short)0, kCB, kRsrcWord3);
            const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc((void *)gy, (short)0, kCB, kRsrcWord3);
            char *lx = smem[stage][0];
            char *ly = smem[stage][1];
#pragma unroll
            for (int i = 0; i < kL1; ++i) {
                const int we = (wsc * 64 + i * kThreads) * 16;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, LDS_PTR(lx + we), 16, off_x, i * kSrcStep, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ry, LDS_PTR(ly + we), 16, off_y, i * kSrcStep, 0, 0);
            }
        };
        const int l32 = lane & 31;
        const int rx0 = wu * 32 * kWB + l32, ry0 = wv * 32 * kWB + l32;
        // 64 KB as a value the optimizer cannot see through: the address
        // registers built on it are computed once, outside the loop
        int hi_base = 65536;
        asm volatile("" : "+s"(hi_base));
        // One k-step: chunk `it` is in registers (fc).  Wait for chunk it+1
        // (this thread's copies: kNS - 2 later chunks may be outstanding) and
        // for this wave's reads of chunk `it`; after the barrier every wave
        // has them, so chunk it's stage takes chunk it + kNS.  Chunk it+1's
        // fragments are then read into fn while chunk it's MFMAs run: the
        // reads first, spread over the first MFMAs, then the copies.
        // `stage` (= it % kNS) is a compile-time constant where the loop
        // below is unrolled by the ring length (FP32 mode, whose MFMAs do not
        // overlap vector instructions): then every LDS read address is a
        // loop-invariant register plus an immediate offset.  The other modes
        // keep a run-time stage: their fragment reads would need more
        // address registers than remain beside 256 accumulators.
        auto step = [&](int it, auto stage, const Frag<MODE> &fc, Frag<MODE> &fn) {
            wait_barrier<(kNS - 2) * kL>();
            // (reads before copies in program order: the compiler cannot
            // tell that they touch different stages and keeps their order)
            const int cur = stage;
            const int ns = (cur + 1) % kNS;
            if constexpr (std::is_integral_v<decltype(stage)>) {
                load_chunk<MODE, kWB>(fn, smem[ns][0], smem[ns][1], rx0, ry0, lane);
            } else {
                // stages past 64 KB are read from a second base (an LDS
                // read's immediate offset stops at 64 KB)
                constexpr int kNext = (decltype(stage)::value + 1) % kNS;
                const char *b = kNext * 2 * kOB < 65536 ? smem[kNext][0]
                                                        : smem_raw + hi_base + (kNext * 2 * kOB - 65536);
                load_chunk<MODE, kWB>(fn, b, b + kOB, rx0, ry0, lane);
            }
            issue_to(it + kNS, cur);
            mma_chunk<MODE, kWB>(fc, acc);
            // Interleave: one fragment read every kA MFMAs, then one copy
            // every kB MFMAs, then the remaining MFMAs.  The reads are
            // spread rather than bunched because the four waves share the
            // CU's LDS bandwidth (~128 B per clock): two 1 KB wave reads per
            // 32-cycle f16 MFMA on every SIMD ask for twice that and stall
            // the MFMAs; one per kA MFMAs stays well below it.
            constexpr int kReads = ChunkWork<MODE, kWB>::kReads, kMfma = ChunkWork<MODE, kWB>::kMfma;
            constexpr int kCopies = 2 * kL1;
            // (the 64 x 64 tile has fewer MFMAs per read: leave room for the copies)
            constexpr int kAFit = (kMfma - kCopies) / kReads > 0 ? (kMfma - kCopies) / kReads : 1;
            constexpr int kA = kAFit < Frag<MODE>::kMfmaPerRead ? kAFit : Frag<MODE>::kMfmaPerRead;
            constexpr int kB = (kMfma - kA * kReads) / (kCopies + 1) > 0 ? (kMfma - kA * kReads) / (kCopies + 1) : 1;
            static_assert(kA * kReads + kB * kCopies <= kMfma, "interleave exceeds the chunk's MFMAs");
#pragma unroll
            for (int i = 0; i < kReads; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, kA, 0);    // MFMA
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);     // LDS read
            }
#pragma unroll
            for (int i = 0; i < kCopies; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, kB, 0);
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);     // VMEM read (copy to LDS)
            }
            __builtin_amdgcn_sched_group_barrier(0x008, kMfma - kA * kReads - kB * kCopies, 0);
        };
        Frag<MODE> f0, f1;
#pragma unroll
        for (int c = 0; c < kNS; ++c) issue_to(c, c);
        wait_barrier<(kNS - 1) * kL>();  // chunk 0
        load_chunk<MODE, kWB>(f0, smem[0][0], smem[0][1], rx0, ry0, lane);
        // keeps the optimizer from merging these reads with the loop's
        // reads into f0 as one read at the top of the loop
        opaque_frag<MODE, kWB>(f0);
        // (the last k-step reads a chunk past the end, unused)
        if constexpr (MODE == QCE_MODE_FP32 && kNS == 4) {
            using S0 = std::integral_constant<int, 0>;
            using S1 = std::integral_constant<int, 1>;
            using S2 = std::integral_constant<int, 2>;
            using S3 = std::integral_constant<int, 3>;
            int it = 0;
            for (; it + 4 <= nk2; it += 4) {
                step(it, S0{}, f0, f1);
                step(it + 1, S1{}, f1, f0);
                step(it + 2, S2{}, f0, f1);
                step(it + 3, S3{}, f1, f0);
            }
            if (it < nk2) {   // two k-steps left: stages 0 and 1 again
                step(it, S0{}, f0, f1);
                step(it + 1, S1{}, f1, f0);
            }
        } else {
            for (int it = 0; it < nk2; it += 2) {
                step(it, it % kNS, f0, f1);
                step(it + 1, (it + 1) % kNS, f1, f0);
            }
        }
        // the copies issued by the last k-steps land before the end
        wait_vmcnt<0>();
    }

    // epilogue: D[j][i] -> C[i][j] (or the split's partial tile)
    const bool alpha_one = g.alpha.x == 1.f && g.alpha.y == 0.f;
    const int l32 = lane & 31, hi = lane >> 5;
#pragma unroll
    for (int ub = 0; ub < kWB; ++ub)
#pragma unroll
        for (int vb = 0; vb < kWB; ++vb) {
            const int64_t i = (int64_t)mb * TILE + wv * 32 * kWB + vb * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t j = (int64_t)nb * TILE + wu * 32 * kWB + ub * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                if (i >= g.m || j >= g.n) continue;
                float re, im;
                if constexpr (MODE == QCE_MODE_FP16X2) {
                    re = acc.re_m[ub][vb][r] + acc.re_c[ub][vb][r] * (1.0f / 2048.0f);
                    im = acc.im_m[ub][vb][r] + acc.im_c[ub][vb][r] * (1.0f / 2048.0f);
                } else if constexpr (MODE == QCE_MODE_BF16X3) {
                    re = acc.re_m[ub][vb][r] + acc.re_c[ub][vb][r];
                    im = acc.im_m[ub][vb][r] + acc.im_c[ub][vb][r];
                } else {
                    re = acc.re_m[ub][vb][r] - acc.re_n[ub][vb][r];
                    im = acc.im_m[ub][vb][r];
                }
                if (split) {
                    g.partial[(int64_t)ks * g.m * g.n + i + j * g.m] = make_float2(re, im);
                    continue;
                }
                if (shift_total) {
                    re = ldexpf(re, -shift_total);
                    im = ldexpf(im, -shift_total);
                }
                float2 out;
                if (alpha_one) {
                    out = make_float2(re, im);
                } else {
                    out = make_float2(g.alpha.x * re - g.alpha.y * im, g.alpha.x * im + g.alpha.y * re);
                }
                float2 *cp = g.C + i + j * g.ldc;
                if (!g.beta_zero) {
                    const float2 c = *cp;
                    out.x += g.beta.x * c.x - g.beta.y * c.y;
                    out.y += g.beta.x * c.y + g.beta.y * c.x;
                }
                *cp = out;
            }
        }
}

// Batched launches: entry blockIdx.z works on its own panels, C, partial
// tiles and device state.
__device__ inline void select_entry(GemmArgs &g, int64_t z) {
    g.panelsA = static_cast<const char *>(g.panelsA) + z * g.bsA;
    g.panelsB = static_cast<const char *>(g.panelsB) + z * g.bsB;
    g.C += z * g.bsC;
    if (g.st) g.st += z;
    if (g.partial) g.partial += z * g.bsPartial;
}

// Forced mode: one kernel per mode and tile.  A 128 x 128 tile holds one
// workgroup per CU; a 64 x 64 tile needs half the LDS and registers, so two
// fit.
template <int MODE, int TILE>
__global__ __launch_bounds__(kThreads, TILE == 128 ? 1 : 2) void gemm_kernel(GemmArgs g, int nbm, int nbn) {
    __shared__ __attribute__((aligned(16))) char smem[smem_bytes<MODE>() * TILE / kPanelRows];
    select_entry(g, blockIdx.z);
    gemm_body<MODE, TILE>(g, nbm, nbn, g.forced_mode, smem, blockIdx.x, blockIdx.y, gridDim.y > 1);
}

// Statistics-selected mode: one launch that reads the device mode flag and
// runs the selected mode's tile (the others never start).
template <int TILE>
__global__ __launch_bounds__(kThreads, TILE == 128 ? 1 : 2) void gemm_auto_kernel(GemmArgs g, int nbm, int nbn) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemBytes * TILE / kPanelRows];
    select_entry(g, blockIdx.z);
    const int mode = g.st->mode;
    const int bid = blockIdx.x, ks = blockIdx.y;
    const bool split = gridDim.y > 1;
    if (mode == QCE_MODE_FP16X2 || mode == QCE_MODE_FP16X2_SCALED)
        gemm_body<QCE_MODE_FP16X2, TILE>(g, nbm, nbn, mode, smem, bid, ks, split);
    else if (mode == QCE_MODE_BF16X3)
        gemm_body<QCE_MODE_BF16X3, TILE>(g, nbm, nbn, mode, smem, bid, ks, split);
    else
        gemm_body<QCE_MODE_FP32, TILE>(g, nbm, nbn, mode, smem, bid, ks, split);
}

// Split-k: add the partial tiles in split order, then shift / alpha / beta
// (output element o of batch entry z).
__device__ inline void reduce_one(GemmArgs g, int splits, int64_t o, int64_t z) {
    select_entry(g, z);
    const int mode = g.st ? g.st->mode : g.forced_mode;
    const int shift_total = (mode == QCE_MODE_FP16X2_SCALED && g.st) ? g.st->shift[0] + g.st->shift[1] : 0;
    float re = 0.f, im = 0.f;
    for (int s = 0; s < splits; ++s) {
        const float2 p = g.partial[(int64_t)s * g.m * g.n + o];
        re += p.x;
        im += p.y;
    }
    if (shift_total) {
        re = ldexpf(re, -shift_total);
        im = ldexpf(im, -shift_total);
    }
    const int64_t i = o % g.m, j = o / g.m;
    float2 out = make_float2(g.alpha.x * re - g.alpha.y * im, g.alpha.x * im + g.alpha.y * re);
    if (g.alpha.x == 1.f && g.alpha.y == 0.f) out = make_float2(re, im);
    float2 *cp = g.C + i + j * g.ldc;
    if (!g.beta_zero) {
        const float2 c = *cp;
        out.x += g.beta.x * c.x - g.beta.y * c.y;
        out.y += g.beta.x * c.y + g.beta.y * c.x;
    }
    *cp = out;
}

__global__ __launch_bounds__(kThreads) void gemm_reduce_kernel(GemmArgs g, int splits) {
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o >= g.m * g.n) return;
    reduce_one(g, splits, o, blockIdx.z);
}

// ---------------------------------------------------------------------------
// Grouped GEMM: GEMMs of different shapes (each possibly a batch) in one
// persistent launch.  The entries' tiles form one sequence (each entry's
// first tile id a multiple of 8, entries ordered by tile cost, heaviest
// first); every XCD owns the ids congruent to its index mod 8 and hands them
// out in increasing order through a device counter, so each XCD works on all
// entries at once, heaviest tiles first, and the tiles of one entry that an
// XCD receives are neighbours (tile_of's XCD ranges).  A workgroup takes
// tiles until its XCD's ids run out; each tile reads its own entry's device
// mode flag, so FP16X2, BF16X3 and FP32 tiles run side by side.  The last
// workgroup to finish clears the counters for the next launch (no memset,
// so the launch can sit in a captured graph).
// ---------------------------------------------------------------------------
__device__ inline int find_entry(const GroupGemmEntry *__restrict__ e, int count, int64_t t, bool red) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((red ? e[mid].red_start : e[mid].tile_start) <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int TILE>
__global__ __launch_bounds__(kThreads, TILE == 128 ? 1 : 2) void gemm_grouped_kernel(
    const GroupGemmEntry *__restrict__ ents, int count, int64_t total, unsigned int *queue) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemBytes * TILE / kPanelRows];
    __shared__ int64_t next;
    const int xcd = blockIdx.x % kXcds;
    for (;;) {
        if (threadIdx.x == 0) next = (int64_t)atomicAdd(&queue[xcd], 1u) * kXcds + xcd;
        __syncthreads();
        const int64_t t = next;
        __syncthreads();  // every wave has read `next`, and the last tile's LDS reads are done
        if (t >= total) break;
        const int e = find_entry(ents, count, t, false);
        const int64_t j = t - ents[e].tile_start;
        if (j >= ents[e].tiles) continue;  // padding between entries
        GemmArgs g = ents[e].g;
        const int nbm = ents[e].nbm, nbn = ents[e].nbn, nsplit = ents[e].nsplit;
        const int64_t per_z = (int64_t)nbm * nbn * nsplit;
        const int64_t z = j / per_z, r = j % per_z;
        const int ks = (int)(r / ((int64_t)nbm * nbn)), bid = (int)(r % ((int64_t)nbm * nbn));
        select_entry(g, z);
        const int mode = g.st ? g.st->mode : g.forced_mode;
        if (mode == QCE_MODE_FP16X2 || mode == QCE_MODE_FP16X2_SCALED)
            gemm_body<QCE_MODE_FP16X2, TILE>(g, nbm, nbn, mode, smem, bid, ks, nsplit > 1);
        else if (mode == QCE_MODE_BF16X3)
            gemm_body<QCE_MODE_BF16X3, TILE>(g, nbm, nbn, mode, smem, bid, ks, nsplit > 1);
        else
            gemm_body<QCE_MODE_FP32, TILE>(g, nbm, nbn, mode, smem, bid, ks, nsplit > 1);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[kXcds], 1u) == gridDim.x - 1) {
            // every workgroup has taken its last id: no counter is read again
            for (int x = 0; x <= kXcds; ++x) atomicExch(&queue[x], 0u);
        }
    }
}

// Split-k sums of the grouped launch's entries that split k.
__global__ __launch_bounds__(kThreads) void gemm_grouped_reduce_kernel(const GroupGemmEntry *__restrict__ ents,
                                                                       int count) {
    const int64_t b = blockIdx.x;
    const int e = find_entry(ents, count, b, true);
    const int64_t j = b - ents[e].red_start;
    if (j >= ents[e].red_blocks || ents[e].nsplit <= 1) return;
    const GemmArgs &g = ents[e].g;
    const int64_t per_z = (g.m * g.n + kThreads - 1) / kThreads;
    const int64_t z = j / per_z;
    const int64_t o = (j % per_z) * kThreads + threadIdx.x;
    if (o >= g.m * g.n) return;
    reduce_one(g, ents[e].nsplit, o, z);
}

__global__ void scale_c_kernel(float2 *C, int64_t m, int64_t n, int64_t ldc, float2 beta,
                               int beta_zero, int64_t bsC) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * n) return;
    C += (int64_t)blockIdx.z * bsC;
    const int64_t i = t % m, j = t / m;
    float2 *cp = C + i + j * ldc;
    if (beta_zero) {
        *cp = make_float2(0.f, 0.f);
    } else {
        const float2 c = *cp;
        *cp = make_float2(beta.x * c.x - beta.y * c.y, beta.x * c.y + beta.y * c.x);
    }
}

// ---------------------------------------------------------------------------
// Short k, narrow C (tall-skinny shapes such as 65536 x 64 x 64): the split
// is done as the operands are loaded, with no panel pass.  A workgroup owns
// 128 rows of C (four waves of 32) and all of its <= 64 columns.  It splits
// op(B) (k x n, at most 128 x 64) into LDS planes once; each wave then loads
// its rows of op(A) chunk by chunk (16 k-values) straight from global memory
// into registers, splits them there, and runs the same MFMA sequence per
// chunk as the panel kernel (the same fragments in the same order, so the
// sums are the same).  Only op(A) and C stream through HBM.
// ---------------------------------------------------------------------------
constexpr int kSkRows = 128;  // rows of C per workgroup
constexpr int kSkCols = 64;   // columns of C: two 32-column blocks

// LDS row of op(B) (one column j of C): kpad values plus 16 bytes, a stride
// that puts 8 consecutive rows' 16-byte fragment reads on distinct banks
__host__ __device__ constexpr int sk_row_bytes(int kpad, int elem) { return kpad * elem + 16; }
__host__ __device__ constexpr int sk_lds_bytes(int kpad) {
    // the largest mode: BF16X3 (6 two-byte planes) vs FP32 (2 four-byte planes)
    return 6 * kSkCols * sk_row_bytes(kpad, 2) > 2 * kSkCols * sk_row_bytes(kpad, 4)
               ? 6 * kSkCols * sk_row_bytes(kpad, 2)
               : 2 * kSkCols * sk_row_bytes(kpad, 4);
}

// The op(A) ring of the k <= 64 kernel: kSkRing stages of one chunk each
// (16 k-values x 128 rows, [k][row]: k-value kk of the chunk's rows is 1 KB
// at kk * 1024).
constexpr int kSkRing = 4;
constexpr int kSkChunkBytes = 16 * kSkRows * 8;
constexpr int kSkStageBytes = kSkRing * kSkChunkBytes;

// Eight 8-byte LDS reads of one lane's op(A) values in a ring stage, at
// addr + 1024 d for its k-offsets d (0-7, or 0-3 and 8-11 for the FP32
// fragment), as one asm block that also waits for them.  The compiler
// would put a wait for every copy still in flight into the ring before an
// LDS read it sees (it cannot tell the stages apart), which undoes the
// ring; the ring's own counted wait and barrier order these reads.
template <bool kFp32Frag>
__device__ __attribute__((always_inline)) inline void ring_read8(uint32_t addr, float2 (&v)[8]) {
    f32x4 r0, r1, r2, r3;
    if constexpr (kFp32Frag) {
        asm volatile(
            "ds_read2st64_b64 %0, %4 offset0:0 offset1:2\n\t"
            "ds_read2st64_b64 %1, %4 offset0:4 offset1:6\n\t"
            "ds_read2st64_b64 %2, %4 offset0:16 offset1:18\n\t"
            "ds_read2st64_b64 %3, %4 offset0:20 offset1:22\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
            : "v"(addr)
            : "memory");
    } else {
        asm volatile(
            "ds_read2st64_b64 %0, %4 offset0:0 offset1:2\n\t"
            "ds_read2st64_b64 %1, %4 offset0:4 offset1:6\n\t"
            "ds_read2st64_b64 %2, %4 offset0:8 offset1:10\n\t"
            "ds_read2st64_b64 %3, %4 offset0:12 offset1:14\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
            : "v"(addr)
            : "memory");
    }
    v[0] = make_float2(r0.x, r0.y);
    v[1] = make_float2(r0.z, r0.w);
    v[2] = make_float2(r1.x, r1.y);
    v[3] = make_float2(r1.z, r1.w);
    v[4] = make_float2(r2.x, r2.y);
    v[5] = make_float2(r2.z, r2.w);
    v[6] = make_float2(r3.x, r3.y);
    v[7] = make_float2(r3.z, r3.w);
}

// The short-k kernel's mode-independent start: the op(A) ring's state with
// its first copies issued, and every op(B) load of the thread issued.
//
// Full row tiles of a rows-contiguous op(A) (k <= 64) stream through a ring
// of kSkRing LDS stages of one chunk each (16 k-values x 128 rows, 16 KB),
// filled by direct buffer loads (no registers held) kSkRing - 1 chunks ahead
// across tile boundaries.  Workgroup b takes a run of consecutive full tiles
// (b * (nfull / G) + min(b, nfull % G) on), so that the tiles in flight at
// once lie spread over all of op(A) and C: the rows of one chunk are lda
// apart, and neighbouring tiles in flight together would put every access of
// the device into a few HBM channels when lda is a large power of two.
// Chunk s of the workgroup is chunk s % nchunks of its (s / nchunks)-th
// tile.
template <int KPAD>
struct SkStart {
    static constexpr int kBPer = kSkCols * KPAD / kThreads;
    bool ring;
    int nchunks, wsc;
    int64_t nfull, G, mine, first_tile, S;
    uint32_t voff, extent;
    // the next chunk to copy: chunk ic of row tile it into stage is (all
    // wave-uniform, advanced by counting: no divisions in the loop)
    int ic, is;
    int64_t it, issued;
    float2 bv[kBPer];  // op(B) element q of this thread (see sk_b_elem)

    // Copies chunk ic of row tile it into stage is and advances to the next
    // chunk.  live = false issues the same four copies through a descriptor
    // of no records (every access out of range: nothing is read) and
    // advances nothing, so that a fixed number of copies is issued either
    // way.
    __device__ __attribute__((always_inline)) void issue(const SmallKArgs &g, char *la, bool live) {
        // rows it*128 .. +127 of k-values 16ic .. 16ic+15: thread (w, lane),
        // copy q moves rows 2 lane, 2 lane + 1 of k-value 16ic + 4q + w
        // (the address is wave-uniform: read it from the first lane, so the
        // descriptor is built in scalar registers)
        const uint64_t a64 = reinterpret_cast<uint64_t>(g.A + it * kSkRows + (int64_t)(16 * ic) * g.lda);
        const uint64_t ua = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(a64 >> 32)) << 32) |
                            (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a64);
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(ua), (short)0, live ? extent : 0u,
                                              kRsrcWord3);
        char *stage = la + is * kSkChunkBytes;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, LDS_PTR(stage + (256 * q + 64 * wsc) * 16), 16, voff,
                                                     (uint32_t)(4 * q * g.lda * 8), 0, 0);
        const int ic1 = ic + 1 == nchunks ? 0 : ic + 1;
        it += live && ic1 == 0 ? 1 : 0;
        ic = live ? ic1 : ic;
        is = live ? (is + 1 == kSkRing ? 0 : is + 1) : is;
        issued += live ? 1 : 0;
    }
};

// Element q of a thread's op(B) loads is (row j, k-value kk) of a 64 x KPAD
// index space (k-values inner when op(B) is k-contiguous, so that lanes read
// consecutive addresses), with compile-time shifts only.
template <int KPAD>
__device__ __attribute__((always_inline)) inline void sk_b_elem(const SmallKArgs &g, int q, int &j, int &kk) {
    static_assert((KPAD & (KPAD - 1)) == 0 && kSkCols == 64, "power-of-two index space");
    const unsigned e = threadIdx.x + (unsigned)(q * kThreads);
    kk = (int)(g.b_kcontig ? (e & (KPAD - 1)) : (e >> 6));
    j = (int)(g.b_kcontig ? (e / KPAD) : (e & 63));
}

template <int KPAD>
__device__ __attribute__((always_inline)) inline void sk_load_b(const SmallKArgs &g, SkStart<KPAD> &r) {
#pragma unroll
    for (int q = 0; q < SkStart<KPAD>::kBPer; ++q) {
        int j, kk;
        sk_b_elem<KPAD>(g, q, j, kk);
        const bool ok = j < g.n && kk < g.k;
        const int64_t idx = !ok ? 0 : g.b_kcontig ? kk + (int64_t)j * g.ldb : j + (int64_t)kk * g.ldb;
        r.bv[q] = g.B[idx];
    }
}

template <int KPAD>
__device__ __attribute__((always_inline)) inline void sk_start(const SmallKArgs &g, char *la, SkStart<KPAD> &r) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kpad = (int)round_up(g.k, kKPad);
    r.nchunks = kpad / kKPad;
    r.ring = KPAD == 64 && g.a_stage;
    r.nfull = g.m / kSkRows;
    r.G = gridDim.x;
    const int64_t per = r.nfull / r.G, rem = r.nfull % r.G;
    r.mine = r.ring ? per + (blockIdx.x < rem ? 1 : 0) : 0;
    r.first_tile = blockIdx.x * per + min((int64_t)blockIdx.x, rem);
    r.S = r.mine * r.nchunks;
    r.wsc = __builtin_amdgcn_readfirstlane(w);
    r.voff = (uint32_t)(16 * lane + r.wsc * g.lda * 8);
    r.extent = (uint32_t)((15 * g.lda + kSkRows) * 8);
    r.ic = 0;
    r.is = 0;
    r.it = r.first_tile;
    r.issued = 0;
    // the first kSkRing - 1 chunks (copies of no records past this
    // workgroup's last chunk, into stages it never reads): a fixed count,
    // which lets the compiler's waits for the loads issued before and after
    // count exactly
    if constexpr (KPAD == 64) {
#pragma unroll
        for (int p = 0; p < kSkRing - 1; ++p) r.issue(g, la, r.issued < r.S);
    }
    // the k <= 64 kernel also issues op(B)'s loads here (the k <= 128 one,
    // whose op(B) takes twice the registers, in its body after the mode is
    // known)
    if constexpr (KPAD == 64) sk_load_b<KPAD>(g, r);
}

template <int MODE, int KPAD>
__device__ __attribute__((always_inline)) inline void smallk_body(const SmallKArgs &g, int mode, int shA, int shB,
                                                                  char *lds, char *la, SkStart<KPAD> &r) {
    constexpr int kE = MODE == QCE_MODE_FP32 ? 4 : 2;
    const int kpad = (int)round_up(g.k, kKPad);
    const int rb = sk_row_bytes(kpad, kE);
    const int pb = kSkCols * rb;
    const int nchunks = kpad / kKPad;

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, l32 = lane & 31, hi = lane >> 5;
    const int64_t ntiles = (g.m + kSkRows - 1) / kSkRows;

    // op(B) -> LDS planes (zeros beyond n and k; k-values from kpad on are
    // not stored)
    constexpr int kBPer = SkStart<KPAD>::kBPer;
    if constexpr (KPAD != 64) sk_load_b<KPAD>(g, r);
#pragma unroll
    for (int q = 0; q < kBPer; ++q) {
        int j, kk;
        sk_b_elem<KPAD>(g, q, j, kk);
        if (kk >= kpad) continue;
        float2 v = make_float2(0.f, 0.f);
        if (j < g.n && kk < g.k) {
            v = r.bv[q];
            if (g.b_conj) v.y = -v.y;  // (padding stays +0)
        }
        char *row = lds + j * rb;
        if constexpr (MODE == QCE_MODE_FP16X2) {
            uint16_t h[4];
            split_fp16x2(v.x, shB, h[0], h[1]);
            split_fp16x2(v.y, shB, h[2], h[3]);
#pragma unroll
            for (int p = 0; p < 4; ++p) *reinterpret_cast<uint16_t *>(row + p * pb + 2 * kk) = h[p];
        } else if constexpr (MODE == QCE_MODE_BF16X3) {
            uint16_t b[6];
            split_bf16x3(v.x, b[0], b[1], b[2]);
            split_bf16x3(v.y, b[3], b[4], b[5]);
#pragma unroll
            for (int p = 0; p < 6; ++p) *reinterpret_cast<uint16_t *>(row + p * pb + 2 * kk) = b[p];
        } else {
            *reinterpret_cast<float *>(row + 4 * kk) = v.x;
            *reinterpret_cast<float *>(row + pb + 4 * kk) = v.y;
        }
    }
    __syncthreads();

    const int nbk = g.n > 32 ? 2 : 1;
    Acc<MODE> acc;
    auto zero_acc = [&]() {
        floatx16 zf;
#pragma unroll
        for (int r = 0; r < 16; ++r) zf[r] = 0.f;
#pragma unroll
        for (int ub = 0; ub < 2; ++ub) {
            acc.re_m[ub][0] = zf;
            acc.im_m[ub][0] = zf;
            if constexpr (MODE != QCE_MODE_FP32) {
                acc.re_c[ub][0] = zf;
                acc.im_c[ub][0] = zf;
            } else {
                acc.re_n[ub][0] = zf;
            }
        }
    };
    // the 8 k-values of op(A) row i this lane supplies in chunk c: 16c + 8hi + u
    // (FP16 / BF16 fragments), or 16c + 8s + 4hi + jj with u = 4s + jj (FP32)
    auto kval = [&](int c, int u) {
        return MODE == QCE_MODE_FP32 ? 16 * c + 8 * (u >> 2) + 4 * hi + (u & 3) : 16 * c + 8 * hi + u;
    };
    // the split and the MFMAs of chunk c (this lane's 8 op(A) values in cur)
    auto mma_chunk = [&](const float2 *cur, int c) {
        if constexpr (MODE == QCE_MODE_FP16X2) {
            uint16_t h[4][8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                split_fp16x2(cur[u].x, shA, h[0][u], h[1][u]);
                split_fp16x2(cur[u].y, shA, h[2][u], h[3][u]);
            }
            u32x4 y[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) y[p] = __builtin_bit_cast(u32x4, pack8(h[p]));
#pragma unroll
            for (int ub = 0; ub < 2; ++ub) {
                if (ub >= nbk) break;
                const char *src = lds + (ub * 32 + l32) * rb + 2 * (16 * c + 8 * hi);
                u32x4 x[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) x[p] = *reinterpret_cast<const u32x4 *>(src + p * pb);
                const u32x4 nx[2] = {neg_halves(x[2]), neg_halves(x[3])};
                fp16x2_block(x, nx, y, acc.re_m[ub][0], acc.im_m[ub][0], acc.re_c[ub][0], acc.im_c[ub][0]);
            }
        } else if constexpr (MODE == QCE_MODE_BF16X3) {
            uint16_t b[6][8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                split_bf16x3(cur[u].x, b[0][u], b[1][u], b[2][u]);
                split_bf16x3(cur[u].y, b[3][u], b[4][u], b[5][u]);
            }
            u32x4 y[6];
#pragma unroll
            for (int p = 0; p < 6; ++p) y[p] = __builtin_bit_cast(u32x4, pack8(b[p]));
#pragma unroll
            for (int ub = 0; ub < 2; ++ub) {
                if (ub >= nbk) break;
                const char *src = lds + (ub * 32 + l32) * rb + 2 * (16 * c + 8 * hi);
                u32x4 x[6];
#pragma unroll
                for (int p = 0; p < 6; ++p) x[p] = *reinterpret_cast<const u32x4 *>(src + p * pb);
                bf16x3_block(x, y, acc.re_m[ub][0], acc.im_m[ub][0], acc.re_c[ub][0], acc.im_c[ub][0]);
            }
        } else {
#pragma unroll
            for (int ub = 0; ub < 2; ++ub) {
                if (ub >= nbk) break;
#pragma unroll
                for (int sh = 0; sh < 2; ++sh) {
                    const char *src = lds + (ub * 32 + l32) * rb + 4 * (16 * c + 8 * sh + 4 * hi);
                    const f32x4 xr = *reinterpret_cast<const f32x4 *>(src);
                    const f32x4 xi = *reinterpret_cast<const f32x4 *>(src + pb);
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const float b_r = cur[4 * sh + jj].x, b_i = cur[4 * sh + jj].y;
                        acc.re_m[ub][0] = mfma32(xr[jj], b_r, acc.re_m[ub][0]);
                        acc.re_n[ub][0] = mfma32(xi[jj], b_i, acc.re_n[ub][0]);
                        acc.im_m[ub][0] = mfma32(xr[jj], b_i, acc.im_m[ub][0]);
                        acc.im_m[ub][0] = mfma32(xi[jj], b_r, acc.im_m[ub][0]);
                    }
                }
            }
        }
    };
    auto epilogue = [&](int64_t i, bool row_ok) {
    const int shift_total = shA + shB;
    const bool alpha_one = g.alpha.x == 1.f && g.alpha.y == 0.f;
    // the common case (C = A B, every column of the block in range, no
    // shift) in a branch of its own: per output the combination and a store
    if (alpha_one && g.beta_zero && shift_total == 0 && row_ok && g.n == nbk * 32) {
        float2 *cp = g.C + i + (int64_t)(4 * hi) * g.ldc;
#pragma unroll
        for (int ub = 0; ub < 2; ++ub) {
            if (ub >= nbk) break;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = ub * 32 + 8 * (r >> 2) + (r & 3);
                float re, im;
                if constexpr (MODE == QCE_MODE_FP16X2) {
                    re = acc.re_m[ub][0][r] + acc.re_c[ub][0][r] * (1.0f / 2048.0f);
                    im = acc.im_m[ub][0][r] + acc.im_c[ub][0][r] * (1.0f / 2048.0f);
                } else if constexpr (MODE == QCE_MODE_BF16X3) {
                    re = acc.re_m[ub][0][r] + acc.re_c[ub][0][r];
                    im = acc.im_m[ub][0][r] + acc.im_c[ub][0][r];
                } else {
                    re = acc.re_m[ub][0][r] - acc.re_n[ub][0][r];
                    im = acc.im_m[ub][0][r];
                }
                // streamed out (C is not read again here), so the lines do not
                // wait in L2 for the end-of-kernel write-back
                const f32x2 val = {re, im};
                __builtin_nontemporal_store(val, reinterpret_cast<f32x2 *>(cp + (int64_t)j * g.ldc));
            }
        }
        return;
    }
#pragma unroll
    for (int ub = 0; ub < 2; ++ub) {
        if (ub >= nbk) break;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t j = ub * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
            if (!row_ok || j >= g.n) continue;
            float re, im;
            if constexpr (MODE == QCE_MODE_FP16X2) {
                re = acc.re_m[ub][0][r] + acc.re_c[ub][0][r] * (1.0f / 2048.0f);
                im = acc.im_m[ub][0][r] + acc.im_c[ub][0][r] * (1.0f / 2048.0f);
            } else if constexpr (MODE == QCE_MODE_BF16X3) {
                re = acc.re_m[ub][0][r] + acc.re_c[ub][0][r];
                im = acc.im_m[ub][0][r] + acc.im_c[ub][0][r];
            } else {
                re = acc.re_m[ub][0][r] - acc.re_n[ub][0][r];
                im = acc.im_m[ub][0][r];
            }
            if (shift_total) {
                re = ldexpf(re, -shift_total);
                im = ldexpf(im, -shift_total);
            }
            float2 out = alpha_one ? make_float2(re, im)
                                   : make_float2(g.alpha.x * re - g.alpha.y * im, g.alpha.x * im + g.alpha.y * re);
            float2 *cp = g.C + i + j * g.ldc;
            if (!g.beta_zero) {
                const float2 cv = *cp;
                out.x += g.beta.x * cv.x - g.beta.y * cv.y;
                out.y += g.beta.x * cv.y + g.beta.y * cv.x;
            }
            *cp = out;
        }
    }
    };

    // the register path below takes the tiles the ring does not (with the
    // ring: the partial tile after the full ones)
    const int64_t first_reg_tile = r.ring ? r.nfull + blockIdx.x : blockIdx.x;
    const int64_t S = r.S;
    if (r.ring) {
        // LDS byte address of this lane's first value in stage 0 (the
        // fragment's first k-value kval(c, 0) - 16 c, then its row)
        const uint32_t ring_base =
            (uint32_t)(uintptr_t)LDS_PTR(la) + (uint32_t)(((kval(0, 0)) * kSkRows + w * 32 + l32) * 8);
        // chunk c of row tile t sits in stage cs
        int c = 0, cs = 0;
        int64_t t = r.first_tile;
        for (int64_t sidx = 0; sidx < S; ++sidx) {
            // chunk sidx has landed once at most the copies issued after it
            // are outstanding (vector memory operations retire in order; the
            // epilogue's stores only make the wait longer)
            static_assert(kSkRing == 4, "the waits below assume up to two chunks in flight after this one");
            const int64_t after = r.issued - 1 - sidx;
            if (after >= 2) wait_vmcnt<8>();
            else if (after == 1) wait_vmcnt<4>();
            else wait_vmcnt<0>();
            __syncthreads();  // every wave's copies of chunk sidx, and every wave done with chunk sidx - 1
            // this lane's values: k-value kval(c, u) - 16 c of the chunk
            // (1 KB apart), row w * 32 + l32
            float2 cur[8];
            const uint32_t ra = ring_base + (uint32_t)(cs * kSkChunkBytes);
            ring_read8<MODE == QCE_MODE_FP32>(ra, cur);
            if (g.a_conj) {
#pragma unroll
                for (int u = 0; u < 8; ++u) cur[u].y = -cur[u].y;
            }
            if (r.issued < S) r.issue(g, la, true);  // into chunk sidx - 1's stage
            if (c == 0) zero_acc();
            mma_chunk(cur, c);
            if (c == nchunks - 1) epilogue(t * kSkRows + w * 32 + l32, true);
            if (++c == nchunks) {
                c = 0;
                ++t;
            }
            if (++cs == kSkRing) cs = 0;
        }
    }
    // the workgroup walks (its remaining) row tiles with op(B) kept in LDS,
    // loading op(A) through registers one chunk ahead
    for (int64_t tile = first_reg_tile; tile < ntiles; tile += gridDim.x) {
        const int64_t i = tile * kSkRows + w * 32 + l32;
        const bool row_ok = i < g.m;
        // the 8 loads are issued (from clamped, valid addresses) before any
        // value is used
        auto load = [&](float2 *v, int c) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kk = kval(c, u);
                const bool ok = row_ok && kk < g.k;
                v[u] = g.A[!ok ? 0 : g.a_kcontig ? kk + i * g.lda : i + (int64_t)kk * g.lda];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (!(row_ok && kval(c, u) < g.k)) v[u] = make_float2(0.f, 0.f);
                else if (g.a_conj) v[u].y = -v[u].y;
            }
        };
        zero_acc();
        float2 cur[8], nxt[8];
        load(cur, 0);
        for (int c = 0; c < nchunks; ++c) {
            if (c + 1 < nchunks) load(nxt, c + 1);
            mma_chunk(cur, c);
#pragma unroll
            for (int u = 0; u < 8; ++u) cur[u] = nxt[u];
        }
        epilogue(i, row_ok);
    }
}

template <int KPAD>
__global__ __launch_bounds__(kThreads) void smallk_kernel(SmallKArgs g) {
    // op(B)'s planes and the op(A) ring (k <= 64 kernel only) in LDS
    // arrays of their own
    __shared__ __attribute__((aligned(16))) char lds[sk_lds_bytes(KPAD)];
    __shared__ __attribute__((aligned(16))) char ring[KPAD == 64 ? kSkStageBytes : 16];
    const int64_t z = blockIdx.z;
    g.A += z * g.bsA;
    g.B += z * g.bsB;
    g.C += z * g.bsC;
    if (g.st) g.st += z;
    // mode-independent loads first -- the selection's records (where they
    // fit in registers), then the op(A) ring's first copies and op(B) --
    // so that the selection's reductions run while the operands arrive
    SelectHead sr;
    const bool early = g.select_here && select_one_pass_fits(g.sel);
    if (early) select_load_head(g.sel, (int)z, sr);
    SkStart<KPAD> r;
    sk_start<KPAD>(g, ring, r);
    int mode, shA = 0, shB = 0;
    if (g.select_here) {
        const SelectDecision d = select_block(g.sel, (int)z, blockIdx.x == 0, early ? &sr : nullptr);
        mode = d.mode;
        shA = d.shift[0];
        shB = d.shift[1];
    } else {
        mode = g.forced_mode >= 0 ? g.forced_mode : g.st->mode;
        if (mode == QCE_MODE_FP16X2_SCALED && g.st) {
            shA = g.st->shift[0];
            shB = g.st->shift[1];
        }
    }
    if (mode == QCE_MODE_FP16X2 || mode == QCE_MODE_FP16X2_SCALED)
        smallk_body<QCE_MODE_FP16X2, KPAD>(g, mode, shA, shB, lds, ring, r);
    else if (mode == QCE_MODE_BF16X3)
        smallk_body<QCE_MODE_BF16X3, KPAD>(g, mode, 0, 0, lds, ring, r);
    else
        smallk_body<QCE_MODE_FP32, KPAD>(g, mode, 0, 0, lds, ring, r);
}

}  // namespace

namespace {
struct TileRule {
    int64_t min_tiles128, min_chunks;
    int tile;
};
#include "tile_table.inc"
}  // namespace

int gemm_tile(int64_t m, int64_t n, int64_t k, int batch) {
    const int64_t tiles = ((m + 127) / 128) * ((n + 127) / 128) * std::max(1, batch);
    const int64_t chunks = round_up(k, kKPad) / kKPad;
    int tile = 128;
    for (const TileRule &r : kTileRules)
        if (tiles >= r.min_tiles128 && chunks >= r.min_chunks) tile = r.tile;
    return tile;
}

int gemm_splits(int64_t m, int64_t n, int64_t k, int batch, int tile) {
    const int64_t tiles = ((m + tile - 1) / tile) * ((n + tile - 1) / tile) * std::max(1, batch);
    const int64_t pads = round_up(k, kKPad) / kKPad;  // chunks of 16 k-values
    // keep >= 16 chunks (256 k-values) per split for 128 x 128 tiles, >= 8
    // for the 64 x 64 tile (a quarter of the MFMAs per chunk)
    const int64_t min_chunks = tile == 64 ? 8 : 16;
    if (tiles >= 256 || pads < 2 * min_chunks) return 1;
    int64_t s = 512 / tiles;                      // aim at ~512 workgroups
    s = std::min<int64_t>(s, pads / min_chunks);
    return (int)std::max<int64_t>(1, s);
}

hipError_t launch_gemm(const GemmArgs &g0, int which, hipStream_t s) {
    GemmArgs g = g0;
    const int tile = g.tile == 64 || g.tile == 128 ? g.tile : gemm_tile(g.m, g.n, g.k, std::max(1, g.batch));
    const int nbm = (int)((g.m + tile - 1) / tile), nbn = (int)((g.n + tile - 1) / tile);
    const int batch = std::max(1, g.batch);
    const int splits = gemm_splits(g.m, g.n, g.k, batch, tile);
    const int64_t pads = round_up(g.k, kKPad) / kKPad;
    g.kpad_per_split = ((pads + splits - 1) / splits) * kKPad;
    const int nsplit = (int)((round_up(g.k, kKPad) + g.kpad_per_split - 1) / g.kpad_per_split);
    g.bsPartial = (int64_t)nsplit * g.m * g.n;
    const dim3 grid((unsigned)(nbm * nbn), (unsigned)nsplit, (unsigned)batch), block(kThreads);
    if (nsplit > 1 && !g.partial) return hipErrorInvalidValue;
    if (tile == 64) {
        if (which < 0)
            hipLaunchKernelGGL(gemm_auto_kernel<64>, grid, block, 0, s, g, nbm, nbn);
        else if (which == QCE_MODE_FP16X2)
            hipLaunchKernelGGL((gemm_kernel<QCE_MODE_FP16X2, 64>), grid, block, 0, s, g, nbm, nbn);
        else if (which == QCE_MODE_BF16X3)
            hipLaunchKernelGGL((gemm_kernel<QCE_MODE_BF16X3, 64>), grid, block, 0, s, g, nbm, nbn);
        else
            hipLaunchKernelGGL((gemm_kernel<QCE_MODE_FP32, 64>), grid, block, 0, s, g, nbm, nbn);
    } else {
        if (which < 0)
            hipLaunchKernelGGL(gemm_auto_kernel<128>, grid, block, 0, s, g, nbm, nbn);
        else if (which == QCE_MODE_FP16X2)
            hipLaunchKernelGGL((gemm_kernel<QCE_MODE_FP16X2, 128>), grid, block, 0, s, g, nbm, nbn);
        else if (which == QCE_MODE_BF16X3)
            hipLaunchKernelGGL((gemm_kernel<QCE_MODE_BF16X3, 128>), grid, block, 0, s, g, nbm, nbn);
        else
            hipLaunchKernelGGL((gemm_kernel<QCE_MODE_FP32, 128>), grid, block, 0, s, g, nbm, nbn);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit == 1) return e;
    const int64_t mn = g.m * g.n;
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((mn + kThreads - 1) / kThreads), 1, (unsigned)batch),
                       block, 0, s, g, nsplit);
    return hipGetLastError();
}

int gemm_group_tile(const GroupGemmEntry *e, int count, int forced_tile) {
    if (forced_tile == 64 || forced_tile == 128) return forced_tile;
    int64_t tiles = 0, k = 0;
    for (int i = 0; i < count; ++i) {
        tiles += ((e[i].g.m + 127) / 128) * ((e[i].g.n + 127) / 128) * std::max(1, e[i].g.batch);
        k = std::max(k, e[i].g.k);
    }
    // the table's rule on the whole launch's output (and its longest k)
    int tile = 128;
    const int64_t chunks = round_up(k, kKPad) / kKPad;
    for (const TileRule &r : kTileRules)
        if (tiles >= r.min_tiles128 && chunks >= r.min_chunks) tile = r.tile;
    return tile;
}

void gemm_group_shape(GroupGemmEntry *e, int count, int tile) {
    int64_t tiles = 0;
    for (int i = 0; i < count; ++i)
        tiles += ((e[i].g.m + tile - 1) / tile) * ((e[i].g.n + tile - 1) / tile) * std::max(1, e[i].g.batch);
    for (int i = 0; i < count; ++i) {
        GemmArgs &g = e[i].g;
        g.tile = tile;
        e[i].nbm = (int)((g.m + tile - 1) / tile);
        e[i].nbn = (int)((g.n + tile - 1) / tile);
        // k splits as for one GEMM, counting the whole launch's tiles
        const int64_t pads = round_up(g.k, kKPad) / kKPad;
        const int64_t min_chunks = tile == 64 ? 8 : 16;
        int64_t s = 1;
        if (tiles < 256 && pads >= 2 * min_chunks) s = std::max<int64_t>(1, std::min<int64_t>(512 / tiles, pads / min_chunks));
        g.kpad_per_split = ((pads + s - 1) / s) * kKPad;
        e[i].nsplit = (int)((round_up(g.k, kKPad) + g.kpad_per_split - 1) / g.kpad_per_split);
        g.bsPartial = e[i].nsplit > 1 ? (int64_t)e[i].nsplit * g.m * g.n : 0;
        e[i].tiles = (int64_t)e[i].nbm * e[i].nbn * e[i].nsplit * std::max(1, g.batch);
        e[i].red_blocks = e[i].nsplit > 1 ? ((g.m * g.n + kThreads - 1) / kThreads) * std::max(1, g.batch) : 0;
    }
}

void gemm_group_schedule(GroupGemmEntry *e, int count, int64_t &total_tiles, int64_t &total_red) {
    // heaviest tiles (most k chunks per tile) first; stable for equal cost
    std::stable_sort(e, e + count, [](const GroupGemmEntry &a, const GroupGemmEntry &b) {
        return a.g.kpad_per_split > b.g.kpad_per_split;
    });
    total_tiles = 0;
    total_red = 0;
    for (int i = 0; i < count; ++i) {
        e[i].tile_start = total_tiles;
        total_tiles = round_up(total_tiles + e[i].tiles, kXcds);
        e[i].red_start = total_red;
        total_red += e[i].red_blocks;
    }
}

hipError_t launch_gemm_grouped(const GroupGemmEntry *dev_entries, int count, int64_t total_tiles,
                               int64_t total_red, int tile, unsigned int *queue, hipStream_t s) {
    if (count <= 0 || total_tiles <= 0) return hipSuccess;
    if (tile != 64 && tile != 128) return hipErrorInvalidValue;
    // one workgroup per resident slot (at most one per tile), a multiple of
    // the XCD count so that every XCD's ids are served
    static int slots[2] = {0, 0};
    int &sl = slots[tile == 64 ? 0 : 1];
    if (sl == 0) {
        int dev = 0, cus = 0, per = 0;
        hipError_t err = hipGetDevice(&dev);
        if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (err == hipSuccess)
            err = tile == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_grouped_kernel<64>, kThreads, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_grouped_kernel<128>, kThreads, 0);
        if (err != hipSuccess) return err;
        sl = std::max(kXcds, (cus * std::max(per, 1)) / kXcds * kXcds);
    }
    const int64_t grid = std::min<int64_t>(sl, round_up(total_tiles, kXcds));
    if (tile == 64)
        hipLaunchKernelGGL(gemm_grouped_kernel<64>, dim3((unsigned)grid), dim3(kThreads), 0, s, dev_entries, count,
                           total_tiles, queue);
    else
        hipLaunchKernelGGL(gemm_grouped_kernel<128>, dim3((unsigned)grid), dim3(kThreads), 0, s, dev_entries, count,
                           total_tiles, queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || total_red == 0) return e;
    hipLaunchKernelGGL(gemm_grouped_reduce_kernel, dim3((unsigned)total_red), dim3(kThreads), 0, s, dev_entries,
                       count);
    return hipGetLastError();
}

size_t gemm_partial_bytes(int64_t m, int64_t n, int64_t k, int batch) {
    // enough for either tile (the launch may be told which)
    size_t most = 0;
    for (int tile : {64, 128}) {
        const int splits = gemm_splits(m, n, k, batch, tile);
        if (splits <= 1) continue;
        const int64_t pads = round_up(k, kKPad) / kKPad;
        const int64_t per = ((pads + splits - 1) / splits) * kKPad;
        const int64_t nsplit = (round_up(k, kKPad) + per - 1) / per;
        if (nsplit > 1) most = std::max(most, (size_t)nsplit * (size_t)(m * n) * sizeof(float2));
    }
    return most;
}

bool smallk_shape(int64_t m, int64_t n, int64_t k) {
    return !irregular_shape(m, n, k) && n <= kSkCols && k <= 128;
}

hipError_t launch_smallk(const SmallKArgs &g, hipStream_t s) {
    if (!smallk_shape(g.m, g.n, g.k)) return hipErrorInvalidValue;
    if (g.forced_mode < 0 && !g.st && !g.select_here) return hipErrorInvalidValue;
    if (g.select_here && (!g.sel.st || !g.sel.rec || g.sel.blocks_a + g.sel.blocks_b <= 0))
        return hipErrorInvalidValue;
    const int batch = std::max(1, g.batch);
    // at most as many workgroups as fit on the device at once: op(B) is
    // split into LDS once per workgroup and reused for every row tile it
    // walks
    const bool short64 = round_up(g.k, kKPad) <= 64;
    static int slots[2] = {0, 0};
    int &sl = slots[short64 ? 0 : 1];
    if (sl == 0) {
        int dev = 0, cus = 0, per = 0;
        hipError_t err = hipGetDevice(&dev);
        if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (err == hipSuccess)
            err = short64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, smallk_kernel<64>, kThreads, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, smallk_kernel<128>, kThreads, 0);
        if (err != hipSuccess) return err;
        sl = std::max(1, cus * std::max(per, 1));
    }
    const int64_t tiles = (g.m + kSkRows - 1) / kSkRows;
    const dim3 grid((unsigned)std::min<int64_t>(tiles, sl), 1, (unsigned)batch), block(kThreads);
    // LDS staging of op(A) (k <= 64 kernel): rows contiguous, 16-byte
    // aligned copies in every batch entry, k a multiple of 16, and every
    // copy's byte offset inside 32 bits
    SmallKArgs q = g;
    const int64_t extent = ((g.k - 1) * g.lda + kSkRows) * 8;
    q.a_stage = short64 && !g.a_kcontig && g.k % kKPad == 0 && g.lda % 2 == 0 &&
                (reinterpret_cast<uintptr_t>(g.A) & 15) == 0 && (batch == 1 || g.bsA % 2 == 0) &&
                extent + 4 * g.lda * 8 < (int64_t(1) << 32);
    if (short64)
        hipLaunchKernelGGL(smallk_kernel<64>, grid, block, 0, s, q);
    else
        hipLaunchKernelGGL(smallk_kernel<128>, grid, block, 0, s, q);
    return hipGetLastError();
}

hipError_t launch_scale_c(float2 *C, int64_t m, int64_t n, int64_t ldc, float2 beta, int beta_zero,
                          hipStream_t s, int batch, int64_t bsC) {
    const int64_t total = m * n;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_c_kernel, dim3((unsigned)((total + 255) / 256), 1, (unsigned)std::max(1, batch)),
                       dim3(256), 0, s, C, m, n, ldc, beta, beta_zero, bsC);
    return hipGetLastError();
}

}  // namespace qce
