// Mode selection from the exponent-statistics records (Sec. 4.1 and 4.2):
// one block of 256 threads adds up a GEMM's per-block records and applies
// the tolerance rule.  Used by the selection launch that follows the
// statistics, and by consumer kernels that take the decision in their own
// prologue (every block of such a kernel reaches the same decision from
// the same integer counts; one block publishes it).
#pragma once

#include "common.hpp"

namespace qce {
namespace {
namespace selimpl {
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
__device__ inline unsigned long long wave_sum64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

}  // namespace selimpl

// Lane operations through DPP (GFX9 controls): no LDS round trip.
constexpr int kDppQuadSwap1 = 0xB1;  // quad_perm [1, 0, 3, 2]: lane ^ 1
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

// inclusive prefix sum over the lanes: within each row of 16 lanes by
// doubling shifts (lanes without a source add 0), then row 1 and 3 add the
// last lane of the row before, rows 2 and 3 the last lane of row 1; with
// rows = 2 only the first 32 lanes are scanned
template <int kRows = 4>
__device__ inline unsigned int lane_scan_add(unsigned int v) {
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr1, 0xf, 0xf, false);
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr2, 0xf, 0xf, false);
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr4, 0xf, 0xf, false);
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr8, 0xf, 0xf, false);
    if constexpr (kRows == 2) {
        v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast15, 0x2, 0xf, false);
    } else {
        v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast15, 0xa, 0xf, false);
        v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast31, 0xc, 0xf, false);
    }
    return v;
}
// sum and maximum over the 64 lanes, in every lane
__device__ inline unsigned int lane_total(unsigned int v) {
    return (unsigned int)__builtin_amdgcn_readlane((int)lane_scan_add(v), 63);
}
__device__ inline int lane_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, kDppRowShr1, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, kDppRowShr2, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, kDppRowShr4, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, kDppRowShr8, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, kDppRowBcast15, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, kDppRowBcast31, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// Workgroup barrier that waits for this wave's LDS operations only: global
// loads issued before the selection (a consumer kernel's own operand
// copies) stay in flight; the selection's record loads are waited for
// where their registers are used.
__device__ __attribute__((always_inline)) inline void sel_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt at their maxima (no wait)
    asm volatile("s_barrier" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// the decision as every thread of the block returns it
struct SelectDecision {
    int mode;
    int shift[2];
};

// Per-operand tolerance level (Sec. 4.1): FP16 if every element but a
// fraction t lies in the FP16 window without shifting (and e_max <= 14: no
// overflow); FP16 with scaling if the window shifted to e_max holds all but
// a fraction t; BF16X3 if all but a fraction t3 lie above its floor and
// e_max <= 126; else FP32.  Non-finite data -> FP32.
__device__ inline int operand_level(const OperandStats &s, int emax, double t, double t3) {
    if (s.nonfinite) return QCE_MODE_FP32;
    if (s.nnz == 0) return QCE_MODE_FP16X2;
    const double nnz = (double)s.nnz;
    if (emax <= kFp16Emax && (double)(s.nnz - s.n1) <= t * nnz) return QCE_MODE_FP16X2;
    if ((double)(s.nnz - s.n2) <= t * nnz) return QCE_MODE_FP16X2_SCALED;
    if (emax <= kBf16x3Emax && (double)(s.nnz - s.n3) <= t3 * nnz) return QCE_MODE_BF16X3;
    return QCE_MODE_FP32;
}

// The decision of batch entry z from its blocks' records (one block of 256
// threads, launched after the statistics launch: the kernel boundary makes
// every record visible, with no device-wide fence in the statistics blocks).
// Thread t takes records t, t + 256, ... of both operands; each pass issues
// the loads of kSelUnroll records before using any (the records come from
// other XCDs' writes, so every round trip is long).
constexpr int kSelUnroll = 4;
// records per thread of the one-pass path (up to 768 records)
constexpr int kSelFast = 3;

// At most kSelFast records per thread, held in registers: counts and
// largest bin, and (where the caller loaded them in the same round) the 32
// cumulative entries, so that stage 2 picks the entry it needs from
// registers.  Lane sums in 32 bits through DPP: a record
// counts at most 256 x 8000 components (< 2^21), so a lane's three stay
// below 2^23 and a wave's sum below 2^29.  Fills red, redmax and emaxbin as
// the general path does.
// a thread's records of the one-pass path (counts and largest bin), loaded
// ahead of their use
struct SelectHead {
    uint4 hdr[kSelFast];
    int mbv[kSelFast];
};
__device__ inline bool select_one_pass_fits(const StatsArgs &g) {
    return g.blocks_a + g.blocks_b <= kSelFast * selimpl::kThreads;
}
// issues the loads of batch entry z's record heads (every thread of the block)
__device__ inline void select_load_head(const StatsArgs &g, int z, SelectHead &r) {
    const int total = g.blocks_a + g.blocks_b;
    const StatsRecord *rec = g.rec + (int64_t)z * total;
#pragma unroll
    for (int u = 0; u < kSelFast; ++u) {
        const int i = min((int)threadIdx.x + u * selimpl::kThreads, total - 1);
        r.hdr[u] = *reinterpret_cast<const uint4 *>(&rec[i].nnz);
        r.mbv[u] = rec[i].maxbin;
    }
}

// kHaveCum: the records' cumulative entries are in cum (registers); else
// stage 2 loads the one entry it needs per record (a consumer kernel that
// preloaded only the heads, keeping its registers for its own operands)
template <bool kHaveCum>
__device__ inline void select_one_pass(const StatsArgs &g, const StatsRecord *rec, int total, SelectHead &r,
                                       const uint4 (&cum)[kSelFast][kRelBins / 4],
                                       unsigned long long (&red)[selimpl::kWaves][2][5],
                                       int (&redmax)[selimpl::kWaves][2], int (&emaxbin)[2]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint4 (&hdr)[kSelFast] = r.hdr;
    int (&mbv)[kSelFast] = r.mbv;
    unsigned int sum[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    int mb[2] = {-1, -1};
#pragma unroll
    for (int u = 0; u < kSelFast; ++u) {
        const int i = (int)threadIdx.x + u * selimpl::kThreads;
        if (i >= total) {
            hdr[u] = make_uint4(0, 0, 0, 0);
            mbv[u] = -1;
        }
        const int o = i < g.blocks_a ? 0 : 1;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (o != q) continue;
            sum[q][0] += hdr[u].x;
            sum[q][1] += hdr[u].y;
            sum[q][2] += hdr[u].z;
            sum[q][3] += hdr[u].w;
            mb[q] = max(mb[q], mbv[u]);
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) sum[q][j] = lane_total(sum[q][j]);
        mb[q] = lane_max(mb[q]);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int j = 0; j < 4; ++j) red[w][q][j] = sum[q][j];
            redmax[w][q] = mb[q];
        }
    }
    sel_barrier();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        int gm = -1;
        for (int v = 0; v < selimpl::kWaves; ++v) gm = max(gm, redmax[v][q]);
        emaxbin[q] = gm;
    }
    // stage 2: the cumulative entry of each record's top bin inside
    // [gmax - 28, gmax], picked from registers by compare and select
    unsigned int n2[2] = {0, 0};
#pragma unroll
    for (int u = 0; u < kSelFast; ++u) {
        const int i = (int)threadIdx.x + u * selimpl::kThreads;
        const int o = i < g.blocks_a ? 0 : 1;
        const int top = kWindowSpan - (emaxbin[o] - mbv[u]);  // highest d inside the window (<= 28)
        unsigned int v = 0;
        if constexpr (kHaveCum) {
#pragma unroll
            for (int q = 0; q < kRelBins / 4; ++q) {
                v = top == 4 * q ? cum[u][q].x : v;
                v = top == 4 * q + 1 ? cum[u][q].y : v;
                v = top == 4 * q + 2 ? cum[u][q].z : v;
                v = top == 4 * q + 3 ? cum[u][q].w : v;
            }
        } else {
            v = rec[min(i, total - 1)].cum[min(max(top, 0), kRelBins - 1)];
            v = top >= 0 ? v : 0u;
        }
        v = i < total && mbv[u] >= 0 ? v : 0u;  // (top < 0 matches no entry)
        n2[0] += o == 0 ? v : 0u;
        n2[1] += o == 1 ? v : 0u;
    }
    n2[0] = lane_total(n2[0]);
    n2[1] = lane_total(n2[1]);
    if (lane == 0) {
        red[w][0][4] = n2[0];
        red[w][1][4] = n2[1];
    }
}

// More records than one round of loads holds: two passes over them, each
// thread issuing the loads of kSelUnroll records before using any.
__device__ inline void select_two_pass(const StatsArgs &g, const StatsRecord *rec, int total,
                                       unsigned long long (&red)[selimpl::kWaves][2][5],
                                       int (&redmax)[selimpl::kWaves][2], int (&emaxbin)[2]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // pass 1: counts and largest bin of each operand (integer sums: the
    // order does not matter); the first pass's largest bins stay in
    // registers for pass 2
    unsigned long long acc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    int mb[2] = {-1, -1};
    int keep[kSelUnroll];
    for (int base = threadIdx.x; base < total; base += kSelUnroll * selimpl::kThreads) {
        uint4 c[kSelUnroll];
        int m[kSelUnroll];
        // loads from clamped indices (no branch between them), masked after
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            const int i = min(base + u * selimpl::kThreads, total - 1);
            c[u] = *reinterpret_cast<const uint4 *>(&rec[i].nnz);
            m[u] = rec[i].maxbin;
        }
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            if (base + u * selimpl::kThreads >= total) {
                c[u] = make_uint4(0, 0, 0, 0);
                m[u] = -1;
            }
        }
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            const int o = base + u * selimpl::kThreads < g.blocks_a ? 0 : 1;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                if (o != q) continue;
                acc[q][0] += c[u].x;
                acc[q][1] += c[u].y;
                acc[q][2] += c[u].z;
                acc[q][3] += c[u].w;
                mb[q] = max(mb[q], m[u]);
            }
            if (base == (int)threadIdx.x) keep[u] = m[u];
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[q][j] = selimpl::wave_sum64(acc[q][j]);
        mb[q] = selimpl::wave_max(mb[q]);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int j = 0; j < 4; ++j) red[w][q][j] = acc[q][j];
            redmax[w][q] = mb[q];
        }
    }
    sel_barrier();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        int gm = -1;
        for (int v = 0; v < selimpl::kWaves; ++v) gm = max(gm, redmax[v][q]);
        emaxbin[q] = gm;
    }
    // pass 2 (stage 2): the part of each block's top bins inside
    // [gmax - 28, gmax] of its operand, one cumulative entry per record
    unsigned long long n2[2] = {0, 0};
    for (int base = threadIdx.x; base < total; base += kSelUnroll * selimpl::kThreads) {
        int m[kSelUnroll];
        if (base == (int)threadIdx.x) {
#pragma unroll
            for (int u = 0; u < kSelUnroll; ++u) m[u] = keep[u];
        } else {
#pragma unroll
            for (int u = 0; u < kSelUnroll; ++u) m[u] = rec[min(base + u * selimpl::kThreads, total - 1)].maxbin;
        }
        unsigned int cv[kSelUnroll];
        bool use[kSelUnroll];
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            const int i = base + u * selimpl::kThreads;
            const int gmax = i < g.blocks_a ? emaxbin[0] : emaxbin[1];
            const int top = kWindowSpan - (gmax - m[u]);  // highest d inside the window (<= 28)
            use[u] = i < total && m[u] >= 0 && top >= 0;
            cv[u] = rec[min(i, total - 1)].cum[min(max(top, 0), kRelBins - 1)];
        }
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) cv[u] = use[u] ? cv[u] : 0u;
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            if (base + u * selimpl::kThreads < g.blocks_a) n2[0] += cv[u];
            else n2[1] += cv[u];
        }
    }
    n2[0] = selimpl::wave_sum64(n2[0]);
    n2[1] = selimpl::wave_sum64(n2[1]);
    if (lane == 0) {
        red[w][0][4] = n2[0];
        red[w][1][4] = n2[1];
    }
}

// The decision of batch entry z (every thread of the block).  pre: the
// thread's record heads already loaded by select_load_head (only where
// select_one_pass_fits), else nullptr.
__device__ inline SelectDecision select_block(const StatsArgs &g, int z, bool publish,
                                              SelectHead *pre = nullptr) {
    const int total = g.blocks_a + g.blocks_b;
    const StatsRecord *rec = g.rec + (int64_t)z * total;
    __shared__ unsigned long long red[selimpl::kWaves][2][5];
    __shared__ int redmax[selimpl::kWaves][2];
    int emaxbin[2];
    if (pre) {
        const uint4 none[kSelFast][kRelBins / 4] = {};
        select_one_pass<false>(g, rec, total, *pre, none, red, redmax, emaxbin);
    } else if (select_one_pass_fits(g)) {
        // one round of loads: heads and cumulative entries
        SelectHead hd;
        uint4 cum[kSelFast][kRelBins / 4];
#pragma unroll
        for (int u = 0; u < kSelFast; ++u) {
            const int i = min((int)threadIdx.x + u * selimpl::kThreads, total - 1);
            hd.hdr[u] = *reinterpret_cast<const uint4 *>(&rec[i].nnz);
            hd.mbv[u] = rec[i].maxbin;
            const uint4 *cp = reinterpret_cast<const uint4 *>(rec[i].cum);
#pragma unroll
            for (int q = 0; q < kRelBins / 4; ++q) cum[u][q] = cp[q];
        }
        select_one_pass<true>(g, rec, total, hd, cum, red, redmax, emaxbin);
    } else {
        select_two_pass(g, rec, total, red, redmax, emaxbin);
    }
    sel_barrier();
    // thread 0 applies the rule; publish: it also writes the device state
    // (mode flag, shifts, the record for the host)
    __shared__ SelectDecision out;
    if (threadIdx.x == 0) {
        OperandStats s[2];
        for (int q = 0; q < 2; ++q) {
            unsigned long long v[5] = {0, 0, 0, 0, 0};
            for (int x = 0; x < selimpl::kWaves; ++x)
                for (int j = 0; j < 5; ++j) v[j] += red[x][q][j];
            s[q].nnz = v[0];
            s[q].n1 = v[1];
            s[q].n3 = v[2];
            s[q].nonfinite = v[3];
            s[q].n2 = v[4];
            s[q].maxbits = 0;
            s[q].pad = 0;
        }
        int level[2], emax[2];
        for (int o = 0; o < 2; ++o) {
            emax[o] = s[o].nnz ? emaxbin[o] - 149 : INT32_MIN;
            level[o] = operand_level(s[o], emax[o], g.t, g.t3);
        }
        const int mode = g.forced >= 0 ? g.forced : max(level[0], level[1]);
        int shv[2] = {0, 0};
        if (mode == QCE_MODE_FP16X2_SCALED)
            for (int o = 0; o < 2; ++o) shv[o] = s[o].nnz ? kFp16Emax - emax[o] : 0;
        out.mode = mode;
        out.shift[0] = shv[0];
        out.shift[1] = shv[1];
        if (publish) {
            DevState *st = g.st + z;
            st->mode = mode;
            st->shift[0] = shv[0];
            st->shift[1] = shv[1];
            if (g.mode_log && z == 0) g.mode_log[g.slot] = mode;
            qce_decision &r = st->last;
            r.mode = mode;
            r.sA = shv[0];
            r.sB = shv[1];
            r.stats_taken = 1;
            for (int o = 0; o < 2; ++o) {
                st->acc[o] = s[o];
                r.nnz[o] = (int64_t)s[o].nnz;
                r.n1[o] = (int64_t)s[o].n1;
                r.n2[o] = (int64_t)s[o].n2;
                r.n3[o] = (int64_t)s[o].n3;
                r.nonfinite[o] = (int64_t)s[o].nonfinite;
                r.emax[o] = emax[o];
            }
        }
    }
    sel_barrier();
    return out;
}

}  // namespace
}  // namespace qce
