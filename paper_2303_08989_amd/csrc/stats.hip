// Exponent statistics and mode selection (Sec. 4.1 and 4.2).
//
// stats1 reads every FP32 component of both operands once (Sec. 4: all
// elements are checked, no sampling) and writes, per block: the nonzero count,
// the stage-1 count n1 = #{|v| >= 2^-14}, the BF16X3-floor count
// n3 = #{|v| >= 2^-110}, the non-finite count and the largest |v| bit
// pattern, from which emax = floor(log2 max|v|) follows.  Positive FP32 bit
// patterns order like their values, so every count is one integer compare of
// the absolute bit pattern.
// stats2 (stage 2): each block first adds up the stage-1 partials of its
// operand; it scans the operand again only when stage 1 failed for it, and
// counts n2 = #{|v| >= 2^(emax-28)}: the elements inside the FP16 window once
// emax is shifted to 14.
// select adds up the partials, turns both operands' statistics into the
// device mode flag and the shifts and keeps a record for the host.  Partials
// are summed in block order (no atomics), so the statistics are exact and
// deterministic, and nothing is copied to the host (Sec. 4.2).
#include "common.hpp"

namespace qce {

namespace {

constexpr int kThreads = 256;

__device__ inline int emax_of_bits(unsigned int maxbits) {
    unsigned int e = maxbits >> 23;
    if (e) return (int)e - 127;
    unsigned int mant = maxbits & 0x7fffffu;  // subnormal: mant * 2^-149
    return -118 - __clz(mant);
}

// threshold bit pattern of 2^e (for e below the subnormal range: smallest
// positive value, i.e. every nonzero counts)
__device__ inline unsigned int pow2_bits(int e) {
    if (e >= -126) return (unsigned int)(e + 127) << 23;
    if (e >= -149) return 1u << (e + 149);
    return 1u;
}

__device__ inline bool stage1_pass(const OperandStats &s, double t) {
    if (s.nnz == 0) return true;
    int emax = emax_of_bits(s.maxbits);
    return emax <= kFp16Emax && (double)(s.nnz - s.n1) <= t * (double)s.nnz;
}

// Visit every FP32 component of a stored column-major complex matrix; the
// work is split over `nblk` blocks starting at block index `blk`.
template <class F>
__device__ inline void scan_matrix(const MatDesc &d, int64_t blk, int64_t nblk, F &f) {
    if (d.rows <= 0 || d.cols <= 0) return;
    const int64_t tid = blk * kThreads + threadIdx.x;
    const int64_t nthr = nblk * kThreads;
    if (d.ld == d.rows || d.cols == 1) {
        const float *p = reinterpret_cast<const float *>(d.ptr);
        const int64_t nf = 2 * d.rows * d.cols;
        if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
            const int64_t n4 = nf >> 2;
            const float4 *p4 = reinterpret_cast<const float4 *>(p);
            int64_t i = tid;
            for (; i + 3 * nthr < n4; i += 4 * nthr) {
                float4 v0 = p4[i], v1 = p4[i + nthr], v2 = p4[i + 2 * nthr], v3 = p4[i + 3 * nthr];
                f(v0.x); f(v0.y); f(v0.z); f(v0.w);
                f(v1.x); f(v1.y); f(v1.z); f(v1.w);
                f(v2.x); f(v2.y); f(v2.z); f(v2.w);
                f(v3.x); f(v3.y); f(v3.z); f(v3.w);
            }
            for (; i < n4; i += nthr) {
                float4 v = p4[i];
                f(v.x); f(v.y); f(v.z); f(v.w);
            }
            for (int64_t j = (n4 << 2) + tid; j < nf; j += nthr) f(p[j]);
        } else {
            const int64_t n2 = nf >> 1;
            const float2 *p2 = reinterpret_cast<const float2 *>(p);
            for (int64_t i = tid; i < n2; i += nthr) {
                float2 v = p2[i];
                f(v.x); f(v.y);
            }
        }
    } else {
        // strided: columns over blocks, rows over threads
        for (int64_t c = blk; c < d.cols; c += nblk) {
            const float2 *col = d.ptr + c * d.ld;
            for (int64_t r = threadIdx.x; r < d.rows; r += kThreads) {
                float2 v = col[r];
                f(v.x); f(v.y);
            }
        }
    }
}

__device__ inline unsigned int abs_bits(float v) { return __float_as_uint(v) & 0x7fffffffu; }

struct Stage1Counter {
    unsigned int gt0 = 0, ge1 = 0, ge3 = 0, inf = 0, maxb = 0;
    __device__ inline void operator()(float v) {
        unsigned int ab = abs_bits(v);
        gt0 += ab != 0u;
        ge1 += ab >= kFp16MinNormalBits;
        ge3 += ab >= kBf16x3FloorBits;
        bool nf = ab >= kInfBits;
        inf += nf;
        maxb = max(maxb, nf ? 0u : ab);
    }
};

struct Stage2Counter {
    unsigned int thr;
    unsigned int ge = 0;
    __device__ inline void operator()(float v) {
        unsigned int ab = abs_bits(v);
        ge += (ab >= thr) & (ab < kInfBits);
    }
};

__device__ inline unsigned long long block_sum(unsigned long long v, unsigned long long *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    unsigned long long r = 0;
    for (int i = 0; i < kThreads / 64; ++i) r += sh[i];
    return r;  // valid in every thread
}

__device__ inline unsigned int block_max(unsigned int v, unsigned long long *sh) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned int)__shfl_xor((int)v, o));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    unsigned int r = 0;
    for (int i = 0; i < kThreads / 64; ++i) r = max(r, (unsigned int)sh[i]);
    return r;  // valid in every thread
}

// Stage-1 totals of one operand from its per-block partials, added in block
// order; every thread of the calling block gets the result.
__device__ inline OperandStats reduce_partials(const DevState *st, int op, int nb, bool with_ge2,
                                               unsigned long long *sh) {
    unsigned long long gt0 = 0, ge1 = 0, ge3 = 0, inf = 0, ge2 = 0;
    unsigned int maxb = 0;
    for (int i = threadIdx.x; i < nb; i += kThreads) {
        const StatsPartial &p = st->part[op][i];
        gt0 += p.gt0;
        ge1 += p.ge1;
        ge3 += p.ge3;
        inf += p.inf;
        maxb = max(maxb, p.maxbits);
        if (with_ge2) ge2 += p.ge2;
    }
    OperandStats s;
    gt0 = block_sum(gt0, sh);
    ge1 = block_sum(ge1, sh);
    ge3 = block_sum(ge3, sh);
    inf = block_sum(inf, sh);
    ge2 = with_ge2 ? block_sum(ge2, sh) : 0;
    s.maxbits = block_max(maxb, sh);
    // every count of "|v| >= x" includes the non-finite values; remove them
    s.nnz = gt0 - inf;
    s.n1 = ge1 - inf;
    s.n3 = ge3 - inf;
    s.n2 = ge2;
    s.nonfinite = inf;
    s.pad = 0;
    return s;
}

__global__ __launch_bounds__(kThreads) void stats1_kernel(MatDesc a, MatDesc b, int blocks_a,
                                                          DevState *st) {
    __shared__ unsigned long long sh[kThreads / 64];
    st += blockIdx.z;
    a.ptr += (int64_t)blockIdx.z * a.bstride;
    b.ptr += (int64_t)blockIdx.z * b.bstride;
    const bool is_a = (int)blockIdx.x < blocks_a;
    const MatDesc &d = is_a ? a : b;
    const int64_t blk = is_a ? blockIdx.x : blockIdx.x - blocks_a;
    const int64_t nblk = is_a ? blocks_a : gridDim.x - blocks_a;
    Stage1Counter c;
    scan_matrix(d, blk, nblk, c);
    const unsigned long long gt0 = block_sum(c.gt0, sh);
    const unsigned long long ge1 = block_sum(c.ge1, sh);
    const unsigned long long ge3 = block_sum(c.ge3, sh);
    const unsigned long long inf = block_sum(c.inf, sh);
    const unsigned int maxb = block_max(c.maxb, sh);
    if (threadIdx.x == 0) {
        StatsPartial &p = st->part[is_a ? 0 : 1][blk];
        p.gt0 = (unsigned int)gt0;
        p.ge1 = (unsigned int)ge1;
        p.ge3 = (unsigned int)ge3;
        p.inf = (unsigned int)inf;
        p.maxbits = maxb;
        p.ge2 = 0;
    }
}

// flag: 0 = stage 2 only for operands failing stage 1, 1 = never, 2 = always
__device__ inline bool stage2_runs(const OperandStats &s, double t, int flag) {
    if (flag == 1 || s.nnz == 0) return false;
    if (flag == 2) return true;
    return s.nonfinite == 0 && !stage1_pass(s, t);
}

__global__ __launch_bounds__(kThreads) void stats2_kernel(MatDesc a, MatDesc b, int blocks_a,
                                                          DevState *st, double t, int flag) {
    __shared__ unsigned long long sh[kThreads / 64];
    st += blockIdx.z;
    a.ptr += (int64_t)blockIdx.z * a.bstride;
    b.ptr += (int64_t)blockIdx.z * b.bstride;
    const bool is_a = (int)blockIdx.x < blocks_a;
    const int op = is_a ? 0 : 1;
    const int64_t blk = is_a ? blockIdx.x : blockIdx.x - blocks_a;
    const int64_t nblk = is_a ? blocks_a : gridDim.x - blocks_a;
    const OperandStats s = reduce_partials(st, op, (int)nblk, false, sh);
    if (!stage2_runs(s, t, flag)) return;  // uniform over the block
    const MatDesc &d = is_a ? a : b;
    Stage2Counter c;
    c.thr = pow2_bits(emax_of_bits(s.maxbits) - kWindowSpan);
    scan_matrix(d, blk, nblk, c);
    const unsigned long long ge = block_sum(c.ge, sh);
    if (threadIdx.x == 0) st->part[op][blk].ge2 = (unsigned int)ge;
}

// Per-operand tolerance level (Sec. 4.1): FP16 if every element but a
// fraction t lies in the FP16 window without shifting; FP16 with scaling if
// the window shifted to emax holds all but a fraction t; BF16X3 if all but a
// fraction t3 lie above its floor; else FP32.  Non-finite data -> FP32.
__device__ inline int operand_level(const OperandStats &s, double t, double t3, bool stage2_ran) {
    if (s.nonfinite) return QCE_MODE_FP32;
    if (s.nnz == 0) return QCE_MODE_FP16X2;
    const double nnz = (double)s.nnz;
    const int emax = emax_of_bits(s.maxbits);
    if (emax <= kFp16Emax && (double)(s.nnz - s.n1) <= t * nnz) return QCE_MODE_FP16X2;
    if (stage2_ran && (double)(s.nnz - s.n2) <= t * nnz) return QCE_MODE_FP16X2_SCALED;
    if (emax <= kBf16x3Emax && (double)(s.nnz - s.n3) <= t3 * nnz) return QCE_MODE_BF16X3;
    return QCE_MODE_FP32;
}

__global__ __launch_bounds__(kThreads) void select_kernel(int blocks_a, int blocks_b, DevState *st,
                                                          double t, double t3, int forced,
                                                          int stage2_flag, int *mode_log, int slot) {
    __shared__ unsigned long long sh[kThreads / 64];
    st += blockIdx.x;                // one block per batch entry
    if (blockIdx.x != 0) mode_log = nullptr;
    OperandStats s[2];
    bool ran[2];
    for (int o = 0; o < 2; ++o) {
        const int nb = o == 0 ? blocks_a : blocks_b;
        s[o] = reduce_partials(st, o, nb, false, sh);
        ran[o] = stage2_runs(s[o], t, stage2_flag);  // uniform over the block
        if (ran[o]) s[o].n2 = reduce_partials(st, o, nb, true, sh).n2;
    }
    if (threadIdx.x != 0) return;
    int level[2];
    for (int o = 0; o < 2; ++o) level[o] = operand_level(s[o], t, t3, ran[o]);
    const int mode = forced >= 0 ? forced : max(level[0], level[1]);
    int shv[2] = {0, 0};
    if (mode == QCE_MODE_FP16X2_SCALED)
        for (int o = 0; o < 2; ++o) shv[o] = s[o].nnz ? kFp16Emax - emax_of_bits(s[o].maxbits) : 0;
    st->mode = mode;
    if (mode_log) mode_log[slot] = mode;
    st->shift[0] = shv[0];
    st->shift[1] = shv[1];
    qce_decision &r = st->last;
    r.mode = mode;
    r.sA = shv[0];
    r.sB = shv[1];
    r.stats_taken = 1;
    for (int o = 0; o < 2; ++o) {
        st->acc[o] = s[o];
        st->stage2[o] = ran[o];
        r.nnz[o] = (int64_t)s[o].nnz;
        r.n1[o] = (int64_t)s[o].n1;
        r.n2[o] = ran[o] ? (int64_t)s[o].n2 : -1;
        r.n3[o] = (int64_t)s[o].n3;
        r.nonfinite[o] = (int64_t)s[o].nonfinite;
        r.emax[o] = s[o].nnz ? emax_of_bits(s[o].maxbits) : INT32_MIN;
    }
}

int stats_blocks(int64_t nf) {
    // enough blocks to cover the device several times, not more than needed
    const int64_t per_block = (int64_t)kThreads * 64;  // >= 64 floats per thread
    int64_t b = (nf + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > 512) b = 512;
    return (int)b;
}

}  // namespace

hipError_t launch_stats1(const MatDesc &a, const MatDesc &b, DevState *st, hipStream_t s,
                         int batch) {
    const int ba = stats_blocks(2 * a.rows * a.cols), bb = stats_blocks(2 * b.rows * b.cols);
    hipLaunchKernelGGL(stats1_kernel, dim3(ba + bb, 1, batch), dim3(kThreads), 0, s, a, b, ba, st);
    return hipGetLastError();
}

hipError_t launch_stats2(const MatDesc &a, const MatDesc &b, DevState *st, double t, int flag,
                         hipStream_t s, int batch) {
    if (flag == 1) return hipSuccess;
    const int ba = stats_blocks(2 * a.rows * a.cols), bb = stats_blocks(2 * b.rows * b.cols);
    hipLaunchKernelGGL(stats2_kernel, dim3(ba + bb, 1, batch), dim3(kThreads), 0, s, a, b, ba, st, t,
                       flag);
    return hipGetLastError();
}

hipError_t launch_select(const MatDesc &a, const MatDesc &b, DevState *st, double t, double t3,
                         int forced_mode, int *mode_log, int slot, hipStream_t s, int batch) {
    // stage-2 flag as used by launch_stats2: forced modes skip stage 2,
    // forced_mode == -2 is the statistics-only entry point (stage 2 always)
    const int flag = forced_mode == -1 ? 0 : (forced_mode == -2 ? 2 : 1);
    const int forced = forced_mode < 0 ? -1 : forced_mode;
    const int ba = stats_blocks(2 * a.rows * a.cols), bb = stats_blocks(2 * b.rows * b.cols);
    hipLaunchKernelGGL(select_kernel, dim3(batch), dim3(kThreads), 0, s, ba, bb, st, t, t3, forced, flag,
                       mode_log, slot);
    return hipGetLastError();
}

}  // namespace qce
