// The element splits of Sec. 2.1 (Eq. 2) and the bfloat16 three-term split,
// shared by the panel writer (split.hip) and the GEMM kernels that split
// their operands as they load them (gemm.hip).  All conversions round to
// nearest even; the subtractions are exact in FP32 and the power-of-two
// scaling is exact (ldexp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qce {

__device__ inline uint16_t f16_bits(float v) {
    _Float16 h = (_Float16)v;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float f16_val(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
__device__ inline uint16_t bf16_bits(float v) {
    __bf16 h = (__bf16)v;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float bf16_val(uint16_t b) { return __uint_as_float((unsigned int)b << 16); }

// FP16 two-term split of x' = x * 2^shift (Eq. 2)
__device__ inline void split_fp16x2(float x, int shift, uint16_t &hi, uint16_t &lo) {
    float xs = ldexpf(x, shift);
    hi = f16_bits(xs);
    float r = xs - f16_val(hi);  // exact
    lo = f16_bits(r * 2048.0f);  // residual scaled by 2^11
}

// bfloat16 three-term split
__device__ inline void split_bf16x3(float x, uint16_t &b0, uint16_t &b1, uint16_t &b2) {
    b0 = bf16_bits(x);
    float r1 = x - bf16_val(b0);  // exact
    b1 = bf16_bits(r1);
    float r2 = r1 - bf16_val(b1);  // exact
    b2 = bf16_bits(r2);
}

__device__ inline uint4 pack8(const uint16_t *v) {
    uint4 r;
    r.x = (unsigned)v[0] | ((unsigned)v[1] << 16);
    r.y = (unsigned)v[2] | ((unsigned)v[3] << 16);
    r.z = (unsigned)v[4] | ((unsigned)v[5] << 16);
    r.w = (unsigned)v[6] | ((unsigned)v[7] << 16);
    return r;
}

}  // namespace qce
