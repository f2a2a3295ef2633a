// tg_device.hpp -- gfx950 device helpers: vector types, MFMA wrappers,
// element conversions.  Included by the kernel translation units only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Bit reinterpretation through a by-value parameter.  (Applying
// __builtin_bit_cast directly to an element of an ext_vector_type value reads
// element 0 with this compiler, so elements are always passed by value.)
__device__ __forceinline__ float as_f32(uint32_t u) {
    return __builtin_bit_cast(float, u);
}
__device__ __forceinline__ uint32_t as_u32(float f) {
    return __builtin_bit_cast(uint32_t, f);
}

// 32x32 output tile, one K-step of the operand type.
//   bf16: K = 16 per instruction, 8 values per lane (one 16-byte chunk).
//   f32:  K = 2 per instruction, 1 value per lane.
//   e4m3: K = 64 per instruction, 32 values per lane (two chunks).
// Lane l supplies row (l % 32) of the A operand and column (l % 32) of the
// B operand; the K positions a lane supplies are the same for A and B, so
// any assignment of K indices to (lane group, register slot) that both
// operands share yields the same dot products.
__device__ __forceinline__ f32x16 mfma_bf16(const i32x4 &a, const i32x4 &b,
                                            f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(
        __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
        0);
}

__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// OCP E4M3 x OCP E4M3 (format code 0 for both operands), unit block scales
// (E8M0 code 127 = 2^0).
__device__ __forceinline__ f32x16 mfma_fp8(const i32x8 &a, const i32x8 &b,
                                           f32x16 c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0,
                                                           127, 0, 127);
}

// 16x16 output tile, K = 32 bf16 per instruction.
__device__ __forceinline__ f32x4 mfma16_bf16(const i32x4 &a, const i32x4 &b,
                                             f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
        0);
}

// Round-to-nearest-even float -> bfloat16 bits (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) {
    return __builtin_bit_cast(float, h << 16);
}

// Four OCP E4M3 codes (one dword) -> four floats, exact.
__device__ __forceinline__ f32x4 e4m3x4_to_f32(uint32_t w) {
    f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
    f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
    return f32x4{lo.x, lo.y, hi.x, hi.y};
}

// Four OCP E4M3 codes -> four bf16 (two dwords), exact: every E4M3 value is
// a bf16 value.  The gfx950 scaled conversion turns two codes into two bf16
// in one instruction; with the scale 1 it is the plain decode.
__device__ __forceinline__ uint2 e4m3x4_to_bf16x4(uint32_t w) {
    typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
    const bf16x2_t lo = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, 1.0f,
                                                                 false);
    const bf16x2_t hi = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, 1.0f,
                                                                 true);
    return uint2{__builtin_bit_cast(uint32_t, lo),
                 __builtin_bit_cast(uint32_t, hi)};
}

__device__ __forceinline__ uint4 ld16(const void *p) {
    return *reinterpret_cast<const uint4 *>(p);
}

__device__ __forceinline__ void st16(void *p, const uint4 &v) {
    *reinterpret_cast<uint4 *>(p) = v;
}

}  // namespace tg
