// gemm_simple.hip -- one tile program per output sub-tensor for requests the
// tiled and decode kernels do not take: any dtype combination, any leading
// dimension or alignment, any partition up to 64 x 64.  Operands are decoded
// element by element into binary32 LDS tiles and contracted with binary32
// FMAs; the program stores only into its own sub-tensor.
#include "tg_device.hpp"
#include "tg_internal.hpp"

namespace tg {
namespace {

// OCP E4M3 code -> binary32 with integer operations only (exact).
__device__ __forceinline__ float e4m3_decode_sw(uint32_t c) {
    uint32_t s = (c & 0x80u) << 24;
    uint32_t em = c & 0x7fu;
    if (em == 0x7fu) return __builtin_bit_cast(float, 0x7fc00000u | s);
    if (em >= 8u)  // normal: exponent e + (127 - 7), mantissa m << 20
        return __builtin_bit_cast(float, s | ((em + (120u << 3)) << 20));
    float v = (float)em * 0x1p-9f;  // subnormal: m * 2^-9
    return s ? -v : v;
}

__device__ __forceinline__ float load_elem(const void *p, int dt, int64_t i) {
    if (dt == TG_F32) return static_cast<const float *>(p)[i];
    if (dt == TG_BF16)
        return bf16_bits_to_f32(static_cast<const uint16_t *>(p)[i]);
    return e4m3_decode_sw(static_cast<const uint8_t *>(p)[i]);
}

constexpr int SBM = 64, SBN = 64, SBK = 32, STH = 256;

__global__ __launch_bounds__(STH) void gemm_simple_kernel(SimpleArgs g) {
    __shared__ float As[SBM][SBK + 1];
    __shared__ float Bs[SBK][SBN + 1];
    const int tiles_n = (g.N + g.bn - 1) / g.bn;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    const int m0 = tm * g.bm, n0 = tn * g.bn;
    const int tid = threadIdx.x;
    constexpr int PER = SBM * SBN / STH;
    float acc[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) acc[j] = 0.0f;

    for (int k0 = 0; k0 < g.K; k0 += SBK) {
        for (int e = tid; e < SBM * SBK; e += STH) {
            int r = e / SBK, kk = e % SBK;
            int row = m0 + r, k = k0 + kk;
            float v = 0.0f;
            if (r < g.bm && row < g.M && k < g.K)
                v = load_elem(g.a, g.a_dtype, (int64_t)row * g.lda + k);
            As[r][kk] = v;
        }
        for (int e = tid; e < SBK * SBN; e += STH) {
            int kk = e / SBN, c = e % SBN;
            int col = n0 + c, k = k0 + kk;
            float v = 0.0f;
            if (c < g.bn && col < g.N && k < g.K) {
                int64_t off = g.b_nk ? (int64_t)col * g.ldb + k
                                     : (int64_t)k * g.ldb + col;
                v = load_elem(g.b, g.b_dtype, off);
            }
            Bs[kk][c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int e = tid + j * STH;
            int r = e / SBN, c = e % SBN;
            float s = acc[j];
#pragma unroll 8
            for (int kk = 0; kk < SBK; ++kk) s = fmaf(As[r][kk], Bs[kk][c], s);
            acc[j] = s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int e = tid + j * STH;
        int r = e / SBN, c = e % SBN;
        int row = m0 + r, col = n0 + c;
        if (r < g.bm && c < g.bn && row < g.M && col < g.N) {
            float x = acc[j];
            if (g.scale_a) x *= g.scale_a[row];
            if (g.scale_b) x *= g.scale_b[col];
            int64_t off = (int64_t)row * g.ldc + col;
            if (g.c_bf16)
                static_cast<uint16_t *>(g.c)[off] = f32_to_bf16_bits(x);
            else
                static_cast<float *>(g.c)[off] = x;
            if (g.wcount) atomicAdd(&g.wcount[(int64_t)row * g.N + col], 1);
        }
    }
}

}  // namespace

hipError_t launch_simple(const SimpleArgs &a, hipStream_t st) {
    int tiles = ((a.M + a.bm - 1) / a.bm) * ((a.N + a.bn - 1) / a.bn);
    hipLaunchKernelGGL(gemm_simple_kernel, dim3(tiles), dim3(STH), 0, st, a);
    return hipGetLastError();
}

}  // namespace tg
