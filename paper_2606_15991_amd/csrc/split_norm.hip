// split_norm.hip -- two memory-bound helpers of the product path.
//
// (1) Split of binary32 operands into bfloat16 planes for the BF16x3 / BF16x6
//     precisions:  hi = bf16(a), mid = bf16(a - hi), lo = bf16(a - hi - mid),
//     each rounded to nearest even (the residuals are exact in binary32).
//     Plane block b of the destination receives plane order[b], so a single
//     bf16 product over the concatenated K axis sums the chosen plane
//     products into one binary32 accumulator.
// (2) Binary64 reductions of the relative Frobenius error of a result
//     against a binary64 reference (the only binary64 arithmetic on the GPU):
//     fixed-order two-pass reduction, no atomics, deterministic.
#include "tg_device.hpp"
#include "tg_internal.hpp"

namespace tg {
namespace {

__global__ void split_rows_kernel(const float *__restrict__ src, int64_t ld,
                                  int32_t rows, int32_t cols, int nplanes,
                                  uint32_t order, uint16_t *__restrict__ dst,
                                  int64_t ldd, int64_t plane_stride) {
    const int64_t total = (int64_t)rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / cols, j = e % cols;
        const float a = src[i * ld + j];
        uint16_t p[3];
        p[0] = f32_to_bf16_bits(a);
        const float r1 = a - bf16_bits_to_f32(p[0]);
        p[1] = f32_to_bf16_bits(r1);
        const float r2 = r1 - bf16_bits_to_f32(p[1]);
        p[2] = f32_to_bf16_bits(r2);
        for (int b = 0; b < nplanes; ++b) {
            const int which = (order >> (4 * b)) & 0xf;
            dst[b * plane_stride + i * ldd + j] = p[which];
        }
    }
}

constexpr int NORM_BLOCKS = 256, NORM_THREADS = 256;

__global__ __launch_bounds__(NORM_THREADS) void norm_partial_kernel(
    const void *__restrict__ c, int c_bf16, const double *__restrict__ r,
    int64_t n, double *__restrict__ out) {
    __shared__ double s_num[NORM_THREADS], s_den[NORM_THREADS];
    double num = 0.0, den = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x; i < n;
         i += (int64_t)NORM_BLOCKS * NORM_THREADS) {
        double cv = c_bf16 ? (double)bf16_bits_to_f32(
                                 static_cast<const uint16_t *>(c)[i])
                           : (double)static_cast<const float *>(c)[i];
        double rv = r[i];
        double d = cv - rv;
        num += d * d;
        den += rv * rv;
    }
    s_num[threadIdx.x] = num;
    s_den[threadIdx.x] = den;
    __syncthreads();
    for (int w = NORM_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_num[threadIdx.x] += s_num[threadIdx.x + w];
            s_den[threadIdx.x] += s_den[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 + 2 * blockIdx.x] = s_num[0];
        out[3 + 2 * blockIdx.x] = s_den[0];
    }
}

__global__ __launch_bounds__(64) void norm_final_kernel(double *out) {
    if (threadIdx.x != 0) return;
    double num = 0.0, den = 0.0;
    for (int b = 0; b < NORM_BLOCKS; ++b) {
        num += out[2 + 2 * b];
        den += out[3 + 2 * b];
    }
    out[0] = num;
    out[1] = den;
}

}  // namespace

hipError_t launch_split_rows(const float *src, int64_t ld, int32_t rows,
                             int32_t cols, int nplanes, const int8_t *order,
                             void *dst, int64_t ldd, int64_t plane_stride,
                             hipStream_t st) {
    uint32_t packed = 0;
    for (int b = 0; b < nplanes; ++b) packed |= (uint32_t)(order[b] & 0xf)
                                                << (4 * b);
    int64_t total = (int64_t)rows * cols;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       st, src, ld, rows, cols, nplanes, packed,
                       static_cast<uint16_t *>(dst), ldd, plane_stride);
    return hipGetLastError();
}

hipError_t launch_error_norm(const void *c, int c_bf16, const double *r,
                             int64_t n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(norm_partial_kernel, dim3(NORM_BLOCKS),
                       dim3(NORM_THREADS), 0, st, c, c_bf16, r, n, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(64), 0, st, out);
    return hipGetLastError();
}

}  // namespace tg
