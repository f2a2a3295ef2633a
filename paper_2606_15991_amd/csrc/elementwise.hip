// elementwise.hip -- z = x + y over a partitioned output: the tile
// programs' add (Sec. 2, the first listing; measured element-wise in
// Sec. 5.1).  z (rows x cols, row stride ldz) is split into bm x bn
// sub-tensors; the program launched as workgroup p owns sub-tensors
// p, p + G, ... of the row-major sub-tensor grid and stores only into them;
// x and y are shared reads.  Every element is added in binary32 and rounded
// once to the storage type: for bf16 operands (8 significant bits) the
// binary32 sum (24 bits >= 2 * 8 + 2) rounded to bf16 equals the correctly
// rounded sum, so the result is the exact sum rounded to nearest even.
//
// gfx950: the work is three HBM streams (two reads, one write), each touched
// once, so the 16-byte chunk loads and stores are non-temporal (they do not
// displace reusable lines from the caches; about 8 % faster at 2^28
// elements than ordinary ones).  Rows whose byte length and start are
// 16-byte aligned move in 16-byte chunks, four chunks of x and y in flight
// per lane before any is added; a row's last partial chunk and unaligned
// operands go element by element.
#include "tg_device.hpp"
#include "tg_internal.hpp"
#include "tg_elementwise.hpp"

namespace tg {
namespace {

constexpr int kAddThreads = 256;
constexpr int kAddUnroll = 4;

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 ld16_stream(const char *p) {
    const u32x4_t v =
        __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(p));
    return uint4{v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ void st16_stream(char *p, const uint4 &v) {
    __builtin_nontemporal_store(u32x4_t{v.x, v.y, v.z, v.w},
                                reinterpret_cast<u32x4_t *>(p));
}

template <int DT>
struct AddTraits;
template <>
struct AddTraits<TG_BF16> {
    static constexpr int ES = 2;
    __device__ static float load(const void *p, int64_t i) {
        const uint32_t b = static_cast<const uint16_t *>(p)[i];
        return __uint_as_float(b << 16);
    }
    __device__ static void store(void *p, int64_t i, float v) {
        static_cast<uint16_t *>(p)[i] = f32_to_bf16_bits(v);
    }
    // eight bf16 sums of a 16-byte chunk pair
    __device__ static uint4 add16(const uint4 &a, const uint4 &b) {
        const uint32_t wa[4] = {a.x, a.y, a.z, a.w};
        const uint32_t wb[4] = {b.x, b.y, b.z, b.w};
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float lo = __uint_as_float(wa[q] << 16) +
                             __uint_as_float(wb[q] << 16);
            const float hi = __uint_as_float(wa[q] & 0xffff0000u) +
                             __uint_as_float(wb[q] & 0xffff0000u);
            w[q] = (uint32_t)f32_to_bf16_bits(lo) |
                   ((uint32_t)f32_to_bf16_bits(hi) << 16);
        }
        return uint4{w[0], w[1], w[2], w[3]};
    }
    // eight bf16 products: the binary32 product of two 8-bit significands
    // is exact unless it falls below the binary32 normal range
    __device__ static uint4 mul16(const uint4 &a, const uint4 &b) {
        const uint32_t wa[4] = {a.x, a.y, a.z, a.w};
        const uint32_t wb[4] = {b.x, b.y, b.z, b.w};
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float lo = __uint_as_float(wa[q] << 16) *
                             __uint_as_float(wb[q] << 16);
            const float hi = __uint_as_float(wa[q] & 0xffff0000u) *
                             __uint_as_float(wb[q] & 0xffff0000u);
            w[q] = (uint32_t)f32_to_bf16_bits(lo) |
                   ((uint32_t)f32_to_bf16_bits(hi) << 16);
        }
        return uint4{w[0], w[1], w[2], w[3]};
    }
    // sum of the squares of the eight values of a chunk
    __device__ static float sumsq16(const uint4 &a) {
        const uint32_t wa[4] = {a.x, a.y, a.z, a.w};
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float lo = __uint_as_float(wa[q] << 16);
            const float hi = __uint_as_float(wa[q] & 0xffff0000u);
            s += lo * lo;
            s += hi * hi;
        }
        return s;
    }
    // x * scale * w for the eight values of a chunk, rounded to bf16
    __device__ static uint4 scale16(const uint4 &a, const uint4 &b, float sc) {
        const uint32_t wa[4] = {a.x, a.y, a.z, a.w};
        const uint32_t wb[4] = {b.x, b.y, b.z, b.w};
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float lo = __uint_as_float(wa[q] << 16) * sc *
                             __uint_as_float(wb[q] << 16);
            const float hi = __uint_as_float(wa[q] & 0xffff0000u) * sc *
                             __uint_as_float(wb[q] & 0xffff0000u);
            w[q] = (uint32_t)f32_to_bf16_bits(lo) |
                   ((uint32_t)f32_to_bf16_bits(hi) << 16);
        }
        return uint4{w[0], w[1], w[2], w[3]};
    }
};
template <>
struct AddTraits<TG_F32> {
    static constexpr int ES = 4;
    __device__ static float load(const void *p, int64_t i) {
        return static_cast<const float *>(p)[i];
    }
    __device__ static void store(void *p, int64_t i, float v) {
        static_cast<float *>(p)[i] = v;
    }
    __device__ static uint4 add16(const uint4 &a, const uint4 &b) {
        return uint4{__float_as_uint(__uint_as_float(a.x) + __uint_as_float(b.x)),
                     __float_as_uint(__uint_as_float(a.y) + __uint_as_float(b.y)),
                     __float_as_uint(__uint_as_float(a.z) + __uint_as_float(b.z)),
                     __float_as_uint(__uint_as_float(a.w) + __uint_as_float(b.w))};
    }
    __device__ static uint4 mul16(const uint4 &a, const uint4 &b) {
        return uint4{__float_as_uint(__uint_as_float(a.x) * __uint_as_float(b.x)),
                     __float_as_uint(__uint_as_float(a.y) * __uint_as_float(b.y)),
                     __float_as_uint(__uint_as_float(a.z) * __uint_as_float(b.z)),
                     __float_as_uint(__uint_as_float(a.w) * __uint_as_float(b.w))};
    }
    __device__ static float sumsq16(const uint4 &a) {
        const float v[4] = {__uint_as_float(a.x), __uint_as_float(a.y),
                            __uint_as_float(a.z), __uint_as_float(a.w)};
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) s += v[q] * v[q];
        return s;
    }
    __device__ static uint4 scale16(const uint4 &a, const uint4 &b, float sc) {
        return uint4{
            __float_as_uint(__uint_as_float(a.x) * sc * __uint_as_float(b.x)),
            __float_as_uint(__uint_as_float(a.y) * sc * __uint_as_float(b.y)),
            __float_as_uint(__uint_as_float(a.z) * sc * __uint_as_float(b.z)),
            __float_as_uint(__uint_as_float(a.w) * sc * __uint_as_float(b.w))};
    }
};

// The binary operation of the element-wise kernels: z = x + y (MUL false)
// or z = x * y (MUL true), one binary32 operation rounded once.
template <int DT, bool MUL>
__device__ __forceinline__ uint4 op16(const uint4 &a, const uint4 &b) {
    if constexpr (MUL) return AddTraits<DT>::mul16(a, b);
    else return AddTraits<DT>::add16(a, b);
}
template <bool MUL>
__device__ __forceinline__ float op1(float a, float b) {
    if constexpr (MUL) return a * b;
    else return a + b;
}

template <int DT, bool VEC, bool MUL>
__device__ __forceinline__ void elementwise_body(const AddArgs &g) {
    using T = AddTraits<DT>;
    constexpr int EPC = 16 / T::ES;               // elements per chunk
    const int64_t tiles_n = (g.cols + g.bn - 1) / g.bn;
    const int64_t tiles = ((g.rows + g.bm - 1) / g.bm) * tiles_n;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t r0 = (t / tiles_n) * g.bm, c0 = (t % tiles_n) * g.bn;
        const int64_t nr = g.rows - r0 < g.bm ? g.rows - r0 : g.bm;
        const int64_t nc = g.cols - c0 < g.bn ? g.cols - c0 : g.bn;
        if constexpr (VEC) {
            // full chunks of every row of the sub-tensor, then the partial
            // chunk that ends a row (bn is a multiple of EPC, so only the
            // last column tile of a row has one)
            const int64_t cpr = nc / EPC;              // full chunks per row
            const int64_t total = nr * cpr;
            // 32-bit division where the sub-tensor's chunk count allows
            const bool small = total < ((int64_t)1 << 31);
            const int64_t step = (int64_t)kAddThreads * kAddUnroll;
            for (int64_t base = threadIdx.x; base < total; base += step) {
                uint4 a[kAddUnroll], b[kAddUnroll];
                int64_t off[kAddUnroll][3];
#pragma unroll
                for (int u = 0; u < kAddUnroll; ++u) {
                    const int64_t q = base + (int64_t)u * kAddThreads;
                    if (q < total) {
                        int64_t r, c;
                        if (small) {
                            const uint32_t qq = (uint32_t)q,
                                           cc = (uint32_t)cpr;
                            r = r0 + qq / cc;
                            c = c0 + (int64_t)(qq % cc) * EPC;
                        } else {
                            r = r0 + q / cpr;
                            c = c0 + (q % cpr) * EPC;
                        }
                        off[u][0] = (r * g.ldx + c) * T::ES;
                        off[u][1] = (r * g.ldy + c) * T::ES;
                        off[u][2] = (r * g.ldz + c) * T::ES;
                        a[u] = ld16_stream(static_cast<const char *>(g.x) +
                                           off[u][0]);
                        b[u] = ld16_stream(static_cast<const char *>(g.y) +
                                           off[u][1]);
                    }
                }
#pragma unroll
                for (int u = 0; u < kAddUnroll; ++u) {
                    const int64_t q = base + (int64_t)u * kAddThreads;
                    if (q < total)
                        st16_stream(static_cast<char *>(g.z) + off[u][2],
                                    op16<DT, MUL>(a[u], b[u]));
                }
            }
            const int64_t rest = nc - cpr * EPC;
            for (int64_t q = threadIdx.x; q < nr * rest; q += kAddThreads) {
                const int64_t r = r0 + q / rest;
                const int64_t c = c0 + cpr * EPC + q % rest;
                T::store(g.z, r * g.ldz + c,
                         op1<MUL>(T::load(g.x, r * g.ldx + c),
                                  T::load(g.y, r * g.ldy + c)));
            }
        } else {
            for (int64_t q = threadIdx.x; q < nr * nc; q += kAddThreads) {
                const int64_t r = r0 + q / nc, c = c0 + q % nc;
                T::store(g.z, r * g.ldz + c,
                         op1<MUL>(T::load(g.x, r * g.ldx + c),
                                  T::load(g.y, r * g.ldy + c)));
            }
        }
        if (g.wcount) {
            // instrumented launches: one count per stored element
            for (int64_t q = threadIdx.x; q < nr * nc; q += kAddThreads)
                atomicAdd(&g.wcount[(r0 + q / nc) * g.cols + c0 + q % nc], 1);
        }
    }
}

template <int DT, bool VEC>
__global__ __launch_bounds__(kAddThreads) void add_kernel(AddArgs g) {
    elementwise_body<DT, VEC, false>(g);
}

template <int DT, bool VEC>
__global__ __launch_bounds__(kAddThreads) void mul_kernel(AddArgs g) {
    elementwise_body<DT, VEC, true>(g);
}

// RMS normalisation (the first step of the decode layer of Sec. 3.2's
// graph-scope listing): y[r, :] = x[r, :] * w / sqrt(mean(x[r, :]^2) + eps).
// y is split into bm x cols sub-tensors (whole rows: a row's scale needs
// every element of the row); program p owns sub-tensors p, p + G, ...  The
// sum of squares is accumulated in binary32 per lane, then over each
// wavefront and the four wavefronts in a fixed order (deterministic); each
// output is x * scale * w in binary32 rounded once to the storage type.
constexpr int kNormThreads = 256;

// With VEC (x, w, y 16-byte aligned, rows a whole number of 16-byte
// chunks apart) each lane moves 16-byte chunks, kNormUnroll of them in
// flight before any is used: a decode row (one program, 5120 bf16) is then
// two or three memory round trips instead of one per element.  The row is
// read twice (the second pass mostly from cache).
constexpr int kNormUnroll = 4;

template <int DT, bool VEC>
__global__ __launch_bounds__(kNormThreads) void rms_norm_kernel(NormArgs g) {
    using T = AddTraits<DT>;
    constexpr int EPC = 16 / T::ES;
    constexpr int U = kNormUnroll;
    __shared__ float red[kNormThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tiles = (g.rows + g.bm - 1) / g.bm;
    const int64_t nch = VEC ? g.cols / EPC : 0;      // whole chunks per row
    const int64_t c_rest = nch * EPC;                // first scalar column
    const char *W = static_cast<const char *>(g.w);
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t r0 = t * g.bm;
        const int64_t nr = g.rows - r0 < g.bm ? g.rows - r0 : g.bm;
        for (int64_t i = 0; i < nr; ++i) {
            const int64_t r = r0 + i;
            const char *X = static_cast<const char *>(g.x) + r * g.ldx * T::ES;
            char *Y = static_cast<char *>(g.y) + r * g.ldy * T::ES;
            float ss = 0.f;
            for (int64_t base = threadIdx.x; base < nch;
                 base += kNormThreads * U) {
                uint4 a[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t q = base + u * kNormThreads;
                    a[u] = q < nch ? ld16(X + q * 16) : uint4{0, 0, 0, 0};
                }
#pragma unroll
                for (int u = 0; u < U; ++u) ss += T::sumsq16(a[u]);
            }
            for (int64_t c = c_rest + threadIdx.x; c < g.cols;
                 c += kNormThreads) {
                const float v = T::load(X, c);
                ss += v * v;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
            if (lane == 0) red[wave] = ss;
            __syncthreads();
            float tot = red[0];
#pragma unroll
            for (int q = 1; q < kNormThreads / 64; ++q) tot += red[q];
            __syncthreads();                  // red is rewritten next row
            const float scale = 1.0f / sqrtf(tot / (float)g.cols + g.eps);
            for (int64_t base = threadIdx.x; base < nch;
                 base += kNormThreads * U) {
                uint4 a[U], b[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t q = base + u * kNormThreads;
                    if (q < nch) {
                        a[u] = ld16(X + q * 16);
                        b[u] = ld16(W + q * 16);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t q = base + u * kNormThreads;
                    if (q < nch) st16(Y + q * 16, T::scale16(a[u], b[u], scale));
                }
            }
            for (int64_t c = c_rest + threadIdx.x; c < g.cols;
                 c += kNormThreads)
                T::store(Y, c, T::load(X, c) * scale * T::load(W, c));
            if (g.wcount) {
                for (int64_t c = threadIdx.x; c < g.cols; c += kNormThreads)
                    atomicAdd(&g.wcount[r * g.cols + c], 1);
            }
        }
    }
}

}  // namespace

template <int DT>
void launch_norm_dt(const NormArgs &a, bool vec, dim3 grid, hipStream_t st) {
    if (vec)
        hipLaunchKernelGGL((rms_norm_kernel<DT, true>), grid,
                           dim3(kNormThreads), 0, st, a);
    else
        hipLaunchKernelGGL((rms_norm_kernel<DT, false>), grid,
                           dim3(kNormThreads), 0, st, a);
}

hipError_t launch_rms_norm(const NormArgs &a, bool vec, int programs,
                           hipStream_t st) {
    if (a.dtype == TG_BF16)
        launch_norm_dt<TG_BF16>(a, vec, dim3(programs), st);
    else if (a.dtype == TG_F32)
        launch_norm_dt<TG_F32>(a, vec, dim3(programs), st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_mul(const AddArgs &a, bool vec, int programs,
                      hipStream_t st) {
    dim3 grid(programs), block(kAddThreads);
    if (a.dtype == TG_BF16) {
        if (vec)
            hipLaunchKernelGGL((mul_kernel<TG_BF16, true>), grid, block, 0,
                               st, a);
        else
            hipLaunchKernelGGL((mul_kernel<TG_BF16, false>), grid, block, 0,
                               st, a);
    } else if (a.dtype == TG_F32) {
        if (vec)
            hipLaunchKernelGGL((mul_kernel<TG_F32, true>), grid, block, 0, st,
                               a);
        else
            hipLaunchKernelGGL((mul_kernel<TG_F32, false>), grid, block, 0,
                               st, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_add(const AddArgs &a, bool vec, int programs,
                      hipStream_t st) {
    dim3 grid(programs), block(kAddThreads);
    if (a.dtype == TG_BF16) {
        if (vec)
            hipLaunchKernelGGL((add_kernel<TG_BF16, true>), grid, block, 0,
                               st, a);
        else
            hipLaunchKernelGGL((add_kernel<TG_BF16, false>), grid, block, 0,
                               st, a);
    } else if (a.dtype == TG_F32) {
        if (vec)
            hipLaunchKernelGGL((add_kernel<TG_F32, true>), grid, block, 0, st,
                               a);
        else
            hipLaunchKernelGGL((add_kernel<TG_F32, false>), grid, block, 0,
                               st, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tg
