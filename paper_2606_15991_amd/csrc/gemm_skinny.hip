// gemm_skinny.hip -- decode-shaped products y[M x N] = x[M x K] . W^T with
// M <= 16 and W stored N x K (bf16, or OCP E4M3 with one fp32 scale per row
// of W, i.e. per output column).
//
// The work is bound by streaming W from HBM once (arithmetic intensity about
// M flop per weight byte).  One tile program owns bn <= 16 RT output columns
// (RT row tiles of 16 weight rows, the rows past its bn repeating its last
// row) for all M rows, so that bn can divide N into a whole number of
// programs per compute unit; its KS wavefronts split
// K between them and stream their share of the weight rows with 16-byte
// loads, several in flight per lane.  With two row tiles every activation
// chunk loaded serves two weight chunks.  The contraction runs on the 16x16x32 bf16 matrix
// instruction with the weight rows as the A operand and the (zero-padded)
// activation rows as the B operand; E4M3 weights are decoded exactly to
// bf16 in registers first (there is no mixed bf16 x e4m3 matrix
// instruction).  The KS partial tiles are summed in LDS in a fixed order,
// and one wavefront stores the sub-tensor: deterministic, no atomics.
//
// Where one program per sub-tensor leaves compute units idle (few output
// columns) or streams too few bytes at once (long rows), the K steps are
// also split over `splitk` programs per sub-tensor (grid y).  Each stores
// its partial tile, unscaled, into its own slice part[s][M][N] of a
// workspace partitioned by (split, sub-tensor); a second launch, whose
// program p owns sub-tensor p of y, sums the slices in split order and
// stores y.  No atomics: the result is the same on every run.
#include "tg_device.hpp"
#include "tg_elementwise.hpp"
#include "tg_internal.hpp"

namespace tg {
namespace {


// 16 bytes at p of which only the first n (0..16) are inside the operand;
// the rest read as zero.  Used for the one chunk per row that straddles K.
__device__ __forceinline__ uint4 ld16_head(const char *p, int n) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int b = 0; b < 16; ++b)
        if (b < n) w[b >> 2] |= (uint32_t)(uint8_t)p[b] << (8 * (b & 3));
    return uint4{w[0], w[1], w[2], w[3]};
}

// Chunk of `epc` elements of `es` bytes starting at element k of a row of
// `K` elements: whole, partial, or past the end.
__device__ __forceinline__ uint4 ld_chunk(const char *row, int k, int K,
                                          int epc, int es) {
    if (k + epc <= K) return ld16(row + (int64_t)k * es);
    if (k < K) return ld16_head(row + (int64_t)k * es, (K - k) * es);
    return uint4{0, 0, 0, 0};
}

// Residual element (m, n), as binary32.
__device__ __forceinline__ float residual_at(const SkinnyArgs &g, int m,
                                             int n) {
    const int64_t off = (int64_t)m * g.ldr + n;
    return g.res_bf16
               ? bf16_bits_to_f32(static_cast<const uint16_t *>(g.res)[off])
               : static_cast<const float *>(g.res)[off];
}

// NORM (1 or 2): the activation rows are RMS-normalised on the fly (the
// normalisation step of the decode layer fused into the product): each
// activation chunk is multiplied by the matching chunk of the normalisation
// weights nw and rounded to bf16 before the contraction, the lanes
// accumulate the squares of the raw activations, and every output of row m
// is multiplied by 1 / sqrt(mean_k x[m, k]^2 + eps).  Every activation
// element of a row is loaded by exactly one lane of one wavefront of the
// program, so the program holds the whole row's sum of squares after its
// reduction.  NORM = 2 first copies the program's slice of nw into LDS and
// reads each chunk from there when it is needed; NORM = 1 (slices longer
// than the LDS budget) loads nw chunks into registers beside the
// activation chunks, which costs a third more registers per lane.
template <int WDT, int KS, bool CBF16, int RT, int NORM>
__device__ __forceinline__ void skinny_body(const SkinnyArgs &g,
                                            const void *nw, float eps) {
    // Elements of K covered by one 16-byte weight load per lane group:
    // bf16: 8 per lane, 4 lane groups -> 32;  e4m3: 16 per lane -> 64.
    constexpr int EPL = WDT == TG_BF16 ? 8 : 16;
    constexpr int KSTEP = 4 * EPL;
    // K steps per super-step: eight weight loads per lane either way
    constexpr int UNROLL = 8 / RT;
    __shared__ f32x4 part[KS][RT][64];
    __shared__ float ssq[NORM ? KS : 1][64];
    extern __shared__ uint4 nw_lds[];   // NORM == 2: this program's nw

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n0 = blockIdx.x * g.bn;
    const int n_end = min(n0 + g.bn, g.N);   // this program's columns
    const int r = lane & 15, grp = lane >> 4;
    const bool xrow_ok = r < g.M;
    const int xrow = xrow_ok ? r : 0;

    const char *W[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        int wrow = n0 + 16 * t + r;
        wrow = wrow < n_end ? wrow : n_end - 1;
        W[t] = static_cast<const char *>(g.w) +
               (int64_t)wrow * g.ldw * (WDT == TG_BF16 ? 2 : 1);
    }
    const uint16_t *X = static_cast<const uint16_t *>(g.x) +
                        (int64_t)xrow * g.ldx;

    f32x4 acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nsteps = (g.K + KSTEP - 1) / KSTEP;
    // this program's K steps: [sb, se) (the whole of K without a split)
    const int sb = blockIdx.y * g.steps_per_split;
    const int se = min(nsteps, sb + g.steps_per_split);
    constexpr int WES = WDT == TG_BF16 ? 2 : 1;
    constexpr int XV = WDT == TG_BF16 ? 1 : 2;   // activation chunks per step
    const char *Xc = reinterpret_cast<const char *>(X);
    const char *NWc = static_cast<const char *>(nw);
    float ss = 0.f;
    // Wave w takes super-steps w, w + KS, ... of UNROLL K steps each: all
    // UNROLL weight and activation chunks of a super-step are loaded before
    // any is contracted, so every lane has UNROLL weight loads in flight
    // (the other wavefronts of the SIMD overlap their own).  Super-steps
    // wholly inside K load without bounds tests: rows beyond the program's
    // columns were clamped to its last row (the repeated loads hit the same
    // cache lines) and activation rows beyond M read row 0, and both only
    // feed outputs that are never stored.  A ragged K tail takes the checked
    // loads.
    // Two register buffers (the wave's next super-step is loaded while the
    // current one is contracted) where the register budget allows: up to
    // 512 threads per program.
    constexpr int NB = KS <= 8 ? 2 : 1;
    uint4 wv[NB][UNROLL][RT], xv[NB][UNROLL][XV];
    uint4 nv[NORM == 1 ? NB : 1][NORM == 1 ? UNROLL : 1][NORM == 1 ? XV : 1];
    const int kb = sb * KSTEP;   // first element of this program's K range
    int s0 = 0;                  // first K step of the buffer contracted
    // NORM == 2: nw[kb, kb + (se - sb) KSTEP) into LDS as 16-byte chunks,
    // zeros past K; run after the first weight loads are issued, so that
    // its round trip overlaps theirs
    auto stage_nw = [&]() {
        if constexpr (NORM == 2) {
            const int chunks = (se - sb) * KSTEP / 8;
            for (int i = threadIdx.x; i < chunks; i += KS * 64)
                nw_lds[i] = ld_chunk(NWc, kb + 8 * i, g.K, 8, 2);
            __syncthreads();
        }
    };
    auto load_fast = [&](int s0, int b) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int k = (s0 + u) * KSTEP + grp * EPL;
#pragma unroll
            for (int t = 0; t < RT; ++t)
                wv[b][u][t] = ld16(W[t] + (int64_t)k * WES);
#pragma unroll
            for (int c = 0; c < XV; ++c) {
                xv[b][u][c] = ld16(Xc + (int64_t)(k + 8 * c) * 2);
                if constexpr (NORM == 1)
                    nv[b][u][c] = ld16(NWc + (int64_t)(k + 8 * c) * 2);
            }
        }
    };
    auto load_checked = [&](int s0, int b) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int k = (s0 + u) * KSTEP + grp * EPL;
            const bool live = s0 + u < se;
#pragma unroll
            for (int t = 0; t < RT; ++t)
                wv[b][u][t] = live ? ld_chunk(W[t], k, g.K, EPL, WES)
                                   : uint4{0, 0, 0, 0};
            const bool ok = live && k < g.K;
#pragma unroll
            for (int c = 0; c < XV; ++c) {
                xv[b][u][c] = ok ? ld_chunk(Xc, k + 8 * c, g.K, 8, 2)
                                 : uint4{0, 0, 0, 0};
                if constexpr (NORM == 1)
                    nv[b][u][c] = ok ? ld_chunk(NWc, k + 8 * c, g.K, 8, 2)
                                     : uint4{0, 0, 0, 0};
            }
        }
    };
    // x * nw rounded to bf16 (round to nearest even, by the packed
    // hardware conversion), eight at a time; squares of x into ss
    auto normed = [&](const uint4 &x, const uint4 &w) -> uint4 {
        typedef float f32x2_t __attribute__((ext_vector_type(2)));
        typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
        const uint32_t xa[4] = {x.x, x.y, x.z, x.w};
        const uint32_t wa[4] = {w.x, w.y, w.z, w.w};
        uint32_t o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float xl = __uint_as_float(xa[q] << 16);
            const float xh = __uint_as_float(xa[q] & 0xffff0000u);
            ss += xl * xl;
            ss += xh * xh;
            const f32x2_t p = {xl * __uint_as_float(wa[q] << 16),
                               xh * __uint_as_float(wa[q] & 0xffff0000u)};
            o[q] = __builtin_bit_cast(
                uint32_t, __builtin_convertvector(p, bf16x2_t));
        }
        return uint4{o[0], o[1], o[2], o[3]};
    };
    // buffer b holds the K steps s0 .. s0 + UNROLL - 1 (s0 as it stands
    // at every call below)
    auto contract = [&](int b) {
        if constexpr (NORM == 1) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
#pragma unroll
                for (int c = 0; c < XV; ++c)
                    xv[b][u][c] = normed(xv[b][u][c], nv[b][u][c]);
        } else if constexpr (NORM == 2) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int k = (s0 + u) * KSTEP + grp * EPL;
#pragma unroll
                for (int c = 0; c < XV; ++c)
                    xv[b][u][c] = normed(xv[b][u][c],
                                         nw_lds[(k - kb) / 8 + c]);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                if constexpr (WDT == TG_BF16) {
                    acc[t] = mfma16_bf16(
                        __builtin_bit_cast(i32x4, wv[b][u][t]),
                        __builtin_bit_cast(i32x4, xv[b][u][0]), acc[t]);
                } else {
                    uint2 w01 = e4m3x4_to_bf16x4(wv[b][u][t].x);
                    uint2 w23 = e4m3x4_to_bf16x4(wv[b][u][t].y);
                    uint2 w45 = e4m3x4_to_bf16x4(wv[b][u][t].z);
                    uint2 w67 = e4m3x4_to_bf16x4(wv[b][u][t].w);
                    i32x4 wa = {(int)w01.x, (int)w01.y, (int)w23.x, (int)w23.y};
                    i32x4 wb = {(int)w45.x, (int)w45.y, (int)w67.x, (int)w67.y};
                    acc[t] = mfma16_bf16(
                        wa, __builtin_bit_cast(i32x4, xv[b][u][0]), acc[t]);
                    acc[t] = mfma16_bf16(
                        wb, __builtin_bit_cast(i32x4, xv[b][u][1]), acc[t]);
                }
            }
    };
    constexpr int STRIDE = KS * UNROLL;
    // steps of this program wholly inside K (split boundaries fall on
    // super-step boundaries, so only the last split has a ragged tail)
    const int nfull = min(g.K / KSTEP, se);
    s0 = sb + wave * UNROLL;
    if constexpr (NB == 2) {
        bool have0 = s0 + UNROLL <= nfull;
        if (have0) load_fast(s0, 0);
        stage_nw();
        while (have0) {
            const int s1 = s0 + STRIDE;
            const bool have1 = s1 + UNROLL <= nfull;
            if (have1) load_fast(s1, NB - 1);
            contract(0);
            s0 = s1;
            if (!have1) break;
            const int s2 = s1 + STRIDE;
            have0 = s2 + UNROLL <= nfull;
            if (have0) load_fast(s2, 0);
            contract(NB - 1);
            s0 = s2;
        }
    } else {
        stage_nw();
        for (; s0 + UNROLL <= nfull; s0 += STRIDE) {
            load_fast(s0, 0);
            contract(0);
        }
    }
    for (; s0 < se; s0 += STRIDE) {           // ragged tail, bounds checked
        load_checked(s0, 0);
        contract(0);
    }

#pragma unroll
    for (int t = 0; t < RT; ++t) part[wave][t][lane] = acc[t];
    if constexpr (NORM) ssq[wave][lane] = ss;
    __syncthreads();
    if (wave != 0) return;
    // 16 x 16 result layout: lane l, register v holds row 4 * (l / 16) + v
    // (a weight row, i.e. output column) and column l % 16 (an output row).
    const int m = lane & 15;
    if (m >= g.M) return;
    if (g.splitk > 1) {
        // partial tile of split blockIdx.y, unscaled, into its own slice
        float *dst = g.part + (int64_t)blockIdx.y * g.M * g.N +
                     (int64_t)m * g.N;
        if constexpr (NORM) {
            if (blockIdx.x == 0 && grp == 0) {
                float tot = 0.f;
#pragma unroll
                for (int w = 0; w < KS; ++w)
#pragma unroll
                    for (int q = 0; q < 4; ++q) tot += ssq[w][m + 16 * q];
                g.ssq_part[blockIdx.y * g.M + m] = tot;
            }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            f32x4 s = part[0][t][lane];
#pragma unroll
            for (int w = 1; w < KS; ++w) {
                f32x4 p = part[w][t][lane];
                s[0] += p[0]; s[1] += p[1]; s[2] += p[2]; s[3] += p[3];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int n = n0 + 16 * t + 4 * grp + v;
                if (n < n_end) dst[n] = s[v];
            }
        }
        return;
    }
    float sa = g.scale_a ? g.scale_a[m] : 1.0f;
    if constexpr (NORM) {
        // row m's squares sit in lanes m, m + 16, m + 32, m + 48 of every
        // wavefront; summed in a fixed order
        float tot = 0.f;
#pragma unroll
        for (int w = 0; w < KS; ++w)
#pragma unroll
            for (int q = 0; q < 4; ++q) tot += ssq[w][m + 16 * q];
        sa *= 1.0f / sqrtf(tot / (float)g.K + eps);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        f32x4 s = part[0][t][lane];
#pragma unroll
        for (int w = 1; w < KS; ++w) {
            f32x4 p = part[w][t][lane];
            s[0] += p[0]; s[1] += p[1]; s[2] += p[2]; s[3] += p[3];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int n = n0 + 16 * t + 4 * grp + v;
            if (n < n_end) {
                float y = s[v] * sa;
                if (g.scale_w) y *= g.scale_w[n];
                if (g.res) y += residual_at(g, m, n);
                int64_t off = (int64_t)m * g.ldy + n;
                if constexpr (CBF16)
                    static_cast<uint16_t *>(g.y)[off] = f32_to_bf16_bits(y);
                else
                    static_cast<float *>(g.y)[off] = y;
                if (g.wcount) atomicAdd(&g.wcount[(int64_t)m * g.N + n], 1);
            }
        }
    }
}

template <int WDT, int KS, bool CBF16, int RT>
__global__ __launch_bounds__(KS * 64) void gemm_skinny_kernel(SkinnyArgs g) {
    skinny_body<WDT, KS, CBF16, RT, 0>(g, nullptr, 0.f);
}

// (bf16 weights, staged nw: three wavefronts per SIMD, as the plain bf16
// product runs; the staged variant fits the register budget for it)
template <int WDT, int KS, bool CBF16, int RT, int NORM>
__global__ __launch_bounds__(KS * 64) __attribute__((amdgpu_waves_per_eu(
    NORM == 2 && WDT == TG_BF16 ? 3 : 1))) void gemm_skinny_norm_kernel(
    SkinnyNormArgs a) {
    skinny_body<WDT, KS, CBF16, RT, NORM>(a.s, a.norm_w, a.eps);
}

// Merge of a split product: program p owns sub-tensor p of y (M rows x bn
// columns); its threads take the sub-tensor's elements in row-major order
// and sum the splitk partial values of each in split order, then apply the
// scales and add the residual.
template <bool CBF16, bool NORM>
__global__ __launch_bounds__(256) void skinny_merge_kernel(SkinnyArgs g,
                                                           float eps) {
    const int n0 = blockIdx.x * g.bn;
    for (int e = threadIdx.x; e < g.M * g.bn; e += 256) {
        const int m = e / g.bn, n = n0 + e % g.bn;
        if (n >= g.N) continue;
        const float *src = g.part + (int64_t)m * g.N + n;
        const int64_t slice = (int64_t)g.M * g.N;
        float v = src[0];
        for (int s = 1; s < g.splitk; ++s) v += src[s * slice];
        float sa = g.scale_a ? g.scale_a[m] : 1.0f;
        if constexpr (NORM) {
            float tot = g.ssq_part[m];
            for (int s = 1; s < g.splitk; ++s) tot += g.ssq_part[s * g.M + m];
            sa *= 1.0f / sqrtf(tot / (float)g.K + eps);
        }
        float y = v * sa;
        if (g.scale_w) y *= g.scale_w[n];
        if (g.res) y += residual_at(g, m, n);
        const int64_t off = (int64_t)m * g.ldy + n;
        if constexpr (CBF16)
            static_cast<uint16_t *>(g.y)[off] = f32_to_bf16_bits(y);
        else
            static_cast<float *>(g.y)[off] = y;
        if (g.wcount) atomicAdd(&g.wcount[(int64_t)m * g.N + n], 1);
    }
}

template <int WDT, int KS, int RT>
hipError_t launch_ks(int c_bf16, const SkinnyArgs &a, hipStream_t st) {
    dim3 grid((a.N + a.bn - 1) / a.bn, a.splitk), block(KS * 64);
    if (c_bf16)
        hipLaunchKernelGGL((gemm_skinny_kernel<WDT, KS, true, RT>), grid,
                           block, 0, st, a);
    else
        hipLaunchKernelGGL((gemm_skinny_kernel<WDT, KS, false, RT>), grid,
                           block, 0, st, a);
    return hipGetLastError();
}

template <int WDT, int RT>
hipError_t launch_w(int c_bf16, int ksplit, const SkinnyArgs &a,
                    hipStream_t st) {
    switch (ksplit) {
    case 1: return launch_ks<WDT, 1, RT>(c_bf16, a, st);
    case 2: return launch_ks<WDT, 2, RT>(c_bf16, a, st);
    case 4: return launch_ks<WDT, 4, RT>(c_bf16, a, st);
    case 8: return launch_ks<WDT, 8, RT>(c_bf16, a, st);
    case 16: return launch_ks<WDT, 16, RT>(c_bf16, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int WDT>
hipError_t launch_bn(int c_bf16, int bn, int ksplit, const SkinnyArgs &a,
                     hipStream_t st) {
    if (bn != a.bn || bn < 1 || bn > 32) return hipErrorInvalidValue;
    if (bn <= 16) return launch_w<WDT, 1>(c_bf16, ksplit, a, st);
    return launch_w<WDT, 2>(c_bf16, ksplit, a, st);
}

// LDS budget of the staged normalisation weights (one program's K range)
constexpr size_t kNormLdsMax = 32768;

template <int WDT, int RT>
hipError_t launch_norm_rt(int c_bf16, int ksplit, const SkinnyNormArgs &a,
                          hipStream_t st) {
    dim3 grid((a.s.N + a.s.bn - 1) / a.s.bn, a.s.splitk);
    // the fused normalisation runs with four wavefronts per program
    if (ksplit != 4) return hipErrorInvalidValue;
    dim3 block(4 * 64);
    constexpr int KSTEP = WDT == TG_BF16 ? 32 : 64;
    const size_t lds = (size_t)a.s.steps_per_split * KSTEP * 2;
    if (lds <= kNormLdsMax) {
        if (c_bf16)
            hipLaunchKernelGGL((gemm_skinny_norm_kernel<WDT, 4, true, RT, 2>),
                               grid, block, lds, st, a);
        else
            hipLaunchKernelGGL((gemm_skinny_norm_kernel<WDT, 4, false, RT, 2>),
                               grid, block, lds, st, a);
    } else {
        if (c_bf16)
            hipLaunchKernelGGL((gemm_skinny_norm_kernel<WDT, 4, true, RT, 1>),
                               grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((gemm_skinny_norm_kernel<WDT, 4, false, RT, 1>),
                               grid, block, 0, st, a);
    }
    return hipGetLastError();
}

template <int WDT>
hipError_t launch_norm_w(int c_bf16, int bn, int ksplit,
                         const SkinnyNormArgs &a, hipStream_t st) {
    if (bn != a.s.bn || bn < 1 || bn > 32) return hipErrorInvalidValue;
    if (bn <= 16) return launch_norm_rt<WDT, 1>(c_bf16, ksplit, a, st);
    return launch_norm_rt<WDT, 2>(c_bf16, ksplit, a, st);
}

}  // namespace

hipError_t launch_skinny_merge(int c_bf16, const SkinnyArgs &a, bool norm,
                               float eps, hipStream_t st) {
    dim3 grid((a.N + a.bn - 1) / a.bn), block(256);
    if (c_bf16) {
        if (norm)
            hipLaunchKernelGGL((skinny_merge_kernel<true, true>), grid, block,
                               0, st, a, eps);
        else
            hipLaunchKernelGGL((skinny_merge_kernel<true, false>), grid,
                               block, 0, st, a, eps);
    } else {
        if (norm)
            hipLaunchKernelGGL((skinny_merge_kernel<false, true>), grid,
                               block, 0, st, a, eps);
        else
            hipLaunchKernelGGL((skinny_merge_kernel<false, false>), grid,
                               block, 0, st, a, eps);
    }
    return hipGetLastError();
}

hipError_t launch_skinny_norm(int w_dtype, int c_bf16, int bn, int ksplit,
                              const SkinnyNormArgs &a, hipStream_t st) {
    if (w_dtype == TG_BF16)
        return launch_norm_w<TG_BF16>(c_bf16, bn, ksplit, a, st);
    if (w_dtype == TG_FP8_E4M3)
        return launch_norm_w<TG_FP8_E4M3>(c_bf16, bn, ksplit, a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_skinny(int w_dtype, int c_bf16, int bn, int ksplit,
                         const SkinnyArgs &a, hipStream_t st) {
    if (w_dtype == TG_BF16)
        return launch_bn<TG_BF16>(c_bf16, bn, ksplit, a, st);
    if (w_dtype == TG_FP8_E4M3)
        return launch_bn<TG_FP8_E4M3>(c_bf16, bn, ksplit, a, st);
    return hipErrorInvalidValue;
}

}  // namespace tg
