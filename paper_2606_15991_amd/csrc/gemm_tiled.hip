// gemm_tiled.hip -- persistent tile programs for C = A . B on gfx950 MFMA.
//
// One workgroup is one tile program of the mapped-partition schedule
// (Sec. 3.6 of the paper): it owns the output sub-tensors
// program_slot(p) + r*G of the traversal order, and for each of them
//   acc = 0; for every K tile: acc += A[BM x BK] . B[BK x BN]; store acc
// into its own BM x BN sub-tensor only.  A and B are read-only.
//
// gfx950 design:
//   * every K tile is 128 bytes deep (64 bf16, 32 f32 or 128 e4m3), so both
//     operands live in LDS as [rows][128 B] with the 16-byte chunk index
//     XOR-swizzled by (row & 7): 16-byte reads and writes of 8 consecutive
//     rows hit 8 distinct chunk positions, i.e. all 32 banks once;
//   * B is held n-major in LDS (k contiguous, like A); a B stored K x N is
//     transposed in registers, 8 x 8 (bf16) or 4 x 4 (f32) blocks at a time,
//     between the coalesced 16-byte global loads and the LDS writes;
//   * two LDS stages: while the MFMAs consume stage s, the next K tile is in
//     flight from global memory into registers and is written into stage
//     s ^ 1 afterwards; one barrier per K tile;
//   * rows of A beyond M and columns of B beyond N are clamped to valid
//     addresses (their products only reach outputs that are never stored),
//     so full K tiles carry no predicates; the K tail is zero-filled.
#include <atomic>

#include "tg_device.hpp"
#include "tg_internal.hpp"

namespace tg {
namespace {

template <int DT>
struct DtypeTraits;
template <>
struct DtypeTraits<TG_BF16> {
    static constexpr int ES = 2;
};
template <>
struct DtypeTraits<TG_F32> {
    static constexpr int ES = 4;
};
template <>
struct DtypeTraits<TG_FP8_E4M3> {
    static constexpr int ES = 1;
};

template <int DT, int BM_, int BN_, int WM_, int WN_, bool BNK_, bool CBF16_>
struct Cfg {
    static constexpr int DTYPE = DT;
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
    static constexpr bool BNK = BNK_, CBF16 = CBF16_;
    static constexpr int ES = DtypeTraits<DT>::ES;
    static constexpr int EPC = 16 / ES;         // elements per 16-byte chunk
    static constexpr int BK = 128 / ES;         // K elements per K tile
    static constexpr int THREADS = WM * WN * 64;
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int FM = TM / 32, FN = TN / 32;
    static constexpr int A_CH = BM * 8 / THREADS;   // A chunks per thread
    static constexpr int B_CH = BN * 8 / THREADS;   // B chunks (n-major B)
    // k-major B: EPC x EPC blocks, (BK / EPC) * (BN / EPC) of them
    static constexpr int B_BLK = (BK / EPC) * (BN / EPC);
    static constexpr int B_BLK_PT = (B_BLK + THREADS - 1) / THREADS;
    static constexpr int STAGE = (BM + BN) * 128;   // bytes per LDS stage
    static_assert(TM % 32 == 0 && TN % 32 == 0, "wave tile");
    static_assert((BM * 8) % THREADS == 0, "A chunk split");
    static_assert(BNK || DT != TG_FP8_E4M3, "e4m3 B must be stored N x K");
    static_assert(!BNK || (BN * 8) % THREADS == 0, "B chunk split");
};

__device__ __forceinline__ int swz(int row, int chunk) {
    return row * 128 + ((chunk ^ (row & 7)) << 4);
}

template <class C>
struct Tile {
    // registers holding the next K tile between its global load and its
    // LDS write
    uint4 ra[C::A_CH];
    uint4 rb[C::BNK ? C::B_CH : C::B_BLK_PT * C::EPC];

    template <bool MASK>
    __device__ __forceinline__ void load(const GemmArgs &g, int m0, int n0,
                                         int k0, int tid) {
        const char *A = static_cast<const char *>(g.a);
        const char *B = static_cast<const char *>(g.b);
#pragma unroll
        for (int i = 0; i < C::A_CH; ++i) {
            int q = i * C::THREADS + tid;
            int r = q >> 3, kc = q & 7;
            int row = m0 + r;
            row = row < g.M ? row : g.M - 1;
            int k = k0 + kc * C::EPC;
            if (MASK && k >= g.K) {
                ra[i] = uint4{0, 0, 0, 0};
            } else {
                ra[i] = ld16(A + ((int64_t)row * g.lda + k) * C::ES);
            }
        }
        if constexpr (C::BNK) {
#pragma unroll
            for (int i = 0; i < C::B_CH; ++i) {
                int q = i * C::THREADS + tid;
                int r = q >> 3, kc = q & 7;
                int row = n0 + r;
                row = row < g.N ? row : g.N - 1;
                int k = k0 + kc * C::EPC;
                if (MASK && k >= g.K) {
                    rb[i] = uint4{0, 0, 0, 0};
                } else {
                    rb[i] = ld16(B + ((int64_t)row * g.ldb + k) * C::ES);
                }
            }
        } else {
            constexpr int NB = C::BN / C::EPC;
#pragma unroll
            for (int i = 0; i < C::B_BLK_PT; ++i) {
                int blk = i * C::THREADS + tid;
                if (C::B_BLK % C::THREADS != 0 && blk >= C::B_BLK) break;
                int kb = blk / NB, nb = blk % NB;
                int col = n0 + nb * C::EPC;
                col = col < g.N ? col : g.N - C::EPC;
#pragma unroll
                for (int r = 0; r < C::EPC; ++r) {
                    int k = k0 + kb * C::EPC + r;
                    if (MASK && k >= g.K) {
                        rb[i * C::EPC + r] = uint4{0, 0, 0, 0};
                    } else {
                        rb[i * C::EPC + r] =
                            ld16(B + ((int64_t)k * g.ldb + col) * C::ES);
                    }
                }
            }
        }
    }

    __device__ __forceinline__ void store(char *stage, int tid) {
        char *As = stage;
        char *Bs = stage + C::BM * 128;
#pragma unroll
        for (int i = 0; i < C::A_CH; ++i) {
            int q = i * C::THREADS + tid;
            st16(As + swz(q >> 3, q & 7), ra[i]);
        }
        if constexpr (C::BNK) {
#pragma unroll
            for (int i = 0; i < C::B_CH; ++i) {
                int q = i * C::THREADS + tid;
                st16(Bs + swz(q >> 3, q & 7), rb[i]);
            }
        } else {
            constexpr int NB = C::BN / C::EPC;
#pragma unroll
            for (int i = 0; i < C::B_BLK_PT; ++i) {
                int blk = i * C::THREADS + tid;
                if (C::B_BLK % C::THREADS != 0 && blk >= C::B_BLK) break;
                int kb = blk / NB, nb = blk % NB;
                const uint4 *r = &rb[i * C::EPC];
                if constexpr (C::ES == 2) {
                    // 8 x 8 bf16 block: rows k, columns n -> chunks (n, k..k+7)
                    const uint32_t *w = reinterpret_cast<const uint32_t *>(r);
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        uint32_t o[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            uint32_t x = w[(2 * j) * 4 + c / 2];
                            uint32_t y = w[(2 * j + 1) * 4 + c / 2];
                            o[j] = (c & 1) ? ((x >> 16) | (y & 0xffff0000u))
                                           : ((x & 0xffffu) | (y << 16));
                        }
                        st16(Bs + swz(nb * 8 + c, kb),
                             uint4{o[0], o[1], o[2], o[3]});
                    }
                } else {
                    // 4 x 4 f32 block
                    const uint32_t *w = reinterpret_cast<const uint32_t *>(r);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        st16(Bs + swz(nb * 4 + c, kb),
                             uint4{w[0 * 4 + c], w[1 * 4 + c], w[2 * 4 + c],
                                   w[3 * 4 + c]});
                    }
                }
            }
        }
    }
};

template <class C>
__device__ __forceinline__ void compute_stage(const char *stage, int wm,
                                              int wn, int lane,
                                              f32x16 (&acc)[C::FM][C::FN]) {
    const char *As = stage;
    const char *Bs = stage + C::BM * 128;
    const int r = lane & 31, half = lane >> 5;
    if constexpr (C::DTYPE == TG_BF16 || C::DTYPE == TG_F32) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int c = 2 * kk + half;
            i32x4 af[C::FM], bfr[C::FN];
#pragma unroll
            for (int f = 0; f < C::FM; ++f)
                af[f] = *reinterpret_cast<const i32x4 *>(
                    As + swz(wm * C::TM + f * 32 + r, c));
#pragma unroll
            for (int f = 0; f < C::FN; ++f)
                bfr[f] = *reinterpret_cast<const i32x4 *>(
                    Bs + swz(wn * C::TN + f * 32 + r, c));
#pragma unroll
            for (int i = 0; i < C::FM; ++i)
#pragma unroll
                for (int j = 0; j < C::FN; ++j) {
                    if constexpr (C::DTYPE == TG_BF16) {
                        acc[i][j] = mfma_bf16(af[i], bfr[j], acc[i][j]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const uint32_t ua = af[i][e], ub = bfr[j][e];
                            acc[i][j] =
                                mfma_f32(as_f32(ua), as_f32(ub), acc[i][j]);
                        }
                    }
                }
        }
    } else {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int c = 4 * kk + 2 * half;
            i32x8 af[C::FM], bfr[C::FN];
#pragma unroll
            for (int f = 0; f < C::FM; ++f) {
                const int row = wm * C::TM + f * 32 + r;
                i32x4 lo = *reinterpret_cast<const i32x4 *>(As + swz(row, c));
                i32x4 hi =
                    *reinterpret_cast<const i32x4 *>(As + swz(row, c + 1));
                af[f] = i32x8{lo[0], lo[1], lo[2], lo[3],
                              hi[0], hi[1], hi[2], hi[3]};
            }
#pragma unroll
            for (int f = 0; f < C::FN; ++f) {
                const int row = wn * C::TN + f * 32 + r;
                i32x4 lo = *reinterpret_cast<const i32x4 *>(Bs + swz(row, c));
                i32x4 hi =
                    *reinterpret_cast<const i32x4 *>(Bs + swz(row, c + 1));
                bfr[f] = i32x8{lo[0], lo[1], lo[2], lo[3],
                               hi[0], hi[1], hi[2], hi[3]};
            }
#pragma unroll
            for (int i = 0; i < C::FM; ++i)
#pragma unroll
                for (int j = 0; j < C::FN; ++j)
                    acc[i][j] = mfma_fp8(af[i], bfr[j], acc[i][j]);
        }
    }
}

// Store one program's accumulators into its own sub-tensor.
// 32 x 32 MFMA result layout: lane l, register v holds
//   row 8 * (v / 4) + 4 * (l / 32) + v % 4,  column l % 32.
template <class C>
__device__ __forceinline__ void epilogue(const GemmArgs &g, int m0, int n0,
                                         int wm, int wn, int lane,
                                         f32x16 (&acc)[C::FM][C::FN]) {
    const int col_l = lane & 31, half = lane >> 5;
#pragma unroll
    for (int j = 0; j < C::FN; ++j) {
        const int col = n0 + wn * C::TN + j * 32 + col_l;
        const bool col_ok = col < g.N;
        const float sb = (g.scale_b && col_ok) ? g.scale_b[col] : 1.0f;
#pragma unroll
        for (int i = 0; i < C::FM; ++i) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm * C::TM + i * 32 + 8 * (v >> 2) +
                                4 * half + (v & 3);
                if (col_ok && row < g.M) {
                    float x = acc[i][j][v];
                    if (g.scale_a) x *= g.scale_a[row];
                    x *= sb;
                    int64_t off = (int64_t)row * g.ldc + col;
                    if constexpr (C::CBF16)
                        static_cast<uint16_t *>(g.c)[off] = f32_to_bf16_bits(x);
                    else
                        static_cast<float *>(g.c)[off] = x;
                    if (g.wcount)
                        atomicAdd(&g.wcount[(int64_t)row * g.N + col], 1);
                }
            }
        }
    }
}

// The body of one owned sub-tensor: zero accumulator, K loop, store.
template <class C>
__device__ __forceinline__ void run_tile(const GemmArgs &g, int tm, int tn,
                                         char *smem) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int m0 = tm * C::BM, n0 = tn * C::BN;

    f32x16 acc[C::FM][C::FN];
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    const int nk_full = g.K / C::BK;
    const int nk = nk_full + (g.K % C::BK != 0);
    Tile<C> t;
    if (nk > 0) {
        if (nk_full > 0)
            t.template load<false>(g, m0, n0, 0, tid);
        else
            t.template load<true>(g, m0, n0, 0, tid);
        t.store(smem, tid);
        __syncthreads();
    }
    for (int kt = 0; kt < nk; ++kt) {
        const int nxt = kt + 1;
        if (nxt < nk_full)
            t.template load<false>(g, m0, n0, nxt * C::BK, tid);
        else if (nxt < nk)
            t.template load<true>(g, m0, n0, nxt * C::BK, tid);
        compute_stage<C>(smem + (kt & 1) * C::STAGE, wm, wn, lane, acc);
        if (nxt < nk) t.store(smem + (nxt & 1) * C::STAGE, tid);
        __syncthreads();
    }
    epilogue<C>(g, m0, n0, wm, wn, lane, acc);
}

template <class C>
__global__ __launch_bounds__(C::THREADS) void gemm_tiled_kernel(GemmArgs g) {
    extern __shared__ __align__(16) char smem[];
    const int G = g.s.n_prog;
    for (int t = program_slot(blockIdx.x, G); t < g.s.n_tiles; t += G) {
        int tm, tn;
        tile_coords(t, g.s, tm, tn);
        run_tile<C>(g, tm, tn, smem);
    }
}

// Grouped launch: programs walk the concatenated sub-tensor lists of all
// problems of the table (binary search on the tile prefix sums).
template <class C>
__global__ __launch_bounds__(C::THREADS) void gemm_grouped_kernel(
    const GroupProblem *__restrict__ tab, int n, int total, int G) {
    extern __shared__ __align__(16) char smem[];
    for (int t = program_slot(blockIdx.x, G); t < total; t += G) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (tab[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
        }
        const GroupProblem &pb = tab[lo];
        GemmArgs g;
        g.a = pb.a; g.b = pb.b; g.c = pb.c;
        g.scale_a = nullptr; g.scale_b = nullptr; g.wcount = nullptr;
        g.lda = pb.lda; g.ldb = pb.ldb; g.ldc = pb.ldc;
        g.M = pb.M; g.N = pb.N; g.K = pb.K;
        g.s.tiles_m = pb.tiles_m; g.s.tiles_n = pb.tiles_n;
        g.s.n_tiles = pb.tiles_m * pb.tiles_n; g.s.n_prog = G;
        g.s.group_m = 8;
        int tm, tn;
        tile_coords(t - pb.tile_begin, g.s, tm, tn);
        run_tile<C>(g, tm, tn, smem);
    }
}

struct VariantEntry {
    TiledVariant v;
    const void *kernel;
    const void *grouped;
    int threads;
    int smem;
};

template <class C>
VariantEntry make_entry() {
    VariantEntry e;
    e.v.dtype = C::DTYPE;
    e.v.bm = C::BM; e.v.bn = C::BN; e.v.bk = C::BK;
    e.v.wm = C::WM; e.v.wn = C::WN;
    e.v.b_nk = C::BNK; e.v.c_bf16 = C::CBF16;
    e.kernel = reinterpret_cast<const void *>(&gemm_tiled_kernel<C>);
    e.grouped = reinterpret_cast<const void *>(&gemm_grouped_kernel<C>);
    e.threads = C::THREADS;
    e.smem = 2 * C::STAGE;
    return e;
}

#define TG_VARIANTS_FOR(DT, BM, BN, WM, WN)                      \
    make_entry<Cfg<DT, BM, BN, WM, WN, false, false>>(),        \
        make_entry<Cfg<DT, BM, BN, WM, WN, false, true>>(),     \
        make_entry<Cfg<DT, BM, BN, WM, WN, true, false>>(),     \
        make_entry<Cfg<DT, BM, BN, WM, WN, true, true>>()

#define TG_VARIANTS_NK(DT, BM, BN, WM, WN)                       \
    make_entry<Cfg<DT, BM, BN, WM, WN, true, false>>(),         \
        make_entry<Cfg<DT, BM, BN, WM, WN, true, true>>()

const VariantEntry *table(int *count) {
    static const VariantEntry entries[] = {
        TG_VARIANTS_FOR(TG_BF16, 256, 256, 2, 2),
        TG_VARIANTS_FOR(TG_BF16, 128, 128, 2, 2),
        TG_VARIANTS_FOR(TG_BF16, 64, 64, 2, 2),
        TG_VARIANTS_FOR(TG_BF16, 32, 32, 1, 1),
        TG_VARIANTS_FOR(TG_F32, 128, 128, 2, 2),
        TG_VARIANTS_FOR(TG_F32, 64, 64, 2, 2),
        TG_VARIANTS_FOR(TG_F32, 32, 32, 1, 1),
        TG_VARIANTS_NK(TG_FP8_E4M3, 256, 256, 2, 2),
        TG_VARIANTS_NK(TG_FP8_E4M3, 128, 128, 2, 2),
        TG_VARIANTS_NK(TG_FP8_E4M3, 64, 64, 2, 2),
        TG_VARIANTS_NK(TG_FP8_E4M3, 32, 32, 1, 1),
    };
    *count = (int)(sizeof(entries) / sizeof(entries[0]));
    return entries;
}

}  // namespace

int tiled_variant_count() {
    int n;
    table(&n);
    return n;
}

const TiledVariant &tiled_variant(int i) {
    int n;
    return table(&n)[i].v;
}

static hipError_t prepare_smem(const VariantEntry &e) {
    // LDS beyond the 64 KiB default is requested once per kernel.
    static std::atomic<int> done[128];
    int n;
    const VariantEntry *base = table(&n);
    int idx = (int)(&e - base);
    if (idx >= 0 && idx < 128 && done[idx].load(std::memory_order_acquire))
        return hipSuccess;
    hipError_t err = hipFuncSetAttribute(
        e.kernel, hipFuncAttributeMaxDynamicSharedMemorySize, e.smem);
    if (err == hipSuccess)
        err = hipFuncSetAttribute(
            e.grouped, hipFuncAttributeMaxDynamicSharedMemorySize, e.smem);
    if (err == hipSuccess && idx >= 0 && idx < 128)
        done[idx].store(1, std::memory_order_release);
    return err;
}

hipError_t launch_tiled(int variant, const GemmArgs &args, hipStream_t st) {
    int n;
    const VariantEntry &e = table(&n)[variant];
    hipError_t err = prepare_smem(e);
    if (err != hipSuccess) return err;
    void *params[] = {const_cast<GemmArgs *>(&args)};
    return hipLaunchKernel(e.kernel, dim3(args.s.n_prog), dim3(e.threads),
                           params, e.smem, st);
}

hipError_t launch_grouped(int variant, const GroupHeader *hdr,
                          const void *table_dev, hipStream_t st) {
    int n;
    const VariantEntry &e = table(&n)[variant];
    hipError_t err = prepare_smem(e);
    if (err != hipSuccess) return err;
    const GroupProblem *tab = static_cast<const GroupProblem *>(table_dev);
    int np = hdr->n, total = hdr->total_tiles, G = hdr->n_prog;
    void *params[] = {&tab, &np, &total, &G};
    return hipLaunchKernel(e.grouped, dim3(G), dim3(e.threads), params,
                           e.smem, st);
}

int tiled_occupancy(int variant) {
    int n;
    const VariantEntry &e = table(&n)[variant];
    int blocks = 0;
    if (prepare_smem(e) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, e.kernel, e.threads, e.smem) != hipSuccess ||
        blocks < 1)
        return 1;
    return blocks;
}

}  // namespace tg
