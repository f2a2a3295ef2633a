// gemm_tiled.hip -- persistent tile programs for C = A . B on gfx950 MFMA.
//
// One workgroup is one tile program of the mapped-partition schedule
// (Sec. 3.6 of the paper): it owns the output sub-tensors
// program_slot(p) + r*G of the traversal order, and for each of them
//   acc = 0; for every K tile: acc += A[BM x BK] . B[BK x BN]; store acc
// into its own BM x BN sub-tensor only.  A and B are read-only.
//
// gfx950 design:
//   * every K tile is RBY = 128 or 64 bytes deep per row (bf16: 64 or 32
//     elements, e4m3: 128 or 64, f32: 32);
//   * k-contiguous operands (A, and B stored N x K) live in LDS as
//     [rows][128 B] with the 16-byte chunk index XOR-swizzled per row so
//     that the 16-byte fragment reads are free of bank conflicts;
//   * bf16 and e4m3 tiles move from HBM to LDS with direct buffer->LDS
//     loads (no staging registers, no LDS write instructions): lane l of a
//     wavefront writes LDS bytes [16 l, 16 l + 16) of a 1 KiB block, so each
//     lane fetches the global chunk that the swizzle assigns to that
//     position; one buffer descriptor per operand and K tile, offsets past
//     its end (rows beyond M or N, K beyond the tail) load zeros;
//   * a bf16 B stored K x N stays k-major in LDS ([BK][BN], chunk index
//     XOR-swizzled by k & 3) and is read with the transposing LDS read,
//     which hands each lane four consecutive k of one column;
//   * a ring of NS = 2 or 4 LDS stages: the loads of the next NS - 1 K tiles
//     are in flight while the MFMAs consume the current one (the HBM/L2
//     latency under full load is about the time of one 64-deep step, so the
//     deeper ring with 32-deep tiles keeps the matrix cores fed); one barrier
//     per K tile; the first K tiles of the program's next sub-tensor are
//     fetched while the current one is stored;
//   * f32 tiles go through registers (B stored K x N transposed 4 x 4 in
//     registers), pipelined the same way;
//   * in the f32 register path rows of A beyond M and columns of B beyond N
//     are clamped to valid addresses (their products only reach outputs that
//     are never stored) and the K tail is zero-filled.
#include <atomic>

#include "tg_device.hpp"
#include "tg_internal.hpp"

namespace tg {
namespace {

typedef __attribute__((address_space(3))) void lds_void;
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

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

template <int DT, int BM_, int BN_, int WM_, int WN_, bool BNK_, bool CBF16_,
          int RBY_ = 128, int NS_ = 2, int SCH_ = TG_SCHED_LOCKSTEP>
struct Cfg {
    static constexpr int DTYPE = DT;
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
    static constexpr bool BNK = BNK_, CBF16 = CBF16_;
    static constexpr int ES = DtypeTraits<DT>::ES;
    static constexpr int EPC = 16 / ES;         // elements per 16-byte chunk
    static constexpr int RBY = RBY_;            // bytes of K per operand row
    static constexpr int NS = NS_;              // LDS stages in the ring
    static constexpr int SCHED = SCH_;          // wavefront schedule
    static constexpr bool PP = SCH_ == TG_SCHED_PINGPONG;
    static constexpr bool XT =
        SCH_ == TG_SCHED_CROSS || SCH_ == TG_SCHED_CROSS_WARM;
    // cross-tile schedule with an L2 warm-up of later K tiles
    static constexpr bool WARM = SCH_ == TG_SCHED_CROSS_WARM;
    static constexpr bool STG = SCH_ == TG_SCHED_STAGED;
    static constexpr bool BLK = SCH_ == TG_SCHED_BULK;
    static constexpr int BK = RBY / ES;         // K elements per K tile
    static constexpr int CPRW = RBY / 16;       // 16-byte chunks per row
    static constexpr int RPK = 1024 / RBY;      // rows per 1 KiB block
    static constexpr int NW = WM * WN;          // wavefronts
    static constexpr int THREADS = NW * 64;
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int FM = TM / 32, FN = TN / 32;
    static constexpr bool DIRECT = ES <= 2;     // direct buffer->LDS loads
    static constexpr bool B_KMAJOR = !BNK && ES == 2;  // [BK][BN] in LDS
    static constexpr int RB = BN * ES;          // bytes per k-major B row
    static constexpr int CPR = RB / 16;         // chunks per k-major B row
    static constexpr int A_CH = BM * 8 / THREADS;   // f32 path: A chunks
    static constexpr int B_CH = BN * 8 / THREADS;   // f32 path: B chunks
    // f32 B stored K x N: EPC x EPC blocks, (BK / EPC) * (BN / EPC) of them
    static constexpr int B_BLK = (BK / EPC) * (BN / EPC);
    static constexpr int B_BLK_PT = (B_BLK + THREADS - 1) / THREADS;
    static constexpr int STAGE = (BM + BN) * RBY;   // bytes per LDS stage
    // Per-row and per-column scales of an owned sub-tensor live in LDS next
    // to the stages, one slot per sub-tensor in flight (NS + 1 slots: the
    // loads run at most NS - 1 K tiles, hence sub-tensors, ahead).
    static constexpr int SCALE_SLOT = (BM + BN) * 4;
    static constexpr int NSLOT = NS + 1;
    static constexpr int SMEM =
        (XT && NS == 3 ? 5 * (STAGE / 2) : NS * STAGE) +
        (WARM ? 256 : 0) +
        (DIRECT && !XT && SCH_ != TG_SCHED_STAGED &&
                 SCH_ != TG_SCHED_BULK
             ? NSLOT * SCALE_SLOT
             : 0);
    static constexpr int LPW = STAGE / 1024 / NW;   // 1 KiB loads per wave
    static_assert(TM % 32 == 0 && TN % 32 == 0, "wave tile");
    static_assert(RBY == 128 || RBY == 64, "K-tile row bytes");
    static_assert(NS == 2 || NS == 4 ||
                      (NS == 5 && XT && !WARM && RBY == 64) ||
                      (NS == 5 && SCH_ == TG_SCHED_BULK) ||
                      (NS == 3 && XT && !WARM && RBY == 128 &&
                       BM == BN),
                  "ring of 2 or 4 stages, 5 of 64-byte rows, or 5 operand "
                  "halves (NS = 3)");
    // NS = 3 with the cross-tile schedule: the LDS holds five operand
    // tiles (A or B of one K tile each) instead of three whole stages.
    static constexpr bool HALVES = XT && NS == 3;
    static_assert(DIRECT || (RBY == 128 && NS == 2), "f32 register path");
    static_assert((BM / RPK) % NW == 0, "A 1 KiB blocks per wave");
    static_assert(B_KMAJOR ? (BK * RB / 1024) % NW == 0
                           : (BN / RPK) % NW == 0, "B 1 KiB blocks per wave");
    static_assert(DIRECT || ((BM * 8) % THREADS == 0 &&
                             (BN * 8) % THREADS == 0), "f32 chunk split");
    static_assert(BNK || DT != TG_FP8_E4M3, "e4m3 B must be stored N x K");
    static_assert(!B_KMAJOR || CPR >= 4, "k-major B rows of >= 64 bytes");
    static_assert(DT != TG_FP8_E4M3 || BK >= 64, "e4m3 K tile >= 64");
    static_assert(LPW * (NS - 1) < 64, "vmcnt range");
    // Wavefronts per SIMD when LDS limits the workgroups per CU (160 KiB):
    // the register budget and scheduling target of the compiler.  Without
    // it the scheduler aims at a higher occupancy than LDS allows and
    // trades the fragment double buffer for fewer registers.
    static constexpr int WG_PER_CU_ = 163840 / SMEM;
    static constexpr int WPE_ = WG_PER_CU_ * NW / 4;
    static constexpr int WPE_MAX_ = DIRECT ? 4 : 2;  // f32: register staging
    static constexpr int WPE = WPE_ < 1 ? 1 : (WPE_ > WPE_MAX_ ? WPE_MAX_ : WPE_);
    static_assert(!PP || (DIRECT && WM == 2 && NW == 8 && NS >= 3),
                  "ping-pong: two groups of four wavefronts, >= 3 stages");
    static_assert(!XT || (DIRECT && DT == TG_BF16 && (BK / 16) % 2 == 0),
                  "cross-tile schedule: bf16, even number of K steps");
    static_assert(!WARM || (NS == 2 && BNK && DT == TG_BF16),
                  "L2 warm-up: two-stage cross-tile ring, B stored N x K");
    static_assert(!BLK || (DT == TG_BF16 && BNK && NS >= 4 &&
                           BK / 16 * (FM + FN) * 4 <= 128),
                  "bulk schedule: bf16, B stored N x K, a ring of at least "
                  "four stages, one K tile of fragments in 64 registers");
    static_assert(!STG || (DT == TG_BF16 && BNK && RBY == 128 && NS == 2),
                  "staged schedule: bf16, B stored N x K, 64-deep K tiles, "
                  "two LDS stages");
};

// Row-major [rows][RBY bytes] operand stage: chunk c of row r sits at chunk
// position c ^ f(r), with f(r) = (r >> 1) & 7 for 128-byte rows and
// ((r >> 1) ^ (r >> 3)) & 3 for 64-byte rows.  Any 16 consecutive rows read
// at one logical chunk then cover 16 distinct 16-byte bank groups of a
// 256-byte bank window (and any 8 of them 8 groups of a 128-byte window), so
// the 16-byte fragment reads are conflict-free.  f is unchanged by a shift
// of 32 rows, so the fragments of one K step, 32 rows apart, sit at one lane
// offset plus constants.
template <class C>
__device__ __forceinline__ int swz_f(int row) {
    if constexpr (C::RBY == 128)
        return (row >> 1) & 7;
    else
        return ((row >> 1) ^ (row >> 3)) & 3;
}
template <class C>
__device__ __forceinline__ int swz(int row, int chunk) {
    return row * C::RBY + ((chunk ^ swz_f<C>(row)) << 4);
}

// Chunk permutation of k-major B rows, by k & 3: the four rows of a 16-lane
// transposing read (and of two such groups read together) land in distinct
// 16-byte bank groups.
template <class C>
__device__ __forceinline__ int swz_kmajor(int k) {
    if constexpr (C::CPR >= 16) {
        constexpr uint32_t tab = 0u | (4u << 8) | (10u << 16) | (14u << 24);
        return (tab >> (8 * (k & 3))) & 0xff;
    } else if constexpr (C::CPR == 8) {
        return 2 * (k & 3);
    } else {
        return 2 * (k & 1);
    }
}

// Vector-memory counter waits, as s_waitcnt instructions the compiler sees
// (its own wait insertion then knows which loads are complete).  Encoding:
// vmcnt in bits [3:0] and [15:14], expcnt [6:4] and lgkmcnt [11:8] at their
// no-wait maxima.
template <int N>
__device__ __forceinline__ void wait_vmem_le() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) |
                               (15 << 8));
}

__device__ __forceinline__ void wait_vmem() { wait_vmem_le<0>(); }

// Workgroup barrier for the K-tile ring.  __syncthreads() carries a
// workgroup-scope fence, which waits for every outstanding global access of
// the wavefront, including the loads of later K tiles that must stay in
// flight.  The ring needs less: this wavefront's LDS reads are complete (so
// a stage may be overwritten after the barrier) and the loads of the tile
// about to be read have landed (waited for by the caller).
__device__ __forceinline__ void ring_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One owned sub-tensor as the kernels see it.
struct Job {
    const char *a;
    const char *b;
    void *c;
    const float *scale_a;
    const float *scale_b;
    int32_t *wcount;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t m0, n0;
    // Load streams of the sub-tensor, fixed for all its K tiles: first
    // byte of its A rows (and of its B rows, or of its B columns in row 0
    // for B stored K x N) and the bytes from there to the operand's end.
    const char *a_row, *b_row;
    int64_t a_rem, b_rem;
};

// ------------------------------------------------------------ tile loads

// Buffer resource of `bytes` bytes at `base` (raw buffer, no stride).
// Lanes whose offset is at or beyond `bytes` read zeros; the direct load
// then writes those zeros into LDS.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base,
                                                           uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base),
                                             (short)0, (int)bytes,
                                             0x00020000);
}

constexpr uint32_t kOutOfRange = 0x80000000u;

// Direct loads are issued from inline assembly.  The compiler's own
// dependency tracking would place waits on the vector-memory counter in
// front of LDS reads it cannot prove disjoint from a load's LDS
// destination, which drains the loads that must stay in flight; the K-tile
// schedules here order every LDS access explicitly instead (counter waits
// before workgroup barriers).
//
// Descriptor words of a raw buffer (no stride) in scalar registers.
__device__ __forceinline__ i32x4 make_srd(const void *base, uint32_t bytes) {
    const uint64_t p = reinterpret_cast<uint64_t>(base);
    i32x4 d;
    d[0] = __builtin_amdgcn_readfirstlane((int)(uint32_t)p);
    d[1] = __builtin_amdgcn_readfirstlane((int)((uint32_t)(p >> 32) & 0xffffu));
    d[2] = __builtin_amdgcn_readfirstlane((int)bytes);
    d[3] = 0x00020000;
    return d;
}

// LDS address of a generic pointer into the workgroup's LDS: its low 32
// bits (the shared aperture occupies the high half of the flat address).
// Taken directly rather than through an address-space cast, which would
// add a null-pointer test to every load.
__device__ __forceinline__ uint32_t lds_addr(const char *p) {
    return __builtin_amdgcn_readfirstlane(
        (int)static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p)));
}

// One 16-byte-per-lane load from buffer `srd` at byte offset `voff` into
// LDS at dst + 16 * lane.  M0 holds the LDS address; one wait state
// separates its write from the load.  The first load after `srd` was
// formed also waits five states, the distance a vector-ALU write of a
// scalar register needs before a vector-memory instruction reads it.
template <bool FIRST>
__device__ __forceinline__ void dma16(const i32x4 &srd, char *dst,
                                      uint32_t voff) {
    const uint32_t lds = lds_addr(dst);
    if constexpr (FIRST)
        asm volatile(
            "s_nop 4\n\ts_mov_b32 m0, %0\n\ts_nop 0\n\t"
            "buffer_load_dwordx4 %1, %2, 0 offen lds"
            :
            : "s"(lds), "v"(voff), "s"(srd)
            : "memory", "m0");
    else
        asm volatile(
            "s_mov_b32 m0, %0\n\ts_nop 0\n\t"
            "buffer_load_dwordx4 %1, %2, 0 offen lds"
            :
            : "s"(lds), "v"(voff), "s"(srd)
            : "memory", "m0");
}

// One 4-byte-per-lane load into LDS at dst + 4 * lane (same protocol as
// dma16).
__device__ __forceinline__ void dma4(const i32x4 &srd, char *dst,
                                     uint32_t voff) {
    const uint32_t lds = lds_addr(dst);
    asm volatile(
        "s_nop 4\n\ts_mov_b32 m0, %0\n\ts_nop 0\n\t"
        "buffer_load_dword %1, %2, 0 offen lds"
        :
        : "s"(lds), "v"(voff), "s"(srd)
        : "memory", "m0");
}

__device__ __forceinline__ uint32_t sat_bytes(int64_t b) {
    return b <= 0 ? 0u : (b >= 0x7fffffff ? 0x7fffffffu : (uint32_t)b);
}

template <class C>
__device__ __forceinline__ void set_streams(Job &j) {
    j.a_row = j.a + (int64_t)j.m0 * j.lda * C::ES;
    j.a_rem = (int64_t)(j.M - j.m0) * j.lda * C::ES;
    if constexpr (C::B_KMAJOR) {
        j.b_row = j.b + (int64_t)j.n0 * C::ES;
        j.b_rem = ((int64_t)j.K * j.ldb - j.n0) * C::ES;
    } else {
        j.b_row = j.b + (int64_t)j.n0 * j.ldb * C::ES;
        j.b_rem = (int64_t)(j.N - j.n0) * j.ldb * C::ES;
    }
}

// Direct HBM -> LDS issue of K tile k0 of one owned sub-tensor.  Each lane
// fetches the 16-byte chunk that the LDS swizzle places at its position:
// lane l of the 1 KiB block rb writes row rb * RPK + l / CPRW at chunk
// position l % CPRW, which holds logical chunk (l % CPRW) ^ f(row).  Rows
// beyond M / N and chunks not wholly inside K read as zeros (out-of-range
// buffer offsets); a chunk straddling K is filled by fill_k_tail.
template <class C, int ROWS>
__device__ __forceinline__ void issue_operand(const char *row0, int64_t rem,
                                              int64_t ld, int k0, int K,
                                              char *dst, int wave, int lane) {
    const int64_t skip = (int64_t)k0 * C::ES;
    const i32x4 srd = make_srd(row0 + skip, sat_bytes(rem - skip));
    const int rsub = lane / C::CPRW, p = lane % C::CPRW;
#pragma unroll
    for (int i = 0; i < ROWS / C::RPK / C::NW; ++i) {
        const int rb = i * C::NW + wave;
        const int row = rb * C::RPK + rsub;           // row within the tile
        const int kc = p ^ swz_f<C>(row);
        const bool kin = k0 + (kc + 1) * C::EPC <= K;
        const uint32_t off = kin ? (uint32_t)((row * ld + kc * C::EPC) * C::ES)
                                 : kOutOfRange;
        if (i == 0)
            dma16<true>(srd, dst + rb * 1024, off);
        else
            dma16<false>(srd, dst + rb * 1024, off);
    }
}

// The A tile of K tile k0 into As.
template <class C>
__device__ __forceinline__ void issue_a(const Job &j, char *As, int k0,
                                        int wave, int lane) {
    issue_operand<C, C::BM>(j.a_row, j.a_rem, j.lda, k0, j.K, As, wave,
                            lane);
}

// The B tile of K tile k0 into Bs.
template <class C>
__device__ __forceinline__ void issue_b(const Job &j, char *Bs, int k0,
                                        int wave, int lane) {
    if constexpr (!C::B_KMAJOR) {
        issue_operand<C, C::BN>(j.b_row, j.b_rem, j.ldb, k0, j.K, Bs,
                                wave, lane);
    } else {
        // k-major B: descriptor from (k0, n0); rows k >= K are past its end,
        // columns >= N are masked per lane
        const int64_t skip = (int64_t)k0 * j.ldb * C::ES;
        const i32x4 srd = make_srd(j.b_row + skip, sat_bytes(j.b_rem - skip));
#pragma unroll
        for (int i = 0; i < C::BK * C::RB / 1024 / C::NW; ++i) {
            const int gi = i * C::NW + wave;
            const int off = gi * 1024 + lane * 16;
            const int k = off / C::RB;
            const int lc = ((off % C::RB) >> 4) ^ swz_kmajor<C>(k);
            const bool nin = j.n0 + lc * C::EPC < j.N;
            const uint32_t voff =
                nin ? (uint32_t)((k * j.ldb + lc * C::EPC) * C::ES)
                    : kOutOfRange;
            if (i == 0)
                dma16<true>(srd, Bs + gi * 1024, voff);
            else
                dma16<false>(srd, Bs + gi * 1024, voff);
        }
    }
}

// parts: bit 0 = the A tile, bit 1 = the B tile, into one stage.
template <class C>
__device__ __forceinline__ void issue_direct(const Job &j, char *stage,
                                             int k0, int wave, int lane,
                                             int parts = 3) {
    if (parts & 1) issue_a<C>(j, stage, k0, wave, lane);
    if (parts & 2) issue_b<C>(j, stage + C::BM * C::RBY, k0, wave, lane);
}

// Scales of one owned sub-tensor into its LDS slot: scale_a[m0 .. m0+BM)
// then scale_b[n0 .. n0+BN), 64 per instruction, instructions dealt out
// over the wavefronts.  Entries beyond M / N load as zeros.
template <class C>
__device__ __forceinline__ void issue_scales(const Job &j, char *slot,
                                             int wave, int lane) {
    constexpr int IA = (C::BM + 63) / 64, IB = (C::BN + 63) / 64;
    if (j.scale_a) {
        const i32x4 srd = make_srd(j.scale_a + j.m0, sat_bytes((int64_t)(j.M - j.m0) * 4));
#pragma unroll
        for (int i = 0; i < IA; ++i)
            if (i % C::NW == wave) {
                const int r = i * 64 + lane;
                dma4(srd, slot + i * 256, r < C::BM ? (uint32_t)(r * 4) : kOutOfRange);
            }
    }
    if (j.scale_b) {
        const i32x4 srd = make_srd(j.scale_b + j.n0, sat_bytes((int64_t)(j.N - j.n0) * 4));
#pragma unroll
        for (int i = 0; i < IB; ++i)
            if ((IA + i) % C::NW == wave) {
                const int c = i * 64 + lane;
                dma4(srd, slot + C::BM * 4 + i * 256,
                     c < C::BN ? (uint32_t)(c * 4) : kOutOfRange);
            }
    }
}

// LDS scale slot of the n-th owned sub-tensor of a program.
template <class C>
__device__ __forceinline__ char *scale_slot(char *smem, int n) {
    return smem + C::NS * C::STAGE + (n % C::NSLOT) * C::SCALE_SLOT;
}

// Register-staged K tile of the f32 path.  load() issues the global reads,
// store() writes LDS.
template <class C>
struct RegTile {
    uint4 ra[C::A_CH];
    static_assert(!C::DIRECT, "register staging is the f32 path");
    uint4 rb[C::BNK ? C::B_CH : C::B_BLK_PT * C::EPC];

    template <bool MASK>
    __device__ __forceinline__ void load(const Job &j, int k0, int tid) {
#pragma unroll
        for (int i = 0; i < C::A_CH; ++i) {
            const int q = i * C::THREADS + tid;
            int row = j.m0 + (q >> 3);
            row = row < j.M ? row : j.M - 1;
            const int k = k0 + (q & 7) * C::EPC;
            if (MASK && k >= j.K)
                ra[i] = uint4{0, 0, 0, 0};
            else
                ra[i] = ld16(j.a + ((int64_t)row * j.lda + k) * C::ES);
        }
        if constexpr (C::BNK) {
#pragma unroll
            for (int i = 0; i < C::B_CH; ++i) {
                const int q = i * C::THREADS + tid;
                int row = j.n0 + (q >> 3);
                row = row < j.N ? row : j.N - 1;
                const int k = k0 + (q & 7) * C::EPC;
                if (MASK && k >= j.K)
                    rb[i] = uint4{0, 0, 0, 0};
                else
                    rb[i] = ld16(j.b + ((int64_t)row * j.ldb + k) * C::ES);
            }
        } else {
            constexpr int NB = C::BN / C::EPC;
#pragma unroll
            for (int i = 0; i < C::B_BLK_PT; ++i) {
                const int blk = i * C::THREADS + tid;
                if (C::B_BLK % C::THREADS != 0 && blk >= C::B_BLK) break;
                const int kb = blk / NB, nb = blk % NB;
                int col = j.n0 + nb * C::EPC;
                col = col < j.N ? col : j.N - C::EPC;
#pragma unroll
                for (int r = 0; r < C::EPC; ++r) {
                    const int k = k0 + kb * C::EPC + r;
                    if (MASK && k >= j.K)
                        rb[i * C::EPC + r] = uint4{0, 0, 0, 0};
                    else
                        rb[i * C::EPC + r] =
                            ld16(j.b + ((int64_t)k * j.ldb + col) * C::ES);
                }
            }
        }
    }

    __device__ __forceinline__ void store(char *stage, int tid) {
        char *As = stage;
        char *Bs = stage + C::BM * C::RBY;
#pragma unroll
        for (int i = 0; i < C::A_CH; ++i) {
            const int q = i * C::THREADS + tid;
            st16(As + swz<C>(q >> 3, q & 7), ra[i]);
        }
        if constexpr (C::BNK) {
#pragma unroll
            for (int i = 0; i < C::B_CH; ++i) {
                const int q = i * C::THREADS + tid;
                st16(Bs + swz<C>(q >> 3, q & 7), rb[i]);
            }
        } else {
            // f32 B stored K x N: 4 x 4 blocks (rows k, columns n) become
            // chunks (n, k .. k+3)
            constexpr int NB = C::BN / C::EPC;
#pragma unroll
            for (int i = 0; i < C::B_BLK_PT; ++i) {
                const int blk = i * C::THREADS + tid;
                if (C::B_BLK % C::THREADS != 0 && blk >= C::B_BLK) break;
                const int kb = blk / NB, nb = blk % NB;
                const uint32_t *w =
                    reinterpret_cast<const uint32_t *>(&rb[i * C::EPC]);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    st16(Bs + swz<C>(nb * 4 + c, kb),
                         uint4{w[0 * 4 + c], w[1 * 4 + c], w[2 * 4 + c],
                               w[3 * 4 + c]});
            }
        }
    }
};

// ---------------------------------------------------------------- compute

// B operand of the 32x32x16 bf16 instruction from a k-major B stage:
// two transposing reads.  In each 16-lane group, lane r names row
// k = kb + r / 4 at columns c0 + 4 (r % 4) .. +3, and lane i of the group
// receives column c0 + i at rows kb .. kb + 3.
template <class C>
__device__ __forceinline__ i32x4 read_b_kmajor(const char *Bs, int kk,
                                               int col0, int lane) {
    const int g = lane >> 4, r = lane & 15;
    const int half = g >> 1, cg = g & 1;
    const int n = col0 + cg * 16 + 4 * (r & 3);
    i32x4 out;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = kk * 16 + half * 8 + q * 4 + (r >> 2);
        const char *p = Bs + k * C::RB +
                        (((n >> 3) ^ swz_kmajor<C>(k)) << 4) + ((n & 7) << 1);
        const s16x4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (lds_s16x4 *)(p));
        const uint32_t v0 = (uint16_t)v[0], v1 = (uint16_t)v[1];
        const uint32_t v2 = (uint16_t)v[2], v3 = (uint16_t)v[3];
        out[2 * q] = (int)(v0 | (v1 << 16));
        out[2 * q + 1] = (int)(v2 | (v3 << 16));
    }
    return out;
}

// hook(kk, KK) runs once per K step kk (after the step's fragment reads are
// issued for bf16 and f32, before them for e4m3); the direct-load programs
// issue the next K tile's loads from it.
template <class C, class Hook>
__device__ __forceinline__ void compute_stage(const char *stage, int wm,
                                              int wn, int lane,
                                              f32x16 (&acc)[C::FM][C::FN],
                                              Hook hook) {
    const char *As = stage;
    const char *Bs = stage + C::BM * C::RBY;
    const int r = lane & 31, half = lane >> 5;
    // Fragment rows are wm * TM + f * 32 + r (A) and wn * TN + f * 32 + r
    // (B): one lane offset per K step, the rest compile-time constants.
    const int sw = swz_f<C>(r);
    const char *Aw = As + wm * C::TM * C::RBY + r * C::RBY;
    const char *Bw = Bs + wn * C::TN * C::RBY + r * C::RBY;
    if constexpr (C::DTYPE == TG_BF16 || C::DTYPE == TG_F32) {
        // fragments of step kk + 1 are read while the MFMAs of step kk run
        i32x4 af[2][C::FM], bfr[2][C::FN];
        auto load = [&](int kk, int s) {
            const int co = ((2 * kk + half) ^ sw) << 4;
#pragma unroll
            for (int f = 0; f < C::FM; ++f)
                af[s][f] = *reinterpret_cast<const i32x4 *>(
                    Aw + f * 32 * C::RBY + co);
#pragma unroll
            for (int f = 0; f < C::FN; ++f) {
                if constexpr (C::B_KMAJOR)
                    bfr[s][f] = read_b_kmajor<C>(Bs, kk, wn * C::TN + f * 32,
                                                 lane);
                else
                    bfr[s][f] = *reinterpret_cast<const i32x4 *>(
                        Bw + f * 32 * C::RBY + co);
            }
        };
        constexpr int KK = C::DTYPE == TG_BF16 ? C::BK / 16 : C::BK / 8;
        load(0, 0);
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            const int s = kk & 1;
            if (kk + 1 < KK) load(kk + 1, s ^ 1);
            hook(kk, KK);
            if constexpr (C::DTYPE == TG_BF16 && C::FM * C::FN >= 8) {
                // interleave the next step's LDS reads with this step's
                // MFMAs: one read after each of the first MFMAs
                constexpr int NR = C::FM + (C::B_KMAJOR ? 2 : 1) * C::FN;
                if (kk + 1 < KK) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < C::FM; ++i)
#pragma unroll
                for (int j = 0; j < C::FN; ++j) {
                    if constexpr (C::DTYPE == TG_BF16) {
                        acc[i][j] = mfma_bf16(af[s][i], bfr[s][j], acc[i][j]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const uint32_t ua = af[s][i][e], ub = bfr[s][j][e];
                            acc[i][j] =
                                mfma_f32(as_f32(ua), as_f32(ub), acc[i][j]);
                        }
                    }
                }
        }
    } else {
#pragma unroll
        for (int kk = 0; kk < C::BK / 64; ++kk) {
            hook(kk, C::BK / 64);   // before this step's fragments are live
            const int c = 4 * kk + 2 * half;
            const int co0 = (c ^ sw) << 4, co1 = ((c + 1) ^ sw) << 4;
            i32x8 af[C::FM], bfr[C::FN];
#pragma unroll
            for (int f = 0; f < C::FM; ++f) {
                i32x4 lo = *reinterpret_cast<const i32x4 *>(Aw + f * 32 * C::RBY + co0);
                i32x4 hi = *reinterpret_cast<const i32x4 *>(Aw + f * 32 * C::RBY + co1);
                af[f] = i32x8{lo[0], lo[1], lo[2], lo[3],
                              hi[0], hi[1], hi[2], hi[3]};
            }
#pragma unroll
            for (int f = 0; f < C::FN; ++f) {
                i32x4 lo = *reinterpret_cast<const i32x4 *>(Bw + f * 32 * C::RBY + co0);
                i32x4 hi = *reinterpret_cast<const i32x4 *>(Bw + f * 32 * C::RBY + co1);
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
// Stores go through a buffer descriptor rooted at the sub-tensor's first
// element with 32-bit offsets; elements outside the output (rows >= M,
// columns >= N) get an out-of-range offset, which the hardware drops.
// `scl`: this sub-tensor's scale slot in LDS (direct-load programs), or
// nullptr to read the scales from global memory.
template <class C>
__device__ __forceinline__ void epilogue(const Job &j, int wm, int wn,
                                         int lane,
                                         f32x16 (&acc)[C::FM][C::FN],
                                         const char *scl) {
    constexpr int OES = C::CBF16 ? 2 : 4;
    // The address arithmetic below is loop-invariant in a persistent
    // program; hidden from the optimiser so that it is formed here, per
    // stored sub-tensor, instead of being hoisted and held in registers
    // across the whole K loop.
    int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)j.ldc);
    int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(j.ldc >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    const int64_t ldc = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    const int col_l = lane & 31, half = lane >> 5;
    const int r0 = wm * C::TM + 4 * half;        // row of v = 0, i = 0
    const int c0 = wn * C::TN + col_l;           // column of jj = 0
    char *base = static_cast<char *>(j.c) +
                 ((int64_t)j.m0 * ldc + j.n0) * OES;
    const __amdgpu_buffer_rsrc_t r = make_rsrc(
        base, sat_bytes(((int64_t)(j.M - j.m0 - 1) * ldc + (j.N - j.n0)) *
                        OES));
    const int rows_left = j.M - j.m0 - r0;       // rows with local index < this
    const int cols_left = j.N - j.n0 - c0;
    // Scales are loaded, and waited for, before any store is issued, and
    // inside the branch that loads them, so that no load of this epilogue
    // is outstanding (or believed outstanding) when the K loop resumes.
    const float *lsa = reinterpret_cast<const float *>(scl);
    const float *lsb = lsa + C::BM;
    float sb[C::FN];
#pragma unroll
    for (int jj = 0; jj < C::FN; ++jj) sb[jj] = 1.0f;
    if (j.scale_b) {
        if (scl) {
#pragma unroll
            for (int jj = 0; jj < C::FN; ++jj) sb[jj] = lsb[c0 + jj * 32];
        } else {
#pragma unroll
            for (int jj = 0; jj < C::FN; ++jj)
                if (jj * 32 < cols_left)
                    sb[jj] = j.scale_b[j.n0 + c0 + jj * 32];
            wait_vmem();
        }
    }
    const uint32_t lane_off = (uint32_t)((r0 * ldc + c0) * OES);
    auto store_rows = [&](int i, const float (&sa)[16]) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int dr = i * 32 + 8 * (v >> 2) + (v & 3);
            const bool row_ok = dr < rows_left;
            const uint32_t roff = lane_off + (uint32_t)(dr * ldc * OES);
#pragma unroll
            for (int jj = 0; jj < C::FN; ++jj) {
                const bool ok = row_ok && jj * 32 < cols_left;
                const uint32_t off = ok ? roff + jj * 32 * OES : kOutOfRange;
                const float x = acc[i][jj][v] * sb[jj] * sa[v];
                if constexpr (C::CBF16)
                    __builtin_amdgcn_raw_buffer_store_b16(
                        (unsigned short)f32_to_bf16_bits(x), r, off, 0, 0);
                else
                    __builtin_amdgcn_raw_buffer_store_b32(
                        __builtin_bit_cast(uint32_t, x), r, off, 0, 0);
            }
        }
    };
    if (!j.scale_a) {
        const float ones[16] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f,
                                1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
#pragma unroll
        for (int i = 0; i < C::FM; ++i) store_rows(i, ones);
    } else {
#pragma unroll
        for (int i = 0; i < C::FM; ++i) {
            float sa[16];
            if (scl) {
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    sa[v] = lsa[r0 + i * 32 + 8 * (v >> 2) + (v & 3)];
            } else {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int dr = i * 32 + 8 * (v >> 2) + (v & 3);
                    sa[v] = dr < rows_left ? j.scale_a[j.m0 + r0 + dr] : 1.0f;
                }
                wait_vmem();
            }
            store_rows(i, sa);
        }
    }
    if (j.wcount) {
        // instrumented launches: one count per stored element
#pragma unroll 1
        for (int i = 0; i < C::FM; ++i)
#pragma unroll 1
            for (int v = 0; v < 16; ++v) {
                const int dr = i * 32 + 8 * (v >> 2) + (v & 3);
                if (dr >= rows_left) continue;
#pragma unroll 1
                for (int jj = 0; jj < C::FN; ++jj)
                    if (jj * 32 < cols_left)
                        atomicAdd(&j.wcount[(int64_t)(j.m0 + r0 + dr) * j.N +
                                            j.n0 + c0 + jj * 32],
                                  1);
            }
    }
}

template <class C>
__device__ __forceinline__ void zero_acc(f32x16 (&acc)[C::FM][C::FN]) {
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
}

// K not a multiple of the 16-byte chunk: the chunk that straddles K was
// loaded as zeros; write its K % EPC valid elements of every row (A, and B
// stored N x K) into LDS one by one.  Called after the stage's loads have
// landed and all wavefronts passed a barrier; a barrier must follow.
template <class C>
__device__ __forceinline__ void fill_k_tail2(const Job &j, char *stage,
                                             char *Bs, int k0, int tid) {
    const int rem = j.K % C::EPC;
    const int kbase = j.K - rem;                  // first element of the chunk
    const int chunk = (kbase - k0) / C::EPC;      // its logical chunk index
    for (int r = tid; r < C::BM; r += C::THREADS) {
        const int row = j.m0 + r;
        char *dst = stage + swz<C>(r, chunk);
        const char *src = j.a + ((int64_t)row * j.lda + kbase) * C::ES;
        for (int e = 0; e < rem; ++e) {
            if constexpr (C::ES == 2)
                reinterpret_cast<uint16_t *>(dst)[e] =
                    row < j.M ? reinterpret_cast<const uint16_t *>(src)[e] : 0;
            else
                reinterpret_cast<uint8_t *>(dst)[e] =
                    row < j.M ? reinterpret_cast<const uint8_t *>(src)[e] : 0;
        }
    }
    if constexpr (!C::B_KMAJOR) {
        for (int r = tid; r < C::BN; r += C::THREADS) {
            const int row = j.n0 + r;
            char *dst = Bs + swz<C>(r, chunk);
            const char *src = j.b + ((int64_t)row * j.ldb + kbase) * C::ES;
            for (int e = 0; e < rem; ++e) {
                if constexpr (C::ES == 2)
                    reinterpret_cast<uint16_t *>(dst)[e] =
                        row < j.N ? reinterpret_cast<const uint16_t *>(src)[e]
                                  : 0;
                else
                    reinterpret_cast<uint8_t *>(dst)[e] =
                        row < j.N ? reinterpret_cast<const uint8_t *>(src)[e]
                                  : 0;
            }
        }
    }
}

template <class C>
__device__ __forceinline__ void fill_k_tail(const Job &j, char *stage, int k0,
                                            int tid) {
    fill_k_tail2<C>(j, stage, stage + C::BM * C::RBY, k0, tid);
}

// ------------------------------------------------------- persistent loops

// Wait until the loads of one K tile have landed while the loads of the
// `later` tiles issued after it (0 <= later <= NS - 2) may still be in
// flight: every wavefront issues the same LPW loads per tile, in tile order.
template <class C>
__device__ __forceinline__ void wait_tile(int later) {
    if constexpr (C::NS >= 4) {
        if (later >= 2) {
            wait_vmem_le<2 * C::LPW>();
            return;
        }
    }
    if constexpr (C::NS >= 3) {
        if (later >= 1) {
            wait_vmem_le<C::LPW>();
            return;
        }
    }
    wait_vmem();
}

// Direct-load programs (bf16, e4m3).  P provides the owned sub-tensors:
// P::n_prog(), P::count(), P::job(t).  The K tiles of all owned sub-tensors
// flow through a ring of NS LDS stages (running index g): tile g lives in
// stage g % NS, and the loads of tiles g+1 .. g+NS-2 are in flight while
// tile g is contracted.
template <class C, class P>
__device__ __forceinline__ void run_direct(const P &prov, char *smem) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int G = prov.n_prog(), total = prov.count();
    int t = program_slot(blockIdx.x, G);
    if (t >= total) return;
    auto stage = [&](int g) { return smem + (g % C::NS) * C::STAGE; };
    auto slot = [&](int n) { return scale_slot<C>(smem, n); };
    Job j = prov.job(t);
    int g = 0, njob = 0;
    {
        const int nk = (j.K + C::BK - 1) / C::BK;
        issue_scales<C>(j, slot(njob), wave, lane);
        for (int s = 0; s < C::NS - 1 && s < nk; ++s)
            issue_direct<C>(j, stage(g + s), s * C::BK, wave, lane);
    }
    f32x16 acc[C::FM][C::FN];
    while (true) {
        const int nk = (j.K + C::BK - 1) / C::BK;
        // the last K tile holds a chunk that straddles K
        const bool ragged = (j.K % C::EPC) != 0;
        zero_acc<C>(acc);
        if (nk == 0) {
            wait_vmem();      // the scales
            ring_barrier();
        }
        for (int kt = 0; kt < nk; ++kt) {
            const int later = nk - 1 - kt < C::NS - 2 ? nk - 1 - kt : C::NS - 2;
            if (kt == 0)
                wait_vmem();   // also covers the previous sub-tensor's stores
            else
                wait_tile<C>(later);
            ring_barrier();
            if (ragged && kt == nk - 1) {
                fill_k_tail<C>(j, stage(g + kt), kt * C::BK, tid);
                __syncthreads();
            }
            // the stage of tile kt - 1 is free: every wavefront passed the
            // barrier above after contracting it.  The loads of tile
            // kt + NS - 1 are issued inside the contraction, the A tile
            // after the first K step's fragment reads and the B tile one
            // step later, so the MFMA pipe is fed while they issue.
            const bool nxt = kt + C::NS - 1 < nk;
            compute_stage<C>(stage(g + kt), wm, wn, lane, acc,
                             [&](int kk, int KK) {
                if (!nxt) return;
                // e4m3 K steps are twice as long: both at the first
                const int parts =
                    C::DTYPE == TG_FP8_E4M3
                        ? (kk == 0 ? 3 : 0)
                        : (kk == 0 ? 1 : 0) | (kk == (KK > 1 ? 1 : 0) ? 2 : 0);
                if (parts)
                    issue_direct<C>(j, stage(g + kt + C::NS - 1),
                                    (kt + C::NS - 1) * C::BK, wave, lane,
                                    parts);
            });
        }
        g += nk;
        // first tiles of the next owned sub-tensor, then store this one; the
        // stages written now are all but the one of the last tile contracted
        t += G;
        const bool more = t < total;
        Job nj;
        if (more) {
            nj = prov.job(t);
            const int nk2 = (nj.K + C::BK - 1) / C::BK;
            issue_scales<C>(nj, slot(njob + 1), wave, lane);
            for (int s = 0; s < C::NS - 1 && s < nk2; ++s)
                issue_direct<C>(nj, stage(g + s), s * C::BK, wave, lane);
        }
        epilogue<C>(j, wm, wn, lane, acc, slot(njob));
        if (!more) break;
        j = nj;
        ++njob;
    }
}

// bf16 fragments of K step kk of a stage: FM A fragments (rows
// wm * TM + f * 32 + lane % 32) and FN B fragments, eight k each.
template <class C>
__device__ __forceinline__ void read_frags2(const char *As, const char *Bs,
                                            int wm, int wn, int lane, int kk,
                                            i32x4 (&af)[C::FM],
                                            i32x4 (&bf)[C::FN]) {
    const int r = lane & 31, half = lane >> 5;
    const int co = ((2 * kk + half) ^ swz_f<C>(r)) << 4;
    const char *Aw = As + wm * C::TM * C::RBY + r * C::RBY + co;
#pragma unroll
    for (int f = 0; f < C::FM; ++f)
        af[f] = *reinterpret_cast<const i32x4 *>(Aw + f * 32 * C::RBY);
#pragma unroll
    for (int f = 0; f < C::FN; ++f) {
        if constexpr (C::B_KMAJOR)
            bf[f] = read_b_kmajor<C>(Bs, kk, wn * C::TN + f * 32, lane);
        else
            bf[f] = *reinterpret_cast<const i32x4 *>(
                Bs + (wn * C::TN + f * 32 + r) * C::RBY + co);
    }
}

template <class C>
__device__ __forceinline__ void read_frags(const char *stage, int wm, int wn,
                                           int lane, int kk,
                                           i32x4 (&af)[C::FM],
                                           i32x4 (&bf)[C::FN]) {
    read_frags2<C>(stage, stage + C::BM * C::RBY, wm, wn, lane, kk, af, bf);
}

// The MFMAs of one K step, with the fragment reads issued just before
// them interleaved one by one (NR of them).
template <class C, int NR>
__device__ __forceinline__ void mfma_step(const i32x4 (&af)[C::FM],
                                          const i32x4 (&bf)[C::FN],
                                          f32x16 (&acc)[C::FM][C::FN]) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < C::FN; ++jj)
            acc[i][jj] = mfma_bf16(af[i], bf[jj], acc[i][jj]);
}


// L2 warm-up of K tile k0 of one owned sub-tensor (B stored N x K): each
// lane touches one 64-byte half of one 128-byte row segment with a 4-byte
// load into a scratch LDS word that nothing reads, so the direct loads
// issued for that tile later hit the XCD's L2.  The traversal map puts an
// 8 x 4 block of sub-tensors on each XCD, so a program touches only the A
// rows whose index is tn mod 4 and the B rows whose index is tm mod 8:
// together the block's programs touch each line once.  Two instructions
// per wavefront.  Where the operands stream from HBM (long K, operands
// larger than the last-level cache) the direct loads of a tile then see
// L2 latency instead of HBM latency; where they already hit the MALL the
// extra requests cost more than they save, so this is a configuration
// of its own.
template <class C>
__device__ __forceinline__ void warm_l2(const Job &j, int k0, char *dummy,
                                        int wave, int lane) {
    constexpr int LA = 2 * (C::BM / 4) / C::NW;    // lanes per wave, A
    constexpr int LB = 2 * (C::BN / 8) / C::NW;    // lanes per wave, B
    static_assert(LA <= 64 && LB <= 64, "warm-up lanes");
    const int pa = (j.n0 / C::BN) & 3, pb = (j.m0 / C::BM) & 7;
    const int64_t skip = (int64_t)k0 * C::ES;
    {
        const i32x4 srd = make_srd(j.a_row + skip, sat_bytes(j.a_rem - skip));
        const int idx = wave * LA + lane;
        const int row = pa + 4 * (idx >> 1);
        const uint32_t off = lane < LA
            ? (uint32_t)(row * j.lda * C::ES + (idx & 1) * 64) : kOutOfRange;
        dma4(srd, dummy, off);
    }
    {
        const i32x4 srd = make_srd(j.b_row + skip, sat_bytes(j.b_rem - skip));
        const int idx = wave * LB + lane;
        const int row = pb + 8 * (idx >> 1);
        const uint32_t off = lane < LB
            ? (uint32_t)(row * j.ldb * C::ES + (idx & 1) * 64) : kOutOfRange;
        dma4(srd, dummy, off);
    }
}

// Cross-tile schedule (bf16).  The barrier that hands over K tile kt + 1
// sits before the last K step of tile kt instead of after it: every
// wavefront has read all of tile kt's fragments by then, so the stage of
// tile kt is free for the loads of tile kt + NS, and the first fragments
// of tile kt + 1 are read while the last MFMAs of tile kt run.  The wait
// for the barrier and the LDS latency of the next tile's first reads are
// thereby covered by MFMA work.  Same ring and load accounting as the
// lock-step loop: tile g in stage g % NS, every wavefront issues LPW loads
// per tile in tile order.
template <class C, class P>
__device__ __forceinline__ void run_direct_xt(const P &prov, char *smem) {
    constexpr int KK = C::BK / 16;                 // K steps per tile (even)
    constexpr int NR = C::FM + (C::B_KMAJOR ? 2 : 1) * C::FN;
    // warm-up distance: tile pend_b + PF is touched when pend_b's B loads
    // are issued, two tile periods before its own direct loads
    constexpr int PF = C::WARM ? 2 : 0;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int G = prov.n_prog(), total = prov.count();
    int t = program_slot(blockIdx.x, G);
    if (t >= total) return;
    auto stage = [&](int g) { return smem + (g % C::NS) * C::STAGE; };
    Job j = prov.job(t);
    int g = 0;
    {
        const int nk = (j.K + C::BK - 1) / C::BK;
        for (int s = 0; s < C::NS - 1 && s < nk; ++s)
            issue_direct<C>(j, stage(g + s), s * C::BK, wave, lane);
    }
    f32x16 acc[C::FM][C::FN];
    i32x4 fa[2][C::FM], fb[2][C::FN];
    while (true) {
        const int nk = (j.K + C::BK - 1) / C::BK;
        const bool ragged = (j.K % C::EPC) != 0;
        zero_acc<C>(acc);
        wait_vmem();          // also covers the previous sub-tensor's stores
        ring_barrier();
        if (nk > 0) {
            if (ragged && nk == 1) {
                fill_k_tail<C>(j, stage(g), 0, tid);
                __syncthreads();
            }
            // the stage of the previous sub-tensor's last tile is free
            if (C::NS - 1 < nk)
                issue_direct<C>(j, stage(g + C::NS - 1),
                                (C::NS - 1) * C::BK, wave, lane);
            read_frags<C>(stage(g), wm, wn, lane, 0, fa[0], fb[0]);
        }
        int pend_b = -1;      // tile whose B loads are still to be issued
        bool pf_out = false;  // warm-up loads issued after the last tile's
        for (int kt = 0; kt < nk; ++kt) {
            char *st = stage(g + kt);
#pragma unroll
            for (int kk = 0; kk < KK - 1; ++kk) {
                const int s = kk & 1;
                read_frags<C>(st, wm, wn, lane, kk + 1, fa[s ^ 1], fb[s ^ 1]);
                mfma_step<C, NR>(fa[s], fb[s], acc);
                if (kk == 0 && pend_b >= 0) {
                    issue_direct<C>(j, stage(g + pend_b), pend_b * C::BK,
                                    wave, lane, 2);
                    if constexpr (PF > 0) {
                        if (pend_b + PF < nk) {
                            warm_l2<C>(j, (pend_b + PF) * C::BK,
                                       smem + C::NS * C::STAGE, wave, lane);
                            pf_out = true;
                        }
                    }
                    pend_b = -1;
                }
            }
            // tile kt + 1 has landed for every wavefront and nobody reads
            // tile kt any more.  After the last tile the barrier and the
            // reads of the (unused) next stage still run, keeping the loop
            // free of a second copy of the MFMAs.
            const int later = nk - 2 - kt < C::NS - 2 ? nk - 2 - kt
                                                      : C::NS - 2;
            // (pinned: the scheduler would otherwise hoist the barrier
            // above the MFMAs of the previous steps)
            __builtin_amdgcn_sched_barrier(0);
            if (PF > 0 && pf_out)
                wait_vmem_le<2>();   // all but the two warm-up loads
            else
                wait_tile<C>(later);
            pf_out = false;
            ring_barrier();
            __builtin_amdgcn_sched_barrier(0);
            if (ragged && kt + 1 == nk - 1) {
                fill_k_tail<C>(j, stage(g + kt + 1), (kt + 1) * C::BK, tid);
                __syncthreads();
            }
            read_frags<C>(stage(g + kt + 1), wm, wn, lane, 0, fa[0], fb[0]);
            mfma_step<C, NR>(fa[1], fb[1], acc);
            if (kt + C::NS < nk) {
                issue_direct<C>(j, st, (kt + C::NS) * C::BK, wave, lane, 1);
                pend_b = kt + C::NS;
            }
        }
        g += nk;
        // first tiles of the next owned sub-tensor into every stage but the
        // one of the last tile contracted, then store this one
        t += G;
        const bool more = t < total;
        Job nj;
        if (more) {
            nj = prov.job(t);
            const int nk2 = (nj.K + C::BK - 1) / C::BK;
            for (int s = 0; s < C::NS - 1 && s < nk2; ++s)
                issue_direct<C>(nj, stage(g + s), s * C::BK, wave, lane);
        }
        epilogue<C>(j, wm, wn, lane, acc, nullptr);
        if (!more) break;
        j = nj;
    }
}

// Cross-tile schedule over a ring of five 32-deep slots (bf16, 64-byte K
// rows; five slots fill the 160 KiB of LDS).  The hand-over barrier comes
// every second slot (a 64-deep unit, four K steps), before the unit's last
// K step as in run_direct_xt.  At a hand-over the two slots of the next
// unit have landed and the slot after them may still be in flight, so half
// of the loads of every unit have two unit periods to land and only the
// other half has one.  Slot q of a sub-tensor (running index g + q) lives
// at position (g + q) % 5; a sub-tensor with an odd number of slots gets
// one more, past K, which loads as zeros.  Per wavefront, slot q is issued
// as one group of LPW loads: slots 0 .. 2 before the sub-tensor's first
// barrier (with the previous sub-tensor's store), slot 2u + 3 after the
// last K step of unit u - 1 and slot 2u + 4 after the first K step of unit
// u, so that the hand-over of unit u waits for all but slot 2u + 4.
template <class C, class P>
__device__ __forceinline__ void run_direct_x5(const P &prov, char *smem) {
    static_assert(C::NS == 5 && C::BK == 32, "five slots of 32 K");
    constexpr int NR = C::FM + (C::B_KMAJOR ? 2 : 1) * C::FN;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int G = prov.n_prog(), total = prov.count();
    int t = program_slot(blockIdx.x, G);
    if (t >= total) return;
    auto slot = [&](int q) { return smem + (q % 5) * C::STAGE; };
    auto nslots = [&](const Job &jb) {
        return (((jb.K + C::BK - 1) / C::BK) + 1) & ~1;
    };
    Job j = prov.job(t);
    int g = 0;
    {
        const int nq = nslots(j);
        for (int q = 0; q < 3 && q < nq; ++q)
            issue_direct<C>(j, slot(g + q), q * C::BK, wave, lane);
    }
    f32x16 acc[C::FM][C::FN];
    i32x4 fa[2][C::FM], fb[2][C::FN];
    while (true) {
        const int nq = nslots(j), nu = nq / 2;
        const bool ragged = (j.K % C::EPC) != 0;
        const int qtail = (j.K + C::BK - 1) / C::BK - 1;  // straddling chunk
        zero_acc<C>(acc);
        wait_vmem();          // also covers the previous sub-tensor's stores
        ring_barrier();
        int pend = -1;        // slot to issue after the next first K step
        if (nu > 0) {
            if (ragged && qtail <= 1) {
                fill_k_tail<C>(j, slot(g + qtail), qtail * C::BK, tid);
                __syncthreads();
            }
            if (3 < nq) issue_direct<C>(j, slot(g + 3), 3 * C::BK, wave, lane);
            if (4 < nq) pend = 4;
            read_frags<C>(slot(g), wm, wn, lane, 0, fa[0], fb[0]);
        }
        for (int u = 0; u < nu; ++u) {
            char *sa = slot(g + 2 * u), *sb = slot(g + 2 * u + 1);
            read_frags<C>(sa, wm, wn, lane, 1, fa[1], fb[1]);
            mfma_step<C, NR>(fa[0], fb[0], acc);
            if (pend >= 0) {
                issue_direct<C>(j, slot(g + pend), pend * C::BK, wave, lane);
                pend = -1;
            }
            read_frags<C>(sb, wm, wn, lane, 0, fa[0], fb[0]);
            mfma_step<C, NR>(fa[1], fb[1], acc);
            read_frags<C>(sb, wm, wn, lane, 1, fa[1], fb[1]);
            mfma_step<C, NR>(fa[0], fb[0], acc);
            // hand-over of unit u + 1 (pinned, as in run_direct_xt); after
            // the last unit it still runs and reads an unused slot
            __builtin_amdgcn_sched_barrier(0);
            if (2 * u + 4 < nq)
                wait_vmem_le<C::LPW>();
            else
                wait_vmem();
            ring_barrier();
            __builtin_amdgcn_sched_barrier(0);
            if (ragged && (qtail >> 1) == u + 1) {
                fill_k_tail<C>(j, slot(g + qtail), qtail * C::BK, tid);
                __syncthreads();
            }
            read_frags<C>(slot(g + 2 * u + 2), wm, wn, lane, 0, fa[0], fb[0]);
            mfma_step<C, NR>(fa[1], fb[1], acc);
            // the positions of unit u are free now
            if (2 * u + 5 < nq)
                issue_direct<C>(j, sa, (2 * u + 5) * C::BK, wave, lane);
            if (2 * u + 6 < nq) pend = 2 * u + 6;
        }
        g += nq;
        // slots 0 .. 2 of the next owned sub-tensor go to the three
        // positions other than those of the last unit, then this one is
        // stored
        t += G;
        const bool more = t < total;
        Job nj;
        if (more) {
            nj = prov.job(t);
            const int nq2 = nslots(nj);
            for (int q = 0; q < 3 && q < nq2; ++q)
                issue_direct<C>(nj, slot(g + q), q * C::BK, wave, lane);
        }
        epilogue<C>(j, wm, wn, lane, acc, nullptr);
        if (!more) break;
        j = nj;
    }
}

// Cross-tile schedule over five operand slots (bf16, 64-deep K tiles,
// BM = BN): each slot holds the A or the B tile of one K tile, so the
// 160 KiB of LDS hold two and a half K tiles.  Operand q of a sub-tensor
// (A of tile t is q = 2t, B is q = 2t + 1; running index g + q) lives in
// slot (g + q) % 5.  At the hand-over of tile kt + 1 (before the last K
// step of tile kt) the slots of tile kt are freed: the B tile of kt + 2
// goes into one right away and the A tile of kt + 3 into the other after
// the next tile's first K step, so that A tiles are in flight for about
// two tile periods and B tiles for about one (two-stage ring: one and a
// bit less).  The hand-over waits for tile kt + 1 while the A tile of
// kt + 2, issued last, may still be in flight.
template <class C, class P>
__device__ __forceinline__ void run_direct_xh(const P &prov, char *smem) {
    static_assert(C::HALVES && C::BM == C::BN, "five operand slots");
    constexpr int KK = C::BK / 16;
    constexpr int NR = C::FM + (C::B_KMAJOR ? 2 : 1) * C::FN;
    constexpr int HALF = C::STAGE / 2;
    constexpr int LPA = C::BM * C::RBY / 1024 / C::NW;  // loads per A tile
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int G = prov.n_prog(), total = prov.count();
    int t = program_slot(blockIdx.x, G);
    if (t >= total) return;
    auto slot = [&](int q) { return smem + (q % 5) * HALF; };
    Job j = prov.job(t);
    int g = 0;
    {
        const int nk = (j.K + C::BK - 1) / C::BK;
        if (nk > 0) {
            issue_a<C>(j, slot(g), 0, wave, lane);
            issue_b<C>(j, slot(g + 1), 0, wave, lane);
        }
        if (nk > 1) issue_a<C>(j, slot(g + 2), C::BK, wave, lane);
    }
    f32x16 acc[C::FM][C::FN];
    i32x4 fa[2][C::FM], fb[2][C::FN];
    while (true) {
        const int nk = (j.K + C::BK - 1) / C::BK;
        const bool ragged = (j.K % C::EPC) != 0;
        zero_acc<C>(acc);
        wait_vmem();          // also covers the previous sub-tensor's stores
        ring_barrier();
        if (nk > 0) {
            if (ragged && nk == 1) {
                fill_k_tail2<C>(j, slot(g), slot(g + 1), 0, tid);
                __syncthreads();
            }
            // the slots of the previous sub-tensor's last tile are free
            if (nk > 1) issue_b<C>(j, slot(g + 3), C::BK, wave, lane);
            read_frags2<C>(slot(g), slot(g + 1), wm, wn, lane, 0, fa[0],
                           fb[0]);
        }
        for (int kt = 0; kt < nk; ++kt) {
            const char *sa = slot(g + 2 * kt), *sb = slot(g + 2 * kt + 1);
#pragma unroll
            for (int kk = 0; kk < KK - 1; ++kk) {
                const int s = kk & 1;
                read_frags2<C>(sa, sb, wm, wn, lane, kk + 1, fa[s ^ 1],
                               fb[s ^ 1]);
                mfma_step<C, NR>(fa[s], fb[s], acc);
                if (kk == 0 && kt + 2 < nk)   // into the slot of B of kt - 1
                    issue_a<C>(j, slot(g + 2 * kt + 4), (kt + 2) * C::BK,
                               wave, lane);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (kt + 2 < nk)
                wait_vmem_le<LPA>();
            else
                wait_vmem();
            ring_barrier();
            __builtin_amdgcn_sched_barrier(0);
            if (ragged && kt + 1 == nk - 1) {
                fill_k_tail2<C>(j, slot(g + 2 * kt + 2), slot(g + 2 * kt + 3),
                                (kt + 1) * C::BK, tid);
                __syncthreads();
            }
            read_frags2<C>(slot(g + 2 * kt + 2), slot(g + 2 * kt + 3), wm, wn,
                           lane, 0, fa[0], fb[0]);
            mfma_step<C, NR>(fa[1], fb[1], acc);
            if (kt + 2 < nk)                  // into the slot of A of kt
                issue_b<C>(j, slot(g + 2 * kt + 5), (kt + 2) * C::BK, wave,
                           lane);
        }
        g += 2 * nk;
        // A and B of the next sub-tensor's first tile and its second A go
        // to the three slots other than those of the last tile, then this
        // one is stored
        t += G;
        const bool more = t < total;
        Job nj;
        if (more) {
            nj = prov.job(t);
            const int nk2 = (nj.K + C::BK - 1) / C::BK;
            if (nk2 > 0) {
                issue_a<C>(nj, slot(g), 0, wave, lane);
                issue_b<C>(nj, slot(g + 1), 0, wave, lane);
            }
            if (nk2 > 1) issue_a<C>(nj, slot(g + 2), C::BK, wave, lane);
        }
        epilogue<C>(j, wm, wn, lane, acc, nullptr);
        if (!more) break;
        j = nj;
    }
}

// Register-staged programs (f32).
template <class C, class P>
__device__ __forceinline__ void run_regs(const P &prov, char *smem) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int G = prov.n_prog(), total = prov.count();
    f32x16 acc[C::FM][C::FN];
    for (int t = program_slot(blockIdx.x, G); t < total; t += G) {
        const Job j = prov.job(t);
        zero_acc<C>(acc);
        const int nk_full = j.K / C::BK;
        const int nk = nk_full + (j.K % C::BK != 0);
        RegTile<C> rt;
        if (nk > 0) {
            if (nk_full > 0)
                rt.template load<false>(j, 0, tid);
            else
                rt.template load<true>(j, 0, tid);
            rt.store(smem, tid);
            __syncthreads();
        }
        for (int kt = 0; kt < nk; ++kt) {
            const int nxt = kt + 1;
            if (nxt < nk_full)
                rt.template load<false>(j, nxt * C::BK, tid);
            else if (nxt < nk)
                rt.template load<true>(j, nxt * C::BK, tid);
            compute_stage<C>(smem + (kt & 1) * C::STAGE, wm, wn, lane, acc,
                             [](int, int) {});
            if (nxt < nk) rt.store(smem + (nxt & 1) * C::STAGE, tid);
            __syncthreads();
        }
        epilogue<C>(j, wm, wn, lane, acc, nullptr);
    }
}

// ------------------------------------------------------ ping-pong schedule
//
// Eight wavefronts in two groups of four (group = wm); the hardware places
// wavefront w on SIMD w % 4, so every SIMD holds one wavefront of each
// group.  The groups run the same sequence of phases, one phase apart:
//   MEM(q):  issue the HBM -> LDS loads of K tile q + NS - 1, then read this
//            wavefront's fragments of K tile q from LDS into registers;
//   COMP(q): the MFMAs of K tile q, from registers only.
// A workgroup barrier separates consecutive phases, so while one group
// contracts, the other group's LDS reads and load issue run on the same
// SIMDs, and the MFMA pipe of each SIMD is fed from one long run of
// independent instructions.  K tiles of consecutive owned sub-tensors form
// one stream q = 0, 1, ...; the loads run NS - 1 tiles ahead.
//
// Ordering (phase k starts at barrier k; group 0 runs MEM(q) in phase 2q
// and COMP(q) in 2q + 1, group 1 one phase later):
//  * tile q is first read in phase 2q: every wavefront waits for its own
//    loads of tile q before barrier 2q (group 0 before MEM(q), group 1
//    before COMP(q - 1));
//  * the loads of tile q + NS - 1 overwrite the stage of tile q - 1, whose
//    last reader (group 1, MEM(q - 1), phase 2q - 1) finished its LDS reads
//    before barrier 2q, the earliest issue of those loads;
//  * both groups pass the same number of barriers: group 1 one extra at the
//    start, group 0 one extra at the end.
template <class C>
struct PPFrag {
    static constexpr bool F8 = C::DTYPE == TG_FP8_E4M3;
    static constexpr int KS = F8 ? C::BK / 64 : C::BK / 16;  // MFMA K steps
    static constexpr int W = F8 ? 2 : 1;                     // i32x4 / operand
    i32x4 a[KS][C::FM][W];
    i32x4 b[KS][C::FN][W];
};

template <class C>
__device__ __forceinline__ void pp_read(const char *stage, int wm, int wn,
                                        int lane, PPFrag<C> &f) {
    const char *As = stage;
    const char *Bs = stage + C::BM * C::RBY;
    const int r = lane & 31, half = lane >> 5;
#pragma unroll
    for (int ks = 0; ks < PPFrag<C>::KS; ++ks) {
        const int c = PPFrag<C>::F8 ? 4 * ks + 2 * half : 2 * ks + half;
#pragma unroll
        for (int i = 0; i < C::FM; ++i)
#pragma unroll
            for (int w = 0; w < PPFrag<C>::W; ++w)
                f.a[ks][i][w] = *reinterpret_cast<const i32x4 *>(
                    As + swz<C>(wm * C::TM + i * 32 + r, c + w));
#pragma unroll
        for (int jj = 0; jj < C::FN; ++jj) {
            if constexpr (C::B_KMAJOR) {
                f.b[ks][jj][0] =
                    read_b_kmajor<C>(Bs, ks, wn * C::TN + jj * 32, lane);
            } else {
#pragma unroll
                for (int w = 0; w < PPFrag<C>::W; ++w)
                    f.b[ks][jj][w] = *reinterpret_cast<const i32x4 *>(
                        Bs + swz<C>(wn * C::TN + jj * 32 + r, c + w));
            }
        }
    }
}

template <class C>
__device__ __forceinline__ void pp_mfma(const PPFrag<C> &f,
                                        f32x16 (&acc)[C::FM][C::FN]) {
#pragma unroll
    for (int ks = 0; ks < PPFrag<C>::KS; ++ks)
#pragma unroll
        for (int i = 0; i < C::FM; ++i)
#pragma unroll
            for (int jj = 0; jj < C::FN; ++jj) {
                if constexpr (PPFrag<C>::F8) {
                    const i32x4 a0 = f.a[ks][i][0], a1 = f.a[ks][i][1];
                    const i32x4 b0 = f.b[ks][jj][0], b1 = f.b[ks][jj][1];
                    acc[i][jj] = mfma_fp8(
                        i32x8{a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2],
                              a1[3]},
                        i32x8{b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2],
                              b1[3]},
                        acc[i][jj]);
                } else {
                    acc[i][jj] = mfma_bf16(f.a[ks][i][0], f.b[ks][jj][0],
                                           acc[i][jj]);
                }
            }
}

// Barrier between two phases: this wavefront's LDS reads are complete, and
// no instruction moves across it.
__device__ __forceinline__ void phase_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    ring_barrier();
    __builtin_amdgcn_sched_barrier(0);
}

// K tiles of one owned sub-tensor in the stream; K = 0 takes one tile of
// zeros (every chunk lies beyond K and loads as zeros).
template <class C>
__device__ __forceinline__ int pp_tiles(int K) {
    const int nk = (K + C::BK - 1) / C::BK;
    return nk > 0 ? nk : 1;
}

// Loads of the K-tile stream in issue order: (owned sub-tensor, K tile).
// A sub-tensor's scales are issued with its first K tile, into the LDS
// slot of its position in the sequence of owned sub-tensors.
template <class C, class P>
struct LoadCursor {
    const P &prov;
    Job j;
    int t, kt, nk, total, G;
    int issued;   // tiles issued so far (stream index of the next one)
    int njob;     // position of j among this program's sub-tensors

    __device__ LoadCursor(const P &p, int t0, int total_, int G_)
        : prov(p), t(t0), kt(0), total(total_), G(G_), issued(0), njob(0) {
        j = prov.job(t);
        nk = pp_tiles<C>(j.K);
    }
    __device__ __forceinline__ void issue(char *smem, int wave, int lane) {
        if (t >= total) return;
        if (kt == 0)
            issue_scales<C>(j, scale_slot<C>(smem, njob), wave, lane);
        issue_direct<C>(j, smem + (issued % C::NS) * C::STAGE, kt * C::BK,
                        wave, lane);
        ++issued;
        if (++kt == nk) {
            kt = 0;
            t += G;
            ++njob;
            if (t < total) {
                j = prov.job(t);
                nk = pp_tiles<C>(j.K);
            }
        }
    }
};

// Wait until this wavefront's loads of stream tile q have landed.  Loads
// complete in issue order; after epilogue stores (dirty) everything is
// drained, since stores need not complete in order with loads.
template <class C>
__device__ __forceinline__ void pp_wait(int q, int issued, bool &dirty) {
    if (q >= issued) return;   // past the end of the stream
    if (dirty) {
        wait_vmem();
        dirty = false;
        return;
    }
    int later = issued - 1 - q;
    later = later < C::NS - 2 ? later : C::NS - 2;
    wait_tile<C>(later);
}

// Ping-pong programs (bf16, e4m3; K a positive multiple of the 16-byte
// chunk, so no tile needs a tail fill).
template <class C, class P>
__device__ __forceinline__ void run_pingpong(const P &prov, char *smem) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int grp = wm;
    const int G = prov.n_prog(), total = prov.count();
    int t = program_slot(blockIdx.x, G);
    if (t >= total) return;
    LoadCursor<C, P> ld(prov, t, total, G);
    for (int s = 0; s < C::NS - 1; ++s) ld.issue(smem, wave, lane);
    Job j = prov.job(t);
    int nk = pp_tiles<C>(j.K);
    int kt = 0, q = 0, njob = 0;
    bool dirty = false;
    f32x16 acc[C::FM][C::FN];
    zero_acc<C>(acc);
    PPFrag<C> f;
    if (grp == 1) {
        pp_wait<C>(0, ld.issued, dirty);
        phase_barrier();
    }
    while (true) {
        // MEM(q)
        if (grp == 0) pp_wait<C>(q, ld.issued, dirty);
        phase_barrier();
        ld.issue(smem, wave, lane);
        pp_read<C>(smem + (q % C::NS) * C::STAGE, wm, wn, lane, f);
        // COMP(q)
        if (grp == 1) pp_wait<C>(q + 1, ld.issued, dirty);
        phase_barrier();
        __builtin_amdgcn_s_setprio(1);
        pp_mfma<C>(f, acc);
        __builtin_amdgcn_s_setprio(0);
        ++q;
        if (++kt == nk) {
            epilogue<C>(j, wm, wn, lane, acc, scale_slot<C>(smem, njob));
            ++njob;
            dirty = true;
            t += G;
            if (t >= total) break;
            j = prov.job(t);
            nk = pp_tiles<C>(j.K);
            kt = 0;
            zero_acc<C>(acc);
        }
    }
    if (grp == 0) phase_barrier();
}


// ------------------------------------------------------- bulk-read ring
//
// Bulk-read schedule (bf16, A and B both k-contiguous).  A K tile's
// fragments are read from LDS into registers all at once, one tile period
// before they are contracted, so its LDS stage is free again as soon as
// every wavefront has read it: with a ring of NS stages the direct loads
// of a tile are issued NS - 1 tile periods before the tile is read (the
// lead time that the HBM and L2 latency under full load asks for), and
// each wavefront holds two tiles of fragments (the one being contracted
// and the next).  Four wavefronts of 128 x 128 outputs, one per SIMD,
// accumulators in the AGPR half of the register file.
//
// The loads run as one stream over the K tiles of all owned sub-tensors
// (tile q of the stream in stage q % NS).  Iteration q, with tile q's
// fragments in registers:
//   wait: this wavefront's reads of tile q are complete and its loads of
//         tile q + 1 have landed; barrier (so for every wavefront);
//   issue the loads of tile q + NS into stage q % NS (tile q's, now free);
//   read tile q + 1's fragments into the other register set, one read
//   slotted after each of the first MFMAs of tile q;
//   after the sub-tensor's last tile, store it and start the next.
// Loads complete in issue order, so waiting until at most the loads of the
// tiles issued after tile q + 1 are outstanding means tile q + 1 has
// landed; epilogue stores in between only make that wait longer.

// One 16-byte-per-lane load into LDS at `lds` + 16 * lane from buffer
// `srd` at byte offset voff + soff (same protocol as dma16; the scalar
// offset carries the distance between a wavefront's 1 KiB blocks).
template <bool FIRST>
__device__ __forceinline__ void dma16_so(const i32x4 &srd, uint32_t lds_,
                                         uint32_t voff, int soff) {
    const uint32_t lds = __builtin_amdgcn_readfirstlane(lds_);
    if constexpr (FIRST)
        asm volatile(
            "s_nop 4\n\ts_mov_b32 m0, %0\n\ts_nop 0\n\t"
            "buffer_load_dwordx4 %1, %2, %3 offen lds"
            :
            : "s"(lds), "v"(voff), "s"(srd), "s"(soff)
            : "memory", "m0");
    else
        asm volatile(
            "s_mov_b32 m0, %0\n\ts_nop 0\n\t"
            "buffer_load_dwordx4 %1, %2, %3 offen lds"
            :
            : "s"(lds), "v"(voff), "s"(srd), "s"(soff)
            : "memory", "m0");
}

// Load stream of one operand of one owned sub-tensor (rows k-contiguous):
// first byte of its rows and the bytes from there to the operand's end,
// the lane's offset within the wavefront's first 1 KiB block (block i of
// the wavefront holds rows i * NW * RPK further down; the swizzle repeats
// every 32 rows, so every block of a lane reads the same logical chunk)
// and the distance between blocks.  K is a whole number of K tiles, so no
// chunk straddles or passes K; rows beyond M / N lie past the buffer's
// end and load zeros.
struct BulkStream {
    const char *row;
    int64_t rem;
    uint32_t voff;
    int32_t stride;
};

template <class C>
__device__ __forceinline__ BulkStream bulk_stream(const char *row0,
                                                  int64_t rem, int64_t ld,
                                                  int wave, int lane) {
    static_assert((C::NW * C::RPK) % 32 == 0, "swizzle period");
    BulkStream s;
    const int row = wave * C::RPK + lane / C::CPRW;
    const int kc = (lane % C::CPRW) ^ swz_f<C>(row);
    s.row = row0;
    s.rem = rem;
    s.voff = (uint32_t)((row * ld + kc * C::EPC) * C::ES);
    s.stride = __builtin_amdgcn_readfirstlane(
        (int)(C::NW * C::RPK * ld * C::ES));
    return s;
}

// This wavefront's ROWS / RPK / NW blocks of one operand of K tile k0.
template <class C, int ROWS>
__device__ __forceinline__ void bulk_issue(const BulkStream &s, int k0,
                                           uint32_t dst, int wave) {
    const int64_t skip = (int64_t)k0 * C::ES;
    const i32x4 srd = make_srd(s.row + skip, sat_bytes(s.rem - skip));
#pragma unroll
    for (int i = 0; i < ROWS / C::RPK / C::NW; ++i) {
        const uint32_t lds = dst + (uint32_t)((i * C::NW + wave) * 1024);
        if (i == 0)
            dma16_so<true>(srd, lds, s.voff, 0);
        else
            dma16_so<false>(srd, lds, s.voff,
                            __builtin_amdgcn_readfirstlane(i * s.stride));
    }
}

// The next K tile of the load stream, ready to issue: buffer resources
// of its A and B rows from its first K column and its LDS stage.
struct BulkTile {
    i32x4 sa, sb;
    uint32_t lds;
    bool live;   // the stream has this tile
};

// Loads of the stream in issue order (owned sub-tensor, K tile).
template <class C, class P>
struct BulkCursor {
    const P &prov;
    BulkStream sa, sb;
    int t, kt, nk, total, G;
    int issued;   // tiles issued so far
    int wave, lane;

    __device__ __forceinline__ void start(int t0) {
        const Job j = prov.job(t0);
        nk = pp_tiles<C>(j.K);
        // K = 0 takes one tile of zeros: an empty buffer range
        const bool k0 = j.K == 0;
        sa = bulk_stream<C>(j.a_row, k0 ? 0 : j.a_rem, j.lda, wave, lane);
        sb = bulk_stream<C>(j.b_row, k0 ? 0 : j.b_rem, j.ldb, wave, lane);
    }
    __device__ BulkCursor(const P &p, int t0, int total_, int G_, int w,
                          int l)
        : prov(p), t(t0), kt(0), total(total_), G(G_), issued(0), wave(w),
          lane(l) {
        start(t0);
    }
    __device__ __forceinline__ BulkTile prepare(char *smem) const {
        BulkTile T;
        T.live = t < total;
        const int64_t skip = (int64_t)kt * C::BK * C::ES;
        T.sa = make_srd(sa.row + skip, sat_bytes(sa.rem - skip));
        T.sb = make_srd(sb.row + skip, sat_bytes(sb.rem - skip));
        T.lds = lds_addr(smem) + (uint32_t)((issued % C::NS) * C::STAGE);
        return T;
    }
    // load r of this wavefront's share of the tile: A blocks first, then B
    __device__ __forceinline__ void load(const BulkTile &T, int r) const {
        constexpr int NA = C::BM / C::RPK / C::NW;
        const bool a = r < NA;
        const int i = a ? r : r - NA;
        const uint32_t lds = T.lds + (a ? 0u : (uint32_t)(C::BM * C::RBY)) +
                             (uint32_t)((i * C::NW + wave) * 1024);
        const BulkStream &st = a ? sa : sb;
        if (i == 0)
            dma16_so<true>(a ? T.sa : T.sb, lds, st.voff, 0);
        else
            dma16_so<false>(a ? T.sa : T.sb, lds, st.voff,
                            __builtin_amdgcn_readfirstlane(i * st.stride));
    }
    __device__ __forceinline__ void advance() {
        ++issued;
        if (++kt == nk) {
            kt = 0;
            t += G;
            if (t < total) start(t);
        }
    }
    __device__ __forceinline__ void issue(char *smem) {
        const BulkTile T = prepare(smem);
        if (!T.live) return;
#pragma unroll
        for (int r = 0; r < C::LPW; ++r) load(T, r);
        advance();
    }
};

template <class C>
struct BulkFrags {
    i32x4 a[C::BK / 16][C::FM];
    i32x4 b[C::BK / 16][C::FN];
};

// Wait until at most the loads of `later` tiles (0 <= later < NS) are
// outstanding.
template <class C>
__device__ __forceinline__ void wait_later(int later) {
    static_assert(C::NS <= 5, "wait table");
    switch (later) {
    case 0: wait_vmem(); break;
    case 1: wait_vmem_le<C::LPW>(); break;
    case 2: wait_vmem_le<2 * C::LPW>(); break;
    case 3: wait_vmem_le<3 * C::LPW>(); break;
    default: wait_vmem_le<(C::NS - 1) * C::LPW>(); break;
    }
}

// Barrier of the bulk-read ring: this wavefront's LDS reads are complete
// (a wait the compiler sees, so that it knows the fragments read before
// are in registers and inserts no waits of its own for them), then the
// workgroup barrier.
__device__ __forceinline__ void bulk_barrier() {
    // lgkmcnt(0); vmcnt and expcnt at their no-wait maxima
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));
    __builtin_amdgcn_s_barrier();
}

// One iteration of the bulk-read ring: contract tile q (fragments in cur)
// and read tile q + 1 into nxt.  The tile's MFMAs are cut into LPW groups;
// one load of tile q + NS leads each group (with one wavefront per SIMD a
// load that waits to issue stalls the MFMAs behind it, so the loads are
// spread over the whole tile period), and the fragment reads of tile
// q + 1 are slotted one after each MFMA of the first groups.
template <class C, class P>
__device__ __forceinline__ void bulk_iter(BulkCursor<C, P> &ld, char *smem,
                                          int q, int wave, int lane, int wm,
                                          int wn, const BulkFrags<C> &cur,
                                          BulkFrags<C> &nxt,
                                          f32x16 (&acc)[C::FM][C::FN]) {
    constexpr int KK = C::BK / 16;
    constexpr int NF = C::FM + C::FN;           // fragments per K step
    constexpr int NRD = KK * NF;                // fragment reads per tile
    constexpr int NM = KK * C::FM * C::FN;      // MFMAs per tile
    constexpr int NG = C::LPW;                  // groups, one load each
    constexpr int MPG = NM / NG;                // MFMAs per group
    static_assert(NM % NG == 0 && NRD % MPG == 0 && NRD / MPG <= NG,
                  "group layout");
    __builtin_amdgcn_sched_barrier(0);
    if (q + 1 < ld.issued) wait_later<C>(ld.issued - q - 2);
    bulk_barrier();
    __builtin_amdgcn_sched_barrier(0);
    const BulkTile T = ld.prepare(smem);
    // (a stale stage is read when tile q + 1 does not exist; unused)
    const char *nst = smem + ((q + 1) % C::NS) * C::STAGE;
    const int r = lane & 31, half = lane >> 5;
    const int sw = swz_f<C>(r);
    const char *Aw = nst + wm * C::TM * C::RBY + r * C::RBY;
    const char *Bw = nst + C::BM * C::RBY + wn * C::TN * C::RBY + r * C::RBY;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        __builtin_amdgcn_sched_barrier(0);
        if (T.live) ld.load(T, g);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int x = g * MPG; x < (g + 1) * MPG; ++x) {
            if (x < NRD) {
                const int kk = x / NF, f = x % NF;
                const int co = ((2 * kk + half) ^ sw) << 4;
                if (f < C::FM)
                    nxt.a[kk][f] = *reinterpret_cast<const i32x4 *>(
                        Aw + f * 32 * C::RBY + co);
                else
                    nxt.b[kk][f - C::FM] = *reinterpret_cast<const i32x4 *>(
                        Bw + (f - C::FM) * 32 * C::RBY + co);
            }
        }
#pragma unroll
        for (int x = g * MPG; x < (g + 1) * MPG; ++x) {
            const int kk = x / (C::FM * C::FN), m = x % (C::FM * C::FN);
            const int i = m / C::FN, jj = m % C::FN;
            acc[i][jj] = mfma_bf16(cur.a[kk][i], cur.b[kk][jj], acc[i][jj]);
        }
#pragma unroll
        for (int x = g * MPG; x < (g + 1) * MPG; ++x) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            if (x < NRD) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (T.live) ld.advance();
}

// Owned sub-tensors one after another; the K tiles of each are taken in
// pairs (register sets fixed at compile time), an odd last tile moves the
// next sub-tensor's first fragments back into set 0.
template <class C, class P>
__device__ __forceinline__ void run_bulk(const P &prov, char *smem) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int G = prov.n_prog(), total = prov.count();
    int t = program_slot(blockIdx.x, G);
    if (t >= total) return;
    BulkCursor<C, P> ld(prov, t, total, G, wave, lane);
    for (int s = 0; s < C::NS; ++s) ld.issue(smem);
    BulkFrags<C> F0, F1;
    wait_later<C>(ld.issued - 1);   // tile 0
    ring_barrier();
#pragma unroll
    for (int kk = 0; kk < C::BK / 16; ++kk)
        read_frags<C>(smem, wm, wn, lane, kk, F0.a[kk], F0.b[kk]);
    f32x16 acc[C::FM][C::FN];
    int q = 0;
    while (true) {
        const Job j = prov.job(t);
        const int nk = pp_tiles<C>(j.K);
        zero_acc<C>(acc);
        int kt = 0;
        for (; kt + 2 <= nk; kt += 2, q += 2) {
            bulk_iter<C, P>(ld, smem, q, wave, lane, wm, wn, F0, F1, acc);
            bulk_iter<C, P>(ld, smem, q + 1, wave, lane, wm, wn, F1, F0,
                            acc);
        }
        if (kt < nk) {
            bulk_iter<C, P>(ld, smem, q, wave, lane, wm, wn, F0, F1, acc);
            ++q;
            F0 = F1;
        }
        epilogue<C>(j, wm, wn, lane, acc, nullptr);
        t += G;
        if (t >= total) break;
    }
}

// ------------------------------------------------- register-staged ring
//
// Staged schedule (bf16, A and B both k-contiguous, 64-deep K tiles): the
// HBM reads of a K tile go into registers, two register sets deep, and
// reach LDS through ordinary 16-byte LDS stores into a ring of two stages.
// With four wavefronts of 128 x 128 outputs (accumulators in the AGPR
// half of the register file) the fragment reads per MFMA are a third
// lower than with eight wavefronts of 128 x 64, and every K tile is read
// from HBM two tile periods before the MFMAs need it: at the start of tile
// kt the registers of tile kt + 1 are stored into the free stage and the
// reads of tile kt + 3 are issued into them, while tile kt + 2 is still in
// flight in the other set.  One barrier per tile, before its last K step
// (as in the cross-tile schedule): by then every wavefront holds the
// tile's last fragments, and tile kt + 1 has been stored.
//
// Register-set indices must be compile-time constants, so tiles are taken
// in pairs.  Each owned sub-tensor starts its own pipeline (the reads of
// its first three tiles are issued after the previous sub-tensor's last
// MFMAs); K must be a whole number of K tiles.  Every tile issues its
// LDS stores and its reads unconditionally (reads past K are out of the
// buffer's range: zeros, no memory access), so that the compiler's
// load-counter bookkeeping sees the same order of outstanding reads on
// every path into the loop and waits only for the older register set.

// This wavefront's share of one K tile in registers: LPW chunks of 16
// bytes per lane, lane l of 1 KiB block rb holding the chunk that belongs
// at byte 16 l of the block (the layout of the direct loads).
template <class C>
struct StagedSet {
    i32x4 v[C::LPW];
};

// Where this wavefront's chunks of one K tile come from: a buffer
// resource per operand (rooted at the tile's first K column, formed in
// scalar registers without branches), one vector offset per operand (block
// i of the wavefront holds rows row + i * NW * RPK; the swizzle does not
// change over multiples of 16 rows, so every block of a lane reads the
// same logical chunk) and the scalar distance between blocks.
struct StagedSrc {
    __amdgpu_buffer_rsrc_t ra, rb;
    uint32_t va, vb;
    int sa, sb;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(
    const char *base, int64_t bytes) {
    const uint64_t p = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    const uint32_t blo = __builtin_amdgcn_readfirstlane((uint32_t)bytes);
    const int32_t bhi = __builtin_amdgcn_readfirstlane((int32_t)(bytes >> 32));
    // clamp to [0, 2^31 - 1]: negative -> 0, at least 2^31 -> 2^31 - 1
    const uint32_t n = bhi < 0 ? 0u
                       : (bhi > 0 || blo > 0x7fffffffu) ? 0x7fffffffu : blo;
    return __builtin_amdgcn_make_buffer_rsrc(
        reinterpret_cast<void *>(((uint64_t)hi << 32) | lo), (short)0,
        (int)n, 0x00020000);
}

template <class C>
__device__ __forceinline__ StagedSrc staged_src(const Job &j, int k0,
                                                int wave, int lane) {
    static_assert((C::NW * C::RPK) % 16 == 0, "swizzle period");
    StagedSrc s;
    const int row = wave * C::RPK + lane / C::CPRW;
    const int kc = (lane % C::CPRW) ^ swz_f<C>(row);
    // tiles past K (the unconditional reads ahead of the last tiles) read
    // an empty buffer: zeros, no memory access
    const int64_t skip = (int64_t)k0 * C::ES;
    const bool live = k0 < j.K;
    s.ra = uniform_rsrc(j.a_row + skip, live ? j.a_rem - skip : 0);
    s.rb = uniform_rsrc(j.b_row + skip, live ? j.b_rem - skip : 0);
    s.va = (uint32_t)((row * j.lda + kc * C::EPC) * C::ES);
    s.vb = (uint32_t)((row * j.ldb + kc * C::EPC) * C::ES);
    s.sa = __builtin_amdgcn_readfirstlane(
        (int)(C::NW * C::RPK * j.lda * C::ES));
    s.sb = __builtin_amdgcn_readfirstlane(
        (int)(C::NW * C::RPK * j.ldb * C::ES));
    return s;
}

// Chunks [LO, HI) of this wavefront's share of a K tile into the register
// set (chunk c < NA is A block c, else B block c - NA).
template <class C, int LO, int HI>
__device__ __forceinline__ void staged_read(const StagedSrc &src,
                                            StagedSet<C> &s) {
    constexpr int NA = C::BM / C::RPK / C::NW;   // A blocks per wavefront
#pragma unroll
    for (int c = LO; c < HI; ++c) {
        if (c < NA)
            s.v[c] = __builtin_bit_cast(
                i32x4, __builtin_amdgcn_raw_buffer_load_b128(
                           src.ra, src.va, c * src.sa, 0));
        else
            s.v[c] = __builtin_bit_cast(
                i32x4, __builtin_amdgcn_raw_buffer_load_b128(
                           src.rb, src.vb, (c - NA) * src.sb, 0));
    }
}

template <class C, int LO, int HI>
__device__ __forceinline__ void staged_write(char *stage, int wave, int lane,
                                             const StagedSet<C> &s) {
    constexpr int NA = C::BM / C::RPK / C::NW;
#pragma unroll
    for (int c = LO; c < HI; ++c) {
        char *base = c < NA ? stage : stage + C::BM * C::RBY;
        const int i = c < NA ? c : c - NA;
        *reinterpret_cast<i32x4 *>(base + (i * C::NW + wave) * 1024 +
                                   lane * 16) = s.v[c];
    }
}

// MFMA slots of a K step that carry one of n evenly spaced instructions.
constexpr uint32_t spread_slots(int n, int slots, int shift) {
    uint32_t m = 0;
    for (int i = 0; i < n; ++i) m |= 1u << ((i * slots / n + shift) % slots);
    return m;
}

// The MFMAs of one K step with, slotted between them, the NREAD fragment
// reads (one after each of the first NREAD MFMAs) and the NWRITE LDS
// stores and NLOAD HBM reads issued just before in program order, spread
// evenly over the step so that the stores do not arrive at the LDS in a
// burst.
template <class C, int NREAD, int NWRITE, int NLOAD>
__device__ __forceinline__ void staged_mfma(const i32x4 (&af)[C::FM],
                                            const i32x4 (&bf)[C::FN],
                                            f32x16 (&acc)[C::FM][C::FN]) {
    constexpr int NM = C::FM * C::FN;
    constexpr uint32_t WS = spread_slots(NWRITE, NM, 0);
    constexpr uint32_t LS = spread_slots(NLOAD, NM, 1);
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if (q < NREAD) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        if ((WS >> q) & 1u) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
        if ((LS >> q) & 1u) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < C::FN; ++jj)
            acc[i][jj] = mfma_bf16(af[i], bf[jj], acc[i][jj]);
}

// One K tile of the staged ring.  Tile kt (stage kt & 1) is contracted;
// set X holds tile kt + 1, which goes into the other stage over the first
// three K steps, each chunk's registers taking the matching chunk of tile
// kt + 3 right after; the other set holds tile kt + 2 (in flight).
template <class C>
__device__ __forceinline__ void staged_tile(
    const Job &j, char *smem, int kt, int nk, int wave, int lane, int wm,
    int wn, StagedSet<C> &X, i32x4 (&fa)[2][C::FM], i32x4 (&fb)[2][C::FN],
    f32x16 (&acc)[C::FM][C::FN]) {
    static_assert(C::BK / 16 == 4 && C::LPW == 16, "four K steps, 16 chunks");
    constexpr int NR = C::FM + C::FN;
    char *st = smem + (kt & 1) * C::STAGE;
    char *nx = smem + ((kt + 1) & 1) * C::STAGE;
    const StagedSrc src = staged_src<C>(j, (kt + 3) * C::BK, wave, lane);
    // one scheduling region per K step, so that each step's interleave
    // pattern takes that step's instructions
    read_frags<C>(st, wm, wn, lane, 1, fa[1], fb[1]);
    staged_write<C, 0, 6>(nx, wave, lane, X);
    staged_read<C, 0, 6>(src, X);
    staged_mfma<C, NR, 6, 6>(fa[0], fb[0], acc);
    __builtin_amdgcn_sched_barrier(0);
    read_frags<C>(st, wm, wn, lane, 2, fa[0], fb[0]);
    staged_write<C, 6, 11>(nx, wave, lane, X);
    staged_read<C, 6, 11>(src, X);
    staged_mfma<C, NR, 5, 5>(fa[1], fb[1], acc);
    __builtin_amdgcn_sched_barrier(0);
    read_frags<C>(st, wm, wn, lane, 3, fa[1], fb[1]);
    staged_write<C, 11, 16>(nx, wave, lane, X);
    staged_read<C, 11, 16>(src, X);
    staged_mfma<C, NR, 5, 5>(fa[0], fb[0], acc);
    // hand-over: tile kt + 1 is stored by every wavefront, nobody reads
    // tile kt any more (its last fragments are in registers)
    __builtin_amdgcn_sched_barrier(0);
    ring_barrier();
    __builtin_amdgcn_sched_barrier(0);
    if (kt + 1 < nk) read_frags<C>(nx, wm, wn, lane, 0, fa[0], fb[0]);
    staged_mfma<C, NR, 0, 0>(fa[1], fb[1], acc);
}

template <class C, class P>
__device__ __forceinline__ void run_staged(const P &prov, char *smem) {
    static_assert(C::BK / 16 % 2 == 0, "even number of K steps");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int G = prov.n_prog(), total = prov.count();
    f32x16 acc[C::FM][C::FN];
    i32x4 fa[2][C::FM], fb[2][C::FN];
    StagedSet<C> S0, S1;
    for (int t = program_slot(blockIdx.x, G); t < total; t += G) {
        const Job j = prov.job(t);
        const int nk = (j.K + C::BK - 1) / C::BK;
        zero_acc<C>(acc);
        if (nk > 0) {
            // pipeline start: tiles 0 and 1 into the sets, tile 0 into
            // stage 0, tile 2 into set 0
            staged_read<C, 0, C::LPW>(staged_src<C>(j, 0, wave, lane), S0);
            staged_read<C, 0, C::LPW>(staged_src<C>(j, C::BK, wave, lane),
                                      S1);
            // the previous sub-tensor's reads of stage 0 ended at its
            // last hand-over barrier
            staged_write<C, 0, C::LPW>(smem, wave, lane, S0);
            staged_read<C, 0, C::LPW>(
                staged_src<C>(j, 2 * C::BK, wave, lane), S0);
            ring_barrier();
            read_frags<C>(smem, wm, wn, lane, 0, fa[0], fb[0]);
            int kt = 0;
            for (; kt + 1 < nk; kt += 2) {
                staged_tile<C>(j, smem, kt, nk, wave, lane, wm, wn, S1, fa,
                               fb, acc);
                staged_tile<C>(j, smem, kt + 1, nk, wave, lane, wm, wn, S0,
                               fa, fb, acc);
            }
            if (kt < nk)
                staged_tile<C>(j, smem, kt, nk, wave, lane, wm, wn, S1, fa,
                               fb, acc);
        }
        epilogue<C>(j, wm, wn, lane, acc, nullptr);
    }
}

// One problem: traversal index -> owned sub-tensor.
template <class C>
struct SingleProvider {
    const GemmArgs &g;
    __device__ int n_prog() const { return g.s.n_prog; }
    __device__ int count() const { return g.s.n_tiles; }
    __device__ Job job(int t) const {
        int tm, tn;
        tile_coords(t, g.s, tm, tn);
        Job j;
        j.a = static_cast<const char *>(g.a);
        j.b = static_cast<const char *>(g.b);
        j.c = g.c;
        // staged programs apply no scales (the host never gives them any),
        // which keeps their epilogue within the register budget
        if constexpr (C::STG) {
            j.scale_a = nullptr; j.scale_b = nullptr;
        } else {
            j.scale_a = g.scale_a; j.scale_b = g.scale_b;
        }
        j.wcount = g.wcount;
        j.lda = g.lda; j.ldb = g.ldb; j.ldc = g.ldc;
        j.M = g.M; j.N = g.N; j.K = g.K;
        j.m0 = tm * C::BM; j.n0 = tn * C::BN;
        set_streams<C>(j);
        return j;
    }
};

// Grouped launch: traversal index -> (problem, owned sub-tensor) by binary
// search on the tile prefix sums of the problem table.
template <class C>
struct GroupProvider {
    const GroupProblem *tab;
    int n, total, G;
    __device__ int n_prog() const { return G; }
    __device__ int count() const { return total; }
    __device__ Job job(int t) const {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
        }
        const GroupProblem &pb = tab[lo];
        Sched s;
        s.tiles_m = pb.tiles_m; s.tiles_n = pb.tiles_n;
        s.n_tiles = pb.tiles_m * pb.tiles_n; s.n_prog = G; s.group_m = 8;
        int tm, tn;
        tile_coords(t - pb.tile_begin, s, tm, tn);
        Job j;
        j.a = static_cast<const char *>(pb.a);
        j.b = static_cast<const char *>(pb.b);
        j.c = pb.c;
        j.scale_a = nullptr; j.scale_b = nullptr; j.wcount = pb.wcount;
        j.lda = pb.lda; j.ldb = pb.ldb; j.ldc = pb.ldc;
        j.M = pb.M; j.N = pb.N; j.K = pb.K;
        j.m0 = tm * C::BM; j.n0 = tn * C::BN;
        set_streams<C>(j);
        return j;
    }
};

template <class C>
__global__ __launch_bounds__(C::THREADS)
__attribute__((amdgpu_waves_per_eu(C::WPE, C::WPE))) void gemm_tiled_kernel(
    GemmArgs g) {
    extern __shared__ __align__(1024) char smem[];
    SingleProvider<C> p{g};
    if constexpr (C::PP)
        run_pingpong<C>(p, smem);
    else if constexpr (C::STG)
        run_staged<C>(p, smem);
    else if constexpr (C::BLK)
        run_bulk<C>(p, smem);
    else if constexpr (C::XT && C::NS == 5)
        run_direct_x5<C>(p, smem);
    else if constexpr (C::HALVES)
        run_direct_xh<C>(p, smem);
    else if constexpr (C::XT)
        run_direct_xt<C>(p, smem);
    else if constexpr (C::DIRECT)
        run_direct<C>(p, smem);
    else
        run_regs<C>(p, smem);
}

template <class C>
__global__ __launch_bounds__(C::THREADS)
__attribute__((amdgpu_waves_per_eu(C::WPE, C::WPE))) void gemm_grouped_kernel(
    const GroupProblem *__restrict__ tab, int n, int total, int G) {
    extern __shared__ __align__(1024) char smem[];
    GroupProvider<C> p{tab, n, total, G};
    if constexpr (C::PP)
        run_pingpong<C>(p, smem);
    else if constexpr (C::STG)
        run_staged<C>(p, smem);
    else if constexpr (C::BLK)
        run_bulk<C>(p, smem);
    else if constexpr (C::XT && C::NS == 5)
        run_direct_x5<C>(p, smem);
    else if constexpr (C::HALVES)
        run_direct_xh<C>(p, smem);
    else if constexpr (C::XT)
        run_direct_xt<C>(p, smem);
    else if constexpr (C::DIRECT)
        run_direct<C>(p, smem);
    else
        run_regs<C>(p, smem);
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
    e.v.bm = C::BM; e.v.bn = C::BN; e.v.bk = C::BK; e.v.stages = C::NS;
    e.v.sched = C::SCHED;
    e.v.wm = C::WM; e.v.wn = C::WN;
    e.v.b_nk = C::BNK; e.v.c_bf16 = C::CBF16;
    e.kernel = reinterpret_cast<const void *>(&gemm_tiled_kernel<C>);
    e.grouped = reinterpret_cast<const void *>(&gemm_grouped_kernel<C>);
    e.threads = C::THREADS;
    e.smem = C::SMEM;
    return e;
}

#define TG_VARIANTS_FOR(DT, BM, BN, WM, WN, RBY, NS)                          \
    make_entry<Cfg<DT, BM, BN, WM, WN, false, false, RBY, NS>>(),             \
        make_entry<Cfg<DT, BM, BN, WM, WN, false, true, RBY, NS>>(),          \
        make_entry<Cfg<DT, BM, BN, WM, WN, true, false, RBY, NS>>(),          \
        make_entry<Cfg<DT, BM, BN, WM, WN, true, true, RBY, NS>>()

#define TG_VARIANTS_NK(DT, BM, BN, WM, WN, RBY, NS)                           \
    make_entry<Cfg<DT, BM, BN, WM, WN, true, false, RBY, NS>>(),              \
        make_entry<Cfg<DT, BM, BN, WM, WN, true, true, RBY, NS>>()

#define TG_VARIANTS_PP(DT, BM, BN, RBY, NS)                                   \
    make_entry<Cfg<DT, BM, BN, 2, 4, false, false, RBY, NS, TG_SCHED_PINGPONG>>(),         \
        make_entry<Cfg<DT, BM, BN, 2, 4, false, true, RBY, NS, TG_SCHED_PINGPONG>>(),      \
        make_entry<Cfg<DT, BM, BN, 2, 4, true, false, RBY, NS, TG_SCHED_PINGPONG>>(),      \
        make_entry<Cfg<DT, BM, BN, 2, 4, true, true, RBY, NS, TG_SCHED_PINGPONG>>()

#define TG_VARIANTS_XT_NK(DT, BM, BN, RBY, NS)                                \
    make_entry<Cfg<DT, BM, BN, 2, 4, true, false, RBY, NS, TG_SCHED_CROSS>>(), \
        make_entry<Cfg<DT, BM, BN, 2, 4, true, true, RBY, NS, TG_SCHED_CROSS>>()

#define TG_VARIANTS_XW_NK(DT, BM, BN)                                         \
    make_entry<Cfg<DT, BM, BN, 2, 4, true, false, 128, 2,                      \
                   TG_SCHED_CROSS_WARM>>(),                                    \
        make_entry<Cfg<DT, BM, BN, 2, 4, true, true, 128, 2,                   \
                       TG_SCHED_CROSS_WARM>>()

#define TG_VARIANTS_XT_KN(DT, BM, BN, RBY, NS)                                \
    make_entry<Cfg<DT, BM, BN, 2, 4, false, false, RBY, NS, TG_SCHED_CROSS>>(), \
        make_entry<Cfg<DT, BM, BN, 2, 4, false, true, RBY, NS, TG_SCHED_CROSS>>()

#define TG_VARIANTS_BLK(DT, BM, BN, WM, WN, RBY, NS)                          \
    make_entry<Cfg<DT, BM, BN, WM, WN, true, false, RBY, NS, TG_SCHED_BULK>>(), \
        make_entry<Cfg<DT, BM, BN, WM, WN, true, true, RBY, NS, TG_SCHED_BULK>>()

#define TG_VARIANTS_STG(DT, BM, BN)                                           \
    make_entry<Cfg<DT, BM, BN, 2, 2, true, false, 128, 2, TG_SCHED_STAGED>>()

#define TG_VARIANTS_PP_NK(DT, BM, BN, RBY, NS)                                \
    make_entry<Cfg<DT, BM, BN, 2, 4, true, false, RBY, NS, TG_SCHED_PINGPONG>>(),          \
        make_entry<Cfg<DT, BM, BN, 2, 4, true, true, RBY, NS, TG_SCHED_PINGPONG>>()

// Table order is preference order: the first variant matching a request's
// dtype, partition, layout and output type is the default.
const VariantEntry *table(int *count) {
    static const VariantEntry entries[] = {
        TG_VARIANTS_XT_NK(TG_BF16, 256, 256, 128, 2),
        TG_VARIANTS_FOR(TG_BF16, 256, 256, 2, 4, 128, 2),
        TG_VARIANTS_XT_KN(TG_BF16, 256, 256, 128, 2),
        TG_VARIANTS_PP(TG_BF16, 256, 256, 64, 4),
        TG_VARIANTS_XT_NK(TG_BF16, 256, 256, 64, 4),
        TG_VARIANTS_XT_KN(TG_BF16, 256, 256, 64, 4),
        TG_VARIANTS_XT_NK(TG_BF16, 256, 256, 128, 3),
        TG_VARIANTS_XT_KN(TG_BF16, 256, 256, 128, 3),
        TG_VARIANTS_XT_NK(TG_BF16, 256, 256, 64, 5),
        TG_VARIANTS_XT_KN(TG_BF16, 256, 256, 64, 5),
        TG_VARIANTS_STG(TG_BF16, 256, 256),
        TG_VARIANTS_XW_NK(TG_BF16, 256, 256),
        TG_VARIANTS_BLK(TG_BF16, 256, 256, 2, 2, 64, 4),
        TG_VARIANTS_BLK(TG_BF16, 256, 256, 2, 4, 64, 4),
        TG_VARIANTS_FOR(TG_BF16, 128, 128, 2, 2, 64, 4),
        TG_VARIANTS_FOR(TG_BF16, 128, 128, 2, 2, 128, 2),
        TG_VARIANTS_FOR(TG_BF16, 64, 64, 2, 2, 128, 2),
        TG_VARIANTS_FOR(TG_BF16, 32, 32, 1, 1, 128, 2),
        TG_VARIANTS_FOR(TG_F32, 128, 128, 2, 2, 128, 2),
        TG_VARIANTS_FOR(TG_F32, 64, 64, 2, 2, 128, 2),
        TG_VARIANTS_FOR(TG_F32, 32, 32, 1, 1, 128, 2),
        TG_VARIANTS_NK(TG_FP8_E4M3, 256, 256, 2, 4, 128, 2),
        TG_VARIANTS_PP_NK(TG_FP8_E4M3, 256, 256, 64, 4),
        TG_VARIANTS_NK(TG_FP8_E4M3, 256, 256, 2, 4, 64, 4),
        TG_VARIANTS_NK(TG_FP8_E4M3, 128, 128, 2, 2, 128, 2),
        TG_VARIANTS_NK(TG_FP8_E4M3, 64, 64, 2, 2, 128, 2),
        TG_VARIANTS_NK(TG_FP8_E4M3, 32, 32, 1, 1, 128, 2),
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

hipError_t launch_grouped(int variant, int n_problems, int total_tiles,
                          int n_prog, const void *table_dev, hipStream_t st) {
    int n;
    const VariantEntry &e = table(&n)[variant];
    hipError_t err = prepare_smem(e);
    if (err != hipSuccess) return err;
    const GroupProblem *tab = static_cast<const GroupProblem *>(table_dev);
    int np = n_problems, total = total_tiles, G = n_prog;
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
