// tg_internal.hpp -- types shared by the host entry points and the kernels.
//
// The tile schedule below is the single definition of the program ->
// sub-tensor map: the kernels walk it on the device and tile_gemm_plan
// exports it on the host, so the map that tile_partition_check validates is
// the one that runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tilegemm.h"

namespace tg {

// Programs of one launch are dispatched round-robin over the XCDs of the
// chip (program p lands on XCD p % kXcds).  MI355X has 8.
constexpr int kXcds = 8;

// Output partition and persistent-program count of one launch.
struct Sched {
    int32_t tiles_m, tiles_n;  // ceil(M / bm), ceil(N / bn)
    int32_t n_tiles;           // tiles_m * tiles_n
    int32_t n_prog;            // persistent programs G (<= n_tiles)
    int32_t group_m;           // tile-rows per band of the traversal order
};

// Slot of program p: programs that share an XCD get a contiguous range of
// slots, so the sub-tensors co-resident on one XCD's L2 are neighbours and
// share A row-blocks and B column-blocks.  A bijection of [0, G) when
// G % kXcds == 0; the identity otherwise.
__host__ __device__ inline int32_t program_slot(int32_t p, int32_t G) {
    if (G % kXcds != 0) return p;
    return (p % kXcds) * (G / kXcds) + p / kXcds;
}

// Linear traversal index t -> sub-tensor (tm, tn): bands of group_m
// tile-rows, column-major inside a band (the last band may be shorter).
// A bijection of [0, tiles_m * tiles_n).
__host__ __device__ inline void tile_coords(int32_t t, const Sched &s,
                                            int32_t &tm, int32_t &tn) {
    int32_t band_tiles = s.group_m * s.tiles_n;
    int32_t band = t / band_tiles;
    int32_t first_m = band * s.group_m;
    int32_t gm = s.tiles_m - first_m;
    if (gm > s.group_m) gm = s.group_m;
    int32_t in = t - band * band_tiles;
    tm = first_m + in % gm;
    tn = in / gm;
}

// Program p owns traversal indices program_slot(p) + r * G, r = 0, 1, ...
// below n_tiles.  tile_id(tm, tn) = tm * tiles_n + tn is the sub-tensor id
// used by tile_partition_check.

// Kernel arguments of one tiled product.
struct GemmArgs {
    const void *a;
    const void *b;
    void *c;
    const float *scale_a;
    const float *scale_b;
    int32_t *wcount;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    Sched s;
};

// One problem of a grouped launch (device-side table entry).
struct GroupProblem {
    const void *a;
    const void *b;
    void *c;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t tiles_m, tiles_n;
    int32_t tile_begin;  // prefix sum of tile counts, in table order
    int32_t c_bf16;      // output dtype: 0 f32, 1 bf16
    int32_t b_nk;        // B stored N x K
    int32_t *wcount;     // M x N store counters (ld N) or NULL
};

// Tiled kernel variants (compile-time instantiations), by index.
struct TiledVariant {
    int32_t dtype;   // tg_dtype of A and B
    int32_t bm, bn, bk, wm, wn;
    int32_t stages;  // LDS stages in the K-tile ring
    int32_t sched;   // tg_sched (lock-step or ping-pong)
    int32_t b_nk;
    int32_t c_bf16;
};

int tiled_variant_count();
const TiledVariant &tiled_variant(int i);
// Enqueue variant i; returns hipSuccess or the launch error.
hipError_t launch_tiled(int variant, const GemmArgs &args, hipStream_t st);
hipError_t launch_grouped(int variant, int n, int total_tiles, int n_prog,
                          const void *table_dev, hipStream_t st);
int tiled_occupancy(int variant);  // resident workgroups per CU

// Skinny (decode-shaped) kernel.
struct SkinnyArgs {
    const void *x;       // M x K bf16 activations
    const void *w;       // N x K weights (bf16 or e4m3)
    void *y;             // M x N output
    const float *scale_a;
    const float *scale_w;  // per output column (row of W)
    int32_t *wcount;
    int64_t ldx, ldw, ldy;
    int32_t M, N, K;
    int32_t bn;          // output columns per program (16 or 32)
    // K split over programs: splitk programs share one sub-tensor's K, each
    // contracting the K steps [s * steps_per_split, (s + 1) *
    // steps_per_split) of its split s; with splitk > 1 they store their
    // partial tiles (unscaled binary32) into part[s][M][N] and, for the
    // fused normalisation, their rows' partial sums of squares into
    // ssq_part[s][M]; a merge launch then owns y.
    int32_t splitk;
    int32_t steps_per_split;
    float *part;
    float *ssq_part;
    // residual R (M x N, leading dimension ldr, bf16 when res_bf16) added
    // to every output before its one rounding, or nullptr
    const void *res;
    int64_t ldr;
    int32_t res_bf16;
};
hipError_t launch_skinny(int w_dtype, int c_bf16, int bn, int ksplit,
                         const SkinnyArgs &a, hipStream_t st);
// Merge of a split decode product: one program per bm x bn sub-tensor of
// y sums the splitk partial tiles in split order, applies the scales (and
// the fused normalisation's row scale when norm is set) and stores y.
hipError_t launch_skinny_merge(int c_bf16, const SkinnyArgs &a, bool norm,
                               float eps, hipStream_t st);

// Simple kernel: any dtype combination, any alignment.
struct SimpleArgs {
    const void *a;
    const void *b;
    void *c;
    const float *scale_a;
    const float *scale_b;
    int32_t *wcount;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t a_dtype, b_dtype, c_bf16, b_nk;
    int32_t bm, bn;
};
hipError_t launch_simple(const SimpleArgs &a, hipStream_t st);

// Split of f32 operands into bf16 planes for the BF16xN precisions.
hipError_t launch_split_rows(const float *src, int64_t ld, int32_t rows,
                             int32_t cols, int nplanes, const int8_t *order,
                             void *dst, int64_t ldd, int64_t plane_stride,
                             hipStream_t st);

hipError_t launch_error_norm(const void *c, int c_bf16, const double *r,
                             int64_t n, double *out, hipStream_t st);

}  // namespace tg
