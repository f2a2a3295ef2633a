// tg_elementwise.hpp -- host-side launch interface of the element-wise
// kernels (add, RMS normalisation) shared by the entry points and the
// kernel sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tilegemm.h"
#include "tg_internal.hpp"

namespace tg {

// Element-wise z = x + y over z's bm x bn partition.
struct AddArgs {
    const void *x;
    const void *y;
    void *z;
    int32_t *wcount;
    int64_t ldx, ldy, ldz;
    int64_t rows, cols;
    int64_t bm, bn;
    int32_t dtype;       // TG_BF16 or TG_F32, all three operands
};
hipError_t launch_add(const AddArgs &a, bool vec, int programs,
                      hipStream_t st);
// Element-wise z = x * y, same arguments.
hipError_t launch_mul(const AddArgs &a, bool vec, int programs,
                      hipStream_t st);

// y = x * w / sqrt(mean(x^2) + eps) per row, over y's bm x cols partition.
struct NormArgs {
    const void *x;
    const void *w;      // one row of cols weights
    void *y;
    int32_t *wcount;
    int64_t ldx, ldy;
    int64_t rows, cols;
    int64_t bm;
    float eps;
    int32_t dtype;      // TG_BF16 or TG_F32: x, w and y
};
hipError_t launch_rms_norm(const NormArgs &a, bool vec, int programs,
                           hipStream_t st);

// Decode product with the RMS normalisation of the activation rows fused
// in: y = diag(1 / sqrt(mean(x^2) + eps)) (x * nw) . W^T (nw: K bf16
// normalisation weights, one per activation column).  Four wavefronts
// per program (ksplit 4).
struct SkinnyNormArgs {
    SkinnyArgs s;
    const void *norm_w;
    float eps;
};
hipError_t launch_skinny_norm(int w_dtype, int c_bf16, int bn, int ksplit,
                              const SkinnyNormArgs &a, hipStream_t st);

}  // namespace tg
