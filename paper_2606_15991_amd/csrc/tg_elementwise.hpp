// tg_elementwise.hpp -- host-side launch interface of the element-wise
// kernels (add, RMS normalisation) shared by the entry points and the
// kernel sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tilegemm.h"

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

}  // namespace tg
