// host_internal.hpp -- host-side pieces shared by the entry points, the
// autotuner and the tile-configuration picker.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/tilegemm.h"

namespace tg {
namespace host {

// The identity of a product for configuration choice.
struct Key {
    int64_t M, N, K;
    int32_t a_dt, b_dt, b_nk, c_bf16, precision;
    bool operator<(const Key &o) const;
    bool operator==(const Key &o) const;
};

// Tuning cache (filled by tile_autotune, consulted by tile_gemm when no
// configuration is given).
bool cache_find(const Key &k, tg_config *cfg);
void cache_put(const Key &k, const tg_config &cfg);

// Learned picker: predicted log(ms) of a configuration from its features.
bool picker_ready();
float picker_predict(const float *feat);

// Picker mode bits (tile_picker_mode).
enum { kUseCache = 1, kUseMlp = 2 };
int picker_mode();

}  // namespace host
}  // namespace tg
