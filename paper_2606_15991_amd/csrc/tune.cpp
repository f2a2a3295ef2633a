// tune.cpp -- configuration choice: exhaustive autotuner, its cache, and the
// learned picker (host inference of the cost-model MLP trained on the GPU
// by the kernels of mlp.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "host_internal.hpp"
#include "tg_internal.hpp"

namespace tg {
namespace host {

bool Key::operator<(const Key &o) const {
    if (M != o.M) return M < o.M;
    if (N != o.N) return N < o.N;
    if (K != o.K) return K < o.K;
    if (a_dt != o.a_dt) return a_dt < o.a_dt;
    if (b_dt != o.b_dt) return b_dt < o.b_dt;
    if (b_nk != o.b_nk) return b_nk < o.b_nk;
    if (c_bf16 != o.c_bf16) return c_bf16 < o.c_bf16;
    return precision < o.precision;
}

bool Key::operator==(const Key &o) const { return !(*this < o) && !(o < *this); }

namespace {
std::mutex g_mu;
std::map<Key, tg_config> g_cache;
int g_mode = kUseCache | kUseMlp;

struct Mlp {
    bool ready = false;
    int n_in = 0, hidden = 0, depth = 0;
    std::vector<float> params, mean, stdev;
};
Mlp g_mlp;
}  // namespace

bool cache_find(const Key &k, tg_config *cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(k);
    if (it == g_cache.end()) return false;
    *cfg = it->second;
    return true;
}

void cache_put(const Key &k, const tg_config &cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[k] = cfg;
}

int picker_mode() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_mode;
}

bool picker_ready() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_mlp.ready;
}

// Forward pass of the cost model, same layout as the GPU kernels:
// depth hidden layers of `hidden` ReLU units, then one linear output.
// Parameters, per layer: W (out x in, row-major) then b (out).
float picker_predict(const float *feat) {
    std::lock_guard<std::mutex> lk(g_mu);
    const Mlp &m = g_mlp;
    std::vector<float> x(m.n_in), y;
    for (int i = 0; i < m.n_in; ++i)
        x[i] = (feat[i] - m.mean[i]) / m.stdev[i];
    const float *w = m.params.data();
    int in = m.n_in;
    for (int l = 0; l <= m.depth; ++l) {
        const int out = l < m.depth ? m.hidden : 1;
        y.assign(out, 0.f);
        const float *b = w + (size_t)out * in;
        for (int o = 0; o < out; ++o) {
            float s = b[o];
            for (int i = 0; i < in; ++i) s += w[(size_t)o * in + i] * x[i];
            y[o] = (l < m.depth && s < 0.f) ? 0.f : s;
        }
        w = b + out;
        x.swap(y);
        in = out;
    }
    return x[0];
}

}  // namespace host
}  // namespace tg

using namespace tg;
using namespace tg::host;

namespace {

host::Key key_from(const tg_in *A, const tg_in *B, const tg_out *C,
                   const tg_opts *o) {
    host::Key k;
    k.M = A->rows;
    k.K = A->cols;
    k.N = B->trans ? B->rows : B->cols;
    k.a_dt = A->dtype;
    k.b_dt = B->dtype;
    k.b_nk = B->trans;
    k.c_bf16 = C->dtype == TG_BF16;
    k.precision = o ? o->precision : TG_PREC_NATIVE;
    return k;
}

}  // namespace

extern "C" {

int32_t tile_picker_mode(int32_t mode) {
    std::lock_guard<std::mutex> lk(g_mu);
    const int32_t old = g_mode;
    if (mode >= 0) g_mode = mode & (kUseCache | kUseMlp);
    return old;
}

size_t tile_mlp_param_count(int32_t n_in, int32_t hidden, int32_t depth) {
    if (n_in <= 0 || hidden <= 0 || depth <= 0) return 0;
    size_t n = (size_t)hidden * n_in + hidden;
    n += (size_t)(depth - 1) * ((size_t)hidden * hidden + hidden);
    n += (size_t)hidden + 1;
    return n;
}

tg_status tile_picker_set(const float *params, int32_t n_in, int32_t hidden,
                          int32_t depth, const float *feat_mean,
                          const float *feat_std) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!params) {
        g_mlp = Mlp();
        return TG_OK;
    }
    if (n_in != TG_PICKER_FEATURES || hidden <= 0 || depth <= 0 ||
        !feat_mean || !feat_std)
        return TG_E_ARG;
    Mlp m;
    m.n_in = n_in;
    m.hidden = hidden;
    m.depth = depth;
    m.params.assign(params, params + tile_mlp_param_count(n_in, hidden, depth));
    m.mean.assign(feat_mean, feat_mean + n_in);
    m.stdev.assign(feat_std, feat_std + n_in);
    for (float &s : m.stdev)
        if (!(s > 0.f)) s = 1.f;
    m.ready = true;
    g_mlp = std::move(m);
    return TG_OK;
}

tg_status tile_picker_predict(const float *feat, float *log_ms) {
    if (!feat || !log_ms) return TG_E_ARG;
    if (!picker_ready()) return TG_E_UNSUPPORTED;
    *log_ms = picker_predict(feat);
    return TG_OK;
}

tg_status tile_autotune(const tg_in *A, const tg_in *B, tg_out *C,
                        const tg_opts *opts, int32_t reps,
                        tg_tune_result *results, int32_t max_results,
                        int32_t *n_results, tg_config *best, tg_stream stream) {
    if (!A || !B || !C || reps <= 0) return TG_E_ARG;
    std::vector<tg_config> cands(128);
    int32_t nc = tile_gemm_candidates(A, B, C, opts, cands.data(), 128);
    if (nc < 0) return TG_E_ARG;
    if (nc == 0) return TG_E_UNSUPPORTED;
    cands.resize(std::min(nc, (int32_t)128));
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return TG_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TG_E_HIP;
    }
    tg_opts o{};
    if (opts) o = *opts;
    o.write_count = nullptr;
    o.checked = 0;
    int32_t bi = -1, nr = 0;
    float best_ms = 0.f;
    tg_status ret = TG_OK;
    for (size_t i = 0; i < cands.size(); ++i) {
        o.config = &cands[i];
        tg_out c = *C;
        tg_status st = tile_gemm(A, B, &c, &o, stream);  // warm-up
        float ms = -1.f;
        if (st == TG_OK) {
            (void)hipEventRecord(e0, hs);
            for (int32_t r = 0; r < reps && st == TG_OK; ++r)
                st = tile_gemm(A, B, &c, &o, stream);
            (void)hipEventRecord(e1, hs);
            if (hipEventSynchronize(e1) != hipSuccess) {
                ret = TG_E_HIP;
                break;
            }
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= (float)reps;
        }
        if (results && nr < max_results) {
            results[nr].cfg = cands[i];
            results[nr].ms = st == TG_OK ? ms : -1.f;
            results[nr].status = st;
            ++nr;
        }
        if (st == TG_OK && (bi < 0 || ms < best_ms)) {
            bi = (int32_t)i;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_results) *n_results = nr;
    if (ret != TG_OK) return ret;
    if (bi < 0) return TG_E_UNSUPPORTED;
    if (best) *best = cands[bi];
    cache_put(key_from(A, B, C, opts), cands[bi]);
    return TG_OK;
}

tg_status tile_autotune_grouped(int32_t n, const tg_in *A, const tg_in *B,
                                tg_out *C, const tg_opts *opts,
                                void *workspace, size_t workspace_bytes,
                                int32_t reps, tg_tune_result *results,
                                int32_t max_results, int32_t *n_results,
                                tg_config *best, tg_grouped_plan *plan,
                                tg_stream stream) {
    if (n <= 0 || !A || !B || !C || !workspace || reps <= 0 || !plan)
        return TG_E_ARG;
    const int b_nk = B[0].trans, c_bf16 = C[0].dtype == TG_BF16;
    std::vector<tg_config> cands;
    for (int i = 0; i < tiled_variant_count(); ++i) {
        const TiledVariant &v = tiled_variant(i);
        if (v.dtype != TG_BF16 || v.b_nk != b_nk || v.c_bf16 != c_bf16)
            continue;
        tg_config c{};
        c.kind = TG_KIND_TILED;
        c.bm = v.bm; c.bn = v.bn; c.bk = v.bk; c.wm = v.wm; c.wn = v.wn;
        c.stages = v.stages; c.sched = v.sched; c.ksplit = 1;
        cands.push_back(c);
    }
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return TG_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TG_E_HIP;
    }
    tg_opts o{};
    if (opts) o = *opts;
    o.write_count = nullptr;
    int32_t bi = -1, nr = 0;
    float best_ms = 0.f;
    tg_status ret = TG_OK;
    for (size_t i = 0; i < cands.size(); ++i) {
        o.config = &cands[i];
        tg_status st = tile_gemm_grouped_prepare(n, A, B, C, &o, workspace,
                                                 workspace_bytes, plan,
                                                 stream);
        // a configuration these problems cannot run is not a candidate
        if (st == TG_E_UNSUPPORTED) continue;
        if (st == TG_OK) st = tile_gemm_grouped(plan, stream);
        float ms = -1.f;
        if (st == TG_OK) {
            (void)hipEventRecord(e0, hs);
            for (int32_t r = 0; r < reps && st == TG_OK; ++r)
                st = tile_gemm_grouped(plan, stream);
            (void)hipEventRecord(e1, hs);
            if (hipEventSynchronize(e1) != hipSuccess) {
                ret = TG_E_HIP;
                break;
            }
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= (float)reps;
        }
        if (results && nr < max_results) {
            results[nr].cfg = cands[i];
            results[nr].ms = st == TG_OK ? ms : -1.f;
            results[nr].status = st;
            ++nr;
        }
        if (st == TG_OK && (bi < 0 || ms < best_ms)) {
            bi = (int32_t)i;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_results) *n_results = nr;
    if (ret != TG_OK) return ret;
    if (bi < 0) return TG_E_UNSUPPORTED;
    o.config = &cands[bi];
    if (opts) o.write_count = opts->write_count;
    tg_status st = tile_gemm_grouped_prepare(n, A, B, C, &o, workspace,
                                             workspace_bytes, plan, stream);
    if (st != TG_OK) return st;
    if (best) *best = cands[bi];
    return TG_OK;
}

tg_status tile_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
    return TG_OK;
}

int32_t tile_tune_cache_size(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int32_t)g_cache.size();
}

// Text format, one entry per line:
//   M N K a_dt b_dt b_nk c_bf16 precision kind bm bn bk wm wn ksplit stages
//   sched splitk
tg_status tile_tune_cache_save(const char *path) {
    if (!path) return TG_E_ARG;
    FILE *f = std::fopen(path, "w");
    if (!f) return TG_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    std::fprintf(f, "# tilegemm tuning cache v4\n");
    for (const auto &kv : g_cache) {
        const Key &k = kv.first;
        const tg_config &c = kv.second;
        std::fprintf(f,
                     "%lld %lld %lld %d %d %d %d %d %d %d %d %d %d %d %d %d "
                     "%d %d\n",
                     (long long)k.M, (long long)k.N, (long long)k.K, k.a_dt,
                     k.b_dt, k.b_nk, k.c_bf16, k.precision, c.kind, c.bm, c.bn,
                     c.bk, c.wm, c.wn, c.ksplit, c.stages, c.sched, c.splitk);
    }
    std::fclose(f);
    return TG_OK;
}

tg_status tile_tune_cache_load(const char *path) {
    if (!path) return TG_E_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return TG_E_ARG;
    char line[512];
    std::map<Key, tg_config> add;
    tg_status st = TG_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        long long M, N, K;
        Key k;
        tg_config c{};
        int n = std::sscanf(
            line,
            "%lld %lld %lld %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d",
            &M, &N, &K, &k.a_dt, &k.b_dt, &k.b_nk, &k.c_bf16, &k.precision,
            &c.kind, &c.bm, &c.bn, &c.bk, &c.wm, &c.wn, &c.ksplit, &c.stages,
            &c.sched, &c.splitk);
        if (n != 18) {
            st = TG_E_ARG;
            break;
        }
        k.M = M; k.N = N; k.K = K;
        add[k] = c;
    }
    std::fclose(f);
    if (st != TG_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &kv : add) g_cache[kv.first] = kv.second;
    return TG_OK;
}

}  // extern "C"
