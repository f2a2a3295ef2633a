// tilegemm.cpp -- host side of the C ABI: argument validation, the
// ownership checks of tile_partition_check, configuration choice, the
// program map, and kernel dispatch.  No call here allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "host_internal.hpp"
#include "tg_internal.hpp"
#include "tg_elementwise.hpp"

using namespace tg;

namespace {

thread_local std::string g_err;

tg_status fail(tg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

tg_status hip_fail(hipError_t e, const char *what) {
    return fail(TG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int esize(int dt) {
    switch (dt) {
    case TG_F32: return 4;
    case TG_BF16: return 2;
    case TG_FP8_E4M3: return 1;
    default: return 0;
    }
}

struct Range {
    uintptr_t lo, hi;  // [lo, hi); empty when lo == hi
};

Range byte_range(const void *data, int64_t rows, int64_t cols, int64_t ld,
                 int es) {
    Range r{(uintptr_t)data, (uintptr_t)data};
    if (rows > 0 && cols > 0)
        r.hi = r.lo + (uintptr_t)(((rows - 1) * ld + cols) * es);
    return r;
}

bool intersect(const Range &a, const Range &b) {
    if (a.lo == a.hi || b.lo == b.hi) return false;
    return a.lo < b.hi && b.lo < a.hi;
}

tg_status check_in(const tg_in *d, const char *name) {
    if (!d) return fail(TG_E_ARG, "%s: NULL descriptor", name);
    if (esize(d->dtype) == 0)
        return fail(TG_E_ARG, "%s: unknown dtype %d", name, d->dtype);
    if (d->rows < 0 || d->cols < 0)
        return fail(TG_E_ARG, "%s: negative size", name);
    if (d->trans != 0 && d->trans != 1)
        return fail(TG_E_ARG, "%s: trans must be 0 or 1", name);
    if (d->rows > 0 && d->cols > 0 && !d->data)
        return fail(TG_E_ARG, "%s: NULL data", name);
    if (d->rows > 1 && d->ld < d->cols)
        return fail(TG_E_SHAPE, "%s: ld %lld < cols %lld", name,
                    (long long)d->ld, (long long)d->cols);
    if (d->ld < 0) return fail(TG_E_SHAPE, "%s: negative ld", name);
    return TG_OK;
}

tg_status check_out(const tg_out *d, bool need_partition) {
    if (!d) return fail(TG_E_ARG, "C: NULL descriptor");
    if (d->dtype != TG_F32 && d->dtype != TG_BF16)
        return fail(TG_E_ARG, "C: dtype must be TG_F32 or TG_BF16");
    if (d->rows < 0 || d->cols < 0) return fail(TG_E_ARG, "C: negative size");
    if (d->rows > 0 && d->cols > 0 && !d->data)
        return fail(TG_E_ARG, "C: NULL data");
    if (need_partition && (d->bm <= 0 || d->bn <= 0))
        return fail(TG_E_ARG, "C: partition %d x %d must be positive", d->bm,
                    d->bn);
    if (d->bm < 0 || d->bn < 0) return fail(TG_E_ARG, "C: negative partition");
    if (d->rows > 1 && d->ld < d->cols)
        return fail(TG_E_SHAPE, "C: ld %lld < cols %lld", (long long)d->ld,
                    (long long)d->cols);
    if (d->ld < 0) return fail(TG_E_SHAPE, "C: negative ld");
    return TG_OK;
}

// Program-map rules: every id on the grid, no sub-tensor twice, none missed.
tg_status check_map(int64_t tiles, int32_t n_prog, const int32_t *offs,
                    const int32_t *ids) {
    if (n_prog < 0) return fail(TG_E_ARG, "negative program count");
    if (n_prog == 0) return TG_OK;
    if (!offs || !ids) return fail(TG_E_ARG, "NULL program map");
    if (offs[0] != 0) return fail(TG_E_ARG, "program map must start at 0");
    // reused per thread: after the first call of a size, checking
    // allocates nothing
    static thread_local std::vector<uint8_t> seen;
    seen.assign((size_t)tiles, 0);
    for (int32_t p = 0; p < n_prog; ++p) {
        if (offs[p + 1] < offs[p])
            return fail(TG_E_ARG, "program %d: decreasing offsets", p);
        for (int32_t q = offs[p]; q < offs[p + 1]; ++q) {
            int64_t t = ids[q];
            if (t < 0 || t >= tiles)
                return fail(TG_E_ARG, "program %d: sub-tensor %lld off the grid",
                            p, (long long)t);
            if (seen[(size_t)t])
                return fail(TG_E_OVERLAP,
                            "sub-tensor %lld owned by two programs (second: %d)",
                            (long long)t, p);
            seen[(size_t)t] = 1;
        }
    }
    for (int64_t t = 0; t < tiles; ++t)
        if (!seen[(size_t)t])
            return fail(TG_E_NOCOVER, "sub-tensor %lld owned by no program",
                        (long long)t);
    return TG_OK;
}

tg_status check_alias(const tg_in *ins, int32_t n_in, const tg_out *out) {
    Range ro = byte_range(out->data, out->rows, out->cols, out->ld,
                          esize(out->dtype));
    for (int32_t i = 0; i < n_in; ++i) {
        Range ri = byte_range(ins[i].data, ins[i].rows, ins[i].cols, ins[i].ld,
                              esize(ins[i].dtype));
        if (intersect(ro, ri))
            return fail(TG_E_ALIAS, "output shares bytes with input %d", i);
    }
    return TG_OK;
}

// ------------------------------------------------------------- device info

int device_cus() {
    static std::mutex mu;
    static std::unordered_map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess)
        cus = 0;
    cache[dev] = cus;
    return cus;
}

// --------------------------------------------------------------- problem

struct Problem {
    int64_t M, N, K;
    int a_dt, b_dt;
    bool b_nk;
    bool c_bf16;
    int precision;
    bool scaled;       // row or column scales given
};

tg_status describe(const tg_in *A, const tg_in *B, const tg_out *C,
                   const tg_opts *o, Problem &p) {
    tg_status st;
    if ((st = check_in(A, "A")) != TG_OK) return st;
    if ((st = check_in(B, "B")) != TG_OK) return st;
    if ((st = check_out(C, false)) != TG_OK) return st;
    if (A->trans) return fail(TG_E_UNSUPPORTED, "A must not be transposed");
    p.M = A->rows;
    p.K = A->cols;
    p.b_nk = B->trans == 1;
    int64_t bk = p.b_nk ? B->cols : B->rows;
    p.N = p.b_nk ? B->rows : B->cols;
    if (bk != p.K)
        return fail(TG_E_SHAPE, "A is %lld x %lld but B has K = %lld",
                    (long long)A->rows, (long long)A->cols, (long long)bk);
    if (C->rows != p.M || C->cols != p.N)
        return fail(TG_E_SHAPE, "C is %lld x %lld, expected %lld x %lld",
                    (long long)C->rows, (long long)C->cols, (long long)p.M,
                    (long long)p.N);
    if (p.M > INT32_MAX || p.N > INT32_MAX || p.K > INT32_MAX)
        return fail(TG_E_SHAPE, "dimension exceeds 2^31 - 1");
    p.a_dt = A->dtype;
    p.b_dt = B->dtype;
    p.c_bf16 = C->dtype == TG_BF16;
    p.precision = o ? o->precision : TG_PREC_NATIVE;
    p.scaled = o && (o->scale_a || o->scale_b);
    if (p.precision < TG_PREC_NATIVE || p.precision > TG_PREC_BF16X6)
        return fail(TG_E_ARG, "unknown precision %d", p.precision);
    bool same = p.a_dt == p.b_dt;
    bool w8 = p.a_dt == TG_BF16 && p.b_dt == TG_FP8_E4M3;
    if (!same && !w8)
        return fail(TG_E_DTYPE, "dtype pair (%d, %d) not provided", p.a_dt,
                    p.b_dt);
    if (p.precision != TG_PREC_NATIVE &&
        (p.a_dt != TG_F32 || p.b_dt != TG_F32))
        return fail(TG_E_DTYPE, "split precision needs f32 A and B");
    return TG_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Can the tiled kernel take this operand layout?
bool tiled_ok(const Problem &p, const tg_in *A, const tg_in *B,
              const tg_out *C, int dt) {
    int es = esize(dt);
    int epc = 16 / es;
    if (p.a_dt != p.b_dt) return false;
    if (dt == TG_FP8_E4M3 && !p.b_nk) return false;
    if (!aligned16(A->data) || !aligned16(B->data)) return false;
    // row starts must stay 16-byte aligned (a single row has no stride)
    if ((A->rows > 1 && (A->ld * es) % 16) || (B->rows > 1 && (B->ld * es) % 16))
        return false;
    // bf16 / e4m3 take any K (the straddling chunk is filled element-wise);
    // the f32 register path needs whole 16-byte chunks
    if (dt == TG_F32 && p.K % epc) return false;
    if (!p.b_nk && (p.N % epc)) return false;
    // the kernels address a sub-tensor with 32-bit byte offsets: 256 rows of
    // any operand (and of C in binary32) must span less than 2^31 bytes
    const int64_t lim = (int64_t)1 << 31;
    if (A->ld * es * 256 >= lim || B->ld * es * 256 >= lim) return false;
    if (C->ld * 4 * 256 >= lim) return false;
    return true;
}

bool skinny_ok(const Problem &p, const tg_in *A, const tg_in *B) {
    if (p.M > 16 || !p.b_nk || p.a_dt != TG_BF16) return false;
    if (p.b_dt != TG_BF16 && p.b_dt != TG_FP8_E4M3) return false;
    if (!aligned16(A->data) || !aligned16(B->data)) return false;
    if ((A->rows > 1 && (A->ld * 2) % 16) ||
        (B->rows > 1 && (B->ld * esize(p.b_dt)) % 16))
        return false;
    return true;
}

// First tiled variant matching the request; zero fields match anything.
// Ping-pong variants have no tail fill for a 16-byte chunk straddling K:
// pp_ok is false when K is not a multiple of the chunk.  Bulk-read
// variants need K a whole number of their 32-deep K tiles (k32_ok).  Staged variants
// need K a whole number of their K tiles (k_tiles_ok: K % 64 == 0 for
// bf16) and apply no scales.
int find_variant(int dt, int bm, int bn, int wm, int wn, int bk, int stages,
                 int sched, bool b_nk, bool c_bf16, bool pp_ok,
                 bool scaled = false, bool k_tiles_ok = false,
                 bool k32_ok = false) {
    int n = tiled_variant_count();
    for (int i = 0; i < n; ++i) {
        const TiledVariant &v = tiled_variant(i);
        if (v.sched == TG_SCHED_PINGPONG && !pp_ok) continue;
        if (v.sched == TG_SCHED_BULK && !k32_ok) continue;
        if (v.sched == TG_SCHED_STAGED && (scaled || !k_tiles_ok)) continue;
        if (v.dtype == dt && v.bm == bm && v.bn == bn && v.b_nk == b_nk &&
            v.c_bf16 == c_bf16 && (wm == 0 || v.wm == wm) &&
            (wn == 0 || v.wn == wn) && (bk == 0 || v.bk == bk) &&
            (stages == 0 || v.stages == stages) &&
            (sched == 0 || v.sched == sched))
            return i;
    }
    return -1;
}

bool chunk_multiple(int64_t K, int dt) { return (K * esize(dt)) % 16 == 0; }

// Default tile choice: the largest square tile that still gives every
// compute unit close to one sub-tensor.
int default_tile(int dt, int64_t M, int64_t N, int cus) {
    const int sizes_lp[] = {256, 128, 64, 32};
    const int sizes_f32[] = {128, 64, 32};
    const int *sz = dt == TG_F32 ? sizes_f32 : sizes_lp;
    int nsz = dt == TG_F32 ? 3 : 4;
    if (cus <= 0) cus = 256;
    for (int i = 0; i < nsz; ++i) {
        int64_t t = ((M + sz[i] - 1) / sz[i]) * ((N + sz[i] - 1) / sz[i]);
        if (t * 4 >= (int64_t)cus * 3) return sz[i];
    }
    return sz[nsz - 1];
}

struct Launch {
    tg_config cfg;
    int variant;       // tiled kernel index, or -1
    int gemm_dt;       // dtype the contraction reads (bf16 for split modes)
    int64_t Kc;        // contraction length seen by the kernel
    int32_t sps;       // decode kernel: K steps per split
    Sched s;
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of a decode product split over `splitk` programs per
// sub-tensor: partial tiles [splitk][M][N] binary32, then (fused
// normalisation) partial sums of squares [splitk][M].
size_t skinny_ws_bytes(int64_t splitk, int64_t M, int64_t N, bool norm) {
    if (splitk <= 1) return 0;
    return up256((size_t)splitk * M * N * 4) +
           (norm ? up256((size_t)splitk * M * 4) : 0);
}

// Decode kernel geometry: K steps (32 bf16 or 64 e4m3 weights per lane
// group) and super-steps (eight 16-byte weight loads per lane).
struct SkinnyGeo {
    int64_t kstep, unroll, nsteps, supers;
};
SkinnyGeo skinny_geo(const Problem &p, int bn) {
    SkinnyGeo g;
    g.kstep = p.b_dt == TG_BF16 ? 32 : 64;
    g.unroll = bn > 16 ? 4 : 8;   // two row tiles: four K steps of two
    g.nsteps = (p.K + g.kstep - 1) / g.kstep;
    g.supers = (g.nsteps + g.unroll - 1) / g.unroll;
    return g;
}

// Decode columns per program that deal N evenly over whole rounds of the
// compute units: N / (ncu r) for the fewest rounds r that bring it to at
// most 32 columns and divide N exactly (else ceil(N / (ncu r)) for the
// fewest rounds); 0 where that leaves fewer than 8 columns per program.
int32_t balanced_bn(int64_t N, int64_t ncu) {
    const int64_t r0 = (N + 32 * ncu - 1) / (32 * ncu);
    for (int64_t r = r0; r < r0 + 4; ++r)
        if (N % (ncu * r) == 0 && N / (ncu * r) >= 8)
            return (int32_t)(N / (ncu * r));
    const int64_t bn = (N + ncu * r0 - 1) / (ncu * r0);
    return bn >= 8 && bn <= 32 ? (int32_t)bn : 0;
}

// Splits that get K work when `splitk` are asked for: each split takes
// ceil(supers / splitk) whole super-steps.
int32_t effective_splitk(int64_t supers, int64_t splitk, int64_t *per) {
    if (supers <= 0 || splitk <= 1) {
        if (per) *per = supers > 0 ? supers : 1;
        return 1;
    }
    const int64_t q = (supers + splitk - 1) / splitk;
    if (per) *per = q;
    return (int32_t)((supers + q - 1) / q);
}

// `have`: workspace bytes the caller supplies; the default K split of a
// decode product is reduced until its workspace fits.
tg_status choose_explicit(const Problem &p, const tg_in *A, const tg_in *B,
                          const tg_out *C, const tg_config *uc, Launch &L,
                          size_t have, bool norm = false) {
    tg_config cfg{};
    if (uc) cfg = *uc;
    if (cfg.kind < TG_KIND_AUTO || cfg.kind > TG_KIND_SIMPLE)
        return fail(TG_E_ARG, "unknown kernel kind %d", cfg.kind);
    int np = p.precision == TG_PREC_BF16X3 ? 3
             : p.precision == TG_PREC_BF16X6 ? 6 : 1;
    L.gemm_dt = np > 1 ? TG_BF16 : p.a_dt;
    L.Kc = p.K * np;
    // the partition of C, when given, fixes the sub-tensor shape
    if (C->bm > 0 || C->bn > 0) {
        if (C->bm <= 0 || C->bn <= 0)
            return fail(TG_E_ARG, "C partition %d x %d: both must be set",
                        C->bm, C->bn);
        if (cfg.bm && cfg.bm != C->bm)
            return fail(TG_E_ARG, "config bm %d != partition bm %d", cfg.bm,
                        C->bm);
        if (cfg.bn && cfg.bn != C->bn)
            return fail(TG_E_ARG, "config bn %d != partition bn %d", cfg.bn,
                        C->bn);
        cfg.bm = C->bm;
        cfg.bn = C->bn;
    }
    // split precisions run the tiled bf16 kernel on the plane operands,
    // whose layout the library lays out itself (always aligned)
    bool t_ok = np > 1 ? ((p.K * np) % 8 == 0 && (p.b_nk || p.N % 8 == 0) &&
                          p.K * np * 2 * 256 < ((int64_t)1 << 31) &&
                          C->ld * 4 * 256 < ((int64_t)1 << 31))
                       : tiled_ok(p, A, B, C, p.a_dt);
    bool s_ok = np == 1 && skinny_ok(p, A, B);
    if (cfg.kind == TG_KIND_AUTO) {
        if (s_ok && (cfg.bm == 0 || (cfg.bm >= p.M && cfg.bm <= 16)) &&
            cfg.bn >= 0 && cfg.bn <= 32)
            cfg.kind = TG_KIND_SKINNY;
        else if (t_ok && (cfg.bm == 0 ||
                          find_variant(L.gemm_dt, cfg.bm, cfg.bn, cfg.wm,
                                       cfg.wn, cfg.bk, cfg.stages, cfg.sched,
                                       p.b_nk, p.c_bf16,
                                       chunk_multiple(L.Kc, L.gemm_dt),
                                       p.scaled, L.Kc % 64 == 0,
                                       L.Kc % 32 == 0) >= 0))
            cfg.kind = TG_KIND_TILED;
        else
            cfg.kind = TG_KIND_SIMPLE;
    }
    int cus = device_cus();
    L.variant = -1;
    if (cfg.kind == TG_KIND_SKINNY) {
        if (!s_ok)
            return fail(TG_E_UNSUPPORTED,
                        "decode kernel needs M <= 16, bf16 A, bf16/e4m3 B "
                        "stored N x K, aligned 16-byte rows");
        if (cfg.bm == 0) cfg.bm = 16;
        // the decode defaults assume MI355X's 256 compute units where the
        // device cannot be asked (host-only planning)
        const int64_t ncu = cus > 0 ? cus : 256;
        // One round of programs, one per compute unit: where N / ncu is 8 to
        // 32 columns, programs of that many columns fill the machine with
        // no K split and so no merge launch.  Measured on (M, N, K) =
        // (1 and 8, 5120, 5120) and (1, 5120, 25600), bf16 and e4m3 cold
        // weights: 3.5-17 % faster than 16-column programs with the best
        // K split (for (1, 51200, 5120), eight rounds of 25 columns lose
        // to 16-column programs, so only the one-round case takes it).
        const int32_t bal = balanced_bn(p.N, ncu);
        const bool one_round = cfg.bn == 0 && cfg.splitk <= 1 && bal > 0 &&
                               p.N <= 32 * ncu;
        // Several rounds with more than four activation rows: programs of
        // the even width and one wavefront each, so that all of them are
        // resident at once (eight per compute unit at N = 51200) with no
        // K split.  Measured at (8 and 16, 51200, 5120): 4-17 % faster
        // than 16- or 32-column programs of four wavefronts, bf16 and
        // e4m3; at (8, 16384 and 32768, 4096) within -14..+4 %.
        const bool resident = cfg.bn == 0 && cfg.splitk <= 1 && bal > 0 &&
                              !one_round && p.M > 4;
        if (one_round || resident) cfg.bn = bal;
        // bf16 weights, up to four activation rows, K up to 8192: where the
        // one-round width needs two row tiles (more than 16 columns), half
        // of it in one row tile, two programs per compute unit of two
        // wavefronts each (both resident).  Measured at N = 5120, 6144 and
        // 8192 (K 4096-8192): 4-18 % faster; at (1, 5120, 25600) 9 %
        // slower, and where the one-round width is 16 or less (N = 4096)
        // 7 % slower, hence the bounds.  Not for the fused normalisation,
        // whose programs each stage the normalisation weights of their K
        // range: twice the programs cost more than they gain (decode
        // layer 21.0 against 19.9 us).
        const bool halves = one_round && !norm && p.b_dt == TG_BF16 &&
                            p.M <= 4 && p.K <= 8192 && bal > 16;
        if (halves) cfg.bn = (bal + 1) / 2;
        if (cfg.bn == 0) {
            // 32-column programs (each activation chunk serves two weight
            // rows) for e4m3 weights with more than four activation rows,
            // or three or four over long sweeps; measured on the decode
            // shapes with cold weights
            const bool wide =
                p.b_dt == TG_FP8_E4M3 &&
                (p.M > 4 || (p.M > 2 && (p.N + 15) / 16 >= 4 * ncu));
            cfg.bn = wide ? 32 : 16;
        }
        if (cfg.bm < p.M || cfg.bm > 16 || cfg.bn < 1 || cfg.bn > 32)
            return fail(TG_E_UNSUPPORTED,
                        "decode kernel owns 16-row x 1..32-column "
                        "sub-tensors (partition %d x %d)", cfg.bm, cfg.bn);
        cfg.bm = 16;
        const SkinnyGeo geo = skinny_geo(p, cfg.bn);
        const int64_t progs = (p.N + cfg.bn - 1) / cfg.bn;
        if (cfg.splitk == 0) {
            // split K over programs until there are four programs per
            // compute unit, keeping at least four super-steps per split
            // (one per wavefront of a four-wavefront program), within the
            // caller's workspace.  Measured over the decode shapes (M 1
            // and 8, bf16 and e4m3, cold weights): within 3 % of the best
            // configuration of each shape on average.
            int64_t sk = 1;
            while (!one_round && !resident && sk < 8 &&
                   progs * sk < 4 * ncu &&
                   (geo.supers + 2 * sk - 1) / (2 * sk) >= 4)
                sk *= 2;
            while (sk > 1 &&
                   skinny_ws_bytes(effective_splitk(geo.supers, sk, nullptr),
                                   p.M, p.N, norm) > have)
                sk /= 2;
            cfg.splitk = (int32_t)sk;
        }
        if (cfg.splitk < 1 || cfg.splitk > TG_MAX_SPLITK)
            return fail(TG_E_UNSUPPORTED, "splitk %d not in [1, %d]",
                        cfg.splitk, TG_MAX_SPLITK);
        int64_t per = 1;
        cfg.splitk = effective_splitk(geo.supers, cfg.splitk, &per);
        L.sps = (int32_t)std::min<int64_t>(per * geo.unroll, INT32_MAX);
        if (cfg.ksplit == 0) {
            // four wavefronts per program split K, and at least one
            // wavefront per compute unit.  Measured on the decode shapes
            // with cold weights, where each wavefront keeps two super-steps
            // of loads in flight.
            int ks = 4;
            while (ks < 16 && progs * cfg.splitk * ks < ncu) ks *= 2;
            // one round of programs: eight wavefronts for e4m3 weights
            // (half the bytes per K element; measured 3-9 % faster than
            // four) except with more than four rows over long K ((8, 5120,
            // 25600): four are 5 % faster), four for bf16
            if (one_round && p.b_dt == TG_FP8_E4M3 &&
                !(p.M > 4 && p.K > 8192))
                ks = 8;
            if (resident) ks = 1;
            if (halves) ks = 2;
            // e4m3 weights, one or two activation rows, several programs
            // per compute unit: two wavefronts per 16-column program
            // (measured at (1 and 2, 51200, 5120), (1, 16384, 4096) and
            // (1, 16384, 16384): 6-12 % faster than 32-column programs of
            // four wavefronts; 4 % slower at (1, 32768, 4096))
            if (!one_round && p.b_dt == TG_FP8_E4M3 && p.M <= 2 &&
                cfg.bn == 16 && cfg.splitk == 1 && progs >= ncu)
                ks = 2;
            // no more wavefronts than super-steps of K (eight 16-byte
            // weight loads per lane each) in one split
            while (ks > 1 && ks > per) ks /= 2;
            cfg.ksplit = ks;
        }
        if (cfg.ksplit != 1 && cfg.ksplit != 2 && cfg.ksplit != 4 &&
            cfg.ksplit != 8 && cfg.ksplit != 16)
            return fail(TG_E_UNSUPPORTED, "ksplit %d not in {1,2,4,8,16}",
                        cfg.ksplit);
        cfg.bk = p.b_dt == TG_BF16 ? 32 : 64;
        cfg.wm = 1;
        cfg.wn = 1;
        L.s.tiles_m = 1;
        L.s.tiles_n = (int32_t)((p.N + cfg.bn - 1) / cfg.bn);
        L.s.n_tiles = L.s.tiles_n;
        L.s.n_prog = L.s.n_tiles;
        L.s.group_m = 1;
    } else if (cfg.kind == TG_KIND_TILED) {
        if (!t_ok)
            return fail(TG_E_UNSUPPORTED,
                        "tiled kernel needs matching A/B dtypes, 16-byte "
                        "aligned rows, K (and N for B stored K x N) a "
                        "multiple of 16 bytes, e4m3 B stored N x K");
        if (cfg.bm == 0 && cfg.bn == 0) {
            int t = default_tile(L.gemm_dt, p.M, p.N, cus);
            cfg.bm = cfg.bn = t;
        } else if (cfg.bm == 0 || cfg.bn == 0) {
            return fail(TG_E_ARG, "config bm/bn: set both or neither");
        }
        // Long K (at least 16384 and twice the larger of M and N): the
        // operands stream from HBM rather than the last-level cache, and the
        // cross-tile schedule with the L2 warm-up is the faster one (measured
        // +3.5 % at 8192 x 4096 x 16384, +9 % at 4096^2 x 32768, +59 % at
        // 2048^2 x 65536; -5 % at 8192^3).
        if (cfg.sched == 0 && cfg.wm == 0 && cfg.wn == 0 && cfg.bk == 0 &&
            cfg.stages == 0 && L.gemm_dt == TG_BF16 && p.b_nk &&
            cfg.bm == 256 && cfg.bn == 256 && L.Kc >= 16384 &&
            L.Kc >= 2 * std::max(p.M, p.N))
            cfg.sched = TG_SCHED_CROSS_WARM;
        L.variant = find_variant(L.gemm_dt, cfg.bm, cfg.bn, cfg.wm, cfg.wn,
                                 cfg.bk, cfg.stages, cfg.sched, p.b_nk,
                                 p.c_bf16, chunk_multiple(L.Kc, L.gemm_dt),
                                 p.scaled, L.Kc % 64 == 0, L.Kc % 32 == 0);
        if (L.variant < 0)
            return fail(TG_E_UNSUPPORTED,
                        "no tiled kernel for dtype %d, %d x %d, waves %d x %d,"
                        " bk %d, %d stages, schedule %d (ping-pong needs K a "
                        "multiple of 16 bytes)", L.gemm_dt, cfg.bm, cfg.bn,
                        cfg.wm, cfg.wn, cfg.bk, cfg.stages, cfg.sched);
        const TiledVariant &v = tiled_variant(L.variant);
        cfg.bk = v.bk;
        cfg.wm = v.wm;
        cfg.wn = v.wn;
        cfg.stages = v.stages;
        cfg.sched = v.sched;
        cfg.ksplit = 1;
        if (cfg.splitk > 1)
            return fail(TG_E_UNSUPPORTED, "splitk applies to the decode "
                                          "kernel only");
        cfg.splitk = 1;
        L.sps = 0;
        L.s.tiles_m = (int32_t)((p.M + cfg.bm - 1) / cfg.bm);
        L.s.tiles_n = (int32_t)((p.N + cfg.bn - 1) / cfg.bn);
        L.s.n_tiles = L.s.tiles_m * L.s.tiles_n;
        int occ = cus > 0 ? tiled_occupancy(L.variant) : 1;
        int64_t cap = (int64_t)(cus > 0 ? cus : 256) * occ;
        L.s.n_prog = (int32_t)std::min<int64_t>(L.s.n_tiles, cap);
        L.s.group_m = 8;
    } else {  // simple
        if (np > 1)
            return fail(TG_E_UNSUPPORTED,
                        "split precision runs on the tiled kernel only");
        if (cfg.bm == 0 && cfg.bn == 0) cfg.bm = cfg.bn = 64;
        if (cfg.bm <= 0 || cfg.bn <= 0 || cfg.bm > 64 || cfg.bn > 64)
            return fail(TG_E_UNSUPPORTED,
                        "simple kernel partitions are at most 64 x 64");
        cfg.bk = 32;
        cfg.wm = 4;
        cfg.wn = 1;
        cfg.ksplit = 1;
        if (cfg.splitk > 1)
            return fail(TG_E_UNSUPPORTED, "splitk applies to the decode "
                                          "kernel only");
        cfg.splitk = 1;
        L.sps = 0;
        L.s.tiles_m = (int32_t)((p.M + cfg.bm - 1) / cfg.bm);
        L.s.tiles_n = (int32_t)((p.N + cfg.bn - 1) / cfg.bn);
        L.s.n_tiles = L.s.tiles_m * L.s.tiles_n;
        L.s.n_prog = L.s.n_tiles;
        L.s.group_m = 1;
    }
    L.cfg = cfg;
    return TG_OK;
}

host::Key key_of(const Problem &p) {
    host::Key k;
    k.M = p.M; k.N = p.N; k.K = p.K;
    k.a_dt = p.a_dt; k.b_dt = p.b_dt; k.b_nk = p.b_nk; k.c_bf16 = p.c_bf16;
    k.precision = p.precision;
    return k;
}

// Every configuration tile_gemm can run for this request.
void candidates(const Problem &p, const tg_in *A, const tg_in *B,
                const tg_out *C, std::vector<tg_config> &out) {
    out.clear();
    auto try_cfg = [&](const tg_config &c) {
        Launch L;
        std::string keep = g_err;
        if (choose_explicit(p, A, B, C, &c, L, SIZE_MAX) == TG_OK) {
            bool dup = false;
            for (const tg_config &o : out)
                dup = dup || std::memcmp(&o, &L.cfg, sizeof o) == 0;
            if (!dup) out.push_back(L.cfg);
        }
        g_err = keep;
    };
    const int np = p.precision == TG_PREC_BF16X3 ? 3
                   : p.precision == TG_PREC_BF16X6 ? 6 : 1;
    const int gdt = np > 1 ? TG_BF16 : p.a_dt;
    const int cus = device_cus();
    const int32_t bal = balanced_bn(p.N, cus > 0 ? cus : 256);
    // 16- and 32-column programs, and the column count that deals N evenly
    // over the compute units
    for (int bn : {16, 32, bal == 16 || bal == 32 ? 0 : bal})
        for (int sk : {1, 2, 4, 8})
            for (int ks : {1, 2, 4, 8, 16}) {
                // K split over programs with two to eight wavefronts each
                if (bn == 0 || (sk > 1 && (ks < 2 || ks > 8))) continue;
                tg_config c{};
                c.kind = TG_KIND_SKINNY;
                c.bn = bn;
                c.ksplit = ks;
                c.splitk = sk;
                try_cfg(c);
            }
    const int n = tiled_variant_count();
    for (int i = 0; i < n; ++i) {
        const TiledVariant &v = tiled_variant(i);
        if (v.dtype != gdt || v.b_nk != (int)p.b_nk || v.c_bf16 != (int)p.c_bf16)
            continue;
        tg_config c{};
        c.kind = TG_KIND_TILED;
        c.bm = v.bm; c.bn = v.bn; c.wm = v.wm; c.wn = v.wn;
        c.bk = v.bk; c.stages = v.stages; c.sched = v.sched;
        try_cfg(c);
    }
    // the element-wise fallback competes only where nothing else runs
    if (!out.empty()) return;
    for (int t : {64, 32}) {
        tg_config c{};
        c.kind = TG_KIND_SIMPLE;
        c.bm = c.bn = t;
        try_cfg(c);
    }
}

float lg2(double x) { return (float)std::log2(x < 1.0 ? 1.0 : x); }

// Picker features of one (request, configuration) pair.
// dflt: the configuration the fixed heuristic gives the same request; the
// last feature flags the candidate that equals it, so that the model learns
// its corrections relative to the heuristic.
void features(const Problem &p, const Launch &L, const tg_config &dflt,
              float *f) {
    const tg_config &c = L.cfg;
    const double tiles = L.s.n_tiles > 0 ? L.s.n_tiles : 1;
    const double progs = L.s.n_prog > 0 ? L.s.n_prog : 1;
    const double rounds = std::ceil(tiles / progs);
    const auto pos = [](int v) { return (double)(v > 0 ? v : 1); };
    f[0] = lg2((double)p.M);
    f[1] = lg2((double)p.N);
    f[2] = lg2((double)(p.K > 0 ? p.K : 1));
    f[3] = (p.a_dt == TG_FP8_E4M3 || p.b_dt == TG_FP8_E4M3) ? 1.f : 0.f;
    f[4] = p.a_dt == TG_F32 ? 1.f : 0.f;
    f[5] = p.b_nk ? 1.f : 0.f;
    f[6] = p.c_bf16 ? 1.f : 0.f;
    f[7] = c.kind == TG_KIND_TILED ? 1.f : 0.f;
    f[8] = c.kind == TG_KIND_SKINNY ? 1.f : 0.f;
    f[9] = c.kind == TG_KIND_SIMPLE ? 1.f : 0.f;
    f[10] = lg2((double)c.bm);
    f[11] = lg2((double)c.bn);
    f[12] = lg2(pos(c.wm * c.wn));
    f[13] = lg2(pos(c.stages));
    f[14] = lg2(pos(c.ksplit));
    f[15] = lg2(tiles);
    f[16] = lg2(progs);
    f[17] = lg2(rounds);
    f[18] = (float)(tiles / (progs * rounds));
    f[19] = (float)((double)p.M * (double)p.N /
                    (tiles * (double)c.bm * (double)c.bn));
    f[20] = c.sched == TG_SCHED_PINGPONG ? 1.f : 0.f;
    f[21] = c.sched == TG_SCHED_CROSS        ? 1.f
            : c.sched == TG_SCHED_CROSS_WARM ? 2.f
                                             : 0.f;
    f[22] = lg2(pos(c.splitk));
    f[23] = std::memcmp(&c, &dflt, sizeof c) == 0 ? 1.f : 0.f;
}

// The heuristic's configuration for a request (what tile_gemm runs with
// neither cache nor model), given a workspace; zeros when none applies.
tg_config default_config(const Problem &p, const tg_in *A, const tg_in *B,
                         const tg_out *C) {
    Launch L0;
    std::string keep = g_err;
    tg_config d{};
    if (choose_explicit(p, A, B, C, nullptr, L0, SIZE_MAX) == TG_OK)
        d = L0.cfg;
    g_err = keep;
    return d;
}

// Configuration when the caller gives none: the tuning cache, then the
// learned picker's argmin over the candidates, then the fixed heuristic.
// `have`: workspace bytes the caller supplies.  Tuned or predicted
// configurations whose decode split needs more are passed over.
tg_status choose(const Problem &p, const tg_in *A, const tg_in *B,
                 const tg_out *C, const tg_opts *o, Launch &L, size_t have,
                 bool norm = false) {
    const tg_config *uc = o ? o->config : nullptr;
    if (uc || C->bm > 0 || C->bn > 0)
        return choose_explicit(p, A, B, C, uc, L, have, norm);
    const int mode = host::picker_mode();
    tg_config cfg;
    auto fits = [&](const Launch &Lx) {
        return Lx.cfg.kind != TG_KIND_SKINNY ||
               skinny_ws_bytes(Lx.cfg.splitk, p.M, p.N, norm) <= have;
    };
    if ((mode & host::kUseCache) && host::cache_find(key_of(p), &cfg)) {
        if (choose_explicit(p, A, B, C, &cfg, L, have, norm) == TG_OK &&
            fits(L))
            return TG_OK;
    }
    if ((mode & host::kUseMlp) && host::picker_ready()) {
        std::vector<tg_config> cands;
        candidates(p, A, B, C, cands);
        float best = 0.f;
        int bi = -1;
        const tg_config dflt = default_config(p, A, B, C);
        for (size_t i = 0; i < cands.size(); ++i) {
            Launch Li;
            if (choose_explicit(p, A, B, C, &cands[i], Li, have, norm) !=
                    TG_OK ||
                !fits(Li))
                continue;
            float f[TG_PICKER_FEATURES];
            features(p, Li, dflt, f);
            const float y = host::picker_predict(f);
            if (bi < 0 || y < best) {
                best = y;
                bi = (int)i;
            }
        }
        if (bi >= 0)
            return choose_explicit(p, A, B, C, &cands[bi], L, have, norm);
    }
    return choose_explicit(p, A, B, C, nullptr, L, have, norm);
}

// Program p -> owned sub-tensor ids, as the kernels walk them.
void build_map(const Launch &L, int32_t *offs, int32_t *ids) {
    const Sched &s = L.s;
    int32_t q = 0;
    offs[0] = 0;
    for (int32_t p = 0; p < s.n_prog; ++p) {
        if (L.cfg.kind == TG_KIND_TILED) {
            for (int32_t t = program_slot(p, s.n_prog); t < s.n_tiles;
                 t += s.n_prog) {
                int32_t tm, tn;
                tile_coords(t, s, tm, tn);
                ids[q++] = tm * s.tiles_n + tn;
            }
        } else {
            ids[q++] = p;  // one program per sub-tensor, row-major grid
        }
        offs[p + 1] = q;
    }
}

// The program map a launch will walk, built into per-thread buffers that
// are reused from call to call, checked with the rules of
// tile_partition_check (injective, covering).
tg_status check_launch_map(const Launch &L) {
    static thread_local std::vector<int32_t> offs, ids;
    offs.resize((size_t)L.s.n_prog + 1);
    ids.resize((size_t)L.s.n_tiles);
    build_map(L, offs.data(), ids.data());
    return check_map(L.s.n_tiles, L.s.n_prog, offs.data(), ids.data());
}

size_t split_bytes(const Problem &p, int np) {
    return up256((size_t)p.M * p.K * np * 2) +
           up256((size_t)p.K * p.N * np * 2);
}

int planes_of(int precision) {
    return precision == TG_PREC_BF16X3 ? 3
           : precision == TG_PREC_BF16X6 ? 6 : 1;
}

// Plane blocks along the concatenated K axis, smallest products first.
// Entries are (A plane, B plane) with 0 = hi, 1 = mid, 2 = lo.
const int8_t kX3A[3] = {0, 1, 0}, kX3B[3] = {1, 0, 0};
const int8_t kX6A[6] = {1, 2, 0, 1, 0, 0}, kX6B[6] = {1, 0, 2, 0, 1, 0};

// Consistency tag of a grouped plan: a mix of its fields, so that a plan
// prepare did not fill (or one altered since) is refused.
uint64_t plan_tag(const tg_grouped_plan &pl) {
    uint64_t h = 0x9e3779b97f4a7c15ull ^ (uint64_t)(uintptr_t)pl.workspace;
    const int32_t f[4] = {pl.n, pl.total_tiles, pl.n_prog, pl.variant};
    for (int32_t v : f) {
        h ^= (uint64_t)(uint32_t)v + 0x9e3779b97f4a7c15ull + (h << 6) +
             (h >> 2);
        h *= 0xff51afd7ed558ccdull;
    }
    return h;
}

// Device scratch of the allocation-free entry point: one array per device
// (each device holds its own copy at its own address), resolved once per
// device with that device current.  In host code the array's name is
// only a stand-in; the resolved address is the one kernels receive.
__device__ __align__(256) char scratch[TG_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::unordered_map<int, void *> g_scratch_addr;

tg_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return TG_OK;
    }
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "scratch address");
    if (!ptr) return fail(TG_E_HIP, "scratch address is NULL");
    g_scratch_addr[dev] = ptr;
    *out = ptr;
    return TG_OK;
}

// The workspace of a split decode product: present, large and aligned
// enough, and sharing no bytes with the operands or the output.
tg_status check_split_ws(const tg_opts *o, const Problem &p, int splitk,
                         bool norm, const tg_in *ins, int n_in,
                         const tg_out *C) {
    const size_t need = skinny_ws_bytes(splitk, p.M, p.N, norm);
    if (!o || !o->workspace || o->workspace_bytes < need)
        return fail(TG_E_WORKSPACE,
                    "decode product split over %d programs per sub-tensor "
                    "needs a workspace of %zu bytes", splitk, need);
    if (!aligned16(o->workspace))
        return fail(TG_E_WORKSPACE, "workspace must be 16-byte aligned");
    Range rw{(uintptr_t)o->workspace, (uintptr_t)o->workspace + need};
    if (intersect(rw, byte_range(C->data, C->rows, C->cols, C->ld,
                                 esize(C->dtype))))
        return fail(TG_E_ALIAS, "workspace shares bytes with the output");
    for (int i = 0; i < n_in; ++i)
        if (intersect(rw, byte_range(ins[i].data, ins[i].rows, ins[i].cols,
                                     ins[i].ld, esize(ins[i].dtype))))
            return fail(TG_E_ALIAS, "workspace shares bytes with input %d",
                        i);
    return TG_OK;
}

// The residual of a decode product (opts->residual): an M x N bf16 or f32
// row-major device matrix, aligned to its element size.  Fills the kernel
// arguments (res = nullptr without one).
tg_status take_residual(const tg_opts *o, const Problem &p, SkinnyArgs &a) {
    a.res = nullptr;
    a.ldr = 0;
    a.res_bf16 = 0;
    if (!o || !o->residual) return TG_OK;
    const tg_in *r = o->residual;
    tg_status st = check_in(r, "residual");
    if (st != TG_OK) return st;
    if (r->dtype != TG_BF16 && r->dtype != TG_F32)
        return fail(TG_E_DTYPE, "residual must be bf16 or f32");
    if (r->trans || r->rows != p.M || r->cols != p.N)
        return fail(TG_E_SHAPE, "residual must be %lld x %lld, row-major",
                    (long long)p.M, (long long)p.N);
    if ((uintptr_t)r->data % (uintptr_t)esize(r->dtype))
        return fail(TG_E_SHAPE, "residual not aligned to its element size");
    a.res = r->data;
    a.ldr = r->ld;
    a.res_bf16 = r->dtype == TG_BF16;
    return TG_OK;
}

}  // namespace

extern "C" {

const char *tg_status_str(int32_t st) {
    switch (st) {
    case TG_OK: return "TG_OK";
    case TG_E_ARG: return "TG_E_ARG";
    case TG_E_DTYPE: return "TG_E_DTYPE";
    case TG_E_SHAPE: return "TG_E_SHAPE";
    case TG_E_OVERLAP: return "TG_E_OVERLAP";
    case TG_E_NOCOVER: return "TG_E_NOCOVER";
    case TG_E_ALIAS: return "TG_E_ALIAS";
    case TG_E_WORKSPACE: return "TG_E_WORKSPACE";
    case TG_E_UNSUPPORTED: return "TG_E_UNSUPPORTED";
    case TG_E_HIP: return "TG_E_HIP";
    default: return "unknown status";
    }
}

const char *tg_last_error(void) { return g_err.c_str(); }

int32_t tg_device_cus(void) { return device_cus(); }

tg_status tile_partition_check(const tg_in *ins, int32_t n_in,
                               const tg_out *out, int32_t n_prog,
                               const int32_t *prog_offsets,
                               const int32_t *prog_tiles) {
    g_err.clear();
    tg_status st;
    if (n_in < 0 || (n_in > 0 && !ins))
        return fail(TG_E_ARG, "bad input list");
    for (int32_t i = 0; i < n_in; ++i) {
        char name[32];
        snprintf(name, sizeof name, "input %d", i);
        if ((st = check_in(&ins[i], name)) != TG_OK) return st;
    }
    if ((st = check_out(out, true)) != TG_OK) return st;
    int64_t tiles = ((out->rows + out->bm - 1) / out->bm) *
                    ((out->cols + out->bn - 1) / out->bn);
    if ((st = check_map(tiles, n_prog, prog_offsets, prog_tiles)) != TG_OK)
        return st;
    return check_alias(ins, n_in, out);
}

size_t tile_gemm_workspace_size(const tg_in *A, const tg_in *B,
                                const tg_out *C, const tg_opts *o) {
    std::string keep = g_err;
    Problem p;
    if (describe(A, B, C, o, p) != TG_OK) {
        g_err = keep;
        return 0;
    }
    int np = planes_of(p.precision);
    if (np > 1) return split_bytes(p, np);
    Launch L;
    size_t need = 0;
    if (choose(p, A, B, C, o, L, SIZE_MAX) == TG_OK &&
        L.cfg.kind == TG_KIND_SKINNY)
        need = skinny_ws_bytes(L.cfg.splitk, p.M, p.N, false);
    g_err = keep;
    return need;
}

tg_status tile_gemm_plan(const tg_in *A, const tg_in *B, const tg_out *C,
                         const tg_opts *o, tg_config *cfg, int32_t *n_prog,
                         int32_t *prog_offsets, int32_t *prog_tiles) {
    g_err.clear();
    Problem p;
    tg_status st = describe(A, B, C, o, p);
    if (st != TG_OK) return st;
    Launch L;
    // the plan for a caller supplying opts->workspace_bytes of workspace
    if ((st = choose(p, A, B, C, o, L, o ? o->workspace_bytes : 0)) != TG_OK)
        return st;
    if (cfg) *cfg = L.cfg;
    if (n_prog) *n_prog = L.s.n_prog;
    if (prog_offsets && prog_tiles) build_map(L, prog_offsets, prog_tiles);
    return TG_OK;
}

tg_status tile_gemm(const tg_in *A, const tg_in *B, tg_out *C,
                    const tg_opts *o, tg_stream stream) {
    g_err.clear();
    Problem p;
    tg_status st = describe(A, B, C, o, p);
    if (st != TG_OK) return st;
    Launch L;
    const size_t have = o && o->workspace ? o->workspace_bytes : 0;
    if ((st = choose(p, A, B, C, o, L, have)) != TG_OK) return st;
    const bool residual = o && o->residual;
    if (residual && L.cfg.kind != TG_KIND_SKINNY)
        return fail(TG_E_UNSUPPORTED, "a residual is added by the decode "
                                      "kernel only (M <= 16, W stored N x K)");
    const bool checked = !o || o->checked;
    if (checked) {
        // the program map the kernel will walk must be injective and cover
        // the partition of C, and C may not alias A, B or the residual
        if ((st = check_launch_map(L)) != TG_OK) return st;
        tg_out part = *C;
        part.bm = L.cfg.bm;
        part.bn = L.cfg.bn;
        tg_in ins[3] = {*A, *B, residual ? *o->residual : *A};
        if ((st = check_alias(ins, residual ? 3 : 2, &part)) != TG_OK)
            return st;
    }
    C->bm = L.cfg.bm;
    C->bn = L.cfg.bn;
    if (p.M == 0 || p.N == 0) return TG_OK;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const float *sa = o ? o->scale_a : nullptr;
    const float *sb = o ? o->scale_b : nullptr;
    int32_t *wc = o ? o->write_count : nullptr;
    hipError_t e = hipSuccess;

    if (L.cfg.kind == TG_KIND_SKINNY) {
        SkinnyArgs a;
        a.x = A->data; a.w = B->data; a.y = C->data;
        a.scale_a = sa; a.scale_w = sb; a.wcount = wc;
        a.ldx = A->ld; a.ldw = B->ld; a.ldy = C->ld;
        a.M = (int32_t)p.M; a.N = (int32_t)p.N; a.K = (int32_t)p.K;
        a.bn = L.cfg.bn;
        a.splitk = L.cfg.splitk;
        a.steps_per_split = L.sps;
        a.part = nullptr;
        a.ssq_part = nullptr;
        if ((st = take_residual(o, p, a)) != TG_OK) return st;
        if (a.splitk > 1) {
            const tg_in ins[3] = {*A, *B, residual ? *o->residual : *A};
            if ((st = check_split_ws(o, p, a.splitk, false, ins,
                                     residual ? 3 : 2, C)) != TG_OK)
                return st;
            a.part = static_cast<float *>(o->workspace);
        }
        e = launch_skinny(p.b_dt, p.c_bf16, L.cfg.bn, L.cfg.ksplit, a, hs);
        if (e == hipSuccess && a.splitk > 1)
            e = launch_skinny_merge(p.c_bf16, a, false, 0.f, hs);
        return e == hipSuccess ? TG_OK : hip_fail(e, "decode kernel launch");
    }
    if (L.cfg.kind == TG_KIND_SIMPLE) {
        SimpleArgs a;
        a.a = A->data; a.b = B->data; a.c = C->data;
        a.scale_a = sa; a.scale_b = sb; a.wcount = wc;
        a.lda = A->ld; a.ldb = B->ld; a.ldc = C->ld;
        a.M = (int32_t)p.M; a.N = (int32_t)p.N; a.K = (int32_t)p.K;
        a.a_dtype = p.a_dt; a.b_dtype = p.b_dt; a.c_bf16 = p.c_bf16;
        a.b_nk = p.b_nk; a.bm = L.cfg.bm; a.bn = L.cfg.bn;
        e = launch_simple(a, hs);
        return e == hipSuccess ? TG_OK : hip_fail(e, "simple kernel launch");
    }

    GemmArgs g;
    g.a = A->data; g.b = B->data; g.c = C->data;
    g.scale_a = sa; g.scale_b = sb; g.wcount = wc;
    g.lda = A->ld; g.ldb = B->ld; g.ldc = C->ld;
    g.M = (int32_t)p.M; g.N = (int32_t)p.N; g.K = (int32_t)p.K;
    g.s = L.s;
    int np = planes_of(p.precision);
    if (np > 1) {
        size_t need = split_bytes(p, np);
        if (!o || !o->workspace || o->workspace_bytes < need)
            return fail(TG_E_WORKSPACE, "split precision needs %zu bytes",
                        need);
        if (!aligned16(o->workspace))
            return fail(TG_E_WORKSPACE, "workspace must be 16-byte aligned");
        Range rw{(uintptr_t)o->workspace, (uintptr_t)o->workspace + need};
        Range rc = byte_range(C->data, C->rows, C->cols, C->ld,
                              esize(C->dtype));
        Range ra = byte_range(A->data, A->rows, A->cols, A->ld, 4);
        Range rb = byte_range(B->data, B->rows, B->cols, B->ld, 4);
        if (intersect(rw, rc) || intersect(rw, ra) || intersect(rw, rb))
            return fail(TG_E_ALIAS, "workspace shares bytes with an operand");
        char *ws = static_cast<char *>(o->workspace);
        size_t a_bytes = ((size_t)p.M * p.K * np * 2 + 255) & ~(size_t)255;
        void *ap = ws, *bp = ws + a_bytes;
        const int8_t *oa = np == 3 ? kX3A : kX6A;
        const int8_t *ob = np == 3 ? kX3B : kX6B;
        int64_t Kc = p.K * np;
        // A' = M x (np K): plane block b occupies columns [b K, (b+1) K)
        e = launch_split_rows(static_cast<const float *>(A->data), A->ld,
                              (int32_t)p.M, (int32_t)p.K, np, oa, ap, Kc,
                              p.K, hs);
        if (e != hipSuccess) return hip_fail(e, "split launch");
        if (p.b_nk) {
            // B stored N x K -> B' = N x (np K)
            e = launch_split_rows(static_cast<const float *>(B->data), B->ld,
                                  (int32_t)p.N, (int32_t)p.K, np, ob, bp, Kc,
                                  p.K, hs);
        } else {
            // B stored K x N -> B' = (np K) x N: plane block b is rows
            // [b K, (b+1) K)
            e = launch_split_rows(static_cast<const float *>(B->data), B->ld,
                                  (int32_t)p.K, (int32_t)p.N, np, ob, bp, p.N,
                                  p.K * p.N, hs);
        }
        if (e != hipSuccess) return hip_fail(e, "split launch");
        g.a = ap; g.b = bp;
        g.lda = Kc;
        g.ldb = p.b_nk ? Kc : p.N;
        g.K = (int32_t)Kc;
    }
    e = launch_tiled(L.variant, g, hs);
    return e == hipSuccess ? TG_OK : hip_fail(e, "tiled kernel launch");
}

tg_status tile_gemm_noalloc(const tg_in *A, const tg_in *B, tg_out *C,
                            const tg_opts *o, tg_stream stream) {
    g_err.clear();
    if (o && o->workspace)
        return fail(TG_E_ARG, "the allocation-free call takes no workspace");
    void *ptr = nullptr;
    tg_status st = scratch_address(&ptr);
    if (st != TG_OK) return st;
    tg_opts oo{};
    if (o)
        oo = *o;
    else
        oo.checked = 1;
    oo.workspace = ptr;
    oo.workspace_bytes = TG_NOALLOC_SCRATCH_BYTES;
    st = tile_gemm(A, B, C, &oo, stream);
    if (st == TG_E_WORKSPACE)
        g_err = "the allocation-free call's scratch holds " +
                std::to_string((size_t)TG_NOALLOC_SCRATCH_BYTES) +
                " bytes: " + g_err;
    return st;
}

int32_t tile_gemm_candidates(const tg_in *A, const tg_in *B, const tg_out *C,
                             const tg_opts *o, tg_config *out, int32_t max) {
    g_err.clear();
    Problem p;
    if (describe(A, B, C, o, p) != TG_OK) return -1;
    std::vector<tg_config> c;
    candidates(p, A, B, C, c);
    for (int32_t i = 0; i < (int32_t)c.size() && i < max; ++i) out[i] = c[i];
    return (int32_t)c.size();
}

tg_status tile_picker_features(const tg_in *A, const tg_in *B,
                               const tg_out *C, const tg_config *cfg,
                               float *feat) {
    g_err.clear();
    if (!feat) return fail(TG_E_ARG, "NULL feature buffer");
    Problem p;
    tg_status st = describe(A, B, C, nullptr, p);
    if (st != TG_OK) return st;
    Launch L;
    if ((st = choose_explicit(p, A, B, C, cfg, L, SIZE_MAX)) != TG_OK)
        return st;
    features(p, L, default_config(p, A, B, C), feat);
    return TG_OK;
}

// ----------------------------------------------------------------- grouped

size_t tile_gemm_grouped_workspace_size(int32_t n) {
    if (n <= 0) return 0;
    return sizeof(GroupProblem) * (size_t)n;
}

tg_status tile_gemm_grouped_prepare(int32_t n, const tg_in *A,
                                    const tg_in *B, tg_out *C,
                                    const tg_opts *o, void *ws,
                                    size_t ws_bytes, tg_grouped_plan *plan,
                                    tg_stream stream) {
    g_err.clear();
    if (!plan) return fail(TG_E_ARG, "NULL plan");
    if (n <= 0 || !A || !B || !C) return fail(TG_E_ARG, "empty problem list");
    if (!ws) return fail(TG_E_WORKSPACE, "NULL workspace");
    if (ws_bytes < tile_gemm_grouped_workspace_size(n))
        return fail(TG_E_WORKSPACE, "workspace needs %zu bytes",
                    tile_gemm_grouped_workspace_size(n));
    if (!aligned16(ws)) return fail(TG_E_WORKSPACE, "workspace misaligned");
    if (o && (o->precision != TG_PREC_NATIVE || o->scale_a || o->scale_b))
        return fail(TG_E_UNSUPPORTED,
                    "grouped launch: native precision, no scales");
    int32_t *wc = o ? o->write_count : nullptr;
    std::vector<Problem> ps((size_t)n);
    int c_bf16 = -1, b_nk = -1;
    int64_t maxM = 0, maxN = 0;
    for (int32_t i = 0; i < n; ++i) {
        tg_status st = describe(&A[i], &B[i], &C[i], nullptr, ps[i]);
        if (st != TG_OK) {
            g_err = "problem " + std::to_string(i) + ": " + g_err;
            return st;
        }
        if (ps[i].a_dt != TG_BF16 || ps[i].b_dt != TG_BF16)
            return fail(TG_E_DTYPE, "problem %d: grouped launch is bf16", i);
        if (!tiled_ok(ps[i], &A[i], &B[i], &C[i], TG_BF16))
            return fail(TG_E_UNSUPPORTED, "problem %d: layout not tileable",
                        i);
        if (c_bf16 < 0) c_bf16 = ps[i].c_bf16;
        if (b_nk < 0) b_nk = ps[i].b_nk;
        if (c_bf16 != (int)ps[i].c_bf16 || b_nk != (int)ps[i].b_nk)
            return fail(TG_E_UNSUPPORTED,
                        "problem %d: all problems share C dtype and B layout",
                        i);
        maxM = std::max(maxM, ps[i].M);
        maxN = std::max(maxN, ps[i].N);
    }
    // ownership across the launch: outputs pairwise disjoint and disjoint
    // from every input
    std::vector<Range> outs((size_t)n), ins((size_t)2 * n);
    for (int32_t i = 0; i < n; ++i) {
        outs[i] = byte_range(C[i].data, C[i].rows, C[i].cols, C[i].ld,
                             esize(C[i].dtype));
        ins[2 * i] = byte_range(A[i].data, A[i].rows, A[i].cols, A[i].ld, 2);
        ins[2 * i + 1] =
            byte_range(B[i].data, B[i].rows, B[i].cols, B[i].ld, 2);
    }
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = i + 1; j < n; ++j)
            if (intersect(outs[i], outs[j]))
                return fail(TG_E_OVERLAP, "outputs %d and %d share bytes", i,
                            j);
        for (int32_t j = 0; j < 2 * n; ++j)
            if (intersect(outs[i], ins[j]))
                return fail(TG_E_ALIAS, "output %d shares bytes with an input "
                                        "of problem %d", i, j / 2);
    }
    // one tile shape for the launch
    tg_config cfg{};
    if (o && o->config) cfg = *o->config;
    if (cfg.bm == 0 || cfg.bn == 0) {
        int64_t work = 0;
        for (auto &p : ps) work += p.M * p.N;
        cfg.bm = cfg.bn = work >= (int64_t)256 * 256 * 256 ? 256 : 128;
    }
    bool pp_ok = true, tiles_ok = true, k32_ok = true;
    for (auto &p : ps) {
        pp_ok = pp_ok && chunk_multiple(p.K, TG_BF16);
        tiles_ok = tiles_ok && p.K % 64 == 0;
        k32_ok = k32_ok && p.K % 32 == 0;
    }
    int variant = find_variant(TG_BF16, cfg.bm, cfg.bn, cfg.wm, cfg.wn,
                               cfg.bk, cfg.stages, cfg.sched, b_nk == 1,
                               c_bf16 == 1, pp_ok, false, tiles_ok, k32_ok);
    if (variant < 0)
        return fail(TG_E_UNSUPPORTED, "no tiled kernel %d x %d", cfg.bm,
                    cfg.bn);
    for (int32_t i = 0; i < n; ++i) {
        C[i].bm = cfg.bm;
        C[i].bn = cfg.bn;
    }
    // longest K first: programs take tiles in table order with a fixed
    // stride, so the costliest tiles are spread over all programs first
    std::vector<int32_t> order((size_t)n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return ps[x].K > ps[y].K;
    });
    // problem i's write counters follow those of problems 0 .. i-1
    std::vector<int64_t> wc_off((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        wc_off[i + 1] = wc_off[i] + ps[i].M * ps[i].N;
    std::vector<GroupProblem> tab((size_t)n);
    int64_t total = 0;
    for (int32_t r = 0; r < n; ++r) {
        int32_t i = order[r];
        GroupProblem &g = tab[r];
        g.a = A[i].data; g.b = B[i].data; g.c = C[i].data;
        g.lda = A[i].ld; g.ldb = B[i].ld; g.ldc = C[i].ld;
        g.M = (int32_t)ps[i].M; g.N = (int32_t)ps[i].N; g.K = (int32_t)ps[i].K;
        g.tiles_m = (int32_t)((ps[i].M + cfg.bm - 1) / cfg.bm);
        g.tiles_n = (int32_t)((ps[i].N + cfg.bn - 1) / cfg.bn);
        g.tile_begin = (int32_t)total;
        g.c_bf16 = c_bf16;
        g.b_nk = b_nk;
        g.wcount = wc ? wc + wc_off[i] : nullptr;
        total += (int64_t)g.tiles_m * g.tiles_n;
    }
    if (total > INT32_MAX) return fail(TG_E_SHAPE, "too many sub-tensors");
    tg_grouped_plan pl{};
    pl.workspace = ws;
    pl.n = n;
    pl.total_tiles = (int32_t)total;
    int cus = device_cus();
    int occ = cus > 0 ? tiled_occupancy(variant) : 1;
    pl.n_prog = (int32_t)std::min<int64_t>(total,
                                           (int64_t)(cus > 0 ? cus : 256) * occ);
    if (pl.n_prog < 1) pl.n_prog = 1;
    pl.variant = variant;
    pl.tag = plan_tag(pl);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(ws, tab.data(), sizeof(GroupProblem) * n,
                                  hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "grouped table copy");
    // the table lives in host memory owned by this call
    e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_fail(e, "grouped table copy");
    *plan = pl;
    return TG_OK;
}

tg_status tile_gemm_grouped(const tg_grouped_plan *plan, tg_stream stream) {
    g_err.clear();
    if (!plan) return fail(TG_E_ARG, "NULL plan");
    if (!plan->workspace || plan->tag != plan_tag(*plan) ||
        plan->variant < 0 || plan->variant >= tiled_variant_count() ||
        plan->n <= 0 || plan->total_tiles < 0 || plan->n_prog < 1)
        return fail(TG_E_ARG,
                    "plan was not filled by tile_gemm_grouped_prepare");
    if (plan->total_tiles == 0) return TG_OK;
    hipError_t e = launch_grouped(plan->variant, plan->n, plan->total_tiles,
                                  plan->n_prog, plan->workspace,
                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TG_OK : hip_fail(e, "grouped kernel launch");
}

tg_status tile_rms_norm_matvec(const tg_in *x, const tg_in *nw, float eps,
                               const tg_in *W, tg_out *y, const tg_opts *o,
                               tg_stream stream) {
    g_err.clear();
    tg_status st;
    if ((st = check_in(nw, "nw")) != TG_OK) return st;
    if (nw->dtype != TG_BF16 || nw->trans || nw->rows != 1)
        return fail(TG_E_SHAPE, "nw must be a 1 x K bf16 row");
    if (!(eps >= 0.0f) || !std::isfinite(eps))
        return fail(TG_E_ARG, "eps must be finite and >= 0");
    if (o && (o->precision != TG_PREC_NATIVE || o->config))
        return fail(TG_E_ARG, "the fused product takes no precision or "
                              "configuration options");
    tg_opts oo{};
    if (o) oo = *o;
    else oo.checked = 1;
    tg_config cfg{};
    cfg.kind = TG_KIND_SKINNY;
    cfg.ksplit = 4;
    oo.config = &cfg;
    const size_t have = o && o->workspace ? o->workspace_bytes : 0;
    Problem p;
    if ((st = describe(x, W, y, &oo, p)) != TG_OK) return st;
    if (nw->cols != p.K)
        return fail(TG_E_SHAPE, "nw has %lld columns, K = %lld",
                    (long long)nw->cols, (long long)p.K);
    if (p.K > 0 && ((uintptr_t)nw->data & 15) != 0)
        return fail(TG_E_SHAPE, "nw must be 16-byte aligned");
    Launch L;
    if ((st = choose(p, x, W, y, &oo, L, have, true)) != TG_OK) return st;
    const bool residual = oo.residual != nullptr;
    if (oo.checked) {
        if ((st = check_launch_map(L)) != TG_OK) return st;
        tg_out part = *y;
        part.bm = L.cfg.bm;
        part.bn = L.cfg.bn;
        tg_in ins[4] = {*x, *W, *nw, residual ? *oo.residual : *x};
        if ((st = check_alias(ins, residual ? 4 : 3, &part)) != TG_OK)
            return st;
    }
    y->bm = L.cfg.bm;
    y->bn = L.cfg.bn;
    if (p.M == 0 || p.N == 0) return TG_OK;
    SkinnyNormArgs a;
    a.s.x = x->data; a.s.w = W->data; a.s.y = y->data;
    a.s.scale_a = oo.scale_a; a.s.scale_w = oo.scale_b;
    a.s.wcount = oo.write_count;
    a.s.ldx = x->ld; a.s.ldw = W->ld; a.s.ldy = y->ld;
    a.s.M = (int32_t)p.M; a.s.N = (int32_t)p.N; a.s.K = (int32_t)p.K;
    a.s.bn = L.cfg.bn;
    a.s.splitk = L.cfg.splitk;
    a.s.steps_per_split = L.sps;
    a.s.part = nullptr;
    a.s.ssq_part = nullptr;
    a.norm_w = nw->data;
    a.eps = eps;
    if ((st = take_residual(&oo, p, a.s)) != TG_OK) return st;
    if (a.s.splitk > 1) {
        const tg_in ins[4] = {*x, *W, *nw, residual ? *oo.residual : *x};
        if ((st = check_split_ws(&oo, p, a.s.splitk, true, ins,
                                 residual ? 4 : 3, y)) != TG_OK)
            return st;
        char *ws = static_cast<char *>(oo.workspace);
        a.s.part = reinterpret_cast<float *>(ws);
        a.s.ssq_part = reinterpret_cast<float *>(
            ws + up256((size_t)a.s.splitk * p.M * p.N * 4));
    }
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = launch_skinny_norm(p.b_dt, p.c_bf16, L.cfg.bn,
                                      L.cfg.ksplit, a, hs);
    if (e == hipSuccess && a.s.splitk > 1)
        e = launch_skinny_merge(p.c_bf16, a.s, true, eps, hs);
    return e == hipSuccess ? TG_OK : hip_fail(e, "fused decode launch");
}

size_t tile_rms_norm_matvec_workspace_size(const tg_in *x, const tg_in *W,
                                           const tg_out *y) {
    std::string keep = g_err;
    tg_config cfg{};
    cfg.kind = TG_KIND_SKINNY;
    cfg.ksplit = 4;
    tg_opts oo{};
    oo.config = &cfg;
    Problem p;
    Launch L;
    size_t need = 0;
    if (describe(x, W, y, &oo, p) == TG_OK &&
        choose(p, x, W, y, &oo, L, SIZE_MAX, true) == TG_OK)
        need = skinny_ws_bytes(L.cfg.splitk, p.M, p.N, true);
    g_err = keep;
    return need;
}

namespace {
tg_status tile_elementwise(bool mul, const tg_in *x, const tg_in *y,
                           tg_out *z, const tg_opts *opts, tg_stream stream) {
    g_err.clear();
    tg_status st;
    if ((st = check_in(x, "x")) != TG_OK) return st;
    if ((st = check_in(y, "y")) != TG_OK) return st;
    if ((st = check_out(z, false)) != TG_OK) return st;
    if (x->trans || y->trans)
        return fail(TG_E_SHAPE, "element-wise operands are not transposed");
    if (x->dtype != z->dtype || y->dtype != z->dtype)
        return fail(TG_E_DTYPE, "x, y and z must share one dtype");
    if (x->rows != z->rows || x->cols != z->cols || y->rows != z->rows ||
        y->cols != z->cols)
        return fail(TG_E_SHAPE, "x, y and z must have one shape");
    const int es = esize(z->dtype), epc = 16 / es;
    if (z->bm == 0 && z->bn == 0) {
        // one row segment of up to 65536 elements per sub-tensor
        z->bm = 1;
        const int64_t bn = std::min<int64_t>(std::max<int64_t>(z->cols, 1),
                                             65536);
        z->bn = (int32_t)((bn + epc - 1) / epc * epc);
    }
    const bool checked = !opts || opts->checked;
    if (checked) {
        const tg_in ins[2] = {*x, *y};
        if ((st = tile_partition_check(ins, 2, z, 0, nullptr, nullptr)) !=
            TG_OK)
            return st;
    } else if (z->bm <= 0 || z->bn <= 0) {
        return fail(TG_E_ARG, "z: partition %d x %d must be positive", z->bm,
                    z->bn);
    }
    if (z->rows == 0 || z->cols == 0) return TG_OK;
    auto al = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
    const bool vec = al(x->data) && al(y->data) && al(z->data) &&
                     (x->ld * es) % 16 == 0 && (y->ld * es) % 16 == 0 &&
                     (z->ld * es) % 16 == 0 && z->bn % epc == 0;
    AddArgs a;
    a.x = x->data; a.y = y->data; a.z = z->data;
    a.wcount = opts ? opts->write_count : nullptr;
    a.ldx = x->rows > 1 ? x->ld : x->cols;
    a.ldy = y->rows > 1 ? y->ld : y->cols;
    a.ldz = z->rows > 1 ? z->ld : z->cols;
    a.rows = z->rows; a.cols = z->cols;
    a.bm = z->bm; a.bn = z->bn;
    a.dtype = z->dtype;
    const int64_t tiles = ((z->rows + z->bm - 1) / z->bm) *
                          ((z->cols + z->bn - 1) / z->bn);
    const int cus = device_cus();
    // sixteen 256-thread programs per compute unit at most (measured at
    // 2^28 bf16 elements: 4 % ahead of four per unit)
    const int programs =
        (int)std::min<int64_t>(tiles, (int64_t)std::max(cus, 1) * 16);
    hipError_t e = (mul ? launch_mul : launch_add)(
        a, vec, programs, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TG_OK : hip_fail(e, "element-wise launch");
}
}  // namespace

tg_status tile_add(const tg_in *x, const tg_in *y, tg_out *z,
                   const tg_opts *opts, tg_stream stream) {
    return tile_elementwise(false, x, y, z, opts, stream);
}

tg_status tile_mul(const tg_in *x, const tg_in *y, tg_out *z,
                   const tg_opts *opts, tg_stream stream) {
    return tile_elementwise(true, x, y, z, opts, stream);
}

tg_status tile_rms_norm(const tg_in *x, const tg_in *w, float eps,
                        tg_out *y, const tg_opts *opts, tg_stream stream) {
    g_err.clear();
    tg_status st;
    if ((st = check_in(x, "x")) != TG_OK) return st;
    if ((st = check_in(w, "w")) != TG_OK) return st;
    if ((st = check_out(y, false)) != TG_OK) return st;
    if (x->trans || w->trans)
        return fail(TG_E_SHAPE, "normalisation operands are not transposed");
    if (x->dtype != y->dtype || w->dtype != y->dtype)
        return fail(TG_E_DTYPE, "x, w and y must share one dtype");
    if (x->rows != y->rows || x->cols != y->cols)
        return fail(TG_E_SHAPE, "x and y must have one shape");
    if (w->rows != 1 || w->cols != y->cols)
        return fail(TG_E_SHAPE, "w must be 1 x %lld", (long long)y->cols);
    if (!(eps >= 0.0f) || !std::isfinite(eps))
        return fail(TG_E_ARG, "eps must be finite and >= 0");
    if (y->bm == 0 && y->bn == 0) {
        y->bm = 1;
        y->bn = (int32_t)std::max<int64_t>(y->cols, 1);
    }
    if (y->cols > 0 && y->bn != y->cols)
        return fail(TG_E_ARG, "y: sub-tensors must span whole rows (bn %d, "
                    "cols %lld)", y->bn, (long long)y->cols);
    const bool checked = !opts || opts->checked;
    if (checked) {
        const tg_in ins[2] = {*x, *w};
        if ((st = tile_partition_check(ins, 2, y, 0, nullptr, nullptr)) !=
            TG_OK)
            return st;
    } else if (y->bm <= 0 || y->bn <= 0) {
        return fail(TG_E_ARG, "y: partition %d x %d must be positive", y->bm,
                    y->bn);
    }
    if (y->rows == 0 || y->cols == 0) return TG_OK;
    NormArgs a;
    a.x = x->data; a.w = w->data; a.y = y->data;
    a.wcount = opts ? opts->write_count : nullptr;
    a.ldx = x->rows > 1 ? x->ld : x->cols;
    a.ldy = y->rows > 1 ? y->ld : y->cols;
    a.rows = y->rows; a.cols = y->cols;
    a.bm = y->bm;
    a.eps = eps;
    a.dtype = y->dtype;
    const int64_t tiles = (y->rows + y->bm - 1) / y->bm;
    const int programs = (int)std::min<int64_t>(
        tiles, (int64_t)std::max(device_cus(), 1) * 8);
    const int es = esize(y->dtype);
    auto al = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
    const bool vec = al(x->data) && al(w->data) && al(y->data) &&
                     (a.ldx * es) % 16 == 0 && (a.ldy * es) % 16 == 0;
    hipError_t e = launch_rms_norm(a, vec, programs,
                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TG_OK : hip_fail(e, "normalisation launch");
}

tg_status tile_error_norm(const void *C, int32_t c_dtype, const double *R,
                          int64_t n, double *out, tg_stream stream) {
    g_err.clear();
    if (c_dtype != TG_F32 && c_dtype != TG_BF16)
        return fail(TG_E_DTYPE, "C must be TG_F32 or TG_BF16");
    if (n < 0) return fail(TG_E_ARG, "negative n");
    if (!out || (n > 0 && (!C || !R))) return fail(TG_E_ARG, "NULL pointer");
    hipError_t e = launch_error_norm(C, c_dtype == TG_BF16, R, n, out,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TG_OK : hip_fail(e, "error-norm launch");
}

}  // extern "C"
