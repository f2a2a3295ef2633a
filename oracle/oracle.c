/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for the
 * tile-partitioned GEMM C = A.B.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or constant with the HIP path.
 *
 * Everything is computed in IEEE binary64 with no blocking, no reordering
 * beyond the plain definition, and no fused multiply-add contraction
 * (built with -ffp-contract=off).
 *
 * Paper passages followed (arxiv 2606.15991, "Fearless Concurrency on the
 * GPU"):
 *   - Sec. 3.6, Listing "GEMM using bounded output sub-tensor indices": each
 *     owned output tile starts from a zero accumulator, sums x-tile . y-tile
 *     products over the K tiles, and is stored once.  Summed over every
 *     tile that is exactly the plain definition R[i][j] = sum_k A[i][k] B[k][j],
 *     which is what oracle_gemm computes.
 *   - Sec. 3.4 (partitioning) and App. A (data-race freedom): the map from
 *     tile programs to output sub-tensors is injective and, with the
 *     partition grid derived from the partition shape, covering; an output
 *     may not alias an immutable input.  oracle_partition_paint checks this
 *     by painting every output element, the brute-force definition.
 *
 * Element formats decoded here (exact, from their published definitions):
 *   - bfloat16: the upper 16 bits of an IEEE binary32.
 *   - OCP 8-bit floating point E4M3 ("e4m3fn"): 1 sign bit, 4 exponent bits
 *     with bias 7, 3 mantissa bits; exponent field 0 is subnormal
 *     (m * 2^-9); S.1111.111 is NaN; there are no infinities; the largest
 *     finite magnitude is 448.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- formats */

double oracle_bf16_to_f64(uint16_t bits)
{
    uint32_t w = ((uint32_t)bits) << 16;
    float f;
    memcpy(&f, &w, sizeof f);
    return (double)f;
}

double oracle_e4m3fn_to_f64(uint8_t code)
{
    int sign = (code >> 7) & 1;
    int e = (code >> 3) & 0xF;
    int m = code & 0x7;
    double v;
    if (e == 0xF && m == 0x7)
        return NAN;
    if (e == 0)
        v = ldexp((double)m, -9);          /* subnormal: m/8 * 2^(1-7) */
    else
        v = ldexp(1.0 + m / 8.0, e - 7);   /* normal: (1 + m/8) * 2^(e-7) */
    return sign ? -v : v;
}

void oracle_decode_bf16(const uint16_t *src, double *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = oracle_bf16_to_f64(src[i]);
}

void oracle_decode_e4m3fn(const uint8_t *src, double *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = oracle_e4m3fn_to_f64(src[i]);
}

void oracle_decode_f32(const float *src, double *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = (double)src[i];
}

/* ------------------------------------------------------------------- GEMM */

/*
 * R[i][j] = sum_{k<K} A[i][k] * B(k, j)       (i < M, j < N)
 *
 * A is M x K row-major with leading dimension lda.
 * B(k, j) = B[k*ldb + j] when b_nk == 0 (B stored K x N row-major),
 *         = B[j*ldb + k] when b_nk != 0 (B stored N x K row-major, i.e. the
 *           weight layout of a decode matrix-vector product).
 * R is M x N row-major with leading dimension ldr.
 * The sum over k runs in increasing k, one product at a time.
 */
void oracle_gemm(int64_t M, int64_t N, int64_t K,
                 const double *A, int64_t lda,
                 const double *B, int64_t ldb, int b_nk,
                 double *R, int64_t ldr)
{
    int64_t i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            double s = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                double b = b_nk ? B[j * ldb + k] : B[k * ldb + j];
                s += A[i * lda + k] * b;
            }
            R[i * ldr + j] = s;
        }
    }
}

/*
 * Same contraction with per-row and per-column scale factors applied to the
 * finished sum:  R[i][j] = sa[i] * sb[j] * sum_k A[i][k] B(k, j).
 * sa == NULL or sb == NULL means all ones.  This is the definition of a
 * GEMM on quantised codes whose real values are code * scale.
 */
void oracle_gemm_scaled(int64_t M, int64_t N, int64_t K,
                        const double *A, int64_t lda,
                        const double *B, int64_t ldb, int b_nk,
                        const double *sa, const double *sb,
                        double *R, int64_t ldr)
{
    oracle_gemm(M, N, K, A, lda, B, ldb, b_nk, R, ldr);
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double s = 1.0;
            if (sa) s *= sa[i];
            if (sb) s *= sb[j];
            R[i * ldr + j] *= s;
        }
}

/*
 * Individual entries R[ii[t]][jj[t]] of the (scaled) product, for spot checks
 * of outputs too large for the full triple loop.
 */
void oracle_gemm_entries(int64_t K,
                         const double *A, int64_t lda,
                         const double *B, int64_t ldb, int b_nk,
                         const double *sa, const double *sb,
                         const int64_t *ii, const int64_t *jj, int64_t n,
                         double *out)
{
    int64_t t;
#pragma omp parallel for schedule(static)
    for (t = 0; t < n; ++t) {
        int64_t i = ii[t], j = jj[t];
        double s = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double b = b_nk ? B[j * ldb + k] : B[k * ldb + j];
            s += A[i * lda + k] * b;
        }
        if (sa) s *= sa[i];
        if (sb) s *= sb[j];
        out[t] = s;
    }
}

/*
 * Relative Frobenius error  ||C - R||_F / ||R||_F  accumulated in binary64.
 * When ||R||_F is zero the result is ||C||_F (absolute error).
 */
double oracle_rel_fro(const double *C, const double *R, int64_t n)
{
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = C[i] - R[i];
        num += d * d;
        den += R[i] * R[i];
    }
    if (den == 0.0)
        return sqrt(num);
    return sqrt(num / den);
}

/* -------------------------------------------------------------- partition */

enum {
    ORACLE_PART_OK = 0,
    ORACLE_PART_ARG = 1,
    ORACLE_PART_NOCOVER = 5,
    ORACLE_PART_OVERLAP = 4
};

/*
 * Paint every element of an M x N output with the number of tile programs
 * that own it.
 *
 * The output is split into bm x bn sub-tensors on a ceil(M/bm) x ceil(N/bn)
 * grid (edge sub-tensors clipped to the output).  Sub-tensor (tm, tn) has the
 * linear id tm * ceil(N/bn) + tn.  Program p owns the sub-tensors
 * prog_tiles[prog_offsets[p] .. prog_offsets[p+1]).  When n_prog == 0 (or the
 * tables are NULL) the plain one-program-per-sub-tensor grid is used.
 *
 * counts (M*N int32, row-major) receives the paint.  Returns
 * ORACLE_PART_OVERLAP if any element is owned twice, else ORACLE_PART_NOCOVER
 * if any element is owned by no program, else ORACLE_PART_OK.  A tile id
 * outside the grid, a negative count or bm/bn <= 0 gives ORACLE_PART_ARG.
 */
int oracle_partition_paint(int64_t M, int64_t N, int64_t bm, int64_t bn,
                           int64_t n_prog, const int32_t *prog_offsets,
                           const int32_t *prog_tiles, int32_t *counts)
{
    if (bm <= 0 || bn <= 0 || M < 0 || N < 0)
        return ORACLE_PART_ARG;
    int64_t tiles_m = (M + bm - 1) / bm, tiles_n = (N + bn - 1) / bn;
    int64_t n_tiles = tiles_m * tiles_n;
    memset(counts, 0, sizeof(int32_t) * (size_t)(M * N));

    int use_map = (n_prog > 0 && prog_offsets && prog_tiles);
    int64_t programs = use_map ? n_prog : n_tiles;
    for (int64_t p = 0; p < programs; ++p) {
        int64_t lo = use_map ? prog_offsets[p] : p;
        int64_t hi = use_map ? prog_offsets[p + 1] : p + 1;
        if (hi < lo)
            return ORACLE_PART_ARG;
        for (int64_t q = lo; q < hi; ++q) {
            int64_t t = use_map ? prog_tiles[q] : q;
            if (t < 0 || t >= n_tiles)
                return ORACLE_PART_ARG;
            int64_t tm = t / tiles_n, tn = t % tiles_n;
            for (int64_t i = tm * bm; i < tm * bm + bm && i < M; ++i)
                for (int64_t j = tn * bn; j < tn * bn + bn && j < N; ++j)
                    counts[i * N + j] += 1;
        }
    }
    int over = 0, hole = 0;
    for (int64_t e = 0; e < M * N; ++e) {
        if (counts[e] > 1) over = 1;
        if (counts[e] == 0) hole = 1;
    }
    if (over) return ORACLE_PART_OVERLAP;
    if (hole) return ORACLE_PART_NOCOVER;
    return ORACLE_PART_OK;
}

/*
 * Byte-range intersection test: do [a, a+na) and [b, b+nb) share a byte?
 * The ranges are those a row-major matrix covers: base .. base +
 * ((rows-1)*ld + cols) * element_size.  Used by the tests to state the
 * aliasing rule (an output may not share memory with an input) from its
 * definition.
 */
int oracle_ranges_intersect(uint64_t a, uint64_t na, uint64_t b, uint64_t nb)
{
    if (na == 0 || nb == 0)
        return 0;
    return a < b + nb && b < a + na;
}

/* ------------------------------------------------------------- threads */

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
