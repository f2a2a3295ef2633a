/*
 * tilegemm.h -- C ABI of the MI355X (gfx950) tile-partitioned GEMM library.
 *
 * The library computes C = A . B with the tile model of arxiv 2606.15991
 * ("Fearless Concurrency on the GPU"):
 *   - the mutable output C is split, before launch, into disjoint BM x BN
 *     sub-tensors (Sec. 3.4, "Partitioning and Ordering");
 *   - a grid of tile programs is derived from that partition; with the
 *     persistent ("mapped partition") schedule of Sec. 3.6 each program owns
 *     a bounded sequence of sub-tensors, the program -> sub-tensor map is
 *     injective, and a program stores only into the sub-tensors it owns;
 *   - the inputs A and B are shared, immutable and never written
 *     (the &Tensor parameters of the launch-boundary type grammar, Sec. 3.1);
 *   - every owned sub-tensor starts from a zero accumulator, sums tile
 *     products over K, and is stored exactly once (Listing "GEMM using
 *     bounded output sub-tensor indices", Sec. 3.6).
 *
 * Conventions shared by every call:
 *   - Matrices are row-major with a leading dimension `ld` (elements between
 *     the starts of consecutive rows, ld >= cols).  A matrix occupies the
 *     bytes [data, data + ((rows-1)*ld + cols) * element_size).
 *   - Pointers named "device" are HIP device pointers (hipMalloc or
 *     torch.cuda memory); "host" pointers are ordinary process memory.
 *   - Ownership (Sec. 3.3, prepare/recover protocol): the library never
 *     frees, retains or reallocates a caller pointer.  Inputs are borrowed
 *     read-only.  Outputs, scales and workspaces are exclusively borrowed
 *     from the call until `stream` reaches the end of the enqueued work; the
 *     caller must not read, write or free them before synchronising that
 *     stream (the unsafe-while-in-flight rule of Sec. 3.2).
 *   - Errors: every argument is validated on the host before anything is
 *     enqueued.  On any error status nothing has been enqueued and outputs
 *     are untouched.  tg_last_error() returns a thread-local message for the
 *     last failing call.  Asynchronous device faults surface at the caller's
 *     stream synchronisation, not through these calls.
 *   - No launch call allocates device memory or synchronises the stream, so
 *     every launch call may be captured into a HIP graph (graph nodes must
 *     be non-allocating, Sec. 3.2 "CUDA graphs").
 */
#ifndef TILEGEMM_H
#define TILEGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A hipStream_t; 0 is the legacy default stream. */
typedef void *tg_stream;

typedef enum tg_status {
    TG_OK = 0,
    TG_E_ARG = 1,         /* NULL pointer, non-positive size, bad enum value */
    TG_E_DTYPE = 2,       /* dtype combination not provided                  */
    TG_E_SHAPE = 3,       /* A.cols != K, C not M x N, ld < cols, ...        */
    TG_E_OVERLAP = 4,     /* a sub-tensor owned by two programs, or two
                             outputs of one launch share bytes               */
    TG_E_NOCOVER = 5,     /* a sub-tensor of the grid is owned by nobody     */
    TG_E_ALIAS = 6,       /* an output shares bytes with an input            */
    TG_E_WORKSPACE = 7,   /* workspace missing, too small or misaligned      */
    TG_E_UNSUPPORTED = 8, /* valid request with no kernel (e.g. a config
                             that is not instantiated, misaligned vectors)  */
    TG_E_HIP = 9          /* the HIP runtime reported an error              */
} tg_status;

typedef enum tg_dtype {
    TG_F32 = 0,           /* IEEE binary32                                   */
    TG_BF16 = 1,          /* bfloat16                                        */
    TG_FP8_E4M3 = 2       /* OCP FP8 E4M3 ("e4m3fn", max 448, no inf)        */
} tg_dtype;

/* Arithmetic of the contraction.  Accumulation is always binary32. */
typedef enum tg_precision {
    TG_PREC_NATIVE = 0,   /* the operands' own type on the matrix cores      */
    TG_PREC_BF16X3 = 1,   /* f32 operands split a = hi + mid (+ rest) into
                             bf16 planes; 3 products hi.hi + hi.mid + mid.hi */
    TG_PREC_BF16X6 = 2    /* 3-way split hi + mid + lo; 6 products hi.hi,
                             hi.mid, mid.hi, hi.lo, lo.hi, mid.mid           */
} tg_precision;

/*
 * Immutable input (a shared read-only tensor).  The descriptor names the
 * stored matrix: `rows` x `cols` row-major with leading dimension `ld`.
 * `trans` = 1 declares that the logical operand is the transpose of the
 * stored matrix (B stored N x K, the weight layout of a decode product);
 * only B may be transposed.
 */
typedef struct tg_in {
    const void *data;     /* device pointer                                  */
    int32_t dtype;        /* tg_dtype                                        */
    int32_t trans;        /* 0 or 1                                          */
    int64_t rows, cols, ld;
} tg_in;

/*
 * Mutable output C (M x N row-major, leading dimension ld) together with its
 * partition shape bm x bn: the output is split into ceil(M/bm) x ceil(N/bn)
 * sub-tensors (edge sub-tensors clipped to the matrix) and each sub-tensor is
 * owned by exactly one tile program.  bm = bn = 0 asks tile_gemm to choose
 * the partition (the tile configuration picker); the chosen shape is
 * written back into the descriptor.
 */
typedef struct tg_out {
    void *data;           /* device pointer                                  */
    int32_t dtype;        /* TG_F32 or TG_BF16 (round to nearest even)       */
    int32_t reserved;
    int64_t rows, cols, ld;
    int32_t bm, bn;
} tg_out;

/*
 * Kernel configuration.  bm x bn must equal the output partition; bk is the
 * K-tile depth; wm x wn is the wavefront grid of one workgroup; stages is
 * the number of K tiles held in LDS at once; sched is the wavefront
 * schedule of the tiled kernel; `kind` selects the kernel family.  Unset
 * fields (0) are filled by the picker.
 */
typedef enum tg_kind {
    TG_KIND_AUTO = 0,
    TG_KIND_TILED = 1,    /* LDS double-buffered MFMA tile program           */
    TG_KIND_SKINNY = 2,   /* decode-shaped (M <= 16) streaming product       */
    TG_KIND_SIMPLE = 3    /* small-tile kernel with no alignment demands     */
} tg_kind;

typedef enum tg_sched {
    TG_SCHED_ANY = 0,
    TG_SCHED_LOCKSTEP = 1, /* all wavefronts load, then all contract         */
    TG_SCHED_PINGPONG = 2, /* two wavefront groups alternate between loading
                              and contracting, one phase apart; needs K a
                              multiple of 16 bytes of the operand type      */
    TG_SCHED_CROSS = 3,    /* lock-step with the hand-over barrier of the
                              next K tile placed before the last K step of
                              the current one (bf16); the default for B
                              stored N x K                                  */
    TG_SCHED_STAGED = 4,   /* four wavefronts of 128 x 128 outputs; each K
                              tile read from HBM into registers two tiles
                              ahead and stored into a two-stage LDS ring
                              (bf16, B stored N x K, binary32 output, no
                              scales, K a multiple of 64)                   */
    TG_SCHED_BULK = 5,     /* four wavefronts of 128 x 128 outputs (or
                              eight of 128 x 64); each K
                              tile's fragments read from LDS into registers
                              in one burst a tile period ahead, freeing its
                              stage for loads NS - 1 tiles ahead (bf16, B
                              stored N x K, K a multiple of 32)             */
    TG_SCHED_CROSS_WARM = 6 /* the cross-tile schedule (two stages, B stored
                              N x K, bf16) touching the L2 lines of the K
                              tile two tiles beyond the one being loaded,
                              so that its direct loads hit the L2 where the
                              operands stream from HBM (long K)             */
} tg_sched;

typedef struct tg_config {
    int32_t kind;         /* tg_kind                                         */
    int32_t bm, bn, bk;
    int32_t wm, wn;
    int32_t ksplit;       /* skinny kernel: wavefronts sharing one tile's K  */
    int32_t stages;       /* tiled kernel: LDS stages of the K-tile ring;
                             with TG_SCHED_CROSS, 3 means five slots of one
                             operand tile each (A or B of a K tile)         */
    int32_t sched;        /* tiled kernel: tg_sched                          */
    int32_t splitk;       /* skinny kernel: programs sharing one sub-tensor's
                             K (1..TG_MAX_SPLITK).  With splitk > 1 each
                             stores its partial tile into a workspace
                             partitioned by (split, sub-tensor) and a second
                             launch, one program per sub-tensor of C, sums
                             them in split order: deterministic, needs a
                             workspace (tile_gemm_workspace_size).  The
                             value is normalised to the splits that get K
                             steps.                                         */
} tg_config;

#define TG_MAX_SPLITK 16

typedef struct tg_opts {
    int32_t precision;    /* tg_precision                                    */
    int32_t checked;      /* 1: run tile_partition_check's rules before the
                             launch (the default); 0: skip them (the
                             unchecked twin used to measure their cost)      */
    const float *scale_a; /* device, M floats or NULL (all ones): row scales */
    const float *scale_b; /* device, N floats or NULL: output-column scales  */
    const tg_config *config; /* host; NULL -> picker                         */
    void *workspace;      /* device, 16-byte aligned; needed by
                             TG_PREC_BF16X3/X6 and by decode products split
                             over programs along K (splitk > 1)             */
    size_t workspace_bytes;
    int32_t *write_count; /* device, M*N int32 (row-major, ld N) or NULL: each
                             store adds 1 to its element's counter, so a
                             correct launch leaves every counter at 1 more
                             than the caller's initial value               */
    const tg_in *residual; /* host descriptor of a device M x N residual R
                             (bf16 or f32, row-major, trans 0), or NULL.
                             Decode products (TG_KIND_SKINNY, and
                             tile_rms_norm_matvec) then store C = (product)
                             + R, the binary32 sum rounded once to C's type:
                             the residual add of the decode layer (Sec. 3.2,
                             graph-scope listing) done by the program that
                             owns each element of C.  R is an immutable
                             input: sharing bytes with C is TG_E_ALIAS (on
                             checked launches; with a split over programs
                             the workspace may not share bytes with it
                             either).  Other kernel kinds return
                             TG_E_UNSUPPORTED.                             */
} tg_opts;

/*
 * tile_partition_check -- the host-side ownership rules of Sec. 3.4 and the
 * data-race-freedom argument of App. A.
 *
 *   ins[0..n_in)   immutable inputs (host array of descriptors)
 *   out            the mutable output with its partition bm x bn
 *   n_prog, prog_offsets[n_prog+1], prog_tiles[...]  optional program map
 *                  (host arrays): program p owns the sub-tensors with linear
 *                  ids prog_tiles[prog_offsets[p] .. prog_offsets[p+1]), where
 *                  sub-tensor (tm, tn) has id tm * ceil(N/bn) + tn.  With
 *                  n_prog == 0 the one-program-per-sub-tensor grid is checked.
 *
 * Returns TG_E_ARG (NULL descriptor or data, bm/bn <= 0, negative sizes, a
 * tile id off the grid), TG_E_SHAPE (ld < cols), TG_E_OVERLAP (a sub-tensor
 * owned twice), TG_E_NOCOVER (a sub-tensor owned by nobody), TG_E_ALIAS (the
 * output's byte range intersects an input's), else TG_OK.  Pure host code:
 * no HIP call is made.
 */
tg_status tile_partition_check(const tg_in *ins, int32_t n_in,
                               const tg_out *out, int32_t n_prog,
                               const int32_t *prog_offsets,
                               const int32_t *prog_tiles);

/*
 * tile_gemm -- C = diag(scale_a) . A . B . diag(scale_b), one launch of tile
 * programs over the partition of C (Sec. 3.6; the decode-shaped product is
 * the matvec of the decode layer in Sec. 3.2's graph-scope listing, bound
 * by the weight stream as in the roofline of Sec. 5.3).
 *
 *   A  M x K (trans must be 0), B  K x N (or stored N x K with trans = 1),
 *   C  M x N with partition bm x bn.
 *   dtypes: A, B both TG_F32, both TG_BF16 or both TG_FP8_E4M3; or
 *   A TG_BF16 with B TG_FP8_E4M3 (weight-only FP8: B is decoded exactly to
 *   bf16 before the contraction).  C is TG_F32 or TG_BF16.
 *   opts may be NULL (native precision, checked, picker).  Precision modes
 *   BF16X3/X6 need f32 A and B and a workspace of
 *   tile_gemm_workspace_size() bytes.  Decode products (M <= 16, B stored
 *   N x K) own sub-tensors of 16 rows x 1..32 columns.  By default the
 *   width deals N evenly over the compute units with no K split where it
 *   can: N / (the compute units) columns where that is 8..32 (half of it,
 *   two programs per compute unit, for bf16 weights with up to four rows
 *   and K <= 8192 when it exceeds 16), or, over several rounds with more
 *   than four rows, an even width of single-wavefront programs all
 *   resident at once; otherwise 16 or 32 columns, and K may be split
 *   over several programs per sub-tensor: an explicit config with
 *   splitk > 1 needs a workspace of tile_gemm_workspace_size() bytes
 *   (TG_E_WORKSPACE without one); the default configuration splits only
 *   when opts carries a workspace that large.  The workspace may not
 *   share bytes with A, B or C (TG_E_ALIAS).
 *   K == 0 stores zeros.  M == 0 or N == 0 enqueues nothing.
 *
 * Every output element is stored exactly once, by the program that owns its
 * sub-tensor; nothing is read from C.
 */
tg_status tile_gemm(const tg_in *A, const tg_in *B, tg_out *C,
                    const tg_opts *opts, tg_stream stream);

/* Workspace bytes tile_gemm needs for these arguments: for opts->config
 * when it is set, else for the configuration tile_gemm chooses when a
 * workspace is supplied (0 when nothing needs one). */
size_t tile_gemm_workspace_size(const tg_in *A, const tg_in *B,
                                const tg_out *C, const tg_opts *opts);

/*
 * tile_gemm_noalloc -- tile_gemm for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Arguments, results and errors as tile_gemm, except
 * that opts->workspace must be NULL (TG_E_ARG otherwise): wherever tile_gemm
 * takes a workspace (BF16X3/X6 planes, a decode product split over programs
 * along K) this call uses a scratch array of TG_NOALLOC_SCRATCH_BYTES that
 * the library holds in each device's memory from its first use until the
 * process ends.  A request whose workspace exceeds it fails with
 * TG_E_WORKSPACE before anything is enqueued (the default decode split is
 * reduced to fit).  Nothing in the scratch needs clearing: every byte a
 * launch reads was written earlier by the same call.  All calls on one
 * device share its scratch, so calls that overlap on one device (different
 * streams, or host threads) race: serialise them.  No allocation, no
 * synchronisation; the first call on a device resolves the scratch's
 * address (a host-side query).
 */
#define TG_NOALLOC_SCRATCH_BYTES (8u << 20)
tg_status tile_gemm_noalloc(const tg_in *A, const tg_in *B, tg_out *C,
                            const tg_opts *opts, tg_stream stream);

/*
 * tile_gemm_plan -- the configuration and program map tile_gemm would use
 * for these arguments, without launching: the host-side derivation of the
 * launch grid from the output partition (Sec. 3.4) and the mapped
 * partition's program -> sub-tensor map (Sec. 3.6), exported so that the
 * ownership rules of App. A can be checked on the very map that runs.  cfg (host) receives the chosen
 * configuration and *n_prog the number of tile programs.  When prog_offsets
 * (n_prog+1 ints) and prog_tiles (ceil(M/bm)*ceil(N/bn) ints) are non-NULL
 * they receive the program -> sub-tensor map, in the format
 * tile_partition_check accepts.  Call once with NULL tables to size them.
 * The plan is the one for a caller supplying opts->workspace_bytes of
 * workspace (the default decode split is reduced to fit it).
 */
tg_status tile_gemm_plan(const tg_in *A, const tg_in *B, const tg_out *C,
                         const tg_opts *opts, tg_config *cfg,
                         int32_t *n_prog, int32_t *prog_offsets,
                         int32_t *prog_tiles);

/*
 * Grouped GEMM: n independent problems C_i = A_i . B_i in ONE persistent
 * launch whose programs walk the concatenated sub-tensor lists of all
 * problems: the mapped-partition schedule of Sec. 3.6 applied across
 * problems, the batched counterpart of the launch-overhead study of
 * Sec. 5.2 and of the GEMM queue of App. B.
 *
 * tile_gemm_grouped_prepare validates every problem (each with the rules of
 * tile_gemm, plus: no two outputs may share bytes, and no output may share
 * bytes with any input of the launch), picks ONE tile configuration for the
 * launch (opts->config when given, else 256 x 256 sub-tensors for large
 * batches and 128 x 128 for small ones; every problem's partition is
 * written back into C[i].bm / C[i].bn), writes the problem table into the
 * caller's device workspace (tile_gemm_grouped_workspace_size(n) bytes,
 * 16-byte aligned) with a copy on `stream` that has completed when prepare
 * returns, and fills the caller's host plan with the launch parameters.
 * Not capturable.  Supported: bf16 A and B, one B layout and one C dtype
 * (f32 or bf16) for all problems, native precision, no scales.
 * opts->write_count (device, or NULL) holds sum_i M_i * N_i int32
 * counters, problem i's block (row-major, leading dimension N_i) after
 * those of problems 0 .. i-1; each store adds 1 to its element's counter.
 *
 * tile_gemm_grouped enqueues the single launch described by the plan (which
 * names its workspace); it allocates nothing and does not synchronise, so
 * it may be captured into a HIP graph and replayed.  Pointers inside the
 * table are those given to prepare; replays recompute the same outputs.
 * The plan is the caller's: the library keeps nothing between the calls.
 * A plan that prepare did not fill (or that was altered) gives TG_E_ARG.
 */
typedef struct tg_grouped_plan {
    const void *workspace; /* device table the plan describes              */
    int32_t n;             /* problems                                     */
    int32_t total_tiles;   /* sub-tensors of all problems                  */
    int32_t n_prog;        /* persistent programs of the launch            */
    int32_t variant;       /* kernel instantiation (library-internal)      */
    uint64_t tag;          /* consistency tag over the fields above        */
} tg_grouped_plan;

size_t tile_gemm_grouped_workspace_size(int32_t n);
tg_status tile_gemm_grouped_prepare(int32_t n, const tg_in *A,
                                    const tg_in *B, tg_out *C,
                                    const tg_opts *opts, void *workspace,
                                    size_t workspace_bytes,
                                    tg_grouped_plan *plan, tg_stream stream);
tg_status tile_gemm_grouped(const tg_grouped_plan *plan, tg_stream stream);

/*
 * tile_add -- z = x + y element by element (Sec. 2, the add of the first
 * listing, measured element-wise in Sec. 5.1), over z's bm x bn partition:
 * each tile program stores only into the sub-tensors it owns, x and y are
 * shared reads.
 * x, y, z: device, one shape (rows x cols, row stride ld), one dtype
 * (TG_BF16 or TG_F32), not transposed.  Each element is added in binary32
 * and rounded once to the dtype (round to nearest even), which for bf16 is
 * the correctly rounded sum.  z->bm = z->bn = 0 selects 1 x 65536
 * sub-tensors (written back into *z).  opts may be NULL; its checked flag
 * (default on) runs tile_partition_check's rules with x and y as inputs,
 * so z may not share bytes with either; opts->write_count counts stores.
 * Errors: TG_E_ARG / TG_E_SHAPE / TG_E_DTYPE before anything is enqueued;
 * TG_E_HIP for a failed launch.  z is exclusively borrowed until the
 * stream passes the launch.
 */
tg_status tile_add(const tg_in *x, const tg_in *y, tg_out *z,
                   const tg_opts *opts, tg_stream stream);

/*
 * tile_mul -- z = x * y element by element: the element-wise kernel of the
 * execution-mode measurement of Sec. 5.2 (y = x . g over one tile).
 * Arguments, partition, checks, errors and ownership as tile_add.  Each
 * product is formed in binary32 and rounded once to the dtype: for TG_F32
 * and for bf16 products of magnitude >= 2^-126 that is the correctly
 * rounded product; smaller bf16 products are rounded first to the binary32
 * subnormal grid (2^-149), then to bf16 (error <= 2^-133, one bf16
 * subnormal step, instead of 2^-134).
 */
tg_status tile_mul(const tg_in *x, const tg_in *y, tg_out *z,
                   const tg_opts *opts, tg_stream stream);

/*
 * tile_rms_norm -- y = x * w / sqrt(mean(x^2) + eps) row by row: the RMS
 * normalisation that opens the decode layer of Sec. 3.2's graph-scope
 * listing (partitioned [1, d]: each program owns whole rows).
 * x, y: device, rows x cols (row stride ld); w: device, 1 x cols; one dtype
 * (TG_BF16 or TG_F32), not transposed.  Sums of squares in binary32 in a
 * fixed order (deterministic); each output x * scale * w is computed in
 * binary32 and rounded once to the dtype.  eps: finite, >= 0.
 * y->bm x y->bn is the partition; bn must equal cols; 0 x 0 selects
 * 1 x cols (written back into *y).  opts may be NULL; its checked flag
 * (default on) applies tile_partition_check's rules with x and w as inputs;
 * opts->write_count counts stores.
 * Errors: TG_E_ARG / TG_E_SHAPE / TG_E_DTYPE before anything is enqueued;
 * TG_E_HIP for a failed launch.  y is exclusively borrowed until the stream
 * passes the launch.
 */
tg_status tile_rms_norm(const tg_in *x, const tg_in *w, float eps, tg_out *y,
                        const tg_opts *opts, tg_stream stream);

/*
 * tile_rms_norm_matvec -- the decode layer's normalisation fused into its
 * product (Sec. 3.2, graph-scope listing: rms_norm then matvec):
 * y = diag(1 / sqrt(mean_k x[m,k]^2 + eps)) . (x * nw) . W^T for M <= 16
 * activation rows.  x: device bf16 M x K; nw: device bf16 1 x K
 * normalisation weights, 16-byte aligned; W: device, stored N x K
 * (trans = 1), bf16 or E4M3 (then opts->scale_b holds its N row scales);
 * y: device M x N, f32 or bf16, partition chosen by the decode kernel
 * (16 x 16 or 16 x 32, written back into *y).  Each x * nw is rounded to
 * bf16 before the contraction; sums of squares and the product accumulate
 * in binary32; the row scale multiplies the binary32 sum.  opts may be NULL;
 * precision and config must be unset.  With opts->workspace (16-byte
 * aligned, tile_rms_norm_matvec_workspace_size bytes, sharing no bytes with
 * x, nw, W or y) the K steps are split over several programs per
 * sub-tensor where that gives the chip more programs; their partial tiles
 * and partial sums of squares go to the workspace and a second launch sums
 * them in split order (deterministic).  Without a workspace K is not split
 * across programs.  Errors as tile_gemm, before anything is enqueued.  y
 * and the workspace are exclusively borrowed until the stream passes the
 * launch.
 */
tg_status tile_rms_norm_matvec(const tg_in *x, const tg_in *nw, float eps,
                               const tg_in *W, tg_out *y, const tg_opts *opts,
                               tg_stream stream);

/* Workspace bytes tile_rms_norm_matvec uses when given one (0: it never
 * splits these arguments).  x, W, y as for tile_rms_norm_matvec. */
size_t tile_rms_norm_matvec_workspace_size(const tg_in *x, const tg_in *W,
                                           const tg_out *y);

/*
 * tile_error_norm -- binary64 reductions for the relative Frobenius error of
 * a result against a binary64 reference, on the GPU (the correctness check
 * that accompanies the GEMM measurement of Sec. 5.1; the paper states its
 * results against a reference without fixing the norm, the relative
 * Frobenius norm is the reading):
 *   out[0] = sum (C[i] - R[i])^2,  out[1] = sum R[i]^2   over i < n
 * C: device, n elements of c_dtype (TG_F32 or TG_BF16), read as a dense
 * array (pass matrices with ld == cols); R: device, n binary64 values.
 * out: device, TG_ERROR_NORM_DOUBLES doubles, all overwritten (entries past
 * the first two hold per-workgroup partial sums).  The summation order is
 * fixed, so repeated calls give identical results.
 */
#define TG_ERROR_NORM_DOUBLES 514
tg_status tile_error_norm(const void *C, int32_t c_dtype, const double *R,
                          int64_t n, double *out, tg_stream stream);

/* ------------------------------------------------------------------------
 * Configuration choice.  The tile shapes of the paper's evaluation are tuned
 * once per problem size (Sec. 5.1); here an exhaustive autotuner times every
 * candidate configuration, a cache keeps the winners, and a learned cost
 * model (an MLP trained on the autotuner's timings by the kernels below)
 * picks configurations for shapes that were never tuned.  tile_gemm with no
 * configuration and no partition uses, in order: the tuning cache, the
 * picker's argmin over tile_gemm_candidates, the fixed default heuristic
 * (tile_picker_mode selects which of the first two are enabled).
 * ---------------------------------------------------------------------- */

/*
 * tile_gemm_candidates -- the configurations the autotuner and the picker
 * choose among for these arguments (honouring C's partition when it is
 * set): every tiled instantiation tile_gemm accepts, and for decode
 * products 16- and 32-column programs plus the width that deals N evenly
 * over whole rounds of the compute units, each with its wavefront counts
 * and K splits.  Writes up to `max` into `out` (host) and returns the total
 * count, or -1 on invalid arguments.  Host only.
 */
int32_t tile_gemm_candidates(const tg_in *A, const tg_in *B, const tg_out *C,
                             const tg_opts *opts, tg_config *out, int32_t max);

typedef struct tg_tune_result {
    tg_config cfg;
    float ms;             /* average launch time, or -1 when it failed       */
    int32_t status;       /* tg_status of the launches                       */
} tg_tune_result;

/*
 * tile_autotune -- run every candidate once (warm-up) then `reps` times on
 * `stream`, timed with HIP events, and record the fastest in the tuning
 * cache.  C is written (any candidate's result).  results (host, up to
 * max_results entries) and best (host) may be NULL.  Synchronises the
 * stream: not capturable.
 */
tg_status tile_autotune(const tg_in *A, const tg_in *B, tg_out *C,
                        const tg_opts *opts, int32_t reps,
                        tg_tune_result *results, int32_t max_results,
                        int32_t *n_results, tg_config *best, tg_stream stream);

/*
 * tile_autotune_grouped -- the autotuner for one grouped launch: every tiled
 * configuration the launch can run (bf16, the problems' B layout and C
 * type) is prepared into `workspace`, launched once (warm-up) and then
 * `reps` times on `stream`, timed with HIP events; the workspace and *plan
 * are left prepared with the fastest, which *best receives (host, may be
 * NULL), and C[i].bm / C[i].bn hold its partition.  Arguments as for
 * tile_gemm_grouped_prepare, whose opts->config it ignores (and whose
 * opts->write_count it does not apply while timing).  Outputs are written
 * (any candidate's results).  Synchronises the stream: not capturable.
 */
tg_status tile_autotune_grouped(int32_t n, const tg_in *A, const tg_in *B,
                                tg_out *C, const tg_opts *opts,
                                void *workspace, size_t workspace_bytes,
                                int32_t reps, tg_tune_result *results,
                                int32_t max_results, int32_t *n_results,
                                tg_config *best, tg_grouped_plan *plan,
                                tg_stream stream);

/* Tuning cache: clear, count, save to / merge from a text file (host). */
tg_status tile_tune_cache_clear(void);
int32_t tile_tune_cache_size(void);
tg_status tile_tune_cache_save(const char *path);
tg_status tile_tune_cache_load(const char *path);

/*
 * Picker.  TG_PICKER_FEATURES numbers describe a (request, configuration)
 * pair, in this order: log2 M, N, K; flags for e4m3 operands, f32 operands,
 * B stored N x K and a bf16 output; the kernel kind (three one-hot flags:
 * tiled, skinny, simple); log2 bm, bn, wavefronts per program, LDS stages
 * and ksplit; log2 of the sub-tensor count, of the program count and of
 * the sub-tensors per program; the fraction of the last round of
 * sub-tensors that has work; the useful fraction of the padded output
 * area; a flag for the ping-pong schedule; 1 for the cross-tile schedule,
 * 2 for the cross-tile schedule with the L2 warm-up, else 0; log2 splitk;
 * a flag for the configuration the fixed heuristic would pick.
 * tile_picker_set installs a cost model (host copy of the parameters in the
 * layout of tile_mlp_*, with per-feature mean and standard deviation used
 * to normalise the features); params == NULL removes it.
 * tile_picker_mode(mode) sets bit 1 = use the tuning cache, bit 2 = use the
 * cost model (mode < 0 only queries) and returns the previous mode.
 */
#define TG_PICKER_FEATURES 24
tg_status tile_picker_features(const tg_in *A, const tg_in *B,
                               const tg_out *C, const tg_config *cfg,
                               float *feat);
tg_status tile_picker_set(const float *params, int32_t n_in, int32_t hidden,
                          int32_t depth, const float *feat_mean,
                          const float *feat_std);
tg_status tile_picker_predict(const float *feat, float *log_ms);
int32_t tile_picker_mode(int32_t mode);

/*
 * Cost-model MLP on the GPU: `depth` hidden ReLU layers of `hidden` units and
 * one linear output.  Parameters (device, binary32), per layer: W (out x in,
 * row-major) then b (out); the output layer has out = 1.  X is batch x n_in
 * row-major (device), y and out are batch values (device).
 *   tile_mlp_forward:   out = MLP(X)
 *   tile_mlp_loss_grad: loss (device, 1 value) = mean (MLP(X) - y)^2 and
 *                       grads (device, same layout as params) = dloss/dparams
 *   tile_mlp_adam:      one Adam step (Kingma & Ba) at step t >= 1 on n
 *                       parameters with moment buffers m, v (device); the
 *                       hyper-parameters are binary64 so that 1 - beta and
 *                       the bias corrections are formed before any rounding
 *                       to binary32
 * ws (device) holds activations: tile_mlp_workspace_bytes bytes.  All
 * reductions run in a fixed order: repeated calls give identical results.
 */
size_t tile_mlp_param_count(int32_t n_in, int32_t hidden, int32_t depth);
size_t tile_mlp_workspace_bytes(int32_t n_in, int32_t hidden, int32_t depth,
                                int32_t batch);
tg_status tile_mlp_forward(const float *params, int32_t n_in, int32_t hidden,
                           int32_t depth, const float *X, int32_t batch,
                           float *out, void *ws, size_t ws_bytes,
                           tg_stream stream);
tg_status tile_mlp_loss_grad(const float *params, int32_t n_in,
                             int32_t hidden, int32_t depth, const float *X,
                             const float *y, int32_t batch, float *grads,
                             float *loss, void *ws, size_t ws_bytes,
                             tg_stream stream);
tg_status tile_mlp_adam(float *params, const float *grads, float *m, float *v,
                        int64_t n, double lr, double beta1, double beta2,
                        double eps, int32_t t, tg_stream stream);

const char *tg_status_str(int32_t status);
const char *tg_last_error(void);

/* Number of compute units of the current device (0 if unknown). */
int32_t tg_device_cus(void);

#ifdef __cplusplus
}
#endif

#endif /* TILEGEMM_H */
