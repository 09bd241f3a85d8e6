/*
 * fmm.h -- C ABI of the MI355X recursive fast matrix multiplication library.
 *
 * The library computes C = A * B by L recursive steps of a bilinear base case
 * <M,K,N;R> given by factor matrices [[U,V,W]] (Benson and Ballard, "A
 * Framework for Practical Parallel Fast Matrix Multiplication", PPoPP 2015,
 * Section 2.2, Equations (1) and (2)).  One step splits A into M x K blocks
 * and B into K x N blocks, forms S_r = sum_i U[i][r] A_i and
 * T_r = sum_j V[j][r] B_j, multiplies M_r = S_r T_r (recursively, or with a
 * classical leaf GEMM) and writes C_k = sum_r W[k][r] M_r (Section 3.1).
 *
 * Conventions for every entry point:
 *  - Matrices are row-major.  A is m x k with leading dimension lda >= k,
 *    B is k x n with ldb >= n, C is m x n with ldc >= n (elements).
 *  - FMM_F64 takes double* A, B, C.  FMM_F32 and FMM_F32_BF16X3 take float*.
 *  - Device pointers.  The caller owns A, B and C; C must not overlap A or B.
 *  - C is overwritten (C = A*B; there is no alpha/beta).
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *    Work is only enqueued: calls return before the GPU finishes.
 *  - Errors are reported by status code; no C++ exception crosses the ABI.
 *    fmm_last_error() returns a message for the calling thread's last error.
 *  - A size of zero (m, k or n) is a valid no-op (with k == 0, C is zeroed).
 *  - Leading dimensions must be below 2^21 elements (FMM_EUNSUPPORTED otherwise):
 *    the leaf kernels address a 128-row tile with 32-bit byte offsets.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan_s *fmm_plan_t;

typedef enum {
    FMM_OK = 0,
    FMM_EINVAL = 1,        /* bad argument: negative size, ld too small, NULL pointer,
                              overlapping C, depth that leaves a leaf dimension < 1 */
    FMM_ENOMEM = 2,        /* workspace beyond the budget, or device allocation failed */
    FMM_EHIP = 3,          /* a HIP runtime or launch failure (message has the HIP error) */
    FMM_EUNSUPPORTED = 4,  /* dtype / option not compiled into this library */
    FMM_EALG = 5           /* unknown algorithm, or a table that fails the Brent check */
} fmm_status;

typedef enum {
    FMM_F64 = 0,           /* binary64 end to end: FP64 additions, FP64 MFMA leaves */
    FMM_F32 = 1,           /* binary32 in/out: FP64-accumulated additions rounded to FP32,
                              FP32 MFMA leaves, FP64 W-combination */
    FMM_F32_BF16X3 = 2     /* binary32 in/out: as FMM_F32, but each leaf product is
                              hi*hi + hi*lo + lo*hi of bf16 splits (FP32 accumulate) */
} fmm_dtype;

/* Stages of one multiply, in execution order (for fmm_run_stage and timing). */
typedef enum {
    FMM_STAGE_FORM_S = 0,  /* S operands from A (Section 3.1, first bullet; 3.2 streaming);
                              for pair_form plans (fmm_plan_info_t) also the T operands */
    FMM_STAGE_FORM_T = 1,  /* T operands from B (nothing for pair_form plans) */
    FMM_STAGE_LEAF = 2,    /* grouped leaf GEMMs M_rho = alpha S_rho T_rho, plus peel strips */
    FMM_STAGE_COMBINE = 3, /* C blocks from the M_rho by W (Section 3.1, third bullet) */
    FMM_NUM_STAGES = 4
} fmm_stage;

/* Operand location codes returned by fmm_plan_operand. */
typedef enum { FMM_LOC_A = 0, FMM_LOC_B = 1, FMM_LOC_C = 2, FMM_LOC_WORKSPACE = 3 } fmm_loc;

typedef struct {
    int64_t m, k, n;             /* problem */
    int levels, dtype;
    int M, K, N, R;              /* base case */
    int64_t m0, k0, n0;          /* core multiple of M^L, K^L, N^L (static peel, Section 3.5) */
    int64_t leaf_m, leaf_k, leaf_n;
    int64_t num_leaves;          /* R^L */
    int64_t num_s_materialized;  /* leaf S operands written to the workspace (the rest are
                                    scaled views of A: single-non-zero columns, Section 3.1) */
    int64_t num_t_materialized;
    int64_t num_gemm_problems;   /* leaves plus peel problems in the grouped launch */
    int64_t gemm_tiles;          /* output tiles of the grouped launch */
    size_t workspace_bytes;
    double leaf_flops;           /* 2 * sum over GEMM problems of m*n*k */
    double classical_flops;      /* 2 m k n, the effective-flop numerator */
    double add_bytes;            /* algorithmic bytes moved by the S, T and W stages */
    double gemm_min_bytes;       /* bytes the leaf stage must read and write at least once */
    int fuse_levels;             /* recursion levels formed / combined per addition pass */
    char alg[80];                /* base case planned ("classical" for a plain GEMM), or one
                                    per level joined by '+'; for "auto" the model's choice */
    int leaf_tile;               /* leaf tile edge asked for (64 / 128), 0: chosen per launch */
    int pair_form;               /* non-zero: S and T are formed by one launch, in the
                                    FMM_STAGE_FORM_S stage (one-level plans of at most 2^20
                                    formation positions, FP64 / FP32); FMM_STAGE_FORM_T then
                                    enqueues nothing */
    double error_bound;          /* predicted bound on the relative Frobenius error of C
                                    against the exact product: e0 * prod over the levels of the
                                    base case's error growth g, e0 = c + (2 + sqrt(k)) u, u the
                                    leaf arithmetic's unit roundoff (2^-53 FP64, 2^-24 FP32),
                                    c = 3 * 2^-16 on the BF16x3 path (split residuals and the
                                    dropped lo*lo term), else 0;
                                    g = sqrt(sum_r |u_r|^2 |v_r|^2 |w_r|^2 / (M K N)) over the
                                    columns of U, V, W (the root-mean-square error growth of one
                                    step for i.i.d. zero-mean operands: 1 classical, 2 Strassen) */
    int leaf_form;               /* non-zero: the leaf GEMM forms S and T while it stages them
                                    (this many term slots per operand: 2), and
                                    fmm_multiply, fmm_multiply_noalloc and fmm_multiply_batched
                                    enqueue no formation stage; fmm_run_stage still runs
                                    FMM_STAGE_FORM_S / FORM_T (they write S and T to the
                                    workspace, where the leaf stage does not read them) */
} fmm_plan_info_t;

/* Options of fmm_plan_ex.  Zero-initialise, then set what you need. */
typedef struct {
    int fuse_levels;   /* 0: library default (2, except 1 for FMM_F32_BF16X3 plans of base
                          cases with R > 8);
                          1 or 2: recursion levels per operand-formation / combination pass */
    int host_only;     /* non-zero: plan on the host only, as fmm_plan_host */
    int use_graph;     /* non-zero: fmm_multiply records its launches once into a HIP graph
                          and replays it; a call with other operand pointers or leading
                          dimensions re-records it (one capture per change).  Ignored while
                          stage timing is on. */
    int defer_device_memory; /* non-zero: allocate nothing on the device; the caller binds
                          fmm_plan_device_bytes(p) bytes with fmm_plan_bind before running */
    int leaf_tile;     /* output tile edge of the leaf GEMM: 128 or 64 (FP64 / FP32 / BF16x3), or
                          256 (BF16x3 leaves with split operands; peel strips then take 128);
                          0 (default): chosen per launch -- BF16x3 leaves 256 when the launch has
                          at least two 256 x 256 tiles per compute unit; FP64 / FP32 launches 32
                          when they have at most half as many 64 x 64 tiles as the device has
                          compute units; otherwise 64 when the launch has fewer 128 x 128 tiles
                          than compute units, else 128.  Every tile edge gives the same bits.
                          Other values: FMM_EINVAL.  Batched launches always choose per launch. */
    double max_error;  /* automatic choice only (alg "auto" or levels -1): the largest
                          error_bound (fmm_plan_info_t) a chosen plan may have; 0: the dtype's
                          default (1e-12 FP64, 1e-4 FP32, 5e-4 BF16x3); < 0: no limit.
                          Plans named explicitly are not limited. */
    int leaf_form;     /* where the leaf operands S and T are formed (Section 3.2's
                          additions): 1 by the formation passes; 2 inside the leaf GEMM,
                          which loads the A (B) blocks of each S (T) column and sums them
                          while it stages the tile, in the passes' order and precision, so
                          the product is bit for bit the same (one-level FP64 / FP32 plans
                          whose U and V columns have at most 2 non-zeros, all +-1: Strassen
                          and its direct sums; else FMM_EINVAL); such launches run 64 x 64
                          (or 32 x 32) tiles whatever leaf_tile asks; 0 (default): 1.  It
                          removes the formation launch and the idle gap before the leaves,
                          but each leaf step issues one load per term, which made leaves
                          with long K up to 2x slower, so it is asked for, not chosen */
} fmm_plan_options_t;

/* Plan C = A*B for an m x k by k x n product with `levels` recursive steps of
 * the base case `alg` ("classical" for a plain GEMM; "strassen_222_7",
 * "fmm_333_23", "fmm_323_15", "fmm_423_20", "fmm_424_26", "classical_222_8")
 * in dtype `dtype` (fmm_dtype).  `alg` may also name one base case per level,
 * top level first, joined by '+' (e.g. "fmm_424_26+strassen_222_7" with
 * levels 2: the composition of different base cases across levels of
 * Section 5.2; the count must equal levels, else FMM_EINVAL; names up to 79
 * characters; such plans run one level per addition pass).  The core
 * (m0, k0, n0) is the largest multiple of the product of the levels' (M, K, N)
 * (M^L, K^L, N^L for one base case); the rest is peeled and multiplied
 * classically inside the same grouped launch (Section 3.5).  Allocates the workspace (all R^L leaf
 * operands and products live at once, the breadth-first layout of Section 4.2)
 * and the descriptor tables on the current HIP device.  On success *out owns
 * them until fmm_plan_destroy.  Errors: FMM_EINVAL (sizes < 0, levels < 0, a
 * leaf dimension < 1), FMM_EALG, FMM_ENOMEM (beyond FMM_HBM_BUDGET bytes, env,
 * or hipMalloc failure), FMM_EHIP. */
fmm_status fmm_plan(fmm_plan_t *out, const char *alg, int64_t m, int64_t k, int64_t n,
                    int levels, int dtype);

/* As fmm_plan, but host-only: computes the decomposition, the peel split, the
 * descriptor tables and the workspace size without touching any device.  The
 * result can be inspected (fmm_plan_info, fmm_plan_operand) but not run:
 * fmm_multiply on it returns FMM_EINVAL. */
fmm_status fmm_plan_host(fmm_plan_t *out, const char *alg, int64_t m, int64_t k, int64_t n,
                         int levels, int dtype);

/* fmm_plan with options (NULL = defaults).  Fusing two levels per addition
 * pass moves fewer bytes (each leaf operand is written once, with no
 * intermediate level), at the cost of more output streams per thread.  The
 * choice changes neither the arithmetic nor its order: results are bitwise
 * identical for every setting. */
fmm_status fmm_plan_ex(fmm_plan_t *out, const char *alg, int64_t m, int64_t k, int64_t n,
                       int levels, int dtype, const fmm_plan_options_t *opts);

/* Device bytes a plan made with defer_device_memory needs: its workspace
 * followed (at a 256-byte boundary) by its descriptor tables. */
size_t fmm_plan_device_bytes(fmm_plan_t p);

/* Gives a defer_device_memory plan the device region mem[0, bytes) (256-byte
 * aligned, bytes >= fmm_plan_device_bytes(p)) and enqueues the upload of its
 * descriptor tables on `stream`.  The caller keeps ownership of mem and must
 * not reuse it while work of the plan is pending; rebinding is allowed between
 * runs.  FMM_EINVAL for a plan that owns its memory, NULL or misaligned mem,
 * too few bytes. */
fmm_status fmm_plan_bind(fmm_plan_t p, void *mem, size_t bytes, void *stream);

/* Enqueue C = A*B on `stream` using plan p.  One multiply may be in flight per
 * plan at a time (the workspace is shared); use one plan per concurrent
 * stream.  Errors: FMM_EINVAL (ld too small, NULL pointer with non-zero size,
 * C overlapping A or B, host-only plan), FMM_EHIP. */
fmm_status fmm_multiply(fmm_plan_t p, const void *A, int64_t lda, const void *B, int64_t ldb,
                        void *C, int64_t ldc, void *stream);

/* Capacity of fmm_multiply_noalloc's device array, in bytes (64 MiB). */
#define FMM_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * enqueue C = A*B with plan p exactly as fmm_multiply does (same kernels, same
 * arithmetic, bitwise the same result), but with the plan's workspace and
 * descriptor tables placed in a fixed device array that the library holds on
 * each GPU from load until the process ends, instead of in the plan's own or
 * bound memory.  Make p with fmm_plan_ex and defer_device_memory (then the
 * plan holds no device memory at all); a plan that owns memory is accepted
 * and its memory is left untouched.  The call allocates nothing: it enqueues
 * the upload of the plan's descriptor tables (a host-to-device copy) and the
 * stage kernels on `stream`.  Limit: fmm_plan_device_bytes(p) must be at most
 * FMM_NOALLOC_MAX_BYTES, else FMM_ENOMEM and nothing is enqueued.  The array
 * is shared by every call on one GPU and keeps the last call's contents
 * (nothing in it needs to start at zero): calls that overlap on one GPU (on
 * different streams, or from several threads without ordering) race and give
 * wrong results; calls ordered on one stream are safe.  Other arguments and
 * errors as fmm_multiply.  Use graph replay or stage timing through
 * fmm_multiply; this call runs the stages directly and records no events. */
fmm_status fmm_multiply_noalloc(fmm_plan_t p, const void *A, int64_t lda, const void *B, int64_t ldb,
                                void *C, int64_t ldc, void *stream);

/* Enqueue count products C[i] = A[i] * B[i], each with its own plan
 * plans[i] (all on the current device, each plan at most once), as one batch:
 * the S and T formations of every request, then grouped leaf launches that
 * hold the leaf products and peel strips of several requests at once (up to
 * 8 plans per launch, one launch series per dtype; Section 3.1's products are
 * independent, so any grouping gives the same results bit for bit), then the
 * combinations.  Per-request arguments and errors as fmm_multiply; on an
 * argument error nothing is enqueued and the message names the request. */
fmm_status fmm_multiply_batched(const fmm_plan_t *plans, const void *const *A, const int64_t *lda,
                                const void *const *B, const int64_t *ldb, void *const *C,
                                const int64_t *ldc, int count, void *stream);

/* Enqueue only one stage of fmm_multiply (same arguments).  Running the four
 * stages in order is exactly fmm_multiply; a stage reads what the earlier
 * stages left in the workspace.  For testing and per-stage timing. */
fmm_status fmm_run_stage(fmm_plan_t p, int stage, const void *A, int64_t lda, const void *B,
                         int64_t ldb, void *C, int64_t ldc, void *stream);

/* Where an operand of leaf `leaf` (0 <= leaf < R^L, most significant digit =
 * top level) lives: side 0 = S (A side), 1 = T (B side), 2 = M (product).
 * *loc is an fmm_loc.  For FMM_LOC_WORKSPACE the operand's element (i, j) is
 * at workspace element *offset + i * (*ld) + j.  For FMM_LOC_A / FMM_LOC_B it
 * is the caller's element (*row + i, *col + j) (a view: no copy is made) and
 * *offset = 0, *ld = 0.  *alpha is the scaling the leaf GEMM applies to the
 * view (single-non-zero columns of U or V).  The element type is the path's
 * (double for FMM_F64, float otherwise).  Any output pointer may be NULL. */
fmm_status fmm_plan_operand(fmm_plan_t p, int side, int64_t leaf, int *loc, int64_t *offset,
                            int64_t *row, int64_t *col, int64_t *ld, double *alpha);

/* Device address of the plan's workspace (NULL for host-only plans). */
void *fmm_plan_workspace(fmm_plan_t p);

size_t fmm_plan_workspace_bytes(fmm_plan_t p);
fmm_status fmm_plan_info(fmm_plan_t p, fmm_plan_info_t *info);

/* Stage timing.  fmm_plan_enable_timing(p, slots) with slots > 0 creates
 * (slots * 5) HIP events once; every later fmm_multiply on p records one event
 * before each stage and one after the last, on its own stream, into a ring of
 * `slots` multiplies (slots = 0 turns recording off).  fmm_plan_stage_ms waits
 * for the recorded multiplies and writes the mean duration of each stage, in
 * milliseconds, over the most recent min(timed, slots) of them. */
fmm_status fmm_plan_enable_timing(fmm_plan_t p, int slots);
fmm_status fmm_plan_stage_ms(fmm_plan_t p, double ms[FMM_NUM_STAGES]);

/* Frees the workspace and tables.  NULL is accepted. */
fmm_status fmm_plan_destroy(fmm_plan_t p);

/* Classical C = A*B with the library's grouped MFMA GEMM kernel (one problem),
 * no plan and no workspace: the same-GPU classical baseline. */
fmm_status fmm_gemm(int dtype, int64_t m, int64_t k, int64_t n, const void *A, int64_t lda,
                    const void *B, int64_t ldb, void *C, int64_t ldc, void *stream);

/* Base-case tables compiled into the library.  fmm_algorithm_coeffs writes
 * the dimensions and, when the arrays are non-NULL, U (MK x R), V (KN x R)
 * and W (MN x R) row-major as int8.  FMM_EALG for an unknown name. */
int fmm_num_algorithms(void);
const char *fmm_algorithm_name(int index);
fmm_status fmm_algorithm_coeffs(const char *alg, int *M, int *K, int *N, int *R,
                                int8_t *U, int8_t *V, int8_t *W);

/* Checks every compiled-in table against the Brent equations (Equation (2))
 * in exact integer arithmetic: FMM_OK or FMM_EALG naming the first failure. */
fmm_status fmm_check_algorithms(void);

const char *fmm_last_error(void);

/* ---- Algorithm and depth selection (model) -------------------------------
 * The paper picks the base case and depth per shape by measurement
 * (Section 5: the best algorithm depends on the shape, and recursion pays only
 * while the leaf product stays efficient).  The library's prior is a cost
 * model, t = leaf_flops / (rate(dtype) * eff(leaf shape)) + add_bytes / BW
 * + launches * t_launch, where eff counts 128 x 128 tile padding, the last
 * partial wave of tiles over the compute units and a per-tile fixed cost in
 * units of K.  fmm_plan with alg "auto" (any base case) or levels -1 (the
 * given base case) plans the model's best candidate whose workspace fits the
 * budget (FMM_HBM_BUDGET bytes, env, else 3/4 of the device's free memory, or
 * of 288 GB on the host).  A measured choice recorded with fmm_tune_record
 * for the exact shape takes precedence (the Python autotuner times the
 * model's best few candidates and records the winner). */
typedef struct {
    char alg[80];        /* "classical", a base-case name, or one per level joined by '+' */
    int levels;
    int fuse_levels;
    int leaf_tile;       /* leaf tile edge of a recorded choice (64 / 128); 0: chosen per launch */
    double model_ms;     /* predicted time */
    double leaf_ms, add_ms;
    size_t workspace_bytes;
    double error_bound;  /* as fmm_plan_info_t::error_bound */
} fmm_candidate_t;

/* Writes up to max candidates for (m, k, n, dtype), best predicted first,
 * restricted to base case `alg` when it is not NULL and not "auto"; *count
 * receives the number written.  Candidates whose workspace exceeds
 * budget_bytes (0 = the default budget above) or whose error bound exceeds
 * max_error (0 = the dtype's default of fmm_plan_options_t::max_error, < 0 =
 * no limit) are left out.  The automatic choice ("auto", levels -1, server
 * requests without a named plan) takes the first candidate of this list, so
 * it never exceeds the error budget; a recorded measured choice
 * (fmm_tune_record) above the budget is ignored. */
fmm_status fmm_rank_candidates(int64_t m, int64_t k, int64_t n, int dtype, const char *alg,
                               size_t budget_bytes, double max_error, fmm_candidate_t *out, int max,
                               int *count);

/* Records a measured choice for the exact shape (m, k, n, dtype) in a
 * process-wide table: later fmm_plan calls with alg "auto" and levels -1 for
 * that shape, and server requests of that shape with alg NULL/"auto" and
 * levels -1, plan it (when its workspace fits the budget) instead of the
 * model's pick, with its fuse_levels and leaf_tile (0, 64 or 128, as in
 * fmm_plan_options_t).  The choice is validated by planning it on the host.
 * fmm_tune_clear empties the table.  Thread-safe. */
fmm_status fmm_tune_record(int64_t m, int64_t k, int64_t n, int dtype, const char *alg, int levels,
                           int fuse_levels, int leaf_tile);
fmm_status fmm_tune_clear(void);

/* ---- Serving runtime: continuous batching ---------------------------------
 * A request queue in front of fmm_multiply_batched.  Requests are admitted in
 * arrival order (within their class, below) while the device arena
 * (workspaces and descriptor tables) has room and a stream of their class
 * has fewer than max_inflight batches pending; each admitted batch is
 * enqueued as one fmm_multiply_batched (or, with use_graph, as one HIP graph
 * recorded from it) on one of the server's streams and followed by one
 * completion event there.  With num_streams = 1 every request shares one
 * stream and batches hold up to max_batch requests.  With 2-4 streams
 * (each of the default priority), stream 0 runs the large requests
 * (2mkn >= large_flops) one per batch, shortest first (fewest flops; a
 * request waiting over 100 ms goes first, oldest first), and the others run
 * the remaining requests in arrival order, in batches of up to max_batch,
 * each batch on the one with the fewest pending batches: a small request
 * never waits behind a large product, and the device interleaves the
 * streams' workgroups as those of running kernels retire.  Planning
 * of the next batches on the host overlaps the running ones on the device.
 * The caller owns A, B and C of every request and keeps them alive until the
 * request completes.  Single-threaded: call every fmm_server_* function of
 * one server from one thread. */
typedef struct fmm_server_s *fmm_server_t;

/* Default large-request threshold (2mkn, flops) with several streams: about
 * 1 ms of the device's FP64 rate. */
#define FMM_SERVER_LARGE_FLOPS 6.0e10
/* arena_bytes = 0: the arena takes the device's free memory at creation less
 * this reserve (bytes) for the callers' operands and outputs. */
#define FMM_SERVER_RESERVE_BYTES (16ull << 30)

typedef struct {
    size_t arena_bytes;  /* device bytes for workspaces and tables (admission budget);
                            0: all free device memory less FMM_SERVER_RESERVE_BYTES */
    int max_batch;       /* requests per batch, 1..64 (leaves of up to 8 share a launch) */
    int max_inflight;    /* batches enqueued and not finished per stream, >= 1 */
    int fuse_levels;     /* as fmm_plan_options_t */
    int use_graph;       /* non-zero: each batch's launches are recorded into a HIP graph
                            (kernel nodes only), instantiated once and launched as one
                            graph; the executable graph is freed when the batch completes */
    double max_error[3]; /* per dtype (index = fmm_dtype): error budget of the automatic
                            choice for requests without a named plan, as
                            fmm_plan_options_t::max_error (0: default, < 0: no limit) */
    int num_streams;     /* 0 or 1: one stream; 2..4: large requests on stream 0, the rest
                            on the others (see above) */
    double large_flops;  /* 2mkn at or above which a request is large (0: the default
                            FMM_SERVER_LARGE_FLOPS); the lanes' split with num_streams >= 2 */
    int small_model;     /* 0 (default): a request below large_flops that names no plan
                            (alg NULL / "auto", levels -1) runs the classical product, whose
                            leaves join the batch's grouped launch; non-zero: the automatic
                            choice for every request.  Large requests always take the
                            automatic choice. */
} fmm_server_options_t;

typedef struct {
    int64_t m, k, n;
    int dtype;
    const char *alg;     /* NULL or "auto": model choice of base case and depth */
    int levels;          /* -1: model choice of depth for `alg` */
    const void *A; int64_t lda;
    const void *B; int64_t ldb;
    void *C; int64_t ldc;
    void *user;          /* returned with the completion */
    int wait_stream;     /* non-zero: the batch that runs the request first waits, on its
                            server stream, for the work enqueued on `stream` before the
                            submit (an event recorded there by fmm_server_submit), e.g. the
                            kernels that write A and B or that still use C's memory */
    void *stream;        /* hipStream_t for wait_stream (NULL: the null stream) */
} fmm_request_t;

typedef struct {
    int64_t id;
    void *user;
    fmm_status status;   /* FMM_OK, or why the request was not run */
    double submit_ms;    /* host steady clock, ms since the server was created */
    double launch_ms;    /* when its batch was enqueued */
    double done_ms;      /* when its batch's completion event was seen */
    int batch_size;
    char alg[80];
    int levels;
    int lane;            /* the server stream its batch ran on (-1: not run) */
} fmm_completion_t;

/* Creates a server on the current device; allocates the arena there.  stream
 * non-NULL: the server's stream 0 (the others, if any, it creates); NULL: it
 * creates all of them.  FMM_ENOMEM when the arena cannot be allocated;
 * FMM_EINVAL for options out of range. */
fmm_status fmm_server_create(fmm_server_t *out, const fmm_server_options_t *opts, void *stream);

/* The arena's size in bytes (as resolved when arena_bytes was 0); 0 for NULL. */
size_t fmm_server_arena_bytes(fmm_server_t s);

/* Queues a request; *id is its sequence number.  The request is validated on
 * the host as fmm_multiply validates its arguments (sizes, dtype, NULL
 * pointers, leading dimensions, C overlapping A or B) and, when it names no
 * plan, planned by the automatic choice; an invalid request is refused here
 * with its own status and never joins a batch.  Does not launch anything by
 * itself. */
fmm_status fmm_server_submit(fmm_server_t s, const fmm_request_t *req, int64_t *id);

/* Makes progress: retires finished batches (frees their arena space) and
 * admits and launches new batches.  Writes up to max_done completions.  With
 * wait non-zero it blocks until at least one request completes if any is
 * pending.  A request that cannot fit the arena even alone, or whose plan
 * fails, completes with that error status. */
fmm_status fmm_server_progress(fmm_server_t s, int wait, fmm_completion_t *done, int max_done,
                               int *num_done);

/* Requests submitted and not yet returned as completions. */
int64_t fmm_server_pending(fmm_server_t s);

/* Waits for pending batches, then frees everything.  Requests still queued
 * are dropped.  NULL is accepted. */
fmm_status fmm_server_destroy(fmm_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H */
