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
    FMM_EUNSUPPORTED = 4,  /* dtype / option not supported by this build */
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
    FMM_STAGE_FORM_S = 0,  /* S operands from A (Section 3.1, first bullet; 3.2 streaming) */
    FMM_STAGE_FORM_T = 1,  /* T operands from B */
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
} fmm_plan_info_t;

/* Options of fmm_plan_ex.  Zero-initialise, then set what you need. */
typedef struct {
    int fuse_levels;   /* 0: library default (2 for base cases with R <= 8, else 1);
                          1 or 2: recursion levels per operand-formation / combination pass */
    int host_only;     /* non-zero: plan on the host only, as fmm_plan_host */
} fmm_plan_options_t;

/* Plan C = A*B for an m x k by k x n product with `levels` recursive steps of
 * the base case `alg` ("classical" for a plain GEMM; "strassen_222_7",
 * "fmm_333_23", "fmm_323_15", "fmm_423_20", "fmm_424_26", "classical_222_8")
 * in dtype `dtype` (fmm_dtype).  The core (m0, k0, n0) is the largest multiple
 * of (M^L, K^L, N^L); the rest is peeled and multiplied classically inside the
 * same grouped launch (Section 3.5).  Allocates the workspace (all R^L leaf
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

/* Enqueue C = A*B on `stream` using plan p.  One multiply may be in flight per
 * plan at a time (the workspace is shared); use one plan per concurrent
 * stream.  Errors: FMM_EINVAL (ld too small, NULL pointer with non-zero size,
 * C overlapping A or B, host-only plan), FMM_EHIP. */
fmm_status fmm_multiply(fmm_plan_t p, const void *A, int64_t lda, const void *B, int64_t ldb,
                        void *C, int64_t ldc, void *stream);

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

#ifdef __cplusplus
}
#endif

#endif /* FMM_H */
