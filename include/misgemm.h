/*
 * misgemm: single-precision GEMM for one AMD Instinct MI355X (gfx950).
 *
 * The operation is the BLAS sgemm that the paper's BLIS-generated library
 * solves (Section III-A):
 *
 *     C = alpha * op(A) * op(B) + beta * C,    op(X) = X or X^T,
 *
 * with op(A) M x K, op(B) K x N and C M x N, every matrix stored column-major
 * (element (r, c) of a matrix with leading dimension ld at offset r + c*ld),
 * M, N and K arbitrary.  The argument order is the classic Fortran BLAS one
 * that the paper's library also generates.
 *
 * Memory and streams.  A, B and C are device pointers on the current HIP
 * device; the caller allocates and owns them, the library never frees them.
 * A and B are read only; C is read (when beta != 0) and written.  C must not
 * overlap A or B (not checked).  Rows r in [M, ldc) of C are never written.
 * `stream` is a hipStream_t passed as void* (NULL = the null stream); every
 * call is asynchronous on it and returns once the work is enqueued.
 *
 * Error convention (every entry point returns int):
 *   0                  success;
 *   < 0                invalid argument, numbered by its position in the
 *                      call, as BLAS xerbla does (-1 = first argument);
 *                      nothing is launched and C is untouched;
 *   1 .. 999           a HIP runtime error code (hipError_t);
 *   >= 1000            a library error, see MISGEMM_E_* below.
 * misgemm_status_string() describes any of them.
 *
 * Degenerate cases follow the reference BLAS: nothing happens when M == 0 or
 * N == 0, or when (alpha == 0 or K == 0) and beta == 1; when alpha == 0 or
 * K == 0, A and B are not read and C = beta * C; when beta == 0, C is not
 * read (NaN or Inf in it does not propagate) and C = alpha * op(A) * op(B).
 */
#ifndef MISGEMM_H
#define MISGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic forms. */
typedef enum {
    /* FP32 matrix-core products (v_mfma_f32_32x32x2_f32), FP32 accumulate. */
    MISGEMM_FP32 = 0,
    /* Split precision: each FP32 operand is written as the sum of three
     * bfloat16 values (round to nearest even, each part rounding what the
     * previous parts left), the six part products whose part indices sum to
     * at most 2 run on BF16 matrix cores with FP32 accumulation, and the
     * result is returned in FP32.  Defined for finite inputs of magnitude
     * below 0x1.fefp127 (the bf16 overflow threshold); tiny inputs (below
     * about 2^-110) lose the exactness of the split. */
    MISGEMM_BF16X3 = 1
} misgemm_mode;

/* Library error codes (>= 1000). */
#define MISGEMM_E_NO_DEVICE        1000 /* no gfx950 device is current          */
#define MISGEMM_E_BAD_CONFIG       1001 /* config id unknown or not for mode     */
#define MISGEMM_E_CAPTURING        1002 /* call not allowed during graph capture */
#define MISGEMM_E_TUNING_FILE      1003 /* tuning file unreadable or malformed   */
#define MISGEMM_E_BATCH            1004 /* bad batch (see bad_index)             */
#define MISGEMM_E_NULL_PLAN        1005 /* plan pointer is NULL                  */
#define MISGEMM_E_TOO_LARGE        1006 /* a size exceeds what the kernels index */
#define MISGEMM_E_SCRATCH          1007 /* needs more than the static scratch    */

/*
 * C = alpha * op(A) * op(B) + beta * C  (Section III-A).
 *
 * transa, transb: 'N'/'n' (op(X) = X) or 'T'/'t'/'C'/'c' (op(X) = X^T; C and
 *   T coincide for real data, as the paper's test parameters c/h do).
 * m, n, k >= 0.  A is m x k (transa = N) or k x m (T), lda >= max(1, rows of
 *   stored A); likewise B is k x n or n x k with ldb; ldc >= max(1, m).
 * mode: a misgemm_mode.
 * Errors: -1 transa, -2 transb, -3 m, -4 n, -5 k, -7 A NULL with work to do,
 *   -8 lda, -9 B NULL, -10 ldb, -12 C NULL, -13 ldc, -14 mode.
 * The kernel configuration (tile shape, wave layout, split-K factor) comes
 * from the loaded tuning table when it holds an entry for the shape, else
 * from built-in heuristics; misgemm_sgemm never picks a packed bf16x3
 * configuration (those need a workspace: misgemm_sgemm_ws).  One choice uses
 * scratch memory that the library owns per (device, stream) -- calls on one
 * stream share it in stream order, calls on different streams never share
 * it: split-K, which the table or the heuristics pick when the C tiles alone
 * would leave CUs idle (each of `splits` workgroups per tile computes a K
 * range and stores its partial tile, splits * tiles * bm * bn * 4 bytes; a
 * second kernel adds the partials in split order and applies alpha/beta, so
 * results are reproducible bit for bit).
 * The scratch is allocated on first need and never while the stream is
 * being captured (the call then runs without it).  When a larger problem
 * outgrows it, the old buffer is freed after the work queued on the stream
 * has finished (the call synchronizes that stream once), unless a call
 * under graph capture used it: a graph may then still reference it, and it
 * is kept until misgemm_release_workspace().  So a caller that never
 * captures holds one buffer per (device, stream), the size of its largest
 * need.  Callers that must not allocate use misgemm_sgemm_ws (caller-owned
 * workspace, no split-K) or misgemm_sgemm_split_noalloc instead.
 */
int misgemm_sgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                  float alpha, const float *A, int64_t lda,
                  const float *B, int64_t ldb,
                  float beta, float *C, int64_t ldc,
                  int mode, void *stream);

/*
 * misgemm_sgemm with an explicit kernel configuration (an index below
 * misgemm_num_configs(); the config's mode must equal `mode`) and tile
 * order: group_m tile-rows of C are walked together so that concurrently
 * running workgroups share panels of op(A) and op(B) in cache (0 = the
 * default, 8).  Used by the autotuner to time every candidate.  Errors as
 * misgemm_sgemm, plus -15 for an unknown config id or one of another mode
 * and -16 for group_m outside [0, 4096].
 */
int misgemm_sgemm_config(char transa, char transb, int64_t m, int64_t n, int64_t k,
                         float alpha, const float *A, int64_t lda,
                         const float *B, int64_t ldb,
                         float beta, float *C, int64_t ldc,
                         int mode, int config_id, int group_m, void *stream);

/*
 * misgemm_sgemm_config with an explicit split-K factor (the GPU form of the
 * partial results the paper sums on the host, Section III-C): splits in
 * [1, 64]; 1 runs the whole K range in every workgroup (as
 * misgemm_sgemm_config), larger values cut K into that many whole-BK ranges
 * (fewer when K has fewer blocks).  config_id < 0 with splits > 1 picks the
 * split-capable configuration of the mode with the smallest tile.  Uses the
 * library scratch of (device, stream) for splits * tiles * bm * bn * 4 bytes
 * of partial tiles; two kernel launches.  Errors as misgemm_sgemm_config,
 * plus -17 for splits outside [1, 64], MISGEMM_E_BAD_CONFIG for a
 * configuration without a split-K variant, MISGEMM_E_CAPTURING when the
 * scratch would have to be allocated during capture.
 */
int misgemm_sgemm_split(char transa, char transb, int64_t m, int64_t n, int64_t k,
                        float alpha, const float *A, int64_t lda,
                        const float *B, int64_t ldb,
                        float beta, float *C, int64_t ldc,
                        int mode, int config_id, int group_m, int splits, void *stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the call of
 * misgemm_sgemm_split (same arguments, errors and results bit for bit) with
 * its split-K partial tiles in a static device array of
 * MISGEMM_STATIC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends.  Allocates nothing and frees nothing.
 * splits * tiles * bm * bn * 4 bytes must fit the array, else
 * MISGEMM_E_SCRATCH (nothing launched); a packed configuration is refused
 * (-15: its panels do not fit).  The array needs no clearing: every partial
 * tile is written before it is read.  Every call on one device shares that
 * device's array: calls that overlap in time on one GPU (other streams,
 * concurrently replayed graphs) race on it; calls on one stream run in
 * order and are safe.  The first call on each device looks the array's
 * address up (hipGetSymbolAddress); make it outside graph capture.
 */
#define MISGEMM_STATIC_SCRATCH_BYTES (64LL << 20)
int misgemm_sgemm_split_noalloc(char transa, char transb, int64_t m, int64_t n, int64_t k,
                                float alpha, const float *A, int64_t lda,
                                const float *B, int64_t ldb,
                                float beta, float *C, int64_t ldc,
                                int mode, int config_id, int group_m, int splits, void *stream);

/*
 * Workspace for the packed bf16x3 path.  Packed configurations first split
 * op(A) and op(B) into bf16 panels (the BLIS packing step: for each block of
 * 16 k, each of the three parts, each row, 16 consecutive values), then run
 * one tile kernel on the panels.  The panels take
 * 6 * ceil(k/16)*16 * (roundup(m,256) + roundup(n,256)) bytes (plus 512).
 *
 * misgemm_workspace_size: bytes misgemm_sgemm_ws needs for the packed path
 *   of this problem (0 for MISGEMM_FP32); negative = argument error as in
 *   misgemm_sgemm.
 * misgemm_sgemm_ws: misgemm_sgemm with a caller-owned device workspace
 *   (16-byte aligned), in which the tuning table's packed bf16x3
 *   configurations may run (a table lists, per shape, its fastest entry,
 *   packed or not, and the fastest non-packed one for misgemm_sgemm).
 *   workspace == NULL: a packed configuration is never chosen and nothing is
 *   allocated; otherwise workspace_bytes must cover misgemm_workspace_size
 *   (-16 if not, -15 if misaligned) and the call allocates nothing
 *   (capturable).  The workspace must not be reused by
 *   another call before this one completes on `stream`.
 * misgemm_sgemm_ws never uses split-K.
 * misgemm_sgemm itself never picks a packed configuration.
 *   misgemm_sgemm_config with an explicit packed configuration uses the
 *   scratch the library owns per (device, stream) for the panels: grown with
 *   hipMalloc when a larger problem arrives (MISGEMM_E_CAPTURING when it
 *   would have to grow while the stream is being captured); outgrown
 *   buffers are freed as described at misgemm_sgemm, except those that
 *   captured graphs may reference.
 * misgemm_release_workspace: synchronizes the current device and frees the
 *   library-owned scratch of that device (all streams); graphs captured
 *   with it must not be replayed afterwards.
 * misgemm_workspace_held: bytes of library-owned scratch the current device
 *   holds (all streams, kept outgrown buffers included); negative status
 *   when no device is current.
 */
int64_t misgemm_workspace_size(char transa, char transb, int64_t m, int64_t n, int64_t k,
                               int mode);
int misgemm_sgemm_ws(char transa, char transb, int64_t m, int64_t n, int64_t k,
                     float alpha, const float *A, int64_t lda,
                     const float *B, int64_t ldb,
                     float beta, float *C, int64_t ldc,
                     int mode, void *workspace, int64_t workspace_bytes, void *stream);
int misgemm_release_workspace(void);
int64_t misgemm_workspace_held(void);

/* Description of one compiled kernel configuration. */
typedef struct {
    int mode;          /* misgemm_mode                                  */
    int bm, bn, bk;    /* workgroup tile: rows of C, columns of C, K step */
    int wm, wn;        /* per-wave tile of C                            */
    int threads;       /* threads per workgroup (64 per wave)           */
    int lds_bytes;     /* LDS used per workgroup                        */
    int packed;        /* 1: operands are first split into packed panels
                          in a workspace (bf16x3 only), 0: split in LDS  */
    int splitk;        /* 1: a split-K variant is compiled               */
    char name[48];     /* e.g. "fp32p_256x256x16_w128x64"              */
} misgemm_config_desc;

/* Number of compiled configurations (ids 0 .. n-1). */
int misgemm_num_configs(void);

/* Fills *out for config `id`; -1 if id is out of range, -2 if out is NULL. */
int misgemm_config_info(int id, misgemm_config_desc *out);

/*
 * Which configuration misgemm_sgemm would pick for this problem (tuning
 * table first, then heuristics; never a packed one), or a negative argument
 * error.
 */
int misgemm_select_config(char transa, char transb, int64_t m, int64_t n, int64_t k,
                          int mode);

/*
 * Load the tuning table written by the autotuner.  Text file: the header
 * line "misgemm-tuning 1", then lines
 *     <mode> <transa> <transb> <m> <n> <k> <config_name> [<group_m> [<splits>]]
 * (a problem is served by the entry of its mode and transposes whose sizes
 * are all within a factor 2 of its own, nearest in summed log-distance;
 * splits 0 or absent = automatic, 1 = none, >= 2 needs a configuration with
 * a split-K variant) and
 *     batch <mode> <config_name>
 * (the default configuration of batched plans); '#' starts a comment line.
 * path == NULL clears the table and returns to the built-in heuristics.
 * The table is replaced only when the whole file parses.  Not thread-safe
 * with concurrent calls of the other entry points.
 * Error: MISGEMM_E_TUNING_FILE.
 */
int misgemm_load_tuning(const char *path);

/* ---------------------------------------------------------------------------
 * Double precision (the paper's dgemm variants, Section IV-B).
 * ------------------------------------------------------------------------- */
typedef enum {
    MISGEMM_D_FP64 = 0, /* FP64 matrix cores (v_mfma_f64_16x16x4_f64), FP64 sums */
    MISGEMM_D_FP32 = 1  /* the paper's "false dgemm": op(A), op(B) rounded to FP32,
                           product on the FP32 path, alpha/beta in FP64         */
} misgemm_dmode;

/*
 * C = alpha * op(A) * op(B) + beta * C for FP64 column-major matrices in
 * device memory; arguments, transposes, degenerate cases and error codes as
 * in misgemm_sgemm (-14: dmode not a misgemm_dmode).  MISGEMM_D_FP32 narrows
 * the stored operands into the library scratch of (device, stream)
 * ((lda*cols(A) + ldb*cols(B) + m*n) * 4 bytes; MISGEMM_E_CAPTURING when it
 * would have to grow during capture), so its result carries FP32 rounding:
 * within tol(K) + 2^-22 of the normalized error bound instead of the FP64
 * max(2K, K+3) * 2^-53.  MISGEMM_D_FP64 allocates nothing.
 */
int misgemm_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                  double alpha, const double *A, int64_t lda,
                  const double *B, int64_t ldb,
                  double beta, double *C, int64_t ldc,
                  int dmode, void *stream);

/* ---------------------------------------------------------------------------
 * LU with partial pivoting and the solve: the Linpack (HPL) workload of the
 * paper's Section IV-C, on the sgemm path.
 * ------------------------------------------------------------------------- */

/*
 * P A = L U for the n x n FP32 matrix A (device, column-major, lda >= n),
 * overwritten by L (unit diagonal not stored) and U.  ipiv (device, n
 * int64): row ipiv[j] (0-based, >= j) was swapped with row j at step j,
 * first row of largest magnitude on ties.  info (device int): 0, or 1 + the
 * first j with a zero pivot (the factorization then completes without
 * dividing that column, as LAPACK's getrf does).  Recursive right-looking
 * algorithm: the trailing updates and the off-diagonal parts of the
 * triangular solves are sgemm calls in `mode` (MISGEMM_FP32 or
 * MISGEMM_BF16X3), except the smallest ones, between two sibling leaves,
 * which the right leaf applies itself in FP32; leaf panels of 8 columns (4
 * when taller than 8192 rows) are factored by one workgroup, and each
 * leaf's interchanges are applied to the rest of the matrix right after
 * it.
 * Asynchronous on `stream`; uses the library scratch of misgemm_sgemm.
 * Errors: -1 n, -2 A, -3 lda, -4 ipiv, -5 info, -6 mode (before any launch).
 */
int misgemm_sgetrf(int64_t n, float *A, int64_t lda, int64_t *ipiv, int *info, int mode,
                   void *stream);

/*
 * Solve A X = B with the factors of misgemm_sgetrf: B (n x nrhs, device,
 * ldb >= n) is overwritten with X (row swaps, then L, then U; the
 * off-diagonal blocks through sgemm in `mode`).  The swaps exchange rows k
 * and ipiv[k] for k = 0 .. n-1 in order, whatever ipiv holds; an entry
 * outside [0, n) is skipped (no access out of bounds).  Errors: -1 n,
 * -2 nrhs, -3 A, -4 lda, -5 ipiv, -6 B, -7 ldb, -8 mode.
 */
int misgemm_sgetrs(int64_t n, int64_t nrhs, const float *A, int64_t lda, const int64_t *ipiv,
                   float *B, int64_t ldb, int mode, void *stream);

/* ---------------------------------------------------------------------------
 * Host-pointer BLAS: for callers whose matrices live in host memory, as the
 * paper's library served unmodified BLAS users (Sections III-A, III-C).
 * ------------------------------------------------------------------------- */

/*
 * misgemm_sgemm / misgemm_dgemm on host matrices, synchronous: A and B are
 * copied into device buffers the library keeps per device (grow-only), C is
 * cut into column panels (about four when n >= 1024) and panel p+1 is copied
 * in while panel p is multiplied and panel p-1 copied back, on three streams
 * of the library's own; C's panels pass through pinned host buffers the
 * library keeps per device (grow-only, hipHostMalloc), gathered from and
 * scattered to the caller's columns by host threads.  Only the m rows of
 * each column of C are written (padding rows untouched) and nothing past
 * the last column of any operand is read.  Calls on one device are
 * serialized.  Returns 0 or an error as
 * misgemm_sgemm / misgemm_dgemm (-14: mode).
 */
int misgemm_sgemm_host(char transa, char transb, int64_t m, int64_t n, int64_t k,
                       float alpha, const float *A, int64_t lda,
                       const float *B, int64_t ldb,
                       float beta, float *C, int64_t ldc, int mode);
int misgemm_dgemm_host(char transa, char transb, int64_t m, int64_t n, int64_t k,
                       double alpha, const double *A, int64_t lda,
                       const double *B, int64_t ldb,
                       double beta, double *C, int64_t ldc, int dmode);

/*
 * The classic Fortran BLAS symbols (every argument by reference, 32-bit
 * integers; trailing hidden string lengths are ignored), on host matrices,
 * through the two functions above: sgemm_ in MISGEMM_FP32 mode (the
 * environment variable MISGEMM_SGEMM_MODE=bf16x3 selects the split form),
 * dgemm_ on FP64 matrix cores.  An invalid argument prints the reference
 * BLAS message " ** On entry to SGEMM  parameter number N had an illegal
 * value" to stderr and returns without touching C.
 */
void sgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
            const float *alpha, const float *A, const int *lda, const float *B, const int *ldb,
            const float *beta, float *C, const int *ldc);
void dgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
            const double *alpha, const double *A, const int *lda, const double *B,
            const int *ldb, const double *beta, double *C, const int *ldc);

/* ---------------------------------------------------------------------------
 * Batched form: many independent sgemm problems in one persistent launch.
 * ------------------------------------------------------------------------- */

/* One problem of a batch; fields as in misgemm_sgemm. */
typedef struct {
    char transa, transb;
    int64_t m, n, k;
    float alpha;
    const float *A;
    int64_t lda;
    const float *B;
    int64_t ldb;
    float beta;
    float *C;
    int64_t ldc;
} misgemm_problem;

typedef struct misgemm_batch misgemm_batch; /* opaque plan */

/*
 * Validate `count` problems, cut every one into C tiles of the chosen
 * configuration, deal the tiles to one list per XCD (problems cut into
 * chunks of consecutive tiles, chunks placed longest first on the least
 * loaded list, so each XCD's L2 serves few problems), order every list by
 * decreasing work (longest first), and upload the problem and tile tables
 * to device memory owned by the plan.
 * config_id < 0 picks the configuration from the tuning table / heuristics;
 * a tuning-table rule "batch2 <mode> <T> <config> <config2>" instead puts
 * the problems with m >= T and n >= T on <config> and the others on
 * <config2>, as two launches that run concurrently (the second on a stream
 * the plan owns, forked from and joined back to the launching stream with
 * events, so misgemm_batch_launch stays capturable).
 * With a packed bf16x3 configuration the plan also owns panels for every
 * problem's split operands (6 bytes per element of op(A) and op(B), rows
 * padded to the tile side), and each launch first packs the operands (one
 * pack kernel over all problems) and then runs the tile kernel on the
 * panels; the operands are read at launch time, as for the other plans.
 * On a bad problem returns that problem's argument error (negative, as for
 * misgemm_sgemm) or MISGEMM_E_BATCH and stores its index in *bad_index.
 * Allocates device memory and synchronizes: NOT capturable (returns
 * MISGEMM_E_CAPTURING if the current device's null stream is capturing).
 * The pointers inside the problems are stored, not copied: the buffers must
 * stay valid while the plan is launched.
 */
int misgemm_batch_plan(const misgemm_problem *problems, int64_t count, int mode,
                       int config_id, misgemm_batch **plan, int64_t *bad_index);

/*
 * Run every problem of the plan in one persistent kernel launch on `stream`.
 * Allocates nothing and does not synchronize, so it may be captured into a
 * HIP graph and replayed.  Launches of one plan on several streams at once
 * race on the plan's C buffers (and, for a two-part plan, on its fork and
 * join events); launches of different plans do not interact.
 */
int misgemm_batch_launch(const misgemm_batch *plan, void *stream);

/* Plan facts: tiles, workgroups launched, config id, total flops 2*m*n*k,
 * and the partition of the tiles over the XCDs.  A two-part plan (a tuned
 * "batch2" rule) reports its larger-problem part in config_id, grid, parts
 * and part_imbalance, the other part's config and grid in second_*; tiles
 * and flops cover both. */
typedef struct {
    int64_t count, tiles, grid;
    int config_id;
    double flops;
    double tile_flops;     /* flops of whole tiles, edges padded (>= flops) */
    int parts;             /* tile lists, one per XCD (1 for tiny batches) */
    double part_imbalance; /* largest list's work / mean list work (>= 1) */
    int second_config_id;  /* -1: one part */
    int64_t second_grid;
    int64_t panel_bytes;   /* device bytes of split operand panels the plan owns
                              (packed bf16x3 configurations; 0 otherwise) */
} misgemm_batch_desc;

int misgemm_batch_info(const misgemm_batch *plan, misgemm_batch_desc *out);

/* Free the plan's device tables (synchronizes the device first). */
int misgemm_batch_destroy(misgemm_batch *plan);

/* ---------------------------------------------------------------------------
 * The split used by MISGEMM_BF16X3, exposed on its own.
 * ------------------------------------------------------------------------- */

/*
 * parts[3*i + t] = bit pattern of the t-th bf16 part of x[i], i < count:
 * part 0 = bf16_rne(x), part 1 = bf16_rne(x - part0), part 2 =
 * bf16_rne(x - part0 - part1), residuals formed in FP32.  x and parts are
 * device pointers.  Errors: -1 x NULL, -2 count < 0, -3 parts NULL.
 */
int misgemm_bf16x3_split(const float *x, int64_t count, uint16_t *parts, void *stream);

/* Human-readable description of a status code. */
const char *misgemm_status_string(int status);

/* Library version string. */
const char *misgemm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MISGEMM_H */
