/*
 * rclupp.h -- C ABI of the MI355X (gfx950) tall-skinny QR library.
 *
 * Computes X = Q R for a tall-skinny X (m x n, m >= n, rank n), Q with
 * orthonormal columns and R upper triangular with a positive diagonal
 * (Section 1 of "A new randomized CholeskyQR based on LU decomposition with
 * partial pivoting", Fan, Guan, Qiao, arXiv 2412.06551), by
 *   RCLUPP   (Algorithm 2)  sketch -> LU of the sketch -> Householder R -> CholeskyQR2
 *   RCLUPPr  (Algorithm 7)  LU of X -> sketch of L -> Householder R -> CholeskyQR2
 * and by the baselines the paper compares with:
 *   CholeskyQR2 (Algorithm 3), Shifted CholeskyQR3 (Algorithm 4),
 *   LU-CholeskyQR2 (Algorithm 5), randomized CholeskyQR (Algorithm 6).
 *
 * Conventions shared by every entry point
 *   - matrix pointers are DEVICE pointers to float64, column-major:
 *     element (i, j) of X is X[i + j*ld]; Q uses the same ld; R is n x n
 *     with leading dimension n and is written in full (zeros below the
 *     diagonal);
 *   - 1 <= n <= RCLUPP_MAX_N, m >= n, ld >= m, and for the sketched
 *     methods n <= s <= m (Section 3: S is s x m with s = O(n)); s and seed
 *     are ignored by the unsketched methods; the tall kernels address a
 *     row tile with 32-bit offsets, so m + 3 ld < 2^29 (else
 *     RCLUPP_ERR_UNSUPPORTED); s <= 4096;
 *   - performance only: X and Q are streamed fastest when every column
 *     starts on a 128-byte line (pointer 128-byte aligned and ld a multiple
 *     of 16); any other ld is supported at a lower rate (the tall passes
 *     then keep lines cached between neighbouring row segments);
 *   - X is read only; X and Q must not overlap; Q and R are written only;
 *   - the sketch is S = G / sqrt(s) with G_ij a standard normal drawn from
 *     Philox4x32-10 (counter = (q lo, q hi, i, 0) with q = floor(j/4), key =
 *     (seed lo, seed hi), Box-Muller on the four 23-bit uniforms giving tall
 *     rows 4q .. 4q+3), a pure function of (seed, i, j); see rclupp_omega;
 *   - all work is enqueued on `stream` (a hipStream_t; NULL = default
 *     stream); calls return before the work finishes and never synchronize
 *     the device, except rclupp_last_info, rclupp_release and the first
 *     autotuned batched call for a batch shape;
 *   - synchronous errors (bad arguments, unsupported sizes, allocation or
 *     launch failures) are returned as an rclupp_status and nothing is
 *     enqueued for them;
 *   - numerical failures found on the device (a zero LU pivot, a Cholesky
 *     pivot that is not positive, non-finite data) are recorded in an
 *     rclupp_info on the device; the kernels after the failing stage see it
 *     and return at once; Q and R are then unspecified.
 *   - calls with different streams and different workspaces may run
 *     concurrently; the 9-argument forms draw their workspace from the
 *     library's stream-ordered pool.
 */
#ifndef RCLUPP_H
#define RCLUPP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RCLUPP_MAX_N 256

/* Synchronous status returned by every entry point. */
typedef enum {
  RCLUPP_OK = 0,
  RCLUPP_ERR_INVALID_ARG = 1, /* a size, pointer or leading dimension is invalid    */
  RCLUPP_ERR_UNSUPPORTED = 2, /* valid but not supported (e.g. n > RCLUPP_MAX_N)      */
  RCLUPP_ERR_ALLOC = 3,       /* device memory could not be obtained                 */
  RCLUPP_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed          */
  RCLUPP_ERR_WORKSPACE = 5,   /* the caller's workspace is smaller than required     */
  RCLUPP_ERR_SCRATCH_LIMIT = 6 /* rclupp_qr_noalloc: the sizes need more workspace than
                                  its fixed RCLUPP_NOALLOC_MAX_BYTES scratch             */
} rclupp_status;

/* Asynchronous numerical outcome, written on the device. */
typedef enum {
  RCLUPP_INFO_OK = 0,
  RCLUPP_INFO_LU_ZERO_PIVOT = 1,  /* LU with partial pivoting met an exactly zero column */
  RCLUPP_INFO_CHOL_BREAKDOWN = 2, /* a Cholesky pivot was not > 0                          */
  RCLUPP_INFO_NONFINITE = 3,      /* the input of a small factorization held NaN or Inf    */
  RCLUPP_INFO_SINGULAR = 4,       /* the preconditioner R_1 has an exactly zero diagonal   */
  RCLUPP_INFO_SYNC_TIMEOUT = 5    /* a bounded wait did not complete: a step of the
                                     multi-workgroup small factorization, or a panel inside
                                     a tournament-pivoting node (should not happen; the
                                     kernel exits rather than hang) */
} rclupp_info_code;

/* Stage = the role of the failing small factorization in the pipeline. */
typedef enum {
  RCLUPP_STAGE_NONE = 0,
  RCLUPP_STAGE_LU = 1,      /* LU of the sketch (RCLUPP) or of X (RCLUPPr, LC2)          */
  RCLUPP_STAGE_QR = 2,      /* R factor of the (sketched) L factor, or chol(M^T M) in LC2 */
  RCLUPP_STAGE_PRECOND = 3, /* R_1 = R_0 N, or the first (shifted) Cholesky               */
  RCLUPP_STAGE_CHOL_A = 4,  /* Cholesky of the first Gram after preconditioning (R_2)     */
  RCLUPP_STAGE_CHOL_B = 5,  /* Cholesky of the second Gram (R_4)                          */
  RCLUPP_STAGE_CHOL_X = 6   /* Cholesky of the extra pass of an escalated mixed-precision call */
} rclupp_stage;

/* index = 1-based column at which the stage failed. reserved: bit 0
 * (RCLUPP_NOTE_ESCALATED) is set when a mixed-precision RCLUPP or RCLUPPr call
 * found its preconditioner too weak for CholeskyQR2 and ran Shifted
 * CholeskyQR3's tail instead (see rclupp_opts). */
typedef struct {
  int32_t code;
  int32_t stage;
  int32_t index;
  int32_t reserved;
} rclupp_info;
#define RCLUPP_NOTE_ESCALATED 1

typedef enum { RCLUPP_PREC_FP64 = 0, RCLUPP_PREC_FP32 = 1, RCLUPP_PREC_BF16 = 2 } rclupp_prec;

/* Options of the full-control forms. A NULL pointer means all defaults (FP64).
 *   sketch_prec: arithmetic of the sketch product S X (or S M): FP64, or FP32 /
 *                BF16 MFMA with FP32 accumulation (the cross-workgroup sum is FP64);
 *   lu_prec:     arithmetic of the LU + Householder preconditioner on the s x n
 *                sketch: FP64 or FP32 (the result R_1 is widened to FP64).
 * Everything else (triangular solves, Gram, Cholesky, the final pass) is FP64.
 * With either option below FP64, RCLUPP and RCLUPPr check on the device that
 * Q_1 = X R_1^{-1} is within CholeskyQR2's range: when the Cholesky of
 * G_1 = Q_1^T Q_1 breaks down, or its diagonal spans more than a factor 1e9,
 * the call takes Algorithm 4's shifted Cholesky of G_1 and one more
 * CholeskyQR pass (Shifted CholeskyQR3 on Q_1; one extra pass over Q) and
 * sets RCLUPP_NOTE_ESCALATED in the outcome. */
typedef struct {
  int32_t sketch_prec;
  int32_t lu_prec;
  int32_t batch_flags; /* rclupp_qr_batched only: RCLUPP_BATCH_* bits       */
  int32_t sketch_kind; /* RCLUPP_SKETCH_GAUSSIAN (0), _COUNT (1) or _SRHT (2) */
  int32_t tall_lu;     /* RCLUPP_TALL_LU_PARTIAL (0) or RCLUPP_TALL_LU_TOURNAMENT */
  int32_t reserved[3];
} rclupp_opts;

/* tall_lu (RCLUPPr, LU-CholeskyQR2): the pivoting of the LU of X.
 *   RCLUPP_TALL_LU_PARTIAL: partial pivoting (LAPACK getrf order), as the
 *     paper's LU of X; M keeps the pivoted row order (the default);
 *   RCLUPP_TALL_LU_TOURNAMENT: tournament pivoting (TSLU, Grigori, Demmel and
 *     Xiang 2011), n <= 128 (else RCLUPP_ERR_UNSUPPORTED): the pivot rows are
 *     chosen by a tree of partial-pivoting eliminations over 256-row blocks
 *     (leaves: ceil(m / 256) blocks of consecutive rows; each node keeps its
 *     first n pivot rows; floor(256 / n) sets merge per node); N and the unit
 *     lower L_11 come from the root; M = P X N^{-1} is one substitution pass
 *     and is kept in X's row order (RCLUPPr's sketch then sees M through a
 *     column permutation of S, a Gaussian matrix of the same distribution).
 *     Its workspace (rclupp_workspace_size) holds, for n > 64, the candidate
 *     rows of the first two merge levels: about (1 + 1/F) (m / 256) n^2 / F
 *     doubles with F = floor(256 / n), 6.4 GB at m = 16,777,216, n = 128.
 *     A node that waits longer than its bounded wait for the previous panel
 *     reports RCLUPP_INFO_SYNC_TIMEOUT (stage LU) rather than hang. */
#define RCLUPP_TALL_LU_PARTIAL 0
#define RCLUPP_TALL_LU_TOURNAMENT 1

/* sketch_kind (RCLUPP, RCLUPPr, randomized CholeskyQR):
 *   RCLUPP_SKETCH_GAUSSIAN: S = G / sqrt(s), G i.i.d. standard normal
 *     (Section 3's Gaussian sketch; the default);
 *   RCLUPP_SKETCH_COUNT: the CountSketch (Section 3 lists it among the common
 *     choices): column j of S holds one entry sigma_j = +-1 in row h_j, drawn
 *     from Philox4x32-10 with counter (q lo, q hi, 0, 1), q = floor(j/4), key
 *     (seed lo, seed hi); word j mod 4 gives h_j = floor(w s / 2^32) and
 *     sigma_j = -1 for odd w, +1 for even. Y = S X is summed in FP64 (X read
 *     once, no generation cost); requires sketch_prec = FP64 and s <= 1792
 *     (else RCLUPP_ERR_UNSUPPORTED). Batches with it run problem by problem.
 *   RCLUPP_SKETCH_SRHT: the subsampled randomized Hadamard transform (Section
 *     3 lists it among the common choices), S = sqrt(m'/s) R H D with m' the
 *     smallest power of two >= m (X taken as padded with zero rows), D the
 *     diagonal of signs d_j, H the Walsh-Hadamard matrix of order m' in
 *     Sylvester order normalized by 1/sqrt(m'), R the rows r_0 .. r_{s-1}:
 *     entry (i, j) of S is (-1)^popcount(r_i & j) d_j / sqrt(s). d_j comes
 *     from Philox4x32-10 with counter (q lo, q hi, 0, 2), q = floor(j/4), key
 *     (seed lo, seed hi), word j mod 4, -1 for odd words; r_i = f3(f2(f1(i)))
 *     on k = log2 m' bits with f1(x) = a1 x + b1, f2(x) = x xor (x >> ceil(k/2)),
 *     f3(x) = a2 x + b2 (mod 2^k), (a1, b1, a2, b2) the words at counter
 *     (0, 0, 0, 3) with a1, a2 made odd: a bijection, so the rows are distinct.
 *     Y = S X is formed as a dense product in the precision of sketch_prec
 *     (the +-1 entries are exact in all three), with no Gaussian generation.
 *     Batches with it run problem by problem. */
#define RCLUPP_SKETCH_GAUSSIAN 0
#define RCLUPP_SKETCH_COUNT 1
#define RCLUPP_SKETCH_SRHT 2

/* batch_flags:
 *   RCLUPP_BATCH_GRAPH: capture the batch's launch sequence into a hipGraph
 *     on first use (keyed by every argument of the call) and replay it;
 *   RCLUPP_BATCH_AUTOTUNE: on the first call for a batch shape (n, s and m
 *     per problem, in 4096-row buckets), time the candidate rows-per-workgroup
 *     of the tall and sketch passes once (synchronizing the stream) and keep
 *     the fastest. Results are deterministic for a given choice; two choices
 *     differ by summation order only. */
#define RCLUPP_BATCH_GRAPH 1
#define RCLUPP_BATCH_AUTOTUNE 2

typedef enum {
  RCLUPP_ALG_RCLUPP = 0,   /* Algorithm 2 */
  RCLUPP_ALG_RCLUPPR = 1,  /* Algorithm 7 */
  RCLUPP_ALG_CHOLQR2 = 2,  /* Algorithm 3 */
  RCLUPP_ALG_SCHOLQR3 = 3, /* Algorithm 4, shift 11(mnu + n(n+1)u) max_j ||X_j||^2 */
  RCLUPP_ALG_LC2 = 4,      /* Algorithm 5 */
  RCLUPP_ALG_RCHOLQR = 5   /* Algorithm 6 */
} rclupp_alg;

/* ---------------------------------------------------------------------------
 * The method entry points (identical signatures). Workspace comes from the
 * library's stream-ordered pool; the numerical outcome is kept per stream and
 * read with rclupp_last_info.
 *   rclupp_qr   : Algorithm 2 (RCLUPP)
 *   rcluppr_qr  : Algorithm 7 (RCLUPPr)
 *   cholqr2_qr  : Algorithm 3 (CholeskyQR2; s, seed ignored)
 *   scholqr3_qr : Algorithm 4 (Shifted CholeskyQR3; s, seed ignored)
 *   lc2_qr      : Algorithm 5 (LU-CholeskyQR2; s, seed ignored)
 *   rcholqr_qr  : Algorithm 6 (randomized CholeskyQR, single sketch)
 * ------------------------------------------------------------------------- */
int rclupp_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
              hipStream_t stream);
int rcluppr_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
               hipStream_t stream);
int cholqr2_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
               hipStream_t stream);
int scholqr3_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
                hipStream_t stream);
int lc2_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
           hipStream_t stream);
int rcholqr_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
               hipStream_t stream);

/* Synchronizes `stream` and copies the outcome of the last 9-argument call
 * enqueued on it to *h_info (host pointer). Returns RCLUPP_ERR_INVALID_ARG if
 * no such call was made on this stream. */
int rclupp_last_info(hipStream_t stream, rclupp_info* h_info);

/* Static description of a status code. */
const char* rclupp_status_string(int status);

/* Frees every object the library keeps for the life of the process: the
 * pinned job tables and cached graphs of the batched form, its capture
 * streams and autotuning results, the stage-timing events and the per-stream
 * outcome slots of the 9-argument forms. It waits for the library's work on
 * the device to finish first. Afterwards the library can be used again
 * (rclupp_last_info then knows no earlier call). Meant for orderly shutdown
 * before the HIP runtime is torn down, e.g. from an exit handler. */
int rclupp_release(void);

/* ---------------------------------------------------------------------------
 * Full-control form: caller-owned workspace and device info.
 *   rclupp_workspace_size: bytes of device workspace needed by rclupp_qr_ex for
 *     these sizes and options (written to *bytes, a host pointer);
 *   rclupp_qr_ex: runs method `alg`; ws is a device buffer of ws_bytes bytes
 *     (256-byte aligned) owned by the caller and used only while the work
 *     runs on `stream`; d_info (device pointer, nullable) receives the outcome.
 * ------------------------------------------------------------------------- */
int rclupp_workspace_size(int alg, int64_t m, int64_t n, int64_t s, const rclupp_opts* opts, size_t* bytes);
int rclupp_qr_ex(int alg, const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q,
                 double* R, const rclupp_opts* opts, void* ws, size_t ws_bytes, rclupp_info* d_info,
                 hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Allocation-free form, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation as rclupp_qr_ex, with the workspace taken
 * from a fixed scratch array of RCLUPP_NOALLOC_MAX_BYTES bytes that the
 * library holds in device memory on every device it runs on, until the
 * process ends. The call allocates nothing (no hipMalloc, hipFree or pinned
 * host memory); the caller passes X, Q, R and, optionally, d_info (device
 * pointer; NULL means the outcome is not reported).
 *   - The workspace layout is rclupp_qr_ex's, except that when it would exceed
 *     the scratch the number of per-workgroup partial sums of the sketch and
 *     of the Gram passes is halved until it fits (results then differ from
 *     rclupp_qr_ex's by the order of those sums only). Sizes that still do not
 *     fit (e.g. RCLUPPr or LC2 with a tall LU whose pivot vector alone needs
 *     4m bytes) return RCLUPP_ERR_SCRATCH_LIMIT and enqueue nothing.
 *   - Every call on a device shares that device's scratch, which keeps the
 *     last call's contents (each call clears what it needs). Calls whose work
 *     overlaps on one device race, and give wrong results: enqueue them on one
 *     stream, or order them with events.
 *   - Other arguments, errors and the outcome are as for rclupp_qr_ex.
 * ------------------------------------------------------------------------- */
#define RCLUPP_NOALLOC_MAX_BYTES ((size_t)128 << 20)

int rclupp_qr_noalloc(int alg, const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed,
                      double* Q, double* R, const rclupp_opts* opts, rclupp_info* d_info, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched form: many independent problems in one call. h_probs is a HOST
 * array of `batch` descriptors whose matrix pointers are device pointers;
 * d_info (device, nullable) receives one rclupp_info per problem. A failure
 * in one problem does not affect the others. The workspace size depends on
 * the whole batch (rclupp_batched_workspace_size).
 * RCLUPP batches whose problems fit the register-resident small kernels
 * (n <= 128, s <= 256) run grouped: problems with equal (n, s) share one
 * launch per pipeline stage (tall and sketch passes split every problem into
 * row chunks, one workgroup each; small stages take one workgroup per
 * problem), optionally graph-captured and autotuned (opts->batch_flags).
 * Other batches run problem after problem with the single-problem pipeline.
 * The job tables are built on the host in pinned memory that the library
 * keeps (reused once the upload that read it has completed, freed by
 * rclupp_release) and uploaded on `stream`; the call does not wait for them.
 * Captured graphs are cached per argument set (16 entries, least recently
 * used evicted; an evicted graph is destroyed once its last replay is done).
 * h_probs is a host array because the grouping, the partition into
 * workgroups and the job tables are planned on the host before anything is
 * enqueued; alg takes the rclupp_alg values as a plain int (ABI-stable).
 * ------------------------------------------------------------------------- */
typedef struct {
  const double* X;
  double* Q;
  double* R;
  int64_t m, n, ld, s;
  uint64_t seed;
} rclupp_problem;

int rclupp_batched_workspace_size(int alg, const rclupp_problem* h_probs, int batch, const rclupp_opts* opts,
                                  size_t* bytes);
int rclupp_qr_batched(int alg, const rclupp_problem* h_probs, int batch, const rclupp_opts* opts, void* ws,
                      size_t ws_bytes, rclupp_info* d_info, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Step entry points: each runs one stage of the pipeline on its own, for
 * testing and profiling. Device pointers, column-major, enqueued on stream.
 * Scratch memory is drawn from the stream-ordered pool.
 * ------------------------------------------------------------------------- */

/* Raw G (unscaled standard normals, float32) of the sketch: G[i + c*s] =
 * z(seed, i, j0 + c) for i < s, c < cols (Section 3, Gaussian sketch). */
int rclupp_omega(uint64_t seed, int64_t s, int64_t j0, int64_t cols, float* G, hipStream_t stream);

/* Raw Philox4x32-10 words for `count` counters (host-visible check of the
 * generator): ctr = device uint32[4*count], key = (k0, k1), out = device
 * uint32[4*count]. */
int rclupp_philox(const uint32_t* ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t stream);

/* Y = S X (s x n, ld s): Algorithm 2 step 1, with `prec` an rclupp_prec.
 * FP64: exact products of the FP32 normals with X, FP64 sums. FP32: X rounded
 * to FP32, FP32 products and sums within a wave. BF16: G and X (through FP32)
 * rounded to BF16, FP32 sums within a wave. All forms add the per-wave and
 * per-workgroup partial sums in FP64 in a fixed order. FP32 and BF16 require
 * m + 16 ld < 2^32 (else RCLUPP_ERR_UNSUPPORTED). */
int rclupp_sketch(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, int prec, double* Y,
                  hipStream_t stream);

/* Y = S X (s x n, ld s) for the SRHT S of RCLUPP_SKETCH_SRHT, with `prec` an
 * rclupp_prec (as rclupp_sketch: FP64, or X rounded to FP32 or BF16); s <= m'
 * (the order of the Hadamard matrix), m < 2^30; FP32 and BF16 require
 * m + 16 ld < 2^32. */
int rclupp_srht(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, int prec, double* Y,
                hipStream_t stream);

/* Y = S X (s x n, ld s) for the CountSketch S of RCLUPP_SKETCH_COUNT (FP64
 * sums, s <= 1792). */
int rclupp_countsketch(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Y,
                       hipStream_t stream);

/* Preconditioner of the sketch (Algorithm 2 steps 2-4, Algorithm 6 step 2):
 * from Y (s x n, ld s) compute R1 (n x n, ld n) = D R_0 N with
 *   lu = 1: [M, N, P] = LU(Y) with partial pivoting, R_0 = R factor of M;
 *   lu = 0: R_0 = R factor of Y, N = I (randomized CholeskyQR);
 * D = sign(diag(R_0 N)). perm (device int32[s], nullable) receives the pivot
 * order (position -> original row); Mout (nullable, s x n, ld s) the unit lower
 * trapezoidal M. `prec` (FP64 or FP32) selects the arithmetic. */
int rclupp_precond(const double* Y, int64_t s, int64_t n, int lu, int prec, double* R1, int32_t* perm, double* Mout,
                   rclupp_info* d_info, hipStream_t stream);

/* Fused tall pass (Algorithm 1 steps 1 and 3 around a given R):
 *   W = X R^{-1} (row-wise substitution; R = NULL means R = I),
 *   G = W^T W (if G != NULL, n x n, ld n),
 * W (m x n, ld ldw) is written if W != NULL; W may equal X (in place). */
int rclupp_trsm_gram(const double* X, int64_t m, int64_t n, int64_t ldx, const double* R, double* W, int64_t ldw,
                     double* G, hipStream_t stream);

/* Cholesky R^T R = G + shift I (upper R, n x n, ld n), shift = 0 or, with
 * scholqr_shift = 1, 11(m n u + n(n+1) u) max_j G_jj (Algorithm 4). If Rprev is
 * not NULL, Rout = R Rprev is also written (nullable). */
int rclupp_chol(const double* G, int64_t n, int64_t m, int scholqr_shift, double* R, const double* Rprev,
                double* Rout, int32_t stage, rclupp_info* d_info, hipStream_t stream);

/* LU with partial pivoting of a tall X (m x n): M (m x n, ld ldm, rows in
 * pivoted order, unit diagonal implied below, N in its upper n x n part as in
 * LAPACK getrf), perm (device int32[m]: position -> original row). M must not
 * overlap X (X is read until the last column has entered M):
 * RCLUPP_ERR_INVALID_ARG otherwise. */
int rclupp_tall_lu(const double* X, int64_t m, int64_t n, int64_t ldx, double* M, int64_t ldm, int32_t* perm,
                   rclupp_info* d_info, hipStream_t stream);

/* Tournament pivoting of a tall X (m x n, n <= 128; see RCLUPP_TALL_LU_TOURNAMENT):
 * sel (device int32[n]) = the pivot rows in pivot order (original indices),
 * N (device, n x n, ld n) = the upper factor, M (m x n, ld ldm, X's row order)
 * = X N^{-1} with rows sel[k] equal to row k of the unit lower L_11, so that
 * X[sel, :] = L_11 N. */
int rclupp_tall_lu_tournament(const double* X, int64_t m, int64_t n, int64_t ldx, double* M, int64_t ldm,
                              int32_t* sel, double* N, rclupp_info* d_info, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Stage timing (profiling aid). rclupp_trace_enable(max_marks > 0) makes every
 * later rclupp_qr_ex call record a hipEvent on its stream before each stage
 * (sketch, sketch_reduce, precond, tall_lu, gram, trsm_gram, gram_reduce,
 * chol, trsm_final) and after its last stage, up to max_marks events in all;
 * max_marks = 0 turns it off. rclupp_trace_read synchronizes on the recorded
 * events, sums the elapsed time per stage name over all traced calls, writes
 * up to max_stages entries (names: max_stages x name_len chars, ms: total
 * milliseconds, launches: number of occurrences; host arrays), sets *count to
 * the number of distinct stages and clears the record.
 * ------------------------------------------------------------------------- */
int rclupp_trace_enable(int max_marks);
int rclupp_trace_read(int max_stages, char* names, int name_len, float* ms, int* launches, int* count);

#ifdef __cplusplus
}
#endif

#endif /* RCLUPP_H */
