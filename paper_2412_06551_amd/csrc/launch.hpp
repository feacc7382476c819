// Host-side launchers of the gfx950 kernels (internal interface between the
// C ABI in capi.hip and the kernel translation units). Every launcher checks
// its own shape assumptions and returns hipSuccess or the launch error.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rclupp {

// ---- batched (grouped) launches ----------------------------------------------
// A batched launch runs one stage for many problems of the same n and s. Each
// workgroup reads an item (problem index, its workgroup index and count within
// that problem) and the problem's job record; the per-problem partition of the
// work is the same as a single launch with `nwg` workgroups.
struct BatchItem {
  int32_t prob, wg, nwg, pad;
};
struct TallJob {
  const double* X;
  int64_t ldx, m, ntiles;
  const double* Rp;
  double* W;
  int64_t ldw;
  double* Gpart;
  const int32_t* info;
};
struct SketchJob {
  const double* X;
  int64_t m, ld, ntiles;
  uint64_t seed;
  double* Ypart;
  const int32_t* info;
};
struct ReduceJob {
  const double* part;  // per-workgroup partials
  double* lvl;         // level-1 sums
  double* out;         // final result (Y or G)
  int32_t nparts, splits;
  const int32_t* info;
};
struct PrecondJob {
  const double* Y;
  double* R1pad;
  double* scratch;
  int32_t* info;
};
struct CholJob {
  const double* G;
  double* Rpad;
  double* Rout;
  const double* Rprev;
  int32_t* info;
  int64_t m;
};

// Padded column count used by the tall kernels: 16, 32, 64, 128 or 256.
int pad_cols(int64_t n);
// Padded sketch rows used by the sketch kernels (multiple of 64).
int64_t pad_sketch_rows(int64_t s);

// Deterministic two-level reduction of per-workgroup partial sums (k_tall.hip):
// lvl[y][e] = sum over the workgroups of split y (in order) of part[b][e].
int reduce_splits(int nparts);
hipError_t launch_partial_sum(const double* part, int nparts, int64_t stride, int splits, double* lvl,
                              const int32_t* info, hipStream_t st);

// ---- sketch (k_sketch.hip) --------------------------------------------------
struct SketchPlan {
  int sm;          // sketch rows per wave (16: one M-block)
  int nn;          // columns (all of them, padded: 16 .. 256)
  int gx;          // row chunks (workgroups per sketch-row group)
  int gy, gz;      // sketch-row groups, column groups (gz = 1)
  bool wm;         // each wave owns its own sketch rows (always)
  int nw;          // waves per workgroup (8, or 4 when s_pad is not a multiple of 128)
  int64_t s_pad;   // padded sketch rows (gy * nw * sm)
  int64_t n_pad;   // padded columns (nn)
  int64_t ntiles;  // 32-row tiles of the tall operand (CountSketch: 4096 / nn rows)
  size_t part_bytes;  // bytes of the per-chunk partial sums and their level-1 sums
  int kind;        // 0 Gaussian, 1 CountSketch (nn = column slice, gz slices; nn = 0: unsupported), 2 SRHT
};
SketchPlan plan_sketch(int64_t m, int64_t n, int64_t s, int prec, int gx_hint);
SketchPlan plan_countsketch(int64_t m, int64_t n, int64_t s, int gx_hint);
// CountSketch partials Ypart[gx][s_pad x n_pad] (the same layout and reduction
// as the Gaussian sketch's, with scale 1).
hipError_t launch_countsketch_partials(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld,
                                       int64_t s, uint64_t seed, double* Ypart, const int32_t* info, hipStream_t st);
// Ypart[gx][s_pad x n_pad] partial sums of G[:, rows] X[rows, :] (G unscaled).
hipError_t launch_sketch_partials(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld, uint64_t seed,
                                  int prec, double* Ypart, const int32_t* info, hipStream_t st);
// Y[i + j*s] = scale * sum_b Ypart[b][i + j*s_pad] for i < s, j < n.
hipError_t launch_sketch_reduce(const SketchPlan& p, const double* Ypart, int64_t s, int64_t n, double scale, double* Y,
                                const int32_t* info, hipStream_t st);
hipError_t launch_omega(uint64_t seed, int64_t s, int64_t j0, int64_t cols, float* G, hipStream_t st);
hipError_t launch_philox(const uint32_t* ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t st);

// ---- tall passes (k_tall.hip) -------------------------------------------------
// R operands of the tall kernels are "padded triangles": NP x NP row-major
// (element (i, j) at i*NP + j) with identity padding beyond n, followed by NP
// reciprocals of the diagonal.
inline size_t padded_r_doubles(int np) { return (size_t)np * np + np; }

struct TallPlan {
  int np;          // padded columns
  int gx;          // workgroups of the passes with a Gram (= Gram partials)
  int gx_solve;    // workgroups of the passes without one
  int64_t ntiles;  // row tiles
  int tile_rows;   // rows per tile
  bool fused_gram; // Gram computed inside the TRSM kernel (np <= 64)
  size_t part_bytes;  // bytes of per-workgroup Gram partials (gx * np * np doubles)
};
TallPlan plan_tall(int64_t m, int64_t n, int gx_hint);
// W = X R^{-1} (R == nullptr: W = X), Gpart (nullable) = per-workgroup W^T W.
// W == nullptr: W is not written. W may equal X.
hipError_t launch_tall_pass(const TallPlan& p, const double* X, int64_t ldx, int64_t m, int64_t n, const double* Rpad,
                            double* W, int64_t ldw, double* Gpart, const int32_t* info, hipStream_t st);
// G (np x np, ld np, upper + mirrored, padded) = sum over workgroup partials.
hipError_t launch_gram_reduce(const TallPlan& p, const double* Gpart, int64_t n, double* G, const int32_t* info,
                              hipStream_t st);

// ---- small dense kernels (k_small.hip) ------------------------------------------
// Preconditioner from the s x n sketch Y (ld s): R1pad (padded triangle) =
// D R_0 N. lu: LU with partial pivoting first (RCLUPP) or not (RCholeskyQR).
// Nin (nullable): an external N (n x n, ld ldn) multiplies R_0 instead of the
// LU's own N (RCLUPPr: N comes from the LU of X). prec: 0 FP64, 1 FP32.
size_t precond_scratch_bytes(int64_t s, int64_t n);
hipError_t launch_precond(const double* Y, int64_t s, int64_t n, int lu, int prec, const double* Nin, int64_t ldn,
                          double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch, int32_t* info,
                          int32_t stage_qr, hipStream_t st);
// Cholesky of G (+ shift) into Rpad; Rout = R * Rprev (both padded or user
// layout). shift_mode: 0 none, 1 = Algorithm 4's shift with m. post: optional
// right factor Npost (LC2: R_1 = D S_c N) with sign fix.
size_t chol_scratch_bytes(int64_t n);
hipError_t launch_chol(const double* G, int ldg, int64_t n, int64_t m, int shift_mode, double* Rpad, double* Rout,
                       int rout_user, const double* Rprev, const double* Npost, int64_t ldnp, double* scratch,
                       int32_t* info, int32_t stage, hipStream_t st);
// Register-resident forms for n <= 128 (k_dense.hip); launch_precond and
// launch_chol route to them. For n > 64 the preconditioner keeps its two n x n
// tables in `scratch` (precond_reg_scratch_bytes()).
bool precond_reg_fits(int64_t s, int64_t n);
size_t precond_reg_scratch_bytes();
hipError_t launch_precond_reg(const double* Y, int64_t s, int64_t n, int lu, int prec, const double* Nin, int64_t ldn,
                              double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch,
                              int32_t* info, int32_t stage_qr, hipStream_t st);
hipError_t launch_chol_reg(const double* G, int ldg, int64_t n, int64_t m, int shift_mode, double* Rpad, double* Rout,
                           int rout_user, const double* Rprev, const double* Npost, int64_t ldnp, int32_t* info,
                           int32_t stage, hipStream_t st);
// Copy a padded triangle to a user n x n matrix.
hipError_t launch_unpad(const double* Rpad, int64_t n, double* R, hipStream_t st);
// Build a padded triangle (R and reciprocal diagonal) from a user n x n matrix.
hipError_t launch_pad(const double* R, int64_t n, double* Rpad, hipStream_t st);
hipError_t launch_set_identity_pad(int np, int64_t n, double* Rpad, hipStream_t st);

// ---- tall LU (k_tall_lu.hip) ----------------------------------------------------
size_t tall_lu_scratch_bytes(int64_t m, int64_t n);
// LU with partial pivoting of X (m x n) into M (rows in pivoted order, N in the
// upper n x n), perm[pos] = original row. Also writes Npad = the n x n factor N
// (user layout n x n, ld n) if Nout != nullptr.
hipError_t launch_tall_lu(const double* X, int64_t m, int64_t n, int64_t ldx, double* M, int64_t ldm, int32_t* perm,
                          double* Nout, double* scratch, int32_t* info, hipStream_t st);
// Tournament pivoting (k_tslu.hip), n <= 128: sel[0..n) = the pivot rows (original
// indices, pivot order), Nout (nullable, n x n, ld n) = N, W (m x n, ld ldw, X's
// row order) = X N^{-1} with the rows sel[k] holding L_11's rows exactly.
int64_t tslu_leaves(int64_t m);
size_t tslu_scratch_bytes(int64_t m, int64_t n);
hipError_t launch_tslu(const double* X, int64_t m, int64_t n, int64_t ldx, double* W, int64_t ldw, int32_t* sel,
                       double* Nout, double* scratch, int32_t* info, hipStream_t st);
// M <- unit lower trapezoid of the packed LU (zero above, one on the diagonal).
hipError_t launch_unit_lower(double* M, int64_t m, int64_t n, int64_t ldm, const int32_t* info, hipStream_t st);

// ---- batched launchers ---------------------------------------------------------
hipError_t launch_sketch_batch(const SketchPlan& p, int64_t n, int prec, const SketchJob* jobs, const BatchItem* items,
                               int nitems, hipStream_t st);
hipError_t launch_sketch_final_batch(const SketchPlan& p, int64_t s, int64_t n, double scale, const ReduceJob* jobs,
                                     int count, hipStream_t st);
hipError_t launch_tall_batch(int np, int n, bool trsm, bool gram, bool write, const TallJob* jobs,
                             const BatchItem* items, int nitems, hipStream_t st);
hipError_t launch_partial_sum_batch(int64_t stride, const ReduceJob* jobs, const BatchItem* items, int nitems,
                                    hipStream_t st);
hipError_t launch_gram_final_batch(int np, int64_t n, const ReduceJob* jobs, int count, hipStream_t st);
hipError_t launch_precond_batch(int64_t s, int64_t n, int prec, const PrecondJob* jobs, int count, int32_t stage_qr,
                                hipStream_t st);
hipError_t launch_chol_batch(int64_t n, int ldg, int rout_user, const CholJob* jobs, int count, int32_t stage,
                             hipStream_t st);

}  // namespace rclupp
