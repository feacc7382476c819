// LU with partial pivoting of the tall X (m x n), P X = M N (Algorithm 7 step
// 1, Algorithm 5 step 1), blocked right-looking:
//   per column k of a panel: one workgroup reduces the per-workgroup argmax
//     partials of |column k| (first row wins ties, LAPACK idamax), swaps rows
//     k and p across all n columns and keeps the pivot row; then every
//     workgroup scales its part of column k and updates the remaining panel
//     columns, and records the argmax partial of column k+1;
//   per panel: U12 = L11^{-1} A12 (one workgroup), then the trailing update
//     A22 -= L21 U12 streams every row once and records the argmax partial of
//     the next panel's first column.
// Three levels of panels: a 4-column panel updates only the rest of its
// 16-column block, a 16-column block only the rest of its 32-column block,
// and a 32-column block the rest of the matrix (each update: U12 of the
// block's rows, then A22 -= L21 U12 with the block's columns of L), so a
// column is streamed once per block of each level that precedes it instead of
// once per panel. Row swaps act on all n columns at once (a row's multipliers
// and its not yet updated entries move together). The per-element update
// order equals that of the unblocked algorithm: every element receives the
// rank-1 updates of the steps in step order, each one fused multiply-add (an
// update applies its block's steps in order).
// M is stored with its rows in pivoted order (position p holds original row
// perm[p]); the upper n x n part holds N as in LAPACK getrf.
// X is not copied into M first: a column enters M when a kernel first updates
// it (the first column step for the first panel, the first update of each
// level for the columns it covers), reading row i from X's row perm[i]; until
// then a row swap only exchanges perm entries (and writes the new pivot row
// into M), since a column no step has updated yet is X's column permuted.
#include <limits.h>

#include "device_common.hpp"
#include "launch.hpp"

namespace rclupp {

constexpr int LU_THREADS = 256;
// panel widths of the three levels (a panel of LU_W0 columns is factored
// column by column; LU_NB bounds the columns one column step reads per row)
constexpr int LU_W0 = 4, LU_W1 = 16, LU_W2 = 32;
constexpr int LU_NB = 8;
static_assert(LU_W0 <= LU_NB, "a column step reads at most LU_NB columns");
constexpr int LU_GRID = 1024;

struct LuPartial {
  double v;
  int idx;
  int bad;
};

// Block reduce (max |v|, lowest index on ties, OR of bad) and write one partial.
__device__ void wg_argmax_write(double v, int idx, int bad, LuPartial* out) {
  __shared__ double sv[LU_THREADS / 64];
  __shared__ int si[LU_THREADS / 64], sb[LU_THREADS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    const int ob = __shfl_xor(bad, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
    bad |= ob;
  }
  if (lane == 0) {
    sv[wave] = v;
    si[wave] = idx;
    sb[wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = sv[0];
    int bi = si[0], bb = sb[0];
    for (int w = 1; w < LU_THREADS / 64; ++w) {
      if (sv[w] > bv || (sv[w] == bv && si[w] < bi)) {
        bv = sv[w];
        bi = si[w];
      }
      bb |= sb[w];
    }
    out->v = bv;
    out->idx = bi;
    out->bad = bb;
  }
}

__device__ __forceinline__ void track(double a, int64_t i, double& best, int& idx, int& bad) {
  if (!is_finite(a)) bad = 1;
  const double v = fabs(a);
  if (v > best) {
    best = v;
    idx = (int)i;
  }
}

// perm = identity, argmax partials of column 0 (read from X).
__global__ __launch_bounds__(LU_THREADS) void k_lu_init(const double* __restrict__ X, int64_t m,
                                                        int32_t* __restrict__ perm, LuPartial* part,
                                                        const int32_t* info) {
  if (info_failed(info)) return;
  double best = -1.0;
  int idx = INT_MAX, bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * LU_THREADS + threadIdx.x; i < m; i += (int64_t)gridDim.x * LU_THREADS) {
    perm[i] = (int32_t)i;
    track(X[i], i, best, idx, bad);
  }
  wg_argmax_write(best, idx, bad, part + blockIdx.x);
}

// Pivot of column k: reduce partials, test, swap rows k and p, keep the pivot row.
// (columns f .. n - 1 are not in M yet: only perm is swapped there, and the
// new pivot row's entries are read from X)
__global__ __launch_bounds__(LU_THREADS) void k_lu_pivot(double* __restrict__ M, int64_t ldm, int n, int k,
                                                         int32_t* __restrict__ perm, const LuPartial* __restrict__ part,
                                                         int nparts, double* __restrict__ prow,
                                                         const double* __restrict__ X, int64_t ldx, int f,
                                                         int32_t* info) {
  __shared__ int s_p, s_fail, s_row;
  __shared__ double rv[LU_THREADS / 64];
  __shared__ int ri[LU_THREADS / 64], rb[LU_THREADS / 64];
  if (info_failed(info)) return;
  // reduce the partials in parallel (max |v|, lowest index on ties, OR of bad:
  // the result does not depend on the order)
  {
    double bv = -1.0;
    int bi = INT_MAX, bb = 0;
    for (int w = threadIdx.x; w < nparts; w += LU_THREADS) {
      const LuPartial q = part[w];
      if (q.v > bv || (q.v == bv && q.idx < bi)) {
        bv = q.v;
        bi = q.idx;
      }
      bb |= q.bad;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      const int ob = __shfl_xor(bb, off);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
      bb |= ob;
    }
    if (lane == 0) {
      rv[wave] = bv;
      ri[wave] = bi;
      rb[wave] = bb;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = rv[0];
    int bi = ri[0], bb = rb[0];
    for (int w = 1; w < LU_THREADS / 64; ++w) {
      if (rv[w] > bv || (rv[w] == bv && ri[w] < bi)) {
        bv = rv[w];
        bi = ri[w];
      }
      bb |= rb[w];
    }
    s_fail = 0;
    if (bb) {
      info_set(info, INFO_NONFINITE, STAGE_LU, k + 1);
      s_fail = 1;
    } else if (!(bv > 0.0)) {
      info_set(info, INFO_LU_ZERO_PIVOT, STAGE_LU, k + 1);
      s_fail = 1;
    }
    s_p = bi;
    if (!s_fail && bi != k) {
      const int32_t t = perm[k];
      perm[k] = perm[bi];
      perm[bi] = t;
    }
    s_row = perm[k];
  }
  __syncthreads();
  if (s_fail) return;
  const int p = s_p;
  const int64_t xk = s_row;
  for (int j = threadIdx.x; j < n; j += LU_THREADS) {
    if (j < f) {
      const double a = M[k + j * ldm];
      const double b = M[p + j * ldm];
      if (p != k) {
        M[k + j * ldm] = b;
        M[p + j * ldm] = a;
      }
      prow[j] = b;
    } else {
      const double b = X[xk + (int64_t)j * ldx];
      M[k + j * ldm] = b;
      prow[j] = b;
    }
  }
}

// Panel update at step k: rows i > k.
// (from_x: the panel's columns enter M here, read from X's rows perm[i])
__global__ __launch_bounds__(LU_THREADS) void k_lu_panel(double* __restrict__ M, int64_t ldm, int64_t m, int k, int c1,
                                                         const double* __restrict__ prow, LuPartial* part,
                                                         int want_next, const double* __restrict__ X, int64_t ldx,
                                                         const int32_t* __restrict__ perm, int from_x,
                                                         const int32_t* info) {
  if (info_failed(info)) return;
  const double piv = prow[k];
  double best = -1.0;
  int idx = INT_MAX, bad = 0;
  for (int64_t i = (int64_t)k + 1 + (int64_t)blockIdx.x * LU_THREADS + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * LU_THREADS) {
    // the row's columns k .. c1 - 1 of the panel (at most LU_NB) are read
    // before any is written, so that their loads are in flight together
    const double* src = from_x ? X + perm[i] : M + i;
    const int64_t ld = from_x ? ldx : ldm;
    double v[LU_NB];
#pragma unroll
    for (int q = 0; q < LU_NB; ++q) v[q] = (k + q < c1) ? src[(int64_t)(k + q) * ld] : 0.0;
    const double l = v[0] / piv;
    M[i + (int64_t)k * ldm] = l;
#pragma unroll
    for (int q = 1; q < LU_NB; ++q) {
      if (k + q < c1) {
        const double a = v[q] - l * prow[k + q];
        M[i + (int64_t)(k + q) * ldm] = a;
        if (q == 1) track(a, i, best, idx, bad);
      }
    }
  }
  if (want_next) wg_argmax_write(best, idx, bad, part + blockIdx.x);
}

// U12 = L11^{-1} A12 in place for the rows c0 .. c1 - 1 (c1 - c0 <= NB) and
// the columns cs .. ce - 1 (at most LU_THREADS of them): forward substitution
// with the unit lower L11 (in LDS), each column in a thread's registers, every
// entry taking its terms in step order.
template <int NB>
__global__ __launch_bounds__(LU_THREADS) void k_lu_trsm12(double* __restrict__ M, int64_t ldm, int c0, int c1, int cs,
                                                          int ce, const int32_t* info) {
  if (info_failed(info)) return;
  __shared__ double L11[NB * NB];  // (r, q) at r + q NB, zero outside the block
  const int nb = c1 - c0;
  for (int e = threadIdx.x; e < NB * NB; e += LU_THREADS) {
    const int r = e % NB, q = e / NB;
    L11[e] = (r < nb && q < nb) ? M[(c0 + r) + (int64_t)(c0 + q) * ldm] : 0.0;
  }
  __syncthreads();
  // one column per thread (ce - cs <= n - 1 < LU_THREADS)
  const int j = cs + (int)threadIdx.x;
  if (j < ce) {
    // rows beyond the block read its last row instead (in range; those
    // entries meet only zero entries of L11 and are not written back)
    const double* col = M + (int64_t)j * ldm;
    double a[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) a[r] = col[c0 + (r < nb ? r : nb - 1)];
    // step q (in order) updates the rows after it
#pragma unroll
    for (int q = 0; q + 1 < NB; ++q) {
#pragma unroll
      for (int r = q + 1; r < NB; ++r) a[r] -= L11[r + q * NB] * a[q];
    }
    double* out = M + (int64_t)j * ldm + c0;
#pragma unroll
    for (int r = 1; r < NB; ++r)
      if (r < nb) out[r] = a[r];
  }
}

// The same for the wider blocks (c1 - c0 <= NB): each thread's column lives in
// LDS instead of registers (128 threads, columns taken in turn), with the same
// order of terms.
constexpr int LU_TRSM_LDS_THREADS = 128;
template <int NB>
__global__ __launch_bounds__(LU_TRSM_LDS_THREADS) void k_lu_trsm12_lds(double* __restrict__ M, int64_t ldm, int c0,
                                                                        int c1, int cs, int ce, const int32_t* info) {
  if (info_failed(info)) return;
  __shared__ double L11[NB * NB];                   // (r, q) at r + q NB
  __shared__ double A[NB * LU_TRSM_LDS_THREADS];   // thread's row r at r * threads + thread
  const int nb = c1 - c0;
  for (int e = threadIdx.x; e < nb * nb; e += LU_TRSM_LDS_THREADS) {
    const int r = e % nb, q = e / nb;
    L11[r + q * NB] = M[(c0 + r) + (int64_t)(c0 + q) * ldm];
  }
  __syncthreads();
  double* a = A + threadIdx.x;
  for (int j = cs + (int)threadIdx.x; j < ce; j += LU_TRSM_LDS_THREADS) {
    const double* col = M + (int64_t)j * ldm + c0;
    for (int r = 0; r < nb; ++r) a[r * LU_TRSM_LDS_THREADS] = col[r];
    for (int q = 0; q + 1 < nb; ++q) {
      const double aq = a[q * LU_TRSM_LDS_THREADS];
      for (int r = q + 1; r < nb; ++r) a[r * LU_TRSM_LDS_THREADS] -= L11[r + q * NB] * aq;
    }
    double* out = M + (int64_t)j * ldm + c0;
    for (int r = 1; r < nb; ++r) out[r] = a[r * LU_TRSM_LDS_THREADS];
  }
}

// A22 -= L21 U12 for the rows c1 .. m - 1 and the columns c1 .. ce - 1, with
// the L columns c0 .. c1 - 1 (c1 - c0 <= NB); records the argmax partial of
// column c1. U12 (nb x nt) is staged in dynamic LDS. Steps beyond nb carry a
// zero multiplier and a zero U12 entry, which leave every element unchanged
// (fma(-0, 0, a) = a, signed zeros included). FROM_X: the columns c1 .. ce - 1
// enter M here, read from X's rows perm[i] (a template argument, so that the
// other form keeps its loads and stores on M alone).
template <int NB, bool FROM_X>
__global__ __launch_bounds__(LU_THREADS) void k_lu_trailing(double* __restrict__ M, int64_t ldm, int64_t m, int c0,
                                                            int c1, int ce, LuPartial* part,
                                                            const double* __restrict__ X, int64_t ldx,
                                                            const int32_t* __restrict__ perm, const int32_t* info) {
  if (info_failed(info)) return;
  extern __shared__ double u[];  // (t, j) at t + j NB
  const int nb = c1 - c0, nt = ce - c1;
  for (int e = threadIdx.x; e < NB * nt; e += LU_THREADS) {
    const int q = e % NB, j = e / NB;
    u[e] = (q < nb) ? M[(c0 + q) + (int64_t)(c1 + j) * ldm] : 0.0;
  }
  __syncthreads();
  double best = -1.0;
  int idx = INT_MAX, bad = 0;
  for (int64_t i = (int64_t)c1 + (int64_t)blockIdx.x * LU_THREADS + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * LU_THREADS) {
    double l[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) l[q] = (q < nb) ? M[i + (int64_t)(c0 + q) * ldm] : 0.0;
    // the row's entry of column c (FROM_X: the row's original in X)
    const double* xr = FROM_X ? X + perm[i] : nullptr;
    auto at = [&](int c) -> const double* { return FROM_X ? xr + (int64_t)c * ldx : M + i + (int64_t)c * ldm; };
    // column c1 first (its argmax partial), then eight columns at a time so
    // that eight loads are in flight per thread, then the rest one by one
    // (issuing the rest's loads together measured no faster)
    {
      double a = *at(c1);
#pragma unroll
      for (int q = 0; q < NB; ++q) a -= l[q] * u[q];
      M[i + (int64_t)c1 * ldm] = a;
      track(a, i, best, idx, bad);
    }
    int j = 1;
    for (; j + 7 < nt; j += 8) {
      double a[8];
#pragma unroll
      for (int w = 0; w < 8; ++w) a[w] = __builtin_nontemporal_load(at(c1 + j + w));
#pragma unroll
      for (int w = 0; w < 8; ++w) {
#pragma unroll
        for (int q = 0; q < NB; ++q) a[w] -= l[q] * u[q + (j + w) * NB];
        __builtin_nontemporal_store(a[w], M + i + (int64_t)(c1 + j + w) * ldm);
      }
    }
    for (; j < nt; ++j) {
      double a = *at(c1 + j);
#pragma unroll
      for (int q = 0; q < NB; ++q) a -= l[q] * u[q + j * NB];
      M[i + (int64_t)(c1 + j) * ldm] = a;
    }
  }
  wg_argmax_write(best, idx, bad, part + blockIdx.x);
}

__global__ void k_lu_extract_n(const double* __restrict__ M, int64_t ldm, int n, double* __restrict__ N,
                               const int32_t* info) {
  if (info_failed(info)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e % n, j = e / n;
  N[e] = (i <= j) ? M[i + (int64_t)j * ldm] : 0.0;
}

__global__ void k_unit_lower(double* __restrict__ M, int64_t ldm, int n, const int32_t* info) {
  if (info_failed(info)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e % n, j = e / n;
  if (i <= j) M[i + (int64_t)j * ldm] = (i == j) ? 1.0 : 0.0;
}

size_t tall_lu_scratch_bytes(int64_t m, int64_t n) {
  (void)n;
  size_t b = (size_t)LU_GRID * sizeof(LuPartial);
  b = (b + 255) / 256 * 256;
  b += ((size_t)RCLUPP_SMALL_MAXN * sizeof(double) + 255) / 256 * 256;  // prow
  (void)m;
  return b;
}

hipError_t launch_tall_lu(const double* X, int64_t m, int64_t n, int64_t ldx, double* M, int64_t ldm, int32_t* perm,
                          double* Nout, double* scratch, int32_t* info, hipStream_t st) {
  if (n < 1 || n > RCLUPP_SMALL_MAXN || m < n) return hipErrorInvalidValue;
  LuPartial* part = (LuPartial*)scratch;
  size_t off = ((size_t)LU_GRID * sizeof(LuPartial) + 255) / 256 * 256;
  double* prow = (double*)((char*)scratch + off);
  int64_t rows_blocks = (m + LU_THREADS - 1) / LU_THREADS;
  const int g = (int)(rows_blocks < LU_GRID ? rows_blocks : LU_GRID);
  hipLaunchKernelGGL(k_lu_init, dim3(g), dim3(LU_THREADS), 0, st, X, m, perm, part, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // columns 0 .. f - 1 are in M; every kernel below updates either columns
  // all in M or columns all outside it, which it then brings in (f grows to
  // the end of its range)
  int f = 0;
  // the update of the columns c1 .. ce - 1 by the steps c0 .. c1 - 1 (U12,
  // then A22 -= L21 U12), which also records the argmax partial of column c1
  auto update = [&](int c0, int c1, int ce) -> hipError_t {
    if (c1 < f && ce > f) return hipErrorInvalidValue;  // not reached: the blocks nest
    const int from_x = c1 >= f ? 1 : 0;
    const size_t lds = (size_t)(ce - c1) * sizeof(double);
#define LU_TRAILING(NB)                                                                                             \
  if (from_x)                                                                                                        \
    hipLaunchKernelGGL((k_lu_trailing<NB, true>), dim3(g), dim3(LU_THREADS), NB * lds, st, M, ldm, m, c0, c1, ce,     \
                       part, X, ldx, perm, info);                                                                    \
  else                                                                                                               \
    hipLaunchKernelGGL((k_lu_trailing<NB, false>), dim3(g), dim3(LU_THREADS), NB * lds, st, M, ldm, m, c0, c1, ce,    \
                       part, X, ldx, perm, info);
    if (c1 - c0 <= LU_W0) {
      hipLaunchKernelGGL(k_lu_trsm12<LU_W0>, dim3(1), dim3(LU_THREADS), 0, st, M, ldm, c0, c1, c1, ce, info);
      LU_TRAILING(LU_W0)
    } else if (c1 - c0 <= LU_W1) {
      hipLaunchKernelGGL(k_lu_trsm12_lds<LU_W1>, dim3(1), dim3(LU_TRSM_LDS_THREADS), 0, st, M, ldm, c0, c1, c1, ce,
                         info);
      LU_TRAILING(LU_W1)
    } else {
      hipLaunchKernelGGL(k_lu_trsm12_lds<LU_W2>, dim3(1), dim3(LU_TRSM_LDS_THREADS), 0, st, M, ldm, c0, c1, c1, ce,
                         info);
      LU_TRAILING(LU_W2)
    }
#undef LU_TRAILING
    if (from_x) f = ce;
    return hipGetLastError();
  };
  // blocks of LU_W2 columns, made of blocks of LU_W1 columns, made of panels
  // of LU_W0 columns; each (sub-)block, once factored, updates the rest of
  // the block that holds it (the outermost: the rest of the matrix)
  for (int b0 = 0; b0 < n; b0 += LU_W2) {
    const int b1 = (int)((b0 + LU_W2 < n) ? b0 + LU_W2 : n);
    for (int s0 = b0; s0 < b1; s0 += LU_W1) {
      const int s1 = (s0 + LU_W1 < b1) ? s0 + LU_W1 : b1;
      for (int c0 = s0; c0 < s1; c0 += LU_W0) {
        const int c1 = (c0 + LU_W0 < s1) ? c0 + LU_W0 : s1;
        for (int k = c0; k < c1; ++k) {
          if (k < f && c1 > f) return hipErrorInvalidValue;  // not reached: panels start outside M or inside it
          hipLaunchKernelGGL(k_lu_pivot, dim3(1), dim3(LU_THREADS), 0, st, M, ldm, (int)n, k, perm, part, g, prow, X,
                             ldx, f, info);
          const int want_next = (k + 1 < c1) ? 1 : 0;
          const int from_x = k >= f ? 1 : 0;
          hipLaunchKernelGGL(k_lu_panel, dim3(g), dim3(LU_THREADS), 0, st, M, ldm, m, k, c1, prow, part, want_next, X,
                             ldx, perm, from_x, info);
          if (from_x) f = c1;
        }
        if (c1 < s1 && (e = update(c0, c1, s1)) != hipSuccess) return e;
      }
      if (s1 < b1 && (e = update(s0, s1, b1)) != hipSuccess) return e;
    }
    if (b1 < n && (e = update(b0, b1, (int)n)) != hipSuccess) return e;
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (Nout) {
    hipLaunchKernelGGL(k_lu_extract_n, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, M, ldm, (int)n, Nout,
                       info);
  }
  return hipGetLastError();
}

hipError_t launch_unit_lower(double* M, int64_t m, int64_t n, int64_t ldm, const int32_t* info, hipStream_t st) {
  (void)m;
  hipLaunchKernelGGL(k_unit_lower, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, M, ldm, (int)n, info);
  return hipGetLastError();
}

}  // namespace rclupp
