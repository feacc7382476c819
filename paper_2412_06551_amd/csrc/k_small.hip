// Small dense stages for the shapes the register-resident kernels of
// k_dense.hip cannot hold (s > 256 or n > 128):
//   k_precond_coop : [M, N, P] = LU(Y) with partial pivoting (eq. elu), R_0 =
//               R factor of M by Householder reflections (eq. eh, Q_s never
//               formed), R_1 = D R_0 N with D = sign(diag(R_0 N)) (eq. ey)
//               (Algorithm 2 steps 2-4; Algorithm 7 steps 3-4 with an external
//               N; Algorithm 6 step 2 without the LU); several workgroups,
//               each step published by its owner and awaited point to point;
//   k_chol_blk : upper Cholesky of G (+ the shift of Algorithm 4) for n in
//               (128, 256], blocked on one workgroup with MFMA trailing updates;
//   k_trmm_pad : the product with an earlier factor (R_3 = R_2 R_1,
//               R = R_4 R_3; eqs. C4, C8) on many workgroups;
//   k_chol    : the column-at-a-time Cholesky with the optional right factor
//               (LC2's R_1 = D S_c N), one workgroup (O(n^3), latency bound);
//               used for that right factor when n > 128.
// k_chol keeps its working copy in LDS when it fits, else in a global scratch
// buffer (same code through generic pointers). Threads form a 64 x 16 grid: tx
// walks rows (contiguous in the column-major layout), ty walks columns; the
// column loops keep SD_U loads in flight per thread (the working copy is in L2
// when it does not fit LDS, and one outstanding load per thread left them
// latency bound).
#include <float.h>
#include <limits.h>

#include "device_common.hpp"
#include "launch.hpp"

namespace rclupp {

constexpr int SD_THREADS = 1024;
constexpr int SD_WAVES = SD_THREADS / 64;
constexpr int SD_U = 4;  // independent loads in flight per thread in the column loops
constexpr size_t SD_LDS_LIMIT = 150 * 1024;

struct ArgMaxSh {
  double v[SD_WAVES];
  int i[SD_WAVES];
  int bad[SD_WAVES];
  int p;
  int pbad;
  double pv;
};

// Block-wide argmax of v (first index wins ties); `bad` is OR-reduced.
__device__ void block_argmax(double& v, int& idx, int& bad, ArgMaxSh* sh) {
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
    sh->v[wave] = v;
    sh->i[wave] = idx;
    sh->bad[wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = sh->v[0];
    int bi = sh->i[0], bb = sh->bad[0];
    for (int w = 1; w < SD_THREADS / 64; ++w) {
      if (sh->v[w] > bv || (sh->v[w] == bv && sh->i[w] < bi)) {
        bv = sh->v[w];
        bi = sh->i[w];
      }
      bb |= sh->bad[w];
    }
    sh->pv = bv;
    sh->p = bi;
    sh->pbad = bb;
  }
  __syncthreads();
  v = sh->pv;
  idx = sh->p;
  bad = sh->pbad;
}


template <typename T>
__device__ __forceinline__ T tabs(T v) {
  return v < T(0) ? -v : v;
}

// Padded triangle: np x np ROW-major (element (i, j) at i*np + j) with the
// identity beyond n, then np reciprocals of the diagonal.
__device__ void write_padded(const double* R /* n x n generic */, int ldr, int n, int np, double* Rpad) {
  for (int e = threadIdx.x; e < np * np; e += SD_THREADS) {
    const int i = e / np, j = e % np;
    double v;
    if (i < n && j < n)
      v = (i <= j) ? R[i + j * ldr] : 0.0;
    else
      v = (i == j) ? 1.0 : 0.0;
    Rpad[e] = v;
  }
  for (int j = threadIdx.x; j < np; j += SD_THREADS) Rpad[np * np + j] = (j < n) ? 1.0 / R[j + j * ldr] : 1.0;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SD_THREADS) void k_chol(const double* __restrict__ G, int ldg, int n, int64_t m,
                                                     int shift_mode, double* Rpad, int np, double* Rout, int rout_user,
                                                     const double* __restrict__ Rprev, const double* __restrict__ Npost,
                                                     int ldnp, double* gA, double* gT, int use_lds, int32_t* info,
                                                     int32_t stage) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ ArgMaxSh amx;
  __shared__ double sh_r;
  __shared__ int fail;
  if (info_failed(info)) return;
  double* A = use_lds ? (double*)smem_raw : gA;  // n x n, ld n
  double* Tm = gT;                               // n x n temporary
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  for (int e = tid; e < n * n; e += SD_THREADS) {
    const int i = e % n, j = e / n;
    A[e] = (i <= j) ? G[i + (int64_t)j * ldg] : 0.0;
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  {
    double v = -1e300;
    int idx = INT_MAX, bad = 0;
    for (int e = tid; e < n * n; e += SD_THREADS) {
      const int i = e % n, j = e / n;
      if (i <= j && !is_finite(A[e]) && j < idx) {
        idx = j;
        bad = 1;
      }
    }
    v = bad ? -(double)idx : -1e300;
    block_argmax(v, idx, bad, &amx);
    if (bad) {
      if (tid == 0) info_set(info, INFO_NONFINITE, stage, (int32_t)(-v) + 1);
      return;
    }
  }
  if (shift_mode == 1) {
    double gm = 0.0;
    int idx = 0, bad = 0;
    for (int j = tid; j < n; j += SD_THREADS) gm = fmax(gm, A[j + j * n]);
    block_argmax(gm, idx, bad, &amx);
    const double u = 0x1p-53;
    const double sigma = 11.0 * ((double)m * (double)n * u + (double)n * (double)(n + 1) * u) * gm;
    for (int j = tid; j < n; j += SD_THREADS) A[j + j * n] += sigma;
    __syncthreads();
  }
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double d = A[k + k * n];
      if (!(d > 0.0)) {
        info_set(info, INFO_CHOL_BREAKDOWN, stage, k + 1);
        fail = 1;
      } else {
        sh_r = sqrt(d);
      }
    }
    __syncthreads();
    if (fail) return;
    const double rkk = sh_r;
    for (int j = k + 1 + tid; j < n; j += SD_THREADS) A[k + j * n] = A[k + j * n] / rkk;
    if (tid == 0) A[k + k * n] = rkk;
    __syncthreads();
    for (int j = k + 1 + ty; j < n; j += SD_WAVES) {
      const double akj = A[k + j * n];
      double* cj = A + (size_t)j * n;
      int i = k + 1 + tx;
      for (; i + 64 * (SD_U - 1) <= j; i += 64 * SD_U) {
        double a[SD_U], l[SD_U];
#pragma unroll
        for (int u = 0; u < SD_U; ++u) {
          a[u] = cj[i + 64 * u];
          l[u] = A[k + (size_t)(i + 64 * u) * n];
        }
#pragma unroll
        for (int u = 0; u < SD_U; ++u) cj[i + 64 * u] = a[u] - l[u] * akj;
      }
      for (; i <= j; i += 64) cj[i] = cj[i] - A[k + (size_t)i * n] * akj;
    }
    __syncthreads();
  }
  // optional right factor with sign fix (LC2: R_1 = D S_c N)
  if (Npost) {
    for (int e = tid; e < n * n; e += SD_THREADS) {
      const int i = e % n, j = e / n;
      double part[SD_U] = {};
      if (i <= j) {
        int k = i;
        for (; k + SD_U - 1 <= j; k += SD_U)
#pragma unroll
          for (int u = 0; u < SD_U; ++u) part[u] += A[i + (k + u) * n] * Npost[k + u + (int64_t)j * ldnp];
        for (; k <= j; ++k) part[0] += A[i + k * n] * Npost[k + (int64_t)j * ldnp];
      }
      double acc = part[0];
#pragma unroll
      for (int u = 1; u < SD_U; ++u) acc += part[u];
      Tm[e] = acc;
    }
    __syncthreads();
    if (tid == 0) {
      for (int i = 0; i < n; ++i) {
        const double d = Tm[i + i * n];
        if (!is_finite(d)) {
          info_set(info, INFO_NONFINITE, STAGE_PRECOND, i + 1);
          fail = 1;
          break;
        }
        if (d == 0.0) {
          info_set(info, INFO_SINGULAR, STAGE_PRECOND, i + 1);
          fail = 1;
          break;
        }
      }
    }
    __syncthreads();
    if (fail) return;
    for (int e = tid; e < n * n; e += SD_THREADS) {
      const int i = e % n;
      const double d = Tm[i + i * n];
      A[e] = (d < 0.0) ? -Tm[e] : Tm[e];
    }
    __syncthreads();
  }
  write_padded(A, n, n, np, Rpad);
  if (Rout) {
    // Rout = R * Rprev, Rprev a padded triangle (ld np)
    for (int e = tid; e < n * n; e += SD_THREADS) {
      const int i = e % n, j = e / n;
      double part[SD_U] = {};
      if (i <= j) {
        int k = i;
        for (; k + SD_U - 1 <= j; k += SD_U)
#pragma unroll
          for (int u = 0; u < SD_U; ++u) part[u] += A[i + (k + u) * n] * Rprev[(int64_t)(k + u) * np + j];
        for (; k <= j; ++k) part[0] += A[i + k * n] * Rprev[(int64_t)k * np + j];
      }
      double acc = part[0];
#pragma unroll
      for (int u = 1; u < SD_U; ++u) acc += part[u];
      if (rout_user)
        Rout[e] = acc;
      else
        Tm[e] = acc;
    }
    if (!rout_user) {
      __syncthreads();
      write_padded(Tm, n, n, np, Rout);
    }
  }
}

// Lane src's value (src a compile-time constant in the unrolled loops below),
// as a wave-uniform scalar.
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src), hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// ---------------------------------------------------------------------------
// Blocked Cholesky for n in (128, 256] without a right factor: the upper
// factor of G (+ the shift of Algorithm 4) by 16-column blocks, right-looking.
// Per block column K:
//   1. the 16 x 16 diagonal block by unblocked steps on 16 lanes of wave 0
//      (lane j holds column j; row k of the block is broadcast lane by lane);
//   2. the block row R_KJ = R_KK^{-T} A_KJ by substitution, one thread per
//      column;
//   3. the trailing update A_IJ -= R_KI^T R_KJ for K < I <= J on FP64 MFMA,
//      16 x 16 blocks dealt round-robin to the waves.
// The matrix is padded to np x np with the identity (its factor is R padded
// with the identity) and kept row-major (element (i, j) at j + i np, the
// padded triangle's own layout) in a global scratch buffer that stays in L2;
// only its upper block triangle is used. Row-major makes every access below
// a run of consecutive addresses across lanes (the MFMA layouts put the
// column index on lane % 16; the block row walks columns across threads). Inside a block every
// entry takes its terms in ascending order (fma; quotients correctly rounded
// from one reciprocal, as in the register-resident kernels); across blocks
// the matrix cores sum four terms at a time, so R agrees with the
// column-at-a-time form to rounding. The one-workgroup column-at-a-time form
// took 10 us per column at n = 256 (its updates are dependent L2 loads).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SD_THREADS) void k_chol_blk(const double* __restrict__ G, int ldg, int n, int64_t m,
                                                         int shift_mode, double* __restrict__ Rpad, int np,
                                                         double* __restrict__ A, int32_t* info, int32_t stage) {
  __shared__ ArgMaxSh amx;
  __shared__ int fail;
  __shared__ double rkk_l[16 * 17];  // R_KK (row i, column j at i * 17 + j)
  __shared__ double yk_l[16];        // RN(1 / r_ii)
  if (info_failed(info)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int nb = np / 16, total = np * np;
  // copy in (eight loads in flight per thread: the copy loops are latency
  // bound on one workgroup) and find the lowest column with a non-finite
  // entry in the upper triangle
  int idx = INT_MAX, bad = 0;
  for (int e0 = tid; e0 < total; e0 += 8 * SD_THREADS) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * SD_THREADS, i = e % np, j = e / np;
      v[u] = (e < total && i < n && j < n) ? (i <= j ? G[i + (int64_t)j * ldg] : 0.0) : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * SD_THREADS, i = e % np, j = e / np;
      if (e < total) {
        A[j + (int64_t)i * np] = v[u];
        if (!is_finite(v[u]) && j < idx) {
          idx = j;
          bad = 1;
        }
      }
    }
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  {
    double v = bad ? -(double)idx : -1e300;
    block_argmax(v, idx, bad, &amx);
    if (bad) {
      if (tid == 0) info_set(info, INFO_NONFINITE, stage, (int32_t)(-v) + 1);
      return;
    }
  }
  if (shift_mode == 1) {
    double gm = 0.0;
    int idx = 0, bad = 0;
    for (int j = tid; j < n; j += SD_THREADS) gm = fmax(gm, A[j + (int64_t)j * np]);  // (the diagonal)
    block_argmax(gm, idx, bad, &amx);
    const double u = 0x1p-53;
    const double sigma = 11.0 * ((double)m * (double)n * u + (double)n * (double)(n + 1) * u) * gm;
    for (int j = tid; j < n; j += SD_THREADS) A[j + (int64_t)j * np] += sigma;
    __syncthreads();
  }
  for (int K = 0; K < nb; ++K) {
    const int k0 = 16 * K;
    // 1. diagonal block
    if (wave == 0) {
      double c[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) c[i] = (lane < 16 && i <= lane) ? A[k0 + lane + (int64_t)(k0 + i) * np] : 0.0;
      // (no early exit: the loops stay unrolled, so every index below is a
      // constant; after a breakdown the remaining steps run on a dummy pivot
      // and nothing is stored)
      bool ok = true;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double d = lane_bcast(c[k], k);
        if (ok && !(d > 0.0)) {
          if (lane == 0) {
            info_set(info, INFO_CHOL_BREAKDOWN, stage, k0 + k + 1);
            fail = 1;
          }
          ok = false;
        }
        const double r = sqrt(ok ? d : 1.0), y = 1.0 / r;
        // row k: r_kj = a_kj / r_kk (Markstein's corrected quotient)
        const double q0 = c[k] * y;
        const double q = __builtin_fma(__builtin_fma(-q0, r, c[k]), y, q0);
        c[k] = (lane == k) ? r : ((lane > k) ? q : c[k]);
        if (lane == 0) yk_l[k] = y;
#pragma unroll
        for (int i = k + 1; i < 16; ++i) {
          const double rki = lane_bcast(c[k], i);
          if (lane >= i) c[i] = __builtin_fma(-rki, c[k], c[i]);
        }
      }
      if (ok && lane < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          if (i <= lane) A[k0 + lane + (int64_t)(k0 + i) * np] = c[i];
          rkk_l[i * 17 + lane] = (i <= lane) ? c[i] : 0.0;
        }
      }
    }
    __syncthreads();
    if (fail) return;
    // 2. block row: column c of the trailing part, x = R_KK^{-T} a
    const int ncol = np - k0 - 16;
    if (tid < ncol) {
      const int64_t col = k0 + 16 + tid;
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = A[col + (int64_t)(k0 + i) * np];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
#pragma unroll
        for (int p = 0; p < i; ++p) x[i] = __builtin_fma(-rkk_l[p * 17 + i], x[p], x[i]);
        const double r = rkk_l[i * 17 + i], y = yk_l[i];
        const double q0 = x[i] * y;
        x[i] = __builtin_fma(__builtin_fma(-q0, r, x[i]), y, q0);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) A[col + (int64_t)(k0 + i) * np] = x[i];
    }
    __syncthreads();
    // 3. trailing blocks K < I <= J
    const int nt = nb - K - 1, nblk = nt * (nt + 1) / 2;
    // (two blocks per round: their L2 loads are in flight together)
    for (int t0 = wave; t0 < nblk; t0 += 2 * SD_WAVES) {
      f64x4 acc[2];
      double fa[2][4], fb[2][4];
      int Ib[2], Jb[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        int J = 0, g = t0 + u * SD_WAVES;
        if (g >= nblk) g = t0;  // (a repeat of the first block, not stored)
        while (g > J) {
          g -= J + 1;
          ++J;
        }
        Ib[u] = K + 1 + g;
        Jb[u] = K + 1 + J;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[u][r] = A[16 * Jb[u] + lr + (int64_t)(16 * Ib[u] + lq + 4 * r) * np];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          fa[u][kk] = -A[16 * Ib[u] + lr + (int64_t)(k0 + 4 * kk + lq) * np];
          fb[u][kk] = A[16 * Jb[u] + lr + (int64_t)(k0 + 4 * kk + lq) * np];
        }
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[u] = mfma_f64(fa[u][kk], fb[u][kk], acc[u]);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (t0 + u * SD_WAVES < nblk) {
#pragma unroll
          for (int r = 0; r < 4; ++r) A[16 * Jb[u] + lr + (int64_t)(16 * Ib[u] + lq + 4 * r) * np] = acc[u][r];
        }
      }
    }
    __syncthreads();
  }
  for (int e0 = tid; e0 < total; e0 += 8 * SD_THREADS) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * SD_THREADS, i = e / np, j = e % np;
      v[u] = (e < total && i <= j) ? A[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * SD_THREADS;
      if (e < total) Rpad[e] = v[u];
    }
  }
  for (int j = tid; j < np; j += SD_THREADS) Rpad[np * np + j] = 1.0 / A[j + (int64_t)j * np];
}

// Rout = R Rprev for two padded triangles (row-major np x np, identity
// padding beyond n; eqs. C4, C8: R_3 = R_2 R_1, R = R_4 R_3) on FP64 MFMA: one
// wave per 16 x 16 output block, R's block row times Rprev's block column over
// K = I..J (both factors are upper triangular). The output is the user layout
// (column-major n x n, zeros below the diagonal) or a padded triangle with the
// reciprocals of its diagonal. Many small workgroups: the single-workgroup
// product read both factors from L2 one dependent load at a time.
__global__ __launch_bounds__(64) void k_trmm_pad(const double* __restrict__ Rpad, const double* __restrict__ Rprev,
                                                 int np, int n, double* __restrict__ Rout, int rout_user,
                                                 const int32_t* info) {
  if (info_failed(info)) return;
  const int nb = np / 16, I = blockIdx.x / nb, J = blockIdx.x % nb;
  const int lane = threadIdx.x, lr = lane & 15, lq = lane >> 4;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int K = I; K <= J; ++K)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double av = Rpad[(int64_t)(16 * I + lr) * np + 16 * K + 4 * kk + lq];
      const double bv = Rprev[(int64_t)(16 * K + 4 * kk + lq) * np + 16 * J + lr];
      acc = mfma_f64(av, bv, acc);
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 16 * I + lq + 4 * r, j = 16 * J + lr;
    if (rout_user) {
      if (i < n && j < n) Rout[i + (int64_t)j * n] = (i > j) ? 0.0 : acc[r];
    } else {
      Rout[(int64_t)i * np + j] = (i < n && j < n) ? ((i > j) ? 0.0 : acc[r]) : (i == j ? 1.0 : 0.0);
      if (i == j) Rout[(int64_t)np * np + i] = (i < n) ? 1.0 / acc[r] : 1.0;
    }
  }
}

__global__ void k_unpad(const double* __restrict__ Rpad, int np, int n, double* __restrict__ R) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e % n, j = e / n;
  R[e] = (i <= j) ? Rpad[i * np + j] : 0.0;
}

__global__ void k_pad(const double* __restrict__ R, int n, int np, double* __restrict__ Rpad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < np * np) {
    const int i = e / np, j = e % np;
    Rpad[e] = (i < n && j < n) ? ((i <= j) ? R[i + j * n] : 0.0) : (i == j ? 1.0 : 0.0);
  }
  if (e < np) Rpad[np * np + e] = (e < n) ? 1.0 / R[e + e * n] : 1.0;
}

// ---------------------------------------------------------------------------
// Preconditioner for the shapes the register-resident kernel cannot hold
// (s > 256 or n > 128), one cooperative launch of G workgroups: column j lives
// in the LDS of workgroup j % G (cpw columns each). The LU steps and then the
// Householder steps form one sequence; step k is published by the owner of
// its column: it finds the pivot (LU) or forms the reflector (Householder),
// writes the pivot or the scale and the multipliers or the reflector into
// slot k mod CP_RING of a ring in global memory, and raises the step's flag.
// Every other workgroup waits for that flag alone (no grid-wide barrier) and
// applies the step to its own columns, in step order. The owner of column
// k + 1 applies step k to that column first and publishes step k + 1 before
// updating its other columns (look-ahead), so the next step's search overlaps
// the other workgroups' updates. Each workgroup counts the steps it has
// finished; an owner reuses a ring slot only when every workgroup is past the
// step that used it last. Rows are swapped physically in every column (the
// finished ones too, as getrf does), so no position bookkeeping is needed. The
// multipliers are true quotients (so the LU factor equals the oracle's bit for
// bit, as k_precond_reg's does); dlarfg's beta = -sign(alpha) hypot(alpha, |x|).
// Every wait is bounded: a wait that does not end records INFO_SYNC_TIMEOUT
// and the kernel exits. A failing owner (zero pivot or non-finite column)
// records it, sets the failure word and raises its flag, so every workgroup
// stops at that step.
// ---------------------------------------------------------------------------
constexpr int CP_THREADS = 256;
constexpr int CP_WAVES = CP_THREADS / 64;
constexpr int CP_RING = 16;  // ring slots of published steps

struct CoopCtl {
  unsigned count, gen;  // grid barrier (start and end of the kernel): arrivals, generation
  int mincol;           // lowest column with a non-finite entry (no LU)
};

// Global state of the flow: control block, step flags (2n), finished-step
// counts (G), and the ring of published vectors (CP_RING slots of s + 1
// doubles: the multipliers or the reflector, then tau). A step's flag carries
// its result: LU step, pivot row + 1 (-1: the step failed); Householder step, 1.
struct CoopState {
  CoopCtl* ctl;
  int* flag;
  int* done;
  double* ring;
};

size_t coop_ctl_bytes() { return (sizeof(CoopCtl) + 255) / 256 * 256; }
size_t coop_state_bytes(int64_t s, int64_t n, int G) {
  return coop_ctl_bytes() + ((size_t)(2 * n + G) * sizeof(int) + 255) / 256 * 256 +
         (size_t)CP_RING * (s + 1) * sizeof(double);
}

__global__ void k_coop_ctl_init(CoopCtl* c, int* words, int nwords) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->count = 0;
    c->gen = 0;
    c->mincol = INT_MAX;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) words[i] = 0;
}

// All G workgroups arrive; false if this workgroup's bounded wait ran out.
// The workgroup barrier makes every wave's stores complete in this CU's L2
// before thread 0's agent-scope release (which writes that L2 back, for the
// other XCDs); thread 0's acquire invalidates this CU's caches before the
// workgroup barrier lets the other waves read. One fence pair per workgroup:
// each is a cache-wide operation.
__device__ bool coop_barrier(CoopCtl* c, unsigned nblocks) {
  __shared__ int timed_out;
  __syncthreads();
  if (threadIdx.x == 0) {
    timed_out = 0;
    __threadfence();  // release: this workgroup's writes before the arrival
    const unsigned g = __hip_atomic_load(&c->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (atomicAdd(&c->count, 1u) == nblocks - 1) {
      __hip_atomic_store(&c->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      atomicAdd(&c->gen, 1u);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&c->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1u << 24)) {
          timed_out = 1;
          break;
        }
      }
    }
    __threadfence();  // acquire: the other workgroups' writes after the wait
  }
  __syncthreads();
  return timed_out == 0;
}

__device__ __forceinline__ int cp_load_i(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double cp_load_d(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish step k with its flag value: every wave's stores of the step are in
// this CU's L2 after the workgroup barrier; thread 0's agent-scope release
// writes them back before the flag rises (the same pattern as coop_barrier's
// arrival).
__device__ void cp_publish(int* flag, int k, int value) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_store(flag + k, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Wait for step k's flag (thread 0, bounded), then acquire; returns the flag
// value to every thread (0 on time-out).
__device__ int cp_wait_flag(const int* flag, int k) {
  __shared__ int value;
  if (threadIdx.x == 0) {
    unsigned spins = 0;
    int v;
    while ((v = cp_load_i(flag + k)) == 0) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 24)) break;
    }
    __threadfence();
    value = v;
  }
  __syncthreads();
  return value;
}

// Before an owner overwrites the ring slot of step k: wait until every
// workgroup has finished step k - CP_RING (wave 0 reads the G counts). The
// smallest count seen is kept in *seen (LDS), so the counts are read again
// only when that bound no longer suffices (about once per CP_RING steps).
// False on time-out.
__device__ bool cp_wait_slot(const int* done, int G, int k, int* seen) {
  __shared__ int timed_out;
  const int need = k - CP_RING + 1;
  if (need <= *seen) return true;  // (uniform: *seen changes only below, before a barrier)
  if (threadIdx.x < 64) {
    unsigned spins = 0;
    int to = 0;
    for (;;) {
      int lo = INT_MAX;
      for (int w = threadIdx.x; w < G; w += 64) lo = min(lo, cp_load_i(done + w));
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) lo = min(lo, __shfl_xor(lo, off));
      if (lo >= need) {
        if (threadIdx.x == 0) *seen = lo;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 24)) {
        to = 1;
        break;
      }
    }
    if (threadIdx.x == 0) timed_out = to;
  }
  __syncthreads();
  return timed_out == 0;
}

// Sum over the workgroup of NV values per thread (each thread gets the sums).
template <int NV, typename T>
__device__ void cp_sum(T (&v)[NV], T* sh /* [CP_WAVES][NV] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off);
    if (lane == 0) sh[wave * NV + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    T r = sh[q];
    for (int w = 1; w < CP_WAVES; ++w) r += sh[w * NV + q];
    v[q] = r;
  }
  __syncthreads();
}

constexpr int CP_MAXC = 8;  // columns per workgroup at most

template <typename T>
__global__ __launch_bounds__(CP_THREADS) void k_precond_coop(const double* __restrict__ Y, int s, int n, int lu,
                                                             const double* __restrict__ Nin, int ldn, double* R1pad,
                                                             int np, double* R1out, int32_t* perm_out, double* Mout,
                                                             double* Ng, double* R0g, int32_t* permg, CoopState st,
                                                             int cpw, int32_t* info, int32_t stage_qr) {
  extern __shared__ __align__(16) unsigned char cp_smem[];
  T* cols = (T*)cp_smem;  // local column q (global g + q G) at q*s
  __shared__ T shr[CP_WAVES * CP_MAXC];
  __shared__ double amv[CP_WAVES];
  __shared__ int ami[CP_WAVES], amb[CP_WAVES];
  __shared__ int my_piv, seen_done;
  __shared__ T my_tau;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const unsigned nb = (unsigned)G;
  CoopCtl* ctl = st.ctl;
  (void)cpw;  // the LDS holds cpw columns; G = ceil(n / cpw) keeps every workgroup's count within it
  // (no workgroup writes info before the first barrier, so all read the same)
  if (info_failed(info)) return;
  auto col = [&](int q) { return cols + (size_t)q * s; };
  auto slot = [&](int k) { return st.ring + (size_t)(k % CP_RING) * (s + 1); };
  const int nloc = (n - g + G - 1) / G;  // columns of this workgroup
  const int lusteps = lu ? n : 0;        // QR step k (column k) is step lusteps + k
#pragma unroll
  for (int q = 0; q < CP_MAXC; ++q) {
    if (q >= nloc) break;
    const int j = g + q * G;
    for (int i = tid; i < s; i += CP_THREADS) col(q)[i] = (T)Y[i + (int64_t)j * s];
  }
  if (tid == 0) seen_done = 0;
  if (!coop_barrier(ctl, nb)) goto timeout;

  if (lu) {
    // owner of column k: pivot search, swap, multipliers, publish (false: failed
    // or timed out, and the workgroup stops)
    auto lu_owner = [&](int k) -> int {
      T* c = col(k / G);
      if (!cp_wait_slot(st.done, G, k, &seen_done)) return -1;
      double best = -1.0;
      int idx = INT_MAX, bad = 0;
      for (int i = k + tid; i < s; i += CP_THREADS) {
        const double a = (double)c[i];
        if (!is_finite(a)) bad = 1;
        const double v = fabs(a);
        if (v > best) {
          best = v;
          idx = i;
        }
      }
      // workgroup argmax, first row on ties
      const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(idx, off);
        const int ob = __shfl_xor(bad, off);
        if (ov > best || (ov == best && oi < idx)) {
          best = ov;
          idx = oi;
        }
        bad |= ob;
      }
      if (lane == 0) {
        amv[wave] = best;
        ami[wave] = idx;
        amb[wave] = bad;
      }
      __syncthreads();
      best = amv[0];
      idx = ami[0];
      bad = amb[0];
      for (int w = 1; w < CP_WAVES; ++w) {
        if (amv[w] > best || (amv[w] == best && ami[w] < idx)) {
          best = amv[w];
          idx = ami[w];
        }
        bad |= amb[w];
      }
      if (bad || !(best > 0.0)) {
        if (tid == 0) info_set(info, bad ? INFO_NONFINITE : INFO_LU_ZERO_PIVOT, STAGE_LU, k + 1);
        cp_publish(st.flag, k, -1);
        return 0;
      }
      const int p = idx;
      const T piv = c[p];
      const T ck = c[k];
      __syncthreads();
      if (tid == 0) {
        c[k] = piv;
        c[p] = ck;
        permg[k] = p;  // pivot history (the permutation is replayed at the end)
        my_piv = p;
      }
      __syncthreads();
      // multipliers RN(x / piv): one reciprocal y = RN(1 / piv), then
      // q0 = RN(x y) and RN(q0 + (x - q0 piv) y), the correctly rounded quotient
      // by Markstein's theorem when y is normal; a subnormal pivot or one above
      // 1 / (smallest normal) divides directly (as the register kernel does)
      const T ap = fabs(piv);
      const T tiny = sizeof(T) == 8 ? (T)DBL_MIN : (T)FLT_MIN;
      const bool direct = ap < tiny || ap > T(1) / tiny;
      const T y = T(1) / piv;
      double* v = slot(k);
      for (int i = k + 1 + tid; i < s; i += CP_THREADS) {
        const T x = c[i];
        T l;
        if (direct) {
          l = x / piv;
        } else {
          const T q0 = x * y;
          l = fma(fma(-q0, piv, x), y, q0);
        }
        c[i] = l;
        v[i] = (double)l;
      }
      cp_publish(st.flag, k, p + 1);
      return 1;
    };
    // step k (pivot row p, multipliers in its slot) on local column q (j > k)
    // or, for a finished column (j < k), the row swap alone; the reads of the
    // two rows happen before the caller's barrier
    auto lu_apply = [&](int k, int p, int q, T akj, T okk) {
      const int j = g + q * G;
      T* c = col(q);
      if (j < k) {
        if (tid == 0 && p != k) {
          c[k] = akj;
          c[p] = okk;
        }
        return;
      }
      const double* v = slot(k);
      for (int i = k + tid; i < s; i += CP_THREADS) {
        if (i == k) {
          c[k] = akj;
        } else {
          const T l = (T)v[i];
          const T a = (i == p) ? okk : c[i];
          c[i] = a - l * akj;
        }
      }
    };

    if (g == 0) {
      const int r = lu_owner(0);
      if (r < 0) goto timeout;
      if (r == 0) return;
    }
    for (int k = 0; k < n; ++k) {
      const int owner = k % G;
      int p;
      if (owner == g) {
        p = my_piv;
      } else {
        const int f = cp_wait_flag(st.flag, k);
        if (f == 0) goto timeout;
        if (f < 0) return;  // the owner failed and recorded it
        p = f - 1;
      }
      // look-ahead: column k + 1 first, then its step
      const int qa = (k + 1 < n && (k + 1) % G == g) ? (k + 1) / G : -1;
      if (qa >= 0) {
        T* c = col(qa);
        const T akj = c[p], okk = c[k];
        __syncthreads();
        lu_apply(k, p, qa, akj, okk);
        __syncthreads();
        const int r = lu_owner(k + 1);
        if (r < 0) goto timeout;
        if (r == 0) return;
      }
      // the other local columns (all but column k itself and the look-ahead one)
      T akj[CP_MAXC], okk[CP_MAXC];
#pragma unroll
      for (int q = 0; q < CP_MAXC; ++q) {
        if (q >= nloc) break;
        const int j = g + q * G;
        if (j != k && q != qa) {
          akj[q] = col(q)[p];
          okk[q] = col(q)[k];
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < CP_MAXC; ++q) {
        if (q >= nloc) break;
        const int j = g + q * G;
        if (j == k || q == qa) continue;
        lu_apply(k, p, q, akj[q], okk[q]);
      }
      __syncthreads();
      if (tid == 0) __hip_atomic_store(st.done + g, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // N = the upper n x n part; M = unit lower trapezoid
#pragma unroll
    for (int q = 0; q < CP_MAXC; ++q) {
      if (q >= nloc) break;
      const int j = g + q * G;
      T* c = col(q);
      for (int i = tid; i < n; i += CP_THREADS) {
        Ng[i + (int64_t)j * n] = (i <= j) ? (double)c[i] : 0.0;
        if (i <= j) c[i] = (i == j) ? T(1) : T(0);
      }
      if (Mout)
        for (int i = tid; i < s; i += CP_THREADS) Mout[i + (int64_t)j * s] = (double)c[i];
    }
    __syncthreads();
  } else {
    // M = Y; N external (upper part) or the identity; non-finite entries of M
    // are reported before the reflections (lowest column)
    int lowest = INT_MAX;
#pragma unroll
    for (int q = 0; q < CP_MAXC; ++q) {
      if (q >= nloc) break;
      const int j = g + q * G;
      for (int i = tid; i < s; i += CP_THREADS)
        if (!is_finite((double)col(q)[i]) && j < lowest) lowest = j;
      for (int i = tid; i < n; i += CP_THREADS)
        Ng[i + (int64_t)j * n] = Nin ? ((i <= j) ? Nin[i + (int64_t)j * ldn] : 0.0) : (i == j ? 1.0 : 0.0);
    }
    if (lowest != INT_MAX) atomicMin(&ctl->mincol, lowest);
    if (!coop_barrier(ctl, nb)) goto timeout;
    const int mc = cp_load_i(&ctl->mincol);
    if (mc != INT_MAX) {
      if (g == 0 && tid == 0) info_set(info, INFO_NONFINITE, stage_qr, mc + 1);
      return;
    }
  }

  {
    // Householder reflections (LAPACK dlarfg convention); column k is step
    // lusteps + k. The owner forms the reflector of its column and publishes
    // it with tau (tau = 0: the identity).
    auto qr_owner = [&](int k) -> bool {
      const int step = lusteps + k;
      T* c = col(k / G);
      if (!cp_wait_slot(st.done, G, step, &seen_done)) return false;
      T part[1] = {T(0)};
      for (int i = k + 1 + tid; i < s; i += CP_THREADS) part[0] += c[i] * c[i];
      cp_sum<1>(part, shr);
      const T al = c[k];
      const T xnorm = sqrt(part[0]);
      T tau = T(0), scal = T(0), beta = al;
      if (xnorm != T(0)) {
        beta = -copysign(hypot(al, xnorm), al);
        tau = (beta - al) / beta;
        scal = T(1) / (al - beta);
      }
      double* v = slot(step);
      if (tau != T(0)) {
        for (int i = k + 1 + tid; i < s; i += CP_THREADS) {
          const T vi = c[i] * scal;
          c[i] = vi;
          v[i] = (double)vi;
        }
      }
      __syncthreads();
      if (tid == 0) {
        if (tau != T(0)) c[k] = beta;
        v[k] = 1.0;
        v[s] = (double)tau;
        my_tau = tau;
      }
      cp_publish(st.flag, step, 1);
      return true;
    };
    if (g == 0 && !qr_owner(0)) goto timeout;
    for (int k = 0; k < n; ++k) {
      const int step = lusteps + k, owner = k % G;
      T tau;
      if (owner == g) {
        tau = my_tau;
      } else {
        if (cp_wait_flag(st.flag, step) == 0) goto timeout;
        tau = (T)slot(step)[s];
      }
      const double* v = slot(step);
      const int qa = (k + 1 < n && (k + 1) % G == g) ? (k + 1) / G : -1;
      if (qa >= 0) {
        // look-ahead: column k + 1 takes reflection k, then forms its own
        if (tau != T(0)) {
          T* c = col(qa);
          T w[1] = {T(0)};
          for (int i = k + tid; i < s; i += CP_THREADS) w[0] += (T)v[i] * c[i];
          cp_sum<1>(w, shr);
          const T tw = tau * w[0];
          for (int i = k + tid; i < s; i += CP_THREADS) c[i] -= tw * (T)v[i];
          __syncthreads();
        }
        if (!qr_owner(k + 1)) goto timeout;
      }
      if (tau != T(0)) {
        // w_j = v^T M(:, j) for the other local columns j > k (one reduction
        // for all), then M(:, j) -= tau w_j v
        T w[CP_MAXC];
        for (int q = 0; q < CP_MAXC; ++q) w[q] = T(0);
        for (int i = k + tid; i < s; i += CP_THREADS) {
          const T vi = (T)v[i];
#pragma unroll
          for (int q = 0; q < CP_MAXC; ++q)
            if (q < nloc && q != qa && g + q * G > k) w[q] += vi * col(q)[i];
        }
        cp_sum<CP_MAXC>(w, shr);
#pragma unroll
        for (int q = 0; q < CP_MAXC; ++q) {
          if (q >= nloc) break;
          if (q == qa || g + q * G <= k) continue;
          T* c = col(q);
          const T tw = tau * w[q];
          for (int i = k + tid; i < s; i += CP_THREADS) c[i] -= tw * (T)v[i];
        }
        __syncthreads();
      }
      if (tid == 0) __hip_atomic_store(st.done + g, step + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }

  // R_0 (rows < n, upper), then R_1 = D R_0 N for this workgroup's columns
#pragma unroll
  for (int q = 0; q < CP_MAXC; ++q) {
    if (q >= nloc) break;
    const int j = g + q * G;
    for (int i = tid; i < n; i += CP_THREADS) R0g[i + (int64_t)j * n] = (i <= j) ? (double)col(q)[i] : 0.0;
  }
  if (!coop_barrier(ctl, nb)) goto timeout;
  {
    // diag(R_0 N) = diag(R_0) diag(N); every workgroup finds the same first failure
    __shared__ int bad_at;
    if (tid == 0) bad_at = INT_MAX;
    __syncthreads();
    for (int i = tid; i < n; i += CP_THREADS) {
      const double d = (double)(T)(cp_load_d(&R0g[i + (int64_t)i * n]) * cp_load_d(&Ng[i + (int64_t)i * n]));
      if (!is_finite(d) || d == 0.0) atomicMin(&bad_at, i);
    }
    __syncthreads();
    if (bad_at != INT_MAX) {
      if (g == 0 && tid == 0) {
        const int i = bad_at;
        const double d = cp_load_d(&R0g[i + (int64_t)i * n]) * cp_load_d(&Ng[i + (int64_t)i * n]);
        info_set(info, is_finite(d) ? INFO_SINGULAR : INFO_NONFINITE, STAGE_PRECOND, i + 1);
      }
      return;
    }
    // columns j = g, g + G, ... < np of the padded triangle
    for (int j = g; j < np; j += G) {
      for (int i = tid; i < np; i += CP_THREADS) {
        double v;
        if (i < n && j < n) {
          T acc = T(0);
          if (i <= j)
            for (int k2 = i; k2 <= j; ++k2) acc += (T)cp_load_d(&R0g[i + (int64_t)k2 * n]) * (T)cp_load_d(&Ng[k2 + (int64_t)j * n]);
          const double dii = (double)(T)(cp_load_d(&R0g[i + (int64_t)i * n]) * cp_load_d(&Ng[i + (int64_t)i * n]));
          v = (i <= j) ? (double)acc : 0.0;
          if (dii < 0.0) v = -v;
          if (R1out) R1out[i + (int64_t)j * n] = v;
        } else {
          v = (i == j) ? 1.0 : 0.0;
        }
        R1pad[(int64_t)i * np + j] = v;
      }
      if (tid == 0) {
        double r = 1.0;
        if (j < n) {
          const double d = (double)(T)(cp_load_d(&R0g[j + (int64_t)j * n]) * cp_load_d(&Ng[j + (int64_t)j * n]));
          r = 1.0 / fabs(d);
        }
        R1pad[(int64_t)np * np + j] = r;
      }
    }
    if (lu && perm_out && g == 0) {
      // replay the pivot history: position k takes the row at position permg[k]
      for (int i = tid; i < s; i += CP_THREADS) perm_out[i] = i;
      __syncthreads();
      if (tid == 0)
        for (int k = 0; k < n; ++k) {
          const int p = permg[k];
          const int32_t t = perm_out[k];
          perm_out[k] = perm_out[p];
          perm_out[p] = t;
        }
    }
  }
  return;
timeout:
  if (threadIdx.x == 0) info_set(info, INFO_SYNC_TIMEOUT, STAGE_LU, 0);
}

// ---------------------------------------------------------------------------
// Launchers. n <= 64 (and s <= 256 for the preconditioner) go to the
// register-resident kernels of k_dense.hip.
// ---------------------------------------------------------------------------
// Workgroups of the multi-workgroup preconditioner: columns per workgroup as
// many as 60 KB of LDS holds, at most CP_MAXC.
static int coop_cpw(int64_t s, size_t elt) {
  int cpw = (int)(61440 / ((size_t)s * elt));
  return cpw > CP_MAXC ? CP_MAXC : cpw;
}

size_t precond_scratch_bytes(int64_t s, int64_t n) {
  // generic kernel: A (s*n) + wv (n) + N (n*n) + R (n*n) in doubles, + perm
  // (s ints), aligned; the multi-workgroup kernel uses 2 n^2 doubles, s ints
  // and its state (control block, step flags and counts, ring); the
  // register-resident kernel for n > 64: its two tables
  size_t b = ((size_t)s * n + n + 2 * (size_t)n * n) * sizeof(double);
  b = (b + 255) / 256 * 256;
  b += ((size_t)s * sizeof(int32_t) + 255) / 256 * 256;
  const int cpw = coop_cpw(s, sizeof(float));
  const int gmax = (int)n;  // G <= n for any cpw >= 1
  (void)cpw;
  size_t flow = ((size_t)2 * n * n * sizeof(double) + 255) / 256 * 256;
  flow += ((size_t)s * sizeof(int32_t) + 255) / 256 * 256;
  flow += coop_state_bytes(s, n, gmax);
  if (flow > b) b = flow;
  if (n > 64 && precond_reg_fits(s, n) && b < precond_reg_scratch_bytes()) b = precond_reg_scratch_bytes();
  return b;
}

template <typename T>
static hipError_t launch_pc_coop(const double* Y, int64_t s, int64_t n, int lu, const double* Nin, int64_t ldn,
                                 double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch,
                                 int32_t* info, int32_t stage_qr, hipStream_t st) {
  const int np = pad_cols(n);
  const int cpw = coop_cpw(s, sizeof(T));
  if (cpw < 1) return hipErrorInvalidValue;
  const int G = (int)((n + cpw - 1) / cpw);
  // scratch: N (n n) | R_0 (n n) doubles | perm (s ints) | control block |
  // step flags (2n ints) and finished-step counts (G ints) | ring (CP_RING (s + 1) doubles)
  double* Ng = scratch;
  double* R0g = Ng + (size_t)n * n;
  size_t off = ((size_t)2 * n * n * sizeof(double) + 255) / 256 * 256;
  int32_t* permg = (int32_t*)((char*)scratch + off);
  off += ((size_t)s * sizeof(int32_t) + 255) / 256 * 256;
  CoopState cs;
  cs.ctl = (CoopCtl*)((char*)scratch + off);
  off += coop_ctl_bytes();
  cs.flag = (int*)((char*)scratch + off);
  cs.done = cs.flag + 2 * n;
  off += ((size_t)(2 * n + G) * sizeof(int) + 255) / 256 * 256;
  cs.ring = (double*)((char*)scratch + off);
  const size_t lds = (size_t)cpw * s * sizeof(T);
  const int nwords = (int)(2 * n + G);
  hipLaunchKernelGGL(k_coop_ctl_init, dim3((nwords + 255) / 256), dim3(256), 0, st, cs.ctl, cs.flag, nwords);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int si = (int)s, ni = (int)n, ldni = (int)ldn;
  void* args[] = {(void*)&Y, &si, &ni, &lu, (void*)&Nin, &ldni, &R1pad, (void*)&np, &R1out, &perm, &Mout,
                  &Ng, &R0g, &permg, &cs, (void*)&cpw, &info, &stage_qr};
  // a cooperative launch: all G workgroups are resident together (the step
  // waits depend on every one of them)
  return hipLaunchCooperativeKernel((const void*)k_precond_coop<T>, dim3(G), dim3(CP_THREADS), args, (unsigned)lds, st);
}

hipError_t launch_precond(const double* Y, int64_t s, int64_t n, int lu, int prec, const double* Nin, int64_t ldn,
                          double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch, int32_t* info,
                          int32_t stage_qr, hipStream_t st) {
  if (s < n || n < 1 || n > 256) return hipErrorInvalidValue;
  if (precond_reg_fits(s, n))
    return launch_precond_reg(Y, s, n, lu, prec, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st);
  if (prec == 1)
    return launch_pc_coop<float>(Y, s, n, lu, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st);
  return launch_pc_coop<double>(Y, s, n, lu, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st);
}

size_t chol_scratch_bytes(int64_t n) { return ((size_t)2 * n * n * sizeof(double) + 255) / 256 * 256; }

hipError_t launch_chol(const double* G, int ldg, int64_t n, int64_t m, int shift_mode, double* Rpad, double* Rout,
                       int rout_user, const double* Rprev, const double* Npost, int64_t ldnp, double* scratch,
                       int32_t* info, int32_t stage, hipStream_t st) {
  if (n < 1 || n > 256) return hipErrorInvalidValue;
  const int np = pad_cols(n);
  if (n <= 128 && !(Npost && Rout))
    return launch_chol_reg(G, ldg, n, m, shift_mode, Rpad, Rout, rout_user, Rprev, Npost, ldnp, info, stage, st);
  if (!Npost) {
    // blocked factor on one workgroup, then the product with the earlier factor
    hipLaunchKernelGGL(k_chol_blk, dim3(1), dim3(SD_THREADS), 0, st, G, ldg, (int)n, m, shift_mode, Rpad, np, scratch,
                       info, stage);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !Rout) return e;
    hipLaunchKernelGGL(k_trmm_pad, dim3((np / 16) * (np / 16)), dim3(64), 0, st, Rpad, Rprev, np, (int)n, Rout,
                       rout_user, info);
    return hipGetLastError();
  }
  const size_t lds = (size_t)n * n * sizeof(double);
  const int use_lds = lds <= SD_LDS_LIMIT;
  double* gA = scratch;
  double* gT = scratch + (size_t)n * n;
  if (use_lds && lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
  }
  // the factor (and its optional right factor) on one workgroup; the product
  // with the earlier factor from the padded result on many
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(SD_THREADS), use_lds ? lds : 0, st, G, ldg, (int)n, m, shift_mode, Rpad, np,
                     nullptr, rout_user, nullptr, Npost, (int)ldnp, gA, gT, use_lds, info, stage);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !Rout) return e;
  const int nb = np / 16;
  hipLaunchKernelGGL(k_trmm_pad, dim3(nb * nb), dim3(64), 0, st, Rpad, Rprev, np, (int)n, Rout, rout_user, info);
  return hipGetLastError();
}

hipError_t launch_unpad(const double* Rpad, int64_t n, double* R, hipStream_t st) {
  const int np = pad_cols(n);
  const int total = (int)(n * n);
  hipLaunchKernelGGL(k_unpad, dim3((total + 255) / 256), dim3(256), 0, st, Rpad, np, (int)n, R);
  return hipGetLastError();
}

hipError_t launch_pad(const double* R, int64_t n, double* Rpad, hipStream_t st) {
  const int np = pad_cols(n);
  const int total = np * np;
  hipLaunchKernelGGL(k_pad, dim3((total + 255) / 256), dim3(256), 0, st, R, (int)n, np, Rpad);
  return hipGetLastError();
}

}  // namespace rclupp
