// Small dense stages on the s x n sketch and the n x n Grams, one workgroup
// each (they are O(s n^2) and O(n^3) and latency bound):
//   k_precond : [M, N, P] = LU(Y) with partial pivoting (eq. elu), R_0 = R
//               factor of M by Householder reflections (eq. eh, Q_s never
//               formed), R_1 = D R_0 N with D = sign(diag(R_0 N)) (eq. ey)
//               (Algorithm 2 steps 2-4; Algorithm 7 steps 3-4 with an external
//               N; Algorithm 6 step 2 without the LU);
//   k_chol    : upper Cholesky of G (+ the shift of Algorithm 4), optional
//               right factor (LC2's R_1 = D S_c N) and product with an earlier
//               factor (R_3 = R_2 R_1, R = R_4 R_3; eqs. C4, C8).
// The working copy lives in LDS when it fits, else in a global scratch buffer
// (same code through generic pointers). Threads form a 64 x 16 grid: tx walks
// rows (contiguous in the column-major layout), ty walks columns; the column
// loops keep SD_U loads in flight per thread (the working copy is in L2 when
// it does not fit LDS, and one outstanding load per thread left them latency
// bound).
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
__device__ T block_sum(T v, T* sh /* [SD_WAVES] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  T r = sh[0];
  for (int w = 1; w < SD_THREADS / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
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
template <typename T>
__global__ __launch_bounds__(SD_THREADS) void k_precond(const double* __restrict__ Y, int s, int n, int lu,
                                                        const double* __restrict__ Nin, int ldn, double* R1pad, int np,
                                                        double* R1out, int32_t* perm_out, double* Mout, T* gA, T* gN,
                                                        T* gR, int32_t* gperm, int use_lds, int32_t* info,
                                                        int32_t stage_qr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ ArgMaxSh amx;
  __shared__ T red[SD_WAVES];
  __shared__ T sc_tau, sc_scal;
  __shared__ int fail;
  if (info_failed(info)) return;
  T* A = use_lds ? (T*)smem_raw : gA;
  T* wv = use_lds ? A + (size_t)s * n : gA + (size_t)s * n;  // n entries
  int32_t* perm = gperm;
  T* N = gN;
  T* R = gR;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;

  for (int e = tid; e < s * n; e += SD_THREADS) A[e] = (T)Y[e];
  if (tid == 0) fail = 0;
  for (int i = tid; i < s; i += SD_THREADS) perm[i] = i;
  __syncthreads();

  // Without the LU, non-finite entries are reported before the Householder
  // steps (lowest column); with the LU each pivot column is checked as it is
  // reached (rows k..s-1 after the earlier updates), as partial pivoting does.
  if (!lu) {
    double v = -1.0;
    int idx = INT_MAX, bad = 0;
    for (int e = tid; e < s * n; e += SD_THREADS)
      if (!is_finite((double)A[e]) && e / s < idx) {
        idx = e / s;
        bad = 1;
      }
    // lowest failing column: reuse the argmax reduction with v = -column
    v = bad ? -(double)idx : -1e300;
    block_argmax(v, idx, bad, &amx);
    if (bad) {
      if (tid == 0) info_set(info, INFO_NONFINITE, stage_qr, (int32_t)(-v) + 1);
      return;
    }
  }

  if (lu) {
    for (int k = 0; k < n; ++k) {
      double best = -1.0;
      int idx = INT_MAX, bad = 0;
      for (int i = k + tid; i < s; i += SD_THREADS) {
        const double a = (double)tabs(A[i + k * s]);
        if (!is_finite(a)) bad = 1;
        if (a > best) {
          best = a;
          idx = i;
        }
      }
      block_argmax(best, idx, bad, &amx);
      if (bad) {
        if (tid == 0) info_set(info, INFO_NONFINITE, STAGE_LU, k + 1);
        return;
      }
      if (best == 0.0) {
        if (tid == 0) info_set(info, INFO_LU_ZERO_PIVOT, STAGE_LU, k + 1);
        return;
      }
      const int p = idx;
      if (p != k) {
        for (int j = tid; j < n; j += SD_THREADS) {
          const T t = A[k + j * s];
          A[k + j * s] = A[p + j * s];
          A[p + j * s] = t;
        }
        if (tid == 0) {
          const int32_t t = perm[k];
          perm[k] = perm[p];
          perm[p] = t;
        }
      }
      __syncthreads();
      const T piv = A[k + k * s];
      for (int i = k + 1 + tid; i < s; i += SD_THREADS) A[i + k * s] = A[i + k * s] / piv;
      __syncthreads();
      for (int j = k + 1 + ty; j < n; j += SD_WAVES) {
        const T akj = A[k + j * s];
        T* cj = A + (size_t)j * s;
        const T* ck = A + (size_t)k * s;
        int i = k + 1 + tx;
        for (; i + 64 * (SD_U - 1) < s; i += 64 * SD_U) {
          T a[SD_U], l[SD_U];
#pragma unroll
          for (int u = 0; u < SD_U; ++u) {
            a[u] = cj[i + 64 * u];
            l[u] = ck[i + 64 * u];
          }
#pragma unroll
          for (int u = 0; u < SD_U; ++u) cj[i + 64 * u] = a[u] - l[u] * akj;
        }
        for (; i < s; i += 64) cj[i] = cj[i] - ck[i] * akj;
      }
      __syncthreads();
    }
    // N = upper n x n; then A := unit lower trapezoidal M
    for (int e = tid; e < n * n; e += SD_THREADS) {
      const int i = e % n, j = e / n;
      N[e] = (i <= j) ? A[i + j * s] : T(0);
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += SD_THREADS) {
      const int i = e % n, j = e / n;
      if (i <= j) A[i + j * s] = (i == j) ? T(1) : T(0);
    }
    __syncthreads();
    if (Mout)
      for (int e = tid; e < s * n; e += SD_THREADS) Mout[e] = (double)A[e];
    if (perm_out)
      for (int i = tid; i < s; i += SD_THREADS) perm_out[i] = perm[i];
  } else {
    for (int e = tid; e < n * n; e += SD_THREADS) {
      const int i = e % n, j = e / n;
      N[e] = Nin ? ((i <= j) ? (T)Nin[i + j * ldn] : T(0)) : (i == j ? T(1) : T(0));
    }
  }
  __syncthreads();

  // Householder R factor of A (s x n), LAPACK dlarfg convention
  for (int k = 0; k < n; ++k) {
    T part = T(0);
    for (int i = k + 1 + tid; i < s; i += SD_THREADS) part += A[i + k * s] * A[i + k * s];
    const T ss = block_sum(part, red);
    if (tid == 0) {
      const T alpha = A[k + k * s];
      const T xnorm = sqrt(ss);
      T tau = T(0), scal = T(0);
      if (xnorm != T(0)) {
        const T beta = -copysign(hypot(alpha, xnorm), alpha);
        tau = (beta - alpha) / beta;
        scal = T(1) / (alpha - beta);
        A[k + k * s] = beta;
      }
      sc_tau = tau;
      sc_scal = scal;
    }
    __syncthreads();
    const T tau = sc_tau, scal = sc_scal;
    if (tau == T(0)) continue;
    for (int i = k + 1 + tid; i < s; i += SD_THREADS) A[i + k * s] *= scal;
    __syncthreads();
    // wv[j] = A[k][j] + sum_{i>k} v_i A[i][j]; one wave per column (strided)
    for (int j = k + 1 + ty; j < n; j += SD_WAVES) {
      const T* cj = A + (size_t)j * s;
      const T* ck = A + (size_t)k * s;
      T part[SD_U];
#pragma unroll
      for (int u = 0; u < SD_U; ++u) part[u] = T(0);
      int i = k + 1 + tx;
      for (; i + 64 * (SD_U - 1) < s; i += 64 * SD_U)
#pragma unroll
        for (int u = 0; u < SD_U; ++u) part[u] += ck[i + 64 * u] * cj[i + 64 * u];
      for (; i < s; i += 64) part[0] += ck[i] * cj[i];
      T acc = part[0];
#pragma unroll
      for (int u = 1; u < SD_U; ++u) acc += part[u];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (tx == 0) wv[j] = A[k + j * s] + acc;
    }
    __syncthreads();
    for (int j = k + 1 + ty; j < n; j += SD_WAVES) {
      const T tw = tau * wv[j];
      T* cj = A + (size_t)j * s;
      const T* ck = A + (size_t)k * s;
      int i = k + tx;
      for (; i + 64 * (SD_U - 1) < s; i += 64 * SD_U) {
        T a[SD_U], v[SD_U];
#pragma unroll
        for (int u = 0; u < SD_U; ++u) {
          a[u] = cj[i + 64 * u];
          v[u] = (i + 64 * u == k) ? T(1) : ck[i + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < SD_U; ++u) cj[i + 64 * u] = a[u] - tw * v[u];
      }
      for (; i < s; i += 64) {
        const T v = (i == k) ? T(1) : ck[i];
        cj[i] -= tw * v;
      }
    }
    __syncthreads();
  }

  // R_1 = R_0 N (upper x upper), then the sign fix D
  for (int e = tid; e < n * n; e += SD_THREADS) {
    const int i = e % n, j = e / n;
    T part[SD_U];
#pragma unroll
    for (int u = 0; u < SD_U; ++u) part[u] = T(0);
    if (i <= j) {
      int k = i;
      for (; k + SD_U - 1 <= j; k += SD_U)
#pragma unroll
        for (int u = 0; u < SD_U; ++u) part[u] += A[i + (size_t)(k + u) * s] * N[k + u + j * n];
      for (; k <= j; ++k) part[0] += A[i + (size_t)k * s] * N[k + j * n];
    }
    T acc = part[0];
#pragma unroll
    for (int u = 1; u < SD_U; ++u) acc += part[u];
    R[e] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < n; ++i) {
      const T d = R[i + i * n];
      if (!is_finite((double)d)) {
        info_set(info, INFO_NONFINITE, STAGE_PRECOND, i + 1);
        fail = 1;
        break;
      }
      if (d == T(0)) {
        info_set(info, INFO_SINGULAR, STAGE_PRECOND, i + 1);
        fail = 1;
        break;
      }
    }
  }
  __syncthreads();
  if (fail) return;
  // widen to double with the signs folded in
  for (int e = tid; e < np * np; e += SD_THREADS) {
    const int i = e / np, j = e % np;
    double v;
    if (i < n && j < n) {
      const double d = (double)R[i + i * n];
      v = (i <= j) ? (double)R[i + j * n] : 0.0;
      if (d < 0.0) v = -v;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    R1pad[e] = v;
    if (R1out && i < n && j < n) R1out[i + j * n] = v;
  }
  __syncthreads();
  for (int j = tid; j < np; j += SD_THREADS) {
    double v = 1.0;
    if (j < n) {
      const double d = (double)R[j + j * n];
      v = 1.0 / (d < 0.0 ? -d : d);
    }
    R1pad[np * np + j] = v;
  }
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
// Launchers. n <= 64 (and s <= 256 for the preconditioner) go to the
// register-resident kernels of k_dense.hip.
// ---------------------------------------------------------------------------
size_t precond_scratch_bytes(int64_t s, int64_t n) {
  // generic kernel: A (s*n) + wv (n) + N (n*n) + R (n*n) in doubles, + perm
  // (s ints), aligned; the register-resident kernel for n > 64: its two tables
  size_t b = ((size_t)s * n + n + 2 * (size_t)n * n) * sizeof(double);
  b = (b + 255) / 256 * 256;
  b += ((size_t)s * sizeof(int32_t) + 255) / 256 * 256;
  if (n > 64 && precond_reg_fits(s, n) && b < precond_reg_scratch_bytes()) b = precond_reg_scratch_bytes();
  return b;
}

template <typename T>
static hipError_t launch_pc(const double* Y, int64_t s, int64_t n, int lu, const double* Nin, int64_t ldn,
                            double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch, int32_t* info,
                            int32_t stage_qr, hipStream_t st) {
  const int np = pad_cols(n);
  T* gA = (T*)scratch;
  T* gN = gA + (size_t)s * n + n;
  T* gR = gN + (size_t)n * n;
  size_t off = ((size_t)s * n + n + 2 * (size_t)n * n) * sizeof(double);
  off = (off + 255) / 256 * 256;
  int32_t* gperm = (int32_t*)((char*)scratch + off);
  const size_t lds = ((size_t)s * n + n) * sizeof(T);
  const int use_lds = lds <= SD_LDS_LIMIT;
  if (use_lds && lds > 64 * 1024) {
    hipError_t e =
        hipFuncSetAttribute((const void*)k_precond<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
  }
  hipLaunchKernelGGL((k_precond<T>), dim3(1), dim3(SD_THREADS), use_lds ? lds : 0, st, Y, (int)s, (int)n, lu, Nin,
                     (int)ldn, R1pad, np, R1out, perm, Mout, gA, gN, gR, gperm, use_lds, info, stage_qr);
  return hipGetLastError();
}

hipError_t launch_precond(const double* Y, int64_t s, int64_t n, int lu, int prec, const double* Nin, int64_t ldn,
                          double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch, int32_t* info,
                          int32_t stage_qr, hipStream_t st) {
  if (s < n || n < 1 || n > 256) return hipErrorInvalidValue;
  if (precond_reg_fits(s, n))
    return launch_precond_reg(Y, s, n, lu, prec, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st);
  if (prec == 1) return launch_pc<float>(Y, s, n, lu, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st);
  return launch_pc<double>(Y, s, n, lu, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st);
}

size_t chol_scratch_bytes(int64_t n) { return ((size_t)2 * n * n * sizeof(double) + 255) / 256 * 256; }

hipError_t launch_chol(const double* G, int ldg, int64_t n, int64_t m, int shift_mode, double* Rpad, double* Rout,
                       int rout_user, const double* Rprev, const double* Npost, int64_t ldnp, double* scratch,
                       int32_t* info, int32_t stage, hipStream_t st) {
  if (n < 1 || n > 256) return hipErrorInvalidValue;
  const int np = pad_cols(n);
  if (n <= 128 && !(Npost && Rout))
    return launch_chol_reg(G, ldg, n, m, shift_mode, Rpad, Rout, rout_user, Rprev, Npost, ldnp, info, stage, st);
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
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(SD_THREADS), use_lds ? lds : 0, st, G, ldg, (int)n, m, shift_mode, Rpad, np,
                     Rout, rout_user, Rprev, Npost, (int)ldnp, gA, gT, use_lds, info, stage);
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
