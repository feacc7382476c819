// Tournament pivoting for the LU of a tall X (TSLU, Grigori, Demmel and Xiang,
// SIAM J. Matrix Anal. Appl. 2011), an alternative to the partial pivoting of
// Algorithm 7 step 1 and Algorithm 5 step 1 for n <= 128:
//   leaves: X is split into L = ceil(m / 256) blocks of consecutive rows
//     (block g: rows floor(g m / L) .. floor((g+1) m / L) - 1, at least n of
//     them); each block is factored by Gaussian elimination with partial
//     pivoting (ties to the smaller position) and its first n pivot rows are
//     its candidates;
//   tree: F = floor(256 / n) consecutive candidate sets are stacked (in set
//     order) and factored the same way; their first n pivot rows are the new
//     candidates; levels repeat until one set is left;
//   root: the last factorization gives the pivot rows sel[0..n) (in pivot
//     order), L_11 (n x n unit lower) and N (n x n upper), with
//     X[sel, :] = L_11 N.
// A block whose column k holds only zeros at the step's candidate positions
// keeps its pivot at position k with no elimination (an exactly singular leaf
// does not stop the tournament); the root reports it as a zero pivot.
// M = P X N^{-1} is then one tall substitution pass over X (the rows of sel
// take L_11 exactly); the caller keeps M in X's row order, which the sketch of
// RCLUPPr sees as a column permutation of a Gaussian matrix.
// One pass over X at the leaves (256-row blocks in LDS-free registers), the
// tree over n-row candidate sets, then the substitution: the m sequential
// column steps of partial pivoting become independent leaf factorizations.
#include <limits.h>

#include "device_common.hpp"
#include "launch.hpp"

namespace rclupp {

constexpr int TS_THREADS = 1024;
constexpr int TS_LEAF = 256;  // rows of a node's block (16 A with A = 16)

__device__ __forceinline__ void ts_info_set(int32_t* info, int32_t code, int32_t stage, int32_t index) {
  // many nodes may fail at once: the first failure wins the code word
  if (info != nullptr && atomicCAS(info, 0, code) == 0) {
    info[1] = stage;
    info[2] = index;
    info[3] = 0;
  }
}

// DPP helpers for 16-lane rows (as in the small dense kernels).
template <int CTRL>
__device__ __forceinline__ int ts_dpp_b32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double ts_dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = ts_dpp_b32<CTRL>((int)b), hi = ts_dpp_b32<CTRL>((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ __forceinline__ void ts_take(double& v, int& key, double ov, int okey) {
  const double a = fabs(v), b = fabs(ov);
  const bool take = (b > a) | ((b == a) & (okey < key));
  v = take ? ov : v;
  key = take ? okey : key;
}
template <int CTRL>
__device__ __forceinline__ void ts_step(double& v, int& key) {
  const double ov = ts_dpp<CTRL>(v);
  const int ok = ts_dpp_b32<CTRL>(key);
  ts_take(v, key, ov, ok);
}

// One node: Gaussian elimination with partial pivoting of r <= 256 rows, n <= 64 CS
// columns, in registers: thread (wave w, lane l) holds columns 4w + l/16 + 64c
// and rows l%16 + 16a (a < 16). Rows never move; positions trade (LDS tables).
//   leaf level (prev == nullptr): node g factors rows floor(g m / L) .. of X;
//   upper levels: node g stacks the sets g F .. of prev (n indices each; the
//     last node may have fewer), nsets sets in all.
// Writes the original indices of its first n pivot rows to sel[g n ..]; the
// root (one node) also writes N and L_11 (n x n, ld n).
template <int CS>
__global__ __launch_bounds__(TS_THREADS) void k_tslu_node(const double* __restrict__ X, int64_t ldx, int64_t m, int n,
                                                          int64_t leaves, const int32_t* __restrict__ prev,
                                                          int64_t nsets, int F, int32_t* __restrict__ sel,
                                                          double* __restrict__ Nout, double* __restrict__ Lout,
                                                          int32_t* info) {
  constexpr int A = 16, SR = 16 * A;
  __shared__ double vb[2][SR];       // multipliers of the step, by (row % 16) * A + row / 16
  __shared__ int posl[SR], rowl[SR];  // position of each local row, row at each position
  __shared__ int64_t orig[SR];        // original row index of each local row
  __shared__ int bc_key[2];
  if (info_failed(info)) return;
  const int64_t g = blockIdx.x;
  const bool root = gridDim.x == 1;
  int r;
  if (!prev) {
    const int64_t r0 = g * m / leaves, r1 = (g + 1) * m / leaves;
    r = (int)(r1 - r0);
    for (int i = threadIdx.x; i < r; i += TS_THREADS) orig[i] = r0 + i;
  } else {
    const int64_t s0 = g * F, s1 = (s0 + F < nsets) ? s0 + F : nsets;
    r = (int)((s1 - s0) * n);
    for (int i = threadIdx.x; i < r; i += TS_THREADS) orig[i] = prev[s0 * n + i];
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tr = lane & 15, col0 = 4 * wave + (lane >> 4);
  for (int i = tid; i < SR; i += TS_THREADS) {
    posl[(i & 15) * A + (i >> 4)] = i;
    rowl[i] = i;
  }
  __syncthreads();
  double x[CS][A];
#pragma unroll
  for (int c = 0; c < CS; ++c)
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const int row = tr + 16 * a, col = col0 + 64 * c;
      x[c][a] = (row < r && col < n) ? X[orig[row] + (int64_t)col * ldx] : 0.0;
    }

#pragma unroll
  for (int kc = 0; kc < CS; ++kc) {
    for (int kk = 0; kk < 64; ++kk) {
      const int k = 64 * kc + kk;
      if (k >= n) break;
      const int buf = k & 1;
      if (wave == (kk >> 2)) {
        // pivot candidates (rows at positions >= k), scanned in register order
        double best = 0.0;
        int key = INT_MAX, bad = 0;
#pragma unroll
        for (int a = 0; a < A; ++a) {
          const int row = tr + 16 * a, pa = posl[tr * A + a];
          const bool live = (row < r) & (pa >= k);
          bad |= live & !is_finite(x[kc][a]);
          ts_take(best, key, live ? x[kc][a] : 0.0, live ? ((pa << 12) | row) : INT_MAX);
        }
        ts_step<0xB1>(best, key);
        ts_step<0x4E>(best, key);
        ts_step<0x141>(best, key);
        ts_step<0x140>(best, key);
        const bool own = (col0 == kk);
        const bool anybad = __ballot(own && bad) != 0;
        if (own) {
          const int prow = key & 4095, ppos = key >> 12;
          const bool zero = !(fabs(best) > 0.0);
          if (anybad || (zero && root)) {
            if (tr == 0) {
              ts_info_set(info, anybad ? INFO_NONFINITE : INFO_LU_ZERO_PIVOT, STAGE_LU, k + 1);
              bc_key[buf] = -1;
            }
          } else {
            // multipliers RN(x / p): Markstein's corrected quotient from one
            // reciprocal y = RN(1 / p), q0 = RN(x y), RN(q0 + (x - q0 p) y), which
            // is the correctly rounded quotient when y is normal (|x / p| <= 1);
            // subnormal pivots and pivots above 1 / (smallest normal) divide
            // directly. A zero pivot column (a singular block below the root)
            // eliminates nothing.
            const double ap = fabs(best);
            const bool direct = ap < 0x1p-1022 || ap > 0x1p1022;
            const double y = zero ? 0.0 : 1.0 / best;
#pragma unroll
            for (int a = 0; a < A; ++a) {
              const int row = tr + 16 * a;
              const bool live = (row < r) & (posl[tr * A + a] >= k) & (row != prow) & !zero;
              double qv;
              if (direct) {
                qv = zero ? 0.0 : x[kc][a] / best;
              } else {
                const double q0 = x[kc][a] * y;
                qv = __builtin_fma(__builtin_fma(-q0, best, x[kc][a]), y, q0);
              }
              const double l = live ? qv : 0.0;
              x[kc][a] = live ? l : x[kc][a];
              vb[buf][tr * A + a] = l;
            }
            if (tr == 0) {
              const int q = rowl[k];
              rowl[k] = prow;
              rowl[ppos] = q;
              posl[(prow & 15) * A + (prow >> 4)] = k;
              posl[(q & 15) * A + (q >> 4)] = ppos;
              bc_key[buf] = key;
            }
          }
        }
      }
      __syncthreads();
      const int pkey = __builtin_amdgcn_readfirstlane(bc_key[buf]);
      if (pkey < 0) return;
      const int prow = pkey & 4095;
      const int ap = prow >> 4, src = (lane & 48) | (prow & 15);
#pragma unroll
      for (int c = kc; c < CS; ++c) {
        if (4 * wave + 3 + 64 * c > k) {
          double u = x[c][0];
#pragma unroll
          for (int a = 1; a < A; ++a)
            if (a == ap) u = x[c][a];
          u = __shfl(u, src);
          if (col0 + 64 * c <= k) u = 0.0;  // columns <= k are final
#pragma unroll
          for (int a = 0; a < A; ++a) x[c][a] = __builtin_fma(-vb[buf][tr * A + a], u, x[c][a]);
        }
      }
    }
    __syncthreads();
  }

  for (int p = tid; p < n; p += TS_THREADS) sel[g * n + p] = (int32_t)orig[rowl[p]];
  if (root) {
#pragma unroll
    for (int c = 0; c < CS; ++c) {
      const int col = col0 + 64 * c;
      if (col >= n) continue;
#pragma unroll
      for (int a = 0; a < A; ++a) {
        const int p = posl[tr * A + a];
        if (tr + 16 * a < r && p < n) {
          Nout[p + (int64_t)col * n] = (col >= p) ? x[c][a] : 0.0;
          Lout[p + (int64_t)col * n] = (col < p) ? x[c][a] : (col == p ? 1.0 : 0.0);
        }
      }
    }
  }
}

// W[sel[k], :] = L_11[k, :] (the pivot rows of M take the exact unit lower factor).
__global__ void k_tslu_scatter(double* W, int64_t ldw, int n, const int32_t* __restrict__ sel,
                               const double* __restrict__ L, const int32_t* info) {
  if (info_failed(info)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int k = e % n, j = e / n;
  W[(int64_t)sel[k] + (int64_t)j * ldw] = L[k + (int64_t)j * n];
}

int64_t tslu_leaves(int64_t m) { return (m + TS_LEAF - 1) / TS_LEAF; }

size_t tslu_scratch_bytes(int64_t m, int64_t n) {
  // candidate sets of two consecutive levels, N and L_11, the padded N
  const size_t sets = (size_t)tslu_leaves(m) * n * sizeof(int32_t);
  const int np = pad_cols(n);
  return 2 * ((sets + 255) / 256 * 256) + 2 * (((size_t)n * n * 8 + 255) / 256 * 256) +
         ((padded_r_doubles(np) * 8 + 255) / 256 * 256);
}

hipError_t launch_tslu(const double* X, int64_t m, int64_t n, int64_t ldx, double* W, int64_t ldw, int32_t* sel,
                       double* Nout, double* scratch, int32_t* info, hipStream_t st) {
  if (n < 1 || n > 128 || m < n) return hipErrorInvalidValue;
  const int64_t leaves = tslu_leaves(m);
  const size_t sets = ((size_t)leaves * n * sizeof(int32_t) + 255) / 256 * 256;
  int32_t* lv[2] = {(int32_t*)scratch, (int32_t*)((char*)scratch + sets)};
  double* Lt = (double*)((char*)scratch + 2 * sets);
  double* Nt = Nout ? Nout : (double*)((char*)Lt + ((size_t)n * n * 8 + 255) / 256 * 256);
  double* Npad = (double*)((char*)Lt + 2 * (((size_t)n * n * 8 + 255) / 256 * 256));
  const int F = TS_LEAF / (int)n;
  auto node = [&](int64_t nodes, const int32_t* prev, int64_t nsets, int32_t* out) {
    if (n <= 64)
      hipLaunchKernelGGL(k_tslu_node<1>, dim3((unsigned)nodes), dim3(TS_THREADS), 0, st, X, ldx, m, (int)n, leaves,
                         prev, nsets, F, out, Nt, Lt, info);
    else
      hipLaunchKernelGGL(k_tslu_node<2>, dim3((unsigned)nodes), dim3(TS_THREADS), 0, st, X, ldx, m, (int)n, leaves,
                         prev, nsets, F, out, Nt, Lt, info);
    return hipGetLastError();
  };
  // leaves, then levels of F-way merges until one set is left (the root
  // writes N and L_11; the final candidates go to `sel`)
  int cur = 0;
  hipError_t e = node(leaves, nullptr, 0, leaves == 1 ? sel : lv[cur]);
  if (e != hipSuccess) return e;
  int64_t nsets = leaves;
  while (nsets > 1) {
    const int64_t nodes = (nsets + F - 1) / F;
    e = node(nodes, lv[cur], nsets, nodes == 1 ? sel : lv[cur ^ 1]);
    if (e != hipSuccess) return e;
    cur ^= 1;
    nsets = nodes;
  }
  // W = X N^{-1} (row-wise substitution on the tall kernels), then the pivot rows
  e = launch_pad(Nt, n, Npad, st);
  if (e != hipSuccess) return e;
  const TallPlan tp = plan_tall(m, n, 0);
  e = launch_tall_pass(tp, X, ldx, m, n, Npad, W, ldw, nullptr, info, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tslu_scatter, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, W, ldw, (int)n, sel, Lt,
                     info);
  return hipGetLastError();
}

}  // namespace rclupp
