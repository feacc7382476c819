// Register-resident small dense stages for n <= 128, one workgroup of 1024
// threads each (these steps are O(s n^2) and O(n^3): their time is the length
// of the chain of dependent column steps, so the layout is chosen to make each
// step short):
//   k_precond_reg : [M, N, P] = LU(Y) with partial pivoting (eq. elu), the R
//                   factor R_0 of M by Householder reflections (eq. eh, Q_s
//                   never formed), R_1 = D R_0 N with D = sign(diag(R_0 N))
//                   (eq. ey). Algorithm 2 steps 2-4; Algorithm 7 steps 3-4
//                   with an external N; Algorithm 6 step 2 without the LU.
//   k_chol_reg    : upper Cholesky of G (+ the shift of Algorithm 4), then an
//                   optional product with an earlier factor (R_3 = R_2 R_1,
//                   R = R_4 R_3; eqs. C4, C8) or an optional right factor with
//                   the sign fix (LC2's R_1 = D S_c N, Algorithm 5).
//
// Layout: thread (wave w, lane l) owns the columns j = 4w + l/16 + 64c
// (c < CS, CS = 1 for n <= 64 and 2 for n <= 128) and the rows i = l%16 + 16a,
// a < A. The 16 lanes of a DPP row therefore hold whole columns: a column
// reduction is four DPP exchanges inside one wave. A column
// step is: the wave owning column k reduces it (pivot search, or the
// reflector's norm), publishes a vector of s values to LDS, one barrier, then
// every thread applies a rank-1 update to the A values it holds. Rows are
// never moved: the LU keeps a position for every row (pivoting swaps
// positions only), so the pivot search scans the rows at positions >= k and
// ties go to the smaller position, as in LAPACK's getrf.
//
// The n x n products (R_0 N, R R_prev, R N) run on FP64 MFMA 16x16x4 from LDS
// tables, one 16 x 16 output block per wave.
#include <limits.h>

#include "device_common.hpp"
#include "launch.hpp"

namespace rclupp {

constexpr int DN_THREADS = 1024;
constexpr int DN_NP = 128;         // largest n handled here

// ---- DPP exchanges within 16-lane rows ----------------------------------------
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <- lane 7-i within each 8
constexpr int DPP_MIRROR = 0x140;       // lane i <- lane 15-i within each 16

template <int CTRL>
__device__ __forceinline__ int dpp_b32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return dpp_b32<CTRL>(v);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(dpp_b32<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_b32<CTRL>((int)b), hi = dpp_b32<CTRL>((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Sum over the 16 lanes of a DPP row. Each exchange pairs lanes that then add
// the same two operands, so every lane ends with the same bits.
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
  v = v + dpp<DPP_XOR1>(v);
  v = v + dpp<DPP_XOR2>(v);
  v = v + dpp<DPP_HALF_MIRROR>(v);
  v = v + dpp<DPP_MIRROR>(v);
  return v;
}

template <typename T>
__device__ __forceinline__ T dn_abs(T v) {
  return v < T(0) ? -v : v;
}

// Pivot candidate order: larger |v| first, then the smaller key (position).
// A strict total order on live candidates (keys are unique), so any reduction
// tree gives the same winner; selects rather than branches (a branch per
// candidate costs an exec-mask save and restore on the search's critical path).
template <typename T>
__device__ __forceinline__ void piv_take(T& v, int& key, T ov, int okey) {
  const T a = dn_abs(v), b = dn_abs(ov);
  const bool take = (b > a) | ((b == a) & (okey < key));
  v = take ? ov : v;
  key = take ? okey : key;
}

template <int CTRL, typename T>
__device__ __forceinline__ void piv_step(T& v, int& key) {
  const T ov = dpp<CTRL>(v);
  const int ok = dpp<CTRL>(key);
  piv_take(v, key, ov, ok);
}

template <typename T>
__device__ __forceinline__ void row16_argmax(T& v, int& key) {
  piv_step<DPP_XOR1>(v, key);
  piv_step<DPP_XOR2>(v, key);
  piv_step<DPP_HALF_MIRROR>(v, key);
  piv_step<DPP_MIRROR>(v, key);
}

__device__ __forceinline__ double dn_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ double dn_min_normal(double) { return 0x1p-1022; }
__device__ __forceinline__ float dn_min_normal(float) { return 0x1p-126f; }
__device__ __forceinline__ float dn_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------------------------
// Preconditioner. A = rows per thread / 16 (s <= 16 A), CS column sets
// (n <= 64 CS). The n x n tables R_0 and N live in LDS for CS = 1 and in the
// global scratch for CS = 2 (row stride 64 CS + 1 either way).
// ---------------------------------------------------------------------------
template <int CS>
constexpr int dn_ld() {
  return 64 * CS + 1;
}
template <typename T, int A, int CS>
constexpr size_t precond_reg_lds() {
  return (CS == 1 ? 2 * 64 * dn_ld<1>() * sizeof(double) : 0) + 2 * 16 * A * sizeof(T) +
         (A > 8 ? 2 * 16 * A * sizeof(int) : 0);
}
size_t precond_reg_scratch_bytes() { return 2 * (size_t)128 * dn_ld<2>() * sizeof(double); }

template <typename T, int A, int CS>
__global__ __launch_bounds__(DN_THREADS) void k_precond_reg(const double* __restrict__ Y, int s, int n, int lu,
                                                            const double* __restrict__ Nin, int ldn, double* R1pad,
                                                            int np, double* R1out, int32_t* perm_out, double* Mout,
                                                            double* gtab, int32_t* info, int32_t stage_qr,
                                                            const PrecondJob* __restrict__ jobs) {
  if (jobs) {  // batched: one workgroup per problem
    const PrecondJob j = jobs[blockIdx.x];
    Y = j.Y, R1pad = j.R1pad, gtab = j.scratch, info = j.info;
  }
  constexpr int SR = 16 * A, LD = dn_ld<CS>(), NT = 64 * CS;
  extern __shared__ __align__(16) unsigned char dn_smem[];
  double* R0l = (CS == 1) ? (double*)dn_smem : gtab;  // R_0(i, j) at i*LD + j
  double* Nl = R0l + NT * LD;                           // N(i, j) at i*LD + j
  T* vb = (T*)(dn_smem + (CS == 1 ? 2 * NT * LD * sizeof(double) : 0));  // [2][SR] step vectors
  // Row positions (lazy pivoting: rows never move, positions trade). Up to 128
  // rows every thread keeps the positions of its rows tr + 16 a in registers
  // (two 16-bit positions per register) and applies each trade itself; the
  // 256-row tiles are at the register limit and keep them in LDS instead
  // (position of row r at (r%16)*A + r/16, and the row at each position),
  // updated by the pivot's owner.
  constexpr bool PREG = A <= 8;
  int* posl = (int*)(vb + 2 * SR);
  int* rowl = posl + SR;
  __shared__ int bc_row[2];
  __shared__ T bc_tau[2];
  __shared__ int bc_min;
  __shared__ double dsg[NT];
  if (info_failed(info)) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tr = lane & 15, col0 = 4 * wave + (lane >> 4);
  T x[CS][A];
#pragma unroll
  for (int c = 0; c < CS; ++c)
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const int row = tr + 16 * a, col = col0 + 64 * c;
      x[c][a] = (row < s && col < n) ? (T)Y[row + (int64_t)col * s] : T(0);
    }
  for (int e = tid; e < 2 * NT * LD; e += DN_THREADS) R0l[e] = 0.0;  // R0l and Nl
  uint32_t posw[PREG ? (A + 1) / 2 : 1];
#pragma unroll
  for (int h = 0; h < (PREG ? (A + 1) / 2 : 1); ++h)
    posw[h] = (uint32_t)(tr + 32 * h) | ((uint32_t)(tr + 32 * h + 16) << 16);
  if (!PREG)
    for (int r = tid; r < SR; r += DN_THREADS) {
      posl[(r & 15) * A + (r >> 4)] = r;
      rowl[r] = r;
    }
  auto pos = [&](int a) -> int {
    if constexpr (PREG)
      return (int)((posw[a >> 1] >> (16 * (a & 1))) & 0xFFFFu);
    else
      return posl[tr * A + a];
  };
  if (tid == 0) {
    bc_min = INT_MAX;
  }
  __syncthreads();

  if (lu) {
#pragma unroll
    for (int kc = 0; kc < CS; ++kc) {
      for (int kk = 0; kk < 64; ++kk) {
        const int k = 64 * kc + kk;
        if (k >= n) break;
        const int buf = k & 1;
        if (wave == (kk >> 2)) {
          // pivot search over the rows at positions >= k of column k
          int pp[A];
#pragma unroll
          for (int a = 0; a < A; ++a) pp[a] = pos(a);
          // candidates (rows not yet pivoted), reduced as a tree
          T cv[A];
          int ck[A], bad = 0;
#pragma unroll
          for (int a = 0; a < A; ++a) {
            const int row = tr + 16 * a;
            const bool live = (row < s) & (pp[a] >= k);
            bad |= live & !is_finite((double)x[kc][a]);
            cv[a] = live ? x[kc][a] : T(0);
            ck[a] = live ? ((pp[a] << 12) | row) : INT_MAX;
          }
#pragma unroll
          for (int w = 1; w < A; w *= 2)
#pragma unroll
            for (int a = 0; a + w < A; a += 2 * w) piv_take(cv[a], ck[a], cv[a + w], ck[a + w]);
          T best = cv[0];
          int key = ck[0];
          row16_argmax(best, key);
          const bool own = (col0 == kk);
          const bool anybad = __ballot(own && bad) != 0;
          if (own) {
            const int prow = key & 4095, ppos = key >> 12;
            const int code = anybad ? INFO_NONFINITE : (dn_abs(best) > T(0) ? 0 : INFO_LU_ZERO_PIVOT);
            if (code) {
              if (tr == 0) {
                info_set(info, code, STAGE_LU, k + 1);
                bc_row[buf] = -1;  // (keys are non-negative)
              }
            } else {
              // multipliers l_i = x_ik / pivot, correctly rounded, for the rows still
              // to eliminate: one division y = RN(1 / pivot), then per entry
              // q0 = RN(x y) and RN(q0 + (x - q0 pivot) y), which is RN(x / pivot)
              // by Markstein's theorem (|x / pivot| <= 1: no overflow; only a
              // subnormal quotient may differ). The per-entry form is three
              // independent FP64 operations; a division sequence is a dozen
              // dependent ones through VCC, so A divisions could not overlap.
              // Every quotient is formed and then selected (no branches).
              // Markstein's theorem needs y = RN(1 / p) normal: a subnormal pivot
              // (|p| below the smallest normal) would overflow 1 / p, and a pivot
              // above 1 / (smallest normal) has a subnormal reciprocal that has
              // lost bits. Such steps divide directly.
              const T ap = dn_abs(best);
              const bool direct = ap < dn_min_normal(best) || ap > T(1) / dn_min_normal(best);
              const T y = T(1) / best;
#pragma unroll
              for (int a = 0; a < A; ++a) {
                const int row = tr + 16 * a;
                const bool live = (row < s) & (pp[a] >= k) & (row != prow);
                T qv;
                if (direct) {
                  qv = x[kc][a] / best;
                } else {
                  const T q0 = x[kc][a] * y;
                  qv = dn_fma(dn_fma(-q0, best, x[kc][a]), y, q0);
                }
                const T l = live ? qv : T(0);
                x[kc][a] = live ? l : x[kc][a];
                vb[buf * SR + tr * A + a] = l;
              }
              if (tr == 0) {
                if (!PREG) {  // positions k and ppos trade rows
                  const int q = rowl[k];
                  rowl[k] = prow;
                  rowl[ppos] = q;
                  posl[(prow & 15) * A + (prow >> 4)] = k;
                  posl[(q & 15) * A + (q >> 4)] = ppos;
                }
                bc_row[buf] = key;  // pivot row and its position
              }
            }
          }
        }
        __syncthreads();
        const int pkey = __builtin_amdgcn_readfirstlane(bc_row[buf]);
        if (pkey < 0) return;
        const int prow = pkey & 4095, ppos = pkey >> 12;
        if constexpr (PREG) {  // positions k and ppos trade rows
#pragma unroll
          for (int a = 0; a < A; ++a) {
            const int pa = pos(a);
            const int np_ = (tr + 16 * a == prow) ? k : (pa == k ? ppos : pa);
            const int sh = 16 * (a & 1);
            posw[a >> 1] = (posw[a >> 1] & ~(0xFFFFu << sh)) | ((uint32_t)np_ << sh);
          }
        }
        const int ap = prow >> 4, src = (lane & 48) | (prow & 15);
#pragma unroll
        for (int c = kc; c < CS; ++c) {
          if (4 * wave + 3 + 64 * c > k) {
            // rank-1 update of the columns j > k with the pivot row's entries
            T u = x[c][0];
#pragma unroll
            for (int a = 1; a < A; ++a)
              if (a == ap) u = x[c][a];
            u = __shfl(u, src);
            // columns <= k are final: a zero factor leaves them unchanged
            if (col0 + 64 * c <= k) u = T(0);
#pragma unroll
            for (int a = 0; a < A; ++a) x[c][a] = dn_fma(-vb[buf * SR + tr * A + a], u, x[c][a]);
          }
        }
      }
    }
    __syncthreads();
  }

  {
  int pp[A];
#pragma unroll
  for (int a = 0; a < A; ++a) pp[a] = pos(a);
  if (lu) {
    // N = the rows at positions < n (upper part); M = unit lower trapezoid
#pragma unroll
    for (int c = 0; c < CS; ++c) {
      const int col = col0 + 64 * c;
#pragma unroll
      for (int a = 0; a < A; ++a) {
        if (pp[a] < n) {
          if (col < n && col >= pp[a]) Nl[pp[a] * LD + col] = (double)x[c][a];
          x[c][a] = (col < pp[a]) ? x[c][a] : (col == pp[a] ? T(1) : T(0));
        }
      }
    }
    if (perm_out) {
      if (PREG) {
        if (tid < 16)
#pragma unroll
          for (int a = 0; a < A; ++a)
            if (tr + 16 * a < s) perm_out[pp[a]] = tr + 16 * a;
      } else {
        for (int p = tid; p < s; p += DN_THREADS) perm_out[p] = rowl[p];
      }
    }
  } else {
    // M = Y; N external (upper part) or the identity. Non-finite entries of M
    // are reported before the reflections (lowest column).
#pragma unroll
    for (int c = 0; c < CS; ++c)
#pragma unroll
      for (int a = 0; a < A; ++a)
        if (tr + 16 * a < s && col0 + 64 * c < n && !is_finite((double)x[c][a])) atomicMin(&bc_min, col0 + 64 * c);
    for (int e = tid; e < n * n; e += DN_THREADS) {
      const int i = e % n, j = e / n;
      Nl[i * LD + j] = Nin ? ((i <= j) ? Nin[i + (int64_t)j * ldn] : 0.0) : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    if (bc_min != INT_MAX) {
      if (tid == 0) info_set(info, INFO_NONFINITE, stage_qr, bc_min + 1);
      return;
    }
  }
  if (Mout) {
#pragma unroll
    for (int c = 0; c < CS; ++c)
#pragma unroll
      for (int a = 0; a < A; ++a)
        if (tr + 16 * a < s && col0 + 64 * c < n) Mout[pp[a] + (int64_t)(col0 + 64 * c) * s] = (double)x[c][a];
  }
  }

  // Householder reflections (LAPACK dlarfg convention) on the rows in position order
#pragma unroll
  for (int kc = 0; kc < CS; ++kc) {
    for (int kk = 0; kk < 64; ++kk) {
      const int k = 64 * kc + kk;
      if (k >= n) break;
      const int buf = k & 1;
      if (wave == (kk >> 2)) {
        int pp[A];
#pragma unroll
        for (int a = 0; a < A; ++a) pp[a] = pos(a);
        T sq = T(0), al = T(0);
#pragma unroll
        for (int a = 0; a < A; ++a) {
          if (pp[a] > k && tr + 16 * a < s) sq = dn_fma(x[kc][a], x[kc][a], sq);
          if (pp[a] == k) al = x[kc][a];
        }
        sq = row16_sum(sq);
        al = row16_sum(al);  // one non-zero term: exact
        if (col0 == kk) {
          // dlarfg: beta = -sign(alpha) ||(alpha, x)||, the norm from the sum of
          // squares already formed (one square root on the critical path)
          T tau = T(0), scal = T(0), beta = al;
          if (sq != T(0)) {
            beta = -copysign(sqrt(dn_fma(al, al, sq)), al);
            tau = (beta - al) / beta;
            scal = T(1) / (al - beta);
          }
          // (selects, not branches: the A entries are independent)
          const bool upd = tau != T(0);
#pragma unroll
          for (int a = 0; a < A; ++a) {
            const bool below = pp[a] > k, diag = pp[a] == k;
            const T v = (below & (tr + 16 * a < s)) ? x[kc][a] * scal : (diag ? T(1) : T(0));
            x[kc][a] = (upd & below) ? v : ((upd & diag) ? beta : x[kc][a]);
            vb[buf * SR + tr * A + a] = v;
          }
          if (tr == 0) bc_tau[buf] = tau;
        }
      }
      __syncthreads();
      const T tau = bc_tau[buf];
      if (tau != T(0)) {
        const T* vv = vb + buf * SR + tr * A;  // re-read from LDS: keeps registers for x
#pragma unroll
        for (int c = kc; c < CS; ++c) {
          if (4 * wave + 3 + 64 * c > k) {
            // w_j = v^T M(:, j); M(:, j) -= tau w_j v for the columns j > k
            T p = T(0);
#pragma unroll
            for (int a = 0; a < A; ++a) p = dn_fma(vv[a], x[c][a], p);
            p = row16_sum(p);
            const T t = (col0 + 64 * c > k) ? tau * p : T(0);
#pragma unroll
            for (int a = 0; a < A; ++a) x[c][a] = dn_fma(-t, vv[a], x[c][a]);
          }
        }
      }
    }
  }

  // R_0: the rows at positions < n, columns >= position
  int pp2[A];
#pragma unroll
  for (int a = 0; a < A; ++a) pp2[a] = pos(a);
#pragma unroll
  for (int c = 0; c < CS; ++c) {
    const int col = col0 + 64 * c;
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const int pa = pp2[a];
      if (pa < n && col < n && col >= pa) R0l[pa * LD + col] = (double)x[c][a];
    }
  }
  __syncthreads();
  // diag(R_0 N) = diag(R_0) diag(N) (both triangular); D and the first failing index
  if (tid < n) {
    const double d = R0l[tid * LD + tid] * Nl[tid * LD + tid];
    dsg[tid] = d;
    if (!is_finite(d) || d == 0.0) atomicMin(&bc_min, tid);
  }
  __syncthreads();
  if (bc_min != INT_MAX) {
    if (tid == 0) info_set(info, is_finite(dsg[bc_min]) ? INFO_SINGULAR : INFO_NONFINITE, STAGE_PRECOND, bc_min + 1);
    return;
  }
  // R_1 = D R_0 N on MFMA: 16 x 16 output blocks, round robin over the waves
  const int nb = np / 16, lr = lane & 15, lq = lane >> 4;
  for (int blk = wave; blk < nb * nb; blk += DN_THREADS / 64) {
    const int I = blk / nb, J = blk % nb;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int K = I; K <= J; ++K)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double av = R0l[(16 * I + lr) * LD + 16 * K + 4 * kk + lq];
        const double bv = Nl[(16 * K + 4 * kk + lq) * LD + 16 * J + lr];
        acc = mfma_f64(av, bv, acc);
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + lq + 4 * r, j = 16 * J + lr;
      double v;
      if (i < n && j < n)
        v = (i > j) ? 0.0 : (dsg[i] < 0.0 ? -acc[r] : acc[r]);
      else
        v = (i == j) ? 1.0 : 0.0;
      R1pad[i * np + j] = v;
      if (R1out && i < n && j < n) R1out[i + (int64_t)j * n] = v;
    }
  }
  if (tid < np) R1pad[np * np + tid] = (tid < n) ? 1.0 / fabs(dsg[tid]) : 1.0;
}

// ---------------------------------------------------------------------------
// Cholesky, right-looking on the full symmetric matrix: thread (columns
// 4w + l/16 + 64c, rows l%16 + 16a, a < 4 CS). Step k: the owner of column k
// forms row k of R (its column, by symmetry) into LDS; every column j > k
// subtracts R(k, :)^T R(k, j). Dynamic LDS: the R table, 64 CS rows of stride
// 64 CS + 1.
// ---------------------------------------------------------------------------
template <int CS>
constexpr size_t chol_reg_lds() {
  return (size_t)64 * CS * dn_ld<CS>() * sizeof(double);
}

template <int CS>
__global__ __launch_bounds__(DN_THREADS) void k_chol_reg(const double* __restrict__ G, int ldg, int n, int64_t m,
                                                         int shift_mode, double* Rpad, int np, double* Rout,
                                                         int rout_user, const double* __restrict__ Rprev,
                                                         const double* __restrict__ Npost, int ldnp, int32_t* info,
                                                         int32_t stage, const CholJob* __restrict__ jobs) {
  if (jobs) {  // batched: one workgroup per problem
    const CholJob j = jobs[blockIdx.x];
    G = j.G, Rpad = j.Rpad, Rout = j.Rout, Rprev = j.Rprev, info = j.info, m = j.m;
  }
  constexpr int LD = dn_ld<CS>(), NT = 64 * CS, A = 4 * CS;
  extern __shared__ __align__(16) unsigned char dn_smem[];
  double* Rl = (double*)dn_smem;  // R(i, j) at i*LD + j
  __shared__ double dg[NT];
  __shared__ int bc_fail, bc_min;
  if (info_failed(info)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tr = lane & 15, col0 = 4 * wave + (lane >> 4);
  double x[CS][A];
  // the upper triangle of G is read; the lower one is its mirror
#pragma unroll
  for (int c = 0; c < CS; ++c)
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const int row = tr + 16 * a, col = col0 + 64 * c;
      x[c][a] =
          (row < n && col < n) ? (row <= col ? G[row + (int64_t)col * ldg] : G[col + (int64_t)row * ldg]) : 0.0;
    }
  for (int e = tid; e < NT * LD; e += DN_THREADS) Rl[e] = 0.0;
  if (tid == 0) {
    bc_fail = 0;
    bc_min = INT_MAX;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CS; ++c)
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const int row = tr + 16 * a, col = col0 + 64 * c;
      if (row <= col && col < n && !is_finite(x[c][a])) atomicMin(&bc_min, col);
      if (row == col && col < n) dg[col] = x[c][a];
    }
  __syncthreads();
  if (bc_min != INT_MAX) {
    if (tid == 0) info_set(info, INFO_NONFINITE, stage, bc_min + 1);
    return;
  }
  if (shift_mode == 1) {
    // Algorithm 4's shift: 11 (m n u + n (n+1) u) max_j G_jj
    double gm = 0.0;
    for (int j = 0; j < n; ++j) gm = fmax(gm, dg[j]);
    const double u = 0x1p-53;
    const double sigma = 11.0 * ((double)m * (double)n * u + (double)n * (double)(n + 1) * u) * gm;
#pragma unroll
    for (int c = 0; c < CS; ++c)
#pragma unroll
      for (int a = 0; a < A; ++a)
        if (tr + 16 * a == col0 + 64 * c && col0 + 64 * c < n) x[c][a] += sigma;
  }
#pragma unroll
  for (int kc = 0; kc < CS; ++kc) {
    for (int kk = 0; kk < 64; ++kk) {
      const int k = 64 * kc + kk;
      if (k >= n) break;
      if (wave == (kk >> 2)) {
        double xs = x[kc][0];
#pragma unroll
        for (int a = 1; a < A; ++a)
          if (a == (k >> 4)) xs = x[kc][a];
        const double d = __shfl(xs, (lane & 48) | (k & 15));
        if (col0 == kk) {
          if (!(d > 0.0)) {
            if (tr == 0) {
              info_set(info, INFO_CHOL_BREAKDOWN, stage, k + 1);
              bc_fail = 1;
            }
          } else {
            // row k of R: r_kj = g_kj / r_kk, each correctly rounded through one
            // reciprocal and Markstein's correction (as the LU multipliers), so
            // the A quotients are independent three-operation chains. r_kk is a
            // square root of a positive double, so it lies in [2^-537, 2^512]
            // and its reciprocal is always normal (the theorem's condition).
            const double rkk = sqrt(d), y = 1.0 / rkk;
#pragma unroll
            for (int a = 0; a < A; ++a) {
              const int row = tr + 16 * a;
              const double q0 = x[kc][a] * y;
              const double q = __builtin_fma(__builtin_fma(-q0, rkk, x[kc][a]), y, q0);
              Rl[k * LD + row] = (row > k) ? q : (row == k ? rkk : 0.0);
            }
          }
        }
      }
      __syncthreads();
      // row k of R read together with the failure flag (one LDS round trip)
      double rk[A];
#pragma unroll
      for (int a = 0; a < A; ++a) rk[a] = Rl[k * LD + tr + 16 * a];
      double rkc[CS];
#pragma unroll
      for (int c = 0; c < CS; ++c) rkc[c] = Rl[k * LD + col0 + 64 * c];
      if (__builtin_amdgcn_readfirstlane(bc_fail)) return;
#pragma unroll
      for (int c = kc; c < CS; ++c) {
        if (4 * wave + 3 + 64 * c > k) {
          const int col = col0 + 64 * c;
          const double rkj = (col > k) ? rkc[c] : 0.0;
#pragma unroll
          for (int a = 0; a < A; ++a) x[c][a] = __builtin_fma(-rk[a], rkj, x[c][a]);
        }
      }
    }
  }

  const int nb = np / 16, lr = lane & 15, lq = lane >> 4;
  if (Npost) {
    // Rpad = D R N (N upper, user layout): diag(R N) = diag(R) diag(N)
    if (tid < n) {
      const double d = Rl[tid * LD + tid] * Npost[tid + (int64_t)tid * ldnp];
      dg[tid] = d;
      if (!is_finite(d) || d == 0.0) atomicMin(&bc_min, tid);
    }
    __syncthreads();
    if (bc_min != INT_MAX) {
      if (tid == 0) info_set(info, is_finite(dg[bc_min]) ? INFO_SINGULAR : INFO_NONFINITE, STAGE_PRECOND, bc_min + 1);
      return;
    }
    for (int blk = wave; blk < nb * nb; blk += DN_THREADS / 64) {
      const int I = blk / nb, J = blk % nb;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int K = I; K <= J; ++K)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int kr = 16 * K + 4 * kk + lq, j = 16 * J + lr;
          const double av = Rl[(16 * I + lr) * LD + 16 * K + 4 * kk + lq];
          const double bv = (kr <= j && j < n) ? Npost[kr + (int64_t)j * ldnp] : 0.0;
          acc = mfma_f64(av, bv, acc);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + lq + 4 * r, j = 16 * J + lr;
        double v;
        if (i < n && j < n)
          v = (i > j) ? 0.0 : (dg[i] < 0.0 ? -acc[r] : acc[r]);
        else
          v = (i == j) ? 1.0 : 0.0;
        Rpad[i * np + j] = v;
      }
    }
    if (tid < np) Rpad[np * np + tid] = (tid < n) ? 1.0 / fabs(dg[tid]) : 1.0;
    return;
  }

  for (int e = tid; e < np * np; e += DN_THREADS) {
    const int i = e / np, j = e % np;
    Rpad[e] = (i < n && j < n) ? Rl[i * LD + j] : (i == j ? 1.0 : 0.0);
  }
  if (tid < np) Rpad[np * np + tid] = (tid < n) ? 1.0 / Rl[tid * LD + tid] : 1.0;
  if (Rout) {
    // Rout = R Rprev, Rprev a padded triangle (row-major, identity padding)
    for (int blk = wave; blk < nb * nb; blk += DN_THREADS / 64) {
      const int I = blk / nb, J = blk % nb;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int K = I; K <= J; ++K)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double av = Rl[(16 * I + lr) * LD + 16 * K + 4 * kk + lq];
          const double bv = Rprev[(int64_t)(16 * K + 4 * kk + lq) * np + 16 * J + lr];
          acc = mfma_f64(av, bv, acc);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + lq + 4 * r, j = 16 * J + lr;
        if (rout_user) {
          if (i < n && j < n) Rout[i + (int64_t)j * n] = (i > j) ? 0.0 : acc[r];
        } else {
          Rout[i * np + j] = (i < n && j < n) ? ((i > j) ? 0.0 : acc[r]) : (i == j ? 1.0 : 0.0);
          if (i == j) Rout[np * np + i] = (i < n) ? 1.0 / acc[r] : 1.0;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
bool precond_reg_fits(int64_t s, int64_t n) { return n >= 1 && n <= DN_NP && s >= n && s <= 256; }

template <typename F>
static hipError_t set_lds(F* fn, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

template <typename T, int A, int CS>
static hipError_t launch_pr(const double* Y, int64_t s, int64_t n, int lu, const double* Nin, int64_t ldn,
                            double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch, int32_t* info,
                            int32_t stage_qr, hipStream_t st) {
  constexpr size_t lds = precond_reg_lds<T, A, CS>();
  static_assert(lds <= 96 * 1024, "LDS budget");
  hipError_t e = set_lds(k_precond_reg<T, A, CS>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_precond_reg<T, A, CS>), dim3(1), dim3(DN_THREADS), lds, st, Y, (int)s, (int)n, lu, Nin,
                     (int)ldn, R1pad, pad_cols(n), R1out, perm, Mout, scratch, info, stage_qr, nullptr);
  return hipGetLastError();
}

template <typename T, int A, int CS>
static hipError_t launch_pr_batch(int64_t s, int64_t n, const PrecondJob* jobs, int count, int32_t stage_qr,
                                  hipStream_t st) {
  constexpr size_t lds = precond_reg_lds<T, A, CS>();
  hipError_t e = set_lds(k_precond_reg<T, A, CS>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_precond_reg<T, A, CS>), dim3((unsigned)count), dim3(DN_THREADS), lds, st, nullptr, (int)s,
                     (int)n, 1, nullptr, 0, nullptr, pad_cols(n), nullptr, nullptr, nullptr, nullptr, nullptr,
                     stage_qr, jobs);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_pr_batch_t(int64_t s, int64_t n, const PrecondJob* jobs, int count, int32_t stage_qr,
                                    hipStream_t st) {
  if (n > 64) {
    if (s <= 128) return launch_pr_batch<T, 8, 2>(s, n, jobs, count, stage_qr, st);
    return launch_pr_batch<T, 16, 2>(s, n, jobs, count, stage_qr, st);
  }
  if (s <= 16) return launch_pr_batch<T, 1, 1>(s, n, jobs, count, stage_qr, st);
  if (s <= 32) return launch_pr_batch<T, 2, 1>(s, n, jobs, count, stage_qr, st);
  if (s <= 64) return launch_pr_batch<T, 4, 1>(s, n, jobs, count, stage_qr, st);
  if (s <= 128) return launch_pr_batch<T, 8, 1>(s, n, jobs, count, stage_qr, st);
  return launch_pr_batch<T, 16, 1>(s, n, jobs, count, stage_qr, st);
}

// Batched LU + Householder preconditioner (RCLUPP), one workgroup per problem.
hipError_t launch_precond_batch(int64_t s, int64_t n, int prec, const PrecondJob* jobs, int count, int32_t stage_qr,
                                hipStream_t st) {
  if (!precond_reg_fits(s, n)) return hipErrorInvalidValue;
  if (count <= 0) return hipSuccess;
  if (prec == 1) return launch_pr_batch_t<float>(s, n, jobs, count, stage_qr, st);
  return launch_pr_batch_t<double>(s, n, jobs, count, stage_qr, st);
}

template <typename T>
static hipError_t launch_pr_t(const double* Y, int64_t s, int64_t n, int lu, const double* Nin, int64_t ldn,
                              double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch,
                              int32_t* info, int32_t stage_qr, hipStream_t st) {
#define PR_ARGS Y, s, n, lu, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st
  if (n > 64) {
    if (s <= 128) return launch_pr<T, 8, 2>(PR_ARGS);
    return launch_pr<T, 16, 2>(PR_ARGS);
  }
  if (s <= 16) return launch_pr<T, 1, 1>(PR_ARGS);
  if (s <= 32) return launch_pr<T, 2, 1>(PR_ARGS);
  if (s <= 64) return launch_pr<T, 4, 1>(PR_ARGS);
  if (s <= 128) return launch_pr<T, 8, 1>(PR_ARGS);
  return launch_pr<T, 16, 1>(PR_ARGS);
#undef PR_ARGS
}

hipError_t launch_precond_reg(const double* Y, int64_t s, int64_t n, int lu, int prec, const double* Nin, int64_t ldn,
                              double* R1pad, double* R1out, int32_t* perm, double* Mout, double* scratch,
                              int32_t* info, int32_t stage_qr, hipStream_t st) {
  if (!precond_reg_fits(s, n)) return hipErrorInvalidValue;
  if (n > 64 && scratch == nullptr) return hipErrorInvalidValue;
  if (prec == 1)
    return launch_pr_t<float>(Y, s, n, lu, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st);
  return launch_pr_t<double>(Y, s, n, lu, Nin, ldn, R1pad, R1out, perm, Mout, scratch, info, stage_qr, st);
}

hipError_t launch_chol_reg(const double* G, int ldg, int64_t n, int64_t m, int shift_mode, double* Rpad, double* Rout,
                           int rout_user, const double* Rprev, const double* Npost, int64_t ldnp, int32_t* info,
                           int32_t stage, hipStream_t st) {
  if (n < 1 || n > DN_NP || (Npost && Rout)) return hipErrorInvalidValue;
  if (n <= 64) {
    constexpr size_t lds = chol_reg_lds<1>();
    hipLaunchKernelGGL(k_chol_reg<1>, dim3(1), dim3(DN_THREADS), lds, st, G, ldg, (int)n, m, shift_mode, Rpad,
                       pad_cols(n), Rout, rout_user, Rprev, Npost, (int)ldnp, info, stage, nullptr);
    return hipGetLastError();
  }
  constexpr size_t lds = chol_reg_lds<2>();
  hipError_t e = set_lds(k_chol_reg<2>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_reg<2>, dim3(1), dim3(DN_THREADS), lds, st, G, ldg, (int)n, m, shift_mode, Rpad,
                     pad_cols(n), Rout, rout_user, Rprev, Npost, (int)ldnp, info, stage, nullptr);
  return hipGetLastError();
}

// Batched Cholesky (+ product with an earlier factor), one workgroup per problem.
hipError_t launch_chol_batch(int64_t n, int ldg, int rout_user, const CholJob* jobs, int count, int32_t stage,
                             hipStream_t st) {
  if (n < 1 || n > DN_NP) return hipErrorInvalidValue;
  if (count <= 0) return hipSuccess;
  if (n <= 64) {
    constexpr size_t lds = chol_reg_lds<1>();
    hipLaunchKernelGGL(k_chol_reg<1>, dim3((unsigned)count), dim3(DN_THREADS), lds, st, nullptr, ldg, (int)n, 0, 0,
                       nullptr, pad_cols(n), nullptr, rout_user, nullptr, nullptr, 0, nullptr, stage, jobs);
    return hipGetLastError();
  }
  constexpr size_t lds = chol_reg_lds<2>();
  hipError_t e = set_lds(k_chol_reg<2>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_reg<2>, dim3((unsigned)count), dim3(DN_THREADS), lds, st, nullptr, ldg, (int)n, 0, 0,
                     nullptr, pad_cols(n), nullptr, rout_user, nullptr, nullptr, 0, nullptr, stage, jobs);
  return hipGetLastError();
}

}  // namespace rclupp
