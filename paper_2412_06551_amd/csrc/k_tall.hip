// Tall passes of CholeskyQR (Algorithm 1 steps 1 and 3) around a small upper
// triangular R:  W = X R^{-1}  and  G = W^T W.
//
// Layout and mapping. One thread owns one row of the tall operand: its n
// entries are read with one coalesced 512-byte access per column per wave
// (column-major data), the row is solved in registers by substitution
//   w_j = (x_j - sum_{i<j} w_i R_ij) / R_jj   (backward stable, eq. ewy; no
//   explicit inverse of the possibly very ill-conditioned R_1),
// with R (wave-uniform) streamed through the scalar data path, and written
// back with the same coalesced pattern. For n <= 64 the Gram partial sum is
// fused: each wave stages its rows (32 at a time) column-major in its own LDS
// region and feeds v_mfma_f64_16x16x4_f64 with 16-column fragments, upper
// 16x16 blocks only. For larger n the substitution walks 64-column blocks
// (earlier blocks of the row are re-read from W, which the thread wrote) and
// the Gram is a separate MFMA pass over W.
// Per-workgroup Gram partials are added in workgroup order by a second kernel.
#include "device_common.hpp"
#include "launch.hpp"

namespace rclupp {

constexpr int TP_THREADS = 256;
constexpr int TP_HALF = 32;           // rows staged per LDS round in the fused Gram
constexpr int TP_LDW = TP_HALF + 1;   // LDS column stride (doubles)

int pad_cols(int64_t n) {
  if (n <= 16) return 16;
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  if (n <= 128) return 128;
  return 256;
}

// ---------------------------------------------------------------------------
// n <= 64: fused substitution + Gram.
// ---------------------------------------------------------------------------
template <int NP, bool TRSM, bool GRAM, bool WRITE>
__global__ __launch_bounds__(TP_THREADS) void k_tall_pass(const double* X, int64_t ldx, int64_t m, int n,
                                                          const double* __restrict__ Rp, double* W, int64_t ldw,
                                                          double* __restrict__ Gpart, int64_t ntiles,
                                                          const int32_t* info) {
  if (info_failed(info)) return;
  constexpr int NBK = NP / 16;
  constexpr int NBLK = NBK * (NBK + 1) / 2;
  __shared__ double lds[GRAM ? 4 * NP * TP_LDW : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  f64x4 gacc[GRAM ? NBLK : 1];
#pragma unroll
  for (int b = 0; b < (GRAM ? NBLK : 1); ++b) gacc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
  double* ws = lds + wave * NP * TP_LDW;

  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row = t * TP_THREADS + tid;
    const bool live = row < m;
    double w[NP];
    {
      const double* xp = X + row;
      const int64_t step = opaque_i64(ldx);
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        w[c] = (live && c < n) ? *xp : 0.0;
        xp += opaque_i64(step);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (TRSM) {
      const cdptr R = opaque_uniform(Rp);  // row-major padded triangle
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        w[j] *= R[NP * NP + j];
#pragma unroll
        for (int k = j + 1; k < NP; ++k) w[k] = __builtin_fma(-w[j], R[j * NP + k], w[k]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (WRITE && live) {
      double* wp = W + row;
      const int64_t step = opaque_i64(ldw);
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        if (c < n) *wp = w[c];
        wp += opaque_i64(step);
      }
    }
    if (GRAM) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if ((lane >> 5) == h) {
#pragma unroll
          for (int c = 0; c < NP; ++c) ws[c * TP_LDW + (lane & 31)] = w[c];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TP_HALF / 4; ++kk) {
          double f[NBK];
#pragma unroll
          for (int ib = 0; ib < NBK; ++ib) f[ib] = ws[(16 * ib + (lane & 15)) * TP_LDW + 4 * kk + (lane >> 4)];
          int b = 0;
#pragma unroll
          for (int jb = 0; jb < NBK; ++jb)
#pragma unroll
            for (int ib = 0; ib <= jb; ++ib) {
              gacc[b] = mfma_f64(f[ib], f[jb], gacc[b]);
              ++b;
            }
        }
        __syncthreads();
      }
    }
  }

  if (GRAM) {
    // sum the four waves in order, then write the workgroup partial (upper blocks)
    double* red = lds;  // NBLK * 4 * 64 doubles <= 4 * NP * TP_LDW
    for (int w = 0; w < 4; ++w) {
      if (wave == w) {
        int b = 0;
#pragma unroll
        for (int jb = 0; jb < NBK; ++jb)
#pragma unroll
          for (int ib = 0; ib <= jb; ++ib) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int idx = (b * 4 + r) * 64 + lane;
              const double v = (w == 0) ? gacc[b][r] : red[idx] + gacc[b][r];
              if (w < 3) {
                red[idx] = v;
              } else {
                const int gi = 16 * ib + (lane >> 4) + 4 * r, gj = 16 * jb + (lane & 15);
                Gpart[(int64_t)blockIdx.x * NP * NP + gi + gj * NP] = v;
              }
            }
            ++b;
          }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// n > 64: blocked substitution (64-column blocks), no Gram.
// ---------------------------------------------------------------------------
template <int NP>
__global__ __launch_bounds__(TP_THREADS) void k_tall_trsm_big(const double* X, int64_t ldx, int64_t m, int n,
                                                              const double* __restrict__ Rp, double* W, int64_t ldw,
                                                              int64_t ntiles, const int32_t* info) {
  if (info_failed(info)) return;
  const int tid = threadIdx.x;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row = t * TP_THREADS + tid;
    if (row >= m) continue;
    for (int cb = 0; cb < NP / 64; ++cb) {
      const int c0 = cb * 64;
      if (c0 >= n) break;
      double acc[64];
#pragma unroll
      for (int c = 0; c < 64; ++c) acc[c] = (c0 + c < n) ? X[row + (int64_t)(c0 + c) * ldx] : 0.0;
      for (int i = 0; i < c0; ++i) {
        const double wi = W[row + (int64_t)i * ldw];
        const cdptr ri = opaque_after(Rp + (int64_t)i * NP + c0, wi);
#pragma unroll
        for (int c = 0; c < 64; ++c) acc[c] = __builtin_fma(-wi, ri[c], acc[c]);
      }
#pragma unroll
      for (int j = 0; j < 64; ++j) {
        const cdptr Rj = opaque_after(Rp + (int64_t)(c0 + j) * NP + c0, acc[j >= 2 ? j - 2 : 0]);
        acc[j] *= Rj[NP * NP - (c0 + j) * NP - c0 + c0 + j];
#pragma unroll
        for (int k = j + 1; k < 64; ++k) acc[k] = __builtin_fma(-acc[j], Rj[k], acc[k]);
      }
#pragma unroll
      for (int c = 0; c < 64; ++c)
        if (c0 + c < n) W[row + (int64_t)(c0 + c) * ldw] = acc[c];
    }
  }
}

// ---------------------------------------------------------------------------
// n > 64: Gram partials of W over 32-row LDS tiles. The upper 16x16 blocks
// are split by block column: workgroup row y and wave w own block columns
// jb = 8 y + w + 4 jj (jj = 0, 1), so each wave keeps at most 2 NP/16
// accumulators; gridDim.y = NP / 128.
// ---------------------------------------------------------------------------
template <int NP>
__global__ __launch_bounds__(TP_THREADS) void k_gram_big(const double* __restrict__ W, int64_t ldw, int64_t m, int n,
                                                         double* __restrict__ Gpart, int64_t ntiles32,
                                                         const int32_t* info) {
  if (info_failed(info)) return;
  constexpr int NBK = NP / 16;
  constexpr int JPW = 2;
  constexpr int MAXB = JPW * NBK;
  __shared__ double lds[NP * TP_LDW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int jbase = 8 * (int)blockIdx.y + wave;
  f64x4 acc[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};

  for (int64_t t = blockIdx.x; t < ntiles32; t += gridDim.x) {
    // load 32 rows x NP columns: thread -> row (tid % 32), columns tid/32 + 8 k
    const int lr = tid & 31, lc = tid >> 5;
    const int64_t row = t * 32 + lr;
#pragma unroll
    for (int k = 0; k < NP / 8; ++k) {
      const int c = lc + 8 * k;
      lds[c * TP_LDW + lr] = (row < m && c < n) ? W[row + (int64_t)c * ldw] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      double f[NBK];
#pragma unroll
      for (int ib = 0; ib < NBK; ++ib) f[ib] = lds[(16 * ib + (lane & 15)) * TP_LDW + 4 * kk + (lane >> 4)];
#pragma unroll
      for (int jj = 0; jj < JPW; ++jj) {
        const int jb = jbase + 4 * jj;
        double fj = f[0];
#pragma unroll
        for (int q = 1; q < NBK; ++q)
          if (q == jb) fj = f[q];
#pragma unroll
        for (int ib = 0; ib < NBK; ++ib)
          if (ib <= jb) acc[jj * NBK + ib] = mfma_f64(f[ib], fj, acc[jj * NBK + ib]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int jj = 0; jj < JPW; ++jj) {
    const int jb = jbase + 4 * jj;
#pragma unroll
    for (int ib = 0; ib < NBK; ++ib) {
      if (ib > jb) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = 16 * ib + (lane >> 4) + 4 * r, gj = 16 * jb + (lane & 15);
        Gpart[(int64_t)blockIdx.x * NP * NP + gi + gj * NP] = acc[jj * NBK + ib][r];
      }
    }
  }
}

// G[i + j*np] = sum_b Gpart[b][i + j*np] for i <= j (mirrored), padded with the
// identity beyond n (so a padded Cholesky stays the identity there).
__global__ void k_gram_reduce(const double* __restrict__ Gpart, int gx, int np, int64_t n, double* __restrict__ G,
                              const int32_t* info) {
  if (info_failed(info)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)np * np) return;
  const int i = (int)(e % np), j = (int)(e / np);
  if (i > j) return;
  double v;
  if (j >= n) {
    v = (i == j) ? 1.0 : 0.0;
  } else {
    const int64_t stride = (int64_t)np * np;
    v = 0.0;
    for (int b = 0; b < gx; ++b) v += Gpart[(int64_t)b * stride + e];
  }
  G[i + (int64_t)j * np] = v;
  G[j + (int64_t)i * np] = v;
}

TallPlan plan_tall(int64_t m, int64_t n, int gx_hint) {
  TallPlan p{};
  p.np = pad_cols(n);
  p.fused_gram = p.np <= 64;
  p.tile_rows = TP_THREADS;
  p.ntiles = (m + TP_THREADS - 1) / TP_THREADS;
  int gx = gx_hint > 0 ? gx_hint : 512;
  if (gx > p.ntiles) gx = (int)p.ntiles;
  if (gx < 1) gx = 1;
  p.gx = gx;
  p.part_bytes = (size_t)gx * p.np * p.np * sizeof(double);
  return p;
}

template <int NP>
static hipError_t launch_tp(const TallPlan& p, const double* X, int64_t ldx, int64_t m, int64_t n, const double* Rp,
                            double* W, int64_t ldw, double* Gpart, const int32_t* info, hipStream_t st) {
  dim3 grid(p.gx), block(TP_THREADS);
  const bool trsm = Rp != nullptr, gram = Gpart != nullptr, write = W != nullptr;
  if (NP <= 64) {
#define TP_CASE(T, G, Wr)                                                                                          \
  if (trsm == T && gram == G && write == Wr) {                                                                     \
    hipLaunchKernelGGL((k_tall_pass<(NP <= 64 ? NP : 64), T, G, Wr>), grid, block, 0, st, X, ldx, m, (int)n, Rp, W, \
                       ldw, Gpart, p.ntiles, info);                                                                 \
    return hipGetLastError();                                                                                       \
  }
    TP_CASE(true, true, true)
    TP_CASE(false, true, false)
#undef TP_CASE
    return hipErrorInvalidValue;
  }
  // n > 64: substitution kernel (if any), then the Gram kernel over W (or X)
  if (trsm) {
    if (!write) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tall_trsm_big<(NP > 64 ? NP : 128)>), grid, block, 0, st, X, ldx, m, (int)n, Rp, W, ldw,
                       p.ntiles, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else if (write) {
    return hipErrorInvalidValue;
  }
  if (gram) {
    const double* src = trsm ? W : X;
    const int64_t lds_ = trsm ? ldw : ldx;
    const int64_t nt32 = (m + 31) / 32;
    dim3 ggrid(p.gx, NP / 128);
    hipLaunchKernelGGL((k_gram_big<(NP > 64 ? NP : 128)>), ggrid, block, 0, st, src, lds_, m, (int)n, Gpart, nt32,
                       info);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_tall_pass(const TallPlan& p, const double* X, int64_t ldx, int64_t m, int64_t n, const double* Rpad,
                            double* W, int64_t ldw, double* Gpart, const int32_t* info, hipStream_t st) {
  switch (p.np) {
    case 16: return launch_tp<16>(p, X, ldx, m, n, Rpad, W, ldw, Gpart, info, st);
    case 32: return launch_tp<32>(p, X, ldx, m, n, Rpad, W, ldw, Gpart, info, st);
    case 64: return launch_tp<64>(p, X, ldx, m, n, Rpad, W, ldw, Gpart, info, st);
    case 128: return launch_tp<128>(p, X, ldx, m, n, Rpad, W, ldw, Gpart, info, st);
    case 256: return launch_tp<256>(p, X, ldx, m, n, Rpad, W, ldw, Gpart, info, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gram_reduce(const TallPlan& p, const double* Gpart, int64_t n, double* G, const int32_t* info,
                              hipStream_t st) {
  const int64_t total = (int64_t)p.np * p.np;
  const int threads = 256;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, st, Gpart,
                     p.gx, p.np, n, G, info);
  return hipGetLastError();
}

}  // namespace rclupp
