// Tall passes of CholeskyQR (Algorithm 1 steps 1 and 3) around a small upper
// triangular R:  W = X R^{-1}  and  G = W^T W.
//
// n <= 64: one fused kernel per pass (k_tall_mfma). The substitution
//   w_j = (x_j - sum_{i<j} w_i R_ij) / R_jj   (row-wise backward stable, eq. ewy
//   and eqs. C3, C7; no explicit inverse of the possibly very ill-conditioned R_1)
// runs blocked on the FP64 matrix cores with the diagonal blocks finished row
// by row in registers; the Gram partial sum of the solved rows is fused.
// n > 64: the same blocked substitution without the fused Gram (the
// off-diagonal fragments are read from R through the cache), then a separate
// MFMA Gram kernel over W.
// Per-workgroup Gram partials are added in a fixed two-level order by
// k_partial_sum and k_gram_final, so results do not depend on timing.
#include <type_traits>

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
// n <= 64: blocked substitution on the matrix cores, fused Gram.
//
// The solve is written transposed, W^T = R^{-T} X^T, in 16-column blocks b,
// right-looking: once block b is solved (substitution over its 16 columns,
// W_b^T = R_{b,b}^{-T} C_b^T), every later block d takes its term
//   C_d^T -= R_{b,d}^T W_b^T                              (v_mfma_f64_16x16x4_f64),
// so C_d^T = X_d^T - sum_{b<d} R_{b,d}^T W_b^T accumulates in ascending b and
// the products for different d are independent.
// MFMA roles: M = the 16 columns of block b, N = 16 rows of X, K = 4 columns of
// an earlier block c. The output layout (lane l, register r holds row l%16,
// column 16b + l/16 + 4r) is exactly the B-operand layout the later blocks
// need (B fragment kk of block c = output register kk, columns 16c + 4kk + k
// in K order), so solved blocks stay in registers and every column takes its
// terms in ascending order. The off-diagonal A fragments (-R_{c,b}^T) are
// built in LDS once per workgroup.
// The diagonal block is solved row by row: the wave's 32 rows go through a
// per-wave LDS transpose so that lane l < 32 holds the 16 block entries of one
// row, which it finishes in registers,
//   w_j = (c_j - sum_{i<j} w_i R_ij) * y_j,   y_j = RN(1/R_jj),
// with fused multiply-adds in ascending i, right-looking (each finished w_i is
// sent to all later columns at once), so the dependent chain per column is one
// multiply-add and one multiply. Multiplying by the rounded reciprocal instead
// of dividing perturbs R_jj by at most 2u relative, so the row-wise bound of
// eq. ewy holds with gamma_{n+1} in place of gamma_n. The R entries and the
// reciprocals are wave-uniform and come through the scalar cache.
// Each wave handles two 16-row blocks (32 rows) for NP <= 64, four waves
// covering a 128-row tile; for NP = 128 each wave handles one 16-row block and
// eight waves cover the 128-row tile (with half the accumulators per wave, four
// waves share a SIMD instead of two, which hides more of the memory latency:
// measured 8 % faster). X and W move in 128-byte row segments.
// The Gram partial sums stage the solved rows in a per-wave LDS region
// (column-major, stride 17) and use v_mfma_f64_16x16x4_f64 on the upper
// 16x16 blocks.
// ---------------------------------------------------------------------------
// 16-row blocks per wave and waves per workgroup: 2 and 4 up to NP = 64, 1 and
// 8 for NP = 128
constexpr int tm_hb(int np) { return np >= 128 ? 1 : 2; }
constexpr int tm_waves(int np) { return np == 128 ? 8 : 4; }
constexpr int tm_tile(int np) { return 16 * tm_waves(np) * tm_hb(np); }  // rows per workgroup tile
constexpr int TM_LDG = 17;                 // Gram staging: 16 rows + pad per column
constexpr int TM_LDT = 18;                 // diagonal transpose: 16 entries + pad per row (16-byte aligned)

// RS, ROFF: R is the ROFF x ROFF-offset NP x NP diagonal block of a padded
// triangle with row stride RS (Rp points at its first entry; the reciprocals
// of its diagonal then sit RS (RS - ROFF) entries further on). The defaults
// are the whole padded triangle.
template <int NP, bool TRSM, bool GRAM, bool WRITE, int RS = NP, int ROFF = 0>
__global__ __launch_bounds__(64 * tm_waves(NP), (NP > 128 ? 1 : 2)) void k_tall_mfma(const double* X, int64_t ldx, int64_t m, int n,
                                                            const double* __restrict__ Rp, double* W, int64_t ldw,
                                                            double* __restrict__ Gpart, int64_t ntiles,
                                                            const int32_t* info, const TallJob* __restrict__ jobs,
                                                            const BatchItem* __restrict__ items) {
  int64_t wg = blockIdx.x, nwg = gridDim.x;
  if (items) {  // batched launch: this workgroup's problem and its place in it
    const BatchItem it = items[blockIdx.x];
    const TallJob j = jobs[it.prob];
    X = j.X, ldx = j.ldx, m = j.m, ntiles = j.ntiles, Rp = j.Rp, W = j.W, ldw = j.ldw, Gpart = j.Gpart;
    info = j.info, wg = it.wg, nwg = it.nwg;
  }
  if (info_failed(info)) return;
  constexpr int NB = NP / 16;                  // column blocks
  constexpr int NOFF = NB * (NB - 1) / 2;      // off-diagonal block pairs c < b
  constexpr int NBLK = NB * (NB + 1) / 2;      // upper Gram blocks
  constexpr int HB = tm_hb(NP), RW = 16 * HB;           // 16-row blocks and rows per wave
  static_assert(!GRAM || tm_waves(NP) == 4, "the fused Gram's staging and reduction assume four waves");
  // per-wave transpose regions; with the Gram they share the per-wave Gram
  // staging regions (used after the solve of the tile), which are larger
  constexpr bool SHARE = GRAM && NP * TM_LDG >= RW * TM_LDT;
  constexpr int TTAB = (TRSM && !SHARE) ? tm_waves(NP) * RW * TM_LDT : 1;
  constexpr int GST = GRAM ? ((4 * NP * TM_LDG > NBLK * 256) ? 4 * NP * TM_LDG : NBLK * 256) : 1;
  // off-diagonal A fragments: an LDS table for NP <= 64, read from R (L2) above
  constexpr bool OG = NP > 128;
  constexpr int OTAB = (TRSM && NOFF > 0 && !OG) ? NOFF * 4 * 64 : 1;  // [pair][kk][lane]
  __shared__ double otab[OTAB];
  __shared__ __align__(16) double gst[GST];
  __shared__ __align__(16) double ttab[TTAB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;

  if (TRSM) {
    // off-diagonal A fragments: otab[(pair*4 + kk)*64 + lane] = -R[16c + 4kk + l/16][16b + l%16]
    for (int e = tid; e < OTAB && NOFF > 0 && !OG; e += 64 * tm_waves(NP)) {
      const int l = e & 63, kk = (e >> 6) & 3, pr = e >> 8;
      int b = 1, c = pr;
      while (c >= b) {
        c -= b;
        ++b;
      }
      otab[e] = -Rp[(16 * c + 4 * kk + (l >> 4)) * RS + 16 * b + (l & 15)];
    }
  }
  __syncthreads();

  f64x4 gacc[GRAM ? NBLK : 1];
#pragma unroll
  for (int g = 0; g < (GRAM ? NBLK : 1); ++g) gacc[g] = f64x4{0.0, 0.0, 0.0, 0.0};
  double* ws = gst + wave * NP * TM_LDG;

  // X tile of this wave in the MFMA B layout. Addresses: a wave-uniform column
  // base (scalar) plus a 32-bit per-lane offset (row + (l/16) ld); requires
  // 3 ld + m < 2^29, checked by the launcher. Streamed once: nontemporal, so X
  // and W do not evict R, the tables and the partials from the caches.
  // (nontemporal only when the column runs fill whole lines)
  const bool ntx = runs_line_aligned(X, ldx), ntw = WRITE && runs_line_aligned(W, ldw);
  auto load_rows = [&](auto nt, int64_t tt, f64x4 (&dst)[HB][NB]) {
    constexpr bool NT = decltype(nt)::value;
    const int64_t r0 = tt * tm_tile(NP) + wave * RW;
#pragma unroll
    for (int h = 0; h < HB; ++h) {
      const int64_t row = r0 + 16 * h + lr;
      const bool live = row < m;
      const uint32_t voff = (uint32_t)(row + (int64_t)lq * ldx);
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * b + lq + 4 * r;
          const double* cb = X + (int64_t)(16 * b + 4 * r) * ldx;
          dst[h][b][r] = (live && col < n) ? stream_load<NT>(cb + voff) : 0.0;
        }
    }
  };
  auto load_x = [&](int64_t tt, f64x4 (&dst)[HB][NB]) {
    if (ntx) load_rows(std::true_type{}, tt, dst);
    else load_rows(std::false_type{}, tt, dst);
  };
  // n = 64 with the Gram: the next tile's loads are issued before this tile's
  // work (64 more registers, still two workgroups per CU), so they are in
  // flight during it. A tile t + nwg belongs to this workgroup alone, so the
  // early read never sees another workgroup's writes, also in place.
  constexpr bool PF = NP == 64 && GRAM && TRSM;
  f64x4 pre[HB][NB];
  if (PF && wg < ntiles) load_x(wg, pre);

  for (int64_t t = wg; t < ntiles; t += nwg) {
    const int64_t row0 = t * tm_tile(NP) + wave * RW;
    f64x4 acc[HB][NB];
    if (PF) {
#pragma unroll
      for (int h = 0; h < HB; ++h)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[h][b] = pre[h][b];
      if (t + nwg < ntiles) load_x(t + nwg, pre);
    } else {
      load_x(t, acc);
    }
    if (TRSM) {
      // opaque per tile: keeps the table reads inside the tile loop (hoisting
      // all of them would need hundreds of registers)
      int dofs = 0;
      asm volatile("" : "+s"(dofs));
      const cdptr Rt = opaque_uniform(Rp);
      // per-lane base of the off-diagonal fragments read from R (NP = 256):
      // kept in VGPRs, so each fragment address is this base plus a constant
      // rather than a scalar base register per (b, kk, d)
      const double* Rl = Rp + lq * RS + lr;
      if (OG) asm volatile("" : "+v"(Rl));
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        // (all terms of the blocks c < b are in: solve the diagonal block b)
        // transpose so that lane l < RW holds row l's 16 entries, substitute in
        // registers, transpose back
        double* tt = SHARE ? gst + wave * NP * TM_LDG : ttab + wave * RW * TM_LDT;
#pragma unroll
        for (int h = 0; h < HB; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) tt[(16 * h + lr) * TM_LDT + lq + 4 * r] = acc[h][b][r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < RW) {
          double v[16];
          const double2* src = (const double2*)(tt + lane * TM_LDT);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const double2 q = src[e];
            v[2 * e] = q.x;
            v[2 * e + 1] = q.y;
          }
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            // the scalar loads of row j run at most two rows ahead of the
            // substitution (all of them at once would not fit the SGPRs)
            const cdptr Rj = (j < 2) ? Rt : opaque_after(Rp, v[j - 2]);
            v[j] *= Rj[RS * (RS - ROFF) + 16 * b + j];
#pragma unroll
            for (int k = j + 1; k < 16; ++k) v[k] = __builtin_fma(-v[j], Rj[(16 * b + j) * RS + 16 * b + k], v[k]);
          }
          double2* dst = (double2*)(tt + lane * TM_LDT);
#pragma unroll
          for (int e = 0; e < 8; ++e) dst[e] = double2{v[2 * e], v[2 * e + 1]};
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int h = 0; h < HB; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[h][b][r] = tt[(16 * h + lr) * TM_LDT + lq + 4 * r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // right-looking: C_d^T -= R_{b,d}^T W_b^T for every later block d > b
        // (each block still takes its terms in ascending column order; the
        // products for different d are independent and pipeline on the MFMA unit)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int d = b + 1; d < NB; ++d) {
            const int pr = d * (d - 1) / 2 + b;
            const double a = OG ? -Rl[(16 * b + 4 * kk) * RS + 16 * d] : otab[dofs + (pr * 4 + kk) * 64 + lane];
#pragma unroll
            for (int h = 0; h < HB; ++h) acc[h][d] = mfma_f64(a, acc[h][b][kk], acc[h][d]);
          }
      }
    }
    if (WRITE) {
      auto store_rows = [&](auto nt) {
        constexpr bool NT = decltype(nt)::value;
#pragma unroll
        for (int h = 0; h < HB; ++h) {
          const int64_t row = row0 + 16 * h + lr;
          const uint32_t voff = (uint32_t)(row + (int64_t)lq * ldw);
          if (row < m) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int col = 16 * b + lq + 4 * r;
                double* cb = W + (int64_t)(16 * b + 4 * r) * ldw;
                if (col < n) stream_store<NT>(acc[h][b][r], cb + voff);
              }
          }
        }
      };
      if (ntw) store_rows(std::true_type{});
      else store_rows(std::false_type{});
    }
    if (GRAM) {
      // stage 16 rows at a time column-major (stride TM_LDG), then Gram fragments
#pragma unroll
      for (int h = 0; h < HB; ++h) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) ws[(16 * b + lq + 4 * r) * TM_LDG + lr] = acc[h][b][r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          double f[NB];
#pragma unroll
          for (int ib = 0; ib < NB; ++ib) f[ib] = ws[(16 * ib + lr) * TM_LDG + 4 * kk + lq];
          int g = 0;
#pragma unroll
          for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int ib = 0; ib <= jb; ++ib) {
              gacc[g] = mfma_f64(f[ib], f[jb], gacc[g]);
              ++g;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }

  if (GRAM) {
    // sum the four waves in order, then write the workgroup partial (upper blocks)
    __syncthreads();
    double* red = gst;  // NBLK * 4 * 64 doubles <= GST
    for (int w = 0; w < 4; ++w) {
      if (wave == w) {
        int g = 0;
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
          for (int ib = 0; ib <= jb; ++ib) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int idx = (g * 4 + r) * 64 + lane;
              const double v = (w == 0) ? gacc[g][r] : red[idx] + gacc[g][r];
              if (w < 3) {
                red[idx] = v;
              } else {
                const int gi = 16 * ib + lq + 4 * r, gj = 16 * jb + lr;
                Gpart[wg * NP * NP + gi + gj * NP] = v;
              }
            }
            ++g;
          }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// n in (128, 256]: the solve is split at column 128,
//   W_1 = X_1 R_11^{-1},   W_2 = (X_2 - W_1 R_12) R_22^{-1},
// the two solves on the 128-column kernel (R_11 and R_22 addressed inside the
// 256 padded triangle) and the product between them here:
//   C_2 = X_2 - W_1 R_12  on v_mfma_f64_16x16x4_f64, written as
//   C_2^T = X_2^T - R_12^T W_1^T, with -R_12^T in LDS as A fragments and W_1^T
//   streamed in the B layout; each entry takes its 128 terms in ascending
//   order. 512 threads, 32 rows per wave, 256-row tiles.
// (Splitting keeps the off-diagonal fragments of the solves in LDS and the
// diagonal substitutions on 32 lanes; the one-kernel 256-column form had to
// read them through the cache one wave-fragment at a time.)
// ---------------------------------------------------------------------------
constexpr int GS_THREADS = 512;
constexpr int GS_TILE = 256;

template <int ND>
constexpr size_t gemm_sub_lds() {
  return (size_t)32 * ND * 64 * sizeof(double);
}

template <int ND>
__global__ __launch_bounds__(GS_THREADS) void k_tall_gemm_sub(const double* X2, int64_t ldx, int64_t m, int n2,
                                                              const double* W1, int64_t ldw1,
                                                              const double* __restrict__ R12, int ldr, double* W2,
                                                              int64_t ldw2, int64_t ntiles, const int32_t* info) {
  if (info_failed(info)) return;
  extern __shared__ __align__(16) unsigned char gs_smem[];
  double* atab = (double*)gs_smem;  // [kk][d][lane] = -R12[4 kk + l/16][16 d + l%16]
  constexpr int HB = 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  for (int e = tid; e < 32 * ND * 64; e += GS_THREADS) {
    const int l = e & 63, d = (e >> 6) % ND, kk = (e >> 6) / ND;
    const int col = 16 * d + (l & 15);
    atab[e] = (col < n2) ? -R12[(int64_t)(4 * kk + (l >> 4)) * ldr + col] : 0.0;
  }
  __syncthreads();
  // nontemporal only when every operand's column runs fill whole lines
  const bool nt = runs_line_aligned(X2, ldx) && runs_line_aligned(W1, ldw1) && runs_line_aligned(W2, ldw2);
  auto tiles = [&](auto ntc) {
  constexpr bool NT = decltype(ntc)::value;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * GS_TILE + wave * 32;
    f64x4 acc[HB][ND];
    // C = X_2 in the output layout: lane l, register r holds row l%16, column 16 d + l/16 + 4 r
#pragma unroll
    for (int h = 0; h < HB; ++h) {
      const int64_t row = row0 + 16 * h + lr;
      const bool live = row < m;
      const uint32_t voff = (uint32_t)(row + (int64_t)lq * ldx);
#pragma unroll
      for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * d + lq + 4 * r;
          const double* cb = X2 + (int64_t)(16 * d + 4 * r) * ldx;
          acc[h][d][r] = (live && col < n2) ? stream_load<NT>(cb + voff) : 0.0;
        }
    }
#pragma unroll 2
    for (int kk = 0; kk < 32; ++kk) {
      // B fragment: lane l holds W_1[row l%16][4 kk + l/16]
      double b[HB];
      const double* wb = W1 + (int64_t)(4 * kk) * ldw1;
#pragma unroll
      for (int h = 0; h < HB; ++h) {
        const int64_t row = row0 + 16 * h + lr;
        const double* p = wb + (uint32_t)(row + (int64_t)lq * ldw1);
        b[h] = (row < m) ? stream_load<NT>(p) : 0.0;
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const double a = atab[(kk * ND + d) * 64 + lane];
#pragma unroll
        for (int h = 0; h < HB; ++h) acc[h][d] = mfma_f64(a, b[h], acc[h][d]);
      }
    }
#pragma unroll
    for (int h = 0; h < HB; ++h) {
      const int64_t row = row0 + 16 * h + lr;
      if (row < m) {
        const uint32_t voff = (uint32_t)(row + (int64_t)lq * ldw2);
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = 16 * d + lq + 4 * r;
            double* cb = W2 + (int64_t)(16 * d + 4 * r) * ldw2;
            if (col < n2) stream_store<NT>(acc[h][d][r], cb + voff);
          }
      }
    }
  }
  };
  if (nt) tiles(std::true_type{});
  else tiles(std::false_type{});
}

// ---------------------------------------------------------------------------
// n > 64: Gram partials of W on the FP64 matrix cores. The NB (NB + 1) / 2
// upper 16 x 16 blocks are dealt round-robin to the NW waves of a workgroup
// (wave w owns blocks w, w + NW, ...), so each block lives in one wave's
// accumulators and the waves' loads are balanced; 32-row tiles of all NP
// columns are double-buffered through LDS (column-major, stride 33). NW = 4
// for NP = 128 (9 blocks per wave), NW = 8 for NP = 256 (17 blocks).
// ---------------------------------------------------------------------------
template <int NP>
constexpr int gram_waves() {
  // 16 waves (n = 256) or 8 (n = 128) in the one or two workgroups that fit a
  // CU's LDS: four or two waves per SIMD, so one wave's LDS fragment reads and
  // barrier waits overlap another's MFMAs (with 8 and 4 waves: 7.5 and 1.9 ms
  // per pass at 4,194,304 rows, now 6.0 and 1.6 ms)
  return NP > 128 ? 16 : 8;
}
template <int NP>
constexpr size_t gram_lds() {
  return (size_t)2 * NP * TP_LDW * sizeof(double);
}

template <int NP>
__global__ __launch_bounds__(64 * gram_waves<NP>()) void k_gram_bal(const double* __restrict__ W, int64_t ldw,
                                                                     int64_t m, int n, double* __restrict__ Gpart,
                                                                     int64_t ntiles32, const int32_t* info,
                                                                     const TallJob* __restrict__ jobs,
                                                                     const BatchItem* __restrict__ items) {
  int64_t wg = blockIdx.x, nwg = gridDim.x;
  if (items) {  // batched: the Gram of the job's W (its X when it has no solve)
    const BatchItem it = items[blockIdx.x];
    const TallJob j = jobs[it.prob];
    W = j.W ? j.W : j.X, ldw = j.W ? j.ldw : j.ldx, m = j.m, ntiles32 = (j.m + 31) / 32, Gpart = j.Gpart;
    info = j.info, wg = it.wg, nwg = it.nwg;
  }
  if (info_failed(info)) return;
  constexpr int NW = gram_waves<NP>(), NT = 64 * NW, NB = NP / 16, NBLK = NB * (NB + 1) / 2;
  constexpr int PB = (NBLK + NW - 1) / NW;  // blocks per wave (at most)
  constexpr int PER = 32 * NP / NT;         // tile entries loaded per thread
  extern __shared__ __align__(16) unsigned char gb_smem[];
  double* lds = (double*)gb_smem;  // [2][NP][TP_LDW]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: block indices stay scalar
  const int lr = lane & 15, lq = lane >> 4;
  // this wave's blocks: (ib, jb) of upper-block index g = wave + NW q, ib <= jb,
  // enumerated column by column
  int bi[PB], bj[PB];
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    int g = wave + NW * q, jb = 0;
    while (g > jb) {
      g -= jb + 1;
      ++jb;
    }
    bi[q] = g;
    bj[q] = jb;
  }
  f64x4 acc[PB];
#pragma unroll
  for (int q = 0; q < PB; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};

  // loader: thread -> row tid % 32, columns tid / 32 + (NT / 32) c
  const int ldr = tid & 31, ldc = tid >> 5;
  double pre[PER];
  // (nontemporal only when the column runs fill whole lines)
  const bool ntw = runs_line_aligned(W, ldw);
  auto load_rows = [&](auto ntc, int64_t t) {
    constexpr bool NTL = decltype(ntc)::value;
    const int64_t row = t * 32 + ldr;
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int col = ldc + (NT / 32) * c;
      pre[c] = (row < m && col < n) ? stream_load<NTL>(W + row + (int64_t)col * ldw) : 0.0;
    }
  };
  auto load = [&](int64_t t) {
    if (ntw) load_rows(std::true_type{}, t);
    else load_rows(std::false_type{}, t);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int c = 0; c < PER; ++c) lds[(buf * NP + ldc + (NT / 32) * c) * TP_LDW + ldr] = pre[c];
  };
  int64_t t = wg;
  int buf = 0;
  if (t < ntiles32) {
    load(t);
    store(0);
  }
  __syncthreads();
  for (; t < ntiles32; t += nwg) {
    const int64_t tn = t + nwg;
    if (tn < ntiles32) load(tn);
    const double* ws = lds + buf * NP * TP_LDW;
#pragma unroll 1
    for (int kk = 0; kk < 8; ++kk) {
      // fragment of column block c at K-step kk: lane l holds W[4 kk + l/16][16 c + l%16]
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        if (wave + NW * q < NBLK) {
          const double fa = ws[(16 * bi[q] + lr) * TP_LDW + 4 * kk + lq];
          const double fb = ws[(16 * bj[q] + lr) * TP_LDW + 4 * kk + lq];
          acc[q] = mfma_f64(fa, fb, acc[q]);
        }
      }
    }
    if (tn < ntiles32) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    if (wave + NW * q < NBLK) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = 16 * bi[q] + lq + 4 * r, gj = 16 * bj[q] + lr;
        Gpart[wg * NP * NP + gi + gj * NP] = acc[q][r];
      }
    }
  }
}

// Level 1 of the deterministic partial-sum reduction: lvl[y][e] = sum of
// part[b][e] over the contiguous chunk of workgroups b assigned to split y
// (in b order). Consecutive threads read consecutive e (coalesced).
__global__ void k_partial_sum(const double* __restrict__ part, int nparts, int64_t stride, int splits,
                              double* __restrict__ lvl, const int32_t* info, const ReduceJob* __restrict__ jobs,
                              const BatchItem* __restrict__ items) {
  int y = blockIdx.y;
  if (items) {  // batched: item = (problem, split index, splits of that problem)
    const BatchItem it = items[blockIdx.y];
    const ReduceJob j = jobs[it.prob];
    part = j.part, nparts = j.nparts, splits = j.splits, lvl = j.lvl, info = j.info, y = it.wg;
  }
  if (info_failed(info)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= stride) return;
  const int per = (nparts + splits - 1) / splits;
  const int b0 = y * per, b1 = (b0 + per < nparts) ? b0 + per : nparts;
  double acc = 0.0;
  #pragma unroll 16
  for (int b = b0; b < b1; ++b) acc += part[(int64_t)b * stride + e];
  lvl[(int64_t)y * stride + e] = acc;
}

// G[i + j*np] = sum_y lvl[y][i + j*np] for i <= j (mirrored), padded with the
// identity beyond n (so a padded Cholesky stays the identity there).
__global__ void k_gram_final(const double* __restrict__ lvl, int splits, int np, int64_t n, double* __restrict__ G,
                             const int32_t* info, const ReduceJob* __restrict__ jobs) {
  if (jobs) {  // batched: blockIdx.y = problem
    const ReduceJob j = jobs[blockIdx.y];
    lvl = j.lvl, splits = j.splits, G = j.out, info = j.info;
  }
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
    #pragma unroll 16
    for (int y = 0; y < splits; ++y) v += lvl[(int64_t)y * stride + e];
  }
  G[i + (int64_t)j * np] = v;
  G[j + (int64_t)i * np] = v;
}

int reduce_splits(int nparts) {
  int sp = nparts / 16;
  if (sp < 1) sp = 1;
  if (sp > 64) sp = 64;
  return sp;
}

hipError_t launch_partial_sum(const double* part, int nparts, int64_t stride, int splits, double* lvl,
                              const int32_t* info, hipStream_t st) {
  const int threads = 256;
  dim3 grid((unsigned)((stride + threads - 1) / threads), (unsigned)splits);
  hipLaunchKernelGGL(k_partial_sum, grid, dim3(threads), 0, st, part, nparts, stride, splits, lvl, info, nullptr,
                     nullptr);
  return hipGetLastError();
}

TallPlan plan_tall(int64_t m, int64_t n, int gx_hint) {
  TallPlan p{};
  p.np = pad_cols(n);
  p.fused_gram = p.np <= 64;
  p.tile_rows = p.fused_gram ? tm_tile(p.np) : TP_THREADS;
  p.ntiles = (m + p.tile_rows - 1) / p.tile_rows;
  // Gram passes: one round of resident workgroups for n <= 64 (two per CU on
  // 256 CUs: register bound), which also keeps the partials few; passes
  // without the Gram (lighter kernel, four per CU) use two rounds
  auto clampg = [&](int g) { return (int)(g > p.ntiles ? p.ntiles : (g < 1 ? 1 : g)); };
  // (n > 64: the Gram kernel keeps one workgroup of 8 waves per CU for n > 128,
  // two of 4 waves for n <= 128)
  p.gx = clampg(gx_hint > 0 ? gx_hint : (p.np == 64 ? 512 : p.np == 256 ? 256 : p.np == 128 ? 512 : 1024));
  p.gx_solve = clampg(gx_hint > 0 ? gx_hint : (p.fused_gram ? 2048 : 1024));
  const int gx = p.gx;
  // per-workgroup partials followed by the level-1 sums of the reduction
  p.part_bytes = ((size_t)gx + reduce_splits(gx)) * p.np * p.np * sizeof(double);
  return p;
}

template <int NP>
static hipError_t launch_tp(const TallPlan& p, const double* X, int64_t ldx, int64_t m, int64_t n, const double* Rp,
                            double* W, int64_t ldw, double* Gpart, const int32_t* info, hipStream_t st) {
  const bool trsm = Rp != nullptr, gram = Gpart != nullptr, write = W != nullptr;
  dim3 grid(gram ? p.gx : p.gx_solve), block(64 * tm_waves(NP <= 64 ? NP : 128));
  if (NP <= 64) {
#define TP_CASE(T, G, Wr)                                                                                          \
  if (trsm == T && gram == G && write == Wr) {                                                                     \
    hipLaunchKernelGGL((k_tall_mfma<(NP <= 64 ? NP : 64), T, G, Wr>), grid, block, 0, st, X, ldx, m, (int)n, Rp, W, \
                       ldw, Gpart, p.ntiles, info, nullptr, nullptr);                                               \
    return hipGetLastError();                                                                                       \
  }
    TP_CASE(true, true, true)
    TP_CASE(true, false, true)
    TP_CASE(false, true, false)
#undef TP_CASE
    return hipErrorInvalidValue;
  }
  // n > 64: blocked substitution on the matrix cores (no fused Gram), then
  // the Gram kernel over W (or X)
  if (trsm && NP == 256) {
    if (!write) return hipErrorInvalidValue;
    // split at column 128: W_1 = X_1 R_11^{-1}; C_2 = X_2 - W_1 R_12; W_2 = C_2 R_22^{-1}
    const int64_t nt = (m + tm_tile(128) - 1) / tm_tile(128);
    dim3 tgrid((unsigned)(p.gx_solve < nt ? p.gx_solve : nt));
    const int n2 = (int)n - 128;
    hipLaunchKernelGGL((k_tall_mfma<128, true, false, true, 256, 0>), tgrid, block, 0, st, X, ldx, m, 128, Rp, W, ldw,
                       nullptr, nt, info, nullptr, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr size_t glds = gemm_sub_lds<8>();
    e = hipFuncSetAttribute((const void*)k_tall_gemm_sub<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds);
    if (e != hipSuccess) return e;
    const int64_t ntg = (m + GS_TILE - 1) / GS_TILE;
    dim3 ggrid((unsigned)(ntg < 256 ? ntg : 256));
    hipLaunchKernelGGL(k_tall_gemm_sub<8>, ggrid, dim3(GS_THREADS), glds, st, X + 128 * ldx, ldx, m, n2, W, ldw,
                       Rp + 128, 256, W + 128 * ldw, ldw, ntg, info);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tall_mfma<128, true, false, true, 256, 128>), tgrid, block, 0, st, W + 128 * ldw, ldw, m, n2,
                       Rp + 128 * 256 + 128, W + 128 * ldw, ldw, nullptr, nt, info, nullptr, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else if (trsm) {
    if (!write) return hipErrorInvalidValue;
    const int64_t nt = (m + tm_tile(NP) - 1) / tm_tile(NP);
    dim3 tgrid((unsigned)(p.gx < nt ? p.gx : nt));
    hipLaunchKernelGGL((k_tall_mfma<(NP > 64 ? NP : 128), true, false, true>), tgrid, block, 0, st, X, ldx, m, (int)n,
                       Rp, W, ldw, nullptr, nt, info, nullptr, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else if (write) {
    return hipErrorInvalidValue;
  }
  if (gram) {
    const double* src = trsm ? W : X;
    const int64_t lds_ = trsm ? ldw : ldx;
    const int64_t nt32 = (m + 31) / 32;
    constexpr int NPG = NP > 64 ? NP : 128;
    constexpr size_t glds = gram_lds<NPG>();
    hipError_t e = hipFuncSetAttribute((const void*)k_gram_bal<NPG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)glds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gram_bal<NPG>), dim3(p.gx), dim3(64 * gram_waves<NPG>()), glds, st, src, lds_, m, (int)n,
                       Gpart, nt32, info, nullptr, nullptr);
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
  // level 1 writes into the tail of the partial buffer's own space is not
  // possible (it is still being read), so the plan reserves lvl after it
  const int64_t stride = (int64_t)p.np * p.np;
  const int splits = reduce_splits(p.gx);
  double* lvl = const_cast<double*>(Gpart) + (int64_t)p.gx * stride;
  hipError_t e = launch_partial_sum(Gpart, p.gx, stride, splits, lvl, info, st);
  if (e != hipSuccess) return e;
  const int threads = 256;
  hipLaunchKernelGGL(k_gram_final, dim3((unsigned)((stride + threads - 1) / threads)), dim3(threads), 0, st, lvl,
                     splits, p.np, n, G, info, nullptr);
  return hipGetLastError();
}

// ---- batched launches (one stage for many problems of the same n) ---------------
// items: one entry per workgroup (problem, its workgroup index and count);
// the same list drives the solve and, for n > 64, the separate Gram kernel,
// so the Gram partials of problem p are its nwg workgroups' sums.
template <int NP>
static hipError_t launch_tall_batch_np(int n, bool trsm, bool gram, bool write, const TallJob* jobs,
                                       const BatchItem* items, int nitems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  dim3 grid((unsigned)nitems), block(64 * tm_waves(NP <= 64 ? NP : 128));
  if (NP <= 64) {
    constexpr int NPS = NP <= 64 ? NP : 64;
    if (trsm && gram && write)
      hipLaunchKernelGGL((k_tall_mfma<NPS, true, true, true>), grid, block, 0, st, nullptr, 0, 0, n, nullptr, nullptr, 0,
                         nullptr, 0, nullptr, jobs, items);
    else if (trsm && !gram && write)
      hipLaunchKernelGGL((k_tall_mfma<NPS, true, false, true>), grid, block, 0, st, nullptr, 0, 0, n, nullptr, nullptr,
                         0, nullptr, 0, nullptr, jobs, items);
    else if (!trsm && gram && !write)
      hipLaunchKernelGGL((k_tall_mfma<NPS, false, true, false>), grid, block, 0, st, nullptr, 0, 0, n, nullptr, nullptr,
                         0, nullptr, 0, nullptr, jobs, items);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  constexpr int NPB = NP > 64 ? NP : 128;
  if (trsm) {
    if (!write) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tall_mfma<NPB, true, false, true>), grid, block, 0, st, nullptr, 0, 0, n, nullptr, nullptr, 0,
                       nullptr, 0, nullptr, jobs, items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (gram) {
    constexpr size_t glds = gram_lds<NPB>();
    hipError_t e = hipFuncSetAttribute((const void*)k_gram_bal<NPB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)glds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gram_bal<NPB>), dim3((unsigned)nitems), dim3(64 * gram_waves<NPB>()), glds, st, nullptr, 0,
                       0, n, nullptr, 0, nullptr, jobs, items);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_tall_batch(int np, int n, bool trsm, bool gram, bool write, const TallJob* jobs,
                             const BatchItem* items, int nitems, hipStream_t st) {
  switch (np) {
    case 16: return launch_tall_batch_np<16>(n, trsm, gram, write, jobs, items, nitems, st);
    case 32: return launch_tall_batch_np<32>(n, trsm, gram, write, jobs, items, nitems, st);
    case 64: return launch_tall_batch_np<64>(n, trsm, gram, write, jobs, items, nitems, st);
    case 128: return launch_tall_batch_np<128>(n, trsm, gram, write, jobs, items, nitems, st);
    case 256: return launch_tall_batch_np<256>(n, trsm, gram, write, jobs, items, nitems, st);
    default: return hipErrorInvalidValue;
  }
}

// Level-1 sums for many problems: items = (problem, split y, splits).
hipError_t launch_partial_sum_batch(int64_t stride, const ReduceJob* jobs, const BatchItem* items, int nitems,
                                    hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const int threads = 256;
  dim3 grid((unsigned)((stride + threads - 1) / threads), (unsigned)nitems);
  hipLaunchKernelGGL(k_partial_sum, grid, dim3(threads), 0, st, nullptr, 0, stride, 1, nullptr, nullptr, jobs, items);
  return hipGetLastError();
}

hipError_t launch_gram_final_batch(int np, int64_t n, const ReduceJob* jobs, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int threads = 256;
  const int64_t stride = (int64_t)np * np;
  dim3 grid((unsigned)((stride + threads - 1) / threads), (unsigned)count);
  hipLaunchKernelGGL(k_gram_final, grid, dim3(threads), 0, st, nullptr, 1, np, n, nullptr, nullptr, jobs);
  return hipGetLastError();
}

}  // namespace rclupp
