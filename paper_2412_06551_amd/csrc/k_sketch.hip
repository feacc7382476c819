// Sketch Y = S X with S = G / sqrt(s) generated on the fly (Algorithm 2 step 1;
// Algorithm 7 step 2 with X = M; Algorithm 6 step 1).
//
// One pass over the tall operand, one kernel for the three arithmetics:
//   FP64: v_mfma_f64_16x16x4_f64, G widened exactly from FP32;
//   FP32: v_mfma_f32_16x16x4_f32, X rounded to FP32 when staged;
//   BF16: v_mfma_f32_16x16x32_bf16, G and X (through FP32) rounded to BF16
//         (round to nearest even); FP32 accumulation inside a wave.
// Work split: every wave owns one 16-row M-block of sketch rows and all
// (padded) columns, so every entry of G is generated exactly once; a
// workgroup of NW waves covers 16 NW sketch rows, and the gy workgroups that
// cover all s rows share each tile of X. Workgroups walk 32-row tiles of X
// (tile c, c + gx, ... for row chunk c), staged in LDS (coalesced column reads,
// double-buffered; the next tile is loaded into registers during the current
// tile's products and converted when it is stored).
// Generation: lane l of an M-block holds sketch row i = l % 16 and the K
// slots of group g = l / 16. One normals4 call gives row i's entries for four
// consecutive tall rows, so the K index is laid out as runs of four rows per
// lane group: for the 16x16x4 forms, K-step ks of a 16-row super-step takes
// tall row 4g + ks in lane group g (one call per lane per super-step); for the
// 16x16x32 BF16 form, lane group g takes rows 8g .. 8g+7 of a 32-row K-step
// (two calls). B (the X tile) is read from LDS in the same K order.
// Launch: gx row chunks x gy sketch-row groups in a 1-D grid. When gx is a
// multiple of 8, workgroup b runs chunk 8 floor(floor(b/8) / gy) + b mod 8,
// sketch group floor(b/8) mod gy: workgroups are dealt to the eight XCDs in
// turn, so the gy workgroups of one chunk run on one XCD at about the same
// time and share its L2 for the tiles of X.
// Each workgroup writes its partial sum (fixed order over its tiles); a second
// kernel adds the partials in chunk order and scales by 1/sqrt(s), so the
// result is deterministic.
// KIND = 2: the SRHT (Section 3 lists the subsampled randomized Hadamard
// transform among the common sketches), S = sqrt(m'/s) R H D with m' the
// smallest power of two >= m: entry (i, j) is (-1)^popcount(r_i & j) d_j /
// sqrt(s). The same kernel forms Y = S X as a dense product: the signs d_j
// are applied to the rows of X as the tile is staged (exact), and the A
// operand is +-1 from the parity of r_i & j (exact in every precision), so the
// generation cost is one Philox call per staged row and a popcount per entry.
// d_j: Philox4x32-10, counter (floor(j/4) lo, hi, 0, 2), word j mod 4, -1 for
// odd words. r_i = f3(f2(f1(i))) on k = log2 m' bits: f1(x) = a1 x + b1, f2(x)
// = x xor (x >> ceil(k/2)), f3(x) = a2 x + b2 (mod 2^k, a1 and a2 odd: a
// bijection, so the sampled rows are distinct), (a1, b1, a2, b2) the words at
// counter (0, 0, 0, 3).
#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace rclupp {

constexpr int SK_TK = 32;  // tall rows per tile

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// LDS tile of the X operand: FP64 and FP32 as [row][col] with row stride NN + 1
// elements (the 16 columns of a B fragment on consecutive banks, the four lane
// groups' rows on different ones); BF16 as [col][row] with column stride
// TK + 8 (a lane's eight consecutive rows are one 16-byte read).
template <int P, int NN>
struct SkTile {
  static constexpr int ELT = P == 0 ? 8 : (P == 1 ? 4 : 2);
  static constexpr int LD = P == 2 ? SK_TK + 8 : NN + 1;
  static constexpr int BYTES = (P == 2 ? NN * LD : SK_TK * LD) * ELT;
};

// The FP32 and BF16 forms of eight waves are held to 128 VGPRs (four waves per
// SIMD: two workgroups per CU), so one workgroup's tile loads are in flight
// while the other computes (their short per-tile work could not hide the load
// latency with one workgroup per CU: 8.3 against 10.5 ms for BF16, 21.6
// against 23.4 ms for FP32 at 4,194,304 x 256, s = 1024).
template <int P, int NN, int NW, int KIND>
__global__ __launch_bounds__(64 * NW, (P != 0 && NW == 8) ? 4 : 1) void k_sketch(const double* __restrict__ X, int64_t m, int n, int64_t ld,
                                                     int64_t ntiles, uint64_t seed, double* __restrict__ Ypart,
                                                     int64_t s_pad, int64_t n_pad, int gy, int xcd_map,
                                                     const int32_t* info, const SketchJob* __restrict__ jobs,
                                                     const BatchItem* __restrict__ items) {
  int64_t chunk, nchunks;
  int sg;
  if (items) {  // batched launch: this workgroup's problem and its row chunk in it
    const BatchItem it = items[blockIdx.x];
    const SketchJob j = jobs[it.prob];
    X = j.X, m = j.m, ld = j.ld, ntiles = j.ntiles, seed = j.seed, Ypart = j.Ypart, info = j.info;
    chunk = it.wg, nchunks = it.nwg, sg = (int)blockIdx.y;
  } else if (xcd_map) {
    const int b = (int)blockIdx.x, k = b >> 3;
    chunk = (int64_t)(k / gy) * 8 + (b & 7);
    sg = k % gy;
    nchunks = gridDim.x / gy;
  } else {
    chunk = blockIdx.x / gy;
    sg = (int)(blockIdx.x % gy);
    nchunks = gridDim.x / gy;
  }
  if (info_failed(info)) return;
  using T = SkTile<P, NN>;
  constexpr int TK = SK_TK, LD = T::LD, NB = NN / 16;
  constexpr int CG = 64 * NW / TK;  // loader column groups
  constexpr int CPT = NN / CG;      // tile columns loaded per thread
  static_assert(CPT >= 1 && NN % CG == 0, "tile columns must cover the loader groups");
  __shared__ __align__(16) unsigned char lds[2 * T::BYTES];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = tid % TK, lc = tid / TK;  // loader: row, first column
  const int ai = lane & 15, ag = lane >> 4;
  const uint32_t srow = (uint32_t)((sg * NW + wave) * 16 + ai);  // this lane's sketch row (A operand)
  // SRHT: the Hadamard row this sketch row samples (rows at or past s are
  // padding and take any row)
  uint32_t hrow = 0;
  if constexpr (KIND == 2) {
    int k = 0;
    while (((int64_t)1 << k) < m) ++k;
    if (k > 0) {
      const philox_out w = philox4x32_10(0u, 0u, 0u, 3u, (uint32_t)seed, (uint32_t)(seed >> 32));
      const uint32_t mask = (uint32_t)((((uint64_t)1) << k) - 1);
      uint32_t x = srow & mask;
      x = ((w.w0 | 1u) * x + w.w1) & mask;
      x ^= x >> ((k + 1) / 2);
      hrow = ((w.w2 | 1u) * x + w.w3) & mask;
    }
  }

  using acc_t = typename std::conditional<P == 0, f64x4, f32x4>::type;
  acc_t acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = acc_t{0, 0, 0, 0};

  double pre[CPT];
  double dpre = 1.0;  // SRHT: the sign d_j of the prefetched row (applied when it is staged)
  auto load_tile = [&](int64_t t) {
    const int64_t row = t * TK + lr;
    if constexpr (P == 0) {
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int col = lc + CG * c;
        pre[c] = (row < m && col < n) ? X[row + (int64_t)col * ld] : 0.0;
      }
    } else {
      // a wave-uniform column base plus a 32-bit per-lane offset (row + lc ld <
      // 2^32: m + 16 ld < 2^32 for the sizes the entry points accept), which
      // keeps no 64-bit address per load in registers
      const uint32_t voff = (uint32_t)(row + (int64_t)lc * ld);
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int col = lc + CG * c;
        const double* cb = X + (int64_t)(CG * c) * ld;
        pre[c] = (row < m && col < n) ? cb[voff] : 0.0;
      }
    }
    if constexpr (KIND == 2) {
      // (the loads stay in flight: the sign multiplies them only in store_tile)
      const uint64_t q = (uint64_t)row >> 2;
      const philox_out w = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), 0u, 2u, (uint32_t)seed, (uint32_t)(seed >> 32));
      const uint32_t wt = (row & 2) ? ((row & 1) ? w.w3 : w.w2) : ((row & 1) ? w.w1 : w.w0);
      dpre = (wt & 1u) ? -1.0 : 1.0;
    }
  };
  auto store_tile = [&](int buf) {
    unsigned char* base = lds + buf * T::BYTES;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = lc + CG * c;
      const double v = KIND == 2 ? dpre * pre[c] : pre[c];  // (a sign change: exact)
      if constexpr (P == 0) {
        ((double*)base)[lr * LD + col] = v;
      } else if constexpr (P == 1) {
        ((float*)base)[lr * LD + col] = (float)v;
      } else {
        ((unsigned short*)base)[col * LD + lr] = (unsigned short)f32_to_bf16_rne((float)v);
      }
    }
  };

  int64_t t = chunk;
  int buf = 0;
  if (t < ntiles) {
    load_tile(t);
    store_tile(0);
  }
  f32x4 zc[TK / 16];  // normals of the current tile (FP64 and FP32 Gaussian forms)
  if constexpr (P != 2 && KIND == 0) {
#pragma unroll
    for (int ss = 0; ss < TK / 16; ++ss) zc[ss] = normals4(seed, (uint64_t)(t * TK + 16 * ss) / 4 + ag, srow);
  }
  __syncthreads();
  for (; t < ntiles; t += nchunks) {
    const int64_t tn = t + nchunks;
    if (tn < ntiles) load_tile(tn);
    const unsigned char* base = lds + buf * T::BYTES;
    if constexpr (P == 2) {
      const unsigned short* xs = (const unsigned short*)base;
      // one K-step of 32 rows: lane group g holds rows 8g .. 8g+7
      uint4 a4;
      if constexpr (KIND == 2) {
        // +-1 in BF16 (0x3F80 / 0xBF80) from the parity of r_i & j
        uint32_t hv[4];
        const uint32_t j0 = (uint32_t)(t * TK) + 8 * ag;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t lo = 0x3F80u | ((__builtin_popcount(hrow & (j0 + 2 * e)) & 1u) << 15);
          const uint32_t hi = 0x3F80u | ((__builtin_popcount(hrow & (j0 + 2 * e + 1)) & 1u) << 15);
          hv[e] = lo | (hi << 16);
        }
        a4 = uint4{hv[0], hv[1], hv[2], hv[3]};
      } else {
        const uint64_t q0 = (uint64_t)(t * TK) / 4 + 2 * ag;
        const f32x4 z0 = normals4(seed, q0, srow), z1 = normals4(seed, q0 + 1, srow);
        a4 = uint4{f32_to_bf16_rne(z0[0]) | (f32_to_bf16_rne(z0[1]) << 16),
                   f32_to_bf16_rne(z0[2]) | (f32_to_bf16_rne(z0[3]) << 16),
                   f32_to_bf16_rne(z1[0]) | (f32_to_bf16_rne(z1[1]) << 16),
                   f32_to_bf16_rne(z1[2]) | (f32_to_bf16_rne(z1[3]) << 16)};
      }
      const bf16x8 A = __builtin_bit_cast(bf16x8, a4);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const uint4 q = *(const uint4*)(xs + (16 * nb + ai) * LD + 8 * ag);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, q), acc[nb], 0, 0, 0);
      }
    } else {
      // the next tile's normals are generated while this tile's products run
      // (their vector-ALU work overlaps the matrix instructions; for tn past
      // the end they are computed and not used)
      f32x4 zn[TK / 16];
      if constexpr (KIND == 0) {
#pragma unroll
        for (int ss = 0; ss < TK / 16; ++ss) zn[ss] = normals4(seed, (uint64_t)(tn * TK + 16 * ss) / 4 + ag, srow);
      }
#pragma unroll
      for (int ss = 0; ss < TK / 16; ++ss) {
        // super-step of 16 rows: K-step ks takes row 16 ss + 4g + ks in lane group g
        f32x4 z;
        if constexpr (KIND == 2) {
          const uint32_t j0 = (uint32_t)(t * TK + 16 * ss) + 4 * ag;
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) z[ks] = (__builtin_popcount(hrow & (j0 + ks)) & 1) ? -1.0f : 1.0f;
        } else {
          z = zc[ss];
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int r = 16 * ss + 4 * ag + ks;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            if constexpr (P == 0) {
              const double bv = ((const double*)base)[r * LD + 16 * nb + ai];
              acc[nb] = mfma_f64((double)z[ks], bv, acc[nb]);
            } else {
              const float bv = ((const float*)base)[r * LD + 16 * nb + ai];
              acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(z[ks], bv, acc[nb], 0, 0, 0);
            }
          }
        }
      }
      if constexpr (P == 1 && KIND == 0) {
        // FP32: interleave explicitly, one product, its B read and two
        // vector-ALU instructions at a time (measured: 9 % faster; the FP64
        // form is fastest as the compiler schedules it)
#pragma unroll
        for (int i = 0; i < TK / 4 * NB; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
        }
      }
      if constexpr (KIND == 0) {
#pragma unroll
        for (int ss = 0; ss < TK / 16; ++ss) zc[ss] = zn[ss];
      }
    }
    if (tn < ntiles) store_tile(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // the wave's 16 x NN partial (FP64 output layout: row l/16 + 4r; FP32: 4(l/16) + r)
  double* out = Ypart + chunk * s_pad * n_pad;
  const int64_t row0 = (int64_t)(sg * NW + wave) * 16;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int crow = (P == 0) ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
      const int64_t col = 16 * nb + (lane & 15);
      out[row0 + crow + col * s_pad] = (double)acc[nb][r];
    }
}

// ---------------------------------------------------------------------------
// CountSketch (Section 3 lists it among the common sketches): column j of S
// has one entry sigma_j = +-1, in row h_j, so Y = S X adds +-row j of X into
// row h_j of Y (no scaling). h_j and sigma_j come from Philox4x32-10 with
// counter (q lo, q hi, 0, 1), q = floor(j/4), key (seed lo, seed hi): word t
// belongs to tall row 4q+t, h = floor(w s / 2^32), sigma = -1 for odd w.
// The pass is HBM-bound (X read once, one add per entry). A workgroup owns a
// row chunk and a slice of NC columns, keeps its s_pad x NC partial of Y in LDS
// and walks tiles of TK = 4096 / NC rows of its slice. Every (row of Y,
// column) sum has one owner, which adds its terms in increasing row order, so
// the result is deterministic without atomics: thread (c, r) owns column c and
// the rows h of Y with h mod R = r (R = 256 / NC). Per tile the rows are
// listed by residue in increasing order (a counting sort: per 64-row chunk a
// ballot per residue gives the counts and each row's rank, one scan the
// offsets), then every thread walks its residue's list.
// The per-chunk partials go through the Gaussian sketch's fixed-order
// reduction with scale 1.
// ---------------------------------------------------------------------------
constexpr int CS_THREADS = 256;
constexpr int CS_TILE = 4096;  // entries of X per tile (TK x NC)

__device__ __forceinline__ void countsketch_hash4(uint64_t seed, uint64_t q, uint32_t s, int h[4], double sg[4]) {
  const philox_out w = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), 0u, 1u, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint32_t ws[4] = {w.w0, w.w1, w.w2, w.w3};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    h[t] = (int)(((uint64_t)ws[t] * (uint64_t)s) >> 32);
    sg[t] = (ws[t] & 1u) ? -1.0 : 1.0;
  }
}

constexpr int cs_tk(int nc) { return CS_TILE / nc; }

size_t countsketch_lds_bytes(int64_t s_pad, int nc) {
  const int R = CS_THREADS / nc, TK = cs_tk(nc), NCH = TK / 64;
  return (size_t)s_pad * nc * 8 + (size_t)TK * (nc + 1) * 8 + (size_t)TK * 8 + (size_t)TK * 4 * 2 +
         (size_t)R * NCH * 4 * 2;
}

template <int NC>
__global__ __launch_bounds__(CS_THREADS) void k_countsketch(const double* __restrict__ X, int64_t m, int n, int64_t ld,
                                                            int64_t ntiles, uint64_t seed, int s,
                                                            double* __restrict__ Ypart, int64_t s_pad, int64_t n_pad,
                                                            const int32_t* info) {
  if (info_failed(info)) return;
  constexpr int R = CS_THREADS / NC, TK = cs_tk(NC), LDT = NC + 1, NCH = TK / 64;
  constexpr int EPT = CS_TILE / CS_THREADS;  // tile entries loaded per thread
  constexpr int CPW = (NCH + 3) / 4;         // 64-row chunks listed per wave
  static_assert(TK % 64 == 0 && R * NC == CS_THREADS, "tile shape");
  extern __shared__ __align__(16) unsigned char cs_smem[];
  double* Y = (double*)cs_smem;         // [s_pad][NC]
  double* xt = Y + s_pad * NC;          // [TK][LDT]
  double* sgn = xt + TK * LDT;          // [TK]
  int* hb = (int*)(sgn + TK);           // [TK] row of Y of each tile row
  int* lst = hb + TK;                   // [TK] tile rows listed by residue
  int* ccnt = lst + TK;                 // [R][NCH] rows of residue q in chunk b
  int* coff = ccnt + R * NCH;           // [R][NCH] their first list position
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t chunk = blockIdx.x, nchunks = gridDim.x;
  const int col0 = (int)blockIdx.y * NC;
  const int c = tid % NC, r = tid / NC;
  for (int64_t e = tid; e < s_pad * NC; e += CS_THREADS) Y[e] = 0.0;
  double pre[EPT];
  auto load = [&](int64_t t) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = tid + CS_THREADS * k, rr = e % TK, cc = e / TK;
      const int64_t row = t * TK + rr;
      const int col = col0 + cc;
      pre[k] = (row < m && col < n) ? X[row + (int64_t)col * ld] : 0.0;
    }
  };
  int64_t t = chunk;
  if (t < ntiles) load(t);
  for (; t < ntiles; t += nchunks) {
    __syncthreads();  // the previous tile's entries and lists are consumed
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = tid + CS_THREADS * k;
      xt[(e % TK) * LDT + e / TK] = pre[k];
    }
    for (int g = tid; g < TK / 4; g += CS_THREADS) {
      int h4[4];
      double s4[4];
      countsketch_hash4(seed, (uint64_t)(t * TK) / 4 + g, (uint32_t)s, h4, s4);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        hb[4 * g + u] = h4[u];
        sgn[4 * g + u] = s4[u];
      }
    }
    __syncthreads();
    // counting sort by residue: counts and ranks per 64-row chunk
    int rank[CPW];
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      const int b = wave + 4 * k;
      rank[k] = 0;
      if (b < NCH) {
        const int res = hb[64 * b + lane] & (R - 1);
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const uint64_t mask = __ballot(res == q);
          if (res == q) rank[k] = __popcll(mask & ((1ull << lane) - 1ull));
          if (lane == 0) ccnt[q * NCH + b] = __popcll(mask);
        }
      }
    }
    __syncthreads();
    if (wave == 0) {  // exclusive scan of the counts in (residue, chunk) order
      constexpr int PER = (R * NCH + 63) / 64;
      int v[PER], sum = 0;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = lane * PER + i;
        v[i] = e < R * NCH ? ccnt[e] : 0;
        sum += v[i];
      }
      int incl = sum;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
      }
      int run = incl - sum;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = lane * PER + i;
        if (e < R * NCH) coff[e] = run;
        run += v[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      const int b = wave + 4 * k;
      if (b < NCH) {
        const int row = 64 * b + lane, res = hb[row] & (R - 1);
        lst[coff[res * NCH + b] + rank[k]] = row;
      }
    }
    if (t + nchunks < ntiles) load(t + nchunks);  // in flight during the adds
    __syncthreads();
    const int k0 = coff[r * NCH], k1 = (r + 1 < R) ? coff[(r + 1) * NCH] : TK;
    for (int k = k0; k < k1; ++k) {
      const int jj = lst[k];
      double* yp = Y + hb[jj] * NC + c;
      *yp = __builtin_fma(sgn[jj], xt[jj * LDT + c], *yp);  // +-x exactly, then one rounding
    }
  }
  __syncthreads();
  double* out = Ypart + chunk * s_pad * n_pad + (int64_t)col0 * s_pad;
  for (int64_t e = tid; e < s_pad * NC; e += CS_THREADS) {
    const int64_t i = e % s_pad, cc = e / s_pad;
    out[i + cc * s_pad] = Y[i * NC + cc];
  }
}

// Y[i + j*s] = scale * sum_y lvl[y][i + j*s_pad] (the level-1 sums of the
// per-workgroup partials, added in split order).
__global__ void k_sketch_final(const double* __restrict__ lvl, int splits, int64_t s, int64_t n, int64_t s_pad,
                               int64_t n_pad, double scale, double* __restrict__ Y, const int32_t* info,
                               const ReduceJob* __restrict__ jobs) {
  if (jobs) {  // batched: blockIdx.y = problem
    const ReduceJob j = jobs[blockIdx.y];
    lvl = j.lvl, splits = j.splits, Y = j.out, info = j.info;
  }
  if (info_failed(info)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s * n) return;
  const int64_t i = e % s, j = e / s;
  const double* p = lvl + i + j * s_pad;
  const int64_t stride = s_pad * n_pad;
  double acc = 0.0;
  #pragma unroll 16
  for (int y = 0; y < splits; ++y) acc += p[(int64_t)y * stride];
  Y[i + j * s] = acc * scale;
}

// G[i + c*s] = z(seed, i, j0 + c): one thread per (sketch row, group of four
// tall rows).
__global__ void k_omega(uint64_t seed, int64_t s, int64_t j0, int64_t cols, float* __restrict__ G) {
  const int64_t q_lo = j0 / 4, q_hi = (j0 + cols - 1) / 4;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s * (q_hi - q_lo + 1)) return;
  const int64_t i = e % s, q = q_lo + e / s;
  const f32x4 z = normals4(seed, (uint64_t)q, (uint32_t)i);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t c = 4 * q + u - j0;
    if (c >= 0 && c < cols) G[i + c * s] = z[u];
  }
}

__global__ void k_philox(const uint32_t* __restrict__ ctr, int64_t count, uint32_t k0, uint32_t k1,
                         uint32_t* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const philox_out w = philox4x32_10(ctr[4 * e], ctr[4 * e + 1], ctr[4 * e + 2], ctr[4 * e + 3], k0, k1);
  out[4 * e] = w.w0;
  out[4 * e + 1] = w.w1;
  out[4 * e + 2] = w.w2;
  out[4 * e + 3] = w.w3;
}

int64_t pad_sketch_rows(int64_t s) { return (s + 63) / 64 * 64; }

SketchPlan plan_sketch(int64_t m, int64_t n, int64_t s, int prec, int gx_hint) {
  SketchPlan p{};
  p.nn = pad_cols(n);  // one column group: every G entry is generated once
  p.gz = 1;
  p.n_pad = p.nn;
  p.s_pad = pad_sketch_rows(s);
  p.sm = 16;
  p.nw = (p.s_pad % 128 == 0) ? 8 : 4;  // s_pad is a multiple of 64
  p.wm = true;
  p.gy = (int)(p.s_pad / (16 * p.nw));
  p.ntiles = (m + SK_TK - 1) / SK_TK;
  (void)prec;
  // about 1024 workgroups in all (eight waves each: two per SIMD), gx a
  // multiple of 8 for the XCD-aware order
  int gx = gx_hint > 0 ? (gx_hint + p.gy - 1) / p.gy : (1024 + p.gy - 1) / p.gy;
  if (gx_hint <= 0 && gx > 8) gx = (gx + 7) / 8 * 8;
  if (gx < 1) gx = 1;
  if (gx > p.ntiles) gx = (int)p.ntiles;
  p.gx = gx;
  // per-workgroup partials followed by the level-1 sums of the reduction
  p.part_bytes = ((size_t)p.gx + reduce_splits(p.gx)) * (size_t)p.s_pad * (size_t)p.n_pad * sizeof(double);
  return p;
}

template <int P, int NN, int NW, int KIND>
static hipError_t launch_sk3(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld, uint64_t seed,
                             double* Ypart, const int32_t* info, const SketchJob* jobs, const BatchItem* items,
                             int nitems, hipStream_t st) {
  dim3 grid, block(64 * NW);
  int xcd = 0;
  if (items) {
    grid = dim3((unsigned)nitems, (unsigned)p.gy);
  } else {
    grid = dim3((unsigned)(p.gx * p.gy));
    xcd = (p.gx % 8 == 0) ? 1 : 0;
  }
  hipLaunchKernelGGL((k_sketch<P, NN, NW, KIND>), grid, block, 0, st, X, m, (int)n, ld, p.ntiles, seed, Ypart, p.s_pad,
                     p.n_pad, p.gy, xcd, info, jobs, items);
  return hipGetLastError();
}

template <int NN, int NW>
static hipError_t launch_sk2(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld, uint64_t seed,
                             int prec, double* Ypart, const int32_t* info, const SketchJob* jobs,
                             const BatchItem* items, int nitems, hipStream_t st) {
  if (p.kind == 2) {
    if (prec == 0) return launch_sk3<0, NN, NW, 2>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
    if (prec == 1) return launch_sk3<1, NN, NW, 2>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
    return launch_sk3<2, NN, NW, 2>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
  }
  if (prec == 0) return launch_sk3<0, NN, NW, 0>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
  if (prec == 1) return launch_sk3<1, NN, NW, 0>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
  return launch_sk3<2, NN, NW, 0>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
}

static hipError_t sketch_dispatch(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld,
                                  uint64_t seed, int prec, double* Ypart, const int32_t* info, const SketchJob* jobs,
                                  const BatchItem* items, int nitems, hipStream_t st) {
  if (prec < 0 || prec > 2 || p.gz != 1 || n > p.nn || (p.kind != 0 && p.kind != 2)) return hipErrorInvalidValue;
#define SK_CASE(NNV, NWV)           \
  if (p.nn == NNV && p.nw == NWV) \
    return launch_sk2<NNV, NWV>(p, X, m, n, ld, seed, prec, Ypart, info, jobs, items, nitems, st);
  SK_CASE(16, 4)
  SK_CASE(16, 8)
  SK_CASE(32, 4)
  SK_CASE(32, 8)
  SK_CASE(64, 4)
  SK_CASE(64, 8)
  SK_CASE(128, 4)
  SK_CASE(128, 8)
  SK_CASE(256, 4)
  SK_CASE(256, 8)
#undef SK_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_sketch_partials(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld, uint64_t seed,
                                  int prec, double* Ypart, const int32_t* info, hipStream_t st) {
  if (p.gx < 1 || p.ntiles < 1) return hipErrorInvalidValue;
  return sketch_dispatch(p, X, m, n, ld, seed, prec, Ypart, info, nullptr, nullptr, 0, st);
}

// Batched: `p` supplies the shape (sm, nn, gy, gz, s_pad, n_pad) shared by the
// problems; items/jobs the per-problem row chunks.
hipError_t launch_sketch_batch(const SketchPlan& p, int64_t n, int prec, const SketchJob* jobs, const BatchItem* items,
                               int nitems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  return sketch_dispatch(p, nullptr, 0, n, 0, 0, prec, nullptr, nullptr, jobs, items, nitems, st);
}

hipError_t launch_sketch_final_batch(const SketchPlan& p, int64_t s, int64_t n, double scale, const ReduceJob* jobs,
                                     int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int threads = 256;
  dim3 grid((unsigned)((s * n + threads - 1) / threads), (unsigned)count);
  hipLaunchKernelGGL(k_sketch_final, grid, dim3(threads), 0, st, nullptr, 1, s, n, p.s_pad, p.n_pad, scale, nullptr,
                     nullptr, jobs);
  return hipGetLastError();
}

hipError_t launch_sketch_reduce(const SketchPlan& p, const double* Ypart, int64_t s, int64_t n, double scale, double* Y,
                                const int32_t* info, hipStream_t st) {
  const int64_t stride = p.s_pad * p.n_pad;
  const int splits = reduce_splits(p.gx);
  double* lvl = const_cast<double*>(Ypart) + (int64_t)p.gx * stride;
  hipError_t e = launch_partial_sum(Ypart, p.gx, stride, splits, lvl, info, st);
  if (e != hipSuccess) return e;
  const int64_t total = s * n;
  const int threads = 256;
  const int64_t blocks = (total + threads - 1) / threads;
  hipLaunchKernelGGL(k_sketch_final, dim3((unsigned)blocks), dim3(threads), 0, st, lvl, splits, s, n, p.s_pad,
                     p.n_pad, scale, Y, info, nullptr);
  return hipGetLastError();
}

hipError_t launch_omega(uint64_t seed, int64_t s, int64_t j0, int64_t cols, float* G, hipStream_t st) {
  if (cols <= 0 || s <= 0) return hipSuccess;
  const int64_t total = s * ((j0 + cols - 1) / 4 - j0 / 4 + 1);
  const int threads = 256;
  hipLaunchKernelGGL(k_omega, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, st, seed, s, j0,
                     cols, G);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int threads = 256;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)((count + threads - 1) / threads)), dim3(threads), 0, st, ctr, count,
                     k0, k1, out);
  return hipGetLastError();
}

SketchPlan plan_countsketch(int64_t m, int64_t n, int64_t s, int gx_hint) {
  SketchPlan p{};
  p.kind = 1;
  p.s_pad = pad_sketch_rows(s);
  p.sm = 0;
  p.nw = 4;
  p.wm = false;
  p.gy = 1;
  const int n16 = pad_cols(n);
  // the widest column slice whose LDS (partial of Y, tile, lists) leaves room
  // for two workgroups per CU, else for one (160 KB)
  int nc = 0;
  for (int cand = 64; cand >= 8 && nc == 0; cand /= 2)
    if (cand <= n16 && countsketch_lds_bytes(p.s_pad, cand) <= 80 * 1024) nc = cand;
  for (int cand = 64; cand >= 8 && nc == 0; cand /= 2)
    if (cand <= n16 && countsketch_lds_bytes(p.s_pad, cand) <= 160 * 1024) nc = cand;
  if (nc == 0) return p;  // nn = 0: unsupported (s above 1792)
  p.nn = nc;
  p.gz = (int)((n + nc - 1) / nc);
  p.n_pad = (int64_t)p.gz * nc;
  p.ntiles = (m + cs_tk(nc) - 1) / cs_tk(nc);
  // about 2048 workgroups, with the partials kept below a sixteenth of X
  int64_t gx = gx_hint > 0 ? gx_hint : (2048 + p.gz - 1) / p.gz;
  const int64_t cap = (m * n) / (16 * p.s_pad * p.n_pad);
  if (gx_hint <= 0 && gx > cap) gx = cap > 8 ? cap : 8;
  if (gx > p.ntiles) gx = p.ntiles;
  if (gx < 1) gx = 1;
  p.gx = (int)gx;
  p.part_bytes = ((size_t)p.gx + reduce_splits(p.gx)) * (size_t)p.s_pad * (size_t)p.n_pad * sizeof(double);
  return p;
}

template <int NC>
static hipError_t launch_cs(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld, int64_t s,
                            uint64_t seed, double* Ypart, const int32_t* info, hipStream_t st) {
  const size_t lds = countsketch_lds_bytes(p.s_pad, NC);
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_countsketch<NC>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_countsketch<NC>, dim3((unsigned)p.gx, (unsigned)p.gz), dim3(CS_THREADS), lds, st, X, m,
                     (int)n, ld, p.ntiles, seed, (int)s, Ypart, p.s_pad, p.n_pad, info);
  return hipGetLastError();
}

hipError_t launch_countsketch_partials(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld,
                                       int64_t s, uint64_t seed, double* Ypart, const int32_t* info, hipStream_t st) {
  if (p.kind != 1 || p.gx < 1 || p.ntiles < 1 || (int64_t)p.gz * p.nn < n || s > p.s_pad) return hipErrorInvalidValue;
  switch (p.nn) {
    case 8: return launch_cs<8>(p, X, m, n, ld, s, seed, Ypart, info, st);
    case 16: return launch_cs<16>(p, X, m, n, ld, s, seed, Ypart, info, st);
    case 32: return launch_cs<32>(p, X, m, n, ld, s, seed, Ypart, info, st);
    case 64: return launch_cs<64>(p, X, m, n, ld, s, seed, Ypart, info, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rclupp
