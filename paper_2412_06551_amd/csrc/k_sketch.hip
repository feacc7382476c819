// Sketch Y = S X with S = G / sqrt(s) generated on the fly (Algorithm 2 step 1;
// Algorithm 7 step 2 with X = M; Algorithm 6 step 1).
//
// One pass over the tall operand. A workgroup owns a group of SM sketch rows
// and NN columns and walks 64-row tiles of X (tile t, t + gridDim.x, ...): the
// tile is staged in LDS (coalesced column reads, double-buffered), each of the
// four waves takes 16 of its rows as four K-steps of v_mfma_f64_16x16x4_f64,
// and the A operand (G) is produced in registers: lane l of a K-step holds the
// G entry of tall row (4 ks + l/16) and slot row (l % 16) of every 16-row
// M-block. Slot rows are mapped to sketch rows so that one Philox call of a
// lane feeds four M-blocks of that same lane:
//   M-block mb = 4a + u, slot i = 4c + t  ->  sketch row 64a + 16c + 4t + u,
// i.e. group q = 16a + 4c + t and output u of Philox(j, q). Every G entry is
// therefore generated exactly once per (workgroup column group).
// Two ways to share a workgroup's tile among its four waves:
//   WM = false: the waves take 16 rows of the tile each and own the same SM
//     sketch rows (summed over the waves at the end); one workgroup column
//     covers SM sketch rows.
//   WM = true (many sketch rows, s >= 4 SM): each wave owns its own SM sketch
//     rows and walks all rows of the tile, so one workgroup covers 4 SM sketch
//     rows and X is read by 4 times fewer workgroup groups.
// Each workgroup writes its partial sum (fixed order over its tiles and
// waves); a second kernel adds the partials in workgroup order and scales by
// 1/sqrt(s), so the result is deterministic.
#include "device_common.hpp"
#include "launch.hpp"

namespace rclupp {

constexpr int SK_TK = 64;  // tall rows per tile
constexpr int SK_THREADS = 256;

template <int SM, int NN, int TK = SK_TK, bool WM = false>
struct SketchLds {
  static constexpr int LDX = NN + 1;
  static constexpr int TILE = TK * LDX;
  static constexpr int RED = WM ? 0 : SM * NN;
  static constexpr int SIZE = (2 * TILE > RED) ? 2 * TILE : RED;
};

// NW waves per workgroup: 4, or 2 with wave-owned rows and 32-row tiles (a
// workgroup then covers 2 SM sketch rows with half the registers and a
// quarter of the LDS, so four workgroups and two waves per SIMD share a CU)
constexpr int sketch_f64_tk(int nw) { return nw == 2 ? 32 : SK_TK; }
template <int SM, int NN, bool WM, int NW>
__global__ __launch_bounds__(64 * NW) void k_sketch_f64(const double* __restrict__ X, int64_t m, int n, int64_t ld,
                                                           int64_t ntiles, uint64_t seed, double* __restrict__ Ypart,
                                                           int64_t s_pad, int64_t n_pad, const int32_t* info,
                                                           const SketchJob* __restrict__ jobs,
                                                           const BatchItem* __restrict__ items) {
  int64_t wg = blockIdx.x, nwg = gridDim.x;
  if (items) {  // batched launch: this workgroup's problem and its place in it
    const BatchItem it = items[blockIdx.x];
    const SketchJob j = jobs[it.prob];
    X = j.X, m = j.m, ld = j.ld, ntiles = j.ntiles, seed = j.seed, Ypart = j.Ypart, info = j.info;
    wg = it.wg, nwg = it.nwg;
  }
  if (info_failed(info)) return;
  constexpr int TK = sketch_f64_tk(NW);
  using L = SketchLds<SM, NN, TK, WM>;
  constexpr int MB = SM / 16, NB = NN / 16, LDX = L::LDX, TILE = L::TILE;
  static_assert(WM || NW == 4, "the row-split form uses four waves");
  constexpr int CG = 64 * NW / TK;  // loader column groups
  constexpr int CPT = NN / CG;      // tile columns loaded per thread
  __shared__ double lds[L::SIZE];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sg = blockIdx.y, col0 = blockIdx.z * NN;
  const int lr = tid % TK, lc0 = (tid / TK) * CPT;  // loader: row, first column

  f64x4 acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

  double pre[CPT];
  auto load_tile = [&](int64_t t) {
    const int64_t row = t * TK + lr;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = col0 + lc0 + c;
      pre[c] = (row < m && col < n) ? X[row + (int64_t)col * ld] : 0.0;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) lds[buf * TILE + lr * LDX + lc0 + c] = pre[c];
  };

  // A-operand slot of this lane: i = lane % 16 = 4c + t, K row = lane / 16
  const int ai = lane & 15, ak = lane >> 4;
  const int grp = WM ? NW * sg + wave : sg;  // this wave's group of SM sketch rows
  const uint32_t qbase = (uint32_t)((grp * SM) / 4 + 4 * (ai >> 2) + (ai & 3));

  int64_t t = wg;
  int buf = 0;
  if (t < ntiles) {
    load_tile(t);
    store_tile(0);
  }
  __syncthreads();
  for (; t < ntiles; t += nwg) {
    const int64_t tn = t + nwg;
    if (tn < ntiles) load_tile(tn);
    const double* xs = lds + buf * TILE;
#pragma unroll 1
    for (int ks = 0; ks < (WM ? TK / 4 : 4); ++ks) {
      const int rloc = (WM ? 0 : 16 * wave) + 4 * ks + ak;
      const int64_t j = t * TK + rloc;
      double b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = xs[rloc * LDX + 16 * nb + ai];
#pragma unroll
      for (int a = 0; a < SM / 64; ++a) {
        f32x4 z = {0.f, 0.f, 0.f, 0.f};
        if (j < m) z = normals4(seed, (uint64_t)j, qbase + 16u * (uint32_t)a);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double av = (double)z[u];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[4 * a + u][nb] = mfma_f64(av, b[nb], acc[4 * a + u][nb]);
        }
      }
    }
    if (tn < ntiles) store_tile(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  if (WM) {  // each wave owns its rows: store them
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t srow = (int64_t)grp * SM + 64 * (a >> 2) + 16 * r + 4 * (lane >> 4) + (a & 3);
          const int64_t col = col0 + 16 * nb + (lane & 15);
          Ypart[wg * s_pad * n_pad + srow + col * s_pad] = acc[a][nb][r];
        }
    return;
  }
  // Sum the four waves' partials in wave order through LDS, then store.
  double* red = lds;
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = ((a * NB + nb) * 4 + r) * 64 + lane;
            const double v = (w == 0) ? acc[a][nb][r] : red[idx] + acc[a][nb][r];
            if (w < 3) {
              red[idx] = v;
            } else {
              // slot row l/16 + 4r of M-block a -> sketch row
              const int64_t srow = (int64_t)sg * SM + 64 * (a >> 2) + 16 * r + 4 * (lane >> 4) + (a & 3);
              const int64_t col = col0 + 16 * nb + (lane & 15);
              Ypart[wg * s_pad * n_pad + srow + col * s_pad] = v;
            }
          }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Mixed-precision sketch: the same walk with the products on the FP32 or BF16
// matrix cores and FP32 accumulation inside a wave; the four waves' partials
// are added in FP64 and the cross-workgroup reduction is the FP64 one above.
//   FP32: v_mfma_f32_16x16x4_f32, G exact (it is generated in FP32), X rounded
//         to FP32 when staged; 64-row tiles, four K-steps of 4 rows per wave.
//   BF16: v_mfma_f32_16x16x32_bf16, G and X rounded to BF16 (round to nearest
//         even; X through FP32); 128-row tiles, one K-step of 32 rows per wave.
//         Operand slots: lane l, element e of A is (row l%16, k = 8(l/16)+e),
//         of B (k = 8(l/16)+e, column l%16).
// Both FP32-output forms return register r of lane l as row 4(l/16) + r,
// column l%16 (the FP64 form returns row l/16 + 4r).
// ---------------------------------------------------------------------------
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <int SM, int NN, bool BF>
struct SketchLpLds {
  static constexpr int TK = BF ? 128 : 64;           // tall rows per tile
  static constexpr int LD = BF ? TK + 8 : NN + 1;    // BF16: [col][row]; FP32: [row][col]
  static constexpr int TILE_BYTES = BF ? NN * LD * 2 : TK * LD * 4;
  static constexpr int RED_BYTES = SM * NN * 8;
  static constexpr int BYTES = (2 * TILE_BYTES > RED_BYTES) ? 2 * TILE_BYTES : RED_BYTES;
};

template <int SM, int NN, bool BF, bool WM>
__global__ __launch_bounds__(SK_THREADS) void k_sketch_lp(const double* __restrict__ X, int64_t m, int n, int64_t ld,
                                                          int64_t ntiles, uint64_t seed, double* __restrict__ Ypart,
                                                          int64_t s_pad, int64_t n_pad, const int32_t* info,
                                                          const SketchJob* __restrict__ jobs,
                                                          const BatchItem* __restrict__ items) {
  int64_t wg = blockIdx.x, nwg = gridDim.x;
  if (items) {  // batched launch: this workgroup's problem and its place in it
    const BatchItem it = items[blockIdx.x];
    const SketchJob j = jobs[it.prob];
    X = j.X, m = j.m, ld = j.ld, ntiles = j.ntiles, seed = j.seed, Ypart = j.Ypart, info = j.info;
    wg = it.wg, nwg = it.nwg;
  }
  if (info_failed(info)) return;
  using L = SketchLpLds<SM, NN, BF>;
  constexpr int MB = SM / 16, NB = NN / 16, TK = L::TK, LD = L::LD;
  constexpr int RPT = TK / 64 * 1;           // loader: rows per thread group
  constexpr int CPT = NN * TK / SK_THREADS;  // tile entries loaded per thread
  __shared__ __align__(16) unsigned char lds_raw[L::BYTES];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sg = blockIdx.y, col0 = blockIdx.z * NN;
  // loader: thread -> row (tid % TK), columns (tid / TK) + (SK_THREADS / TK) c
  constexpr int CSTEP = SK_THREADS / TK;
  const int lrow = tid % TK, lcol0 = tid / TK;
  (void)RPT;

  f32x4 acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  // prefetch registers: FP32 keeps the FP64 values as loaded (converting at
  // load time would wait for every load before the tile's products, so the
  // loads would not overlap them); BF16 (a 128-row tile, twice the entries)
  // packs pairs of columns per word to stay within the registers
  constexpr int PRE = BF ? CPT / 2 : 1;
  uint32_t prb[PRE];
  double pre[BF ? 1 : CPT];
  auto load_tile = [&](int64_t t) {
    const int64_t row = t * TK + lrow;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = col0 + lcol0 + CSTEP * c;
      if constexpr (BF) {
        const float v = (row < m && col < n) ? (float)X[row + (int64_t)col * ld] : 0.f;
        const uint32_t h = f32_to_bf16_rne(v);
        prb[c >> 1] = (c & 1) ? (prb[c >> 1] | (h << 16)) : h;
      } else {
        pre[c] = (row < m && col < n) ? X[row + (int64_t)col * ld] : 0.0;
      }
    }
  };
  auto store_tile = [&](int buf) {
    if constexpr (BF) {
      unsigned short* xs = (unsigned short*)(lds_raw + buf * L::TILE_BYTES);
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        xs[(lcol0 + CSTEP * c) * LD + lrow] = (unsigned short)((c & 1) ? (prb[c >> 1] >> 16) : (prb[c >> 1] & 0xFFFFu));
    } else {
      float* xs = (float*)(lds_raw + buf * L::TILE_BYTES);
#pragma unroll
      for (int c = 0; c < CPT; ++c) xs[lrow * LD + lcol0 + CSTEP * c] = (float)pre[c];
    }
  };

  const int ai = lane & 15, ag = lane >> 4;
  const int grp = WM ? 4 * sg + wave : sg;  // this wave's group of SM sketch rows
  const uint32_t qbase = (uint32_t)((grp * SM) / 4 + 4 * (ai >> 2) + (ai & 3));

  int64_t t = wg;
  int buf = 0;
  if (t < ntiles) {
    load_tile(t);
    store_tile(0);
  }
  __syncthreads();
  for (; t < ntiles; t += nwg) {
    const int64_t tn = t + nwg;
    if (tn < ntiles) load_tile(tn);
    if constexpr (BF) {
      const unsigned short* xs = (const unsigned short*)(lds_raw + buf * L::TILE_BYTES);
#pragma unroll 1
      for (int ks = 0; ks < (WM ? 4 : 1); ++ks) {
      const int r0 = (WM ? 32 * ks : 32 * wave) + 8 * ag;  // this lane's 8 tall rows within the tile
      bf16x8 b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const uint4 q = *(const uint4*)(xs + (16 * nb + ai) * LD + r0);
        b[nb] = __builtin_bit_cast(bf16x8, q);
      }
      const int64_t j0 = t * TK + r0;
#pragma unroll
      for (int a = 0; a < SM / 64; ++a) {
        // packed BF16 pairs: pk[u][e/2] holds elements e, e+1 of M-block 4a+u
        uint32_t pk[4][4];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          f32x4 z0 = {0.f, 0.f, 0.f, 0.f}, z1 = {0.f, 0.f, 0.f, 0.f};
          if (j0 + e < m) z0 = normals4(seed, (uint64_t)(j0 + e), qbase + 16u * (uint32_t)a);
          if (j0 + e + 1 < m) z1 = normals4(seed, (uint64_t)(j0 + e + 1), qbase + 16u * (uint32_t)a);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            pk[u][e >> 1] = (uint32_t)f32_to_bf16_rne(z0[u]) | ((uint32_t)f32_to_bf16_rne(z1[u]) << 16);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint4 q4 = {pk[u][0], pk[u][1], pk[u][2], pk[u][3]};
          const bf16x8 A = __builtin_bit_cast(bf16x8, q4);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[4 * a + u][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, b[nb], acc[4 * a + u][nb], 0, 0, 0);
        }
      }
      }
    } else {
      const float* xs = (const float*)(lds_raw + buf * L::TILE_BYTES);
#pragma unroll 1
      for (int ks = 0; ks < (WM ? 16 : 4); ++ks) {
        const int rloc = (WM ? 0 : 16 * wave) + 4 * ks + ag;
        const int64_t j = t * TK + rloc;
        float b[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) b[nb] = xs[rloc * LD + 16 * nb + ai];
#pragma unroll
        for (int a = 0; a < SM / 64; ++a) {
          f32x4 z = {0.f, 0.f, 0.f, 0.f};
          if (j < m) z = normals4(seed, (uint64_t)j, qbase + 16u * (uint32_t)a);
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              acc[4 * a + u][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(z[u], b[nb], acc[4 * a + u][nb], 0, 0, 0);
        }
      }
    }
    if (tn < ntiles) store_tile(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  if (WM) {  // each wave owns its rows: store them (FP64)
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int slot = 4 * (lane >> 4) + r;
          const int64_t srow = (int64_t)grp * SM + 64 * (a >> 2) + 16 * (slot >> 2) + 4 * (slot & 3) + (a & 3);
          const int64_t col = col0 + 16 * nb + (lane & 15);
          Ypart[wg * s_pad * n_pad + srow + col * s_pad] = (double)acc[a][nb][r];
        }
    return;
  }
  // Sum the four waves' partials in wave order (FP64) through LDS, then store.
  double* red = (double*)lds_raw;
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = ((a * NB + nb) * 4 + r) * 64 + lane;
            const double v = (w == 0) ? (double)acc[a][nb][r] : red[idx] + (double)acc[a][nb][r];
            if (w < 3) {
              red[idx] = v;
            } else {
              // slot row of M-block a -> sketch row 64(a/4) + 16c + 4t + a%4 for slot 4c + t
              const int slot = 4 * (lane >> 4) + r;
              const int64_t srow = (int64_t)sg * SM + 64 * (a >> 2) + 16 * (slot >> 2) + 4 * (slot & 3) + (a & 3);
              const int64_t col = col0 + 16 * nb + (lane & 15);
              Ypart[wg * s_pad * n_pad + srow + col * s_pad] = v;
            }
          }
    }
    __syncthreads();
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

__global__ void k_omega(uint64_t seed, int64_t s, int64_t j0, int64_t cols, float* __restrict__ G) {
  const int64_t q4 = (s + 3) / 4;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= q4 * cols) return;
  const int64_t q = e % q4, c = e / q4;
  const f32x4 z = normals4(seed, (uint64_t)(j0 + c), (uint32_t)q);
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (4 * q + u < s) G[4 * q + u + c * s] = z[u];
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
  if (n <= 16) {
    p.nn = 16;
  } else if (n <= 32) {
    p.nn = 32;
  } else if (n <= 64) {
    p.nn = 64;
  } else {
    p.nn = 128;
  }
  p.s_pad = pad_sketch_rows(s);
  // accumulators per wave: (sm/16)(nn/16) f64x4 <= 32
  const int max_sm = (p.nn == 16) ? 256 : (p.nn == 32) ? 256 : (p.nn == 64) ? 128 : 64;
  p.sm = 64;
  while (p.sm * 2 <= max_sm && p.s_pad % (p.sm * 2) == 0) p.sm *= 2;
  // four or more row groups: give each wave its own group (X read 4x less)
  p.wm = p.s_pad % (4 * p.sm) == 0;
  p.nw = 4;
  if (prec == 0 && !p.wm && p.sm >= 128 && p.s_pad % 128 == 0) {
    // FP64 with two 64-row groups' worth of rows: 64-row groups owned by the
    // waves instead (a 128-row group needs all 512 registers of a wave)
    p.sm = 64;
    p.wm = true;
    p.nw = (p.s_pad % 256 == 0) ? 4 : 2;
  }
  p.gy = (int)(p.s_pad / (p.wm ? p.nw * p.sm : p.sm));
  p.gz = (int)((n + p.nn - 1) / p.nn);
  p.n_pad = (int64_t)p.gz * p.nn;
  const int tk = (prec == 2) ? 128 : (prec == 0 ? sketch_f64_tk(p.nw) : SK_TK);  // BF16 tiles are 128 rows
  p.ntiles = (m + tk - 1) / tk;
  int gx = gx_hint > 0 ? gx_hint : 512 * 4 / p.nw;  // 2048 waves in all
  const int per_chunk = p.gy * p.gz;
  if (per_chunk > 1) gx = (gx + per_chunk - 1) / per_chunk;
  if (gx < 1) gx = 1;
  if (gx > p.ntiles) gx = (int)p.ntiles;
  p.gx = gx;
  // per-workgroup partials followed by the level-1 sums of the reduction
  p.part_bytes = ((size_t)p.gx + reduce_splits(p.gx)) * (size_t)p.s_pad * (size_t)p.n_pad * sizeof(double);
  return p;
}

template <int SM, int NN, bool WM>
static hipError_t launch_sk_wm(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld, uint64_t seed,
                               int prec, double* Ypart, const int32_t* info, const SketchJob* jobs,
                               const BatchItem* items, int nitems, hipStream_t st) {
  dim3 grid(items ? (unsigned)nitems : (unsigned)p.gx, p.gy, p.gz);
  if (prec == 0 && WM && p.nw == 2)
    hipLaunchKernelGGL((k_sketch_f64<SM, NN, WM, (WM ? 2 : 4)>), grid, dim3(128), 0, st, X, m, (int)n, ld, p.ntiles,
                       seed, Ypart, p.s_pad, p.n_pad, info, jobs, items);
  else if (prec == 0)
    hipLaunchKernelGGL((k_sketch_f64<SM, NN, WM, 4>), grid, dim3(SK_THREADS), 0, st, X, m, (int)n, ld, p.ntiles, seed,
                       Ypart, p.s_pad, p.n_pad, info, jobs, items);
  else if (prec == 1)
    hipLaunchKernelGGL((k_sketch_lp<SM, NN, false, WM>), grid, dim3(SK_THREADS), 0, st, X, m, (int)n, ld, p.ntiles,
                       seed, Ypart, p.s_pad, p.n_pad, info, jobs, items);
  else
    hipLaunchKernelGGL((k_sketch_lp<SM, NN, true, WM>), grid, dim3(SK_THREADS), 0, st, X, m, (int)n, ld, p.ntiles,
                       seed, Ypart, p.s_pad, p.n_pad, info, jobs, items);
  return hipGetLastError();
}

template <int SM, int NN>
static hipError_t launch_sk(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld, uint64_t seed,
                            int prec, double* Ypart, const int32_t* info, const SketchJob* jobs,
                            const BatchItem* items, int nitems, hipStream_t st) {
  if (p.wm) return launch_sk_wm<SM, NN, true>(p, X, m, n, ld, seed, prec, Ypart, info, jobs, items, nitems, st);
  return launch_sk_wm<SM, NN, false>(p, X, m, n, ld, seed, prec, Ypart, info, jobs, items, nitems, st);
}

static hipError_t sketch_dispatch(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld,
                                  uint64_t seed, int prec, double* Ypart, const int32_t* info, const SketchJob* jobs,
                                  const BatchItem* items, int nitems, hipStream_t st) {
  if (prec < 0 || prec > 2) return hipErrorInvalidValue;
#define SK_CASE(SMV, NNV)        \
  if (p.sm == SMV && p.nn == NNV) \
    return launch_sk<SMV, NNV>(p, X, m, n, ld, seed, prec, Ypart, info, jobs, items, nitems, st);
  SK_CASE(64, 16)
  SK_CASE(128, 16)
  SK_CASE(256, 16)
  SK_CASE(64, 32)
  SK_CASE(128, 32)
  SK_CASE(256, 32)
  SK_CASE(64, 64)
  SK_CASE(128, 64)
  SK_CASE(64, 128)
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
  const int64_t total = (s + 3) / 4 * cols;
  if (total <= 0) return hipSuccess;
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

}  // namespace rclupp
