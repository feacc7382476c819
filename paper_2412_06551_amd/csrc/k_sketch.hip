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

template <int P, int NN, int NW>
__global__ __launch_bounds__(64 * NW) void k_sketch(const double* __restrict__ X, int64_t m, int n, int64_t ld,
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

  using acc_t = typename std::conditional<P == 0, f64x4, f32x4>::type;
  acc_t acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = acc_t{0, 0, 0, 0};

  double pre[CPT];
  auto load_tile = [&](int64_t t) {
    const int64_t row = t * TK + lr;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = lc + CG * c;
      pre[c] = (row < m && col < n) ? X[row + (int64_t)col * ld] : 0.0;
    }
  };
  auto store_tile = [&](int buf) {
    unsigned char* base = lds + buf * T::BYTES;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = lc + CG * c;
      if constexpr (P == 0) {
        ((double*)base)[lr * LD + col] = pre[c];
      } else if constexpr (P == 1) {
        ((float*)base)[lr * LD + col] = (float)pre[c];
      } else {
        ((unsigned short*)base)[col * LD + lr] = (unsigned short)f32_to_bf16_rne((float)pre[c]);
      }
    }
  };

  int64_t t = chunk;
  int buf = 0;
  if (t < ntiles) {
    load_tile(t);
    store_tile(0);
  }
  __syncthreads();
  for (; t < ntiles; t += nchunks) {
    const int64_t tn = t + nchunks;
    if (tn < ntiles) load_tile(tn);
    const unsigned char* base = lds + buf * T::BYTES;
    if constexpr (P == 2) {
      const unsigned short* xs = (const unsigned short*)base;
      // one K-step of 32 rows: lane group g holds rows 8g .. 8g+7
      const uint64_t q0 = (uint64_t)(t * TK) / 4 + 2 * ag;
      const f32x4 z0 = normals4(seed, q0, srow), z1 = normals4(seed, q0 + 1, srow);
      const uint4 a4 = {f32_to_bf16_rne(z0[0]) | (f32_to_bf16_rne(z0[1]) << 16),
                        f32_to_bf16_rne(z0[2]) | (f32_to_bf16_rne(z0[3]) << 16),
                        f32_to_bf16_rne(z1[0]) | (f32_to_bf16_rne(z1[1]) << 16),
                        f32_to_bf16_rne(z1[2]) | (f32_to_bf16_rne(z1[3]) << 16)};
      const bf16x8 A = __builtin_bit_cast(bf16x8, a4);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const uint4 q = *(const uint4*)(xs + (16 * nb + ai) * LD + 8 * ag);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, q), acc[nb], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ss = 0; ss < TK / 16; ++ss) {
        // super-step of 16 rows: K-step ks takes row 16 ss + 4g + ks in lane group g
        const f32x4 z = normals4(seed, (uint64_t)(t * TK + 16 * ss) / 4 + ag, srow);
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

template <int P, int NN, int NW>
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
  hipLaunchKernelGGL((k_sketch<P, NN, NW>), grid, block, 0, st, X, m, (int)n, ld, p.ntiles, seed, Ypart, p.s_pad,
                     p.n_pad, p.gy, xcd, info, jobs, items);
  return hipGetLastError();
}

template <int NN, int NW>
static hipError_t launch_sk2(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld, uint64_t seed,
                             int prec, double* Ypart, const int32_t* info, const SketchJob* jobs,
                             const BatchItem* items, int nitems, hipStream_t st) {
  if (prec == 0) return launch_sk3<0, NN, NW>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
  if (prec == 1) return launch_sk3<1, NN, NW>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
  return launch_sk3<2, NN, NW>(p, X, m, n, ld, seed, Ypart, info, jobs, items, nitems, st);
}

static hipError_t sketch_dispatch(const SketchPlan& p, const double* X, int64_t m, int64_t n, int64_t ld,
                                  uint64_t seed, int prec, double* Ypart, const int32_t* info, const SketchJob* jobs,
                                  const BatchItem* items, int nitems, hipStream_t st) {
  if (prec < 0 || prec > 2 || p.gz != 1 || n > p.nn) return hipErrorInvalidValue;
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

}  // namespace rclupp
