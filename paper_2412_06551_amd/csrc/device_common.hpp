// Device-side helpers shared by the gfx950 kernels: the counter-based Gaussian
// generator of the sketch, MFMA fragment types, info handling, and launch-shape
// constants. Column-major float64 throughout (element (i, j) at A[i + j*ld]).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Largest supported column count (the C ABI's RCLUPP_MAX_N).
#define RCLUPP_SMALL_MAXN 256

namespace rclupp {

// Asynchronous outcome codes and stages (the values the C ABI documents).
enum : int32_t { INFO_OK = 0, INFO_LU_ZERO_PIVOT = 1, INFO_CHOL_BREAKDOWN = 2, INFO_NONFINITE = 3, INFO_SINGULAR = 4,
                INFO_SYNC_TIMEOUT = 5 };
enum : int32_t { STAGE_LU = 1, STAGE_QR = 2, STAGE_PRECOND = 3, STAGE_CHOL_A = 4, STAGE_CHOL_B = 5 };

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64: C[16x16] += A[16x4] B[4x16].
//   A operand: lane l holds A[l % 16][l / 16]
//   B operand: lane l holds B[l / 16][l % 16]
//   C/D:       lane l, register r holds C[l / 16 + 4 r][l % 16]
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Gaussian sketch entries. Section 3 takes S = G / sqrt(s) with G i.i.d.
// standard normal; here G_ij = z(seed, i, j) is a pure function of its indices:
//   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
//   counter = (floor(j/4) mod 2^32, floor(j/4) div 2^32, i, 0), key = (seed lo, seed hi);
//   each 32-bit word w gives u = (floor(w / 2^9) + 1/2) 2^-23, an odd multiple
//   of 2^-24 in (0, 1) that float32 holds exactly;
//   Box-Muller: (u0, u1) -> tall rows 4q, 4q+1 and (u2, u3) -> 4q+2, 4q+3 of
//   sketch row i (q = floor(j/4)):
//     z = sqrt(-2 ln u_a) * (cos 2 pi u_b, sin 2 pi u_b), in float32.
// One call thus gives one sketch row's entries for four consecutive tall rows,
// which is the run of the K index that one lane holds in the MFMA operands.
// ---------------------------------------------------------------------------
struct philox_out {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ philox_out philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                    uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ float word_to_uniform(uint32_t w) {
  return (float)(w >> 9) * 0x1p-23f + 0x1p-24f;  // exact: (2k+1) 2^-24
}

// The four normals of (sketch row i, tall-row group q): G[i][4q .. 4q+3].
__device__ __forceinline__ f32x4 normals4(uint64_t seed, uint64_t q, uint32_t i) {
  const philox_out w = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), i, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
  const float u0 = word_to_uniform(w.w0), u1 = word_to_uniform(w.w1);
  const float u2 = word_to_uniform(w.w2), u3 = word_to_uniform(w.w3);
  // Box-Muller on the hardware transcendentals: log2, square root, and sine
  // and cosine of 2 pi x taken in revolutions (one instruction each; within
  // 8 float32 ulps of max(|z|, 1) of the correctly rounded transform, checked
  // against the library functions on 2^24 draws)
  const float k = -2.0f * 0.693147180559945309f;  // -2 ln 2: ln u = ln 2 log2 u
  const float r0 = __builtin_amdgcn_sqrtf(k * __builtin_amdgcn_logf(u0));
  const float r1 = __builtin_amdgcn_sqrtf(k * __builtin_amdgcn_logf(u2));
  f32x4 z;
  z[0] = r0 * __builtin_amdgcn_cosf(u1);
  z[1] = r0 * __builtin_amdgcn_sinf(u1);
  z[2] = r1 * __builtin_amdgcn_cosf(u3);
  z[3] = r1 * __builtin_amdgcn_sinf(u3);
  return z;
}

// ---------------------------------------------------------------------------
// Device-side outcome record.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool info_failed(const int32_t* info) {
  return info != nullptr && __builtin_nontemporal_load(info) != 0;
}

// Only one thread of one workgroup records a failure at a time in every
// stage that can fail, so a plain vector store suffices.
__device__ __forceinline__ void info_set(int32_t* info, int32_t code, int32_t stage, int32_t index) {
  if (info != nullptr && info[0] == 0) {
    info[1] = stage;
    info[2] = index;
    info[3] = 0;
    __threadfence();
    info[0] = code;
  }
}

__device__ __forceinline__ bool is_finite(double v) { return __builtin_isfinite(v); }

// Streaming hints for the tall operands. A 16-row run of one column (a
// quarter of a wave's load or store) fills one 128-byte line only when the
// column starts on a line: base 128-byte aligned and ld a multiple of 16
// elements. With any other leading dimension every run straddles two lines
// whose other parts belong to the neighbouring runs, and a nontemporal access
// lets the line leave the caches before the neighbour reaches it (measured:
// more than twice the time of a pass). The kernels then use ordinary accesses.
__device__ __forceinline__ bool runs_line_aligned(const void* p, int64_t ld) {
  return ((ld & 15) == 0) && (((uintptr_t)p & 127) == 0);
}
template <bool NT>
__device__ __forceinline__ double stream_load(const double* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void stream_store(double v, double* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Makes a wave-uniform pointer opaque to the optimizer and returns it as a
// constant-address-space pointer, so loads through it are scalar loads issued
// where they are consumed (inside a row-tile loop) rather than hoisted out of
// the loop, which would overflow the scalar register file.
typedef __attribute__((address_space(4))) const double* cdptr;
__device__ __forceinline__ cdptr opaque_uniform(const double* p) {
  asm volatile("" : "+s"(p));
  return (cdptr)p;
}

// As opaque_uniform, and the loads through the result may not be issued
// before `dep` is available (bounds how far ahead the scalar loads run).
__device__ __forceinline__ cdptr opaque_after(const double* p, double dep) {
  asm volatile("" : "+s"(p) : "v"(dep));
  return (cdptr)p;
}

// Same for a uniform 64-bit integer (a column stride): keeps per-column
// address arithmetic next to its load instead of hoisting one scalar register
// pair per column out of the row-tile loop.
__device__ __forceinline__ int64_t opaque_i64(int64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

}  // namespace rclupp
