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

constexpr int TS_ROWS = 256;  // rows of a node's block
constexpr int TS_CPW = 8;     // columns of the block held by one wave

__device__ __forceinline__ void ts_info_set(int32_t* info, int32_t code, int32_t stage, int32_t index) {
  // many nodes may fail at once: the first failure wins the code word
  if (info != nullptr && atomicCAS(info, 0, code) == 0) {
    info[1] = stage;
    info[2] = index;
    info[3] = 0;
  }
}

// lane `ln` (wave-uniform) of a double held in VGPRs
__device__ __forceinline__ double ts_readlane(double v, int ln) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, ln), hi = __builtin_amdgcn_readlane((int)(b >> 32), ln);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
// Wave maximum / minimum by DPP: butterflies within each 16-lane row (quad
// permutations, half-row and row mirrors), then the row broadcasts
// (row_bcast:15 = 0x142 into rows 1 and 3, row_bcast:31 = 0x143 into rows 2
// and 3) carry the result into the last row; it is read from lane 63. The
// moved operand of a lane without a source is the operation's identity,
// which lets the compiler fold each move into the max or min instruction.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned ts_dpp_umax(unsigned v) {
  return max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ unsigned ts_wave_umax(unsigned v) {
  v = ts_dpp_umax<0xB1, 0xF>(v);
  v = ts_dpp_umax<0x4E, 0xF>(v);
  v = ts_dpp_umax<0x141, 0xF>(v);
  v = ts_dpp_umax<0x140, 0xF>(v);
  v = ts_dpp_umax<0x142, 0xA>(v);
  v = ts_dpp_umax<0x143, 0xC>(v);
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ int ts_dpp_min(int v) {
  return min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ int ts_wave_min(int v) {
  v = ts_dpp_min<0xB1, 0xF>(v);
  v = ts_dpp_min<0x4E, 0xF>(v);
  v = ts_dpp_min<0x141, 0xF>(v);
  v = ts_dpp_min<0x140, 0xF>(v);
  v = ts_dpp_min<0x142, 0xA>(v);
  v = ts_dpp_min<0x143, 0xC>(v);
  return __builtin_amdgcn_readlane(v, 63);
}

// Shared state of one node.
struct TsShared {
  double l[2][TS_CPW][TS_ROWS];  // multipliers of the steps of a panel, by local row (two panels in flight)
  int key[2][TS_CPW];            // pivots of those steps: (position << 9) | (sign << 8) | row
  int flag[2][TS_CPW];           // p + 1 once step c of panel p is published
  int posl[TS_ROWS];             // position of each local row
  int rowat[TS_ROWS];            // local row at each of the first n positions (at the end)
  int fail[2];                   // failure seen after the barrier that publishes panel p, in slot p % 2
                                 // (set during the window before it, read after it: no wave reads a
                                 // slot while another may still set it)
};

// x[c] -= l u_c for the register columns c in [C0, 8), u_c being column c of
// the pivot row of the step (row = key & 255: lane row % 64, register row
// row / 64, both wave-uniform; one branch on the register row: reading all
// four register rows and selecting measured slower).
template <int C0>
__device__ __forceinline__ void ts_apply(double (&x)[TS_CPW][4], const double (&l)[4], int key) {
  if constexpr (C0 < TS_CPW) {
    const int prow = key & 255, pa = prow >> 6, pl = prow & 63;
    double u[TS_CPW];
#define TS_READ_ROW(A) \
  _Pragma("unroll") for (int c = C0; c < TS_CPW; ++c) u[c] = ts_readlane(x[c][A], pl);
    switch (pa) {
      case 0: TS_READ_ROW(0) break;
      case 1: TS_READ_ROW(1) break;
      case 2: TS_READ_ROW(2) break;
      default: TS_READ_ROW(3) break;
    }
#undef TS_READ_ROW
#pragma unroll
    for (int c = C0; c < TS_CPW; ++c)
#pragma unroll
      for (int a = 0; a < 4; ++a) x[c][a] = __builtin_fma(-l[a], u[c], x[c][a]);
  }
}

// The pivot of step k on register column C (pos: the positions of the lane's
// rows after step k - 1): the largest |x| over the rows at positions >= k,
// ties to the smaller position (a wave maximum over the bit patterns of |x|,
// then the key of the row that attains it, or the wave minimum of the keys
// when several do), and the multipliers RN(x / p) of the other live rows into
// l (zero for rows that are not eliminated). Publishes the multipliers (ls),
// the key (ks), the position swap and then the step's flag (fs = fv); pos
// becomes the positions after step k. Returns the key, or -1 (with zero
// multipliers, and the failure flag set) if the column is not finite or, at
// the root, zero.
template <int C>
__device__ __forceinline__ int ts_pivot(double (&x)[TS_CPW][4], int (&pos)[4], double (&l)[4], double* ls, int* ks,
                                        int* fs, int fv, TsShared& sh, int k, int r, int lane, bool root,
                                        int32_t* info) {
  // |x| compared through its bit pattern (the order of non-negative
  // doubles): first the high words (a live row's plus one, zero for the
  // others), then, only when several rows share the largest, the low words
  unsigned hv[4], lo[4];
  bool live[4], bad = false;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    live[a] = (lane + 64 * a < r) & (pos[a] >= k);
    const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(x[C][a]));
    hv[a] = live[a] ? (unsigned)(bits >> 32) + 1u : 0u;
    lo[a] = (unsigned)bits;
    bad |= live[a] & !is_finite(x[C][a]);
  }
  // independent of the pivot, so formed beside the reductions below: the
  // row now at position k, and whether any live entry is not finite
  unsigned long long atk = 0;
  int qa = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const unsigned long long bk = __ballot(pos[a] == k);
    if (bk != 0) {
      atk = bk;
      qa = a;
    }
  }
  const int q = 64 * qa + __builtin_ctzll(atk);
  const bool anybad = __ballot(bad) != 0;
  const unsigned hm = ts_wave_umax(max(max(hv[0], hv[1]), max(hv[2], hv[3])));
  // nc rows attain it; lw is the lane of one of them (of the only one when
  // nc = 1)
  bool cand[4];
  int nc = 0;
  unsigned long long anyc = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    cand[a] = hv[a] == hm;
    const unsigned long long at = __ballot(cand[a]);
    nc += __builtin_popcountll(at);
    anyc |= at;
  }
  int lw = __builtin_ctzll(anyc);
  // common case first: one row has the largest high word; otherwise the low
  // words of those rows decide, behind a branch laid out of line (a taken
  // branch costs a wave about as much as a dozen dependent instructions)
  unsigned lm = (unsigned)__builtin_amdgcn_readlane((int)(cand[0] ? lo[0] : cand[1] ? lo[1] : cand[2] ? lo[2] : lo[3]), lw);
  if (__builtin_expect(nc != 1, 0)) {
    lm = ts_wave_umax(max(max(cand[0] ? lo[0] : 0u, cand[1] ? lo[1] : 0u),
                          max(cand[2] ? lo[2] : 0u, cand[3] ? lo[3] : 0u)));
    nc = 0;
    anyc = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      cand[a] = cand[a] & (lo[a] == lm);
      const unsigned long long at = __ballot(cand[a]);
      nc += __builtin_popcountll(at);
      anyc |= at;
    }
    lw = __builtin_ctzll(anyc);
  }
  const double best = __longlong_as_double((long long)(((unsigned long long)(hm - 1u) << 32) | lm));
  // RN(1 / |p|), formed while the keys are reduced (RN(1 / -b) = -RN(1 / b))
  const double yb = 1.0 / best;
  // the key of the row attaining it (read from its lane), or the wave
  // minimum of the keys when several do; the key carries the entry's sign
  // below the position, which decides nothing (positions are distinct)
  int kc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
    kc[a] = cand[a] ? ((pos[a] << 9) | ((x[C][a] < 0.0) << 8) | (lane + 64 * a)) : INT_MAX;
  const int kl = min(min(kc[0], kc[1]), min(kc[2], kc[3]));
  int key = __builtin_amdgcn_readlane(kl, lw);
  // the tests of the rare cases below (a failure; a pivot the corrected
  // quotient does not cover)
  const bool zero = !(best > 0.0);
  const bool failed = anybad || (zero && root);
  const bool odd = zero || best < 0x1p-1022 || best > 0x1p1022;
  // the reciprocal, the key and those tests are independent chains: keep
  // them in one block, ahead of the branches below, so that their latencies
  // overlap
  __asm__ volatile("" ::"v"(yb), "s"((int)failed | ((int)odd << 1)));
  if (__builtin_expect(nc != 1, 0)) key = ts_wave_min(kl);
  if (__builtin_expect(failed, 0)) {
    if (lane == 0) {
      ts_info_set(info, anybad ? INFO_NONFINITE : INFO_LU_ZERO_PIVOT, STAGE_LU, k + 1);
      sh.fail[(k / TS_CPW) & 1] = 1;
      *ks = -1;
      *fs = fv;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) l[a] = 0.0;
    return -1;
  }
  const int prow = key & 255, ppos = key >> 9;
  const bool pneg = (key >> 8) & 1;
  const double p = pneg ? -best : best;
  // multipliers RN(x / p): Markstein's corrected quotient from one reciprocal
  // y = RN(1 / p), q0 = RN(x y), RN(q0 + (x - q0 p) y), the correctly rounded
  // quotient when y is normal (|x / p| <= 1); subnormal pivots and pivots
  // above 1 / (smallest normal) divide directly (rare: formed after the
  // common case). A zero pivot column (a singular block below the root)
  // eliminates nothing.
  const double y = pneg ? -yb : yb;
  double qv[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double q0 = x[C][a] * y;
    qv[a] = __builtin_fma(__builtin_fma(-q0, p, x[C][a]), y, q0);
  }
  if (__builtin_expect(odd, 0)) {
#pragma unroll
    for (int a = 0; a < 4; ++a) qv[a] = zero ? 0.0 : x[C][a] / p;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = lane + 64 * a;
    const bool elim = live[a] & (row != prow) & !zero;
    l[a] = elim ? qv[a] : 0.0;
    x[C][a] = elim ? qv[a] : x[C][a];
    ls[row] = l[a];
  }
  // one lane publishes the key, the position swap (the pivot row moves to k,
  // the row at k to its place) and then the step's flag
  if (lane == 0) {
    *ks = key;
    sh.posl[q] = ppos;
    sh.posl[prow] = k;
    __hip_atomic_store(fs, fv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) pos[a] = (lane + 64 * a == prow) ? k : (pos[a] == k ? ppos : pos[a]);
  return key;
}

// Steps 8w .. 8w+7 (those below n) on the wave that holds their columns: the
// unblocked elimination of its 8 columns (each pivot, then that step applied
// to the wave's columns after it), published step by step into panel buffer
// w % 2 (multipliers, key, then the step's flag: the LDS executes one wave's
// accesses in issue order, so a wave that reads the flag and then the step
// sees the step; no wait for the writes is needed before the flag).
__device__ __forceinline__ void ts_panel(double (&x)[TS_CPW][4], int (&pos)[4], TsShared& sh, int w, int n, int r,
                                         int lane, bool root, int32_t* info) {
  const int b = w & 1;
  double l[4];
  // A failed pivot sets the node's failure flag and the node stops at the
  // next barrier; the rest of the panel still runs (on meaningless values,
  // with every index in range: a key of -1 names row 255), which keeps one
  // path through the registers.
#define TS_PANEL_STEP(C)                                                                                    \
  if (TS_CPW * w + C < n) {                                                                                 \
    const int key = ts_pivot<C>(x, pos, l, sh.l[b][C], &sh.key[b][C], &sh.flag[b][C], w + 1, sh, TS_CPW * w + C, r, \
                                lane, root, info);                                                          \
    ts_apply<C + 1>(x, l, key);                                                                             \
  }
  // the panel is the node's critical path: its wave issues first
  __builtin_amdgcn_s_setprio(3);
  TS_PANEL_STEP(0)
  TS_PANEL_STEP(1)
  TS_PANEL_STEP(2)
  TS_PANEL_STEP(3)
  TS_PANEL_STEP(4)
  TS_PANEL_STEP(5)
  TS_PANEL_STEP(6)
  TS_PANEL_STEP(7)
#undef TS_PANEL_STEP
  __builtin_amdgcn_s_setprio(0);
}

// Step c of panel p (published) on a wave's own columns.
__device__ __forceinline__ void ts_follow(double (&x)[TS_CPW][4], const TsShared& sh, int p, int c, int lane) {
  const int b = p & 1;
  const int key = __builtin_amdgcn_readfirstlane(sh.key[b][c]);
  double l[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) l[a] = sh.l[b][c][lane + 64 * a];
  ts_apply<0>(x, l, key);
}

// One node: Gaussian elimination with partial pivoting of r <= 256 rows and
// n <= 8 NWV columns, in registers: wave w holds columns 8w .. 8w+7, lane l
// the rows l, l+64, l+128, l+192. Rows never move; positions trade (an LDS
// table, and registers in the wave that chooses the pivots). Blocked by
// panels of 8 columns: the wave that holds a panel eliminates it on its own
// and publishes its 8 steps; after one barrier the waves that hold later
// columns apply them, and the wave of the next panel then eliminates that
// one. Every element receives the updates of the steps in step order, each
// as one fused multiply-add, as in the unblocked elimination.
//   leaf level (prev == nullptr): node g factors rows floor(g m / L) .. of X;
//   upper levels: node g stacks the sets g F .. of prev (n indices each; the
//     last node may have fewer), nsets sets in all, whose rows of X it reads
//     from cin (set s: n x n, ld n, rows in the set's order) when the level
//     below forwarded them, else from X by index.
// Writes the original indices of its first n pivot rows to sel[g n ..] and,
// with cout, those rows of X (set g), so that the next level reads them
// contiguously instead of gathering them from X (for n > 64: measured 3 %
// faster at 16,777,216 x 128, 20 % slower at 1,048,576 x 64); the root (one
// node) writes N and L_11 (n x n, ld n).
template <int NWV>
__global__ __launch_bounds__(64 * NWV, NWV >= 4 ? 4 : NWV) void k_tslu_node(
    const double* __restrict__ X, int64_t ldx, int64_t m, int n, int64_t leaves, const int32_t* __restrict__ prev,
    int64_t nsets, int F, int32_t* __restrict__ sel, const double* __restrict__ cin, double* __restrict__ cout,
    double* __restrict__ Nout, double* __restrict__ Lout, int32_t* info) {
  __shared__ TsShared sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) sh.fail[0] = sh.fail[1] = info_failed(info) ? 1 : 0;
  for (int i = tid; i < TS_ROWS; i += 64 * NWV) sh.posl[i] = i;
  for (int i = tid; i < 2 * TS_CPW; i += 64 * NWV) sh.flag[i / TS_CPW][i % TS_CPW] = 0;
  __syncthreads();
  if (sh.fail[0]) return;
  const int64_t g = blockIdx.x;
  const bool root = gridDim.x == 1;
  // local row i is X's row r0 + i (leaves) or prev[s0 n + i] (upper levels)
  int r;
  int64_t r0 = 0, s0 = 0;
  if (!prev) {
    r0 = g * m / leaves;
    r = (int)((g + 1) * m / leaves - r0);
  } else {
    s0 = g * F;
    const int64_t s1 = (s0 + F < nsets) ? s0 + F : nsets;
    r = (int)((s1 - s0) * n);
  }
  auto orig = [&](int row) -> int64_t { return prev ? (int64_t)prev[s0 * n + row] : r0 + row; };
  // the block: from the stacked sets when the level below forwarded them,
  // else from X
  const int64_t nn = (int64_t)n * n;
  double x[TS_CPW][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = lane + 64 * a;
    const double* src = nullptr;
    int64_t ld = 0;
    if (row < r) {
      src = cin ? cin + (s0 + row / n) * nn + row % n : X + orig(row);
      ld = cin ? n : ldx;
    }
#pragma unroll
    for (int c = 0; c < TS_CPW; ++c) {
      const int col = TS_CPW * wave + c;
      x[c][a] = (row < r && col < n) ? src[(int64_t)col * ld] : 0.0;
    }
  }
  int pos[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) pos[a] = lane + 64 * a;
  const int np = (n + TS_CPW - 1) / TS_CPW;  // panels
  // j = -1: wave 0 eliminates panel 0 (one copy of the panel code for all
  // panels keeps the kernel's instructions few)
  for (int j = -1; j < np; ++j) {
    if (j >= 0) {
      __syncthreads();  // panel j published
      if (sh.fail[j & 1]) return;
    }
    if (wave > j && TS_CPW * wave < n) {
      // the steps of panel j on this wave's columns, in step order (the wave
      // of panel j + 1 applied them while they were published)
      if (j >= 0 && wave != j + 1) {
#pragma unroll 1
        for (int c = 0; c < TS_CPW && TS_CPW * j + c < n; ++c) ts_follow(x, sh, j, c, lane);
      }
      if (wave == j + 1) {
        // the next panel: its wave takes the positions from the table
#pragma unroll
        for (int a = 0; a < 4; ++a) pos[a] = sh.posl[lane + 64 * a];
        ts_panel(x, pos, sh, wave, n, r, lane, root, info);
      } else if (wave == j + 2) {
        // the wave of panel j + 2 applies the steps of panel j + 1 as they
        // are published, so that it can start its own panel at the barrier
        // (a bounded wait: on time-out the node fails)
#pragma unroll 1
        for (int c = 0; c < TS_CPW && TS_CPW * (j + 1) + c < n; ++c) {
          unsigned spins = 0;
          while (__hip_atomic_load(&sh.flag[(j + 1) & 1][c], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != j + 2) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 22)) break;
          }
          if (spins > (1u << 22)) {
            if (lane == 0) {
              ts_info_set(info, INFO_SYNC_TIMEOUT, STAGE_LU, TS_CPW * (j + 1) + c + 1);
              sh.fail[(j + 1) & 1] = 1;
            }
            break;
          }
          ts_follow(x, sh, j + 1, c, lane);
        }
      }
    }
  }
  __syncthreads();
  if (sh.fail[0] | sh.fail[1]) return;
  if (wave == 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int row = lane + 64 * a;
      const int p = sh.posl[row];
      if (row < r && p < n) sel[g * n + p] = (int32_t)orig(row);
    }
  }
  if (cout) {
    // the candidates' rows of X, in pivot order, for the next level (first
    // the local row at each of the first n positions)
    for (int row = tid; row < r; row += 64 * NWV) {
      const int p = sh.posl[row];
      if (p < n) sh.rowat[p] = row;
    }
    __syncthreads();
    // each wave its own columns, lane l the positions l and l + 64
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int p = lane + 64 * a;
      if (p >= n) continue;
      const int row = sh.rowat[p];
      const double* src = cin ? cin + (s0 + row / n) * nn + row % n : X + orig(row);
      const int64_t ld = cin ? n : ldx;
#pragma unroll
      for (int c = 0; c < TS_CPW; ++c) {
        const int col = TS_CPW * wave + c;
        if (col < n) cout[g * nn + (int64_t)col * n + p] = src[(int64_t)col * ld];
      }
    }
  }
  if (root) {
#pragma unroll
    for (int c = 0; c < TS_CPW; ++c) {
      const int col = TS_CPW * wave + c;
      if (col >= n) continue;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int row = lane + 64 * a;
        const int p = sh.posl[row];
        if (row < r && p < n) {
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

int64_t tslu_leaves(int64_t m) { return (m + TS_ROWS - 1) / TS_ROWS; }

static size_t tslu_al(size_t b) { return (b + 255) / 256 * 256; }

static bool tslu_forward(int64_t n) { return n > 64; }

// The sizes of the forwarded rows of the first and second merge levels (the
// leaves do not forward: the first merge level gathers 2n rows from two
// neighbouring 256-row blocks of X, nearly as fast as the leaves read theirs,
// and writing the leaves' candidates cost more than it saved).
static size_t tslu_fwd_bytes(int64_t m, int64_t n, int level) {
  if (!tslu_forward(n)) return 0;
  const int64_t F = TS_ROWS / n;
  int64_t nodes = tslu_leaves(m);
  for (int l = 0; l < level; ++l) nodes = (nodes + F - 1) / F;
  return (size_t)nodes * n * n * sizeof(double);
}

size_t tslu_scratch_bytes(int64_t m, int64_t n) {
  // candidate sets of two consecutive levels (indices, and for n > 64 the
  // rows of X of the merge levels' candidates), N and L_11, the padded N
  const int64_t leaves = tslu_leaves(m);
  const size_t sets = (size_t)leaves * n * sizeof(int32_t);
  const size_t c0 = tslu_fwd_bytes(m, n, 1), c1 = tslu_fwd_bytes(m, n, 2);
  const int np = pad_cols(n);
  return 2 * tslu_al(sets) + tslu_al(c0) + tslu_al(c1) + 2 * tslu_al((size_t)n * n * 8) +
         tslu_al(padded_r_doubles(np) * 8);
}

hipError_t launch_tslu(const double* X, int64_t m, int64_t n, int64_t ldx, double* W, int64_t ldw, int32_t* sel,
                       double* Nout, double* scratch, int32_t* info, hipStream_t st) {
  if (n < 1 || n > TS_CPW * 16 || m < n) return hipErrorInvalidValue;
  const int64_t leaves = tslu_leaves(m);
  const int F = TS_ROWS / (int)n;
  const size_t sets = tslu_al((size_t)leaves * n * sizeof(int32_t));
  const bool fwd = tslu_forward(n);
  const size_t c0 = tslu_al(tslu_fwd_bytes(m, n, 1)), c1 = tslu_al(tslu_fwd_bytes(m, n, 2));
  char* sp = (char*)scratch;
  int32_t* lv[2] = {(int32_t*)sp, (int32_t*)(sp + sets)};
  double* cv[2] = {(double*)(sp + 2 * sets), (double*)(sp + 2 * sets + c0)};
  double* Lt = (double*)(sp + 2 * sets + c0 + c1);
  double* Nt = Nout ? Nout : (double*)((char*)Lt + tslu_al((size_t)n * n * 8));
  double* Npad = (double*)((char*)Lt + 2 * tslu_al((size_t)n * n * 8));
  // waves per node: one per 8 columns, rounded up to a power of two
  const int64_t wv = (n + TS_CPW - 1) / TS_CPW;
  auto node = [&](int64_t nodes, const int32_t* prev, int64_t nsets, int32_t* out, const double* cin, double* cout) {
#define TS_LAUNCH(NWV)                                                                                           \
  hipLaunchKernelGGL(k_tslu_node<NWV>, dim3((unsigned)nodes), dim3(64 * NWV), 0, st, X, ldx, m, (int)n, leaves, \
                     prev, nsets, F, out, cin, cout, Nt, Lt, info)
    if (wv <= 1)
      TS_LAUNCH(1);
    else if (wv <= 2)
      TS_LAUNCH(2);
    else if (wv <= 4)
      TS_LAUNCH(4);
    else if (wv <= 8)
      TS_LAUNCH(8);
    else
      TS_LAUNCH(16);
#undef TS_LAUNCH
    return hipGetLastError();
  };
  // leaves, then levels of F-way merges until one set is left (the root
  // writes N and L_11; the final candidates go to `sel`)
  // (the merge levels' candidates' rows of X: the first level's in cv[0],
  // then alternately in cv[1] and cv[0], each level's output no larger than
  // its buffer; the first merge level gathers from X)
  int cur = 0;
  hipError_t e = node(leaves, nullptr, 0, leaves == 1 ? sel : lv[cur], nullptr, nullptr);
  if (e != hipSuccess) return e;
  int64_t nsets = leaves;
  int level = 1;
  while (nsets > 1) {
    const int64_t nodes = (nsets + F - 1) / F;
    const double* cin = (fwd && level >= 2) ? cv[level & 1] : nullptr;
    double* cout = (fwd && nodes > 1) ? cv[(level + 1) & 1] : nullptr;
    e = node(nodes, lv[cur], nsets, nodes == 1 ? sel : lv[cur ^ 1], cin, cout);
    if (e != hipSuccess) return e;
    cur ^= 1;
    nsets = nodes;
    ++level;
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
