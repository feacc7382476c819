// C ABI of the tall-skinny QR library (declarations and contracts in
// include/rclupp.h). Host side only: argument validation, workspace layout,
// and the stream-ordered launch sequence of each method.
//
// Method pipelines (every arrow is one or two kernels on the caller's stream):
//   RCLUPP   (Alg. 2): sketch(X) -> Y -> LU + Householder R + D R_0 N -> R_1
//                      -> CholeskyQR2 tail
//   RCLUPPr  (Alg. 7): tall LU(X) -> M (in Q), N -> sketch(M) -> Householder R
//                      of M_s -> D R_0 N -> R_1 -> CholeskyQR2 tail
//   CholeskyQR2 (Alg. 3): Gram(X) -> chol -> R_1 -> one CholeskyQR step
//   SCholeskyQR3 (Alg. 4): Gram(X) -> shifted chol -> R_1 -> CholeskyQR2 tail
//   LC2 (Alg. 5):      tall LU(X) -> Gram(M) -> chol -> D S_c N = R_1 -> one step
//   RCholeskyQR (Alg. 6): sketch(X) -> Householder R -> R_1 -> one step
// CholeskyQR2 tail (eqs. C1-C8): Q_1 = X R_1^{-1} with G_1 fused -> R_2 =
// chol(G_1), R_3 = R_2 R_1 -> Q_2 = Q_1 R_2^{-1} in place with G_2 fused ->
// R_4 = chol(G_2), R = R_4 R_3 -> Q = Q_2 R_4^{-1} in place.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rclupp.h"
#include "launch.hpp"

using namespace rclupp;

// Workspace of the allocation-free entry point rclupp_qr_noalloc. Every device
// the library runs on holds its own copy (loaded with the library's code
// object, kept until the process ends). In host code this name is only a
// stand-in for the symbol: the device address of the current device's copy
// comes from hipGetSymbolAddress (noalloc_scratch below) and is the only form
// passed to kernels.
static __device__ __align__(256) unsigned char noalloc_ws[RCLUPP_NOALLOC_MAX_BYTES];

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

bool sketched(int alg) { return alg == RCLUPP_ALG_RCLUPP || alg == RCLUPP_ALG_RCLUPPR || alg == RCLUPP_ALG_RCHOLQR; }
bool uses_tall_lu(int alg) { return alg == RCLUPP_ALG_RCLUPPR || alg == RCLUPP_ALG_LC2; }

struct Layout {
  size_t info = 0, gates = 0, ypart = 0, y = 0, r1 = 0, r2 = 0, r3 = 0, r4 = 0, gpart = 0, g = 0, small = 0,
         perm = 0, nmat = 0, lu = 0, total = 0;
  SketchPlan sk{};
  TallPlan tp{};
  bool tslu = false;  // the tall LU takes tournament pivoting
};

int validate(int alg, int64_t m, int64_t n, int64_t ld, int64_t s, const rclupp_opts* o) {
  if (alg < RCLUPP_ALG_RCLUPP || alg > RCLUPP_ALG_RCHOLQR) return RCLUPP_ERR_INVALID_ARG;
  if (n < 1 || m < n || ld < m) return RCLUPP_ERR_INVALID_ARG;
  if (n > RCLUPP_MAX_N) return RCLUPP_ERR_UNSUPPORTED;
  if (m > (int64_t)INT32_MAX && uses_tall_lu(alg)) return RCLUPP_ERR_UNSUPPORTED;
  if (sketched(alg) && (s < n || s > m)) return RCLUPP_ERR_INVALID_ARG;
  if (sketched(alg) && s > 4096) return RCLUPP_ERR_UNSUPPORTED;
  // the tall kernels address a row tile with 32-bit byte offsets
  if (m + 3 * ld >= ((int64_t)1 << 29)) return RCLUPP_ERR_UNSUPPORTED;
  if (o) {
    if (o->sketch_prec < 0 || o->sketch_prec > 2 || o->lu_prec < 0 || o->lu_prec > 1) return RCLUPP_ERR_INVALID_ARG;
    if (o->sketch_kind != RCLUPP_SKETCH_GAUSSIAN && o->sketch_kind != RCLUPP_SKETCH_COUNT &&
        o->sketch_kind != RCLUPP_SKETCH_SRHT)
      return RCLUPP_ERR_INVALID_ARG;
    if (o->tall_lu != RCLUPP_TALL_LU_PARTIAL && o->tall_lu != RCLUPP_TALL_LU_TOURNAMENT) return RCLUPP_ERR_INVALID_ARG;
    if (o->tall_lu == RCLUPP_TALL_LU_TOURNAMENT && uses_tall_lu(alg) && n > 128) return RCLUPP_ERR_UNSUPPORTED;
    if (o->sketch_kind == RCLUPP_SKETCH_COUNT && sketched(alg)) {
      if (o->sketch_prec != RCLUPP_PREC_FP64) return RCLUPP_ERR_UNSUPPORTED;
      if (plan_countsketch(m, n, s, 0).nn == 0) return RCLUPP_ERR_UNSUPPORTED;
    }
  }
  return RCLUPP_OK;
}

// Grid hints: 0 = the planners' defaults (or the RCLUPP_TALL_GRID /
// RCLUPP_SKETCH_GRID environment overrides); a positive value fixes the number
// of workgroups of the tall passes or of the sketch, which sets the number of
// per-workgroup partial sums kept in the workspace.
Layout make_layout(int alg, int64_t m, int64_t n, int64_t s, const rclupp_opts* o, int tall_grid = 0,
                   int sketch_grid = 0) {
  Layout L;
  const int sk_prec = o ? o->sketch_prec : 0;
  L.tp = plan_tall(m, n, tall_grid > 0 ? tall_grid : env_int("RCLUPP_TALL_GRID", 0));
  const int np = L.tp.np;
  const size_t rbytes = align_up(padded_r_doubles(np) * sizeof(double));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(bytes);
    return at;
  };
  L.info = take(sizeof(rclupp_info));
  L.gates = take(3 * sizeof(rclupp_info));
  if (sketched(alg)) {
    const int grid_hint = sketch_grid > 0 ? sketch_grid : env_int("RCLUPP_SKETCH_GRID", 0);
    L.sk = (o && o->sketch_kind == RCLUPP_SKETCH_COUNT) ? plan_countsketch(m, n, s, grid_hint)
                                                        : plan_sketch(m, n, s, sk_prec, grid_hint);
    if (o && o->sketch_kind == RCLUPP_SKETCH_SRHT) L.sk.kind = 2;
    L.ypart = take(L.sk.part_bytes);
    L.y = take((size_t)s * n * sizeof(double));
  }
  L.r1 = take(rbytes);
  L.r2 = take(rbytes);
  L.r3 = take(rbytes);
  L.r4 = take(rbytes);
  L.gpart = take(L.tp.part_bytes);
  L.g = take((size_t)np * np * sizeof(double));
  size_t small = chol_scratch_bytes(n);
  if (sketched(alg)) {
    const size_t pc = precond_scratch_bytes(s, n);
    if (pc > small) small = pc;
  }
  L.small = take(small);
  if (uses_tall_lu(alg)) {
    L.tslu = o && o->tall_lu == RCLUPP_TALL_LU_TOURNAMENT;
    L.perm = take((size_t)(L.tslu ? n : m) * sizeof(int32_t));
    L.nmat = take((size_t)n * n * sizeof(double));
    L.lu = take(L.tslu ? tslu_scratch_bytes(m, n) : tall_lu_scratch_bytes(m, n));
  }
  L.total = off;
  return L;
}

__global__ void k_zero_info(rclupp_info* info) {
  if (threadIdx.x == 0) {
    info->code = 0;
    info->stage = 0;
    info->index = 0;
    info->reserved = 0;
  }
}

#define HIPCHK(expr)                        \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return RCLUPP_ERR_HIP; \
  } while (0)

// ---- optional stage timing: an event is recorded on the stream before every
// stage of rclupp_qr_ex and after its last one (profiling aid, off by default).
struct TraceMark {
  const char* name;  // stage that starts at this mark (nullptr = end of a call)
  hipEvent_t ev;
};
std::mutex g_trace_mu;
bool g_trace_on = false;
std::vector<hipEvent_t> g_trace_pool;
std::vector<TraceMark> g_trace_marks;

void trace_mark(const char* name, hipStream_t st) {
  if (!g_trace_on) return;
  std::lock_guard<std::mutex> lk(g_trace_mu);
  if (g_trace_marks.size() >= g_trace_pool.size()) return;
  hipEvent_t ev = g_trace_pool[g_trace_marks.size()];
  if (hipEventRecord(ev, st) == hipSuccess) g_trace_marks.push_back({name, ev});
}
#define STAGE(name) trace_mark(name, st)

// The CholeskyQR2 tail, Q holds nothing yet: Q_1 = X R_1^{-1} is the first pass.
int tail_cholqr2(const Layout& L, char* ws, const double* X, int64_t m, int64_t n, int64_t ld, double* Q, double* R,
                 int32_t* info, hipStream_t st) {
  double* r1 = (double*)(ws + L.r1);
  double* r2 = (double*)(ws + L.r2);
  double* r3 = (double*)(ws + L.r3);
  double* r4 = (double*)(ws + L.r4);
  double* gpart = (double*)(ws + L.gpart);
  double* g = (double*)(ws + L.g);
  double* small = (double*)(ws + L.small);
  const int np = L.tp.np;
  STAGE("trsm_gram");
  HIPCHK(launch_tall_pass(L.tp, X, ld, m, n, r1, Q, ld, gpart, info, st));
  STAGE("gram_reduce");
  HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, info, st));
  STAGE("chol");
  HIPCHK(launch_chol(g, np, n, m, 0, r2, r3, 0, r1, nullptr, 0, small, info, RCLUPP_STAGE_CHOL_A, st));
  STAGE("trsm_gram");
  HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, r2, Q, ld, gpart, info, st));
  STAGE("gram_reduce");
  HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, info, st));
  STAGE("chol");
  HIPCHK(launch_chol(g, np, n, m, 0, r4, R, 1, r3, nullptr, 0, small, info, RCLUPP_STAGE_CHOL_B, st));
  STAGE("trsm_final");
  HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, r4, Q, ld, nullptr, info, st));
  return RCLUPP_OK;
}

// One CholeskyQR step after the preconditioner (Algorithms 3, 5, 6).
int tail_cholqr1(const Layout& L, char* ws, const double* X, int64_t m, int64_t n, int64_t ld, double* Q, double* R,
                 int32_t* info, hipStream_t st) {
  double* r1 = (double*)(ws + L.r1);
  double* r2 = (double*)(ws + L.r2);
  double* gpart = (double*)(ws + L.gpart);
  double* g = (double*)(ws + L.g);
  double* small = (double*)(ws + L.small);
  const int np = L.tp.np;
  STAGE("trsm_gram");
  HIPCHK(launch_tall_pass(L.tp, X, ld, m, n, r1, Q, ld, gpart, info, st));
  STAGE("gram_reduce");
  HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, info, st));
  STAGE("chol");
  HIPCHK(launch_chol(g, np, n, m, 0, r2, R, 1, r1, nullptr, 0, small, info, RCLUPP_STAGE_CHOL_A, st));
  STAGE("trsm_final");
  HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, r2, Q, ld, nullptr, info, st));
  return RCLUPP_OK;
}

// ---- escalation of the mixed-precision forms ------------------------------------
// An FP32 or BF16 sketch rounds X (or M) before the product, so R_1 is the R
// factor of a perturbed matrix and kappa(Q_1) grows like kappa(X) times the
// rounding unit of the sketch (about 2^-9 kappa(X) for BF16). Past CholeskyQR2's
// range (Lemma 3.1) the first Cholesky breaks down, or its factor spans many
// orders of magnitude. Then the tail takes Algorithm 4's shifted Cholesky of
// G_1 instead (which always succeeds for kappa(Q_1) up to about u^{-1}) and one
// more CholeskyQR pass, i.e. Shifted CholeskyQR3 applied to Q_1. The decision
// is taken on the device: the stages it controls are launched every time and
// return at once when their gate record is closed, so the launch sequence is
// fixed (graph-capturable). info->reserved bit 0 records that it happened.
constexpr int32_t kGateClosed = -1;      // a gate record that makes its stages return at once
// max/min diag(R_2) (a lower bound of kappa(Q_1)) beyond which the tail
// escalates even though the Cholesky did not break down. Measured on the SVD
// family (n = 64 and 256, FP32 and BF16 sketches): whenever the first Cholesky
// succeeded, CholeskyQR2 was accurate (orthogonality near 1e-14), up to a
// ratio of 1.1e8 (kappa(R_2) = 4e8); past that the Cholesky broke down. The
// bound is a safety margin above that range, not a tuned switch.
constexpr double kEscalateRatio = 1e9;

__global__ void k_gate_copy(const rclupp_info* info, rclupp_info* g) {
  if (threadIdx.x == 0) *g = *info;
}

// After the unshifted Cholesky of G_1 (outcome gA, factor in the padded
// triangle r2): open gate gS for the shifted Cholesky when gA reports a
// breakdown or diag(R_2) spans more than `ratio`; any other failure of gA
// becomes the call's outcome. One wave.
__global__ void k_escalate_decide(rclupp_info* info, const rclupp_info* gA, rclupp_info* gS, const double* r2, int np,
                                  int n, double ratio) {
  const int t = threadIdx.x;
  double mx = 0.0, mn = __builtin_inf();
  for (int j = t; j < n; j += 64) {
    const double d = r2[(size_t)j * np + j];
    mx = fmax(mx, d);
    mn = fmin(mn, d);
  }
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o));
    mn = fmin(mn, __shfl_xor(mn, o));
  }
  if (t != 0) return;
  *gS = rclupp_info{kGateClosed, 0, 0, 0};
  if (info->code != 0) return;
  const bool broke = gA->code == RCLUPP_INFO_CHOL_BREAKDOWN;
  const bool weak = gA->code == 0 && !(mx <= ratio * mn);
  if (broke || weak) {
    *gS = rclupp_info{0, 0, 0, 0};
    info->reserved |= 1;
  } else if (gA->code != 0) {
    *info = *gA;
  }
}

// Gate g is open when nothing has failed and the call escalated.
__global__ void k_gate_open(const rclupp_info* info, rclupp_info* g) {
  if (threadIdx.x == 0) {
    const bool run = info->code == 0 && (info->reserved & 1);
    *g = run ? rclupp_info{0, 0, 0, 0} : rclupp_info{kGateClosed, 0, 0, 0};
  }
}

// A failure recorded by the stages behind gate g becomes the call's outcome.
__global__ void k_gate_close(const rclupp_info* g, rclupp_info* info) {
  if (threadIdx.x == 0 && g->code > 0 && info->code == 0) *info = *g;
}

// dst = src (count doubles) when gate g is open.
__global__ void k_copy_gated(const double* src, double* dst, int count, const rclupp_info* g) {
  if (g->code != 0) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

// The CholeskyQR2 tail with the escalation above (mixed-precision forms).
int tail_cholqr2_escalating(const Layout& L, char* ws, const double* X, int64_t m, int64_t n, int64_t ld, double* Q,
                            double* R, int32_t* info32, hipStream_t st) {
  rclupp_info* info = (rclupp_info*)info32;
  rclupp_info* gA = (rclupp_info*)(ws + L.gates);
  rclupp_info* gS = gA + 1;
  rclupp_info* gX = gA + 2;
  double* r1 = (double*)(ws + L.r1);
  double* r2 = (double*)(ws + L.r2);
  double* r3 = (double*)(ws + L.r3);
  double* r4 = (double*)(ws + L.r4);
  double* gpart = (double*)(ws + L.gpart);
  double* g = (double*)(ws + L.g);
  double* small = (double*)(ws + L.small);
  const int np = L.tp.np;
  STAGE("trsm_gram");
  HIPCHK(launch_tall_pass(L.tp, X, ld, m, n, r1, Q, ld, gpart, info32, st));
  STAGE("gram_reduce");
  HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, info32, st));
  STAGE("chol");
  hipLaunchKernelGGL(k_gate_copy, dim3(1), dim3(64), 0, st, info, gA);
  HIPCHK(hipGetLastError());
  HIPCHK(launch_chol(g, np, n, m, 0, r2, r3, 0, r1, nullptr, 0, small, (int32_t*)gA, RCLUPP_STAGE_CHOL_A, st));
  hipLaunchKernelGGL(k_escalate_decide, dim3(1), dim3(64), 0, st, info, gA, gS, r2, np, (int)n, kEscalateRatio);
  HIPCHK(hipGetLastError());
  HIPCHK(launch_chol(g, np, n, m, 1, r2, r3, 0, r1, nullptr, 0, small, (int32_t*)gS, RCLUPP_STAGE_CHOL_A, st));
  hipLaunchKernelGGL(k_gate_close, dim3(1), dim3(64), 0, st, gS, info);
  HIPCHK(hipGetLastError());
  STAGE("trsm_gram");
  HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, r2, Q, ld, gpart, info32, st));
  STAGE("gram_reduce");
  HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, info32, st));
  // the extra CholeskyQR pass (gate gX): R_x = chol(G_2), R_3 <- R_x R_3, Q <- Q R_x^{-1}, G
  STAGE("escalation");
  hipLaunchKernelGGL(k_gate_open, dim3(1), dim3(64), 0, st, info, gX);
  HIPCHK(hipGetLastError());
  HIPCHK(launch_chol(g, np, n, m, 0, r2, r4, 0, r3, nullptr, 0, small, (int32_t*)gX, RCLUPP_STAGE_CHOL_X, st));
  HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, r2, Q, ld, gpart, (int32_t*)gX, st));
  HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, (int32_t*)gX, st));
  const int pad_count = (int)padded_r_doubles(np);
  hipLaunchKernelGGL(k_copy_gated, dim3((pad_count + 255) / 256), dim3(256), 0, st, r4, r3, pad_count, gX);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_gate_close, dim3(1), dim3(64), 0, st, gX, info);
  HIPCHK(hipGetLastError());
  STAGE("chol");
  HIPCHK(launch_chol(g, np, n, m, 0, r4, R, 1, r3, nullptr, 0, small, info32, RCLUPP_STAGE_CHOL_B, st));
  STAGE("trsm_final");
  HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, r4, Q, ld, nullptr, info32, st));
  return RCLUPP_OK;
}

int sketch_into(const Layout& L, char* ws, const double* A, int64_t m, int64_t n, int64_t lda, int64_t s,
                uint64_t seed, int prec, int32_t* info, hipStream_t st) {
  double* ypart = (double*)(ws + L.ypart);
  double* y = (double*)(ws + L.y);
  STAGE("sketch");
  if (L.sk.kind == 1) {
    HIPCHK(launch_countsketch_partials(L.sk, A, m, n, lda, s, seed, ypart, info, st));
    STAGE("sketch_reduce");
    HIPCHK(launch_sketch_reduce(L.sk, ypart, s, n, 1.0, y, info, st));
    return RCLUPP_OK;
  }
  HIPCHK(launch_sketch_partials(L.sk, A, m, n, lda, seed, prec, ypart, info, st));
  STAGE("sketch_reduce");
  HIPCHK(launch_sketch_reduce(L.sk, ypart, s, n, 1.0 / std::sqrt((double)s), y, info, st));
  return RCLUPP_OK;
}

// The LU of X for RCLUPPr and LC2: M into Q (pivoted row order for partial
// pivoting, X's row order for tournament pivoting), N into the workspace.
hipError_t tall_lu_into(const Layout& L, char* ws, const double* X, int64_t m, int64_t n, int64_t ld, double* Q,
                        int32_t* info, hipStream_t st) {
  int32_t* perm = (int32_t*)(ws + L.perm);
  double* nmat = (double*)(ws + L.nmat);
  if (L.tslu) return launch_tslu(X, m, n, ld, Q, ld, perm, nmat, (double*)(ws + L.lu), info, st);
  hipError_t e = launch_tall_lu(X, m, n, ld, Q, ld, perm, nmat, (double*)(ws + L.lu), info, st);
  if (e != hipSuccess) return e;
  return launch_unit_lower(Q, m, n, ld, info, st);
}

int run_method(int alg, const Layout& L, char* ws, const double* X, int64_t m, int64_t n, int64_t ld, int64_t s,
               uint64_t seed, double* Q, double* R, const rclupp_opts* o, int32_t* info, hipStream_t st) {
  const int sk_prec = o ? o->sketch_prec : 0;
  const int lu_prec = o ? o->lu_prec : 0;
  const int np = L.tp.np;
  double* r1 = (double*)(ws + L.r1);
  double* gpart = (double*)(ws + L.gpart);
  double* g = (double*)(ws + L.g);
  double* small = (double*)(ws + L.small);
  // reduced-precision preconditioners take the escalating tail
  auto tail2 = (sk_prec != RCLUPP_PREC_FP64 || lu_prec != RCLUPP_PREC_FP64) ? tail_cholqr2_escalating : tail_cholqr2;
  int rc;
  switch (alg) {
    case RCLUPP_ALG_RCLUPP:
      if ((rc = sketch_into(L, ws, X, m, n, ld, s, seed, sk_prec, info, st))) return rc;
      STAGE("precond");
      HIPCHK(launch_precond((double*)(ws + L.y), s, n, 1, lu_prec, nullptr, 0, r1, nullptr, nullptr, nullptr, small,
                            info, RCLUPP_STAGE_QR, st));
      return tail2(L, ws, X, m, n, ld, Q, R, info, st);
    case RCLUPP_ALG_RCHOLQR:
      if ((rc = sketch_into(L, ws, X, m, n, ld, s, seed, sk_prec, info, st))) return rc;
      STAGE("precond");
      HIPCHK(launch_precond((double*)(ws + L.y), s, n, 0, lu_prec, nullptr, 0, r1, nullptr, nullptr, nullptr, small,
                            info, RCLUPP_STAGE_QR, st));
      return tail_cholqr1(L, ws, X, m, n, ld, Q, R, info, st);
    case RCLUPP_ALG_RCLUPPR: {
      double* nmat = (double*)(ws + L.nmat);
      STAGE("tall_lu");
      HIPCHK(tall_lu_into(L, ws, X, m, n, ld, Q, info, st));
      if ((rc = sketch_into(L, ws, Q, m, n, ld, s, seed, sk_prec, info, st))) return rc;
      STAGE("precond");
      HIPCHK(launch_precond((double*)(ws + L.y), s, n, 0, lu_prec, nmat, n, r1, nullptr, nullptr, nullptr, small, info,
                            RCLUPP_STAGE_QR, st));
      return tail2(L, ws, X, m, n, ld, Q, R, info, st);
    }
    case RCLUPP_ALG_CHOLQR2:
      STAGE("gram");
      HIPCHK(launch_tall_pass(L.tp, X, ld, m, n, nullptr, nullptr, ld, gpart, info, st));
      STAGE("gram_reduce");
      HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, info, st));
      STAGE("chol");
      HIPCHK(launch_chol(g, np, n, m, 0, r1, nullptr, 0, nullptr, nullptr, 0, small, info, RCLUPP_STAGE_PRECOND, st));
      return tail_cholqr1(L, ws, X, m, n, ld, Q, R, info, st);
    case RCLUPP_ALG_SCHOLQR3:
      STAGE("gram");
      HIPCHK(launch_tall_pass(L.tp, X, ld, m, n, nullptr, nullptr, ld, gpart, info, st));
      STAGE("gram_reduce");
      HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, info, st));
      STAGE("chol");
      HIPCHK(launch_chol(g, np, n, m, 1, r1, nullptr, 0, nullptr, nullptr, 0, small, info, RCLUPP_STAGE_PRECOND, st));
      return tail_cholqr2(L, ws, X, m, n, ld, Q, R, info, st);
    case RCLUPP_ALG_LC2: {
      double* nmat = (double*)(ws + L.nmat);
      STAGE("tall_lu");
      HIPCHK(tall_lu_into(L, ws, X, m, n, ld, Q, info, st));
      STAGE("gram");
      HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, nullptr, nullptr, ld, gpart, info, st));
      STAGE("gram_reduce");
      HIPCHK(launch_gram_reduce(L.tp, gpart, n, g, info, st));
      STAGE("chol");
      HIPCHK(launch_chol(g, np, n, m, 0, r1, nullptr, 0, nullptr, nmat, n, small, info, RCLUPP_STAGE_QR, st));
      return tail_cholqr1(L, ws, X, m, n, ld, Q, R, info, st);
    }
    default:
      return RCLUPP_ERR_INVALID_ARG;
  }
}

// ---- allocation-free form: the device address of noalloc_ws per device ------------
std::mutex g_noalloc_mu;
std::map<int, char*> g_noalloc_addr;

// Looked up once per device, with that device current (the caller's).
int noalloc_scratch(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RCLUPP_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_addr.find(dev);
  if (it == g_noalloc_addr.end()) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_ws)) != hipSuccess || p == nullptr) return RCLUPP_ERR_HIP;
    if (((uintptr_t)p) % kAlign) return RCLUPP_ERR_HIP;
    it = g_noalloc_addr.emplace(dev, (char*)p).first;
  }
  *out = it->second;
  return RCLUPP_OK;
}

// ---- per-stream outcome of the 9-argument forms ---------------------------------
std::mutex g_mu;
std::map<hipStream_t, rclupp_info*> g_last;

rclupp_info* last_slot(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_last.find(st);
  if (it != g_last.end()) return it->second;
  rclupp_info* p = nullptr;
  if (hipHostMalloc((void**)&p, sizeof(rclupp_info), hipHostMallocDefault) != hipSuccess) return nullptr;
  std::memset(p, 0, sizeof(rclupp_info));
  g_last[st] = p;
  return p;
}

int simple_entry(int alg, const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q,
                 double* R, hipStream_t st) {
  int rc = validate(alg, m, n, ld, s, nullptr);
  if (rc) return rc;
  if (!X || !Q || !R) return RCLUPP_ERR_INVALID_ARG;
  size_t bytes = 0;
  rc = rclupp_workspace_size(alg, m, n, s, nullptr, &bytes);
  if (rc) return rc;
  rclupp_info* slot = last_slot(st);
  if (!slot) return RCLUPP_ERR_ALLOC;
  void* ws = nullptr;
  if (hipMallocAsync(&ws, bytes, st) != hipSuccess) return RCLUPP_ERR_ALLOC;
  rclupp_info* d_info = (rclupp_info*)((char*)ws + make_layout(alg, m, n, s, nullptr).info);
  rc = rclupp_qr_ex(alg, X, m, n, ld, s, seed, Q, R, nullptr, ws, bytes, d_info, st);
  if (rc == RCLUPP_OK) {
    if (hipMemcpyAsync(slot, d_info, sizeof(rclupp_info), hipMemcpyDeviceToHost, st) != hipSuccess) rc = RCLUPP_ERR_HIP;
  }
  if (hipFreeAsync(ws, st) != hipSuccess && rc == RCLUPP_OK) rc = RCLUPP_ERR_HIP;
  return rc;
}

// Clears the outcome record and enqueues method `alg` in the workspace `w`
// (laid out by L) on `st`.
int run_in_workspace(int alg, const Layout& L, char* w, const double* X, int64_t m, int64_t n, int64_t ld, int64_t s,
                     uint64_t seed, double* Q, double* R, const rclupp_opts* opts, rclupp_info* d_info,
                     hipStream_t st) {
  rclupp_info* info = d_info ? d_info : (rclupp_info*)(w + L.info);
  hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(64), 0, st, info);
  if (hipGetLastError() != hipSuccess) return RCLUPP_ERR_HIP;
  const int rc = run_method(alg, L, w, X, m, n, ld, s, seed, Q, R, opts, (int32_t*)info, st);
  trace_mark(nullptr, st);
  return rc;
}

// The layout of rclupp_qr_ex for these sizes, with the number of per-workgroup
// partial sums (the grid of the sketch, then of the Gram passes, whichever
// holds more bytes) halved until the whole workspace fits in `cap` bytes. The
// passes without a Gram keep their own grid (they keep no partials). False if
// nothing fits (e.g. the m-long pivot vector of the tall LU).
bool fit_layout(int alg, int64_t m, int64_t n, int64_t s, const rclupp_opts* o, size_t cap, Layout* out) {
  Layout L = make_layout(alg, m, n, s, o);
  const int solve_grid = L.tp.gx_solve;
  int tall_grid = L.tp.gx;
  int sketch_grid = 0;
  while (L.total > cap) {
    const size_t sb = sketched(alg) ? L.sk.part_bytes : 0;
    // (the Gaussian plan reads its hint as workgroups in all, the CountSketch
    // plan as row chunks)
    const int sk_half = L.sk.kind == 1 ? L.sk.gx / 2 : (L.sk.gx / 2) * L.sk.gy * L.sk.gz;
    if (sketched(alg) && sb >= L.tp.part_bytes && L.sk.gx > 1) {
      sketch_grid = sk_half;
    } else if (L.tp.gx > 1) {
      tall_grid = L.tp.gx / 2;
    } else if (sketched(alg) && L.sk.gx > 1) {
      sketch_grid = sk_half;
    } else {
      return false;
    }
    L = make_layout(alg, m, n, s, o, tall_grid, sketch_grid);
  }
  L.tp.gx_solve = solve_grid;
  *out = L;
  return true;
}

template <typename F>
int with_scratch(size_t bytes, hipStream_t st, F&& f) {
  void* p = nullptr;
  if (bytes == 0) bytes = kAlign;
  if (hipMallocAsync(&p, bytes, st) != hipSuccess) return RCLUPP_ERR_ALLOC;
  int rc = f((char*)p);
  if (hipFreeAsync(p, st) != hipSuccess && rc == RCLUPP_OK) rc = RCLUPP_ERR_HIP;
  return rc;
}

}  // namespace

extern "C" {

const char* rclupp_status_string(int status) {
  switch (status) {
    case RCLUPP_OK: return "ok";
    case RCLUPP_ERR_INVALID_ARG: return "invalid argument";
    case RCLUPP_ERR_UNSUPPORTED: return "unsupported size or option";
    case RCLUPP_ERR_ALLOC: return "device allocation failed";
    case RCLUPP_ERR_HIP: return "HIP runtime or launch error";
    case RCLUPP_ERR_WORKSPACE: return "workspace too small";
    case RCLUPP_ERR_SCRATCH_LIMIT: return "sizes need more than the fixed scratch of rclupp_qr_noalloc";
    default: return "unknown status";
  }
}

int rclupp_workspace_size(int alg, int64_t m, int64_t n, int64_t s, const rclupp_opts* opts, size_t* bytes) {
  if (!bytes) return RCLUPP_ERR_INVALID_ARG;
  int rc = validate(alg, m, n, m, s, opts);
  if (rc) return rc;
  *bytes = make_layout(alg, m, n, s, opts).total;
  return RCLUPP_OK;
}

int rclupp_qr_ex(int alg, const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q,
                 double* R, const rclupp_opts* opts, void* ws, size_t ws_bytes, rclupp_info* d_info,
                 hipStream_t stream) {
  int rc = validate(alg, m, n, ld, s, opts);
  if (rc) return rc;
  if (!X || !Q || !R || !ws) return RCLUPP_ERR_INVALID_ARG;
  if (((uintptr_t)ws) % kAlign) return RCLUPP_ERR_INVALID_ARG;
  const Layout L = make_layout(alg, m, n, s, opts);
  if (ws_bytes < L.total) return RCLUPP_ERR_WORKSPACE;
  return run_in_workspace(alg, L, (char*)ws, X, m, n, ld, s, seed, Q, R, opts, d_info, stream);
}

int rclupp_qr_noalloc(int alg, const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed,
                      double* Q, double* R, const rclupp_opts* opts, rclupp_info* d_info, hipStream_t stream) {
  int rc = validate(alg, m, n, ld, s, opts);
  if (rc) return rc;
  if (!X || !Q || !R) return RCLUPP_ERR_INVALID_ARG;
  Layout L;
  if (!fit_layout(alg, m, n, s, opts, RCLUPP_NOALLOC_MAX_BYTES, &L)) return RCLUPP_ERR_SCRATCH_LIMIT;
  char* w = nullptr;
  if ((rc = noalloc_scratch(&w))) return rc;
  return run_in_workspace(alg, L, w, X, m, n, ld, s, seed, Q, R, opts, d_info, stream);
}

int rclupp_trace_enable(int max_marks) {
  std::lock_guard<std::mutex> lk(g_trace_mu);
  g_trace_marks.clear();
  if (max_marks <= 0) {
    g_trace_on = false;
    return RCLUPP_OK;
  }
  while ((int)g_trace_pool.size() < max_marks) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return RCLUPP_ERR_HIP;
    g_trace_pool.push_back(ev);
  }
  g_trace_on = true;
  return RCLUPP_OK;
}

int rclupp_trace_read(int max_stages, char* names, int name_len, float* ms, int* launches, int* count) {
  if (!count || (max_stages > 0 && (!names || !ms || !launches || name_len < 2))) return RCLUPP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_trace_mu);
  std::vector<std::string> keys;
  std::vector<float> tot;
  std::vector<int> cnt;
  for (size_t i = 0; i + 1 < g_trace_marks.size(); ++i) {
    if (!g_trace_marks[i].name) continue;
    if (hipEventSynchronize(g_trace_marks[i + 1].ev) != hipSuccess) return RCLUPP_ERR_HIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_trace_marks[i].ev, g_trace_marks[i + 1].ev) != hipSuccess) return RCLUPP_ERR_HIP;
    size_t k = 0;
    while (k < keys.size() && keys[k] != g_trace_marks[i].name) ++k;
    if (k == keys.size()) {
      keys.push_back(g_trace_marks[i].name);
      tot.push_back(0.f);
      cnt.push_back(0);
    }
    tot[k] += t;
    cnt[k] += 1;
  }
  *count = (int)keys.size();
  for (int k = 0; k < (int)keys.size() && k < max_stages; ++k) {
    std::strncpy(names + (size_t)k * name_len, keys[k].c_str(), (size_t)name_len - 1);
    names[(size_t)k * name_len + name_len - 1] = 0;
    ms[k] = tot[k];
    launches[k] = cnt[k];
  }
  g_trace_marks.clear();
  return RCLUPP_OK;
}

int rclupp_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
              hipStream_t stream) {
  return simple_entry(RCLUPP_ALG_RCLUPP, X, m, n, ld, s, seed, Q, R, stream);
}
int rcluppr_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
               hipStream_t stream) {
  return simple_entry(RCLUPP_ALG_RCLUPPR, X, m, n, ld, s, seed, Q, R, stream);
}
int cholqr2_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
               hipStream_t stream) {
  return simple_entry(RCLUPP_ALG_CHOLQR2, X, m, n, ld, s, seed, Q, R, stream);
}
int scholqr3_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
                hipStream_t stream) {
  return simple_entry(RCLUPP_ALG_SCHOLQR3, X, m, n, ld, s, seed, Q, R, stream);
}
int lc2_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
           hipStream_t stream) {
  return simple_entry(RCLUPP_ALG_LC2, X, m, n, ld, s, seed, Q, R, stream);
}
int rcholqr_qr(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Q, double* R,
               hipStream_t stream) {
  return simple_entry(RCLUPP_ALG_RCHOLQR, X, m, n, ld, s, seed, Q, R, stream);
}

int rclupp_last_info(hipStream_t stream, rclupp_info* h_info) {
  if (!h_info) return RCLUPP_ERR_INVALID_ARG;
  rclupp_info* slot = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_last.find(stream);
    if (it == g_last.end()) return RCLUPP_ERR_INVALID_ARG;
    slot = it->second;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return RCLUPP_ERR_HIP;
  *h_info = *slot;
  return RCLUPP_OK;
}

}  // extern "C"

namespace {

// ---- batched ----------------------------------------------------------------------
// RCLUPP problems are grouped by (n, s). Every stage of the pipeline is one
// launch per group over all its problems (workgroup -> (problem, chunk) items;
// the small stages take one workgroup per problem), so a batch of any size is a
// fixed, short launch sequence. With RCLUPP_BATCH_GRAPH that sequence is
// captured once into a hipGraph (keyed by the call's arguments) and replayed;
// with RCLUPP_BATCH_AUTOTUNE the rows per workgroup of the tall and sketch
// passes are chosen per batch shape by timing the candidates once. Other
// methods, and shapes beyond the register-resident small kernels, run one
// problem after another with the single-problem pipeline.
// Tuning knobs of a grouped batch: tall tiles (64 or 128 rows) per workgroup
// of the tall passes, and 32-row tiles per workgroup of the sketch.
struct BatchTune {
  int tall_tpw;
  int sk_tpw;
};
// (more tiles per workgroup: fewer per-workgroup partial sums to write and
// add, each s_pad x n_pad or np x np doubles; fewer: more parallelism for the
// short problems)
constexpr int kTuneTall[] = {4, 8, 16, 32, 64};
constexpr int kTuneSketch[] = {16, 32, 64, 128, 256, 512, 1024};
constexpr int kNumTuneTall = (int)(sizeof(kTuneTall) / sizeof(kTuneTall[0]));
constexpr int kNumTuneSketch = (int)(sizeof(kTuneSketch) / sizeof(kTuneSketch[0]));
constexpr BatchTune kDefaultTune = {8, 32};

struct BatchProbPlan {
  int b;             // index in the caller's array
  SketchPlan sk;     // this problem's sketch partition
  int64_t tiles;     // tall tiles
  int tall_wg;       // tall workgroups
  size_t ypart, y, r1, r2, r3, r4, gpart, g, scratch;  // workspace offsets
};
struct BatchGroupPlan {
  int64_t n, s;
  int np;
  std::vector<BatchProbPlan> probs;
};
struct BatchPlan {
  std::vector<BatchGroupPlan> groups;
  size_t table_off = 0, table_bytes = 0, info_off = 0, total = 0;
  bool grouped = false;
};

bool batch_groupable(int alg, const rclupp_problem* h, int batch, const rclupp_opts* o) {
  if (alg != RCLUPP_ALG_RCLUPP || batch <= 0) return false;
  if (o && o->sketch_kind != RCLUPP_SKETCH_GAUSSIAN) return false;
  for (int b = 0; b < batch; ++b)
    if (!precond_reg_fits(h[b].s, h[b].n)) return false;
  return true;
}

int64_t tall_tiles(int64_t m, int np) { return (m + (np > 128 ? 64 : 128) - 1) / (np > 128 ? 64 : 128); }

BatchPlan make_batch_plan(const rclupp_problem* h, int batch, const rclupp_opts* o, BatchTune tune) {
  const int tpw = tune.tall_tpw;
  BatchPlan P;
  const int prec = o ? o->sketch_prec : 0;
  std::map<std::pair<int64_t, int64_t>, int> gi;
  for (int b = 0; b < batch; ++b) {
    auto key = std::make_pair(h[b].n, h[b].s);
    auto it = gi.find(key);
    if (it == gi.end()) {
      gi[key] = (int)P.groups.size();
      BatchGroupPlan g;
      g.n = h[b].n;
      g.s = h[b].s;
      g.np = pad_cols(h[b].n);
      P.groups.push_back(g);
      it = gi.find(key);
    }
    BatchProbPlan pp{};
    pp.b = b;
    pp.sk = plan_sketch(h[b].m, h[b].n, h[b].s, prec, 0);
    int64_t skw = (pp.sk.ntiles + tune.sk_tpw - 1) / tune.sk_tpw;
    if (skw > 1024) skw = 1024;
    pp.sk.gx = (int)(skw < 1 ? 1 : skw);
    pp.sk.part_bytes = ((size_t)pp.sk.gx + reduce_splits(pp.sk.gx)) * pp.sk.s_pad * pp.sk.n_pad * sizeof(double);
    pp.tiles = tall_tiles(h[b].m, P.groups[it->second].np);
    int64_t tw = (pp.tiles + tpw - 1) / tpw;
    if (tw > 1024) tw = 1024;
    pp.tall_wg = (int)(tw < 1 ? 1 : tw);
    P.groups[it->second].probs.push_back(pp);
  }
  // workspace: per-problem regions, then the per-problem info records (when
  // the caller passes none), then the job tables
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(bytes);
    return at;
  };
  for (auto& g : P.groups) {
    const size_t rb = padded_r_doubles(g.np) * sizeof(double);
    for (auto& pp : g.probs) {
      pp.ypart = take(pp.sk.part_bytes);
      pp.y = take((size_t)g.s * g.n * sizeof(double));
      pp.r1 = take(rb);
      pp.r2 = take(rb);
      pp.r3 = take(rb);
      pp.r4 = take(rb);
      pp.gpart = take(((size_t)pp.tall_wg + reduce_splits(pp.tall_wg)) * g.np * g.np * sizeof(double));
      pp.g = take((size_t)g.np * g.np * sizeof(double));
      pp.scratch = g.n > 64 ? take(precond_reg_scratch_bytes()) : 0;
    }
  }
  P.info_off = take((size_t)batch * sizeof(rclupp_info));
  // tables (upper bound: every group's arrays, see build_tables)
  size_t tb = 0;
  for (auto& g : P.groups) {
    size_t items = 0, cnt = g.probs.size();
    for (auto& pp : g.probs) items += 2 * (size_t)pp.sk.gx + 2 * (size_t)pp.tall_wg + 64 * 4;
    tb += items * sizeof(BatchItem) + cnt * (sizeof(SketchJob) + 3 * sizeof(ReduceJob) + sizeof(PrecondJob) +
                                             3 * sizeof(TallJob) + 2 * sizeof(CholJob)) + 16 * kAlign;
  }
  P.table_bytes = tb;
  P.table_off = take(tb);
  P.total = off;
  P.grouped = true;
  return P;
}

// Host image of the job tables of one group, at its offsets in the table area.
struct GroupTables {
  size_t sk_jobs, sk_items, ysum_jobs, ysum_items, pc_jobs, t1, t2, t3, t_items, g_jobs, g_items, c1, c2;
  int n_sk_items, n_ysum_items, n_t_items, n_g_items;
};

template <typename T>
size_t put(std::vector<unsigned char>& img, size_t& at, const std::vector<T>& v) {
  const size_t o = at;
  const size_t bytes = v.size() * sizeof(T);
  if (o + bytes > img.size()) img.resize(o + bytes);
  if (bytes) std::memcpy(img.data() + o, v.data(), bytes);
  at = align_up(o + bytes);
  return o;
}

std::vector<GroupTables> build_tables(const BatchPlan& P, const rclupp_problem* h, char* ws, rclupp_info* infos,
                                      std::vector<unsigned char>& img) {
  std::vector<GroupTables> out;
  size_t at = 0;
  for (const auto& g : P.groups) {
    GroupTables T{};
    std::vector<SketchJob> skj;
    std::vector<BatchItem> ski, ysi, ti, gii;
    std::vector<ReduceJob> ysj, gj;
    std::vector<PrecondJob> pcj;
    std::vector<TallJob> t1, t2, t3;
    std::vector<CholJob> c1, c2;
    const int64_t sz = g.np;
    for (size_t k = 0; k < g.probs.size(); ++k) {
      const BatchProbPlan& pp = g.probs[k];
      const rclupp_problem& p = h[pp.b];
      int32_t* info = (int32_t*)(infos + pp.b);
      double* ypart = (double*)(ws + pp.ypart);
      double* y = (double*)(ws + pp.y);
      double* r1 = (double*)(ws + pp.r1);
      double* r2 = (double*)(ws + pp.r2);
      double* r3 = (double*)(ws + pp.r3);
      double* r4 = (double*)(ws + pp.r4);
      double* gpart = (double*)(ws + pp.gpart);
      double* gm = (double*)(ws + pp.g);
      double* scr = pp.scratch ? (double*)(ws + pp.scratch) : nullptr;
      const int pk = (int)k;
      skj.push_back({p.X, p.m, p.ld, pp.sk.ntiles, p.seed, ypart, info});
      for (int w = 0; w < pp.sk.gx; ++w) ski.push_back({pk, w, pp.sk.gx, 0});
      const int ysp = reduce_splits(pp.sk.gx);
      const int64_t ystride = pp.sk.s_pad * pp.sk.n_pad;
      ysj.push_back({ypart, ypart + (int64_t)pp.sk.gx * ystride, y, pp.sk.gx, ysp, info});
      for (int w = 0; w < ysp; ++w) ysi.push_back({pk, w, ysp, 0});
      pcj.push_back({y, r1, scr, info});
      t1.push_back({p.X, p.ld, p.m, pp.tiles, r1, p.Q, p.ld, gpart, info});
      t2.push_back({p.Q, p.ld, p.m, pp.tiles, r2, p.Q, p.ld, gpart, info});
      t3.push_back({p.Q, p.ld, p.m, pp.tiles, r4, p.Q, p.ld, nullptr, info});
      for (int w = 0; w < pp.tall_wg; ++w) ti.push_back({pk, w, pp.tall_wg, 0});
      const int gsp = reduce_splits(pp.tall_wg);
      gj.push_back({gpart, gpart + (int64_t)pp.tall_wg * sz * sz, gm, pp.tall_wg, gsp, info});
      for (int w = 0; w < gsp; ++w) gii.push_back({pk, w, gsp, 0});
      c1.push_back({gm, r2, r3, r1, info, p.m});
      c2.push_back({gm, r4, p.R, r3, info, p.m});
    }
    T.sk_jobs = put(img, at, skj);
    T.sk_items = put(img, at, ski);
    T.ysum_jobs = put(img, at, ysj);
    T.ysum_items = put(img, at, ysi);
    T.pc_jobs = put(img, at, pcj);
    T.t1 = put(img, at, t1);
    T.t2 = put(img, at, t2);
    T.t3 = put(img, at, t3);
    T.t_items = put(img, at, ti);
    T.g_jobs = put(img, at, gj);
    T.g_items = put(img, at, gii);
    T.c1 = put(img, at, c1);
    T.c2 = put(img, at, c2);
    T.n_sk_items = (int)ski.size();
    T.n_ysum_items = (int)ysi.size();
    T.n_t_items = (int)ti.size();
    T.n_g_items = (int)gii.size();
    out.push_back(T);
  }
  img.resize(at);
  return out;
}

__global__ void k_zero_infos(rclupp_info* info, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) info[i] = rclupp_info{0, 0, 0, 0};
}

// Side streams of the grouped batch (one set per device, default priority):
// the (n, s) groups are independent, so each runs on its own stream between a
// fork and a join event; one group's small stages (one workgroup per problem)
// then overlap with another group's tall passes. Also inside a captured graph,
// where the events become the branches' dependencies.
constexpr int kSideStreams = 4;
struct SideStreams {
  hipStream_t s[kSideStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSideStreams] = {};
  bool ok = false;  // all created (else the groups run one after another on the caller's stream)
};
std::map<int, SideStreams> g_side;  // guarded by g_batch_mu

SideStreams* side_streams() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  auto it = g_side.find(dev);
  if (it != g_side.end()) return it->second.ok ? &it->second : nullptr;
  SideStreams ss;
  bool ok = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < kSideStreams && ok; ++i) {
    ok = hipStreamCreateWithFlags(&ss.s[i], hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&ss.join[i], hipEventDisableTiming) == hipSuccess;
  }
  ss.ok = ok;
  auto& slot = g_side[dev];
  slot = ss;  // kept (and freed by rclupp_release) even if incomplete
  return ok ? &slot : nullptr;
}

// The launch sequence of a grouped batch (tables already in place on `st`).
int batch_launch(const BatchPlan& P, const std::vector<GroupTables>& GT, char* tab, rclupp_info* infos, int batch,
                 const rclupp_opts* o, hipStream_t st) {
  const int sk_prec = o ? o->sketch_prec : 0;
  const int lu_prec = o ? o->lu_prec : 0;
  hipLaunchKernelGGL(k_zero_infos, dim3((batch + 255) / 256), dim3(256), 0, st, infos, batch);
  HIPCHK(hipGetLastError());
  SideStreams* side = P.groups.size() > 1 ? side_streams() : nullptr;
  if (side) HIPCHK(hipEventRecord(side->fork, st));
  const hipStream_t main_st = st;
  for (size_t gi = 0; gi < P.groups.size(); ++gi) {
    if (side) {
      st = side->s[gi % kSideStreams];
      if (gi < (size_t)kSideStreams) HIPCHK(hipStreamWaitEvent(st, side->fork, 0));
    }
    const BatchGroupPlan& g = P.groups[gi];
    const GroupTables& T = GT[gi];
    const int cnt = (int)g.probs.size();
    const SketchPlan& shape = g.probs[0].sk;
    const int64_t ystride = shape.s_pad * shape.n_pad, gstride = (int64_t)g.np * g.np;
    auto J = [&](size_t off) { return (void*)(tab + off); };
    HIPCHK(launch_sketch_batch(shape, g.n, sk_prec, (const SketchJob*)J(T.sk_jobs), (const BatchItem*)J(T.sk_items),
                               T.n_sk_items, st));
    HIPCHK(launch_partial_sum_batch(ystride, (const ReduceJob*)J(T.ysum_jobs), (const BatchItem*)J(T.ysum_items),
                                    T.n_ysum_items, st));
    HIPCHK(launch_sketch_final_batch(shape, g.s, g.n, 1.0 / std::sqrt((double)g.s), (const ReduceJob*)J(T.ysum_jobs),
                                     cnt, st));
    HIPCHK(launch_precond_batch(g.s, g.n, lu_prec, (const PrecondJob*)J(T.pc_jobs), cnt, RCLUPP_STAGE_QR, st));
    const BatchItem* ti = (const BatchItem*)J(T.t_items);
    const ReduceJob* gj = (const ReduceJob*)J(T.g_jobs);
    const BatchItem* gii = (const BatchItem*)J(T.g_items);
    HIPCHK(launch_tall_batch(g.np, (int)g.n, true, true, true, (const TallJob*)J(T.t1), ti, T.n_t_items, st));
    HIPCHK(launch_partial_sum_batch(gstride, gj, gii, T.n_g_items, st));
    HIPCHK(launch_gram_final_batch(g.np, g.n, gj, cnt, st));
    HIPCHK(launch_chol_batch(g.n, g.np, 0, (const CholJob*)J(T.c1), cnt, RCLUPP_STAGE_CHOL_A, st));
    HIPCHK(launch_tall_batch(g.np, (int)g.n, true, true, true, (const TallJob*)J(T.t2), ti, T.n_t_items, st));
    HIPCHK(launch_partial_sum_batch(gstride, gj, gii, T.n_g_items, st));
    HIPCHK(launch_gram_final_batch(g.np, g.n, gj, cnt, st));
    HIPCHK(launch_chol_batch(g.n, g.np, 1, (const CholJob*)J(T.c2), cnt, RCLUPP_STAGE_CHOL_B, st));
    HIPCHK(launch_tall_batch(g.np, (int)g.n, true, false, true, (const TallJob*)J(T.t3), ti, T.n_t_items, st));
  }
  if (side) {
    const size_t used = P.groups.size() < (size_t)kSideStreams ? P.groups.size() : (size_t)kSideStreams;
    for (size_t i = 0; i < used; ++i) {
      HIPCHK(hipEventRecord(side->join[i], side->s[i]));
      HIPCHK(hipStreamWaitEvent(main_st, side->join[i], 0));
    }
  }
  return RCLUPP_OK;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

// ---- pinned staging of the job tables ---------------------------------------------
// The tables are built on the host and uploaded on the stream, so their pinned
// source must outlive the upload (for a captured graph: every replay). Buffers
// come from a pool and are reused only once the event recorded after their
// last use has completed; that is polled, never waited for. When no buffer is
// free a new one is allocated (hipHostMalloc does not synchronize; hipHostFree
// does, so buffers are freed only by rclupp_release).
struct PinnedBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;  // recorded after the last enqueued use
  bool held = false;          // in use by a call being enqueued or by a cached graph
  bool recorded = false;      // `done` has been recorded at least once
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  PinnedBuf* tables = nullptr;   // pinned image the captured copy reads on every replay
  hipEvent_t launched = nullptr; // recorded after every replay
  bool replayed = false;
  uint64_t tick = 0;             // last use (least recently used entries are evicted first)
};
struct RetiredExec {
  hipGraphExec_t exec;
  hipEvent_t launched;
  bool replayed;
};

std::mutex g_batch_mu;  // guards everything below
std::vector<PinnedBuf*> g_pinned;
std::map<uint64_t, GraphEntry> g_graphs;
std::vector<RetiredExec> g_retired;  // evicted graphs whose last replay may still run
uint64_t g_tick = 0;
std::map<uint64_t, BatchTune> g_tuned;  // (architecture, batch shape) -> tuned knobs
std::map<int, hipStream_t> g_capture_stream;
constexpr size_t kGraphCacheEntries = 16;

PinnedBuf* pinned_acquire(size_t bytes) {
  for (PinnedBuf* b : g_pinned) {
    if (b->held || b->bytes < bytes) continue;
    if (b->recorded && hipEventQuery(b->done) != hipSuccess) continue;  // in flight (or unknown)
    b->held = true;
    return b;
  }
  PinnedBuf* b = new PinnedBuf;
  b->bytes = bytes < 4096 ? 4096 : bytes;
  if (hipHostMalloc(&b->ptr, b->bytes, hipHostMallocDefault) != hipSuccess) {
    delete b;
    return nullptr;
  }
  if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
    g_pinned.push_back(b);  // kept (held) so that rclupp_release frees it
    b->held = true;
    return nullptr;
  }
  b->held = true;
  g_pinned.push_back(b);
  return b;
}

// The buffer becomes reusable once the work enqueued so far on `st` is done.
// If the event cannot be recorded the buffer stays held (never reused).
int pinned_release_after(PinnedBuf* b, hipStream_t st) {
  if (hipEventRecord(b->done, st) != hipSuccess) return RCLUPP_ERR_HIP;
  b->recorded = true;
  b->held = false;
  return RCLUPP_OK;
}

// Destroys the retired graph executables whose last replay has completed.
void reap_retired() {
  for (size_t i = 0; i < g_retired.size();) {
    RetiredExec& r = g_retired[i];
    if (r.replayed && hipEventQuery(r.launched) != hipSuccess) {
      ++i;
      continue;
    }
    (void)hipGraphExecDestroy(r.exec);
    (void)hipEventDestroy(r.launched);
    g_retired[i] = g_retired.back();
    g_retired.pop_back();
  }
}

uint64_t shape_key(const rclupp_problem* h, int batch, const rclupp_opts* o) {
  uint64_t k = 1469598103934665603ull;
  for (int b = 0; b < batch; ++b) {
    const int64_t v[3] = {h[b].n, h[b].s, (h[b].m + 4095) / 4096};
    k = fnv1a(k, v, sizeof(v));
  }
  const int32_t pr[3] = {o ? o->sketch_prec : 0, o ? o->lu_prec : 0, o ? o->sketch_kind : 0};
  return fnv1a(k, pr, sizeof(pr));
}

// Host side of a grouped run: the job tables written into a pinned buffer
// (held by the caller until it releases or hands it to a graph entry).
struct BatchPrep {
  std::vector<GroupTables> gt;
  PinnedBuf* buf = nullptr;
  size_t bytes = 0;
};

int batch_prepare(const BatchPlan& P, const rclupp_problem* h, char* ws, rclupp_info* infos, BatchPrep* out) {
  std::vector<unsigned char> img;
  out->gt = build_tables(P, h, ws, infos, img);
  if (img.size() > P.table_bytes) return RCLUPP_ERR_WORKSPACE;
  out->bytes = img.size() ? img.size() : 1;
  out->buf = pinned_acquire(out->bytes);
  if (!out->buf) return RCLUPP_ERR_ALLOC;
  if (!img.empty()) std::memcpy(out->buf->ptr, img.data(), img.size());
  return RCLUPP_OK;
}

// Stream part of a grouped run: the table upload, then the launch sequence.
int batch_enqueue(const BatchPlan& P, const BatchPrep& prep, int batch, const rclupp_opts* o, char* ws,
                  rclupp_info* infos, hipStream_t st) {
  if (hipMemcpyAsync(ws + P.table_off, prep.buf->ptr, prep.bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return RCLUPP_ERR_HIP;
  return batch_launch(P, prep.gt, ws + P.table_off, infos, batch, o, st);
}

// Enqueues one grouped run (tables, upload, launches) and hands the pinned
// buffer back to the pool behind an event. Called with g_batch_mu held.
int batch_run_once(const BatchPlan& P, const rclupp_problem* h, int batch, const rclupp_opts* o, char* ws,
                   rclupp_info* infos, hipStream_t st) {
  BatchPrep prep;
  int rc = batch_prepare(P, h, ws, infos, &prep);
  if (rc == RCLUPP_OK) rc = batch_enqueue(P, prep, batch, o, ws, infos, st);
  if (prep.buf) {
    const int rr = pinned_release_after(prep.buf, st);
    if (rc == RCLUPP_OK) rc = rr;
  }
  return rc;
}

// ---- persistent tuning cache ------------------------------------------------------
// Tuned knobs are kept in memory and, unless RCLUPP_TUNE_CACHE is "off", in a
// text file (RCLUPP_TUNE_CACHE, else $HOME/.cache/rclupp_batch_tune.txt) with
// one "key tall_tpw sk_tpw" line per batch shape; the key hashes the device's
// architecture name with the shape key (n, s and m in 4096-row buckets per
// problem, the precisions). The file is read once per process and appended to
// after each tuning; any I/O failure leaves the in-memory table in charge.
std::string tune_cache_path() {
  const char* e = std::getenv("RCLUPP_TUNE_CACHE");
  if (e && std::strcmp(e, "off") == 0) return std::string();
  if (e && *e) return std::string(e);
  const char* home = std::getenv("HOME");
  if (!home || !*home) return std::string();
  return std::string(home) + "/.cache/rclupp_batch_tune.txt";
}

bool g_tune_file_read = false;

void tune_cache_load() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  unsigned long long key = 0;
  int a = 0, b = 0;
  auto known = [](int v, const int* c, int nc) {
    for (int i = 0; i < nc; ++i)
      if (c[i] == v) return true;
    return false;
  };
  // only candidate values are taken (the workspace size assumes them)
  while (std::fscanf(f, "%llx %d %d", &key, &a, &b) == 3)
    if (known(a, kTuneTall, kNumTuneTall) && known(b, kTuneSketch, kNumTuneSketch))
      g_tuned[(uint64_t)key] = BatchTune{a, b};
  std::fclose(f);
}

void tune_cache_store(uint64_t key, BatchTune t) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%016llx %d %d\n", (unsigned long long)key, t.tall_tpw, t.sk_tpw);
  std::fclose(f);
}

uint64_t arch_key(uint64_t k) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return k;
  return fnv1a(k, prop.gcnArchName, std::strlen(prop.gcnArchName));
}

// Times one complete grouped run of `t` on `stream` (waits for it); < 0 if the
// plan does not fit the workspace.
int time_candidate(const rclupp_problem* h, int batch, const rclupp_opts* o, char* ws, size_t ws_bytes,
                   rclupp_info* d_info, hipStream_t stream, BatchTune t, hipEvent_t e0, hipEvent_t e1, float* ms) {
  BatchPlan P = make_batch_plan(h, batch, o, t);
  *ms = -1.f;
  if (P.total > ws_bytes) return RCLUPP_OK;
  rclupp_info* infos = d_info ? d_info : (rclupp_info*)(ws + P.info_off);
  if (hipEventRecord(e0, stream) != hipSuccess) return RCLUPP_ERR_HIP;
  int rc = batch_run_once(P, h, batch, o, ws, infos, stream);
  if (rc) return rc;
  if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return RCLUPP_ERR_HIP;
  (void)hipEventElapsedTime(ms, e0, e1);
  return RCLUPP_OK;
}

int batched_grouped(int alg, const rclupp_problem* h, int batch, const rclupp_opts* o, void* ws_v, size_t ws_bytes,
                    rclupp_info* d_info, hipStream_t stream) {
  (void)alg;
  char* ws = (char*)ws_v;
  const int flags = o ? o->batch_flags : 0;
  BatchTune tune = kDefaultTune;
  const uint64_t skey = shape_key(h, batch, o);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  reap_retired();
  if (flags & RCLUPP_BATCH_AUTOTUNE) {
    tune_cache_load();
    const uint64_t tkey = arch_key(skey);
    auto it = g_tuned.find(tkey);
    if (it != g_tuned.end()) {
      tune = it->second;
    } else {
      // coordinate search, one complete batch per candidate (this waits for
      // the stream, as the header states): the tall passes' tiles per
      // workgroup with the default sketch, then the sketch's with that choice
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) != hipSuccess) return RCLUPP_ERR_HIP;
      if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return RCLUPP_ERR_HIP;
      }
      int rc = RCLUPP_OK;
      float best = -1.f;
      BatchTune best_t = kDefaultTune;
      for (int cand : kTuneTall) {
        float ms = 0.f;
        const BatchTune t{cand, kDefaultTune.sk_tpw};
        if ((rc = time_candidate(h, batch, o, ws, ws_bytes, d_info, stream, t, e0, e1, &ms))) break;
        if (ms >= 0.f && (best < 0.f || ms < best)) {
          best = ms;
          best_t = t;
        }
      }
      for (int cand : kTuneSketch) {
        if (rc || cand == best_t.sk_tpw) continue;
        float ms = 0.f;
        const BatchTune t{best_t.tall_tpw, cand};
        if ((rc = time_candidate(h, batch, o, ws, ws_bytes, d_info, stream, t, e0, e1, &ms))) break;
        if (ms >= 0.f && (best < 0.f || ms < best)) {
          best = ms;
          best_t = t;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (rc) return rc;
      tune = best_t;
      g_tuned[tkey] = tune;
      tune_cache_store(tkey, tune);
    }
  }
  BatchPlan P = make_batch_plan(h, batch, o, tune);
  if (P.total > ws_bytes) return RCLUPP_ERR_WORKSPACE;
  rclupp_info* infos = d_info ? d_info : (rclupp_info*)(ws + P.info_off);
  if (!(flags & RCLUPP_BATCH_GRAPH)) return batch_run_once(P, h, batch, o, ws, infos, stream);
  // graph: key = every argument that the captured sequence depends on
  uint64_t key = fnv1a(skey, h, sizeof(rclupp_problem) * (size_t)batch);
  const void* ptrs[3] = {ws_v, (const void*)d_info, nullptr};
  key = fnv1a(key, ptrs, sizeof(ptrs));
  key = fnv1a(key, &tune, sizeof(tune));
  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RCLUPP_ERR_HIP;
    hipStream_t cs = g_capture_stream[dev];
    if (!cs) {
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return RCLUPP_ERR_HIP;
      g_capture_stream[dev] = cs;
    }
    GraphEntry e;
    if (hipEventCreateWithFlags(&e.launched, hipEventDisableTiming) != hipSuccess) return RCLUPP_ERR_HIP;
    BatchPrep prep;
    int rc = batch_prepare(P, h, ws, infos, &prep);
    hipGraph_t graph = nullptr;
    if (rc == RCLUPP_OK) {
      if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = RCLUPP_ERR_HIP;
      } else {
        rc = batch_enqueue(P, prep, batch, o, ws, infos, cs);
        const hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (rc == RCLUPP_OK && ec != hipSuccess) rc = RCLUPP_ERR_HIP;
      }
    }
    if (rc == RCLUPP_OK && hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = RCLUPP_ERR_HIP;
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) {
      // nothing was enqueued from the buffer: it is free again at once
      if (prep.buf) prep.buf->held = false;
      (void)hipEventDestroy(e.launched);
      return rc;
    }
    e.tables = prep.buf;
    if (g_graphs.size() >= kGraphCacheEntries) {
      // evict the least recently used entry: its pinned tables return to the
      // pool behind the event of its last replay, and the executable is
      // destroyed once that replay has completed (reap_retired)
      auto old = g_graphs.begin();
      for (auto jt = g_graphs.begin(); jt != g_graphs.end(); ++jt)
        if (jt->second.tick < old->second.tick) old = jt;
      GraphEntry& v = old->second;
      v.tables->held = false;  // its `done` event already follows the last replay
      g_retired.push_back({v.exec, v.launched, v.replayed});
      g_graphs.erase(old);
      reap_retired();
    }
    it = g_graphs.emplace(key, e).first;
  }
  GraphEntry& ge = it->second;
  ge.tick = ++g_tick;
  if (hipGraphLaunch(ge.exec, stream) != hipSuccess) return RCLUPP_ERR_HIP;
  // both events follow this replay: the entry's (for its executable) and the
  // pinned buffer's (for reuse of the tables after eviction)
  if (hipEventRecord(ge.launched, stream) != hipSuccess) return RCLUPP_ERR_HIP;
  ge.replayed = true;
  if (hipEventRecord(ge.tables->done, stream) != hipSuccess) return RCLUPP_ERR_HIP;
  ge.tables->recorded = true;
  return RCLUPP_OK;
}

// Frees every process-lifetime object of the library (rclupp_release).
int release_all() {
  int rc = RCLUPP_OK;
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto& kv : g_graphs) {
      GraphEntry& v = kv.second;
      if (v.replayed && hipEventSynchronize(v.launched) != hipSuccess) rc = RCLUPP_ERR_HIP;
      if (hipGraphExecDestroy(v.exec) != hipSuccess) rc = RCLUPP_ERR_HIP;
      (void)hipEventDestroy(v.launched);
      if (v.tables) v.tables->held = false;
    }
    g_graphs.clear();
    for (RetiredExec& r : g_retired) {
      if (r.replayed && hipEventSynchronize(r.launched) != hipSuccess) rc = RCLUPP_ERR_HIP;
      (void)hipGraphExecDestroy(r.exec);
      (void)hipEventDestroy(r.launched);
    }
    g_retired.clear();
    for (PinnedBuf* b : g_pinned) {
      if (b->recorded && hipEventSynchronize(b->done) != hipSuccess) rc = RCLUPP_ERR_HIP;
      if (b->done) (void)hipEventDestroy(b->done);
      if (b->ptr && hipHostFree(b->ptr) != hipSuccess) rc = RCLUPP_ERR_HIP;
      delete b;
    }
    g_pinned.clear();
    for (auto& kv : g_capture_stream)
      if (kv.second && hipStreamDestroy(kv.second) != hipSuccess) rc = RCLUPP_ERR_HIP;
    g_capture_stream.clear();
    for (auto& kv : g_side) {
      SideStreams& ss = kv.second;
      for (int i = 0; i < kSideStreams; ++i) {
        if (ss.s[i] && hipStreamSynchronize(ss.s[i]) != hipSuccess) rc = RCLUPP_ERR_HIP;
        if (ss.s[i] && hipStreamDestroy(ss.s[i]) != hipSuccess) rc = RCLUPP_ERR_HIP;
        if (ss.join[i]) (void)hipEventDestroy(ss.join[i]);
      }
      if (ss.fork) (void)hipEventDestroy(ss.fork);
    }
    g_side.clear();
    g_tuned.clear();
    g_tune_file_read = false;
  }
  {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    g_trace_on = false;
    g_trace_marks.clear();
    for (hipEvent_t ev : g_trace_pool) {
      if (hipEventSynchronize(ev) != hipSuccess) rc = RCLUPP_ERR_HIP;
      (void)hipEventDestroy(ev);
    }
    g_trace_pool.clear();
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    // (hipHostFree waits for the device, so the outcome copies enqueued into
    // the slots have completed before they are freed)
    for (auto& kv : g_last)
      if (hipHostFree(kv.second) != hipSuccess) rc = RCLUPP_ERR_HIP;
    g_last.clear();
  }
  return rc;
}

}  // namespace

extern "C" {

int rclupp_release(void) { return release_all(); }

int rclupp_batched_workspace_size(int alg, const rclupp_problem* h_probs, int batch, const rclupp_opts* opts,
                                  size_t* bytes) {
  if (!bytes || batch < 0 || (batch > 0 && !h_probs)) return RCLUPP_ERR_INVALID_ARG;
  size_t mx = 0;
  for (int b = 0; b < batch; ++b) {
    const rclupp_problem& p = h_probs[b];
    int rc = validate(alg, p.m, p.n, p.ld, p.s, opts);
    if (rc) return rc;
    if (!p.X || !p.Q || !p.R) return RCLUPP_ERR_INVALID_ARG;
    const size_t t = make_layout(alg, p.m, p.n, p.s, opts).total;
    if (t > mx) mx = t;
  }
  if (batch_groupable(alg, h_probs, batch, opts)) {
    // the largest plan among the tuning candidates (fewest rows per workgroup)
    for (int ct : kTuneTall)
      for (int cs : kTuneSketch) {
        const size_t t = make_batch_plan(h_probs, batch, opts, BatchTune{ct, cs}).total;
        if (t > mx) mx = t;
      }
  }
  *bytes = mx > 0 ? mx : kAlign;
  return RCLUPP_OK;
}

int rclupp_qr_batched(int alg, const rclupp_problem* h_probs, int batch, const rclupp_opts* opts, void* ws,
                      size_t ws_bytes, rclupp_info* d_info, hipStream_t stream) {
  size_t need = 0;
  int rc = rclupp_batched_workspace_size(alg, h_probs, batch, opts, &need);
  if (rc) return rc;
  if (!ws) return RCLUPP_ERR_INVALID_ARG;
  if (ws_bytes < need) return RCLUPP_ERR_WORKSPACE;
  if (batch_groupable(alg, h_probs, batch, opts))
    return batched_grouped(alg, h_probs, batch, opts, ws, ws_bytes, d_info, stream);
  for (int b = 0; b < batch; ++b) {
    const rclupp_problem& p = h_probs[b];
    rc = rclupp_qr_ex(alg, p.X, p.m, p.n, p.ld, p.s, p.seed, p.Q, p.R, opts, ws, ws_bytes,
                      d_info ? d_info + b : nullptr, stream);
    if (rc) return rc;
  }
  return RCLUPP_OK;
}

// ---- step entry points -------------------------------------------------------------
int rclupp_omega(uint64_t seed, int64_t s, int64_t j0, int64_t cols, float* G, hipStream_t stream) {
  if (s < 1 || cols < 0 || j0 < 0 || (cols > 0 && !G)) return RCLUPP_ERR_INVALID_ARG;
  return launch_omega(seed, s, j0, cols, G, stream) == hipSuccess ? RCLUPP_OK : RCLUPP_ERR_HIP;
}

int rclupp_philox(const uint32_t* ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t stream) {
  if (count < 0 || (count > 0 && (!ctr || !out))) return RCLUPP_ERR_INVALID_ARG;
  return launch_philox(ctr, count, k0, k1, out, stream) == hipSuccess ? RCLUPP_OK : RCLUPP_ERR_HIP;
}

int rclupp_sketch(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, int prec, double* Y,
                  hipStream_t stream) {
  if (!X || !Y || n < 1 || m < 1 || ld < m || s < 1) return RCLUPP_ERR_INVALID_ARG;
  if (n > RCLUPP_MAX_N || s > 4096) return RCLUPP_ERR_UNSUPPORTED;
  if (prec < RCLUPP_PREC_FP64 || prec > RCLUPP_PREC_BF16) return RCLUPP_ERR_INVALID_ARG;
  // the reduced-precision loaders address a tile row with 32-bit element offsets
  if (prec != RCLUPP_PREC_FP64 && m + 16 * ld >= ((int64_t)1 << 32)) return RCLUPP_ERR_UNSUPPORTED;
  const SketchPlan sk = plan_sketch(m, n, s, prec, env_int("RCLUPP_SKETCH_GRID", 0));
  return with_scratch(sk.part_bytes, stream, [&](char* p) {
    if (launch_sketch_partials(sk, X, m, n, ld, seed, prec, (double*)p, nullptr, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    if (launch_sketch_reduce(sk, (double*)p, s, n, 1.0 / std::sqrt((double)s), Y, nullptr, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    return (int)RCLUPP_OK;
  });
}

int rclupp_srht(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, int prec, double* Y,
                hipStream_t stream) {
  if (!X || !Y || n < 1 || m < 1 || ld < m || s < 1) return RCLUPP_ERR_INVALID_ARG;
  if (n > RCLUPP_MAX_N || s > 4096 || m >= ((int64_t)1 << 30)) return RCLUPP_ERR_UNSUPPORTED;
  if (prec < RCLUPP_PREC_FP64 || prec > RCLUPP_PREC_BF16) return RCLUPP_ERR_INVALID_ARG;
  if (prec != RCLUPP_PREC_FP64 && m + 16 * ld >= ((int64_t)1 << 32)) return RCLUPP_ERR_UNSUPPORTED;
  int64_t mp = 1;
  while (mp < m) mp *= 2;
  if (s > mp) return RCLUPP_ERR_INVALID_ARG;  // s distinct rows of the order-m' Hadamard matrix
  SketchPlan sk = plan_sketch(m, n, s, prec, env_int("RCLUPP_SKETCH_GRID", 0));
  sk.kind = 2;
  return with_scratch(sk.part_bytes, stream, [&](char* p) {
    if (launch_sketch_partials(sk, X, m, n, ld, seed, prec, (double*)p, nullptr, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    if (launch_sketch_reduce(sk, (double*)p, s, n, 1.0 / std::sqrt((double)s), Y, nullptr, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    return (int)RCLUPP_OK;
  });
}

int rclupp_countsketch(const double* X, int64_t m, int64_t n, int64_t ld, int64_t s, uint64_t seed, double* Y,
                       hipStream_t stream) {
  if (!X || !Y || n < 1 || m < 1 || ld < m || s < 1) return RCLUPP_ERR_INVALID_ARG;
  if (n > RCLUPP_MAX_N) return RCLUPP_ERR_UNSUPPORTED;
  const SketchPlan sk = plan_countsketch(m, n, s, env_int("RCLUPP_SKETCH_GRID", 0));
  if (sk.nn == 0) return RCLUPP_ERR_UNSUPPORTED;
  return with_scratch(sk.part_bytes, stream, [&](char* p) {
    if (launch_countsketch_partials(sk, X, m, n, ld, s, seed, (double*)p, nullptr, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    if (launch_sketch_reduce(sk, (double*)p, s, n, 1.0, Y, nullptr, stream) != hipSuccess) return (int)RCLUPP_ERR_HIP;
    return (int)RCLUPP_OK;
  });
}

int rclupp_precond(const double* Y, int64_t s, int64_t n, int lu, int prec, double* R1, int32_t* perm, double* Mout,
                   rclupp_info* d_info, hipStream_t stream) {
  if (!Y || !R1 || n < 1 || s < n) return RCLUPP_ERR_INVALID_ARG;
  if (n > RCLUPP_MAX_N || s > 4096) return RCLUPP_ERR_UNSUPPORTED;
  if (prec != RCLUPP_PREC_FP64 && prec != RCLUPP_PREC_FP32) return RCLUPP_ERR_INVALID_ARG;
  const int np = pad_cols(n);
  const size_t rb = align_up(padded_r_doubles(np) * sizeof(double));
  const size_t sb = precond_scratch_bytes(s, n);
  return with_scratch(rb + sb + kAlign, stream, [&](char* p) {
    int32_t* info = d_info ? (int32_t*)d_info : (int32_t*)(p + rb + sb);
    if (!d_info) hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(64), 0, stream, (rclupp_info*)info);
    if (launch_precond(Y, s, n, lu ? 1 : 0, prec, nullptr, 0, (double*)p, R1, perm, Mout, (double*)(p + rb), info,
                       RCLUPP_STAGE_QR, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    return (int)RCLUPP_OK;
  });
}

int rclupp_trsm_gram(const double* X, int64_t m, int64_t n, int64_t ldx, const double* R, double* W, int64_t ldw,
                     double* G, hipStream_t stream) {
  if (!X || n < 1 || m < 1 || ldx < m) return RCLUPP_ERR_INVALID_ARG;
  if (n > RCLUPP_MAX_N) return RCLUPP_ERR_UNSUPPORTED;
  if (m + 3 * ldx >= ((int64_t)1 << 29) || (W && m + 3 * ldw >= ((int64_t)1 << 29)))
    return RCLUPP_ERR_UNSUPPORTED;
  if (W && ldw < m) return RCLUPP_ERR_INVALID_ARG;
  if (R && !W) return RCLUPP_ERR_INVALID_ARG;
  if (!R && W) return RCLUPP_ERR_INVALID_ARG;
  if (!G && !W) return RCLUPP_ERR_INVALID_ARG;
  const TallPlan tp = plan_tall(m, n, env_int("RCLUPP_TALL_GRID", 0));
  const int np = tp.np;
  const size_t rb = align_up(padded_r_doubles(np) * sizeof(double));
  const size_t gb = align_up((size_t)np * np * sizeof(double));
  return with_scratch(rb + tp.part_bytes + gb, stream, [&](char* p) {
    double* rpad = (double*)p;
    double* gpart = (double*)(p + rb);
    double* gfull = (double*)(p + rb + align_up(tp.part_bytes));
    if (R && launch_pad(R, n, rpad, stream) != hipSuccess) return (int)RCLUPP_ERR_HIP;
    // (the Gram partials only when G is asked for: a solve alone skips the Gram)
    if (launch_tall_pass(tp, X, ldx, m, n, R ? rpad : nullptr, W, W ? ldw : ldx, G ? gpart : nullptr, nullptr,
                         stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    if (G) {
      if (launch_gram_reduce(tp, gpart, n, gfull, nullptr, stream) != hipSuccess) return (int)RCLUPP_ERR_HIP;
      if (hipMemcpy2DAsync(G, n * sizeof(double), gfull, np * sizeof(double), n * sizeof(double), n,
                           hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return (int)RCLUPP_ERR_HIP;
    }
    return (int)RCLUPP_OK;
  });
}

int rclupp_chol(const double* G, int64_t n, int64_t m, int scholqr_shift, double* R, const double* Rprev,
                double* Rout, int32_t stage, rclupp_info* d_info, hipStream_t stream) {
  if (!G || !R || n < 1) return RCLUPP_ERR_INVALID_ARG;
  if (n > RCLUPP_MAX_N) return RCLUPP_ERR_UNSUPPORTED;
  if ((Rprev == nullptr) != (Rout == nullptr)) return RCLUPP_ERR_INVALID_ARG;
  const int np = pad_cols(n);
  const size_t rb = align_up(padded_r_doubles(np) * sizeof(double));
  const size_t sb = chol_scratch_bytes(n);
  return with_scratch(2 * rb + sb + kAlign, stream, [&](char* p) {
    double* rpad = (double*)p;
    double* prevpad = (double*)(p + rb);
    int32_t* info = d_info ? (int32_t*)d_info : (int32_t*)(p + 2 * rb + sb);
    if (!d_info) hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(64), 0, stream, (rclupp_info*)info);
    if (Rprev && launch_pad(Rprev, n, prevpad, stream) != hipSuccess) return (int)RCLUPP_ERR_HIP;
    if (launch_chol(G, (int)n, n, m, scholqr_shift ? 1 : 0, rpad, Rout, 1, Rprev ? prevpad : nullptr, nullptr, 0,
                    (double*)(p + 2 * rb), info, stage, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    if (launch_unpad(rpad, n, R, stream) != hipSuccess) return (int)RCLUPP_ERR_HIP;
    return (int)RCLUPP_OK;
  });
}

int rclupp_tall_lu_tournament(const double* X, int64_t m, int64_t n, int64_t ldx, double* M, int64_t ldm,
                              int32_t* sel, double* N, rclupp_info* d_info, hipStream_t stream) {
  if (!X || !M || !sel || !N || n < 1 || m < n || ldx < m || ldm < m) return RCLUPP_ERR_INVALID_ARG;
  if (n > 128 || m > (int64_t)INT32_MAX) return RCLUPP_ERR_UNSUPPORTED;
  if (m + 3 * ldx >= ((int64_t)1 << 29) || m + 3 * ldm >= ((int64_t)1 << 29)) return RCLUPP_ERR_UNSUPPORTED;
  const size_t sb = tslu_scratch_bytes(m, n);
  return with_scratch(sb + kAlign, stream, [&](char* p) {
    int32_t* info = d_info ? (int32_t*)d_info : (int32_t*)(p + sb);
    if (!d_info) hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(64), 0, stream, (rclupp_info*)info);
    if (launch_tslu(X, m, n, ldx, M, ldm, sel, N, (double*)p, info, stream) != hipSuccess) return (int)RCLUPP_ERR_HIP;
    return (int)RCLUPP_OK;
  });
}

int rclupp_tall_lu(const double* X, int64_t m, int64_t n, int64_t ldx, double* M, int64_t ldm, int32_t* perm,
                   rclupp_info* d_info, hipStream_t stream) {
  if (!X || !M || !perm || n < 1 || m < n || ldx < m || ldm < m) return RCLUPP_ERR_INVALID_ARG;
  // X is read until the last column has entered M: the two must not overlap
  const uintptr_t x0 = (uintptr_t)X, x1 = (uintptr_t)(X + (n - 1) * ldx + m);
  const uintptr_t m0 = (uintptr_t)M, m1 = (uintptr_t)(M + (n - 1) * ldm + m);
  if (x0 < m1 && m0 < x1) return RCLUPP_ERR_INVALID_ARG;
  if (n > RCLUPP_MAX_N || m > (int64_t)INT32_MAX) return RCLUPP_ERR_UNSUPPORTED;
  const size_t sb = tall_lu_scratch_bytes(m, n);
  return with_scratch(sb + kAlign, stream, [&](char* p) {
    int32_t* info = d_info ? (int32_t*)d_info : (int32_t*)(p + sb);
    if (!d_info) hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(64), 0, stream, (rclupp_info*)info);
    if (launch_tall_lu(X, m, n, ldx, M, ldm, perm, nullptr, (double*)p, info, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    return (int)RCLUPP_OK;
  });
}

}  // extern "C"
