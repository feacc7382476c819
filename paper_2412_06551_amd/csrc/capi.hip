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

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rclupp.h"
#include "launch.hpp"

using namespace rclupp;

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
  size_t info = 0, ypart = 0, y = 0, r1 = 0, r2 = 0, r3 = 0, r4 = 0, gpart = 0, g = 0, small = 0, perm = 0,
         nmat = 0, lu = 0, total = 0;
  SketchPlan sk{};
  TallPlan tp{};
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
  }
  return RCLUPP_OK;
}

Layout make_layout(int alg, int64_t m, int64_t n, int64_t s, const rclupp_opts* o) {
  Layout L;
  const int sk_prec = o ? o->sketch_prec : 0;
  L.tp = plan_tall(m, n, env_int("RCLUPP_TALL_GRID", 0));
  const int np = L.tp.np;
  const size_t rbytes = align_up(padded_r_doubles(np) * sizeof(double));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(bytes);
    return at;
  };
  L.info = take(sizeof(rclupp_info));
  if (sketched(alg)) {
    L.sk = plan_sketch(m, n, s, sk_prec, env_int("RCLUPP_SKETCH_GRID", 0));
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
    L.perm = take((size_t)m * sizeof(int32_t));
    L.nmat = take((size_t)n * n * sizeof(double));
    L.lu = take(tall_lu_scratch_bytes(m, n));
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
  HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, r4, Q, ld, gpart, info, st));  // Gram unused
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
  HIPCHK(launch_tall_pass(L.tp, Q, ld, m, n, r2, Q, ld, gpart, info, st));  // Gram unused
  return RCLUPP_OK;
}

int sketch_into(const Layout& L, char* ws, const double* A, int64_t m, int64_t n, int64_t lda, int64_t s,
                uint64_t seed, int prec, int32_t* info, hipStream_t st) {
  double* ypart = (double*)(ws + L.ypart);
  double* y = (double*)(ws + L.y);
  STAGE("sketch");
  HIPCHK(launch_sketch_partials(L.sk, A, m, n, lda, seed, prec, ypart, info, st));
  STAGE("sketch_reduce");
  HIPCHK(launch_sketch_reduce(L.sk, ypart, s, n, 1.0 / std::sqrt((double)s), y, info, st));
  return RCLUPP_OK;
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
  int rc;
  switch (alg) {
    case RCLUPP_ALG_RCLUPP:
      if ((rc = sketch_into(L, ws, X, m, n, ld, s, seed, sk_prec, info, st))) return rc;
      STAGE("precond");
      HIPCHK(launch_precond((double*)(ws + L.y), s, n, 1, lu_prec, nullptr, 0, r1, nullptr, nullptr, nullptr, small,
                            info, RCLUPP_STAGE_QR, st));
      return tail_cholqr2(L, ws, X, m, n, ld, Q, R, info, st);
    case RCLUPP_ALG_RCHOLQR:
      if ((rc = sketch_into(L, ws, X, m, n, ld, s, seed, sk_prec, info, st))) return rc;
      STAGE("precond");
      HIPCHK(launch_precond((double*)(ws + L.y), s, n, 0, lu_prec, nullptr, 0, r1, nullptr, nullptr, nullptr, small,
                            info, RCLUPP_STAGE_QR, st));
      return tail_cholqr1(L, ws, X, m, n, ld, Q, R, info, st);
    case RCLUPP_ALG_RCLUPPR: {
      int32_t* perm = (int32_t*)(ws + L.perm);
      double* nmat = (double*)(ws + L.nmat);
      STAGE("tall_lu");
      HIPCHK(launch_tall_lu(X, m, n, ld, Q, ld, perm, nmat, (double*)(ws + L.lu), info, st));
      HIPCHK(launch_unit_lower(Q, m, n, ld, info, st));
      if ((rc = sketch_into(L, ws, Q, m, n, ld, s, seed, sk_prec, info, st))) return rc;
      STAGE("precond");
      HIPCHK(launch_precond((double*)(ws + L.y), s, n, 0, lu_prec, nmat, n, r1, nullptr, nullptr, nullptr, small, info,
                            RCLUPP_STAGE_QR, st));
      return tail_cholqr2(L, ws, X, m, n, ld, Q, R, info, st);
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
      int32_t* perm = (int32_t*)(ws + L.perm);
      double* nmat = (double*)(ws + L.nmat);
      STAGE("tall_lu");
      HIPCHK(launch_tall_lu(X, m, n, ld, Q, ld, perm, nmat, (double*)(ws + L.lu), info, st));
      HIPCHK(launch_unit_lower(Q, m, n, ld, info, st));
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
  char* w = (char*)ws;
  rclupp_info* info = d_info ? d_info : (rclupp_info*)(w + L.info);
  hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(64), 0, stream, info);
  if (hipGetLastError() != hipSuccess) return RCLUPP_ERR_HIP;
  const int rc2 = run_method(alg, L, w, X, m, n, ld, s, seed, Q, R, opts, (int32_t*)info, stream);
  trace_mark(nullptr, stream);
  return rc2;
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

// ---- batched: one problem after another on the stream (same kernels) ------------
int rclupp_batched_workspace_size(int alg, const rclupp_problem* h_probs, int batch, const rclupp_opts* opts,
                                  size_t* bytes) {
  if (!bytes || batch < 0 || (batch > 0 && !h_probs)) return RCLUPP_ERR_INVALID_ARG;
  size_t mx = 0;
  for (int b = 0; b < batch; ++b) {
    const rclupp_problem& p = h_probs[b];
    int rc = validate(alg, p.m, p.n, p.ld, p.s, opts);
    if (rc) return rc;
    const size_t t = make_layout(alg, p.m, p.n, p.s, opts).total;
    if (t > mx) mx = t;
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
  const SketchPlan sk = plan_sketch(m, n, s, prec, env_int("RCLUPP_SKETCH_GRID", 0));
  return with_scratch(sk.part_bytes, stream, [&](char* p) {
    if (launch_sketch_partials(sk, X, m, n, ld, seed, prec, (double*)p, nullptr, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
    if (launch_sketch_reduce(sk, (double*)p, s, n, 1.0 / std::sqrt((double)s), Y, nullptr, stream) != hipSuccess)
      return (int)RCLUPP_ERR_HIP;
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
    // the n <= 64 substitution kernel always forms the Gram partials as well
    if (launch_tall_pass(tp, X, ldx, m, n, R ? rpad : nullptr, W, W ? ldw : ldx, (G || R) ? gpart : nullptr, nullptr,
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

int rclupp_tall_lu(const double* X, int64_t m, int64_t n, int64_t ldx, double* M, int64_t ldm, int32_t* perm,
                   rclupp_info* d_info, hipStream_t stream) {
  if (!X || !M || !perm || n < 1 || m < n || ldx < m || ldm < m) return RCLUPP_ERR_INVALID_ARG;
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
