// C-ABI entry points of libprohd: argument validation, workspace sizing,
// error strings and kernel timing.  Kernels live in k_*.hip.

#include <math.h>

#include <cmath>

#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace prohd {

// Defined in k_hd.hip / k_project.hip.
prohd_status hd_candidates(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                           const int32_t* idxA, const int64_t* dnA, int64_t capA,
                           const int32_t* idxB, const int64_t* dnB, int64_t capB, uint32_t flags,
                           prohd_result* out, void* ws, size_t ws_bytes, hipStream_t s);
prohd_status hd_exact(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      uint32_t flags, prohd_result* out, float* nn2A, float* nn2B, void* ws,
                      size_t ws_bytes, hipStream_t s);
prohd_status project_run(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                         int32_t m, bool dirs_given, float* dirs, float* projA, float* projB,
                         double* evals, int32_t* status, void* ws, size_t ws_bytes, hipStream_t s);

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_err;
}
void set_error(const std::string& msg) { g_err = msg; }
prohd_status fail(prohd_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

// ------------------------------------------------------------ device info
int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// ----------------------------------------------------------------- timing
namespace {
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_pool;
thread_local int g_open = -1;
thread_local bool g_capturing = false;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool profiling() { return g_prof_on && !g_capturing; }

void set_capturing(bool on) { g_capturing = on; }

void profile_begin(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfRec r{name, take_event(), take_event()};
  if (!r.a || !r.b) return;
  hipEventRecord(r.a, s);
  g_prof.push_back(r);
  g_open = (int)g_prof.size() - 1;
}

void profile_end(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (g_open >= 0 && g_open < (int)g_prof.size()) hipEventRecord(g_prof[g_open].b, s);
  g_open = -1;
}

}  // namespace prohd

using namespace prohd;

namespace {

bool bad_ptr(const void* p) { return p == nullptr; }

prohd_status check_sets(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D) {
  if (bad_ptr(A) || bad_ptr(B)) return fail(PROHD_EINVAL, "A and B must be non-null device pointers");
  if (nA < 1 || nB < 1) return fail(PROHD_EINVAL, "nA and nB must be >= 1");
  if (nA >= (int64_t(1) << 31) || nB >= (int64_t(1) << 31))
    return fail(PROHD_EINVAL, "nA and nB must be < 2^31");
  if (D < 1) return fail(PROHD_EINVAL, "D must be >= 1");
  if (D > PROHD_MAX_DIM) return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM (256)");
  return PROHD_OK;
}

prohd_status finish(prohd_status st, uint32_t flags, hipStream_t s, const int32_t* dev_status) {
  if (st != PROHD_OK) return st;
  if (flags & PROHD_SYNC) {
    PROHD_HIP(hipStreamSynchronize(s));
    if (dev_status) {
      int32_t h = 0;
      PROHD_HIP(hipMemcpy(&h, dev_status, sizeof(h), hipMemcpyDeviceToHost));
      if (h != PROHD_OK) return fail((prohd_status)h, "device reported status " + std::to_string(h));
    }
  }
  return PROHD_OK;
}

// Scratch memory of exact_hd_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[PROHD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

prohd_status scratch_address(void** p) {
  int dev = -1;
  PROHD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PROHD_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess || q == nullptr)
      return fail(PROHD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = q;
  }
  *p = g_scratch_ptr[dev];
  return PROHD_OK;
}

}  // namespace

extern "C" {

size_t prohd_workspace_size(int64_t nA, int64_t nB, int32_t D, int32_t ndirs, int64_t capA,
                            int64_t capB) {
  if (nA < 1 || nB < 1 || D < 1 || D > PROHD_MAX_DIM || ndirs < 1 || ndirs > PROHD_MAX_DIRS ||
      capA < 0 || capB < 0)
    return 0;
  if (capA == 0 || capA > nA) capA = nA;
  if (capB == 0 || capB > nB) capB = nB;
  size_t need = project_ws_bytes(nA, nB, D, ndirs);
  need = std::max(need, select_ws_bytes(2 * ndirs, std::max(nA, nB)) +
                            compact_ws_bytes(std::max(nA, nB)) + (size_t)(nA + nB) + 1024);
  need = std::max(need, hd_ws_bytes(nA, nB, D, capA, capB, true, PROHD_PREC_BF16 | PROHD_PRUNE));
  need = std::max(need, hd_ws_bytes(nA, nB, D, capA, capB, false, PROHD_PREC_BF16 | PROHD_PRUNE));
  need = std::max(need, exact_ws_bytes(nA, nB, D, PROHD_PREC_BF16 | PROHD_PRUNE));
  return need;
}

int32_t prohd_default_m(int32_t D) { return (D < 1 || D > PROHD_MAX_DIM) ? 0 : default_m(D); }

int32_t prohd_prune_levels(int64_t nA, int64_t nB, int64_t capA, int64_t capB, uint32_t flags) {
  if (nA < 1 || nB < 1 || capA < 1 || capB < 1 || capA > nA || capB > nB) return 0;
  return hd_prune_levels(capA, capB, nA, nB, flags);
}

prohd_status prohd_alpha_k(double alpha, int64_t n, int32_t m, int32_t* k) {
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(PROHD_EINVAL, "alpha must be positive and finite");
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(PROHD_EINVAL, "n must be in [1, 2^31)");
  if (m < 1 || m + 1 > PROHD_MAX_DIRS) return fail(PROHD_EINVAL, "m must be in [1, PROHD_MAX_DIRS - 1]");
  if (bad_ptr(k)) return fail(PROHD_EINVAL, "k must be a non-null host array of m + 1 entries");
  k[0] = (int32_t)alpha_k(alpha, n);
  for (int d = 1; d <= m; ++d) k[d] = (int32_t)alpha_k(alpha / m, n);
  return PROHD_OK;
}

prohd_status prohd_project(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                           int32_t m, uint32_t flags, float* dirs, float* projA, float* projB,
                           double* evals, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  prohd_status st = check_sets(A, nA, B, nB, D);
  if (st) return st;
  if (flags & ~(uint32_t)(PROHD_DIRS_GIVEN | PROHD_SYNC)) return fail(PROHD_EINVAL, "unknown flag");
  if (m < 1 || m > D) return fail(PROHD_EINVAL, "m must satisfy 1 <= m <= D");
  if (m + 1 > PROHD_MAX_DIRS) return fail(PROHD_EUNSUPPORTED, "m + 1 exceeds PROHD_MAX_DIRS");
  if (bad_ptr(dirs) || bad_ptr(projA) || bad_ptr(projB))
    return fail(PROHD_EINVAL, "dirs, projA and projB must be non-null");
  if (bad_ptr(ws)) return fail(PROHD_EINVAL, "workspace must be non-null");
  if (ws_bytes < project_ws_bytes(nA, nB, D, m + 1)) return fail(PROHD_EWORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  st = project_run(A, nA, B, nB, D, m, (flags & PROHD_DIRS_GIVEN) != 0, dirs, projA, projB, evals,
                   status, ws, ws_bytes, s);
  return finish(st, flags, s, status);
}

prohd_status prohd_select(const float* projA, int64_t nA, const float* projB, int64_t nB,
                          int32_t ndirs, const int32_t* kA, const int32_t* kB, int32_t* idxA,
                          int64_t capA, int64_t* nselA, int32_t* idxB, int64_t capB, int64_t* nselB,
                          void* ws, size_t ws_bytes, void* stream) {
  if (bad_ptr(projA) || bad_ptr(projB)) return fail(PROHD_EINVAL, "projections must be non-null");
  if (nA < 1 || nB < 1 || nA >= (int64_t(1) << 31) || nB >= (int64_t(1) << 31))
    return fail(PROHD_EINVAL, "nA and nB must be in [1, 2^31)");
  if (ndirs < 1) return fail(PROHD_EINVAL, "ndirs must be >= 1");
  if (ndirs > PROHD_MAX_DIRS) return fail(PROHD_EUNSUPPORTED, "ndirs exceeds PROHD_MAX_DIRS");
  if (bad_ptr(kA) || bad_ptr(kB)) return fail(PROHD_EINVAL, "kA and kB must be non-null host arrays");
  if (bad_ptr(idxA) || bad_ptr(idxB) || bad_ptr(nselA) || bad_ptr(nselB))
    return fail(PROHD_EINVAL, "index outputs must be non-null");
  if (bad_ptr(ws)) return fail(PROHD_EINVAL, "workspace must be non-null");
  int64_t boundA = 0, boundB = 0;
  for (int d = 0; d < ndirs; ++d) {
    if (kA[d] < 1 || kB[d] < 1) return fail(PROHD_EINVAL, "every k must be >= 1");
    boundA += 2 * std::min<int64_t>(kA[d], nA);
    boundB += 2 * std::min<int64_t>(kB[d], nB);
  }
  boundA = std::min(boundA, nA);
  boundB = std::min(boundB, nB);
  if (capA < boundA || capB < boundB)
    return fail(PROHD_EINVAL, "capA/capB below min(n, sum 2k): the index list could overflow");
  const int nseg = 2 * ndirs;
  Arena ar(ws);
  uint8_t* fA = ar.take<uint8_t>(nA);
  uint8_t* fB = ar.take<uint8_t>(nB);
  const size_t sel_bytes = select_ws_bytes(nseg, std::max(nA, nB));
  void* sel_ws = ar.take<char>(sel_bytes);
  const size_t cmp_bytes = compact_ws_bytes(std::max(nA, nB));
  void* cmp_ws = ar.take<char>(cmp_bytes);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  prohd_status st = zero_bytes(fA, (size_t)nA, s);
  if (st) return st;
  st = zero_bytes(fB, (size_t)nB, s);
  if (st) return st;
  std::vector<SelSegment> segs;
  segs.reserve(nseg);
  for (int d = 0; d < ndirs; ++d) {
    const int32_t ka = (int32_t)std::min<int64_t>(kA[d], nA);
    const int32_t kb = (int32_t)std::min<int64_t>(kB[d], nB);
    segs.push_back(SelSegment{projA + (size_t)d * nA, nA, nullptr, ka, ka, fA});
    segs.push_back(SelSegment{projB + (size_t)d * nB, nB, nullptr, kb, kb, fB});
  }
  st = select_mark(segs.data(), nseg, sel_ws, sel_bytes, s);
  if (st) return st;
  return compact_flags2(fA, nA, idxA, capA, nselA, fB, nB, idxB, capB, nselB, cmp_ws, cmp_bytes, s);
}

prohd_status prohd_top_keys(const float* vals, int64_t n, const int64_t* dev_n, int32_t k,
                            int32_t* idx, int64_t* count, void* ws, size_t ws_bytes,
                            void* stream) {
  if ((n > 0 && bad_ptr(vals)) || bad_ptr(idx) || bad_ptr(count) || bad_ptr(ws))
    return fail(PROHD_EINVAL, "vals (when n > 0), idx, count and ws must be non-null");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(PROHD_EINVAL, "n must be in [0, 2^31)");
  if (k < 0 || k > 64) return fail(PROHD_EINVAL, "k must be in [0, 64]");
  if (ws_bytes < PROHD_TOPK_WS_BYTES) return fail(PROHD_EWORKSPACE, "workspace too small");
  const TopSegment seg{reinterpret_cast<const uint32_t*>(vals), n, dev_n, k, idx, count};
  return top_keys(&seg, 1, ws, ws_bytes, (hipStream_t)stream);
}

prohd_status prohd_hd(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      const int32_t* idxA, const int64_t* nselA, const int32_t* idxB,
                      const int64_t* nselB, int64_t capA, int64_t capB, uint32_t flags,
                      prohd_result* out, void* ws, size_t ws_bytes, void* stream) {
  prohd_status st = check_sets(A, nA, B, nB, D);
  if (st) return st;
  if (flags & ~(uint32_t)(PROHD_INNER_FULL | PROHD_PREC_BF16 | PROHD_PREC_FP8 | PROHD_SYNC | PROHD_PRUNE))
    return fail(PROHD_EINVAL, "unknown flag");
  if ((flags & PROHD_PREC_BF16) && (flags & PROHD_PREC_FP8))
    return fail(PROHD_EINVAL, "PROHD_PREC_BF16 and PROHD_PREC_FP8 are exclusive");
  if (bad_ptr(idxA) || bad_ptr(idxB) || bad_ptr(nselA) || bad_ptr(nselB))
    return fail(PROHD_EINVAL, "index inputs must be non-null");
  if (capA < 1 || capB < 1 || capA > nA || capB > nB)
    return fail(PROHD_EINVAL, "capA/capB must be in [1, n]");
  if (bad_ptr(out)) return fail(PROHD_EINVAL, "out must be non-null");
  if (bad_ptr(ws)) return fail(PROHD_EINVAL, "workspace must be non-null");
  const bool full = (flags & PROHD_INNER_FULL) != 0;
  if (ws_bytes < hd_ws_bytes(nA, nB, D, capA, capB, full, flags))
    return fail(PROHD_EWORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  st = hd_candidates(A, nA, B, nB, D, idxA, nselA, capA, idxB, nselB, capB, flags, out, ws, ws_bytes, s);
  return finish(st, flags, s, out ? &out->status : nullptr);
}

prohd_status exact_hd(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      uint32_t flags, prohd_result* out, float* nn2A, float* nn2B, void* ws,
                      size_t ws_bytes, void* stream) {
  prohd_status st = check_sets(A, nA, B, nB, D);
  if (st) return st;
  if (flags & ~(uint32_t)(PROHD_PREC_BF16 | PROHD_PREC_FP8 | PROHD_SYNC | PROHD_PRUNE))
    return fail(PROHD_EINVAL, "unknown flag");
  if ((flags & PROHD_PREC_BF16) && (flags & PROHD_PREC_FP8))
    return fail(PROHD_EINVAL, "PROHD_PREC_BF16 and PROHD_PREC_FP8 are exclusive");
  if (bad_ptr(out)) return fail(PROHD_EINVAL, "out must be non-null");
  if (bad_ptr(ws)) return fail(PROHD_EINVAL, "workspace must be non-null");
  if (ws_bytes < exact_ws_bytes(nA, nB, D, flags)) return fail(PROHD_EWORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  st = hd_exact(A, nA, B, nB, D, flags, out, nn2A, nn2B, ws, ws_bytes, s);
  return finish(st, flags, s, out ? &out->status : nullptr);
}

prohd_status exact_hd_noalloc(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                              uint32_t flags, prohd_result* out, float* nn2A, float* nn2B,
                              void* stream) {
  prohd_status st = check_sets(A, nA, B, nB, D);
  if (st) return st;
  if (flags & ~(uint32_t)(PROHD_PREC_BF16 | PROHD_PREC_FP8))
    return fail(PROHD_EINVAL, "exact_hd_noalloc: only PROHD_PREC_BF16 / PROHD_PREC_FP8 are accepted");
  if ((flags & PROHD_PREC_BF16) && (flags & PROHD_PREC_FP8))
    return fail(PROHD_EINVAL, "PROHD_PREC_BF16 and PROHD_PREC_FP8 are exclusive");
  if (bad_ptr(out)) return fail(PROHD_EINVAL, "out must be non-null");
  const size_t need = exact_ws_bytes(nA, nB, D, flags);
  if (need > PROHD_NOALLOC_SCRATCH_BYTES)
    return fail(PROHD_EWORKSPACE, "exact_hd_noalloc: the sets need " + std::to_string(need) +
                                      " bytes of scratch, above PROHD_NOALLOC_SCRATCH_BYTES (" +
                                      std::to_string((size_t)PROHD_NOALLOC_SCRATCH_BYTES) + ")");
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st) return st;
  return hd_exact(A, nA, B, nB, D, flags, out, nn2A, nn2B, ws, PROHD_NOALLOC_SCRATCH_BYTES,
                  (hipStream_t)stream);
}

// ------------------------------------------------------- adaptive alpha
// Host-driven schedule over device work: one projection and one certificate,
// then per alpha one selection and one inner-full distance; the host reads
// the 80-byte result after each step to decide whether to go on.
namespace {

struct AdaptiveLayout {
  float* dirs;
  float* projA;
  float* projB;
  int32_t* pstatus;
  int32_t* idxA;
  int32_t* idxB;
  int64_t* cnt;
  prohd_cert* cert;
  void* sub;
  size_t sub_bytes;
};

int64_t alpha_cap(double alpha, int64_t n, int32_t m) {
  int64_t s = 2 * alpha_k(alpha, n);
  for (int d = 1; d <= m; ++d) s += 2 * alpha_k(alpha / m, n);
  return std::min(n, s);
}

AdaptiveLayout adaptive_layout(Arena& ar, int64_t nA, int64_t nB, int32_t D, int32_t m,
                               double alpha_max, uint32_t flags) {
  AdaptiveLayout L{};
  const int32_t nd = m + 1;
  const int64_t capA = alpha_cap(alpha_max, nA, m), capB = alpha_cap(alpha_max, nB, m);
  L.dirs = ar.take<float>((size_t)nd * D);
  L.projA = ar.take<float>((size_t)nd * nA);
  L.projB = ar.take<float>((size_t)nd * nB);
  L.pstatus = ar.take<int32_t>(64);
  L.idxA = ar.take<int32_t>(capA);
  L.idxB = ar.take<int32_t>(capB);
  L.cnt = ar.take<int64_t>(2);
  L.cert = ar.take<prohd_cert>(1);
  size_t sub = project_ws_bytes(nA, nB, D, nd);
  sub = std::max(sub, select_ws_bytes(2 * nd, std::max(nA, nB)) + compact_ws_bytes(std::max(nA, nB)) +
                          (size_t)(nA + nB) + 1024);
  sub = std::max(sub, hd_ws_bytes(nA, nB, D, capA, capB, true, flags | PROHD_PRUNE));
  sub = std::max(sub, cert_ws_bytes(D, nd));
  L.sub_bytes = sub;
  L.sub = ar.take<char>(sub);
  return L;
}

}  // namespace

size_t prohd_adaptive_workspace_size(int64_t nA, int64_t nB, int32_t D, double alpha_max,
                                     uint32_t flags) {
  if (nA < 1 || nB < 1 || D < 1 || D > PROHD_MAX_DIM || !(alpha_max > 0.0) || !std::isfinite(alpha_max))
    return 0;
  Arena ar(nullptr);
  adaptive_layout(ar, nA, nB, D, default_m(D), alpha_max, flags);
  return ar.used + 256;
}

prohd_status prohd_adaptive(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                            double alpha0, double growth, double alpha_max, double tol,
                            uint32_t flags, prohd_result* out, prohd_adaptive_result* res,
                            void* ws, size_t ws_bytes, void* stream) {
  prohd_status st = check_sets(A, nA, B, nB, D);
  if (st) return st;
  if (flags & ~(uint32_t)(PROHD_PREC_BF16 | PROHD_PREC_FP8)) return fail(PROHD_EINVAL, "unknown flag");
  if ((flags & PROHD_PREC_BF16) && (flags & PROHD_PREC_FP8))
    return fail(PROHD_EINVAL, "PROHD_PREC_BF16 and PROHD_PREC_FP8 are exclusive");
  if (!(alpha0 > 0.0) || !(alpha_max >= alpha0) || !std::isfinite(alpha_max))
    return fail(PROHD_EINVAL, "need 0 < alpha0 <= alpha_max < inf");
  if (!(growth > 1.0) || !std::isfinite(growth)) return fail(PROHD_EINVAL, "growth must be > 1");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(PROHD_EINVAL, "tol must be >= 0");
  if (bad_ptr(out) || bad_ptr(res) || bad_ptr(ws)) return fail(PROHD_EINVAL, "out, res and ws must be non-null");
  const int32_t m = default_m(D);
  if (m + 1 > PROHD_MAX_DIRS) return fail(PROHD_EUNSUPPORTED, "m + 1 exceeds PROHD_MAX_DIRS");
  Arena ar(ws);
  const AdaptiveLayout L = adaptive_layout(ar, nA, nB, D, m, alpha_max, flags);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const int32_t nd = m + 1;
  st = project_run(A, nA, B, nB, D, m, false, L.dirs, L.projA, L.projB, nullptr, L.pstatus, L.sub,
                   L.sub_bytes, s);
  if (st) return st;
  st = cert_run(A, nA, B, nB, D, L.dirs, nd, L.projA, L.projB, nullptr, L.cert, L.sub, L.sub_bytes, s);
  if (st) return st;
  prohd_cert cert{};
  int32_t pst = 0;
  PROHD_HIP(hipMemcpyAsync(&cert, L.cert, sizeof(cert), hipMemcpyDeviceToHost, s));
  PROHD_HIP(hipMemcpyAsync(&pst, L.pstatus, sizeof(pst), hipMemcpyDeviceToHost, s));
  PROHD_HIP(hipStreamSynchronize(s));
  if (pst != PROHD_OK) return fail((prohd_status)pst, "projection reported status " + std::to_string(pst));
  if (cert.status != PROHD_OK)
    return fail((prohd_status)cert.status, "certificate reported status " + std::to_string(cert.status));
  const int64_t capA = alpha_cap(alpha_max, nA, m), capB = alpha_cap(alpha_max, nB, m);
  std::vector<int32_t> kA(nd), kB(nd);
  double alpha = alpha0, prev = -1.0;
  for (int32_t j = 0;; ++j) {
    const double a = std::min(alpha, alpha_max);
    st = prohd_alpha_k(a, nA, m, kA.data());
    if (!st) st = prohd_alpha_k(a, nB, m, kB.data());
    if (!st)
      st = prohd_select(L.projA, nA, L.projB, nB, nd, kA.data(), kB.data(), L.idxA, capA, L.cnt,
                        L.idxB, capB, L.cnt + 1, L.sub, L.sub_bytes, s);
    if (!st)
      st = prohd_hd(A, nA, B, nB, D, L.idxA, L.cnt, L.idxB, L.cnt + 1, alpha_cap(a, nA, m),
                    alpha_cap(a, nB, m), flags | PROHD_INNER_FULL | PROHD_PRUNE | PROHD_SYNC, out, L.sub,
                    L.sub_bytes, s);
    if (st) return st;
    prohd_result r{};
    PROHD_HIP(hipMemcpy(&r, out, sizeof(r), hipMemcpyDeviceToHost));
    const double F = r.H;
    const double lb = std::max(cert.hu_lo, F);
    int32_t reason = 0;
    if (cert.ub - lb <= tol * lb) reason = 1;
    else if (j >= 1 && F - prev <= tol * F) reason = 2;
    else if (a >= alpha_max) reason = 3;
    if (reason) {
      res->alpha = a;
      res->H = F;
      res->lb = lb;
      res->ub = cert.ub;
      res->change = j >= 1 && F > 0.0 ? (F - prev) / F : -1.0;
      res->nA_sel = r.nA_sel;
      res->nB_sel = r.nB_sel;
      res->steps = j + 1;
      res->reason = reason;
      return PROHD_OK;
    }
    prev = F;
    alpha *= growth;
  }
}

size_t prohd_mlp_param_count(int32_t D) {
  if (D < 1 || D > PROHD_MAX_DIM) return 0;
  return mlp_param_count(D);
}

size_t prohd_mlp_workspace_size(int64_t rows, int32_t D) {
  if (rows < 1 || D < 1 || D > PROHD_MAX_DIM) return 0;
  return mlp_ws_bytes(rows, D);
}

prohd_status prohd_mlp_init(float* params, int32_t D, uint64_t seed, void* stream) {
  if (bad_ptr(params)) return fail(PROHD_EINVAL, "params must be non-null");
  if (D < 1) return fail(PROHD_EINVAL, "D must be >= 1");
  if (D > PROHD_MAX_DIM) return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM (256)");
  return mlp_init(params, D, seed, (hipStream_t)stream);
}

prohd_status prohd_mlp_score(const float* X, int64_t n, int32_t D, const float* c_other,
                             const float* params, float* scores, void* ws, size_t ws_bytes,
                             void* stream) {
  if (bad_ptr(X) || bad_ptr(c_other) || bad_ptr(params) || bad_ptr(scores) || bad_ptr(ws))
    return fail(PROHD_EINVAL, "null pointer");
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(PROHD_EINVAL, "n must be in [1, 2^31)");
  if (D < 1) return fail(PROHD_EINVAL, "D must be >= 1");
  if (D > PROHD_MAX_DIM) return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM (256)");
  if (ws_bytes < mlp_ws_bytes(n, D)) return fail(PROHD_EWORKSPACE, "workspace too small");
  return mlp_score(X, n, D, c_other, params, scores, ws, ws_bytes, (hipStream_t)stream);
}

prohd_status prohd_mlp_grad(const float* X, int32_t D, const float* c_other, const float* labels,
                            const int32_t* idx, int64_t batch, float pos_weight,
                            const float* params, float* grad, float* loss, void* ws,
                            size_t ws_bytes, void* stream) {
  if (bad_ptr(X) || bad_ptr(c_other) || bad_ptr(labels) || bad_ptr(idx) || bad_ptr(params) ||
      bad_ptr(grad) || bad_ptr(loss) || bad_ptr(ws))
    return fail(PROHD_EINVAL, "null pointer");
  if (batch < 1 || batch > 65536) return fail(PROHD_EINVAL, "batch must be in [1, 65536]");
  if (D < 1) return fail(PROHD_EINVAL, "D must be >= 1");
  if (D > PROHD_MAX_DIM) return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM (256)");
  if (!(pos_weight > 0.f)) return fail(PROHD_EINVAL, "pos_weight must be > 0");
  if (ws_bytes < mlp_ws_bytes(batch, D)) return fail(PROHD_EWORKSPACE, "workspace too small");
  return mlp_grad(X, D, c_other, labels, idx, batch, pos_weight, params, grad, loss, ws, ws_bytes,
                  (hipStream_t)stream);
}

prohd_status prohd_mlp_adamw(float* params, const float* grad, float* m, float* v, int32_t D,
                             int64_t t, float lr, float weight_decay, float beta1, float beta2,
                             float eps, void* stream) {
  if (bad_ptr(params) || bad_ptr(grad) || bad_ptr(m) || bad_ptr(v)) return fail(PROHD_EINVAL, "null pointer");
  if (D < 1) return fail(PROHD_EINVAL, "D must be >= 1");
  if (D > PROHD_MAX_DIM) return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM (256)");
  if (t < 1) return fail(PROHD_EINVAL, "t must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr >= 0.f))
    return fail(PROHD_EINVAL, "bad AdamW hyper-parameters");
  return mlp_adamw(params, grad, m, v, D, t, lr, weight_decay, beta1, beta2, eps, (hipStream_t)stream);
}

prohd_status prohd_mlp_train_step(const float* X, int32_t D, const float* c_other,
                                  const float* labels, const int32_t* idx, int64_t batch,
                                  float pos_weight, float* params, float* grad, float* m, float* v,
                                  int64_t t, float lr, float weight_decay, float beta1, float beta2,
                                  float eps, float* loss, void* ws, size_t ws_bytes, void* stream) {
  if (bad_ptr(m) || bad_ptr(v)) return fail(PROHD_EINVAL, "null pointer");
  if (t < 1) return fail(PROHD_EINVAL, "t must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr >= 0.f))
    return fail(PROHD_EINVAL, "bad AdamW hyper-parameters");
  prohd_status st = prohd_mlp_grad(X, D, c_other, labels, idx, batch, pos_weight, params, grad, loss,
                                   ws, ws_bytes, stream);
  if (st) return st;
  return prohd_mlp_adamw(params, grad, m, v, D, t, lr, weight_decay, beta1, beta2, eps, stream);
}

prohd_status prohd_centroid(const float* X, int64_t n, int32_t D, float* mean, void* ws,
                            size_t ws_bytes, void* stream) {
  if (bad_ptr(X) || bad_ptr(mean) || bad_ptr(ws)) return fail(PROHD_EINVAL, "null pointer");
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(PROHD_EINVAL, "n must be in [1, 2^31)");
  if (D < 1) return fail(PROHD_EINVAL, "D must be >= 1");
  if (D > PROHD_MAX_DIM) return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM (256)");
  if (ws_bytes < PROHD_CENTROID_WS_BYTES(D) || ws_bytes < centroid_ws_bytes(D))
    return fail(PROHD_EWORKSPACE, "workspace too small");
  return centroid_run(X, n, D, mean, ws, ws_bytes, (hipStream_t)stream);
}

size_t prohd_certificate_workspace_size(int32_t D, int32_t ndirs) {
  if (D < 1 || D > PROHD_MAX_DIM || ndirs < 1 || ndirs > PROHD_MAX_DIRS) return 0;
  return cert_ws_bytes(D, ndirs);
}

prohd_status prohd_certificate(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                               const float* dirs, int32_t ndirs, const float* projA,
                               const float* projB, const prohd_result* lower, prohd_cert* out,
                               void* ws, size_t ws_bytes, void* stream) {
  prohd_status st = check_sets(A, nA, B, nB, D);
  if (st) return st;
  if (bad_ptr(dirs) || bad_ptr(projA) || bad_ptr(projB) || bad_ptr(out) || bad_ptr(ws))
    return fail(PROHD_EINVAL, "dirs, projA, projB, out and ws must be non-null");
  if (ndirs < 1) return fail(PROHD_EINVAL, "ndirs must be >= 1");
  if (ndirs > PROHD_MAX_DIRS) return fail(PROHD_EUNSUPPORTED, "ndirs exceeds PROHD_MAX_DIRS (64)");
  if (ws_bytes < cert_ws_bytes(D, ndirs)) return fail(PROHD_EWORKSPACE, "workspace too small");
  return cert_run(A, nA, B, nB, D, dirs, ndirs, projA, projB, lower, out, ws, ws_bytes,
                  (hipStream_t)stream);
}

prohd_status prohd_select_scored(const float* scoresA, int64_t nA, int32_t sA,
                                 const float* scoresB, int64_t nB, int32_t sB,
                                 int32_t* idxA, int64_t capA, int64_t* nselA,
                                 int32_t* idxB, int64_t capB, int64_t* nselB,
                                 void* ws, size_t ws_bytes, void* stream) {
  if (bad_ptr(scoresA) || bad_ptr(scoresB) || bad_ptr(idxA) || bad_ptr(idxB) || bad_ptr(nselA) ||
      bad_ptr(nselB) || bad_ptr(ws))
    return fail(PROHD_EINVAL, "null pointer");
  if (nA < 1 || nB < 1 || nA >= (int64_t(1) << 31) || nB >= (int64_t(1) << 31))
    return fail(PROHD_EINVAL, "nA and nB must be in [1, 2^31)");
  if (sA < 0 || sB < 0) return fail(PROHD_EINVAL, "sA and sB must be >= 0");
  if (capA < std::min<int64_t>(nA, sA) || capB < std::min<int64_t>(nB, sB) || capA > nA || capB > nB)
    return fail(PROHD_EINVAL, "capacities must lie in [min(n, s), n]");
  Arena ar(ws);
  uint8_t* fA = ar.take<uint8_t>(nA);
  uint8_t* fB = ar.take<uint8_t>(nB);
  const size_t sel_bytes = select_ws_bytes(2, std::max(nA, nB));
  void* sel_ws = ar.take<char>(sel_bytes);
  const size_t cmp_bytes = compact_ws_bytes(std::max(nA, nB));
  void* cmp_ws = ar.take<char>(cmp_bytes);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  prohd_status st = zero_bytes(fA, (size_t)nA, s);
  if (!st) st = zero_bytes(fB, (size_t)nB, s);
  if (!st) st = scatter_index_flags(idxA, nselA, capA, fA, s);
  if (!st) st = scatter_index_flags(idxB, nselB, capB, fB, s);
  if (st) return st;
  SelSegment segs[2] = {
      SelSegment{scoresA, nA, nullptr, 0, (int32_t)std::min<int64_t>(sA, nA), fA},
      SelSegment{scoresB, nB, nullptr, 0, (int32_t)std::min<int64_t>(sB, nB), fB}};
  st = select_mark(segs, 2, sel_ws, sel_bytes, s);
  if (!st) st = compact_flags2(fA, nA, idxA, capA, nselA, fB, nB, idxB, capB, nselB, cmp_ws, cmp_bytes, s);
  return st;
}

const char* prohd_last_error(void) { return g_err.c_str(); }

const char* prohd_version(void) { return "prohd-gfx950 0.1.0"; }

prohd_status prohd_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return PROHD_OK;
}

prohd_status prohd_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof) {
    hipEventSynchronize(r.b);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_prof.clear();
  return PROHD_OK;
}

prohd_status prohd_profile_read(const char* name, int64_t* launches, double* total_ms) {
  if (!name || !launches || !total_ms) return fail(PROHD_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int64_t n = 0;
  double ms = 0.0;
  for (auto& r : g_prof) {
    if (r.name.find(name) == std::string::npos) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(PROHD_EDEVICE, "event synchronize failed");
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(PROHD_EDEVICE, "elapsed time failed");
    ms += t;
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  return PROHD_OK;
}

}  // extern "C"
