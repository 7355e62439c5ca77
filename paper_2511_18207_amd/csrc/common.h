// Internal declarations shared by the translation units of libprohd.
// Not part of the public ABI (see include/prohd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "prohd.h"

namespace prohd {

// ----------------------------------------------------------------- errors
void set_error(const std::string& msg);
prohd_status fail(prohd_status code, const std::string& msg);

#define PROHD_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return ::prohd::fail(PROHD_EDEVICE, std::string(#call) + ": " +          \
                                              hipGetErrorString(e_));          \
  } while (0)

// ------------------------------------------------------------ kernel timing
bool profiling();
// While a launch sequence is being captured into a graph, kernel timing is
// suspended (events of a capture are graph nodes, not timestamps).
void set_capturing(bool on);
void profile_begin(const char* name, hipStream_t s);
void profile_end(hipStream_t s);

// Launches a kernel (optionally bracketed by timing events) and checks the
// launch.  Usage: PROHD_LAUNCH("name", kern, grid, block, lds, stream, args...)
#define PROHD_LAUNCH(name, kern, grid, block, lds, stream, ...)                \
  do {                                                                         \
    const bool prof_ = ::prohd::profiling();                                   \
    if (prof_) ::prohd::profile_begin(name, stream);                           \
    hipLaunchKernelGGL(kern, grid, block, lds, stream, __VA_ARGS__);           \
    hipError_t le_ = hipGetLastError();                                        \
    if (le_ != hipSuccess)                                                     \
      return ::prohd::fail(PROHD_EDEVICE,                                      \
                           std::string("launch ") + name + ": " +              \
                               hipGetErrorString(le_));                        \
    if (prof_) ::prohd::profile_end(stream);                                   \
  } while (0)

// ---------------------------------------------------------------- workspace
// Bump allocator over the caller's workspace.  With base == nullptr it only
// counts bytes (used by the size queries).
struct Arena {
  char* base;
  size_t used = 0;
  explicit Arena(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// Device properties needed for launch shaping (cached per device).
int cu_count();

// Padded dimension used by the tile kernels: 16, 32, 64, 128 or 256.
inline int pad_dim(int D) {
  int p = 16;
  while (p < D) p *= 2;
  return p;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Alpha mode of Alg. 3 (host): m = floor(sqrt(D)) principal components;
// per set of n rows, k = max(1, floor(alpha n)) per end on the centroid axis
// (Alg. 1) and max(1, floor((alpha / m) n)) per end on each component (Alg. 2
// with alpha' = alpha / m), clipped to n.  The floor is taken of
// alpha n + 1e-9, so a decimal alpha does not lose an integer to binary
// rounding (0.29 * 100 = 28.999...).
inline int32_t default_m(int32_t D) {
  if (D < 1) return 0;
  int32_t m = 1;
  while ((int64_t)(m + 1) * (m + 1) <= D) ++m;
  return m;
}
inline int64_t alpha_k(double alpha, int64_t n) {
  const double f = alpha * (double)n + 1e-9;
  const int64_t k = f >= (double)n ? n : (int64_t)f;   // floor of a non-negative value
  return k < 1 ? 1 : (k > n ? n : k);
}

// Device status word values (int32), shared by kernels.
constexpr int32_t ST_OK = PROHD_OK;
constexpr int32_t ST_NONFINITE = PROHD_ENONFINITE;
constexpr int32_t ST_EMPTY = PROHD_EINVAL;

// ------------------------------------------------------------- sub-systems
// Extreme selection (k_select.hip).  Each segment is a float32 array;
// `lo`/`hi` are the numbers of smallest / largest entries to keep under the
// order (value, index), ties to the smaller index at both ends.  Kept
// entries set flag bytes; `n` may be read from device (dev_n) when non-null.
struct SelSegment {
  const float* vals;
  int64_t n;        // host bound on the length
  const int64_t* dev_n;  // device length, or nullptr (use n)
  int32_t lo, hi;   // counts per end (0 = none); clipped to the length
  uint8_t* flags;   // flag bytes to set (length >= n)
};
size_t select_ws_bytes(int nseg, int64_t max_n);
prohd_status select_mark(const SelSegment* segs, int nseg, void* ws, size_t ws_bytes,
                         hipStream_t s);
// Compaction of flag bytes into an ascending index list + device count;
// at most `cap` entries are written (and counted).
size_t compact_ws_bytes(int64_t n);
// Two arrays at once (host lengths; grid y = array).
prohd_status compact_flags2(const uint8_t* fA, int64_t nA, int32_t* idxA, int64_t capA, int64_t* countA,
                            const uint8_t* fB, int64_t nB, int32_t* idxB, int64_t capB, int64_t* countB,
                            void* ws, size_t ws_bytes, hipStream_t s);
// The k <= 64 largest keys of up to two arrays under the same order (larger
// float value first; equal values: smaller index first), as ascending index
// lists with a device count of min(k, length).  `keys` are float32 bit
// patterns; the length is read from dev_n (clipped to n) when non-null.
struct TopSegment {
  const uint32_t* keys;
  int64_t n;              // host bound on the length
  const int64_t* dev_n;   // device length, or nullptr (use n)
  int32_t k;              // entries to keep, at most 64
  int32_t* idx;           // k entries
  int64_t* count;         // 1 entry
};
size_t topk_ws_bytes(int64_t max_n);
prohd_status top_keys(const TopSegment* segs, int nseg, void* ws, size_t ws_bytes, hipStream_t s);
// flags[idx[i]] = 1 for the first *count entries (count clipped to cap).
prohd_status scatter_index_flags(const int32_t* idx, const int64_t* count, int64_t cap,
                                 uint8_t* flags, hipStream_t s);
// Fill bytes with zero through a kernel (graph-friendly; no memset nodes).
prohd_status zero_bytes(void* p, size_t bytes, hipStream_t s);

// Distance core (k_hd.hip).
size_t hd_ws_bytes(int64_t nA, int64_t nB, int32_t D, int64_t capA, int64_t capB, bool full,
                   uint32_t flags);
size_t exact_ws_bytes(int64_t nA, int64_t nB, int32_t D, uint32_t flags);
int hd_prune_levels(int64_t capA, int64_t capB, int64_t nA, int64_t nB, uint32_t flags);
// Exact distance of one pair (exact_hd without argument checks).
prohd_status hd_exact(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      uint32_t flags, prohd_result* out, float* nn2A, float* nn2B, void* ws,
                      size_t ws_bytes, hipStream_t s);

// Column means of one set (k_mean.hip).
size_t centroid_ws_bytes(int32_t D);
prohd_status centroid_run(const float* X, int64_t n, int32_t D, float* mean, void* ws,
                          size_t ws_bytes, hipStream_t s);

// Error certificate (k_cert.hip).
size_t cert_ws_bytes(int32_t D, int32_t ndirs);
prohd_status cert_run(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      const float* dirs, int32_t ndirs, const float* PA, const float* PB,
                      const prohd_result* lower, prohd_cert* out, void* ws, size_t ws_bytes,
                      hipStream_t s);

// Learned proposal scorer (k_mlp.hip).
size_t mlp_param_count(int32_t D);
size_t mlp_ws_bytes(int64_t rows, int32_t D);
prohd_status mlp_init(float* params, int32_t D, uint64_t seed, hipStream_t s);
prohd_status mlp_score(const float* X, int64_t n, int32_t D, const float* c_other,
                       const float* params, float* scores, void* ws, size_t ws_bytes,
                       hipStream_t s);
prohd_status mlp_grad(const float* X, int32_t D, const float* c_other, const float* labels,
                      const int32_t* idx, int64_t batch, float pos_weight, const float* params,
                      float* grad, float* loss, void* ws, size_t ws_bytes, hipStream_t s);
prohd_status mlp_adamw(float* params, const float* grad, float* m, float* v, int32_t D, int64_t t,
                       float lr, float wd, float b1, float b2, float eps, hipStream_t s);

// Direction finding and projection (k_stats.hip, k_eig.hip, k_project.hip).
size_t project_ws_bytes(int64_t nA, int64_t nB, int32_t D, int32_t ndirs);

}  // namespace prohd
