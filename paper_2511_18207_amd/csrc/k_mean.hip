// Column means of one point set (the set centroid of Alg. 1, exposed on its
// own for the features of the learned proposal), accumulated in float64.
//
// colsum_part: work-group b sums rows [b*rows, (b+1)*rows) -- the 256
// threads form 256/D row groups (at least one), each reading whole rows, so
// consecutive threads touch consecutive addresses; the groups combine in LDS.
// colsum_final adds the partials in block order (deterministic).

#include <algorithm>

#include "common.h"

namespace prohd {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxParts = 1024;

__global__ __launch_bounds__(kThreads) void colsum_part(const float* __restrict__ X, int64_t n, int D,
                                                       int64_t rows, double* __restrict__ part) {
  __shared__ double red[kThreads];
  const int groups = D >= kThreads ? 1 : kThreads / D;
  const int g = threadIdx.x / D;
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int64_t r1 = r0 + rows < n ? r0 + rows : n;
  for (int c0 = 0; c0 < D; c0 += kThreads) {
    const int c = c0 + (int)(threadIdx.x % (unsigned)(D >= kThreads ? kThreads : D));
    // four independent partial sums (fixed order), added at the end
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (g < groups && c < D) {
      int64_t r = r0 + g;
      for (; r + 3 * groups < r1; r += 4 * groups) {
        a0 += (double)X[r * D + c];
        a1 += (double)X[(r + groups) * D + c];
        a2 += (double)X[(r + 2 * groups) * D + c];
        a3 += (double)X[(r + 3 * groups) * D + c];
      }
      for (; r < r1; r += groups) a0 += (double)X[r * D + c];
    }
    const double acc = (a0 + a1) + (a2 + a3);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < (unsigned)(D >= kThreads ? kThreads : D) && c < D) {
      double t = 0.0;
      for (int q = 0; q < groups; ++q) t += red[q * D + threadIdx.x];
      part[(size_t)blockIdx.x * D + c] = t;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void colsum_final(const double* __restrict__ part, int nparts,
                                                        int D, int64_t n, float* __restrict__ mean) {
  for (int c = threadIdx.x; c < D; c += blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < nparts; ++b) t += part[(size_t)b * D + c];
    mean[c] = (float)(t / (double)n);
  }
}

}  // namespace

size_t centroid_ws_bytes(int32_t D) { return (size_t)kMaxParts * (size_t)D * sizeof(double) + 256; }

prohd_status centroid_run(const float* X, int64_t n, int32_t D, float* mean, void* ws, size_t ws_bytes,
                          hipStream_t s) {
  if (ws_bytes < centroid_ws_bytes(D)) return fail(PROHD_EWORKSPACE, "centroid: workspace too small");
  const int64_t rows = std::max<int64_t>(256, cdiv(n, kMaxParts));
  const int nparts = (int)cdiv(n, rows);
  double* part = (double*)ws;
  PROHD_LAUNCH("centroid_part", colsum_part, dim3(nparts), dim3(kThreads), 0, s, X, n, (int)D, rows,
               part);
  PROHD_LAUNCH("centroid_final", colsum_final, dim3(1), dim3(kThreads), 0, s, part, nparts, (int)D, n,
               mean);
  return PROHD_OK;
}

}  // namespace prohd
