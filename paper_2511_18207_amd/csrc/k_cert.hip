// Error certificate for a ProHD result (Sec. II-E): for every direction u
// the projected distance H_u (1-D Hausdorff distance of the projections)
// and the spread delta(u) (largest distance of a point of A u B from a line
// parallel to u) bound the true distance,
//     H_u <= H <= H_u + 2 delta(u),
// because |a - b| <= |a.u - b.u| + |a_perp| + |b_perp| for the components
// orthogonal to the line.  The bound holds for any line parallel to u; the
// line through the centroid c of A u B keeps delta small.
//
// The certificate is rigorous for the float32 inputs:
//   * delta: |x - c|^2 is summed in float64 from exactly converted values;
//     the component along u, t = x.u - c.u, comes from the float32
//     projection, whose error is at most (D + 2) 2^-24 (|x| + |x - c|) (a
//     float32 dot product of D terms, and |u| within 2^-23 of 1 on both
//     x.u and c.u); |t| is shrunk by that bound before delta^2 = |x - c|^2 -
//     t^2 is formed, so delta is never underestimated.
//   * H_u: the projections of the target set are binned (8 192 bins over
//     the range of both sets; each work-group bins its share in LDS and
//     merges); each bin keeps its smallest and largest value.
//     For a query value a, every target value lies in a's own bin or beyond
//     the nearest non-empty bins on either side, so the distance to the
//     interval [min, max] of those (up to three) bins bounds min_b |a - b|
//     from below and the distance to their end values bounds it from above.
//     The maxima over the query set bound h_u; both directed parts give
//     H_u.  Both bounds then widen by twice the projection error.
// lb = max(max_u lower H_u, an optional lower value such as the
// inner-minimum-over-the-full-set result of prohd_hd); ub = min_u (upper
// H_u + 2 delta(u)).

#include <algorithm>

#include "common.h"

namespace prohd {
namespace {

constexpr int kBins = 8192;
constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t okey(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u << 1) == 0u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ukey(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}
// non-negative doubles order like their bit patterns
__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x > 0.0 ? x : 0.0);
}
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

struct CertWs {
  float* c;                     // D: centroid of A u B (float32, the line's point)
  double* cu;                   // ndirs: c.u
  double* cA;                   // D float64 column means (scratch)
  float* fA;                    // D float32 means of A
  float* fB;                    // D float32 means of B
  uint32_t* pk;                 // ndirs x 2: min / max projection keys
  unsigned long long* del2;     // ndirs: largest delta^2 (bits)
  unsigned long long* nmax;     // 1: largest |x|^2 (bits)
  unsigned long long* hu;       // ndirs x 2 (target set) x 2 (lo, hi): directed bounds (bits)
  uint32_t* bmin;               // 2 x ndirs x kBins keys
  uint32_t* bmax;
  int32_t* left;                // 2 x ndirs x kBins: last non-empty bin <= b (or -1)
  int32_t* right;               // 2 x ndirs x kBins: first non-empty bin >= b (or kBins)
  void* mean_ws;
  size_t mean_bytes;
};

CertWs cert_layout(Arena& ar, int D, int ndirs) {
  CertWs w;
  w.c = ar.take<float>(D);
  w.cu = ar.take<double>(ndirs);
  w.cA = ar.take<double>(D);
  w.fA = ar.take<float>(D);
  w.fB = ar.take<float>(D);
  w.pk = ar.take<uint32_t>(2 * ndirs);
  w.del2 = ar.take<unsigned long long>(ndirs);
  w.nmax = ar.take<unsigned long long>(1);
  w.hu = ar.take<unsigned long long>(4 * ndirs);
  const size_t nb = (size_t)2 * ndirs * kBins;
  w.bmin = ar.take<uint32_t>(nb);
  w.bmax = ar.take<uint32_t>(nb);
  w.left = ar.take<int32_t>(nb);
  w.right = ar.take<int32_t>(nb);
  w.mean_bytes = centroid_ws_bytes(D);
  w.mean_ws = ar.take<char>(w.mean_bytes);
  return w;
}

__global__ void cert_init(CertWs w, int ndirs) {
  const int64_t nb = (int64_t)2 * ndirs * kBins;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nb; e += (int64_t)gridDim.x * blockDim.x) {
    w.bmin[e] = 0xFFFFFFFFu;
    w.bmax[e] = 0u;
    if (e < ndirs) {
      w.pk[2 * e] = 0xFFFFFFFFu;
      w.pk[2 * e + 1] = 0u;
      w.del2[e] = 0ull;
    }
    if (e < 4 * ndirs) w.hu[e] = 0ull;
    if (e == 0) *w.nmax = 0ull;
  }
}

// c = (nA cA + nB cB) / (nA + nB) in float64, stored as float32; c.u per
// direction in float64 from the float32 values.
__global__ void cert_center(CertWs w, const float* __restrict__ dirs, int ndirs, int D, int64_t nA,
                            int64_t nB) {
  __shared__ float cs[PROHD_MAX_DIM];
  const double N = (double)(nA + nB);
  for (int k = threadIdx.x; k < D; k += blockDim.x) {
    const float v = (float)(((double)nA * (double)w.fA[k] + (double)nB * (double)w.fB[k]) / N);
    cs[k] = v;
    w.c[k] = v;
  }
  __syncthreads();
  for (int d = threadIdx.x; d < ndirs; d += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < D; ++k) s += (double)cs[k] * (double)dirs[(size_t)d * D + k];
    w.cu[d] = s;
  }
}

__device__ __forceinline__ double wave_sum64(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// One wave per row: |x - c|^2 and |x|^2 in float64; lane d < ndirs then
// handles direction d (delta^2 with the projection error margin, range of
// the projections).  Rows of A, then rows of B.
__global__ __launch_bounds__(kThreads) void cert_rows(const float* __restrict__ A, int64_t nA,
                                                      const float* __restrict__ B, int64_t nB, int D,
                                                      const float* __restrict__ PA,
                                                      const float* __restrict__ PB, int ndirs,
                                                      CertWs w) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kThreads) >> 6;
  const double cu = lane < ndirs ? w.cu[lane] : 0.0;
  const double eps = (double)(D + 2) * 5.9604644775390625e-08 * 1.0001;   // (D + 2) 2^-24 (1 + 1e-4)
  double dmax = 0.0, nmx = 0.0;
  uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
  for (int64_t r = wid; r < nA + nB; r += nw) {
    const bool inA = r < nA;
    const int64_t i = inA ? r : r - nA;
    const float* x = (inA ? A : B) + i * D;
    double s = 0.0, q = 0.0;
    for (int k = lane; k < D; k += 64) {
      const double xv = (double)x[k];
      const double dv = xv - (double)w.c[k];
      s = fma(dv, dv, s);
      q = fma(xv, xv, q);
    }
    s = wave_sum64(s);
    q = wave_sum64(q);
    nmx = fmax(nmx, q);
    if (lane < ndirs) {
      const int64_t n = inA ? nA : nB;
      const float pv = (inA ? PA : PB)[(size_t)lane * n + i];
      // margin: dot-product rounding plus |u| != 1 on both x.u and c.u
      const double t = fabs((double)pv - cu) - eps * (sqrt(q) + sqrt(s));
      const double tt = t > 0.0 ? t : 0.0;
      dmax = fmax(dmax, s - tt * tt);
      const uint32_t k = okey(pv);
      kmin = min(kmin, k);
      kmax = max(kmax, k);
    }
  }
  if (lane < ndirs) {
    atomicMax(&w.del2[lane], dbits(dmax));
    atomicMin(&w.pk[2 * lane], kmin);
    atomicMax(&w.pk[2 * lane + 1], kmax);
  }
  if (lane == 0) atomicMax(w.nmax, dbits(nmx));
}

struct BinMap {
  double lo, scale;
};

__device__ __forceinline__ BinMap bin_map(const CertWs& w, int d) {
  const double lo = (double)ukey(w.pk[2 * d]), hi = (double)ukey(w.pk[2 * d + 1]);
  BinMap m;
  m.lo = lo;
  m.scale = hi > lo ? (double)kBins / (hi - lo) : 0.0;
  return m;
}

__device__ __forceinline__ int bin_of(const BinMap& m, float v) {
  const double b = floor(((double)v - m.lo) * m.scale);
  return b < 0.0 ? 0 : (b >= (double)kBins ? kBins - 1 : (int)b);
}

// Bin statistics of the target set s (0: A, 1: B) for direction blockIdx.y:
// each work-group keeps private LDS bins for its share of the values, then
// merges its non-empty bins into the global ones.
__global__ __launch_bounds__(kThreads) void cert_bins(const float* __restrict__ P, int64_t n, int s,
                                                      int ndirs, CertWs w) {
  __shared__ uint32_t lmn[kBins], lmx[kBins];
  const int d = blockIdx.y;
  const BinMap m = bin_map(w, d);
  for (int b = threadIdx.x; b < kBins; b += kThreads) {
    lmn[b] = 0xFFFFFFFFu;
    lmx[b] = 0u;
  }
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const float v = P[(size_t)d * n + i];
    const int b = bin_of(m, v);
    const uint32_t k = okey(v);
    atomicMin(&lmn[b], k);
    atomicMax(&lmx[b], k);
  }
  __syncthreads();
  uint32_t* bmn = w.bmin + ((size_t)s * ndirs + d) * kBins;
  uint32_t* bmx = w.bmax + ((size_t)s * ndirs + d) * kBins;
  for (int b = threadIdx.x; b < kBins; b += kThreads) {
    if (lmx[b] != 0u) {
      atomicMin(&bmn[b], lmn[b]);
      atomicMax(&bmx[b], lmx[b]);
    }
  }
}

// Nearest non-empty bins: one work-group per (target set, direction).
__global__ __launch_bounds__(1024) void cert_scan(int ndirs, CertWs w) {
  constexpr int PER = kBins / 1024;
  static_assert(PER >= 1 && kBins % 1024 == 0, "bins per thread");
  __shared__ int32_t lastv[1024], firstv[1024];
  const size_t base = (size_t)blockIdx.x * kBins;
  const int t = threadIdx.x;
  int32_t last = -1, first = kBins;
  for (int q = 0; q < PER; ++q) {
    const int b = t * PER + q;
    if (w.bmax[base + b] != 0u) last = b;
  }
  for (int q = PER - 1; q >= 0; --q) {
    const int b = t * PER + q;
    if (w.bmax[base + b] != 0u) first = b;
  }
  lastv[t] = last;
  firstv[t] = first;
  __syncthreads();
  // inclusive max-scan (last) and suffix min-scan (first) over the threads
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t a = t >= off ? lastv[t - off] : -1;
    const int32_t f = t + off < 1024 ? firstv[t + off] : kBins;
    __syncthreads();
    lastv[t] = max(lastv[t], a);
    firstv[t] = min(firstv[t], f);
    __syncthreads();
  }
  int32_t run = t > 0 ? lastv[t - 1] : -1;
  for (int q = 0; q < PER; ++q) {
    const int b = t * PER + q;
    if (w.bmax[base + b] != 0u) run = b;
    w.left[base + b] = run;
  }
  run = t < 1023 ? firstv[t + 1] : kBins;
  for (int q = PER - 1; q >= 0; --q) {
    const int b = t * PER + q;
    if (w.bmax[base + b] != 0u) run = b;
    w.right[base + b] = run;
  }
}

// Directed bounds of h_u(Q, S): queries from P (set 1 - s), targets of set
// s; the target's bin tables are staged in LDS once per work-group.
__global__ __launch_bounds__(kThreads) void cert_query(const float* __restrict__ P, int64_t n, int s,
                                                       int ndirs, CertWs w) {
  __shared__ float tmn[kBins], tmx[kBins];
  __shared__ int16_t tl[kBins], tr[kBins];
  __shared__ unsigned long long rlo[kThreads / 64], rhi[kThreads / 64];
  const int d = blockIdx.y;
  const BinMap m = bin_map(w, d);
  const size_t base = ((size_t)s * ndirs + d) * kBins;
  for (int b = threadIdx.x; b < kBins; b += kThreads) {
    const bool ne = w.bmax[base + b] != 0u;
    tmn[b] = ne ? ukey(w.bmin[base + b]) : 0.f;
    tmx[b] = ne ? ukey(w.bmax[base + b]) : 0.f;
    tl[b] = (int16_t)w.left[base + b];
    tr[b] = (int16_t)(w.right[base + b] < kBins ? w.right[base + b] : -1);
  }
  __syncthreads();
  double lo_max = 0.0, hi_max = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const float v = P[(size_t)d * n + i];
    const double a = (double)v;
    const int b = bin_of(m, v);
    int cand[3];
    cand[0] = (tl[b] == b) ? b : -1;              // own bin when non-empty
    cand[1] = b > 0 ? tl[b - 1] : -1;             // nearest non-empty below
    cand[2] = b < kBins - 1 ? tr[b + 1] : -1;     // nearest non-empty above
    double lo = 1.0e308, hi = 1.0e308;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = cand[c];
      if (k >= 0) {
        const double mn = (double)tmn[k], mx = (double)tmx[k];
        const double dist = a < mn ? mn - a : (a > mx ? a - mx : 0.0);
        lo = fmin(lo, dist);
        hi = fmin(hi, fmin(fabs(a - mn), fabs(a - mx)));
      }
    }
    lo_max = fmax(lo_max, lo);
    hi_max = fmax(hi_max, hi);
  }
  // work-group maxima, then one atomic per work-group
  unsigned long long bl = dbits(lo_max), bh = dbits(hi_max);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long ol = __shfl_xor(bl, off), oh = __shfl_xor(bh, off);
    bl = ol > bl ? ol : bl;
    bh = oh > bh ? oh : bh;
  }
  if ((threadIdx.x & 63) == 0) {
    rlo[threadIdx.x >> 6] = bl;
    rhi[threadIdx.x >> 6] = bh;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kThreads / 64; ++q) {
      bl = rlo[q] > bl ? rlo[q] : bl;
      bh = rhi[q] > bh ? rhi[q] : bh;
    }
    atomicMax(&w.hu[4 * d + 2 * s], bl);
    atomicMax(&w.hu[4 * d + 2 * s + 1], bh);
  }
}

__global__ void cert_final(CertWs w, int ndirs, int D, const prohd_result* __restrict__ lower,
                           prohd_cert* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double emax = (double)(D + 2) * 5.9604644775390625e-08 * 1.0001 * sqrt(bitsd(*w.nmax));
  double hu_lo = 0.0, hu_hi = 0.0, ub = 1.0e308, dmin = 1.0e308;
  int best = 0;
  for (int d = 0; d < ndirs; ++d) {
    const double lo = fmax(0.0, fmax(bitsd(w.hu[4 * d]), bitsd(w.hu[4 * d + 2])) - 2.0 * emax);
    const double hi = fmax(bitsd(w.hu[4 * d + 1]), bitsd(w.hu[4 * d + 3])) + 2.0 * emax;
    const double del = sqrt(bitsd(w.del2[d])) * (1.0 + 1e-15);
    hu_lo = fmax(hu_lo, lo);
    hu_hi = fmax(hu_hi, hi);
    dmin = fmin(dmin, del);
    if (hi + 2.0 * del < ub) {
      ub = hi + 2.0 * del;
      best = d;
    }
  }
  prohd_cert r;
  r.lb = hu_lo;
  if (lower && lower->status == 0) r.lb = fmax(r.lb, lower->H);
  r.ub = ub;
  r.hu_lo = hu_lo;
  r.hu_hi = hu_hi;
  r.delta_min = dmin;
  r.proj_err = emax;
  r.best_dir = best;
  r.status = 0;
  *out = r;
}

}  // namespace

size_t cert_ws_bytes(int32_t D, int32_t ndirs) {
  Arena ar(nullptr);
  cert_layout(ar, D, ndirs);
  return ar.used + 256;
}

prohd_status cert_run(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      const float* dirs, int32_t ndirs, const float* PA, const float* PB,
                      const prohd_result* lower, prohd_cert* out, void* ws, size_t ws_bytes,
                      hipStream_t s) {
  Arena ar(ws);
  CertWs w = cert_layout(ar, D, ndirs);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "certificate: workspace too small");
  const int cus = cu_count();
  PROHD_LAUNCH("cert_init", cert_init, dim3(std::min<int64_t>(cdiv((int64_t)2 * ndirs * kBins, kThreads), 4096)),
               dim3(kThreads), 0, s, w, (int)ndirs);
  prohd_status st = centroid_run(A, nA, D, w.fA, w.mean_ws, w.mean_bytes, s);
  if (!st) st = centroid_run(B, nB, D, w.fB, w.mean_ws, w.mean_bytes, s);
  if (st) return st;
  PROHD_LAUNCH("cert_center", cert_center, dim3(1), dim3(kThreads), 0, s, w, dirs, (int)ndirs, (int)D, nA,
               nB);
  const int64_t waves = std::min<int64_t>(nA + nB, (int64_t)cus * 32);
  PROHD_LAUNCH("cert_rows", cert_rows, dim3((unsigned)cdiv(waves * 64, kThreads)), dim3(kThreads), 0, s, A,
               nA, B, nB, (int)D, PA, PB, (int)ndirs, w);
  const int64_t ns[2] = {nA, nB};
  const float* Ps[2] = {PA, PB};
  for (int t = 0; t < 2; ++t) {
    const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(ns[t], 16 * kThreads), std::max(1, 2 * cus / ndirs))),
                 (unsigned)ndirs);
    PROHD_LAUNCH("cert_bins", cert_bins, g, dim3(kThreads), 0, s, Ps[t], ns[t], t, (int)ndirs, w);
  }
  PROHD_LAUNCH("cert_scan", cert_scan, dim3((unsigned)(2 * ndirs)), dim3(1024), 0, s, (int)ndirs, w);
  for (int t = 0; t < 2; ++t) {   // target set t, queries from the other set
    const int q = 1 - t;
    const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(ns[q], 16 * kThreads), std::max(1, 2 * cus / ndirs))),
                 (unsigned)ndirs);
    PROHD_LAUNCH("cert_query", cert_query, g, dim3(kThreads), 0, s, Ps[q], ns[q], t, (int)ndirs, w);
  }
  PROHD_LAUNCH("cert_final", cert_final, dim3(1), dim3(64), 0, s, w, (int)ndirs, (int)D, lower, out);
  return PROHD_OK;
}

}  // namespace prohd
