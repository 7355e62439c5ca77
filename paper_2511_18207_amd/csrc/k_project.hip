// Directions and projections: the projection steps of the paper's Alg. 1
// (onto the centroid axis) and Alg. 2 (onto each principal component), for
// both sets, plus the driver that chains statistics -> eigensolve ->
// projection without a host synchronisation.
//
// project_rows streams the n x D rows once from HBM (coalesced float4 loads
// into an LDS tile of 64 rows, the next tile prefetched in registers while
// the current one is used).  Each of the four waves takes a quarter of the
// columns; lane = row.  Directions are read transposed (D x 8 per group), so
// the eight values a k-step needs are wave-uniform scalar loads and the inner
// loop is eight FMAs per LDS read.  Quarter sums meet in LDS and are written
// direction-major: P[d * n + i], one coalesced store per direction.
// This pass is bound by HBM bandwidth: 4 D bytes read and 4 (m+1) bytes
// written per row.

#include "common.h"

namespace prohd {

size_t stats_ws_bytes(int64_t nA, int64_t nB, int32_t D);
prohd_status stats_run(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                       double* C, double* u0, int32_t* status, void* ws, size_t ws_bytes,
                       hipStream_t s);
size_t eig_ws_bytes(int32_t D, int32_t m);
prohd_status eig_run(double* C, int32_t D, int32_t m, const double* u0, float* dirs, double* evals,
                     const int32_t* status, void* ws, size_t ws_bytes, hipStream_t s);

namespace {

constexpr int kRows = 64;     // rows per tile
constexpr int kThreads = 256;

// Ut[k * ndp + d] = dirs[d * D + k] for d < ndirs, zero elsewhere.
__global__ void transpose_dirs(const float* __restrict__ dirs, int ndirs, int D, int DP, int ndp,
                               float* __restrict__ Ut) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < DP * ndp; e += gridDim.x * blockDim.x) {
    const int k = e / ndp, d = e - k * ndp;
    Ut[e] = (d < ndirs && k < D) ? dirs[(size_t)d * D + k] : 0.f;
  }
}

template <int DP, bool VEC>
__global__ __launch_bounds__(kThreads) void project_rows(const float* __restrict__ A, int64_t nA,
                                                         const float* __restrict__ B, int64_t nB,
                                                         int D, const float* __restrict__ Ut,
                                                         int ndirs, int ndp,
                                                         float* __restrict__ PA,
                                                         float* __restrict__ PB) {
  constexpr int ST = DP + 4;                        // LDS row stride (floats)
  constexpr int KW = DP / 4;                        // columns per wave
  constexpr int NF = VEC ? (kRows * DP / 4 + kThreads - 1) / kThreads   // float4 per thread
                         : (kRows * DP + kThreads - 1) / kThreads;      // floats per thread
  __shared__ __attribute__((aligned(16))) float tile[kRows * ST];
  __shared__ float red[4][8][kRows];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int64_t tilesA = (nA + kRows - 1) / kRows;
  const int64_t tiles = tilesA + (nB + kRows - 1) / kRows;
  const int ngroups = (ndirs + 7) / 8;

  // LDS destinations of this thread's loads (identical for every tile)
  int dst[NF];
  const int D4 = D / 4;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const int f = tid + kThreads * i;
    if (VEC) {
      const int r = f / (D4 > 0 ? D4 : 1), c4 = f - r * D4;
      dst[i] = (f < kRows * D4) ? r * ST + 4 * c4 : -1;
    } else {
      const int r = f / D, c = f - r * D;
      dst[i] = (f < kRows * D) ? r * ST + c : -1;
    }
  }
  float4 buf4[VEC ? NF : 1];
  float buf1[VEC ? 1 : NF];

  auto load = [&](int64_t tl) {
    const bool inA = tl < tilesA;
    const float* X = inA ? A : B;
    const int64_t n = inA ? nA : nB;
    const int64_t r0 = (inA ? tl : tl - tilesA) * kRows;
    const int64_t lim = (min<int64_t>(n, r0 + kRows) - r0) * D;  // valid floats in the tile
    const float* base = X + r0 * D;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int f = tid + kThreads * i;
      if (VEC) {
        buf4[i] = (4 * (int64_t)f < lim && dst[i] >= 0)
                      ? reinterpret_cast<const float4*>(base)[f]
                      : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        buf1[i] = ((int64_t)f < lim && dst[i] >= 0) ? base[f] : 0.f;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      if (dst[i] >= 0) {
        if (VEC) *reinterpret_cast<float4*>(&tile[dst[i]]) = buf4[i];
        else tile[dst[i]] = buf1[i];
      }
    }
  };

  int64_t tl = blockIdx.x;
  if (tl < tiles) load(tl);
  for (; tl < tiles; tl += gridDim.x) {
    // pad columns D..DP stay zero: clear once per tile when D < DP
    __syncthreads();
    if (D < DP) {
      for (int e = tid; e < kRows * ST; e += kThreads) tile[e] = 0.f;
      __syncthreads();
    }
    store();
    __syncthreads();
    const int64_t nxt = tl + gridDim.x;
    if (nxt < tiles) load(nxt);

    const bool inA = tl < tilesA;
    const int64_t n = inA ? nA : nB;
    const int64_t r0 = (inA ? tl : tl - tilesA) * kRows;
    float* P = inA ? PA : PB;
    const float* xr = &tile[lane * ST + wave * KW];
    for (int g = 0; g < ngroups; ++g) {
      float acc[8];
#pragma unroll
      for (int d = 0; d < 8; ++d) acc[d] = 0.f;
      const float* u = Ut + (size_t)(wave * KW) * ndp + 8 * g;
#pragma unroll 4
      for (int k = 0; k < KW; ++k) {
        const float x = xr[k];
        const float* uk = u + (size_t)k * ndp;
#pragma unroll
        for (int d = 0; d < 8; ++d) acc[d] = fmaf(x, uk[d], acc[d]);
      }
#pragma unroll
      for (int d = 0; d < 8; ++d) red[wave][d][lane] = acc[d];
      __syncthreads();
      // 256 threads: row = tid % 64, two directions each
      {
        const int row = tid & 63;
        const int d0 = (tid >> 6) * 2;
#pragma unroll
        for (int dd = 0; dd < 2; ++dd) {
          const int d = d0 + dd;
          const float v = (red[0][d][row] + red[1][d][row]) + (red[2][d][row] + red[3][d][row]);
          const int dir = 8 * g + d;
          if (dir < ndirs && r0 + row < n) P[(size_t)dir * n + r0 + row] = v;
        }
      }
      __syncthreads();
    }
  }
}

struct ProjLayout {
  int32_t* status;
  double* C;
  double* u0;
  float* Ut;
  void* sub;
  size_t sub_bytes;
};

ProjLayout proj_layout(Arena& ar, int64_t nA, int64_t nB, int D, int ndirs) {
  ProjLayout L;
  const int DP = pad_dim(D);
  const int ndp = ((ndirs + 7) / 8) * 8;
  L.status = ar.take<int32_t>(64);
  L.C = ar.take<double>((size_t)DP * DP);
  L.u0 = ar.take<double>(DP);
  L.Ut = ar.take<float>((size_t)DP * ndp);
  L.sub_bytes = std::max(stats_ws_bytes(nA, nB, D), eig_ws_bytes(D, ndirs - 1));
  L.sub = ar.take<char>(L.sub_bytes);
  return L;
}

template <int DP>
prohd_status launch_project(const float* A, int64_t nA, const float* B, int64_t nB, int D,
                            const float* Ut, int ndirs, int ndp, float* PA, float* PB,
                            hipStream_t s) {
  const int64_t tiles = cdiv(nA, kRows) + cdiv(nB, kRows);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, 2 * cu_count()));
  const bool vec = (D % 4 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0);
  if (vec) {
    PROHD_LAUNCH("project_rows", (project_rows<DP, true>), dim3(grid), dim3(kThreads), 0, s, A, nA, B,
                 nB, D, Ut, ndirs, ndp, PA, PB);
  } else {
    PROHD_LAUNCH("project_rows", (project_rows<DP, false>), dim3(grid), dim3(kThreads), 0, s, A, nA, B,
                 nB, D, Ut, ndirs, ndp, PA, PB);
  }
  return PROHD_OK;
}

}  // namespace

size_t project_ws_bytes(int64_t nA, int64_t nB, int32_t D, int32_t ndirs) {
  Arena ar(nullptr);
  proj_layout(ar, nA, nB, D, ndirs);
  return ar.used + 256;
}

prohd_status project_run(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                         int32_t m, bool dirs_given, float* dirs, float* projA, float* projB,
                         double* evals, int32_t* status, void* ws, size_t ws_bytes, hipStream_t s) {
  const int ndirs = m + 1;
  Arena ar(ws);
  ProjLayout L = proj_layout(ar, nA, nB, D, ndirs);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "project: workspace too small");
  int32_t* st = status ? status : L.status;
  prohd_status r = zero_bytes(st, sizeof(int32_t), s);
  if (r) return r;
  if (!dirs_given) {
    r = stats_run(A, nA, B, nB, D, L.C, L.u0, st, L.sub, L.sub_bytes, s);
    if (r) return r;
    r = eig_run(L.C, D, m, L.u0, dirs, evals, st, L.sub, L.sub_bytes, s);
    if (r) return r;
  }
  const int DP = pad_dim(D);
  const int ndp = ((ndirs + 7) / 8) * 8;
  PROHD_LAUNCH("project_dirs", transpose_dirs, dim3(std::max(1, std::min(64, DP * ndp / 256))),
               dim3(256), 0, s, dirs, ndirs, D, DP, ndp, L.Ut);
  switch (DP) {
    case 16: return launch_project<16>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    case 32: return launch_project<32>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    case 64: return launch_project<64>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    case 128: return launch_project<128>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    case 256: return launch_project<256>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    default: return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM");
  }
}

}  // namespace prohd
