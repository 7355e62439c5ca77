// Directions and projections: the projection steps of the paper's Alg. 1
// (onto the centroid axis) and Alg. 2 (onto each principal component), for
// both sets, plus the driver that chains statistics -> eigensolve ->
// projection without a host synchronisation.
//
// project_rows streams the n x D rows once from HBM: a work-group of 512
// threads owns 512 rows (one per thread) and walks their columns in chunks of
// 32 (coalesced 128-byte row segments staged through LDS, the next chunk
// prefetched in registers while the current one is used).  The directions
// (up to 32 per launch) are stored k-major and read as wave-uniform scalar
// loads, so a k-step is one LDS read of x feeding 8-32 FMAs with scalar
// operands; the finished row writes P[d * n + i] (coalesced across the wave
// per direction).
// This pass is bound by HBM bandwidth: 4 D bytes read and 4 (m+1) bytes
// written per row.

#include "batch.h"
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

constexpr int kTileRows = 512;  // rows per tile: one per thread
constexpr int kThreads = 512;

// Directions in blocks of 32: block b (directions 32b..) is stored k-major,
// Ut[32 b DP + k nd8 + j] = dirs[32 b + j][k], nd8 = 8 ceil(nd/8) for the
// nd directions of that block; zero for k >= D.
__global__ void transpose_dirs(const float* __restrict__ dirs, int ndirs, int D, int DP,
                               float* __restrict__ Ut) {
  const int nblk = (ndirs + 31) / 32;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nblk * 32 * DP; e += gridDim.x * blockDim.x) {
    const int b = e / (32 * DP);
    const int r = e - b * 32 * DP;
    const int nd = min(32, ndirs - 32 * b);
    const int nd8 = 8 * ((nd + 7) / 8);
    const int k = r / nd8, j = r - k * nd8;
    if (k >= DP) continue;
    Ut[(size_t)b * 32 * DP + r] = (j < nd && k < D) ? dirs[(size_t)(32 * b + j) * D + k] : 0.f;
  }
}

template <int DP, int NG, bool VEC>
__global__ __launch_bounds__(kThreads) void project_rows(const float* __restrict__ A, int64_t nA,
                                                         const float* __restrict__ B, int64_t nB,
                                                         int D, const float* __restrict__ Ut,
                                                         int ndirs,
                                                         float* __restrict__ PA,
                                                         float* __restrict__ PB) {
  constexpr int KC = DP < 32 ? DP : 32;             // columns per chunk
  constexpr int NCH = DP / KC;                      // chunks per row
  constexpr int ST = KC + 4;                        // LDS row stride (floats)
  constexpr int ND = 8 * NG;                        // directions, padded
  constexpr int F4R = KC / 4;                       // float4 per row chunk
  constexpr int NF = kTileRows * F4R / kThreads;    // float4 per thread per chunk
  __shared__ __attribute__((aligned(16))) float xt[kTileRows * ST];
  const int tid = threadIdx.x;
  const int64_t tilesA = (nA + kTileRows - 1) / kTileRows;
  const int64_t tiles = tilesA + (nB + kTileRows - 1) / kTileRows;

  float4 buf[NF];
  // chunk c of tile tl: row f / F4R, float4 f % F4R of columns [c KC, c KC + KC)
  auto load = [&](int64_t tl, int c) {
    const bool inA = tl < tilesA;
    const float* X = inA ? A : B;
    const int64_t n = inA ? nA : nB;
    const int64_t r0 = (inA ? tl : tl - tilesA) * kTileRows;
    const int rows = (int)min<int64_t>(kTileRows, n - r0);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int f = tid + kThreads * i;
      const int r = f / F4R, j = f - r * F4R;
      const int k = c * KC + 4 * j;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < rows) {
        const float* src = X + (r0 + r) * D + k;
        if (VEC) {
          if (k < D) v = *reinterpret_cast<const float4*>(src);
        } else {
          if (k + 0 < D) v.x = src[0];
          if (k + 1 < D) v.y = src[1];
          if (k + 2 < D) v.z = src[2];
          if (k + 3 < D) v.w = src[3];
        }
      }
      buf[i] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int f = tid + kThreads * i;
      const int r = f / F4R, j = f - r * F4R;
      *reinterpret_cast<float4*>(&xt[r * ST + 4 * j]) = buf[i];
    }
  };

  int64_t tl = blockIdx.x;
  if (tl < tiles) load(tl, 0);
  for (; tl < tiles; tl += gridDim.x) {
    float acc[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] = 0.f;
    for (int c = 0; c < NCH; ++c) {
      __syncthreads();
      store();
      __syncthreads();
      // prefetch the next chunk (or the first chunk of the next tile)
      if (c + 1 < NCH) load(tl, c + 1);
      else if (tl + gridDim.x < tiles) load(tl + gridDim.x, 0);
      // row tid: x from LDS; direction values are wave-uniform scalar loads
      // (all waves work on the same chunk, so its KC x ND values stay in the
      // scalar cache)
      const float* xr = &xt[tid * ST];
      const float* uc = Ut + (size_t)(c * KC) * ND;
#pragma unroll 2
      for (int k4 = 0; k4 < KC / 4; ++k4) {
        const float4 x = *reinterpret_cast<const float4*>(xr + 4 * k4);
        const float xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const float* uk = uc + (4 * k4 + kk) * ND;
#pragma unroll
          for (int d4 = 0; d4 < ND / 4; ++d4) {
            const float4 u = *reinterpret_cast<const float4*>(uk + 4 * d4);
            acc[4 * d4 + 0] = fmaf(xs[kk], u.x, acc[4 * d4 + 0]);
            acc[4 * d4 + 1] = fmaf(xs[kk], u.y, acc[4 * d4 + 1]);
            acc[4 * d4 + 2] = fmaf(xs[kk], u.z, acc[4 * d4 + 2]);
            acc[4 * d4 + 3] = fmaf(xs[kk], u.w, acc[4 * d4 + 3]);
          }
        }
      }
    }
    const bool inA = tl < tilesA;
    const int64_t n = inA ? nA : nB;
    const int64_t row = (inA ? tl : tl - tilesA) * kTileRows + tid;
    float* P = inA ? PA : PB;
    if (row < n) {
#pragma unroll
      for (int d = 0; d < ND; ++d)
        if (d < ndirs) P[(size_t)d * n + row] = acc[d];
    }
  }
}

// Batched: one item = one 512-row tile of one set of one pair (directions
// of that pair, at most 32, in Ut as above).  Same per-row arithmetic as
// project_rows; the next chunk of the tile is prefetched in registers.
template <int DP, int NG, bool VEC>
__global__ __launch_bounds__(kThreads) void project_batch(const ProjJob* __restrict__ jobs, int njobs,
                                                          int D, const float* __restrict__ Ubase) {
  constexpr int KC = DP < 32 ? DP : 32;
  constexpr int NCH = DP / KC;
  constexpr int ST = KC + 4;
  constexpr int ND = 8 * NG;
  constexpr int F4R = KC / 4;
  constexpr int NF = kTileRows * F4R / kThreads;
  __shared__ __attribute__((aligned(16))) float xt[kTileRows * ST];
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const ProjJob j = jobs[it];
    const int rows = (int)min<int64_t>(kTileRows, j.n - j.r0);
    float4 buf[NF];
    auto load = [&](int c) {
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const int f = tid + kThreads * i;
        const int r = f / F4R, q = f - r * F4R;
        const int k = c * KC + 4 * q;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < rows) {
          const float* src = j.X + (j.r0 + r) * D + k;
          if (VEC) {
            if (k < D) v = *reinterpret_cast<const float4*>(src);
          } else {
            if (k + 0 < D) v.x = src[0];
            if (k + 1 < D) v.y = src[1];
            if (k + 2 < D) v.z = src[2];
            if (k + 3 < D) v.w = src[3];
          }
        }
        buf[i] = v;
      }
    };
    float acc[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] = 0.f;
    load(0);
    for (int c = 0; c < NCH; ++c) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const int f = tid + kThreads * i;
        const int r = f / F4R, q = f - r * F4R;
        *reinterpret_cast<float4*>(&xt[r * ST + 4 * q]) = buf[i];
      }
      __syncthreads();
      if (c + 1 < NCH) load(c + 1);
      const float* xr = &xt[tid * ST];
      const float* uc = Ubase + j.ut_off + (size_t)(c * KC) * ND;
#pragma unroll 2
      for (int k4 = 0; k4 < KC / 4; ++k4) {
        const float4 x = *reinterpret_cast<const float4*>(xr + 4 * k4);
        const float xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const float* uk = uc + (4 * k4 + kk) * ND;
#pragma unroll
          for (int d4 = 0; d4 < ND / 4; ++d4) {
            const float4 u = *reinterpret_cast<const float4*>(uk + 4 * d4);
            acc[4 * d4 + 0] = fmaf(xs[kk], u.x, acc[4 * d4 + 0]);
            acc[4 * d4 + 1] = fmaf(xs[kk], u.y, acc[4 * d4 + 1]);
            acc[4 * d4 + 2] = fmaf(xs[kk], u.z, acc[4 * d4 + 2]);
            acc[4 * d4 + 3] = fmaf(xs[kk], u.w, acc[4 * d4 + 3]);
          }
        }
      }
    }
    const int64_t row = j.r0 + tid;
    if (tid < rows) {
#pragma unroll
      for (int d = 0; d < ND; ++d)
        if (d < j.ndirs) j.P[(size_t)d * j.n + row] = acc[d];
    }
  }
}

// Batched transpose: one work-group per job.
__global__ void transpose_batch(const TransJob* __restrict__ jobs, int njobs, int D, int DP) {
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const TransJob j = jobs[it];
    const int nblk = (j.ndirs + 31) / 32;
    for (int e = threadIdx.x; e < nblk * 32 * DP; e += blockDim.x) {
      const int b = e / (32 * DP);
      const int r = e - b * 32 * DP;
      const int nd = min(32, j.ndirs - 32 * b);
      const int nd8 = 8 * ((nd + 7) / 8);
      const int k = r / nd8, q = r - k * nd8;
      if (k >= DP) continue;
      j.Ut[(size_t)b * 32 * DP + r] = (q < nd && k < D) ? j.dirs[(size_t)(32 * b + q) * D + k] : 0.f;
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
  L.Ut = ar.take<float>((size_t)DP * ((ndirs + 31) / 32) * 32);
  L.sub_bytes = std::max(stats_ws_bytes(nA, nB, D), eig_ws_bytes(D, ndirs - 1));
  L.sub = ar.take<char>(L.sub_bytes);
  return L;
}

template <int DP, int NG>
prohd_status launch_project_ng(const float* A, int64_t nA, const float* B, int64_t nB, int D,
                               const float* Ut, int ndirs, float* PA, float* PB, hipStream_t s) {
  const int64_t tiles = cdiv(nA, kTileRows) + cdiv(nB, kTileRows);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cu_count()));
  const bool vec = (D % 4 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0);
  if (vec) {
    PROHD_LAUNCH("project_rows", (project_rows<DP, NG, true>), dim3(grid), dim3(kThreads), 0, s, A, nA,
                 B, nB, D, Ut, ndirs, PA, PB);
  } else {
    PROHD_LAUNCH("project_rows", (project_rows<DP, NG, false>), dim3(grid), dim3(kThreads), 0, s, A,
                 nA, B, nB, D, Ut, ndirs, PA, PB);
  }
  return PROHD_OK;
}

// Direction groups of 8 per launch: 1, 2, 3 or 4 groups (up to 32 directions).
template <int DP>
prohd_status launch_project(const float* A, int64_t nA, const float* B, int64_t nB, int D,
                            const float* Ut, int ndirs, int ndp, float* PA, float* PB,
                            hipStream_t s) {
  for (int d0 = 0; d0 < ndirs; d0 += 32) {
    const int nd = std::min(32, ndirs - d0);
    const int ng = (nd + 7) / 8;
    const float* U = Ut + (size_t)d0 * DP;   // Ut is stored per 32-direction block
    float* pa = PA + (size_t)d0 * nA;
    float* pb = PB + (size_t)d0 * nB;
    prohd_status r;
    switch (ng) {
      case 1: r = launch_project_ng<DP, 1>(A, nA, B, nB, D, U, nd, pa, pb, s); break;
      case 2: r = launch_project_ng<DP, 2>(A, nA, B, nB, D, U, nd, pa, pb, s); break;
      case 3: r = launch_project_ng<DP, 3>(A, nA, B, nB, D, U, nd, pa, pb, s); break;
      default: r = launch_project_ng<DP, 4>(A, nA, B, nB, D, U, nd, pa, pb, s); break;
    }
    if (r) return r;
  }
  (void)ndp;
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
               dim3(256), 0, s, dirs, ndirs, D, DP, L.Ut);
  switch (DP) {
    case 16: return launch_project<16>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    case 32: return launch_project<32>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    case 64: return launch_project<64>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    case 128: return launch_project<128>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    case 256: return launch_project<256>(A, nA, B, nB, D, L.Ut, ndirs, ndp, projA, projB, s);
    default: return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM");
  }
}

template <int DP, int NG>
prohd_status batch_project_ng(int D, bool vec, const float* U, const ProjJob* jobs, int njobs, int grid,
                              hipStream_t s) {
  if (vec) {
    PROHD_LAUNCH("batch_project", (project_batch<DP, NG, true>), dim3(grid), dim3(kThreads), 0, s, jobs,
                 njobs, D, U);
  } else {
    PROHD_LAUNCH("batch_project", (project_batch<DP, NG, false>), dim3(grid), dim3(kThreads), 0, s, jobs,
                 njobs, D, U);
  }
  return PROHD_OK;
}

template <int DP>
prohd_status batch_project_dp(int D, int ndirs, bool vec, const float* U, const ProjJob* jobs, int njobs,
                              int grid, hipStream_t s) {
  switch ((ndirs + 7) / 8) {
    case 1: return batch_project_ng<DP, 1>(D, vec, U, jobs, njobs, grid, s);
    case 2: return batch_project_ng<DP, 2>(D, vec, U, jobs, njobs, grid, s);
    case 3: return batch_project_ng<DP, 3>(D, vec, U, jobs, njobs, grid, s);
    case 4: return batch_project_ng<DP, 4>(D, vec, U, jobs, njobs, grid, s);
    default: return fail(PROHD_EUNSUPPORTED, "batched projection: more than 32 directions");
  }
}

prohd_status batch_project(int DP, int D, int ndirs, bool vec, const float* U, const ProjJob* jobs,
                           int njobs, int grid, hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  vec = vec && D % 4 == 0;
  switch (DP) {
    case 16: return batch_project_dp<16>(D, ndirs, vec, U, jobs, njobs, grid, s);
    case 32: return batch_project_dp<32>(D, ndirs, vec, U, jobs, njobs, grid, s);
    case 64: return batch_project_dp<64>(D, ndirs, vec, U, jobs, njobs, grid, s);
    case 128: return batch_project_dp<128>(D, ndirs, vec, U, jobs, njobs, grid, s);
    case 256: return batch_project_dp<256>(D, ndirs, vec, U, jobs, njobs, grid, s);
    default: return fail(PROHD_EUNSUPPORTED, "batched: unsupported padded dimension");
  }
}

prohd_status batch_transpose(int D, int DP, const TransJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  const int grid = std::min(njobs, 8 * cu_count());
  PROHD_LAUNCH("batch_transpose", transpose_batch, dim3(grid), dim3(256), 0, s, jobs, njobs, D, DP);
  return PROHD_OK;
}

}  // namespace prohd
