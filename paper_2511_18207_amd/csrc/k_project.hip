// Directions and projections: the projection steps of the paper's Alg. 1
// (onto the centroid axis) and Alg. 2 (onto each principal component), for
// both sets, plus the host routine that chains statistics -> eigensolve ->
// projection without a host synchronisation.
//
// The projection of n rows onto up to 33 directions is a skinny product
// (n x D) (D x nd) done on the FP32 matrix cores: v_mfma_f32_16x16x4f32 with
// the directions as the 16-row A operand and 16 points as the B operand, so
// the 16 x 16 result block holds direction-major values that store straight
// into P[d * n + i] (16 consecutive points = 64 contiguous bytes per
// direction).  A wave owns 16 rows at a time and reads them straight from HBM
// into registers: lane (p, g) = (lane % 16, lane / 16) holds the float4s
// x[p][16 t + 4 g .. + 3], t = 0 .. D/16 - 1, so the four lane groups of a
// point read 64 contiguous bytes per load and the contraction index k is
// permuted identically for both operands (MFMA step (t, c) contracts
// k = 16 t + 4 g + c in lane group g).  The directions sit in LDS for the
// whole launch (one copy per work-group, row stride DP + 4 so that the 16
// directions of a read hit distinct banks).  Direction counts of 16 n + 1
// (the default m + 1 = 17) take the last direction on the vector ALUs with
// the same operands, reduced over the four lane groups at the end.
// No LDS barrier sits in the row loop; latency is hidden by occupancy.
// This pass is bound by HBM bandwidth: 4 D bytes read and 4 (m+1) bytes
// written per row; the matrix cores need about 40 % of their peak at the
// HBM rate for 17 directions at D = 256.

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

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kBlockRows = 16;     // rows per wave step (the MFMA's N)
constexpr int kJobRows = 512;      // rows per batched job
constexpr int kMaxGroup = 33;      // directions per launch: 2 MFMA blocks + 1 on the ALUs
constexpr int kBufferFlags = 0x00020000;   // buffer descriptor word 3 (32-bit data, CDNA)
constexpr int kRunBlocks = 4;      // 16-row blocks per run of the single-pair kernel
// staging row stride (floats): 68 puts the four lane groups of a result
// write (directions 4 apart) on disjoint LDS banks
constexpr int kStgStride = 68;

// directions [d0, d0 + nd) of row-major dirs (ndirs x D) -> LDS rows of
// stride DP + 4, zero beyond nd and beyond D
template <int DP, int NDL>
__device__ __forceinline__ void stage_dirs(float* us, const float* __restrict__ dirs, int d0, int nd,
                                           int D) {
  constexpr int S = DP + 4;
  for (int e = threadIdx.x; e < NDL * DP; e += kThreads) {
    const int d = e / DP, k = e - d * DP;
    us[d * S + k] = (d < nd && k < D) ? dirs[(size_t)(d0 + d) * D + k] : 0.f;
  }
}

// One wave: rows [r0, r0 + 16) of X (n rows) onto the nd staged directions;
// P points at the projection of the first staged direction (row stride n).
// The rows are read with buffer loads whose range is the block's live rows,
// so a dead lane (row >= n) reads zeros without a branch; a column k >= D of
// a live row reads the next row or zero and meets a zero direction entry
// (the staged directions are zero beyond D).  Inputs are taken to be finite.
// With stg, the results go to this wave's LDS staging rows instead (row d at
// stg + d * kStgStride, points at columns scol .. scol + 15) for a store of
// whole runs later.
template <int DP, int NB, bool TAIL, bool VEC>
__device__ __forceinline__ void proj_block(const float* __restrict__ X, int64_t n, int64_t r0, int D,
                                           const float* us, int nd, float* __restrict__ P,
                                           float* stg = nullptr, int scol = 0) {
  constexpr int S = DP + 4;
  constexpr int T = DP / 16;
  const int lane = threadIdx.x & 63;
  const int p = lane & 15, g = lane >> 4;
  const int live_rows = (int)min<int64_t>(kBlockRows, n - r0);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(X + r0 * D), 0, live_rows * D * 4, kBufferFlags);
  const int voff = (p * D + 4 * g) * 4;
  float4 x[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (VEC) {
      x[t] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 64 * t, 0, 0));
    } else {
      x[t] = make_float4(
          __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff + 64 * t + 0, 0, 0)),
          __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff + 64 * t + 4, 0, 0)),
          __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff + 64 * t + 8, 0, 0)),
          __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff + 64 * t + 12, 0, 0)));
    }
  }
  const int64_t row = r0 + p;
  const bool live = p < live_rows;
  floatx4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
  float tl = 0.f;
  // direction operands of step t, read one step ahead; the scheduling
  // barrier keeps the compiler from hoisting every LDS read of the block
  // (that would double the registers and halve the occupancy)
  const float* ua = us + p * S + 4 * g;
  const float* ut = us + 16 * NB * S + 4 * g;
  float4 a[NB], at;
#pragma unroll
  for (int b = 0; b < NB; ++b) a[b] = *reinterpret_cast<const float4*>(ua + 16 * b * S);
  if (TAIL) at = *reinterpret_cast<const float4*>(ut);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    float4 an[NB], atn;
    if (t + 1 < T) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        an[b] = *reinterpret_cast<const float4*>(ua + 16 * b * S + 16 * (t + 1));
      if (TAIL) atn = *reinterpret_cast<const float4*>(ut + 16 * (t + 1));
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].x, x[t].x, acc[b], 0, 0, 0);
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].y, x[t].y, acc[b], 0, 0, 0);
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].z, x[t].z, acc[b], 0, 0, 0);
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].w, x[t].w, acc[b], 0, 0, 0);
    }
    if (TAIL) {
      tl = fmaf(at.x, x[t].x, tl);
      tl = fmaf(at.y, x[t].y, tl);
      tl = fmaf(at.z, x[t].z, tl);
      tl = fmaf(at.w, x[t].w, tl);
      asm volatile("" : "+v"(tl));   // keep the chain in step with the MFMAs
    }
    if (t + 1 < T) {
#pragma unroll
      for (int b = 0; b < NB; ++b) a[b] = an[b];
      if (TAIL) at = atn;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // result block b: lane (p, g) holds directions 16 b + 4 g + v of point p
  if (stg) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) stg[(16 * b + 4 * g + v) * kStgStride + scol + p] = acc[b][v];
    if (TAIL) {
      tl += __shfl_xor(tl, 16);
      tl += __shfl_xor(tl, 32);
      if (g == 0) stg[(16 * NB) * kStgStride + scol + p] = tl;
    }
    return;
  }
  float* q = P + (live ? row : 0);
  if (live) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int d = 16 * b + 4 * g + v;
        if (d < nd) q[(int64_t)d * n] = acc[b][v];
      }
  }
  if (TAIL) {
    tl += __shfl_xor(tl, 16);
    tl += __shfl_xor(tl, 32);
    if (live && g == 0 && 16 * NB < nd) q[(int64_t)(16 * NB) * n] = tl;
  }
}

// Single pair (rows read as float4s): every wave walks runs of kRunBlocks
// 16-row blocks (64 rows) of A, then B (runs w, w + W, ... over the W waves
// of the grid);
// directions [d0, d0 + nd).  A run's results are staged in LDS and each
// direction's 64 values leave in one 256-byte store: stored block by block,
// every direction took a 64-byte piece per block, half a cache line, and the
// projection pass lost about a seventh of its time to the writes.
template <int DP, int NB, bool TAIL, bool VEC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void project_mfma(const float* __restrict__ A, int64_t nA,
                                                         const float* __restrict__ B, int64_t nB,
                                                         int D, const float* __restrict__ dirs,
                                                         int d0, int nd, float* __restrict__ PA,
                                                         float* __restrict__ PB) {
  constexpr int NDL = 16 * NB + (TAIL ? 1 : 0);
  constexpr int RR = kRunBlocks * kBlockRows;   // rows per run
  __shared__ __attribute__((aligned(16))) float us[NDL * (DP + 4)];
  stage_dirs<DP, NDL>(us, dirs, d0, nd, D);
  __syncthreads();
  const int64_t W = (int64_t)gridDim.x * kWaves;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if constexpr (!VEC) {
    // rows read a float at a time (unaligned or D % 4 != 0): blocks of 16
    // rows stored directly (the staging registers would not fit beside the
    // scalar loads)
    const int64_t bA = (nA + kBlockRows - 1) / kBlockRows;
    const int64_t nblk = bA + (nB + kBlockRows - 1) / kBlockRows;
    for (int64_t b = (int64_t)blockIdx.x * kWaves + wave; b < nblk; b += W) {
      const bool inA = b < bA;
      const int64_t n = inA ? nA : nB;
      float* P = inA ? PA + (size_t)d0 * nA : PB + (size_t)d0 * nB;
      proj_block<DP, NB, TAIL, VEC>(inA ? A : B, n, (inA ? b : b - bA) * kBlockRows, D, us, nd, P);
    }
    return;
  }
  __shared__ float stg_all[kWaves][NDL * kStgStride];
  const int64_t rA = (nA + RR - 1) / RR;
  const int64_t nrun = rA + (nB + RR - 1) / RR;
  const int lane = threadIdx.x & 63;
  float* stg = stg_all[wave];
  for (int64_t r = (int64_t)blockIdx.x * kWaves + wave; r < nrun; r += W) {
    const bool inA = r < rA;
    const int64_t n = inA ? nA : nB;
    const int64_t r0 = (inA ? r : r - rA) * RR;
    float* P = inA ? PA + (size_t)d0 * nA : PB + (size_t)d0 * nB;
    const float* X = inA ? A : B;
#pragma unroll
    for (int e = 0; e < kRunBlocks; ++e)
      if (r0 + e * kBlockRows < n)   // uniform
        proj_block<DP, NB, TAIL, VEC>(X, n, r0 + e * kBlockRows, D, us, nd, P, stg, e * kBlockRows);
    // the staging rows were written by this wave only: its own LDS writes
    // complete before the reads below (no barrier)
    const bool live = r0 + lane < n;
#pragma unroll 4
    for (int d = 0; d < nd && d < NDL; ++d) {
      const float v = stg[d * kStgStride + lane];
      if (live) P[(int64_t)d * n + r0 + lane] = v;
    }
  }
}

// Batched: one item = one 512-row tile of one set of one pair; the pair's
// directions (all of them, at most 33) are staged per item.
template <int DP, int NB, bool TAIL, bool VEC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void project_batch(const ProjJob* __restrict__ jobs, int njobs,
                                                          int D) {
  constexpr int NDL = 16 * NB + (TAIL ? 1 : 0);
  __shared__ __attribute__((aligned(16))) float us[NDL * (DP + 4)];
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const ProjJob j = jobs[it];
    __syncthreads();   // the previous item's reads of us are done
    stage_dirs<DP, NDL>(us, j.dirs, 0, j.ndirs, D);
    __syncthreads();
    for (int b = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); b < kJobRows / kBlockRows;
         b += kWaves) {
      const int64_t r0 = j.r0 + (int64_t)b * kBlockRows;
      if (r0 >= j.n) break;
      proj_block<DP, NB, TAIL, VEC>(j.X, j.n, r0, D, us, j.ndirs, j.P);
    }
  }
}

// (NB, TAIL) for a group of nd <= 33 directions
inline void group_shape(int nd, int& nb, bool& tail) {
  nb = nd <= 17 ? 1 : 2;
  tail = nd == 17 || nd == 33;
}

// persistent grid: resident work-groups per CU (from the kernel's own
// register and LDS use) times the CU count, capped by the work
template <typename K>
int resident_grid(K kernel, int64_t work_groups) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 2;
  return (int)std::max<int64_t>(1, std::min<int64_t>(work_groups, (int64_t)per_cu * cu_count()));
}

struct ProjLayout {
  int32_t* status;
  double* C;
  double* u0;
  void* sub;
  size_t sub_bytes;
};

ProjLayout proj_layout(Arena& ar, int64_t nA, int64_t nB, int D, int ndirs) {
  ProjLayout L;
  const int DP = pad_dim(D);
  L.status = ar.take<int32_t>(64);
  L.C = ar.take<double>((size_t)DP * DP);
  L.u0 = ar.take<double>(DP);
  L.sub_bytes = std::max(stats_ws_bytes(nA, nB, D), eig_ws_bytes(D, ndirs - 1));
  L.sub = ar.take<char>(L.sub_bytes);
  return L;
}

template <int DP, int NB, bool TAIL>
prohd_status launch_group(const float* A, int64_t nA, const float* B, int64_t nB, int D,
                          const float* dirs, int d0, int nd, float* PA, float* PB, hipStream_t s) {
  const bool vec = (D % 4 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0);
  // work-groups with work: runs of kRunBlocks blocks (staged form), blocks otherwise
  const int64_t rows_per = vec ? kRunBlocks * kBlockRows : kBlockRows;
  const int64_t wgs = cdiv(cdiv(nA, rows_per) + cdiv(nB, rows_per), kWaves);
  if (vec) {
    // eight times the resident work-groups: measured at 2M + 2M rows,
    // D = 256, 17 directions, 0.87 ms at one resident round, 0.85 ms at
    // eight (later work-groups start as earlier ones drain)
    static const int per = resident_grid(project_mfma<DP, NB, TAIL, true>, 1 << 30);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(wgs, (int64_t)per * 8));
    PROHD_LAUNCH("project_mfma", (project_mfma<DP, NB, TAIL, true>), dim3(grid), dim3(kThreads), 0, s,
                 A, nA, B, nB, D, dirs, d0, nd, PA, PB);
  } else {
    static const int per = resident_grid(project_mfma<DP, NB, TAIL, false>, 1 << 30);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(wgs, per));
    PROHD_LAUNCH("project_mfma", (project_mfma<DP, NB, TAIL, false>), dim3(grid), dim3(kThreads), 0, s,
                 A, nA, B, nB, D, dirs, d0, nd, PA, PB);
  }
  return PROHD_OK;
}

// Directions in groups of at most 33 per launch.
template <int DP>
prohd_status launch_project(const float* A, int64_t nA, const float* B, int64_t nB, int D,
                            const float* dirs, int ndirs, float* PA, float* PB, hipStream_t s) {
  for (int d0 = 0; d0 < ndirs; d0 += kMaxGroup) {
    const int nd = std::min(kMaxGroup, ndirs - d0);
    int nb;
    bool tail;
    group_shape(nd, nb, tail);
    prohd_status r;
    if (nb == 1)
      r = tail ? launch_group<DP, 1, true>(A, nA, B, nB, D, dirs, d0, nd, PA, PB, s)
               : launch_group<DP, 1, false>(A, nA, B, nB, D, dirs, d0, nd, PA, PB, s);
    else
      r = tail ? launch_group<DP, 2, true>(A, nA, B, nB, D, dirs, d0, nd, PA, PB, s)
               : launch_group<DP, 2, false>(A, nA, B, nB, D, dirs, d0, nd, PA, PB, s);
    if (r) return r;
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
  switch (pad_dim(D)) {
    case 16: return launch_project<16>(A, nA, B, nB, D, dirs, ndirs, projA, projB, s);
    case 32: return launch_project<32>(A, nA, B, nB, D, dirs, ndirs, projA, projB, s);
    case 64: return launch_project<64>(A, nA, B, nB, D, dirs, ndirs, projA, projB, s);
    case 128: return launch_project<128>(A, nA, B, nB, D, dirs, ndirs, projA, projB, s);
    case 256: return launch_project<256>(A, nA, B, nB, D, dirs, ndirs, projA, projB, s);
    default: return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM");
  }
}

template <int DP, int NB, bool TAIL>
prohd_status batch_project_g(int D, bool vec, const ProjJob* jobs, int njobs, int grid, hipStream_t s) {
  if (vec) {
    PROHD_LAUNCH("batch_project", (project_batch<DP, NB, TAIL, true>), dim3(grid), dim3(kThreads), 0, s,
                 jobs, njobs, D);
  } else {
    PROHD_LAUNCH("batch_project", (project_batch<DP, NB, TAIL, false>), dim3(grid), dim3(kThreads), 0,
                 s, jobs, njobs, D);
  }
  return PROHD_OK;
}

template <int DP>
prohd_status batch_project_dp(int D, int ndirs, bool vec, const ProjJob* jobs, int njobs, int grid,
                              hipStream_t s) {
  if (ndirs < 1 || ndirs > kMaxGroup)
    return fail(PROHD_EUNSUPPORTED, "batched projection: more than 33 directions");
  int nb;
  bool tail;
  group_shape(ndirs, nb, tail);
  if (nb == 1)
    return tail ? batch_project_g<DP, 1, true>(D, vec, jobs, njobs, grid, s)
                : batch_project_g<DP, 1, false>(D, vec, jobs, njobs, grid, s);
  return tail ? batch_project_g<DP, 2, true>(D, vec, jobs, njobs, grid, s)
              : batch_project_g<DP, 2, false>(D, vec, jobs, njobs, grid, s);
}

prohd_status batch_project(int DP, int D, int ndirs, bool vec, const ProjJob* jobs, int njobs, int grid,
                           hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  vec = vec && D % 4 == 0;
  switch (DP) {
    case 16: return batch_project_dp<16>(D, ndirs, vec, jobs, njobs, grid, s);
    case 32: return batch_project_dp<32>(D, ndirs, vec, jobs, njobs, grid, s);
    case 64: return batch_project_dp<64>(D, ndirs, vec, jobs, njobs, grid, s);
    case 128: return batch_project_dp<128>(D, ndirs, vec, jobs, njobs, grid, s);
    case 256: return batch_project_dp<256>(D, ndirs, vec, jobs, njobs, grid, s);
    default: return fail(PROHD_EUNSUPPORTED, "batched: unsupported padded dimension");
  }
}

}  // namespace prohd
