// Hausdorff distance kernels: the candidate distance of ProHD and the exact
// brute-force distance, on gfx950 matrix cores.
//
// Definitions: Eq. (1) of the paper, h(X,Y) = max_x min_y ||x - y||, and the
// candidate form H-hat (Sec. II-A, Alg. 3), which is the same distance over
// the selected rows.
//
// Pipeline for one pair of row sets (X, Y):
//   prep     rows are shifted by a common point s (translation leaves every
//            distance unchanged and shrinks |x|^2, which bounds the rounding of
//            the expansion below), padded with zeros to DP in {16..256}
//            columns, and their squared norms taken; non-finite input raises
//            the status word.  For the candidate distance, prep gathers the
//            selected rows.
//   tile     one work-group holds 256 rows of X as matrix-core A operands in
//            registers (32 rows per wave, the k range split between the two
//            half-waves) and streams Y through LDS 32 rows at a time.  Each
//            32x32 block of dot products comes from DP/2 v_mfma_f32_32x32x2f32
//            issues; the epilogue forms d2 = |x|^2 + |y|^2 - 2 x.y, keeps a
//            running row minimum in registers across all Y blocks and reduces
//            the block's column minima through LDS into a global atomicMin.
//            Y may be split across work-groups so that small X still fills
//            every compute unit; row minima then meet in a global atomicMin.
//            Minima are kept as float bit patterns of non-negative values,
//            whose unsigned order is the float order.
//   refine   the R rows with the largest approximate minimum (R = 256, or all
//            rows if fewer) are re-measured against every row of Y by float32
//            direct differences sum (x_k - y_k)^2, keeping the arg-min (smallest
//            index on ties).
//   finalize the largest refined minimum per direction gives the witness pair,
//            whose distance is recomputed in float64 from the original rows.

#include "common.h"

namespace prohd {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kRefineRows = 256;   // rows re-measured per direction
constexpr uint32_t kInfBits = 0x7f800000u;

__device__ __forceinline__ uint32_t clamp_bits(float d) {
  // d2 from the expansion may round below zero; the minimum of clamped values
  // equals the clamped minimum.  (d > 0) also maps -0.0 and NaN to +0.0.
  return __float_as_uint(d > 0.f ? d : 0.f);
}

// Device count clipped to the host bound (capacity), or the host count.
__device__ __forceinline__ int64_t dev_or(const int64_t* p, int64_t v) {
  if (!p) return v;
  const int64_t d = *p;
  return d < v ? (d > 0 ? d : 0) : v;
}

// ------------------------------------------------------------------ prep
// Xp[i] = pad(X[src(i)] - s), xn[i] = |Xp[i]|^2, for i < n (device count or
// host count).  src(i) = idx ? idx[i] : i.  s = X0[shift_idx ? *shift_idx : 0]
// taken from the FIRST set so both sets share it.  One wave per row.
template <int DP>
__global__ __launch_bounds__(256) void prep_rows(const float* __restrict__ X, int D,
                                                 const int32_t* __restrict__ idx,
                                                 const int64_t* __restrict__ dn, int64_t hn,
                                                 const float* __restrict__ S,
                                                 const int32_t* __restrict__ sidx,
                                                 const int64_t* __restrict__ sdn,
                                                 float* __restrict__ Xp, float* __restrict__ xn,
                                                 int32_t* __restrict__ status) {
  const int64_t n = dev_or(dn, hn);
  if (n <= 0) return;
  const int lane = threadIdx.x & 63;
  // shift row: first selected row of the first set (row 0 if none selected)
  const int64_t s_row = (sidx && (!sdn || *sdn > 0)) ? (int64_t)sidx[0] : 0;
  const float* srow = S + s_row * D;
  constexpr int PER = (DP + 63) / 64;
  float sv[PER];
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int k = lane + 64 * c;
    sv[c] = (k < D) ? srow[k] : 0.f;
  }
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
    const int64_t src = idx ? (int64_t)idx[i] : i;
    const float* xr = X + src * D;
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int k = lane + 64 * c;
      if (k < DP) {
        float v = 0.f;
        if (k < D) {
          const float x = xr[k];
          bad |= !(x - x == 0.f);  // NaN or Inf
          v = x - sv[c];
        }
        Xp[i * DP + k] = v;
        acc = fmaf(v, v, acc);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) xn[i] = acc;
  }
  if (bad) atomicOr(status, ST_NONFINITE);
}

__global__ void fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ------------------------------------------------------------------ tile
constexpr int kTileRows = 256;  // rows of X per work-group (8 waves x 32)
constexpr int kBN = 32;         // rows of Y per LDS block

template <int DP, bool COLMIN>
__global__ __launch_bounds__(512) void dist_tile(const float* __restrict__ Xp,
                                                 const float* __restrict__ xn,
                                                 const int64_t* __restrict__ dnX, int64_t hnX,
                                                 const float* __restrict__ Yp,
                                                 const float* __restrict__ yn,
                                                 const int64_t* __restrict__ dnY, int64_t hnY,
                                                 int ysplit, uint32_t* __restrict__ rowmin,
                                                 uint32_t* __restrict__ colmin) {
  constexpr int KH = DP / 2;       // k values per half-wave
  constexpr int ST = DP + 4;       // LDS row stride (floats): conflict-free b128 reads
  constexpr int NV4 = kBN * DP / 4;             // float4s per Y block
  constexpr int PF = (NV4 + 511) / 512;         // float4s per thread per block
  __shared__ __attribute__((aligned(16))) float ys[2][kBN * ST];
  __shared__ float yns[2][kBN];
  __shared__ uint32_t cmin[2][kBN];

  const int64_t nX = dev_or(dnX, hnX);
  const int64_t nY = dev_or(dnY, hnY);
  const int xblk = blockIdx.x / ysplit;
  const int ysi = blockIdx.x - xblk * ysplit;
  const int64_t x0 = (int64_t)xblk * kTileRows;
  if (x0 >= nX) return;
  const int64_t chunk = ((nY + ysplit - 1) / ysplit + kBN - 1) / kBN * kBN;
  const int64_t yb = (int64_t)ysi * chunk;
  const int64_t ye = min(nY, yb + chunk);
  if (yb >= ye) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 5;   // half-wave: k range [g*KH, g*KH + KH)
  const int c = lane & 31;   // row (A operand) / column (B operand) within the 32-block

  // A operand: row x0 + 32*wave + c, k in [g*KH, g*KH + KH)
  float a[KH];
  {
    const int64_t xr = x0 + 32 * wave + c;
    if (xr < nX) {
      const float4* src = reinterpret_cast<const float4*>(Xp + xr * DP + g * KH);
#pragma unroll
      for (int j = 0; j < KH / 4; ++j) {
        const float4 v = src[j];
        a[4 * j] = v.x; a[4 * j + 1] = v.y; a[4 * j + 2] = v.z; a[4 * j + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < KH; ++j) a[j] = 0.f;
    }
  }
  // |x|^2 of the 16 accumulator rows this lane holds: row 8*(v/4) + 4*g + v%4
  float xq[16];
  float rmin[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t r = x0 + 32 * wave + 8 * (v >> 2) + 4 * g + (v & 3);
    xq[v] = (r < nX) ? xn[r] : __uint_as_float(kInfBits);
    rmin[v] = __uint_as_float(kInfBits);
  }

  auto load_block = [&](int64_t y0, float4 (&buf)[PF], float& ynv) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int f = tid + 512 * p;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (f < NV4) {
        const int r = f / (DP / 4);
        const int k4 = f - r * (DP / 4);
        if (y0 + r < ye) v = reinterpret_cast<const float4*>(Yp + (y0 + r) * DP)[k4];
      }
      buf[p] = v;
    }
    ynv = (tid < kBN && y0 + tid < ye) ? yn[y0 + tid] : __uint_as_float(kInfBits);
  };
  auto store_block = [&](int b, const float4 (&buf)[PF], float ynv) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int f = tid + 512 * p;
      if (f < NV4) {
        const int r = f / (DP / 4);
        const int k4 = f - r * (DP / 4);
        *reinterpret_cast<float4*>(&ys[b][r * ST + 4 * k4]) = buf[p];
      }
    }
    if (tid < kBN) {
      yns[b][tid] = ynv;
      cmin[b][tid] = kInfBits;
    }
  };

  float4 pf[PF];
  float pyn;
  load_block(yb, pf, pyn);
  store_block(0, pf, pyn);
  __syncthreads();

  int cur = 0;
  for (int64_t y0 = yb; y0 < ye; y0 += kBN) {
    const bool more = y0 + kBN < ye;
    if (more) load_block(y0 + kBN, pf, pyn);

    // one accumulator: dependent 32x32x2 issues with the same destination
    // accumulate back to back in the matrix pipe
    floatx16 acc = {0.f};
    const float* yrow = &ys[cur][c * ST + g * KH];
#pragma unroll
    for (int s = 0; s < KH; s += 4) {
      const float4 b = *reinterpret_cast<const float4*>(yrow + s);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 0], b.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 1], b.y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 2], b.z, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 3], b.w, acc, 0, 0, 0);
    }
    // epilogue: lane holds column c of the block, rows 8*(v/4) + 4*g + v%4
    const float ynv = yns[cur][c];
    float cm = __uint_as_float(kInfBits);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float d = fmaf(-2.f, acc[v], xq[v] + ynv);
      rmin[v] = fminf(rmin[v], d);
      cm = fminf(cm, d);
    }
    if (COLMIN) {
      cm = fminf(cm, __shfl_xor(cm, 32));
      if (g == 0) atomicMin(&cmin[cur][c], clamp_bits(cm));
    }
    if (more) store_block(cur ^ 1, pf, pyn);
    __syncthreads();
    if (COLMIN && wave == 0 && lane < kBN) {
      const uint32_t v = cmin[cur][lane];
      if (y0 + lane < ye) atomicMin(&colmin[y0 + lane], v);
    }
    cur ^= 1;
  }

  // row minima: reduce over the 32 lanes of each half-wave (same rows)
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    float x = rmin[v];
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) x = fminf(x, __shfl_xor(x, off));
    rmin[v] = x;
  }
  float mine = __uint_as_float(kInfBits);
#pragma unroll
  for (int v = 0; v < 16; ++v) mine = (c == v) ? rmin[v] : mine;
  if (c < 16) {
    const int64_t r = x0 + 32 * wave + 8 * (c >> 2) + 4 * g + (c & 3);
    if (r < nX) atomicMin(&rowmin[r], clamp_bits(mine));
  }
}

// ---------------------------------------------------------------- refine
// best[r] = min over y of (bits(sum_k (x_k - y_k)^2) << 32 | y) for the
// candidate rows cand[r], r < R.
template <int DP>
__global__ __launch_bounds__(256) void refine_rows(const float* __restrict__ Xp,
                                                   const int32_t* __restrict__ cand,
                                                   const int64_t* __restrict__ dR,
                                                   const float* __restrict__ Yp,
                                                   const int64_t* __restrict__ dnY, int64_t hnY,
                                                   int ysplit,
                                                   unsigned long long* __restrict__ best) {
  constexpr int RB = 8;     // candidate rows per work-group
  constexpr int BN = 64;    // Y rows per LDS block
  constexpr int ST = DP + 4;
  __shared__ __attribute__((aligned(16))) float xs[RB * DP];
  __shared__ __attribute__((aligned(16))) float ysm[BN * ST];
  const int64_t R = *dR;
  const int64_t nY = dev_or(dnY, hnY);
  const int cb = blockIdx.x / ysplit;
  const int ysi = blockIdx.x - cb * ysplit;
  if ((int64_t)cb * RB >= R) return;
  const int64_t chunk = ((nY + ysplit - 1) / ysplit + BN - 1) / BN * BN;
  const int64_t yb = (int64_t)ysi * chunk;
  const int64_t ye = min(nY, yb + chunk);
  if (yb >= ye) return;
  const int tid = threadIdx.x;
  for (int f = tid; f < RB * DP; f += 256) {
    const int r = f / DP, k = f - r * DP;
    const int64_t cr = (int64_t)cb * RB + r;
    xs[f] = (cr < R) ? Xp[(int64_t)cand[cr] * DP + k] : 0.f;
  }
  const int q = tid >> 6;   // candidate pair 2q, 2q+1 (one per wave: broadcast reads)
  const int j = tid & 63;   // Y row within the block
  float b0 = __uint_as_float(kInfBits), b1 = b0;
  int64_t i0 = 0, i1 = 0;
  for (int64_t y0 = yb; y0 < ye; y0 += BN) {
    __syncthreads();
    for (int f = tid; f < BN * DP / 4; f += 256) {
      const int r = f / (DP / 4), k4 = f - r * (DP / 4);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (y0 + r < ye) v = reinterpret_cast<const float4*>(Yp + (y0 + r) * DP)[k4];
      *reinterpret_cast<float4*>(&ysm[r * ST + 4 * k4]) = v;
    }
    __syncthreads();
    if (y0 + j < ye) {
      float s0[4] = {0.f, 0.f, 0.f, 0.f}, s1[4] = {0.f, 0.f, 0.f, 0.f};
      const float* yr = &ysm[j * ST];
      const float* x0r = &xs[(2 * q) * DP];
      const float* x1r = &xs[(2 * q + 1) * DP];
#pragma unroll 8
      for (int k = 0; k < DP; k += 4) {
        const float4 y = *reinterpret_cast<const float4*>(yr + k);
        const float4 u = *reinterpret_cast<const float4*>(x0r + k);
        const float4 w = *reinterpret_cast<const float4*>(x1r + k);
        float t;
        t = u.x - y.x; s0[0] = fmaf(t, t, s0[0]);
        t = u.y - y.y; s0[1] = fmaf(t, t, s0[1]);
        t = u.z - y.z; s0[2] = fmaf(t, t, s0[2]);
        t = u.w - y.w; s0[3] = fmaf(t, t, s0[3]);
        t = w.x - y.x; s1[0] = fmaf(t, t, s1[0]);
        t = w.y - y.y; s1[1] = fmaf(t, t, s1[1]);
        t = w.z - y.z; s1[2] = fmaf(t, t, s1[2]);
        t = w.w - y.w; s1[3] = fmaf(t, t, s1[3]);
      }
      const float d0 = (s0[0] + s0[1]) + (s0[2] + s0[3]);
      const float d1 = (s1[0] + s1[1]) + (s1[2] + s1[3]);
      if (d0 < b0) { b0 = d0; i0 = y0 + j; }
      if (d1 < b1) { b1 = d1; i1 = y0 + j; }
    }
  }
  unsigned long long p0 = ((unsigned long long)__float_as_uint(b0) << 32) | (unsigned long long)(uint32_t)i0;
  unsigned long long p1 = ((unsigned long long)__float_as_uint(b1) << 32) | (unsigned long long)(uint32_t)i1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o0 = __shfl_xor(p0, off);
    const unsigned long long o1 = __shfl_xor(p1, off);
    p0 = o0 < p0 ? o0 : p0;
    p1 = o1 < p1 ? o1 : p1;
  }
  if (j == 0) {
    const int64_t r0 = (int64_t)cb * RB + 2 * q;
    if (r0 < R) atomicMin(&best[r0], p0);
    if (r0 + 1 < R) atomicMin(&best[r0 + 1], p1);
  }
}

// -------------------------------------------------------------- finalize
struct DirIn {
  const unsigned long long* best;  // refined minima
  const int32_t* cand;             // candidate rows (indices into the X list)
  const int64_t* dR;               // number of candidates
  const int32_t* mapX;             // X list -> original rows (or null)
  const int32_t* mapY;             // Y list -> original rows (or null)
  const float* Xo;                 // original X rows
  const float* Yo;                 // original Y rows
};

__device__ double pair_dist64(const float* __restrict__ X, int64_t i, const float* __restrict__ Y,
                              int64_t j, int D, double* red) {
  double s = 0.0;
  for (int k = threadIdx.x; k < D; k += blockDim.x) {
    const double t = (double)X[i * D + k] - (double)Y[j * D + k];
    s = fma(t, t, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sqrt(red[0]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void finalize(DirIn ab, DirIn ba, int D,
                                                const int64_t* __restrict__ dnA, int64_t hnA,
                                                const int64_t* __restrict__ dnB, int64_t hnB,
                                                const int32_t* __restrict__ status,
                                                prohd_result* __restrict__ out) {
  __shared__ double red[256];
  __shared__ unsigned long long bestp[256];
  int64_t wx[2], wy[2];
  double h[2];
  const int64_t nA = dev_or(dnA, hnA), nB = dev_or(dnB, hnB);
  int32_t st = *status;
  if (nA < 1 || nB < 1) st = st ? st : ST_EMPTY;
  for (int dir = 0; dir < 2; ++dir) {
    const DirIn& d = dir == 0 ? ab : ba;
    const int64_t R = (st == ST_OK) ? *d.dR : 0;
    // largest refined minimum; ties -> smallest candidate position
    unsigned long long m = 0ull;
    for (int64_t r = threadIdx.x; r < R; r += blockDim.x) {
      const unsigned long long v = ((d.best[r] >> 32) << 32) | (0xFFFFFFFFull - (unsigned long long)r);
      m = v > m ? v : m;
    }
    bestp[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) bestp[threadIdx.x] = max(bestp[threadIdx.x], bestp[threadIdx.x + w]);
      __syncthreads();
    }
    const unsigned long long top = bestp[0];
    __syncthreads();
    if (R > 0) {
      const int64_t r = (int64_t)(0xFFFFFFFFull - (top & 0xFFFFFFFFull));
      const int64_t xi = d.cand[r];
      const int64_t yi = (int64_t)(d.best[r] & 0xFFFFFFFFull);
      wx[dir] = d.mapX ? (int64_t)d.mapX[xi] : xi;
      wy[dir] = d.mapY ? (int64_t)d.mapY[yi] : yi;
      h[dir] = pair_dist64(d.Xo, wx[dir], d.Yo, wy[dir], D, red);
    } else {
      wx[dir] = wy[dir] = -1;
      h[dir] = 0.0;
    }
  }
  if (threadIdx.x == 0) {
    prohd_result r;
    r.hAB = h[0];
    r.hBA = h[1];
    r.H = h[0] > h[1] ? h[0] : h[1];
    r.ab_a = wx[0];
    r.ab_b = wy[0];
    r.ba_b = wx[1];
    r.ba_a = wy[1];
    r.nA_sel = nA;
    r.nB_sel = nB;
    r.status = st;
    r.refined = 0;
    *out = r;
  }
}

__global__ void store_refined(prohd_result* out, const int64_t* dR1, const int64_t* dR2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out->refined = (int32_t)max(*dR1, *dR2);
}

// ------------------------------------------------------------ host side
struct PrepSet {
  float* p;       // padded rows, cap x DP
  float* n;       // squared norms, cap
};

// ysplit so that (x blocks) x (ysplit) fills the compute units in whole waves
// of work-groups, with at least `min_blocks` Y blocks per work-group.
int choose_split(int64_t xblocks, int64_t ny, int64_t min_rows) {
  const int64_t cus = cu_count();
  const int64_t max_split = std::max<int64_t>(1, ny / std::max<int64_t>(1, min_rows));
  int best = 1;
  double best_eff = -1.0;
  for (int64_t s = 1; s <= std::min<int64_t>(max_split, 4096); ++s) {
    const int64_t tot = xblocks * s;
    const int64_t waves = cdiv(tot, cus);
    double eff = (double)tot / (double)(waves * cus);
    // prefer fewer splits unless the fill improves noticeably
    if (eff > best_eff + 0.02) {
      best_eff = eff;
      best = (int)s;
    }
    if (tot >= 8 * cus && eff > 0.97) break;
  }
  return best;
}

template <int DP>
prohd_status launch_prep(const float* X, int D, const int32_t* idx, const int64_t* dn, int64_t cap,
                         const float* S, const int32_t* sidx, const int64_t* sdn, PrepSet o,
                         int32_t* status, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(cap, 4), 8 * cu_count()));
  PROHD_LAUNCH("hd_prep", prep_rows<DP>, dim3(grid), dim3(256), 0, s, X, D, idx, dn, cap, S, sidx,
               sdn, o.p, o.n, status);
  return PROHD_OK;
}

template <int DP>
prohd_status launch_tile(PrepSet X, const int64_t* dnX, int64_t capX, PrepSet Y, const int64_t* dnY,
                         int64_t capY, uint32_t* rowmin, uint32_t* colmin, hipStream_t s) {
  const int64_t xblocks = cdiv(capX, kTileRows);
  const int split = choose_split(xblocks, capY, 4 * kBN);
  const int64_t grid = xblocks * split;
  if (grid > 0x7fffffff) return fail(PROHD_EUNSUPPORTED, "tile grid too large");
  if (colmin) {
    PROHD_LAUNCH("hd_tile", (dist_tile<DP, true>), dim3((unsigned)grid), dim3(512), 0, s, X.p, X.n,
                 dnX, capX, Y.p, Y.n, dnY, capY, split, rowmin, colmin);
  } else {
    PROHD_LAUNCH("hd_tile", (dist_tile<DP, false>), dim3((unsigned)grid), dim3(512), 0, s, X.p, X.n,
                 dnX, capX, Y.p, Y.n, dnY, capY, split, rowmin, colmin);
  }
  return PROHD_OK;
}

template <int DP>
prohd_status launch_refine(const float* Xp, const int32_t* cand, const int64_t* dR, const float* Yp,
                           const int64_t* dnY, int64_t capY, unsigned long long* best,
                           hipStream_t s) {
  const int64_t cblocks = cdiv(kRefineRows, 8);
  const int split = choose_split(cblocks, capY, 256);
  PROHD_LAUNCH("hd_refine", refine_rows<DP>, dim3((unsigned)(cblocks * split)), dim3(256), 0, s, Xp,
               cand, dR, Yp, dnY, capY, split, best);
  return PROHD_OK;
}

// One directed refinement: top-R of `mins` (n entries), then refine vs Y.
struct DirWork {
  uint8_t* flags;   // n bytes
  int32_t* cand;    // kRefineRows
  int64_t* count;   // 1
  unsigned long long* best;  // kRefineRows
};

struct HdLayout {
  PrepSet xa, xb;          // prepared candidate (or full) rows
  PrepSet fa, fb;          // full prepared rows (inner-full mode)
  uint32_t* rowA;          // minima of A-side rows
  uint32_t* rowB;          // minima of B-side rows
  DirWork w[2];
  int32_t* status;
  void* sel_ws;
  size_t sel_bytes;
};

HdLayout hd_layout(Arena& ar, int64_t capA, int64_t capB, int64_t nA, int64_t nB, int DP,
                   bool full) {
  HdLayout L{};
  L.status = ar.take<int32_t>(64);
  L.xa.p = ar.take<float>((size_t)capA * DP);
  L.xa.n = ar.take<float>(capA);
  L.xb.p = ar.take<float>((size_t)capB * DP);
  L.xb.n = ar.take<float>(capB);
  if (full) {
    L.fa.p = ar.take<float>((size_t)nA * DP);
    L.fa.n = ar.take<float>(nA);
    L.fb.p = ar.take<float>((size_t)nB * DP);
    L.fb.n = ar.take<float>(nB);
  }
  L.rowA = ar.take<uint32_t>(capA);
  L.rowB = ar.take<uint32_t>(capB);
  const int64_t caps[2] = {capA, capB};
  for (int d = 0; d < 2; ++d) {
    L.w[d].flags = ar.take<uint8_t>(caps[d]);
    L.w[d].cand = ar.take<int32_t>(kRefineRows);
    L.w[d].count = ar.take<int64_t>(1);
    L.w[d].best = ar.take<unsigned long long>(kRefineRows);
  }
  const int64_t mx = std::max(capA, capB);
  L.sel_bytes = std::max(select_ws_bytes(1, mx), compact_ws_bytes(mx));
  L.sel_ws = ar.take<char>(L.sel_bytes);
  return L;
}

// Top-R rows of `mins` (device length dn / host n) -> w.cand / w.count.
prohd_status top_rows(const uint32_t* mins, int64_t n, const int64_t* dn, DirWork& w, void* sel_ws,
                      size_t sel_bytes, hipStream_t s) {
  prohd_status st = zero_bytes(w.flags, (size_t)n, s);
  if (st) return st;
  SelSegment seg{reinterpret_cast<const float*>(mins), n, dn, 0, kRefineRows, w.flags};
  st = select_mark(&seg, 1, sel_ws, sel_bytes, s);
  if (st) return st;
  return compact_flags(w.flags, n, dn, w.cand, w.count, sel_ws, sel_bytes, s);
}

prohd_status init_mins(uint32_t* p, int64_t n, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 4096));
  PROHD_LAUNCH("hd_fill", fill_u32, dim3(grid), dim3(256), 0, s, p, n, kInfBits);
  return PROHD_OK;
}

prohd_status init_best(unsigned long long* p, hipStream_t s) {
  PROHD_LAUNCH("hd_fill", fill_u64, dim3(1), dim3(256), 0, s, p, (int64_t)kRefineRows, ~0ull);
  return PROHD_OK;
}

#define PROHD_TRY(x)                 \
  do {                               \
    prohd_status st_ = (x);          \
    if (st_ != PROHD_OK) return st_; \
  } while (0)

// Shared driver.  Mode: exact (idx null), candidates, or candidates with the
// inner minimum over the full other set.
template <int DP>
prohd_status run_hd(const float* A, int64_t nA, const float* B, int64_t nB, int D,
                    const int32_t* idxA, const int64_t* dnA, int64_t capA, const int32_t* idxB,
                    const int64_t* dnB, int64_t capB, bool full, prohd_result* out, float* nn2A,
                    float* nn2B, void* ws, size_t ws_bytes, hipStream_t s) {
  Arena ar(ws);
  HdLayout L = hd_layout(ar, capA, capB, nA, nB, DP, full);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "hd: workspace too small");
  PROHD_TRY(zero_bytes(L.status, sizeof(int32_t) * 64, s));
  // common shift: the first (selected) row of A
  const int32_t* sidx = idxA;
  PROHD_TRY(launch_prep<DP>(A, D, idxA, dnA, capA, A, sidx, dnA, L.xa, L.status, s));
  PROHD_TRY(launch_prep<DP>(B, D, idxB, dnB, capB, A, sidx, dnA, L.xb, L.status, s));
  PROHD_TRY(init_mins(L.rowA, capA, s));
  PROHD_TRY(init_mins(L.rowB, capB, s));
  for (int d = 0; d < 2; ++d) PROHD_TRY(init_best(L.w[d].best, s));
  DirIn ab{}, ba{};
  if (!full) {
    PROHD_TRY(launch_tile<DP>(L.xa, dnA, capA, L.xb, dnB, capB, L.rowA, L.rowB, s));
    PROHD_TRY(top_rows(L.rowA, capA, dnA, L.w[0], L.sel_ws, L.sel_bytes, s));
    PROHD_TRY(top_rows(L.rowB, capB, dnB, L.w[1], L.sel_ws, L.sel_bytes, s));
    PROHD_TRY(launch_refine<DP>(L.xa.p, L.w[0].cand, L.w[0].count, L.xb.p, dnB, capB, L.w[0].best, s));
    PROHD_TRY(launch_refine<DP>(L.xb.p, L.w[1].cand, L.w[1].count, L.xa.p, dnA, capA, L.w[1].best, s));
    ab = DirIn{L.w[0].best, L.w[0].cand, L.w[0].count, idxA, idxB, A, B};
    ba = DirIn{L.w[1].best, L.w[1].cand, L.w[1].count, idxB, idxA, B, A};
  } else {
    PROHD_TRY(launch_prep<DP>(A, D, nullptr, nullptr, nA, A, sidx, dnA, L.fa, L.status, s));
    PROHD_TRY(launch_prep<DP>(B, D, nullptr, nullptr, nB, A, sidx, dnA, L.fb, L.status, s));
    PROHD_TRY(launch_tile<DP>(L.xa, dnA, capA, L.fb, nullptr, nB, L.rowA, nullptr, s));
    PROHD_TRY(launch_tile<DP>(L.xb, dnB, capB, L.fa, nullptr, nA, L.rowB, nullptr, s));
    PROHD_TRY(top_rows(L.rowA, capA, dnA, L.w[0], L.sel_ws, L.sel_bytes, s));
    PROHD_TRY(top_rows(L.rowB, capB, dnB, L.w[1], L.sel_ws, L.sel_bytes, s));
    PROHD_TRY(launch_refine<DP>(L.xa.p, L.w[0].cand, L.w[0].count, L.fb.p, nullptr, nB, L.w[0].best, s));
    PROHD_TRY(launch_refine<DP>(L.xb.p, L.w[1].cand, L.w[1].count, L.fa.p, nullptr, nA, L.w[1].best, s));
    ab = DirIn{L.w[0].best, L.w[0].cand, L.w[0].count, idxA, nullptr, A, B};
    ba = DirIn{L.w[1].best, L.w[1].cand, L.w[1].count, idxB, nullptr, B, A};
  }
  PROHD_LAUNCH("hd_finalize", finalize, dim3(1), dim3(256), 0, s, ab, ba, D, dnA, capA, dnB, capB,
               L.status, out);
  PROHD_LAUNCH("hd_finalize", store_refined, dim3(1), dim3(64), 0, s, out, L.w[0].count, L.w[1].count);
  if (nn2A) PROHD_HIP(hipMemcpyAsync(nn2A, L.rowA, sizeof(float) * capA, hipMemcpyDeviceToDevice, s));
  if (nn2B) PROHD_HIP(hipMemcpyAsync(nn2B, L.rowB, sizeof(float) * capB, hipMemcpyDeviceToDevice, s));
  return PROHD_OK;
}

template <class F>
prohd_status by_dp(int D, F&& f) {
  switch (pad_dim(D)) {
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    default: return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM");
  }
}

}  // namespace

size_t hd_ws_bytes(int64_t nA, int64_t nB, int32_t D, int64_t capA, int64_t capB, bool full) {
  Arena ar(nullptr);
  hd_layout(ar, capA, capB, nA, nB, pad_dim(D), full);
  return ar.used + 256;
}

size_t exact_ws_bytes(int64_t nA, int64_t nB, int32_t D) {
  Arena ar(nullptr);
  hd_layout(ar, nA, nB, nA, nB, pad_dim(D), false);
  return ar.used + 256;
}

prohd_status hd_candidates(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                           const int32_t* idxA, const int64_t* dnA, int64_t capA,
                           const int32_t* idxB, const int64_t* dnB, int64_t capB, bool full,
                           prohd_result* out, void* ws, size_t ws_bytes, hipStream_t s) {
  return by_dp(D, [&](auto dp) {
    return run_hd<decltype(dp)::value>(A, nA, B, nB, D, idxA, dnA, capA, idxB, dnB, capB, full, out,
                                       nullptr, nullptr, ws, ws_bytes, s);
  });
}

prohd_status hd_exact(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      prohd_result* out, float* nn2A, float* nn2B, void* ws, size_t ws_bytes,
                      hipStream_t s) {
  return by_dp(D, [&](auto dp) {
    return run_hd<decltype(dp)::value>(A, nA, B, nB, D, nullptr, nullptr, nA, nullptr, nullptr, nB,
                                       false, out, nn2A, nn2B, ws, ws_bytes, s);
  });
}

}  // namespace prohd
