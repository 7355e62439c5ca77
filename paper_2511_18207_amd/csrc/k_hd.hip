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
//   bounds   from each row's approximate minimum, certified bounds L <= t <=
//            U of its true minimum t (the search's worst-case rounding and
//            quantisation error, see min_upper / min_lower); the directed
//            distance lies in [max L, max U].
//   refine   every row whose U reaches max L is re-measured against every
//            row of Y in float64 (matrix-core float64 expansion of the
//            exactly converted rows), keeping the arg-min (smallest index on
//            ties); on ordinary data these are a handful of rows.
//   finalize the largest refined minimum per direction gives the witness pair,
//            whose distance is recomputed in float64 from the original rows.
//   pruning  optionally (PROHD_PRUNE) the search runs in levels against
//            subsets of Y first (a subset minimum bounds the full minimum
//            from above), dropping rows whose U falls below max L.
// The batched form runs the same bound rule per pair (keys_batch,
// uncertain_batch, refine_dyn_batch) without pruning; its exact mode sends
// the pairs large enough for pruning through the single-pair path.

#include "batch.h"
#include "common.h"

namespace prohd {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kSeedRows = 64;      // rows that seed the lower bound (at most 64: top_keys)
constexpr int kShortList = 64;     // lists searched as the inner side of a tile
constexpr uint32_t kInfBits = 0x7f800000u;

__device__ __forceinline__ uint32_t clamp_bits(float d) {
  // d2 from the expansion may round below zero; the minimum of clamped values
  // equals the clamped minimum.  (d > 0) also maps -0.0 and NaN to +0.0.
  return __float_as_uint(d > 0.f ? d : 0.f);
}

// Running minimum as the median of (acc, d, ninf) with ninf = -inf held in
// a scalar register.  Equal to fminf for non-NaN operands; fminf on a value
// carried across blocks first gets a quieting max(acc, acc) from the
// compiler, the median needs none.  The empty asm hides the constant, which
// the compiler would otherwise fold the median back into a minimum with.
__device__ __forceinline__ float neg_inf_sreg() {
  float v = __uint_as_float(0xff800000u);
  asm volatile("" : "+s"(v));
  return v;
}
__device__ __forceinline__ float run_min(float acc, float d, float ninf) {
  return __builtin_amdgcn_fmed3f(acc, d, ninf);
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
__device__ __forceinline__ void prep_body(const float* __restrict__ X, int D,
                                          const int32_t* __restrict__ idx,
                                          const int64_t* __restrict__ dn, int64_t hn,
                                          const float* __restrict__ S,
                                          const int32_t* __restrict__ sidx,
                                          const int64_t* __restrict__ sdn,
                                          float* __restrict__ Xp, float* __restrict__ xn,
                                          int32_t* __restrict__ status,
                                          uint32_t* __restrict__ maxabs, int bx, int nbx) {
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
  float amax = 0.f;
  for (int64_t i = (int64_t)bx * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)nbx * 4) {
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
        amax = fmaxf(amax, fabsf(v));
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) xn[i] = acc;
  }
  if (bad) atomicOr(status, ST_NONFINITE);
  if (maxabs) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    if ((threadIdx.x & 63) == 0 && amax == amax) atomicMax(maxabs, __float_as_uint(amax));
  }
}

// Both sets in one launch (grid y = set; the shift row is shared).
struct PrepDir {
  const float* X;
  const int32_t* idx;
  const int64_t* dn;
  int64_t hn;
  float* Xp;
  float* xn;
};
struct PrepPair {
  PrepDir j[2];
  const float* S;
  const int32_t* sidx;
  const int64_t* sdn;
  int32_t* status;
  uint32_t* maxabs;
  int D;
};

template <int DP>
__global__ __launch_bounds__(256) void prep_rows(const PrepPair P) {
  const PrepDir J = P.j[blockIdx.y];
  prep_body<DP>(J.X, P.D, J.idx, J.dn, J.hn, P.S, P.sidx, P.sdn, J.Xp, J.xn, P.status, P.maxabs, blockIdx.x,
                gridDim.x);
}

__global__ void fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Several word fills in one launch (grid y = job): the clears and +inf
// initialisations of a search, which would otherwise take a launch each.
constexpr int kFillJobs = 8;
struct FillJob {
  uint32_t* p;
  int64_t n;
  uint32_t v;
};
struct FillPack {
  FillJob j[kFillJobs];
};
__global__ void fill_multi(const FillPack P) {
  const FillJob f = P.j[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.n; i += (int64_t)gridDim.x * blockDim.x)
    f.p[i] = f.v;
}

__global__ void fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ------------------------------------------------------------------ tile
// raw buffer descriptor word 3 for gfx950: offsets past num_records read zero
constexpr int kBufferFlags = 0x00020000;

constexpr int kTileRows = 256;  // rows of X per work-group (8 waves x 32)
constexpr int kBN = 32;         // columns (Y rows) of one 32 x 32 subtile

// Y rows per LDS buffer.  At D = 256 a buffer holds two subtiles, copied
// from memory straight into LDS (one 1 KiB row per wave instruction, no
// staging registers), so there is one barrier per 64 columns; narrower rows
// stage one subtile at a time through registers.
template <int DP>
__host__ __device__ constexpr int tile_bn() { return DP == 256 ? 2 * kBN : kBN; }

// One segment of the distance matrix: X rows [x0, x0 + kTileRows) against
// Y rows [yb, ye).  Row minima go to rowmin, column minima (COLMIN) to colmin,
// both as order-preserving bit patterns through atomicMin.  BNT: Y rows per
// LDS buffer (one 32-row subtile when Y has no more rows than that, so a
// tile against a short Y does not multiply padding).
template <int DP, bool COLMIN, bool GX = false, int BNT = tile_bn<DP>()>
__device__ __forceinline__ void dist_seg(const float* __restrict__ Xp, const float* __restrict__ xn,
                                         const int32_t* __restrict__ xidx,
                                         int64_t nX, const float* __restrict__ Yp,
                                         const float* __restrict__ yn, int64_t x0, int64_t yb,
                                         int64_t ye, uint32_t* __restrict__ rowmin,
                                         uint32_t* __restrict__ colmin) {
  constexpr int KH = DP / 2;       // k values per half-wave
  constexpr int ST = DP + 4;       // LDS row stride (floats): conflict-free b128 reads
  constexpr int BN = BNT;
  static_assert(BN % kBN == 0 && BN % 8 == 0, "whole subtiles");
  constexpr int NSUB = BN / kBN;   // subtiles per buffer
  constexpr bool DMA = DP == 256;  // rows of 1 KiB go straight into LDS
  constexpr int NV4 = BN * DP / 4;              // float4s per Y block
  constexpr int PF = DMA ? 1 : (NV4 + 511) / 512;   // float4s per thread per block
  // the two Y buffers are distinct objects, and the loop below names them
  // statically, so the compiler can tell that the copy into one does not
  // touch the reads of the other (no wait for the copy in flight before the
  // reads)
  __shared__ __attribute__((aligned(16))) float ys0[BN * ST];
  __shared__ __attribute__((aligned(16))) float ys1[BN * ST];
  __shared__ float yns0[BN], yns1[BN];
  __shared__ uint32_t cmin0[BN], cmin1[BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 5;   // half-wave: k range [g*KH, g*KH + KH)
  const int c = lane & 31;   // row (A operand) / column (B operand) within the 32-block

  // A operand: row x0 + 32*wave + c, k in [g*KH, g*KH + KH) (GX: the row
  // of that position in the list xidx)
  float a[KH];
  if constexpr (DMA) {
    // 1 KiB rows: each wave copies its 32 rows into its slice of the second
    // Y buffer (free until the first Y block is in, XR = BN / 8 rows) XR
    // rows at a time, one row per instruction (64 lanes x 16 contiguous
    // bytes; a row past nX has an empty range and reads zeros), then the
    // lanes of those rows read their half rows.  Loaded straight into
    // registers, each instruction touched 64 cache lines (every lane its
    // own row).
    constexpr int XR = BN / 8;
    float* xs = ys1 + wave * XR * ST;
#pragma unroll
    for (int p8 = 0; p8 < 32 / XR; ++p8) {
      if (x0 + 32 * wave + XR * p8 >= nX) {   // uniform: no live row in this pass
        if (c / XR == p8) {
#pragma unroll
          for (int j = 0; j < KH; ++j) a[j] = 0.f;
        }
        continue;
      }
#pragma unroll
      for (int r = 0; r < XR; ++r) {
        const int64_t xr = x0 + 32 * wave + XR * p8 + r;
        const int64_t xm = xr < nX ? (GX ? (int64_t)xidx[xr] : xr) : 0;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(Xp + xm * DP), 0, xr < nX ? DP * 4 : 0, kBufferFlags);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(xs + r * ST), 16, 4 * lane * 4, 0, 0, 0);
      }
      __builtin_amdgcn_s_waitcnt(0);   // this wave's row copies have landed
      if (c / XR == p8) {
        const float4* src = reinterpret_cast<const float4*>(xs + (c % XR) * ST + g * KH);
#pragma unroll
        for (int j = 0; j < KH / 4; ++j) {
          const float4 v = src[j];
          a[4 * j] = v.x; a[4 * j + 1] = v.y; a[4 * j + 2] = v.z; a[4 * j + 3] = v.w;
        }
      }
      // the slice is refilled by the next pass: this wave's reads come first
      __builtin_amdgcn_s_waitcnt(0);
    }
  } else {
    const int64_t xr = x0 + 32 * wave + c;
    if (xr < nX) {
      const int64_t xm = GX ? (int64_t)xidx[xr] : xr;
      const float4* src = reinterpret_cast<const float4*>(Xp + xm * DP + g * KH);
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
    xq[v] = (r < nX) ? xn[GX ? (int64_t)xidx[r] : r] : __uint_as_float(kInfBits);
    rmin[v] = __uint_as_float(kInfBits);
  }

  // Y block at y0 into buffer b: DMA rows past ye read as zero (buffer
  // range), register-staged rows past ye are zero-filled
  auto load_block = [&](int64_t y0, float* ysb, float4 (&buf)[PF], float& ynv) {
    if constexpr (DMA) {
      const int rows = (int)min<int64_t>(BN, ye - y0);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(Yp + y0 * DP), 0, rows * DP * 4, kBufferFlags);
#pragma unroll
      for (int r = wave; r < BN; r += 8)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(ysb + r * ST), 16,
            (r * DP + 4 * lane) * 4, 0, 0, 0);
    } else {
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
    }
    ynv = (tid < BN && y0 + tid < ye) ? yn[y0 + tid] : __uint_as_float(kInfBits);
  };
  auto store_block = [&](float* ysb, float* ynb, uint32_t* cmb, const float4 (&buf)[PF], float ynv) {
    if constexpr (!DMA) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int f = tid + 512 * p;
        if (f < NV4) {
          const int r = f / (DP / 4);
          const int k4 = f - r * (DP / 4);
          *reinterpret_cast<float4*>(ysb + r * ST + 4 * k4) = buf[p];
        }
      }
    }
    if (tid < BN) {
      ynb[tid] = ynv;
      cmb[tid] = kInfBits;
    }
  };

  float4 pf[PF];
  float pyn;
  load_block(yb, ys0, pf, pyn);
  store_block(ys0, yns0, cmin0, pf, pyn);
  if (DMA) __builtin_amdgcn_s_waitcnt(0);   // this wave's row copies have landed
  __syncthreads();

  // block at y0 in buffer cur (cy), the next one copied into nyb
  // (every LDS array is named statically at each call, for the same reason)
  auto block = [&](int64_t y0, float* cy, float* cyn, uint32_t* ccm, float* ny, float* nyn,
                   uint32_t* ncm) {
    const bool more = y0 + BN < ye;
    if (more) load_block(y0 + BN, ny, pf, pyn);
    float cms[NSUB];   // column minima of each subtile (lanes g == 0 hold them)
#pragma unroll
    for (int sub = 0; sub < NSUB; ++sub) {
      // one accumulator: dependent 32x32x2 issues with the same destination
      // accumulate back to back in the matrix pipe
      floatx16 acc = {0.f};
      const float* yrow = cy + (kBN * sub + c) * ST + g * KH;
      // raised issue priority while this wave's matrix ops go out, normal
      // again for the epilogue, so that the other wave on the SIMD gets the
      // issue slots for its vector work in between
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int s = 0; s < KH; s += 4) {
        const float4 b = *reinterpret_cast<const float4*>(yrow + s);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 0], b.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 1], b.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 2], b.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 3], b.w, acc, 0, 0, 0);
      }
      __builtin_amdgcn_s_setprio(0);
      // epilogue: lane holds column c of the subtile, rows 8*(v/4) + 4*g + v%4
      const float ynv = cyn[kBN * sub + c];
      float cm = __uint_as_float(kInfBits);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float d = fmaf(-2.f, acc[v], xq[v] + ynv);
        rmin[v] = fminf(rmin[v], d);
        cm = fminf(cm, d);
      }
      cms[sub] = COLMIN ? fminf(cm, __shfl_xor(cm, 32)) : cm;
    }
    // LDS writes after the wait for this wave's row copies: the compiler
    // would otherwise hold each of them until every copy in flight landed
    if (DMA) __builtin_amdgcn_s_waitcnt(0);
    if (COLMIN && g == 0) {
#pragma unroll
      for (int sub = 0; sub < NSUB; ++sub) atomicMin(&ccm[kBN * sub + c], clamp_bits(cms[sub]));
    }
    if (more) store_block(ny, nyn, ncm, pf, pyn);
    __syncthreads();
    // column minima of the block: wave 0 (which also resets cmin of the
    // other buffer, so this read precedes that write in program order)
    if (COLMIN && wave == 0 && lane < BN) {
      const uint32_t v = ccm[lane];
      if (y0 + lane < ye) atomicMin(&colmin[y0 + lane], v);
    }
  };
  for (int64_t y0 = yb; y0 < ye; y0 += 2 * BN) {
    block(y0, ys0, yns0, cmin0, ys1, yns1, cmin1);
    if (y0 + BN < ye) block(y0 + BN, ys1, yns1, cmin1, ys0, yns0, cmin0);
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
    if (r < nX && rowmin) atomicMin(&rowmin[r], clamp_bits(mine));
  }
}

// Work-group bx of a (row tile) x (ysplit Y chunks) grid.
template <int DP, bool COLMIN>
__device__ __forceinline__ void dist_tile_body(const float* __restrict__ Xp,
                                               const float* __restrict__ xn,
                                               const int64_t* __restrict__ dnX, int64_t hnX,
                                               const float* __restrict__ Yp,
                                               const float* __restrict__ yn,
                                               const int64_t* __restrict__ dnY, int64_t hnY,
                                               int ysplit, uint32_t* __restrict__ rowmin,
                                               uint32_t* __restrict__ colmin, int bx) {
  const int64_t nX = dev_or(dnX, hnX);
  const int64_t nY = dev_or(dnY, hnY);
  const int xblk = bx / ysplit;
  const int ysi = bx - xblk * ysplit;
  const int64_t x0 = (int64_t)xblk * kTileRows;
  if (x0 >= nX) return;
  constexpr int BN = tile_bn<DP>();
  const int64_t chunk = ((nY + ysplit - 1) / ysplit + BN - 1) / BN * BN;
  const int64_t yb = (int64_t)ysi * chunk;
  const int64_t ye = min(nY, yb + chunk);
  if (yb >= ye) return;
  dist_seg<DP, COLMIN>(Xp, xn, nullptr, nX, Yp, yn, x0, yb, ye, rowmin, colmin);
}

// Chunk count of a persistent tile launch.  The matrix is cut into xt x S
// (row tile, Y chunk) items that G work-groups take in whole rounds; the
// items left over after the last whole round are shared out in equal
// contiguous ranges of Y blocks (tile_schedule), which balances the work
// for any S but reads those blocks without the in-step L2 sharing.  So S is
// the smallest split (S <= min(16, nyb)) that leaves at most 5 % of a round
// over, else the one that leaves the fewest.  Decided on the device from the
// actual counts.
__device__ __forceinline__ int64_t tile_split(int64_t xt, int64_t nyb, int64_t G) {
  int64_t S = 1, best = G;
  for (int64_t s = 1; s <= 16 && s <= nyb; ++s) {
    const int64_t left = xt * s % G;
    if (left < best) {
      best = left;
      S = s;
    }
    if (left * 20 <= G) break;
  }
  return S;
}

// Work of this work-group in a persistent tile launch: whole rounds of
// chunk-major items (item i: chunk i / xt, row tile i % xt; work-group b
// takes items b, b + G, ...), then its share of the leftover items' Y blocks.
// seg(row tile, first block, end block) runs one segment; every thread of
// the work-group reaches the same calls.
// (bx, G: this work-group's place among the G that share the pair.)
template <class Seg>
__device__ __forceinline__ void tile_schedule(int64_t xt, int64_t nyb, int64_t S, int64_t bx, int64_t G,
                                              Seg&& seg) {
  const int64_t items = xt * S;
  const int64_t full = items / G * G;
  for (int64_t i = bx; i < full; i += G) {
    const int64_t ysi = i / xt, xblk = i - ysi * xt;
    seg(xblk, ysi * nyb / S, (ysi + 1) * nyb / S);
  }
  // leftover items as cmax block slots each (chunks differ by one block at
  // most; slots past a chunk's end are empty), cut into G equal ranges
  const int64_t left = items - full;
  if (left == 0) return;
  const int64_t cmax = (nyb + S - 1) / S;
  const int64_t cells = left * cmax;
  int64_t w = cells * bx / G;
  const int64_t hi = cells * (bx + 1) / G;
  while (w < hi) {
    const int64_t q = w / cmax;
    const int64_t end = min(hi, (q + 1) * cmax);
    const int64_t i = full + q;
    const int64_t ysi = i / xt, xblk = i - ysi * xt;
    const int64_t c0 = ysi * nyb / S, c1 = (ysi + 1) * nyb / S;
    const int64_t b0 = c0 + (w - q * cmax), b1 = min(c1, c0 + (end - q * cmax));
    if (b0 < b1) seg(xblk, b0, b1);
    w = end;
  }
}

// Persistent form for one pair (schedule: tile_schedule).  The items of one
// round start together at the beginning of their chunk and sweep it in step,
// so the work-groups of an XCD (ids congruent modulo 8), which hold
// consecutive items of one or two chunks, read each Y block at about the same
// time and one L2 fill serves them all.
template <int DP, bool COLMIN, bool GX = false, int BNT = tile_bn<DP>()>
__global__ __launch_bounds__(512) void dist_tile(const float* __restrict__ Xp,
                                                 const float* __restrict__ xn,
                                                 const int32_t* __restrict__ xidx,
                                                 const int64_t* __restrict__ dnX, int64_t hnX,
                                                 const float* __restrict__ Yp,
                                                 const float* __restrict__ yn,
                                                 const int64_t* __restrict__ dnY, int64_t hnY,
                                                 uint32_t* __restrict__ rowmin,
                                                 uint32_t* __restrict__ colmin) {
  constexpr int BN = BNT;
  const int64_t nX = dev_or(dnX, hnX);
  const int64_t nY = dev_or(dnY, hnY);
  const int64_t xt = (nX + kTileRows - 1) / kTileRows;
  const int64_t nyb = (nY + BN - 1) / BN;
  if (xt == 0 || nyb == 0) return;
  const int64_t S = tile_split(xt, nyb, gridDim.x);
  tile_schedule(xt, nyb, S, blockIdx.x, gridDim.x, [&](int64_t xblk, int64_t b0, int64_t b1) {
    __syncthreads();  // LDS of the previous segment is no longer read
    dist_seg<DP, COLMIN, GX, BNT>(Xp, xn, xidx, nX, Yp, yn, xblk * kTileRows, b0 * BN,
                                  min(nY, b1 * BN), rowmin, colmin);
  });
}

// Both directions of a search in one launch: work-groups [0, g0) run the
// first direction's schedule among themselves, the rest the second's (g0 a
// multiple of 8 where the grid allows, so a work-group's XCD is the same
// in both numberings).  Two directions of a few hundred row tiles each fill
// the chip together where one alone leaves it half idle.
struct TileDir {
  const float* Xp;
  const float* xn;
  const int32_t* xidx;
  const int64_t* dnX;
  int64_t hnX;
  const float* Yp;
  const float* yn;
  const int64_t* dnY;
  int64_t hnY;
  uint32_t* rowmin;
  uint32_t* colmin;
};
struct TilePair {
  TileDir d[2];
  int32_t g0;
};

template <int DP, bool COLMIN, bool GX, int BNT>
__global__ __launch_bounds__(512) void dist_tile2(const TilePair P) {
  constexpr int BN = BNT;
  const bool second = (int)blockIdx.x >= P.g0;   // uniform
  const TileDir d = P.d[second ? 1 : 0];
  const int64_t G = second ? (int64_t)gridDim.x - P.g0 : P.g0;
  const int64_t bx = second ? (int64_t)blockIdx.x - P.g0 : blockIdx.x;
  const int64_t nX = dev_or(d.dnX, d.hnX);
  const int64_t nY = dev_or(d.dnY, d.hnY);
  const int64_t xt = (nX + kTileRows - 1) / kTileRows;
  const int64_t nyb = (nY + BN - 1) / BN;
  if (xt == 0 || nyb == 0) return;
  const int64_t S = tile_split(xt, nyb, G);
  tile_schedule(xt, nyb, S, bx, G, [&](int64_t xblk, int64_t b0, int64_t b1) {
    __syncthreads();  // LDS of the previous segment is no longer read
    dist_seg<DP, COLMIN, GX, BNT>(d.Xp, d.xn, d.xidx, nX, d.Yp, d.yn, xblk * kTileRows, b0 * BN,
                                  min(nY, b1 * BN), d.rowmin, d.colmin);
  });
}

// ------------------------------------------------- low-precision copies
// Matrix-core input formats: bfloat16 (round to nearest even) and OCP
// float8 e4m3 with one power-of-two scale for both sets, chosen from the
// largest |shifted value| so that scaled values stay below 224 (e4m3 max 448).
enum { FMT_F32 = 0, FMT_BF16 = 1, FMT_FP8 = 2 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

// Row length of the low-precision copies: float8 ops take 64 k per op, so
// rows are padded to at least 64 columns.
__host__ __device__ constexpr int qdim(int DP, int fmt) { return fmt == FMT_FP8 && DP < 64 ? 64 : DP; }

__device__ __forceinline__ float fp8_scale(const uint32_t* maxabs) {
  const float m = __uint_as_float(*maxabs);
  if (!(m > 0.f) || !(m < 3.0e38f)) return 1.f;
  // at most 2^60, so that scale^2 and the tile's 2 / scale^2 stay finite
  // normal numbers (values below about 2e-16 then quantise coarsely; the
  // FP64 refinement still measures the witnesses exactly)
  return exp2f(fminf(floorf(log2f(224.f / m)), 60.f));
}

// Xq[i] = quantised Xp[i] (DP elements), qn[i] = |dequantised row|^2.
template <int DP, int FMT>
__global__ __launch_bounds__(256) void quant_rows(const float* __restrict__ Xp,
                                                  const int64_t* __restrict__ dn, int64_t hn,
                                                  const uint32_t* __restrict__ maxabs,
                                                  void* __restrict__ Xq, float* __restrict__ qn) {
  constexpr int QD = qdim(DP, FMT);
  const int64_t n = dev_or(dn, hn);
  const int lane = threadIdx.x & 63;
  const float sc = (FMT == FMT_FP8) ? fp8_scale(maxabs) : 1.f;
  const float isc = 1.f / sc;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
    float acc = 0.f;
    // each lane converts pairs of elements k = 2 (lane + 64 c)
    for (int k = 2 * lane; k < QD; k += 128) {
      const float v0 = k < DP ? Xp[i * DP + k] : 0.f;
      const float v1 = k + 1 < DP ? Xp[i * DP + k + 1] : 0.f;
      if (FMT == FMT_BF16) {
        const __bf16 b0 = (__bf16)v0, b1 = (__bf16)v1;
        __bf16* q = reinterpret_cast<__bf16*>(Xq) + i * QD + k;
        q[0] = b0;
        q[1] = b1;
        const float d0 = (float)b0, d1 = (float)b1;
        acc = fmaf(d0, d0, acc);
        acc = fmaf(d1, d1, acc);
      } else {
        const int pk = __builtin_amdgcn_cvt_pk_fp8_f32(v0 * sc, v1 * sc, 0, false);
        uint8_t* q = reinterpret_cast<uint8_t*>(Xq) + i * QD + k;
        q[0] = (uint8_t)(pk & 0xff);
        q[1] = (uint8_t)((pk >> 8) & 0xff);
        const float d0 = __builtin_amdgcn_cvt_f32_fp8(pk, 0) * isc;
        const float d1 = __builtin_amdgcn_cvt_f32_fp8(pk, 1) * isc;
        acc = fmaf(d0, d0, acc);
        acc = fmaf(d1, d1, acc);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) qn[i] = acc;
  }
}

// Same contract as dist_tile, on bfloat16 / float8 inputs with float32
// accumulation: v_mfma_f32_32x32x16_bf16 (K = 16) or
// v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales (K = 64).  Each lane
// supplies K/2 consecutive k of its half-wave's k range per op.  A wave holds
// two 32-row sets of X (512 rows per work-group), so every B operand read
// from LDS feeds two ops: at these input widths one op per 32 or 64 cycles
// would otherwise need the whole LDS bandwidth.  Y blocks of 128 rows (four
// 32-column subtiles) per LDS buffer; rows of 256 bytes or more are copied
// from memory straight into LDS (4-byte pieces, so the padded row stride that
// keeps the b128 reads conflict-free survives), narrower rows through
// registers.  Where the registers allow, two accumulator sets let the
// epilogue of one subtile run while the next subtile's ops execute.
template <int FMT>
struct LpFmt {
  static constexpr int KPM = FMT == FMT_BF16 ? 16 : 64;   // k per op
  static constexpr int EB = FMT == FMT_BF16 ? 2 : 1;      // bytes per element
  static constexpr int LB = KPM / 2 * EB;                 // bytes per lane per op (16 or 32)
};

constexpr int kLpBN = 128;   // Y rows per LDS buffer
constexpr int kLpXS = 2;     // 32-row X sets per wave
constexpr int kLpTileRows = kTileRows * kLpXS;

template <int DP, int FMT, bool COLMIN, bool GX = false>
__device__ __forceinline__ void dist_seg_lp(const uint8_t* __restrict__ Xq,
                                            const float* __restrict__ xn,
                                            const int32_t* __restrict__ xidx, int64_t nX,
                                            const uint8_t* __restrict__ Yq,
                                            const float* __restrict__ yn, int64_t x0, int64_t yb,
                                            int64_t ye, const uint32_t* __restrict__ maxabs,
                                            uint32_t* __restrict__ rowmin,
                                            uint32_t* __restrict__ colmin) {
  using F = LpFmt<FMT>;
  constexpr int XS = kLpXS;
  constexpr int RB = DP * F::EB;            // bytes per row
  constexpr int STB = RB + 16;              // LDS row stride (bytes): conflict-free b128
  constexpr int NS = DP / F::KPM;           // ops per 32x32 subtile
  constexpr int NA = RB / 2 / 16;           // 16-byte chunks of a lane's A operand
  constexpr bool DMA = RB % 256 == 0;       // rows copied straight into LDS
  constexpr int NV = kLpBN * RB / 16;       // 16-byte chunks per Y buffer (register path)
  constexpr int PF = DMA ? 1 : (NV + 511) / 512;
  // overlapped subtiles need a second accumulator set: not at BF16 and
  // D = 256, whose two X sets already fill the registers
  constexpr bool ILV = FMT == FMT_FP8 || DP <= 128;
  // distinct LDS objects per buffer, named statically below (as in
  // dist_seg): the compiler then sees that the copy into one buffer does
  // not touch the reads of the other
  __shared__ __attribute__((aligned(16))) uint8_t ys0[kLpBN * STB];
  __shared__ __attribute__((aligned(16))) uint8_t ys1[kLpBN * STB];
  __shared__ float yns0[kLpBN], yns1[kLpBN];
  __shared__ uint32_t cmin0[kLpBN], cmin1[kLpBN];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 5;
  const int c = lane & 31;
  const float ninf = neg_inf_sreg();
  float dscale = -2.f;
  if (FMT == FMT_FP8) {
    const float sc = fp8_scale(maxabs);
    dscale = -2.f / (sc * sc);
  }

  // X set x of this wave: rows x0 + 32 (XS wave + x) ..  xc holds
  // |x|^2 / dscale (a power-of-two multiple, exact) in the accumulator
  // layout: it is the first op's C operand, so the accumulator ends at
  // |x|^2 / dscale + (quantised x).(quantised y), and d2 = dscale acc + |y|^2
  // costs one multiply-add.
  uint4 a[XS][NA];
  floatx16 xc[XS];
  float rmin[XS][16];
  const float inv_dscale = 1.f / dscale;
#pragma unroll
  for (int x = 0; x < XS; ++x) {
    const int64_t rb0 = x0 + 32 * (XS * wave + x);
    const int64_t xr = rb0 + c;
    if (xr < nX) {
      const int64_t xm = GX ? (int64_t)xidx[xr] : xr;
      const uint4* src = reinterpret_cast<const uint4*>(Xq + xm * RB + g * (RB / 2));
#pragma unroll
      for (int j = 0; j < NA; ++j) a[x][j] = src[j];
    } else {
#pragma unroll
      for (int j = 0; j < NA; ++j) a[x][j] = make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t r = rb0 + 8 * (v >> 2) + 4 * g + (v & 3);
      xc[x][v] = ((r < nX) ? xn[GX ? (int64_t)xidx[r] : r] : __uint_as_float(kInfBits)) * inv_dscale;
      rmin[x][v] = __uint_as_float(kInfBits);
    }
  }

  // Y block -> LDS buffer b.  DMA: 4-byte pieces, RB / 256 instructions per
  // row, spread over the waves; the buffer range ends at the last valid row,
  // so rows past the end read as zero.
  auto load_block = [&](int64_t y0, uint8_t* ysb, uint4 (&buf)[PF], float& ynv) {
    if constexpr (DMA) {
      const int rows = (int)min<int64_t>(kLpBN, ye - y0);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<uint8_t*>(Yq + y0 * RB), 0, rows * RB, kBufferFlags);
      constexpr int PPR = RB / 256;   // pieces per row
      for (int i = wave; i < kLpBN * PPR; i += 8) {
        const int r = i / PPR, h = i - r * PPR;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(ysb + r * STB + 256 * h), 4,
            r * RB + 256 * h + 4 * lane, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int f = tid + 512 * p;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (f < NV) {
          const int r = f / (RB / 16);
          const int q = f - r * (RB / 16);
          if (y0 + r < ye) v = reinterpret_cast<const uint4*>(Yq + (y0 + r) * RB)[q];
        }
        buf[p] = v;
      }
    }
    ynv = (tid < kLpBN && y0 + tid < ye) ? yn[y0 + tid] : __uint_as_float(kInfBits);
  };
  auto store_block = [&](uint8_t* ysb, float* ynb, uint32_t* cmb, const uint4 (&buf)[PF],
                         float ynv) {
    if constexpr (!DMA) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int f = tid + 512 * p;
        if (f < NV) {
          const int r = f / (RB / 16);
          const int q = f - r * (RB / 16);
          *reinterpret_cast<uint4*>(ysb + r * STB + 16 * q) = buf[p];
        }
      }
    }
    if (tid < kLpBN) {
      ynb[tid] = ynv;
      cmb[tid] = kInfBits;
    }
  };
  // one 32-column subtile against both X sets: each B read feeds XS ops
  auto subtile = [&](const uint8_t* cy, int t, floatx16 (&acc)[XS]) {
    __builtin_amdgcn_s_setprio(1);   // issue priority while the ops go out
#pragma unroll
    for (int x = 0; x < XS; ++x) acc[x] = xc[x];
    const uint8_t* yrow = cy + (32 * t + c) * STB + g * (RB / 2);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if constexpr (FMT == FMT_BF16) {
        const uint4 bv = *reinterpret_cast<const uint4*>(yrow + 16 * s);
#pragma unroll
        for (int x = 0; x < XS; ++x)
          acc[x] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[x][s]),
                                                           __builtin_bit_cast(bf16x8, bv), acc[x], 0, 0, 0);
      } else {
        const uint4 b0 = *reinterpret_cast<const uint4*>(yrow + 32 * s);
        const uint4 b1 = *reinterpret_cast<const uint4*>(yrow + 32 * s + 16);
        const intx8 bw = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w,
                          (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
#pragma unroll
        for (int x = 0; x < XS; ++x) {
          const intx8 av = {(int)a[x][2 * s].x, (int)a[x][2 * s].y, (int)a[x][2 * s].z,
                            (int)a[x][2 * s].w, (int)a[x][2 * s + 1].x, (int)a[x][2 * s + 1].y,
                            (int)a[x][2 * s + 1].z, (int)a[x][2 * s + 1].w};
          // formats 0/0 = e4m3 for both operands; scales 0x7f = 2^0
          acc[x] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bw, acc[x], 0, 0, 0, 0x7f7f7f7f,
                                                                   0, 0x7f7f7f7f);
        }
      }
    }
  };
  // returns the subtile's column minima (lanes g == 0 hold them)
  auto epilogue = [&](const float* cyn, int t, const floatx16 (&acc)[XS]) {
    __builtin_amdgcn_s_setprio(0);
    const float ynv = cyn[32 * t + c];
    float cm = __uint_as_float(kInfBits);
#pragma unroll
    for (int x = 0; x < XS; ++x)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float d = fmaf(dscale, acc[x][v], ynv);
        rmin[x][v] = run_min(rmin[x][v], d, ninf);
        cm = fminf(cm, d);
      }
    return COLMIN ? run_min(cm, __shfl_xor(cm, 32), ninf) : cm;
  };

  uint4 pf[PF];
  float pyn;
  load_block(yb, ys0, pf, pyn);
  store_block(ys0, yns0, cmin0, pf, pyn);
  if (DMA) __builtin_amdgcn_s_waitcnt(0);   // this wave's row copies have landed
  __syncthreads();

  // block at y0 in buffer cy (norms cyn, column minima ccm); the next block
  // is copied into ny
  auto block = [&](int64_t y0, const uint8_t* cy, const float* cyn, uint32_t* ccm, uint8_t* ny,
                   float* nyn, uint32_t* ncm) {
    const bool more = y0 + kLpBN < ye;
    if (more) load_block(y0 + kLpBN, ny, pf, pyn);
    const int nsub = (int)min<int64_t>(4, (ye - y0 + 31) / 32);
    float cms[4];
    if constexpr (ILV) {
      // two accumulator sets: one subtile's epilogue runs while the next
      // subtile's ops execute
      floatx16 p0[XS], p1[XS];
      subtile(cy, 0, p0);
      if (nsub > 1) subtile(cy, 1, p1);
      cms[0] = epilogue(cyn, 0, p0);
      if (nsub > 2) subtile(cy, 2, p0);
      if (nsub > 1) cms[1] = epilogue(cyn, 1, p1);
      if (nsub > 3) subtile(cy, 3, p1);
      if (nsub > 2) cms[2] = epilogue(cyn, 2, p0);
      if (nsub > 3) cms[3] = epilogue(cyn, 3, p1);
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < nsub) {
          floatx16 acc[XS];
          subtile(cy, t, acc);
          cms[t] = epilogue(cyn, t, acc);
        }
      }
    }
    // LDS writes after the wait for this wave's row copies (the compiler
    // would otherwise hold each of them until every copy in flight landed)
    if (DMA) __builtin_amdgcn_s_waitcnt(0);
    if (COLMIN && g == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nsub) atomicMin(&ccm[32 * t + c], clamp_bits(cms[t]));
    }
    if (more) store_block(ny, nyn, ncm, pf, pyn);
    __syncthreads();
    if (COLMIN && tid < kLpBN) {
      const uint32_t v = ccm[tid];
      if (y0 + tid < ye) atomicMin(&colmin[y0 + tid], v);
    }
  };
  for (int64_t y0 = yb; y0 < ye; y0 += 2 * kLpBN) {
    block(y0, ys0, yns0, cmin0, ys1, yns1, cmin1);
    if (y0 + kLpBN < ye) block(y0 + kLpBN, ys1, yns1, cmin1, ys0, yns0, cmin0);
  }

  // row minima: reduce over the 32 lanes of each half-wave (same rows)
#pragma unroll
  for (int x = 0; x < XS; ++x) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float t = rmin[x][v];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) t = run_min(t, __shfl_xor(t, off), ninf);
      rmin[x][v] = t;
    }
    float mine = __uint_as_float(kInfBits);
#pragma unroll
    for (int v = 0; v < 16; ++v) mine = (c == v) ? rmin[x][v] : mine;
    if (c < 16) {
      const int64_t r = x0 + 32 * (XS * wave + x) + 8 * (c >> 2) + 4 * g + (c & 3);
      if (r < nX && rowmin) atomicMin(&rowmin[r], clamp_bits(mine));
    }
  }
}

// Persistent form of the low-precision tile (same schedule as dist_tile).
template <int DP, int FMT, bool COLMIN, bool GX = false>
__global__ __launch_bounds__(512) void dist_tile_lp(const uint8_t* __restrict__ Xq,
                                                     const float* __restrict__ xn,
                                                     const int32_t* __restrict__ xidx,
                                                     const int64_t* __restrict__ dnX, int64_t hnX,
                                                     const uint8_t* __restrict__ Yq,
                                                     const float* __restrict__ yn,
                                                     const int64_t* __restrict__ dnY, int64_t hnY,
                                                     const uint32_t* __restrict__ maxabs,
                                                     uint32_t* __restrict__ rowmin,
                                                     uint32_t* __restrict__ colmin) {
  const int64_t nX = dev_or(dnX, hnX);
  const int64_t nY = dev_or(dnY, hnY);
  const int64_t xt = (nX + kLpTileRows - 1) / kLpTileRows;
  const int64_t nyb = (nY + kLpBN - 1) / kLpBN;
  if (xt == 0 || nyb == 0) return;
  const int64_t S = tile_split(xt, nyb, gridDim.x);
  tile_schedule(xt, nyb, S, blockIdx.x, gridDim.x, [&](int64_t xblk, int64_t b0, int64_t b1) {
    __syncthreads();  // LDS of the previous segment is no longer read
    dist_seg_lp<DP, FMT, COLMIN, GX>(Xq, xn, xidx, nX, Yq, yn, xblk * kLpTileRows, b0 * kLpBN,
                                 min(nY, b1 * kLpBN), maxabs, rowmin, colmin);
  });
}

// ---------------------------------------------------------------- refine
// best[r] = min over y of (bits(float(d2)) << 32 | y), ties to the smallest y,
// for candidate rows cand[r], r < R, with d2 = |x|^2 + |y|^2 - 2 x.y evaluated
// in float64 (v_mfma_f64_16x16x4f64 on the exactly converted float32 rows):
// the expansion's rounding is ~1e-16 |x|^2, far below float32 resolution.
// A wave owns 16 candidate rows (A operands in registers); Y streams through
// LDS as float64, 32 rows per block (two 16-column accumulators).
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Candidate block cb (rows 64 cb .. 64 cb + 63 of cand[0..R)) against Y
// chunk ysi of ysplit.  Every thread of the work-group makes the same call;
// LDS is reused from one call to the next (each Y block starts at a barrier).
template <int DP>
__device__ __forceinline__ void refine_block(const float* __restrict__ Xp,
                                             const int32_t* __restrict__ cand, int64_t R,
                                             const float* __restrict__ Yp, int64_t nY, int ysplit,
                                             int ysi, int64_t cb,
                                             unsigned long long* __restrict__ best) {
  constexpr int KS = DP / 4;        // k steps of the 16x16x4 op
  constexpr int BNY = 32;           // Y rows per LDS block
  constexpr int STY = DP + 4;       // LDS row stride (doubles)
  __shared__ double ys[BNY * STY];
  __shared__ double yq[BNY];
  if (cb * 64 >= R) return;
  const int64_t chunk = ((nY + ysplit - 1) / ysplit + BNY - 1) / BNY * BNY;
  const int64_t yb = (int64_t)ysi * chunk;
  const int64_t ye = min(nY, yb + chunk);
  if (yb >= ye) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int i16 = lane & 15;   // A row / B column within the 16-block
  const int kq = lane >> 4;    // k within the group of four

  // A operands: candidate row 64 cb + 16 wave + i16, k = 4 s + kq
  const int64_t cr = cb * 64 + 16 * wave + i16;
  const float* xrow = (cr < R) ? (Xp + (int64_t)cand[cr] * DP) : nullptr;
  double a[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) a[s] = xrow ? (double)xrow[4 * s + kq] : 0.0;
  // |x|^2 in float64 for the four rows this lane's results cover (l/16 + 4v)
  double xq[4];
  {
    double part = 0.0;
#pragma unroll
    for (int s = 0; s < KS; ++s) part = fma(a[s], a[s], part);
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);   // lanes with equal i16 hold |x_row i16|^2
#pragma unroll
    for (int v = 0; v < 4; ++v) xq[v] = __shfl(part, kq + 4 * v);
  }
  double bv[4];
  int bi[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    bv[v] = __longlong_as_double(0x7ff0000000000000ll);
    bi[v] = 0x7fffffff;
  }
  for (int64_t y0 = yb; y0 < ye; y0 += BNY) {
    __syncthreads();
    // stage 32 rows as float64 and their squared norms (8 threads per row;
    // at DP >= 32 each thread moves float4 runs, all loads of a row issued
    // before the conversions)
    {
      const int r = tid >> 3, part = tid & 7;
      const bool ok = y0 + r < ye;
      const float* src = Yp + (y0 + r) * DP;
      double sq = 0.0;
      if constexpr (DP >= 32) {
        constexpr int NQ = DP / 32;   // float4 runs per thread
        float4 q[NQ];
#pragma unroll
        for (int j = 0; j < NQ; ++j)
          q[j] = ok ? *reinterpret_cast<const float4*>(src + 4 * part + 32 * j)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
          const int k = 4 * part + 32 * j;
          const double v0 = q[j].x, v1 = q[j].y, v2 = q[j].z, v3 = q[j].w;
          ys[r * STY + k] = v0;
          ys[r * STY + k + 1] = v1;
          ys[r * STY + k + 2] = v2;
          ys[r * STY + k + 3] = v3;
          sq = fma(v0, v0, sq);
          sq = fma(v1, v1, sq);
          sq = fma(v2, v2, sq);
          sq = fma(v3, v3, sq);
        }
      } else {
#pragma unroll 4
        for (int k = part; k < DP; k += 8) {
          const double v = ok ? (double)src[k] : 0.0;
          ys[r * STY + k] = v;
          sq = fma(v, v, sq);
        }
      }
      sq += __shfl_xor(sq, 1);
      sq += __shfl_xor(sq, 2);
      sq += __shfl_xor(sq, 4);
      if (part == 0) yq[r] = ok ? sq : __longlong_as_double(0x7ff0000000000000ll);
    }
    __syncthreads();
    doublex4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
    const double* b0 = &ys[i16 * STY + kq];
    const double* b1 = &ys[(16 + i16) * STY + kq];
    // fully unrolled: a partial unroll leaves the accumulators crossing a
    // loop edge, which the compiler pays for with register-class copies
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b0[4 * s], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b1[4 * s], c1, 0, 0, 0);
    }
    // element v of lane l: row l/16 + 4 v, column l%16 (of each 16 block)
    const double q0 = yq[i16], q1 = yq[16 + i16];
    const int j0 = (int)(y0 + i16), j1 = (int)(y0 + 16 + i16);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double d0 = xq[v] + q0 - 2.0 * c0[v];
      const double d1 = xq[v] + q1 - 2.0 * c1[v];
      if (d0 < bv[v]) { bv[v] = d0; bi[v] = j0; }
      if (d1 < bv[v]) { bv[v] = d1; bi[v] = j1; }
    }
  }
  // reduce over the 16 lanes sharing rows; ties -> smallest index
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float f = bv[v] > 0.0 ? (float)bv[v] : 0.f;
    unsigned long long p = ((unsigned long long)__float_as_uint(f) << 32) | (uint32_t)bi[v];
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const unsigned long long o = __shfl_xor(p, off);
      p = o < p ? o : p;
    }
    const int64_t r = cb * 64 + 16 * wave + kq + 4 * v;
    if (i16 == 0 && r < R) atomicMin(&best[r], p);
  }
}

// Few rows (R <= kThinRows): the float64 pass as direct differences on the
// vector ALUs, each wave measuring whole Y rows of its chunk (lane l holds
// dimensions l, l + 64, ...; loads of 256 contiguous bytes), the R rows in
// registers; the matrix-core block would spend 64 rows' work on them.  Same
// Y chunking, packing (float32 bits of d^2, then the index) and arg-min
// rule (ties -> smallest index) as refine_block.  The waves' minima meet in
// LDS and each work-group makes one atomic per row (every work-group's
// atomic hits the same R words, so their number sets the tail).
constexpr int kThinRows = 8;

template <int DP>
__device__ __forceinline__ void refine_thin(const float* __restrict__ Xp,
                                            const int32_t* __restrict__ cand, int64_t R,
                                            const float* __restrict__ Yp, int64_t nY, int ysplit,
                                            int ysi, unsigned long long* __restrict__ best) {
  constexpr int BNY = 32;
  constexpr int NJ = DP >= 64 ? DP / 64 : 1;
  const int64_t chunk = ((nY + ysplit - 1) / ysplit + BNY - 1) / BNY * BNY;
  const int64_t yb = (int64_t)ysi * chunk;
  const int64_t ye = min(nY, yb + chunk);
  if (yb >= ye) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  double xv[kThinRows][NJ];
#pragma unroll
  for (int r = 0; r < kThinRows; ++r)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int k = lane + 64 * j;
      xv[r][j] = (r < R && k < DP) ? (double)Xp[(int64_t)cand[r] * DP + k] : 0.0;
    }
  double bv[kThinRows];
  int bi[kThinRows];
#pragma unroll
  for (int r = 0; r < kThinRows; ++r) {
    bv[r] = __longlong_as_double(0x7ff0000000000000ll);
    bi[r] = 0x7fffffff;
  }
  // UY rows per step, all their loads issued before any use
  constexpr int UY = 4;
  for (int64_t y0 = yb + (int64_t)UY * wave; y0 < ye; y0 += (int64_t)UY * nw) {
    // unconditional loads (rows clamped to the chunk, columns to the row);
    // rows past the chunk are skipped below, columns past DP zeroed
    float yf[UY][NJ];
#pragma unroll
    for (int u = 0; u < UY; ++u) {
      const int64_t yy = min(y0 + u, ye - 1);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int k = lane + 64 * j;
        const float v = Yp[yy * DP + (k < DP ? k : 0)];
        yf[u][j] = k < DP ? v : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < UY; ++u) {
      if (y0 + u >= ye) break;
#pragma unroll
      for (int r = 0; r < kThinRows; ++r) {
        if (r >= R) break;
        double sq = 0.0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const double t = xv[r][j] - (double)yf[u][j];
          sq = fma(t, t, sq);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
        if (sq < bv[r]) {
          bv[r] = sq;
          bi[r] = (int)(y0 + u);
        }
      }
    }
  }
  __shared__ unsigned long long red[kThinRows][16];
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < kThinRows; ++r) {
      const float f = bv[r] > 0.0 ? (float)bv[r] : 0.f;
      red[r][wave] = ((unsigned long long)__float_as_uint(f) << 32) | (uint32_t)bi[r];
    }
  }
  __syncthreads();
  if ((int64_t)threadIdx.x < R) {
    unsigned long long k = red[threadIdx.x][0];
    for (int w = 1; w < nw; ++w) k = red[threadIdx.x][w] < k ? red[threadIdx.x][w] : k;
    atomicMin(&best[threadIdx.x], k);
  }
}

// Second refinement pass: the candidate count is known only on the device,
// so the grid is (groups) x (ysplit Y chunks) and each work-group walks the
// candidate blocks cb = group, group + groups, ...; with no candidates (the
// usual case) every work-group returns at once.
template <int DP>
__device__ __forceinline__ void refine_dyn_body(const float* __restrict__ Xp,
                                                const int32_t* __restrict__ cand,
                                                const int64_t* __restrict__ dR,
                                                const float* __restrict__ Yp,
                                                const int64_t* __restrict__ dnY, int64_t hnY,
                                                int ysplit, unsigned long long* __restrict__ best,
                                                int bx, int nbx) {
  const int64_t R = *dR;
  const int64_t nY = dev_or(dnY, hnY);
  const int groups = nbx / ysplit;
  const int g = bx / ysplit;
  const int ysi = bx - g * ysplit;
  if (R <= kThinRows) return;   // refine_rows_thin takes these
  for (int64_t cb = g; cb * 64 < R; cb += groups)
    refine_block<DP>(Xp, cand, R, Yp, nY, ysplit, ysi, cb, best);
}

// Both directions in one launch (grid y = direction).
struct RefineDir {
  const float* Xp;            // outer rows (prepared)
  const int32_t* cand;        // listed outer rows
  const int64_t* dR;          // their device count
  const float* Yp;            // inner set (prepared)
  const int64_t* dnY;         // its device length, or null
  int64_t hnY;                // its host bound
  unsigned long long* best;   // per listed row: (float bits of d^2, index)
};
struct RefinePair {
  RefineDir d[2];
};

template <int DP>
__global__ __launch_bounds__(256) void refine_rows_dyn(const RefinePair P) {
  const RefineDir d = P.d[blockIdx.y];
  refine_dyn_body<DP>(d.Xp, d.cand, d.dR, d.Yp, d.dnY, d.hnY, gridDim.x, d.best, blockIdx.x, gridDim.x);
}

// The same pass for R <= kThinRows rows (a kernel of its own: it needs far
// fewer registers than the matrix-core block, so more waves hide the
// memory latency); with more rows it returns at once.
template <int DP>
__global__ __launch_bounds__(256) void refine_rows_thin(const RefinePair P) {
  const RefineDir d = P.d[blockIdx.y];
  const int64_t R = *d.dR;
  if (R < 1 || R > kThinRows) return;
  refine_thin<DP>(d.Xp, d.cand, R, d.Yp, dev_or(d.dnY, d.hnY), gridDim.x, blockIdx.x, d.best);
}

// ------------------------------------------------- certified refinement
// The tile search gives each row x an approximate squared minimum m2 of its
// distance to the other set.  Which rows the float64 refinement re-measures
// follows from a bound of the search error, so that the maximum it returns
// is the exact directed distance (up to the float64 rounding of the
// re-measured rows) for any data, not only where the approximate minima
// happen to rank the witness among the first rows.
//
// Error model.  x, y are the shifted float32 rows; xq, yq the copies the
// tile multiplies (x, y themselves in float32; rounded to nearest bfloat16,
// or to e4m3 after the power-of-two scale sc, in the low-precision formats);
// K is the number of products per dot product (padded width).
//   quantisation  |xq - x| <= uq |x| + a        uq = 2^-8 (bfloat16: round to
//                 nearest even), 2^-3 (e4m3: one unit in the last place, which
//                 holds for any rounding of the conversion), 0 (float32); a
//                 covers subnormals: sqrt(K) 2^-9 / sc for e4m3 (one subnormal
//                 step), sqrt(K) 2^-126 (operands flushed to zero) otherwise
//   expansion     |m2~ - |xq - yq|^2| <= c (|xq| + |yq|)^2 + eta  per pair,
//                 c = 2 (K + 4) 2^-24: twice the worst-case error of a float32
//                 sum of the K products and the two norms in any order; eta =
//                 16 (K + 4) 2^-126 (flushed subnormal products; / sc^2 for e4m3)
// For the row y* the search found (squared value m2) let t = |x - y*|; with
// S >= |x| one has |x| + |y*| <= 2 S + t, so
//   |xq - y*q| >= p t - b,               p = 1 - uq, b = 2 (uq S + a)
//   |xq - y*q|^2 <= m2 + eta + (r t + e)^2,  r = sqrt(c)(1 + uq),
//                                            e = sqrt(c)(2 (1 + uq) S + 2 a)
// and (p t - b)^2 - (r t + e)^2 <= m2 + eta.  The larger root of that
// quadratic bounds t, and the row's true minimum is at most t:
//   U = ((p b + r e) + sqrt((p e + r b)^2 + (p^2 - r^2)(m2 + eta))) / (p^2 - r^2).
// U replaces m2 as the ranking key (bits of U^2 rounded up to float32, in
// place): the first refinement takes the 256 rows with the largest U; then
// every other row whose U exceeds the largest refined minimum is refined
// too (uncertain_rows + refine_rows_dyn, usually nothing), after which no
// unrefined row can exceed the returned maximum.
struct SearchModel {
  double c, uq, a, eta;
};

__device__ __forceinline__ SearchModel search_model(int K, int fmt, const uint32_t* maxabs) {
  SearchModel q;
  q.c = 2.0 * (K + 4) * 0x1p-24;
  q.eta = 16.0 * (K + 4) * 0x1p-126;
  q.uq = 0.0;
  q.a = sqrt((double)K) * 0x1p-126;
  if (fmt == FMT_BF16) q.uq = 0x1p-8;
  if (fmt == FMT_FP8) {
    const double sc = fp8_scale(maxabs);
    q.uq = 0x1p-3;
    q.a = sqrt((double)K) * 0x1p-9 / sc;
    q.eta /= sc * sc;
  }
  return q;
}

__device__ __forceinline__ double min_upper(double m2, double S, const SearchModel& q) {
  const double rc = sqrt(q.c);
  const double p = 1.0 - q.uq, b = 2.0 * (q.uq * S + q.a);
  const double r = rc * (1.0 + q.uq), e = rc * (2.0 * (1.0 + q.uq) * S + 2.0 * q.a);
  const double den = p * p - r * r;
  const double g = p * e + r * b;
  return ((p * b + r * e) + sqrt(g * g + den * (m2 + q.eta))) / den;
}

// float32 bits of the smallest float >= v (v >= 0)
__device__ __forceinline__ uint32_t bits_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
  return __float_as_uint(f);
}

// float32 bits of the largest float <= v (v >= 0)
__device__ __forceinline__ uint32_t bits_down(double v) {
  float f = (float)v;
  if ((double)f > v) f = __uint_as_float(__float_as_uint(f) - 1u);
  return __float_as_uint(f);
}

// mins[i] (bits of the approximate squared minimum) -> bits of U^2 rounded
// up, for the rows i < n.  xn[i]: float32 |x_i|^2 of the shifted row (DP
// terms, so |x|^2 <= xn (1 + 2 (DP + 2) 2^-24)).
// With `map`, entry i belongs to row map[i] (norm xn[map[i]]).
__device__ __forceinline__ void bound_keys_body(uint32_t* __restrict__ mins,
                                                const float* __restrict__ xn, int64_t n, int DP,
                                                int K, int fmt, const uint32_t* __restrict__ maxabs,
                                                int64_t i0, int64_t stride,
                                                const int32_t* __restrict__ map = nullptr) {
  const SearchModel q = search_model(K, fmt, maxabs);
  const double grow = 1.0 + 2.0 * (DP + 2) * 0x1p-24;
  for (int64_t i = i0; i < n; i += stride) {
    const double m2 = (double)__uint_as_float(mins[i]);
    const double S = sqrt((double)xn[map ? (int64_t)map[i] : i] * grow);
    const double U = min_upper(m2, S, q);
    mins[i] = bits_up(U * U * (1.0 + 0x1p-40));
  }
}

// Lower bound L of a row's true minimum t' from the search's approximate
// squared minimum m2: for the true nearest row y', m2 <= d~(x, y') and, with
// the same error model and symbols as min_upper,
//   m2 <= ((1 + uq) t' + b)^2 + (r t' + e)^2 + eta,
// whose right side increases with t' >= 0; L is the root of equality (0
// when m2 - eta <= b^2 + e^2).  A stored minimum clamped at zero gives 0.
__device__ __forceinline__ double min_lower(double m2, double S, const SearchModel& q) {
  const double rc = sqrt(q.c);
  const double P = 1.0 + q.uq, b = 2.0 * (q.uq * S + q.a);
  const double r = rc * (1.0 + q.uq), e = rc * (2.0 * (1.0 + q.uq) * S + 2.0 * q.a);
  const double w = m2 - q.eta - b * b - e * e;   // -(constant term)
  if (!(w > 0.0)) return 0.0;
  const double A2 = P * P + r * r, B1 = P * b + r * e;
  return w / (B1 + sqrt(B1 * B1 + A2 * w));
}

// Row bounds of one direction's search results: key[i] (bits of the row's
// approximate squared minimum) -> bits of U^2 rounded up, as bound_keys_body;
// with `hlow`, the largest L^2 (rounded down) over the rows is merged into
// *hlow (float bits of non-negative values order as unsigned integers).
// `zero` (optional) is cleared: the count of the list the next step fills.
struct BoundJob {
  uint32_t* key;
  const float* xn;          // norms of the outer rows (indexed through map)
  const int32_t* map;       // entry i -> outer row map[i] (or null: i)
  const int64_t* dn;        // entries (device) or null
  int64_t hn;               // entries (host bound)
  uint32_t* hlow;           // or null
  int64_t* zero;            // or null
};
struct BoundPair {
  BoundJob d[2];
};

__global__ __launch_bounds__(256) void row_bounds(const BoundPair P, int DP, int K, int fmt,
                                                  const uint32_t* __restrict__ maxabs) {
  const BoundJob& j = P.d[blockIdx.y];
  if (j.zero && blockIdx.x == 0 && threadIdx.x == 0) *j.zero = 0;
  const SearchModel q = search_model(K, fmt, maxabs);
  const double grow = 1.0 + 2.0 * (DP + 2) * 0x1p-24;
  const int64_t n = dev_or(j.dn, j.hn);
  double lmax = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double m2 = (double)__uint_as_float(j.key[i]);
    const double S = sqrt((double)j.xn[j.map ? (int64_t)j.map[i] : i] * grow);
    const double U = min_upper(m2, S, q);
    j.key[i] = bits_up(U * U * (1.0 + 0x1p-40));
    if (j.hlow) lmax = fmax(lmax, min_lower(m2, S, q));
  }
  if (!j.hlow) return;
  uint32_t lb = bits_down(lmax * lmax * (1.0 - 0x1p-40));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lb = max(lb, (uint32_t)__shfl_xor(lb, o));
  if ((threadIdx.x & 63) == 0 && lb > 0) atomicMax(j.hlow, lb);
}

// Rows that may hold the directed distance: every entry whose key (U^2 of
// its row) is at least *hlow (the largest certified L^2) is appended to
// cand (as map[i], or i), with best[pos] = ~0 for the float64 pass that
// follows.  Order of the list: arbitrary (wave-aggregated atomic appends);
// everything that reads it is order-independent.  The count must be zero
// before the launch.  Nothing is appended after a device error.
struct AppendJob {
  const uint32_t* key;
  const int32_t* map;
  const int64_t* dn;
  int64_t hn;
  const uint32_t* hlow;
  int32_t* cand;
  int64_t* count;
  unsigned long long* best;
};
struct AppendPair {
  AppendJob d[2];
};

__global__ __launch_bounds__(256) void append_uncertain(const AppendPair P,
                                                        const int32_t* __restrict__ status) {
  const AppendJob& j = P.d[blockIdx.y];
  if (*status != ST_OK) return;
  const int64_t n = dev_or(j.dn, j.hn);
  const uint32_t tb = *j.hlow;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs the same number of iterations
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
    const int64_t i = base + lane;
    const bool on = i < n && j.key[i] >= tb;
    const unsigned long long m = __ballot(on);
    if (m == 0) continue;
    unsigned long long at = 0;
    if (lane == 0) at = atomicAdd(reinterpret_cast<unsigned long long*>(j.count), (unsigned long long)__popcll(m));
    at = __shfl(at, 0);
    if (on) {
      const int64_t pos = (int64_t)at + __popcll(m & ((1ull << lane) - 1ull));
      j.cand[pos] = j.map ? j.map[i] : (int32_t)i;
      j.best[pos] = ~0ull;
    }
  }
}

// Pruned search: the subset of a prepared set made of its rows at positions
// 0, F, 2F, ... (all of them, float32 and low-precision copies with their
// norms); *dsub = number of subset rows.  One wave per row.  The search
// runs levels of strides 16^L, ..., 16, 1 (see prune_levels).
constexpr int kPruneMaxLevels = 4;       // strides up to 16^4
constexpr int64_t kPruneMinRows = 16384;   // smaller sets are searched in full

template <int DP, int FMT>
__global__ __launch_bounds__(256) void gather_subset(const float* __restrict__ Xp,
                                                     const float* __restrict__ xn,
                                                     const uint8_t* __restrict__ Xq,
                                                     const float* __restrict__ xqn,
                                                     const int64_t* __restrict__ dn, int64_t hn,
                                                     float* __restrict__ Sp, float* __restrict__ sn,
                                                     uint8_t* __restrict__ Sq, float* __restrict__ sqn,
                                                     int64_t* __restrict__ dsub, int F) {
  constexpr int QB = FMT == FMT_F32 ? 0 : qdim(DP, FMT) * (FMT == FMT_BF16 ? 2 : 1);   // bytes per row
  const int64_t n = dev_or(dn, hn);
  const int64_t ns = (n + F - 1) / F;
  if (blockIdx.x == 0 && threadIdx.x == 0) *dsub = ns;
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < ns; i += (int64_t)gridDim.x * 4) {
    const int64_t src = i * F;
    for (int k = lane; k < DP; k += 64) Sp[i * DP + k] = Xp[src * DP + k];
    if constexpr (QB > 0) {
      for (int k = 4 * lane; k < QB; k += 256)
        *reinterpret_cast<uint32_t*>(Sq + i * QB + k) = *reinterpret_cast<const uint32_t*>(Xq + src * QB + k);
    }
    if (lane == 0) {
      sn[i] = xn[src];
      if constexpr (QB > 0) sqn[i] = xqn[src];
    }
  }
}

// A short list of rows as a set of its own: when the device count of the
// list `idx` is at most `limit`, rows idx[0..count) of X (float32 and
// low-precision copies with their norms) are copied to S and *dsmall =
// count, *dbig = 0; otherwise nothing is copied, *dsmall = 0 and *dbig =
// count.  The search of a short list runs with the list as the inner side
// of the tile (column minima), a long one with the listed rows as its outer
// side; each launch sees an empty side when it is not the one.  One wave
// per row.
// Both directions' lists in one launch (grid y = direction).
struct GatherJob {
  const float* Xp;
  const float* xn;
  const uint8_t* Xq;
  const float* xqn;
  const int32_t* idx;
  const int64_t* dcount;
  float* Sp;
  float* sn;
  uint8_t* Sq;
  float* sqn;
  int64_t* dsmall;
  int64_t* dbig;
};
struct GatherPair {
  GatherJob j[2];
  int32_t limit;
};

template <int DP, int FMT>
__global__ __launch_bounds__(256) void gather_list(const GatherPair P) {
  constexpr int QB = FMT == FMT_F32 ? 0 : qdim(DP, FMT) * (FMT == FMT_BF16 ? 2 : 1);   // bytes per row
  const GatherJob J = P.j[blockIdx.y];
  const int64_t n = *J.dcount;
  const bool small = n <= P.limit;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *J.dsmall = small ? n : 0;
    if (J.dbig) *J.dbig = small ? 0 : n;
  }
  if (!small) return;
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
    const int64_t src = J.idx[i];
    for (int k = lane; k < DP; k += 64) J.Sp[i * DP + k] = J.Xp[src * DP + k];
    if constexpr (QB > 0) {
      for (int k = 4 * lane; k < QB; k += 256)
        *reinterpret_cast<uint32_t*>(J.Sq + i * QB + k) = *reinterpret_cast<const uint32_t*>(J.Xq + src * QB + k);
    }
    if (lane == 0) {
      J.sn[i] = J.xn[src];
      if constexpr (QB > 0) J.sqn[i] = J.xqn[src];
    }
  }
}

// Exclusive prefix sum over a work-group of NT threads; *total gets the sum.
template <int NT>
__device__ __forceinline__ uint32_t wg_excl_sum(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  __syncthreads();   // the previous call's reads of lds are done
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    const uint32_t x = lds[k];
    before += k < w ? x : 0u;
    tot += x;
  }
  *total = tot;
  return before + inc - v;
}

// The rows of one direction the float64 pass must re-measure (one
// work-group, batched form): with `hlow`, every row whose key (U^2) reaches
// the largest certified L^2; without, every row not re-measured yet whose
// key exceeds the largest re-measured minimum (lowered by 2^-20 of itself
// to cover its rounding to float32 and the float64 expansion).  Their
// indices go to cand2 in ascending order (the order does not depend on
// timing), count2 gets their number and best2 the initial value of their
// minima.
template <int NT>
__device__ __forceinline__ void uncertain_body(const UncJob& j, uint32_t* lds) {
  const int tid = threadIdx.x;
  const bool ok = *j.status == ST_OK;
  int64_t n;
  int64_t tb;   // rows with key > tb are listed
  if (j.hlow) {
    // keys reaching the largest lower bound (with none above zero: every
    // row, so that the list is never empty)
    n = ok ? dev_or(j.dn, j.hn) : 0;
    tb = (int64_t)*j.hlow - 1;
  } else {
    const int64_t R = ok ? *j.dR : 0;
    n = R > 0 ? dev_or(j.dn, j.hn) : 0;
    uint32_t hb = 0;
    for (int64_t r = tid; r < R; r += NT) hb = max(hb, (uint32_t)(j.best[r] >> 32));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) hb = max(hb, (uint32_t)__shfl_xor(hb, o));
    __syncthreads();
    if ((tid & 63) == 0) lds[tid >> 6] = hb;
    __syncthreads();
    hb = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) hb = max(hb, lds[k]);
    tb = (int64_t)bits_down((double)__uint_as_float(hb) * (1.0 - 0x1p-20));
  }
  constexpr int Q = 8;
  int64_t base = 0;
  for (int64_t c0 = 0; c0 < n; c0 += (int64_t)NT * Q) {
    uint32_t f = 0, cnt = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = c0 + (int64_t)tid * Q + q;
      const bool on = i < n && (!j.top || j.top[i] == 0) && (int64_t)j.key[i] > tb;
      f |= (on ? 1u : 0u) << q;
      cnt += on ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t pos = wg_excl_sum<NT>(cnt, lds, &tot);
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if ((f >> q) & 1u) {
        const int64_t i = c0 + (int64_t)tid * Q + q;
        j.cand2[base + pos++] = j.map ? j.map[i] : (int32_t)i;
      }
    base += tot;
  }
  if (tid == 0) *j.count2 = base;
  for (int64_t i = tid; i < base; i += NT) j.best2[i] = ~0ull;
}

// -------------------------------------------------------------- finalize
struct DirIn {
  const unsigned long long* best;  // refined minima, first pass
  const int32_t* cand;             // its rows (indices into the X list)
  const int64_t* dR;               // its number of rows
  const unsigned long long* best2; // second pass (uncertain rows), or null
  const int32_t* cand2;
  const int64_t* dR2;
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

__device__ __forceinline__ void finalize_body(const DirIn& ab, const DirIn& ba, int D,
                                              const int64_t* __restrict__ dnA, int64_t hnA,
                                              const int64_t* __restrict__ dnB, int64_t hnB,
                                              const int32_t* __restrict__ status,
                                              prohd_result* __restrict__ out) {
  __shared__ double red[256];
  __shared__ unsigned long long bestp[256];
  __shared__ int64_t bestpos[256];
  int64_t wx[2], wy[2];
  double h[2];
  const int64_t nA = dev_or(dnA, hnA), nB = dev_or(dnB, hnB);
  int32_t st = *status;
  if (nA < 1 || nB < 1) st = st ? st : ST_EMPTY;
  int64_t refined = 0;
  for (int dir = 0; dir < 2; ++dir) {
    const DirIn& d = dir == 0 ? ab : ba;
    const int64_t R = (st == ST_OK && d.dR) ? *d.dR : 0;
    const int64_t R2 = (st == ST_OK && d.dR2) ? *d.dR2 : 0;
    refined = R + R2 > refined ? R + R2 : refined;
    // largest refined minimum over both passes; ties -> smallest row of the
    // X list (low word: its complement), then the first pass
    unsigned long long m = 0ull;
    int64_t mpos = -1;
    for (int64_t r = threadIdx.x; r < R + R2; r += blockDim.x) {
      const bool first = r < R;
      const unsigned long long b = first ? d.best[r] : d.best2[r - R];
      const uint32_t xi = (uint32_t)(first ? d.cand[r] : d.cand2[r - R]);
      const unsigned long long v = ((b >> 32) << 32) | (0xFFFFFFFFull - xi);
      if (v > m) {
        m = v;
        mpos = r;
      }
    }
    bestp[threadIdx.x] = m;
    bestpos[threadIdx.x] = mpos;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        const unsigned long long o = bestp[threadIdx.x + w];
        if (o > bestp[threadIdx.x] ||
            (o == bestp[threadIdx.x] && bestpos[threadIdx.x + w] < bestpos[threadIdx.x])) {
          bestp[threadIdx.x] = o;
          bestpos[threadIdx.x] = bestpos[threadIdx.x + w];
        }
      }
      __syncthreads();
    }
    const int64_t r = bestpos[0];
    __syncthreads();
    if (r >= 0) {
      const bool first = r < R;
      const int64_t xi = first ? d.cand[r] : d.cand2[r - R];
      const unsigned long long b = first ? d.best[r] : d.best2[r - R];
      const int64_t yi = (int64_t)(b & 0xFFFFFFFFull);
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
    r.refined = (int32_t)refined;
    *out = r;
  }
}

__global__ __launch_bounds__(256) void finalize(DirIn ab, DirIn ba, int D,
                                                const int64_t* __restrict__ dnA, int64_t hnA,
                                                const int64_t* __restrict__ dnB, int64_t hnB,
                                                const int32_t* __restrict__ status,
                                                prohd_result* __restrict__ out) {
  finalize_body(ab, ba, D, dnA, hnA, dnB, hnB, status, out);
}


// ------------------------------------------------------------ batched
// Persistent versions: each work-group walks the item table and runs the
// single-pair body of its job with the item's block index.
template <int DP>
__global__ __launch_bounds__(256) void prep_batch(const PrepJob* __restrict__ jobs, int D,
                                                  const BItem* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    if (w.job < 0) continue;
    const PrepJob j = jobs[w.job];
    prep_body<DP>(j.X, D, j.idx, j.dn, j.hn, j.S, j.sidx, j.sdn, j.Xp, j.xn, j.status, nullptr, w.bx,
                  j.nbx);
  }
}

template <int DP>
__global__ __launch_bounds__(512) void tile_batch(const TileJob* __restrict__ jobs,
                                                  const BItem* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    if (w.job < 0) continue;
    const TileJob j = jobs[w.job];
    __syncthreads();  // LDS of the previous item is no longer read
    dist_tile_body<DP, true>(j.Xp, j.xn, j.dnX, j.hnX, j.Yp, j.yn, j.dnY, j.hnY, j.ysplit, j.rowmin,
                             j.colmin, w.bx);
  }
}

__global__ __launch_bounds__(256) void finalize_batch(const FinalJob* __restrict__ jobs, int njobs) {
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const FinalJob j = jobs[it];
    const DirIn ab{j.ab.best, j.ab.cand, j.ab.dR, j.ab.best2, j.ab.cand2, j.ab.dR2,
                   j.ab.mapX, j.ab.mapY, j.ab.Xo, j.ab.Yo};
    const DirIn ba{j.ba.best, j.ba.cand, j.ba.dR, j.ba.best2, j.ba.cand2, j.ba.dR2,
                   j.ba.mapX, j.ba.mapY, j.ba.Xo, j.ba.Yo};
    __syncthreads();
    finalize_body(ab, ba, j.D, j.dnA, j.hnA, j.dnB, j.hnB, j.status, j.out);
  }
}

// Bound keys of one side's rows, in place over its row minima (float32
// tiles: K = DP).
__global__ __launch_bounds__(256) void keys_batch(const KeyJob* __restrict__ jobs, int DP,
                                                  const BItem* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    if (w.job < 0) continue;
    const KeyJob j = jobs[w.job];
    if (!j.hlow) {
      bound_keys_body(j.mins, j.xn, dev_or(j.dn, j.hn), DP, DP, FMT_F32, nullptr,
                      (int64_t)w.bx * blockDim.x + threadIdx.x, (int64_t)j.nbx * blockDim.x);
      continue;
    }
    // upper bounds as keys, and the largest lower bound into *hlow
    const SearchModel q = search_model(DP, FMT_F32, nullptr);
    const double grow = 1.0 + 2.0 * (DP + 2) * 0x1p-24;
    const int64_t n = dev_or(j.dn, j.hn);
    double lmax = 0.0;
    for (int64_t i = (int64_t)w.bx * blockDim.x + threadIdx.x; i < n; i += (int64_t)j.nbx * blockDim.x) {
      const double m2 = (double)__uint_as_float(j.mins[i]);
      const double S = sqrt((double)j.xn[i] * grow);
      const double U = min_upper(m2, S, q);
      j.mins[i] = bits_up(U * U * (1.0 + 0x1p-40));
      lmax = fmax(lmax, min_lower(m2, S, q));
    }
    uint32_t lb = bits_down(lmax * lmax * (1.0 - 0x1p-40));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lb = max(lb, (uint32_t)__shfl_xor(lb, o));
    if ((threadIdx.x & 63) == 0 && lb > 0) atomicMax(j.hlow, lb);
  }
}

constexpr int kUncBatchT = 256;

__global__ __launch_bounds__(kUncBatchT) void uncertain_batch(const UncJob* __restrict__ jobs,
                                                              int njobs) {
  __shared__ uint32_t lds[kUncBatchT / 64];
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const UncJob j = jobs[it];
    __syncthreads();
    uncertain_body<kUncBatchT>(j, lds);
  }
}

// Second refinement pass of many pairs: item (job, Y chunk) walks every
// candidate block of its job's device count (none in the usual case).
template <int DP>
__global__ __launch_bounds__(256) void refine_dyn_batch(const RefineJob* __restrict__ jobs,
                                                        const BItem* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    if (w.job < 0) continue;
    const RefineJob j = jobs[w.job];
    const int64_t R = *j.dR;
    const int64_t nY = dev_or(j.dnY, j.hnY);
    for (int64_t cb = 0; cb * 64 < R; ++cb)
      refine_block<DP>(j.Xp, j.cand, R, j.Yp, nY, j.ysplit, w.bx, cb, j.best);
  }
}

// ------------------------------------------------------------ host side
struct PrepSet {
  float* p = nullptr;      // padded float32 rows, cap x DP
  float* n = nullptr;      // squared norms, cap
  uint8_t* q = nullptr;    // low-precision rows (bf16 / fp8), cap x DP
  float* qn = nullptr;     // squared norms of the dequantised rows
};

template <int DP>
prohd_status launch_prep2(const PrepPair& P, hipStream_t s) {
  const int64_t cap = std::max(P.j[0].hn, P.j[1].hn);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(cap, 4), 8 * cu_count()));
  PROHD_LAUNCH("hd_prep", prep_rows<DP>, dim3(grid, 2), dim3(256), 0, s, P);
  return PROHD_OK;
}

template <int DP>
prohd_status launch_quant(int fmt, PrepSet o, const int64_t* dn, int64_t cap, const uint32_t* maxabs,
                          hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(cap, 4), 8 * cu_count()));
  if (fmt == FMT_BF16) {
    PROHD_LAUNCH("hd_quant", (quant_rows<DP, FMT_BF16>), dim3(grid), dim3(256), 0, s, o.p, dn, cap,
                 maxabs, (void*)o.q, o.qn);
  } else {
    PROHD_LAUNCH("hd_quant", (quant_rows<DP, FMT_FP8>), dim3(grid), dim3(256), 0, s, o.p, dn, cap,
                 maxabs, (void*)o.q, o.qn);
  }
  return PROHD_OK;
}

// resident work-groups of a persistent tile kernel (from its register and
// LDS use), capped by the items of the matrix
template <typename K>
int64_t tile_grid(K kernel, int64_t items) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 512, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)per_cu * cu_count()));
}

// One distance-tile launch: X rows (all of X, or with `xidx` the rows it
// lists; row minima then go to positions of the list) against Y rows.
template <int DP, bool COLMIN, bool GX>
prohd_status launch_tile_k(int fmt, PrepSet X, const int32_t* xidx, const int64_t* dnX, int64_t capX,
                           PrepSet Y, const int64_t* dnY, int64_t capY, const uint32_t* maxabs,
                           uint32_t* rowmin, uint32_t* colmin, hipStream_t s) {
  // one resident work-group per slot, at most one per (row tile, Y block)
  // the capacities allow: a few rows against a large Y still fill the chip
  // (the kernel shares the Y blocks of its items out over the work-groups)
  // timing names: "hd_tile*" for every form; "_rows" row minima only,
  // "_gx" listed rows
  const dim3 T(512);
  if (fmt == FMT_F32) {
    const char* name = GX ? "hd_tile_gx" : COLMIN ? "hd_tile" : "hd_tile_rows";
    auto k32 = dist_tile<DP, COLMIN, GX, kBN>;
    const int64_t xt = cdiv(capX, kTileRows);
    if (tile_bn<DP>() > kBN &&
        (capY <= kBN || (capY <= 2 * kBN && xt <= 2 * tile_grid(k32, int64_t(1) << 40)))) {
      // a sparse pruning level (at most 32 Y rows), or a short list against
      // at most two rounds of row tiles: buffers of 32 rows, so padding
      // does not double the work below 32 rows, and the items of a second,
      // partial round are half-size (with more row tiles the second Y
      // subtile's items would each load their X rows again)
      const int64_t items = xt * cdiv(capY, kBN);
      auto k = k32;
      PROHD_LAUNCH(name, k, dim3((unsigned)tile_grid(k, items)), T, 0, s, X.p, X.n, xidx, dnX, capX,
                   Y.p, Y.n, dnY, capY, rowmin, colmin);
      return PROHD_OK;
    }
    const int64_t items = cdiv(capX, kTileRows) * cdiv(capY, tile_bn<DP>());
    auto k = dist_tile<DP, COLMIN, GX>;
    PROHD_LAUNCH(name, k, dim3((unsigned)tile_grid(k, items)), T, 0, s, X.p, X.n, xidx, dnX, capX,
                 Y.p, Y.n, dnY, capY, rowmin, colmin);
    return PROHD_OK;
  }
  const int64_t items = cdiv(capX, kLpTileRows) * cdiv(capY, kLpBN);
  if (fmt == FMT_BF16) {
    auto k = dist_tile_lp<qdim(DP, FMT_BF16), FMT_BF16, COLMIN, GX>;
    const char* name = GX ? "hd_tile_bf16_gx" : COLMIN ? "hd_tile_bf16" : "hd_tile_bf16_rows";
    PROHD_LAUNCH(name, k, dim3((unsigned)tile_grid(k, items)), T, 0, s, X.q, X.qn, xidx, dnX,
                 capX, Y.q, Y.qn, dnY, capY, maxabs, rowmin, colmin);
  } else {
    auto k = dist_tile_lp<qdim(DP, FMT_FP8), FMT_FP8, COLMIN, GX>;
    const char* name = GX ? "hd_tile_fp8_gx" : COLMIN ? "hd_tile_fp8" : "hd_tile_fp8_rows";
    PROHD_LAUNCH(name, k, dim3((unsigned)tile_grid(k, items)), T, 0, s, X.q, X.qn, xidx, dnX,
                 capX, Y.q, Y.qn, dnY, capY, maxabs, rowmin, colmin);
  }
  return PROHD_OK;
}

template <int DP>
prohd_status launch_tile(int fmt, PrepSet X, const int64_t* dnX, int64_t capX, PrepSet Y,
                         const int64_t* dnY, int64_t capY, const uint32_t* maxabs, uint32_t* rowmin,
                         uint32_t* colmin, hipStream_t s, const int32_t* xidx = nullptr) {
  if (xidx) {
    if (colmin) return fail(PROHD_EINVAL, "hd: listed rows take row minima only");
    return launch_tile_k<DP, false, true>(fmt, X, xidx, dnX, capX, Y, dnY, capY, maxabs, rowmin,
                                          nullptr, s);
  }
  if (colmin)
    return launch_tile_k<DP, true, false>(fmt, X, nullptr, dnX, capX, Y, dnY, capY, maxabs, rowmin,
                                          colmin, s);
  return launch_tile_k<DP, false, false>(fmt, X, nullptr, dnX, capX, Y, dnY, capY, maxabs, rowmin,
                                         nullptr, s);
}


// One direction of a tile search (the arguments of launch_tile).
struct TileArgs {
  PrepSet X;
  const int64_t* dnX;
  int64_t capX;
  PrepSet Y;
  const int64_t* dnY;
  int64_t capY;
  uint32_t* rowmin;
  uint32_t* colmin;
  const int32_t* xidx;
};

// Both directions of one kind in one float32 launch (dist_tile2) when they
// take the same tile form; otherwise, or in the low-precision formats, one
// launch each.
template <int DP, bool COLMIN, bool GX>
prohd_status launch_tile_pair_k(int fmt, const TileArgs& a, const TileArgs& b, const uint32_t* maxabs,
                                hipStream_t s) {
  auto one = [&](const TileArgs& t) {
    return launch_tile_k<DP, COLMIN, GX>(fmt, t.X, t.xidx, t.dnX, t.capX, t.Y, t.dnY, t.capY, maxabs,
                                         t.rowmin, t.colmin, s);
  };
  auto use32 = [&](const TileArgs& t) {
    const int64_t xt = cdiv(t.capX, kTileRows);
    return tile_bn<DP>() > kBN &&
           (t.capY <= kBN || (t.capY <= 2 * kBN && xt <= 2 * tile_grid(dist_tile<DP, COLMIN, GX, kBN>,
                                                                     int64_t(1) << 40)));
  };
  if (fmt != FMT_F32 || use32(a) != use32(b)) {
    const prohd_status st = one(a);
    return st != PROHD_OK ? st : one(b);
  }
  const bool b32 = use32(a);
  const int bn = b32 ? kBN : tile_bn<DP>();
  const int64_t ia = cdiv(a.capX, kTileRows) * cdiv(a.capY, bn);
  const int64_t ib = cdiv(b.capX, kTileRows) * cdiv(b.capY, bn);
  TilePair P{};
  P.d[0] = TileDir{a.X.p, a.X.n, a.xidx, a.dnX, a.capX, a.Y.p, a.Y.n, a.dnY, a.capY, a.rowmin, a.colmin};
  P.d[1] = TileDir{b.X.p, b.X.n, b.xidx, b.dnX, b.capX, b.Y.p, b.Y.n, b.dnY, b.capY, b.rowmin, b.colmin};
  auto kp32 = dist_tile2<DP, COLMIN, GX, kBN>;
  auto kp = dist_tile2<DP, COLMIN, GX, tile_bn<DP>()>;
  const int64_t grid = b32 ? tile_grid(kp32, ia + ib) : tile_grid(kp, ia + ib);
  if (grid < 2) {
    const prohd_status st = one(a);
    return st != PROHD_OK ? st : one(b);
  }
  int64_t g0 = grid * ia / (ia + ib);
  if (grid >= 16) g0 = (g0 + 4) / 8 * 8;
  P.g0 = (int32_t)std::min<int64_t>(grid - 1, std::max<int64_t>(1, g0));
  const char* name = GX ? "hd_tile_gx" : COLMIN ? "hd_tile" : "hd_tile_rows";
  if (b32) {
    PROHD_LAUNCH(name, kp32, dim3((unsigned)grid), dim3(512), 0, s, P);
  } else {
    PROHD_LAUNCH(name, kp, dim3((unsigned)grid), dim3(512), 0, s, P);
  }
  return PROHD_OK;
}

template <int DP>
prohd_status launch_tile_pair(int fmt, const TileArgs& a, const TileArgs& b, const uint32_t* maxabs,
                              hipStream_t s) {
  if ((a.xidx != nullptr) != (b.xidx != nullptr) || (a.colmin != nullptr) != (b.colmin != nullptr))
    return fail(PROHD_EINVAL, "hd: a tile pair of two kinds");
  if (a.xidx) {
    if (a.colmin) return fail(PROHD_EINVAL, "hd: listed rows take row minima only");
    return launch_tile_pair_k<DP, false, true>(fmt, a, b, maxabs, s);
  }
  if (a.colmin) return launch_tile_pair_k<DP, true, false>(fmt, a, b, maxabs, s);
  return launch_tile_pair_k<DP, false, false>(fmt, a, b, maxabs, s);
}

// Per direction: the seed rows of the pruned search (top-kSeedRows of the
// first level's bounds) and the list of rows the float64 pass re-measures.
struct DirWork {
  int32_t* cand;    // kSeedRows
  int64_t* count;   // 1
  int32_t* cand2;   // n: rows of the float64 pass (or of a pruning level)
  int64_t* count2;  // 1
  unsigned long long* best2;  // n
};

// Pruned search (per direction): the row minima of the listed rows at the
// current level, and two row lists (a level reads one, writes the other).
struct PruneWork {
  uint32_t* rowF;                 // cap
  int32_t* cand[2];               // cap each
  int64_t* count[2];              // 1 each
  unsigned long long* best[2];    // cap each
};

struct HdLayout {
  uint32_t* hlow;          // [2] largest certified L^2 per direction (bits)
  uint32_t* rowS[2];       // minima of the seed rows
  PrepSet sh[2];           // short lists (seeds, last pruning level) as sets
  int64_t* dshort;         // [2][2]: rows of sh[d] / of the long-list search
  PrepSet xa, xb;          // prepared candidate (or full) rows
  PrepSet fa, fb;          // full prepared rows (inner-full mode)
  int nlev;                // pruned search: subset levels (0: not pruned)
  PrepSet sub[2][kPruneMaxLevels];   // per direction, its inner set's subsets
  int64_t* dsub;           // [2][kPruneMaxLevels] subset row counts
  uint32_t* rowA;          // minima of A-side rows
  uint32_t* rowB;          // minima of B-side rows
  DirWork w[2];
  PruneWork pw[2];
  int32_t* status;
  uint32_t* maxabs;        // largest |shifted value| (float bits), fp8 scale
  void* top_ws;            // wave lists of the seed selection
  size_t top_bytes;
};

void take_set(Arena& ar, PrepSet& o, int64_t rows, int DP, int fmt) {
  o.p = ar.take<float>((size_t)rows * DP);
  o.n = ar.take<float>(rows);
  if (fmt != FMT_F32) {
    o.q = ar.take<uint8_t>((size_t)rows * qdim(DP, fmt) * (fmt == FMT_BF16 ? 2 : 1));
    o.qn = ar.take<float>(rows);
  }
}

// Levels of the pruned search for inner sets of at least n rows: strides
// 16^nlev, ..., 16 (level j: 16^(nlev - j)), the coarsest subset keeping
// at least 16 rows, at most kPruneMaxLevels levels.
int prune_levels(int64_t n) {
  int lev = 1;
  while (lev < kPruneMaxLevels && n / ((int64_t)1 << (4 * (lev + 1))) >= 16) ++lev;
  return lev;
}
int64_t prune_stride(int nlev, int j) { return (int64_t)1 << (4 * (nlev - j)); }

HdLayout hd_layout(Arena& ar, int64_t capA, int64_t capB, int64_t nA, int64_t nB, int DP,
                   bool full, int fmt, bool prune) {
  HdLayout L{};
  L.status = ar.take<int32_t>(64);
  L.maxabs = ar.take<uint32_t>(64);
  L.hlow = ar.take<uint32_t>(64);
  take_set(ar, L.xa, capA, DP, fmt);
  take_set(ar, L.xb, capB, DP, fmt);
  if (full) {
    take_set(ar, L.fa, nA, DP, fmt);
    take_set(ar, L.fb, nB, DP, fmt);
  }
  L.rowA = ar.take<uint32_t>(capA);
  L.rowB = ar.take<uint32_t>(capB);
  for (int d = 0; d < 2; ++d) {   // seeds and short lists (every mode)
    L.rowS[d] = ar.take<uint32_t>(kSeedRows);
    take_set(ar, L.sh[d], std::max(kSeedRows, kShortList), DP, fmt);
  }
  L.dshort = ar.take<int64_t>(4);
  const int64_t caps[2] = {capA, capB};
  for (int d = 0; d < 2; ++d) {
    L.w[d].cand = ar.take<int32_t>(kSeedRows);
    L.w[d].count = ar.take<int64_t>(1);
    L.w[d].cand2 = ar.take<int32_t>(caps[d]);
    L.w[d].count2 = ar.take<int64_t>(1);
    L.w[d].best2 = ar.take<unsigned long long>(caps[d]);
  }
  L.nlev = 0;
  if (prune) {
    const int64_t ycap[2] = {full ? nB : capB, full ? nA : capA};
    L.nlev = prune_levels(std::min(ycap[0], ycap[1]));
    L.dsub = ar.take<int64_t>(2 * kPruneMaxLevels);
    for (int d = 0; d < 2; ++d) {
      for (int j = 0; j < L.nlev; ++j)
        take_set(ar, L.sub[d][j], cdiv(ycap[d], prune_stride(L.nlev, j)), DP, fmt);
      L.pw[d].rowF = ar.take<uint32_t>(caps[d]);
      for (int b = 0; b < 2; ++b) {
        L.pw[d].cand[b] = ar.take<int32_t>(caps[d]);
        L.pw[d].count[b] = ar.take<int64_t>(1);
        L.pw[d].best[b] = ar.take<unsigned long long>(caps[d]);
      }
    }
  }
  L.top_bytes = topk_ws_bytes(std::max(capA, capB));
  L.top_ws = ar.take<char>(L.top_bytes);
  return L;
}

// Top-k rows (k <= 64) of both directions' minima (`mins[d]`, device length
// dn[d], host bound n[d]) -> w[d].cand / w[d].count; two launches for both.
prohd_status top_rows2(const uint32_t* const mins[2], const int64_t n[2], const int64_t* const dn[2],
                       DirWork* w, void* top_ws, size_t top_bytes, hipStream_t s, int k) {
  TopSegment seg[2];
  for (int d = 0; d < 2; ++d) seg[d] = TopSegment{mins[d], n[d], dn[d], k, w[d].cand, w[d].count};
  return top_keys(seg, 2, top_ws, top_bytes, s);
}

// Bound keys in place of the row minima (see the certified refinement).
// Row bounds of both directions (one launch; grid y = direction).
prohd_status launch_bounds(const BoundPair& P, int64_t cap, int DP, int fmt, const uint32_t* maxabs,
                           hipStream_t s) {
  const int K = fmt == FMT_F32 ? DP : qdim(DP, fmt);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(cap, 256), 4 * cu_count()));
  PROHD_LAUNCH("hd_keys", row_bounds, dim3(grid, 2), dim3(256), 0, s, P, DP, K, fmt, maxabs);
  return PROHD_OK;
}

// Uncertain rows of both directions (one launch; grid y = direction).
prohd_status launch_append(const AppendPair& P, int64_t cap, const int32_t* status, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(cap, 256), 4 * cu_count()));
  PROHD_LAUNCH("hd_uncertain", append_uncertain, dim3(grid, 2), dim3(256), 0, s, P, status);
  return PROHD_OK;
}

template <int DP>
prohd_status launch_subset(int fmt, PrepSet X, const int64_t* dn, int64_t cap, int64_t F, PrepSet S,
                           int64_t* dsub, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(cdiv(cap, F), 4), 1024));
  if (fmt == FMT_F32) {
    PROHD_LAUNCH("hd_subset", (gather_subset<DP, FMT_F32>), dim3(grid), dim3(256), 0, s, X.p, X.n, X.q,
                 X.qn, dn, cap, S.p, S.n, S.q, S.qn, dsub, (int)F);
  } else if (fmt == FMT_BF16) {
    PROHD_LAUNCH("hd_subset", (gather_subset<DP, FMT_BF16>), dim3(grid), dim3(256), 0, s, X.p, X.n, X.q,
                 X.qn, dn, cap, S.p, S.n, S.q, S.qn, dsub, (int)F);
  } else {
    PROHD_LAUNCH("hd_subset", (gather_subset<DP, FMT_FP8>), dim3(grid), dim3(256), 0, s, X.p, X.n, X.q,
                 X.qn, dn, cap, S.p, S.n, S.q, S.qn, dsub, (int)F);
  }
  return PROHD_OK;
}

template <int DP>
prohd_status launch_gather_lists(int fmt, const GatherPair& P, hipStream_t s) {
  const dim3 g((unsigned)cdiv(P.limit, 4), 2);
  if (fmt == FMT_F32) {
    PROHD_LAUNCH("hd_gather", (gather_list<DP, FMT_F32>), g, dim3(256), 0, s, P);
  } else if (fmt == FMT_BF16) {
    PROHD_LAUNCH("hd_gather", (gather_list<DP, FMT_BF16>), g, dim3(256), 0, s, P);
  } else {
    PROHD_LAUNCH("hd_gather", (gather_list<DP, FMT_FP8>), g, dim3(256), 0, s, P);
  }
  return PROHD_OK;
}

// Second refinement pass of one direction: cand2 / count2 / best2 against
// Y (device count known only on the device).
template <int DP>
prohd_status launch_refine_pair(const RefinePair& P, hipStream_t s) {
  const int64_t capY = std::max(P.d[0].hnY, P.d[1].hnY);
  const int split = (int)std::max<int64_t>(1, std::min<int64_t>(2 * (int64_t)cu_count(), capY / 128));
  PROHD_LAUNCH("hd_dyn_refine", refine_rows_dyn<DP>, dim3((unsigned)split, 2), dim3(256), 0, s, P);
  const int tsplit = (int)std::max<int64_t>(1, std::min<int64_t>(8 * (int64_t)cu_count(), capY / 256));
  PROHD_LAUNCH("hd_dyn_refine", refine_rows_thin<DP>, dim3((unsigned)tsplit, 2), dim3(256), 0, s, P);
  return PROHD_OK;
}

prohd_status fill_words(const FillJob* jobs, int njobs, hipStream_t s) {
  if (njobs < 1 || njobs > kFillJobs) return fail(PROHD_EINVAL, "fill_words: 1 to 8 jobs");
  FillPack P{};
  int64_t mx = 1;
  for (int i = 0; i < njobs; ++i) {
    P.j[i] = jobs[i];
    mx = std::max(mx, jobs[i].n);
  }
  const int grid = (int)std::min<int64_t>(1024, cdiv(mx, 256));
  PROHD_LAUNCH("hd_fill", fill_multi, dim3(grid, njobs), dim3(256), 0, s, P);
  return PROHD_OK;
}


#define PROHD_TRY(x)                 \
  do {                               \
    prohd_status st_ = (x);          \
    if (st_ != PROHD_OK) return st_; \
  } while (0)

// Shared driver.  Mode: exact (idx null), candidates, or candidates with the
// inner minimum over the full other set; fmt selects the tile input format.
template <int DP>
prohd_status run_hd(const float* A, int64_t nA, const float* B, int64_t nB, int D,
                    const int32_t* idxA, const int64_t* dnA, int64_t capA, const int32_t* idxB,
                    const int64_t* dnB, int64_t capB, bool full, int fmt, bool prune,
                    prohd_result* out, float* nn2A, float* nn2B, void* ws, size_t ws_bytes,
                    hipStream_t s) {
  Arena ar(ws);
  HdLayout L = hd_layout(ar, capA, capB, nA, nB, DP, full, fmt, prune);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "hd: workspace too small");
  {
    // status words, the fp8 scale and the lower bounds cleared; every row
    // minimum (outer rows of both directions, seed rows) set to +inf
    const FillJob f[7] = {{(uint32_t*)L.status, 64, 0u}, {L.maxabs, 64, 0u}, {L.hlow, 64, 0u},
                          {L.rowA, capA, kInfBits},      {L.rowB, capB, kInfBits},
                          {L.rowS[0], kSeedRows, kInfBits}, {L.rowS[1], kSeedRows, kInfBits}};
    PROHD_TRY(fill_words(f, 7, s));
  }
  uint32_t* mx = fmt == FMT_FP8 ? L.maxabs : nullptr;
  // common shift: the first (selected) row of A
  const int32_t* sidx = idxA;
  {
    PrepPair pp{{PrepDir{A, idxA, dnA, capA, L.xa.p, L.xa.n}, PrepDir{B, idxB, dnB, capB, L.xb.p, L.xb.n}},
                A, sidx, dnA, L.status, mx, D};
    PROHD_TRY(launch_prep2<DP>(pp, s));
  }
  if (full) {
    PrepPair pf{{PrepDir{A, nullptr, nullptr, nA, L.fa.p, L.fa.n}, PrepDir{B, nullptr, nullptr, nB, L.fb.p, L.fb.n}},
                A, sidx, dnA, L.status, mx, D};
    PROHD_TRY(launch_prep2<DP>(pf, s));
  }
  if (fmt != FMT_F32) {
    PROHD_TRY(launch_quant<DP>(fmt, L.xa, dnA, capA, L.maxabs, s));
    PROHD_TRY(launch_quant<DP>(fmt, L.xb, dnB, capB, L.maxabs, s));
    if (full) {
      PROHD_TRY(launch_quant<DP>(fmt, L.fa, nullptr, nA, L.maxabs, s));
      PROHD_TRY(launch_quant<DP>(fmt, L.fb, nullptr, nB, L.maxabs, s));
    }
  }
  const uint32_t* const mins2[2] = {L.rowA, L.rowB};
  const int64_t caps2[2] = {capA, capB};
  const int64_t* const dns2[2] = {dnA, dnB};
  PrepSet ysA = full ? L.fa : L.xa;   // the inner sets of the two directions
  PrepSet ysB = full ? L.fb : L.xb;
  const int64_t* ydnA = full ? nullptr : dnA;
  const int64_t* ydnB = full ? nullptr : dnB;
  const int64_t ycapA = full ? nA : capA;
  const int64_t ycapB = full ? nB : capB;
  // per direction d: outer rows xs[d], inner set ys[d] (A -> B, then B -> A)
  const PrepSet xs[2] = {L.xa, L.xb};
  const PrepSet ys[2] = {ysB, ysA};
  const int64_t* const ydn[2] = {ydnB, ydnA};
  const int64_t ycap[2] = {ycapB, ycapA};
  uint32_t* const rmin[2] = {L.rowA, L.rowB};
  const int64_t cmax = std::max(capA, capB);
  // The rows the float64 pass re-measures (cand2 / count2 / best2 of each
  // direction): every row whose certified upper bound U of its true minimum
  // reaches the largest certified lower bound L of any row's true minimum
  // (the directed distance lies between the two).
  const int32_t* cand2[2] = {L.w[0].cand2, L.w[1].cand2};
  const int64_t* count2[2] = {L.w[0].count2, L.w[1].count2};
  unsigned long long* best2[2] = {L.w[0].best2, L.w[1].best2};
  // Seeds: the kSeedRows rows with the largest upper bounds (keys in
  // rmin[d]), searched against the whole inner set with the float32 tile
  // (whose error bound is tight in every precision form), raise the lower
  // bound; `zero` lists the counts the next append fills.
  auto seeds = [&](int64_t* const zero[2]) -> prohd_status {
    PROHD_TRY(top_rows2(mins2, caps2, dns2, L.w, L.top_ws, L.top_bytes, s, kSeedRows));
    BoundPair sp{};
    TileArgs ta[2];
    GatherPair gp{};
    gp.limit = kSeedRows;
    for (int d = 0; d < 2; ++d) {
      // the seed rows as the inner side of a tile whose outer side is the
      // whole inner set: their minima come out as column minima
      gp.j[d] = GatherJob{xs[d].p, xs[d].n, xs[d].q, xs[d].qn, L.w[d].cand, L.w[d].count, L.sh[d].p,
                          L.sh[d].n, L.sh[d].q, L.sh[d].qn, L.dshort + 2 * d, nullptr};
      ta[d] = TileArgs{ys[d], ydn[d], ycap[d], L.sh[d], L.dshort + 2 * d, kSeedRows, nullptr, L.rowS[d],
                       nullptr};
      sp.d[d] = BoundJob{L.rowS[d], xs[d].n, L.w[d].cand, L.w[d].count, kSeedRows, L.hlow + d, zero[d]};
    }
    PROHD_TRY(launch_gather_lists<DP>(FMT_F32, gp, s));
    PROHD_TRY(launch_tile_pair<DP>(FMT_F32, ta[0], ta[1], L.maxabs, s));
    return launch_bounds(sp, kSeedRows, DP, FMT_F32, L.maxabs, s);
  };
  int64_t* const zero2[2] = {L.w[0].count2, L.w[1].count2};
  if (L.nlev == 0) {
    // one search of every outer row against its whole inner set
    if (!full) {
      PROHD_TRY(launch_tile<DP>(fmt, L.xa, dnA, capA, L.xb, dnB, capB, L.maxabs, L.rowA, L.rowB, s));
    } else {
      PROHD_TRY(launch_tile<DP>(fmt, L.xa, dnA, capA, L.fb, nullptr, nB, L.maxabs, L.rowA, nullptr, s));
      PROHD_TRY(launch_tile<DP>(fmt, L.xb, dnB, capB, L.fa, nullptr, nA, L.maxabs, L.rowB, nullptr, s));
    }
    if (nn2A) PROHD_HIP(hipMemcpyAsync(nn2A, L.rowA, sizeof(float) * capA, hipMemcpyDeviceToDevice, s));
    if (nn2B) PROHD_HIP(hipMemcpyAsync(nn2B, L.rowB, sizeof(float) * capB, hipMemcpyDeviceToDevice, s));
    BoundPair bp{};
    AppendPair ap{};
    for (int d = 0; d < 2; ++d) {
      bp.d[d] = BoundJob{rmin[d], xs[d].n, nullptr, dns2[d], caps2[d], L.hlow + d, L.w[d].count2};
      ap.d[d] = AppendJob{rmin[d], nullptr, dns2[d], caps2[d], L.hlow + d, L.w[d].cand2, L.w[d].count2,
                          L.w[d].best2};
    }
    PROHD_TRY(launch_bounds(bp, cmax, DP, fmt, L.maxabs, s));
    // the low-precision forms' lower bounds are loose (e4m3 rounds to 4
    // significant bits): seeds tighten them
    if (fmt != FMT_F32) PROHD_TRY(seeds(zero2));
    PROHD_TRY(launch_append(ap, cmax, L.status, s));
  } else {
    // Pruned search.  A row's minimum over any subset of its inner set
    // bounds its minimum over the whole set from above, so U from a subset
    // search is still an upper bound; lower bounds come only from searches
    // over the whole inner set.  Level 1: every row against the coarsest
    // subset.
    for (int d = 0; d < 2; ++d)
      for (int j = 0; j < L.nlev; ++j)
        PROHD_TRY(launch_subset<DP>(fmt, ys[d], ydn[d], ycap[d], prune_stride(L.nlev, j), L.sub[d][j],
                                    L.dsub + d * kPruneMaxLevels + j, s));
    {
      TileArgs ta[2];
      for (int d = 0; d < 2; ++d)
        ta[d] = TileArgs{xs[d], dns2[d], caps2[d], L.sub[d][0], L.dsub + d * kPruneMaxLevels,
                         cdiv(ycap[d], prune_stride(L.nlev, 0)), rmin[d], nullptr, nullptr};
      PROHD_TRY(launch_tile_pair<DP>(fmt, ta[0], ta[1], L.maxabs, s));
    }
    BoundPair bp{};
    for (int d = 0; d < 2; ++d)
      bp.d[d] = BoundJob{rmin[d], xs[d].n, nullptr, dns2[d], caps2[d], nullptr, nullptr};
    PROHD_TRY(launch_bounds(bp, cmax, DP, fmt, L.maxabs, s));
    // the seeds give the first lower bound
    PROHD_TRY(seeds(zero2));
    AppendPair ap{};
    for (int d = 0; d < 2; ++d)
      ap.d[d] = AppendJob{rmin[d], nullptr, dns2[d], caps2[d], L.hlow + d, L.w[d].cand2, L.w[d].count2,
                          L.w[d].best2};
    PROHD_TRY(launch_append(ap, cmax, L.status, s));
    // finer levels: the listed rows against a 16 times larger subset, the
    // last against the whole inner set (which also raises the lower bound)
    for (int j = 1; j <= L.nlev; ++j) {
      const int b = (j - 1) & 1;   // list this level writes
      const bool last = j == L.nlev;
      const FillJob fr[2] = {{L.pw[0].rowF, caps2[0], kInfBits}, {L.pw[1].rowF, caps2[1], kInfBits}};
      PROHD_TRY(fill_words(fr, 2, s));
      if (!last) {
        TileArgs ta[2];
        for (int d = 0; d < 2; ++d)
          ta[d] = TileArgs{xs[d], count2[d], caps2[d], L.sub[d][j], L.dsub + d * kPruneMaxLevels + j,
                           cdiv(ycap[d], prune_stride(L.nlev, j)), L.pw[d].rowF, nullptr, cand2[d]};
        PROHD_TRY(launch_tile_pair<DP>(fmt, ta[0], ta[1], L.maxabs, s));
      } else {
        // against the whole inner set: a short list as the inner side of
        // a tile over the inner set, a long one as the outer side
        TileArgs tc[2], tr[2];
        GatherPair gp{};
        gp.limit = kShortList;
        for (int d = 0; d < 2; ++d) {
          int64_t* dsm = L.dshort + 2 * d;
          gp.j[d] = GatherJob{xs[d].p, xs[d].n, xs[d].q, xs[d].qn, cand2[d], count2[d], L.sh[d].p, L.sh[d].n,
                              L.sh[d].q, L.sh[d].qn, dsm, dsm + 1};
          tc[d] = TileArgs{ys[d], ydn[d], ycap[d], L.sh[d], dsm, kShortList, nullptr, L.pw[d].rowF, nullptr};
          tr[d] = TileArgs{xs[d], dsm + 1, caps2[d], ys[d], ydn[d], ycap[d], L.pw[d].rowF, nullptr, cand2[d]};
        }
        PROHD_TRY(launch_gather_lists<DP>(fmt, gp, s));
        PROHD_TRY(launch_tile_pair<DP>(fmt, tc[0], tc[1], L.maxabs, s));
        PROHD_TRY(launch_tile_pair<DP>(fmt, tr[0], tr[1], L.maxabs, s));
      }
      for (int d = 0; d < 2; ++d) {
        bp.d[d] = BoundJob{L.pw[d].rowF, xs[d].n, cand2[d], count2[d], caps2[d], last ? L.hlow + d : nullptr,
                           L.pw[d].count[b]};
        ap.d[d] = AppendJob{L.pw[d].rowF, cand2[d], count2[d], caps2[d], L.hlow + d, L.pw[d].cand[b],
                            L.pw[d].count[b], L.pw[d].best[b]};
      }
      PROHD_TRY(launch_bounds(bp, cmax, DP, fmt, L.maxabs, s));
      PROHD_TRY(launch_append(ap, cmax, L.status, s));
      for (int d = 0; d < 2; ++d) {
        cand2[d] = L.pw[d].cand[b];
        count2[d] = L.pw[d].count[b];
        best2[d] = L.pw[d].best[b];
      }
    }
  }
  {
    RefinePair rp{};
    rp.d[0] = RefineDir{L.xa.p, cand2[0], count2[0], ysB.p, ydnB, ycapB, best2[0]};
    rp.d[1] = RefineDir{L.xb.p, cand2[1], count2[1], ysA.p, ydnA, ycapA, best2[1]};
    PROHD_TRY(launch_refine_pair<DP>(rp, s));
  }
  const DirIn ab{nullptr, nullptr, nullptr, best2[0], cand2[0], count2[0], idxA, full ? nullptr : idxB, A, B};
  const DirIn ba{nullptr, nullptr, nullptr, best2[1], cand2[1], count2[1], idxB, full ? nullptr : idxA, B, A};
  PROHD_LAUNCH("hd_finalize", finalize, dim3(1), dim3(256), 0, s, ab, ba, D, dnA, capA, dnB, capB,
               L.status, out);
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

int fmt_of(uint32_t flags) {
  if (flags & PROHD_PREC_FP8) return FMT_FP8;
  if (flags & PROHD_PREC_BF16) return FMT_BF16;
  return FMT_F32;
}

}  // namespace

// Pruned search when asked for, on outer row lists large enough to profit
// (smaller ones: the unpruned search, same value); the inner sets are at
// least as large (the other list, or in inner-full mode the whole set).
bool use_prune(uint32_t flags, int64_t capA, int64_t capB) {
  return (flags & PROHD_PRUNE) && capA >= kPruneMinRows && capB >= kPruneMinRows;
}

int hd_prune_levels(int64_t capA, int64_t capB, int64_t nA, int64_t nB, uint32_t flags) {
  if (!use_prune(flags, capA, capB)) return 0;
  const bool full = (flags & PROHD_INNER_FULL) != 0;
  return prune_levels(std::min(full ? nB : capB, full ? nA : capA));
}

size_t hd_ws_bytes(int64_t nA, int64_t nB, int32_t D, int64_t capA, int64_t capB, bool full,
                   uint32_t flags) {
  Arena ar(nullptr);
  hd_layout(ar, capA, capB, nA, nB, pad_dim(D), full, fmt_of(flags), use_prune(flags, capA, capB));
  return ar.used + 256;
}

size_t exact_ws_bytes(int64_t nA, int64_t nB, int32_t D, uint32_t flags) {
  Arena ar(nullptr);
  hd_layout(ar, nA, nB, nA, nB, pad_dim(D), false, fmt_of(flags), use_prune(flags, nA, nB));
  return ar.used + 256;
}

prohd_status hd_candidates(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                           const int32_t* idxA, const int64_t* dnA, int64_t capA,
                           const int32_t* idxB, const int64_t* dnB, int64_t capB, uint32_t flags,
                           prohd_result* out, void* ws, size_t ws_bytes, hipStream_t s) {
  const bool full = (flags & PROHD_INNER_FULL) != 0;
  const int fmt = fmt_of(flags);
  const bool prune = use_prune(flags, capA, capB);
  return by_dp(D, [&](auto dp) {
    return run_hd<decltype(dp)::value>(A, nA, B, nB, D, idxA, dnA, capA, idxB, dnB, capB, full, fmt,
                                       prune, out, nullptr, nullptr, ws, ws_bytes, s);
  });
}

prohd_status hd_exact(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      uint32_t flags, prohd_result* out, float* nn2A, float* nn2B, void* ws,
                      size_t ws_bytes, hipStream_t s) {
  const int fmt = fmt_of(flags);
  // the per-row minima asked for (nn2) come from the full search
  const bool prune = !nn2A && !nn2B && use_prune(flags, nA, nB);
  return by_dp(D, [&](auto dp) {
    return run_hd<decltype(dp)::value>(A, nA, B, nB, D, nullptr, nullptr, nA, nullptr, nullptr, nB,
                                       false, fmt, prune, out, nn2A, nn2B, ws, ws_bytes, s);
  });
}

template <class F>
prohd_status by_dp_batch(int DP, F&& f) {
  switch (DP) {
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    default: return fail(PROHD_EUNSUPPORTED, "batched: unsupported padded dimension");
  }
}

prohd_status batch_prep(int DP, int D, const PrepJob* jobs, const BItem* items, int nitems, int grid,
                        hipStream_t s) {
  if (nitems <= 0) return PROHD_OK;
  return by_dp_batch(DP, [&](auto dp) {
    PROHD_LAUNCH("batch_prep", prep_batch<decltype(dp)::value>, dim3(grid), dim3(256), 0, s, jobs, D,
                 items, nitems);
    return PROHD_OK;
  });
}

prohd_status batch_tile(int DP, const TileJob* jobs, const BItem* items, int nitems, int grid,
                        hipStream_t s) {
  if (nitems <= 0) return PROHD_OK;
  return by_dp_batch(DP, [&](auto dp) {
    PROHD_LAUNCH("batch_tile", tile_batch<decltype(dp)::value>, dim3(grid), dim3(512), 0, s, jobs,
                 items, nitems);
    return PROHD_OK;
  });
}

prohd_status batch_keys(int DP, const KeyJob* jobs, const BItem* items, int nitems, int grid,
                        hipStream_t s) {
  if (nitems <= 0) return PROHD_OK;
  PROHD_LAUNCH("batch_keys", keys_batch, dim3(grid), dim3(256), 0, s, jobs, DP, items, nitems);
  return PROHD_OK;
}

prohd_status batch_uncertain(const UncJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  const int grid = std::min(njobs, 8 * cu_count());
  PROHD_LAUNCH("batch_uncertain", uncertain_batch, dim3(grid), dim3(kUncBatchT), 0, s, jobs, njobs);
  return PROHD_OK;
}

prohd_status batch_refine_dyn(int DP, const RefineJob* jobs, const BItem* items, int nitems, int grid,
                              hipStream_t s) {
  if (nitems <= 0) return PROHD_OK;
  return by_dp_batch(DP, [&](auto dp) {
    PROHD_LAUNCH("batch_refine2", refine_dyn_batch<decltype(dp)::value>, dim3(grid), dim3(256), 0, s,
                 jobs, items, nitems);
    return PROHD_OK;
  });
}

prohd_status batch_finalize(const FinalJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  const int grid = std::min(njobs, 4 * cu_count());
  PROHD_LAUNCH("batch_finalize", finalize_batch, dim3(grid), dim3(256), 0, s, jobs, njobs);
  return PROHD_OK;
}

prohd_status batch_fill32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return PROHD_OK;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 4096));
  PROHD_LAUNCH("batch_fill", fill_u32, dim3(grid), dim3(256), 0, s, p, n, v);
  return PROHD_OK;
}

prohd_status batch_fill64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return PROHD_OK;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 4096));
  PROHD_LAUNCH("batch_fill", fill_u64, dim3(grid), dim3(256), 0, s, p, n, v);
  return PROHD_OK;
}

}  // namespace prohd
