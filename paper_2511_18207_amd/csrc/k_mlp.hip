// Learned candidate proposal: a scorer MLP 2D -> 256 -> 128 -> 1 (GELU,
// bfloat16 weights and activations into the matrix cores, float32
// accumulation and master weights) over the per-point features
// f = [x, x - c_other], with its own forward, backward and AdamW kernels.
//
// This extends the paper's candidate selection (the per-direction extremes
// of Alg. 1 / Alg. 2): the highest-scoring points of each set are added to
// the selected rows before the candidate distance is taken.
//
// Flat float32 parameter layout: [W1 (256 x 2D), b1 (256), W2 (128 x 256),
// b2 (128), w3 (128), b3 (1)].
//
// One general bfloat16 GEMM (64 x 64 output tile per 4-wave work-group,
// v_mfma_f32_32x32x16_bf16, K staged through LDS 32 at a time, operands at
// arbitrary strides) serves every product; epilogues add the bias and GELU
// (forward), multiply by GELU' (backward through an activation) or store the
// float32 sums (weight gradients).

#include <math.h>

#include "common.h"

namespace prohd {
namespace {

constexpr int kH1 = 256;
constexpr int kH2 = 128;
constexpr int kHeadPart = kH2 + 2;             // head partial: gw3, gb3, loss
constexpr int64_t kPartFloats = 4 << 20;       // split-K / column-sum partials (16 MiB)

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum { EPI_F32 = 0, EPI_BIAS_GELU = 1, EPI_GELU_BWD = 2 };

struct GemmArgs {
  const __bf16* A;
  int64_t lam, lak;   // A(m, k) = A[m lam + k lak]
  const __bf16* B;
  int64_t lbk, lbn;   // B(k, n) = B[k lbk + n lbn]
  int M, N, K;
  int64_t ldc;
  float* outf;        // EPI_F32: sums; EPI_BIAS_GELU: pre-activation z (may be null)
  __bf16* outh;       // EPI_BIAS_GELU: gelu(z); EPI_GELU_BWD: acc * gelu'(zin)
  const float* bias;  // EPI_BIAS_GELU
  const float* zin;   // EPI_GELU_BWD: pre-activation, same layout as the output
  int kper;           // K range of split z = blockIdx.z: [z kper, (z + 1) kper)
  float* part;        // EPI_F32 with several splits: partial sums [z][M][N]
  int amode, bmode;   // operand staging: 0 scalar, 1 K-contiguous, 2 M/N-contiguous
};

// Stage the 64 x 32 tile X(r0 + r, k0 + k) = P[r lr + k lk] into S[r][k]
// (row stride ST).  Full tiles of a vector-friendly operand move 8 values
// per thread in one 16-byte load; edge tiles and other layouts go element by
// element with zero fill.
template <int ST>
__device__ __forceinline__ void stage(const __bf16* __restrict__ P, int64_t lr, int64_t lk, int R,
                                      int kend, int r0, int k0, int mode, __bf16* __restrict__ S,
                                      int tid) {
  const bool full = (r0 + 64 <= R) && (k0 + 32 <= kend);
  if (full && mode == 1) {
    const int r = tid >> 2, kk = (tid & 3) * 8;
    *reinterpret_cast<bf16x8*>(&S[r * ST + kk]) =
        *reinterpret_cast<const bf16x8*>(&P[(int64_t)(r0 + r) * lr + (k0 + kk)]);
  } else if (full && mode == 2) {
    const int kk = tid >> 3, rr = (tid & 7) * 8;
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(&P[(r0 + rr) + (int64_t)(k0 + kk) * lk]);
#pragma unroll
    for (int j = 0; j < 8; ++j) S[(rr + j) * ST + kk] = v[j];
  } else {
    const int r = tid >> 2, kk = (tid & 3) * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + kk + j;
      S[r * ST + kk + j] = (r0 + r < R && k < kend) ? P[(int64_t)(r0 + r) * lr + (int64_t)k * lk] : (__bf16)0.f;
    }
  }
}

template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16(GemmArgs g) {
  constexpr int KC = 32;
  constexpr int ST = KC + 8;   // LDS row stride (bf16): 80 bytes, 16-byte aligned rows
  __shared__ __attribute__((aligned(16))) __bf16 As[64 * ST];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[64 * ST];   // n-major: Bs[n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = 32 * (wave >> 1), wn = 32 * (wave & 1);
  const int gsel = lane >> 5, c = lane & 31;
  floatx16 acc = {0.f};
  // staging: thread -> (row r = tid / 4, k group of 8 = (tid % 4) * 8)
  const int kbeg = blockIdx.z * g.kper;
  const int kend = min(g.K, kbeg + g.kper);
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    __syncthreads();
    stage<ST>(g.A, g.lam, g.lak, g.M, kend, m0, k0, g.amode, As, tid);
    stage<ST>(g.B, g.lbn, g.lbk, g.N, kend, n0, k0, g.bmode, Bs, tid);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[(wm + c) * ST + 16 * s + 8 * gsel]);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[(wn + c) * ST + 16 * s + 8 * gsel]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
  }
  // lane holds column wn + c, rows wm + 8 (v/4) + 4 gsel + v%4
  const int n = n0 + wn + c;
  if (n >= g.N) return;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm + 8 * (v >> 2) + 4 * gsel + (v & 3);
    if (m >= g.M) continue;
    const int64_t o = (int64_t)m * g.ldc + n;
    if (EPI == EPI_F32) {
      if (g.part)
        g.part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = acc[v];
      else
        g.outf[o] = acc[v];
    } else if (EPI == EPI_BIAS_GELU) {
      const float z = acc[v] + g.bias[n];
      if (g.outf) g.outf[o] = z;
      g.outh[o] = (__bf16)gelu(z);
    } else {
      g.outh[o] = (__bf16)(acc[v] * gelu_grad(g.zin[o]));
    }
  }
}

// F[i] = [x, x - c] of row idx[i] (or i), bfloat16, 2D per row.
__global__ void features(const float* __restrict__ X, int D, const int32_t* __restrict__ idx,
                         int64_t n, const float* __restrict__ c, __bf16* __restrict__ F) {
  const int64_t total = n * 2 * D;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / (2 * D);
    const int k = (int)(e - i * 2 * D);
    const int64_t r = idx ? (int64_t)idx[i] : i;
    const float v = k < D ? X[r * D + k] : X[r * D + (k - D)] - c[k - D];
    F[e] = (__bf16)v;
  }
}

// ------------------------------------------------------- fused scoring
// Scores only (no gradients): the feature layer folded,
//   W1 [x; x - c] + b1 = (W1a + W1b) x + (b1 - W1b c),
// W1a / W1b the halves of W1 acting on x and on x - c (fold_w1, once per
// call: W1f = bf16(W1a + W1b) padded to KD columns, b1f = b1 - W1b c in
// float64), then one launch over 64-row tiles: the tile's rows are read once
// (float32 -> bfloat16 into LDS), layer 1 (64 x KD times KD x 256) and
// layer 2 (64 x 256 times 256 x 128) run on v_mfma_f32_32x32x16_bf16 with
// the weights read from L2 (192 KiB at D = 256, shared by every tile), the
// GELU activations stay in LDS, and the head w3 . h2 + b3 is reduced in
// registers.  The GELU's erf is the rational approximation 7.1.26 of
// Abramowitz and Stegun (Handbook of Mathematical Functions, absolute error
// below 1.5e-7), far below the bfloat16 rounding (2^-9) of the activations.

// GELU(z) = z Phi(z) = max(z, 0) - |z| erfc(|z| / sqrt 2) / 2, with
// erfc(a) = t P(t) e^{-a^2}, t = 1 / (1 + p a) for a >= 0 (7.1.26); the
// halving and 1 / sqrt 2 are folded into the constants, e^{-a^2} is
// exp2(-z^2 log2(e) / 2).
__device__ __forceinline__ float gelu_fast(float z) {
  const float az = fabsf(z);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, az, 1.f));   // 1 ulp
  float p = 0.5f * 1.061405429f;
  p = fmaf(p, t, 0.5f * -1.453152027f);
  p = fmaf(p, t, 0.5f * 1.421413741f);
  p = fmaf(p, t, 0.5f * -0.284496736f);
  p = fmaf(p, t, 0.5f * 0.254829592f);
  const float e = __builtin_amdgcn_exp2f(z * z * -0.72134752044448170f);   // e^{-z^2 / 2}
  return fmaf(-az * (p * t), e, fmaxf(z, 0.f));
}

constexpr int kScoreRows = 64;   // rows per scoring tile

// Weight operands in load order.  Wave w of the scoring kernel reads, for
// product step s, the 8 values k = 16 s + 8 g .. + 7 of unit 32 b + c in
// lane (c, g) (b = the wave's 32-unit block); stored at
// ((b KS + s) 64 + 32 g + c) 8, one load instruction of a wave reads 1 KiB
// of contiguous memory (8 cache lines instead of 32).  KS = K / 16.
__device__ __forceinline__ int64_t opnd_index(int j, int k, int KS) {
  const int b = j >> 5, c = j & 31, s = k >> 4, g = (k >> 3) & 1, e = k & 7;
  return ((((int64_t)b * KS + s) * 64 + 32 * g + c) << 3) + e;
}

// W1f (operand order) of bf16(W1[j][k] + W1[j][D + k]) for k < D, 0 up to
// KD; b1f[j] = b1[j] - sum_k W1[j][D + k] c[k] (float64 sum).  Block j =
// unit j.
__global__ __launch_bounds__(256) void fold_w1(const float* __restrict__ W1, const float* __restrict__ b1,
                                               int D, int KD, const float* __restrict__ c,
                                               __bf16* __restrict__ W1f, float* __restrict__ b1f) {
  __shared__ double red[256];
  const int j = blockIdx.x, tid = threadIdx.x;
  const float* w = W1 + (int64_t)j * 2 * D;
  double acc = 0.0;
  for (int k = tid; k < KD; k += 256) {
    W1f[opnd_index(j, k, KD / 16)] = k < D ? (__bf16)(w[k] + w[D + k]) : (__bf16)0.f;
    if (k < D) acc += (double)w[D + k] * (double)c[k];
  }
  red[tid] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) b1f[j] = (float)((double)b1[j] - red[0]);
}

// W2 (128 x 256, float32) -> bfloat16 in operand order.
__global__ __launch_bounds__(256) void w2_operands(const float* __restrict__ W2, __bf16* __restrict__ W2o) {
  const int j = blockIdx.x;
  for (int k = threadIdx.x; k < kH1; k += 256) W2o[opnd_index(j, k, kH1 / 16)] = (__bf16)W2[j * kH1 + k];
}

// One 64-row tile per work-group of 8 waves; the rows (bfloat16, stride
// KD + 8) and then the layer-1 activations (stride 264) share one LDS
// buffer, so three work-groups fit on a compute unit.  VEC: rows read as
// float4 (D a multiple of 4, 16-byte aligned X).
constexpr int kScoreT = 512;

template <int KD, bool VEC>
__global__ __launch_bounds__(kScoreT, 3) void score_fused(const float* __restrict__ X, int64_t n, int D,
                                                          const __bf16* __restrict__ W1f,   // operand order
                                                          const float* __restrict__ b1f,
                                                          const __bf16* __restrict__ W2b,   // operand order
                                                          const float* __restrict__ b2,
                                                          const float* __restrict__ w3,
                                                          const float* __restrict__ b3,
                                                          float* __restrict__ scores) {
  constexpr int R = kScoreRows;
  constexpr int NT = kScoreT;
  constexpr int STX = KD + 8;    // bfloat16 row strides: 16-byte aligned rows
  constexpr int STH = kH1 + 8;
  __shared__ __attribute__((aligned(16))) __bf16 buf[R * STH];
  __shared__ float rs[R][4];
  __bf16* const Xs = buf;
  __bf16* const Hs = buf;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, g = lane >> 5, c = lane & 31;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  // stage the tile's rows as bfloat16 (rows past n and columns past D are
  // 0); all of a thread's loads are issued before the first conversion
  if constexpr (VEC) {
    constexpr int NL = (R * (KD / 4) + NT - 1) / NT;   // float4 loads per thread
    float4 v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + NT * q;
      const int r = e / (KD / 4), k = 4 * (e - r * (KD / 4));
      v[q] = (e < R * (KD / 4) && r0 + r < n && k < D)
                 ? *reinterpret_cast<const float4*>(X + (r0 + r) * D + k)
                 : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + NT * q;
      if (e < R * (KD / 4)) {
        const int r = e / (KD / 4), k = 4 * (e - r * (KD / 4));
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        const bf16x4 q4 = {(__bf16)v[q].x, (__bf16)v[q].y, (__bf16)v[q].z, (__bf16)v[q].w};
        *reinterpret_cast<bf16x4*>(&Xs[r * STX + k]) = q4;   // one 8-byte store
      }
    }
  } else {
    constexpr int NL = (R * KD + NT - 1) / NT;         // elements per thread
    float v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + NT * q;
      const int r = e / KD, k = e - r * KD;
      v[q] = (e < R * KD && r0 + r < n && k < D) ? X[(r0 + r) * D + k] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + NT * q;
      if (e < R * KD) Xs[(e / KD) * STX + (e % KD)] = (__bf16)v[q];
    }
  }
  __syncthreads();
  // layer 1: wave w owns units [32 w, 32 w + 32) for all 64 rows; its
  // weight operands for the whole K range are loaded before the first
  // product (one L2 latency per tile)
  {
    floatx16 acc0 = {0.f}, acc1 = {0.f};
    const __bf16* wb = W1f + ((int64_t)w * (KD / 16) * 64 + lane) * 8;
    bf16x8 Bw[KD / 16];
#pragma unroll
    for (int s = 0; s < KD / 16; ++s) Bw[s] = *reinterpret_cast<const bf16x8*>(wb + 512 * s);
#pragma unroll
    for (int s = 0; s < KD / 16; ++s) {
      const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&Xs[c * STX + 16 * s + 8 * g]);
      const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&Xs[(32 + c) * STX + 16 * s + 8 * g]);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, Bw[s], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, Bw[s], acc1, 0, 0, 0);
    }
    __syncthreads();   // every wave's reads of the rows are done: Hs replaces them
    // lane holds unit 32 w + c, rows 32 i + 8 (v / 4) + 4 g + v % 4
    const int u = 32 * w + c;
    const float bu = b1f[u];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = 8 * (q >> 2) + 4 * g + (q & 3);
      Hs[r * STH + u] = (__bf16)gelu_fast(acc0[q] + bu);
      Hs[(32 + r) * STH + u] = (__bf16)gelu_fast(acc1[q] + bu);
    }
  }
  __syncthreads();
  // layer 2: wave w owns units [32 (w % 4), +32) for rows [32 (w / 4), +32);
  // the head then sums gelu(z2) w3 over those 32 units per row
  const int cb = w & 3, rb = w >> 2;
  floatx16 acc2 = {0.f};
  const __bf16* wb = W2b + ((int64_t)cb * (kH1 / 16) * 64 + lane) * 8;
  bf16x8 B2[kH1 / 16];
#pragma unroll
  for (int s = 0; s < kH1 / 16; ++s) B2[s] = *reinterpret_cast<const bf16x8*>(wb + 512 * s);
#pragma unroll
  for (int s = 0; s < kH1 / 16; ++s) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(&Hs[(32 * rb + c) * STH + 16 * s + 8 * g]);
    acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, B2[s], acc2, 0, 0, 0);
  }
  const int u = 32 * cb + c;
  const float bu = b2[u], wu = w3[u];
  float h[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) h[q] = gelu_fast(acc2[q] + bu) * wu;
  // butterfly over the 32 lanes of the half-wave: after the step with
  // offset o a lane keeps the half of its list selected by bit o of c, so
  // lane c (c < 16 after four steps; the offset-16 step then adds the two
  // copies) ends with the 32-lane sum of entry c % 16, row 32 rb +
  // 8 ((c % 16) / 4) + 4 g + c % 4.  The choice between the halves is a bit
  // mask, not a select of array entries, which the compiler would turn into
  // a run-time index into the whole register array.
#pragma unroll
  for (int o = 8, len = 16; o >= 1; o >>= 1, len >>= 1) {
    const uint32_t m = (c & o) ? 0xffffffffu : 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < len / 2) {
        const uint32_t lo = __float_as_uint(h[q]), up = __float_as_uint(h[q + len / 2]);
        const uint32_t d = (lo ^ up) & m;
        const float keep = __uint_as_float(lo ^ d);   // up when the bit is set
        const float send = __uint_as_float(up ^ d);   // lo when the bit is set
        h[q] = keep + __shfl_xor(send, o);
      }
    }
  }
  const float tot = h[0] + __shfl_xor(h[0], 16);
  if (c < 16) rs[32 * rb + 8 * (c >> 2) + 4 * g + (c & 3)][cb] = tot;
  __syncthreads();
  if (tid < R && r0 + tid < n)
    scores[r0 + tid] = ((rs[tid][0] + rs[tid][1]) + (rs[tid][2] + rs[tid][3])) + b3[0];
}

// s[i] = w3 . h2[i] + b3 (one wave per row).
__global__ void head_fwd(const __bf16* __restrict__ H2, int64_t n, const float* __restrict__ w3,
                         const float* __restrict__ b3, float* __restrict__ s) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); i < n;
       i += (int64_t)gridDim.x * (blockDim.x / 64)) {
    float a = (float)H2[i * kH2 + lane] * w3[lane] + (float)H2[i * kH2 + 64 + lane] * w3[64 + lane];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if (lane == 0) s[i] = a + b3[0];
  }
}

// Loss and the gradient at the head: ds = (pw y (sig - 1) + (1 - y) sig) / n,
// dZ2 = ds w3 * gelu'(z2), grads of w3 and b3, summed loss.  A work-group
// of 256 threads handles 64 rows; thread j < 128 owns hidden unit j.
__global__ __launch_bounds__(256) void head_bwd(const __bf16* __restrict__ H2,
                                                const float* __restrict__ Z2,
                                                const float* __restrict__ s,
                                                const float* __restrict__ labels,
                                                const int32_t* __restrict__ idx, int64_t n,
                                                float pos_weight, const float* __restrict__ w3,
                                                __bf16* __restrict__ dZ2, float* __restrict__ part) {
  __shared__ float dsv[64];
  __shared__ float lsum[64];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int64_t i = r0 + tid;
    float ds = 0.f, l = 0.f;
    if (i < n) {
      const float y = labels[idx ? idx[i] : i];
      const float sv = s[i];
      const float sig = 1.f / (1.f + expf(-sv));
      // softplus(-s) and softplus(s), stable
      const float spn = fmaxf(-sv, 0.f) + log1pf(expf(-fabsf(sv)));
      const float spp = fmaxf(sv, 0.f) + log1pf(expf(-fabsf(sv)));
      l = pos_weight * y * spn + (1.f - y) * spp;
      ds = (pos_weight * y * (sig - 1.f) + (1.f - y) * sig) / (float)n;
    }
    dsv[tid] = ds;
    lsum[tid] = l;
  }
  __syncthreads();
  const int j = tid & 127, half = tid >> 7;
  float g = 0.f;
  for (int rr = half; rr < 64; rr += 2) {
    const int64_t i = r0 + rr;
    if (i >= n) break;
    const float ds = dsv[rr];
    g += ds * (float)H2[i * kH2 + j];
    dZ2[i * kH2 + j] = (__bf16)(ds * w3[j] * gelu_grad(Z2[i * kH2 + j]));
  }
  // per-block partials [130]: gw3 (128), gb3, loss; halves combine in LDS
  __shared__ float gsum[256];
  gsum[tid] = g;
  __syncthreads();
  float* pp = part + (size_t)blockIdx.x * kHeadPart;
  if (tid < 128) pp[tid] = gsum[tid] + gsum[tid + 128];
  if (tid == 0) {
    float a = 0.f, b = 0.f;
    for (int rr = 0; rr < 64; ++rr) {
      a += dsv[rr];
      b += lsum[rr];
    }
    pp[128] = a;
    pp[129] = b / (float)n;
  }
}

// Sums of the head partials over blocks, in block order.
__global__ void head_reduce(const float* __restrict__ part, int nblk, float* __restrict__ gw3,
                            float* __restrict__ gb3, float* __restrict__ loss) {
  const int j = threadIdx.x;
  if (j >= kHeadPart) return;
  float a = 0.f;
  for (int b = 0; b < nblk; ++b) a += part[(size_t)b * kHeadPart + j];
  if (j < 128) gw3[j] = a;
  else if (j == 128) gb3[0] = a;
  else loss[0] = a;
}

// out[m ldc + n] = sum over z of part[z][m][n] (split order, deterministic).
__global__ void split_reduce(const float* __restrict__ part, int splits, int M, int N,
                             float* __restrict__ out, int64_t ldc) {
  const int64_t MN = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < MN;
       e += (int64_t)gridDim.x * blockDim.x) {
    float a = 0.f;
    for (int z = 0; z < splits; ++z) a += part[(int64_t)z * MN + e];
    out[(e / N) * ldc + (e % N)] = a;
  }
}

// Partial column sums of a bfloat16 matrix (n x N, N <= 256): block g sums
// rows [256 g, 256 g + 256) into part[g][N].
__global__ void colsum_part(const __bf16* __restrict__ M, int64_t n, int N, float* __restrict__ part) {
  const int j = threadIdx.x;
  if (j >= N) return;
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int64_t r1 = r0 + 256 < n ? r0 + 256 : n;
  float a = 0.f;
  for (int64_t i = r0; i < r1; ++i) a += (float)M[i * N + j];
  part[(size_t)blockIdx.x * N + j] = a;
}

// bfloat16 copies of W1 and W2 from the float32 master.
__global__ void to_bf16(const float* __restrict__ src, int64_t n, __bf16* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (__bf16)src[e];
}

__global__ void adamw_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, int64_t n, float lr, float wd, float b1, float b2,
                             float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float mh = me / c1, vh = ve / c2;
    p[e] -= lr * (mh / (sqrtf(vh) + eps) + wd * p[e]);
  }
}

// Deterministic initialisation: U(-a, a) with a = sqrt(6 / (fan_in + fan_out))
// for the weight matrices (counter-based hash of (seed, index)); biases 0.
__device__ __forceinline__ float hash_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed * 0x9E3779B97F4A7C15ull + i * 0xBF58476D1CE4E5B9ull + 0x94D049BB133111EBull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (float)((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f;
}

__global__ void init_params(float* __restrict__ p, int D, uint64_t seed) {
  const int64_t F = 2 * D;
  const int64_t oW1 = 0, ob1 = kH1 * F, oW2 = ob1 + kH1, ob2 = oW2 + kH2 * kH1, ow3 = ob2 + kH2,
                ob3 = ow3 + kH2, total = ob3 + 1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    float a = 0.f;
    if (e < ob1) a = sqrtf(6.f / (float)(F + kH1));
    else if (e >= oW2 && e < ob2) a = sqrtf(6.f / (float)(kH1 + kH2));
    else if (e >= ow3 && e < ob3) a = sqrtf(6.f / (float)(kH2 + 1));
    p[e] = a * hash_uniform(seed, (uint64_t)e);
  }
}

struct Layout {
  int64_t F, oW1, ob1, oW2, ob2, ow3, ob3, total;
};

Layout layout(int D) {
  Layout L;
  L.F = 2 * D;
  L.oW1 = 0;
  L.ob1 = kH1 * L.F;
  L.oW2 = L.ob1 + kH1;
  L.ob2 = L.oW2 + (int64_t)kH2 * kH1;
  L.ow3 = L.ob2 + kH2;
  L.ob3 = L.ow3 + kH2;
  L.total = L.ob3 + 1;
  return L;
}

struct MlpWs {
  __bf16* Fb;    // chunk x 2D
  float* Z1;     // chunk x 256
  __bf16* H1;
  float* Z2;     // chunk x 128
  __bf16* H2;
  __bf16* dZ2;
  __bf16* dZ1;
  __bf16* W1b;
  __bf16* W2b;
  __bf16* W1f;   // folded layer 1 (scoring): 256 x 256 at most
  float* b1f;
  float* s;      // chunk
  float* part;   // split-K, column-sum and head partials
};

constexpr int64_t kChunk = 65536;   // rows per forward chunk

MlpWs mlp_layout(Arena& ar, int64_t rows, int D) {
  MlpWs W;
  W.Fb = ar.take<__bf16>((size_t)rows * 2 * D);
  W.Z1 = ar.take<float>((size_t)rows * kH1);
  W.H1 = ar.take<__bf16>((size_t)rows * kH1);
  W.Z2 = ar.take<float>((size_t)rows * kH2);
  W.H2 = ar.take<__bf16>((size_t)rows * kH2);
  W.dZ2 = ar.take<__bf16>((size_t)rows * kH2);
  W.dZ1 = ar.take<__bf16>((size_t)rows * kH1);
  W.W1b = ar.take<__bf16>((size_t)kH1 * 2 * D);
  W.W2b = ar.take<__bf16>((size_t)kH2 * kH1);
  W.W1f = ar.take<__bf16>((size_t)kH1 * 256);
  W.b1f = ar.take<float>(kH1);
  W.s = ar.take<float>(rows);
  W.part = ar.take<float>((size_t)kPartFloats);
  return W;
}

int vec_mode(const __bf16* P, int64_t lr, int64_t lk) {
  if (((uintptr_t)P & 15) != 0) return 0;
  if (lk == 1 && lr % 8 == 0) return 1;
  if (lr == 1 && lk % 8 == 0) return 2;
  return 0;
}

// Launches one product.  With `part` (EPI_F32 only) a long K is split over
// blockIdx.z so that the grid has ~2048 work-groups; the partial sums are
// then added in split order.
template <int EPI>
prohd_status gemm(GemmArgs g, hipStream_t s, float* part = nullptr) {
  g.amode = vec_mode(g.A, g.lam, g.lak);
  g.bmode = vec_mode(g.B, g.lbn, g.lbk);
  const int64_t tiles = cdiv(g.N, 64) * cdiv(g.M, 64);
  int64_t splits = 1;
  if (EPI == EPI_F32 && part) {
    splits = std::min<int64_t>(cdiv(g.K, 128), cdiv(2048, tiles));
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, kPartFloats / ((int64_t)g.M * g.N)));
  }
  g.kper = (int)(cdiv(cdiv(g.K, splits), 32) * 32);
  splits = std::max<int64_t>(1, cdiv(g.K, g.kper));
  g.part = splits > 1 ? part : nullptr;
  const dim3 grid((unsigned)cdiv(g.N, 64), (unsigned)cdiv(g.M, 64), (unsigned)splits);
  PROHD_LAUNCH("mlp_gemm", gemm_bf16<EPI>, grid, dim3(256), 0, s, g);
  if (splits > 1) {
    const int64_t MN = (int64_t)g.M * g.N;
    PROHD_LAUNCH("mlp_split_reduce", split_reduce, dim3((unsigned)std::min<int64_t>(cdiv(MN, 256), 1024)),
                 dim3(256), 0, s, (const float*)part, (int)splits, g.M, g.N, g.outf, g.ldc);
  }
  return PROHD_OK;
}

prohd_status colsum(const __bf16* M, int64_t n, int N, float* out, float* part, hipStream_t s) {
  const int nblk = (int)cdiv(n, 256);
  PROHD_LAUNCH("mlp_colsum", colsum_part, dim3(nblk), dim3(256), 0, s, M, n, N, part);
  PROHD_LAUNCH("mlp_split_reduce", split_reduce, dim3(1), dim3(256), 0, s, (const float*)part, nblk, 1,
               N, out, (int64_t)N);
  return PROHD_OK;
}

#define MLP_TRY(x)                   \
  do {                               \
    prohd_status st_ = (x);          \
    if (st_ != PROHD_OK) return st_; \
  } while (0)

// Forward over rows [0, n) of a chunk (features already in W.Fb).
prohd_status forward(const MlpWs& W, int64_t n, int D, const float* params, hipStream_t s) {
  const Layout L = layout(D);
  GemmArgs g1{W.Fb, L.F, 1, W.W1b, 1, L.F, (int)n, kH1, (int)L.F, kH1, W.Z1, W.H1, params + L.ob1, nullptr};
  MLP_TRY(gemm<EPI_BIAS_GELU>(g1, s));
  GemmArgs g2{W.H1, kH1, 1, W.W2b, 1, kH1, (int)n, kH2, kH1, kH2, W.Z2, W.H2, params + L.ob2, nullptr};
  MLP_TRY(gemm<EPI_BIAS_GELU>(g2, s));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 4), 4096));
  PROHD_LAUNCH("mlp_head", head_fwd, dim3(grid), dim3(256), 0, s, W.H2, n, params + L.ow3,
               params + L.ob3, W.s);
  return PROHD_OK;
}

prohd_status weights_bf16(const MlpWs& W, int D, const float* params, hipStream_t s) {
  const Layout L = layout(D);
  PROHD_LAUNCH("mlp_cvt", to_bf16, dim3(256), dim3(256), 0, s, params + L.oW1, (int64_t)kH1 * L.F, W.W1b);
  PROHD_LAUNCH("mlp_cvt", to_bf16, dim3(128), dim3(256), 0, s, params + L.oW2, (int64_t)kH2 * kH1, W.W2b);
  return PROHD_OK;
}

}  // namespace

size_t mlp_param_count(int32_t D) { return (size_t)layout(D).total; }

size_t mlp_ws_bytes(int64_t rows, int32_t D) {
  Arena ar(nullptr);
  mlp_layout(ar, std::min<int64_t>(std::max<int64_t>(rows, 1), kChunk), D);
  return ar.used + 256;
}

prohd_status mlp_init(float* params, int32_t D, uint64_t seed, hipStream_t s) {
  PROHD_LAUNCH("mlp_init", init_params, dim3(256), dim3(256), 0, s, params, D, seed);
  return PROHD_OK;
}

template <int KD>
prohd_status launch_score(const float* X, int64_t n, int D, const MlpWs& W, const float* params,
                          float* scores, hipStream_t s) {
  const Layout L = layout(D);
  const dim3 grid((unsigned)cdiv(n, kScoreRows));
  if (D % 4 == 0 && ((uintptr_t)X & 15) == 0) {
    PROHD_LAUNCH("mlp_score", (score_fused<KD, true>), grid, dim3(kScoreT), 0, s, X, n, D, W.W1f, W.b1f,
                 W.W2b, params + L.ob2, params + L.ow3, params + L.ob3, scores);
  } else {
    PROHD_LAUNCH("mlp_score", (score_fused<KD, false>), grid, dim3(kScoreT), 0, s, X, n, D, W.W1f, W.b1f,
                 W.W2b, params + L.ob2, params + L.ow3, params + L.ob3, scores);
  }
  return PROHD_OK;
}

prohd_status mlp_score(const float* X, int64_t n, int32_t D, const float* c_other,
                       const float* params, float* scores, void* ws, size_t ws_bytes,
                       hipStream_t s) {
  Arena ar(ws);
  MlpWs W = mlp_layout(ar, std::min<int64_t>(n, kChunk), D);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "mlp: workspace too small");
  const Layout L = layout(D);
  const int KD = pad_dim(D);
  PROHD_LAUNCH("mlp_fold", fold_w1, dim3(kH1), dim3(256), 0, s, params + L.oW1, params + L.ob1, D, KD,
               c_other, W.W1f, W.b1f);
  PROHD_LAUNCH("mlp_cvt", w2_operands, dim3(kH2), dim3(256), 0, s, params + L.oW2, W.W2b);
  switch (KD) {
    case 16: return launch_score<16>(X, n, D, W, params, scores, s);
    case 32: return launch_score<32>(X, n, D, W, params, scores, s);
    case 64: return launch_score<64>(X, n, D, W, params, scores, s);
    case 128: return launch_score<128>(X, n, D, W, params, scores, s);
    default: return launch_score<256>(X, n, D, W, params, scores, s);
  }
}

prohd_status mlp_grad(const float* X, int32_t D, const float* c_other, const float* labels,
                      const int32_t* idx, int64_t batch, float pos_weight, const float* params,
                      float* grad, float* loss, void* ws, size_t ws_bytes, hipStream_t s) {
  const Layout L = layout(D);
  if (batch > kChunk) return fail(PROHD_EINVAL, "mlp: batch exceeds 65536 rows");
  Arena ar(ws);
  MlpWs W = mlp_layout(ar, batch, D);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "mlp: workspace too small");
  MLP_TRY(weights_bf16(W, D, params, s));
  PROHD_LAUNCH("mlp_features", features, dim3(2048), dim3(256), 0, s, X, D, idx, batch, c_other, W.Fb);
  MLP_TRY(forward(W, batch, D, params, s));
  const int hblk = (int)cdiv(batch, 64);
  PROHD_LAUNCH("mlp_head_bwd", head_bwd, dim3((unsigned)hblk), dim3(256), 0, s, W.H2, W.Z2, W.s, labels,
               idx, batch, pos_weight, params + L.ow3, W.dZ2, W.part);
  PROHD_LAUNCH("mlp_head_reduce", head_reduce, dim3(1), dim3(192), 0, s, (const float*)W.part, hblk,
               grad + L.ow3, grad + L.ob3, loss);
  // dW2 = dZ2^T H1 ; db2 = colsum dZ2
  GemmArgs gw2{W.dZ2, 1, kH2, W.H1, kH1, 1, kH2, kH1, (int)batch, kH1, grad + L.oW2, nullptr, nullptr, nullptr};
  MLP_TRY(gemm<EPI_F32>(gw2, s, W.part));
  MLP_TRY(colsum(W.dZ2, batch, kH2, grad + L.ob2, W.part, s));
  // dZ1 = (dZ2 W2) * gelu'(z1)
  GemmArgs gd1{W.dZ2, kH2, 1, W.W2b, kH1, 1, (int)batch, kH1, kH2, kH1, nullptr, W.dZ1, nullptr, W.Z1};
  MLP_TRY(gemm<EPI_GELU_BWD>(gd1, s));
  // dW1 = dZ1^T F ; db1 = colsum dZ1
  GemmArgs gw1{W.dZ1, 1, kH1, W.Fb, L.F, 1, kH1, (int)L.F, (int)batch, L.F, grad + L.oW1, nullptr, nullptr, nullptr};
  MLP_TRY(gemm<EPI_F32>(gw1, s, W.part));
  MLP_TRY(colsum(W.dZ1, batch, kH1, grad + L.ob1, W.part, s));
  return PROHD_OK;
}

prohd_status mlp_adamw(float* params, const float* grad, float* m, float* v, int32_t D, int64_t t,
                       float lr, float wd, float b1, float b2, float eps, hipStream_t s) {
  const int64_t n = layout(D).total;
  const float c1 = (float)(1.0 - pow((double)b1, (double)t));
  const float c2 = (float)(1.0 - pow((double)b2, (double)t));
  PROHD_LAUNCH("mlp_adamw", adamw_kernel, dim3(256), dim3(256), 0, s, params, grad, m, v, n, lr, wd, b1,
               b2, eps, c1, c2);
  return PROHD_OK;
}

}  // namespace prohd
