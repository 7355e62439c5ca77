// Top-m eigenvectors of the union covariance, float64, in one work-group:
// the "top m principal components" step of the paper's Alg. 2.
//
//   1. Householder tridiagonalisation  C = Q T Q^T  (Q = H_0 H_1 ... H_{n-3},
//      H_j = I - tau_j v_j v_j^T); per step one symmetric matrix-vector
//      product and one rank-2 update, spread over all threads.  With the
//      wide work-group and n >= 64 the lower triangle is held in registers
//      (16 x 16 tiles, each lane a 2 x 2 block); otherwise it lives in LDS
//      (n <= 64) or in L2-resident global memory.  The reflectors go to
//      global memory.
//   2. Eigenvalues of T by bisection on Sturm counts; when only the m + 1
//      largest are needed, multisection with one 16-lane group per
//      eigenvalue.
//   3. Eigenvectors of T for the m largest eigenvalues by inverse iteration
//      with a pivoted tridiagonal LU, one substitution thread per vector;
//      eigenvalues closer than 1e-3 of the spectral radius form a cluster
//      whose members iterate together, orthogonalised after every
//      substitution against the earlier members of their cluster (modified
//      Gram-Schmidt in index order, one wave per cluster) and normalised.
//   4. Back-transformation z = Q y (reflectors staged through LDS, the dot
//      products of a wave's vectors reduced together per reflector), unit
//      length, sign fixed so the largest-magnitude entry is positive (first
//      index on ties).
// Rows and columns beyond D (padding to n = 16..256) carry -1 on the
// diagonal and zeros elsewhere, so they stay decoupled and below every real
// (non-negative) eigenvalue.

#include <type_traits>

#include "batch.h"
#include "common.h"

namespace prohd {

size_t eig_ws_bytes(int32_t D, int32_t m);
prohd_status eig_run(double* C, int32_t D, int32_t m, const double* u0, float* dirs, double* evals,
                     const int32_t* status, void* ws, size_t ws_bytes, hipStream_t s);

namespace {

// Work-group shape.  The single-pair solve is latency bound and uses a wide
// work-group (512 threads with 256 registers each, the matrix held in
// registers, 8-16 inverse-iteration slots); the batched solve may instead
// use a narrow one (256 threads, 4 slots, matrix in LDS up to D = 64 and in
// global memory above) so that several problems share a compute unit.
// With the wide work-group and DP >= 64 the matrix is held in registers during
// the tridiagonalisation (REG); LDS then only holds vectors and, later, the
// inverse-iteration slots and reflector chunks.
template <int DP, int NT_ = (DP >= 64 ? 512 : 256), int SLOTS_ = 16,
          bool LDSMAT = (DP <= 32), int MAXD_ = PROHD_MAX_DIRS>
struct EigShape {
  static constexpr int NT = NT_;                        // threads
  static constexpr int SLOTS = SLOTS_;                  // concurrent inverse-iteration workers
  static constexpr int MAXD = MAXD_;                    // largest m + 1 handled
  static constexpr int NQ = NT / DP;                    // threads per column
  static constexpr int QS = DP / NQ > 0 ? DP / NQ : 1;  // rows per thread
  static constexpr bool REG = NT == 512 && DP >= 64;    // register-resident matrix
  static constexpr bool IN_LDS = LDSMAT && !REG;        // matrix in LDS
  static constexpr int SS = 4 * DP + 1;                 // LU slot stride (odd)
  // LDS region reused: matrix (when in LDS) or the register form's vectors
  // and its last 64 x 64 block, then LU slots, then reflector chunks
  static constexpr int BIG0 = IN_LDS ? (DP * DP > SLOTS * SS ? DP * DP : SLOTS * SS) : SLOTS * SS;
  static constexpr int BIG = REG && BIG0 < 64 * 65 + 128 ? 64 * 65 + 128 : BIG0;
  static constexpr int VROWS = BIG / DP;                // reflector rows per chunk
};

template <int DP>
using EigNarrow = EigShape<DP, 256, 4, (DP <= 64), 32>;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// Sum over the work-group; every thread gets the result.
template <int NT>
__device__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Lane permutations through DPP (no LDS round trip), on both halves of a
// double.  CTRL: 0xB1 quad_perm [1,0,3,2] (xor 1), 0x4E quad_perm [2,3,0,1]
// (xor 2), 0x141 row_half_mirror (lane i of 8 <- 7 - i), 0x128 row_ror 8
// (xor 8 within 16 lanes).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  // every lane has a valid source under these controls, so no "old" value
  // is needed (the plain move form leaves the destination free instead of
  // tying it to a copied or zeroed register)
  const int l2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  const int h2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __hiloint2double(h2, l2);
}

// Sum over the 8 consecutive lanes of each group of 8; every lane of the
// group gets the same bits.
__device__ __forceinline__ double sum8(double x) {
  x += dpp_d<0xB1>(x);
  x += dpp_d<0x4E>(x);
  x += dpp_d<0x141>(x);
  return x;
}

// Sum over the whole wave (all lanes active), returned wave-uniform: DPP
// within rows of 16 lanes, then the four row sums read from lanes 0, 16, 32
// and 48 in a fixed order.
__device__ __forceinline__ double wave_sum_dpp(double x) {
  x = sum8(x);
  x += dpp_d<0x128>(x);
  auto rl = [&](int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
  };
  return (rl(0) + rl(16)) + (rl(32) + rl(48));
}

// Sum over lanes congruent modulo 8 (the 8 lanes l % 8 == r).
__device__ __forceinline__ double sum_mod8(double x) {
  x += dpp_d<0x128>(x);
  x += __shfl_xor(x, 16);
  x += __shfl_xor(x, 32);
  return x;
}

// Householder tridiagonalisation with the symmetric matrix in registers.
// The lower triangle is cut into 16 x 16 tiles (I >= J; diagonal tiles hold
// both triangles).  Wave w owns the tile rows w and NB-1-w (NB + 1 tiles per
// wave); lane l holds the 2 x 2 block at tile rows 2 (l % 8).. and columns
// 2 (l / 8)..  Per step j: the owners of column j publish it in LDS; every
// wave forms the reflector v (Householder vector of the column below the
// subdiagonal) from it; the trailing matvec p = tau A v is summed per wave
// (row sums accumulated over a tile row before one cross-lane reduction,
// column sums reduced within groups of 8 lanes per tile) into two private
// LDS rows, then across waves in a fixed order; every wave forms K = (tau/2) p.v
// and the tiles take the rank-2 update A -= v w^T + w v^T, w = p - K v, in
// registers.  Writes d, e, tau and the reflectors (Vg rows) as the LDS /
// global variant does.
//
// The step is a chain of short phases between three barriers, bound by LDS
// latency and LDS issue rather than arithmetic: every length-DP vector is
// read once per phase with all of a lane's loads in flight together, the
// tile loops fetch the column entries of tile u + 2 while tile u is worked
// on, and the partial sums are plain stores (no LDS atomics).  The reflector
// rows go to global memory from the last wave, which owns the fewest tiles.
template <int DP, int NT>
__device__ __forceinline__ void tridiag_reg(const double* __restrict__ Mg, double* __restrict__ Vg,
                                            double* col0, double* pbuf0, double* col1, double* pbuf1,
                                            double* pw, double* red, double* dd, double* ee,
                                            double* tau) {
  constexpr int W = NT / 64;
  constexpr int NB = DP / 16;
  constexpr int TPW = NB + 1;          // tiles of tile rows RA and RB
  constexpr int PR = DP / 64;          // entries of a length-DP vector per lane
  static_assert(NB / 2 <= W, "one pair of tile rows per wave");
  static_assert(DP % 64 == 0, "register path: DP a multiple of 64");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool owner = wave < NB / 2;
  const int RA = wave, RB = NB - 1 - wave;
  const int rb = lane & 7, cb = lane >> 3;
  double a[TPW][2][2];
  // tile u: row RA for u <= RA (J = u), else row RB (J = u - RA - 1)
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int I = u <= RA ? RA : RB, J = u <= RA ? u : u - RA - 1;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        a[u][i][q] = owner ? Mg[(size_t)(16 * I + 2 * rb + i) * DP + 16 * J + 2 * cb + q] : 0.0;
  }
  // two partial rows of p per wave, written with plain stores (an LDS
  // atomic costs the compute unit several times a load): pwA takes the
  // column sums of the row-RA tiles (blocks J < RA) and the row sums of row
  // RA, pwB those of row RB.  Within a step no entry is written twice;
  // blocks a wave never writes stay zero from here on, and entries of
  // skipped tiles keep stale values at indices <= j, which p never reads.
  double* pwA = pw + (size_t)(2 * wave) * DP;
  double* pwB = pwA + DP;
  // per-wave copies of the step's v and w (only this wave reads them, in
  // program order after its own writes, so no barrier guards them)
  double* vp = pw + (size_t)(2 * W + wave) * DP;
  double* wp = pw + (size_t)(3 * W + wave) * DP;
#pragma unroll
  for (int r = 0; r < 2 * PR; ++r) pwA[lane + 64 * r] = 0.0;
  struct Pair {
    double x, y;
  };
  // entries 16 J + 2 cb and + 1 of a length-DP vector, J the tile column of tile u
  auto tcol = [&](int u) { return u <= RA ? u : u - RA - 1; };
  auto colpair = [&](const double* x, int u) {
    const int J = tcol(u);
    return Pair{x[16 * J + 2 * cb], x[16 * J + 2 * cb + 1]};
  };
  auto rowpair = [&](const double* x, int I) { return Pair{x[16 * I + 2 * rb], x[16 * I + 2 * rb + 1]}; };
  // the matrix loads complete here, before the step loop (a wait on them
  // inside the loop would also wait, every step, for the reflector stores)
  __builtin_amdgcn_s_waitcnt(0);
  // one step; QJ = j % 2 is a compile-time constant so that the column
  // element is picked without indexing the register array
  // col and pbuf alternate between two buffers by step parity, so a step
  // can publish its column while slower waves still read the previous
  // step's in their rank-2 update (no barrier at the start of a step)
  auto step = [&](const int j, auto QJ) {
    double* col = decltype(QJ)::value ? col1 : col0;
    double* pbuf = decltype(QJ)::value ? pbuf1 : pbuf0;
    const int rb2 = 2 * rb;
    const int Jj = j >> 4, cj = (j & 15) >> 1;
    if (owner && cb == cj) {
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int I = u <= RA ? RA : RB, J = u <= RA ? u : u - RA - 1;
        if (J == Jj) {
          col[16 * I + rb2] = a[u][0][decltype(QJ)::value];
          col[16 * I + rb2 + 1] = a[u][1][decltype(QJ)::value];
        }
      }
    }
    __syncthreads();
    // reflector (every wave computes the same values in the same order)
    double ck[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r) ck[r] = col[lane + 64 * r];
    const double alpha = col[j + 1];
    double s2 = 0.0;
#pragma unroll
    for (int r = 0; r < PR; ++r) {
      const int k = lane + 64 * r;
      s2 += (k > j + 1) ? ck[r] * ck[r] : 0.0;
    }
    const double sigma = wave_sum_dpp(s2);
    double tj = 0.0, beta = alpha, scale = 0.0;
    if (sigma > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tj = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v once per step into this wave's copy: every later use is one load
    double vk[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r) {
      const int k = lane + 64 * r;
      vk[r] = k == j + 1 ? 1.0 : (k > j + 1 ? ck[r] * scale : 0.0);
      vp[k] = vk[r];
    }
    if (tid == 0) {
      ee[j] = beta;
      tau[j] = tj;
    }
    if (wave == W - 1) {
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        const int k = lane + 64 * r;
        if (k == j) dd[j] = ck[r];
        Vg[(size_t)j * DP + k] = vk[r];
      }
    }
    if (tj == 0.0) return;   // uniform: nothing below the subdiagonal
    // p = A v over the trailing block, per wave
    if (owner) {
      double pa0 = 0.0, pa1 = 0.0, pb0 = 0.0, pb1 = 0.0;
      const Pair va = rowpair(vp, RA), vb = rowpair(vp, RB);
      Pair vq[TPW];
      vq[0] = colpair(vp, 0);
      vq[1] = colpair(vp, 1);
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        if (u + 2 < TPW) vq[u + 2] = colpair(vp, u + 2);
        const bool rowA = u <= RA;
        const int J = tcol(u);
        const int I = rowA ? RA : RB;
        if (16 * J + 15 > j) {   // uniform per wave
          const int c0 = 16 * J + 2 * cb;
          const double vc0 = vq[u].x, vc1 = vq[u].y;
          const double vr0 = rowA ? va.x : vb.x, vr1 = rowA ? va.y : vb.y;
          const double r0s = a[u][0][0] * vc0 + a[u][0][1] * vc1;
          const double r1s = a[u][1][0] * vc0 + a[u][1][1] * vc1;
          if (rowA) {
            pa0 += r0s;
            pa1 += r1s;
          } else {
            pb0 += r0s;
            pb1 += r1s;
          }
          if (I > J) {
            // column sums over the 8 row-pair lanes
            const double pc0 = sum8(a[u][0][0] * vr0 + a[u][1][0] * vr1);
            const double pc1 = sum8(a[u][0][1] * vr0 + a[u][1][1] * vr1);
            if (rb == 0) {
              double* dst = rowA ? pwA : pwB;
              dst[c0] = pc0;
              dst[c0 + 1] = pc1;
            }
          }
        }
      }
      pa0 = sum_mod8(pa0);
      pa1 = sum_mod8(pa1);
      pb0 = sum_mod8(pb0);
      pb1 = sum_mod8(pb1);
      if (cb == 0) {
        pwA[16 * RA + rb2] = pa0;
        pwA[16 * RA + rb2 + 1] = pa1;
        pwB[16 * RB + rb2] = pb0;
        pwB[16 * RB + rb2 + 1] = pb1;
      }
    }
    __syncthreads();
    // p in a fixed order over waves
    if (tid < DP) {
      double p = 0.0;
      if (tid > j) {
#pragma unroll
        for (int w = 0; w < NB; ++w) p += pw[(size_t)w * DP + tid];
        p *= tj;
      }
      pbuf[tid] = p;
    }
    __syncthreads();
    // K = (tau / 2) p.v (each wave, same order); w_k = p_k - K v_k
    double pk[PR], vv[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r) {
      pk[r] = pbuf[lane + 64 * r];
      vv[r] = vp[lane + 64 * r];
    }
    double kd = 0.0;
#pragma unroll
    for (int r = 0; r < PR; ++r) kd += pk[r] * vv[r];
    const double K = 0.5 * tj * wave_sum_dpp(kd);
    if (!owner) return;
#pragma unroll
    for (int r = 0; r < PR; ++r) {
      const int k = lane + 64 * r;
      wp[k] = k > j ? pk[r] - K * vv[r] : 0.0;
    }
    const Pair wa = rowpair(wp, RA), wb = rowpair(wp, RB);
    const Pair va = rowpair(vp, RA), vb = rowpair(vp, RB);
    // A -= v w^T + w v^T
    Pair vq[TPW], wq[TPW];
    vq[0] = colpair(vp, 0);
    wq[0] = colpair(wp, 0);
    vq[1] = colpair(vp, 1);
    wq[1] = colpair(wp, 1);
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      if (u + 2 < TPW) {
        vq[u + 2] = colpair(vp, u + 2);
        wq[u + 2] = colpair(wp, u + 2);
      }
      const bool rowA = u <= RA;
      const int J = rowA ? u : u - RA - 1;
      if (16 * J + 15 > j) {
        const double vc0 = vq[u].x, vc1 = vq[u].y, wc0 = wq[u].x, wc1 = wq[u].y;
        const double vr0 = rowA ? va.x : vb.x, vr1 = rowA ? va.y : vb.y;
        const double wr0 = rowA ? wa.x : wb.x, wr1 = rowA ? wa.y : wb.y;
        // two fused steps per element (a - v w^T, then - w v^T)
        a[u][0][0] = fma(-wr0, vc0, fma(-vr0, wc0, a[u][0][0]));
        a[u][0][1] = fma(-wr0, vc1, fma(-vr0, wc1, a[u][0][1]));
        a[u][1][0] = fma(-wr1, vc0, fma(-vr1, wc0, a[u][1][0]));
        a[u][1][1] = fma(-wr1, vc1, fma(-vr1, wc1, a[u][1][1]));
      }
    }
  };
  // The last M - 2 steps (trailing block of at most M = 64 rows) go to one
  // wave with the block in LDS: a step of the register form costs about the
  // same whatever the trailing size (three barriers and the chain of short
  // phases; about 7 500 cycles per step at D = 256 once the block is
  // small), while one wave with its own row per lane needs no barrier.
  constexpr int M = 64;
  constexpr int J0 = DP - M;   // even
  for (int j = 0; j < J0; j += 2) {
    step(j, std::integral_constant<int, 0>{});
    step(j + 1, std::integral_constant<int, 1>{});
  }
  __syncthreads();   // every wave's last rank-2 update is done; pw is free
  // the trailing M x M block (rows / columns J0 ..) into LDS, both
  // triangles, row stride M + 1
  constexpr int MS = M + 1;
  double* Am = pw;
  double* vs2 = pw + M * MS;
  double* ws2 = vs2 + M;
  if (owner) {
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const int I = u <= RA ? RA : RB, J = u <= RA ? u : u - RA - 1;
      if (16 * J >= J0) {   // then 16 I >= J0 as well (I >= J)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int r = 16 * I + 2 * rb + i - J0, cc = 16 * J + 2 * cb + q - J0;
            Am[r * MS + cc] = a[u][i][q];
            if (I > J) Am[cc * MS + r] = a[u][i][q];
          }
      }
    }
  }
  __syncthreads();
  if (wave == 0) {
    const int l = lane;   // local row
    for (int j = J0; j < DP - 2; ++j) {
      const int jl = j - J0;
      const double ajl = Am[l * MS + jl];
      const double alpha = Am[(jl + 1) * MS + jl];
      const double sigma = wave_sum_dpp(l > jl + 1 ? ajl * ajl : 0.0);
      double tj = 0.0, beta = alpha, scale = 0.0;
      if (sigma > 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      const double vk = l == jl + 1 ? 1.0 : (l > jl + 1 ? ajl * scale : 0.0);
      if (l == 0) {
        ee[j] = beta;
        tau[j] = tj;
        dd[j] = Am[jl * MS + jl];
      }
#pragma unroll
      for (int r = 0; r < PR; ++r) {   // entries J0 + l are in the last lane block
        const int k = lane + 64 * r;
        Vg[(size_t)j * DP + k] = k >= J0 ? vk : 0.0;
      }
      if (tj == 0.0) continue;   // uniform
      vs2[l] = vk;
      // p = tau A v over rows / columns past jl (this lane's row), then
      // K = (tau / 2) p.v and w = p - K v
      // (in chunks of 16 columns, the live ones only; the entries of v and
      // w at or before jl are zero, so whole chunks need no masks)
      double pp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k0 = 0; k0 < M; k0 += 16) {
        if (k0 + 15 <= jl) continue;   // uniform
        double av[16], vv2[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          av[q] = Am[l * MS + k0 + q];
          vv2[q] = vs2[k0 + q];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) pp[q & 3] = fma(av[q], vv2[q], pp[q & 3]);
      }
      double p = (pp[0] + pp[1]) + (pp[2] + pp[3]);
      p = l > jl ? p * tj : 0.0;
      const double K = 0.5 * tj * wave_sum_dpp(p * vk);
      const double wk = l > jl ? p - K * vk : 0.0;
      ws2[l] = wk;
      // A -= v w^T + w v^T on this lane's row (two fused steps per element)
      // (rows at or before jl have v = w = 0 and stay as they are)
#pragma unroll
      for (int k0 = 0; k0 < M; k0 += 16) {
        if (k0 + 15 <= jl) continue;   // uniform
        double av[16], vv2[16], wv2[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          av[q] = Am[l * MS + k0 + q];
          vv2[q] = vs2[k0 + q];
          wv2[q] = ws2[k0 + q];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) Am[l * MS + k0 + q] = fma(-wk, vv2[q], fma(-vk, wv2[q], av[q]));
      }
    }
    if (l == 0) {
      dd[DP - 2] = Am[(M - 2) * MS + M - 2];
      dd[DP - 1] = Am[(M - 1) * MS + M - 1];
      ee[DP - 2] = Am[(M - 1) * MS + M - 2];
    }
  }
  if (tid == 0) {
    ee[DP - 1] = 0.0;
    tau[DP - 2] = tau[DP - 1] = 0.0;
  }
  __syncthreads();
}

// Number of eigenvalues of the tridiagonal T (diagonal d, squared
// off-diagonal e2) below x: the negative pivots of T - x I (Sturm sequence),
// each pivot kept at least pivmin away from zero.
template <int DP>
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, double pivmin, double x) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < DP; ++i) {
    double r = __builtin_amdgcn_rcp(q);   // 1/q, refined by one Newton step
    r = fma(r, fma(-q, r, 1.0), r);
    q = d[i] - x - e2[i - 1] * r;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Eigenvalue bounds of T: Gershgorin interval [gl, gu], the largest squared
// off-diagonal.  Minima and maxima are exact, so every caller and every
// reduction order gets the same bits.
struct TriBounds {
  double gl, gu, tnorm, pivmin;
};

__device__ __forceinline__ double gersh_radius(const double* e, int i, int n) {
  return (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
}

// Unit length and canonical sign (largest-magnitude entry positive, first
// index on ties) of one vector held by one wave, lane l holding entries
// l + 64 r; written as float32 row 1 + c of dirs (entries below D).
template <int DP, int PR>
__device__ __forceinline__ void finish_vector(const double (&z)[PR], int lane, int c, int D,
                                              float* __restrict__ dirs) {
  double s2 = 0.0, bv = -1.0, sv = 0.0;
  int bk = 0x7fffffff;
#pragma unroll
  for (int r = 0; r < PR; ++r) {
    const int k = lane + 64 * r;
    if (k < DP) {
      s2 += z[r] * z[r];
      const double a = fabs(z[r]);
      if (a > bv || (a == bv && k < bk)) {
        bv = a;
        bk = k;
        sv = z[r];
      }
    }
  }
  s2 = wave_sum(s2);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off);
    const int ok2 = __shfl_xor(bk, off);
    const double os = __shfl_xor(sv, off);
    if (ov > bv || (ov == bv && ok2 < bk)) {
      bv = ov;
      bk = ok2;
      sv = os;
    }
  }
  const double f = (sv < 0.0 ? -1.0 : 1.0) / sqrt(s2);
#pragma unroll
  for (int r = 0; r < PR; ++r) {
    const int k = lane + 64 * r;
    if (k < D) dirs[(size_t)(1 + c) * D + k] = (float)(z[r] * f);
  }
}

// The stages of the solve run either in one work-group (ALL: the batched
// form, one job per work-group) or split over four launches for one
// matrix: TRI (tridiagonalisation, d / e / tau to global memory), then a
// multi-work-group bisection, then VEC (inverse iteration from the stored T
// and eigenvalues), then a multi-work-group back-transformation.
enum EigMode { EIG_ALL = 0, EIG_TRI = 1, EIG_VEC = 2 };

__device__ __forceinline__ double start_value(int k, int c) {
  // deterministic pseudo-random start vector entry in (-1, 1)
  uint32_t h = (uint32_t)k * 0x9E3779B1u ^ ((uint32_t)c + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return ((double)(h & 0xFFFFFFu) / 8388608.0) - 1.0 + 1.0 / 16777216.0;
}

// tri: 4 DP doubles (d, e, tau, eigenvalues), used by the split modes.
template <int DP, class S, int MODE = EIG_ALL>
__device__ __forceinline__ void eig_body(
    double* __restrict__ Mg, int D, int m, double* __restrict__ Vg, double* __restrict__ Yg,
    const double* __restrict__ u0, float* __restrict__ dirs, double* __restrict__ evals,
    const int32_t* __restrict__ status, double* __restrict__ tri = nullptr) {
  constexpr int NT = S::NT;
  __shared__ double big[S::BIG];
  __shared__ double vs[DP], wv[DP], part[S::NQ][DP];
  __shared__ double dd[DP], ee[DP], e2[DP], tau[DP], lam[DP];
  __shared__ double red[NT / 64];
  __shared__ uint8_t piv[S::SLOTS][DP + 4];
  __shared__ int lead_of[64];

  const int t = threadIdx.x;
  const bool ok = (status == nullptr) || (*status == 0);

  double* M = S::IN_LDS ? big : Mg;
  if (S::IN_LDS && MODE != EIG_VEC) {
    for (int e = t; e < DP * DP; e += NT) big[e] = Mg[e];
  }
  __syncthreads();

  // ---------------------------------------------------- 1. tridiagonalise
  if constexpr (MODE == EIG_VEC) {
    if (t < DP) {
      dd[t] = tri[t];
      ee[t] = tri[DP + t];
      tau[t] = tri[2 * DP + t];
      lam[t] = tri[3 * DP + t];
    }
    __syncthreads();
  } else if constexpr (S::REG) {
    static_assert(S::NQ >= 2, "the second column / p buffers live in part");
    static_assert(S::BIG >= 4 * (NT / 64) * DP, "per-wave p partials, v and w live in big");
    static_assert(S::BIG >= 64 * 65 + 128, "the last 64 x 64 block and two vectors live in big");
    tridiag_reg<DP, NT>(Mg, Vg, vs, wv, part[0], part[1], big, red, dd, ee, tau);
  } else {
    const int ci = t % DP;        // column owned in the matvec / update
    const int cq = t / DP;        // row block of that column
    const int k0 = cq * S::QS;
    const int k1 = k0 + S::QS;
    __shared__ double sq[S::NQ];
    // sigma of column 0 below the subdiagonal
    double sigma = block_sum<NT>((t > 1 && t < DP) ? M[(size_t)t * DP] * M[(size_t)t * DP] : 0.0, red);
    for (int j = 0; j < DP - 2; ++j) {
      const double xk = (t > j + 1 && t < DP) ? M[(size_t)t * DP + j] : 0.0;
      const double alpha = M[(size_t)(j + 1) * DP + j];
      double tj = 0.0, beta = alpha, scale = 0.0;
      if (sigma > 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      if (t < DP) {
        const double v = (t == j + 1) ? 1.0 : (t > j + 1 ? xk * scale : 0.0);
        vs[t] = v;
        Vg[(size_t)j * DP + t] = v;
      }
      if (t == 0) {
        ee[j] = beta;
        tau[j] = tj;
        dd[j] = M[(size_t)j * DP + j];
      }
      __syncthreads();
      if (tj != 0.0) {  // uniform
        // p = tau * M v over the trailing block (rows k > j, columns > j)
        if (ci > j) {
          double acc = 0.0;
          const int kb = k0 > j + 1 ? k0 : j + 1;
  #pragma unroll 8
          for (int k = kb; k < k1; ++k) acc += M[(size_t)k * DP + ci] * vs[k];
          part[cq][ci] = acc;
        }
        __syncthreads();
        double p = 0.0, v = 0.0;
        if (t < DP && t > j) {
  #pragma unroll
          for (int q = 0; q < S::NQ; ++q) p += part[q][t];
          p *= tj;
          v = vs[t];
        }
        const double K = 0.5 * tj * block_sum<NT>(p * v, red);
        if (t < DP) wv[t] = (t > j) ? p - K * v : 0.0;
        __syncthreads();
        // M -= v w^T + w v^T on the trailing block; the owners of column j+1
        // also sum its squares below the next subdiagonal (next step's sigma)
        double s2 = 0.0;
        if (ci > j) {
          const double vi = vs[ci], wi = wv[ci];
          const int kb = k0 > j + 1 ? k0 : j + 1;
  #pragma unroll 8
          for (int k = kb; k < k1; ++k) {
            const double nv = M[(size_t)k * DP + ci] - (vs[k] * wi + wv[k] * vi);
            M[(size_t)k * DP + ci] = nv;
            s2 += (k > j + 2) ? nv * nv : 0.0;
          }
        }
        if (ci == j + 1) sq[cq] = s2;
        __syncthreads();
        sigma = 0.0;
  #pragma unroll
        for (int q = 0; q < S::NQ; ++q) sigma += sq[q];
      } else {
        const double nx = (t > j + 2 && t < DP) ? M[(size_t)t * DP + j + 1] : 0.0;
        sigma = block_sum<NT>(nx * nx, red);
      }
    }
    if (t == 0) {
      dd[DP - 2] = M[(size_t)(DP - 2) * DP + DP - 2];
      dd[DP - 1] = M[(size_t)(DP - 1) * DP + DP - 1];
      ee[DP - 2] = M[(size_t)(DP - 1) * DP + DP - 2];
      ee[DP - 1] = 0.0;
      tau[DP - 2] = tau[DP - 1] = 0.0;
    }
    __syncthreads();
  }

  if constexpr (MODE == EIG_TRI) {
    if (t < DP) {
      tri[t] = dd[t];
      tri[DP + t] = ee[t];
      tri[2 * DP + t] = tau[t];
    }
    return;
  }

  // ------------------------------------------------------- 2. bisection
  if (t < DP) e2[t] = ee[t] * ee[t];
  __syncthreads();
  double gl = 0.0, gu = 0.0, emax = 0.0;
  for (int i = 0; i < DP; ++i) {
    const double r = gersh_radius(ee, i, DP);
    gl = (i == 0) ? dd[i] - r : fmin(gl, dd[i] - r);
    gu = (i == 0) ? dd[i] + r : fmax(gu, dd[i] + r);
    emax = fmax(emax, e2[i]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = 1e-290 * fmax(1.0, emax);
  // count(x) = number of eigenvalues below x (Sturm sequence of T - x I)
  auto sturm = [&](double x) { return sturm_count<DP>(dd, e2, pivmin, x); };
  if (MODE == EIG_VEC) {
    // eigenvalues from the bisection launch
  } else if (evals == nullptr && NT >= 512) {
    // only the m + 1 largest and the smallest real eigenvalue are used:
    // 16-way multisection, one group of 16 lanes per eigenvalue
    constexpr int G = 16;
    const int grp = t / G, gi = t % G;
    const int ne = m + 2;
    for (int base = 0; base < ne; base += NT / G) {
      const int e = base + grp;
      if (e < ne) {   // uniform per group of 16 lanes
        const int idx = e <= m ? DP - 1 - e : DP - D;
        double lo = gl - 1e-14 * tnorm - pivmin, hi = gu + 1e-14 * tnorm + pivmin;
        for (int it = 0; it < 40; ++it) {
          const double w = hi - lo;
          if (!(w > 2.2e-16 * (fmax(fabs(lo), fabs(hi)) + tnorm) + pivmin)) break;
          const double x = lo + w * (double)(gi + 1) / (double)(G + 1);
          const unsigned long long bal = __ballot(sturm(x) <= idx);
          const int k = __popcll((bal >> (t & 63 & ~(G - 1))) & 0xFFFFull);
          const double nlo = k > 0 ? lo + w * (double)k / (double)(G + 1) : lo;
          const double nhi = k < G ? lo + w * (double)(k + 1) / (double)(G + 1) : hi;
          if (!(nlo >= lo && nhi <= hi && nlo < nhi)) break;
          lo = nlo;
          hi = nhi;
        }
        if (gi == 0) lam[idx] = 0.5 * (lo + hi);
      }
    }
  } else if (t < DP) {
    // lam[t] = (t+1)-th smallest eigenvalue: count(x) = #eigenvalues < x
    double lo = gl - 1e-14 * tnorm - pivmin, hi = gu + 1e-14 * tnorm + pivmin;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      if (hi - lo <= 2.2e-16 * (fmax(fabs(lo), fabs(hi)) + tnorm) + pivmin) break;
      if (sturm(mid) >= t + 1) hi = mid; else lo = mid;
    }
    lam[t] = 0.5 * (lo + hi);
  }
  __syncthreads();

  // ------------------------------------------------ 3. inverse iteration
  // vectors c = 0..m-1 (descending eigenvalue); clusters by gap < ortol.
  // Rounds of SLOTS vectors: one thread per vector factors T - lc I
  // (pivoted LU) and runs the substitutions; after each substitution the
  // waves orthogonalise every vector against the earlier members of its
  // cluster (modified Gram-Schmidt in index order, 64 lanes per vector; one
  // wave per cluster, so members of a cluster stay in order) and scale it to
  // unit length.  Members of one cluster iterate together, so a large
  // cluster costs no more substitutions than a separated eigenvalue.
  const double lmax = fmax(fabs(lam[DP - 1]), fabs(lam[DP - D]));
  const double ortol = 1e-3 * lmax;
  const double tol = 2.2e-16 * fmax(tnorm, 1e-300);
  __shared__ double shift[S::MAXD];
  if (t == 0) {
    int lead = 0;
    double prev = 0.0;
    for (int c = 0; c < m; ++c) {
      if (c > 0 && lam[DP - c] - lam[DP - 1 - c] >= ortol) lead = c;
      lead_of[c] = lead;
      // equal eigenvalues inside a cluster get shifts 10 tol apart
      double lc = lam[DP - 1 - c];
      if (c > lead && lc > prev - 10.0 * tol) lc = prev - 10.0 * tol;
      prev = lc;
      shift[c] = lc;
    }
  }
  __syncthreads();
  // Slots: U0 inverse, U1, L and x of one vector each, S::SS doubles apart
  // (an odd stride puts the 16 substitution threads' entries in different
  // LDS banks; so does the padded pivot row).
  double* slot_base = big;
  constexpr int SS = S::SS;
  constexpr int NWV = NT / 64;
  constexpr int PRV = (DP + 63) / 64;     // entries of a vector per lane
  constexpr int SB = 8;                   // substitution block
  const int lane3 = t & 63, wave3 = t >> 6;
  for (int r0 = 0; r0 < m; r0 += S::SLOTS) {
    const int nr = min(S::SLOTS, m - r0);
    double* U0 = slot_base + (size_t)(t < S::SLOTS ? t : 0) * SS;
    double* U1 = U0 + DP;
    double* Lm = U0 + 2 * DP;
    double* x = U0 + 3 * DP;
    uint8_t* pv = piv[t < S::SLOTS ? t : 0];
    if (t < nr && ok) {
      const int c = r0 + t;
      const double lc = shift[c];
      // pivoted LU of T - lc I, without branches: the pivot choice selects
      // the operands of one reciprocal
      double dcur = dd[0] - lc, ucur = ee[0];
      for (int i = 0; i < DP - 1; ++i) {
        const double sub = ee[i];
        const double an = dd[i + 1] - lc;
        const double bn = (i + 1 < DP - 1) ? ee[i + 1] : 0.0;
        const bool keep = fabs(dcur) >= fabs(sub);   // no row interchange
        double dpiv = dcur;
        if (fabs(dpiv) < tol) dpiv = dpiv < 0.0 ? -tol : tol;
        const double rp = 1.0 / (keep ? dpiv : sub);
        const double mult = (keep ? sub : dcur) * rp;
        U0[i] = rp;
        U1[i] = keep ? ucur : an;
        Lm[i] = mult;
        pv[i] = keep ? 0 : 1;
        const double dn = keep ? an - mult * ucur : ucur - mult * an;
        ucur = keep ? bn : -mult * bn;
        dcur = dn;
      }
      if (fabs(dcur) < tol) dcur = dcur < 0.0 ? -tol : tol;
      U0[DP - 1] = 1.0 / dcur;
      // start vector (zero on padding rows keeps them exactly zero)
      for (int k = 0; k < DP; ++k) x[k] = (k < D) ? start_value(k, c) : 0.0;
    }
    // three iterations: the shifts are the bisection's eigenvalues (float64
    // resolution), so one solve already leaves another eigenvector's share
    // below (shift error) / (gap to it) and the next two take it to rounding
    // (a gap under 1e-3 of the spectral radius makes a cluster, whose members
    // are orthogonalised after every solve)
    for (int it = 0; it < 3; ++it) {
      if (t < nr && ok) {
        // forward: apply the row interchanges and multipliers.  The running
        // row stays in a register; the operands of SB steps are read into
        // registers before those steps (x[i + 1] is read before step i + 1
        // writes it, as in the step order), so a block costs one LDS round
        // trip rather than one per step.
        double carry = x[0];
        for (int ib = 0; ib < DP - 1; ib += SB) {
          double xn[SB], lm[SB];
          bool sw[SB];
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            const int i = min(ib + q, DP - 2);
            xn[q] = x[i + 1];
            lm[q] = Lm[i];
            sw[q] = pv[i] != 0;
          }
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            const int i = ib + q;
            if (i < DP - 1) {
              const double bi = sw[q] ? xn[q] : carry, bnx = sw[q] ? carry : xn[q];
              x[i] = bi;
              carry = bnx - lm[q] * bi;
            }
          }
        }
        x[DP - 1] = carry;
        // backward: U has diagonal, first and (when pivoted) second
        // superdiagonal; blocks of SB steps as above
        double x2 = 0.0, x1 = x[DP - 1] * U0[DP - 1];
        x[DP - 1] = x1;
        for (int ib = DP - 2; ib >= 0; ib -= SB) {
          double xo[SB], u1[SB], u0[SB], u2[SB];
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            const int i = max(ib - q, 0);
            const double e1 = ee[i + 1 < DP ? i + 1 : i];
            xo[q] = x[i];
            u1[q] = U1[i];
            u0[q] = U0[i];
            u2[q] = (pv[i] && i + 2 < DP) ? e1 : 0.0;
          }
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            const int i = ib - q;
            if (i >= 0) {
              const double xi = (xo[q] - u1[q] * x1 - u2[q] * x2) * u0[q];
              x[i] = xi;
              x2 = x1;
              x1 = xi;
            }
          }
        }
      }
      __syncthreads();
      if (ok) {
        for (int v = 0; v < nr; ++v) {
          const int c = r0 + v;
          if (lead_of[c] % NWV != wave3) continue;   // wave-uniform
          double* xv = slot_base + (size_t)v * SS + 3 * DP;
          double xr[PRV];
#pragma unroll
          for (int r = 0; r < PRV; ++r) {
            const int k = lane3 + 64 * r;
            xr[r] = k < DP ? xv[k] : 0.0;
          }
          for (int p = lead_of[c]; p < c; ++p) {
            const double* yp = p < r0 ? Yg + (size_t)p * DP : slot_base + (size_t)(p - r0) * SS + 3 * DP;
            double yr[PRV];
#pragma unroll
            for (int r = 0; r < PRV; ++r) {
              const int k = lane3 + 64 * r;
              yr[r] = k < DP ? yp[k] : 0.0;
            }
            double d = 0.0;
#pragma unroll
            for (int r = 0; r < PRV; ++r) d += xr[r] * yr[r];
            d = wave_sum_dpp(d);
#pragma unroll
            for (int r = 0; r < PRV; ++r) xr[r] -= d * yr[r];
          }
          double mx = 0.0;
#pragma unroll
          for (int r = 0; r < PRV; ++r) mx = fmax(mx, fabs(xr[r]));
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
          if (!(mx > 0.0)) mx = 1.0;
          double s2 = 0.0;
#pragma unroll
          for (int r = 0; r < PRV; ++r) {
            xr[r] = xr[r] / mx;
            s2 += xr[r] * xr[r];
          }
          const double inv = 1.0 / sqrt(wave_sum_dpp(s2));
#pragma unroll
          for (int r = 0; r < PRV; ++r) {
            const int k = lane3 + 64 * r;
            if (k < DP) xv[k] = xr[r] * inv;
          }
        }
      }
      __syncthreads();
    }
    for (int e = t; e < nr * DP; e += NT) {
      const int v = e / DP, k = e - v * DP;
      Yg[(size_t)(r0 + v) * DP + k] = slot_base[(size_t)v * SS + 3 * DP + k];
    }
    __syncthreads();
  }

  // ------------------------------------------------ 4. back-transform
  if constexpr (MODE == EIG_VEC) {   // the back-transformation launch follows
    if (t < D) {
      dirs[t] = (float)u0[t];
      if (evals) evals[t] = lam[DP - 1 - t];
    }
    return;
  }
  // wave w transforms vectors c = w, w + NW, ...; lane holds entries
  // k = lane + 64 r.  Per reflector the wave forms the dot products of all
  // its vectors first and reduces them together (independent cross-lane
  // chains overlap); NV = 2 covers m <= 2 NW (the default m = 16 on eight
  // waves) without carrying empty vectors through the reductions.
  constexpr int PR = (DP + 63) / 64;
  constexpr int NW = NT / 64;
  constexpr int VPW = (S::MAXD - 1 + NW - 1) / NW;
  const int lane = t & 63, wave = t >> 6;
  double z[VPW][PR];
#pragma unroll
  for (int v = 0; v < VPW; ++v) {
    const int c = wave + NW * v;
#pragma unroll
    for (int r = 0; r < PR; ++r) {
      const int k = lane + 64 * r;
      z[v][r] = (c < m && k < DP && ok) ? Yg[(size_t)c * DP + k] : 0.0;
    }
  }
  auto apply = [&](auto NVC) {
    constexpr int NV = decltype(NVC)::value;
    for (int hi = DP - 3; hi >= 0; hi -= S::VROWS) {
      const int lo = hi - S::VROWS + 1 > 0 ? hi - S::VROWS + 1 : 0;
      __syncthreads();
      // chunk of reflector rows into LDS, eight loads in flight per thread
      const int ne = (hi - lo + 1) * DP;
      for (int e0 = t; e0 < ne; e0 += 8 * NT) {
        double tmp[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) tmp[q] = Vg[(size_t)lo * DP + min(e0 + q * NT, ne - 1)];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (e0 + q * NT < ne) big[e0 + q * NT] = tmp[q];
      }
      __syncthreads();
      for (int j = hi; j >= lo; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;
        const double* vj = big + (size_t)(j - lo) * DP;
        double vr[PR];
#pragma unroll
        for (int r = 0; r < PR; ++r) vr[r] = vj[(lane + 64 * r) % DP];
        double d[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          d[v] = 0.0;
#pragma unroll
          for (int r = 0; r < PR; ++r)
            if (lane + 64 * r < DP) d[v] += vr[r] * z[v][r];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) d[v] = tj * wave_sum_dpp(d[v]);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int r = 0; r < PR; ++r)
            if (lane + 64 * r < DP) z[v][r] -= d[v] * vr[r];
      }
    }
  };
  if (m <= 2 * NW)
    apply(std::integral_constant<int, 2 < VPW ? 2 : VPW>{});
  else
    apply(std::integral_constant<int, VPW>{});
  // unit length, canonical sign, float32 output rows 1..m
#pragma unroll
  for (int v = 0; v < VPW; ++v) {
    const int c = wave + NW * v;
    if (c < m) finish_vector<DP>(z[v], lane, c, D, dirs);
  }
  if (t < D) {
    dirs[t] = (float)u0[t];
    if (evals) evals[t] = lam[DP - 1 - t];
  }
}

template <int DP>
__global__ __launch_bounds__(EigShape<DP>::NT) void eig_tri_kernel(double* __restrict__ Mg, int D,
                                                                    double* __restrict__ Vg,
                                                                    double* __restrict__ tri) {
  eig_body<DP, EigShape<DP>, EIG_TRI>(Mg, D, 0, Vg, nullptr, nullptr, nullptr, nullptr, nullptr, tri);
}

template <int DP>
__global__ __launch_bounds__(EigShape<DP>::NT) void eig_vec_kernel(
    int D, int m, double* __restrict__ Vg, double* __restrict__ Yg, const double* __restrict__ u0,
    float* __restrict__ dirs, double* __restrict__ evals, const int32_t* __restrict__ status,
    double* __restrict__ tri) {
  eig_body<DP, EigShape<DP>, EIG_VEC>(nullptr, D, m, Vg, Yg, u0, dirs, evals, status, tri);
}

// Bisection over work-groups: work-group b finds one eigenvalue of the
// stored T (index DP-1-b, the (b+1)-th largest; with all == 0 the last
// work-group takes the smallest real one, DP-D) by 256-way multisection,
// one Sturm count per thread and step, so an interval shrinks 257-fold per
// step (about seven steps to float64 resolution).  The stopping rule and
// the final midpoint are those of the one-work-group solve.
constexpr int kBisectThreads = 256;

template <int DP>
__global__ __launch_bounds__(kBisectThreads) void eig_bisect_kernel(double* __restrict__ tri, int D,
                                                                    int m, int all) {
  constexpr int G = kBisectThreads;
  __shared__ double d[DP], e2[DP];
  __shared__ double rmin[G / 64], rmax[G / 64], rem[G / 64];
  __shared__ int cnt[2][G / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int b = blockIdx.x;
  const int idx = all ? DP - 1 - b : (b <= m ? DP - 1 - b : DP - D);
  const double* te = tri + DP;
  double lo_t = 0.0, hi_t = 0.0, e2_t = 0.0;
  if (t < DP) {
    d[t] = tri[t];
    e2[t] = te[t] * te[t];
    const double r = gersh_radius(te, t, DP);
    lo_t = tri[t] - r;
    hi_t = tri[t] + r;
    e2_t = e2[t];
  } else {   // threads past DP repeat entry 0: minima and maxima unchanged
    const double r = gersh_radius(te, 0, DP);
    lo_t = tri[0] - r;
    hi_t = tri[0] + r;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo_t = fmin(lo_t, __shfl_xor(lo_t, off));
    hi_t = fmax(hi_t, __shfl_xor(hi_t, off));
    e2_t = fmax(e2_t, __shfl_xor(e2_t, off));
  }
  if (lane == 0) {
    rmin[wave] = lo_t;
    rmax[wave] = hi_t;
    rem[wave] = e2_t;
  }
  __syncthreads();
  double gl = rmin[0], gu = rmax[0], emax = rem[0];
#pragma unroll
  for (int w = 1; w < G / 64; ++w) {
    gl = fmin(gl, rmin[w]);
    gu = fmax(gu, rmax[w]);
    emax = fmax(emax, rem[w]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = 1e-290 * fmax(1.0, emax);
  double lo = gl - 1e-14 * tnorm - pivmin, hi = gu + 1e-14 * tnorm + pivmin;
  for (int it = 0; it < 64; ++it) {
    const double w = hi - lo;
    if (!(w > 2.2e-16 * (fmax(fabs(lo), fabs(hi)) + tnorm) + pivmin)) break;
    const double x = lo + w * (double)(t + 1) / (double)(G + 1);
    const unsigned long long bal = __ballot(sturm_count<DP>(d, e2, pivmin, x) <= idx);
    if (lane == 0) cnt[it & 1][wave] = __popcll(bal);
    __syncthreads();
    int k = 0;
#pragma unroll
    for (int q = 0; q < G / 64; ++q) k += cnt[it & 1][q];
    const double nlo = k > 0 ? lo + w * (double)k / (double)(G + 1) : lo;
    const double nhi = k < G ? lo + w * (double)(k + 1) / (double)(G + 1) : hi;
    if (!(nlo >= lo && nhi <= hi && nlo < nhi)) break;
    lo = nlo;
    hi = nhi;
  }
  if (t == 0) tri[3 * DP + idx] = 0.5 * (lo + hi);
}

// Back-transformation over work-groups: work-group c (one wave) turns
// eigenvector c of T into z = H_0 H_1 ... H_{DP-3} y, lane l holding entries
// l + 64 r, with the arithmetic and order of the one-work-group form; the
// reflector rows come from global memory (L2) a block of kBackRows ahead of
// their use, so one vector's chain of dot products and updates never waits
// for memory.  Then unit length and canonical sign (row 1 + c of dirs).
constexpr int kBackRows = 8;

template <int DP>
__global__ __launch_bounds__(64) void eig_back_kernel(const double* __restrict__ Vg,
                                                      const double* __restrict__ Yg,
                                                      const double* __restrict__ tri, int D,
                                                      float* __restrict__ dirs,
                                                      const int32_t* __restrict__ status) {
  constexpr int PR = (DP + 63) / 64;
  constexpr int SB = kBackRows;
  const int c = blockIdx.x, lane = threadIdx.x;
  const bool ok = (status == nullptr) || (*status == 0);
  const double* tau = tri + 2 * DP;
  double z[PR];
#pragma unroll
  for (int r = 0; r < PR; ++r) {
    const int k = lane + 64 * r;
    z[r] = (k < DP && ok) ? Yg[(size_t)c * DP + k] : 0.0;
  }
  double vb[2][SB][PR], tb[2][SB];
  // reflectors jb, jb - 1, ..., jb - SB + 1 (those >= 0) into buffer b
  auto fetch = [&](auto B, int jb) {
    constexpr int b = decltype(B)::value;
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int j = jb - q, jj = j > 0 ? j : 0;
      tb[b][q] = j >= 0 ? tau[jj] : 0.0;
#pragma unroll
      for (int r = 0; r < PR; ++r) vb[b][q][r] = Vg[(size_t)jj * DP + (lane + 64 * r) % DP];
    }
  };
  auto apply = [&](auto B, int jb) {
    constexpr int b = decltype(B)::value;
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const double tj = tb[b][q];
      if (jb - q < 0 || tj == 0.0) continue;   // uniform
      double d = 0.0;
#pragma unroll
      for (int r = 0; r < PR; ++r)
        if (lane + 64 * r < DP) d += vb[b][q][r] * z[r];
      d = tj * wave_sum_dpp(d);
#pragma unroll
      for (int r = 0; r < PR; ++r)
        if (lane + 64 * r < DP) z[r] -= d * vb[b][q][r];
    }
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  fetch(B0{}, DP - 3);
  for (int jb = DP - 3; jb >= 0; jb -= 2 * SB) {
    fetch(B1{}, jb - SB);
    apply(B0{}, jb);
    fetch(B0{}, jb - 2 * SB);
    apply(B1{}, jb - SB);
  }
  finish_vector<DP>(z, lane, c, D, dirs);
}

// One work-group per job (pair).
template <int DP, class S>
__global__ __launch_bounds__(S::NT) void eig_batch(const EigJob* __restrict__ jobs, int D, int njobs) {
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const EigJob j = jobs[it];
    __syncthreads();
    eig_body<DP, S>(j.C, D, j.m, j.V, j.Y, j.u0, j.dirs, nullptr, j.status);
  }
}

template <int DP>
prohd_status eig_dp(double* C, int32_t D, int32_t m, const double* u0, float* dirs, double* evals,
                    const int32_t* status, void* ws, size_t ws_bytes, hipStream_t s) {
  Arena ar(ws);
  double* V = ar.take<double>((size_t)DP * DP);
  double* Y = ar.take<double>((size_t)PROHD_MAX_DIRS * DP);
  double* T = ar.take<double>((size_t)4 * DP);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "eig: workspace too small");
  // eigenvalues wanted: all D real ones with evals, else the m + 1 largest
  // and the smallest real one
  const int all = evals != nullptr;
  const int nb = all ? D : m + 2;
  PROHD_LAUNCH("eig_tri", eig_tri_kernel<DP>, dim3(1), dim3(EigShape<DP>::NT), 0, s, C, D, V, T);
  PROHD_LAUNCH("eig_bisect", eig_bisect_kernel<DP>, dim3(nb), dim3(kBisectThreads), 0, s, T, D, m, all);
  PROHD_LAUNCH("eig_vec", eig_vec_kernel<DP>, dim3(1), dim3(EigShape<DP>::NT), 0, s, D, m, V, Y, u0, dirs,
               evals, status, T);
  if (m > 0) PROHD_LAUNCH("eig_back", eig_back_kernel<DP>, dim3(m), dim3(64), 0, s, V, Y, T, D, dirs, status);
  return PROHD_OK;
}

}  // namespace

size_t eig_ws_bytes(int32_t D, int32_t m) {
  (void)m;
  const int DP = pad_dim(D);
  Arena ar(nullptr);
  ar.take<double>((size_t)DP * DP);
  ar.take<double>((size_t)PROHD_MAX_DIRS * DP);
  ar.take<double>((size_t)4 * DP);
  return ar.used + 256;
}

prohd_status eig_run(double* C, int32_t D, int32_t m, const double* u0, float* dirs, double* evals,
                     const int32_t* status, void* ws, size_t ws_bytes, hipStream_t s) {
  switch (pad_dim(D)) {
    case 16: return eig_dp<16>(C, D, m, u0, dirs, evals, status, ws, ws_bytes, s);
    case 32: return eig_dp<32>(C, D, m, u0, dirs, evals, status, ws, ws_bytes, s);
    case 64: return eig_dp<64>(C, D, m, u0, dirs, evals, status, ws, ws_bytes, s);
    case 128: return eig_dp<128>(C, D, m, u0, dirs, evals, status, ws, ws_bytes, s);
    case 256: return eig_dp<256>(C, D, m, u0, dirs, evals, status, ws, ws_bytes, s);
    default: return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM");
  }
}

size_t eig_job_doubles(int DP) { return (size_t)DP * DP + (size_t)PROHD_MAX_DIRS * DP; }

template <int DP, class S>
prohd_status batch_eig_shape(int D, const EigJob* jobs, int njobs, int per_cu, hipStream_t s) {
  const int grid = std::min(njobs, per_cu * cu_count());
  PROHD_LAUNCH("batch_eig", (eig_batch<DP, S>), dim3(grid), dim3(S::NT), 0, s, jobs, D, njobs);
  return PROHD_OK;
}

template <int DP>
prohd_status batch_eig_dp(int D, const EigJob* jobs, int njobs, bool narrow, hipStream_t s) {
  if (narrow) return batch_eig_shape<DP, EigNarrow<DP>>(D, jobs, njobs, 4, s);
  return batch_eig_shape<DP, EigShape<DP>>(D, jobs, njobs, 2, s);
}

prohd_status batch_eig(int DP, int D, const EigJob* jobs, int njobs, bool narrow, hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  switch (DP) {
    case 16: return batch_eig_dp<16>(D, jobs, njobs, narrow, s);
    case 32: return batch_eig_dp<32>(D, jobs, njobs, narrow, s);
    case 64: return batch_eig_dp<64>(D, jobs, njobs, narrow, s);
    case 128: return batch_eig_dp<128>(D, jobs, njobs, narrow, s);
    case 256: return batch_eig_dp<256>(D, jobs, njobs, narrow, s);
    default: return fail(PROHD_EUNSUPPORTED, "batched: unsupported padded dimension");
  }
}

}  // namespace prohd

