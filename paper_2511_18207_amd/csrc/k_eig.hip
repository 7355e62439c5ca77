// Top-m eigenvectors of the union covariance, float64, in one work-group:
// the "top m principal components" step of the paper's Alg. 2.
//
//   1. Householder tridiagonalisation  C = Q T Q^T  (Q = H_0 H_1 ... H_{n-3},
//      H_j = I - tau_j v_j v_j^T); per step one symmetric matrix-vector
//      product and one rank-2 update, spread over all threads.  The matrix
//      lives in LDS for n <= 128 and in (L2-resident) global memory for
//      n = 256; the reflectors go to global memory.
//   2. All eigenvalues of T by bisection on Sturm counts (one per thread).
//   3. Eigenvectors of T for the m largest eigenvalues by inverse iteration
//      with a pivoted tridiagonal LU; eigenvalues closer than 1e-3 of the
//      spectral radius form a cluster and are solved in turn by one thread
//      with modified Gram-Schmidt against the earlier members.
//   4. Back-transformation z = Q y (reflectors staged through LDS), unit
//      length, sign fixed so the largest-magnitude entry is positive (first
//      index on ties).
// Rows and columns beyond D (padding to n = 16..256) carry -1 on the
// diagonal and zeros elsewhere, so they stay decoupled and below every real
// (non-negative) eigenvalue.

#include "batch.h"
#include "common.h"

namespace prohd {

size_t eig_ws_bytes(int32_t D, int32_t m);
prohd_status eig_run(double* C, int32_t D, int32_t m, const double* u0, float* dirs, double* evals,
                     const int32_t* status, void* ws, size_t ws_bytes, hipStream_t s);

namespace {

constexpr int kSlots = 16;   // concurrent inverse-iteration workers

template <int DP>
struct EigShape {
  static constexpr int NT = DP >= 64 ? 1024 : 256;     // threads
  static constexpr int NQ = NT / DP;                    // threads per column
  static constexpr int QS = DP / NQ > 0 ? DP / NQ : 1;  // rows per thread
  static constexpr bool IN_LDS = DP <= 128;             // matrix in LDS
  // LDS region reused: matrix (n <= 128), then LU slots, then reflector chunks
  static constexpr int BIG = IN_LDS ? (DP * DP > 4 * kSlots * DP ? DP * DP : 4 * kSlots * DP)
                                    : 4 * kSlots * DP;
  static constexpr int VROWS = BIG / DP;                // reflector rows per chunk
};

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

__device__ __forceinline__ double start_value(int k, int c) {
  // deterministic pseudo-random start vector entry in (-1, 1)
  uint32_t h = (uint32_t)k * 0x9E3779B1u ^ ((uint32_t)c + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return ((double)(h & 0xFFFFFFu) / 8388608.0) - 1.0 + 1.0 / 16777216.0;
}

template <int DP>
__device__ __forceinline__ void eig_body(
    double* __restrict__ Mg, int D, int m, double* __restrict__ Vg, double* __restrict__ Yg,
    const double* __restrict__ u0, float* __restrict__ dirs, double* __restrict__ evals,
    const int32_t* __restrict__ status) {
  using S = EigShape<DP>;
  constexpr int NT = S::NT;
  __shared__ double big[S::BIG];
  __shared__ double vs[DP], wv[DP], part[S::NQ][DP];
  __shared__ double dd[DP], ee[DP], e2[DP], tau[DP], lam[DP];
  __shared__ double red[NT / 64];
  __shared__ uint8_t piv[kSlots][DP];
  __shared__ int lead_of[64];

  const int t = threadIdx.x;
  const bool ok = (status == nullptr) || (*status == 0);

  double* M = S::IN_LDS ? big : Mg;
  if (S::IN_LDS) {
    for (int e = t; e < DP * DP; e += NT) big[e] = Mg[e];
  }
  __syncthreads();

  // ---------------------------------------------------- 1. tridiagonalise
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

  // ------------------------------------------------------- 2. bisection
  if (t < DP) e2[t] = ee[t] * ee[t];
  __syncthreads();
  double gl = 0.0, gu = 0.0, emax = 0.0;
  for (int i = 0; i < DP; ++i) {
    const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i < DP - 1 ? fabs(ee[i]) : 0.0);
    gl = (i == 0) ? dd[i] - r : fmin(gl, dd[i] - r);
    gu = (i == 0) ? dd[i] + r : fmax(gu, dd[i] + r);
    emax = fmax(emax, e2[i]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = 1e-290 * fmax(1.0, emax);
  if (t < DP) {
    // lam[t] = (t+1)-th smallest eigenvalue: count(x) = #eigenvalues < x
    double lo = gl - 1e-14 * tnorm - pivmin, hi = gu + 1e-14 * tnorm + pivmin;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      if (hi - lo <= 2.2e-16 * (fmax(fabs(lo), fabs(hi)) + tnorm) + pivmin) break;
      int cnt = 0;
      double q = dd[0] - mid;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      for (int i = 1; i < DP; ++i) {
        double r = __builtin_amdgcn_rcp(q);   // 1/q, refined by one Newton step
        r = fma(r, fma(-q, r, 1.0), r);
        q = dd[i] - mid - e2[i - 1] * r;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
      }
      if (cnt >= t + 1) hi = mid; else lo = mid;
    }
    lam[t] = 0.5 * (lo + hi);
  }
  __syncthreads();

  // ------------------------------------------------ 3. inverse iteration
  // vectors c = 0..m-1 (descending eigenvalue); clusters by gap < ortol
  const double lmax = fmax(fabs(lam[DP - 1]), fabs(lam[DP - D]));
  const double ortol = 1e-3 * lmax;
  const double tol = 2.2e-16 * fmax(tnorm, 1e-300);
  if (t == 0) {
    int lead = 0;
    for (int c = 0; c < m; ++c) {
      if (c > 0 && lam[DP - c] - lam[DP - 1 - c] >= ortol) lead = c;
      lead_of[c] = lead;
    }
  }
  __syncthreads();
  double* slot_base = big;  // kSlots x 4 x DP doubles: U0 inverse, U1, L, x
  // leaders take slots in rounds of kSlots
  for (int round = 0; round * kSlots < m; ++round) {
    const int c0 = t;  // candidate leader index handled by this thread
    const int leader = round * kSlots + c0;
    if (c0 < kSlots && leader < m && lead_of[leader] == leader && ok) {
      double* U0 = slot_base + (size_t)c0 * 4 * DP;
      double* U1 = U0 + DP;
      double* Lm = U0 + 2 * DP;
      double* x = U0 + 3 * DP;
      uint8_t* pv = piv[c0];
      double prev = 0.0;
      for (int c = leader; c < m && lead_of[c] == leader; ++c) {
        double lc = lam[DP - 1 - c];
        if (c > leader && lc > prev - 10.0 * tol) lc = prev - 10.0 * tol;
        prev = lc;
        // pivoted LU of T - lc I
        double dcur = dd[0] - lc, ucur = ee[0];
        for (int i = 0; i < DP - 1; ++i) {
          const double sub = ee[i];
          const double an = dd[i + 1] - lc;
          const double bn = (i + 1 < DP - 1) ? ee[i + 1] : 0.0;
          if (fabs(dcur) >= fabs(sub)) {
            double dpiv = dcur;
            if (fabs(dpiv) < tol) dpiv = dpiv < 0.0 ? -tol : tol;
            const double mult = sub / dpiv;
            U0[i] = 1.0 / dpiv;
            U1[i] = ucur;
            Lm[i] = mult;
            pv[i] = 0;
            dcur = an - mult * ucur;
            ucur = bn;
          } else {
            const double mult = dcur / sub;
            U0[i] = 1.0 / sub;
            U1[i] = an;
            Lm[i] = mult;
            pv[i] = 1;
            dcur = ucur - mult * an;
            ucur = -mult * bn;
          }
        }
        if (fabs(dcur) < tol) dcur = dcur < 0.0 ? -tol : tol;
        U0[DP - 1] = 1.0 / dcur;
        // start vector (zero on padding rows keeps them exactly zero)
        for (int k = 0; k < DP; ++k) x[k] = (k < D) ? start_value(k, c) : 0.0;
        for (int it = 0; it < 5; ++it) {
          // forward: apply the row interchanges and multipliers
          for (int i = 0; i < DP - 1; ++i) {
            double bi = x[i], bn = x[i + 1];
            if (pv[i]) {
              const double tmp = bi;
              bi = bn;
              bn = tmp;
            }
            x[i] = bi;
            x[i + 1] = bn - Lm[i] * bi;
          }
          // backward: U has diagonal, first and (when pivoted) second superdiagonal
          double x2 = 0.0, x1 = x[DP - 1] * U0[DP - 1];
          x[DP - 1] = x1;
          for (int i = DP - 2; i >= 0; --i) {
            const double u2 = (pv[i] && i + 2 < DP) ? ee[i + 1] : 0.0;
            const double xi = (x[i] - U1[i] * x1 - u2 * x2) * U0[i];
            x[i] = xi;
            x2 = x1;
            x1 = xi;
          }
          // orthogonalise against the earlier members of the cluster
          for (int p = leader; p < c; ++p) {
            const double* yp = Yg + (size_t)p * DP;
            double d = 0.0;
            for (int k = 0; k < DP; ++k) d += x[k] * yp[k];
            for (int k = 0; k < DP; ++k) x[k] -= d * yp[k];
          }
          double mx = 0.0;
          for (int k = 0; k < DP; ++k) mx = fmax(mx, fabs(x[k]));
          if (!(mx > 0.0)) mx = 1.0;
          double s2 = 0.0;
          for (int k = 0; k < DP; ++k) {
            x[k] /= mx;
            s2 += x[k] * x[k];
          }
          const double inv = 1.0 / sqrt(s2);
          for (int k = 0; k < DP; ++k) x[k] *= inv;
        }
        double* yc = Yg + (size_t)c * DP;
        for (int k = 0; k < DP; ++k) yc[k] = x[k];
      }
    }
    __syncthreads();
  }

  // ------------------------------------------------ 4. back-transform
  // wave w transforms vectors c = w, w + NW, ...; lane holds entries
  // k = lane + 64 r.
  constexpr int PR = (DP + 63) / 64;
  constexpr int NW = NT / 64;
  constexpr int VPW = (PROHD_MAX_DIRS - 1 + NW - 1) / NW;
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
  for (int hi = DP - 3; hi >= 0; hi -= S::VROWS) {
    const int lo = hi - S::VROWS + 1 > 0 ? hi - S::VROWS + 1 : 0;
    __syncthreads();
    for (int e = t; e < (hi - lo + 1) * DP; e += NT) big[e] = Vg[(size_t)lo * DP + e];
    __syncthreads();
    for (int j = hi; j >= lo; --j) {
      const double tj = tau[j];
      if (tj == 0.0) continue;
      const double* vj = big + (size_t)(j - lo) * DP;
#pragma unroll
      for (int v = 0; v < VPW; ++v) {
        const int c = wave + NW * v;
        if (c < m) {
          double d = 0.0;
#pragma unroll
          for (int r = 0; r < PR; ++r) {
            const int k = lane + 64 * r;
            if (k < DP) d += vj[k] * z[v][r];
          }
          d = tj * wave_sum(d);
#pragma unroll
          for (int r = 0; r < PR; ++r) {
            const int k = lane + 64 * r;
            if (k < DP) z[v][r] -= d * vj[k];
          }
        }
      }
    }
  }
  // unit length, canonical sign, float32 output rows 1..m
#pragma unroll
  for (int v = 0; v < VPW; ++v) {
    const int c = wave + NW * v;
    if (c < m) {
      double s2 = 0.0, bv = -1.0, sv = 0.0;
      int bk = 0x7fffffff;
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        const int k = lane + 64 * r;
        if (k < DP) {
          s2 += z[v][r] * z[v][r];
          const double a = fabs(z[v][r]);
          if (a > bv || (a == bv && k < bk)) {
            bv = a;
            bk = k;
            sv = z[v][r];
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
        if (k < D) dirs[(size_t)(1 + c) * D + k] = (float)(z[v][r] * f);
      }
    }
  }
  if (t < D) {
    dirs[t] = (float)u0[t];
    if (evals) evals[t] = lam[DP - 1 - t];
  }
}

template <int DP>
__global__ __launch_bounds__(EigShape<DP>::NT) void eig_kernel(
    double* __restrict__ Mg, int D, int m, double* __restrict__ Vg, double* __restrict__ Yg,
    const double* __restrict__ u0, float* __restrict__ dirs, double* __restrict__ evals,
    const int32_t* __restrict__ status) {
  eig_body<DP>(Mg, D, m, Vg, Yg, u0, dirs, evals, status);
}

// One work-group per job (pair).
template <int DP>
__global__ __launch_bounds__(EigShape<DP>::NT) void eig_batch(const EigJob* __restrict__ jobs, int D,
                                                              int njobs) {
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const EigJob j = jobs[it];
    __syncthreads();
    eig_body<DP>(j.C, D, j.m, j.V, j.Y, j.u0, j.dirs, nullptr, j.status);
  }
}

template <int DP>
prohd_status eig_dp(double* C, int32_t D, int32_t m, const double* u0, float* dirs, double* evals,
                    const int32_t* status, void* ws, size_t ws_bytes, hipStream_t s) {
  Arena ar(ws);
  double* V = ar.take<double>((size_t)DP * DP);
  double* Y = ar.take<double>((size_t)PROHD_MAX_DIRS * DP);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "eig: workspace too small");
  PROHD_LAUNCH("eig", eig_kernel<DP>, dim3(1), dim3(EigShape<DP>::NT), 0, s, C, D, m, V, Y, u0, dirs,
               evals, status);
  return PROHD_OK;
}

}  // namespace

size_t eig_ws_bytes(int32_t D, int32_t m) {
  (void)m;
  const int DP = pad_dim(D);
  Arena ar(nullptr);
  ar.take<double>((size_t)DP * DP);
  ar.take<double>((size_t)PROHD_MAX_DIRS * DP);
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

prohd_status batch_eig(int DP, int D, const EigJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  const int grid = std::min(njobs, 2 * cu_count());
  switch (DP) {
    case 16: PROHD_LAUNCH("batch_eig", eig_batch<16>, dim3(grid), dim3(EigShape<16>::NT), 0, s, jobs, D, njobs); break;
    case 32: PROHD_LAUNCH("batch_eig", eig_batch<32>, dim3(grid), dim3(EigShape<32>::NT), 0, s, jobs, D, njobs); break;
    case 64: PROHD_LAUNCH("batch_eig", eig_batch<64>, dim3(grid), dim3(EigShape<64>::NT), 0, s, jobs, D, njobs); break;
    case 128: PROHD_LAUNCH("batch_eig", eig_batch<128>, dim3(grid), dim3(EigShape<128>::NT), 0, s, jobs, D, njobs); break;
    case 256: PROHD_LAUNCH("batch_eig", eig_batch<256>, dim3(grid), dim3(EigShape<256>::NT), 0, s, jobs, D, njobs); break;
    default: return fail(PROHD_EUNSUPPORTED, "batched: unsupported padded dimension");
  }
  return PROHD_OK;
}

}  // namespace prohd
