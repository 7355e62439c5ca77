// First pass over the two point sets: per-set sums (centroids, paper Alg. 1)
// and the Gram matrix of the stacked union [A; B] (covariance for the
// principal components, Alg. 2), in float64 on the matrix cores.
//
// Rows are shifted by s = A[0] (converted to float64; the difference of two
// float32 values is exact in float64), so the accumulated Gram
//   G = sum_r (z_r - s)(z_r - s)^T
// stays well conditioned when the data sit far from the origin; the
// covariance is then C = (G - N mu_w mu_w^T) / (N - 1) with mu_w the mean of
// the shifted rows.
//
// gram_partial: TSPLIT work-groups per slice of rows of one set, each owning
// a share of the upper-triangle super-blocks (SB x SB blocks of 16 x 16),
// one super-block per wave.  Rows arrive in chunks of RC rows copied
// straight from HBM into LDS as float32 (buffer loads into LDS, no
// registers), double-buffered so that the next chunk streams in while the
// matrix cores work on the current one; one barrier per chunk.  For every
// group of four rows, lane l reads w[row l/16][16*I + l%16] for its blocks,
// converts to float64 and subtracts the shift (exact), and the 16x16 Gram
// block (I, J) gains one v_mfma_f64_16x16x4_f64 with A operand = block I and
// B operand = block J (the four rows are the k index).  Only blocks with
// I <= J are formed.  The waves that own a diagonal super-block also add the
// shifted values into the per-set column sums (each column has exactly one
// diagonal super-block) and check them for non-finite input.  The
// work-group writes its partial blocks and its columns' sums; gram_reduce
// adds the partials in a fixed order (deterministic) and writes C (padded
// to DP x DP: rows/columns >= D hold -1 on the diagonal, which keeps those
// padding directions below every real eigenvalue), the centroid axis (dirs
// row 0) and the status word.

#include <type_traits>
#include <utility>

#include "batch.h"
#include "common.h"

namespace prohd {

size_t stats_ws_bytes(int64_t nA, int64_t nB, int32_t D);
prohd_status stats_run(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                       double* C, double* u0, int32_t* status, void* ws, size_t ws_bytes,
                       hipStream_t s);

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int DP>
struct GramShape {
  static constexpr int NB = DP / 16;                    // 16-column blocks
  static constexpr int T = NB * (NB + 1) / 2;           // blocks with I <= J
  static constexpr int SB = DP >= 32 ? 2 : 1;           // super-block edge (blocks)
  static constexpr int NS = NB / SB;                    // super-blocks per edge
  static constexpr int TS = NS * (NS + 1) / 2;          // upper super-blocks
  static constexpr int TSPLIT = DP >= 256 ? 3 : 1;      // work-groups per row slice
  static constexpr int TSW = (TS + TSPLIT - 1) / TSPLIT;  // super-blocks per work-group
  static constexpr int WAVES = TSW > 4 ? TSW : 4;       // one super-block per wave
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int RC = 64;                         // rows per chunk
  static constexpr int CHUNK = RC * DP;                 // floats per LDS buffer
};

// Upper-triangle index of block (I, J), I <= J, rows enumerated in order.
__host__ __device__ constexpr int cblock_t(int I, int J, int nb) { return I * nb - I * (I - 1) / 2 + (J - I); }

// Super-block s (0..TS-1) -> (P, Q), P <= Q, in units of SB blocks.
constexpr int csb_p(int s, int ns) {
  int i = 0;
  while (i < ns && s >= ns - i) { s -= ns - i; ++i; }
  return i < ns ? i : 0;
}
constexpr int csb_q(int s, int ns) {
  int i = 0;
  while (i < ns && s >= ns - i) { s -= ns - i; ++i; }
  return i < ns ? i + s : 0;
}

// Super-block s -> (P, Q), P <= Q (wave-uniform values).
__device__ __forceinline__ void sb_pq(int s, int ns, int& P, int& Q) {
  int i = 0, rem = s;
  while (rem >= ns - i) {
    rem -= ns - i;
    ++i;
  }
  P = i;
  Q = i + rem;
}

// Block t (0..T-1) -> (I, J), I <= J, enumerated row by row.
__device__ __forceinline__ void block_ij(int t, int nb, int& I, int& J) {
  int i = 0, rem = t;
  while (rem >= nb - i) {
    rem -= nb - i;
    ++i;
  }
  I = i;
  J = i + rem;
}

// Gram partial of rows [r_begin, r_end) of X, shifted by the row `shift`;
// super-block share ts of TSPLIT; writes gp (T x 256) and, for the columns
// of its diagonal super-blocks, sp (2 DP sums: set A's, then set B's).
template <int DP>
__device__ __forceinline__ void gram_body(const float* __restrict__ shift, const float* __restrict__ X,
                                          int64_t r_begin, int64_t r_end, int D, int ts, bool setA,
                                          double* __restrict__ gp, double* __restrict__ spo,
                                          int32_t* __restrict__ status) {
  using S = GramShape<DP>;
  constexpr int RC = S::RC;
  constexpr int SB = S::SB;
  __shared__ __attribute__((aligned(16))) float xs[2][S::CHUNK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int col = lane & 15;   // column within a 16-block
  const int rsub = lane >> 4;  // row within a group of four
  const bool vec = (D & 3) == 0;

  // chunk c: rows [r_begin + c RC, ..) = one contiguous run of floats, copied
  // to LDS in 1 KiB (vec: 16 bytes per lane) or 256-byte pieces; the buffer
  // range ends at the slice's last row, so the rest reads as zero
  const int64_t nch = (r_end - r_begin + RC - 1) / RC;
  auto copy = [&](int64_t c) {
    const int64_t r0 = r_begin + c * RC;
    const int rows = (int)min<int64_t>(RC, r_end - r0);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(X + r0 * D), 0, rows * D * 4, 0x00020000);
    float* dst = xs[c & 1];
    if (vec) {
      const int pieces = (RC * D + 255) / 256;
      for (int i = wave; i < pieces; i += S::WAVES)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(dst + 256 * i), 16, (256 * i + 4 * lane) * 4, 0,
            0, 0);
    } else {
      const int pieces = (RC * D + 63) / 64;
      for (int i = wave; i < pieces; i += S::WAVES)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(dst + 64 * i), 4, (64 * i + lane) * 4, 0, 0, 0);
    }
  };

  // this wave's super-block s = ts TSW + wave: block rows P SB.., columns Q SB..
  int sp = -1, sq = -1;
  {
    const int sidx = ts * S::TSW + wave;
    if (wave < S::TSW && sidx < S::TS) sb_pq(sidx, S::NS, sp, sq);
  }
  const bool diag = sp >= 0 && sp == sq;
  int ca[SB], cb[SB];          // this lane's column in each block
  double sha[SB], shb[SB];     // the shift at those columns
  double sum[SB];
#pragma unroll
  for (int x = 0; x < SB; ++x) {
    ca[x] = 16 * (max(sp, 0) * SB + x) + col;
    cb[x] = 16 * (max(sq, 0) * SB + x) + col;
    sha[x] = ca[x] < D ? (double)shift[ca[x]] : 0.0;
    shb[x] = cb[x] < D ? (double)shift[cb[x]] : 0.0;
    sum[x] = 0.0;
  }
  bool bad = false;
  doublex4 acc[SB * SB];
#pragma unroll
  for (int x = 0; x < SB * SB; ++x) acc[x] = doublex4{0.0, 0.0, 0.0, 0.0};

  if (nch > 0) copy(0);
  for (int64_t c = 0; c < nch; ++c) {
    // chunk c has landed (every wave waited for its own copies), and every
    // wave is done with chunk c - 1, whose buffer the next copy overwrites
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 1 < nch) copy(c + 1);
    if (sp < 0) continue;
    const float* buf = xs[c & 1];
    const int lim = (int)min<int64_t>(RC, r_end - (r_begin + c * RC));
    if (lim == RC && D == DP) {
      // full chunk, no padding columns: no masks; each step reads the next
      // step's values ahead (the scheduling barrier keeps that order).  The
      // loop is instantiated separately for diagonal and off-diagonal
      // super-blocks (DG is wave-uniform), so neither carries the other's
      // branches.
      const float* bq = buf + rsub * DP;
      auto fast = [&](auto DGC) {
        constexpr bool DG = decltype(DGC)::value;
        float f[SB], g[SB];
#pragma unroll
        for (int x = 0; x < SB; ++x) {
          f[x] = bq[ca[x]];
          g[x] = DG ? 0.f : bq[cb[x]];
        }
#pragma unroll
        for (int q = 0; q < RC / 4; ++q) {
          float nf[SB], ng[SB];
#pragma unroll
          for (int x = 0; x < SB; ++x) {
            nf[x] = q + 1 < RC / 4 ? bq[4 * (q + 1) * DP + ca[x]] : 0.f;
            ng[x] = (q + 1 < RC / 4 && !DG) ? bq[4 * (q + 1) * DP + cb[x]] : 0.f;
          }
          double a[SB], b[SB];
#pragma unroll
          for (int x = 0; x < SB; ++x) {
            a[x] = (double)f[x] - sha[x];
            b[x] = DG ? a[x] : (double)g[x] - shb[x];
            if (DG) {
              bad |= !(f[x] - f[x] == 0.f);
              sum[x] += a[x];
            }
          }
#pragma unroll
          for (int x = 0; x < SB; ++x)
#pragma unroll
            for (int y = 0; y < SB; ++y)
              if (!DG || x <= y)
                acc[x * SB + y] =
                    __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x * SB + y], 0, 0, 0);
#pragma unroll
          for (int x = 0; x < SB; ++x) {
            f[x] = nf[x];
            g[x] = ng[x];
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      if (diag)
        fast(std::true_type{});
      else
        fast(std::false_type{});
      continue;
    }
#pragma unroll 2
    for (int q = 0; q < RC / 4; ++q) {
      const int row = 4 * q + rsub;
      const bool live = row < lim;
      const float* rp = buf + row * D;
      double a[SB], b[SB];
#pragma unroll
      for (int x = 0; x < SB; ++x) {
        const bool oka = live && ca[x] < D, okb = live && cb[x] < D;
        const float fa = rp[ca[x]], fb = rp[cb[x]];
        a[x] = oka ? (double)fa - sha[x] : 0.0;
        b[x] = okb ? (double)fb - shb[x] : 0.0;
        if (diag) {
          bad |= oka && !(fa - fa == 0.f);
          sum[x] += a[x];
        }
      }
#pragma unroll
      for (int x = 0; x < SB; ++x)
#pragma unroll
        for (int y = 0; y < SB; ++y)
          if (!diag || x <= y)
            acc[x * SB + y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x * SB + y], 0, 0, 0);
    }
  }
  if (bad) atomicOr(status, ST_NONFINITE);

  // live blocks: element v of lane l of the 16x16x4 f64 result is row
  // l/16 + 4 v, column l%16
  if (sp >= 0) {
#pragma unroll
    for (int x = 0; x < SB; ++x)
#pragma unroll
      for (int y = 0; y < SB; ++y) {
        const int I = sp * SB + x, J = sq * SB + y;
        if (I <= J) {
          const int t = cblock_t(I, J, S::NB);
#pragma unroll
          for (int v = 0; v < 4; ++v)
            gp[(size_t)t * 256 + (rsub + 4 * v) * 16 + col] = acc[x * SB + y][v];
        }
      }
  }
  // column sums of the diagonal super-blocks: the four row phases of a
  // column sit in lanes col, col + 16, col + 32, col + 48
  if (diag) {
#pragma unroll
    for (int x = 0; x < SB; ++x) {
      double v = sum[x];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (rsub == 0) {
        spo[setA ? ca[x] : DP + ca[x]] = v;
        spo[setA ? DP + ca[x] : ca[x]] = 0.0;
      }
    }
  }
}

template <int DP>
__global__ __launch_bounds__(GramShape<DP>::THREADS) void gram_partial(const float* __restrict__ A, int64_t nA,
                                                    const float* __restrict__ B, int64_t nB,
                                                    int D, int64_t rows_per_wg, int nslices,
                                                    double* __restrict__ gpart,
                                                    double* __restrict__ spart,
                                                    int32_t* __restrict__ status) {
  using S = GramShape<DP>;
  // row slices [0, wgA) of A, then of B; TSPLIT work-groups per slice share
  // its super-blocks and get ids congruent mod 8 (one XCD, one L2)
  const int xcd = blockIdx.x & 7;
  const int q8 = blockIdx.x >> 3;
  const int ts = q8 % S::TSPLIT;
  const int slice = (q8 / S::TSPLIT) * 8 + xcd;
  if (slice >= nslices) return;
  const int64_t wgA = (nA + rows_per_wg - 1) / rows_per_wg;
  const bool setA = (int64_t)slice < wgA;
  const float* X = setA ? A : B;
  const int64_t nX = setA ? nA : nB;
  const int64_t r_begin = (setA ? (int64_t)slice : (int64_t)slice - wgA) * rows_per_wg;
  const int64_t r_end = min(nX, r_begin + rows_per_wg);
  gram_body<DP>(A, X, r_begin, r_end, D, ts, setA, gpart + (size_t)slice * S::T * 256,
                spart + (size_t)slice * 2 * DP, status);
}

// D in (128, 256] (padded width 256), single pair and batched: one
// work-group of 16 waves per row slice forms all 136 upper-triangle
// 16 x 16 blocks.  Matrix and vector
// instructions of one SIMD share its issue (a probe loop of independent
// v_mfma_f64_16x16x4f64 loses about 4.4 cycles per 64 for every vector op
// beside it), so each value is converted to float64 and shifted once, into
// an LDS tile, instead of by every wave that uses it (5.5 times over):
//   per 32-row chunk: the rows arrive by DMA (float32, double-buffered);
//   after a barrier each thread converts 8 values of one column (its
//   shift in a register) into the float64 tile; after a second barrier
//   the waves multiply from it.
//   waves 0-11   a 32 x 64 unit (block rows 2P, 2P+1 x block columns 4Q'..
//                4Q'+3, all above the diagonal quads): 8 ops per 4 rows;
//   waves 12-15  a diagonal 64 x 64 quad (block rows = columns 4Q..4Q+3,
//                the 10 blocks with I <= J): 10 ops per 4 rows.
// With waves assigned to SIMDs round-robin each SIMD gets three units and
// one quad: 3 x 8 + 10 = 34 ops per group of four rows on every SIMD.
// The converting threads also sum their column (each column is converted
// by exactly the four threads t = c, c + 256, c + 512, c + 768) and check
// it for non-finite values at the end (an Inf or NaN anywhere in a column
// makes its float64 sum non-finite; finite float32 values cannot overflow
// it).
constexpr int kG256Units[12][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3},
                                   {2, 2}, {2, 3}, {3, 2}, {3, 3}, {4, 3}, {5, 3}};
constexpr int kG256RC = 32;           // rows per chunk
constexpr int kG256ST = 256 + 16;     // float64 tile row stride (doubles)

// The multiply phase of one wave kind (DG: diagonal quad, else a 32 x 64
// unit) over one chunk of the float64 tile; accumulators live in the
// caller's loop (one instantiation per kind, so the register allocation is
// the larger kind's).
template <bool DG>
__device__ __forceinline__ void g256_mul(const double* __restrict__ t64, int ca0, int cb0, int rsub,
                                         doublex4* acc) {
  constexpr int NA = DG ? 4 : 2;
  constexpr int NBV = DG ? 0 : 4;
  auto rd = [&](int q, double (&a)[NA], double (&b)[NBV > 0 ? NBV : 1]) {
    const double* rp = t64 + (4 * q + rsub) * kG256ST;
#pragma unroll
    for (int x = 0; x < NA; ++x) a[x] = rp[ca0 + 16 * x];
#pragma unroll
    for (int y = 0; y < NBV; ++y) b[y] = rp[cb0 + 16 * y];
  };
  double a[NA], b[NBV > 0 ? NBV : 1];
  rd(0, a, b);
#pragma unroll
  for (int q = 0; q < kG256RC / 4; ++q) {
    double na[NA], nb[NBV > 0 ? NBV : 1];
    if (q + 1 < kG256RC / 4) rd(q + 1, na, nb);
    if constexpr (DG) {
      int k = 0;
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = x; y < 4; ++y, ++k)
          acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], a[y], acc[k], 0, 0, 0);
    } else {
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[4 * x + y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[4 * x + y], 0, 0, 0);
    }
    if (q + 1 < kG256RC / 4) {
#pragma unroll
      for (int x = 0; x < NA; ++x) a[x] = na[x];
#pragma unroll
      for (int y = 0; y < NBV; ++y) b[y] = nb[y];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <bool DG>
__device__ __forceinline__ void g256_slice(const float* __restrict__ X, int64_t r_begin, int64_t r_end,
                                           int D, int br, int bc, double shv, float (*xs)[kG256RC * 256],
                                           double* t64, double* __restrict__ gp, double& csum) {
  constexpr int DP = 256, NB = 16, RC = kG256RC;
  constexpr int NACC = DG ? 10 : 8;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int col = lane & 15, rsub = lane >> 4;
  const int ca0 = 16 * br + col, cb0 = 16 * bc + col;
  const int ccol = tid & 255, crow = tid >> 8;   // conversion: column, first row
  const int64_t nch = (r_end - r_begin + RC - 1) / RC;
  // chunk c: 32 rows of D floats, one contiguous run copied in 1 KiB (D a
  // multiple of 4: 16 bytes per lane) or 256-byte pieces; rows past the
  // slice's end read as zero (buffer range)
  const bool vec = (D & 3) == 0;
  auto copy = [&](int64_t c) {
    const int64_t r0 = r_begin + c * RC;
    const int rows = (int)min<int64_t>(RC, r_end - r0);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(X + r0 * D), 0, rows * D * 4, 0x00020000);
    float* dst = xs[c & 1];
    if (vec) {
      for (int i = wave; i < (RC * D) / 256; i += 16)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(dst + 256 * i), 16, (256 * i + 4 * lane) * 4, 0,
            0, 0);
    } else {
      for (int i = wave; i < (RC * D + 63) / 64; i += 16)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void*)(dst + 64 * i), 4, (64 * i + lane) * 4, 0, 0, 0);
    }
  };
  doublex4 acc[NACC];
#pragma unroll
  for (int x = 0; x < NACC; ++x) acc[x] = doublex4{0.0, 0.0, 0.0, 0.0};
  if (nch > 0) copy(0);
  for (int64_t c = 0; c < nch; ++c) {
    // chunk c has landed (every wave waited for its own copies), and every
    // wave is done with the float64 tile of chunk c - 1
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const float* buf = xs[c & 1];
    const int lim = (int)min<int64_t>(RC, r_end - (r_begin + c * RC));
    // convert and shift: rows crow, crow + 4, ... of column ccol; rows past
    // the slice's end and columns past D become zero
    const bool cin = ccol < D;
    const int cc = cin ? ccol : D - 1;
#pragma unroll
    for (int k = 0; k < RC / 4; ++k) {
      const int r = crow + 4 * k;
      const double v = (double)buf[r * D + cc] - shv;
      const double z = (r < lim && cin) ? v : 0.0;
      csum += z;
      t64[r * kG256ST + ccol] = z;
    }
    __syncthreads();
    // buffer c & 1 is free: the copy of chunk c + 2 can go in after the
    // multiply phase of this chunk started; chunk c + 1 goes into the other
    if (c + 1 < nch) copy(c + 1);
    g256_mul<DG>(t64, ca0, cb0, rsub, acc);
  }
  // element v of lane l of the 16x16x4 f64 result is row l/16 + 4 v, column l%16
  int k = 0;
#pragma unroll
  for (int x = 0; x < (DG ? 4 : 2); ++x)
#pragma unroll
    for (int y = DG ? x : 0; y < 4; ++y, ++k) {
      const int t = cblock_t(br + x, bc + y, NB);
#pragma unroll
      for (int v = 0; v < 4; ++v) gp[(size_t)t * 256 + (rsub + 4 * v) * 16 + col] = acc[k][v];
    }
}

// Rows [r_begin, r_end) of X (one set's rows, D columns), shifted by the
// row `shift`: partial blocks gp (T x 256) and, for set A (setA) or B, the
// column sums spo (2 x 256).  All 1 024 threads reach every barrier.
__device__ __forceinline__ void gram256_body(const float* __restrict__ shift, const float* __restrict__ X,
                                             int64_t r_begin, int64_t r_end, int D, bool setA,
                                             double* __restrict__ gp, double* __restrict__ spo,
                                             int32_t* __restrict__ status, float (*xs)[kG256RC * 256],
                                             double* t64, double (*red)[256]) {
  constexpr int DP = 256;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool diag = wave >= 12;
  const int br = diag ? 4 * (wave - 12) : 2 * kG256Units[diag ? 0 : wave][0];
  const int bc = diag ? br : 4 * kG256Units[diag ? 0 : wave][1];
  const int ccol = tid & 255;
  const double shv = ccol < D ? (double)shift[ccol] : 0.0;   // the shift at this thread's column
  double csum = 0.0;
  if (diag)
    g256_slice<true>(X, r_begin, r_end, D, br, bc, shv, xs, t64, gp, csum);
  else
    g256_slice<false>(X, r_begin, r_end, D, br, bc, shv, xs, t64, gp, csum);
  // column sums: the four threads of a column, in a fixed order
  red[tid >> 8][ccol] = csum;
  __syncthreads();
  if (tid < DP) {
    const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
    spo[setA ? tid : DP + tid] = v;
    spo[setA ? DP + tid : tid] = 0.0;
    if (!(v - v == 0.0)) atomicOr(status, ST_NONFINITE);
  }
}

__global__ __launch_bounds__(1024) void gram_partial256(const float* __restrict__ A, int64_t nA,
                                                        const float* __restrict__ B, int64_t nB, int D,
                                                        int64_t rows_per_wg, int nslices,
                                                        double* __restrict__ gpart,
                                                        double* __restrict__ spart,
                                                        int32_t* __restrict__ status) {
  constexpr int DP = 256, NB = 16, T = NB * (NB + 1) / 2;
  __shared__ __attribute__((aligned(16))) float xs[2][kG256RC * 256];
  __shared__ __attribute__((aligned(16))) double t64[kG256RC * kG256ST];
  __shared__ double red[4][256];
  const int slice = blockIdx.x;
  if (slice >= nslices) return;
  const int64_t wgA = (nA + rows_per_wg - 1) / rows_per_wg;
  const bool setA = (int64_t)slice < wgA;
  const int64_t nX = setA ? nA : nB;
  const int64_t r_begin = (setA ? (int64_t)slice : (int64_t)slice - wgA) * rows_per_wg;
  const int64_t r_end = min(nX, r_begin + rows_per_wg);
  gram256_body(A, setA ? A : B, r_begin, r_end, D, setA, gpart + (size_t)slice * T * 256,
               spart + (size_t)slice * 2 * DP, status, xs, t64, red);
}

// Batched, padded width 256: one item per slice job.
__global__ __launch_bounds__(1024) void gram_batch256(const GramJob* __restrict__ jobs, int D,
                                                      const BItem* __restrict__ items, int nitems) {
  __shared__ __attribute__((aligned(16))) float xs[2][kG256RC * 256];
  __shared__ __attribute__((aligned(16))) double t64[kG256RC * kG256ST];
  __shared__ double red[4][256];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    if (w.job < 0) continue;
    const GramJob j = jobs[w.job];
    __syncthreads();   // the previous item's LDS reads are done
    gram256_body(j.shift, j.X, j.r_begin, j.r_end, D, j.setA != 0, j.gp, j.sp, j.status, xs, t64, red);
  }
}

// Batched: item (slice job, ts); the host orders items so that the TSPLIT
// shares of a slice are congruent modulo 8 (same XCD) for a grid that is a
// multiple of 8.
template <int DP>
__global__ __launch_bounds__(GramShape<DP>::THREADS) void gram_batch(const GramJob* __restrict__ jobs,
                                                                    int D,
                                                                    const BItem* __restrict__ items,
                                                                    int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    if (w.job < 0) continue;
    const GramJob j = jobs[w.job];
    __syncthreads();
    gram_body<DP>(j.shift, j.X, j.r_begin, j.r_end, D, w.bx, j.setA != 0, j.gp, j.sp, j.status);
  }
}

// Sums the partials (fixed order), forms the covariance and the centroid axis.
template <int DP>
__device__ __forceinline__ void gram_reduce_body(const double* __restrict__ gpart,
                                                 const double* __restrict__ spart, int nwg,
                                                 int64_t nA, int64_t nB, int D,
                                                 double* __restrict__ C, double* __restrict__ u0,
                                                 int bx, int nbx) {
  using S = GramShape<DP>;
  constexpr int NB = S::NB;
  __shared__ double sA[DP], sB[DP];
  __shared__ double red[256];
  for (int k = threadIdx.x; k < DP; k += blockDim.x) {
    double a = 0.0, b = 0.0;
    int g = 0;
    for (; g + 8 <= nwg; g += 8) {
      double va[8], vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        va[u] = spart[(size_t)(g + u) * 2 * DP + k];
        vb[u] = spart[(size_t)(g + u) * 2 * DP + DP + k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a += va[u];
        b += vb[u];
      }
    }
    for (; g < nwg; ++g) {
      a += spart[(size_t)g * 2 * DP + k];
      b += spart[(size_t)g * 2 * DP + DP + k];
    }
    sA[k] = a;
    sB[k] = b;
  }
  __syncthreads();
  const double N = (double)(nA + nB);
  const double inv = 1.0 / (double)((nA + nB) > 1 ? (nA + nB - 1) : 1);
  // covariance entries, one Gram element per thread iteration
  for (int e = bx * blockDim.x + threadIdx.x; e < S::T * 256; e += nbx * blockDim.x) {
    const int t = e >> 8;
    const int i = (e >> 4) & 15;
    const int j = e & 15;
    int I, J;
    block_ij(t, NB, I, J);
    // a diagonal tile holds both (i, j) and (j, i), which the matrix cores
    // may round differently: the lower one (i >= j) writes both positions,
    // so that no two threads race on an entry and C is the same bits on
    // every run
    if (I == J && i < j) continue;
    // partials added in slice order; loads issued eight at a time so the
    // sum does not wait on one memory round trip per slice
    double g = 0.0;
    const double* gq = gpart + (size_t)t * 256 + i * 16 + j;
    const size_t gs = (size_t)S::T * 256;
    int w = 0;
    for (; w + 8 <= nwg; w += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = gq[(size_t)(w + u) * gs];
#pragma unroll
      for (int u = 0; u < 8; ++u) g += v[u];
    }
    for (; w < nwg; ++w) g += gq[(size_t)w * gs];
    const int r = 16 * I + i, c = 16 * J + j;
    double v;
    if (r < D && c < D) {
      const double mr = (sA[r] + sB[r]) / N, mc = (sA[c] + sB[c]) / N;
      v = (g - N * mr * mc) * inv;
    } else {
      v = (r == c) ? -1.0 : 0.0;
    }
    C[(size_t)r * DP + c] = v;
    C[(size_t)c * DP + r] = v;
  }
  if (bx != 0) return;
  // centroid axis: mean(B) - mean(A) = sB/nB - sA/nA (the shift cancels)
  double nrm2 = 0.0;
  for (int k = threadIdx.x; k < D; k += blockDim.x) {
    const double d = sB[k] / (double)nB - sA[k] / (double)nA;
    nrm2 += d * d;
  }
  red[threadIdx.x] = nrm2;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  for (int k = threadIdx.x; k < D; k += blockDim.x) {
    const double d = sB[k] / (double)nB - sA[k] / (double)nA;
    u0[k] = (nrm < 1e-9) ? (k == 0 ? 1.0 : 0.0) : d / nrm;
  }
}

template <int DP>
__global__ __launch_bounds__(256) void gram_reduce(const double* __restrict__ gpart,
                                                   const double* __restrict__ spart, int nwg,
                                                   int64_t nA, int64_t nB, int D,
                                                   double* __restrict__ C, double* __restrict__ u0) {
  gram_reduce_body<DP>(gpart, spart, nwg, nA, nB, D, C, u0, blockIdx.x, gridDim.x);
}

template <int DP>
__global__ __launch_bounds__(256) void gram_reduce_batch(const GramRedJob* __restrict__ jobs, int D,
                                                         int njobs, int per_job) {
  for (int it = blockIdx.x; it < njobs * per_job; it += gridDim.x) {
    const GramRedJob j = jobs[it / per_job];
    __syncthreads();
    gram_reduce_body<DP>(j.gpart, j.spart, j.nwg, j.nA, j.nB, D, j.C, j.u0, it % per_job, per_job);
  }
}

struct StatsLayout {
  double* gpart;
  double* spart;
  int64_t rows;  // rows per work-group (multiple of the 64-row chunk)
  int nwg;       // work-groups: ceil(nA/rows) over A, then ceil(nB/rows) over B
};

StatsLayout stats_layout(Arena& ar, int64_t nA, int64_t nB, int DP, int cus) {
  StatsLayout L;
  const int64_t N = nA + nB;
  const int64_t target = std::max<int64_t>(1, std::min<int64_t>(cus, cdiv(N, 1024)));
  L.rows = cdiv(cdiv(N, target), 64) * 64;   // whole chunks
  L.nwg = (int)(cdiv(nA, L.rows) + cdiv(nB, L.rows));
  const int nb = DP / 16;
  const int T = nb * (nb + 1) / 2;
  L.gpart = ar.take<double>((size_t)L.nwg * T * 256);
  L.spart = ar.take<double>((size_t)L.nwg * 2 * DP);
  return L;
}

template <int DP>
prohd_status stats_dp(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D, double* C,
                      double* u0, int32_t* status, void* ws, size_t ws_bytes, hipStream_t s) {
  Arena ar(ws);
  StatsLayout L = stats_layout(ar, nA, nB, DP, cu_count());
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "stats: workspace too small");
  const int nwg = L.nwg;
  if constexpr (DP == 256) {
    PROHD_LAUNCH("stats_gram", gram_partial256, dim3(nwg), dim3(1024), 0, s, A, nA, B, nB, D, L.rows, nwg,
                 L.gpart, L.spart, status);
  } else {
    const int grid = (int)(cdiv(nwg, 8) * 8) * GramShape<DP>::TSPLIT;
    PROHD_LAUNCH("stats_gram", gram_partial<DP>, dim3(grid), dim3(GramShape<DP>::THREADS), 0, s, A,
                 nA, B, nB, D, L.rows, nwg, L.gpart, L.spart, status);
  }
  const int nb = DP / 16;
  const int T = nb * (nb + 1) / 2;
  const int rgrid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv((int64_t)T * 256, 256), 256));
  PROHD_LAUNCH("stats_reduce", gram_reduce<DP>, dim3(rgrid), dim3(256), 0, s, L.gpart, L.spart, nwg,
               nA, nB, D, C, u0);
  return PROHD_OK;
}

}  // namespace

size_t stats_ws_bytes(int64_t nA, int64_t nB, int32_t D) {
  Arena ar(nullptr);
  // the run uses at most as many work-groups as with this CU count
  stats_layout(ar, nA, nB, pad_dim(D), 1);
  Arena ar2(nullptr);
  stats_layout(ar2, nA, nB, pad_dim(D), 1024);
  ar.used = std::max(ar.used, ar2.used);
  return ar.used + 256;
}

prohd_status stats_run(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                       double* C, double* u0, int32_t* status, void* ws, size_t ws_bytes,
                       hipStream_t s) {
  switch (pad_dim(D)) {
    case 16: return stats_dp<16>(A, nA, B, nB, D, C, u0, status, ws, ws_bytes, s);
    case 32: return stats_dp<32>(A, nA, B, nB, D, C, u0, status, ws, ws_bytes, s);
    case 64: return stats_dp<64>(A, nA, B, nB, D, C, u0, status, ws, ws_bytes, s);
    case 128: return stats_dp<128>(A, nA, B, nB, D, C, u0, status, ws, ws_bytes, s);
    case 256: return stats_dp<256>(A, nA, B, nB, D, C, u0, status, ws, ws_bytes, s);
    default: return fail(PROHD_EUNSUPPORTED, "D exceeds PROHD_MAX_DIM");
  }
}

template <class F>
prohd_status by_dp_stats(int DP, F&& f) {
  switch (DP) {
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    default: return fail(PROHD_EUNSUPPORTED, "batched: unsupported padded dimension");
  }
}

int gram_tsplit(int DP) {
  if (DP == 256) return 1;   // gram_batch256: one work-group per slice
  int v = 1;
  by_dp_stats(DP, [&](auto dp) { v = GramShape<decltype(dp)::value>::TSPLIT; return PROHD_OK; });
  return v;
}

int gram_rows_quantum(int DP) {
  if (DP == 256) return kG256RC;
  int v = 32;
  by_dp_stats(DP, [&](auto dp) { v = GramShape<decltype(dp)::value>::RC; return PROHD_OK; });
  return v;
}

size_t gram_partial_doubles(int DP) {
  size_t v = 0;
  by_dp_stats(DP, [&](auto dp) { v = (size_t)GramShape<decltype(dp)::value>::T * 256; return PROHD_OK; });
  return v;
}

prohd_status batch_gram(int DP, int D, const GramJob* jobs, const BItem* items, int nitems, int grid,
                        hipStream_t s) {
  if (nitems <= 0) return PROHD_OK;
  if (DP == 256) {
    PROHD_LAUNCH("batch_gram", gram_batch256, dim3(grid), dim3(1024), 0, s, jobs, D, items, nitems);
    return PROHD_OK;
  }
  return by_dp_stats(DP, [&](auto dp) {
    constexpr int V = decltype(dp)::value;
    PROHD_LAUNCH("batch_gram", gram_batch<V>, dim3(grid), dim3(GramShape<V>::THREADS), 0, s, jobs, D,
                 items, nitems);
    return PROHD_OK;
  });
}

prohd_status batch_gram_reduce(int DP, int D, const GramRedJob* jobs, int njobs, int per_job,
                               hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  const int grid = (int)std::min<int64_t>((int64_t)njobs * per_job, 8 * cu_count());
  return by_dp_stats(DP, [&](auto dp) {
    PROHD_LAUNCH("batch_gram_reduce", gram_reduce_batch<decltype(dp)::value>, dim3(grid), dim3(256), 0,
                 s, jobs, D, njobs, per_job);
    return PROHD_OK;
  });
}

}  // namespace prohd
