// Extreme selection: the k smallest and k largest entries of float32 arrays
// under the total order (value, index), by radix selection on the device.
//
// This is the "argsort, keep the first k and the last k, keep the unique
// indices" step of the paper's Alg. 1 and Alg. 2, without a sort: only the
// k-th key from each end is located (three histogram passes over 11/11/10
// bits of an order-preserving 32-bit key), then every entry is compared with
// it.  Entries equal to the k-th key are taken in index order until the
// count is reached, so ties go to the smaller index at both ends.  When few
// entries share the first 22 bits with the k-th key, the third pass is
// skipped: the compare pass collects them and a small kernel ranks them.
//
// Kept entries set a flag byte; flags of several arrays (directions) may
// point to one buffer, which yields their union.  compact_flags2() turns the
// flags into an ascending index list with a device-side count.
//
// Every launch reads its array lengths from device memory when asked to, so
// a whole chain runs without a host synchronisation.

#include "batch.h"
#include "common.h"

namespace prohd {
namespace {

constexpr int kBins = 2048;          // 11-bit digits
constexpr int kHistChunk = 16384;    // elements per histogram work-group
constexpr int kMarkChunk = 4096;     // elements per tie-count / mark work-group
constexpr int kThreads = 256;

struct EndState {
  uint32_t prefix;  // key bits fixed so far
  uint32_t mask;    // which bits of prefix are fixed
  int32_t need;     // entries still to take among those matching prefix
  int32_t active;   // 1 if this end selects anything
  int32_t eq;       // entries in the last located digit (after the final
                    // pass: entries equal to the k-th key)
  int32_t buf;      // 1: after the second digit the entries sharing the
                    // 22-bit prefix fit a buffer; the mark pass collects them
                    // and buf_finish ranks them (no third pass)
};

// Entries of one end that share the 22-bit prefix, as (ranking key, index)
// composites where a smaller composite ranks first: the key at the bottom
// end, its complement at the top (equal keys then rank by index).
constexpr int kBufCap = 1024;

constexpr int kUnr = 8;   // loads in flight per thread in the streaming passes

struct SegDev {
  const float* vals;
  const int64_t* dev_n;
  int64_t n;
  uint8_t* flags;
  int32_t lo, hi;
};

// Segment descriptors travel as a kernel argument (no host-to-device copy,
// so a chain of launches can be captured in a graph).
constexpr int kSegPerLaunch = 64;   // 64 x 40-byte descriptors: 2.6 KB of kernel arguments
struct SegPack {
  SegDev s[kSegPerLaunch];
  int32_t nseg;   // segments in this pack
  int32_t base;   // global index of s[0] (state / histogram slot)
};

// Order-preserving key: a < b (as floats, -0 == +0) <=> key(a) < key(b).
__device__ __forceinline__ uint32_t fkey(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u << 1) == 0u) u = 0u;  // -0.0 -> +0.0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ int64_t seg_len(const SegDev& s) {
  return s.dev_n ? min(*s.dev_n, s.n) : s.n;
}

__global__ void init_state(const SegPack P, EndState* __restrict__ st, uint32_t* __restrict__ hist,
                           int32_t* __restrict__ bufn) {
  const int lid = blockIdx.x;
  if (lid >= P.nseg) return;
  const SegDev s = P.s[lid];
  const int sid = P.base + lid;
  const int64_t n = seg_len(s);
  if (threadIdx.x < 2) {
    const int e = threadIdx.x;
    const int64_t k = e == 0 ? s.lo : s.hi;
    const int64_t need = k < n ? k : n;
    EndState es;
    es.prefix = 0u;
    es.mask = 0u;
    es.need = (int32_t)(need > 0 ? need : 0);
    es.active = need > 0 ? 1 : 0;
    es.eq = 0;
    es.buf = 0;
    st[2 * sid + e] = es;
    bufn[2 * sid + e] = 0;
  }
  uint32_t* h = hist + (size_t)sid * 2 * kBins;
  for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x) h[i] = 0u;
}

// One digit pass: histogram of the digit at `shift` over entries whose key
// matches the prefix fixed so far, separately for the two ends.
__global__ __launch_bounds__(kThreads) void digit_hist(const SegPack P,
                                                      const EndState* __restrict__ st,
                                                      uint32_t* __restrict__ hist,
                                                      int shift, uint32_t dmask) {
  __shared__ uint32_t h[2][kBins];
  const SegDev s = P.s[blockIdx.y];
  const int sid = P.base + blockIdx.y;
  const int64_t n = seg_len(s);
  const int64_t base = (int64_t)blockIdx.x * kHistChunk;
  if (base >= n) return;
  const EndState e0 = st[2 * sid], e1 = st[2 * sid + 1];
  // buffered ends (see EndState::buf) need no further digit
  const bool a0 = e0.active && !e0.buf, a1 = e1.active && !e1.buf;
  if (!a0 && !a1) return;
  for (int i = threadIdx.x; i < 2 * kBins; i += kThreads) (&h[0][0])[i] = 0u;
  __syncthreads();
  const int64_t end = min(n, base + kHistChunk);
  // both ends still on the same prefix (always so in the first pass): one
  // histogram serves both
  const bool same = a0 && a1 && e0.mask == e1.mask && e0.prefix == e1.prefix;
  for (int64_t i0 = base; i0 < end; i0 += (int64_t)kThreads * kUnr) {
    uint32_t keys[kUnr];
#pragma unroll
    for (int u = 0; u < kUnr; ++u) keys[u] = fkey(s.vals[min(i0 + u * kThreads + threadIdx.x, end - 1)]);
#pragma unroll
    for (int u = 0; u < kUnr; ++u) {
      if (i0 + u * kThreads + threadIdx.x >= end) continue;
      const uint32_t key = keys[u];
      const uint32_t d = (key >> shift) & dmask;
      if (a0 && (key & e0.mask) == e0.prefix) atomicAdd(&h[0][d], 1u);
      if (!same && a1 && (key & e1.mask) == e1.prefix) atomicAdd(&h[1][d], 1u);
    }
  }
  __syncthreads();
  uint32_t* g = hist + (size_t)sid * 2 * kBins;
  for (int i = threadIdx.x; i < 2 * kBins; i += kThreads) {
    const uint32_t v = same ? h[0][i & (kBins - 1)] : (&h[0][0])[i];
    if (v) atomicAdd(&g[i], v);
  }
}

// Finds, per (segment, end), the digit holding the need-th entry, fixes it in
// the prefix, and clears the histogram for the next pass.
__global__ __launch_bounds__(kThreads) void digit_scan(EndState* __restrict__ st,
                                                      uint32_t* __restrict__ hist,
                                                      int shift, uint32_t dmask) {
  const int sid = blockIdx.x >> 1;
  const int e = blockIdx.x & 1;
  uint32_t* h = hist + (size_t)sid * 2 * kBins + (size_t)e * kBins;
  EndState es = st[2 * sid + e];
  __shared__ uint32_t part[kThreads];
  __shared__ uint32_t sel[3];
  constexpr int per = kBins / kThreads;  // 8 bins per thread
  const int nb = (int)dmask + 1;
  // ascending order of digits for the bottom end, descending for the top
  uint32_t v[per];
  uint32_t tot = 0;
  for (int j = 0; j < per; ++j) {
    const int pos = threadIdx.x * per + j;  // position in scan order
    const int bin = e == 0 ? pos : (nb - 1 - pos);
    v[j] = (pos < nb) ? h[bin] : 0u;
    tot += v[j];
  }
  part[threadIdx.x] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int t = 0; t < kThreads; ++t) {
      const uint32_t x = part[t];
      part[t] = acc;
      acc += x;
    }
  }
  __syncthreads();
  const bool live = es.active && !es.buf;
  if (live) {
    uint32_t acc = part[threadIdx.x];
    const uint32_t need = (uint32_t)es.need;
    for (int j = 0; j < per; ++j) {
      if (acc < need && acc + v[j] >= need) {
        const int pos = threadIdx.x * per + j;
        sel[0] = (uint32_t)(e == 0 ? pos : (nb - 1 - pos));
        sel[1] = acc;
        sel[2] = v[j];
      }
      acc += v[j];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && live) {
    es.prefix |= sel[0] << shift;
    es.mask |= dmask << shift;
    es.need -= (int32_t)sel[1];
    es.eq = (int32_t)sel[2];
    if (shift == 10) es.buf = es.eq <= kBufCap ? 1 : 0;
    st[2 * sid + e] = es;
  }
  for (int i = threadIdx.x; i < kBins; i += kThreads) h[i] = 0u;
}

// Number of entries equal to the located key, per chunk and end.
__global__ __launch_bounds__(kThreads) void tie_count(const SegPack P,
                                                     const EndState* __restrict__ st,
                                                     uint32_t* __restrict__ tcnt,
                                                     int nchunks) {
  const SegDev s = P.s[blockIdx.y];
  const int sid = P.base + blockIdx.y;
  const int64_t n = seg_len(s);
  const int64_t base = (int64_t)blockIdx.x * kMarkChunk;
  __shared__ uint32_t c[2];
  if (threadIdx.x < 2) c[threadIdx.x] = 0u;
  __syncthreads();
  const EndState e0 = st[2 * sid], e1 = st[2 * sid + 1];
  // ends whose ties all fit (need == eq) take them without ranking: no count
  const bool c0 = e0.active && !e0.buf && e0.need < e0.eq, c1 = e1.active && !e1.buf && e1.need < e1.eq;
  uint32_t m0 = 0, m1 = 0;
  const int64_t end = min(n, base + kMarkChunk);
  if (c0 || c1) {
    for (int64_t i0 = base; i0 < end; i0 += (int64_t)kThreads * kUnr) {
      uint32_t keys[kUnr];
#pragma unroll
      for (int u = 0; u < kUnr; ++u) keys[u] = fkey(s.vals[min(i0 + u * kThreads + threadIdx.x, end - 1)]);
#pragma unroll
      for (int u = 0; u < kUnr; ++u) {
        const bool in = i0 + u * kThreads + threadIdx.x < end;
        m0 += (in && c0 && keys[u] == e0.prefix);
        m1 += (in && c1 && keys[u] == e1.prefix);
      }
    }
  }
  if (m0) atomicAdd(&c[0], m0);
  if (m1) atomicAdd(&c[1], m1);
  __syncthreads();
  if (threadIdx.x < 2) tcnt[((size_t)sid * 2 + threadIdx.x) * nchunks + blockIdx.x] = c[threadIdx.x];
}

// Exclusive prefix over chunks (per segment and end), in place.
__device__ __forceinline__ void chunk_scan_body(uint32_t* __restrict__ c, int nchunks,
                                                int64_t* __restrict__ total, int64_t cap) {
  __shared__ uint32_t part[kThreads];
  const int per = (nchunks + kThreads - 1) / kThreads;
  uint32_t s = 0;
  for (int j = 0; j < per; ++j) {
    const int i = threadIdx.x * per + j;
    if (i < nchunks) s += c[i];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int t = 0; t < kThreads; ++t) {
      const uint32_t x = part[t];
      part[t] = acc;
      acc += x;
    }
    if (total) *total = (int64_t)acc < cap ? (int64_t)acc : cap;
  }
  __syncthreads();
  uint32_t acc = part[threadIdx.x];
  for (int j = 0; j < per; ++j) {
    const int i = threadIdx.x * per + j;
    if (i < nchunks) {
      const uint32_t x = c[i];
      c[i] = acc;
      acc += x;
    }
  }
}

__global__ __launch_bounds__(kThreads) void chunk_scan(uint32_t* __restrict__ cnt, int nchunks,
                                                      int64_t* __restrict__ total, int64_t cap) {
  chunk_scan_body(cnt + (size_t)blockIdx.x * nchunks, nchunks, total ? total + blockIdx.x : nullptr, cap);
}

// Block-wide exclusive prefix of a 0/1 predicate in thread order; returns the
// prefix for this thread and writes the block total to *tot.
__device__ __forceinline__ uint32_t block_excl_scan(bool p, uint32_t* wsum, uint32_t* tot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t bal = __ballot(p);
  const uint32_t in_wave = (uint32_t)__popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
  if (lane == 0) wsum[wave] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t x = wsum[w];
    before += (w < wave) ? x : 0u;
    all += x;
  }
  *tot = all;
  __syncthreads();
  return before + in_wave;
}

__global__ __launch_bounds__(kThreads) void mark(const SegPack P,
                                                const EndState* __restrict__ st,
                                                const uint32_t* __restrict__ toff,
                                                int nchunks, int32_t* __restrict__ bufn,
                                                unsigned long long* __restrict__ bufv) {
  const SegDev s = P.s[blockIdx.y];
  const int sid = P.base + blockIdx.y;
  const int64_t n = seg_len(s);
  const int64_t base = (int64_t)blockIdx.x * kMarkChunk;
  if (base >= n) return;
  const EndState e0 = st[2 * sid], e1 = st[2 * sid + 1];
  if (!e0.active && !e1.active) return;
  // buffered ends: keep what lies strictly beyond the 22-bit prefix, collect
  // what shares it
  const bool b0 = e0.active && e0.buf, b1 = e1.active && e1.buf;
  auto buffered = [&](uint32_t key, int64_t i) {
    bool keep = false;
    if (b0) {
      const uint32_t m = key & e0.mask;
      keep |= m < e0.prefix;
      if (m == e0.prefix) {
        const int32_t at = atomicAdd(&bufn[2 * sid], 1);
        if (at < kBufCap)
          bufv[(size_t)(2 * sid) * kBufCap + at] = ((unsigned long long)key << 32) | (uint32_t)i;
      }
    }
    if (b1) {
      const uint32_t m = key & e1.mask;
      keep |= m > e1.prefix;
      if (m == e1.prefix) {
        const int32_t at = atomicAdd(&bufn[2 * sid + 1], 1);
        if (at < kBufCap)
          bufv[(size_t)(2 * sid + 1) * kBufCap + at] = ((unsigned long long)(~key) << 32) | (uint32_t)i;
      }
    }
    return keep;
  };
  const bool c0 = e0.active && !e0.buf, c1 = e1.active && !e1.buf;   // classic ends
  if ((!c0 || e0.need >= e0.eq) && (!c1 || e1.need >= e1.eq)) {
    // every tie of a classic end fits: keep key <= k-th key (bottom) and
    // key >= k-th key (top), no ranking
    const int64_t end = min(n, base + kMarkChunk);
    for (int64_t i0 = base; i0 < end; i0 += (int64_t)kThreads * kUnr) {
      uint32_t keys[kUnr];
#pragma unroll
      for (int u = 0; u < kUnr; ++u) keys[u] = fkey(s.vals[min(i0 + u * kThreads + threadIdx.x, end - 1)]);
#pragma unroll
      for (int u = 0; u < kUnr; ++u) {
        const int64_t i = i0 + u * kThreads + threadIdx.x;
        if (i >= end) continue;
        bool keep = (c0 && keys[u] <= e0.prefix) || (c1 && keys[u] >= e1.prefix);
        if (b0 || b1) keep |= buffered(keys[u], i);
        if (keep) s.flags[i] = 1;
      }
    }
    return;
  }
  __shared__ uint32_t wsum[kThreads / 64];
  uint32_t r0 = toff[((size_t)sid * 2 + 0) * nchunks + blockIdx.x];
  uint32_t r1 = toff[((size_t)sid * 2 + 1) * nchunks + blockIdx.x];
  for (int it = 0; it < kMarkChunk / kThreads; ++it) {
    const int64_t i = base + (int64_t)it * kThreads + threadIdx.x;
    const bool in = i < n;
    const uint32_t key = in ? fkey(s.vals[i]) : 0u;
    const bool t0 = in && c0 && key == e0.prefix;
    const bool t1 = in && c1 && key == e1.prefix;
    uint32_t tot0, tot1;
    const uint32_t p0 = block_excl_scan(t0, wsum, &tot0);
    const uint32_t p1 = block_excl_scan(t1, wsum, &tot1);
    bool keep = false;
    if (in && c0) keep |= key < e0.prefix || (t0 && r0 + p0 < (uint32_t)e0.need);
    if (in && c1) keep |= key > e1.prefix || (t1 && r1 + p1 < (uint32_t)e1.need);
    if (in && (b0 || b1)) keep |= buffered(key, i);
    if (keep) s.flags[i] = 1;
    r0 += tot0;
    r1 += tot1;
  }
}

// The collected entries of each buffered end: an entry is kept when fewer
// than `need` entries of its buffer rank before it (one work-group per
// segment and end; at most kBufCap entries, ranked by counting).
__global__ __launch_bounds__(kThreads) void buf_finish(const SegPack P, const EndState* __restrict__ st,
                                                      const int32_t* __restrict__ bufn,
                                                      const unsigned long long* __restrict__ bufv) {
  const int lid = blockIdx.x >> 1, e = blockIdx.x & 1;
  const int sid = P.base + lid;
  const EndState es = st[2 * sid + e];
  if (!es.active || !es.buf) return;
  const int nb = min(bufn[2 * sid + e], kBufCap);
  __shared__ unsigned long long v[kBufCap];
  for (int j = threadIdx.x; j < nb; j += kThreads) v[j] = bufv[(size_t)(2 * sid + e) * kBufCap + j];
  __syncthreads();
  const SegDev s = P.s[lid];
  for (int j = threadIdx.x; j < nb; j += kThreads) {
    const unsigned long long mine = v[j];
    int rank = 0;
    for (int q = 0; q < nb; ++q) rank += v[q] < mine ? 1 : 0;
    if (rank < es.need) s.flags[(uint32_t)mine] = 1;
  }
}

// ------------------------------------------------------------- compaction
__device__ __forceinline__ void flag_count_body(const uint8_t* __restrict__ f, int64_t hn,
                                                const int64_t* __restrict__ dn,
                                                uint32_t* __restrict__ cnt) {
  const int64_t n = dn ? min(*dn, hn) : hn;
  const int64_t base = (int64_t)blockIdx.x * kMarkChunk;
  uint32_t m = 0;
  for (int64_t i = base + threadIdx.x; i < min(n, base + kMarkChunk); i += kThreads) m += f[i] != 0;
  __shared__ uint32_t c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  if (m) atomicAdd(&c, m);
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

__global__ __launch_bounds__(kThreads) void flag_count(const uint8_t* __restrict__ f, int64_t hn,
                                                      const int64_t* __restrict__ dn,
                                                      uint32_t* __restrict__ cnt) {
  flag_count_body(f, hn, dn, cnt);
}

__device__ __forceinline__ void flag_write_body(const uint8_t* __restrict__ f, int64_t hn,
                                                const int64_t* __restrict__ dn,
                                                const uint32_t* __restrict__ off,
                                                int32_t* __restrict__ idx, int64_t cap) {
  const int64_t n = dn ? min(*dn, hn) : hn;
  const int64_t base = (int64_t)blockIdx.x * kMarkChunk;
  if (base >= n) return;
  __shared__ uint32_t wsum[kThreads / 64];
  uint32_t r = off[blockIdx.x];
  for (int it = 0; it < kMarkChunk / kThreads; ++it) {
    const int64_t i = base + (int64_t)it * kThreads + threadIdx.x;
    const bool p = i < n && f[i] != 0;
    uint32_t tot;
    const uint32_t pre = block_excl_scan(p, wsum, &tot);
    if (p && (int64_t)(r + pre) < cap) idx[r + pre] = (int32_t)i;
    r += tot;
  }
}

__global__ __launch_bounds__(kThreads) void flag_write(const uint8_t* __restrict__ f, int64_t hn,
                                                      const int64_t* __restrict__ dn,
                                                      const uint32_t* __restrict__ off,
                                                      int32_t* __restrict__ idx, int64_t cap) {
  flag_write_body(f, hn, dn, off, idx, cap);
}

// Two flag arrays compacted together (grid y = array; chunk counts of
// array a at cnt + a * nchunks, nchunks covering the longer one).
struct CompactDir {
  const uint8_t* f;
  int64_t n;
  int32_t* idx;
  int64_t cap;
  int64_t* count;
};
struct CompactPair {
  CompactDir d[2];
  uint32_t* cnt;
  int32_t nchunks;
};

__global__ __launch_bounds__(kThreads) void flag_count2(const CompactPair P) {
  const CompactDir d = P.d[blockIdx.y];
  flag_count_body(d.f, d.n, nullptr, P.cnt + (size_t)blockIdx.y * P.nchunks);
}

__global__ __launch_bounds__(kThreads) void chunk_scan2(const CompactPair P) {
  const CompactDir d = P.d[blockIdx.x];
  chunk_scan_body(P.cnt + (size_t)blockIdx.x * P.nchunks, P.nchunks, d.count, d.cap);
}

__global__ __launch_bounds__(kThreads) void flag_write2(const CompactPair P) {
  const CompactDir d = P.d[blockIdx.y];
  flag_write_body(d.f, d.n, nullptr, P.cnt + (size_t)blockIdx.y * P.nchunks, d.idx, d.cap);
}

// flags[idx[i]] = 1 for i < *count
__global__ void scatter_flags(const int32_t* __restrict__ idx, const int64_t* __restrict__ count,
                              int64_t cap, uint8_t* __restrict__ flags) {
  const int64_t n = min(*count, cap);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flags[idx[i]] = 1;
}

__global__ void zero_kernel(uint32_t* __restrict__ p, size_t words, uint8_t* __restrict__ tail,
                            int tail_bytes) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < tail_bytes) tail[threadIdx.x] = 0;
}

// ------------------------------------------------ batched (one WG / segment)
// For many short segments (up to a few 10^5 values each) one work-group per
// segment does the whole selection with LDS histograms: three digit passes
// (11/11/10 bits) fix the k-th key from each end (the high end uses the
// complemented key, so equal values still rank by index), then one pass
// marks.  Entries equal to the k-th key are all taken when they fit; only
// otherwise a second, index-ordered pass ranks them (ties to the smaller
// index, as in the multi-launch selection).
constexpr int kSegT = 256;
constexpr int kSegBins = 2048;
constexpr int kSegUnr = 8;   // loads in flight per thread in the streaming passes
constexpr int kSegBufCap = 512;   // collected entries per end (LDS)

// Exclusive prefix over the work-group (NT threads); *total gets the sum.
template <int NT>
__device__ __forceinline__ uint32_t wg_excl_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint32_t t = lds[w];
    base += (w < wave) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// Selection of one segment by one work-group (LDS scratch passed in); the
// caller runs it uniformly over the work-group.
template <int NT>
__device__ __forceinline__ void select_seg_body(const SegJob& j, uint32_t (*hist)[kSegBins],
                                                uint32_t* scan_lds, uint32_t* s_bin,
                                                uint32_t* s_before,
                                                unsigned long long (*sbuf)[kSegBufCap],
                                                uint32_t* sbn) {
  const int tid = threadIdx.x;
  int64_t n = j.dn ? *j.dn : j.n;
  n = n < j.n ? (n > 0 ? n : 0) : j.n;
  const uint32_t k[2] = {(uint32_t)min<int64_t>(j.lo, n), (uint32_t)min<int64_t>(j.hi, n)};
  if (n == 0 || (k[0] == 0 && k[1] == 0)) return;
  uint32_t pre[2] = {0u, 0u}, rem[2] = {k[0], k[1]}, eq[2] = {0u, 0u};
  // buffered end: after the second digit at most kSegBufCap entries share
  // its 22-bit prefix; the mark pass collects them in LDS and ranks them,
  // and the third digit is skipped
  bool buf[2] = {false, false};
  const int shifts[3] = {21, 10, 0};
  const uint32_t masks[3] = {0x7FFu, 0x7FFu, 0x3FFu};
  const uint32_t pmasks[3] = {0u, 0xFFE00000u, 0xFFFFFC00u};
  for (int p = 0; p < 3; ++p) {
    if (p == 2 && (!k[0] || buf[0]) && (!k[1] || buf[1])) break;   // uniform
    __syncthreads();
    for (int b = tid; b < 2 * kSegBins; b += NT) (&hist[0][0])[b] = 0u;
    __syncthreads();
    // kSegUnr loads in flight per thread (indices clamped, so the loads are
    // unconditional), then their histogram updates
    for (int64_t i0 = 0; i0 < n; i0 += (int64_t)NT * kSegUnr) {
      uint32_t keys[kSegUnr];
#pragma unroll
      for (int u = 0; u < kSegUnr; ++u) keys[u] = fkey(j.vals[min(i0 + u * NT + tid, n - 1)]);
#pragma unroll
      for (int u = 0; u < kSegUnr; ++u) {
        if (i0 + u * NT + tid >= n) continue;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const uint32_t ke = e ? ~keys[u] : keys[u];
          if (k[e] && !buf[e] && (ke & pmasks[p]) == pre[e])
            atomicAdd(&hist[e][(ke >> shifts[p]) & masks[p]], 1u);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (!k[e] || buf[e]) continue;   // uniform
      uint32_t loc = 0;
#pragma unroll
      for (int b = 0; b < kSegBins / NT; ++b) loc += hist[e][tid * (kSegBins / NT) + b];
      uint32_t tot;
      const uint32_t ex = wg_excl_scan<NT>(loc, scan_lds, &tot);
      if (ex < rem[e] && rem[e] <= ex + loc) {
        uint32_t acc = ex;
        for (int b = 0; b < kSegBins / NT; ++b) {
          const int bin = tid * (kSegBins / NT) + b;
          const uint32_t h = hist[e][bin];
          if (acc + h >= rem[e]) {
            s_bin[e] = (uint32_t)bin;
            s_before[e] = acc;
            break;
          }
          acc += h;
        }
      }
      __syncthreads();
      pre[e] |= s_bin[e] << shifts[p];
      rem[e] -= s_before[e];
      if (p >= 1) eq[e] = hist[e][s_bin[e]];
      if (p == 1) buf[e] = eq[e] <= (uint32_t)kSegBufCap;
      __syncthreads();
    }
  }
  // mark: below the k-th key, and ties when all of them fit
  bool ordered[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) ordered[e] = k[e] && !buf[e] && rem[e] < eq[e];
  if (tid < 2) sbn[tid] = 0u;
  __syncthreads();
  for (int64_t i0 = 0; i0 < n; i0 += (int64_t)NT * kSegUnr) {
    uint32_t keys[kSegUnr];
#pragma unroll
    for (int u = 0; u < kSegUnr; ++u) keys[u] = fkey(j.vals[min(i0 + u * NT + tid, n - 1)]);
#pragma unroll
    for (int u = 0; u < kSegUnr; ++u) {
      const int64_t i = i0 + u * NT + tid;
      bool f = false;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const uint32_t ke = e ? ~keys[u] : keys[u];
        if (k[e] && !buf[e]) f |= ke < pre[e] || (ke == pre[e] && !ordered[e]);
        if (k[e] && buf[e] && i < n) {
          const uint32_t m = ke & 0xFFFFFC00u;
          f |= m < pre[e];
          if (m == pre[e]) {
            const uint32_t at = atomicAdd(&sbn[e], 1u);
            if (at < (uint32_t)kSegBufCap) sbuf[e][at] = ((unsigned long long)ke << 32) | (uint32_t)i;
          }
        }
      }
      if (f && i < n) j.flags[i] = 1;
    }
  }
  // buffered ends: an entry is kept when fewer than rem entries of its
  // buffer rank before it (composites: key, then index)
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if (!k[e] || !buf[e]) continue;   // uniform
    const uint32_t nb = min(sbn[e], (uint32_t)kSegBufCap);
    for (uint32_t q = tid; q < nb; q += NT) {
      const unsigned long long mine = sbuf[e][q];
      uint32_t rank = 0;
      for (uint32_t r = 0; r < nb; ++r) rank += sbuf[e][r] < mine ? 1u : 0u;
      if (rank < rem[e]) j.flags[(uint32_t)mine] = 1;
    }
  }
  // ties that do not all fit: rank them in index order
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if (!ordered[e]) continue;   // uniform
    uint32_t taken = 0;
    for (int64_t c0 = 0; c0 < n; c0 += NT) {
      const int64_t i = c0 + tid;
      bool tie = false;
      if (i < n) {
        const uint32_t key = fkey(j.vals[i]);
        tie = (e ? ~key : key) == pre[e];
      }
      uint32_t tot;
      const uint32_t ex = wg_excl_scan<NT>(tie ? 1u : 0u, scan_lds, &tot);
      if (tie && taken + ex < rem[e]) j.flags[i] = 1;
      taken += tot;
      if (taken >= rem[e]) break;   // uniform
    }
  }
}

__global__ __launch_bounds__(kSegT) void select_seg(const SegJob* __restrict__ jobs, int njobs) {
  __shared__ uint32_t hist[2][kSegBins];
  __shared__ uint32_t scan_lds[kSegT / 64];
  __shared__ uint32_t s_bin[2], s_before[2];
  __shared__ unsigned long long sbuf[2][kSegBufCap];
  __shared__ uint32_t sbn[2];
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const SegJob j = jobs[it];
    select_seg_body<kSegT>(j, hist, scan_lds, s_bin, s_before, sbuf, sbn);
  }
}

// Compaction of one flag array into ascending indices (at most cap) and its
// count; one work-group per job.
template <int NT>
__device__ __forceinline__ void compact_seg_body(const CompactJob& j, uint32_t* scan_lds) {
  const int tid = threadIdx.x;
  int64_t n = j.dn ? *j.dn : j.n;
  n = n < j.n ? (n > 0 ? n : 0) : j.n;
  // 16 consecutive flags per thread per chunk (loads clamped, so all 16 are
  // in flight together), one work-group scan per chunk
  constexpr int Q = 16;
  int64_t base = 0;
  for (int64_t c0 = 0; c0 < n; c0 += Q * NT) {
    uint8_t fb[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) fb[q] = j.flags[min(c0 + Q * tid + q, n - 1)];
    uint32_t f = 0, cnt = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const bool on = c0 + Q * tid + q < n && fb[q];
      f |= (on ? 1u : 0u) << q;
      cnt += on ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t pos = wg_excl_scan<NT>(cnt, scan_lds, &tot);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if ((f >> q) & 1u) {
        const int64_t o = base + pos;
        if (o < j.cap) j.idx[o] = (int32_t)(c0 + Q * tid + q);
        ++pos;
      }
    }
    base += tot;
  }
  if (tid == 0) *j.count = base < j.cap ? base : j.cap;
}

__global__ __launch_bounds__(kSegT) void compact_seg(const CompactJob* __restrict__ jobs, int njobs) {
  __shared__ uint32_t scan_lds[kSegT / 64];
  for (int it = blockIdx.x; it < njobs; it += gridDim.x) {
    const CompactJob j = jobs[it];
    __syncthreads();
    compact_seg_body<kSegT>(j, scan_lds);
  }
}

// The k <= 64 largest keys of an array under the order above (larger key
// first; equal keys: smaller index first), in two launches.  An entry
// becomes one 64-bit composite, the order-preserving key in the high word
// and the complemented index in the low word, so composites are distinct
// and compare in that order; 0 marks an empty slot (the low word of a real
// entry is at least 2^31).  Every wave reduces blocks of 64 x kTopR entries
// to the 64 largest composites seen so far with bitonic networks across its
// lanes (each register of 64 entries sorted, then sorted lists merged
// pairwise, keeping the larger half).  The second launch merges the waves'
// lists the same way in one work-group per array and writes the k indices
// in ascending order with their count.
constexpr int kTopR = 8;                  // entries per lane per block
constexpr int kTopBlock = 64 * kTopR;     // entries per wave per block
constexpr int kTopMaxWaves = 1024;        // wave lists per array
constexpr int kTopT = 256;                // first launch: 4 waves per work-group
constexpr int kTopFinalT = 1024;          // second launch: 16 waves
constexpr int kTopFinalR = 16;            // its lists per wave per block

struct TopDev {
  const uint32_t* keys;
  const int64_t* dev_n;
  int64_t n;
  int32_t* idx;
  int64_t* count;
  int32_t k;
};
struct TopPack {
  TopDev s[2];
  unsigned long long* part;   // [nseg][nwaves][64] wave lists
  int32_t nwaves;             // per array (a multiple of 4)
  int32_t nseg;
};

__device__ __forceinline__ int64_t top_len(const TopDev& t) {
  const int64_t n = t.dev_n ? min(*t.dev_n, t.n) : t.n;
  return n > 0 ? n : 0;
}

__device__ __forceinline__ unsigned long long top_comp(uint32_t bits, int64_t i) {
  return ((unsigned long long)fkey(__uint_as_float(bits)) << 32) |
         (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
}

// Lane l's value from lane l ^ J (both words): DPP for J = 1, 2 (quad
// permutes) and 8 (rotation by 8 within a row of 16 lanes), a cross-lane
// permute otherwise.  All lanes active.
template <int J>
__device__ __forceinline__ unsigned long long lane_xor(unsigned long long x) {
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  uint32_t l2, h2;
  if constexpr (J == 1 || J == 2 || J == 8) {
    constexpr int CTRL = J == 1 ? 0xB1 : (J == 2 ? 0x4E : 0x128);
    l2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, CTRL, 0xF, 0xF, true);
    h2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, CTRL, 0xF, 0xF, true);
  } else {
    l2 = __shfl_xor(lo, J);
    h2 = __shfl_xor(hi, J);
  }
  return ((unsigned long long)h2 << 32) | l2;
}

// Compare-exchange with lane l ^ J: the lower lane of the pair keeps the
// larger value in a descending run (the smaller in an ascending one).
template <int J>
__device__ __forceinline__ unsigned long long cx(unsigned long long x, int lane, bool desc) {
  const unsigned long long y = lane_xor<J>(x);
  const bool keep_max = ((lane & J) == 0) == desc;
  return keep_max == (x > y) ? x : y;
}

// A bitonic sequence across the 64 lanes into descending (DESC) or
// ascending order.
template <bool DESC>
__device__ __forceinline__ unsigned long long bitonic_merge(unsigned long long x, int lane) {
  x = cx<32>(x, lane, DESC);
  x = cx<16>(x, lane, DESC);
  x = cx<8>(x, lane, DESC);
  x = cx<4>(x, lane, DESC);
  x = cx<2>(x, lane, DESC);
  return cx<1>(x, lane, DESC);
}

// Any 64 values across the lanes into descending (DESC) or ascending order:
// runs of K = 2, 4, .., 32 lanes sorted in alternating directions (the
// run's direction is DESC where lane & K is 0), each pair of runs then
// merged as one bitonic run of 2K.
template <bool DESC>
__device__ __forceinline__ unsigned long long bitonic_sort(unsigned long long x, int lane) {
  bool d = ((lane & 2) == 0) == DESC;
  x = cx<1>(x, lane, d);
  d = ((lane & 4) == 0) == DESC;
  x = cx<2>(x, lane, d);
  x = cx<1>(x, lane, d);
  d = ((lane & 8) == 0) == DESC;
  x = cx<4>(x, lane, d);
  x = cx<2>(x, lane, d);
  x = cx<1>(x, lane, d);
  d = ((lane & 16) == 0) == DESC;
  x = cx<8>(x, lane, d);
  x = cx<4>(x, lane, d);
  x = cx<2>(x, lane, d);
  x = cx<1>(x, lane, d);
  d = ((lane & 32) == 0) == DESC;
  x = cx<16>(x, lane, d);
  x = cx<8>(x, lane, d);
  x = cx<4>(x, lane, d);
  x = cx<2>(x, lane, d);
  x = cx<1>(x, lane, d);
  return bitonic_merge<DESC>(x, lane);
}

// The 64 largest of R >= 2 sorted lists across the lanes (list q descending
// for even q, ascending for odd q), descending (DESC) or ascending.  The
// lane-wise larger of a descending and an ascending list is a bitonic
// sequence holding the 64 largest of the two; pairs are merged level by
// level, the results again alternating in direction.
template <int R, bool DESC>
__device__ __forceinline__ unsigned long long top64_lists(unsigned long long (&e)[R], int lane) {
  static_assert(R >= 2 && (R & (R - 1)) == 0, "R: a power of two, at least 2");
#pragma unroll
  for (int w = R; w > 1; w >>= 1) {
#pragma unroll
    for (int q = 0; q < w / 2; ++q) {
      const unsigned long long a = e[2 * q], b = e[2 * q + 1];
      const unsigned long long c = a > b ? a : b;
      const bool d = w == 2 ? DESC : (q & 1) == 0;
      e[q] = d ? bitonic_merge<true>(c, lane) : bitonic_merge<false>(c, lane);
    }
  }
  return e[0];
}

// One block of a wave: the 64 largest of its R x 64 unsorted entries e and
// its carried list c (descending), descending: lane l gets the l-th largest
// (0 where fewer than l + 1 entries are non-empty).  Called by the whole
// wave.
template <int R>
__device__ __forceinline__ unsigned long long block_top64(unsigned long long (&e)[R],
                                                          unsigned long long c, int lane) {
#pragma unroll
  for (int q = 0; q < R; ++q)
    e[q] = (q & 1) == 0 ? bitonic_sort<true>(e[q], lane) : bitonic_sort<false>(e[q], lane);
  const unsigned long long t = top64_lists<R, false>(e, lane);
  return bitonic_merge<true>(c > t ? c : t, lane);
}

// The same for R sorted lists (alternating directions, as top64_lists).
template <int R>
__device__ __forceinline__ unsigned long long lists_top64(unsigned long long (&e)[R],
                                                          unsigned long long c, int lane) {
  const unsigned long long t = top64_lists<R, false>(e, lane);
  return bitonic_merge<true>(c > t ? c : t, lane);
}

__global__ __launch_bounds__(kTopT) void top_part(const TopPack P) {
  const TopDev t = P.s[blockIdx.y];
  const int64_t n = top_len(t);
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (kTopT / 64) + (threadIdx.x >> 6);
  // wave gw takes the blocks gw, gw + nwaves, ... (loads clamped, so the
  // R loads of a lane are unconditional and in flight together)
  const int64_t nblk = (n + kTopBlock - 1) / kTopBlock;
  unsigned long long best = 0;
  for (int64_t b = gw; b < nblk; b += P.nwaves) {
    unsigned long long e[kTopR];
#pragma unroll
    for (int q = 0; q < kTopR; ++q) {
      const int64_t i = b * kTopBlock + q * 64 + lane;
      const uint32_t bits = t.keys[min(i, n - 1)];
      e[q] = i < n ? top_comp(bits, i) : 0ull;
    }
    best = block_top64<kTopR>(e, best, lane);
  }
  P.part[((size_t)blockIdx.y * P.nwaves + gw) * 64 + lane] = best;
}

__global__ __launch_bounds__(kTopFinalT) void top_final(const TopPack P) {
  __shared__ unsigned long long lists[kTopFinalT / 64][64];
  const TopDev t = P.s[blockIdx.x];
  const unsigned long long* part = P.part + (size_t)blockIdx.x * P.nwaves * 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave w merges the lists w R, .., w R + R - 1, then (w + 16) R, ..; odd
  // lists of a block are read back to front (ascending)
  constexpr int R = kTopFinalR;
  const int nblk = (P.nwaves + R - 1) / R;
  unsigned long long best = 0;
  for (int b = wave; b < nblk; b += kTopFinalT / 64) {
    unsigned long long e[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int g = b * R + q;
      const unsigned long long v = part[(size_t)min(g, P.nwaves - 1) * 64 + ((q & 1) ? 63 - lane : lane)];
      e[q] = g < P.nwaves ? v : 0ull;
    }
    best = lists_top64<R>(e, best, lane);
  }
  lists[wave][lane] = best;
  __syncthreads();
  if (wave != 0) return;
  unsigned long long e[kTopFinalT / 64];
#pragma unroll
  for (int q = 0; q < kTopFinalT / 64; ++q) e[q] = lists[q][(q & 1) ? 63 - lane : lane];
  const unsigned long long top = top64_lists<kTopFinalT / 64, true>(e, lane);
  const int64_t n = top_len(t);
  const int k = (int)min<int64_t>(t.k, n);
  // lanes below k hold the k largest; their indices in ascending order
  const bool on = lane < k;
  const uint32_t idx = on ? 0xFFFFFFFFu - (uint32_t)top : 0xFFFFFFFFu;
  int rank = 0;
  for (int j = 0; j < 64; ++j) rank += __shfl(idx, j) < idx ? 1 : 0;
  if (on) t.idx[rank] = (int32_t)idx;
  if (lane == 0) *t.count = k;
}

int top_waves(int64_t max_n) {
  const int64_t w = std::min<int64_t>(kTopMaxWaves, std::max<int64_t>(1, cdiv(max_n, kTopBlock)));
  return (int)cdiv(w, 4) * 4;
}

struct SelLayout {
  EndState* st;
  uint32_t* hist;
  uint32_t* tie;
  int32_t* bufn;                 // [nseg][2] collected entries
  unsigned long long* bufv;      // [nseg][2][kBufCap]
  int nchunks;
};

SelLayout sel_layout(Arena& ar, int nseg, int64_t max_n) {
  SelLayout L;
  L.nchunks = (int)std::max<int64_t>(1, cdiv(max_n, kMarkChunk));
  L.st = ar.take<EndState>(2 * nseg);
  L.hist = ar.take<uint32_t>((size_t)nseg * 2 * kBins);
  L.tie = ar.take<uint32_t>((size_t)nseg * 2 * L.nchunks);
  L.bufn = ar.take<int32_t>(2 * nseg);
  L.bufv = ar.take<unsigned long long>((size_t)2 * nseg * kBufCap);
  return L;
}

}  // namespace

size_t select_ws_bytes(int nseg, int64_t max_n) {
  Arena ar(nullptr);
  sel_layout(ar, nseg, max_n);
  return ar.used + 256;
}

prohd_status select_mark(const SelSegment* segs, int nseg, void* ws, size_t ws_bytes,
                         hipStream_t s) {
  if (nseg <= 0) return PROHD_OK;
  int64_t max_n = 1;
  for (int i = 0; i < nseg; ++i) max_n = std::max<int64_t>(max_n, segs[i].n);
  Arena ar(ws);
  SelLayout L = sel_layout(ar, nseg, max_n);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "select: workspace too small");
  const int hchunks = (int)std::max<int64_t>(1, cdiv(max_n, kHistChunk));
  const int shifts[3] = {21, 10, 0};
  const uint32_t masks[3] = {0x7FFu, 0x7FFu, 0x3FFu};
  for (int g0 = 0; g0 < nseg; g0 += kSegPerLaunch) {
    SegPack P;
    P.nseg = std::min(kSegPerLaunch, nseg - g0);
    P.base = g0;
    for (int i = 0; i < kSegPerLaunch; ++i) {
      SegDev d{};
      if (i < P.nseg) {
        const SelSegment& q = segs[g0 + i];
        d.vals = q.vals;
        d.dev_n = q.dev_n;
        d.n = q.n;
        d.flags = q.flags;
        d.lo = q.lo;
        d.hi = q.hi;
      }
      P.s[i] = d;
    }
    const int ns = P.nseg;
    PROHD_LAUNCH("select_init", init_state, dim3(ns), dim3(kThreads), 0, s, P, L.st, L.hist, L.bufn);
    for (int p = 0; p < 3; ++p) {
      PROHD_LAUNCH("select_hist", digit_hist, dim3(hchunks, ns), dim3(kThreads), 0, s, P, L.st,
                   L.hist, shifts[p], masks[p]);
      PROHD_LAUNCH("select_scan", digit_scan, dim3(2 * ns), dim3(kThreads), 0, s,
                   L.st + 2 * g0, L.hist + (size_t)g0 * 2 * kBins, shifts[p], masks[p]);
    }
    PROHD_LAUNCH("select_ties", tie_count, dim3(L.nchunks, ns), dim3(kThreads), 0, s, P, L.st,
                 L.tie, L.nchunks);
    PROHD_LAUNCH("select_tiescan", chunk_scan, dim3(2 * ns), dim3(kThreads), 0, s,
                 L.tie + (size_t)g0 * 2 * L.nchunks, L.nchunks, (int64_t*)nullptr, (int64_t)0);
    PROHD_LAUNCH("select_mark", mark, dim3(L.nchunks, ns), dim3(kThreads), 0, s, P, L.st, L.tie,
                 L.nchunks, L.bufn, L.bufv);
    PROHD_LAUNCH("select_buf", buf_finish, dim3(2 * ns), dim3(kThreads), 0, s, P, L.st, L.bufn, L.bufv);
  }
  return PROHD_OK;
}

size_t compact_ws_bytes(int64_t n) {
  Arena ar(nullptr);
  ar.take<uint32_t>((size_t)2 * std::max<int64_t>(1, cdiv(n, kMarkChunk)));   // room for a pair
  return ar.used + 256;
}

prohd_status compact_flags2(const uint8_t* fA, int64_t nA, int32_t* idxA, int64_t capA, int64_t* countA,
                            const uint8_t* fB, int64_t nB, int32_t* idxB, int64_t capB, int64_t* countB,
                            void* ws, size_t ws_bytes, hipStream_t s) {
  CompactPair P{};
  P.nchunks = (int)std::max<int64_t>(1, cdiv(std::max(nA, nB), kMarkChunk));
  Arena ar(ws);
  P.cnt = ar.take<uint32_t>((size_t)2 * P.nchunks);
  if (ar.used > ws_bytes) return fail(PROHD_EWORKSPACE, "compact: workspace too small");
  P.d[0] = CompactDir{fA, nA, idxA, capA, countA};
  P.d[1] = CompactDir{fB, nB, idxB, capB, countB};
  PROHD_LAUNCH("compact_count", flag_count2, dim3(P.nchunks, 2), dim3(kThreads), 0, s, P);
  PROHD_LAUNCH("compact_scan", chunk_scan2, dim3(2), dim3(kThreads), 0, s, P);
  PROHD_LAUNCH("compact_write", flag_write2, dim3(P.nchunks, 2), dim3(kThreads), 0, s, P);
  return PROHD_OK;
}

prohd_status scatter_index_flags(const int32_t* idx, const int64_t* count, int64_t cap, uint8_t* flags,
                                 hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(cap, 256), 1024));
  PROHD_LAUNCH("select_scatter", scatter_flags, dim3(grid), dim3(256), 0, s, idx, count, cap, flags);
  return PROHD_OK;
}

size_t topk_ws_bytes(int64_t max_n) {
  return (size_t)2 * top_waves(max_n) * 64 * sizeof(unsigned long long) + 256;
}

prohd_status top_keys(const TopSegment* segs, int nseg, void* ws, size_t ws_bytes, hipStream_t s) {
  if (nseg <= 0) return PROHD_OK;
  if (nseg > 2) return fail(PROHD_EINVAL, "top_keys: at most 2 arrays");
  int64_t max_n = 1;
  for (int i = 0; i < nseg; ++i) {
    if (segs[i].k < 0 || segs[i].k > 64) return fail(PROHD_EINVAL, "top_keys: k outside [0, 64]");
    if (segs[i].n > INT32_MAX) return fail(PROHD_EINVAL, "top_keys: more than 2^31 - 1 entries");
    max_n = std::max<int64_t>(max_n, segs[i].n);
  }
  TopPack P{};
  P.nwaves = top_waves(max_n);
  P.nseg = nseg;
  if ((size_t)nseg * P.nwaves * 64 * sizeof(unsigned long long) > ws_bytes)
    return fail(PROHD_EWORKSPACE, "top_keys: workspace too small");
  P.part = static_cast<unsigned long long*>(ws);
  for (int i = 0; i < nseg; ++i) {
    const TopSegment& g = segs[i];
    P.s[i] = TopDev{g.keys, g.dev_n, g.n, g.idx, g.count, g.k};
  }
  PROHD_LAUNCH("top_part", top_part, dim3(P.nwaves / (kTopT / 64), nseg), dim3(kTopT), 0, s, P);
  PROHD_LAUNCH("top_final", top_final, dim3(nseg), dim3(kTopFinalT), 0, s, P);
  return PROHD_OK;
}

prohd_status zero_bytes(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return PROHD_OK;
  // Workspace carve-outs are 256-byte aligned; whole words first, then bytes.
  const size_t words = bytes / 4;
  const int tail = (int)(bytes - words * 4);
  const int grid = (int)std::min<size_t>(4096, std::max<size_t>(1, cdiv((int64_t)words, 256 * 4)));
  PROHD_LAUNCH("zero", zero_kernel, dim3(grid), dim3(256), 0, s, (uint32_t*)p, words,
               (uint8_t*)p + words * 4, tail);
  return PROHD_OK;
}

prohd_status batch_select(const SegJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  const int grid = std::min(njobs, 16 * cu_count());
  PROHD_LAUNCH("batch_select", select_seg, dim3(grid), dim3(kSegT), 0, s, jobs, njobs);
  return PROHD_OK;
}

prohd_status batch_compact(const CompactJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return PROHD_OK;
  const int grid = std::min(njobs, 16 * cu_count());
  PROHD_LAUNCH("batch_compact", compact_seg, dim3(grid), dim3(kSegT), 0, s, jobs, njobs);
  return PROHD_OK;
}

}  // namespace prohd
