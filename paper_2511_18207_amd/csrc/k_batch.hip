// Batched form: ProHD (Alg. 3 per pair, alpha mode) or the exact distance of
// Eq. (1) for P independent pairs of uneven sizes, with per-pair dimension D.
//
// A plan fixes the pair sizes.  Binding it to concrete buffers (the packed
// point sets, the result array and a workspace) builds the work tables on
// the host, uploads them once, and captures the whole launch sequence into
// one graph on a private stream; a run is then a single graph launch on the
// caller's stream.  Every launch is a persistent kernel (batch.h) that walks
// a table of work items, so small pairs cost a few table entries instead of
// launches.  Pairs are grouped by D (the kernels are specialised on the
// padded width and take D as an argument), and within a group items are
// ordered by decreasing cost so that the static round-robin over
// work-groups ends with small items.
//
// Work shapes (rows per Gram slice, Y rows per distance item, work-groups
// per compute unit of the persistent launches) come from a tuning table;
// prohd_batch_tune measures candidate shapes on the bound batch with the
// library's kernel timers and keeps the fastest.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "batch.h"
#include "common.h"

using namespace prohd;

namespace {



struct Tuning {
  int gram_rows = 6144;   // rows per Gram slice
  int gram_mult = 2;      // Gram work-groups per compute unit
  int proj_mult = 4;      // projection work-groups per compute unit
  int tile_yc = 8192;     // Y rows per distance item
  int tile_mult = 2;      // distance work-groups per compute unit
  int refine_yc = 8192;   // Y rows per refinement item
  int eig_narrow = 0;     // eigensolver work-group: 1 narrow (256 threads), 0 wide (512)
};

struct Pair {
  int64_t nA, nB;
  int32_t D, DP, m;
  int64_t offA, offB;          // element offsets in the packed sets
  int64_t capA, capB;          // selection capacities (ProHD)
  std::vector<int32_t> kA, kB;
};


// per-pair pieces of the workspace
struct PairWs {
  int32_t* status;
  int64_t* cnt;       // [2] selected counts (ProHD)
  uint32_t* hlow;     // [2] largest certified lower bound (squared, float bits) per direction
  int64_t* ccnt2;     // [2] counts of the rows the float64 pass re-measures
  unsigned long long* best2[2];   // float64 pass (one entry per row)
  int32_t* cand2[2];
  uint32_t* row[2];   // row minima (then bound keys) of the A side / B side rows
  float* xp[2];       // prepared rows (DP wide)
  float* xn[2];
  // ProHD only
  uint8_t* flags[2];
  int32_t* idx[2];
  double* gpart;
  double* spart;
  int nsl[2];
  double* C;
  double* u0;
  double* V;
  double* Y;
  float* dirs;
  float* proj[2];
};

struct Layout {
  std::vector<PairWs> p;
  void* single_ws;          // workspace of the pruned single-pair searches
  size_t single_bytes;
  int32_t* status;
  uint32_t* hlow;
  uint32_t* row;
  int64_t nrow;
  uint8_t* flags;
  int64_t nflags;
};

}  // namespace

struct prohd_batch {
  int32_t P = 0;
  double alpha = 0.01;
  std::vector<Pair> pairs;
  std::vector<int32_t> dims;   // distinct D values, ascending
  Tuning tune;
  // binding
  bool bound = false;
  uint32_t mode = 0;
  const float* A = nullptr;
  const float* B = nullptr;
  prohd_result* out = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* dtab = nullptr;
  size_t dtab_bytes = 0;
  std::vector<std::function<prohd_status(hipStream_t)>> launches;
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // completion of the last run on the caller's stream: a rebuild (new
  // binding or tuning) rewrites or frees the device tables and the graph,
  // which a run still in flight on another stream may be reading
  hipEvent_t done = nullptr;
  bool pending = false;
};

namespace {

// Exact mode: pairs large enough for the pruned search (both sets at least
// 16 384 rows) run it one after another, through the single-pair path, in
// the same launch list; the batched tables hold the others.
bool pruned_pair(const Pair& q, uint32_t mode) {
  return mode == PROHD_BATCH_EXACT && hd_prune_levels(q.nA, q.nB, q.nA, q.nB, PROHD_PRUNE) > 0;
}

int64_t side_rows(const Pair& q, int set, uint32_t mode) {
  if (pruned_pair(q, mode)) return 0;
  if (mode == PROHD_BATCH_EXACT) return set ? q.nB : q.nA;
  return set ? q.capB : q.capA;
}

Layout make_layout(Arena& ar, const prohd_batch& b, uint32_t mode, const Tuning& t) {
  Layout L;
  const int P = b.P;
  L.p.resize(P);
  L.status = ar.take<int32_t>(P);
  int64_t* cnt = ar.take<int64_t>(2 * (size_t)P);
  L.hlow = ar.take<uint32_t>(2 * (size_t)P);
  L.nrow = 0;
  for (const Pair& q : b.pairs) L.nrow += side_rows(q, 0, mode) + side_rows(q, 1, mode);
  L.row = ar.take<uint32_t>(L.nrow);
  int64_t* ccnt2 = ar.take<int64_t>(2 * (size_t)P);
  int32_t* cand2 = ar.take<int32_t>(L.nrow);
  unsigned long long* best2 = ar.take<unsigned long long>(L.nrow);
  L.nflags = 0;
  if (mode == PROHD_BATCH_PROHD)
    for (const Pair& q : b.pairs) L.nflags += q.nA + q.nB;
  L.flags = mode == PROHD_BATCH_PROHD ? ar.take<uint8_t>(L.nflags) : nullptr;
  L.single_bytes = 0;
  for (const Pair& q : b.pairs)
    if (pruned_pair(q, mode))
      L.single_bytes = std::max(L.single_bytes, exact_ws_bytes(q.nA, q.nB, q.D, PROHD_PRUNE));
  L.single_ws = L.single_bytes ? ar.take<char>(L.single_bytes) : nullptr;
  int64_t ro = 0, fo = 0;
  for (int i = 0; i < P; ++i) {
    const Pair& q = b.pairs[i];
    PairWs& w = L.p[i];
    w.status = L.status + i;
    w.cnt = cnt + 2 * i;
    w.hlow = L.hlow + 2 * i;
    w.ccnt2 = ccnt2 + 2 * i;
    for (int s = 0; s < 2; ++s) {
      const int64_t r = side_rows(q, s, mode);
      w.cand2[s] = cand2 + ro;
      w.best2[s] = best2 + ro;
      w.row[s] = L.row + ro;
      ro += r;
      w.xp[s] = ar.take<float>((size_t)r * q.DP);
      w.xn[s] = ar.take<float>(r);
      w.flags[s] = nullptr;
      w.idx[s] = nullptr;
      w.proj[s] = nullptr;
    }
    if (mode == PROHD_BATCH_PROHD) {
      w.flags[0] = L.flags + fo;
      fo += q.nA;
      w.flags[1] = L.flags + fo;
      fo += q.nB;
      w.idx[0] = ar.take<int32_t>(q.capA);
      w.idx[1] = ar.take<int32_t>(q.capB);
      w.nsl[0] = (int)cdiv(q.nA, t.gram_rows);
      w.nsl[1] = (int)cdiv(q.nB, t.gram_rows);
      const int nsl = w.nsl[0] + w.nsl[1];
      w.gpart = ar.take<double>((size_t)nsl * gram_partial_doubles(q.DP));
      w.spart = ar.take<double>((size_t)nsl * 2 * q.DP);
      w.C = ar.take<double>((size_t)q.DP * q.DP);
      w.u0 = ar.take<double>(q.DP);
      w.V = ar.take<double>(eig_job_doubles(q.DP));
      w.Y = w.V + (size_t)q.DP * q.DP;
      w.dirs = ar.take<float>((size_t)(q.m + 1) * q.D);
      w.proj[0] = ar.take<float>((size_t)(q.m + 1) * q.nA);
      w.proj[1] = ar.take<float>((size_t)(q.m + 1) * q.nB);
    }
  }
  return L;
}

// Host tables, concatenated into one device buffer.
struct Tables {
  std::vector<char> host;
  size_t add(const void* p, size_t bytes) {
    const size_t o = (host.size() + 255) / 256 * 256;
    host.resize(o + bytes);
    if (bytes) std::memcpy(host.data() + o, p, bytes);
    return o;
  }
  template <class T>
  size_t add(const std::vector<T>& v) {
    return add(v.data(), v.size() * sizeof(T));
  }
};

prohd_status mark_done(prohd_batch* b, hipStream_t s) {
  if (!b->done && hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
    b->done = nullptr;
    return fail(PROHD_EDEVICE, "batch: cannot create the completion event");
  }
  if (hipEventRecord(b->done, s) != hipSuccess) return fail(PROHD_EDEVICE, "batch: cannot record completion");
  b->pending = true;
  return PROHD_OK;
}

prohd_status wait_done(prohd_batch* b) {
  if (b->pending && b->done) {
    b->pending = false;
    if (hipEventSynchronize(b->done) != hipSuccess) return fail(PROHD_EDEVICE, "batch: previous run failed");
  }
  return PROHD_OK;
}

void release_graph(prohd_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Order pair indices of one D group by decreasing size (largest work first).
std::vector<int> group(const prohd_batch* b, int D) {
  std::vector<int> g;
  for (int i = 0; i < b->P; ++i)
    if (b->pairs[i].D == D) g.push_back(i);
  std::stable_sort(g.begin(), g.end(), [&](int x, int y) {
    return b->pairs[x].nA + b->pairs[x].nB > b->pairs[y].nA + b->pairs[y].nB;
  });
  return g;
}

int persist(int64_t items, int mult) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)mult * cu_count()));
}

// Builds the tables and the launch list for the current binding.
prohd_status build(prohd_batch* b) {
  const uint32_t mode = b->mode;
  const Tuning t = b->tune;
  Arena ar(b->ws);
  Layout L = make_layout(ar, *b, mode, t);
  if (ar.used > b->ws_bytes) return fail(PROHD_EWORKSPACE, "batch: workspace too small");
  Tables T;
  struct Rec {
    int D, DP, m;
    size_t gram_jobs, gram_items, red_jobs, eig_jobs, proj_jobs, seg_jobs, cmp_jobs;
    int n_gram_items, n_red, n_eig, n_proj, n_seg, n_cmp;
    size_t prep_jobs, prep_items, tile_jobs, tile_items, key_jobs, key_items, unc_jobs, ref2_jobs,
        ref2_items, fin_jobs;
    int n_prep_items, n_tile_items, n_key_items, n_unc, n_ref2_items,
        n_fin;
  };
  std::vector<Rec> recs;
  const bool prohd = mode == PROHD_BATCH_PROHD;
  for (int D : b->dims) {
    const std::vector<int> g = group(b, D);
    Rec r{};
    r.D = D;
    r.DP = pad_dim(D);
    r.m = b->pairs[g[0]].m;
    const int DP = r.DP;
    if (prohd) {
      // Gram slices; items in groups of 8 slices x TSPLIT shares x 8 (XCD)
      std::vector<GramJob> gj;
      std::vector<GramRedJob> rj;
      std::vector<EigJob> ej;
      std::vector<ProjJob> pj;
      std::vector<SegJob> sj;
      std::vector<CompactJob> cj;
      for (int i : g) {
        const Pair& q = b->pairs[i];
        const PairWs& w = L.p[i];
        const float* Ap = b->A + q.offA;
        const float* Bp = b->B + q.offB;
        const size_t TD = gram_partial_doubles(DP);
        int sl = 0;
        for (int s = 0; s < 2; ++s) {
          const int64_t n = s ? q.nB : q.nA;
          for (int64_t r0 = 0; r0 < n; r0 += t.gram_rows, ++sl)
            gj.push_back(GramJob{s ? Bp : Ap, Ap, r0, std::min<int64_t>(n, r0 + t.gram_rows),
                                 w.gpart + (size_t)sl * TD, w.spart + (size_t)sl * 2 * DP, s == 0,
                                 w.status});
        }
        rj.push_back(GramRedJob{w.gpart, w.spart, sl, q.nA, q.nB, w.C, w.u0});
        ej.push_back(EigJob{w.C, w.V, w.Y, w.u0, w.dirs, w.status, q.m});
        for (int s = 0; s < 2; ++s) {
          const int64_t n = s ? q.nB : q.nA;
          for (int64_t r0 = 0; r0 < n; r0 += 512)
            pj.push_back(ProjJob{s ? Bp : Ap, n, r0, w.dirs, w.proj[s], q.m + 1});
          for (int d = 0; d <= q.m; ++d) {
            const int32_t k = s ? q.kB[d] : q.kA[d];
            sj.push_back(SegJob{w.proj[s] + (size_t)d * n, n, nullptr, k, k, w.flags[s]});
          }
          cj.push_back(CompactJob{w.flags[s], n, nullptr, w.idx[s], s ? q.capB : q.capA, w.cnt + s});
        }
      }
      const int ts = gram_tsplit(DP);
      std::vector<BItem> gi;
      const int nsl = (int)gj.size();
      for (int g8 = 0; g8 < nsl; g8 += 8)
        for (int sh = 0; sh < ts; ++sh)
          for (int x = 0; x < 8; ++x) gi.push_back(BItem{g8 + x < nsl ? g8 + x : -1, sh});
      r.gram_jobs = T.add(gj);
      r.gram_items = T.add(gi);
      r.n_gram_items = (int)gi.size();
      r.red_jobs = T.add(rj);
      r.n_red = (int)rj.size();
      r.eig_jobs = T.add(ej);
      r.n_eig = (int)ej.size();
      r.proj_jobs = T.add(pj);
      r.n_proj = (int)pj.size();
      r.seg_jobs = T.add(sj);
      r.n_seg = (int)sj.size();
      r.cmp_jobs = T.add(cj);
      r.n_cmp = (int)cj.size();
    }
    // distance stage (both modes)
    std::vector<PrepJob> prj;
    std::vector<BItem> pri;
    std::vector<TileJob> tlj;
    std::vector<BItem> tli;
    std::vector<KeyJob> kyj;
    std::vector<BItem> kyi;
    std::vector<UncJob> ucj;
    std::vector<RefineJob> r2j;
    std::vector<BItem> r2i;
    std::vector<FinalJob> fj;
    for (int i : g) {
      const Pair& q = b->pairs[i];
      if (pruned_pair(q, mode)) continue;
      const PairWs& w = L.p[i];
      const float* Ap = b->A + q.offA;
      const float* Bp = b->B + q.offB;
      const int64_t rA = side_rows(q, 0, mode), rB = side_rows(q, 1, mode);
      const int64_t* dA = prohd ? w.cnt : nullptr;
      const int64_t* dB = prohd ? w.cnt + 1 : nullptr;
      for (int s = 0; s < 2; ++s) {
        const int64_t r = s ? rB : rA;
        const int nbx = (int)std::max<int64_t>(1, cdiv(r, 64));
        const int job = (int)prj.size();
        prj.push_back(PrepJob{s ? Bp : Ap, prohd ? w.idx[s] : nullptr, s ? dB : dA, r, Ap,
                              prohd ? w.idx[0] : nullptr, dA, w.xp[s], w.xn[s], w.status, nbx});
        for (int x = 0; x < nbx; ++x) pri.push_back(BItem{job, x});
      }
      const int ysplit = (int)std::max<int64_t>(1, cdiv(rB, t.tile_yc));
      const int job = (int)tlj.size();
      tlj.push_back(TileJob{w.xp[0], w.xn[0], dA, rA, w.xp[1], w.xn[1], dB, rB, ysplit, w.row[0],
                            w.row[1]});
      const int64_t nbt = cdiv(rA, 256) * ysplit;
      for (int64_t x = 0; x < nbt; ++x) tli.push_back(BItem{job, (int)x});
      for (int s = 0; s < 2; ++s) {
        const int64_t r = s ? rB : rA;
        const int64_t ry = s ? rA : rB;
        const int ys = (int)std::max<int64_t>(1, cdiv(ry, t.refine_yc));
        // upper bounds as keys in place of the row minima and the largest
        // lower bound, then every row whose upper bound reaches it, and
        // their float64 re-measurement
        const int kbx = (int)std::max<int64_t>(1, cdiv(r, 256));
        const int kjob = (int)kyj.size();
        kyj.push_back(KeyJob{w.row[s], w.xn[s], s ? dB : dA, r, kbx, w.hlow + s});
        for (int x = 0; x < kbx; ++x) kyi.push_back(BItem{kjob, x});
        ucj.push_back(UncJob{w.row[s], nullptr, nullptr, s ? dB : dA, r, nullptr, nullptr, w.status,
                             w.cand2[s], w.ccnt2 + s, w.best2[s], w.hlow + s});
        const int r2job = (int)r2j.size();
        r2j.push_back(RefineJob{w.xp[s], w.cand2[s], w.ccnt2 + s, w.xp[1 - s], s ? dA : dB, ry, ys,
                                w.best2[s]});
        for (int x = 0; x < ys; ++x) r2i.push_back(BItem{r2job, x});
      }
      FinalJob f{};
      f.ab = FinalDir{nullptr, nullptr, nullptr, w.best2[0], w.cand2[0], w.ccnt2,
                      prohd ? w.idx[0] : nullptr, prohd ? w.idx[1] : nullptr, Ap, Bp};
      f.ba = FinalDir{nullptr, nullptr, nullptr, w.best2[1], w.cand2[1], w.ccnt2 + 1,
                      prohd ? w.idx[1] : nullptr, prohd ? w.idx[0] : nullptr, Bp, Ap};
      f.dnA = dA;
      f.hnA = rA;
      f.dnB = dB;
      f.hnB = rB;
      f.status = w.status;
      f.out = b->out + i;
      f.D = q.D;
      fj.push_back(f);
    }
    r.prep_jobs = T.add(prj);
    r.prep_items = T.add(pri);
    r.n_prep_items = (int)pri.size();
    r.tile_jobs = T.add(tlj);
    r.tile_items = T.add(tli);
    r.n_tile_items = (int)tli.size();
    r.key_jobs = T.add(kyj);
    r.key_items = T.add(kyi);
    r.n_key_items = (int)kyi.size();
    r.unc_jobs = T.add(ucj);
    r.n_unc = (int)ucj.size();
    r.ref2_jobs = T.add(r2j);
    r.ref2_items = T.add(r2i);
    r.n_ref2_items = (int)r2i.size();
    r.fin_jobs = T.add(fj);
    r.n_fin = (int)fj.size();
    recs.push_back(r);
  }
  // upload
  if (b->dtab_bytes < T.host.size()) {
    if (b->dtab) hipFree(b->dtab);
    b->dtab = nullptr;
    b->dtab_bytes = 0;
    if (hipMalloc(&b->dtab, std::max<size_t>(T.host.size(), 256)) != hipSuccess)
      return fail(PROHD_EDEVICE, "batch: cannot allocate the work tables");
    b->dtab_bytes = std::max<size_t>(T.host.size(), 256);
  }
  if (!T.host.empty() && hipMemcpy(b->dtab, T.host.data(), T.host.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(PROHD_EDEVICE, "batch: cannot upload the work tables");
  char* base = static_cast<char*>(b->dtab);
  auto at = [base](size_t o) { return (const void*)(base + o); };

  auto& Ls = b->launches;
  Ls.clear();
  // initial state: statuses and lower bounds (adjacent), flags, minima
  int32_t* status = L.status;
  const int P = b->P;
  uint32_t* row = L.row;
  const int64_t nrow = L.nrow;
  uint8_t* flags = L.flags;
  const int64_t nflags = L.nflags;
  uint32_t* hlow = L.hlow;
  Ls.push_back([=](hipStream_t s) { return zero_bytes(status, sizeof(int32_t) * P, s); });
  Ls.push_back([=](hipStream_t s) { return zero_bytes(hlow, sizeof(uint32_t) * 2 * P, s); });
  if (prohd) Ls.push_back([=](hipStream_t s) { return zero_bytes(flags, (size_t)nflags, s); });
  if (nrow > 0) Ls.push_back([=](hipStream_t s) { return batch_fill32(row, nrow, 0x7f800000u, s); });
  for (const Rec& r : recs) {
    if (!prohd) continue;
    const int gram_grid = (int)(cdiv(persist(r.n_gram_items, t.gram_mult), 8) * 8);
    Ls.push_back([=](hipStream_t s) {
      return batch_gram(r.DP, r.D, (const GramJob*)at(r.gram_jobs), (const BItem*)at(r.gram_items),
                        r.n_gram_items, gram_grid, s);
    });
    Ls.push_back([=](hipStream_t s) {
      return batch_gram_reduce(r.DP, r.D, (const GramRedJob*)at(r.red_jobs), r.n_red, 4, s);
    });
    const bool narrow = t.eig_narrow != 0 && r.m < 32;
    Ls.push_back([=](hipStream_t s) {
      return batch_eig(r.DP, r.D, (const EigJob*)at(r.eig_jobs), r.n_eig, narrow, s);
    });
    const int pgrid = persist(r.n_proj, t.proj_mult);
    const bool vec = ((uintptr_t)b->A % 16 == 0) && ((uintptr_t)b->B % 16 == 0);
    Ls.push_back([=](hipStream_t s) {
      return batch_project(r.DP, r.D, r.m + 1, vec, (const ProjJob*)at(r.proj_jobs), r.n_proj,
                           pgrid, s);
    });
    Ls.push_back([=](hipStream_t s) { return batch_select((const SegJob*)at(r.seg_jobs), r.n_seg, s); });
    Ls.push_back([=](hipStream_t s) { return batch_compact((const CompactJob*)at(r.cmp_jobs), r.n_cmp, s); });
  }
  // the pruned single-pair searches (largest first, as the groups)
  for (int D : b->dims)
    for (int i : group(b, D)) {
      const Pair& q = b->pairs[i];
      if (!pruned_pair(q, mode)) continue;
      const float* Ap = b->A + q.offA;
      const float* Bp = b->B + q.offB;
      prohd_result* o = b->out + i;
      void* sw = L.single_ws;
      const size_t sb = L.single_bytes;
      Ls.push_back([=](hipStream_t s) {
        return hd_exact(Ap, q.nA, Bp, q.nB, q.D, PROHD_PRUNE, o, nullptr, nullptr, sw, sb, s);
      });
    }
  for (const Rec& r : recs) {
    if (r.n_fin == 0) continue;   // every pair of this width took the pruned search
    const int prep_grid = persist(r.n_prep_items, 8);
    const int tile_grid = persist(r.n_tile_items, t.tile_mult);
    Ls.push_back([=](hipStream_t s) {
      return batch_prep(r.DP, r.D, (const PrepJob*)at(r.prep_jobs), (const BItem*)at(r.prep_items),
                        r.n_prep_items, prep_grid, s);
    });
    Ls.push_back([=](hipStream_t s) {
      return batch_tile(r.DP, (const TileJob*)at(r.tile_jobs), (const BItem*)at(r.tile_items),
                        r.n_tile_items, tile_grid, s);
    });
    const int key_grid = persist(r.n_key_items, 8);
    Ls.push_back([=](hipStream_t s) {
      return batch_keys(r.DP, (const KeyJob*)at(r.key_jobs), (const BItem*)at(r.key_items),
                        r.n_key_items, key_grid, s);
    });
    Ls.push_back([=](hipStream_t s) { return batch_uncertain((const UncJob*)at(r.unc_jobs), r.n_unc, s); });
    const int ref2_grid = persist(r.n_ref2_items, 4);
    Ls.push_back([=](hipStream_t s) {
      return batch_refine_dyn(r.DP, (const RefineJob*)at(r.ref2_jobs), (const BItem*)at(r.ref2_items),
                              r.n_ref2_items, ref2_grid, s);
    });
    Ls.push_back([=](hipStream_t s) { return batch_finalize((const FinalJob*)at(r.fin_jobs), r.n_fin, s); });
  }
  return PROHD_OK;
}

prohd_status run_list(prohd_batch* b, hipStream_t s) {
  for (auto& f : b->launches) {
    const prohd_status st = f(s);
    if (st) return st;
  }
  return PROHD_OK;
}

prohd_status capture(prohd_batch* b) {
  release_graph(b);
  if (!b->cs && hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess)
    return fail(PROHD_EDEVICE, "batch: cannot create the capture stream");
  if (hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(PROHD_EDEVICE, "batch: cannot begin graph capture");
  set_capturing(true);
  const prohd_status st = run_list(b, b->cs);
  set_capturing(false);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cs, &g);
  if (st) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess || !g) return fail(PROHD_EDEVICE, "batch: graph capture failed");
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    release_graph(b);
    return fail(PROHD_EDEVICE, "batch: cannot instantiate the graph");
  }
  return PROHD_OK;
}

prohd_status bind(prohd_batch* b, uint32_t mode, const float* A, const float* B, prohd_result* out,
                  void* ws, size_t ws_bytes) {
  if (b->bound && b->mode == mode && b->A == A && b->B == B && b->out == out && b->ws == ws &&
      b->ws_bytes == ws_bytes)
    return PROHD_OK;
  const prohd_status w = wait_done(b);   // no run in flight reads the tables or the graph
  if (w) return w;
  release_graph(b);
  b->bound = false;
  b->mode = mode;
  b->A = A;
  b->B = B;
  b->out = out;
  b->ws = ws;
  b->ws_bytes = ws_bytes;
  const prohd_status st = build(b);
  if (st) return st;
  b->bound = true;
  return PROHD_OK;
}

size_t ws_size(const prohd_batch* b, uint32_t mode, const Tuning& t) {
  Arena ar(nullptr);
  make_layout(ar, *b, mode, t);
  return ar.used + 256;
}

prohd_status check_run(const prohd_batch* b, uint32_t mode, const float* A, const float* B,
                       const prohd_result* out, const void* ws) {
  if (!b) return fail(PROHD_EINVAL, "plan must be non-null");
  if (mode != PROHD_BATCH_PROHD && mode != PROHD_BATCH_EXACT)
    return fail(PROHD_EINVAL, "mode must be PROHD_BATCH_PROHD or PROHD_BATCH_EXACT");
  if (!A || !B || !out || !ws) return fail(PROHD_EINVAL, "A, B, out and ws must be non-null");
  return PROHD_OK;
}

bool json_int(const std::string& txt, const char* key, int* v) {
  const std::string k = std::string("\"") + key + "\"";
  const size_t p = txt.find(k);
  if (p == std::string::npos) return false;
  const size_t c = txt.find(':', p + k.size());
  if (c == std::string::npos) return false;
  char* end = nullptr;
  const long x = std::strtol(txt.c_str() + c + 1, &end, 10);
  if (end == txt.c_str() + c + 1 || x <= 0 || x > (1L << 30)) return false;
  *v = (int)x;
  return true;
}

}  // namespace

extern "C" {

prohd_status prohd_batch_create(int32_t P, const int64_t* nA, const int64_t* nB, const int32_t* D,
                                double alpha, prohd_batch** plan) {
  if (!plan) return fail(PROHD_EINVAL, "plan must be non-null");
  *plan = nullptr;
  if (P < 1) return fail(PROHD_EINVAL, "P must be >= 1");
  if (!nA || !nB || !D) return fail(PROHD_EINVAL, "nA, nB and D must be non-null host arrays");
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(PROHD_EINVAL, "alpha must lie in (0, 1]");
  prohd_batch* b = new prohd_batch();
  b->P = P;
  b->alpha = alpha;
  b->pairs.resize(P);
  int64_t oa = 0, ob = 0;
  for (int i = 0; i < P; ++i) {
    Pair& q = b->pairs[i];
    if (nA[i] < 1 || nB[i] < 1 || nA[i] >= (int64_t(1) << 31) || nB[i] >= (int64_t(1) << 31)) {
      delete b;
      return fail(PROHD_EINVAL, "pair sizes must lie in [1, 2^31)");
    }
    if (D[i] < 1 || D[i] > PROHD_MAX_DIM) {
      delete b;
      return fail(D[i] < 1 ? PROHD_EINVAL : PROHD_EUNSUPPORTED, "pair dimension must lie in [1, 256]");
    }
    q.nA = nA[i];
    q.nB = nB[i];
    q.D = D[i];
    q.DP = pad_dim(D[i]);
    q.m = default_m(D[i]);
    q.offA = oa;
    q.offB = ob;
    oa += q.nA * q.D;
    ob += q.nB * q.D;
    q.kA.resize(q.m + 1);
    q.kB.resize(q.m + 1);
    int64_t sA = 0, sB = 0;
    for (int d = 0; d <= q.m; ++d) {
      const double a = d == 0 ? alpha : alpha / q.m;
      q.kA[d] = (int32_t)alpha_k(a, q.nA);
      q.kB[d] = (int32_t)alpha_k(a, q.nB);
      sA += 2 * (int64_t)q.kA[d];
      sB += 2 * (int64_t)q.kB[d];
    }
    q.capA = std::min<int64_t>(q.nA, sA);
    q.capB = std::min<int64_t>(q.nB, sB);
    if (std::find(b->dims.begin(), b->dims.end(), q.D) == b->dims.end()) b->dims.push_back(q.D);
  }
  std::sort(b->dims.begin(), b->dims.end());
  *plan = b;
  return PROHD_OK;
}

void prohd_batch_destroy(prohd_batch* plan) {
  if (!plan) return;
  wait_done(plan);
  if (plan->done) hipEventDestroy(plan->done);
  release_graph(plan);
  if (plan->cs) hipStreamDestroy(plan->cs);
  if (plan->dtab) hipFree(plan->dtab);
  delete plan;
}

size_t prohd_batch_workspace_size(const prohd_batch* plan, uint32_t mode) {
  if (!plan || (mode != PROHD_BATCH_PROHD && mode != PROHD_BATCH_EXACT)) return 0;
  // the Gram slice count depends on the tuned slice length: take the worst
  // (shortest) candidate so that a later tune never needs more
  Tuning t = plan->tune;
  t.gram_rows = std::min(t.gram_rows, 3072);
  return std::max(ws_size(plan, mode, t), ws_size(plan, mode, plan->tune));
}

prohd_status prohd_batch_run(prohd_batch* plan, uint32_t mode, const float* A, const float* B,
                             prohd_result* out, void* ws, size_t ws_bytes, uint32_t flags,
                             void* stream) {
  prohd_status st = check_run(plan, mode, A, B, out, ws);
  if (st) return st;
  if (flags & ~(uint32_t)(PROHD_BATCH_EAGER | PROHD_SYNC)) return fail(PROHD_EINVAL, "unknown flag bits");
  st = bind(plan, mode, A, B, out, ws, ws_bytes);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (flags & PROHD_BATCH_EAGER) {
    st = run_list(plan, s);
  } else {
    if (!plan->exec) {
      st = capture(plan);
      if (st) return st;
    }
    if (hipGraphLaunch(plan->exec, s) != hipSuccess) return fail(PROHD_EDEVICE, "batch: graph launch failed");
  }
  if (st) return st;
  st = mark_done(plan, s);
  if (st) return st;
  if (flags & PROHD_SYNC) {
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PROHD_EDEVICE, "batch: stream error");
  }
  return PROHD_OK;
}

prohd_status prohd_batch_tune(prohd_batch* plan, uint32_t mode, const float* A, const float* B,
                              prohd_result* out, void* ws, size_t ws_bytes, void* stream,
                              const char* json_path) {
  prohd_status st = check_run(plan, mode, A, B, out, ws);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  struct Knob {
    const char* name;
    int Tuning::*field;
    std::vector<int> values;
    const char* kernel;   // timer name whose total is minimised
  };
  std::vector<Knob> knobs;
  if (mode == PROHD_BATCH_PROHD) {
    knobs.push_back({"eig_narrow", &Tuning::eig_narrow, {0, 1}, "batch_eig"});
    knobs.push_back({"gram_rows", &Tuning::gram_rows, {3072, 6144, 12288, 24576}, "batch_gram"});
    knobs.push_back({"gram_mult", &Tuning::gram_mult, {1, 2, 3}, "batch_gram"});
    knobs.push_back({"proj_mult", &Tuning::proj_mult, {2, 4, 8}, "batch_project"});
    knobs.push_back({"tile_yc", &Tuning::tile_yc, {1024, 4096, 16384}, "batch_tile"});
  } else {
    knobs.push_back({"tile_yc", &Tuning::tile_yc, {4096, 8192, 16384}, "batch_tile"});
    knobs.push_back({"tile_mult", &Tuning::tile_mult, {1, 2}, "batch_tile"});
    knobs.push_back({"refine_yc", &Tuning::refine_yc, {8192, 32768}, "batch_refine"});
  }
  std::string trials;
  for (const Knob& k : knobs) {
    int best_v = plan->tune.*(k.field);
    double best_ms = -1.0;
    for (int v : k.values) {
      Tuning t = plan->tune;
      t.*(k.field) = v;
      if (ws_size(plan, mode, t) > ws_bytes) continue;
      plan->tune = t;
      plan->bound = false;
      st = bind(plan, mode, A, B, out, ws, ws_bytes);
      if (!st) st = run_list(plan, s);   // warm
      if (!st) st = prohd_profile_reset();
      if (!st) st = prohd_profile_enable(1);
      if (!st) st = run_list(plan, s);
      if (!st) st = mark_done(plan, s);
      int64_t n = 0;
      double ms = 0.0;
      if (!st) st = prohd_profile_read(k.kernel, &n, &ms);
      prohd_profile_enable(0);
      if (st) return st;
      char buf[160];
      std::snprintf(buf, sizeof(buf), "%s{\"knob\": \"%s\", \"value\": %d, \"ms\": %.4f}",
                    trials.empty() ? "" : ", ", k.name, v, ms);
      trials += buf;
      if (best_ms < 0.0 || ms < best_ms) {
        best_ms = ms;
        best_v = v;
      }
    }
    plan->tune.*(k.field) = best_v;
  }
  plan->bound = false;
  release_graph(plan);
  prohd_profile_reset();
  if (json_path && *json_path) {
    FILE* f = std::fopen(json_path, "w");
    if (!f) return fail(PROHD_EINVAL, "cannot write the tuning file");
    const Tuning& t = plan->tune;
    std::fprintf(f,
                 "{\"mode\": \"%s\", \"pairs\": %d, \"cus\": %d, \"knobs\": {\"gram_rows\": %d, "
                 "\"gram_mult\": %d, \"proj_mult\": %d, \"tile_yc\": %d, \"tile_mult\": %d, "
                 "\"refine_yc\": %d, \"eig_narrow\": %d}, \"trials\": [%s]}\n",
                 mode == PROHD_BATCH_PROHD ? "prohd" : "exact", plan->P, cu_count(), t.gram_rows,
                 t.gram_mult, t.proj_mult, t.tile_yc, t.tile_mult, t.refine_yc, t.eig_narrow,
                 trials.c_str());
    std::fclose(f);
  }
  return PROHD_OK;
}

prohd_status prohd_batch_load_tuning(prohd_batch* plan, const char* json_path) {
  if (!plan || !json_path) return fail(PROHD_EINVAL, "plan and path must be non-null");
  FILE* f = std::fopen(json_path, "r");
  if (!f) return fail(PROHD_EINVAL, "cannot read the tuning file");
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
  std::fclose(f);
  const size_t kp = txt.find("\"knobs\"");
  if (kp == std::string::npos) return fail(PROHD_EINVAL, "tuning file has no knobs");
  const std::string knobs = txt.substr(kp, txt.find('}', kp) - kp);
  Tuning t = plan->tune;
  json_int(knobs, "gram_rows", &t.gram_rows);
  json_int(knobs, "gram_mult", &t.gram_mult);
  json_int(knobs, "proj_mult", &t.proj_mult);
  json_int(knobs, "tile_yc", &t.tile_yc);
  json_int(knobs, "tile_mult", &t.tile_mult);
  json_int(knobs, "refine_yc", &t.refine_yc);
  int en = 0;
  if (knobs.find("\"eig_narrow\"") != std::string::npos) {
    const size_t c = knobs.find(':', knobs.find("\"eig_narrow\""));
    en = c != std::string::npos ? std::atoi(knobs.c_str() + c + 1) : 1;
    t.eig_narrow = en != 0;
  }
  plan->tune = t;
  plan->bound = false;
  release_graph(plan);
  return PROHD_OK;
}

}  // extern "C"
