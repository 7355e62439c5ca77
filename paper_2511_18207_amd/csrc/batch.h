// Batched form: many independent pairs per launch.
//
// Every batched kernel is persistent: a grid of at most a few work-groups per
// compute unit walks a device table of work items (blockIdx.x, then strides
// of gridDim.x).  A work item names a job (one pair, set or direction) and a
// block index inside it, and the kernel runs the same device body as the
// single-pair kernel with that block index.  The host builds the tables once
// per plan (k_batch.hip); the launches themselves take only device pointers
// and counts, so the whole chain can be captured in one graph.
#pragma once

#include "common.h"

namespace prohd {

struct BItem {
  int32_t job;  // index into the job table (-1: nothing to do)
  int32_t bx;   // block index inside the job
};

// prep: gather (optional), shift, pad, norms
struct PrepJob {
  const float* X;
  const int32_t* idx;   // rows to gather, or null (all rows)
  const int64_t* dn;    // device row count, or null
  int64_t hn;           // host bound on the row count
  const float* S;       // set holding the shift row
  const int32_t* sidx;  // shift row = S[sidx[0]] (or S[0] when null / empty)
  const int64_t* sdn;
  float* Xp;
  float* xn;
  int32_t* status;
  int32_t nbx;          // blocks of this job (rows are strided over them)
};

// float32 distance tile with row and column minima
struct TileJob {
  const float* Xp;
  const float* xn;
  const int64_t* dnX;
  int64_t hnX;
  const float* Yp;
  const float* yn;
  const int64_t* dnY;
  int64_t hnY;
  int32_t ysplit;
  uint32_t* rowmin;
  uint32_t* colmin;
};

// float64 refinement of the candidate rows of one direction
struct RefineJob {
  const float* Xp;
  const int32_t* cand;
  const int64_t* dR;
  const float* Yp;
  const int64_t* dnY;
  int64_t hnY;
  int32_t ysplit;
  unsigned long long* best;
};

// bound keys of one side's rows, in place over its row minima
struct KeyJob {
  uint32_t* mins;
  const float* xn;
  const int64_t* dn;
  int64_t hn;
  int32_t nbx;          // blocks of this job (rows are strided over them)
  uint32_t* hlow;       // largest certified L^2 of the rows (float bits, atomicMax), or null
};

// rows of one direction that may hold the directed distance (one
// work-group each) -> cand2 (ascending), count2, best2 initialised: with
// `hlow`, every row whose key reaches it (the largest certified lower
// bound); else every row whose key exceeds the largest first-pass minimum
// and is not one of the first pass's rows
struct UncJob {
  const uint32_t* key;               // bound keys (float bits)
  const uint8_t* top;                // rows of the first refinement (flag 1), or null
  const int32_t* map;                // entry -> row (cand2 gets map[i]), or null
  const int64_t* dn;                 // device row count, or null
  int64_t hn;                        // host bound on the row count
  const unsigned long long* best;    // first-pass minima
  const int64_t* dR;                 // first-pass count
  const int32_t* status;
  int32_t* cand2;                    // capacity hn
  int64_t* count2;
  unsigned long long* best2;         // capacity hn
  const uint32_t* hlow;              // or null
};

// one directed half of the final witness search
struct FinalDir {
  const unsigned long long* best;
  const int32_t* cand;
  const int64_t* dR;
  const unsigned long long* best2;   // second refinement pass (or null)
  const int32_t* cand2;
  const int64_t* dR2;
  const int32_t* mapX;
  const int32_t* mapY;
  const float* Xo;
  const float* Yo;
};

struct FinalJob {
  FinalDir ab, ba;
  const int64_t* dnA;
  int64_t hnA;
  const int64_t* dnB;
  int64_t hnB;
  const int32_t* status;
  prohd_result* out;
  int32_t D;
};

// Gram partial of one row slice of one set (rows [r_begin, r_end) of X)
struct GramJob {
  const float* X;
  const float* shift;   // first row of the pair's A
  int64_t r_begin, r_end;
  double* gp;           // T x 256 partial blocks of this slice
  double* sp;           // 2 DP partial column sums of this slice
  int32_t setA;
  int32_t* status;
};

struct GramRedJob {
  const double* gpart;  // first slice partial of the pair
  const double* spart;
  int32_t nwg;          // slices of the pair
  int64_t nA, nB;
  double* C;
  double* u0;
};

struct EigJob {
  double* C;
  double* V;
  double* Y;
  const double* u0;
  float* dirs;
  const int32_t* status;
  int32_t m;
};

// one 512-row tile of one set; dirs: the pair's ndirs x D directions
struct ProjJob {
  const float* X;
  int64_t n;
  int64_t r0;
  const float* dirs;
  float* P;
  int32_t ndirs;
};

// extreme selection of one segment (one work-group each)
struct SegJob {
  const float* vals;
  int64_t n;
  const int64_t* dn;
  int32_t lo, hi;
  uint8_t* flags;
};

struct CompactJob {
  const uint8_t* flags;
  int64_t n;
  const int64_t* dn;
  int32_t* idx;
  int64_t cap;
  int64_t* count;
};

// Launchers (grid = persistent work-groups; items/jobs are device tables).
prohd_status batch_prep(int DP, int D, const PrepJob* jobs, const BItem* items, int nitems, int grid,
                        hipStream_t s);
prohd_status batch_tile(int DP, const TileJob* jobs, const BItem* items, int nitems, int grid,
                        hipStream_t s);
prohd_status batch_keys(int DP, const KeyJob* jobs, const BItem* items, int nitems, int grid,
                        hipStream_t s);
prohd_status batch_uncertain(const UncJob* jobs, int njobs, hipStream_t s);
// items (job, Y chunk); each walks every candidate block of its job's count
prohd_status batch_refine_dyn(int DP, const RefineJob* jobs, const BItem* items, int nitems, int grid,
                              hipStream_t s);
prohd_status batch_finalize(const FinalJob* jobs, int njobs, hipStream_t s);
prohd_status batch_fill32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
prohd_status batch_fill64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
int gram_tsplit(int DP);
int gram_rows_quantum(int DP);
size_t gram_partial_doubles(int DP);
prohd_status batch_gram(int DP, int D, const GramJob* jobs, const BItem* items, int nitems, int grid,
                        hipStream_t s);
prohd_status batch_gram_reduce(int DP, int D, const GramRedJob* jobs, int njobs, int per_job,
                               hipStream_t s);
size_t eig_job_doubles(int DP);
// narrow: 256-thread work-groups (several problems per compute unit), m < 32
prohd_status batch_eig(int DP, int D, const EigJob* jobs, int njobs, bool narrow, hipStream_t s);
// vec: float4 row loads (D % 4 == 0 and 16-byte aligned packed sets);
// ndirs <= 33
prohd_status batch_project(int DP, int D, int ndirs, bool vec, const ProjJob* jobs, int njobs, int grid,
                           hipStream_t s);
prohd_status batch_select(const SegJob* jobs, int njobs, hipStream_t s);
prohd_status batch_compact(const CompactJob* jobs, int njobs, hipStream_t s);

}  // namespace prohd
