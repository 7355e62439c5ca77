/*
 * prohd.h -- C ABI of the MI355X (gfx950) ProHD hot path.
 *
 * ProHD (projection-based Hausdorff approximation, arXiv 2511.18207) keeps,
 * for each of a few directions -- the centroid axis and the top principal
 * components of the union of the two sets -- the points of each set whose
 * projections are extreme, and computes the Hausdorff distance of the two
 * kept subsets.  This library runs every step of that path, and the exact
 * brute-force distance it approximates, as HIP kernels on one GPU:
 *
 *   prohd_project  centroid axis + top-m principal directions, projections
 *                  (paper Alg. 1 centroid/axis/projection steps, Alg. 2
 *                  stacking/PCA/normalisation/projection steps)
 *   prohd_select   per-direction k smallest / k largest, union, unique
 *                  (Alg. 1 and Alg. 2 argsort/extreme/union steps, Alg. 3
 *                  union of the two index sets)
 *   prohd_hd       directed and symmetric Hausdorff distance over the
 *                  selected rows (Sec. II-A definition of H-hat, Alg. 3
 *                  subset extraction and distance steps)
 *   exact_hd       exact Hausdorff distance, Eq. (1)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Point sets are DEVICE pointers to row-major float32 arrays, n rows of
 *    D floats, row stride D, 4-byte aligned (16-byte aligned is faster).
 *    1 <= D <= PROHD_MAX_DIM.  Row counts are < 2^31.
 *  - All device pointers are owned by the caller.  The library never frees
 *    or retains them, and allocates no device memory: every scratch byte
 *    comes from the caller's workspace `ws` (device memory, 256-byte
 *    aligned, at least prohd_workspace_size() bytes).
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 *    the default stream).  Calls that share a workspace must be ordered on
 *    one stream.  Distinct streams with distinct workspaces may run
 *    concurrently from different host threads.
 *  - Host-side argument errors are returned before anything is enqueued.
 *    Errors found on the device (non-finite input) are written to the
 *    `status` field of a prohd_result and, when PROHD_SYNC is set, the call
 *    waits for the stream and returns that status.
 *  - On any non-OK return, prohd_last_error() gives a message (per host
 *    thread).
 *  - Distances are Euclidean (not squared).  Index outputs are 0-based
 *    int32, ascending and unique.  Witness indices refer to rows of the
 *    ORIGINAL A and B.
 */
#ifndef PROHD_H
#define PROHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PROHD_MAX_DIM 256
#define PROHD_MAX_DIRS 64

typedef enum {
  PROHD_OK = 0,
  PROHD_EINVAL = 1,       /* bad argument: NULL pointer, size, k, flag      */
  PROHD_ENONFINITE = 2,   /* NaN or Inf found in an input set (device)      */
  PROHD_EWORKSPACE = 3,   /* ws_bytes below the size the call needs         */
  PROHD_EDEVICE = 4,      /* a HIP runtime call failed                      */
  PROHD_EUNSUPPORTED = 5  /* D > PROHD_MAX_DIM or ndirs > PROHD_MAX_DIRS    */
} prohd_status;

/* Flags (bitwise OR). */
enum {
  PROHD_DIRS_GIVEN = 1u << 0, /* prohd_project: `dirs` is an input          */
  PROHD_INNER_FULL = 1u << 1, /* prohd_hd: inner minimum over the whole other
                                 set: max{h(A_sel,B), h(B_sel,A)} <= H(A,B)  */
  PROHD_PREC_BF16 = 1u << 2,  /* prohd_hd / exact_hd: distance search tiles
                                 in bfloat16 (float32 accumulation)          */
  PROHD_PREC_FP8 = 1u << 3,   /* ... in float8 e4m3 with one power-of-two
                                 scale (float32 accumulation)                */
  PROHD_SYNC = 1u << 4,       /* wait for the stream; return device status  */
  PROHD_PRUNE = 1u << 5       /* prohd_hd / exact_hd: pruned distance
                                 search, same result (see prohd_hd)          */
};

/* Result of prohd_hd / exact_hd, written by the device into caller memory. */
typedef struct {
  double H;        /* max(hAB, hBA)                                          */
  double hAB;      /* directed distance from (selected) A to (selected) B    */
  double hBA;      /* directed distance from (selected) B to (selected) A    */
  int64_t ab_a;    /* row of A realising hAB                                 */
  int64_t ab_b;    /* its nearest row of B                                   */
  int64_t ba_b;    /* row of B realising hBA                                 */
  int64_t ba_a;    /* its nearest row of A                                   */
  int64_t nA_sel;  /* rows of A taken part (nA for exact_hd)                 */
  int64_t nB_sel;  /* rows of B taken part (nB for exact_hd)                 */
  int32_t status;  /* prohd_status of the device-side work                   */
  int32_t refined; /* rows re-measured in float64, the larger of the two
                      directions (first pass: up to 256; more when the search
                      error bound leaves rows uncertain)                    */
} prohd_result;

/*
 * Bytes of workspace that any entry point needs for sets of nA and nB rows
 * in dimension D with `ndirs` directions (m+1) and selection capacities
 * capA / capB (0 lets the library use nA / nB).  Pure host function.
 * Returns 0 for invalid sizes.
 */
size_t prohd_workspace_size(int64_t nA, int64_t nB, int32_t D, int32_t ndirs,
                            int64_t capA, int64_t capB);

/*
 * Alpha mode of Alg. 3 (host functions, no device work).
 *
 * prohd_default_m -- m = floor(sqrt(D)), the number of principal components
 * Alg. 3 uses; 0 when D is outside [1, PROHD_MAX_DIM].
 *
 * prohd_alpha_k -- the per-direction counts for prohd_select in alpha mode,
 * for a set of n rows and m components:
 *   k[0]      = max(1, floor(alpha n))        per end on the centroid axis
 *               (Alg. 1, its k rule)
 *   k[1..m]   = max(1, floor((alpha / m) n))  per end on each component
 *               (Alg. 2 called by Alg. 3 with alpha' = alpha / m)
 * each clipped to n; the floor is taken of alpha n + 1e-9, so that a decimal
 * alpha does not lose an integer to binary rounding.
 *   k    HOST int32 array of m + 1 entries, output
 * Errors: EINVAL (alpha not positive and finite, n outside [1, 2^31),
 * m outside [1, PROHD_MAX_DIRS - 1], k null).
 */
int32_t prohd_default_m(int32_t D);
prohd_status prohd_alpha_k(double alpha, int64_t n, int32_t m, int32_t* k);

/*
 * prohd_project -- directions and projections.
 *
 * Computes, unless PROHD_DIRS_GIVEN is set:
 *   dirs row 0   : the centroid axis u = (mean(B) - mean(A)) / ||.||, or the
 *                  first basis vector e_1 when ||mean(B) - mean(A)|| < 1e-9
 *                  (Alg. 1, axis step, with X = A and Y = B as Alg. 3 calls
 *                  it);
 *   dirs rows 1..m: the m principal components of the stacked union [A; B]
 *                  (eigenvectors of its centred covariance, largest
 *                  eigenvalue first), unit length, sign fixed so the
 *                  largest-magnitude entry is positive (Alg. 2, PCA and
 *                  normalisation steps).
 * Means, covariance and eigensolve are float64 on the device.
 * Then projA[d*nA + i] = A_i . dirs_d and projB[d*nB + j] = B_j . dirs_d
 * (float32; Alg. 1 and Alg. 2 projection steps), for d = 0..m.
 *
 *   A, B     device float32, nA x D and nB x D
 *   m        number of principal directions, 1 <= m <= D, m + 1 <= PROHD_MAX_DIRS
 *   dirs     device float32, (m+1) x D row-major: output, or input when
 *            PROHD_DIRS_GIVEN (rows are then used as given)
 *   projA    device float32, (m+1) x nA (direction-major), output
 *   projB    device float32, (m+1) x nB, output
 *   evals    device float64, D entries, output (descending covariance
 *            eigenvalues), or NULL; untouched when PROHD_DIRS_GIVEN
 *   status   device int32, output: PROHD_OK or PROHD_ENONFINITE
 *            (NaN/Inf in A or B), or NULL
 * Errors: EINVAL (NULL, n < 1, m out of range), EUNSUPPORTED (D too large),
 * EWORKSPACE, EDEVICE.
 */
prohd_status prohd_project(const float* A, int64_t nA, const float* B, int64_t nB,
                           int32_t D, int32_t m, uint32_t flags, float* dirs,
                           float* projA, float* projB, double* evals,
                           int32_t* status, void* ws, size_t ws_bytes, void* stream);

/*
 * prohd_select -- extreme-candidate selection and union.
 *
 * For every direction d (0 <= d < ndirs) and each set, keeps the kA[d]
 * (resp. kB[d]) smallest and the same number of largest projections, under
 * the total order (value, index): ties go to the smaller index at BOTH ends;
 * -0.0 equals +0.0.  k is clipped to the set size.  The kept indices of all
 * directions and both ends are unioned into ascending unique lists
 * (Alg. 1 and Alg. 2 extreme steps, Alg. 3 union step).
 *
 *   projA    device float32, ndirs x nA (as written by prohd_project)
 *   projB    device float32, ndirs x nB
 *   kA, kB   HOST int32 arrays of ndirs entries, each >= 1
 *   idxA     device int32, capacity capA: output, ascending unique rows of A
 *   nselA    device int64: output, number of entries written to idxA
 *   idxB, capB, nselB: the same for B
 * capA must be >= min(nA, sum_d 2*min(kA[d], nA)) (so the list cannot
 * overflow); likewise capB.  Projections must be finite.
 * Errors: EINVAL, EUNSUPPORTED (ndirs > PROHD_MAX_DIRS), EWORKSPACE, EDEVICE.
 */
prohd_status prohd_select(const float* projA, int64_t nA, const float* projB, int64_t nB,
                          int32_t ndirs, const int32_t* kA, const int32_t* kB,
                          int32_t* idxA, int64_t capA, int64_t* nselA,
                          int32_t* idxB, int64_t capB, int64_t* nselB,
                          void* ws, size_t ws_bytes, void* stream);

/*
 * prohd_top_keys -- the k <= 64 largest entries of one float32 array under
 * the order of prohd_select (larger value first; equal values: smaller index
 * first; -0.0 equals +0.0), as an ascending index list.  prohd_hd's pruned
 * search takes its seed rows this way (the rows with the largest upper
 * bounds); the ordering rule is that of the extreme step of Alg. 1 and
 * Alg. 2.
 *
 *   vals   device float32, n entries, no NaN (+-inf allowed); may be NULL
 *          when n is 0
 *   n      host bound on the length, 0 <= n < 2^31
 *   dev_n  device int64 or NULL: when non-null the length is min(*dev_n, n)
 *          (a negative count is 0), read on the device
 *   k      0 <= k <= 64
 *   idx    device int32, at least k entries: output, ascending
 *   count  device int64: output, min(k, length)
 *   ws     device workspace, ws_bytes >= PROHD_TOPK_WS_BYTES
 * Two kernel launches on `stream`, no host synchronisation.
 * Errors: EINVAL (null pointers, n or k out of range), EWORKSPACE, EDEVICE.
 */
#define PROHD_TOPK_WS_BYTES ((size_t)(512u * 1024u + 256u))
prohd_status prohd_top_keys(const float* vals, int64_t n, const int64_t* dev_n, int32_t k,
                            int32_t* idx, int64_t* count, void* ws, size_t ws_bytes,
                            void* stream);

/*
 * prohd_hd -- Hausdorff distance over the selected rows.
 *
 * Default: H-hat = max{ max_{a in A_sel} min_{b in B_sel} ||a-b||,
 *                       max_{b in B_sel} min_{a in A_sel} ||b-a|| }
 * (Sec. II-A definition of H-hat; Alg. 3 extraction and distance steps).
 * With PROHD_INNER_FULL: max{ h(A_sel, B), h(B_sel, A) } (inner minimum
 * over the whole other set), which never exceeds H(A,B).
 *
 * Distances are searched with float32 (or, with PROHD_PREC_BF16 /
 * PROHD_PREC_FP8, bfloat16 / e4m3) matrix-core tiles of |a|^2 + |b|^2 - 2 a.b
 * on rows shifted by a common point.  Each outer row gets an upper bound of
 * its true minimum from the search's worst-case rounding and quantisation
 * error; the 256 rows with the largest bounds, and then every further row
 * whose bound exceeds the largest re-measured minimum, are re-measured
 * against every inner row with the float64 expansion on the matrix cores
 * (the float32 rows converted exactly), and the final witness pair is
 * measured in float64 from the original rows.  So no row whose true minimum
 * could exceed the returned value is left out, for any data (on data whose
 * nearest-neighbour distances the expansion cannot resolve, such as a set
 * against a slightly moved copy of itself, that may be every row).  Range:
 * the search forms float32 squared distances of the shifted rows, so these
 * must stay below float32's maximum (coordinates spread by up to about
 * 1e18); wider sets saturate the search and the witness pair is then not
 * guaranteed.
 *
 * With PROHD_PRUNE (ignored when either side has fewer than 16384 outer
 * rows) the search runs in levels.  The first measures every outer row
 * against every F-th row of its inner set (rows 0, F, 2F, ... of the
 * selected list, or of the whole set in inner-full mode; F = 16^L with L
 * the largest level count in [1, 4] that leaves at least 16 rows of the
 * smaller inner set): the minimum over a subset bounds the row's minimum
 * over the whole inner set from above.  The 256 rows with the largest such
 * bounds are re-measured in float64 against the whole inner set; a row
 * whose bound does not exceed the largest re-measured minimum cannot hold
 * the directed distance and is dropped.  Each further level searches the
 * remaining rows against a 16 times larger subset (F/16, ..., 16, and last
 * the whole inner set) and drops rows by the same rule; what the last level
 * leaves is re-measured as above.  The result is the same witness and value
 * as without the flag; the work falls from about nA nB to about nA nB / F
 * when few rows remain (the usual case) and rises by at most 1/15 when no
 * row can be dropped.
 *
 *   A, B            device float32 point sets (nA x D, nB x D)
 *   idxA, nselA     device: selected rows of A (ascending int32) and their
 *                   count (int64), as written by prohd_select; likewise B
 *   capA, capB      host: upper bounds of *nselA / *nselB (grid sizing);
 *                   the device counts must not exceed them
 *   out             device prohd_result, output
 * Errors: EINVAL, EUNSUPPORTED, EWORKSPACE, EDEVICE; with PROHD_SYNC the
 * device status (ENONFINITE, or EINVAL for an empty selection).
 */
prohd_status prohd_hd(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      const int32_t* idxA, const int64_t* nselA,
                      const int32_t* idxB, const int64_t* nselB,
                      int64_t capA, int64_t capB, uint32_t flags,
                      prohd_result* out, void* ws, size_t ws_bytes, void* stream);

/*
 * prohd_prune_levels -- subset levels L of the pruned search that prohd_hd
 * (capacities capA / capB, `flags`) runs on sets of nA / nB rows: the first
 * level searches against every 16^L-th row of the inner set; 0 when the
 * call is not pruned (no PROHD_PRUNE, or a capacity below 16384).  For
 * exact_hd pass capA = nA, capB = nB.  Pure host function; 0 for invalid
 * sizes.
 */
int32_t prohd_prune_levels(int64_t nA, int64_t nB, int64_t capA, int64_t capB, uint32_t flags);

/*
 * exact_hd -- exact Hausdorff distance H(A,B) of Eq. (1), both directed
 * parts and witnesses, by brute force over all nA x nB pairs (float32
 * matrix-core tiles + refinement as in prohd_hd).
 *
 *   nn2A   device float32, nA entries, or NULL: per row of A the squared
 *          distance to its nearest row of B, as found by the float32 tile
 *          search (before refinement); likewise nn2B (nB entries).  When
 *          either is non-null PROHD_PRUNE is ignored (every row's minimum is
 *          then searched over the whole other set).
 * Errors: as prohd_hd.
 */
prohd_status exact_hd(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                      uint32_t flags, prohd_result* out, float* nn2A, float* nn2B,
                      void* ws, size_t ws_bytes, void* stream);

/*
 * exact_hd_noalloc -- exact_hd without a workspace argument and without any
 * allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * Computes what exact_hd computes, with the same kernels, into `out` (and
 * nn2A / nn2B when non-null).  Its scratch is a file-scope device array of
 * PROHD_NOALLOC_SCRATCH_BYTES (64 MiB) in the library, one per GPU, held
 * until the process ends; the sets must fit in it (the same bytes as
 * exact_hd's workspace: about (nA + nB) (4 DP + 42) bytes in float32, with
 * DP = D rounded up to a power of two >= 16, plus 2 DP per row for bfloat16
 * or 1 DP for float8; e.g. nA + nB up to about 60 000 rows at D = 256,
 * 380 000 at D = 32), otherwise PROHD_EWORKSPACE before any launch.  The
 * first call on a device looks up that device's copy of the array; the
 * call then makes no allocation of any kind (no hipMalloc, no library
 * allocation) and every launch is a kernel (no memset), so it can be
 * captured into a graph.  Kernel timing (prohd_profile_enable) must be off.
 *
 * Every call on a GPU uses that GPU's one array, which keeps the previous
 * call's contents (each call initialises what it needs): calls that overlap
 * in time on one GPU -- on different streams, or from different threads --
 * race on it and give undefined results.  Serialise them.
 *
 *   flags  PROHD_PREC_BF16 or PROHD_PREC_FP8 (or 0); PROHD_SYNC is not
 *          accepted (the call never blocks: read out->status after the
 *          stream has completed)
 * Errors: EINVAL, EUNSUPPORTED, EWORKSPACE (sets too large for the
 * scratch), EDEVICE.
 */
#define PROHD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
prohd_status exact_hd_noalloc(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                              uint32_t flags, prohd_result* out, float* nn2A, float* nn2B,
                              void* stream);

/*
 * Learned candidate proposal (an extension of the candidate selection of
 * Alg. 1 / Alg. 2, not in the paper).  A scorer MLP 2D -> 256 -> 128 -> 1
 * with GELU activations reads the per-point features f = [x, x - c_other]
 * (c_other: centroid of the other set) and scores how likely a point is to
 * be a Hausdorff witness.  Matrix products run on bfloat16 weights and
 * activations with float32 accumulation; parameters are a float32 master
 * vector, layout [W1 (256 x 2D row-major), b1 (256), W2 (128 x 256),
 * b2 (128), w3 (128), b3 (1)].  All pointers are device memory.
 */
/* Number of float32 parameters for dimension D (host). */
size_t prohd_mlp_param_count(int32_t D);
/* Workspace bytes for scoring or a gradient step over up to `rows` rows. */
size_t prohd_mlp_workspace_size(int64_t rows, int32_t D);
/* Deterministic initialisation of `params` (uniform Glorot weights, zero
 * biases) from `seed`. */
prohd_status prohd_mlp_init(float* params, int32_t D, uint64_t seed, void* stream);
/* scores[i] = network(f(X_i)) for i < n. */
prohd_status prohd_mlp_score(const float* X, int64_t n, int32_t D, const float* c_other,
                             const float* params, float* scores, void* ws, size_t ws_bytes,
                             void* stream);
/* Gradient of the mean weighted binary cross-entropy with logits
 *   l = pos_weight * y softplus(-s) + (1 - y) softplus(s)
 * over the batch rows X[idx[i]] (labels[idx[i]] in {0, 1}), i < batch
 * (batch <= 65536).  grad: param_count floats (overwritten); loss: one float. */
prohd_status prohd_mlp_grad(const float* X, int32_t D, const float* c_other, const float* labels,
                            const int32_t* idx, int64_t batch, float pos_weight,
                            const float* params, float* grad, float* loss, void* ws,
                            size_t ws_bytes, void* stream);
/* One AdamW step (decoupled weight decay) at step number t >= 1. */
prohd_status prohd_mlp_adamw(float* params, const float* grad, float* m, float* v, int32_t D,
                             int64_t t, float lr, float weight_decay, float beta1, float beta2,
                             float eps, void* stream);
/* One training step: prohd_mlp_grad, then prohd_mlp_adamw at step t with
 * the gradient it wrote (grad is overwritten). */
prohd_status prohd_mlp_train_step(const float* X, int32_t D, const float* c_other,
                                  const float* labels, const int32_t* idx, int64_t batch,
                                  float pos_weight, float* params, float* grad, float* m, float* v,
                                  int64_t t, float lr, float weight_decay, float beta1, float beta2,
                                  float eps, float* loss, void* ws, size_t ws_bytes, void* stream);
/* Centroid (column mean, float64 accumulation, float32 result) of the n x D
 * set X (Alg. 1 forms it for both sets); the scorer's c_other.  `mean`: D
 * floats, device.  ws_bytes must be >= PROHD_CENTROID_WS_BYTES(D). */
#define PROHD_CENTROID_WS_BYTES(D) ((size_t)1024 * (size_t)(D) * 8u + 256u)
prohd_status prohd_centroid(const float* X, int64_t n, int32_t D, float* mean, void* ws,
                            size_t ws_bytes, void* stream);
/* Adds the sA (sB) highest-scoring rows of A (B) to the selected lists
 * idxA/nselA (idxB/nselB) in place: the result is the ascending unique union.
 * Ties in the scores go to the smaller index.  capA must be >= min(nA,
 * capacity bound of the existing list + sA); likewise capB. */
prohd_status prohd_select_scored(const float* scoresA, int64_t nA, int32_t sA,
                                 const float* scoresB, int64_t nB, int32_t sB,
                                 int32_t* idxA, int64_t capA, int64_t* nselA,
                                 int32_t* idxB, int64_t capB, int64_t* nselB,
                                 void* ws, size_t ws_bytes, void* stream);

/*
 * Batched form: P independent pairs (uneven sizes, each with its own D) in
 * one graph of persistent launches.  Pair i's rows are packed row-major:
 * A holds nA[0] x D[0] floats, then nA[1] x D[1], ...; likewise B.
 *
 *   prohd_batch_create   host plan for fixed sizes; alpha-mode ProHD with
 *                        m = floor(sqrt(D)) per pair (Alg. 1-3).  The plan
 *                        owns a small device table area and a private
 *                        capture stream (freed by prohd_batch_destroy).
 *   prohd_batch_run      mode PROHD_BATCH_PROHD: Alg. 3's candidate value
 *                        per pair (as prohd_project + prohd_select +
 *                        prohd_hd); PROHD_BATCH_EXACT: Eq. (1) per pair (as
 *                        exact_hd; pairs whose sets both have at least
 *                        16384 rows take exact_hd's pruned search, one
 *                        after another in the same launch list, the others
 *                        the batched kernels).  out[i] receives pair i's
 *                        result (device
 *                        memory, P entries).  The first run with a given
 *                        (mode, A, B, out, ws) builds the work tables and
 *                        captures the launches into a graph; later runs
 *                        launch that graph on `stream`.  PROHD_BATCH_EAGER
 *                        launches the kernels directly instead; PROHD_SYNC
 *                        waits for completion.  Not thread-safe per plan.
 *   prohd_batch_tune     times candidate work shapes (rows per covariance
 *                        slice, rows per distance item, work-groups per
 *                        compute unit) on the bound batch with the kernel
 *                        timers, keeps the fastest and, when json_path is
 *                        non-null, writes them with the trials as JSON.
 *   prohd_batch_load_tuning  reads such a file back.
 * Errors: EINVAL (arguments), EUNSUPPORTED (D > 256), EWORKSPACE,
 * EDEVICE.  Device-detected errors (non-finite rows) go to out[i].status.
 */
typedef struct prohd_batch prohd_batch;
#define PROHD_BATCH_PROHD 0u
#define PROHD_BATCH_EXACT 1u
#define PROHD_BATCH_EAGER (1u << 5)
prohd_status prohd_batch_create(int32_t P, const int64_t* nA, const int64_t* nB, const int32_t* D,
                                double alpha, prohd_batch** plan);
void prohd_batch_destroy(prohd_batch* plan);
size_t prohd_batch_workspace_size(const prohd_batch* plan, uint32_t mode);
prohd_status prohd_batch_run(prohd_batch* plan, uint32_t mode, const float* A, const float* B,
                             prohd_result* out, void* ws, size_t ws_bytes, uint32_t flags,
                             void* stream);
prohd_status prohd_batch_tune(prohd_batch* plan, uint32_t mode, const float* A, const float* B,
                              prohd_result* out, void* ws, size_t ws_bytes, void* stream,
                              const char* json_path);
prohd_status prohd_batch_load_tuning(prohd_batch* plan, const char* json_path);

/*
 * prohd_certificate -- a certified interval for the true distance H(A,B)
 * from the projections ProHD already made (Sec. II-E: H_u <= H <= H_u +
 * 2 delta(u) for every direction u, delta measured from the line through
 * the centroid of A u B, which the bound allows since H and H_u are
 * translation invariant).
 *
 *   dirs, projA, projB  the outputs of prohd_project (ndirs = m + 1 rows).
 *   lower   device prohd_result whose H is known to be <= H(A,B) -- the
 *           result of prohd_hd with PROHD_INNER_FULL -- or NULL.
 *   out     device prohd_cert: lb <= H(A,B) <= ub, with lb = max(max_u lower
 *           bound of H_u, lower->H) and ub = min_u (upper bound of H_u +
 *           2 delta(u)); hu_lo / hu_hi bound H_U = max_u H_u; delta_min =
 *           min_u delta(u); proj_err = bound of the float32 projection
 *           error used to widen the H_u bounds; best_dir = the u giving ub.
 * The bounds account for float32 rounding of the projections (rigorous for
 * finite inputs).  Workspace: prohd_certificate_workspace_size(D, ndirs).
 * Errors: EINVAL, EUNSUPPORTED (D > 256 or ndirs > 64), EWORKSPACE.
 */
typedef struct {
  double lb, ub;
  double hu_lo, hu_hi;
  double delta_min;
  double proj_err;
  int32_t best_dir;
  int32_t status;
} prohd_cert;

size_t prohd_certificate_workspace_size(int32_t D, int32_t ndirs);
prohd_status prohd_certificate(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                               const float* dirs, int32_t ndirs, const float* projA,
                               const float* projB, const prohd_result* lower, prohd_cert* out,
                               void* ws, size_t ws_bytes, void* stream);

/*
 * prohd_adaptive -- alpha chosen under an error budget (this library's
 * schedule for the adaptive alpha the paper's Conclusion names as future
 * work; Sec. III shows the error falling as alpha grows).
 *
 * Directions (Alg. 1, Alg. 2, m = floor(sqrt(D))) and projections are
 * computed once, with the Sec. II-E certificate of those directions
 * (prohd_certificate: hu_lo <= H_U and ub >= H(A,B)).  Then for
 * alpha_j = min(alpha0 growth^j, alpha_max), j = 0, 1, ..., the alpha-mode
 * candidates (prohd_alpha_k, prohd_select) give the inner-full value
 *   F_j = max{ h(A_sel, B), h(B_sel, A) }   (prohd_hd with PROHD_INNER_FULL),
 * which never exceeds H(A,B) and cannot decrease as alpha grows (the
 * candidate sets are nested).  The schedule stops at the first j with
 *   ub - max(hu_lo, F_j) <= tol max(hu_lo, F_j)   reason 1 (certified gap)
 *   j >= 1 and F_j - F_{j-1} <= tol F_j          reason 2 (converged)
 *   alpha_j >= alpha_max                         reason 3
 * Only reason 1 certifies the relative error; reason 2 is the empirical
 * rule (no further gain from a growth-fold larger alpha).
 *
 *   alpha0, growth, alpha_max   0 < alpha0 <= alpha_max, growth > 1
 *   tol      relative budget (>= 0)
 *   flags    PROHD_PREC_BF16 / PROHD_PREC_FP8 for the distance search (or 0)
 *   out      device prohd_result: the last step's inner-full result
 *   res      HOST prohd_adaptive_result, output
 * Workspace: prohd_adaptive_workspace_size(nA, nB, D, alpha_max, flags).
 * The call blocks: it reads each step's result on the host (the schedule is
 * decided there).  Errors: EINVAL, EUNSUPPORTED, EWORKSPACE, EDEVICE, and
 * the device status of the projection / distance (ENONFINITE).
 */
typedef struct {
  double alpha;     /* alpha of the last step                               */
  double H;         /* its inner-full value F (<= H(A,B))                   */
  double lb, ub;    /* certified interval: lb = max(hu_lo, F) <= H <= ub    */
  double change;    /* (F_j - F_{j-1}) / F_j of the last step, -1 at j = 0   */
  int64_t nA_sel, nB_sel;  /* candidate-set sizes of the last step          */
  int32_t steps;    /* alphas tried                                         */
  int32_t reason;   /* 1 certified gap, 2 converged, 3 alpha_max reached    */
} prohd_adaptive_result;

size_t prohd_adaptive_workspace_size(int64_t nA, int64_t nB, int32_t D, double alpha_max,
                                     uint32_t flags);
prohd_status prohd_adaptive(const float* A, int64_t nA, const float* B, int64_t nB, int32_t D,
                            double alpha0, double growth, double alpha_max, double tol,
                            uint32_t flags, prohd_result* out, prohd_adaptive_result* res,
                            void* ws, size_t ws_bytes, void* stream);

/* Message of the last non-OK return on this host thread ("" if none). */
const char* prohd_last_error(void);

/* Library version string. */
const char* prohd_version(void);

/*
 * Kernel timing (host).  While enabled, every kernel the library launches
 * is bracketed by HIP events on the stream it runs on.  prohd_profile_read
 * waits for those events and returns, for kernels whose name contains
 * `name`, the number of launches and their summed duration in ms since the
 * last reset.  Returns PROHD_OK or EINVAL / EDEVICE.
 */
prohd_status prohd_profile_enable(int32_t on);
prohd_status prohd_profile_reset(void);
prohd_status prohd_profile_read(const char* name, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* PROHD_H */
