/* Row and column minima of one block of squared distances -- test
 * infrastructure only (part of the FP64 oracle; nothing in the product links
 * it).
 *
 * Given G = Q R^T for a block of rows of Q (rows i0 .. i0+nq-1) and of R
 * (rows j0 .. j0+nr-1), the squared Euclidean distance of Eq. (1) is
 *   d2(i, j) = |q_i|^2 + |r_j|^2 - 2 G[i][j]        (FP64 throughout).
 * nn_block keeps, per row i, the smallest d2 over the block's columns and
 * its column index (rowd / rowj), and per column j the smallest d2 over the
 * block's rows and its row index (cold / coli).  Indices are visited in
 * ascending order and only a strictly smaller value replaces the kept one,
 * so ties keep the smallest index (the oracle's tie rule), also across
 * blocks when the caller visits blocks in ascending index order.
 *
 * Plain loops.  OpenMP gives each thread a contiguous range of rows; a
 * thread keeps its own column minima, and these are merged in thread order
 * (ascending rows), so the result does not depend on the thread count.  The
 * row minimum is found in two scans of the row (the smallest value, then the
 * first column that reaches it), which gives the same value and index as one
 * scan with a strict comparison.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

int nn_block(const double* G, int64_t nq, int64_t nr, const double* qn, const double* rn,
             int64_t i0, int64_t j0, double* rowd, int64_t* rowj, double* cold, int64_t* coli) {
  const int T = omp_get_max_threads();
  double* cd = (double*)malloc(sizeof(double) * (size_t)T * (size_t)nr);
  int64_t* ci = (int64_t*)malloc(sizeof(int64_t) * (size_t)T * (size_t)nr);
  if (!cd || !ci) {
    free(cd);
    free(ci);
    return 1;
  }
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    const int nt = omp_get_num_threads();
    double* mycd = cd + (size_t)t * nr;
    int64_t* myci = ci + (size_t)t * nr;
    for (int64_t j = 0; j < nr; ++j) {
      mycd[j] = INFINITY;
      myci[j] = -1;
    }
    const int64_t r0 = nq * t / nt, r1 = nq * (t + 1) / nt;
    for (int64_t i = r0; i < r1; ++i) {
      const double* g = G + i * nr;
      const double q = qn[i];
      const int64_t ii = i0 + i;
      double m = rowd[i];
#pragma omp simd reduction(min : m)
      for (int64_t j = 0; j < nr; ++j) {
        const double d2 = q + rn[j] - 2.0 * g[j];
        m = d2 < m ? d2 : m;
        const int lt = d2 < mycd[j];
        mycd[j] = lt ? d2 : mycd[j];
        myci[j] = lt ? ii : myci[j];
      }
      if (m < rowd[i]) {
        for (int64_t j = 0; j < nr; ++j) {
          if (q + rn[j] - 2.0 * g[j] == m) {
            rowd[i] = m;
            rowj[i] = j0 + j;
            break;
          }
        }
      }
    }
#pragma omp barrier
    /* merge the threads' column minima in thread order */
#pragma omp for schedule(static)
    for (int64_t j = 0; j < nr; ++j) {
      for (int s = 0; s < nt; ++s) {
        const double v = cd[(size_t)s * nr + j];
        if (v < cold[j]) {
          cold[j] = v;
          coli[j] = ci[(size_t)s * nr + j];
        }
      }
    }
  }
  free(cd);
  free(ci);
  return 0;
}
