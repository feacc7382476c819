/*
 * Accuracy metrics used by the tests (TEST INFRASTRUCTURE ONLY).
 *
 *   orthogonality  ||Q^T Q - I||_F
 *   residual       ||Q R - X||_F   (and ||X||_F for the relative form)
 *
 * These are the two accuracy measures of the paper's experiments (Section 5).
 * Every dot product is evaluated with the compensated "Dot2" scheme of Ogita,
 * Rump and Oishi (SIAM J. Sci. Comput. 26, 2005): error-free TwoSum and
 * TwoProduct (via fma) accumulate the rounding errors, so the measured value
 * is not polluted by the checker's own rounding, even for m in the millions.
 * Loops run over fixed row blocks in order, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CHK_BLOCK 2048

static inline void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}
static inline void two_prod(double a, double b, double* p, double* e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

/* orth = ||Q^T Q - I||_F, Q m x n (ld ldq). */
double chk_orthogonality(const double* Q, int64_t m, int64_t n, int64_t ldq) {
  size_t np = (size_t)n * (size_t)n;
  double* hi = (double*)calloc(np, sizeof(double));
  double* lo = (double*)calloc(np, sizeof(double));
  for (int64_t r0 = 0; r0 < m; r0 += CHK_BLOCK) {
    int64_t r1 = r0 + CHK_BLOCK < m ? r0 + CHK_BLOCK : m;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
      const double* qj = Q + j * ldq;
      for (int64_t i = 0; i <= j; ++i) {
        const double* qi = Q + i * ldq;
        double s = hi[i + j * n], c = lo[i + j * n];
        for (int64_t r = r0; r < r1; ++r) {
          double p, ep, es;
          two_prod(qi[r], qj[r], &p, &ep);
          two_sum(s, p, &s, &es);
          c += ep + es;
        }
        hi[i + j * n] = s;
        lo[i + j * n] = c;
      }
    }
  }
  double acc = 0.0;
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) {
      double t = (hi[i + j * n] - (i == j ? 1.0 : 0.0)) + lo[i + j * n];
      acc += (i == j ? 1.0 : 2.0) * t * t;
    }
  free(hi);
  free(lo);
  return sqrt(acc);
}

/* res = ||Q R - X||_F with R upper triangular (n x n, ld n); xnorm = ||X||_F. */
void chk_residual(const double* X, int64_t ldx, const double* Q, int64_t ldq, const double* R, int64_t m, int64_t n,
                  double* res, double* xnorm) {
  int64_t nblk = (m + CHK_BLOCK - 1) / CHK_BLOCK;
  double* pr = (double*)calloc((size_t)nblk, sizeof(double));
  double* px = (double*)calloc((size_t)nblk, sizeof(double));
#pragma omp parallel
  {
    double* qrow = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
    for (int64_t b = 0; b < nblk; ++b) {
      int64_t r0 = b * CHK_BLOCK, r1 = r0 + CHK_BLOCK < m ? r0 + CHK_BLOCK : m;
      double sr = 0.0, sx = 0.0;
      for (int64_t r = r0; r < r1; ++r) {
        for (int64_t k = 0; k < n; ++k) qrow[k] = Q[r + k * ldq];
        for (int64_t j = 0; j < n; ++j) {
          double x = X[r + j * ldx];
          double s = -x, c = 0.0;
          for (int64_t k = 0; k <= j; ++k) {
            double p, ep, es;
            two_prod(qrow[k], R[k + j * n], &p, &ep);
            two_sum(s, p, &s, &es);
            c += ep + es;
          }
          double t = s + c;
          sr += t * t;
          sx += x * x;
        }
      }
      pr[b] = sr;
      px[b] = sx;
    }
    free(qrow);
  }
  double a = 0.0, bx = 0.0;
  for (int64_t b = 0; b < nblk; ++b) {
    a += pr[b];
    bx += px[b];
  }
  free(pr);
  free(px);
  *res = sqrt(a);
  *xnorm = sqrt(bx);
}
