/*
 * CPU FP64 oracle for the randomized LU-preconditioned CholeskyQR methods
 * (RCLUPP, RCLUPPr) and the baselines they are compared with (CholeskyQR2,
 * Shifted CholeskyQR3, LU-CholeskyQR2, randomized CholeskyQR).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, step-by-step
 * reference that the GPU library is checked against. Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no
 * code, header, table or constant with the GPU library.
 *
 * Conventions
 *   - every matrix is float64, column-major: element (i, j) of a matrix with
 *     leading dimension ld sits at A[i + j*ld];
 *   - X is m x n with m >= n (Section 1: tall-skinny, full column rank);
 *   - info is int32[4] = {code, stage, index (1-based column), 0}.
 *
 * Readings where the paper is silent (they are listed with reasons in the
 * design notes of the repository):
 *   - the sketch S = G / sqrt(s) (Section 3, Gaussian sketch) uses
 *     G_ij = z(seed, i, j) from Philox4x32-10 (Salmon et al., SC'11) with
 *     counter (q lo, q hi, i, 0), q = floor(j/4), and key (seed lo, seed hi);
 *     the four output words give u_t = (floor(w_t / 2^9) + 1/2) * 2^-23 and
 *     the Box-Muller pairs (u0,u1) -> tall rows 4q, 4q+1 and (u2,u3) -> 4q+2,
 *     4q+3; each normal is rounded to float32;
 *   - sums over the tall dimension (sketch, Gram, norms) are taken
 *     sequentially inside blocks of ORC_BLOCK rows, and the block partial sums
 *     are added in block order;
 *   - LU with partial pivoting picks the first row of largest magnitude;
 *   - Householder vectors follow the LAPACK dlarfg convention; only R is kept;
 *   - R_1 gets the signs of its diagonal folded in (row scaling by +-1) so the
 *     final R has a positive diagonal;
 *   - the triangular solve is row-wise substitution (no explicit inverse);
 *   - the elimination of the LU and the sums of the substitution use fused
 *     multiply-add (one rounding per term) and true division; the error model
 *     of Section 3 (eqs. elu and ewy) bounds either choice, but outcomes on
 *     problems outside its conditions (kappa(M) kappa(N) near 1/u) depend on it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_BLOCK 4096

/* Multiply-add of the LU elimination and of the substitution. The oracle's
 * reading is one rounding per term (fused). Built with -DORC_SEPARATE_MULADD
 * the product and the sum are rounded separately: the other reading, kept to
 * record how outcomes outside the conditions of eq. (s4) depend on it. */
#ifdef ORC_SEPARATE_MULADD
#define ORC_MULADD(a, b, c) ((a) * (b) + (c))
#else
#define ORC_MULADD(a, b, c) fma((a), (b), (c))
#endif

/* info codes */
#define ORC_OK 0
#define ORC_LU_ZERO_PIVOT 1
#define ORC_CHOL_BREAKDOWN 2
#define ORC_NONFINITE 3
#define ORC_SINGULAR 4
/* stages: the role of the small factorization in the pipeline */
#define ORC_ST_LU 1      /* LU with partial pivoting (of the sketch, or of X)      */
#define ORC_ST_QR 2      /* R factor of the (sketched) L factor                     */
#define ORC_ST_PRECOND 3 /* preconditioner R_1 (R_0 N, or the first Cholesky)       */
#define ORC_ST_CHOL_A 4  /* Cholesky of the first Gram after preconditioning (R_2)  */
#define ORC_ST_CHOL_B 5  /* Cholesky of the second Gram (R_4)                       */

static void set_info(int32_t* info, int32_t code, int32_t stage, int64_t index) {
  if (info && info[0] == ORC_OK) {
    info[0] = code;
    info[1] = stage;
    info[2] = (int32_t)index;
    info[3] = 0;
  }
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the      */
/* Philox S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and the Weyl key    */
/* schedule 0x9E3779B9 / 0xBB67AE85.                                        */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Four standard normals of sketch row i for tall rows 4q..4q+3 (Box-Muller).
 * The transform is evaluated in double and each normal rounded to float. */
void orc_normals4(uint64_t seed, uint64_t q, uint32_t i, float z[4]) {
  uint32_t ctr[4] = {(uint32_t)q, (uint32_t)(q >> 32), i, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  double u[4];
  for (int t = 0; t < 4; ++t) u[t] = ((double)(w[t] >> 9) + 0.5) * 0x1p-23;
  const double two_pi = 6.283185307179586476925286766559;
  double r0 = sqrt(-2.0 * log(u[0]));
  double r1 = sqrt(-2.0 * log(u[2]));
  z[0] = (float)(r0 * cos(two_pi * u[1]));
  z[1] = (float)(r0 * sin(two_pi * u[1]));
  z[2] = (float)(r1 * cos(two_pi * u[3]));
  z[3] = (float)(r1 * sin(two_pi * u[3]));
}

/* Columns 4q .. 4q+3 of Omega = G / sqrt(s): out[t*s + i] = z(seed, i, 4q+t) / sqrt(s). */
static void omega_group(uint64_t seed, uint64_t q, int64_t s, double* out) {
  double scale = 1.0 / sqrt((double)s);
  for (int64_t i = 0; i < s; ++i) {
    float z[4];
    orc_normals4(seed, q, (uint32_t)i, z);
    for (int t = 0; t < 4; ++t) out[t * s + i] = (double)z[t] * scale;
  }
}

/* Omega[:, j0 .. j0+cols) materialised (s x cols, ld s). */
void orc_omega(uint64_t seed, int64_t s, int64_t j0, int64_t cols, double* Om) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < cols; ++c) {
    double* om4 = (double*)malloc(sizeof(double) * 4 * (size_t)s);
    const uint64_t j = (uint64_t)(j0 + c);
    omega_group(seed, j / 4, s, om4);
    memcpy(Om + c * s, om4 + (j % 4) * s, sizeof(double) * (size_t)s);
    free(om4);
  }
}

/* ------------------------------------------------------------------------ */
/* Sketch Y = Omega X (Algorithm 2, first step; Algorithm 7, second step).   */
/* Omega column index j is the row index of the tall operand.               */
/* ------------------------------------------------------------------------ */
void orc_sketch(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Y) {
  int64_t nblk = (m + ORC_BLOCK - 1) / ORC_BLOCK;
  int64_t batch = 2 * (int64_t)orc_max_threads();
  size_t psz = (size_t)s * (size_t)n;
  double* part = (double*)malloc(sizeof(double) * psz * (size_t)batch);
  for (size_t e = 0; e < psz; ++e) Y[e] = 0.0;
  for (int64_t b0 = 0; b0 < nblk; b0 += batch) {
    int64_t nb = (nblk - b0 < batch) ? (nblk - b0) : batch;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t bb = 0; bb < nb; ++bb) {
      double* P = part + (size_t)bb * psz;
      double* om4 = (double*)malloc(sizeof(double) * 4 * (size_t)s);
      for (size_t e = 0; e < psz; ++e) P[e] = 0.0;
      int64_t r0 = (b0 + bb) * ORC_BLOCK; /* a multiple of 4 */
      int64_t r1 = r0 + ORC_BLOCK < m ? r0 + ORC_BLOCK : m;
      for (int64_t j = r0; j < r1; ++j) {
        if (j % 4 == 0) omega_group(seed, (uint64_t)j / 4, s, om4);
        const double* om = om4 + (j % 4) * s;
        for (int64_t k = 0; k < n; ++k) {
          double xjk = X[j + k * ldx];
          double* Pk = P + k * s;
          for (int64_t i = 0; i < s; ++i) Pk[i] += om[i] * xjk;
        }
      }
      free(om4);
    }
    for (int64_t bb = 0; bb < nb; ++bb) {
      const double* P = part + (size_t)bb * psz;
      for (size_t e = 0; e < psz; ++e) Y[e] += P[e];
    }
  }
  free(part);
}

/* ------------------------------------------------------------------------ */
/* CountSketch (Section 3 names it among the common choices of S): column j  */
/* of S has a single entry sigma_j = +-1, in row h_j, so Y = S X adds +-row  */
/* j of X into row h_j of Y (no scaling: E[S^T S] = I). h_j and sigma_j are  */
/* drawn from Philox4x32-10 with counter (q lo, q hi, 0, 1), q = floor(j/4)  */
/* (the Gaussian sketch's counters end in 0), key (seed lo, seed hi): word t */
/* belongs to tall row 4q+t and gives h = floor(w s / 2^32), sigma = +1 for  */
/* even w and -1 for odd w.                                                  */
/* ------------------------------------------------------------------------ */
void orc_countsketch_hash(uint64_t seed, uint64_t j, int64_t s, int64_t* h, double* sigma) {
  uint64_t q = j / 4;
  uint32_t ctr[4] = {(uint32_t)q, (uint32_t)(q >> 32), 0u, 1u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  uint32_t word = w[j % 4];
  *h = (int64_t)(((uint64_t)word * (uint64_t)s) >> 32);
  *sigma = (word & 1u) ? -1.0 : 1.0;
}

/* Y = S X with the rows added in increasing order inside blocks of ORC_BLOCK
 * rows and the block sums added in block order (as the Gaussian sketch). */
void orc_countsketch(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Y) {
  int64_t nblk = (m + ORC_BLOCK - 1) / ORC_BLOCK;
  int64_t batch = 2 * (int64_t)orc_max_threads();
  size_t psz = (size_t)s * (size_t)n;
  double* part = (double*)malloc(sizeof(double) * psz * (size_t)batch);
  for (size_t e = 0; e < psz; ++e) Y[e] = 0.0;
  for (int64_t b0 = 0; b0 < nblk; b0 += batch) {
    int64_t nb = (nblk - b0 < batch) ? (nblk - b0) : batch;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t bb = 0; bb < nb; ++bb) {
      double* P = part + (size_t)bb * psz;
      for (size_t e = 0; e < psz; ++e) P[e] = 0.0;
      int64_t r0 = (b0 + bb) * ORC_BLOCK;
      int64_t r1 = r0 + ORC_BLOCK < m ? r0 + ORC_BLOCK : m;
      for (int64_t j = r0; j < r1; ++j) {
        int64_t h;
        double sg;
        orc_countsketch_hash(seed, (uint64_t)j, s, &h, &sg);
        for (int64_t k = 0; k < n; ++k) P[h + k * s] += sg * X[j + k * ldx];
      }
    }
    for (int64_t bb = 0; bb < nb; ++bb) {
      const double* P = part + (size_t)bb * psz;
      for (size_t e = 0; e < psz; ++e) Y[e] += P[e];
    }
  }
  free(part);
}

/* ------------------------------------------------------------------------ */
/* SRHT, the subsampled randomized Hadamard transform (Section 3 lists it     */
/* among the common sketches): S = sqrt(m'/s) R H D, with m' = 2^k the       */
/* smallest power of two >= m (X taken as padded with zero rows), D = diag   */
/* of random signs d_j, H the Walsh-Hadamard matrix of order m' normalized   */
/* by 1/sqrt(m') (Sylvester order: H[r][j] = (-1)^popcount(r & j) / sqrt(m')) */
/* and R the s rows r_0 .. r_{s-1} of a random permutation of [0, m').       */
/* Entry (i, j) of S is thus (-1)^popcount(r_i & j) d_j / sqrt(s).           */
/* d_j: Philox4x32-10 with counter (q lo, q hi, 0, 2), q = floor(j/4), key   */
/* (seed lo, seed hi); word j mod 4, d_j = -1 for odd words.                 */
/* r_i = pi(i), pi(x) = f3(f2(f1(x))) on k-bit integers: f1(x) = a1 x + b1,  */
/* f2(x) = x xor (x >> ceil(k/2)), f3(x) = a2 x + b2 (mod 2^k; a1, a2 odd);   */
/* each step is a bijection of [0, 2^k), so the r_i are distinct. (a1, b1,   */
/* a2, b2) = the words of Philox4x32-10 at counter (0, 0, 0, 3), a1 and a2    */
/* with their low bit set.                                                   */
/* ------------------------------------------------------------------------ */
static int srht_log2(int64_t m) {
  int k = 0;
  while (((int64_t)1 << k) < m) ++k;
  return k;
}

double orc_srht_sign(uint64_t seed, uint64_t j) {
  uint64_t q = j / 4;
  uint32_t ctr[4] = {(uint32_t)q, (uint32_t)(q >> 32), 0u, 2u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  return (w[j % 4] & 1u) ? -1.0 : 1.0;
}

int64_t orc_srht_row(uint64_t seed, int64_t m, int64_t i) {
  const int k = srht_log2(m);
  if (k == 0) return 0;
  uint32_t ctr[4] = {0u, 0u, 0u, 3u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  const uint64_t mask = ((uint64_t)1 << k) - 1;
  uint64_t x = (uint64_t)i;
  x = ((uint64_t)(w[0] | 1u) * x + w[1]) & mask;
  x = x ^ (x >> ((k + 1) / 2));
  x = ((uint64_t)(w[2] | 1u) * x + w[3]) & mask;
  return (int64_t)x;
}

/* Y = S X, summed as the Gaussian sketch (rows in order inside blocks of
 * ORC_BLOCK rows, the block sums in block order). */
void orc_srht(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Y) {
  int64_t nblk = (m + ORC_BLOCK - 1) / ORC_BLOCK;
  int64_t batch = 2 * (int64_t)orc_max_threads();
  size_t psz = (size_t)s * (size_t)n;
  double* part = (double*)malloc(sizeof(double) * psz * (size_t)batch);
  int64_t* r = (int64_t*)malloc(sizeof(int64_t) * (size_t)s);
  const double scale = 1.0 / sqrt((double)s);
  for (int64_t i = 0; i < s; ++i) r[i] = orc_srht_row(seed, m, i);
  for (size_t e = 0; e < psz; ++e) Y[e] = 0.0;
  for (int64_t b0 = 0; b0 < nblk; b0 += batch) {
    int64_t nb = (nblk - b0 < batch) ? (nblk - b0) : batch;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t bb = 0; bb < nb; ++bb) {
      double* P = part + (size_t)bb * psz;
      double* col = (double*)malloc(sizeof(double) * (size_t)s);
      for (size_t e = 0; e < psz; ++e) P[e] = 0.0;
      int64_t r0 = (b0 + bb) * ORC_BLOCK;
      int64_t r1 = r0 + ORC_BLOCK < m ? r0 + ORC_BLOCK : m;
      for (int64_t j = r0; j < r1; ++j) {
        const double d = orc_srht_sign(seed, (uint64_t)j) * scale;
        for (int64_t i = 0; i < s; ++i) col[i] = (__builtin_popcountll((uint64_t)(r[i] & j)) & 1) ? -d : d;
        for (int64_t k = 0; k < n; ++k) {
          double xjk = X[j + k * ldx];
          double* Pk = P + k * s;
          for (int64_t i = 0; i < s; ++i) Pk[i] += col[i] * xjk;
        }
      }
      free(col);
    }
    for (int64_t bb = 0; bb < nb; ++bb) {
      const double* P = part + (size_t)bb * psz;
      for (size_t e = 0; e < psz; ++e) Y[e] += P[e];
    }
  }
  free(r);
  free(part);
}

/* The sketch of a method: Gaussian (no sketch flag), CountSketch or SRHT. */
#define ORC_SKETCH_COUNT 1
#define ORC_LU_TOURNAMENT 2 /* RCLUPPr, LC2: tournament pivoting (orc_tslu) */
#define ORC_SKETCH_SRHT 4
static void method_sketch(int flags, const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed,
                          double* Y) {
  if (flags & ORC_SKETCH_COUNT)
    orc_countsketch(X, m, n, ldx, s, seed, Y);
  else if (flags & ORC_SKETCH_SRHT)
    orc_srht(X, m, n, ldx, s, seed, Y);
  else
    orc_sketch(X, m, n, ldx, s, seed, Y);
}

/* ------------------------------------------------------------------------ */
/* Gram matrix G = W^T W (Algorithm 1, first step), upper triangle summed,   */
/* then mirrored.                                                           */
/* ------------------------------------------------------------------------ */
void orc_gram(const double* W, int64_t m, int64_t n, int64_t ldw, double* G) {
  int64_t nblk = (m + ORC_BLOCK - 1) / ORC_BLOCK;
  int64_t batch = 2 * (int64_t)orc_max_threads();
  size_t psz = (size_t)n * (size_t)n;
  double* part = (double*)malloc(sizeof(double) * psz * (size_t)batch);
  for (size_t e = 0; e < psz; ++e) G[e] = 0.0;
  for (int64_t b0 = 0; b0 < nblk; b0 += batch) {
    int64_t nb = (nblk - b0 < batch) ? (nblk - b0) : batch;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t bb = 0; bb < nb; ++bb) {
      double* P = part + (size_t)bb * psz;
      int64_t r0 = (b0 + bb) * ORC_BLOCK;
      int64_t r1 = r0 + ORC_BLOCK < m ? r0 + ORC_BLOCK : m;
      for (int64_t j = 0; j < n; ++j) {
        const double* wj = W + j * ldw;
        for (int64_t i = 0; i <= j; ++i) {
          const double* wi = W + i * ldw;
          double acc = 0.0;
          for (int64_t r = r0; r < r1; ++r) acc += wi[r] * wj[r];
          P[i + j * n] = acc;
        }
      }
    }
    for (int64_t bb = 0; bb < nb; ++bb) {
      const double* P = part + (size_t)bb * psz;
      for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i <= j; ++i) G[i + j * n] += P[i + j * n];
    }
  }
  free(part);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = j + 1; i < n; ++i) G[i + j * n] = G[j + i * n];
}

/* ------------------------------------------------------------------------ */
/* LU with partial pivoting, P A = M N (Algorithm 2 step 2, Algorithm 5/7    */
/* step 1), in place on A (r x n, r >= n). On return the strict lower part   */
/* of A holds M (unit diagonal implied) and the upper n x n part holds N.    */
/* perm[p] = original index of the row now at position p.                   */
/* Returns 0, or the failing column k+1 with info set.                      */
/* ------------------------------------------------------------------------ */
int orc_gepp(double* A, int64_t r, int64_t n, int64_t lda, int64_t* perm, int32_t* info, int32_t stage) {
  for (int64_t i = 0; i < r; ++i) perm[i] = i;
  for (int64_t k = 0; k < n; ++k) {
    double* ak = A + k * lda;
    int64_t p = k;
    double best = -1.0;
    for (int64_t i = k; i < r; ++i) {
      double v = ak[i];
      if (!isfinite(v)) {
        set_info(info, ORC_NONFINITE, stage, k + 1);
        return (int)(k + 1);
      }
      if (fabs(v) > best) {
        best = fabs(v);
        p = i;
      }
    }
    if (best == 0.0) {
      set_info(info, ORC_LU_ZERO_PIVOT, stage, k + 1);
      return (int)(k + 1);
    }
    if (p != k) {
      for (int64_t j = 0; j < n; ++j) {
        double t = A[k + j * lda];
        A[k + j * lda] = A[p + j * lda];
        A[p + j * lda] = t;
      }
      int64_t t = perm[k];
      perm[k] = perm[p];
      perm[p] = t;
    }
    double piv = ak[k];
#pragma omp parallel for schedule(static)
    for (int64_t i0 = k + 1; i0 < r; i0 += ORC_BLOCK) {
      int64_t i1 = i0 + ORC_BLOCK < r ? i0 + ORC_BLOCK : r;
      for (int64_t i = i0; i < i1; ++i) ak[i] = ak[i] / piv;
      for (int64_t j = k + 1; j < n; ++j) {
        double akj = A[k + j * lda];
        double* aj = A + j * lda;
        for (int64_t i = i0; i < i1; ++i) aj[i] = ORC_MULADD(-ak[i], akj, aj[i]);
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Tournament pivoting (TSLU: Grigori, Demmel and Xiang, SIAM J. Matrix     */
/* Anal. Appl. 2011) for the LU of a tall X with n <= 128, as an alternative */
/* to partial pivoting in Algorithm 7 step 1 and Algorithm 5 step 1:         */
/*   leaves: L = ceil(m / 256) blocks of consecutive rows, block g holding   */
/*     rows floor(g m / L) .. floor((g+1) m / L) - 1; each is factored with  */
/*     partial pivoting (ties to the smaller position) and its first n pivot */
/*     rows are its candidates;                                              */
/*   tree: F = floor(256 / n) consecutive candidate sets stacked in set      */
/*     order are factored the same way, keeping their first n pivot rows,    */
/*     until one set is left;                                                */
/*   root: the last factorization gives sel (pivot order), L_11 and N.       */
/* A column whose candidates are all zero keeps its pivot at position k and  */
/* eliminates nothing below the root; at the root it is a zero pivot.        */
/* ------------------------------------------------------------------------ */
static int tslu_factor(double* A, int64_t r, int64_t n, int64_t* idx, int root, int32_t* info) {
  for (int64_t k = 0; k < n; ++k) {
    double* ak = A + k * r;
    int64_t p = k;
    double best = -1.0;
    for (int64_t i = k; i < r; ++i) {
      if (!isfinite(ak[i])) {
        set_info(info, ORC_NONFINITE, ORC_ST_LU, k + 1);
        return 1;
      }
      if (fabs(ak[i]) > best) {
        best = fabs(ak[i]);
        p = i;
      }
    }
    if (best == 0.0) {
      if (root) {
        set_info(info, ORC_LU_ZERO_PIVOT, ORC_ST_LU, k + 1);
        return 1;
      }
      continue;
    }
    if (p != k) {
      for (int64_t j = 0; j < n; ++j) {
        double t = A[k + j * r];
        A[k + j * r] = A[p + j * r];
        A[p + j * r] = t;
      }
      int64_t t = idx[k];
      idx[k] = idx[p];
      idx[p] = t;
    }
    double piv = ak[k];
    for (int64_t i = k + 1; i < r; ++i) ak[i] = ak[i] / piv;
    for (int64_t j = k + 1; j < n; ++j) {
      double akj = A[k + j * r];
      double* aj = A + j * r;
      for (int64_t i = k + 1; i < r; ++i) aj[i] = ORC_MULADD(-ak[i], akj, aj[i]);
    }
  }
  return 0;
}

/* One tournament node: the r rows idx[0..r) of X (in that order) factored;
 * out[0..n) = its first n pivot rows; the root also gives N and L_11. */
static int tslu_node(const double* X, int64_t ldx, int64_t n, const int64_t* rows, int64_t r, int root, int64_t* out,
                     double* N, double* L11, int32_t* info) {
  double* A = (double*)malloc(sizeof(double) * (size_t)(r * n));
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)r);
  for (int64_t i = 0; i < r; ++i) {
    idx[i] = rows[i];
    for (int64_t k = 0; k < n; ++k) A[i + k * r] = X[rows[i] + k * ldx];
  }
  int rc = tslu_factor(A, r, n, idx, root, info);
  if (!rc) {
    for (int64_t p = 0; p < n; ++p) out[p] = idx[p];
    if (root)
      for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
          N[i + j * n] = (i <= j) ? A[i + j * r] : 0.0;
          L11[i + j * n] = (i > j) ? A[i + j * r] : (i == j ? 1.0 : 0.0);
        }
  }
  free(A);
  free(idx);
  return rc;
}

void orc_trsm(const double* X, int64_t m, int64_t n, int64_t ldx, const double* R, double* W, int64_t ldw);

/* sel (n), N, L_11 (n x n) of the tournament; M (m x n, ld ldm, X's row order)
 * = X N^{-1} by row-wise substitution, rows sel[k] replaced by row k of L_11. */
int orc_tslu(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t* sel, double* N, double* L11, double* M,
             int64_t ldm, int32_t* info) {
  const int64_t L = (m + 255) / 256, F = 256 / n;
  int64_t nsets = L;
  int64_t* sets = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L * n));
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L * n));
  int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * 256);
  int rc = 0;
  for (int64_t g = 0; g < L && !rc; ++g) {
    const int64_t r0 = g * m / L, r1 = (g + 1) * m / L;
    for (int64_t i = r0; i < r1; ++i) rows[i - r0] = i;
    rc = tslu_node(X, ldx, n, rows, r1 - r0, L == 1, L == 1 ? sel : sets + g * n, N, L11, info);
  }
  while (!rc && nsets > 1) {
    const int64_t nodes = (nsets + F - 1) / F;
    for (int64_t g = 0; g < nodes && !rc; ++g) {
      const int64_t s0 = g * F, s1 = (s0 + F < nsets) ? s0 + F : nsets;
      rc = tslu_node(X, ldx, n, sets + s0 * n, (s1 - s0) * n, nodes == 1, nodes == 1 ? sel : next + g * n, N, L11,
                     info);
    }
    int64_t* t = sets;
    sets = next;
    next = t;
    nsets = nodes;
  }
  if (!rc && M) {
    orc_trsm(X, m, n, ldx, N, M, ldm);
    for (int64_t k = 0; k < n; ++k)
      for (int64_t j = 0; j < n; ++j) M[sel[k] + j * ldm] = L11[k + j * n];
  }
  free(sets);
  free(next);
  free(rows);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Thin Householder QR, R factor only (Algorithm 2 step 3): A (r x n, r>=n)  */
/* is overwritten by the reflectors; R (n x n, ld n) receives the upper      */
/* triangle. Reflector k: beta = -sign(alpha) ||(alpha, x)||,                */
/* tau = (beta - alpha)/beta, v = (1, x/(alpha - beta)) (LAPACK dlarfg).     */
/* ------------------------------------------------------------------------ */
void orc_house_r(double* A, int64_t r, int64_t n, int64_t lda, double* R) {
  for (int64_t k = 0; k < n; ++k) {
    double* ak = A + k * lda;
    double alpha = ak[k];
    double ss = 0.0;
    for (int64_t i = k + 1; i < r; ++i) ss += ak[i] * ak[i];
    double xnorm = sqrt(ss);
    double tau = 0.0;
    if (xnorm != 0.0) {
      double beta = -copysign(hypot(alpha, xnorm), alpha);
      tau = (beta - alpha) / beta;
      double scal = 1.0 / (alpha - beta);
      for (int64_t i = k + 1; i < r; ++i) ak[i] *= scal;
      ak[k] = beta;
    }
    if (tau != 0.0) {
      for (int64_t j = k + 1; j < n; ++j) {
        double* aj = A + j * lda;
        double w = aj[k];
        for (int64_t i = k + 1; i < r; ++i) w += ak[i] * aj[i];
        aj[k] -= tau * w;
        for (int64_t i = k + 1; i < r; ++i) aj[i] -= tau * w * ak[i];
      }
    }
  }
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) R[i + j * n] = (i <= j) ? A[i + j * lda] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Cholesky, upper factor: R^T R = G (+ shift I). Reads the upper triangle. */
/* Breakdown when a pivot is not > 0 (Algorithm 1 step 2).                  */
/* ------------------------------------------------------------------------ */
int orc_chol(const double* G, int64_t n, double shift, double* R, int32_t* info, int32_t stage) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i)
      if (!isfinite(G[i + j * n])) {
        set_info(info, ORC_NONFINITE, stage, j + 1);
        return (int)(j + 1);
      }
  for (int64_t e = 0; e < n * n; ++e) R[e] = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double d = G[j + j * n] + shift;
    for (int64_t k = 0; k < j; ++k) d -= R[k + j * n] * R[k + j * n];
    if (!(d > 0.0)) {
      set_info(info, ORC_CHOL_BREAKDOWN, stage, j + 1);
      return (int)(j + 1);
    }
    double rjj = sqrt(d);
    R[j + j * n] = rjj;
    for (int64_t l = j + 1; l < n; ++l) {
      double a = G[j + l * n];
      for (int64_t k = 0; k < j; ++k) a -= R[k + j * n] * R[k + l * n];
      R[j + l * n] = a / rjj;
    }
  }
  return 0;
}

/* W = X R^{-1}, R upper (n x n, ld n): for each row x, solve w R = x by     */
/* substitution w_j = (x_j - sum_{i<j} w_i R_ij) / R_jj. W may equal X.     */
void orc_trsm(const double* X, int64_t m, int64_t n, int64_t ldx, const double* R, double* W, int64_t ldw) {
#pragma omp parallel
  {
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
      for (int64_t j = 0; j < n; ++j) {
        double acc = X[r + j * ldx];
        for (int64_t i = 0; i < j; ++i) acc = ORC_MULADD(-w[i], R[i + j * n], acc);
        w[j] = acc / R[j + j * n];
      }
      for (int64_t j = 0; j < n; ++j) W[r + j * ldw] = w[j];
    }
    free(w);
  }
}

/* C = A B for upper-triangular A, B (n x n, ld n). C may not alias. */
void orc_trmm(const double* A, const double* B, int64_t n, double* C) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      if (i <= j)
        for (int64_t k = i; k <= j; ++k) acc += A[i + k * n] * B[k + j * n];
      C[i + j * n] = acc;
    }
}

/* R <- D R with D = sign(diag R); a zero diagonal entry is a failure.      */
static int sign_fix(double* R, int64_t n, int32_t* info, int32_t stage) {
  for (int64_t i = 0; i < n; ++i) {
    double d = R[i + i * n];
    if (!isfinite(d)) {
      set_info(info, ORC_NONFINITE, stage, i + 1);
      return 1;
    }
    if (d == 0.0) {
      set_info(info, ORC_SINGULAR, stage, i + 1);
      return 1;
    }
    if (d < 0.0)
      for (int64_t j = i; j < n; ++j) R[i + j * n] = -R[i + j * n];
  }
  return 0;
}

static int any_nonfinite(const double* A, int64_t r, int64_t n, int64_t lda, int64_t* col) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < r; ++i)
      if (!isfinite(A[i + j * lda])) {
        *col = j;
        return 1;
      }
  return 0;
}

/* One CholeskyQR step on Q in place (Algorithm 1): G = Q^T Q, Rc = chol(G), */
/* Q <- Q Rc^{-1}.                                                           */
static int cholqr_step(double* Q, int64_t m, int64_t n, int64_t ldq, double* Rc, int32_t* info, int32_t stage) {
  double* G = (double*)malloc(sizeof(double) * (size_t)(n * n));
  orc_gram(Q, m, n, ldq, G);
  int rc = orc_chol(G, n, 0.0, Rc, info, stage);
  free(G);
  if (rc) return rc;
  orc_trsm(Q, m, n, ldq, Rc, Q, ldq);
  return 0;
}

/* Optional intermediates returned to the tests: R1 (preconditioner), R2, R4
 * (Cholesky factors of the two Grams; R4 unused by one-step tails). */
typedef struct {
  double* R1;
  double* R2;
  double* R4;
} orc_aux;

static void copy_nn(double* dst, const double* src, int64_t n) {
  if (dst) memcpy(dst, src, sizeof(double) * (size_t)(n * n));
}

/* CholeskyQR2 tail (equations C1-C8): Q holds Q_1 = X R_1^{-1} on entry.
 * R = R_4 (R_2 R_1). */
static int cholqr2_tail(double* Q, int64_t m, int64_t n, int64_t ldq, const double* R1, double* R, int32_t* info,
                        orc_aux* aux) {
  size_t nn = (size_t)(n * n);
  double* R2 = (double*)calloc(nn, sizeof(double));
  double* R3 = (double*)calloc(nn, sizeof(double));
  double* R4 = (double*)calloc(nn, sizeof(double));
  int rc = cholqr_step(Q, m, n, ldq, R2, info, ORC_ST_CHOL_A);
  if (!rc) {
    orc_trmm(R2, R1, n, R3);
    rc = cholqr_step(Q, m, n, ldq, R4, info, ORC_ST_CHOL_B);
    if (!rc) orc_trmm(R4, R3, n, R);
  }
  if (aux) {
    copy_nn(aux->R2, R2, n);
    copy_nn(aux->R4, R4, n);
  }
  free(R2);
  free(R3);
  free(R4);
  return rc;
}

/* One-CholeskyQR tail (Algorithm 5 steps 6-7, Algorithm 6 steps 4-5). */
static int cholqr1_tail(double* Q, int64_t m, int64_t n, int64_t ldq, const double* R1, double* R, int32_t* info,
                        orc_aux* aux) {
  size_t nn = (size_t)(n * n);
  double* Z = (double*)calloc(nn, sizeof(double));
  int rc = cholqr_step(Q, m, n, ldq, Z, info, ORC_ST_CHOL_A);
  if (!rc) orc_trmm(Z, R1, n, R);
  if (aux) copy_nn(aux->R2, Z, n);
  free(Z);
  return rc;
}

static void copy_tall(const double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) memcpy(Q + j * ldq, X + j * ldx, sizeof(double) * (size_t)m);
}

/* Unit lower-trapezoidal M (r x n, ld r) from the packed LU in A. */
static void unpack_m(const double* A, int64_t r, int64_t n, int64_t lda, double* M) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < r; ++i) M[i + j * r] = (i > j) ? A[i + j * lda] : (i == j ? 1.0 : 0.0);
}
static void unpack_n(const double* A, int64_t n, int64_t lda, double* N) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) N[i + j * n] = (i <= j) ? A[i + j * lda] : 0.0;
}

/* R_1 = D R_0 N with the sign fix (Algorithm 2 step 4). */
static int make_r1(const double* R0, const double* N, int64_t n, double* R1, int32_t* info) {
  orc_trmm(R0, N, n, R1);
  return sign_fix(R1, n, info, ORC_ST_PRECOND);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: RCLUPP.                                                      */
/* ------------------------------------------------------------------------ */
int orc_rclupp_f(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Q, int64_t ldq,
                 double* R, int32_t* info, double* R1_out, double* R2_out, double* R4_out, int flags) {
  orc_aux aux = {R1_out, R2_out, R4_out};
  size_t nn = (size_t)(n * n);
  int rc = 0;
  if (info) memset(info, 0, 4 * sizeof(int32_t));
  double* Y = (double*)malloc(sizeof(double) * (size_t)(s * n));
  double* Mf = (double*)malloc(sizeof(double) * (size_t)(s * n));
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)s);
  double* N = (double*)calloc(nn, sizeof(double));
  double* R0 = (double*)calloc(nn, sizeof(double));
  double* R1 = (double*)calloc(nn, sizeof(double));
  method_sketch(flags, X, m, n, ldx, s, seed, Y);             /* X_s = S X          */
  rc = orc_gepp(Y, s, n, s, perm, info, ORC_ST_LU);           /* [M, N, P] = LU(X_s) */
  if (!rc) {
    unpack_m(Y, s, n, s, Mf);
    unpack_n(Y, n, s, N);
    int64_t col;
    if (any_nonfinite(Mf, s, n, s, &col)) {
      set_info(info, ORC_NONFINITE, ORC_ST_QR, col + 1);
      rc = 1;
    } else {
      orc_house_r(Mf, s, n, s, R0);                           /* [Q_s, R_0] = HQR(M) */
      rc = make_r1(R0, N, n, R1, info);                       /* R_1 = R_0 N         */
    }
  }
  if (!rc) {
    copy_nn(aux.R1, R1, n);
    orc_trsm(X, m, n, ldx, R1, Q, ldq);                       /* Q_1 = X R_1^{-1}    */
    rc = cholqr2_tail(Q, m, n, ldq, R1, R, info, &aux);       /* CholeskyQR2, R=Z R_1 */
  }
  free(Y); free(Mf); free(perm); free(N); free(R0); free(R1);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 7: RCLUPPr (LU of X first, then the sketch of its L factor).   */
/* The sketch's column index is the row position in the pivoted order.      */
/* ------------------------------------------------------------------------ */
int orc_rcluppr_f(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Q,
                  int64_t ldq, double* R, int32_t* info, double* R1_out, double* R2_out, double* R4_out, int flags) {
  orc_aux aux = {R1_out, R2_out, R4_out};
  size_t nn = (size_t)(n * n);
  int rc = 0;
  if (info) memset(info, 0, 4 * sizeof(int32_t));
  double* A = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n);
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
  double* N = (double*)calloc(nn, sizeof(double));
  double* Ms = (double*)malloc(sizeof(double) * (size_t)(s * n));
  double* R0 = (double*)calloc(nn, sizeof(double));
  double* R1 = (double*)calloc(nn, sizeof(double));
  if (flags & ORC_LU_TOURNAMENT) {
    /* [M, N, P] by tournament pivoting; M in X's row order */
    double* L11 = (double*)malloc(sizeof(double) * nn);
    rc = orc_tslu(X, m, n, ldx, perm, N, L11, A, m, info);
    free(L11);
  } else {
    copy_tall(X, m, n, ldx, A, m);
    rc = orc_gepp(A, m, n, m, perm, info, ORC_ST_LU);        /* [M, N, P] = LU(X)   */
    if (!rc) {
      unpack_n(A, n, m, N);
      /* M in place: unit diagonal, zeros above (the packed U part is not M). */
#pragma omp parallel for schedule(static)
      for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < j; ++i) A[i + j * m] = 0.0;
        A[j + j * m] = 1.0;
      }
    }
  }
  if (!rc) {
    method_sketch(flags, A, m, n, m, s, seed, Ms);            /* M_s = S M           */
    int64_t col;
    if (any_nonfinite(Ms, s, n, s, &col)) {
      set_info(info, ORC_NONFINITE, ORC_ST_QR, col + 1);
      rc = 1;
    } else {
      orc_house_r(Ms, s, n, s, R0);                           /* R_0 = HQR(M_s)      */
      rc = make_r1(R0, N, n, R1, info);                       /* R_1 = R_0 N         */
    }
  }
  free(A);
  free(perm);
  if (!rc) {
    copy_nn(aux.R1, R1, n);
    orc_trsm(X, m, n, ldx, R1, Q, ldq);                       /* Q_1 = X R_1^{-1}    */
    rc = cholqr2_tail(Q, m, n, ldq, R1, R, info, &aux);
  }
  free(N); free(Ms); free(R0); free(R1);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3: CholeskyQR2.                                                */
/* ------------------------------------------------------------------------ */
int orc_cholqr2(const double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* R, int32_t* info,
                double* R1_out, double* R2_out) {
  orc_aux aux = {R1_out, R2_out, NULL};
  size_t nn = (size_t)(n * n);
  if (info) memset(info, 0, 4 * sizeof(int32_t));
  double* G = (double*)malloc(sizeof(double) * nn);
  double* R1 = (double*)calloc(nn, sizeof(double));
  orc_gram(X, m, n, ldx, G);
  int rc = orc_chol(G, n, 0.0, R1, info, ORC_ST_PRECOND);     /* first CholeskyQR  */
  if (!rc) {
    copy_nn(aux.R1, R1, n);
    orc_trsm(X, m, n, ldx, R1, Q, ldq);
    rc = cholqr1_tail(Q, m, n, ldq, R1, R, info, &aux);       /* second CholeskyQR */
  }
  free(G);
  free(R1);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 4: Shifted CholeskyQR3 with s = 11(mnu + n(n+1)u) ||X||_g^2,    */
/* ||X||_g = max column 2-norm (Definition 2.1), u = 2^-53.                  */
/* ------------------------------------------------------------------------ */
double orc_scholqr3_shift(int64_t m, int64_t n, double g_max_diag) {
  const double u = 0x1p-53;
  return 11.0 * ((double)m * (double)n * u + (double)n * (double)(n + 1) * u) * g_max_diag;
}

int orc_scholqr3(const double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* R, int32_t* info,
                 double* R1_out, double* R2_out, double* R4_out) {
  orc_aux aux = {R1_out, R2_out, R4_out};
  size_t nn = (size_t)(n * n);
  if (info) memset(info, 0, 4 * sizeof(int32_t));
  double* G = (double*)malloc(sizeof(double) * nn);
  double* R1 = (double*)calloc(nn, sizeof(double));
  orc_gram(X, m, n, ldx, G);
  double gmax = 0.0;
  for (int64_t j = 0; j < n; ++j)
    if (G[j + j * n] > gmax) gmax = G[j + j * n];
  double sigma = orc_scholqr3_shift(m, n, gmax);
  int rc = orc_chol(G, n, sigma, R1, info, ORC_ST_PRECOND);   /* chol(G + sI)      */
  if (!rc) {
    copy_nn(aux.R1, R1, n);
    orc_trsm(X, m, n, ldx, R1, Q, ldq);
    rc = cholqr2_tail(Q, m, n, ldq, R1, R, info, &aux);
  }
  free(G);
  free(R1);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 5: LU-CholeskyQR2 (LC2). The Cholesky factor of M^T M is named  */
/* S_c here (the paper reuses the letter S).                                 */
/* ------------------------------------------------------------------------ */
int orc_lc2_f(const double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* R, int32_t* info,
              double* R1_out, double* R2_out, int flags) {
  orc_aux aux = {R1_out, R2_out, NULL};
  size_t nn = (size_t)(n * n);
  int rc = 0;
  if (info) memset(info, 0, 4 * sizeof(int32_t));
  double* A = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n);
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
  double* N = (double*)calloc(nn, sizeof(double));
  double* G = (double*)malloc(sizeof(double) * nn);
  double* Sc = (double*)calloc(nn, sizeof(double));
  double* R1 = (double*)calloc(nn, sizeof(double));
  if (flags & ORC_LU_TOURNAMENT) {
    double* L11 = (double*)malloc(sizeof(double) * nn);
    rc = orc_tslu(X, m, n, ldx, perm, N, L11, A, m, info);   /* M in X's row order  */
    free(L11);
  } else {
    copy_tall(X, m, n, ldx, A, m);
    rc = orc_gepp(A, m, n, m, perm, info, ORC_ST_LU);        /* [M, N, P] = LU(X)   */
    if (!rc) {
      unpack_n(A, n, m, N);
#pragma omp parallel for schedule(static)
      for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < j; ++i) A[i + j * m] = 0.0;
        A[j + j * m] = 1.0;
      }
    }
  }
  if (!rc) {
    orc_gram(A, m, n, m, G);                                  /* G = M^T M           */
    rc = orc_chol(G, n, 0.0, Sc, info, ORC_ST_QR);            /* S_c = chol(G)       */
    if (!rc) rc = make_r1(Sc, N, n, R1, info);                /* R_1 = S_c N         */
  }
  free(A);
  free(perm);
  if (!rc) {
    copy_nn(aux.R1, R1, n);
    orc_trsm(X, m, n, ldx, R1, Q, ldq);                       /* Q_1 = X R_1^{-1}    */
    rc = cholqr1_tail(Q, m, n, ldq, R1, R, info, &aux);       /* one CholeskyQR      */
  }
  free(N); free(G); free(Sc); free(R1);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 6: randomized CholeskyQR (single Gaussian sketch).             */
/* ------------------------------------------------------------------------ */
int orc_rcholqr_f(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Q,
                  int64_t ldq, double* R, int32_t* info, double* R1_out, double* R2_out, int flags) {
  orc_aux aux = {R1_out, R2_out, NULL};
  size_t nn = (size_t)(n * n);
  int rc = 0;
  if (info) memset(info, 0, 4 * sizeof(int32_t));
  double* K = (double*)malloc(sizeof(double) * (size_t)(s * n));
  double* R1 = (double*)calloc(nn, sizeof(double));
  method_sketch(flags, X, m, n, ldx, s, seed, K);             /* K = S X             */
  int64_t col;
  if (any_nonfinite(K, s, n, s, &col)) {
    set_info(info, ORC_NONFINITE, ORC_ST_QR, col + 1);
    rc = 1;
  } else {
    orc_house_r(K, s, n, s, R1);                              /* R_1 = HQR(K)        */
    rc = sign_fix(R1, n, info, ORC_ST_PRECOND);
  }
  if (!rc) {
    copy_nn(aux.R1, R1, n);
    orc_trsm(X, m, n, ldx, R1, Q, ldq);
    rc = cholqr1_tail(Q, m, n, ldq, R1, R, info, &aux);
  }
  free(K);
  free(R1);
  return rc;
}

/* The methods with the Gaussian sketch (flags = 0). */
int orc_rclupp(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Q, int64_t ldq,
               double* R, int32_t* info, double* R1_out, double* R2_out, double* R4_out) {
  return orc_rclupp_f(X, m, n, ldx, s, seed, Q, ldq, R, info, R1_out, R2_out, R4_out, 0);
}
int orc_rcluppr(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Q, int64_t ldq,
                double* R, int32_t* info, double* R1_out, double* R2_out, double* R4_out) {
  return orc_rcluppr_f(X, m, n, ldx, s, seed, Q, ldq, R, info, R1_out, R2_out, R4_out, 0);
}
int orc_rcholqr(const double* X, int64_t m, int64_t n, int64_t ldx, int64_t s, uint64_t seed, double* Q, int64_t ldq,
                double* R, int32_t* info, double* R1_out, double* R2_out) {
  return orc_rcholqr_f(X, m, n, ldx, s, seed, Q, ldq, R, info, R1_out, R2_out, 0);
}
int orc_lc2(const double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* R, int32_t* info,
            double* R1_out, double* R2_out) {
  return orc_lc2_f(X, m, n, ldx, Q, ldq, R, info, R1_out, R2_out, 0);
}
