/*
 * CPU oracle for the product-reduced Taylor matrix exponential
 * (Bader, Blanes, Casas, "An improved algorithm to compute the exponential of a matrix").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or helper
 * with the GPU library: every constant below is transcribed here from the paper, and
 * every routine is a plain loop nest written for readability, not speed.
 *
 * Build: gcc -O3 -fPIC -shared -ffp-contract=off -fopenmp (no FMA contraction and no
 * reassociation, so the rounding of each operation is the textbook one).
 *
 * Matrices are n x n, row-major, contiguous (a[i*n + j]).  Complex matrices are
 * interleaved (re, im) pairs.  "ld" routines compute in 80-bit x87 long double, "d"
 * routines in IEEE double.
 *
 * Contents and the passage each follows:
 *   or_norm1           1-norm  max_j sum_i |a_ij|                      (Sec. 1 / Sec. 4: norm of A)
 *   or_expm_taylor     e^A by the plain Taylor series T_n = sum A^k/k! (Sec. 3, eq. tay.exp)
 *                      with scaling and squaring (Sec. 1, eq. eses); own scaling ||X|| <= 1/2
 *   or_expm_taylor_z   the same for complex A
 *   or_expm_pade26     diagonal Pade r_26 (Sec. 1, eqs. eq.24 and eq.pade26) + squaring
 *   or_reduced_Tm      T_m(X) by the product-reduced sequences: T_8 (eq. Algorithm83eA),
 *                      T_12 (eq. poly12), T_18 (eq. poly.18); T_1, T_2, T_4 written as
 *                      I+X, I+X+X^2/2, I+X+X^2(I/2+X/6+X^2/24) (the paper says only that
 *                      they follow the Paterson-Stockmeyer pattern, Sec. 3)
 *   or_expm_reduced    T_m(A/2^s)^(2^s) for a given (m, s): the method's own output
 *   or_select_plain    (m, s) from ||A||_1 against theta_m (Sec. 1, eq. eq.theta; Table 2;
 *                      product counts Table 3)
 *   or_select_alpha    (m, s) from alpha_p = max(d_p, d_{p+1}), d_k = ||A^k||^(1/k), formed
 *                      explicitly (the refinement of the norm cited by the paper in Sec. 1)
 *   or_powers_norms    ||A^k||_1, k = 1..kmax, from explicit powers
 *   or_expm_apply      e^A v for a few vectors v by the series itself (Sec. 1) applied to
 *                      A / q, q times (and or_expm_apply_z for complex A)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;
typedef long double complex ldc;

/* ------------------------------------------------------------------------------------ */
/* Plain dense kernels in long double.                                                   */
/* ------------------------------------------------------------------------------------ */

static ld *ld_alloc(int64_t n) { return (ld *)calloc((size_t)(n * n), sizeof(ld)); }
static ldc *ldc_alloc(int64_t n) { return (ldc *)calloc((size_t)(n * n), sizeof(ldc)); }

/* C = A * B, the textbook triple loop (i, k, j order so the inner loop is contiguous). */
static void mm_ld(int64_t n, const ld *A, const ld *B, ld *C) {
  for (int64_t i = 0; i < n * n; ++i) C[i] = 0.0L;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < n; ++k) {
      ld a = A[i * n + k];
      if (a == 0.0L) continue;
      for (int64_t j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
    }
}

static void mm_d(int64_t n, const double *A, const double *B, double *C) {
  for (int64_t i = 0; i < n * n; ++i) C[i] = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < n; ++k) {
      double a = A[i * n + k];
      if (a == 0.0) continue;
      for (int64_t j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
    }
}

static void mm_ldc(int64_t n, const ldc *A, const ldc *B, ldc *C) {
  for (int64_t i = 0; i < n * n; ++i) C[i] = 0.0L;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < n; ++k) {
      ldc a = A[i * n + k];
      if (a == 0.0L) continue;
      for (int64_t j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
    }
}

static ld norm1_ld(int64_t n, const ld *A) {
  ld best = 0.0L;
  for (int64_t j = 0; j < n; ++j) {
    ld s = 0.0L;
    for (int64_t i = 0; i < n; ++i) s += fabsl(A[i * n + j]);
    if (s > best) best = s;
  }
  return best;
}

static ld norm1_ldc(int64_t n, const ldc *A) {
  ld best = 0.0L;
  for (int64_t j = 0; j < n; ++j) {
    ld s = 0.0L;
    for (int64_t i = 0; i < n; ++i) s += cabsl(A[i * n + j]);
    if (s > best) best = s;
  }
  return best;
}

static void set_identity_ld(int64_t n, ld *A) {
  for (int64_t i = 0; i < n * n; ++i) A[i] = 0.0L;
  for (int64_t i = 0; i < n; ++i) A[i * n + i] = 1.0L;
}

/* ------------------------------------------------------------------------------------ */
/* 1-norm.                                                                               */
/* ------------------------------------------------------------------------------------ */

double or_norm1(int64_t n, const double *A) {
  ld best = 0.0L;
  for (int64_t j = 0; j < n; ++j) {
    ld s = 0.0L;
    for (int64_t i = 0; i < n; ++i) s += fabsl((ld)A[i * n + j]);
    if (s > best) best = s;
  }
  return (double)best;
}

double or_norm1_z(int64_t n, const double *Az) {
  ld best = 0.0L;
  for (int64_t j = 0; j < n; ++j) {
    ld s = 0.0L;
    for (int64_t i = 0; i < n; ++i) {
      ld re = Az[2 * (i * n + j)], im = Az[2 * (i * n + j) + 1];
      s += hypotl(re, im);
    }
    if (s > best) best = s;
  }
  return (double)best;
}

/* Smallest s >= 0 with x * 2^-s <= bound (exact: scaling by a power of two is exact). */
static int scale_exponent(ld x, ld bound) {
  int s = 0;
  if (!(x > bound)) return 0;
  /* start near the answer, then correct by exact comparisons */
  s = (int)ceill(log2l(x / bound));
  if (s < 0) s = 0;
  while (s > 0 && x <= ldexpl(bound, s - 1)) --s;
  while (x > ldexpl(bound, s)) ++s;
  return s;
}

/* ------------------------------------------------------------------------------------ */
/* Direct Taylor summation with scaling and squaring.                                    */
/* ------------------------------------------------------------------------------------ */

/*
 * e^A: X = A / 2^s with s the smallest non-negative integer for which ||X||_1 <= 1/2
 * (deliberately not the method's own (m, s) rule), S = sum_k X^k / k! accumulated term by
 * term (P_0 = I, P_k = P_{k-1} X / k) until ||P_k||_1 <= 2^-64 ||S||_1 (or P_k = 0), then S
 * squared s times.  prec = 1: long double throughout; prec = 0: double throughout.
 * Returns the number of series terms used (>= 0), or -1 on a non-finite input.
 */
int or_expm_taylor(int64_t n, const double *A, double *E, int prec, int *s_out) {
  for (int64_t i = 0; i < n * n; ++i)
    if (!isfinite(A[i])) return -1;
  ld eta = (ld)or_norm1(n, A);
  int s = scale_exponent(eta, 0.5L);
  if (s_out) *s_out = s;
  int terms = 0;
  if (prec) {
    ld *X = ld_alloc(n), *P = ld_alloc(n), *Q = ld_alloc(n), *S = ld_alloc(n);
    for (int64_t i = 0; i < n * n; ++i) X[i] = ldexpl((ld)A[i], -s);
    set_identity_ld(n, P);
    set_identity_ld(n, S);
    for (int k = 1; k <= 60; ++k) {
      mm_ld(n, P, X, Q);
      for (int64_t i = 0; i < n * n; ++i) P[i] = Q[i] / (ld)k;
      for (int64_t i = 0; i < n * n; ++i) S[i] += P[i];
      terms = k;
      ld pn = norm1_ld(n, P);
      if (pn == 0.0L || pn <= ldexpl(norm1_ld(n, S), -64)) break;
    }
    for (int r = 0; r < s; ++r) {
      mm_ld(n, S, S, Q);
      memcpy(S, Q, sizeof(ld) * (size_t)(n * n));
    }
    for (int64_t i = 0; i < n * n; ++i) E[i] = (double)S[i];
    free(X); free(P); free(Q); free(S);
  } else {
    double *X = malloc(sizeof(double) * n * n), *P = malloc(sizeof(double) * n * n);
    double *Q = malloc(sizeof(double) * n * n), *S = malloc(sizeof(double) * n * n);
    for (int64_t i = 0; i < n * n; ++i) { X[i] = ldexp(A[i], -s); P[i] = 0.0; S[i] = 0.0; }
    for (int64_t i = 0; i < n; ++i) { P[i * n + i] = 1.0; S[i * n + i] = 1.0; }
    for (int k = 1; k <= 60; ++k) {
      mm_d(n, P, X, Q);
      for (int64_t i = 0; i < n * n; ++i) P[i] = Q[i] / (double)k;
      for (int64_t i = 0; i < n * n; ++i) S[i] += P[i];
      terms = k;
      double pn = or_norm1(n, P);
      if (pn == 0.0 || pn <= ldexp(or_norm1(n, S), -64)) break;
    }
    for (int r = 0; r < s; ++r) {
      mm_d(n, S, S, Q);
      memcpy(S, Q, sizeof(double) * (size_t)(n * n));
    }
    memcpy(E, S, sizeof(double) * (size_t)(n * n));
    free(X); free(P); free(Q); free(S);
  }
  return terms;
}

/* Complex A (interleaved re, im), long double complex throughout.  Same scheme as above. */
int or_expm_taylor_z(int64_t n, const double *Az, double *Ez, int *s_out) {
  for (int64_t i = 0; i < 2 * n * n; ++i)
    if (!isfinite(Az[i])) return -1;
  ld eta = (ld)or_norm1_z(n, Az);
  int s = scale_exponent(eta, 0.5L);
  if (s_out) *s_out = s;
  ldc *X = ldc_alloc(n), *P = ldc_alloc(n), *Q = ldc_alloc(n), *S = ldc_alloc(n);
  for (int64_t i = 0; i < n * n; ++i)
    X[i] = ldexpl((ld)Az[2 * i], -s) + I * ldexpl((ld)Az[2 * i + 1], -s);
  for (int64_t i = 0; i < n; ++i) { P[i * n + i] = 1.0L; S[i * n + i] = 1.0L; }
  int terms = 0;
  for (int k = 1; k <= 60; ++k) {
    mm_ldc(n, P, X, Q);
    for (int64_t i = 0; i < n * n; ++i) P[i] = Q[i] / (ld)k;
    for (int64_t i = 0; i < n * n; ++i) S[i] += P[i];
    terms = k;
    ld pn = norm1_ldc(n, P);
    if (pn == 0.0L || pn <= ldexpl(norm1_ldc(n, S), -64)) break;
  }
  for (int r = 0; r < s; ++r) {
    mm_ldc(n, S, S, Q);
    memcpy(S, Q, sizeof(ldc) * (size_t)(n * n));
  }
  for (int64_t i = 0; i < n * n; ++i) { Ez[2 * i] = (double)creall(S[i]); Ez[2 * i + 1] = (double)cimagl(S[i]); }
  free(X); free(P); free(Q); free(S);
  return terms;
}

/*
 * e^A applied to k vectors, from the series definition e^B w = sum_j B^j w / j! (Sec. 1) and
 * e^A = (e^(A/q))^q: with q = max(1, ceil(||A||_1 / 2)), the series of B = A / q is applied q
 * times (||B||_1 <= 2, so no term exceeds e^2 ||w||_1 and little cancels), each time
 * t_0 = w, t_j = B t_{j-1} / j, w <- sum of the t_j, in long double (real A: A row-major
 * n x n; complex A: interleaved).  A series stops at the first j with j >= 2 ||B||_1 and
 * ||t_j||_1 <= 2^-64 ||sum||_1: from there on each term is at most half the one before
 * (||B||_1 / (j + 1) < 1/2), so the neglected tail is at most ||t_j||_1.  V and out hold the k
 * vectors one after the other (k x n, each contiguous).  Returns the number of applications q,
 * or -1 when a series needs more than 1000 terms.  OpenMP over the vectors.  Meant for
 * sampled columns of e^A (v = e_j) at orders where forming e^A on the CPU is too slow.
 */
static int64_t apply_steps(ld eta) {
  const ld q = ceill(eta / 2.0L);
  return q < 1.0L ? 1 : (int64_t)q;
}

int or_expm_apply(int64_t n, const double *A, int64_t k, const double *V, double *out) {
  const ld eta = (ld)or_norm1(n, A);
  const int64_t q = apply_steps(eta);
  const ld beta = eta / (ld)q;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int64_t c = 0; c < k; ++c) {
    ld *w = malloc(sizeof(ld) * n), *t = malloc(sizeof(ld) * n), *u = malloc(sizeof(ld) * n);
    for (int64_t i = 0; i < n; ++i) w[i] = V[c * n + i];
    for (int64_t step = 0; step < q && !bad; ++step) {
      for (int64_t i = 0; i < n; ++i) t[i] = w[i];
      int j;
      for (j = 1; j <= 1000; ++j) {
        for (int64_t i = 0; i < n; ++i) {
          ld acc = 0.0L;
          for (int64_t p = 0; p < n; ++p) acc += (ld)A[i * n + p] * t[p];
          u[i] = acc / ((ld)q * (ld)j);
        }
        ld tn = 0.0L, sn = 0.0L;
        for (int64_t i = 0; i < n; ++i) { t[i] = u[i]; w[i] += t[i]; tn += fabsl(t[i]); sn += fabsl(w[i]); }
        if ((ld)j >= 2.0L * beta && tn <= ldexpl(sn, -64)) break;
      }
      if (j > 1000) bad += 1;
    }
    for (int64_t i = 0; i < n; ++i) out[c * n + i] = (double)w[i];
    free(w); free(t); free(u);
  }
  return bad ? -1 : (int)q;
}

int or_expm_apply_z(int64_t n, const double *Az, int64_t k, const double *Vz, double *outz) {
  const ld eta = (ld)or_norm1_z(n, Az);
  const int64_t q = apply_steps(eta);
  const ld beta = eta / (ld)q;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int64_t c = 0; c < k; ++c) {
    ldc *w = malloc(sizeof(ldc) * n), *t = malloc(sizeof(ldc) * n), *u = malloc(sizeof(ldc) * n);
    for (int64_t i = 0; i < n; ++i) w[i] = Vz[2 * (c * n + i)] + I * Vz[2 * (c * n + i) + 1];
    for (int64_t step = 0; step < q && !bad; ++step) {
      for (int64_t i = 0; i < n; ++i) t[i] = w[i];
      int j;
      for (j = 1; j <= 1000; ++j) {
        for (int64_t i = 0; i < n; ++i) {
          ldc acc = 0.0L;
          for (int64_t p = 0; p < n; ++p)
            acc += ((ld)Az[2 * (i * n + p)] + I * (ld)Az[2 * (i * n + p) + 1]) * t[p];
          u[i] = acc / ((ld)q * (ld)j);
        }
        ld tn = 0.0L, sn = 0.0L;
        for (int64_t i = 0; i < n; ++i) { t[i] = u[i]; w[i] += t[i]; tn += cabsl(t[i]); sn += cabsl(w[i]); }
        if ((ld)j >= 2.0L * beta && tn <= ldexpl(sn, -64)) break;
      }
      if (j > 1000) bad += 1;
    }
    for (int64_t i = 0; i < n; ++i) { outz[2 * (c * n + i)] = (double)creall(w[i]); outz[2 * (c * n + i) + 1] = (double)cimagl(w[i]); }
    free(w); free(t); free(u);
  }
  return bad ? -1 : (int)q;
}

/* Batched direct Taylor in double or long double, one OpenMP task per matrix. */
/* Threads of the batch routines (OpenMP over matrices): set, and the number a parallel region
 * then runs with. */
#include <omp.h>
void or_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }

int or_expm_taylor_batch(int64_t count, const int64_t *ns, const int64_t *offsets, const double *A,
                         double *E, int prec, int *s_out) {
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int64_t b = 0; b < count; ++b) {
    int s = 0;
    int t = or_expm_taylor(ns[b], A + offsets[b], E + offsets[b], prec, &s);
    if (s_out) s_out[b] = s;
    if (t < 0) bad += 1;
  }
  return bad;
}

/* ------------------------------------------------------------------------------------ */
/* Diagonal Pade r_26 (cross-check reference, as used for the paper's stability study). */
/* ------------------------------------------------------------------------------------ */

/* Solve M R = B for R by Gaussian elimination with partial pivoting (long double). */
static int lu_solve_ld(int64_t n, ld *M, ld *B) {
  int64_t *piv = malloc(sizeof(int64_t) * n);
  for (int64_t k = 0; k < n; ++k) {
    int64_t p = k;
    ld best = fabsl(M[k * n + k]);
    for (int64_t i = k + 1; i < n; ++i)
      if (fabsl(M[i * n + k]) > best) { best = fabsl(M[i * n + k]); p = i; }
    if (best == 0.0L) { free(piv); return -1; }
    piv[k] = p;
    if (p != k) {
      for (int64_t j = 0; j < n; ++j) {
        ld t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t;
        t = B[k * n + j]; B[k * n + j] = B[p * n + j]; B[p * n + j] = t;
      }
    }
    for (int64_t i = k + 1; i < n; ++i) {
      ld f = M[i * n + k] / M[k * n + k];
      if (f == 0.0L) continue;
      for (int64_t j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
      for (int64_t j = 0; j < n; ++j) B[i * n + j] -= f * B[k * n + j];
    }
  }
  /* back substitution, all right-hand sides */
  for (int64_t i = n - 1; i >= 0; --i) {
    for (int64_t j = 0; j < n; ++j) {
      ld v = B[i * n + j];
      for (int64_t k = i + 1; k < n; ++k) v -= M[i * n + k] * B[k * n + j];
      B[i * n + j] = v / M[i * n + i];
    }
  }
  free(piv);
  return 0;
}

/*
 * r_26(A/2^s)^(2^s) in long double.  Coefficients of p_13: b_j = (26-j)! 13! / (26! (13-j)! j!)
 * (eq. eq.24 with m = 13).  u_13 and v_13 are assembled as in eq. eq.pade26 from
 * A_2 = A^2, A_4 = A_2^2, A_6 = A_2 A_4; then (v_13 - u_13) R = u_13 + v_13.
 * s = smallest s >= 0 with ||A||_1 / 2^s <= theta26 (theta26 is passed in).
 * Returns 0, or -1 on a non-finite input or a singular denominator.
 */
int or_expm_pade26(int64_t n, const double *A, double *E, double theta26, int *s_out) {
  for (int64_t i = 0; i < n * n; ++i)
    if (!isfinite(A[i])) return -1;
  ld eta = (ld)or_norm1(n, A);
  int s = scale_exponent(eta, (ld)theta26);
  if (s_out) *s_out = s;
  ld b[14];
  for (int j = 0; j <= 13; ++j) {
    /* (26-j)! 13! / (26! (13-j)! j!) as a running product to stay in range */
    ld v = 1.0L;
    for (int t = 0; t < j; ++t) v *= (ld)(13 - t) / (ld)(26 - t); /* 13!/(13-j)! * (26-j)!/26! */
    for (int t = 2; t <= j; ++t) v /= (ld)t;                      /* / j! */
    b[j] = v;
  }
  ld *X = ld_alloc(n), *A2 = ld_alloc(n), *A4 = ld_alloc(n), *A6 = ld_alloc(n);
  ld *T1 = ld_alloc(n), *T2 = ld_alloc(n), *U = ld_alloc(n), *V = ld_alloc(n);
  for (int64_t i = 0; i < n * n; ++i) X[i] = ldexpl((ld)A[i], -s);
  mm_ld(n, X, X, A2);
  mm_ld(n, A2, A2, A4);
  mm_ld(n, A2, A4, A6);
  /* u_13 = X ( A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I ) */
  for (int64_t i = 0; i < n * n; ++i) T1[i] = b[13] * A6[i] + b[11] * A4[i] + b[9] * A2[i];
  mm_ld(n, A6, T1, T2);
  for (int64_t i = 0; i < n * n; ++i) T2[i] += b[7] * A6[i] + b[5] * A4[i] + b[3] * A2[i];
  for (int64_t i = 0; i < n; ++i) T2[i * n + i] += b[1];
  mm_ld(n, X, T2, U);
  /* v_13 = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I */
  for (int64_t i = 0; i < n * n; ++i) T1[i] = b[12] * A6[i] + b[10] * A4[i] + b[8] * A2[i];
  mm_ld(n, A6, T1, V);
  for (int64_t i = 0; i < n * n; ++i) V[i] += b[6] * A6[i] + b[4] * A4[i] + b[2] * A2[i];
  for (int64_t i = 0; i < n; ++i) V[i * n + i] += b[0];
  /* (-u + v) R = u + v */
  for (int64_t i = 0; i < n * n; ++i) { T1[i] = V[i] - U[i]; T2[i] = U[i] + V[i]; }
  int rc = lu_solve_ld(n, T1, T2);
  for (int r = 0; r < s && rc == 0; ++r) {
    mm_ld(n, T2, T2, T1);
    memcpy(T2, T1, sizeof(ld) * (size_t)(n * n));
  }
  for (int64_t i = 0; i < n * n; ++i) E[i] = (double)T2[i];
  free(X); free(A2); free(A4); free(A6); free(T1); free(T2); free(U); free(V);
  return rc;
}

/* r_2m(A / 2^s)^(2^s) for a given (m, s), r_2m = p_m(X) / p_m(-X) with p_m of eq. eq.24
 * summed term by term over plain powers X^j (not the grouped forms of eqs. eq.pade10 /
 * eq.pade26), one LU solve with partial pivoting, s squarings; long double.  Returns 0, or -1
 * for a singular denominator. */
int or_pade_ms(int64_t n, const double *A, int m, int s, double *E) {
  ld b[32];
  for (int j = 0; j <= m; ++j) {
    ld v = 1.0L;
    for (int t = 0; t < j; ++t) v *= (ld)(m - t) / (ld)(2 * m - t);
    for (int t = 2; t <= j; ++t) v /= (ld)t;
    b[j] = v;
  }
  ld *X = ld_alloc(n), *P = ld_alloc(n), *T = ld_alloc(n), *Pp = ld_alloc(n), *Q = ld_alloc(n);
  for (int64_t i = 0; i < n * n; ++i) X[i] = ldexpl((ld)A[i], -s);
  for (int64_t i = 0; i < n; ++i) P[i * n + i] = 1.0L; /* X^0 */
  for (int j = 0; j <= m; ++j) {
    if (j > 0) {
      mm_ld(n, P, X, T);
      memcpy(P, T, sizeof(ld) * (size_t)(n * n));
    }
    const ld sg = (j % 2) ? -1.0L : 1.0L;
    for (int64_t i = 0; i < n * n; ++i) {
      Pp[i] += b[j] * P[i];
      Q[i] += sg * b[j] * P[i];
    }
  }
  int rc = lu_solve_ld(n, Q, Pp); /* Pp <- Q^{-1} Pp */
  for (int r = 0; r < s && rc == 0; ++r) {
    mm_ld(n, Pp, Pp, T);
    memcpy(Pp, T, sizeof(ld) * (size_t)(n * n));
  }
  for (int64_t i = 0; i < n * n; ++i) E[i] = (double)Pp[i];
  free(X); free(P); free(T); free(Pp); free(Q);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* The product-reduced Taylor sequences (Sec. 3).                                        */
/* ------------------------------------------------------------------------------------ */

/* Coefficients of eq. poly12, in the order a_{0..3, j}, j = 1..4, as printed. */
static const ld T12_a[4][4] = {
    /* a_{i,1} */ {9.0198e-16L, 0.46932117595418237389L, -0.20099424927047284052L, -0.04623946134063071740L},
    /* a_{i,2} */ {5.31597895759871264183L, 1.19926790417132231573L, 0.01179296240992997031L, 0.01108844528519167989L},
    /* a_{i,3} */ {0.18188869982170434744L, 0.05502798439925399070L, 0.09351590770535414968L, 0.00610700528898058230L},
    /* a_{i,4} */ {-2.0861320e-13L, -0.13181061013830184015L, -0.02027855540589259079L, -0.00675951846863086359L},
};

/* Coefficients of eq. poly.18.  B_1 uses a_{i,1} (i = 0..3); B_{j+1} uses b_{i,j}, j = 1..4,
 * over the powers (I, A, A_2, A_3, A_6). */
static const ld T18_a1[4] = {0.0L, -0.100365581030144620L, -0.0080292464824115696L, -0.0008921384980457299L};
static const ld T18_b[4][5] = {
    /* b_{0,1}, b_{1,1}, b_{2,1}, b_{3,1}, b_{6,1} */
    {0.0L, 0.39784974949964507614L, 1.36783778460411719922L, 0.49828962252538267755L, -0.0006378981945947233L},
    /* b_{.,2} */
    {-10.967639605296206259L, 1.68015813878906197182L, 0.05717798464788655127L, -0.0069821012248805208L, 0.00003349750170860705L},
    /* b_{.,3} */
    {-0.0904316832390810561L, -0.0676404519071381907L, 0.06759613017704596460L, 0.02955525704293155274L, -0.0000139180257516060L},
    /* b_{.,4} */
    {0.0L, 0.0L, -0.0923364619367118592L, -0.0169364939002081717L, -0.0000140086798182036L},
};

/* lincomb: D = c0 I + c1 P1 + c2 P2 + c3 P3 + c4 P4 (any P may be NULL with c = 0). */
static void lincomb_ld(int64_t n, ld *D, ld c0, ld c1, const ld *P1, ld c2, const ld *P2, ld c3,
                       const ld *P3, ld c4, const ld *P4) {
  for (int64_t i = 0; i < n * n; ++i) {
    ld v = 0.0L;
    if (P1) v += c1 * P1[i];
    if (P2) v += c2 * P2[i];
    if (P3) v += c3 * P3[i];
    if (P4) v += c4 * P4[i];
    D[i] = v;
  }
  for (int64_t i = 0; i < n; ++i) D[i * n + i] += c0;
}

/* T_m(X) in long double, m in {1, 2, 4, 8, 12, 18}.  Returns the number of matrix products
 * used, or -1 for an unsupported m. */
static int reduced_Tm_ld(int64_t n, const ld *X, int m, ld *T) {
  ld *X2 = ld_alloc(n), *W1 = ld_alloc(n), *W2 = ld_alloc(n), *W3 = ld_alloc(n);
  int products = -1;
  if (m == 1) {
    lincomb_ld(n, T, 1.0L, 1.0L, X, 0, NULL, 0, NULL, 0, NULL);
    products = 0;
  } else if (m == 2) {
    mm_ld(n, X, X, X2);
    lincomb_ld(n, T, 1.0L, 1.0L, X, 0.5L, X2, 0, NULL, 0, NULL);
    products = 1;
  } else if (m == 4) {
    mm_ld(n, X, X, X2);
    lincomb_ld(n, W1, 0.5L, 1.0L / 6.0L, X, 1.0L / 24.0L, X2, 0, NULL, 0, NULL);
    mm_ld(n, X2, W1, W2);
    lincomb_ld(n, T, 1.0L, 1.0L, X, 1.0L, W2, 0, NULL, 0, NULL);
    products = 2;
  } else if (m == 8) {
    /* eq. Algorithm83eA with x3 = 2/3 */
    const ld r = sqrtl(177.0L), x3 = 2.0L / 3.0L;
    const ld x1 = x3 * (1.0L + r) / 88.0L, x2 = (1.0L + r) / 352.0L * x3;
    const ld x4 = (-271.0L + 29.0L * r) / (315.0L * x3), x5 = 11.0L * (-1.0L + r) / (1260.0L * x3);
    const ld x6 = 11.0L * (-9.0L + r) / (5040.0L * x3), x7 = (89.0L - r) / (5040.0L * x3 * x3);
    const ld y0 = 1.0L, y1 = 1.0L, y2 = (857.0L - 58.0L * r) / 630.0L;
    mm_ld(n, X, X, X2);                                                  /* A_2 */
    lincomb_ld(n, W1, 0.0L, x1, X, x2, X2, 0, NULL, 0, NULL);             /* x1 A + x2 A_2 */
    mm_ld(n, X2, W1, W2);                                                /* A_4 */
    lincomb_ld(n, W1, 0.0L, x3, X2, 1.0L, W2, 0, NULL, 0, NULL);          /* x3 A_2 + A_4 */
    lincomb_ld(n, W3, x4, x5, X, x6, X2, x7, W2, 0, NULL);                /* x4 I + x5 A + x6 A_2 + x7 A_4 */
    mm_ld(n, W1, W3, W2);                                                /* A_8 */
    lincomb_ld(n, T, y0, y1, X, y2, X2, 1.0L, W2, 0, NULL);               /* T_8 */
    products = 3;
  } else if (m == 12) {
    ld *X3 = ld_alloc(n), *B1 = ld_alloc(n), *B2 = ld_alloc(n), *B3 = ld_alloc(n), *B4 = ld_alloc(n);
    mm_ld(n, X, X, X2);
    mm_ld(n, X2, X, X3);
    const ld(*a)[4] = T12_a;
    lincomb_ld(n, B1, a[0][0], a[0][1], X, a[0][2], X2, a[0][3], X3, 0, NULL);
    lincomb_ld(n, B2, a[1][0], a[1][1], X, a[1][2], X2, a[1][3], X3, 0, NULL);
    lincomb_ld(n, B3, a[2][0], a[2][1], X, a[2][2], X2, a[2][3], X3, 0, NULL);
    lincomb_ld(n, B4, a[3][0], a[3][1], X, a[3][2], X2, a[3][3], X3, 0, NULL);
    mm_ld(n, B4, B4, W1);                                    /* B_4^2 */
    for (int64_t i = 0; i < n * n; ++i) W1[i] += B3[i];      /* A_6 = B_3 + B_4^2 */
    for (int64_t i = 0; i < n * n; ++i) W2[i] = B2[i] + W1[i];
    mm_ld(n, W2, W1, W3);                                    /* (B_2 + A_6) A_6 */
    for (int64_t i = 0; i < n * n; ++i) T[i] = B1[i] + W3[i];
    products = 4;
    free(X3); free(B1); free(B2); free(B3); free(B4);
  } else if (m == 18) {
    ld *X3 = ld_alloc(n), *X6 = ld_alloc(n), *B[6];
    for (int j = 1; j <= 5; ++j) B[j] = ld_alloc(n);
    mm_ld(n, X, X, X2);
    mm_ld(n, X2, X, X3);
    mm_ld(n, X3, X3, X6);
    lincomb_ld(n, B[1], T18_a1[0], T18_a1[1], X, T18_a1[2], X2, T18_a1[3], X3, 0, NULL);
    for (int j = 1; j <= 4; ++j) {
      const ld *c = T18_b[j - 1];
      lincomb_ld(n, B[j + 1], c[0], c[1], X, c[2], X2, c[3], X3, c[4], X6);
    }
    mm_ld(n, B[1], B[5], W1);                                /* B_1 B_5 */
    for (int64_t i = 0; i < n * n; ++i) W1[i] += B[4][i];    /* A_9 */
    for (int64_t i = 0; i < n * n; ++i) W2[i] = B[3][i] + W1[i];
    mm_ld(n, W2, W1, W3);                                    /* (B_3 + A_9) A_9 */
    for (int64_t i = 0; i < n * n; ++i) T[i] = B[2][i] + W3[i];
    products = 5;
    free(X3); free(X6);
    for (int j = 1; j <= 5; ++j) free(B[j]);
  }
  free(X2); free(W1); free(W2); free(W3);
  return products;
}

/* T_m(X) for a double X, evaluated in long double, rounded to double.  Returns the number of
 * matrix products, or -1 for an unsupported m. */
int or_reduced_Tm(int64_t n, const double *X, int m, double *T) {
  ld *Xl = ld_alloc(n), *Tl = ld_alloc(n);
  for (int64_t i = 0; i < n * n; ++i) Xl[i] = X[i];
  int p = reduced_Tm_ld(n, Xl, m, Tl);
  for (int64_t i = 0; i < n * n; ++i) T[i] = (double)Tl[i];
  free(Xl); free(Tl);
  return p;
}

/* T_m(A / 2^s)^(2^s) in long double: the method's own result for a given (m, s), free of
 * the GPU's rounding.  Returns the total number of products (polynomial + squarings). */
int or_expm_reduced(int64_t n, const double *A, int m, int s, double *E) {
  ld *X = ld_alloc(n), *T = ld_alloc(n), *Q = ld_alloc(n);
  for (int64_t i = 0; i < n * n; ++i) X[i] = ldexpl((ld)A[i], -s);
  int p = reduced_Tm_ld(n, X, m, T);
  for (int r = 0; r < s && p >= 0; ++r) {
    mm_ld(n, T, T, Q);
    memcpy(T, Q, sizeof(ld) * (size_t)(n * n));
  }
  for (int64_t i = 0; i < n * n; ++i) E[i] = (double)T[i];
  free(X); free(T); free(Q);
  return p < 0 ? -1 : p + s;
}

/* ------------------------------------------------------------------------------------ */
/* (m, s) selection.                                                                     */
/* ------------------------------------------------------------------------------------ */

static const int SEL_M[6] = {1, 2, 4, 8, 12, 18};
static const int SEL_PI[6] = {0, 1, 2, 3, 4, 5}; /* products per degree, Table 3 */

/*
 * Plain rule: for each degree m with threshold theta[i] (theta[0..5] for m = 1, 2, 4, 8, 12,
 * 18), the scaling s_m is the smallest s >= 0 with eta_m / 2^s <= theta_m (inclusive bound,
 * eq. eq.theta); the cost is products(m) + s_m; the cheapest wins, and a tie goes to the
 * smaller s (fewer squarings).  eta[i] is the norm quantity used for degree i (the same
 * ||A||_1 for every degree in the plain rule).
 */
static void select_from_eta(const ld *eta, const double *theta, int *m_out, int *s_out) {
  int best_i = -1, best_cost = 0, best_s = 0;
  for (int i = 0; i < 6; ++i) {
    int s = scale_exponent(eta[i], (ld)theta[i]);
    int cost = SEL_PI[i] + s;
    if (best_i < 0 || cost < best_cost || (cost == best_cost && s < best_s)) {
      best_i = i; best_cost = cost; best_s = s;
    }
  }
  *m_out = SEL_M[best_i];
  *s_out = best_s;
}

void or_select_plain(double eta, const double *theta, int *m_out, int *s_out) {
  ld e[6];
  for (int i = 0; i < 6; ++i) e[i] = eta;
  select_from_eta(e, theta, m_out, s_out);
}

/* ||A^k||_1 for k = 1..kmax from explicit powers in long double; out[k-1]. */
void or_powers_norms(int64_t n, const double *A, int kmax, double *out) {
  ld *P = ld_alloc(n), *Q = ld_alloc(n), *X = ld_alloc(n);
  for (int64_t i = 0; i < n * n; ++i) { X[i] = A[i]; P[i] = A[i]; }
  for (int k = 1; k <= kmax; ++k) {
    out[k - 1] = (double)norm1_ld(n, P);
    if (k < kmax) {
      mm_ld(n, P, X, Q);
      memcpy(P, Q, sizeof(ld) * (size_t)(n * n));
    }
  }
  free(P); free(Q); free(X);
}

/*
 * Selection from alpha_p = max(d_p, d_{p+1}), d_k = ||A^k||_1^(1/k), with p restricted to
 * p (p - 1) <= m + 1 for degree m (the series of the backward error of T_m starts at power
 * m + 1).  For each degree the norm quantity is min over admissible p of alpha_p; the rest is
 * the plain rule.  dk[0..4] = d_1..d_5 are supplied by the caller (exact values from
 * or_powers_norms, or upper bounds).
 */
void or_select_alpha(const double *dk, const double *theta, int *m_out, int *s_out) {
  ld e[6];
  for (int i = 0; i < 6; ++i) {
    int m = SEL_M[i];
    ld best = -1.0L;
    for (int p = 1; p <= 4; ++p) {
      if (p * (p - 1) > m + 1) break;
      ld a = dk[p - 1] > dk[p] ? dk[p - 1] : dk[p];
      if (best < 0 || a < best) best = a;
    }
    e[i] = best;
  }
  select_from_eta(e, theta, m_out, s_out);
}

/*
 * Label rule of the learned selector: degrees m >= 12 judge the alpha bound with dk_hi
 * (exact d_3, because those degrees form A^3), degrees m <= 8 with dk_lo (d_3 only through
 * its bound).  Otherwise as or_select_alpha.
 */
void or_select_alpha_split(const double *dk_lo, const double *dk_hi, const double *theta, int *m_out,
                           int *s_out) {
  ld e[6];
  for (int i = 0; i < 6; ++i) {
    const int m = SEL_M[i];
    const double *dk = m >= 12 ? dk_hi : dk_lo;
    ld best = -1.0L;
    for (int p = 1; p <= 4; ++p) {
      if (p * (p - 1) > m + 1) break;
      ld a = dk[p - 1] > dk[p] ? dk[p - 1] : dk[p];
      if (best < 0 || a < best) best = a;
    }
    e[i] = best;
  }
  select_from_eta(e, theta, m_out, s_out);
}
