// Internal declarations of the gfx950 matrix-exponential library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/expm.h"

namespace expm {

// Degrees of the product-reduced Taylor family and their product counts (Table 3; T_1, T_2,
// T_4 take 0, 1, 2 products).
constexpr int kNumDeg = 6;
constexpr int kDeg[kNumDeg] = {1, 2, 4, 8, 12, 18};
constexpr int kProducts[kNumDeg] = {0, 1, 2, 3, 4, 5};

// Comparison method of Sec. 4: the plain Taylor polynomial evaluated by the Paterson-Stockmeyer
// rule in Horner form (eq. poli9), with the degrees k products reach (Table 3).  Degrees 6, 9
// and 12 use the base A^3, degree 16 the base A^4; degrees 1, 2 and 4 coincide with T_1, T_2,
// T_4 above.
constexpr int kNumPs = 7;
constexpr int kPsDeg[kNumPs] = {1, 2, 4, 6, 9, 12, 16};
constexpr int kPsProducts[kNumPs] = {0, 1, 2, 3, 4, 5, 6};
__host__ __device__ inline int ps_base(int m) { return m == 16 ? 4 : 3; }

// Comparison method of Sec. 2: diagonal Pade r_10 and r_26 (eqs. eq.pade10, eq.pade26) with
// 3 and 6 products plus one solve, costed as 4/3 of a product (so costs are kept in thirds).
constexpr int kNumPade = 2;
constexpr int kPadeDeg[kNumPade] = {10, 26};
constexpr int kPadeCost3[kNumPade] = {3 * 3 + 4, 3 * 6 + 4};

// Coefficients and thresholds handed to the kernels by value.
struct Consts {
  double theta[kNumDeg];  // theta_m(u) for m = 1, 2, 4, 8, 12, 18
  // T_8, eq. Algorithm83eA (x3 = 2/3): x1..x7 in t8[0..6], y0, y1, y2 in t8[7..9].
  double t8[10];
  // T_12, eq. poly12: t12[j][i] = a_{i, j+1}, i = power 0..3 (I, A, A^2, A^3), j = B index - 1.
  double t12[4][4];
  // T_18, eq. poly.18: B_1 = sum_i t18a[i] A^i (i = 0..3); B_{j+2} = t18b[j] over
  // (I, A, A^2, A^3, A^6), i.e. t18b[j][*] = b_{*, j+1}.
  double t18a[4];
  double t18b[4][5];
  double theta_ps[kNumPs];  // theta_m(u) for the Paterson-Stockmeyer degrees (Table 2)
  // Pade r_10, r_26: b_j of p_m (eq. eq.24, m = 5 and 13) and theta_10, theta_26 (Table 1;
  // zero when u is not one of the two printed rows: the method is then unavailable)
  double pade5[6];
  double pade13[14];
  double theta_pade[kNumPade];
};

// Builds Consts for accuracy u (host; thresholds cached per u).  Returns false for u outside
// the supported range.
bool make_consts(double u, Consts *out);
// theta_m(u), host.
bool theta_of(int m, double u, double *out);

// Smallest s >= 0 with eta / 2^s <= theta (exact: scaling by 2^s is exact).  For eta > theta
// (both positive, finite, normal) write eta = me 2^ee and theta = mt 2^et with me, mt in
// [1/2, 1): eta <= theta 2^s iff me / mt <= 2^(et + s - ee), and me / mt lies in (1/2, 2), so
// s = ee - et when me <= mt and ee - et + 1 otherwise.  Both are read off the bit patterns.
__host__ __device__ inline int scale_exp(double eta, double theta) {
  if (!(eta > theta)) return 0;
  const unsigned long long be = __builtin_bit_cast(unsigned long long, eta);
  const unsigned long long bt = __builtin_bit_cast(unsigned long long, theta);
  const unsigned long long kFrac = (1ull << 52) - 1;
  const int ee = (int)((be >> 52) & 0x7ff), et = (int)((bt >> 52) & 0x7ff);
  return ee - et + ((be & kFrac) > (bt & kFrac) ? 1 : 0);
}

// The kernels scale A by 2^-sp (sp: the plain rule's s) when it is loaded, before any power
// is formed, so every matrix they hold stays in range whatever ||A|| is.  The norm of a power
// of the scaled matrix is that of A^k times 2^-k sp: unscale_norm gives ||A^k|| back (exactly;
// +inf when it overflows, which the ALPHA rule then treats as no better than ||A||).  nk < 0
// (power not formed) passes through.
__host__ __device__ inline double unscale_norm(double nk, int k, int sp) { return nk < 0 ? nk : ldexp(nk, k * sp); }

// Norm quantities for the ALPHA rule from ||A||, ||A^2||, ||A^3|| (n2, n3 < 0: not formed,
// replaced by submultiplicative bounds).  d[k-1] >= ||A^k||^(1/k), k = 1..5.
__host__ __device__ inline void alpha_d(double n1, double n2, double n3, double d[5]) {
  if (n2 < 0) n2 = n1 * n1;
  if (n3 < 0) n3 = fmin(n1 * n2, n1 * n1 * n1);
  double n4 = fmin(n2 * n2, n3 * n1);
  double n5 = fmin(n2 * n3, n4 * n1);
  d[0] = n1;
  d[1] = sqrt(n2);
  d[2] = cbrt(n3);
  d[3] = sqrt(sqrt(n4));
  d[4] = pow(n5, 0.2);
}

// Norm quantity for degree index i: ||A||_1 (PLAIN) or the smallest admissible
// alpha_p = max(d_p, d_{p+1}) with p (p - 1) <= m + 1 (ALPHA), d from alpha_d.
__host__ __device__ inline double eta_for_degree(int i, int alpha, double n1, const double d[5]) {
  if (!alpha) return n1;
  const int m = kDeg[i];
  double eta = n1;  // p = 1: alpha_1 = max(d_1, d_2) = d_1
  for (int p = 2; p <= 4; ++p) {
    if (p * (p - 1) > m + 1) break;
    const double a = fmax(d[p - 1], d[p]);
    if (a < eta) eta = a;
  }
  return eta;
}

__host__ __device__ inline int degree_index(int m) {
  for (int i = 0; i < kNumDeg; ++i)
    if (kDeg[i] == m) return i;
  return -1;
}

// (m, s) selection: for each degree, s_m = scale_exp(eta_m, theta_m) with eta_m from
// eta_for_degree; cost = products + s_m; cheapest wins, ties go to the smaller s.
__host__ __device__ inline void select_ms(const double *theta, int alpha, double n1, double n2,
                                          double n3, int *m_out, int *s_out) {
  double d[5];
  if (alpha) alpha_d(n1, n2, n3, d);
  int best = -1, best_cost = 0, best_s = 0;
  for (int i = 0; i < kNumDeg; ++i) {
    const int s = scale_exp(eta_for_degree(i, alpha, n1, d), theta[i]);
    const int cost = kProducts[i] + s;
    if (best < 0 || cost < best_cost || (cost == best_cost && s < best_s)) {
      best = i; best_cost = cost; best_s = s;
    }
  }
  *m_out = kDeg[best];
  *s_out = best_s;
}

// (m, s) of the Paterson-Stockmeyer comparison method: the same rule over the degrees and
// product counts of kPsDeg / kPsProducts, from eta = ||A||_1.
__host__ __device__ inline void select_ps(const double *theta_ps, double eta, int *m_out, int *s_out) {
  int best = -1, best_cost = 0, best_s = 0;
  for (int i = 0; i < kNumPs; ++i) {
    const int s = scale_exp(eta, theta_ps[i]);
    const int cost = kPsProducts[i] + s;
    if (best < 0 || cost < best_cost || (cost == best_cost && s < best_s)) {
      best = i; best_cost = cost; best_s = s;
    }
  }
  *m_out = kPsDeg[best];
  *s_out = best_s;
}

// (2m, s) of the Pade comparison method: the smallest s with eta <= theta_2m 2^s for 2m = 10,
// 26; the cheaper of the two (products + 4/3 + s), ties to the smaller s.
__host__ __device__ inline void select_pade(const double *theta_pade, double eta, int *m_out, int *s_out) {
  int best = -1, best_cost = 0, best_s = 0;
  for (int i = 0; i < kNumPade; ++i) {
    const int s = scale_exp(eta, theta_pade[i]);
    const int cost = kPadeCost3[i] + 3 * s;
    if (best < 0 || cost < best_cost || (cost == best_cost && s < best_s)) {
      best = i; best_cost = cost; best_s = s;
    }
  }
  *m_out = kPadeDeg[best];
  *s_out = best_s;
}

// Training label of the learned selector: the cheapest (m, s) that passes the alpha bound
// with the information the selector has when it decides: ||A||, ||A^2|| always; ||A^3|| only
// for m >= 12 (those degrees form A^3 anyway); smaller degrees use its submultiplicative
// bound.  Ties go to the smaller s.
__host__ __device__ inline void learned_label(const double *theta, double n1, double n2, double n3,
                                              int *m_out, int *s_out) {
  double dlo[5], dhi[5];
  alpha_d(n1, n2, -1.0, dlo);
  alpha_d(n1, n2, n3, dhi);
  int best = -1, best_cost = 0, best_s = 0;
  for (int i = 0; i < kNumDeg; ++i) {
    const double *d = kDeg[i] >= 12 ? dhi : dlo;
    const int s = scale_exp(eta_for_degree(i, 1, n1, d), theta[i]);
    const int cost = kProducts[i] + s;
    if (best < 0 || cost < best_cost || (cost == best_cost && s < best_s)) {
      best = i; best_cost = cost; best_s = s;
    }
  }
  *m_out = kDeg[best];
  *s_out = best_s;
}

// Acceptance test of a proposed (m, s): the alpha bound with ||A^3|| when given (n3 >= 0),
// else its bound.  True iff the backward error of T_m at X = A / 2^s stays below u.
__host__ __device__ inline bool proposal_ok(const double *theta, double n1, double n2, double n3, int m, int s) {
  const int i = degree_index(m);
  if (i < 0 || s < 0) return false;
  double d[5];
  alpha_d(n1, n2, n3, d);
  return scale_exp(eta_for_degree(i, 1, n1, d), theta[i]) <= s;
}

}  // namespace expm
