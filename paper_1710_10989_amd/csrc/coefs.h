// Per-degree coefficient layout read by the GEMM epilogues and elementwise passes.
#pragma once
#include <math.h>

#include "expm_internal.h"

namespace expm {

// Scaled coefficients for degree m and scaling s: a coefficient of X^k becomes
// coef * 2^(-s k) on the stored power A^k.  Layout per degree as the epilogues read it.
__host__ __device__ inline void make_coefs(const Consts &k, int m, int s, double *c) {
  const double h1 = ldexp(1.0, -s), h2 = ldexp(1.0, -2 * s), h3 = ldexp(1.0, -3 * s),
               h6 = ldexp(1.0, -6 * s);
  switch (m) {
    case 1: c[0] = h1; break;
    case 2: c[0] = h1; c[1] = 0.5 * h2; break;
    case 4:
      c[0] = h1; c[1] = h2;                            // T = I + h1 A + h2 (A^2 W)
      c[2] = 0.5; c[3] = h1 / 6.0; c[4] = h2 / 24.0;   // W = I/2 + X/6 + X^2/24
      break;
    case 8:
      c[0] = k.t8[0] * h1; c[1] = k.t8[1] * h2;       // W1 = x1 X + x2 X^2
      c[2] = h2;                                        // A_4 = h2 (A^2 W1)
      c[3] = k.t8[2] * h2;                              // L = x3 X^2 + A_4
      c[4] = k.t8[3]; c[5] = k.t8[4] * h1; c[6] = k.t8[5] * h2; c[7] = k.t8[6];  // R
      c[8] = k.t8[7]; c[9] = k.t8[8] * h1; c[10] = k.t8[9] * h2;  // y0 I + y1 X + y2 X^2
      break;
    case 12:
      for (int j = 0; j < 4; ++j) {
        c[4 * j + 0] = k.t12[j][0];
        c[4 * j + 1] = k.t12[j][1] * h1;
        c[4 * j + 2] = k.t12[j][2] * h2;
        c[4 * j + 3] = k.t12[j][3] * h3;
      }
      break;
    case 18:
      c[0] = k.t18a[0]; c[1] = k.t18a[1] * h1; c[2] = k.t18a[2] * h2; c[3] = k.t18a[3] * h3;
      for (int j = 0; j < 4; ++j) {
        c[4 + 5 * j + 0] = k.t18b[j][0];
        c[4 + 5 * j + 1] = k.t18b[j][1] * h1;
        c[4 + 5 * j + 2] = k.t18b[j][2] * h2;
        c[4 + 5 * j + 3] = k.t18b[j][3] * h3;
        c[4 + 5 * j + 4] = k.t18b[j][4] * h6;
      }
      break;
  }
}

// Coefficients of the Paterson-Stockmeyer evaluation of degree m in {6, 9, 12, 16} (eq. poli9)
// at X = A / 2^s, a_k = 2^(-s k) / k!, in blocks of four per Horner step: block j holds the
// coefficients of I, A, A^2, A^3 in F_j = sum_i a_(q j + i) A^i (q the base; with q = 3 the
// fourth slot is 0, except in the innermost block, where it carries a_m of the term a_m A^3);
// with q = 4, c[16] = a_16 multiplies A^4 in the innermost block.  Then
// T = F_0 + (F_1 + (... + F_(r-1) ...) A^q) A^q, r = m / q.
__host__ __device__ inline void make_ps_coefs(int m, int s, double *c) {
  // 1/k! for k <= 16: every k! there is an exact double, so each quotient is correctly rounded
  constexpr double kInvFact[17] = {1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0,
                                   1.0 / 5040.0, 1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0,
                                   1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0,
                                   1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0};
  const int q = ps_base(m), r = m / q;
  for (int i = 0; i < 17; ++i) c[i] = 0.0;
  for (int j = 0; j < r; ++j)
    for (int i = 0; i < q; ++i) c[4 * j + i] = ldexp(kInvFact[q * j + i], -s * (q * j + i));
  if (q == 3) c[4 * (r - 1) + 3] = ldexp(kInvFact[m], -s * m);
  else c[16] = ldexp(kInvFact[16], -s * 16);
}

}  // namespace expm
