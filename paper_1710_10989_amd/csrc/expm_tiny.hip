// One wavefront per matrix of real order <= 16: the batched exponential of small matrices and
// the fourth-order Magnus step built on it (exponential integrators, concluding remarks).
//
// At np = 16 the resident workgroup kernels keep three of their four waves idle.  Here every
// wave takes its own matrix.  A 16 x 16 matrix in the D layout of the 16x16x4 FP64 MFMA is one
// register quad per lane (lane l, register r: row 4 r + l / 16, column l % 16); that layout is
// also the B-operand layout of the same MFMA for k rows 4 r .. 4 r + 3, so the right operand
// of a product is fed from the lane's own registers.  The left operand goes through a 16 x 17
// LDS tile private to the wave (odd stride: the 16 rows of a fragment read fall in distinct
// banks).  No workgroup barrier is needed: one wave's LDS operations complete in issue order,
// and a wavefront-scope fence keeps the compiler from reordering them.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "coefs.h"
#include "expm_fused.h"
#include "expm_internal.h"
#include "tile_gemm.h"

namespace expm {
namespace {

constexpr int kTinyW = 4;          // waves per workgroup
constexpr int kTinyLd = 17;        // LDS row stride (doubles)
constexpr int kTinyTile = 16 * kTinyLd;

typedef double q4[4];

__device__ inline void wsync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ inline int lane_id() { return threadIdx.x & 63; }

// A wave-uniform double in scalar registers.
__device__ inline double tuni(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)u);
  const int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

struct TLane {
  int lr, lk;
  __device__ TLane() {
    const int l = lane_id();
    lr = l & 15;
    lk = l >> 4;
  }
  __device__ int row(int r) const { return 4 * r + lk; }
  __device__ double delta(int r) const { return 4 * r + lk == lr ? 1.0 : 0.0; }
};

__device__ inline void t_zero(q4 &x) {
#pragma unroll
  for (int r = 0; r < 4; ++r) x[r] = 0.0;
}

__device__ inline void t_copy(q4 &d, const q4 &x) {
#pragma unroll
  for (int r = 0; r < 4; ++r) d[r] = x[r];
}

// LDS tile <- register matrix (own elements).
__device__ inline void t_put(double *L, const TLane &ln, const q4 &x) {
  wsync();
#pragma unroll
  for (int r = 0; r < 4; ++r) L[ln.row(r) * kTinyLd + ln.lr] = x[r];
  wsync();
}

// acc += L * R, L in the wave's LDS tile, R in registers.
__device__ inline void t_gemm(const double *L, const TLane &ln, const q4 &R, q4 &acc) {
  dbl4 c = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
  for (int q = 0; q < 4; ++q) c = __builtin_amdgcn_mfma_f64_16x16x4f64(L[ln.lr * kTinyLd + 4 * q + ln.lk], R[q], c, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = c[r];
}

// acc += L * L.
__device__ inline void t_gemm_sq(const double *L, const TLane &ln, q4 &acc) {
  dbl4 c = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
  for (int q = 0; q < 4; ++q)
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(L[ln.lr * kTinyLd + 4 * q + ln.lk], L[ln.row(q) * kTinyLd + ln.lr], c, 0,
                                             0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = c[r];
}

// 1-norm (largest column sum of |x|), the same value on every lane.
__device__ inline double t_norm1(const q4 &x) {
  double s = fabs(x[0]) + fabs(x[1]) + fabs(x[2]) + fabs(x[3]);
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) s = fmax(s, __shfl_xor(s, o));
  return tuni(s);
}

// 1-norm of an interleaved complex nin x nin matrix (nin <= 8), sum_i |z_ij| maximised over the
// columns j: lane j < nin sums its column.
__device__ __noinline__ double t_norm1_z(const double *A, int nin) {
  cgdouble *Ag = gptr(A);
  const int l = lane_id();
  double s = 0.0;
  if (l < nin)
    for (int r = 0; r < nin; ++r) s += hypot(Ag[2 * (r * nin + l)], Ag[2 * (r * nin + l) + 1]);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s = fmax(s, __shfl_xor(s, o));
  return tuni(s);
}

// Loads matrix (n x n real, or the real form [[X, -Y], [Y, X]] of an nin x nin interleaved
// complex matrix, n = 2 nin) zero-padded to 16 x 16.
__device__ inline void t_load(const double *A, int n, int nin, int cx, const TLane &ln, q4 &x) {
  cgdouble *Ag = gptr(A);
  const int c = ln.lr;
  if (!cx && n == 16) {  // full tile: no bounds to check
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = Ag[ln.row(r) * 16 + c];
    return;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = ln.row(r);
    double v = 0.0;
    if (row < n && c < n) {
      if (!cx) {
        v = Ag[row * n + c];
      } else {
        const int ri = row < nin ? row : row - nin, ci = c < nin ? c : c - nin;
        const bool im = (row < nin) != (c < nin);
        v = Ag[2 * (ri * nin + ci) + (im ? 1 : 0)];
        if (row < nin && c >= nin) v = -v;
      }
    }
    x[r] = v;
  }
}

__device__ inline void t_store(double *E, int n, int nin, int cx, const TLane &ln, const q4 &x) {
  gdouble *Eg = gptr(E);
  const int c = ln.lr;
  if (!cx && n == 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) Eg[ln.row(r) * 16 + c] = x[r];
    return;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = ln.row(r);
    if (!cx) {
      if (row < n && c < n) Eg[row * n + c] = x[r];
    } else if (c < nin) {
      if (row < nin) Eg[2 * (row * nin + c)] = x[r];
      else if (row < n) Eg[2 * ((row - nin) * nin + c) + 1] = x[r];
    }
  }
}

// Plain rule (eq. theta, Table 2) on bit patterns: for finite eta >= 0 and theta > 0 the
// order of the doubles is the order of their bit patterns, and the smallest s >= 0 with
// eta <= theta 2^s is 0 when eta <= theta, else the exponent difference plus one when eta's
// mantissa exceeds theta's.  Integer work on wave-uniform values; cost products + s, the
// cheapest degree wins, ties to the smaller s.
struct Theta {
  double t[kNumDeg];
};

__device__ inline void t_select_plain(const Theta &th, double eta, int *m_out, int *s_out) {
  const unsigned long long be = __builtin_bit_cast(unsigned long long, eta);
  const unsigned long long kFrac = (1ull << 52) - 1;
  int bm = kDeg[kNumDeg - 1], bs = 0, bc = 1 << 30;
#pragma unroll
  for (int i = 0; i < kNumDeg; ++i) {
    const unsigned long long bt = __builtin_bit_cast(unsigned long long, th.t[i]);
    const int si = be <= bt ? 0
                            : (int)((be >> 52) & 0x7ff) - (int)((bt >> 52) & 0x7ff) + ((be & kFrac) > (bt & kFrac) ? 1 : 0);
    const int ci = kProducts[i] + si;
    if (ci < bc || (ci == bc && si < bs)) { bm = kDeg[i]; bs = si; bc = ci; }
  }
  *m_out = bm;
  *s_out = bs;
}

// Selection (eq. theta; Table 2), then T_m(A / 2^s) (eqs. Algorithm83eA, poly12, poly.18) and
// s squarings, all within the wave.  X0 = A on entry; the result is left in AC.  The scaling
// is applied to the matrices (X = 2^-s A exactly, X^2 = 2^-2s A^2, ...), so the polynomial
// coefficients are the constants themselves.  Returns false when only (m, s) was asked for.
template <int SEL>
__device__ bool t_expm(const Consts &K, const Theta &th, double *L, const TLane &ln, q4 &X0, double eta,
                       int select_only, int *m_out, int *s_out, q4 &AC) {
  int m, s;
  t_select_plain(th, eta, &m, &s);
  m = __builtin_amdgcn_readfirstlane(m);
  s = __builtin_amdgcn_readfirstlane(s);
  const int m_plain = m, s_plain = s;
  q4 X1, X2;
  // X_p = 2^-sp A (sp the plain rule's s) before any power is formed: every matrix stays in range
#pragma unroll
  for (int r = 0; r < 4; ++r) X0[r] = ldexp(X0[r], -s);
  if (m_plain >= 2) {
    t_put(L, ln, X0);
    t_zero(X1);
    t_gemm(L, ln, X0, X1);  // X_p^2
  }
  if (m_plain >= 12) {
    t_zero(X2);
    t_gemm(L, ln, X1, X2);  // X_p^3
  }
  if (SEL == EXPM_SEL_ALPHA) {
    if (m_plain >= 2) {
      // a plain degree below 12 means s = 0 and an alpha degree of at most 8: A^3 is not needed;
      // ||A^k|| = 2^(k sp) ||X_p^k||
      const double n2 = unscale_norm(t_norm1(X1), 2, s_plain);
      const double n3 = m_plain >= 12 ? unscale_norm(t_norm1(X2), 3, s_plain) : -1.0;
      select_ms(K.theta, 1, eta, n2, n3, &m, &s);
      m = __builtin_amdgcn_readfirstlane(m);
      s = __builtin_amdgcn_readfirstlane(s);
    }
    // X^k = 2^(k (sp - s)) X_p^k, exactly
    const int dsc = s_plain - s;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      X0[r] = ldexp(X0[r], dsc);
      X1[r] = ldexp(X1[r], 2 * dsc);
      X2[r] = ldexp(X2[r], 3 * dsc);
    }
  }
  *m_out = m;
  *s_out = s;
  if (select_only) return false;
  // coefficients of the chosen degree only (scalar registers); the scaling is in the matrices
  auto coefs = [&](auto deg, double *c, int count) {
    double t[24];
    make_coefs(K, decltype(deg)::value, 0, t);
    for (int j = 0; j < count; ++j) c[j] = tuni(t[j]);
  };
  if (m == 1) {
    double c[1];
    coefs(std::integral_constant<int, 1>(), c, 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) AC[r] = ln.delta(r) + c[0] * X0[r];
  } else if (m == 2) {
    double c[2];
    coefs(std::integral_constant<int, 2>(), c, 2);
#pragma unroll
    for (int r = 0; r < 4; ++r) AC[r] = ln.delta(r) + c[0] * X0[r] + c[1] * X1[r];
  } else if (m == 4) {
    // T = I + c0 A + c1 (A^2 W), A^2 W = (c3 A + c4 A^2) A^2 + c2 A^2
    double c[5];
    coefs(std::integral_constant<int, 4>(), c, 5);
    q4 W;
#pragma unroll
    for (int r = 0; r < 4; ++r) W[r] = c[3] * X0[r] + c[4] * X1[r];
    t_put(L, ln, W);
    t_zero(AC);
    t_gemm(L, ln, X1, AC);
#pragma unroll
    for (int r = 0; r < 4; ++r) AC[r] = ln.delta(r) + c[0] * X0[r] + c[1] * (AC[r] + c[2] * X1[r]);
  } else if (m == 8) {
    // V = (c0 A + c1 A^2) A^2; A_4 = c2 V; T = (c3 A^2 + A_4)(c4 I + c5 A + c6 A^2 + c7 A_4)
    //   + c8 I + c9 A + c10 A^2
    double c[11];
    coefs(std::integral_constant<int, 8>(), c, 11);
    q4 W, V, R;
#pragma unroll
    for (int r = 0; r < 4; ++r) W[r] = c[0] * X0[r] + c[1] * X1[r];
    t_put(L, ln, W);
    t_zero(V);
    t_gemm(L, ln, X1, V);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double d = ln.delta(r), a4 = c[2] * V[r];
      W[r] = c[3] * X1[r] + a4;
      R[r] = c[4] * d + c[5] * X0[r] + c[6] * X1[r] + c[7] * a4;
      AC[r] = c[8] * d + c[9] * X0[r] + c[10] * X1[r];
    }
    t_put(L, ln, W);
    t_gemm(L, ln, R, AC);
  } else if (m == 12) {
    // B_j over (I, A, A^2, A^3); A_6 = B_3 + B_4 B_4; T = B_1 + (B_2 + A_6) A_6
    double c[16];
    coefs(std::integral_constant<int, 12>(), c, 16);
    q4 B1, B2, B3, B4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double d = ln.delta(r);
      B1[r] = c[0] * d + c[1] * X0[r] + c[2] * X1[r] + c[3] * X2[r];
      B2[r] = c[4] * d + c[5] * X0[r] + c[6] * X1[r] + c[7] * X2[r];
      B3[r] = c[8] * d + c[9] * X0[r] + c[10] * X1[r] + c[11] * X2[r];
      B4[r] = c[12] * d + c[13] * X0[r] + c[14] * X1[r] + c[15] * X2[r];
    }
    t_put(L, ln, B4);
    t_gemm_sq(L, ln, B3);  // A_6
#pragma unroll
    for (int r = 0; r < 4; ++r) B2[r] += B3[r];
    t_put(L, ln, B2);
    t_copy(AC, B1);
    t_gemm(L, ln, B3, AC);
  } else {
    // A^6 = A^3 A^3; B_1 over (I, A, A^2, A^3), B_2..B_5 over (I, A, A^2, A^3, A^6);
    // A_9 = B_1 B_5 + B_4; T = B_2 + (B_3 + A_9) A_9
    double c[24];
    coefs(std::integral_constant<int, 18>(), c, 24);
    q4 X6, B2, B3, B4, B5;
    t_put(L, ln, X2);
    t_zero(X6);
    t_gemm_sq(L, ln, X6);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double d = ln.delta(r), a1 = X0[r], a2 = X1[r], a3 = X2[r], a6 = X6[r];
      X2[r] = c[0] * d + c[1] * a1 + c[2] * a2 + c[3] * a3;  // B_1
      B2[r] = c[4] * d + c[5] * a1 + c[6] * a2 + c[7] * a3 + c[8] * a6;
      B3[r] = c[9] * d + c[10] * a1 + c[11] * a2 + c[12] * a3 + c[13] * a6;
      B4[r] = c[14] * d + c[15] * a1 + c[16] * a2 + c[17] * a3 + c[18] * a6;
      B5[r] = c[19] * d + c[20] * a1 + c[21] * a2 + c[22] * a3 + c[23] * a6;
    }
    t_put(L, ln, X2);
    t_gemm(L, ln, B5, B4);  // A_9
#pragma unroll
    for (int r = 0; r < 4; ++r) B3[r] += B4[r];
    t_put(L, ln, B3);
    t_copy(AC, B2);
    t_gemm(L, ln, B4, AC);
  }
  for (int q = 0; q < s; ++q) {
    t_put(L, ln, AC);
    t_zero(AC);
    t_gemm_sq(L, ln, AC);
  }
  return true;
}


__device__ inline void t_squarings(double *L, const TLane &ln, int s, q4 &AC) {
  for (int q = 0; q < s; ++q) {
    t_put(L, ln, AC);
    t_zero(AC);
    t_gemm_sq(L, ln, AC);
  }
}

// 1/k!, k <= 16 (every k! there is an exact double, so each quotient is correctly rounded).
constexpr double kTInvFact[17] = {1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0,
                                  1.0 / 5040.0, 1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0,
                                  1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0,
                                  1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0};

// Innermost term and Horner steps of eq. poli9, degree M = Q R with base X^Q: X0..X3 hold X,
// X^2, X^3 (and X^4 when Q = 4), X = 2^-s A, so the coefficients are c_k = 1/k! themselves
// (compile-time constants).  F_j = sum_(i < Q) c_(Q j + i) X^i;
// T = F_0 + (F_1 + (... + (F_(R-1) + c_M X^Q) X^Q ...) X^Q) X^Q.
template <int Q, int R>
__device__ inline void t_ps_horner(double *L, const TLane &ln, const q4 &X0, const q4 &X1, const q4 &X2,
                                   const q4 &X3, q4 &AC) {
  auto F = [&](auto jc, int r) {
    constexpr int j = decltype(jc)::value;
    double v = kTInvFact[Q * j] * ln.delta(r) + kTInvFact[Q * j + 1] * X0[r] + kTInvFact[Q * j + 2] * X1[r];
    if constexpr (Q == 4) v += kTInvFact[Q * j + 3] * X2[r];
    return v;
  };
  q4 Rm;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    Rm[r] = F(std::integral_constant<int, R - 1>(), r);
    if constexpr (Q == 4) Rm[r] += kTInvFact[Q * R] * X3[r];
    else Rm[r] += kTInvFact[Q * R] * X2[r];
  }
  auto step = [&](auto jc) {
    t_put(L, ln, Rm);
#pragma unroll
    for (int r = 0; r < 4; ++r) AC[r] = F(jc, r);
    if constexpr (Q == 4) t_gemm(L, ln, X3, AC);  // F_j + R_(j+1) X^4
    else t_gemm(L, ln, X2, AC);                   // F_j + R_(j+1) X^3
    t_copy(Rm, AC);
  };
  if constexpr (R >= 4) step(std::integral_constant<int, 2>());
  if constexpr (R >= 3) step(std::integral_constant<int, 1>());
  step(std::integral_constant<int, 0>());
}

// The Paterson-Stockmeyer comparison (Sec. 4, eq. poli9): (m, s) over the degrees of Table 3,
// then the plain Taylor polynomial in Horner form, then s squarings.
__device__ bool t_expm_ps(const Consts &K, double *L, const TLane &ln, q4 &X0, double eta, int select_only,
                          int *m_out, int *s_out, q4 &AC) {
  int m, s;
  select_ps(K.theta_ps, eta, &m, &s);
  m = __builtin_amdgcn_readfirstlane(m);
  s = __builtin_amdgcn_readfirstlane(s);
  *m_out = m;
  *s_out = s;
  if (select_only) return false;
#pragma unroll
  for (int r = 0; r < 4; ++r) X0[r] = ldexp(X0[r], -s);
  q4 X1, X2, X3;
  if (m >= 2) {
    t_put(L, ln, X0);
    t_zero(X1);
    t_gemm(L, ln, X0, X1);  // X^2
  }
  if (m >= 6) {
    t_zero(X2);
    t_gemm(L, ln, X1, X2);  // X^3
  }
  if (m == 16) {
    t_put(L, ln, X1);
    t_zero(X3);
    t_gemm(L, ln, X1, X3);  // X^4 = X^2 X^2
  }
  if (m <= 4) {
    double c[5];
    make_coefs(K, m, 0, c);
#pragma unroll
    for (int j = 0; j < 5; ++j) c[j] = tuni(c[j]);
    if (m == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) AC[r] = ln.delta(r) + c[0] * X0[r];
    } else if (m == 2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) AC[r] = ln.delta(r) + c[0] * X0[r] + c[1] * X1[r];
    } else {
      q4 W;
#pragma unroll
      for (int r = 0; r < 4; ++r) W[r] = c[3] * X0[r] + c[4] * X1[r];
      t_put(L, ln, W);
      t_zero(AC);
      t_gemm(L, ln, X1, AC);
#pragma unroll
      for (int r = 0; r < 4; ++r) AC[r] = ln.delta(r) + c[0] * X0[r] + c[1] * (AC[r] + c[2] * X1[r]);
    }
  } else {
    if (m == 6) t_ps_horner<3, 2>(L, ln, X0, X1, X2, X3, AC);
    else if (m == 9) t_ps_horner<3, 3>(L, ln, X0, X1, X2, X3, AC);
    else if (m == 12) t_ps_horner<3, 4>(L, ln, X0, X1, X2, X3, AC);
    else t_ps_horner<4, 4>(L, ln, X0, X1, X2, X3, AC);
  }
  t_squarings(L, ln, s, AC);
  return true;
}

constexpr int kGjLd = 33;  // row stride of the wave's 16 x 32 elimination tile

// Solves M R = B in place on the wave's tile G = [M | B] (16 rows, columns 0..15 and 16..31):
// Gauss-Jordan elimination with partial pivoting (row k takes the largest |M[i][k]|, i >= k).
// Lane l eliminates row l / 4 over columns 8 (l % 4) .. 8 (l % 4) + 7.
__device__ inline void t_gauss_jordan(double *G) {
  const int lane = lane_id();
  const int gi = lane >> 2, gc = (lane & 3) * 8;
  for (int k = 0; k < 16; ++k) {
    wsync();
    double v = (lane >= k && lane < 16) ? fabs(G[lane * kGjLd + k]) : -1.0;
    int idx = lane;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const double ov = __shfl_xor(v, o);
      const int oi = __shfl_xor(idx, o);
      if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    const int p = __builtin_amdgcn_readfirstlane(idx);  // lane 0 holds the argmax of lanes 0..15
    if (p != k && lane < 32) {
      const double x = G[k * kGjLd + lane], y = G[p * kGjLd + lane];
      G[k * kGjLd + lane] = y;
      G[p * kGjLd + lane] = x;
    }
    wsync();
    const double piv = G[k * kGjLd + k];
    wsync();
    if (lane < 32) G[k * kGjLd + lane] = G[k * kGjLd + lane] / piv;
    wsync();
    const double f = G[gi * kGjLd + k];
    wsync();
    if (gi != k) {
#pragma unroll
      for (int t = 0; t < 8; ++t) G[gi * kGjLd + gc + t] -= f * G[k * kGjLd + gc + t];
    }
  }
  wsync();
}

// The Pade comparison (Sec. 2): (2m, s) by select_pade, r_10 (eq. eq.pade10) or r_26
// (eq. eq.pade26) at X = 2^-s A, the solve (-U + V) R = U + V, then s squarings.
__device__ bool t_expm_pade(const Consts &K, double *L, double *G, const TLane &ln, q4 &X0, double eta,
                            int select_only, int *m_out, int *s_out, q4 &AC) {
  int m, s;
  select_pade(K.theta_pade, eta, &m, &s);
  m = __builtin_amdgcn_readfirstlane(m);
  s = __builtin_amdgcn_readfirstlane(s);
  *m_out = m;
  *s_out = s;
  if (select_only) return false;
#pragma unroll
  for (int r = 0; r < 4; ++r) X0[r] = ldexp(X0[r], -s);
  q4 A2, A4, U, V;
  t_put(L, ln, X0);
  t_zero(A2);
  t_gemm(L, ln, X0, A2);  // A_2
  t_put(L, ln, A2);
  t_zero(A4);
  t_gemm(L, ln, A2, A4);  // A_4
  if (m == 10) {
    double b[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) b[j] = tuni(K.pade5[j]);
    q4 W;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double d = ln.delta(r);
      W[r] = b[5] * A4[r] + b[3] * A2[r] + b[1] * d;
      V[r] = b[4] * A4[r] + b[2] * A2[r] + b[0] * d;
    }
    t_put(L, ln, X0);
    t_zero(U);
    t_gemm(L, ln, W, U);  // u_5 = A (b5 A_4 + b3 A_2 + b1 I)
  } else {
    double b[14];
#pragma unroll
    for (int j = 0; j < 14; ++j) b[j] = tuni(K.pade13[j]);
    q4 A6, W, Z;
    t_zero(A6);
    t_gemm(L, ln, A4, A6);  // A_6 = A_2 A_4 (A_2 still in L)
#pragma unroll
    for (int r = 0; r < 4; ++r) W[r] = b[13] * A6[r] + b[11] * A4[r] + b[9] * A2[r];
    t_put(L, ln, A6);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      Z[r] = b[7] * A6[r] + b[5] * A4[r] + b[3] * A2[r] + b[1] * ln.delta(r);
    t_gemm(L, ln, W, Z);  // A_6 (b13 A_6 + b11 A_4 + b9 A_2) + b7 A_6 + b5 A_4 + b3 A_2 + b1 I
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      W[r] = b[12] * A6[r] + b[10] * A4[r] + b[8] * A2[r];
      V[r] = b[6] * A6[r] + b[4] * A4[r] + b[2] * A2[r] + b[0] * ln.delta(r);
    }
    t_gemm(L, ln, W, V);  // v_13 (A_6 still in L)
    t_put(L, ln, X0);
    t_zero(U);
    t_gemm(L, ln, Z, U);  // u_13 = A ( ... )
  }
  wsync();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    G[ln.row(r) * kGjLd + ln.lr] = V[r] - U[r];
    G[ln.row(r) * kGjLd + 16 + ln.lr] = V[r] + U[r];
  }
  t_gauss_jordan(G);
#pragma unroll
  for (int r = 0; r < 4; ++r) AC[r] = G[ln.row(r) * kGjLd + 16 + ln.lr];
  t_squarings(L, ln, s, AC);
  return true;
}

__device__ inline void copy_consts(const Consts &src, Consts *dst) {
  const double *s = reinterpret_cast<const double *>(&src);
  double *d = reinterpret_cast<double *>(dst);
  for (int e = threadIdx.x; e < (int)(sizeof(Consts) / sizeof(double)); e += blockDim.x) d[e] = s[e];
  __syncthreads();
}

// Matrices of this wave: a static stride over the sweep's range [lo, hi), read from the
// work queue's bounds when there is a queue.  Matrices of one padded order cost about the
// same, and one atomic per matrix on a counter shared by thousands of waves would serialise
// in L2, so this sweep takes no counter.
struct TSweep {
  int64_t lo, hi, next, stride;
  __device__ explicit TSweep(const FusedArgs &a) {
    const int64_t wave = (int64_t)blockIdx.x * kTinyW + (threadIdx.x >> 6);
    if (a.queue) {
      lo = (int64_t)a.queue[kQBound + a.q_lo];
      hi = (int64_t)a.queue[kQBound + a.q_hi];
    } else {
      lo = a.lo;
      hi = a.hi;
    }
    next = lo + wave;
    stride = (int64_t)gridDim.x * kTinyW;
  }
  __device__ int64_t pop() {
    const int64_t idx = next;
    next += stride;
    return idx;
  }
};

// Matrix of a queue entry: index, orders and element offset, read by the whole wave.
struct TItem {
  int64_t b, off;
  int nin, n;
};

__device__ inline TItem t_item(const FusedArgs &a, int64_t idx) {
  TItem it;
  it.b = a.order ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[idx]) : idx;
  it.nin = __builtin_amdgcn_readfirstlane(a.ns ? a.ns[it.b] : a.n_uniform);
  it.n = a.cplx ? 2 * it.nin : it.nin;
  it.off = (a.offs ? a.offs[it.b] : it.b * (int64_t)it.nin * it.nin) * (a.cplx ? 2 : 1);
  return it;
}

// Persistent: each wave takes matrices from its sweep until the range is empty.  The next
// matrix's load is issued before the current one is computed, so every wave keeps an HBM
// read in flight while its MFMA chain runs.
template <int SEL, int METHOD>
__global__ __launch_bounds__(64 * kTinyW, SEL == EXPM_SEL_PLAIN ? 4 : 2) void expm_tiny_kernel(FusedArgs a) {
  __shared__ double tiles[kTinyW * kTinyTile];
  __shared__ double gj[METHOD == 2 ? kTinyW * 16 * kGjLd : 1];
  __shared__ Consts K;
  copy_consts(a.k, &K);
  Theta th;
#pragma unroll
  for (int i = 0; i < kNumDeg; ++i) th.t[i] = a.k.theta[i];
  double *L = tiles + (threadIdx.x >> 6) * kTinyTile;
  const TLane ln;
  const int cx = a.cplx;
  TSweep sw(a);
  int64_t idx = sw.pop();
  TItem cur;
  q4 Xc;
  if (idx < sw.hi) {
    cur = t_item(a, idx);
    if (cur.nin >= 1 && cur.n <= 16) t_load(a.A + cur.off, cur.n, cur.nin, cx, ln, Xc);
  }
  while (idx < sw.hi) {
    const int64_t nidx = sw.pop();
    TItem nxt;
    q4 Xn;
    if (nidx < sw.hi) {
      nxt = t_item(a, nidx);
      if (nxt.nin >= 1 && nxt.n <= 16) t_load(a.A + nxt.off, nxt.n, nxt.nin, cx, ln, Xn);
    }
    const int64_t b = cur.b;
    const int nin = cur.nin, n = cur.n;
    const int64_t off = cur.off;
    const bool head = lane_id() == 0;
    // ||A||_1 (a complex input's is that of A itself); taken only when the input is finite
    const bool finite = nin >= 1 && n <= 16 &&
                        !__any(!isfinite(Xc[0]) || !isfinite(Xc[1]) || !isfinite(Xc[2]) || !isfinite(Xc[3]));
    const double eta = !finite ? 0.0 : cx ? t_norm1_z(a.A + off, nin) : t_norm1(Xc);
    if (nin < 1 || n > 16) {
      if (head) {
        a.m_out[b] = -1; a.s_out[b] = -1;
        if (a.status) a.status[b] = (nin < 1 || n > a.np_max) ? EXPM_E_INVALID_ARG : EXPM_E_UNSUPPORTED;
      }
    } else if (!finite || !(eta <= __DBL_MAX__)) {
      // (a 1-norm that overflows is refused like a non-finite entry)
      if (a.E)
        for (int e = lane_id(); e < nin * nin * (cx ? 2 : 1); e += 64) a.E[off + e] = __builtin_nan("");
      if (head) {
        a.m_out[b] = -1; a.s_out[b] = -1;
        if (a.status) a.status[b] = EXPM_E_NONFINITE;
      }
    } else {
      q4 AC;
      int m, s;
      bool full;
      if constexpr (METHOD == 1) full = t_expm_ps(K, L, ln, Xc, eta, a.select_only, &m, &s, AC);
      else if constexpr (METHOD == 2)
        full = t_expm_pade(K, L, gj + (threadIdx.x >> 6) * 16 * kGjLd, ln, Xc, eta, a.select_only, &m, &s, AC);
      else full = t_expm<SEL>(K, th, L, ln, Xc, eta, a.select_only, &m, &s, AC);
      if (head) {
        a.m_out[b] = m; a.s_out[b] = s;
        if (a.status) a.status[b] = EXPM_OK;
      }
      if (full) t_store(a.E + off, n, nin, cx, ln, AC);
    }
    idx = nidx;
    cur = nxt;
    t_copy(Xc, Xn);
  }
}

struct MagnusArgs {
  const double *S0, *S1, *Yin;
  double *Yout;
  const double *u1, *u2;
  int32_t *m_out, *s_out, *status;
  int64_t batch, s_stride;
  int n;
  double h, k_comm;  // h and sqrt(3) h^2 / 12
  Consts k;
};

// One fourth-order Magnus step per wave:
//   Omega = h S0 + (h/2)(u1 + u2) S1 + (sqrt(3) h^2 / 12)(u1 - u2)(S0 S1 - S1 S0),
//   Y <- e^Omega Y.
template <int SEL>
__global__ __launch_bounds__(64 * kTinyW, SEL == EXPM_SEL_PLAIN ? 4 : 2) void expm_magnus4_kernel(MagnusArgs a) {
  __shared__ double tiles[kTinyW * kTinyTile];
  __shared__ Consts K;
  copy_consts(a.k, &K);
  Theta th;
#pragma unroll
  for (int i = 0; i < kNumDeg; ++i) th.t[i] = a.k.theta[i];
  double *L = tiles + (threadIdx.x >> 6) * kTinyTile;
  const TLane ln;
  const int n = a.n;
  const int64_t stride = (int64_t)gridDim.x * kTinyW;
  for (int64_t b = (int64_t)blockIdx.x * kTinyW + (threadIdx.x >> 6); b < a.batch; b += stride) {
    const bool head = lane_id() == 0;
    const int64_t so = b * a.s_stride, yo = b * (int64_t)n * n;
    q4 S0, S1, Y, C, AC;
    t_load(a.S0 + so, n, n, 0, ln, S0);
    t_load(a.S1 + so, n, n, 0, ln, S1);
    t_load(a.Yin + yo, n, n, 0, ln, Y);
    const double u1 = tuni(a.u1[b]), u2 = tuni(a.u2[b]);
    bool bad = !isfinite(u1) || !isfinite(u2);
#pragma unroll
    for (int r = 0; r < 4; ++r) bad = bad || !isfinite(S0[r]) || !isfinite(S1[r]) || !isfinite(Y[r]);
    if (__any(bad)) {
      for (int e = lane_id(); e < n * n; e += 64) a.Yout[yo + e] = __builtin_nan("");
      if (head) {
        a.m_out[b] = -1; a.s_out[b] = -1;
        if (a.status) a.status[b] = EXPM_E_NONFINITE;
      }
      continue;
    }
    // Omega, with the commutator S0 S1 - S1 S0 from two products
    q4 P, W;
    t_zero(P);
    t_put(L, ln, S0);
    t_gemm(L, ln, S1, P);  // S0 S1
    t_zero(C);
    t_put(L, ln, S1);
    t_gemm(L, ln, S0, C);  // S1 S0
    const double ca = a.h, cb = 0.5 * a.h * (u1 + u2), cc = a.k_comm * (u1 - u2);
#pragma unroll
    for (int r = 0; r < 4; ++r) W[r] = ca * S0[r] + cb * S1[r] + cc * (P[r] - C[r]);
    int m, s;
    t_expm<SEL>(K, th, L, ln, W, t_norm1(W), 0, &m, &s, AC);
    t_put(L, ln, AC);
    t_zero(C);
    t_gemm(L, ln, Y, C);
    t_store(a.Yout + yo, n, n, 0, ln, C);
    if (head) {
      a.m_out[b] = m; a.s_out[b] = s;
      if (a.status) a.status[b] = EXPM_OK;
    }
  }
}

}  // namespace

int tiny_max_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, expm_tiny_kernel<EXPM_SEL_PLAIN, 0>, 64 * kTinyW, 0) !=
      hipSuccess)
    return 1;
  return nb < 1 ? 1 : nb;
}

hipError_t launch_tiny(const FusedArgs &a, int grid, hipStream_t st) {
  if (a.method == 1)
    hipLaunchKernelGGL((expm_tiny_kernel<EXPM_SEL_PLAIN, 1>), dim3(grid), dim3(64 * kTinyW), 0, st, a);
  else if (a.method == 2)
    hipLaunchKernelGGL((expm_tiny_kernel<EXPM_SEL_PLAIN, 2>), dim3(grid), dim3(64 * kTinyW), 0, st, a);
  else if (a.sel == EXPM_SEL_ALPHA)
    hipLaunchKernelGGL((expm_tiny_kernel<EXPM_SEL_ALPHA, 0>), dim3(grid), dim3(64 * kTinyW), 0, st, a);
  else
    hipLaunchKernelGGL((expm_tiny_kernel<EXPM_SEL_PLAIN, 0>), dim3(grid), dim3(64 * kTinyW), 0, st, a);
  return hipGetLastError();
}

int tiny_waves_per_block() { return kTinyW; }

hipError_t launch_magnus4(const double *S0, const double *S1, int64_t s_stride, const double *Yin, double *Yout,
                          const double *u1, const double *u2, int n, int64_t batch, double h, int sel,
                          const Consts &k, int32_t *m_out, int32_t *s_out, int32_t *status, int grid,
                          hipStream_t st) {
  MagnusArgs a;
  a.S0 = S0; a.S1 = S1; a.Yin = Yin; a.Yout = Yout; a.u1 = u1; a.u2 = u2;
  a.m_out = m_out; a.s_out = s_out; a.status = status;
  a.batch = batch; a.s_stride = s_stride; a.n = n;
  a.h = h;
  a.k_comm = sqrt(3.0) * h * h / 12.0;
  a.k = k;
  if (sel == EXPM_SEL_ALPHA)
    hipLaunchKernelGGL(expm_magnus4_kernel<EXPM_SEL_ALPHA>, dim3(grid), dim3(64 * kTinyW), 0, st, a);
  else
    hipLaunchKernelGGL(expm_magnus4_kernel<EXPM_SEL_PLAIN>, dim3(grid), dim3(64 * kTinyW), 0, st, a);
  return hipGetLastError();
}

}  // namespace expm
