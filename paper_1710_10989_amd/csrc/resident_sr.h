// Split-row resident evaluation for real orders np = 80, 96 (T = np / 16 = 5, 6): both operands
// of every product resident in LDS, 12 waves per workgroup.
//
// At these orders two np x np matrices fit in LDS together (2 x 72 KiB at np = 96), so the
// right operand of a product need not come from registers.  Then a column tile can be split
// between two waves: wave w owns column tile j = w % T and the row half H = w / T of it (row
// tiles i0 .. i0 + RT - 1, RT = ceil(T / 2) for the upper half, floor for the lower).  A
// register matrix costs a wave 8 RT VGPRs (24 at np = 96) instead of 8 T, so no matrix has to be
// parked, and 12 waves (3 per SIMD) keep the four SIMDs evenly loaded where the 8-wave scheme
// leaves two of them with one working wave.  Each product L R writes the operands it needs into
// the two LDS matrices (L1 left, L2 right; a square reads both from L1), then every wave
// accumulates its RT tiles: per k step RT left-operand reads, one right-operand read and RT
// MFMAs.  Register and LDS layouts are those of the 8-wave scheme (resident.h).
//
// Included by expm_fused.hip after resident.h.
#pragma once

namespace expm {
namespace {

constexpr int kSrNW = 12;     // waves per workgroup
constexpr int kSrTMin = 5;    // orders served: T = 5, 6
constexpr int kSrTMax = 6;

__shared__ double g_sr1[96 * 96];
__shared__ double g_sr2[96 * 96];
__shared__ double sh_colpart[2][96];

// Geometry of the lane's tile within the split: H = row half (compile time), RT row tiles
// starting at tile I0.
template <int T, int H>
struct SrGeo {
  static constexpr int RT = H == 0 ? (T + 1) / 2 : T / 2;
  static constexpr int I0 = H == 0 ? 0 : (T + 1) / 2;
  static constexpr int S = Res<T>::S;
};

struct SrLane {
  int j, lr, lk, col;
  __device__ explicit SrLane(int T) {
    const int tid = opq(threadIdx.x);
    const int w = tid >> 6, lane = tid & 63;
    j = w % T;
    lr = lane & 15;
    lk = lane >> 4;
    col = 16 * j + lr;
  }
};

// LDS offsets of the lane's own elements (row 16 (I0 + i) + 4 r + lk, column col).
template <int T, int H>
struct SrOwn {
  typedef SrGeo<T, H> G;
  int b[4];
  int dd;
  __device__ explicit SrOwn(const SrLane &ln) {
    const int lk = opq(ln.lk), col = opq(ln.col);
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = lk * G::S + (col ^ swz(4 * r + lk));
    dd = col - lk;
  }
  __device__ int at(int i, int r) const { return b[r] + (16 * (G::I0 + i) + 4 * r) * G::S; }
  __device__ double delta(int i, int r) const { return dd == 16 * (G::I0 + i) + 4 * r ? 1.0 : 0.0; }
};

template <int T, int H>
__device__ inline void sr_put(double *L, const SrLane &ln, const dbl4 (&x)[SrGeo<T, H>::RT]) {
  const SrOwn<T, H> o(ln);
#pragma unroll
  for (int i = 0; i < SrGeo<T, H>::RT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) L[o.at(i, r)] = x[i][r];
}

// acc += Lm * Rm over the lane's tiles, both operands resident in LDS (they may coincide).
template <int T, int H>
__device__ inline void sr_gemm(const double *Lm, const double *Rm, const SrLane &ln,
                               dbl4 (&acc)[SrGeo<T, H>::RT]) {
  typedef SrGeo<T, H> G;
  constexpr int S = G::S, RT = G::RT;
  const int lr = opq(ln.lr), lk = opq(ln.lk), col = opq(ln.col);
  const double *Lrow = Lm + (16 * G::I0 + lr) * S;
  const int sw = swz(lr);
  int cb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) cb[r] = lk * S + (col ^ swz(4 * r + lk));
  double a[2][RT], bq[2];
  auto fetch = [&](int q, double (&da)[RT], double &db) {
    const int kc = (4 * q + lk) ^ sw;
#pragma unroll
    for (int i = 0; i < RT; ++i) da[i] = Lrow[i * 16 * S + kc];
    db = Rm[cb[q & 3] + 4 * q * S];
  };
  fetch(0, a[0], bq[0]);
#pragma unroll
  for (int q = 0; q < 4 * T; ++q) {
    if (q + 1 < 4 * T) fetch(q + 1, a[(q + 1) & 1], bq[(q + 1) & 1]);
#pragma unroll
    for (int i = 0; i < RT; ++i)
      acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q & 1][i], bq[q & 1], acc[i], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Workgroup maximum over columns of the per-column sums f(column partials of both halves).
// Each wave passes its lanes' partial sums over its RT tiles (column col); returns the maximum
// column total to every thread.
__device__ inline double sr_colmax(double part, const SrLane &ln, int H, bool act, int np, double *red) {
  part += __shfl_xor(part, 16);
  part += __shfl_xor(part, 32);
  if (act && ln.lk == 0) sh_colpart[H][ln.col] = part;
  __syncthreads();
  const int t = threadIdx.x;
  const double v = t < np ? sh_colpart[0][t] + sh_colpart[1][t] : 0.0;
  __syncthreads();
  return wg_max<kSrNW>(v, red);
}

template <int T, int H>
__device__ inline double sr_abs_part(const dbl4 (&x)[SrGeo<T, H>::RT]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < SrGeo<T, H>::RT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) s += fabs(x[i][r]);
  return s;
}

// Runs the method on matrix b of real order n (np = 16 T) in the split-row scheme.  H: this
// wave's row half; IDLE: waves beyond 2 T (T = 5) take part in barriers and reductions only.
template <int SEL, int T, int H, bool IDLE>
__device__ __attribute__((always_inline)) void run_sr(const FusedArgs &a, int64_t b, int n, int nin, int cx, int64_t off, double *red) {
  typedef SrGeo<T, H> G;
  constexpr int RT = G::RT, S = G::S;
  constexpr bool act = !IDLE;
  double *L1 = g_sr1, *L2 = g_sr2;
  const int tid = threadIdx.x;
  const SrLane ln(T);
  dbl4 X0[RT];

  // ---- load A (real form of a complex input) into X0 and L1; finiteness, 1-norm ----
  int bad = 0;
  double csum = 0.0;
  if constexpr (act) {
    cgdouble *Ag = gptr(a.A + off);
    const int lk = opq(ln.lk), c = opq(ln.col);
    const bool cin = c < n;
    const int cc = cin ? c : n - 1;
    if (!cx) {
      // real input: one buffer load per element at a 32-bit byte offset; padding rows and
      // columns lie past the buffer's n^2 elements and read as zero
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(ufp(a.A + off), 0, n * n * 8, kBufWord3);
      const int lb = cin ? (lk * n + c) * 8 : n * n * 8;
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const u2v v = __builtin_amdgcn_raw_buffer_load_b64(rs, lb + (16 * (G::I0 + i) + 4 * r) * n * 8, 0, 0);
          X0[i][r] = __longlong_as_double((long long)(((unsigned long long)v[1] << 32) | v[0]));
        }
    } else {
      const int ci = cc < nin ? cc : cc - nin;
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (G::I0 + i) + 4 * r + lk;
          const int rr = row < n ? row : n - 1;
          const int ri = rr < nin ? rr : rr - nin;
          const bool im = (rr < nin) != (cc < nin);
          X0[i][r] = Ag[2 * ((size_t)ri * nin + ci) + (im ? 1 : 0)];
        }
    }
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (G::I0 + i) + 4 * r + lk;
        double x = X0[i][r];
        if (cx && (row < nin) && !(cc < nin)) x = -x;  // -Y block of the real form
        x = (row < n && cin) ? x : 0.0;
        X0[i][r] = x;
        bad |= !isfinite(x);
        csum += fabs(x);
      }
    if (cx) {
      // complex input: the 1-norm of A itself, sum_i |z_ij| over the columns of the X block
      csum = 0.0;
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (G::I0 + i) + 4 * r + lk;
          if (row < nin && c < nin) csum += hypot(X0[i][r], Ag[2 * ((size_t)row * nin + c) + 1]);
        }
    }
  }
  bad = ufi(__syncthreads_or(bad));
  const double eta = sr_colmax(csum, ln, H, act, 16 * T, red);
  // a 1-norm that overflows (finite entries) is refused like a non-finite entry
  if (bad || !(eta <= __DBL_MAX__)) {
    double *E = a.E ? a.E + off : nullptr;
    if (E) for (int e = tid; e < nin * nin * (cx ? 2 : 1); e += 64 * kSrNW) E[e] = __builtin_nan("");
    if (tid == 0) {
      a.m_out[b] = -1; a.s_out[b] = -1;
      if (a.status) a.status[b] = EXPM_E_NONFINITE;
    }
    __syncthreads();
    return;
  }

  int m_rule, s_plain;
  select_ms(sh_consts.theta, 0, eta, -1.0, -1.0, &m_rule, &s_plain);
  m_rule = ufi(m_rule);
  s_plain = ufi(s_plain);
  // X_p = 2^-sp A (sp the plain rule's s, exact) into L1: every power formed from here on
  // stays in range
  if constexpr (act) {
    if (s_plain > 0) {
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) X0[i][r] = ldexp(X0[i][r], -s_plain);
    }
    sr_put<T, H>(L1, ln, X0);
  }
  __syncthreads();

  // The rest of the method, per degree under the plain rule (see run_res).
  auto rest = [&](auto Mc) __attribute__((always_inline)) {
    constexpr int MC = decltype(Mc)::value;
    const int m_plain = MC == 0 ? m_rule : MC == 2 ? (m_rule <= 1 ? 1 : 2) : MC;
    int m = m_plain, s = s_plain;
    dbl4 X1[RT], X2[RT], X3[RT], AC[RT];

    // ---- A^2 (X1) = A A from L1; the norms the selector needs; A^3 (X2) at most once ----
    if (m_plain >= 2) {
      if constexpr (act) {
        zero<RT>(X1);
        sr_gemm<T, H>(L1, L1, ln, X1);
      }
    }
    double n2 = -1.0, n3 = -1.0;
    bool need3 = false;
    int mq = 0, sq = 0;
    if (SEL == EXPM_SEL_ALPHA && m_plain >= 2) {
      n2 = unscale_norm(sr_colmax(act ? sr_abs_part<T, H>(X1) : 0.0, ln, H, act, 16 * T, red), 2, s_plain);
      need3 = m_plain >= 12;
    } else if (SEL == EXPM_SEL_LEARNED && m_plain >= 2) {
      n2 = unscale_norm(sr_colmax(act ? sr_abs_part<T, H>(X1) : 0.0, ln, H, act, 16 * T, red), 2, s_plain);
      double tr = 0.0, asy = 0.0;
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
        const int lk = opq(ln.lk), col = opq(ln.col);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            tr += o.delta(i, r) * X0[i][r];
            const int row = 16 * (G::I0 + i) + 4 * r + lk;  // A^T element from the resident A
            asy += fabs(X0[i][r] - L1[col * S + (row ^ swz(col))]);
          }
      }
      tr = ldexp(wg_sum<kSrNW>(act ? tr : 0.0, red), s_plain);  // of A, not of X_p
      asy = ldexp(sr_colmax(act ? asy : 0.0, ln, H, act, 16 * T, red), s_plain);
      const int cls = ufi(res_mlp<64 * kSrNW>(eta, n2, tr, asy, n));
      mlp_class_ms(cls, &mq, &sq);
      if (mq >= 12) {
        need3 = true;  // the acceptance test uses ||A^3||
      } else {
        const bool ok = ufi(res_proposal_ok(sh_consts.theta, eta, n2, -1.0, mq, sq)) != 0;
        if (ok) { m = mq; s = sq; }
        if (tid == 0) atomicAdd(&g_learned_counts[ok ? 0 : 1], 1ull);
        need3 = m >= 12;
      }
    } else {
      need3 = m_plain >= 12;
    }
    if (need3) {
      if constexpr (act) sr_put<T, H>(L2, ln, X1);  // L2 is idle since the last matrix
      __syncthreads();
      if constexpr (act) {
        zero<RT>(X2);
        sr_gemm<T, H>(L1, L2, ln, X2);
      }
      if (SEL == EXPM_SEL_ALPHA) {
        n3 = unscale_norm(sr_colmax(act ? sr_abs_part<T, H>(X2) : 0.0, ln, H, act, 16 * T, red), 3, s_plain);
        if (tid == 0) res_select(sh_consts.theta, 1, eta, n2, n3, &sh_ms[0], &sh_ms[1]);
        __syncthreads();
        m = ufi(sh_ms[0]); s = ufi(sh_ms[1]);
      } else if (SEL == EXPM_SEL_LEARNED && mq >= 12) {
        n3 = unscale_norm(sr_colmax(act ? sr_abs_part<T, H>(X2) : 0.0, ln, H, act, 16 * T, red), 3, s_plain);
        const bool ok = ufi(res_proposal_ok(sh_consts.theta, eta, n2, n3, mq, sq)) != 0;
        if (ok) { m = mq; s = sq; }
        if (tid == 0) atomicAdd(&g_learned_counts[ok ? 0 : 1], 1ull);
      }
    } else if (SEL == EXPM_SEL_ALPHA && m_plain >= 2) {
      if (tid == 0) res_select(sh_consts.theta, 1, eta, n2, -1.0, &sh_ms[0], &sh_ms[1]);
      __syncthreads();
      m = ufi(sh_ms[0]); s = ufi(sh_ms[1]);
    }
    if (tid == 0) {
      a.m_out[b] = m; a.s_out[b] = s;
      if (a.status) a.status[b] = EXPM_OK;
    }
    if (a.select_only) {
      __syncthreads();
      return;
    }
    // The powers held so far are those of X_p; the other rules may have chosen s != sp:
    // X^k = 2^(k (sp - s)) X_p^k, rescaled exactly.
    const int dsc = s_plain - s;
    if (SEL != EXPM_SEL_PLAIN && dsc != 0 && act) {
  #pragma unroll
      for (int i = 0; i < RT; ++i)
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          X0[i][r] = ldexp(X0[i][r], dsc);
          if (m_plain >= 2) X1[i][r] = ldexp(X1[i][r], 2 * dsc);
          if (need3) X2[i][r] = ldexp(X2[i][r], 3 * dsc);
        }
    }
    // coefficients of the chosen degree (the scaling is in the matrices)
    auto coefs = [&](auto deg, double *c, int count) {
      double t[24];
      make_coefs(sh_consts, decltype(deg)::value, 0, t);
      for (int j = 0; j < count; ++j) c[j] = uni(t[j]);
    };

    // ---- T_m(X) into AC (X0 = X, X1 = X^2, X2 = X^3 where formed) ----
    __syncthreads();  // every product so far has finished reading L1 and L2
    if (m <= 2) {
      double c[2];
      if (m == 2) coefs(std::integral_constant<int, 2>(), c, 2);
      else { coefs(std::integral_constant<int, 1>(), c, 1); c[1] = 0.0; }
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r)
            AC[i][r] = o.delta(i, r) + c[0] * X0[i][r] + (m == 2 ? c[1] * X1[i][r] : 0.0);
      }
    } else if (m == 4) {
      // T = I + c0 A + c1 V, V = A^2 W = A^2 (c2 I + c3 A + c4 A^2)
      double c[5];
      coefs(std::integral_constant<int, 4>(), c, 5);
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
        sr_put<T, H>(L1, ln, X1);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) L2[o.at(i, r)] = c[2] * o.delta(i, r) + c[3] * X0[i][r] + c[4] * X1[i][r];
      }
      __syncthreads();
      if constexpr (act) {
        zero<RT>(AC);
        sr_gemm<T, H>(L1, L2, ln, AC);
        const SrOwn<T, H> o(ln);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) AC[i][r] = o.delta(i, r) + c[0] * X0[i][r] + c[1] * AC[i][r];
      }
    } else if (m == 8) {
      // V = A^2 W1 (W1 = c0 A + c1 A^2); A_4 = c2 V; Lm = c3 A^2 + A_4;
      // Rm = c4 I + c5 A + c6 A^2 + c7 A_4; T = Lm Rm + c8 I + c9 A + c10 A^2   (eq. Algorithm83eA)
      double c[11];
      coefs(std::integral_constant<int, 8>(), c, 11);
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
        sr_put<T, H>(L1, ln, X1);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) L2[o.at(i, r)] = c[0] * X0[i][r] + c[1] * X1[i][r];
      }
      __syncthreads();
      if constexpr (act) {
        zero<RT>(X2);
        sr_gemm<T, H>(L1, L2, ln, X2);  // V
      }
      __syncthreads();
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double d = o.delta(i, r), a1 = X0[i][r], a2 = X1[i][r], a4 = c[2] * X2[i][r];
            L1[o.at(i, r)] = c[3] * a2 + a4;                                 // Lm
            L2[o.at(i, r)] = c[4] * d + c[5] * a1 + c[6] * a2 + c[7] * a4;   // Rm
            AC[i][r] = c[8] * d + c[9] * a1 + c[10] * a2;
          }
      }
      __syncthreads();
      if constexpr (act) sr_gemm<T, H>(L1, L2, ln, AC);
    } else if (m == 12) {
      // B_j over (I, A, A^2, A^3); A_6 = B_3 + B_4^2; T = B_1 + (B_2 + A_6) A_6   (eq. poly12)
      double k[16];
      coefs(std::integral_constant<int, 12>(), k, 16);
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double d = o.delta(i, r), a1 = X0[i][r], a2 = X1[i][r], a3 = X2[i][r];
            L1[o.at(i, r)] = k[12] * d + k[13] * a1 + k[14] * a2 + k[15] * a3;  // B_4
            X0[i][r] = k[0] * d + k[1] * a1 + k[2] * a2 + k[3] * a3;            // B_1
            X1[i][r] = k[4] * d + k[5] * a1 + k[6] * a2 + k[7] * a3;            // B_2
            AC[i][r] = k[8] * d + k[9] * a1 + k[10] * a2 + k[11] * a3;          // B_3
          }
      }
      __syncthreads();
      if constexpr (act) sr_gemm<T, H>(L1, L1, ln, AC);  // A_6 = B_3 + B_4 B_4
      __syncthreads();
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            L1[o.at(i, r)] = X1[i][r] + AC[i][r];  // Y = B_2 + A_6
            L2[o.at(i, r)] = AC[i][r];             // A_6
          }
      }
      __syncthreads();
      if constexpr (act) {
        sr_gemm<T, H>(L1, L2, ln, X0);  // T = B_1 + Y A_6
  #pragma unroll
        for (int i = 0; i < RT; ++i) AC[i] = X0[i];
      }
    } else {
      // m == 18: A^6 = A^3 A^3; B_1 over (I, A, A^2, A^3), B_2..B_5 over (I, A, A^2, A^3, A^6);
      // A_9 = B_1 B_5 + B_4; T = B_2 + (B_3 + A_9) A_9   (eq. poly.18)
      double k[24];
      coefs(std::integral_constant<int, 18>(), k, 24);
      if constexpr (act) sr_put<T, H>(L1, ln, X2);
      __syncthreads();
      if constexpr (act) {
        zero<RT>(X3);
        sr_gemm<T, H>(L1, L1, ln, X3);  // A^6
      }
      __syncthreads();
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double d = o.delta(i, r), a1 = X0[i][r], a2 = X1[i][r], a3 = X2[i][r], a6 = X3[i][r];
            L1[o.at(i, r)] = k[0] * d + k[1] * a1 + k[2] * a2 + k[3] * a3;                       // B_1
            X0[i][r] = k[4] * d + k[5] * a1 + k[6] * a2 + k[7] * a3 + k[8] * a6;               // B_2
            X1[i][r] = k[9] * d + k[10] * a1 + k[11] * a2 + k[12] * a3 + k[13] * a6;           // B_3
            AC[i][r] = k[14] * d + k[15] * a1 + k[16] * a2 + k[17] * a3 + k[18] * a6;          // B_4
            L2[o.at(i, r)] = k[19] * d + k[20] * a1 + k[21] * a2 + k[22] * a3 + k[23] * a6;    // B_5
          }
      }
      __syncthreads();
      if constexpr (act) sr_gemm<T, H>(L1, L2, ln, AC);  // A_9 = B_1 B_5 + B_4
      __syncthreads();
      if constexpr (act) {
        const SrOwn<T, H> o(ln);
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            L1[o.at(i, r)] = X1[i][r] + AC[i][r];  // Y = B_3 + A_9
            L2[o.at(i, r)] = AC[i][r];             // A_9
          }
      }
      __syncthreads();
      if constexpr (act) {
        sr_gemm<T, H>(L1, L2, ln, X0);  // T = B_2 + Y A_9
  #pragma unroll
        for (int i = 0; i < RT; ++i) AC[i] = X0[i];
      }
    }

    // ---- s squarings: the resident matrix is both operands ----
    for (int q = 0; q < s; ++q) {
      __syncthreads();
      if constexpr (act) sr_put<T, H>(L1, ln, AC);
      __syncthreads();
      if constexpr (act) {
        zero<RT>(AC);
        sr_gemm<T, H>(L1, L1, ln, AC);
      }
    }

    // ---- e^A ----
    if constexpr (act) {
      gdouble *E = gptr(a.E + off);
      const int lk = opq(ln.lk), col = opq(ln.col);
      if (!cx) {
        // real output through a buffer over the n^2 elements; stores of padding rows and
        // columns fall past its end and are dropped
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(ufp(a.E + off), 0, n * n * 8, kBufWord3);
        const int lb = col < n ? (lk * n + col) * 8 : n * n * 8;
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            const unsigned long long u = (unsigned long long)__double_as_longlong(AC[i][r]);
            __builtin_amdgcn_raw_buffer_store_b64(u2v{(unsigned)u, (unsigned)(u >> 32)}, rs,
                                                  lb + (16 * (G::I0 + i) + 4 * r) * n * 8, 0, 0);
          }
      } else {
  #pragma unroll
        for (int i = 0; i < RT; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) put_dst(E, n, nin, cx, 16 * (G::I0 + i) + 4 * r + lk, col, AC[i][r]);
      }
    }
    __syncthreads();
  };
  if constexpr (SEL == EXPM_SEL_PLAIN) {
    switch (m_rule) {
      case 18: rest(std::integral_constant<int, 18>()); break;
      case 12: rest(std::integral_constant<int, 12>()); break;
      case 8: rest(std::integral_constant<int, 8>()); break;
      case 4: rest(std::integral_constant<int, 4>()); break;
      default: rest(std::integral_constant<int, 2>()); break;
    }
  } else {
    rest(std::integral_constant<int, 0>());
  }
}

template <int SEL>
__device__ __attribute__((always_inline)) void run_sr_dispatch(const FusedArgs &a, int64_t b, double *red) {
  const int tid = threadIdx.x;
  // the order and the offset both depend on b only: both loads are issued before either is used
  const int32_t nraw = a.ns ? ((__attribute__((address_space(1))) const int32_t *)a.ns)[b] : a.n_uniform;
  const int64_t oraw = a.offs ? ((__attribute__((address_space(1))) const int64_t *)a.offs)[b] : 0;
  const int nin = ufi(nraw);
  const int cx = a.cplx;
  const int n = cx ? 2 * nin : nin;
  const int64_t off = (a.offs ? ufl(oraw) : b * (int64_t)nin * nin) * (cx ? 2 : 1);
  const int t = (n + 15) >> 4;
  if (nin < 1 || n > a.np_max || t < kSrTMin || t > kSrTMax) {  // invalid order, or wrong variant
    if (tid == 0) {
      a.m_out[b] = -1; a.s_out[b] = -1;
      if (a.status) a.status[b] = (nin < 1 || n > a.np_max) ? EXPM_E_INVALID_ARG : EXPM_E_UNSUPPORTED;
    }
    return;
  }
  const int w = (int)(threadIdx.x >> 6);  // wave-uniform
  if (t == 6) {
    if (w < 6) run_sr<SEL, 6, 0, false>(a, b, n, nin, cx, off, red);
    else run_sr<SEL, 6, 1, false>(a, b, n, nin, cx, off, red);
  } else {
    if (w < 5) run_sr<SEL, 5, 0, false>(a, b, n, nin, cx, off, red);
    else if (w < 10) run_sr<SEL, 5, 1, false>(a, b, n, nin, cx, off, red);
    else run_sr<SEL, 5, 1, true>(a, b, n, nin, cx, off, red);
  }
}

}  // namespace
}  // namespace expm
