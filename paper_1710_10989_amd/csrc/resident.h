// On-chip resident evaluation for real orders np <= 128 (np = n rounded up to 16): one
// workgroup per matrix.  Besides the input and the output, only up to two parked matrices
// (np >= 96) cross HBM.
//
// Data placement.  Wave w owns the column tile w (columns 16 w .. 16 w + 15) of every matrix
// it holds in registers, as the D layout of the 16x16x4 FP64 MFMA: register r of row tile i
// of lane l holds M[16 i + 4 r + l / 16][16 w + l % 16].  That layout is exactly the B-operand
// layout of the same MFMA for rows 4 q .. 4 q + 3 of M (q = 4 i + r), so a product L * R with
// R held in registers needs no data movement for R: per k step q each lane feeds its own
// element R(q).  The left operand L is the one matrix resident in LDS (the whole np x np
// matrix, 128 KiB at np = 128); lane l reads L[16 i + l % 16][4 q + l / 16] for row tile i.
// Every product of the method has at most one operand that is not at hand in registers
// (powers of A commute, so each product can be ordered to make that operand L), and the two
// products whose operands are equal (squarings, A^3 A^3, B_4 B_4) read both from LDS.
//
// LDS layout: row stride S (np rounded up to 32 doubles), element (r, c) at
// r S + (c ^ swz(r)) with swz(r) = (r & 15) | ((r & 1) << 4).  The XOR keeps the three access
// patterns conflict-free whether the banks repeat every 128 or every 256 bytes: left-operand
// reads (16 rows x 2 adjacent k per 32 lanes), right-operand reads and D-layout writes (2 rows x
// 16 adjacent columns per 32 lanes).
//
// Included by expm_fused.hip (shares the selection helpers and the learned-selector state).
#pragma once
#include <type_traits>

namespace expm {
namespace {

constexpr int kResTMax = 8;  // np <= 128

template <int T>
struct Res {
  static constexpr int NP = 16 * T;
  static constexpr int S = (NP + 31) & ~31;
};

__shared__ double g_res8[128 * 128];
__shared__ double g_res4[64 * 64];
__shared__ Consts sh_consts;  // copy of the kernel's constants for the out-of-line helpers
template <int NW>
__device__ inline double *res_lds() {
  if constexpr (NW == 4) return g_res4;
  else return g_res8;
}

__device__ inline int swz(int r) { return (r & 15) | ((r & 1) << 4); }

// Fourth word of a raw (untyped) buffer resource on gfx9-family targets: 32-bit data format.
constexpr int kBufWord3 = 0x00020000;
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

// Opaque copy: address arithmetic derived from it is redone at each use instead of being
// hoisted into registers that stay live across the whole matrix.
__device__ inline int opq(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Wave-uniform integer moved to a scalar register: branches on it are then uniform
// branches, not exec-masked regions that keep both sides' values alive.
__device__ inline int ufi(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline int64_t ufl(int64_t x) {
  return (int64_t)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(x >> 32)) << 32) |
                   (unsigned)__builtin_amdgcn_readfirstlane((int)x));
}

// A wave-uniform address moved to scalar registers (a buffer resource built on it then needs
// no per-access waterfall over the lanes' copies).
__device__ inline void *ufp(const void *p) {
  const unsigned long long u = (unsigned long long)p;
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return (void *)(((unsigned long long)hi << 32) | lo);
}

// A wave-uniform double moved to scalar registers (coefficients of the linear combinations).
__device__ inline double uni(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)u);
  const int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Per-lane geometry of the owned column tile.
struct Lane {
  int w, lr, lk, col;
  __device__ Lane() {
    const int tid = opq(threadIdx.x);  // recomputed per matrix, not held across the sweep
    w = tid >> 6;
    const int lane = tid & 63;
    lr = lane & 15;
    lk = lane >> 4;
    col = 16 * w + lr;
  }
  __device__ int row(int i, int r) const { return 16 * i + 4 * r + lk; }
};

// LDS offsets of the lane's own elements: at(i, r) = own element (row 16 i + 4 r + lk, column
// col); dd marks the diagonal: element (i, r) is on it iff 16 i + 4 r == dd.
template <int T>
struct Own {
  static constexpr int S = Res<T>::S;
  int b[4];
  int dd;
  __device__ explicit Own(const Lane &ln) {
    const int lk = opq(ln.lk), col = opq(ln.col);
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = lk * S + (col ^ swz(4 * r + lk));
    dd = col - lk;
  }
  __device__ int at(int i, int r) const { return b[r] + (16 * i + 4 * r) * S; }
  __device__ double delta(int i, int r) const { return dd == 16 * i + 4 * r ? 1.0 : 0.0; }
};

template <int T>
__device__ inline void zero(dbl4 (&x)[T]) {
#pragma unroll
  for (int i = 0; i < T; ++i) x[i] = dbl4{0.0, 0.0, 0.0, 0.0};
}

// Writes the lane's elements of a register matrix into the resident LDS matrix.
template <int T>
__device__ inline void to_lds(double *L, const Lane &ln, const dbl4 (&x)[T]) {
  const Own<T> o(ln);
#pragma unroll
  for (int i = 0; i < T; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) L[o.at(i, r)] = x[i][r];
}

// Reads the lane's elements of the resident LDS matrix into a register matrix.
template <int T>
__device__ inline void from_lds(const double *L, const Lane &ln, dbl4 (&x)[T]) {
  const Own<T> o(ln);
#pragma unroll
  for (int i = 0; i < T; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) x[i][r] = L[o.at(i, r)];
}

// acc += L * R over the owned column tile: L resident in LDS, R(q) the lane's B operand of k
// step q (rows 4 q .. 4 q + 3 of R).  The left-operand fragments of step q + 1 are read while
// step q multiplies; a scheduling barrier per step keeps the compiler from hoisting more
// steps' reads (which would cost registers the resident matrices need).
template <int T, class RF>
__device__ inline void rgemm(const double *L, const Lane &ln, const RF &rf, dbl4 (&acc)[T]) {
  constexpr int S = Res<T>::S;
  const int lr = opq(ln.lr), lk = opq(ln.lk);
  const double *Lrow = L + lr * S;
  const int sw = swz(lr);  // rows 16 i + lr share the swizzle
  double a[2][T];
  auto fetch = [&](int q, double (&dst)[T]) {
    const int kc = (4 * q + lk) ^ sw;
#pragma unroll
    for (int i = 0; i < T; ++i) dst[i] = Lrow[i * 16 * S + kc];
  };
  fetch(0, a[0]);
#pragma unroll
  for (int q = 0; q < 4 * T; ++q) {
    if (q + 1 < 4 * T) fetch(q + 1, a[(q + 1) & 1]);
    const double b = rf(q);
#pragma unroll
    for (int i = 0; i < T; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q & 1][i], b, acc[i], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// acc += L * R with R held in registers.
template <int T>
__device__ inline void rgemm_reg(const double *L, const Lane &ln, const dbl4 (&R)[T], dbl4 (&acc)[T]) {
  rgemm<T>(L, ln, [&](int q) { return R[q >> 2][q & 3]; }, acc);
}

// acc += L * L (both operands from the resident matrix; the B operand of k step q is the
// lane's element of rows 4 q .. 4 q + 3 in its own columns).
template <int T>
__device__ inline void rgemm_sq(const double *L, const Lane &ln, dbl4 (&acc)[T]) {
  constexpr int S = Res<T>::S;
  const int lk = opq(ln.lk), col = opq(ln.col);
  int cb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) cb[r] = lk * S + (col ^ swz(4 * r + lk));
  rgemm<T>(L, ln, [&](int q) { return L[cb[q & 3] + 4 * q * S]; }, acc);
}

// Workgroup maximum of a per-lane value (every thread passes one; returns it to all).
template <int NW>
__device__ inline double wg_max(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) r = fmax(r, red[k]);
  __syncthreads();
  return r;
}

template <int NW>
__device__ inline double wg_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) r += red[k];
  __syncthreads();
  return r;
}

// Column sums of |x| over the owned tile, reduced over the 4 row groups of a column; the
// workgroup maximum is the 1-norm of the register matrix.
template <int T>
__device__ inline double col_abs_sum(const dbl4 (&x)[T]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < T; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) s += fabs(x[i][r]);
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}

template <int NW, int T>
__device__ inline double norm1(const dbl4 (&x)[T], bool act, double *red) {
  return wg_max<NW>(act ? col_abs_sum<T>(x) : 0.0, red);  // act: compile-time in the callers
}

// Matrices parked in the workgroup's HBM slot (two regions of NW * T * 64 dbl4 each): lane l
// of wave w keeps its element (i, r) at ((w T + i) 4 + r) 64 + l of the region, so every
// access of a wave is 512 contiguous bytes, and each lane reads back only what it wrote.
template <int NW, int T>
struct Park {
  // Two addressings, chosen per order by measurement: for np >= 112 a buffer resource over
  // the region plus this lane's byte offset (each access is one VGPR offset and a constant
  // scalar offset, so no per-element 64-bit addresses are formed or kept: the register
  // budget is tightest there); below, plain global addressing.
  static constexpr bool kBuf = T >= 7;
  __amdgpu_buffer_rsrc_t rs;
  gdouble *s;
  int base;  // element offset (global form) or byte offset (buffer form) of this lane
  __device__ Park(double *slot, int region) {
    constexpr int kRegion = NW * T * 4 * 64;  // doubles
    const int tid = opq(threadIdx.x);
    const int lane_off = (tid >> 6) * (T * 4 * 64) + (tid & 63);
    if constexpr (kBuf) {
      rs = __builtin_amdgcn_make_buffer_rsrc(slot + (size_t)region * kRegion, 0, kRegion * 8, kBufWord3);
      base = lane_off * 8;
    } else {
      s = gptr(slot);
      base = region * kRegion + lane_off;
    }
  }
  __device__ double get(int i, int r) const {
    if constexpr (kBuf) {
      const u2v v = __builtin_amdgcn_raw_buffer_load_b64(rs, base, (i * 4 + r) * 512, 0);
      return __longlong_as_double((long long)(((unsigned long long)v[1] << 32) | v[0]));
    } else {
      return s[base + (i * 4 + r) * 64];
    }
  }
  __device__ void put(int i, int r, double x) const {
    if constexpr (kBuf) {
      const unsigned long long u = (unsigned long long)__double_as_longlong(x);
      __builtin_amdgcn_raw_buffer_store_b64(u2v{(unsigned)u, (unsigned)(u >> 32)}, rs, base, (i * 4 + r) * 512, 0);
    } else {
      s[base + (i * 4 + r) * 64] = x;
    }
  }
  __device__ void put_all(const dbl4 (&x)[T]) const {
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) put(i, r, x[i][r]);
  }
  __device__ void get_all(dbl4 (&x)[T]) const {
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) x[i][r] = get(i, r);
  }
};

// Calls f(i, r, v) for every owned element (i, r), v the element of a matrix held either in
// registers (X) or, when PARKED, in the slot P.  Parked elements arrive in chunks of 8 with the
// next chunk in flight; a scheduling barrier per chunk keeps the compiler from issuing every
// chunk's loads up front (which would need the registers parking saves).
template <bool PARKED, int NW, int T, class F>
__device__ inline void each_elem(const Park<NW, T> &P, const dbl4 (&X)[T], const F &f) {
  if constexpr (!PARKED) {
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) f(i, r, X[i][r]);
  } else {
    constexpr int NE = 4 * T, CH = 8, NC = (NE + CH - 1) / CH;
    double buf[2][CH];
    auto fetch = [&](int g, double (&d)[CH]) {
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (g * CH + u < NE) d[u] = P.get((g * CH + u) >> 2, (g * CH + u) & 3);
    };
    fetch(0, buf[0]);
#pragma unroll
    for (int g = 0; g < NC; ++g) {
      if (g + 1 < NC) fetch(g + 1, buf[(g + 1) & 1]);
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (g * CH + u < NE) f((g * CH + u) >> 2, (g * CH + u) & 3, buf[g & 1][u]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// The alpha rule's selection work runs out of line: it executes once per matrix on one
// thread, and inlined its math-library code (roots, powers) would compete for registers with
// the register-held matrices.  The plain rule and the coefficients are cheap and inline.
__device__ __noinline__ void res_select(const double *theta, int alpha, double n1, double n2, double n3, int *m,
                                        int *s) {
  select_ms(theta, alpha, n1, n2, n3, m, s);
}
__device__ __noinline__ int res_proposal_ok(const double *theta, double n1, double n2, double n3, int m, int s) {
  return proposal_ok(theta, n1, n2, n3, m, s) ? 1 : 0;
}

// Copies the kernel's constants to LDS (the helpers above take pointers; a pointer into the
// kernel argument itself would force a private copy of the whole argument block).
template <int NW>
__device__ inline void res_init(const FusedArgs &a) {
  const double *src = reinterpret_cast<const double *>(&a.k);
  double *dst = reinterpret_cast<double *>(&sh_consts);
  for (int e = threadIdx.x; e < (int)(sizeof(Consts) / sizeof(double)); e += 64 * NW) dst[e] = src[e];
  __syncthreads();
}
template <int NT>
__device__ __noinline__ int res_mlp(double n1, double n2, double tr, double asym, int n) {
  return mlp_infer<NT>(n1, n2, tr, asym, n);
}

// Runs the method on matrix b of real order n (np = 16 T) with the resident scheme; SEL is the
// (m, s) rule, a compile-time parameter so that the plain rule's kernel carries none of the
// other rules' code and registers.  Waves
// beyond T own no column tile (IDLE): they run the same control flow, barriers and
// reductions without touching the matrices.  IDLE is a compile-time parameter so that the
// working waves update their register matrices unconditionally (a run-time guard around an
// update would keep the old and the new values alive together).
template <int NW, int SEL, int T, bool IDLE>
__device__ __attribute__((always_inline)) void run_res(const FusedArgs &a, int64_t b, int n, int nin, int cx, int64_t off, double *slot,
                        double *red) {
  double *L = res_lds<NW>();
  const int tid = threadIdx.x;
  const Lane ln;
  constexpr bool act = !IDLE;
  dbl4 X0[T];

  // ---- load A (real form of a complex input); finiteness, 1-norm; then X_p = 2^-sp A with sp
  // the plain rule's s (exact), into LDS: every power formed from here on stays in range. ----
  int bad = 0;
  double csum = 0.0;
  if constexpr (act) {
    cgdouble *Ag = gptr(a.A + off);
    const int lk = opq(ln.lk), c = opq(ln.col);
    const bool cin = c < n;
    const int cc = cin ? c : n - 1;
    if (!cx) {
      // real input: one buffer load per element at a 32-bit byte offset, issued back to back
      // with no per-element branch or 64-bit address; padding rows and columns lie past the
      // buffer's n^2 elements and read as zero
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(ufp(a.A + off), 0, n * n * 8, kBufWord3);
      const int lb = cin ? (lk * n + c) * 8 : n * n * 8;
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const u2v v = __builtin_amdgcn_raw_buffer_load_b64(rs, lb + (16 * i + 4 * r) * n * 8, 0, 0);
          X0[i][r] = __longlong_as_double((long long)(((unsigned long long)v[1] << 32) | v[0]));
        }
    } else {
      // complex input (real form): every lane loads (indices clamped into the matrix) and
      // zeroes what lies outside
      const int ci = cc < nin ? cc : cc - nin;
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * i + 4 * r + lk;
          const int rr = row < n ? row : n - 1;
          const int ri = rr < nin ? rr : rr - nin;
          const bool im = (rr < nin) != (cc < nin);
          X0[i][r] = Ag[2 * ((size_t)ri * nin + ci) + (im ? 1 : 0)];
        }
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * i + 4 * r + lk;
          double x = X0[i][r];
          if ((row < nin) && !(cc < nin)) x = -x;  // -Y block of the real form
          X0[i][r] = (row < n && cin) ? x : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        bad |= !isfinite(X0[i][r]);
        csum += fabs(X0[i][r]);
      }
    if (cx) {
      // complex input: the 1-norm of A itself, sum_i |z_ij| over the columns of the X block
      // (which holds the real parts; the imaginary parts are read beside them)
      csum = 0.0;
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * i + 4 * r + lk;
          if (row < nin && c < nin) csum += hypot(X0[i][r], Ag[2 * ((size_t)row * nin + c) + 1]);
        }
    }
    csum += __shfl_xor(csum, 16);
    csum += __shfl_xor(csum, 32);
  }
  bad = ufi(__syncthreads_or(bad));
  const double eta = wg_max<NW>(csum, red);
  // a 1-norm that overflows (finite entries) is refused like a non-finite entry
  if (bad || !(eta <= __DBL_MAX__)) {
    double *E = a.E ? a.E + off : nullptr;
    if (E) for (int e = tid; e < nin * nin * (cx ? 2 : 1); e += 64 * NW) E[e] = __builtin_nan("");
    if (tid == 0) {
      a.m_out[b] = -1; a.s_out[b] = -1;
      if (a.status) a.status[b] = EXPM_E_NONFINITE;
    }
    __syncthreads();
    return;
  }

  // plain rule, evaluated by every lane on the (uniform) norm: integer work on bit patterns
  int m_rule, s_plain;
  select_ms(sh_consts.theta, 0, eta, -1.0, -1.0, &m_rule, &s_plain);
  m_rule = ufi(m_rule);
  s_plain = ufi(s_plain);
  if constexpr (act) {
    if (s_plain > 0) {
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) X0[i][r] = ldexp(X0[i][r], -s_plain);
    }
    to_lds<T>(L, ln, X0);
  }
  __syncthreads();

  // The rest of the method.  Under the plain rule the degree is known here, so it runs once
  // per degree, each with the degree as a compile-time constant and its own register matrices
  // (their registers are allotted per degree, so one degree's pressure does not spill
  // another's); under the other rules, once with the degree chosen at run time.
  auto rest = [&](auto Mc) __attribute__((always_inline)) {
    constexpr int MC = decltype(Mc)::value;
    const int m_plain = MC == 0 ? m_rule : MC == 2 ? (m_rule <= 1 ? 1 : 2) : MC;
    int m = m_plain, s = s_plain;
    dbl4 X1[T], X2[T], AC[T];

    // ---- A^2 (X1), the norms the selector needs, then A^3 (X2) at most once ----
    if (m_plain >= 2 && !IDLE) {
      zero<T>(X1);
      rgemm_reg<T>(L, ln, X0, X1);
    }
    double n2 = -1.0, n3 = -1.0;
    bool need3 = false;
    int mq = 0, sq = 0;
    if (SEL == EXPM_SEL_ALPHA && m_plain >= 2) {
      n2 = unscale_norm(norm1<NW, T>(X1, act, red), 2, s_plain);
      need3 = m_plain >= 12;
    } else if (SEL == EXPM_SEL_LEARNED && m_plain >= 2) {
      n2 = unscale_norm(norm1<NW, T>(X1, act, red), 2, s_plain);
      double tr = 0.0, asy = 0.0;
      if constexpr (act) {
        constexpr int S = Res<T>::S;
        const Own<T> o(ln);
        const int lk = opq(ln.lk), col = opq(ln.col);
  #pragma unroll
        for (int i = 0; i < T; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            tr += o.delta(i, r) * X0[i][r];
            const int row = 16 * i + 4 * r + lk;  // A^T element from the resident A
            asy += fabs(X0[i][r] - L[col * S + (row ^ swz(col))]);
          }
        asy += __shfl_xor(asy, 16);
        asy += __shfl_xor(asy, 32);
      }
      tr = ldexp(wg_sum<NW>(act ? tr : 0.0, red), s_plain);  // of A, not of X_p
      asy = ldexp(wg_max<NW>(act ? asy : 0.0, red), s_plain);
      const int cls = ufi(res_mlp<64 * NW>(eta, n2, tr, asy, n));
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

    // From here on A is read elementwise only.  At np >= 96 on 8 waves, B_3 of the degree-18
    // stage waits in the workgroup's HBM slot (region 1) and B_1 of the degree-12 stage in
    // region 0; under the alpha and learned rules (one body for every degree) so does A
    // (region 0), so that no phase holds more than two register matrices besides the
    // accumulator.  Under the plain rule each degree has registers of its own and A stays in
    // X0 (B_1 of the degree-12 stage is still parked: held in registers through the product
    // B_4 B_4 it was partly spilled and reloaded one element at a time).
    constexpr bool kPark = NW == 8 && T >= kResParkT;
    constexpr bool kParkA = kPark && MC == 0;
    constexpr bool kParkB1 = kPark && (MC == 0 || MC == 12);
    const Park<NW, T> P0(slot, 0), P1(slot, 1);
    if constexpr (kParkA) {
      if constexpr (act) P0.put_all(X0);
    }

    if (need3) {
      if constexpr (act) {
        zero<T>(X2);
        rgemm_reg<T>(L, ln, X1, X2);
      }
      if (SEL == EXPM_SEL_ALPHA) {
        n3 = unscale_norm(norm1<NW, T>(X2, act, red), 3, s_plain);
        if (tid == 0) res_select(sh_consts.theta, 1, eta, n2, n3, &sh_ms[0], &sh_ms[1]);
        __syncthreads();
        m = ufi(sh_ms[0]); s = ufi(sh_ms[1]);
      } else if (SEL == EXPM_SEL_LEARNED && mq >= 12) {
        n3 = unscale_norm(norm1<NW, T>(X2, act, red), 3, s_plain);
        const bool ok = ufi(res_proposal_ok(sh_consts.theta, eta, n2, n3, mq, sq)) != 0;
        if (ok) { m = mq; s = sq; }
        if (tid == 0) atomicAdd(&g_learned_counts[ok ? 0 : 1], 1ull);
      }
    } else if (SEL == EXPM_SEL_ALPHA && m_plain >= 2) {
      // plain m < 12 implies s = 0 and an alpha choice of m <= 8: A^3 is never needed here
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
    // The powers held so far are those of X_p = 2^-sp A; the other rules may have chosen s != sp:
    // X = 2^(sp - s) X_p, so X^k = 2^(k (sp - s)) X_p^k, rescaled exactly here (A itself when its
    // elements are read below, through x1).
    const int dsc = s_plain - s;
    if (SEL != EXPM_SEL_PLAIN && dsc != 0 && act) {
      if (m_plain >= 2) {
  #pragma unroll
        for (int i = 0; i < T; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) X1[i][r] = ldexp(X1[i][r], 2 * dsc);
      }
      if (need3) {
  #pragma unroll
        for (int i = 0; i < T; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) X2[i][r] = ldexp(X2[i][r], 3 * dsc);
      }
    }
    auto x1 = [&](double v) {
      if constexpr (SEL == EXPM_SEL_PLAIN) return v;
      else return ldexp(v, dsc);
    };
    // coefficients of degree M (the scaling is in the matrices), computed by every lane from the
    // constants in LDS and moved to scalar registers
    auto coefs = [&](auto deg, double *c, int count) {
      double t[24];
      make_coefs(sh_consts, decltype(deg)::value, 0, t);
      for (int j = 0; j < count; ++j) c[j] = uni(t[j]);
    };

    // ---- T_m(X) into AC.  Products of polynomials in A commute, so each product is
    // ordered to make the operand that is not at hand in registers the resident one.  Every
    // elementwise pass writes its results in place of inputs that die with it, so no pass
    // holds more register matrices than the product that follows it. ----
    if (m <= 2) {
      double c[2];
      if (m == 2) coefs(std::integral_constant<int, 2>(), c, 2);
      else { coefs(std::integral_constant<int, 1>(), c, 1); c[1] = 0.0; }
      if constexpr (act) {
        const Own<T> o(ln);
        each_elem<kParkA>(P0, X0, [&](int i, int r, double a1r) {
          const double a1 = x1(a1r);
          X1[i][r] = o.delta(i, r) + c[0] * a1 + (m == 2 ? c[1] * X1[i][r] : 0.0);
        });
  #pragma unroll
        for (int i = 0; i < T; ++i) AC[i] = X1[i];
      }
    } else if (m == 4) {
      // T = I + c0 A + c1 V, V = A^2 W = (c3 A + c4 A^2) A^2 + c2 A^2
      double c[5];
      coefs(std::integral_constant<int, 4>(), c, 5);
      __syncthreads();
      if constexpr (act) {
        const Own<T> o(ln);
        each_elem<kParkA>(P0, X0, [&](int i, int r, double a1r) {
          const double a1 = x1(a1r); L[o.at(i, r)] = c[3] * a1 + c[4] * X1[i][r]; });
      }
      __syncthreads();
      if constexpr (act) {
        zero<T>(AC);
        rgemm_reg<T>(L, ln, X1, AC);
        const Own<T> o(ln);
        each_elem<kParkA>(P0, X0, [&](int i, int r, double a1r) {
          const double a1 = x1(a1r);
          AC[i][r] = o.delta(i, r) + c[0] * a1 + c[1] * (AC[i][r] + c[2] * X1[i][r]);
        });
      }
    } else if (m == 8) {
      // V = W1 A^2 (W1 = c0 A + c1 A^2); A_4 = c2 V; Lm = c3 A^2 + A_4;
      // Rm = c4 I + c5 A + c6 A^2 + c7 A_4; T = Lm Rm + c8 I + c9 A + c10 A^2   (eq. Algorithm83eA)
      double c[11];
      coefs(std::integral_constant<int, 8>(), c, 11);
      __syncthreads();
      if constexpr (act) {
        const Own<T> o(ln);
        each_elem<kParkA>(P0, X0, [&](int i, int r, double a1r) {
          const double a1 = x1(a1r); L[o.at(i, r)] = c[0] * a1 + c[1] * X1[i][r]; });
      }
      __syncthreads();
      if constexpr (act) {
        zero<T>(AC);
        rgemm_reg<T>(L, ln, X1, AC);  // V
      }
      __syncthreads();
      if constexpr (act) {
        const Own<T> o(ln);
        each_elem<kParkA>(P0, X0, [&](int i, int r, double a1r) {
          const double a1 = x1(a1r);
          const double d = o.delta(i, r), a2 = X1[i][r], a4 = c[2] * AC[i][r];
          L[o.at(i, r)] = c[3] * a2 + a4;                                 // Lm
          X1[i][r] = c[4] * d + c[5] * a1 + c[6] * a2 + c[7] * a4;         // Rm
          AC[i][r] = c[8] * d + c[9] * a1 + c[10] * a2;
        });
      }
      __syncthreads();
      if constexpr (act) rgemm_reg<T>(L, ln, X1, AC);
    } else if (m == 12) {
      // B_j over (I, A, A^2, A^3); A_6 = B_3 + B_4^2; T = B_1 + (B_2 + A_6) A_6   (eq. poly12)
      double k[16];
      coefs(std::integral_constant<int, 12>(), k, 16);
      __syncthreads();
      if constexpr (act) {
        const Own<T> o(ln);
        each_elem<kParkA>(P0, X0, [&](int i, int r, double a1r) {
          const double a1 = x1(a1r);
          const double d = o.delta(i, r), a2 = X1[i][r], a3 = X2[i][r];
          L[o.at(i, r)] = k[12] * d + k[13] * a1 + k[14] * a2 + k[15] * a3;  // B_4
          const double b1 = k[0] * d + k[1] * a1 + k[2] * a2 + k[3] * a3;
          if constexpr (kParkB1) P0.put(i, r, b1);
          else X0[i][r] = b1;
          X1[i][r] = k[4] * d + k[5] * a1 + k[6] * a2 + k[7] * a3;   // B_2
          X2[i][r] = k[8] * d + k[9] * a1 + k[10] * a2 + k[11] * a3;  // B_3
        });
      }
      __syncthreads();
      if constexpr (act) {
        rgemm_sq<T>(L, ln, X2);  // A_6 = B_3 + B_4 B_4
  #pragma unroll
        for (int i = 0; i < T; ++i) X1[i] += X2[i];  // Y = B_2 + A_6
      }
      __syncthreads();
      if constexpr (act) {
        to_lds<T>(L, ln, X1);
        if constexpr (kParkB1) P0.get_all(X1);  // B_1
        else {
  #pragma unroll
          for (int i = 0; i < T; ++i) X1[i] = X0[i];
        }
      }
      __syncthreads();
      if constexpr (act) {
        rgemm_reg<T>(L, ln, X2, X1);  // T = B_1 + Y A_6
  #pragma unroll
        for (int i = 0; i < T; ++i) AC[i] = X1[i];
      }
    } else {
      // m == 18: A^6 = A^3 A^3; B_1 over (I, A, A^2, A^3), B_2..B_5 over (I, A, A^2, A^3, A^6);
      // A_9 = B_1 B_5 + B_4; T = B_2 + (B_3 + A_9) A_9   (eq. poly.18)
      double k[24];
      coefs(std::integral_constant<int, 18>(), k, 24);
      __syncthreads();
      if constexpr (act) to_lds<T>(L, ln, X2);
      __syncthreads();
      if constexpr (act) {
        zero<T>(AC);
        rgemm_sq<T>(L, ln, AC);  // A^6
      }
      __syncthreads();
      if constexpr (act) {
        const Own<T> o(ln);
        each_elem<kParkA>(P0, X0, [&](int i, int r, double a1r) {
          const double a1 = x1(a1r);
          const double d = o.delta(i, r), a2 = X1[i][r], a3 = L[o.at(i, r)], a6 = AC[i][r];
          L[o.at(i, r)] = k[0] * d + k[1] * a1 + k[2] * a2 + k[3] * a3;  // B_1
          const double b2 = k[4] * d + k[5] * a1 + k[6] * a2 + k[7] * a3 + k[8] * a6;
          const double b3 = k[9] * d + k[10] * a1 + k[11] * a2 + k[12] * a3 + k[13] * a6;
          X0[i][r] = b2;
          if constexpr (kPark) P1.put(i, r, b3);
          else X2[i][r] = b3;
          AC[i][r] = k[14] * d + k[15] * a1 + k[16] * a2 + k[17] * a3 + k[18] * a6;  // B_4
          X1[i][r] = k[19] * d + k[20] * a1 + k[21] * a2 + k[22] * a3 + k[23] * a6;  // B_5
        });
      }
      __syncthreads();
      if constexpr (act) {
        rgemm_reg<T>(L, ln, X1, AC);  // A_9 = B_1 B_5 + B_4
      }
      __syncthreads();
      if constexpr (act) {  // Y = B_3 + A_9 becomes the resident matrix
        const Own<T> o(ln);
        each_elem<kPark>(P1, X2, [&](int i, int r, double b3) { L[o.at(i, r)] = b3 + AC[i][r]; });
      }
      __syncthreads();
      if constexpr (act) {
        rgemm_reg<T>(L, ln, AC, X0);  // T = B_2 + Y A_9
  #pragma unroll
        for (int i = 0; i < T; ++i) AC[i] = X0[i];
      }
    }

    // ---- s squarings: the resident matrix is both operands ----
    for (int q = 0; q < s; ++q) {
      __syncthreads();
      if constexpr (act) to_lds<T>(L, ln, AC);
      __syncthreads();
      if constexpr (act) {
        zero<T>(AC);
        rgemm_sq<T>(L, ln, AC);
      }
    }

    // ---- e^A ----
    if constexpr (act) {
      gdouble *E = gptr(a.E + off);
      const int lk = opq(ln.lk), col = opq(ln.col);
      if (!cx) {
        // real output: row-major through a buffer over the n^2 elements; stores of padding
        // rows and columns fall past its end and are dropped
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(ufp(a.E + off), 0, n * n * 8, kBufWord3);
        const int lb = col < n ? (lk * n + col) * 8 : n * n * 8;
  #pragma unroll
        for (int i = 0; i < T; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            const unsigned long long u = (unsigned long long)__double_as_longlong(AC[i][r]);
            __builtin_amdgcn_raw_buffer_store_b64(u2v{(unsigned)u, (unsigned)(u >> 32)}, rs, lb + (16 * i + 4 * r) * n * 8, 0, 0);
          }
      } else {
  #pragma unroll
        for (int i = 0; i < T; ++i)
  #pragma unroll
          for (int r = 0; r < 4; ++r) put_dst(E, n, nin, cx, 16 * i + 4 * r + lk, col, AC[i][r]);
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

template <int NW, int SEL>
__device__ __attribute__((always_inline)) void run_res_dispatch(const FusedArgs &a, int64_t b, double *slot, double *red) {
  const int tid = threadIdx.x;
  // the order and the offset both depend on b only: both loads are issued before either is used
  const int32_t nraw = a.ns ? ((__attribute__((address_space(1))) const int32_t *)a.ns)[b] : a.n_uniform;
  const int64_t oraw = a.offs ? ((__attribute__((address_space(1))) const int64_t *)a.offs)[b] : 0;
  const int nin = ufi(nraw);
  const int cx = a.cplx;
  const int n = cx ? 2 * nin : nin;
  const int64_t off = (a.offs ? ufl(oraw) : b * (int64_t)nin * nin) * (cx ? 2 : 1);
  const int t = (n + 15) >> 4;
  const bool fits = NW == 8 ? (t > kRes6T && t <= kResT) : (t >= 1 && t < kSplitT);
  if (nin < 1 || n > a.np_max || !fits) {  // invalid order, or routed to the wrong variant
    if (tid == 0) {
      a.m_out[b] = -1; a.s_out[b] = -1;
      if (a.status) a.status[b] = (nin < 1 || n > a.np_max) ? EXPM_E_INVALID_ARG : EXPM_E_UNSUPPORTED;
    }
    return;
  }
  const bool idle = (int)(threadIdx.x >> 6) >= t;  // wave-uniform
  if constexpr (NW == 8) {
    if (t == 7) {
      idle ? run_res<8, SEL, 7, true>(a, b, n, nin, cx, off, slot, red)
           : run_res<8, SEL, 7, false>(a, b, n, nin, cx, off, slot, red);
    } else {
      run_res<8, SEL, 8, false>(a, b, n, nin, cx, off, slot, red);
    }
  } else {
    switch (t) {
      case 1: idle ? run_res<4, SEL, 1, true>(a, b, n, nin, cx, off, slot, red)
                   : run_res<4, SEL, 1, false>(a, b, n, nin, cx, off, slot, red); break;
      case 2: idle ? run_res<4, SEL, 2, true>(a, b, n, nin, cx, off, slot, red)
                   : run_res<4, SEL, 2, false>(a, b, n, nin, cx, off, slot, red); break;
      case 3: idle ? run_res<4, SEL, 3, true>(a, b, n, nin, cx, off, slot, red)
                   : run_res<4, SEL, 3, false>(a, b, n, nin, cx, off, slot, red); break;
      default: run_res<4, SEL, 4, false>(a, b, n, nin, cx, off, slot, red); break;
    }
  }
}

}  // namespace
}  // namespace expm
