// Workgroup FP64 MFMA tile engine: acc(BM x BN) = P[m0 : m0+BM, 0:K] * Q[0:K, n0 : n0+BN]
// for row-major operands in device memory.
//
// Pipeline.  K is walked in panels of KP = 16.  Panels travel from global memory straight
// into LDS with global_load_lds_dwordx4 (gfx950: each lane moves 16 bytes to
// LDS base + 16 * lane, no registers involved), into a ring of three LDS stages.  Panel
// kp + 2 is in flight while panel kp is multiplied, and one workgroup barrier per panel both
// publishes panel kp and retires the stage that panel kp + 2 overwrites.  The ring is unrolled
// by three so every stage is a distinct __shared__ array: the compiler then sees that the
// fragment reads of one stage never alias the in-flight writes of another.
//
// LDS layouts (16-byte chunks):
//   P stage: BM rows x 8 chunks (128 B per row).  Chunk c of row r sits in slot
//            c ^ ((r >> 1) & 7): an A fragment reads 16 rows of one column, and the swizzle
//            puts those 16 reads in 16 distinct bank groups.
//   Q stage: 16 rows x BN/2 chunks.  When BN/2 is a multiple of 16, odd rows swap 128-byte
//            halves (slot c ^ 8), so the four 16-lane groups of a B fragment use both bank
//            halves.
//
// MFMA operand layouts (gfx950): 16x16x4 f64 and f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; 16x16x32 bf16: lane l supplies 8 elements of row l % 16 of A and of
// column l % 16 of B, the same k for both (lane group l / 16 covers 8 of the 32).
// Accumulator register r of lane l holds D[4 r + l / 16][l % 16] for f64,
// D[4 (l / 16) + r][l % 16] for the f32-accumulating forms.
#pragma once
#include <hip/hip_runtime.h>

namespace expm {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const dv2 cgdv2;
typedef short shr4 __attribute__((ext_vector_type(4)));

// Arithmetic of the products: PREC_F64 (v_mfma_f64_16x16x4, tile_gemm on FP64 operands),
// PREC_F32 (operands rounded to FP32, v_mfma_f32_16x16x4, FP32 accumulation), PREC_BF16X3
// (each FP64 operand split into three bfloat16 terms hi + mid + lo; the six products hi*hi,
// hi*mid, mid*hi, hi*lo, lo*hi, mid*mid by v_mfma_f32_16x16x32_bf16, FP32 accumulation); the
// two reduced forms run tile_gemm_lp on operand planes made once per product.
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };
template <int PREC> struct AccOf { typedef dbl4 T; };
template <> struct AccOf<PREC_F32> { typedef flt4 T; };
template <> struct AccOf<PREC_BF16X3> { typedef flt4 T; };

// Round-to-nearest-even bfloat16 of a float (the 16 high bits).
__device__ inline short bf16_rne(float f) {
  const unsigned u = __float_as_uint(f);
  return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline double bf16_to_double(short h) { return (double)__uint_as_float(((unsigned)(unsigned short)h) << 16); }

// x = hi + mid + lo + O(2^-24 |x|), each term a bfloat16; the remainders are exact in FP64.
__device__ inline void split3(double x, short &hi, short &mid, short &lo) {
  hi = bf16_rne((float)x);
  const double r1 = x - bf16_to_double(hi);
  mid = bf16_rne((float)r1);
  const double r2 = r1 - bf16_to_double(mid);
  lo = bf16_rne((float)r2);
}
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const double cgdouble;
typedef __attribute__((address_space(1))) const void *gvoidp;
typedef __attribute__((address_space(3))) void *lvoidp;
__device__ inline gdouble *gptr(double *p) { return (gdouble *)p; }
__device__ inline cgdouble *gptr(const double *p) { return (cgdouble *)p; }

constexpr int kKP = 16;

// NW waves; chunk BM x BN; waves in a WR x WC grid, each owning BR x BC 16x16 tiles.
template <int NW_, int BM_, int BN_, int WR_, int WC_, int BR_, int BC_>
struct TileShape {
  static constexpr int NW = NW_, BM = BM_, BN = BN_, WR = WR_, WC = WC_, BR = BR_, BC = BC_;
  static constexpr int TPW = BR * BC;
  static constexpr int P_STAGE = BM * kKP;          // doubles
  static constexpr int Q_STAGE = kKP * BN;          // doubles
  static constexpr int P_INSTR = BM * kKP / 128;    // wave instructions (64 x 16 B) per panel
  static constexpr int Q_INSTR = kKP * BN / 128;
  static constexpr int INSTR = P_INSTR + Q_INSTR;
  static constexpr int MIN_INSTR_PER_WAVE = INSTR / NW;  // waves issue floor or ceil of this
  static constexpr bool Q_SWZ = ((BN / 2) % 16) == 0;
  static_assert(BM % 16 == 0 && BN % 16 == 0, "tile multiple of 16");
  static_assert(WR * WC <= NW, "wave grid");
  static_assert(P_INSTR * 128 == BM * kKP && Q_INSTR * 128 == kKP * BN, "whole wave loads");
};

template <class S>
struct TileLds {
  double p[3][S::P_STAGE];
  double q[3][S::Q_STAGE];
};

// Workgroup barrier for the panel ring.  __syncthreads() (and even an LDS-scoped fence)
// makes the compiler wait for every outstanding vector-memory operation, including the
// in-flight LDS-DMA panels.  Here the caller waits for exactly the panel it needs
// (wait_vmcnt), this wave's LDS reads are drained (lgkmcnt(0)), and s_barrier publishes both;
// the memory clobber keeps the compiler from moving LDS accesses across it.
__device__ inline void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// s_waitcnt with vmcnt <= n and the other counters unconstrained (gfx9 encoding).
template <int n>
__device__ inline void wait_vmcnt() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Issues the direct-to-LDS loads of panel kp (columns k0 .. k0+15 of P's rows m0.., rows
// k0 .. k0+15 of Q's columns n0..) into stage buffers lp, lq.  Rows of P at or beyond M,
// columns of Q at or beyond N and k at or beyond K are clamped to valid addresses: those LDS
// entries only feed accumulators that are never stored, or are skipped (k tail).
template <class S>
__device__ inline void issue_panel(cgdouble *P, int ldp, cgdouble *Q, int ldq, int M, int N, int K,
                                   int m0, int n0, int k0, double *lp, double *lq) {
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));  // opaque: addresses are rebuilt per panel, not held live
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < (S::INSTR + S::NW - 1) / S::NW; ++i) {
    const int ins = i * S::NW + wave;  // wave-uniform instruction index
    if (ins < S::P_INSTR) {
      const int j = ins * 64 + lane;   // chunk index in the P stage
      const int r = j >> 3, slot = j & 7;
      const int c = slot ^ ((r >> 1) & 7);
      int k = k0 + 2 * c;
      if (k >= K) k = 0;
      const int row = (m0 + r < M) ? m0 + r : 0;
      __builtin_amdgcn_global_load_lds((gvoidp)(P + (size_t)row * ldp + k),
                                       (lvoidp)(lp + ins * 128), 16, 0, 0);
    } else if (ins < S::INSTR) {
      const int qi = ins - S::P_INSTR;
      const int j = qi * 64 + lane;    // chunk index in the Q stage
      const int r = j / (S::BN / 2), slot = j % (S::BN / 2);
      const int c = S::Q_SWZ ? (slot ^ ((r & 1) << 3)) : slot;
      int k = k0 + r;
      if (k >= K) k = 0;
      const int col = (n0 + 2 * c < N) ? n0 + 2 * c : 0;
      __builtin_amdgcn_global_load_lds((gvoidp)(Q + (size_t)k * ldq + col),
                                       (lvoidp)(lq + qi * 128), 16, 0, 0);
    }
  }
}

// Multiplies the panel held in (lp, lq) into acc: kend = 16, or fewer for a K tail (a tail
// only occurs with PREC_F64 on orders that are odd multiples of 16).
template <class S, int PREC, bool NEG = false>
__device__ inline void mma_panel(const double *lp, const double *lq, int wr_row, int wc_col, int kend,
                                 typename AccOf<PREC>::T (&acc)[S::TPW]) {
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const int lr = lane & 15, lk = lane >> 4;
  static_assert(PREC == PREC_F64, "reduced precisions run tile_gemm_lp on operand planes");
  {
    // Blocks of 9+ tiles keep only two k steps of fragments in flight (register budget).
    constexpr int KU = S::TPW >= 9 ? 2 : 4;
#pragma unroll KU
    for (int kk = 0; kk < kKP; kk += 4) {
      if (kk < kend) {
        const int k = kk + lk;
        double a[S::BR], b[S::BC];
#pragma unroll
        for (int i = 0; i < S::BR; ++i) {
          const int r = wr_row + i * 16 + lr;  // row within the chunk
          const int slot = (k >> 1) ^ ((r >> 1) & 7);
          a[i] = NEG ? -lp[r * kKP + 2 * slot + (k & 1)] : lp[r * kKP + 2 * slot + (k & 1)];
        }
#pragma unroll
        for (int j = 0; j < S::BC; ++j) {
          const int col = wc_col + j * 16 + lr;  // column within the chunk
          const int slot = S::Q_SWZ ? ((col >> 1) ^ ((k & 1) << 3)) : (col >> 1);
          b[j] = lq[k * S::BN + 2 * slot + (col & 1)];
        }
#pragma unroll
        for (int i = 0; i < S::BR; ++i)
#pragma unroll
          for (int j = 0; j < S::BC; ++j) {
            acc[i * S::BC + j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i * S::BC + j], 0, 0, 0);
          }
      }
    }
  }
}

// Full K loop for one chunk.  `active`: this wave owns a block inside the matrix.  The caller
// must have passed a workgroup barrier since the stages were last read.  On return every
// panel load has completed, but other waves may still be reading the last stage.  acc = P Q,
// or with ACC acc += P Q, or with NEG acc -= P Q (the four real products of a complex one).
template <class S, int PREC = PREC_F64, bool ACC = false, bool NEG = false>
__device__ inline void tile_gemm(cgdouble *P, int ldp, cgdouble *Q, int ldq, int M, int N, int K,
                                 int m0, int n0, TileLds<S> &L, bool active, int wr_row, int wc_col,
                                 typename AccOf<PREC>::T (&acc)[S::TPW]) {
  typedef typename AccOf<PREC>::T AT;
  if constexpr (!ACC) {
#pragma unroll
    for (int i = 0; i < S::TPW; ++i) acc[i] = AT{0, 0, 0, 0};
  }
  const int npan = (K + kKP - 1) / kKP;
  issue_panel<S>(P, ldp, Q, ldq, M, N, K, m0, n0, 0, L.p[0], L.q[0]);
  if (npan > 1) issue_panel<S>(P, ldp, Q, ldq, M, N, K, m0, n0, kKP, L.p[1], L.q[1]);
  // One step: wait for panel kp, publish it, refill the stage freed by panel kp - 1, multiply.
  auto step = [&](int kp, double *lp, double *lq, double *np_p, double *np_q) {
    if (kp + 1 < npan) wait_vmcnt<S::MIN_INSTR_PER_WAVE>(); else wait_vmcnt<0>();
    lds_barrier();
    if (kp + 2 < npan) issue_panel<S>(P, ldp, Q, ldq, M, N, K, m0, n0, (kp + 2) * kKP, np_p, np_q);
    const int kend = (K - kp * kKP) < kKP ? (K - kp * kKP) : kKP;
    if (active) mma_panel<S, PREC, NEG>(lp, lq, wr_row, wc_col, kend, acc);
  };
  for (int kp = 0; kp < npan; kp += 3) {
    step(kp, L.p[0], L.q[0], L.p[2], L.q[2]);
    if (kp + 1 < npan) step(kp + 1, L.p[1], L.q[1], L.p[0], L.q[0]);
    if (kp + 2 < npan) step(kp + 2, L.p[2], L.q[2], L.p[1], L.q[1]);
  }
}

// ---------------------------------------------------------------------------------------
// Reduced-precision tile engine on operand planes made once per product (lg_planes_kernel):
// PREC_BF16X3: three bfloat16 planes hi, mid, lo per operand (the successive roundings of
// split3), six products per k block by v_mfma_f32_16x16x32_bf16 (gfx950: K = 32 per
// instruction, 8 bfloat16 per lane and operand); PREC_F32: one float plane per operand,
// v_mfma_f32_16x16x4_f32.  FP32 accumulation in both.  The left operand's planes are
// row-major (P[row][k]); the right operand's are stored transposed (Q^T[col][k]), so both
// fragments are 16-byte LDS reads along k.  K is walked in panels of 32 through a ring of
// three LDS stages filled by direct-to-LDS loads, as in tile_gemm.  The k order inside an
// MFMA block only permutes the terms of each dot product: lane group g supplies the same k
// values (8 g .. 8 g + 7 of the panel) to both operands.
//
// LDS layout per plane stage: rows of 32 elements (64 B bf16 / 128 B float) in 16-byte
// chunks; chunk c of row r sits in slot c ^ ((r >> 2) & 3) (bf16) or c ^ ((r >> 1) & 7)
// (float), so the 16 rows of a fragment read land in distinct banks.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shr8 __attribute__((ext_vector_type(8)));
typedef float flt8 __attribute__((ext_vector_type(8)));
template <int PREC> struct LpOf;
template <> struct LpOf<PREC_BF16X3> {
  typedef short E;
  static constexpr int PL = 3, EPC = 8, CPR = 4;
  __device__ static int swz(int r) { return (r >> 2) & 3; }
};
template <> struct LpOf<PREC_F32> {
  typedef float E;
  static constexpr int PL = 1, EPC = 4, CPR = 8;
  __device__ static int swz(int r) { return (r >> 1) & 7; }
};
constexpr int kLpKP = 32;

template <class S, int PREC>
struct LpLds {
  typedef typename LpOf<PREC>::E E;
  static constexpr int PST = LpOf<PREC>::PL * S::BM * kLpKP;  // elements per P stage
  static constexpr int QST = LpOf<PREC>::PL * S::BN * kLpKP;  // elements per Q stage
  static constexpr int P_INSTR = LpOf<PREC>::PL * S::BM * LpOf<PREC>::CPR / 64;
  static constexpr int Q_INSTR = LpOf<PREC>::PL * S::BN * LpOf<PREC>::CPR / 64;
  static constexpr int INSTR = P_INSTR + Q_INSTR;
  static_assert(P_INSTR * 64 == LpOf<PREC>::PL * S::BM * LpOf<PREC>::CPR, "whole wave loads");
  static_assert(Q_INSTR * 64 == LpOf<PREC>::PL * S::BN * LpOf<PREC>::CPR, "whole wave loads");
  static_assert(INSTR % S::NW == 0, "every wave issues the same number of loads");
  E p[3][PST];
  E q[3][QST];
};

// Direct-to-LDS loads of panel k0 .. k0 + 31: P planes rows m0.., Q^T planes rows n0.. (rows
// beyond M or N clamped to row 0: they only feed accumulators that are never stored).
template <class S, int PREC>
__device__ inline void issue_panel_lp(const typename LpOf<PREC>::E *P, const typename LpOf<PREC>::E *QT,
                                      size_t pstride, int ld, int M, int N, int m0, int n0, int k0,
                                      typename LpOf<PREC>::E *lp, typename LpOf<PREC>::E *lq) {
  typedef LpOf<PREC> O;
  typedef LpLds<S, PREC> LL;
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < LL::INSTR / S::NW; ++i) {
    const int ins = i * S::NW + wave;  // wave-uniform
    const bool isq = ins >= LL::P_INSTR;
    const int qi = isq ? ins - LL::P_INSTR : ins;
    const int j = qi * 64 + lane;  // chunk in the stage: plane, row, slot
    const int rows = isq ? S::BN : S::BM;
    const int pl = j / (rows * O::CPR), rem = j - pl * rows * O::CPR;
    const int r = rem / O::CPR, slot = rem - r * O::CPR;
    const int c = slot ^ O::swz(r);
    const int lim = isq ? N : M, o0 = isq ? n0 : m0;
    const int row = (o0 + r < lim) ? o0 + r : 0;
    const typename O::E *src = (isq ? QT : P) + (size_t)pl * pstride + (size_t)row * ld + k0 + c * O::EPC;
    typename O::E *dst = (isq ? lq : lp) + qi * 64 * O::EPC;
    __builtin_amdgcn_global_load_lds((gvoidp)src, (lvoidp)dst, 16, 0, 0);
  }
}

template <class S, int PREC>
__device__ inline void mma_panel_lp(const typename LpOf<PREC>::E *lp, const typename LpOf<PREC>::E *lq, int wr_row,
                                    int wc_col, flt4 (&acc)[S::TPW]) {
  typedef LpOf<PREC> O;
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const int lr = lane & 15, g = lane >> 4;
  if constexpr (PREC == PREC_BF16X3) {
    shr8 a[3][S::BR], b[3][S::BC];
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int r = wr_row + i * 16 + lr;
#pragma unroll
      for (int pl = 0; pl < 3; ++pl)
        a[pl][i] = *(const shr8 *)(lp + (pl * S::BM + r) * kLpKP + (g ^ O::swz(r)) * O::EPC);
    }
#pragma unroll
    for (int j = 0; j < S::BC; ++j) {
      const int cc = wc_col + j * 16 + lr;
#pragma unroll
      for (int pl = 0; pl < 3; ++pl)
        b[pl][j] = *(const shr8 *)(lq + (pl * S::BN + cc) * kLpKP + (g ^ O::swz(cc)) * O::EPC);
    }
    auto mf = [](const shr8 &x, const shr8 &y, flt4 c) {
      return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, x), __builtin_bit_cast(bf16x8, y), c,
                                                     0, 0, 0);
    };
#pragma unroll
    for (int i = 0; i < S::BR; ++i)
#pragma unroll
      for (int j = 0; j < S::BC; ++j) {
        flt4 c = acc[i * S::BC + j];
        // smallest terms first: mid*mid, hi*lo, lo*hi, hi*mid, mid*hi, hi*hi
        c = mf(a[1][i], b[1][j], c);
        c = mf(a[0][i], b[2][j], c);
        c = mf(a[2][i], b[0][j], c);
        c = mf(a[0][i], b[1][j], c);
        c = mf(a[1][i], b[0][j], c);
        c = mf(a[0][i], b[0][j], c);
        acc[i * S::BC + j] = c;
      }
  } else {
    flt8 a[S::BR], b[S::BC];
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int r = wr_row + i * 16 + lr;
      const float *row = lp + r * kLpKP;
      const flt4 lo = *(const flt4 *)(row + ((2 * g) ^ O::swz(r)) * O::EPC);
      const flt4 hi = *(const flt4 *)(row + ((2 * g + 1) ^ O::swz(r)) * O::EPC);
      a[i] = flt8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
#pragma unroll
    for (int j = 0; j < S::BC; ++j) {
      const int cc = wc_col + j * 16 + lr;
      const float *row = lq + cc * kLpKP;
      const flt4 lo = *(const flt4 *)(row + ((2 * g) ^ O::swz(cc)) * O::EPC);
      const flt4 hi = *(const flt4 *)(row + ((2 * g + 1) ^ O::swz(cc)) * O::EPC);
      b[j] = flt8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int i = 0; i < S::BR; ++i)
#pragma unroll
        for (int j = 0; j < S::BC; ++j)
          acc[i * S::BC + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j][t], acc[i * S::BC + j], 0, 0, 0);
  }
}

// Full K loop of one chunk on operand planes (K a multiple of 32).  Same contract as
// tile_gemm: the caller has passed a workgroup barrier since the stages were last read.
template <class S, int PREC>
__device__ inline void tile_gemm_lp(const typename LpOf<PREC>::E *P, const typename LpOf<PREC>::E *QT,
                                    size_t pstride, int ld, int M, int N, int K, int m0, int n0,
                                    LpLds<S, PREC> &L, bool active, int wr_row, int wc_col, flt4 (&acc)[S::TPW]) {
  typedef LpLds<S, PREC> LL;
#pragma unroll
  for (int i = 0; i < S::TPW; ++i) acc[i] = flt4{0, 0, 0, 0};
  const int npan = K / kLpKP;
  constexpr int PER_WAVE = LL::INSTR / S::NW;
  issue_panel_lp<S, PREC>(P, QT, pstride, ld, M, N, m0, n0, 0, L.p[0], L.q[0]);
  if (npan > 1) issue_panel_lp<S, PREC>(P, QT, pstride, ld, M, N, m0, n0, kLpKP, L.p[1], L.q[1]);
  auto step = [&](int kp, const typename LL::E *lp, const typename LL::E *lq, typename LL::E *np_p,
                  typename LL::E *np_q) {
    if (kp + 1 < npan) wait_vmcnt<PER_WAVE>(); else wait_vmcnt<0>();
    lds_barrier();
    if (kp + 2 < npan) issue_panel_lp<S, PREC>(P, QT, pstride, ld, M, N, m0, n0, (kp + 2) * kLpKP, np_p, np_q);
    if (active) mma_panel_lp<S, PREC>(lp, lq, wr_row, wc_col, acc);
  };
  for (int kp = 0; kp < npan; kp += 3) {
    step(kp, L.p[0], L.q[0], L.p[2], L.q[2]);
    if (kp + 1 < npan) step(kp + 1, L.p[1], L.q[1], L.p[0], L.q[0]);
    if (kp + 2 < npan) step(kp + 2, L.p[2], L.q[2], L.p[1], L.q[1]);
  }
}

}  // namespace expm
