// Tiled multi-workgroup path for large orders: every GEMM is one launch over
// (output tiles) x (matrices of the group), each workgroup computing one 128 x 128 tile with
// the 8-wave direct-to-LDS tile engine and applying the fused epilogue of that step.
//
// Steps per group of matrices (all of order n, zero padded to np = multiple of 128):
//   load: copy A into buffer 0 (real form for complex input), partial column sums;
//   norm: column sums reduced in a fixed order, maximum by an integer atomic on the bit
//         pattern of the non-negative doubles (deterministic);
//   select: (m, s) per matrix on the device, scaled coefficients per matrix;
//   read (m, s) back once; group the matrices by degree and squaring count;
//   powers, product stage (the same epilogue kinds as the fused path), s squarings.
// Zero padding is exact for the same reason as in the fused path (block-diagonal powers).
//
// Reduced-precision forms: the powers and the first GEMM of the product stage run in FP32 or
// BF16x3 (FP32 accumulation); the last product of the stage, which carries the O(1) identity
// part of T_m (for T_18: (B_3 + A_9) A_9 with constant term about (-11.06)(-0.090) = 1), and
// the s squarings, whose error grows 2^s-fold, stay FP64, as do the norms and the selection.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "coefs.h"
#include "expm_large.h"
#include "gemm_block.h"

namespace expm {

namespace {

typedef TileShape<8, 128, 128, 4, 2, 2, 4> LS;
// LDS pool of the reduced-precision products: the three-stage ring of bfloat16 planes
// (144 KiB), reused as the chunk copy of C
constexpr int kPoolLp = 18432;
static_assert(kLargeTile * 129 <= kPoolLp, "tile copy exceeds the reduced-precision pool");
constexpr int LDC_L = 129;
static_assert(kLargeTile * LDC_L <= kPool8, "tile copy exceeds the LDS pool");

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Buffer selectors resolved per matrix inside the kernels.
enum BufSel {
  SEL_T = 100,       // buffer holding T: 2 for m >= 8, else 3
  SEL_TDST = 101,    // destination of T: e^A when s == 0, else SEL_T
  SEL_SQSRC = 200,   // squaring source in round r: SEL_T ^ ((r - 1) & 1)
  SEL_SQDST = 201,   // squaring destination in round r: e^A when r == s, else source ^ 1
  SEL_NONE = -1
};

struct MatCtx {
  double *buf0;      // first work buffer of the matrix
  size_t bstride;    // doubles between buffers
  int m, s;
};

struct LargeArgs {
  double *ws;              // group work buffers
  size_t mstride, bstride; // doubles per matrix / per buffer
  int np, n, nin, cplx;
  const double *A;
  double *E;
  int64_t io_stride;       // doubles between consecutive inputs / outputs
  int64_t g0;              // global index of the group's first matrix
  const int32_t *m_arr, *s_arr;  // global arrays
  const double *coef;      // group coefficients, 64 per matrix
  const int32_t *list;     // matrices (group-relative) of this launch
  int round;               // squaring round (1-based) for SEL_SQ*
  int ps;                  // Paterson-Stockmeyer comparison method
  int pade;                // diagonal Pade comparison method (m = 2m' = 10 or 26)
  int32_t *piv;            // per matrix: np row pivots of the Pade denominator's LU
  const int *flags;        // per matrix: bit 0 non-finite input, bit 1 not upper triangular
  int coff;                // first coefficient of this step in the matrix's 64
  void *planes;            // operand planes of reduced-precision products (2 PL np^2
                           // elements per matrix: left-operand planes, then right-operand)
  int32_t *shift;          // per matrix: exponents e0, e1, e2 of the pending rescale
                           // B_k *= 2^e_k of buffers 0, 1, 2 (lg_rescale_kernel)
  // step description
  int kind;                // epilogue kind (GEMM) or elementwise kind
  int p, q, b0, b1, b2, in0, in1, o[5], dst;
};

// Buffer of T.  Reduced sequences: 2 for m >= 8, else 3.  Paterson-Stockmeyer (A^2, A^3 in
// 1, 2, A^4 in 3, Horner partial sums in 6 and 7): 3 with the base A^3, 5 with the base A^4,
// so that neither operand of the last Horner step is its destination.
// Pade (r_10: V - U and V + U in 6, 7; r_26: in 4, 5): T is the numerator's buffer, which the
// solve overwrites with r = (V - U)^-1 (V + U); the squarings alternate with the denominator's.
__device__ inline int resolve_t(int m, int ps, int pade) {
  if (pade) return m == 10 ? 7 : 5;
  if (ps && m >= 6) return ps_base(m) == 4 ? 5 : 3;
  return m >= 8 ? 2 : 3;
}

// Pointer of a selector for matrix (group-relative) mi; returns nullptr for e^A (the caller
// then writes the output matrix).
__device__ inline double *sel_ptr(const LargeArgs &a, int mi, int sel, int m, int s) {
  double *base = a.ws + (size_t)mi * a.mstride;
  int k = sel;
  const int t = resolve_t(m, a.ps, a.pade);
  if (sel == SEL_T) k = t;
  else if (sel == SEL_TDST) { if (s == 0) return nullptr; k = t; }
  else if (sel == SEL_SQSRC) k = t ^ ((a.round - 1) & 1);
  else if (sel == SEL_SQDST) { if (a.round == s) return nullptr; k = t ^ ((a.round - 1) & 1) ^ 1; }
  if (k < 0) return nullptr;
  return base + (size_t)k * a.bstride;
}

__global__ void lg_zero_kernel(unsigned long long *norms, int64_t nnorms, int *flags, int64_t nflags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nnorms) norms[i] = 0ull;
  if (i < nflags) flags[i] = 0;
}

// Copy of the group's inputs into buffer 0 (zero padded, real form for complex input) and
// partial column sums of |A| over kLargeRB rows.  Grid (np / 256, np / kLargeRB, count).
__global__ __launch_bounds__(256) void lg_load_kernel(LargeArgs a, double *partial, int nrb, int *flags) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= a.np) return;
  const int rb = blockIdx.y;
  const int mi = blockIdx.z;
  const int n = a.n, nin = a.nin, np = a.np, cx = a.cplx;
  cgdouble *A = gptr(a.A + (a.g0 + mi) * a.io_stride);
  gdouble *B0 = gptr(a.ws + (size_t)mi * a.mstride);
  double acc = 0.0;
  int bad = 0, lower = 0;
  for (int r0 = rb * kLargeRB; r0 < (rb + 1) * kLargeRB; r0 += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = r0 + u;
      double x = 0.0;
      if (r < n && col < n) {
        if (cx == 2) {  // native complex: the real part here, the imaginary one below
          x = A[2 * ((size_t)r * n + col)];
        } else if (!cx) {
          x = A[(size_t)r * n + col];
        } else {
          const int ri = r < nin ? r : r - nin, ci = col < nin ? col : col - nin;
          const bool im = (r < nin) != (col < nin);
          x = A[2 * ((size_t)ri * nin + ci) + (im ? 1 : 0)];
          if (im && r < nin) x = -x;
        }
      }
      v[u] = x;
    }
    if (cx == 2) {
      const size_t nn = (size_t)np * np;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int r = r0 + u;
        const double y = (r < n && col < n) ? A[2 * ((size_t)r * n + col) + 1] : 0.0;
        bad |= !isfinite(v[u]) || !isfinite(y);
        acc += hypot(v[u], y);  // |z| (a-1: the 1-norm of the complex matrix)
        B0[(size_t)r * np + col] = v[u];
        B0[nn + (size_t)r * np + col] = y;
      }
      continue;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      bad |= !isfinite(v[u]);
      lower |= (r0 + u > col) && v[u] != 0.0;
      acc += fabs(v[u]);
      B0[(size_t)(r0 + u) * np + col] = v[u];
    }
  }
  partial[((size_t)mi * nrb + rb) * np + col] = acc;
  if (bad || lower) atomicOr(&flags[mi], (bad ? 1 : 0) | (lower ? 2 : 0));
}

// Triangular refinement (concluding remarks; the technique of the alpha_p paper it cites): for
// an upper triangular input, the current iterate approximates e^(2^(r - s) A) after round r of
// the squarings (r = 0: T_m itself).  Its diagonal is set to exp(2^(r-s) a_ii) and its first
// superdiagonal to the exact (1, 2) entry of the exponential of the 2 x 2 block
// [[x1, y], [0, x2]] = 2^(r-s) [[a_ii, a_i,i+1], [0, a_i+1,i+1]]:
//   y exp((x1 + x2) / 2) sinh(d) / d,  d = (x2 - x1) / 2   (y exp(x1) when d = 0).
// The iterate lives where that round wrote it (a work buffer, or e^A after the last round).
// Grid (ceil(n / 256), count).
__global__ __launch_bounds__(256) void lg_tri_fix_kernel(LargeArgs a) {
  const int mi = a.list[blockIdx.y];
  const int64_t gb = a.g0 + mi;
  const int m = a.m_arr[gb], s = a.s_arr[gb];
  if (m < 1 || (a.flags[mi] & 2)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int n = a.n, np = a.np;
  if (i >= n) return;
  // the caller's input (real, n x n): the product stage reuses the work buffer that held A
  cgdouble *A = gptr(a.A + gb * a.io_stride);
  double *dstp = sel_ptr(a, mi, a.round == 0 ? SEL_TDST : SEL_SQDST, m, s);
  gdouble *dst = dstp ? gptr(dstp) : gptr(a.E + gb * a.io_stride);
  const int ld = dstp ? np : n;
  const double f = ldexp(1.0, a.round - s);
  const double x1 = f * A[(size_t)i * n + i];
  dst[(size_t)i * ld + i] = exp(x1);
  if (i + 1 < n) {
    const double x2 = f * A[(size_t)(i + 1) * n + i + 1], y = f * A[(size_t)i * n + i + 1];
    const double d = 0.5 * (x2 - x1);
    const double sh = d == 0.0 ? 1.0 : sinh(d) / d;
    dst[(size_t)i * ld + i + 1] = y * exp(0.5 * (x1 + x2)) * sh;
  }
}

// Partial column sums of |buffer sel| for the listed matrices.  Grid (np / 256, nrb, count).
__global__ __launch_bounds__(256) void lg_colsum_kernel(LargeArgs a, int sel, double *partial, int nrb) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= a.np) return;
  const int rb = blockIdx.y;
  const int mi = a.list[blockIdx.z];
  cgdouble *B = gptr(a.ws + (size_t)mi * a.mstride + (size_t)sel * a.bstride);
  double acc = 0.0;
  const size_t nn = (size_t)a.np * a.np;
  for (int r0 = rb * kLargeRB; r0 < (rb + 1) * kLargeRB; r0 += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = B[(size_t)(r0 + u) * a.np + col];
    if (a.cplx == 2) {
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += hypot(v[u], B[nn + (size_t)(r0 + u) * a.np + col]);
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += fabs(v[u]);
    }
  }
  partial[((size_t)mi * nrb + rb) * a.np + col] = acc;
}

// Column sums in row-block order, then the maximum over columns into norms[mi] (bit pattern
// of a non-negative double, monotone as an unsigned integer).  Grid (np / 256, count).
__global__ __launch_bounds__(256) void lg_colmax_kernel(LargeArgs a, const double *partial, int nrb,
                                                        unsigned long long *norms, int use_list) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  const int mi = use_list ? a.list[blockIdx.y] : blockIdx.y;
  double s = 0.0;
  if (col < a.np)
    for (int rb = 0; rb < nrb; ++rb) s += partial[((size_t)mi * nrb + rb) * a.np + col];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(&norms[mi], (unsigned long long)__double_as_longlong(red[0]));
}

// (m, s) and coefficients per matrix, and the rescale that puts the scaling into the matrices:
// buffer 0 holds A after the load, so the first pass (alpha = 0) asks for X = 2^-s A (s of the
// plain rule, or of the Paterson-Stockmeyer rule), exactly, before any power is formed; the
// coefficients are then the constants themselves.  alpha = 1 (after A^2, A^3 of that X_p =
// 2^-sp A were formed where the plain degree forms them; their norms are those of X_p^k)
// recomputes sp, takes ||A^k|| = 2^(k sp) ||X_p^k||, selects, and asks for
// X^k = 2^(k (sp - s)) X_p^k.  A 1-norm that overflows (finite entries) is refused like a
// non-finite entry.
__global__ void lg_select_kernel(LargeArgs a, int count, int stride, const unsigned long long *norms,
                                 const int *flags, int alpha, Consts k, int32_t *status, double *coef) {
  const int mi = blockIdx.x * blockDim.x + threadIdx.x;
  if (mi >= count) return;
  const int64_t gb = a.g0 + mi;
  int32_t *m_arr = const_cast<int32_t *>(a.m_arr), *s_arr = const_cast<int32_t *>(a.s_arr);
  int32_t *sh = a.shift + 3 * mi;
  sh[0] = sh[1] = sh[2] = 0;
  const double eta = __longlong_as_double((long long)norms[mi]);
  if ((flags[mi] & 1) || !(eta <= __DBL_MAX__)) {
    m_arr[gb] = -1; s_arr[gb] = -1;
    if (status) status[gb] = EXPM_E_NONFINITE;
    return;
  }
  int m, s;
  if (a.pade) {
    // Sec. 2: r_10 or r_26, the cheaper with the solve costed 4/3 of a product (Table 1 theta);
    // coefficients b_0 .. b_m' of p_m' (eq. eq.24)
    select_pade(k.theta_pade, eta, &m, &s);
    m_arr[gb] = m; s_arr[gb] = s;
    if (status) status[gb] = EXPM_OK;
    double *cf = coef + (size_t)mi * 64;
    if (m == 10) for (int j = 0; j < 6; ++j) cf[j] = k.pade5[j];
    else for (int j = 0; j < 14; ++j) cf[j] = k.pade13[j];
    sh[0] = -s;
    return;
  }
  if (a.ps) {
    select_ps(k.theta_ps, eta, &m, &s);
    m_arr[gb] = m; s_arr[gb] = s;
    if (status) status[gb] = EXPM_OK;
    if (m >= 6) make_ps_coefs(m, 0, coef + (size_t)mi * 64);
    else make_coefs(k, m, 0, coef + (size_t)mi * 64);
    sh[0] = -s;
    return;
  }
  select_ms(k.theta, 0, eta, -1.0, -1.0, &m, &s);
  const int sp = s;
  if (alpha && m >= 2) {
    const double n2 = unscale_norm(__longlong_as_double((long long)norms[stride + mi]), 2, sp);
    const double n3 = m >= 12 ? unscale_norm(__longlong_as_double((long long)norms[2 * stride + mi]), 3, sp) : -1.0;
    select_ms(k.theta, 1, eta, n2, n3, &m, &s);
    sh[0] = sp - s; sh[1] = 2 * (sp - s); sh[2] = 3 * (sp - s);
  } else if (!alpha) {
    sh[0] = -sp;
  }
  m_arr[gb] = m; s_arr[gb] = s;
  if (status) status[gb] = EXPM_OK;
  make_coefs(k, m, 0, coef + (size_t)mi * 64);
}

// B_k *= 2^e_k (exact) for buffers k < nbuf of every matrix of the group with e_k != 0.
// Grid (np * np / 1024, count).
__global__ __launch_bounds__(256) void lg_rescale_kernel(LargeArgs a, int nbuf) {
  const int mi = blockIdx.y;
  const int64_t total = (int64_t)a.np * a.np * (a.cplx == 2 ? 2 : 1);
  for (int k = 0; k < nbuf; ++k) {
    const int e2 = a.shift[3 * mi + k];
    if (e2 == 0) continue;
    gdouble *B = gptr(a.ws + (size_t)mi * a.mstride + (size_t)k * a.bstride);
    for (int u = 0; u < 4; ++u) {
      const int64_t e = ((int64_t)blockIdx.x * 4 + u) * 256 + threadIdx.x;
      if (e < total) B[e] = ldexp(B[e], e2);
    }
  }
}

// Thread 0 of a GEMM tile fills the LDS descriptor of the step for matrix mi.
__device__ inline void fill_desc(const LargeArgs &a, int mi, int64_t gb, int m, int s) {
  EpiDesc &d = g_ep;
  d.P = sel_ptr(a, mi, a.p, m, s);
  d.Q = sel_ptr(a, mi, a.q, m, s);
  d.b0 = sel_ptr(a, mi, 0, m, s); d.b1 = sel_ptr(a, mi, 1, m, s); d.b2 = sel_ptr(a, mi, 2, m, s);
  d.in0 = a.in0 >= 0 ? sel_ptr(a, mi, a.in0, m, s) : nullptr;
  d.in1 = a.in1 >= 0 ? sel_ptr(a, mi, a.in1, m, s) : nullptr;
  for (int j = 0; j < 5; ++j) d.o[j] = a.o[j] >= 0 ? sel_ptr(a, mi, a.o[j], m, s) : nullptr;
  double *dst = sel_ptr(a, mi, a.dst, m, s);
  if (dst) {
    d.dst = dst; d.dst_ld = a.np; d.dst_nvalid = a.np; d.cplx = 0;
  } else {
    d.dst = a.E + gb * a.io_stride; d.dst_ld = a.n; d.dst_nvalid = a.nin; d.cplx = a.cplx;
  }
  d.idw = 1.0;
  d.kind = a.kind;
  d.np = a.np;
  for (int i = 0; i < 64; ++i) d.c[i] = i + a.coff < 64 ? a.coef[(size_t)mi * 64 + a.coff + i] : 0.0;
}

// Native complex steps (cplx == 2): every buffer holds the real plane and then the imaginary
// one (nn elements apart).  After the real plane's epilogue thread 0 points the descriptor at
// the imaginary planes: inputs and outputs move by nn (the output matrix e^A by one double, to
// the imaginary members), and the identity terms drop out (real coefficients).
__device__ inline void desc_to_imag(size_t nn) {
  EpiDesc &d = g_ep;
  d.b0 += nn; d.b1 += nn; d.b2 += nn;
  if (d.in0) d.in0 += nn;
  if (d.in1) d.in1 += nn;
  for (int j = 0; j < 5; ++j)
    if (d.o[j]) d.o[j] += nn;
  d.dst += d.cplx == 2 ? 1 : nn;
  d.idw = 0.0;
}

// One 128 x 128 output tile of an FP64 GEMM step for matrix list[blockIdx.y].  Native
// complex: the real plane of the tile from two real products (Re P Re Q - Im P Im Q) and its
// epilogue, then the imaginary plane (Re P Im Q + Im P Re Q) and its epilogue.
template <int PREC>
__global__ __launch_bounds__(512, 1) void lg_gemm_kernel(LargeArgs a) {
  const int mi = a.list[blockIdx.y];
  const int64_t gb = a.g0 + mi;
  const int m = a.m_arr[gb], s = a.s_arr[gb];
  const int tiles = a.np / kLargeTile;
  const int tm = blockIdx.x / tiles, tn = blockIdx.x - tm * tiles;
  if (threadIdx.x == 0) fill_desc(a, mi, gb, m, s);
  __syncthreads();
  TileLds<LS> &L = *reinterpret_cast<TileLds<LS> *>(lds_pool<8>());
  const int wave = threadIdx.x >> 6;
  const int wr = wave / LS::WC, wc = wave % LS::WC;
  const int wr_row = wr * LS::BR * 16, wc_col = wc * LS::BC * 16;
  const int m0 = tm * kLargeTile, n0 = tn * kLargeTile;
  typename AccOf<PREC>::T acc[LS::TPW];
  double *cbuf = lds_pool<8>();
  auto finish = [&]() {
    if (a.kind == EK_STORE) {
      store_acc<LS, PREC>(acc, m0 + wr_row, n0 + wc_col);
      return;
    }
    __syncthreads();
    stage_acc<LS, LDC_L, PREC>(cbuf, acc, wr_row, wc_col);
    __syncthreads();
    run_epilogue<8>(cbuf, m0, n0, kLargeTile, kLargeTile, LDC_L);
  };
  cgdouble *P = gptr(g_ep.P), *Q = gptr(g_ep.Q);
  if (a.cplx != 2) {
    tile_gemm<LS, PREC>(P, a.np, Q, a.np, a.np, a.np, a.np, m0, n0, L, true, wr_row, wc_col, acc);
    finish();
    return;
  }
  const size_t nn = (size_t)a.np * a.np;
  tile_gemm<LS, PREC>(P, a.np, Q, a.np, a.np, a.np, a.np, m0, n0, L, true, wr_row, wc_col, acc);
  __syncthreads();
  tile_gemm<LS, PREC, true, true>(P + nn, a.np, Q + nn, a.np, a.np, a.np, a.np, m0, n0, L, true, wr_row, wc_col, acc);
  finish();
  __syncthreads();
  if (threadIdx.x == 0) desc_to_imag(nn);
  __syncthreads();
  tile_gemm<LS, PREC>(P, a.np, Q + nn, a.np, a.np, a.np, a.np, m0, n0, L, true, wr_row, wc_col, acc);
  __syncthreads();
  tile_gemm<LS, PREC, true>(P + nn, a.np, Q, a.np, a.np, a.np, a.np, m0, n0, L, true, wr_row, wc_col, acc);
  finish();
}

// Operand planes of a reduced-precision product (tile_gemm_lp): the FP64 buffer `sel` of each
// listed matrix, converted once, into the matrix's plane region: forms bit 0 row-major planes
// at the left-operand slot, bit 1 transposed planes at the right-operand slot.  BF16X3: hi,
// mid, lo = successive bfloat16 roundings (split3); F32: the FP32 rounding.  A 64 x 64 tile per
// workgroup, transposed through LDS.  Grid (np / 64, np / 64, count).
template <int PREC>
__global__ __launch_bounds__(256) void lg_planes_kernel(LargeArgs a, int sel, int forms) {
  typedef typename LpOf<PREC>::E E;
  constexpr int PL = LpOf<PREC>::PL;
  __shared__ double t[64][65];
  const int mi = a.list[blockIdx.z];
  const int64_t gb = a.g0 + mi;
  const int m = a.m_arr[gb], s = a.s_arr[gb];
  cgdouble *B = gptr((const double *)sel_ptr(a, mi, sel, m, s));
  const int np = a.np;
  const size_t nn = (size_t)np * np;
  E *base = (E *)a.planes + (size_t)mi * (2 * PL) * nn;
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  auto put = [&](E *dst, size_t e, double x) {
    if constexpr (PREC == PREC_BF16X3) {
      short h, md, l;
      split3(x, h, md, l);
      dst[e] = h; dst[nn + e] = md; dst[2 * nn + e] = l;
    } else {
      dst[e] = (float)x;
    }
  };
  for (int rr = ty; rr < 64; rr += 4) {
    const double x = B[(size_t)(r0 + rr) * np + c0 + tx];
    t[rr][tx] = x;
    if (forms & 1) put(base, (size_t)(r0 + rr) * np + c0 + tx, x);
  }
  if (forms & 2) {
    __syncthreads();
    for (int rr = ty; rr < 64; rr += 4) put(base + PL * nn, (size_t)(c0 + rr) * np + r0 + tx, t[tx][rr]);
  }
}

// One 128 x 128 output tile of a reduced-precision product on operand planes (left operand
// row-major planes, right operand transposed planes of the matrix's plane region), then the
// step's epilogue, as lg_gemm_kernel.
__shared__ double g_pool_lp[kPoolLp];
template <int PREC>
__global__ __launch_bounds__(512, 1) void lg_gemm_lp_kernel(LargeArgs a) {
  typedef typename LpOf<PREC>::E E;
  constexpr int PL = LpOf<PREC>::PL;
  static_assert(sizeof(LpLds<LS, PREC>) <= sizeof(g_pool_lp), "stage ring exceeds the pool");
  const int mi = a.list[blockIdx.y];
  const int64_t gb = a.g0 + mi;
  const int m = a.m_arr[gb], s = a.s_arr[gb];
  const int tiles = a.np / kLargeTile;
  const int tm = blockIdx.x / tiles, tn = blockIdx.x - tm * tiles;
  if (threadIdx.x == 0) fill_desc(a, mi, gb, m, s);
  __syncthreads();
  LpLds<LS, PREC> &L = *reinterpret_cast<LpLds<LS, PREC> *>(g_pool_lp);
  const int wave = threadIdx.x >> 6;
  const int wr = wave / LS::WC, wc = wave % LS::WC;
  const int wr_row = wr * LS::BR * 16, wc_col = wc * LS::BC * 16;
  const int m0 = tm * kLargeTile, n0 = tn * kLargeTile;
  const size_t nn = (size_t)a.np * a.np;
  const E *P = (const E *)a.planes + (size_t)mi * (2 * PL) * nn;
  flt4 acc[LS::TPW];
  tile_gemm_lp<LS, PREC>(P, P + PL * nn, nn, a.np, a.np, a.np, a.np, m0, n0, L, true, wr_row, wc_col, acc);
  if (a.kind == EK_STORE) {
    store_acc<LS, PREC>(acc, m0 + wr_row, n0 + wc_col);
    return;
  }
  __syncthreads();
  stage_acc<LS, LDC_L, PREC>(g_pool_lp, acc, wr_row, wc_col);
  __syncthreads();
  run_epilogue<8>(g_pool_lp, m0, n0, kLargeTile, kLargeTile, LDC_L);
}

// Elementwise steps (no product), kinds LC1, LC2 (T = I + c0 A [+ c1 A^2]), LC4W, LC8W,
// LC12.  Grid (np * np / (256 * 4), count).
// LCPS: innermost Horner term of eq. poli9, F_(r-1) (+ a_16 A^4 for the base A^4), from the
// coefficient block at coff.
// LCPADE: the even and odd parts' inner sums of eq. eq.pade26 (r_26: W1 = b13 X^6 + b11 X^4 +
// b9 X^2, Z1 = b7 X^6 + b5 X^4 + b3 X^2 + b1 I, W2 = b12 X^6 + b10 X^4 + b8 X^2, Z2 = b6 X^6 +
// b4 X^4 + b2 X^2 + b0 I into 4, 5, 6, 7; r_10: W = b5 X^4 + b3 X^2 + b1 I, V = b4 X^4 + b2 X^2 +
// b0 I into 4, 5) from X^2, X^4, X^6 in 1, 2, 3.  LCCOPY: dst = buffer in0.
enum ElemKind { LC1 = 0, LC2 = 1, LC4W = 2, LC8W = 3, LC12 = 4, LCNAN = 5, LCPS = 6, LCPADE = 7, LCCOPY = 8 };

__global__ __launch_bounds__(256) void lg_elem_kernel(LargeArgs a) {
  const int mi = a.list[blockIdx.y];
  const int64_t gb = a.g0 + mi;
  const int m = a.m_arr[gb], s = a.s_arr[gb];
  const double *c = a.coef + (size_t)mi * 64;
  cgdouble *B0 = gptr(sel_ptr(a, mi, 0, m, s));
  cgdouble *B1 = gptr(sel_ptr(a, mi, 1, m, s));
  cgdouble *B2 = gptr(sel_ptr(a, mi, 2, m, s));
  double *dstp = a.kind == LCNAN ? nullptr : sel_ptr(a, mi, a.dst, m, s);
  gdouble *dst0 = dstp ? gptr(dstp) : gptr(a.E + gb * a.io_stride);
  const int dld = dstp ? a.np : a.n, dnv = dstp ? a.np : a.nin, dcx = dstp ? 0 : a.cplx;
  const int np = a.np;
  // native complex: the elements of the imaginary planes follow those of the real ones (no
  // identity there); e indexes the buffers directly either way
  const int64_t nn = (int64_t)np * np, total = nn * (a.cplx == 2 ? 2 : 1);
  for (int u = 0; u < 4; ++u) {
    const int64_t e = ((int64_t)blockIdx.x * 4 + u) * 256 + threadIdx.x;
    if (e >= total) break;
    const bool im = e >= nn;
    const int64_t e1 = im ? e - nn : e;
    const int r = (int)(e1 / np), cc = (int)(e1 - (int64_t)r * np);
    const double id = (r == cc && !im) ? 1.0 : 0.0;
    gdouble *dst = dst0 + (im ? (dstp ? nn : 1) : 0);
    switch (a.kind) {
      case LC1: put_dst(dst, dld, dnv, dcx, r, cc, id + c[0] * B0[e]); break;
      case LC2: put_dst(dst, dld, dnv, dcx, r, cc, id + c[0] * B0[e] + c[1] * B1[e]); break;
      case LC4W: gptr(sel_ptr(a, mi, 2, m, s))[e] = c[2] * id + c[3] * B0[e] + c[4] * B1[e]; break;
      case LC8W: gptr(sel_ptr(a, mi, 2, m, s))[e] = c[0] * B0[e] + c[1] * B1[e]; break;
      case LCNAN: put_dst(dst, dld, dnv, dcx, r, cc, __builtin_nan("")); break;
      case LCCOPY: put_dst(dst, dld, dnv, dcx, r, cc, gptr(sel_ptr(a, mi, a.in0, m, s))[e]); break;
      case LCPADE: {
        const double x2 = B1[e], x4 = B2[e];
        if (m == 10) {
          gptr(sel_ptr(a, mi, 4, m, s))[e] = c[5] * x4 + c[3] * x2 + c[1] * id;
          gptr(sel_ptr(a, mi, 5, m, s))[e] = c[4] * x4 + c[2] * x2 + c[0] * id;
        } else {
          const double x6 = gptr(sel_ptr(a, mi, 3, m, s))[e];
          gptr(sel_ptr(a, mi, 4, m, s))[e] = c[13] * x6 + c[11] * x4 + c[9] * x2;
          gptr(sel_ptr(a, mi, 5, m, s))[e] = c[7] * x6 + c[5] * x4 + c[3] * x2 + c[1] * id;
          gptr(sel_ptr(a, mi, 6, m, s))[e] = c[12] * x6 + c[10] * x4 + c[8] * x2;
          gptr(sel_ptr(a, mi, 7, m, s))[e] = c[6] * x6 + c[4] * x4 + c[2] * x2 + c[0] * id;
        }
      } break;
      case LCPS: {
        const double *k = c + a.coff;
        double t = k[0] * id + k[1] * B0[e] + k[2] * B1[e] + k[3] * B2[e];
        if (m == 16) t += k[4] * gptr(sel_ptr(a, mi, 3, m, s))[e];
        gptr(dstp)[e] = t;
      } break;
      case LC12: {
        const double x1 = B0[e], x2 = B1[e], x3 = B2[e];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          gptr(sel_ptr(a, mi, 3 + j, m, s))[e] = c[4 * j] * id + c[4 * j + 1] * x1 + c[4 * j + 2] * x2 + c[4 * j + 3] * x3;
      } break;
    }
  }
}

// ---- Pade comparison method: the solve (V - U) R = V + U (Sec. 2; an inverse costed as 4/3
// of a product) by LU factorization with partial pivoting, in blocks of kLuNB columns.  The
// right-hand side rides along as extra columns, so the factorization leaves L^-1 P (V + U) in
// its place; back substitution with U then gives R there.  Steps per block k: the panel's LU
// (one workgroup per matrix, the panel rows in registers), the panel's row swaps on every
// other column, the unit-lower block solve of the block row, the trailing update by the MFMA
// tile engine (K = kLuNB).  Then, blocks from the bottom: the upper block solve and the update
// of the rows above.  The denominator lives in buffer 6 (r_10) or 4 (r_26), the numerator in
// the next one.
constexpr int kLuNB = 32;

__device__ inline int lu_mbuf(int m) { return m == 10 ? 6 : 4; }

// Panel: columns [k, k + 32) of rows [k, np); thread t holds rows t + 1024 q (q < RPT).
// Pivot = largest |a| in the column (the smallest row on ties), as LAPACK's getf2.
template <int RPT>
__global__ __launch_bounds__(1024) void lg_lu_panel_kernel(LargeArgs a, int k) {
  const int mi = a.list[blockIdx.x];
  const int m = a.m_arr[a.g0 + mi];
  const int np = a.np;
  gdouble *M = gptr(a.ws + (size_t)mi * a.mstride + (size_t)lu_mbuf(m) * a.bstride);
  int32_t *piv = a.piv + (size_t)mi * np;
  __shared__ double rowA[kLuNB], rowB[kLuNB], wv[16];
  __shared__ int wi[16], sp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double v[RPT][kLuNB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = tid + 1024 * q;
#pragma unroll
    for (int c = 0; c < kLuNB; ++c) v[q][c] = (i >= k && i < np) ? M[(size_t)i * np + k + c] : 0.0;
  }
#pragma clang loop unroll(full)
  for (int j = 0; j < kLuNB; ++j) {
    const int col = k + j;
    double best = -1.0;
    int bi = np;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = tid + 1024 * q;
      const double x = fabs(v[q][j]);
      if (i >= col && i < np && x > best) { best = x; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { wv[wave] = best; wi[wave] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = wv[0];
      int ii = wi[0];
      for (int w = 1; w < 16; ++w)
        if (wv[w] > b || (wv[w] == b && wi[w] < ii)) { b = wv[w]; ii = wi[w]; }
      sp = ii;
      piv[col] = ii;
    }
    __syncthreads();
    const int p = sp;
    // rows col and p trade places (their owners pass them through LDS)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = tid + 1024 * q;
      if (i == col) {
#pragma unroll
        for (int c = 0; c < kLuNB; ++c) rowA[c] = v[q][c];
      }
      if (i == p) {
#pragma unroll
        for (int c = 0; c < kLuNB; ++c) rowB[c] = v[q][c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = tid + 1024 * q;
      if (p != col && i == col) {
#pragma unroll
        for (int c = 0; c < kLuNB; ++c) v[q][c] = rowB[c];
      }
      if (p != col && i == p) {
#pragma unroll
        for (int c = 0; c < kLuNB; ++c) v[q][c] = rowA[c];
      }
    }
    // rowB is the pivot row now at `col`: multipliers and the rank-1 update of the panel
    const double d = rowB[j];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = tid + 1024 * q;
      if (i > col && i < np) {
        const double l = v[q][j] / d;
        v[q][j] = l;
#pragma unroll
        for (int c = j + 1; c < kLuNB; ++c) v[q][c] -= l * rowB[c];
      }
    }
    __syncthreads();  // rowA, rowB are rewritten by the next column
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = tid + 1024 * q;
    if (i >= k && i < np)
#pragma unroll
      for (int c = 0; c < kLuNB; ++c) M[(size_t)i * np + k + c] = v[q][c];
  }
}

// The panel's row swaps on every other column of the denominator and on the numerator.
// Thread per column of the augmented [M | R]; grid (2 np / 256, count).
__global__ __launch_bounds__(256) void lg_lu_swap_kernel(LargeArgs a, int k) {
  const int mi = a.list[blockIdx.y];
  const int m = a.m_arr[a.g0 + mi];
  const int np = a.np;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= 2 * np) return;
  const int cc = c < np ? c : c - np;
  if (c < np && cc >= k && cc < k + kLuNB) return;  // the panel swapped its own rows
  gdouble *B = gptr(a.ws + (size_t)mi * a.mstride + (size_t)(lu_mbuf(m) + (c < np ? 0 : 1)) * a.bstride);
  const int32_t *piv = a.piv + (size_t)mi * np;
  for (int j = 0; j < kLuNB; ++j) {
    const int p = piv[k + j];
    if (p != k + j) {
      const double t = B[(size_t)(k + j) * np + cc];
      B[(size_t)(k + j) * np + cc] = B[(size_t)p * np + cc];
      B[(size_t)p * np + cc] = t;
    }
  }
}

// Block row k of U and of L^-1 P R: x <- L11^-1 x for the columns right of the panel and every
// numerator column (L11 unit lower, in LDS).  Thread per column; grid
// (((np - k - 32) + np) / 256, count).
__global__ __launch_bounds__(256) void lg_lu_fsub_kernel(LargeArgs a, int k) {
  const int mi = a.list[blockIdx.y];
  const int m = a.m_arr[a.g0 + mi];
  const int np = a.np;
  gdouble *M = gptr(a.ws + (size_t)mi * a.mstride + (size_t)lu_mbuf(m) * a.bstride);
  __shared__ double Lk[kLuNB][kLuNB + 1];
  for (int e = threadIdx.x; e < kLuNB * kLuNB; e += 256) Lk[e / kLuNB][e % kLuNB] = M[(size_t)(k + e / kLuNB) * np + k + e % kLuNB];
  __syncthreads();
  const int nm = np - k - kLuNB;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nm + np) return;
  gdouble *B = c < nm ? M : gptr(a.ws + (size_t)mi * a.mstride + (size_t)(lu_mbuf(m) + 1) * a.bstride);
  const int cc = c < nm ? k + kLuNB + c : c - nm;
  double x[kLuNB];
#pragma unroll
  for (int i = 0; i < kLuNB; ++i) x[i] = B[(size_t)(k + i) * np + cc];
#pragma unroll
  for (int i = 1; i < kLuNB; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) x[i] -= Lk[i][j] * x[j];
#pragma unroll
  for (int i = 0; i < kLuNB; ++i) B[(size_t)(k + i) * np + cc] = x[i];
}

// Block row k of R: x <- U11^-1 x for every numerator column (U11 upper, in LDS).  Grid
// (np / 256, count).
__global__ __launch_bounds__(256) void lg_lu_bsub_kernel(LargeArgs a, int k) {
  const int mi = a.list[blockIdx.y];
  const int m = a.m_arr[a.g0 + mi];
  const int np = a.np;
  gdouble *M = gptr(a.ws + (size_t)mi * a.mstride + (size_t)lu_mbuf(m) * a.bstride);
  gdouble *R = gptr(a.ws + (size_t)mi * a.mstride + (size_t)(lu_mbuf(m) + 1) * a.bstride);
  __shared__ double Uk[kLuNB][kLuNB + 1];
  for (int e = threadIdx.x; e < kLuNB * kLuNB; e += 256) Uk[e / kLuNB][e % kLuNB] = M[(size_t)(k + e / kLuNB) * np + k + e % kLuNB];
  __syncthreads();
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= np) return;
  double x[kLuNB];
#pragma unroll
  for (int i = 0; i < kLuNB; ++i) x[i] = R[(size_t)(k + i) * np + c];
#pragma unroll
  for (int i = kLuNB - 1; i >= 0; --i) {
#pragma unroll
    for (int j = i + 1; j < kLuNB; ++j) x[i] -= Uk[i][j] * x[j];
    x[i] /= Uk[i][i];
  }
#pragma unroll
  for (int i = 0; i < kLuNB; ++i) R[(size_t)(k + i) * np + c] = x[i];
}

// dst -= P Q with K = 32 on 128 x 128 tiles: P = columns [pcol, pcol + 32) of the denominator,
// Q = rows [qrow, qrow + 32); output rows [r_lo, r_hi) of the denominator's columns
// [mcol, np) (Q and dst the denominator) followed by every numerator column (Q and dst the
// numerator).  Grid (row tiles x column tiles, count).
__global__ __launch_bounds__(512, 1) void lg_lu_gemm_kernel(LargeArgs a, int pcol, int qrow, int r_lo, int r_hi,
                                                           int mcol) {
  const int mi = a.list[blockIdx.y];
  const int m = a.m_arr[a.g0 + mi];
  const int np = a.np;
  double *M = a.ws + (size_t)mi * a.mstride + (size_t)lu_mbuf(m) * a.bstride;
  double *R = M + a.bstride;
  const int tcm = mcol < np ? (np - mcol + kLargeTile - 1) / kLargeTile : 0;
  const int tcn = tcm + np / kLargeTile;
  const int tm = blockIdx.x / tcn, tn = blockIdx.x - tm * tcn;
  const int m0 = r_lo + tm * kLargeTile;
  const bool inm = tn < tcm;
  double *Qb = inm ? M : R;
  const int n0 = inm ? mcol + tn * kLargeTile : (tn - tcm) * kLargeTile;
  TileLds<LS> &L = *reinterpret_cast<TileLds<LS> *>(lds_pool<8>());
  const int wave = threadIdx.x >> 6;
  const int wr = wave / LS::WC, wc = wave % LS::WC;
  const int wr_row = wr * LS::BR * 16, wc_col = wc * LS::BC * 16;
  dbl4 acc[LS::TPW];
  tile_gemm<LS>(gptr(M + pcol), np, gptr(Qb + (size_t)qrow * np), np, r_hi, np, kLuNB, m0, n0, L, true, wr_row,
                wc_col, acc);
  gdouble *D = gptr(Qb);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < LS::BR; ++i)
#pragma unroll
    for (int j = 0; j < LS::BC; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr_row + 16 * i + 4 * r + (lane >> 4), col = n0 + wc_col + 16 * j + (lane & 15);
        if (row < r_hi && col < np) D[(size_t)row * np + col] -= acc[i * LS::BC + j][r];
      }
}

}  // namespace

LargeLayout large_layout(int64_t n_real, int64_t batch, int prec, int tiles_per_launch, int planes) {
  LargeLayout L;
  L.n = n_real;
  L.np = (n_real + kLargeTile - 1) / kLargeTile * kLargeTile;
  const int64_t tiles = (L.np / kLargeTile) * (L.np / kLargeTile);
  int64_t g = (tiles_per_launch + tiles - 1) / tiles;   // about that many output tiles per launch
  if (g < 1) g = 1;
  if (g > batch) g = batch;
  L.group = g;
  L.nrb = L.np / kLargeRB;
  const size_t nn = (size_t)L.np * L.np;
  L.bufs_off = 0;
  L.partial_off = align_up(L.bufs_off + (size_t)g * kLargeBufs * planes * nn * sizeof(double));
  L.norms_off = align_up(L.partial_off + (size_t)g * L.nrb * L.np * sizeof(double));
  L.flags_off = align_up(L.norms_off + (size_t)3 * g * sizeof(unsigned long long));
  L.coef_off = align_up(L.flags_off + (size_t)g * sizeof(int));
  L.list_off = align_up(L.coef_off + (size_t)g * 64 * sizeof(double));
  L.shift_off = align_up(L.list_off + (size_t)g * 64 * sizeof(int32_t));
  // operand planes: BF16X3 2 x 3 bfloat16 planes per matrix, FP32 and FP32_ALL 2 float planes
  const size_t plane_bytes = prec == EXPM_PREC_BF16X3 ? 12 : prec == EXPM_PREC_FP64 ? 0 : 8;
  L.planes_off = align_up(L.shift_off + (size_t)g * 3 * sizeof(int32_t));
  L.piv_off = align_up(L.planes_off + (size_t)g * plane_bytes * nn);
  L.total = align_up(L.piv_off + (size_t)g * L.np * sizeof(int32_t));
  return L;
}

namespace {

struct Launcher {
  const LargeCall &c;
  const LargeLayout &L;
  LargeArgs base;
  hipStream_t st;
  int32_t *list_dev;
  bool ok = true;

  std::vector<std::vector<int32_t>> keep;  // host copies stay alive until the group's sync

  // Uploads `idx` as the launch list and returns the device pointer (slots are reused in
  // stream order: a later copy into a slot runs after the kernels that read it).
  const int32_t *upload(const std::vector<int32_t> &idx, int slot) {
    int32_t *d = list_dev + (size_t)(slot % 64) * L.group;
    keep.push_back(idx);
    if (hipMemcpyAsync(d, keep.back().data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess)
      ok = false;
    return d;
  }

  int prec = PREC_F64;  // arithmetic of the polynomial products (set per call by run_large)

  void gemm(const std::vector<int32_t> &idx, int slot, int kind, int p, int q, int dst,
            int in0 = SEL_NONE, int in1 = SEL_NONE, std::vector<int> o = {}, int round = 0,
            bool reduced = false, int coff = 0) {
    if (idx.empty() || !ok) return;
    LargeArgs a = base;
    a.list = upload(idx, slot);
    a.kind = kind; a.p = p; a.q = q; a.dst = dst; a.in0 = in0; a.in1 = in1; a.round = round;
    a.coff = coff;
    for (int j = 0; j < 5; ++j) a.o[j] = j < (int)o.size() ? o[j] : SEL_NONE;
    const int tiles = (int)((L.np / kLargeTile) * (L.np / kLargeTile));
    // EXPM_PREC_FP32_ALL: every product in FP32; otherwise the reduced form covers the powers
    // and the first product of the stage, and the rest stays FP64
    const int pr = prec == EXPM_PREC_FP32_ALL ? PREC_F32 : reduced ? prec : PREC_F64;
    const dim3 grid(tiles, (unsigned)idx.size());
    if (pr == PREC_F64) {
      hipLaunchKernelGGL(lg_gemm_kernel<PREC_F64>, grid, dim3(512), 0, st, a);
    } else {
      // operands converted once into planes (both forms from one read when P = Q), then the
      // product on the planes
      const dim3 pg((unsigned)(L.np / 64), (unsigned)(L.np / 64), (unsigned)idx.size());
      if (pr == PREC_F32) {
        if (p == q) hipLaunchKernelGGL(lg_planes_kernel<PREC_F32>, pg, dim3(256), 0, st, a, p, 3);
        else {
          hipLaunchKernelGGL(lg_planes_kernel<PREC_F32>, pg, dim3(256), 0, st, a, p, 1);
          hipLaunchKernelGGL(lg_planes_kernel<PREC_F32>, pg, dim3(256), 0, st, a, q, 2);
        }
        hipLaunchKernelGGL(lg_gemm_lp_kernel<PREC_F32>, grid, dim3(512), 0, st, a);
      } else {
        if (p == q) hipLaunchKernelGGL(lg_planes_kernel<PREC_BF16X3>, pg, dim3(256), 0, st, a, p, 3);
        else {
          hipLaunchKernelGGL(lg_planes_kernel<PREC_BF16X3>, pg, dim3(256), 0, st, a, p, 1);
          hipLaunchKernelGGL(lg_planes_kernel<PREC_BF16X3>, pg, dim3(256), 0, st, a, q, 2);
        }
        hipLaunchKernelGGL(lg_gemm_lp_kernel<PREC_BF16X3>, grid, dim3(512), 0, st, a);
      }
    }
    if (hipGetLastError() != hipSuccess) ok = false;
  }

  // the Pade solve of the listed matrices (their denominators and numerators in place)
  void lu(const std::vector<int32_t> &idx, int slot) {
    if (idx.empty() || !ok) return;
    LargeArgs a = base;
    a.list = upload(idx, slot);
    const int np = (int)L.np;
    const unsigned cnt = (unsigned)idx.size();
    const int ct = np / kLargeTile;
    for (int k = 0; k < np && ok; k += kLuNB) {
      if (np <= 1024) hipLaunchKernelGGL(lg_lu_panel_kernel<1>, dim3(cnt), dim3(1024), 0, st, a, k);
      else hipLaunchKernelGGL(lg_lu_panel_kernel<2>, dim3(cnt), dim3(1024), 0, st, a, k);
      hipLaunchKernelGGL(lg_lu_swap_kernel, dim3((unsigned)((2 * np + 255) / 256), cnt), dim3(256), 0, st, a, k);
      const int rest = np - k - kLuNB;
      hipLaunchKernelGGL(lg_lu_fsub_kernel, dim3((unsigned)((rest + np + 255) / 256), cnt), dim3(256), 0, st, a, k);
      if (rest > 0) {
        const int rt = (rest + kLargeTile - 1) / kLargeTile;
        hipLaunchKernelGGL(lg_lu_gemm_kernel, dim3((unsigned)(rt * (rt + ct)), cnt), dim3(512), 0, st, a, k, k,
                           k + kLuNB, np, k + kLuNB);
      }
      if (hipGetLastError() != hipSuccess) ok = false;
    }
    for (int k = np - kLuNB; k >= 0 && ok; k -= kLuNB) {
      hipLaunchKernelGGL(lg_lu_bsub_kernel, dim3((unsigned)((np + 255) / 256), cnt), dim3(256), 0, st, a, k);
      if (k > 0) {
        const int rt = (k + kLargeTile - 1) / kLargeTile;
        hipLaunchKernelGGL(lg_lu_gemm_kernel, dim3((unsigned)(rt * ct), cnt), dim3(512), 0, st, a, k, k, 0, k, np);
      }
      if (hipGetLastError() != hipSuccess) ok = false;
    }
  }

  // triangular refinement of the iterate after squaring round `round` (0: T_m)
  void tri(const std::vector<int32_t> &idx, int slot, int round) {
    if (idx.empty() || !ok) return;
    LargeArgs a = base;
    a.list = upload(idx, slot);
    a.round = round;
    hipLaunchKernelGGL(lg_tri_fix_kernel, dim3((unsigned)((L.n + 255) / 256), (unsigned)idx.size()), dim3(256), 0, st,
                       a);
    if (hipGetLastError() != hipSuccess) ok = false;
  }

  void elem(const std::vector<int32_t> &idx, int slot, int kind, int dst, int coff = 0, int in0 = SEL_NONE) {
    if (idx.empty() || !ok) return;
    LargeArgs a = base;
    a.list = upload(idx, slot);
    a.kind = kind; a.dst = dst; a.in0 = in0;
    a.coff = coff;
    const int64_t blocks = (L.np * L.np * (c.cplx == 2 ? 2 : 1) + 1023) / 1024;
    hipLaunchKernelGGL(lg_elem_kernel, dim3((unsigned)blocks, (unsigned)idx.size()), dim3(256), 0, st, a);
    if (hipGetLastError() != hipSuccess) ok = false;
  }
};

}  // namespace

expm_status_t run_large(const LargeCall &c, hipStream_t st) {
  // real order the kernels run on: the real form for cplx == 1; the complex order itself for
  // the native complex path (cplx == 2, two planes per buffer)
  const int64_t n = c.cplx == 1 ? 2 * c.nin : c.nin;
  const int planes = c.cplx == 2 ? 2 : 1;
  LargeLayout L = large_layout(n, c.batch, c.prec, c.tiles, planes);
  if (!c.ws || c.ws_bytes < L.total) return EXPM_E_WORKSPACE;
  char *base = (char *)c.ws;
  double *bufs = (double *)(base + L.bufs_off);
  double *partial = (double *)(base + L.partial_off);
  unsigned long long *norms = (unsigned long long *)(base + L.norms_off);
  int *flags = (int *)(base + L.flags_off);
  double *coef = (double *)(base + L.coef_off);
  int32_t *lists = (int32_t *)(base + L.list_off);
  int32_t *shift = (int32_t *)(base + L.shift_off);
  int32_t *piv = (int32_t *)(base + L.piv_off);

  LargeArgs a;
  memset(&a, 0, sizeof(a));
  a.ws = bufs;
  a.bstride = (size_t)L.np * L.np * planes;
  a.mstride = kLargeBufs * a.bstride;
  a.np = (int)L.np; a.n = (int)n; a.nin = (int)c.nin; a.cplx = c.cplx;
  a.A = c.A; a.E = c.E;
  a.io_stride = c.nin * c.nin * (c.cplx ? 2 : 1);
  a.m_arr = c.m_out; a.s_arr = c.s_out;
  a.coef = coef;
  a.ps = c.ps;
  a.pade = c.pade;
  a.piv = piv;
  a.flags = flags;
  a.shift = shift;
  a.planes = base + L.planes_off;
  for (int j = 0; j < 5; ++j) a.o[j] = SEL_NONE;
  const unsigned rs_blocks = (unsigned)((L.np * L.np * (c.cplx == 2 ? 2 : 1) + 1023) / 1024);

  std::vector<int32_t> mh, sh;
  for (int64_t g0 = 0; g0 < c.batch; g0 += L.group) {
    const int cnt = (int)std::min<int64_t>(L.group, c.batch - g0);
    a.g0 = g0;
    Launcher run{c, L, a, st, lists};
    run.prec = c.prec;
    std::vector<int32_t> all(cnt);
    for (int i = 0; i < cnt; ++i) all[i] = i;
    // norms (3 per matrix) and non-finite flags start at zero
    hipLaunchKernelGGL(lg_zero_kernel, dim3((unsigned)((3 * L.group + 255) / 256)), dim3(256), 0, st, norms,
                       3 * L.group, flags, L.group);
    hipLaunchKernelGGL(lg_load_kernel, dim3((unsigned)((L.np + 255) / 256), (unsigned)L.nrb, cnt),
                       dim3(256), 0, st, a, partial, (int)L.nrb, flags);
    hipLaunchKernelGGL(lg_colmax_kernel, dim3((unsigned)((L.np + 255) / 256), cnt), dim3(256), 0, st, a, partial, (int)L.nrb,
                       norms, 0);
    if (hipGetLastError() != hipSuccess) return EXPM_E_HIP;
    if (c.sel == EXPM_SEL_ALPHA) {
      // plain choice first: it says which powers the method forms anyway
      hipLaunchKernelGGL(lg_select_kernel, dim3((cnt + 63) / 64), dim3(64), 0, st, a, cnt, (int)L.group, norms,
                         flags, 0, c.k, c.status, coef);
      hipLaunchKernelGGL(lg_rescale_kernel, dim3(rs_blocks, cnt), dim3(256), 0, st, a, 1);
      mh.assign(cnt, 0);
      if (hipMemcpyAsync(mh.data(), c.m_out + g0, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return EXPM_E_HIP;
      std::vector<int32_t> l2, l3;
      for (int i = 0; i < cnt; ++i) {
        if (mh[i] >= 2) l2.push_back(i);
        if (mh[i] >= 12) l3.push_back(i);
      }
      run.gemm(l2, 0, EK_STORE, 0, 0, 1, SEL_NONE, SEL_NONE, {}, 0, true);
      run.gemm(l3, 1, EK_STORE, 1, 0, 2, SEL_NONE, SEL_NONE, {}, 0, true);
      LargeArgs b2 = a;
      if (!l2.empty()) {
        b2.list = run.upload(l2, 2);
        hipLaunchKernelGGL(lg_colsum_kernel, dim3((unsigned)((L.np + 255) / 256), (unsigned)L.nrb, (unsigned)l2.size()),
                           dim3(256), 0, st, b2, 1, partial, (int)L.nrb);
        hipLaunchKernelGGL(lg_colmax_kernel, dim3((unsigned)((L.np + 255) / 256), (unsigned)l2.size()), dim3(256), 0, st, b2,
                           partial, (int)L.nrb, norms + L.group, 1);
      }
      if (!l3.empty()) {
        b2.list = run.upload(l3, 3);
        hipLaunchKernelGGL(lg_colsum_kernel, dim3((unsigned)((L.np + 255) / 256), (unsigned)L.nrb, (unsigned)l3.size()),
                           dim3(256), 0, st, b2, 2, partial, (int)L.nrb);
        hipLaunchKernelGGL(lg_colmax_kernel, dim3((unsigned)((L.np + 255) / 256), (unsigned)l3.size()), dim3(256), 0, st, b2,
                           partial, (int)L.nrb, norms + 2 * L.group, 1);
      }
      // the alpha selection reads norms[group + i] and norms[2 group + i]
      hipLaunchKernelGGL(lg_select_kernel, dim3((cnt + 63) / 64), dim3(64), 0, st, a, cnt, (int)L.group, norms,
                         flags, 1, c.k, c.status, coef);
      if (!c.select_only) hipLaunchKernelGGL(lg_rescale_kernel, dim3(rs_blocks, cnt), dim3(256), 0, st, a, 3);
    } else {
      hipLaunchKernelGGL(lg_select_kernel, dim3((cnt + 63) / 64), dim3(64), 0, st, a, cnt, (int)L.group, norms,
                         flags, 0, c.k, c.status, coef);
      if (!c.select_only) hipLaunchKernelGGL(lg_rescale_kernel, dim3(rs_blocks, cnt), dim3(256), 0, st, a, 1);
    }
    if (hipGetLastError() != hipSuccess || !run.ok) return EXPM_E_HIP;
    mh.assign(cnt, 0);
    sh.assign(cnt, 0);
    if (hipMemcpyAsync(mh.data(), c.m_out + g0, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(sh.data(), c.s_out + g0, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return EXPM_E_HIP;
    if (c.select_only) continue;

    // ---- powers (the alpha path formed them already) ----
    std::vector<int32_t> l2, l3, l4, lm[27], lnan, l0;
    int smax = 0;
    for (int i = 0; i < cnt; ++i) {
      const int m = mh[i];
      if (m < 1) { lnan.push_back(i); continue; }  // non-finite input
      if (c.pade) {  // m = 2m' = 10 or 26
        l2.push_back(i);
        lm[m].push_back(i);
        if (sh[i] == 0) l0.push_back(i);
        smax = std::max(smax, (int)sh[i]);
        continue;
      }
      if (m >= 2) l2.push_back(i);
      if (m >= (c.ps ? 6 : 12)) l3.push_back(i);
      if (c.ps && m == 16) l4.push_back(i);
      lm[m].push_back(i);
      smax = std::max(smax, (int)sh[i]);
    }
    if (c.pade) {
      // eqs. eq.pade10 / eq.pade26: X^2, X^4 (and X^6 for r_26), the inner sums, then the odd
      // part U by the last product, whose epilogue writes the denominator V - U and the
      // numerator V + U; r_26 forms V = X^6 W2 + Z2 and Y = X^6 W1 + Z1 first (U = X Y)
      run.gemm(l2, 0, EK_STORE, 0, 0, 1);
      run.gemm(l2, 1, EK_STORE, 1, 1, 2);
      run.gemm(lm[26], 2, EK_STORE, 2, 1, 3);
      run.elem(l2, 3, LCPADE, SEL_NONE);
      run.gemm(lm[10], 4, EK_PADE, 0, 4, SEL_NONE, 5, SEL_NONE, {6, 7});
      run.gemm(lm[26], 5, EK_ADD1, 3, 4, 1, 5);
      run.gemm(lm[26], 5, EK_ADD1, 3, 6, 2, 7);
      run.gemm(lm[26], 5, EK_PADE, 0, 1, SEL_NONE, 2, SEL_NONE, {4, 5});
      run.lu(l2, 6);
      run.elem(l0, 7, LCCOPY, SEL_TDST, 0, SEL_T);  // no squaring: e^A = r itself
    } else if (c.sel != EXPM_SEL_ALPHA) {
      run.gemm(l2, 0, EK_STORE, 0, 0, 1, SEL_NONE, SEL_NONE, {}, 0, true);
      run.gemm(l3, 1, EK_STORE, 1, 0, 2, SEL_NONE, SEL_NONE, {}, 0, true);
    }
    run.gemm(l4, 20, EK_STORE, 1, 1, 3);  // A^4 = A^2 A^2 (base of the degree-16 rule)
    run.elem(lnan, 1, LCNAN, SEL_NONE);
    std::vector<int32_t> lvalid;
    for (int i = 0; i < cnt; ++i)
      if (mh[i] >= 1) lvalid.push_back(i);
    // ---- product stage per degree (Pade: done above) ----
    run.elem(lm[1], 2, LC1, SEL_TDST);
    run.elem(lm[2], 3, LC2, SEL_TDST);
    run.elem(lm[4], 4, LC4W, 2);
    run.gemm(lm[4], 4, EK_M4, 1, 2, SEL_TDST);
    if (c.ps) {
      // eq. poli9: innermost term F_(r-1) (+ a_16 A^4) into buffer 6, then r - 1 Horner steps
      // R <- F_j + R A^q alternating between buffers 6 and 7; the last one writes T
      for (int m : {6, 9, 12, 16}) {
        const int q = m == 16 ? 4 : 3, r = m / q, qb = q == 4 ? 3 : 2, slot = 21 + q + r;
        run.elem(lm[m], slot, LCPS, 6, 4 * (r - 1));
        int cur = 6;
        for (int j = r - 2; j >= 0; --j) {
          const int dst = j == 0 ? (int)SEL_TDST : (cur == 6 ? 7 : 6);
          run.gemm(lm[m], slot, EK_PSH, cur, qb, dst, SEL_NONE, SEL_NONE, {}, 0, false, 4 * j);
          cur = dst;
        }
      }
    } else {
      run.elem(lm[8], 5, LC8W, 2);
      run.gemm(lm[8], 5, EK_M8A, 1, 2, SEL_NONE, SEL_NONE, SEL_NONE, {3, 4}, 0, true);
      run.gemm(lm[8], 5, EK_M8B, 3, 4, SEL_TDST);
      run.elem(lm[12], 6, LC12, SEL_NONE);
      run.gemm(lm[12], 6, EK_SPLIT2, 6, 6, SEL_NONE, 5, 4, {0, 1}, 0, true);
      run.gemm(lm[12], 6, EK_ADD1, 1, 0, SEL_TDST, 3);
      run.gemm(lm[18], 7, EK_M18A, 2, 2, SEL_NONE, SEL_NONE, SEL_NONE, {3, 4, 5, 6, 7}, 0, true);
      run.gemm(lm[18], 7, EK_SPLIT2, 3, 7, SEL_NONE, 6, 5, {0, 1}, 0, true);
      run.gemm(lm[18], 7, EK_ADD1, 1, 0, SEL_TDST, 4);
    }
    // ---- squarings: round r covers the matrices with s >= r ----
    if (c.tri) run.tri(lvalid, 30, 0);
    for (int r = 1; r <= smax; ++r) {
      std::vector<int32_t> lr;
      for (int i = 0; i < cnt; ++i)
        if (mh[i] >= 1 && sh[i] >= r) lr.push_back(i);
      run.gemm(lr, 8 + (r & 1) * 8, EK_STORE, SEL_SQSRC, SEL_SQSRC, SEL_SQDST, SEL_NONE, SEL_NONE, {}, r);
      if (c.tri) run.tri(lr, 8 + (r & 1) * 8, r);
    }
    if (!run.ok) return EXPM_E_HIP;
    // lists are uploaded asynchronously from host vectors that die here: finish the group
    if (hipStreamSynchronize(st) != hipSuccess) return EXPM_E_HIP;
  }
  return EXPM_OK;
}

}  // namespace expm
