// Workgroup-level FP64 GEMM for matrices resident in device memory (order np = 16 T,
// T = 1..16): C = P * Q, followed by a fused elementwise epilogue chosen at run time.
//
// Two workgroup shapes share the code: NW = 4 waves (orders up to 64, several workgroups
// per CU) and NW = 8 waves (orders 80..256, one workgroup per CU, chunks of 96 x 128 or
// 128 x 128).  For each
// order class T the chunk and wave decomposition is fixed at compile time (TileFor); the
// K loop is the direct-to-LDS pipeline of tile_gemm.h.
//
// Epilogues.  A plain product (EK_STORE) is stored from the accumulators: lanes 0..15 of a
// register cover 16 consecutive columns of one row.  Every other kind first copies the chunk
// of C into LDS and then walks it with consecutive threads on consecutive columns; each thread
// gathers the global inputs of 8 elements before computing, so the loads overlap.
//
// The operands, the epilogue kind and its arguments come from the LDS descriptor g_ep, filled
// by thread 0 before the call.  LDS objects are file-scope so every access stays ds_*.
#pragma once
#include <hip/hip_runtime.h>

#include "tile_gemm.h"

namespace expm {

constexpr int kNpMax = 256;

// Epilogue kinds.  v is the product element at (row, col); e = row * np + col indexes the
// workspace buffers; "id" is the identity element (1 on the diagonal).
enum EpiKind {
  EK_STORE = 0,   // dst = v
  EK_M4 = 1,      // dst = id + c0 b0 + c1 v                         (T_4)
  EK_M8A = 2,     // a4 = c2 v; o0 = c3 b1 + a4; o1 = c4 id + c5 b0 + c6 b1 + c7 a4   (T_8)
  EK_M8B = 3,     // dst = v + c8 id + c9 b0 + c10 b1               (T_8)
  EK_ADD1 = 4,    // dst = v + in0
  EK_SPLIT2 = 5,  // o0 = v + in0; o1 = o0 + in1
  EK_M18A = 6,    // o0..o4 = B_1..B_5 of the degree-18 sequence from (id, b0, b1, b2, v)
  EK_PSH = 7,     // dst = v + c0 id + c1 b0 + c2 b1 + c3 b2   (a Horner step of eq. poli9)
  EK_PADE = 8     // o0 = in0 - v, o1 = in0 + v: with v = U, in0 = V the denominator V - U and the
                  // numerator V + U of the diagonal Pade approximant (eq. eq.pade26)
};

struct EpiDesc {
  const double *P, *Q;
  const double *b0, *b1, *b2, *in0, *in1;
  double *o[5];
  double *dst;
  int kind, np, dst_ld, dst_nvalid;
  int cplx;  // 1: dst is an interleaved complex n x n matrix (n = dst_nvalid) holding the
             // realified result: rows 0..n-1 carry the real part, rows n..2n-1 the imaginary;
             // 2: dst points at the real or imaginary member of an interleaved complex n x n
             // matrix, and the result is that part (a plane of the native complex path)
  double idw;  // weight of the identity terms (1; 0 for the imaginary plane of a complex step)
  double c[64];
};

// Store of one element of a result to the destination described by (dst, ld, nv, cplx).
// Real: element (r, c) of the leading nv x nv block.  Complex (realified 2nv x 2nv matrix
// [[Re, -Im], [Im, Re]]): column c < nv of the upper half is Re, of the lower half Im.
__device__ inline void put_dst(gdouble *dst, int ld, int nv, int cplx, int r, int c, double v) {
  if (!cplx) {
    if (r < nv && c < nv) dst[r * ld + c] = v;
  } else if (cplx == 2) {
    if (r < nv && c < nv) dst[2 * (r * nv + c)] = v;
  } else if (c < nv) {
    if (r < nv) dst[2 * (r * nv + c)] = v;
    else if (r < 2 * nv) dst[2 * ((r - nv) * nv + c) + 1] = v;
  }
}

__shared__ EpiDesc g_ep;

// Decomposition per (waves, order class).
template <int NW, int T> struct TileFor;
template <> struct TileFor<4, 1> { typedef TileShape<4, 16, 16, 1, 1, 1, 1> S; };
template <> struct TileFor<4, 2> { typedef TileShape<4, 32, 32, 2, 2, 1, 1> S; };
template <> struct TileFor<4, 3> { typedef TileShape<4, 48, 48, 3, 1, 1, 3> S; };
template <> struct TileFor<4, 4> { typedef TileShape<4, 64, 64, 2, 2, 2, 2> S; };
template <int T> struct TileFor<8, T> { typedef TileShape<8, 128, 128, 4, 2, 2, 4> S; };
template <> struct TileFor<8, 5> { typedef TileShape<8, 96, 128, 2, 4, 3, 2> S; };
template <> struct TileFor<8, 6> { typedef TileShape<8, 96, 128, 2, 4, 3, 2> S; };

// LDS pools: the stage ring, reused after the K loop as the chunk copy of C.
constexpr int kPool4 = 3 * (64 * 16 + 16 * 64);  // 3 stages of 64 x 16 + 16 x 64; >= 64 x (64 + 1)
constexpr int kPool8 = 128 * 129;   // >= 3 stages of 128 x 16 + 16 x 128, >= 128 x (128 + 1)
__shared__ double g_pool4[kPool4];
__shared__ double g_pool8[kPool8];
template <int NW> __device__ inline double *lds_pool() {
  if constexpr (NW == 4) return g_pool4;
  else return g_pool8;
}

// Walks the LDS copy of a chunk (ld ldc) with consecutive threads on consecutive columns.
// Each thread gathers the NIN global inputs of kEpiU elements before computing.
constexpr int kEpiU = 8;

template <int NW, int NIN, class F>
__device__ inline void for_chunk(const double *cbuf, int row0, int col0, int rows, int cols, int ldc,
                                 int np, cgdouble *const (&in)[NIN > 0 ? NIN : 1], const F &f) {
  constexpr int NT = 64 * NW;
  const int total = rows * cols;
  for (int base = threadIdx.x; base < total; base += NT * kEpiU) {
    double v[kEpiU], x[kEpiU][NIN > 0 ? NIN : 1];
    int rr[kEpiU], cc[kEpiU];
#pragma unroll
    for (int u = 0; u < kEpiU; ++u) {
      const int e = base + u * NT;
      rr[u] = -1;
      if (e < total) {
        const int r = e / cols, c = e - r * cols;
        rr[u] = row0 + r;
        cc[u] = col0 + c;
        v[u] = cbuf[r * ldc + c];
        const int g = rr[u] * np + cc[u];
#pragma unroll
        for (int k = 0; k < NIN; ++k) x[u][k] = in[k][g];
      }
    }
#pragma unroll
    for (int u = 0; u < kEpiU; ++u)
      if (rr[u] >= 0) f(rr[u], cc[u], rr[u] * np + cc[u], v[u], x[u]);
  }
}

template <int NW>
__device__ inline void run_epilogue(const double *cbuf, int row0, int col0, int rows, int cols, int ldc) {
  const int np = g_ep.np;
  const double *c = g_ep.c;
  const double idw = g_ep.idw;
  switch (g_ep.kind) {
    case EK_M4: {
      gdouble *dst = gptr(g_ep.dst);
      const int ld = g_ep.dst_ld, nv = g_ep.dst_nvalid, cx = g_ep.cplx;
      const double c0 = c[0], c1 = c[1];
      cgdouble *const in[1] = {gptr(g_ep.b0)};
      for_chunk<NW, 1>(cbuf, row0, col0, rows, cols, ldc, np, in, [&](int r, int cc, int, double v, const double *x) {
        const double t = (r == cc ? idw : 0.0) + c0 * x[0] + c1 * v;
        put_dst(dst, ld, nv, cx, r, cc, t);
      });
    } break;
    case EK_M8A: {
      gdouble *o0 = gptr(g_ep.o[0]), *o1 = gptr(g_ep.o[1]);
      const double c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5], c6 = c[6], c7 = c[7];
      cgdouble *const in[2] = {gptr(g_ep.b0), gptr(g_ep.b1)};
      for_chunk<NW, 2>(cbuf, row0, col0, rows, cols, ldc, np, in, [&](int r, int cc, int e, double v, const double *x) {
        const double a4 = c2 * v;
        o0[e] = c3 * x[1] + a4;
        o1[e] = (r == cc ? c4 * idw : 0.0) + c5 * x[0] + c6 * x[1] + c7 * a4;
      });
    } break;
    case EK_M8B: {
      gdouble *dst = gptr(g_ep.dst);
      const int ld = g_ep.dst_ld, nv = g_ep.dst_nvalid, cx = g_ep.cplx;
      const double c8 = c[8], c9 = c[9], c10 = c[10];
      cgdouble *const in[2] = {gptr(g_ep.b0), gptr(g_ep.b1)};
      for_chunk<NW, 2>(cbuf, row0, col0, rows, cols, ldc, np, in, [&](int r, int cc, int, double v, const double *x) {
        const double t = v + (r == cc ? c8 * idw : 0.0) + c9 * x[0] + c10 * x[1];
        put_dst(dst, ld, nv, cx, r, cc, t);
      });
    } break;
    case EK_ADD1: {
      gdouble *dst = gptr(g_ep.dst);
      const int ld = g_ep.dst_ld, nv = g_ep.dst_nvalid, cx = g_ep.cplx;
      cgdouble *const in[1] = {gptr(g_ep.in0)};
      for_chunk<NW, 1>(cbuf, row0, col0, rows, cols, ldc, np, in, [&](int r, int cc, int, double v, const double *x) {
        const double t = v + x[0];
        put_dst(dst, ld, nv, cx, r, cc, t);
      });
    } break;
    case EK_SPLIT2: {
      gdouble *o0 = gptr(g_ep.o[0]), *o1 = gptr(g_ep.o[1]);
      cgdouble *const in[2] = {gptr(g_ep.in0), gptr(g_ep.in1)};
      for_chunk<NW, 2>(cbuf, row0, col0, rows, cols, ldc, np, in, [&](int, int, int e, double v, const double *x) {
        const double t = v + x[0];
        o0[e] = t;
        o1[e] = t + x[1];
      });
    } break;
    case EK_M18A: {
      gdouble *o0 = gptr(g_ep.o[0]), *o1 = gptr(g_ep.o[1]), *o2 = gptr(g_ep.o[2]), *o3 = gptr(g_ep.o[3]),
              *o4 = gptr(g_ep.o[4]);
      double k[24];
#pragma unroll
      for (int i = 0; i < 24; ++i) k[i] = c[i];
      cgdouble *const in[3] = {gptr(g_ep.b0), gptr(g_ep.b1), gptr(g_ep.b2)};
      for_chunk<NW, 3>(cbuf, row0, col0, rows, cols, ldc, np, in, [&](int r, int cc, int e, double v, const double *x) {
        const double id = (r == cc) ? idw : 0.0;
        const double x1 = x[0], x2 = x[1], x3 = x[2];
        o0[e] = k[0] * id + k[1] * x1 + k[2] * x2 + k[3] * x3;
        o1[e] = k[4] * id + k[5] * x1 + k[6] * x2 + k[7] * x3 + k[8] * v;
        o2[e] = k[9] * id + k[10] * x1 + k[11] * x2 + k[12] * x3 + k[13] * v;
        o3[e] = k[14] * id + k[15] * x1 + k[16] * x2 + k[17] * x3 + k[18] * v;
        o4[e] = k[19] * id + k[20] * x1 + k[21] * x2 + k[22] * x3 + k[23] * v;
      });
    } break;
    case EK_PSH: {
      gdouble *dst = gptr(g_ep.dst);
      const int ld = g_ep.dst_ld, nv = g_ep.dst_nvalid, cx = g_ep.cplx;
      const double c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3];
      cgdouble *const in[3] = {gptr(g_ep.b0), gptr(g_ep.b1), gptr(g_ep.b2)};
      for_chunk<NW, 3>(cbuf, row0, col0, rows, cols, ldc, np, in, [&](int r, int cc, int, double v, const double *x) {
        const double t = v + (r == cc ? c0 * idw : 0.0) + c1 * x[0] + c2 * x[1] + c3 * x[2];
        put_dst(dst, ld, nv, cx, r, cc, t);
      });
    } break;
    case EK_PADE: {
      gdouble *o0 = gptr(g_ep.o[0]), *o1 = gptr(g_ep.o[1]);
      cgdouble *const in[1] = {gptr(g_ep.in0)};
      for_chunk<NW, 1>(cbuf, row0, col0, rows, cols, ldc, np, in, [&](int, int, int e, double v, const double *x) {
        o0[e] = x[0] - v;
        o1[e] = x[0] + v;
      });
    } break;
    default: break;
  }
}

// Plain product: each lane stores its accumulators to the g_ep destination (lanes 0..15 of
// a register cover 16 consecutive columns of one row).  (row0, col0): the wave's block.
template <class S, int PREC = PREC_F64>
__device__ inline void store_acc(const typename AccOf<PREC>::T (&acc)[S::TPW], int row0, int col0) {
  gdouble *dst = gptr(g_ep.dst);
  int ld = g_ep.dst_ld;
  const int nv = g_ep.dst_nvalid, cx = g_ep.cplx;
  asm volatile("" : "+v"(ld));  // keep the store addresses out of the K loop
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < S::BR; ++i)
#pragma unroll
    for (int j = 0; j < S::BC; ++j) {
      const int col = col0 + j * 16 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + i * 16 + (PREC == PREC_F64 ? 4 * r + lk : 4 * lk + r);
        put_dst(dst, ld, nv, cx, row, col, (double)acc[i * S::BC + j][r]);
      }
    }
}

// Stages the wave's accumulators into the chunk copy (ld LDC) at chunk-relative (r0, c0).
template <class S, int LDC, int PREC = PREC_F64>
__device__ inline void stage_acc(double *cbuf, const typename AccOf<PREC>::T (&acc)[S::TPW], int r0, int c0) {
  const int lane = threadIdx.x & 63;
  int lrow = lane >> 4;
  asm volatile("" : "+v"(lrow));
  const int lr = lane & 15;
#pragma unroll
  for (int i = 0; i < S::BR; ++i)
#pragma unroll
    for (int j = 0; j < S::BC; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        cbuf[(r0 + i * 16 + (PREC == PREC_F64 ? 4 * r + lrow : 4 * lrow + r)) * LDC + c0 + j * 16 + lr] =
            (double)acc[i * S::BC + j][r];
}

template <int NW, int T>
__device__ __noinline__ void gemm_t() {
  typedef typename TileFor<NW, T>::S S;
  constexpr int np = 16 * T;
  constexpr int LDC = S::BN + 1;
  static_assert(3 * (S::P_STAGE + S::Q_STAGE) <= (NW == 4 ? kPool4 : kPool8), "stage ring exceeds pool");
  static_assert(S::BM * LDC <= (NW == 4 ? kPool4 : kPool8), "chunk copy exceeds pool");
  TileLds<S> &L = *reinterpret_cast<TileLds<S> *>(lds_pool<NW>());
  cgdouble *P = gptr(g_ep.P);
  cgdouble *Q = gptr(g_ep.Q);
  const int wave = threadIdx.x >> 6;
  const bool has_block = wave < S::WR * S::WC;
  const int wr = wave / S::WC, wc = wave % S::WC;
  const int kind = g_ep.kind;

#pragma unroll 1
  for (int m0 = 0; m0 < np; m0 += S::BM) {
#pragma unroll 1
    for (int n0 = 0; n0 < np; n0 += S::BN) {
      const int wr_row = wr * S::BR * 16, wc_col = wc * S::BC * 16;  // within the chunk
      const bool active = has_block && m0 + wr_row < np && n0 + wc_col < np;
      dbl4 acc[S::TPW];
      tile_gemm<S>(P, np, Q, np, np, np, np, m0, n0, L, active, wr_row, wc_col, acc);
      if (kind == EK_STORE) {
        if (active) store_acc<S>(acc, m0 + wr_row, n0 + wc_col);
        __syncthreads();  // the next chunk's loads reuse the stage ring
        continue;
      }
      __syncthreads();  // stage ring retired: it becomes the chunk copy of C
      double *cbuf = lds_pool<NW>();
      if (active) stage_acc<S, LDC>(cbuf, acc, wr_row, wc_col);
      __syncthreads();
      const int rows = (np - m0) < S::BM ? (np - m0) : S::BM;
      const int cols = (np - n0) < S::BN ? (np - n0) : S::BN;
      run_epilogue<NW>(cbuf, m0, n0, rows, cols, LDC);
      __syncthreads();  // chunk copy consumed before the next chunk's loads
    }
  }
}

// C = P * Q with the epilogue described by g_ep (np = g_ep.np).  NW = 4 serves np <= 64,
// NW = 8 serves np in 80..256.
template <int NW>
__device__ inline void gemm_block() {
  const int t = g_ep.np >> 4;
  if constexpr (NW == 4) {
    switch (t) {
      case 1: gemm_t<4, 1>(); break;
      case 2: gemm_t<4, 2>(); break;
      case 3: gemm_t<4, 3>(); break;
      default: gemm_t<4, 4>(); break;
    }
  } else {
    switch (t) {
      case 5: gemm_t<8, 5>(); break;
      case 6: gemm_t<8, 6>(); break;
      case 7: gemm_t<8, 7>(); break;
      case 8: gemm_t<8, 8>(); break;
      case 9: gemm_t<8, 9>(); break;
      case 10: gemm_t<8, 10>(); break;
      case 11: gemm_t<8, 11>(); break;
      case 12: gemm_t<8, 12>(); break;
      case 13: gemm_t<8, 13>(); break;
      case 14: gemm_t<8, 14>(); break;
      case 15: gemm_t<8, 15>(); break;
      default: gemm_t<8, 16>(); break;
    }
  }
}

}  // namespace expm
