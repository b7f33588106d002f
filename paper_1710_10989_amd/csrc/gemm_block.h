// Workgroup-level FP64 MFMA GEMM for matrices resident in device memory (order np = 16 T,
// T = 1..16): C = P * Q, with a fused elementwise epilogue chosen at run time.
//
// Decomposition (compile time per T).  The output is a T x T grid of 16 x 16 tiles.  The four
// waves form a WR x WC grid; each wave owns a BR x BC block of tiles, so one "chunk" covers
// (WR BR) x (WC BC) tiles and the chunks are walked in row-major order.  A wave whose block
// lies entirely outside the matrix skips the arithmetic (wave-uniform branch); tiles of a
// partially covered block are computed on clamped indices and never stored.
//
// Data path.  For every chunk the K dimension is walked in panels of 16: the P panel
// (chunk rows x 16) and the Q panel (16 x chunk columns) are loaded from global memory into
// registers one panel ahead (software prefetch), written to LDS, and consumed by
// v_mfma_f64_16x16x4_f64.  Per 4-wide k step a wave reads BR A-fragments and BC B-fragments
// from LDS for BR * BC MFMAs.  At the end of the chunk the accumulators are written to an
// LDS copy of the chunk (sharing the panel storage), and the epilogue walks that copy with
// consecutive threads on consecutive columns, so its global reads and writes are coalesced
// and it holds no accumulator registers.
//
// The operands, the epilogue kind and its arguments come from the workgroup's LDS
// descriptor g_ep, filled before the call.  All LDS objects are file-scope __shared__
// variables so every access compiles to ds_read / ds_write even in outlined functions.
//
// MFMA operand layout (gfx950, 16x16x4 f64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l holds D[4 r + l / 16][l % 16].
#pragma once
#include <hip/hip_runtime.h>

namespace expm {

typedef double dbl4 __attribute__((ext_vector_type(4)));
// Pointers read back from the LDS descriptor are generic; casting them to the global address
// space lets the compiler emit global_load / global_store instead of flat accesses.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const double cgdouble;
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const dv2 cgdv2;
__device__ inline gdouble *gptr(double *p) { return (gdouble *)p; }
__device__ inline cgdouble *gptr(const double *p) { return (cgdouble *)p; }

constexpr int kThreads = 256;  // four wave64s
constexpr int kKP = 16;        // K panel width
constexpr int kNpMax = 256;

template <int T> struct TileCfg { static constexpr int WR = 2, WC = 2, BR = 2, BC = 4; };
template <> struct TileCfg<1> { static constexpr int WR = 1, WC = 1, BR = 1, BC = 1; };
template <> struct TileCfg<2> { static constexpr int WR = 2, WC = 2, BR = 1, BC = 1; };
template <> struct TileCfg<3> { static constexpr int WR = 4, WC = 1, BR = 1, BC = 3; };
template <> struct TileCfg<4> { static constexpr int WR = 2, WC = 2, BR = 2, BC = 2; };
template <> struct TileCfg<5> { static constexpr int WR = 4, WC = 1, BR = 1, BC = 5; };
template <> struct TileCfg<6> { static constexpr int WR = 2, WC = 2, BR = 3, BC = 3; };
template <> struct TileCfg<7> { static constexpr int WR = 4, WC = 1, BR = 1, BC = 7; };

// LDS: panels (P <= 96 rows x (16 + 1), Q 16 x (<= 128 + 1)) or, after the K loop, the chunk
// of C (<= 96 x (96 + 1) or 64 x (128 + 1)).  The +1 staggers banks.
constexpr int kLdsP = 96 * (kKP + 1);
constexpr int kLdsQ = kKP * (128 + 1);
constexpr int kLdsC = 96 * 97;
struct GemmPanels {
  double p[kLdsP];
  double q[kLdsQ];
};
union GemmSmem {
  GemmPanels pan;
  double c[kLdsC];
};

// Epilogue kinds.  v is the product element at (row, col); e = row * np + col indexes the
// workspace buffers; "id" is the identity element (1 on the diagonal).
enum EpiKind {
  EK_STORE = 0,   // dst = v
  EK_M4 = 1,      // dst = id + c0 b0 + c1 v                         (T_4)
  EK_M8A = 2,     // a4 = c2 v; o0 = c3 b1 + a4; o1 = c4 id + c5 b0 + c6 b1 + c7 a4   (T_8)
  EK_M8B = 3,     // dst = v + c8 id + c9 b0 + c10 b1               (T_8)
  EK_ADD1 = 4,    // dst = v + in0
  EK_SPLIT2 = 5,  // o0 = v + in0; o1 = o0 + in1
  EK_M18A = 6     // o0..o4 = B_1..B_5 of the degree-18 sequence from (id, b0, b1, b2, v)
};

struct EpiDesc {
  const double *P, *Q;
  const double *b0, *b1, *b2, *in0, *in1;
  double *o[5];
  double *dst;
  int kind, np, dst_ld, dst_nvalid;
  double c[64];
};

__shared__ GemmSmem g_sm;
__shared__ EpiDesc g_ep;

template <class F>
__device__ inline void for_chunk(int row0, int col0, int rows, int cols, int ldc, const F &f) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    const int r = e / cols, cc = e - r * cols;
    f(row0 + r, col0 + cc, g_sm.c[r * ldc + cc]);
  }
}

__device__ inline void run_epilogue(int row0, int col0, int rows, int cols, int ldc) {
  const int np = g_ep.np;
  const double *c = g_ep.c;
  switch (g_ep.kind) {
    case EK_STORE: {
      gdouble *dst = gptr(g_ep.dst);
      const int ld = g_ep.dst_ld, nv = g_ep.dst_nvalid;
      for_chunk(row0, col0, rows, cols, ldc, [&](int r, int cc, double v) {
        if (r < nv && cc < nv) dst[(size_t)r * ld + cc] = v;
      });
    } break;
    case EK_M4: {
      gdouble *dst = gptr(g_ep.dst);
      const int ld = g_ep.dst_ld, nv = g_ep.dst_nvalid;
      cgdouble *b0 = gptr(g_ep.b0);
      const double c0 = c[0], c1 = c[1];
      for_chunk(row0, col0, rows, cols, ldc, [&](int r, int cc, double v) {
        const size_t e = (size_t)r * np + cc;
        const double t = (r == cc ? 1.0 : 0.0) + c0 * b0[e] + c1 * v;
        if (r < nv && cc < nv) dst[(size_t)r * ld + cc] = t;
      });
    } break;
    case EK_M8A: {
      cgdouble *b0 = gptr(g_ep.b0), *b1 = gptr(g_ep.b1);
      gdouble *o0 = gptr(g_ep.o[0]), *o1 = gptr(g_ep.o[1]);
      const double c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5], c6 = c[6], c7 = c[7];
      for_chunk(row0, col0, rows, cols, ldc, [&](int r, int cc, double v) {
        const size_t e = (size_t)r * np + cc;
        const double a4 = c2 * v, x2 = b1[e];
        o0[e] = c3 * x2 + a4;
        o1[e] = (r == cc ? c4 : 0.0) + c5 * b0[e] + c6 * x2 + c7 * a4;
      });
    } break;
    case EK_M8B: {
      gdouble *dst = gptr(g_ep.dst);
      const int ld = g_ep.dst_ld, nv = g_ep.dst_nvalid;
      cgdouble *b0 = gptr(g_ep.b0), *b1 = gptr(g_ep.b1);
      const double c8 = c[8], c9 = c[9], c10 = c[10];
      for_chunk(row0, col0, rows, cols, ldc, [&](int r, int cc, double v) {
        const size_t e = (size_t)r * np + cc;
        const double t = v + (r == cc ? c8 : 0.0) + c9 * b0[e] + c10 * b1[e];
        if (r < nv && cc < nv) dst[(size_t)r * ld + cc] = t;
      });
    } break;
    case EK_ADD1: {
      gdouble *dst = gptr(g_ep.dst);
      const int ld = g_ep.dst_ld, nv = g_ep.dst_nvalid;
      cgdouble *in0 = gptr(g_ep.in0);
      for_chunk(row0, col0, rows, cols, ldc, [&](int r, int cc, double v) {
        const size_t e = (size_t)r * np + cc;
        const double t = v + in0[e];
        if (r < nv && cc < nv) dst[(size_t)r * ld + cc] = t;
      });
    } break;
    case EK_SPLIT2: {
      cgdouble *in0 = gptr(g_ep.in0), *in1 = gptr(g_ep.in1);
      gdouble *o0 = gptr(g_ep.o[0]), *o1 = gptr(g_ep.o[1]);
      for_chunk(row0, col0, rows, cols, ldc, [&](int r, int cc, double v) {
        const size_t e = (size_t)r * np + cc;
        const double t = v + in0[e];
        o0[e] = t;
        o1[e] = t + in1[e];
      });
    } break;
    case EK_M18A: {
      cgdouble *b0 = gptr(g_ep.b0), *b1 = gptr(g_ep.b1), *b2 = gptr(g_ep.b2);
      gdouble *o0 = gptr(g_ep.o[0]), *o1 = gptr(g_ep.o[1]), *o2 = gptr(g_ep.o[2]), *o3 = gptr(g_ep.o[3]), *o4 = gptr(g_ep.o[4]);
      for_chunk(row0, col0, rows, cols, ldc, [&](int r, int cc, double v) {
        const size_t e = (size_t)r * np + cc;
        const double id = (r == cc) ? 1.0 : 0.0;
        const double x1 = b0[e], x2 = b1[e], x3 = b2[e];
        o0[e] = c[0] * id + c[1] * x1 + c[2] * x2 + c[3] * x3;
        o1[e] = c[4] * id + c[5] * x1 + c[6] * x2 + c[7] * x3 + c[8] * v;
        o2[e] = c[9] * id + c[10] * x1 + c[11] * x2 + c[12] * x3 + c[13] * v;
        o3[e] = c[14] * id + c[15] * x1 + c[16] * x2 + c[17] * x3 + c[18] * v;
        o4[e] = c[19] * id + c[20] * x1 + c[21] * x2 + c[22] * x3 + c[23] * v;
      });
    } break;
  }
}

template <int T>
__device__ __noinline__ void gemm_t() {
  typedef TileCfg<T> C;
  constexpr int np = 16 * T;
  constexpr int CR = C::WR * C::BR, CC = C::WC * C::BC;   // chunk size in tiles
  constexpr int PROWS = CR * 16, QCOLS = CC * 16;
  constexpr int LDP = kKP + 1, LDQ = QCOLS + 1, LDC = QCOLS + 1;
  constexpr int PPT = (PROWS * 8 + kThreads - 1) / kThreads;  // P double2 per thread
  constexpr int QPT = (QCOLS * 8 + kThreads - 1) / kThreads;  // Q double2 per thread
  constexpr int NPAN = np / kKP;
  constexpr int TPW = C::BR * C::BC;
  static_assert(PROWS <= 96 && QCOLS <= 128 && PROWS * LDC <= kLdsC, "chunk exceeds LDS budget");

  cgdouble *__restrict__ P = gptr(g_ep.P);
  cgdouble *__restrict__ Q = gptr(g_ep.Q);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const bool has_block = wave < C::WR * C::WC;
  const int wr = wave / C::WC, wc = wave % C::WC;

#pragma unroll 1
  for (int cr0 = 0; cr0 < T; cr0 += CR) {
#pragma unroll 1
    for (int cc0 = 0; cc0 < T; cc0 += CC) {
      const int br0 = cr0 + wr * C::BR, bc0 = cc0 + wc * C::BC;
      const bool active = has_block && br0 < T && bc0 < T;
      dbl4 acc[TPW];
#pragma unroll
      for (int i = 0; i < TPW; ++i) acc[i] = dbl4{0.0, 0.0, 0.0, 0.0};
      int aoff[C::BR], boff[C::BC];
#pragma unroll
      for (int i = 0; i < C::BR; ++i) aoff[i] = ((br0 - cr0 + i) * 16 + lr) * LDP + lk;
#pragma unroll
      for (int j = 0; j < C::BC; ++j) boff[j] = lk * LDQ + (bc0 - cc0 + j) * 16 + lr;

      dv2 rp[PPT], rq[QPT];
      auto load_panel = [&](int kp) {
        const int k0 = kp * kKP;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
          const int idx = tid + i * kThreads;
          const int r = idx >> 3, c2 = idx & 7;
          if (idx < PROWS * 8 && cr0 * 16 + r < np)
            rp[i] = *reinterpret_cast<cgdv2 *>(P + (size_t)(cr0 * 16 + r) * np + k0 + 2 * c2);
        }
#pragma unroll
        for (int i = 0; i < QPT; ++i) {
          const int idx = tid + i * kThreads;
          const int r = idx / (QCOLS / 2), c2 = idx % (QCOLS / 2);
          if (idx < QCOLS * 8 && cc0 * 16 + 2 * c2 < np)
            rq[i] = *reinterpret_cast<cgdv2 *>(Q + (size_t)(k0 + r) * np + cc0 * 16 + 2 * c2);
        }
      };
      auto store_panel = [&]() {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
          const int idx = tid + i * kThreads;
          const int r = idx >> 3, c2 = idx & 7;
          if (idx < PROWS * 8 && cr0 * 16 + r < np) {
            g_sm.pan.p[r * LDP + 2 * c2] = rp[i].x;
            g_sm.pan.p[r * LDP + 2 * c2 + 1] = rp[i].y;
          }
        }
#pragma unroll
        for (int i = 0; i < QPT; ++i) {
          const int idx = tid + i * kThreads;
          const int r = idx / (QCOLS / 2), c2 = idx % (QCOLS / 2);
          if (idx < QCOLS * 8 && cc0 * 16 + 2 * c2 < np) {
            g_sm.pan.q[r * LDQ + 2 * c2] = rq[i].x;
            g_sm.pan.q[r * LDQ + 2 * c2 + 1] = rq[i].y;
          }
        }
      };

      load_panel(0);
#pragma unroll 1
      for (int kp = 0; kp < NPAN; ++kp) {
        __syncthreads();  // previous panel (or previous chunk's C copy) consumed
        store_panel();
        __syncthreads();
        if (kp + 1 < NPAN) load_panel(kp + 1);
        if (active) {
#pragma unroll
          for (int kk = 0; kk < kKP; kk += 4) {
            double a[C::BR], b[C::BC];
#pragma unroll
            for (int i = 0; i < C::BR; ++i) a[i] = g_sm.pan.p[aoff[i] + kk];
#pragma unroll
            for (int j = 0; j < C::BC; ++j) b[j] = g_sm.pan.q[boff[j] + kk * LDQ];
#pragma unroll
            for (int i = 0; i < C::BR; ++i)
#pragma unroll
              for (int j = 0; j < C::BC; ++j)
                acc[i * C::BC + j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i * C::BC + j], 0, 0, 0);
          }
        }
      }
      __syncthreads();  // panels consumed: the chunk copy of C reuses their storage
      if (active) {
#pragma unroll
        for (int i = 0; i < C::BR; ++i)
#pragma unroll
          for (int j = 0; j < C::BC; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              g_sm.c[((br0 - cr0 + i) * 16 + 4 * r + lk) * LDC + (bc0 - cc0 + j) * 16 + lr] = acc[i * C::BC + j][r];
      }
      __syncthreads();
      const int rows = ((T - cr0) < CR ? (T - cr0) : CR) * 16;
      const int cols = ((T - cc0) < CC ? (T - cc0) : CC) * 16;
      run_epilogue(cr0 * 16, cc0 * 16, rows, cols, LDC);
    }
  }
  __syncthreads();  // outputs visible to the whole workgroup before the next step
}

// C = P * Q with the epilogue described by g_ep (np = g_ep.np, a multiple of 16, <= 256).
__device__ inline void gemm_block() {
  switch (g_ep.np >> 4) {
    case 1: gemm_t<1>(); break;
    case 2: gemm_t<2>(); break;
    case 3: gemm_t<3>(); break;
    case 4: gemm_t<4>(); break;
    case 5: gemm_t<5>(); break;
    case 6: gemm_t<6>(); break;
    case 7: gemm_t<7>(); break;
    case 8: gemm_t<8>(); break;
    case 9: gemm_t<9>(); break;
    case 10: gemm_t<10>(); break;
    case 11: gemm_t<11>(); break;
    case 12: gemm_t<12>(); break;
    case 13: gemm_t<13>(); break;
    case 14: gemm_t<14>(); break;
    case 15: gemm_t<15>(); break;
    default: gemm_t<16>(); break;
  }
}

}  // namespace expm
