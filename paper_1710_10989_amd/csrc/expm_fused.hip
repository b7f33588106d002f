// Persistent fused kernels: e^A for matrices of order n <= 256, one workgroup per matrix.
//
// Each workgroup pops matrices from a device work queue (largest order first, then largest
// cost estimate first) and runs the whole method for it: copy A into a zero-padded np x np
// buffer (np = n rounded up to 16) while taking the 1-norm, choose (m, s), form the powers
// A^2, A^3 with MFMA GEMMs, build the linear combinations of the product-reduced sequence in
// GEMM epilogues, run the product stage and the s squarings, and write e^A.  Zero padding is
// exact: every polynomial in the padded matrix is block diagonal, so the leading n x n block
// is p(A).
//
// Scaling (Sec. 1, eq. eses): X^k = 2^(-sk) A^k goes into the coefficients of the linear
// combinations, so the stored powers are those of A, with no pass over a matrix, whenever no
// power up to the sixth can overflow (||A||_1 <= 2^150).  Above that the matrix is scaled once
// its 1-norm is known, to X_p = 2^(-s_p) A with s_p the plain rule's s (exact), and only the
// difference between the chosen s and s_p goes into the coefficients (or, when that difference
// is extreme, into the matrices).
//
// Two instantiations: 8 waves (orders 80..256, one workgroup per CU) take the front of the
// queue, 4 waves (orders up to 64, two workgroups per CU) take the rest.
//
// Workspace: one slot of 8 np_max^2 doubles per resident workgroup; a matrix of order n uses
// the first 8 np^2 doubles of its workgroup's slot.
#include <hip/hip_runtime.h>
#include <math.h>

#include "expm_fused.h"
#include "expm_internal.h"
#include "coefs.h"
#include "gemm_block.h"
#include "mlp.h"

namespace expm {

// Learned selector state: MLP parameters, feature normalisation (mean[8], std[8]) and the
// accepted / rejected proposal counters.
__device__ float g_mlp_params[kMlpParams];
__device__ double g_mlp_norm[2 * kMlpIn];
__device__ unsigned long long g_learned_counts[2];

namespace {

constexpr int kBufs = kFusedBufs;
__shared__ int sh_ms[2];
__shared__ float sh_mlp[8 + 64 + 64 + 16];

// Column sums of |B| over an np x np buffer (thread j owns column j), reduced to the maximum.
template <int NT>
__device__ double block_norm1(const double *B, int np, double *red) {
  const int tid = threadIdx.x;
  double s = 0.0;
  if (tid < np) {
    cgdouble *Bg = gptr(B);
    for (int i = 0; i < np; i += 16) {  // np is a multiple of 16: 16 loads in flight
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = Bg[(i + u) * np + tid];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += fabs(v[u]);
    }
  }
  red[tid] = s;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Trace of an np x np buffer.
template <int NT>
__device__ double block_trace(const double *B, int np, double *red) {
  const int tid = threadIdx.x;
  red[tid] = tid < np ? B[tid * np + tid] : 0.0;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// ||B - B^T||_1 of an np x np buffer (thread j owns column j).  Per block of 16 rows a thread
// issues 16 coalesced column loads and reads the 16 mirror elements of its own row as eight
// contiguous 16-byte loads, all before accumulating.
template <int NT>
__device__ double block_asym1(const double *B, int np, double *red) {
  const int tid = threadIdx.x;
  double s = 0.0;
  if (tid < np) {
    cgdouble *Bg = gptr(B);
    for (int i = 0; i < np; i += 16) {
      double col[16];
      dv2 row[8];
#pragma unroll
      for (int u = 0; u < 16; ++u) col[u] = Bg[(i + u) * np + tid];
#pragma unroll
      for (int u = 0; u < 8; ++u) row[u] = *reinterpret_cast<cgdv2 *>(Bg + tid * np + i + 2 * u);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s += fabs(col[2 * u] - row[u].x);
        s += fabs(col[2 * u + 1] - row[u].y);
      }
    }
  }
  red[tid] = s;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// The learned selector's 8 raw features from ||A||, ||A^2||, tr A, ||A - A^T||, n:
// log2 d_1 .. log2 d_5 (d_3..d_5 by their submultiplicative bounds), log2 n,
// |tr A| / ||A||_1, ||A - A^T||_1 / (2 ||A||_1).
__device__ inline void learned_features(double n1, double n2, double tr, double asym, int n, double *f) {
  double d[5];
  alpha_d(n1, n2, -1.0, d);
  for (int k = 0; k < 5; ++k) f[k] = log2(fmax(d[k], 1e-300));
  f[5] = log2((double)n);
  f[6] = n1 > 0.0 ? fabs(tr) / n1 : 0.0;
  f[7] = n1 > 0.0 ? asym / (2.0 * n1) : 0.0;
}

// MLP inference (weights in g_mlp_params, feature normalisation in g_mlp_norm); returns the
// proposed class.  Threads 0..63 evaluate the hidden units.
template <int NT>
__device__ int mlp_infer(double n1, double n2, double tr, double asym, int n) {
  const int tid = threadIdx.x;
  const float *W = g_mlp_params;
  if (tid == 0) {
    double f[8];
    learned_features(n1, n2, tr, asym, n, f);
    for (int k = 0; k < kMlpIn; ++k) sh_mlp[k] = (float)((f[k] - g_mlp_norm[k]) / g_mlp_norm[kMlpIn + k]);
  }
  __syncthreads();
  if (tid < kMlpH) {
    float acc = W[kMlpB1 + tid];
    for (int k = 0; k < kMlpIn; ++k) acc += W[kMlpW1 + tid * kMlpIn + k] * sh_mlp[k];
    sh_mlp[8 + tid] = fmaxf(acc, 0.0f);
  }
  __syncthreads();
  if (tid < kMlpH) {
    float acc = W[kMlpB2 + tid];
    for (int k = 0; k < kMlpH; ++k) acc += W[kMlpW2 + tid * kMlpH + k] * sh_mlp[8 + k];
    sh_mlp[72 + tid] = fmaxf(acc, 0.0f);
  }
  __syncthreads();
  if (tid < kMlpOut) {
    float acc = W[kMlpB3 + tid];
    for (int k = 0; k < kMlpH; ++k) acc += W[kMlpW3 + tid * kMlpH + k] * sh_mlp[72 + k];
    sh_mlp[136 + tid] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    int best = 0;
    for (int c = 1; c < kMlpOut; ++c)
      if (sh_mlp[136 + c] > sh_mlp[136 + best]) best = c;
    sh_ms[0] = best;
  }
  __syncthreads();
  const int cls = sh_ms[0];
  __syncthreads();
  return cls;
}

// Elementwise pass over the np x np index space: each thread gathers the NIN inputs of
// kEpiU elements before computing, then calls f(row, col, e, x).
template <int NT, int NIN, class F>
__device__ void for_each_elem(int np, const double *const (&inp)[NIN], const F &f) {
  const int total = np * np;
  cgdouble *in[NIN];
#pragma unroll
  for (int k = 0; k < NIN; ++k) in[k] = gptr(inp[k]);
  for (int base = threadIdx.x; base < total; base += NT * kEpiU) {
    double x[kEpiU][NIN];
#pragma unroll
    for (int u = 0; u < kEpiU; ++u) {
      const int e = base + u * NT;
      if (e < total) {
#pragma unroll
        for (int k = 0; k < NIN; ++k) x[u][k] = in[k][e];
      }
    }
#pragma unroll
    for (int u = 0; u < kEpiU; ++u) {
      const int e = base + u * NT;
      if (e < total) {
        const int row = e / np, col = e - row * np;
        f(row, col, e, x[u]);
      }
    }
  }
  __syncthreads();
}



// One GEMM step: thread 0 fills the LDS descriptor through `set`, then all threads run it.
template <int NW, class S>
__device__ void gemm_step(const S &set) {
  if (threadIdx.x == 0) {
    g_ep.idw = 1.0;
    set(g_ep);
  }
  __syncthreads();
  gemm_block<NW>();
  __syncthreads();
}

// Runs the method on one matrix.
template <int NW>
__device__ void run_one(const FusedArgs &a, int64_t b, double *slot, double *red) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  const int nin = a.ns ? a.ns[b] : a.n_uniform;  // order of the input (complex or real)
  const int cx = a.cplx;
  const int n = cx ? 2 * nin : nin;              // order of the real matrix the method runs on
  const int64_t off = (a.offs ? a.offs[b] : b * (int64_t)nin * nin) * (cx ? 2 : 1);  // in doubles
  if (nin < 1 || n > a.np_max) {
    if (tid == 0) {
      a.m_out[b] = -1; a.s_out[b] = -1;
      if (a.status) a.status[b] = EXPM_E_INVALID_ARG;
    }
    return;
  }
  const int np = (n + 15) & ~15;
  if ((NW == 4) != ((np >> 4) < kSplitT)) {  // matrix routed to the wrong variant
    if (tid == 0) {
      a.m_out[b] = -1; a.s_out[b] = -1;
      if (a.status) a.status[b] = EXPM_E_UNSUPPORTED;
    }
    return;
  }
  const size_t nn = (size_t)np * np;
  double *buf[kBufs];
  for (int i = 0; i < kBufs; ++i) buf[i] = slot + i * nn;
  const double *A = a.A + off;
  double *E = a.E ? a.E + off : nullptr;

  // ---- load A into buf0 (zero padded) and take ||A||_1 (thread j owns column j).  A complex
  // input Z = X + iY is loaded as its real form [[X, -Y], [Y, X]] (an algebra homomorphism,
  // so the real exponential of that matrix is the real form of e^Z). ----
  double colsum = 0.0;
  int bad = 0;
  if (tid < np) {
    cgdouble *Ag = gptr(A);
    gdouble *B0g = gptr(buf[0]);
    for (int i = 0; i < np; i += 16) {  // 16 loads in flight, then 16 stores
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int r = i + u;
        double x = 0.0;
        if (r < n && tid < n) {
          if (!cx) {
            x = Ag[(size_t)r * n + tid];
          } else {
            const int ri = r < nin ? r : r - nin, ci = tid < nin ? tid : tid - nin;
            const bool im = (r < nin) != (tid < nin);
            x = Ag[2 * ((size_t)ri * nin + ci) + (im ? 1 : 0)];
            if (im && r < nin) x = -x;
          }
        }
        v[u] = x;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        bad |= !isfinite(v[u]);
        colsum += fabs(v[u]);
        B0g[(i + u) * np + tid] = v[u];
      }
    }
    if (cx) {  // complex input: the 1-norm of A itself, sum_i |z_ij|
      colsum = 0.0;
      if (tid < nin) {
#pragma unroll 8
        for (int r = 0; r < nin; ++r) colsum += hypot(Ag[2 * ((size_t)r * nin + tid)], Ag[2 * ((size_t)r * nin + tid) + 1]);
      }
    }
  }
  bad = __syncthreads_or(bad);
  red[tid] = colsum;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double eta = red[0];
  __syncthreads();

  // a 1-norm that overflows (finite entries) is refused like a non-finite entry
  if (bad || !(eta <= __DBL_MAX__)) {
    if (E) for (int e = tid; e < nin * nin * (cx ? 2 : 1); e += NT) E[e] = __builtin_nan("");
    if (tid == 0) {
      a.m_out[b] = -1; a.s_out[b] = -1;
      if (a.status) a.status[b] = EXPM_E_NONFINITE;
    }
    __syncthreads();
    return;
  }

  if (tid == 0) select_ms(a.k.theta, 0, eta, -1.0, -1.0, &sh_ms[0], &sh_ms[1]);
  __syncthreads();
  const int m_plain = sh_ms[0], s_plain = sh_ms[1];
  // buffer B *= 2^e exactly (elementwise)
  // (16 loads in flight per thread, then 16 stores: a pass costs a few memory latencies, not
  // one per element)
  auto rescale = [&](double *B, int e2) {
    if (e2 == 0) return;
    gdouble *Bg = gptr(B);
    for (int e0 = tid; e0 < (int)nn; e0 += 16 * NT) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + u * NT;
        v[u] = e < (int)nn ? Bg[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + u * NT;
        if (e < (int)nn) Bg[e] = ldexp(v[u], e2);
      }
    }
    __syncthreads();
  };
  // The buffer holds X_b = 2^eb A: A itself (eb = 0) when no power up to the sixth can overflow
  // (||A||_1 <= 2^150), else X_p = 2^-sp A (sp the plain rule's s), whose powers stay in range
  // at any norm.  Either way exact.
  const int eb = eta <= 0x1p150 ? 0 : -s_plain;
  rescale(buf[0], eb);

  // ---- powers A^2 (buffer 1), A^3 (buffer 2) as the selection needs them ----
  bool have2 = false, have3 = false;
  double n2 = -1.0, n3 = -1.0;
  auto form2 = [&]() {
    if (have2) return;
    gemm_step<NW>([&](EpiDesc &d) {
      d.P = buf[0]; d.Q = buf[0]; d.kind = EK_STORE; d.np = np;
      d.dst = buf[1]; d.dst_ld = np; d.dst_nvalid = np; d.cplx = 0;
    });
    have2 = true;
  };
  auto form3 = [&]() {
    form2();
    if (have3) return;
    gemm_step<NW>([&](EpiDesc &d) {
      d.P = buf[1]; d.Q = buf[0]; d.kind = EK_STORE; d.np = np;
      d.dst = buf[2]; d.dst_ld = np; d.dst_nvalid = np; d.cplx = 0;
    });
    have3 = true;
  };
  int m = m_plain, s = s_plain;
  if (a.features) {
    // feature row and training label of the learned selector (no e^A)
    form3();
    n2 = unscale_norm(block_norm1<NT>(buf[1], np, red), 2, -eb);
    n3 = unscale_norm(block_norm1<NT>(buf[2], np, red), 3, -eb);
    const double tr = ldexp(block_trace<NT>(buf[0], np, red), -eb);
    const double asym = ldexp(block_asym1<NT>(buf[0], np, red), -eb);
    if (tid == 0) {
      double *row = a.features + b * kFeatRow;
      learned_features(eta, n2, tr, asym, n, row);
      int lm, ls, am, as;
      learned_label(a.k.theta, eta, n2, n3, &lm, &ls);
      select_ms(a.k.theta, 1, eta, m_plain >= 2 ? n2 : -1.0, m_plain >= 12 ? n3 : -1.0, &am, &as);
      row[8] = eta; row[9] = n2; row[10] = n3; row[11] = mlp_ms_class(lm, ls);
      row[12] = m_plain; row[13] = s_plain; row[14] = am; row[15] = as;
      a.m_out[b] = lm; a.s_out[b] = ls;
      if (a.status) a.status[b] = EXPM_OK;
    }
    __syncthreads();
    return;
  } else if (a.sel == EXPM_SEL_ALPHA) {
    if (m_plain >= 2) { form2(); n2 = unscale_norm(block_norm1<NT>(buf[1], np, red), 2, -eb); }
    if (m_plain >= 12) { form3(); n3 = unscale_norm(block_norm1<NT>(buf[2], np, red), 3, -eb); }
    if (m_plain >= 2) {
      if (tid == 0) select_ms(a.k.theta, 1, eta, n2, n3, &sh_ms[0], &sh_ms[1]);
      __syncthreads();
      m = sh_ms[0]; s = sh_ms[1];
    }
  } else if (a.sel == EXPM_SEL_LEARNED && m_plain >= 2) {
    // proposal from the MLP on features available once A^2 exists; kept only if the alpha
    // bound holds for it (with ||A^3|| when the proposal forms A^3 anyway), else the plain rule
    form2();
    n2 = unscale_norm(block_norm1<NT>(buf[1], np, red), 2, -eb);
    const double tr = ldexp(block_trace<NT>(buf[0], np, red), -eb);
    const double asym = ldexp(block_asym1<NT>(buf[0], np, red), -eb);
    const int cls = mlp_infer<NT>(eta, n2, tr, asym, n);
    int mq, sq;
    mlp_class_ms(cls, &mq, &sq);
    if (mq >= 12) { form3(); n3 = unscale_norm(block_norm1<NT>(buf[2], np, red), 3, -eb); }
    const bool ok = proposal_ok(a.k.theta, eta, n2, mq >= 12 ? n3 : -1.0, mq, sq);
    if (ok) { m = mq; s = sq; } else { m = m_plain; s = s_plain; }
    if (tid == 0) atomicAdd(&g_learned_counts[ok ? 0 : 1], 1ull);
  }
  // X = 2^-s A = 2^-sc X_b with sc = s + eb, so X^k = 2^(-k sc) X_b^k.  The factors go into the
  // coefficients when they stay far from overflow (|sc| <= 150: k sc is within the exponent
  // range for k <= 6); otherwise the powers formed so far are rescaled (exact) and the missing
  // ones are formed from X itself.  No pass over a buffer in the common case.
  const int sc = s + eb;
  const bool fold = sc >= -150 && sc <= 150;
  if (!fold) {
    rescale(buf[0], -sc);
    if (have2) rescale(buf[1], -2 * sc);
    if (have3) rescale(buf[2], -3 * sc);
  }
  if (m >= 2) form2();
  if (m >= 12) form3();
  if (tid == 0) {
    make_coefs(a.k, m, fold ? sc : 0, g_ep.c);
    a.m_out[b] = m; a.s_out[b] = s;
    if (a.status) a.status[b] = EXPM_OK;
  }
  __syncthreads();
  if (a.select_only) return;

  const double *c = g_ep.c;
  const int tb = (m >= 8) ? 2 : 3;  // buffer holding T when s > 0
  // destination of T: e^A itself when there is no squaring, else a workspace buffer
  double *Tp = (s == 0) ? E : buf[tb];
  const int Tld = (s == 0) ? n : np, Tnv = (s == 0) ? nin : np, Tcx = (s == 0) ? cx : 0;
  double *B0 = buf[0], *B1 = buf[1], *B2 = buf[2];
  auto base = [&](EpiDesc &d) {
    d.np = np; d.b0 = B0; d.b1 = B1; d.b2 = B2;
    d.dst = Tp; d.dst_ld = Tld; d.dst_nvalid = Tnv; d.cplx = Tcx;
  };
  gdouble *Tg = gptr(Tp);

  if (m == 1) {
    const double c0 = c[0];
    const double *in[1] = {B0};
    for_each_elem<NT, 1>(np, in, [&](int r, int cc, int, const double *x) {
      put_dst(Tg, Tld, Tnv, Tcx, r, cc, (r == cc ? 1.0 : 0.0) + c0 * x[0]);
    });
  } else if (m == 2) {
    const double c0 = c[0], c1 = c[1];
    const double *in[2] = {B0, B1};
    for_each_elem<NT, 2>(np, in, [&](int r, int cc, int, const double *x) {
      put_dst(Tg, Tld, Tnv, Tcx, r, cc, (r == cc ? 1.0 : 0.0) + c0 * x[0] + c1 * x[1]);
    });
  } else if (m == 4) {
    double *W = buf[2];
    const double c2 = c[2], c3 = c[3], c4 = c[4];
    const double *in[2] = {B0, B1};
    for_each_elem<NT, 2>(np, in, [&](int r, int cc, int e, const double *x) {
      W[e] = (r == cc ? c2 : 0.0) + c3 * x[0] + c4 * x[1];
    });
    gemm_step<NW>([&](EpiDesc &d) { base(d); d.P = B1; d.Q = W; d.kind = EK_M4; });
  } else if (m == 8) {
    double *W1 = buf[2], *L = buf[3], *Rm = buf[4];
    const double c0 = c[0], c1 = c[1];
    const double *in[2] = {B0, B1};
    for_each_elem<NT, 2>(np, in, [&](int, int, int e, const double *x) { W1[e] = c0 * x[0] + c1 * x[1]; });
    gemm_step<NW>([&](EpiDesc &d) { base(d); d.P = B1; d.Q = W1; d.kind = EK_M8A; d.o[0] = L; d.o[1] = Rm; });
    gemm_step<NW>([&](EpiDesc &d) { base(d); d.P = L; d.Q = Rm; d.kind = EK_M8B; });
  } else if (m == 12) {
    double *Bq0 = buf[3], *Bq1 = buf[4], *Bq2 = buf[5], *Bq3 = buf[6];
    double cf[16];
    for (int i = 0; i < 16; ++i) cf[i] = c[i];
    const double *in[3] = {B0, B1, B2};
    for_each_elem<NT, 3>(np, in, [&](int r, int cc, int e, const double *x) {
      const double id = (r == cc) ? 1.0 : 0.0;
      const double x1 = x[0], x2 = x[1], x3 = x[2];
      Bq0[e] = cf[0] * id + cf[1] * x1 + cf[2] * x2 + cf[3] * x3;
      Bq1[e] = cf[4] * id + cf[5] * x1 + cf[6] * x2 + cf[7] * x3;
      Bq2[e] = cf[8] * id + cf[9] * x1 + cf[10] * x2 + cf[11] * x3;
      Bq3[e] = cf[12] * id + cf[13] * x1 + cf[14] * x2 + cf[15] * x3;
    });
    double *A6 = buf[0], *Y = buf[1];
    // A_6 = B_3 + B_4^2 ; Y = B_2 + A_6
    gemm_step<NW>([&](EpiDesc &d) {
      base(d); d.P = Bq3; d.Q = Bq3; d.kind = EK_SPLIT2; d.in0 = Bq2; d.in1 = Bq1; d.o[0] = A6; d.o[1] = Y;
    });
    // T_12 = B_1 + Y A_6
    gemm_step<NW>([&](EpiDesc &d) { base(d); d.P = Y; d.Q = A6; d.kind = EK_ADD1; d.in0 = Bq0; });
  } else {  // m == 18
    double *Bq[5] = {buf[3], buf[4], buf[5], buf[6], buf[7]};
    // A^6 = A^3 A^3; the epilogue forms B_1..B_5 from (I, A, A^2, A^3, A^6)
    gemm_step<NW>([&](EpiDesc &d) {
      base(d); d.P = B2; d.Q = B2; d.kind = EK_M18A;
      for (int j = 0; j < 5; ++j) d.o[j] = Bq[j];
    });
    double *A9 = buf[0], *Y = buf[1];
    // A_9 = B_1 B_5 + B_4 ; Y = B_3 + A_9
    gemm_step<NW>([&](EpiDesc &d) {
      base(d); d.P = Bq[0]; d.Q = Bq[4]; d.kind = EK_SPLIT2; d.in0 = Bq[3]; d.in1 = Bq[2]; d.o[0] = A9; d.o[1] = Y;
    });
    // T_18 = B_2 + Y A_9
    gemm_step<NW>([&](EpiDesc &d) { base(d); d.P = Y; d.Q = A9; d.kind = EK_ADD1; d.in0 = Bq[1]; });
  }

  // ---- s squarings, ping-pong between buffers tb and tb^1 ----
  int cur = tb;
  for (int rsq = 1; rsq <= s; ++rsq) {
    const int nxt = cur ^ 1;
    const bool last = (rsq == s);
    gemm_step<NW>([&](EpiDesc &d) {
      d.np = np; d.P = buf[cur]; d.Q = buf[cur]; d.kind = EK_STORE;
      d.dst = last ? E : buf[nxt]; d.dst_ld = last ? n : np; d.dst_nvalid = last ? nin : np;
      d.cplx = last ? cx : 0;
    });
    cur = nxt;
  }
}

}  // namespace

// Sweep range and counter of one launch: queue words when the batch is sorted on the device,
// else the static range.
struct Sweep {
  int64_t lo, hi;
  unsigned long long *ctr;
};
__device__ inline Sweep sweep_of(const FusedArgs &a) {
  Sweep w;
  if (a.queue) {
    w.lo = (int64_t)a.queue[kQBound + a.q_lo];
    w.hi = (int64_t)a.queue[kQBound + a.q_hi];
    w.ctr = &a.queue[a.q_ctr];
  } else {
    w.lo = a.lo;
    w.hi = a.hi;
    w.ctr = nullptr;
  }
  return w;
}

// Persistent loop: each workgroup pops the next queue entry of its range until it is empty.
template <class F>
__device__ __attribute__((always_inline)) inline void sweep(const FusedArgs &a, const F &run) {
  __shared__ int64_t sh_idx;
  const Sweep w = sweep_of(a);
  for (int64_t it = w.lo + blockIdx.x;; it += gridDim.x) {
    int64_t idx = it;
    if (w.ctr) {
      if (threadIdx.x == 0) sh_idx = w.lo + (int64_t)atomicAdd(w.ctr, 1ull);
      __syncthreads();
      const long long v = sh_idx;
      idx = (int64_t)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
                      (unsigned)__builtin_amdgcn_readfirstlane((int)v));
      __syncthreads();
    }
    if (idx >= w.hi) break;
    // entry and matrix index are uniform: keep them in scalar registers
    const int64_t b = a.order ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[idx]) : idx;
    run(b);
    __syncthreads();
  }
}

template <int NW>
__global__ __launch_bounds__(64 * NW, NW == 4 ? 2 : 1) void expm_fused_kernel(FusedArgs a) {
  __shared__ double red[64 * NW + 16];
  double *slot = a.slots + (size_t)blockIdx.x * a.slot_doubles;
  sweep(a, [&](int64_t b) { run_one<NW>(a, b, slot, red); });
}

}  // namespace expm

#include "resident.h"
#include "resident_sr.h"

namespace expm {
namespace {

// OCC workgroups per CU.  8 waves: one (its LDS matrix takes 128 KiB).  4 waves (orders up to
// 64): three in the plain rule's batched sweeps, 168 VGPRs each, which the per-degree
// instantiation leaves without spills below order 64 (measured against two per CU: the sweep
// 1.5 % shorter); two, with 256 VGPRs, under the other rules and for calls whose matrices are
// all of order 49..64, where the degree-12 and degree-18 stages would spill at 168.
template <int NW, int SEL, int OCC>
__global__ __launch_bounds__(64 * NW, OCC) void expm_resident_kernel(FusedArgs a) {
  __shared__ double red[64 * NW + 16];
  double *slot = a.slots ? a.slots + (size_t)blockIdx.x * a.slot_doubles : nullptr;
  res_init<NW>(a);
  // (inlined all the way down: an out-of-line call would copy the kernel arguments to private
  // memory and spill the register matrices around it)
  sweep(a, [&](int64_t b) __attribute__((always_inline)) { run_res_dispatch<NW, SEL>(a, b, slot, red); });
}

template <int SEL>
__global__ __launch_bounds__(64 * kSrNW, 3) void expm_sr_kernel(FusedArgs a) {
  __shared__ double red[64 * kSrNW + 16];
  res_init<kSrNW>(a);
  sweep(a, [&](int64_t b) __attribute__((always_inline)) { run_sr_dispatch<SEL>(a, b, red); });
}

}  // namespace

// Cost key of each matrix for the work-queue order: the binary exponent of the mean absolute
// row sum of four sampled rows of the real form (an estimate of the mean column sum, a cheap
// stand-in for ||A||_1, which decides m and s), biased into 1..kKeyBins-1; 0 when the sample
// is empty, zero or not finite.  One wave per matrix reads at most four rows of it.  The key
// only orders the work: every matrix is still evaluated from its exact norm.
__global__ __launch_bounds__(256) void expm_cost_key_kernel(const double *A, const int64_t *offs, const int32_t *ns,
                                                            int n_uniform, int64_t batch, int cplx, uint8_t *key) {
  const int lane = threadIdx.x & 63;
  for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < batch; b += (int64_t)gridDim.x * 4) {
    const int nin = ns ? ns[b] : n_uniform;
    const int64_t ob = offs ? offs[b] : 0;  // issued beside the order's load, not after it
    const int n = cplx ? 2 * nin : nin;
    double acc = 0.0;
    int rows = 0;
    if (nin >= 1 && n <= kNpMax) {
      const int64_t off = (offs ? ob : b * (int64_t)nin * nin) * (cplx ? 2 : 1);
      const int len = cplx ? 2 * nin : nin;  // doubles per input row; a complex row's |re| + |im|
                                             // is the row sum of its row of the real form
      rows = nin < 4 ? nin : 4;
      for (int k = 0; k < rows; ++k) {
        const double *row = A + off + (int64_t)(((2 * k + 1) * nin) / (2 * rows)) * len;
        for (int j = lane; j < len; j += 64) acc += fabs(row[j]);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
      int k = 0;
      if (rows > 0 && acc > 0.0 && isfinite(acc)) {
        const int e = ilogb(acc / rows) + kKeyBias;
        k = e < 1 ? 1 : (e > kKeyBins - 1 ? kKeyBins - 1 : e);
      }
      key[b] = (uint8_t)k;
    }
  }
}

// Counting sort of the batch into the work-queue order: by padded real order, largest first,
// and within an order by cost key, largest first (the longest jobs are claimed first, so a
// sweep does not end on a few expensive matrices claimed late); resets the counters and
// records the range bounds.  One workgroup of 1024 threads; key may be null (all keys 0).
__global__ __launch_bounds__(1024) void expm_order_kernel(const int32_t *ns, int n_uniform, int np_max,
                                                          const uint8_t *key, int64_t batch, int cplx,
                                                          int32_t *order, unsigned long long *queue) {
  constexpr int kCls = 18, kBins = kCls * kKeyBins;
  static_assert(kBins <= 2 * 1024, "two bins per thread in the scan");
  __shared__ int hist[kBins], start[kBins], part[16];
  const int tid = threadIdx.x;
  for (int i = tid; i < kBins; i += 1024) hist[i] = 0;
  __syncthreads();
  auto bin = [&](int64_t b) {
    const int nin = ns ? ns[b] : n_uniform;
    const int n = cplx ? 2 * nin : nin;  // order of the real matrix the method runs on
    // class 0 for np = 256 ... 15 for np = 16; 17 for an invalid order (also one above the
    // call's n_max, which no sweep of the call would otherwise reach): drained with np = 16,
    // whose kernels report it
    const int cls = (nin < 1 || n > np_max) ? 17 : 16 - ((n + 15) >> 4);
    const int k = key ? (int)key[b] : 0;
    return cls * kKeyBins + (kKeyBins - 1 - k);
  };
  // each thread's first kHeld bins stay in registers for the scatter below
  constexpr int kHeld = 8;
  int held[kHeld];
#pragma unroll
  for (int j = 0; j < kHeld; ++j) {
    const int64_t b = tid + (int64_t)j * 1024;
    held[j] = b < batch ? bin(b) : 0;
  }
#pragma unroll
  for (int j = 0; j < kHeld; ++j)
    if (tid + (int64_t)j * 1024 < batch) atomicAdd(&hist[held[j]], 1);
  for (int64_t b = tid + (int64_t)kHeld * 1024; b < batch; b += 1024) atomicAdd(&hist[bin(b)], 1);
  __syncthreads();
  // exclusive scan of the bins: thread t owns bins 2t and 2t + 1; inclusive scans within each
  // wave, then each wave adds the totals of the waves before it
  const int b0 = 2 * tid, b1 = 2 * tid + 1;
  const int h0 = b0 < kBins ? hist[b0] : 0, h1 = b1 < kBins ? hist[b1] : 0;
  const int lane = tid & 63, wv = tid >> 6;
  int v = h0 + h1;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  if (lane == 63) part[wv] = v;
  __syncthreads();
  for (int k = 0; k < wv; ++k) v += part[k];
  if (b0 < kBins) start[b0] = v - h0 - h1;
  if (b1 < kBins) start[b1] = v - h1;
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < kQBound; ++i) queue[i] = 0ull;
    queue[kQBound + 0] = 0ull;
    queue[kQBound + 1] = (unsigned long long)start[(16 - kResT) * kKeyBins];        // np <= 128
    queue[kQBound + 2] = (unsigned long long)start[(16 - kRes6T) * kKeyBins];       // np <= 96
    queue[kQBound + 3] = (unsigned long long)start[(16 - kSplitT + 1) * kKeyBins];  // np <= 64
    queue[kQBound + 4] = (unsigned long long)start[15 * kKeyBins];                  // np = 16
    queue[kQBound + 5] = (unsigned long long)batch;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kHeld; ++j) {
    const int64_t b = tid + (int64_t)j * 1024;
    if (b < batch) order[atomicAdd(&start[held[j]], 1)] = (int32_t)b;
  }
  for (int64_t b = tid + (int64_t)kHeld * 1024; b < batch; b += 1024)
    order[atomicAdd(&start[bin(b)], 1)] = (int32_t)b;
}

int fused_max_blocks_per_cu(int nw) {
  int nb = 0;
  hipError_t e = nw == 8
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, expm_fused_kernel<8>, 512, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, expm_fused_kernel<4>, 256, 0);
  if (e != hipSuccess) return 1;
  return nb < 1 ? 1 : nb;
}

hipError_t launch_fused(const FusedArgs &a, int nw, int grid, hipStream_t st) {
  if (nw == 8) hipLaunchKernelGGL(expm_fused_kernel<8>, dim3(grid), dim3(512), 0, st, a);
  else hipLaunchKernelGGL(expm_fused_kernel<4>, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

int resident_max_blocks_per_cu(int nw) {
  int nb = 0;
  hipError_t e = nw == 8    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, expm_resident_kernel<8, EXPM_SEL_PLAIN, 1>, 512, 0)
                 : nw == 12 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, expm_sr_kernel<EXPM_SEL_PLAIN>, 768, 0)
                 : nw == 5  ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, expm_resident_kernel<4, EXPM_SEL_PLAIN, 2>, 256, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, expm_resident_kernel<4, EXPM_SEL_PLAIN, 3>, 256, 0);
  if (e != hipSuccess) return 1;
  return nb < 1 ? 1 : nb;
}

// Every selector variant of a kernel has the same launch bounds and LDS footprint.
template <int NW, int OCC>
static void launch_res_sel(const FusedArgs &a, int grid, hipStream_t st) {
  switch (a.sel) {
    case EXPM_SEL_ALPHA: hipLaunchKernelGGL((expm_resident_kernel<NW, EXPM_SEL_ALPHA, OCC>), dim3(grid), dim3(64 * NW), 0, st, a); break;
    case EXPM_SEL_LEARNED: hipLaunchKernelGGL((expm_resident_kernel<NW, EXPM_SEL_LEARNED, OCC>), dim3(grid), dim3(64 * NW), 0, st, a); break;
    default: hipLaunchKernelGGL((expm_resident_kernel<NW, EXPM_SEL_PLAIN, OCC>), dim3(grid), dim3(64 * NW), 0, st, a); break;
  }
}

hipError_t launch_resident(const FusedArgs &a, int nw, int grid, hipStream_t st) {
  if (nw == 8) {
    launch_res_sel<8, 1>(a, grid, st);
  } else if (nw == 12) {
    switch (a.sel) {
      case EXPM_SEL_ALPHA: hipLaunchKernelGGL((expm_sr_kernel<EXPM_SEL_ALPHA>), dim3(grid), dim3(64 * kSrNW), 0, st, a); break;
      case EXPM_SEL_LEARNED: hipLaunchKernelGGL((expm_sr_kernel<EXPM_SEL_LEARNED>), dim3(grid), dim3(64 * kSrNW), 0, st, a); break;
      default: hipLaunchKernelGGL((expm_sr_kernel<EXPM_SEL_PLAIN>), dim3(grid), dim3(64 * kSrNW), 0, st, a); break;
    }
  } else if (nw == 5 || a.sel != EXPM_SEL_PLAIN) {
    // the alpha and learned rules' 4-wave kernels keep two workgroups per CU (at three their
    // run-time degree spills)
    launch_res_sel<4, 2>(a, grid, st);
  } else {
    hipLaunchKernelGGL((expm_resident_kernel<4, EXPM_SEL_PLAIN, 3>), dim3(grid), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_order(const double *A, const int64_t *offs, const int32_t *ns, int n_uniform, int np_max,
                        int64_t batch, int cplx, uint8_t *key, int32_t *order, unsigned long long *queue,
                        hipStream_t st) {
  if (key) {
    const int64_t g = (batch + 3) / 4;
    hipLaunchKernelGGL(expm_cost_key_kernel, dim3((unsigned)(g < 2048 ? g : 2048)), dim3(256), 0, st, A, offs, ns,
                       n_uniform, batch, cplx, key);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(expm_order_kernel, dim3(1), dim3(1024), 0, st, ns, n_uniform, np_max < kNpMax ? np_max : kNpMax,
                     (const uint8_t *)key, batch, cplx, order, queue);
  return hipGetLastError();
}

}  // namespace expm

namespace expm {

hipError_t learned_set(const float *params_dev, const double *norm_host, hipStream_t st) {
  hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_mlp_params), params_dev, kMlpParams * sizeof(float), 0,
                                        hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_mlp_norm), norm_host, 2 * kMlpIn * sizeof(double), 0,
                             hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  const unsigned long long z[2] = {0ull, 0ull};
  e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_learned_counts), z, sizeof(z), 0, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t learned_counts(unsigned long long out[2]) {
  return hipMemcpyFromSymbol(out, HIP_SYMBOL(g_learned_counts), 2 * sizeof(unsigned long long));
}

}  // namespace expm
