// Tiled multi-workgroup path for real orders above 256 (complex orders above 128).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "expm_internal.h"

namespace expm {

constexpr int kLargeTile = 128;   // output tile of one workgroup
constexpr int kLargeBufs = 8;     // n x n work buffers per matrix
constexpr int kLargeRB = 64;      // rows per workgroup in the norm passes
constexpr int kPadeNpMax = 2048;  // largest padded real order of the tiled Pade solve

struct LargeLayout {
  int64_t n;        // order of the real matrix the method runs on (2 * input order if complex)
  int64_t np;       // n rounded up to kLargeTile
  int64_t group;    // matrices processed together
  int64_t nrb;      // row blocks of the norm passes
  size_t bufs_off, partial_off, norms_off, flags_off, coef_off, list_off, shift_off, planes_off, piv_off, total;
};

// prec: expm_prec_t of the call (the reduced forms need room for operand planes); tiles:
// output tiles per launch (the group holds about that many tiles' worth of matrices).
// planes: 2 for the native complex path (every buffer holds a real and an imaginary plane).
LargeLayout large_layout(int64_t n_real, int64_t batch, int prec, int tiles, int planes);

struct LargeCall {
  const double *A;    // first input; matrix b at A + b * in_stride doubles
  double *E;          // first output, same layout
  int64_t nin;        // input order (complex or real)
  int cplx;           // interleaved complex input / output: 1 run on the real form (order 2 nin),
                      // 2 native complex (planar buffers, four real products per product)
  int64_t batch;
  int sel;            // EXPM_SEL_PLAIN or EXPM_SEL_ALPHA
  int prec;           // PREC_F64 / PREC_F32 / PREC_BF16X3 for the reduced steps
  int select_only;
  int ps;             // Paterson-Stockmeyer comparison method (EXPM_FLAG_PS)
  int pade;           // diagonal Pade comparison method (EXPM_FLAG_PADE), real order <= 2048
  int tri;            // triangular refinement (EXPM_FLAG_TRI)
  int tiles;          // output tiles per launch
  int32_t *m_out, *s_out, *status;  // device, one per matrix
  void *ws;
  size_t ws_bytes;
  Consts k;
};

// Runs the method on a uniform batch of large matrices.  Synchronises the stream once per
// group to read the chosen (m, s) back.
expm_status_t run_large(const LargeCall &c, hipStream_t st);

}  // namespace expm
