// Launch interface of the persistent fused kernels (orders n <= 256).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "expm_internal.h"

namespace expm {

// Orders with np / 16 >= kSplitT run on the 8-wave kernel, the rest on the 4-wave kernel.
constexpr int kSplitT = 5;

struct FusedArgs {
  const double *A;        // packed inputs
  double *E;              // packed outputs (nullptr when select_only)
  const int64_t *offs;    // per-matrix element offsets (nullptr: b * n_uniform^2)
  const int32_t *ns;      // per-matrix orders (nullptr: n_uniform)
  const int32_t *order;   // work-queue order (nullptr: identity)
  unsigned long long *queue;  // [counter 8-wave, counter 4-wave, split]; nullptr: static
  int32_t *m_out, *s_out, *status;
  double *slots;          // gridDim.x slots of slot_doubles doubles (per kernel variant)
  size_t slot_doubles;
  int64_t batch;
  int64_t split;          // used when queue == nullptr
  int n_uniform;
  int np_max;             // largest padded order the slots can hold
  int sel;                // expm_sel_t
  int select_only;
  int cplx;               // inputs / outputs are interleaved complex (run on the real form)
  double *features;       // feature rows of the learned selector (kFeatRow doubles per
                          // matrix); when set no e^A is computed
  Consts k;
};

// Feature row: f0..f7 (raw features), ||A||, ||A^2||, ||A^3||, label class, plain m, plain s,
// alpha m, alpha s.
constexpr int kFeatRow = 16;
hipError_t learned_set(const float *params_dev, const double *norm_host, hipStream_t st);
hipError_t learned_counts(unsigned long long out[2]);


constexpr int kFusedBufs = 8;
int fused_max_blocks_per_cu(int nw);
hipError_t launch_fused(const FusedArgs &a, int nw, int grid, hipStream_t st);
hipError_t launch_order(const int32_t *ns, int64_t batch, int cplx, int32_t *order,
                        unsigned long long *queue, hipStream_t st);

}  // namespace expm
