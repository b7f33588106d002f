// Launch interface of the persistent fused kernels (orders n <= 256).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "expm_internal.h"

namespace expm {

// Orders with np / 16 >= kSplitT run on 8-wave workgroups, the rest on 4-wave workgroups.
constexpr int kSplitT = 5;
// Largest np / 16 of the resident kernels (np <= 128).
constexpr int kResT = 8;
// The 8-wave resident kernel parks up to two matrices in HBM from np / 16 >= kResParkT on;
// per np / 16 its slot needs 2 regions x 8 waves x 4 x 64 doubles.
constexpr int kResParkT = 5;
constexpr int kResParkDoublesPerT = 2 * 8 * 4 * 64;

// Orders np 80..96 (np / 16 = 5, 6) run on the split-row resident kernel (12 waves).
constexpr int kRes6T = 6;

// Work-queue words written by the order kernel: [0, kQBound) counters of up to six sweeps;
// [kQBound, kQBound + 6) range bounds of the sorted order (largest real order first):
// 0, first entry with np <= 128, with np <= 96, with np <= 64, with np = 16, batch.
constexpr int kQBound = 8;
constexpr int kQWords = 16;
// Cost keys (one byte per matrix) order the entries of one order largest first: binary
// exponent of a sampled mean row sum plus kKeyBias, clamped to 1..kKeyBins-1.
constexpr int kKeyBins = 64;
constexpr int kKeyBias = 32;

struct FusedArgs {
  const double *A;        // packed inputs
  double *E;              // packed outputs (nullptr when select_only)
  const int64_t *offs;    // per-matrix element offsets (nullptr: b * n_uniform^2)
  const int32_t *ns;      // per-matrix orders (nullptr: n_uniform)
  const int32_t *order;   // work-queue order (nullptr: identity)
  unsigned long long *queue;  // kQWords words (see below); nullptr: static range [lo, hi)
  int32_t *m_out, *s_out, *status;
  double *slots;          // gridDim.x slots of slot_doubles doubles (per kernel variant)
  size_t slot_doubles;
  int q_ctr, q_lo, q_hi;  // this sweep's counter word and its range bounds queue[kQBound + q_lo],
                          // queue[kQBound + q_hi]
  int64_t lo, hi;         // static range (queue == nullptr)
  int64_t batch;
  int n_uniform;
  int np_max;             // largest padded order the slots can hold
  int sel;                // expm_sel_t
  int select_only;
  int method;             // 0 product-reduced T_m; 1 Paterson-Stockmeyer; 2 Pade (one-wave kernel)
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
// Resident kernels (np <= 128: 8 waves for np 112..128, split-row 12 waves for np 80..96,
// 4 waves for np <= 64).
int resident_max_blocks_per_cu(int nw);
// One wave per matrix of real order <= 16 (expm_tiny.hip): persistent launch over the sweep
// described by a (queue range or static range), PLAIN or ALPHA rule.
int tiny_max_blocks_per_cu();
int tiny_waves_per_block();
hipError_t launch_tiny(const FusedArgs &a, int grid, hipStream_t st);
// Fourth-order Magnus steps, one system of order n <= 16 per wave (expm_tiny.hip).
hipError_t launch_magnus4(const double *S0, const double *S1, int64_t s_stride, const double *Yin, double *Yout,
                          const double *u1, const double *u2, int n, int64_t batch, double h, int sel,
                          const Consts &k, int32_t *m_out, int32_t *s_out, int32_t *status, int grid,
                          hipStream_t st);
// nw = 8, 12, 4; 5: the 4-wave kernel at two workgroups per CU (calls whose matrices are all of
// order 49..64), where nw = 4 runs three per CU (batched sweeps)
hipError_t launch_resident(const FusedArgs &a, int nw, int grid, hipStream_t st);
// Work-queue order of a batch: cost keys of every matrix (into key, batch bytes; skipped when
// key is null), then the counting sort by (real order, key) into order and the queue words.
// Orders above np_max (the call's largest padded real order) are classed invalid.
hipError_t launch_order(const double *A, const int64_t *offs, const int32_t *ns, int n_uniform, int np_max,
                        int64_t batch, int cplx, uint8_t *key, int32_t *order, unsigned long long *queue,
                        hipStream_t st);

}  // namespace expm
