// C ABI of the matrix-exponential library (declarations and contracts in include/expm.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <initializer_list>
#include <map>
#include <mutex>

#include "expm_fused.h"
#include "expm_internal.h"
#include "expm_large.h"
#include "mlp.h"

namespace expm {
size_t mlp_scratch_floats(int B);
hipError_t mlp_forward(const float *params, const float *X, int B, float *scratch, float *logits, hipStream_t st);
hipError_t mlp_grad(const float *params, const float *X, const int *y, int B, float *scratch, float *grads,
                    float *loss, hipStream_t st);
hipError_t mlp_adam_step(float *params, const float *grads, float *m, float *v, int step, float lr, hipStream_t st);
}  // namespace expm

using namespace expm;

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kFusedNMax = 256;  // orders handled by the fused kernel
constexpr int kMaxSlots = 1024;         // upper bound on resident fused workgroups

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int64_t pad16(int64_t n) { return (n + 15) & ~int64_t(15); }
int np_max_t(int64_t n) { return (int)(pad16(n) >> 4); }

// FP64 and BF16X3 target the double row of the thresholds (truncation below 1e-15, so the
// split's FP32 accumulation dominates the error); FP32 uses the single row.
double default_u(int prec) { return prec == EXPM_PREC_FP32 || prec == EXPM_PREC_FP32_ALL ? 0x1p-24 : 0x1p-53; }

expm_status_t check_opts(const expm_opts_t *o, double *u) {
  if (!o) return EXPM_E_INVALID_ARG;
  if (o->dtype != EXPM_F64 && o->dtype != EXPM_C128) return EXPM_E_INVALID_ARG;
  if (o->prec < EXPM_PREC_FP64 || o->prec > EXPM_PREC_FP32_ALL) return EXPM_E_INVALID_ARG;
  if (o->sel < EXPM_SEL_PLAIN || o->sel > EXPM_SEL_LEARNED) return EXPM_E_INVALID_ARG;
  if (o->flags != 0 && o->flags != EXPM_FLAG_PS && o->flags != EXPM_FLAG_PADE && o->flags != EXPM_FLAG_TRI)
    return EXPM_E_INVALID_ARG;
  double uu = o->u == 0.0 ? default_u(o->prec) : o->u;
  if (!(uu >= 0x1p-53 && uu <= 0x1p-10)) return EXPM_E_INVALID_ARG;
  *u = uu;
  return EXPM_OK;
}

// Resident workgroups per CU of the four sweep kernels on the current device (cached).
struct FusedCaps {
  int cus = 0, per4 = 1, per8 = 1, res4 = 1, res6 = 1, res8 = 1, tiny = 1, res4w = 1;
};

FusedCaps fused_caps() {
  static FusedCaps caps;
  static bool init = false;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  if (!init) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
      caps.cus = cus;
      caps.per4 = fused_max_blocks_per_cu(4);
      caps.per8 = fused_max_blocks_per_cu(8);
      caps.res4 = resident_max_blocks_per_cu(4);
      caps.res4w = resident_max_blocks_per_cu(5);
      caps.res6 = resident_max_blocks_per_cu(12);
      caps.res8 = resident_max_blocks_per_cu(8);
      caps.tiny = tiny_max_blocks_per_cu();
      init = true;
    } else {
      caps.cus = 0;  // no device visible: size for the largest launch, do not cache
    }
  }
  return caps;
}

// K_RES6: split-row kernel, np 80..96; K_TINY: one wave per matrix, np 16; K_RES4W: the 4-wave
// kernel at two workgroups per CU (uniform calls of np 64; not tunable, it has no per_cu entry)
enum Kern { K_FUSED4, K_FUSED8, K_RES4, K_RES6, K_RES8, K_TINY, K_RES4W };

// Launch configuration installed by expm_tune_set (process-wide; zero fields = defaults).
std::mutex g_tune_mu;
expm_tune_t g_tune = {};
expm_tune_t tune_now() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tune;
}
constexpr int kDefaultTiles = 2048;

// Persistent grid of sweep kernel k for `batch` matrices: resident workgroups per CU (the
// occupancy maximum, or fewer when tuned; layouts size their slots with tuned = false).
int grid_for(Kern k, int64_t batch, bool tuned = true) {
  FusedCaps c = fused_caps();
  if (tuned && k != K_RES4W) {
    const int t = tune_now().per_cu[k];
    if (t > 0) {
      int *per = k == K_FUSED4 ? &c.per4 : k == K_FUSED8 ? &c.per8 : k == K_RES4 ? &c.res4
               : k == K_RES6 ? &c.res6 : k == K_RES8 ? &c.res8 : &c.tiny;
      if (t < *per) *per = t;
    }
  }
  if (k == K_TINY) {  // one matrix per wave; no per-workgroup slot
    const int64_t w = tiny_waves_per_block();
    const int64_t need = (batch + w - 1) / w;
    const int64_t cap = c.cus > 0 ? (int64_t)c.cus * c.tiny : 8192;
    return (int)(need < cap ? need : cap);
  }
  const int per = k == K_FUSED4 ? c.per4 : k == K_FUSED8 ? c.per8 : k == K_RES4 ? c.res4 : k == K_RES6 ? c.res6
                : k == K_RES4W ? c.res4w : c.res8;
  int cap = c.cus > 0 ? c.cus * per : kMaxSlots;
  if (cap > kMaxSlots) cap = kMaxSlots;
  return (int)(batch < cap ? batch : cap);
}

struct FusedLayout {
  size_t queue_off, order_off, key_off, slots8_off, slots4_off, slotsr_off, total;
  size_t slot8_doubles, slot4_doubles, slotr_doubles;
  int slots8, slots4, slotsr;
};

// Workspace of the fused path.  Separate slot arrays per sweep kernel, so the sweeps may run
// concurrently: the global-memory kernels (8 buffers per slot; the 8-wave one serves np >= 80,
// the 4-wave one np <= 64 — the resident kernels cover np <= 128 except for the learned
// selector's feature rows) and the 8-wave resident kernel (two parked matrices per slot, for
// np >= 96).
FusedLayout fused_layout(int64_t n_max, int64_t batch) {
  FusedLayout L;
  const int64_t np = pad16(n_max);
  const int64_t np4 = std::min<int64_t>(np, 16 * (kSplitT - 1));
  const int64_t tr = std::min<int64_t>(np_max_t(n_max), kResT);
  L.slots4 = grid_for(K_FUSED4, batch, false);
  L.slots8 = np_max_t(n_max) >= kSplitT ? grid_for(K_FUSED8, batch, false) : 0;
  L.slotsr = tr > kRes6T ? grid_for(K_RES8, batch, false) : 0;  // the 8-wave resident kernel: np 112, 128
  L.slot8_doubles = (size_t)kFusedBufs * np * np;
  L.slot4_doubles = (size_t)kFusedBufs * np4 * np4;
  L.slotr_doubles = (size_t)kResParkDoublesPerT * tr;
  L.queue_off = 0;
  L.order_off = kAlign;
  L.key_off = L.order_off + align_up(sizeof(int32_t) * (size_t)batch);
  L.slots8_off = L.key_off + align_up((size_t)batch);
  L.slots4_off = L.slots8_off + align_up((size_t)L.slots8 * L.slot8_doubles * sizeof(double));
  L.slotsr_off = L.slots4_off + align_up((size_t)L.slots4 * L.slot4_doubles * sizeof(double));
  L.total = L.slotsr_off + (size_t)L.slotsr * L.slotr_doubles * sizeof(double);
  return L;
}

// ---- expm_batched_noalloc: the fused path's scratch in a device array of the library ----
// Real orders <= 128 only (the on-chip kernels: the global-memory kernels' slots are not
// needed), at most kNoAllocBatch matrices, at most kNoAllocSlots 8-wave resident workgroups
// (one per CU on MI355X).  Layout: queue words | order (int32 x batch) | cost keys (batch
// bytes) | park slots of the 8-wave resident kernel.
constexpr int64_t kNoAllocBatch = 65536;
constexpr int kNoAllocSlots = 256;
constexpr size_t kNoAllocParkOff = kAlign + ((sizeof(int32_t) * kNoAllocBatch + kAlign - 1) & ~(kAlign - 1)) +
                                   ((kNoAllocBatch + kAlign - 1) & ~(kAlign - 1));
constexpr size_t kScratchBytes =
    kNoAllocParkOff + (size_t)kNoAllocSlots * kResParkDoublesPerT * kResT * sizeof(double);  // 64.3 MiB

// Held by every device the library runs on until the process ends.  Host code never uses this
// name as an address: noalloc_scratch() looks up the device address once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up once per device, with that
// device current); nullptr on a HIP error.
void *noalloc_scratch() {
  static std::map<int, void *> per_dev;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  auto it = per_dev.find(dev);
  if (it != per_dev.end()) return it->second;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
  per_dev.emplace(dev, ptr);
  return ptr;
}

// Layout of the fused path's scratch inside `scratch` for `batch` matrices of real order
// <= 128: no global-memory slots; the 8-wave resident sweep gets at most kNoAllocSlots slots
// (its grid is capped to them).
FusedLayout noalloc_layout(int64_t nr_max, int64_t batch) {
  FusedLayout L;
  memset(&L, 0, sizeof(L));
  const int64_t tr = std::min<int64_t>(np_max_t(nr_max), kResT);
  L.slotsr = tr > kRes6T ? std::min(grid_for(K_RES8, batch, false), kNoAllocSlots) : 0;
  L.slotr_doubles = (size_t)kResParkDoublesPerT * tr;
  L.queue_off = 0;
  L.order_off = kAlign;
  L.key_off = L.order_off + align_up(sizeof(int32_t) * (size_t)batch);
  L.slots8_off = L.slots4_off = L.slotsr_off = kNoAllocParkOff;
  L.total = kNoAllocParkOff + (size_t)L.slotsr * L.slotr_doubles * sizeof(double);
  return L;
}

// Output tiles per launch of the tiled path for precision `prec` (tuned or the default).
int tiles_per_launch(int prec) {
  const int t = tune_now().tiles_per_launch[prec];
  return t > 0 ? t : kDefaultTiles;
}

// Second stream of the current device for the sweeps that run beside the 8-wave resident
// sweep (created once per device, default priority), with the fork and join events.  The
// mutex makes each call's record/wait pairs atomic, so concurrent host threads cannot
// interleave them.
struct ForkJoin {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_fj_mu;

bool fork_join_for_device(ForkJoin *out) {
  static std::map<int, ForkJoin> per_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  auto it = per_dev.find(dev);
  if (it == per_dev.end()) {
    ForkJoin f;
    if (hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&f.fork, hipEventDisableTiming) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&f.join, hipEventDisableTiming) != hipSuccess) return false;
    it = per_dev.emplace(dev, f).first;
  }
  *out = it->second;
  return true;
}

}  // namespace

extern "C" {

const char *expm_status_string(expm_status_t st) {
  switch (st) {
    case EXPM_OK: return "ok";
    case EXPM_E_INVALID_ARG: return "invalid argument";
    case EXPM_E_NONFINITE: return "non-finite input";
    case EXPM_E_WORKSPACE: return "workspace too small";
    case EXPM_E_HIP: return "HIP runtime error";
    case EXPM_E_UNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

expm_status_t expm_theta(int32_t m, double u, double *theta_out) {
  if (!theta_out) return EXPM_E_INVALID_ARG;
  return theta_of(m, u, theta_out) ? EXPM_OK : EXPM_E_INVALID_ARG;
}

expm_status_t expm_select_rule(const double *norms, int32_t sel, double u, int32_t *m_out,
                               int32_t *s_out) {
  if (!norms || !m_out || !s_out) return EXPM_E_INVALID_ARG;
  if (sel != EXPM_SEL_PLAIN && sel != EXPM_SEL_ALPHA) return EXPM_E_INVALID_ARG;
  if (!(norms[0] >= 0.0) || !isfinite(norms[0])) return EXPM_E_NONFINITE;
  Consts k;
  if (!make_consts(u, &k)) return EXPM_E_INVALID_ARG;
  int m, s;
  select_ms(k.theta, sel == EXPM_SEL_ALPHA, norms[0], norms[1], norms[2], &m, &s);
  *m_out = m;
  *s_out = s;
  return EXPM_OK;
}

// The reduced forms, the triangular refinement and the Paterson-Stockmeyer comparison above
// real order 16 run the tiled path (the Pade comparison exists for real orders <= 16 only).
static int64_t real_order(const expm_opts_t *o, int64_t n);
static bool tiled_only(const expm_opts_t *o, int64_t n = 0) {
  return o->prec != EXPM_PREC_FP64 || (o->flags & EXPM_FLAG_TRI) ||
         ((o->flags & (EXPM_FLAG_PS | EXPM_FLAG_PADE)) && real_order(o, n) > 16);
}
// Comparison methods on the fused kernels: FP64, plain rule, real order <= 16 (one wave per
// matrix), Pade only for the two printed rows of u.
static expm_status_t method_check(const expm_opts_t *o, int64_t n, double u) {
  if (o->flags == 0) return EXPM_OK;
  if (o->flags == EXPM_FLAG_TRI) return o->dtype == EXPM_F64 ? EXPM_OK : EXPM_E_UNSUPPORTED;
  if (o->prec != EXPM_PREC_FP64 || o->sel != EXPM_SEL_PLAIN) return EXPM_E_UNSUPPORTED;
  if ((o->flags & EXPM_FLAG_PADE) && (real_order(o, n) > kPadeNpMax || (u != 0x1p-53 && u != 0x1p-24)))
    return EXPM_E_UNSUPPORTED;
  return EXPM_OK;
}

// Order of the real matrix the method runs on: complex inputs use their real form (except on
// the tiled path's native complex route, which keeps the complex order; see native_complex).
static int64_t real_order(const expm_opts_t *o, int64_t n) { return o->dtype == EXPM_C128 ? 2 * n : n; }

// Complex inputs on the tiled path run natively (planar real and imaginary buffers, a complex
// product as four real MFMA products, (m, s) from the complex 1-norm) in FP64 with the
// product-reduced Taylor method or Paterson-Stockmeyer; the reduced-precision forms and Pade
// run on the real form.
static bool native_complex(const expm_opts_t *o) {
  return o->dtype == EXPM_C128 && o->prec == EXPM_PREC_FP64 && !(o->flags & EXPM_FLAG_PADE);
}

size_t expm_workspace_bytes(int64_t n_max, int64_t batch, const expm_opts_t *opts) {
  double u;
  if (n_max < 1 || batch < 1 || check_opts(opts, &u) != EXPM_OK) return 0;
  const int64_t nr = real_order(opts, n_max);
  if (nr <= kFusedNMax && !tiled_only(opts, n_max)) return fused_layout(nr, batch).total;
  if (native_complex(opts)) return large_layout(n_max, batch, opts->prec, tiles_per_launch(opts->prec), 2).total;
  return large_layout(nr, batch, opts->prec, tiles_per_launch(opts->prec), 1).total;
}

// stage: -1 all phases; 0 sort the batch into the work queue; 1 sweep of the 8-wave resident
// kernel (real orders 112..128); 2 sweeps of every other order, i.e. stages 3, 4, 5 in turn:
// 3 np 144..256 on the 8-wave global-memory kernel, 4 np 80..96 on the split-row resident
// kernel, 5 np 32..64 on the 4-wave resident kernel and np 16 on the one-wave kernel.
// Stages 1..5 need stage 0 first and are independent of each other.  Feature rows (learned
// selector) run on the global-memory kernels.
static expm_status_t run_fused(const void *A, void *E, const int64_t *offs, const int32_t *ns,
                               int64_t batch, int64_t n_uniform, int64_t n_max,
                               const expm_opts_t *opts, double u, int32_t *m_dev, int32_t *s_dev,
                               int32_t *status_dev, void *ws, size_t ws_bytes, void *stream,
                               int select_only, int stage = -1, double *features = nullptr,
                               const FusedLayout *given = nullptr) {
  // n_uniform and n_max are input orders; the kernels pad the real order.  `given`: a layout
  // of the caller's (the no-allocation variant), whose sweeps then all run on `stream`.
  const int cplx = opts->dtype == EXPM_C128;
  const int64_t nr_max = real_order(opts, n_max), nr_uni = real_order(opts, n_uniform);
  FusedLayout L = given ? *given : fused_layout(nr_max, batch);
  if (!ws || ws_bytes < L.total) return EXPM_E_WORKSPACE;
  if (((uintptr_t)ws) % kAlign) return EXPM_E_INVALID_ARG;
  FusedArgs a;
  memset(&a, 0, sizeof(a));
  if (!make_consts(u, &a.k)) return EXPM_E_INVALID_ARG;
  a.A = (const double *)A;
  a.E = (double *)E;
  a.offs = offs;
  a.ns = ns;
  a.m_out = m_dev;
  a.s_out = s_dev;
  a.status = status_dev;
  char *base = (char *)ws;
  a.batch = batch;
  a.n_uniform = (int)n_uniform;
  a.np_max = (int)pad16(nr_max);
  a.cplx = cplx;
  a.sel = opts->sel;  // every kernel runs all three rules
  a.method = (opts->flags & EXPM_FLAG_PS) ? 1 : (opts->flags & EXPM_FLAG_PADE) ? 2 : 0;
  a.select_only = select_only;
  a.features = features;
  a.lo = 0;
  a.hi = batch;
  hipStream_t st = (hipStream_t)stream;
  FusedArgs f8 = a, f4 = a, r8 = a, r6 = a, r4 = a, tn = a;
  f8.slots = (double *)(base + L.slots8_off);
  f8.slot_doubles = L.slot8_doubles;
  f4.slots = (double *)(base + L.slots4_off);
  f4.slot_doubles = L.slot4_doubles;
  r8.slots = L.slotsr > 0 ? (double *)(base + L.slotsr_off) : nullptr;
  r8.slot_doubles = L.slotr_doubles;
  r6.slots = r4.slots = tn.slots = nullptr;
  r6.slot_doubles = r4.slot_doubles = tn.slot_doubles = 0;
  // np = 16 runs one matrix per wave, except under the learned selector (whose network
  // lives with the workgroup kernels) or when tuned onto the 4-wave kernel
  const expm_tune_t tune = tune_now();
  const bool tiny = opts->sel != EXPM_SEL_LEARNED && tune.small_kernel != 2;
  const int tmax = np_max_t(nr_max);
  auto go = [&](Kern k, FusedArgs &x, int ctr, int lo, int hi) -> bool {
    x.q_ctr = ctr; x.q_lo = lo; x.q_hi = hi;
    int grid;
    hipError_t e;
    switch (k) {
      case K_FUSED8: grid = std::min(L.slots8, grid_for(K_FUSED8, batch)); e = launch_fused(x, 8, grid, st); break;
      case K_FUSED4: grid = std::min(L.slots4, grid_for(K_FUSED4, batch)); e = launch_fused(x, 4, grid, st); break;
      case K_RES8:
        grid = std::min(grid_for(K_RES8, batch), L.slotsr);
        if (grid < 1) return false;
        e = launch_resident(x, 8, grid, st);
        break;
      case K_RES6: grid = grid_for(K_RES6, batch); e = launch_resident(x, 12, grid, st); break;
      case K_TINY: grid = grid_for(K_TINY, batch); e = launch_tiny(x, grid, st); break;
      case K_RES4W: grid = grid_for(K_RES4W, batch); e = launch_resident(x, 5, grid, st); break;
      default:  // K_RES4: three workgroups per CU under the plain rule, two otherwise
        if (x.sel == EXPM_SEL_PLAIN) {
          grid = grid_for(K_RES4, batch);
          e = launch_resident(x, 4, grid, st);
        } else {
          grid = grid_for(K_RES4W, batch);
          e = launch_resident(x, 5, grid, st);
        }
        break;
    }
    return e == hipSuccess;
  };
  // queue words: counters 0 (np 144..256), 1 (112..128), 2 (80..96), 3 (32..64, or <= 64
  // without the one-wave kernel), 4 (feature rows of np <= 64), 5 (np 16); bounds
  // kQBound + 0..5 (see the order kernel)
  if (ns) {
    int32_t *order = (int32_t *)(base + L.order_off);
    unsigned long long *queue = (unsigned long long *)(base + L.queue_off);
    f8.order = f4.order = r8.order = r6.order = r4.order = tn.order = order;
    f8.queue = f4.queue = r8.queue = r6.queue = r4.queue = tn.queue = queue;
    uint8_t *key = (uint8_t *)(base + L.key_off);
    if ((stage == -1 || stage == 0) &&
        launch_order(a.A, offs, ns, (int)n_uniform, a.np_max, batch, cplx, key, order, queue, st) != hipSuccess)
      return EXPM_E_HIP;
    if (features) {
      // global-memory kernels: np >= 80 on 8 waves, the rest on 4 waves
      if (tmax >= kSplitT && !go(K_FUSED8, f8, 0, 0, 3)) return EXPM_E_HIP;
      if (!go(K_FUSED4, f4, 4, 3, 5)) return EXPM_E_HIP;
      return EXPM_OK;
    }
    // largest orders first; each sweep drains its own range of the sorted queue.  A full call
    // runs the sweeps as two chains on the caller's stream and a second stream (fork after
    // the sort, join before return), so the sweeps share the CUs instead of each waiting for
    // the previous one's last matrices.
    // sub-sweeps: 3 np 144..256, 4 np 80..96, 5 np 32..64 (np <= 64 without the one-wave
    // kernel), 6 np 16 on the one-wave kernel
    auto sub = [&](int k) -> bool {
      switch (k) {
        case 3: return tmax <= kResT || go(K_FUSED8, f8, 0, 0, 1);
        case 4: return tmax < kSplitT || go(K_RES6, r6, 2, 2, 3);
        case 5: return tiny ? go(K_RES4, r4, 3, 3, 4) : go(K_RES4, r4, 3, 3, 5);
        default: return !tiny || go(K_TINY, tn, 5, 4, 5);
      }
    };
    auto on = [&](hipStream_t s2, std::initializer_list<int> ks) -> bool {
      const hipStream_t keep = st;
      st = s2;
      bool ok = true;
      for (int k : ks) ok = ok && sub(k);
      st = keep;
      return ok;
    };
    if (stage == 1) return (tmax <= kRes6T || go(K_RES8, r8, 1, 1, 2)) ? EXPM_OK : EXPM_E_HIP;
    if (stage == 2) return on(st, {3, 4, 5, 6}) ? EXPM_OK : EXPM_E_HIP;
    if (stage == 5) return on(st, {5, 6}) ? EXPM_OK : EXPM_E_HIP;
    if (stage >= 3) return sub(stage) ? EXPM_OK : EXPM_E_HIP;
    if (stage == -1 && given) {
      // no second stream (creating one is not for callers that cannot allocate): the sweeps
      // in turn on the caller's stream
      if (!((tmax <= kRes6T || go(K_RES8, r8, 1, 1, 2)) && on(st, {3, 4, 5, 6}))) return EXPM_E_HIP;
    } else if (stage == -1 && tune.arrangement[opts->sel] == 1) {
      // every sweep in turn on the caller's stream
      if (!((tmax <= kRes6T || go(K_RES8, r8, 1, 1, 2)) && on(st, {3, 4, 5, 6}))) return EXPM_E_HIP;
    } else if (stage == -1) {
      std::lock_guard<std::mutex> lk(g_fj_mu);
      ForkJoin fj;
      if (!fork_join_for_device(&fj)) return EXPM_E_HIP;
      if (hipEventRecord(fj.fork, st) != hipSuccess || hipStreamWaitEvent(fj.side, fj.fork, 0) != hipSuccess)
        return EXPM_E_HIP;
      // two chains side by side; arrangement 0 (default, the best measured before tuning): np
      // 144..256, 80..96 and 16 on the second stream, 112..128 then 32..64 on the caller's;
      // 2: (144..256, 80..96) beside (112..128, 32..64, 16); 3: everything but 112..128 on the
      // second stream
      const int arr = tune.arrangement[opts->sel];
      const bool ok2 = arr == 2 ? on(fj.side, {3, 4}) : arr == 3 ? on(fj.side, {3, 4, 5, 6}) : on(fj.side, {3, 4, 6});
      const bool ok1 = (tmax <= kRes6T || go(K_RES8, r8, 1, 1, 2)) &&
                       (arr == 2 ? (sub(5) && sub(6)) : arr == 3 ? true : sub(5));
      if (hipEventRecord(fj.join, fj.side) != hipSuccess || hipStreamWaitEvent(st, fj.join, 0) != hipSuccess)
        return EXPM_E_HIP;
      if (!ok1 || !ok2) return EXPM_E_HIP;
    }
  } else {
    const int t = np_max_t(nr_uni);
    const Kern k = t > kResT ? K_FUSED8
                   : t > kRes6T ? K_RES8
                   : t >= kSplitT ? K_RES6
                   : (t == 1 && (tiny || a.method)) ? K_TINY
                   : t == kSplitT - 1 ? K_RES4W : K_RES4;
    bool ok;
    if (k != K_TINY && batch > grid_for(k, batch)) {
      // more matrices than one round of the persistent grid: walk a queue ordered by the cost
      // estimate (longest jobs first), the one order class's range of it
      int32_t *order = (int32_t *)(base + L.order_off);
      unsigned long long *queue = (unsigned long long *)(base + L.queue_off);
      uint8_t *key = (uint8_t *)(base + L.key_off);
      f8.order = r8.order = r6.order = r4.order = order;
      f8.queue = r8.queue = r6.queue = r4.queue = queue;
      if (launch_order(a.A, nullptr, nullptr, (int)n_uniform, a.np_max, batch, cplx, key, order, queue, st) != hipSuccess)
        return EXPM_E_HIP;
      ok = k == K_FUSED8 ? go(K_FUSED8, f8, 0, 0, 1)
           : k == K_RES8 ? go(K_RES8, r8, 1, 1, 2)
           : k == K_RES6 ? go(K_RES6, r6, 2, 2, 3)
                         : go(k, r4, 3, 3, 5);
    } else {
      // one matrix per workgroup at most (or one wave per matrix): the static range
      ok = k == K_FUSED8 ? go(K_FUSED8, f8, 0, 0, 0)
           : k == K_RES8 ? go(K_RES8, r8, 1, 0, 0)
           : k == K_RES6 ? go(K_RES6, r6, 2, 0, 0)
           : k == K_TINY ? go(K_TINY, tn, 5, 0, 0)
                         : go(k, r4, 3, 0, 0);
    }
    if (!ok) return EXPM_E_HIP;
  }
  return EXPM_OK;
}

static expm_status_t run_large_call(const void *A, void *E, int64_t n, int64_t batch, const expm_opts_t *opts,
                                    double u, int32_t *m_dev, int32_t *s_dev, int32_t *status_dev, void *ws,
                                    size_t ws_bytes, void *stream, int select_only) {
  if (((uintptr_t)ws) % kAlign) return EXPM_E_INVALID_ARG;
  const bool ps = (opts->flags & EXPM_FLAG_PS) != 0;
  if (ps && (opts->prec != EXPM_PREC_FP64 || opts->sel != EXPM_SEL_PLAIN)) return EXPM_E_UNSUPPORTED;
  LargeCall c;
  memset(&c, 0, sizeof(c));
  if (!make_consts(u, &c.k)) return EXPM_E_INVALID_ARG;
  c.A = (const double *)A;
  c.E = (double *)E;
  c.nin = n;
  c.cplx = opts->dtype != EXPM_C128 ? 0 : native_complex(opts) ? 2 : 1;
  c.batch = batch;
  c.sel = opts->sel == EXPM_SEL_LEARNED ? EXPM_SEL_ALPHA : opts->sel;
  c.prec = opts->prec;  // expm_prec_t values match PREC_F64 / PREC_F32 / PREC_BF16X3
  c.select_only = select_only;
  c.ps = ps ? 1 : 0;
  c.pade = (opts->flags & EXPM_FLAG_PADE) ? 1 : 0;
  c.tri = (opts->flags & EXPM_FLAG_TRI) ? 1 : 0;
  c.m_out = m_dev;
  c.s_out = s_dev;
  c.status = status_dev;
  c.tiles = tiles_per_launch(opts->prec);
  c.ws = ws;
  c.ws_bytes = ws_bytes;
  return run_large(c, (hipStream_t)stream);
}

expm_status_t expm_select(const void *A_dev, int64_t n, const expm_opts_t *opts, int32_t *m_dev,
                          int32_t *s_dev, void *ws_dev, size_t ws_bytes, void *stream) {
  double u;
  expm_status_t st = check_opts(opts, &u);
  if (st != EXPM_OK) return st;
  if (!A_dev || !m_dev || !s_dev || n < 1) return EXPM_E_INVALID_ARG;
  if ((st = method_check(opts, n, u)) != EXPM_OK) return st;
  if (real_order(opts, n) > kFusedNMax || tiled_only(opts, n))
    return run_large_call(A_dev, nullptr, n, 1, opts, u, m_dev, s_dev, nullptr, ws_dev, ws_bytes, stream, 1);
  return run_fused(A_dev, nullptr, nullptr, nullptr, 1, n, n, opts, u, m_dev, s_dev, nullptr,
                   ws_dev, ws_bytes, stream, 1);
}

expm_status_t expm_taylor(const void *A_dev, void *E_dev, int64_t n, const expm_opts_t *opts,
                          int32_t *m_dev, int32_t *s_dev, int32_t *status_dev, void *ws_dev,
                          size_t ws_bytes, void *stream) {
  double u;
  expm_status_t st = check_opts(opts, &u);
  if (st != EXPM_OK) return st;
  if (!A_dev || !E_dev || !m_dev || !s_dev || n < 1 || A_dev == E_dev) return EXPM_E_INVALID_ARG;
  if ((st = method_check(opts, n, u)) != EXPM_OK) return st;
  if (real_order(opts, n) > kFusedNMax || tiled_only(opts, n))
    return run_large_call(A_dev, E_dev, n, 1, opts, u, m_dev, s_dev, status_dev, ws_dev, ws_bytes, stream, 0);
  return run_fused(A_dev, E_dev, nullptr, nullptr, 1, n, n, opts, u, m_dev, s_dev, status_dev,
                   ws_dev, ws_bytes, stream, 0);
}

expm_status_t expm_batched(const void *A_dev, void *E_dev, const int64_t *offsets_dev,
                           const int32_t *n_dev, int64_t batch, int64_t n_max,
                           const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                           int32_t *status_dev, void *ws_dev, size_t ws_bytes, void *stream) {
  double u;
  expm_status_t st = check_opts(opts, &u);
  if (st != EXPM_OK) return st;
  if (!A_dev || !E_dev || !offsets_dev || !n_dev || !m_dev || !s_dev || batch < 1 || n_max < 1 ||
      A_dev == E_dev)
    return EXPM_E_INVALID_ARG;
  if (real_order(opts, n_max) > kFusedNMax || tiled_only(opts) || opts->flags) return EXPM_E_UNSUPPORTED;
  return run_fused(A_dev, E_dev, offsets_dev, n_dev, batch, 0, n_max, opts, u, m_dev, s_dev,
                   status_dev, ws_dev, ws_bytes, stream, 0);
}

expm_status_t expm_batched_noalloc(const void *A_dev, void *E_dev, const int64_t *offsets_dev,
                                   const int32_t *n_dev, int64_t batch, int64_t n_max, const expm_opts_t *opts,
                                   int32_t *m_dev, int32_t *s_dev, int32_t *status_dev, void *stream) {
  double u;
  expm_status_t st = check_opts(opts, &u);
  if (st != EXPM_OK) return st;
  if (!A_dev || !E_dev || !offsets_dev || !n_dev || !m_dev || !s_dev || batch < 1 || n_max < 1 ||
      A_dev == E_dev)
    return EXPM_E_INVALID_ARG;
  if (tiled_only(opts) || opts->flags) return EXPM_E_UNSUPPORTED;
  if (real_order(opts, n_max) > 16 * kResT || batch > kNoAllocBatch) return EXPM_E_WORKSPACE;
  void *ws = noalloc_scratch();
  if (!ws) return EXPM_E_HIP;
  const FusedLayout L = noalloc_layout(real_order(opts, n_max), batch);
  if (L.total > kScratchBytes) return EXPM_E_WORKSPACE;
  return run_fused(A_dev, E_dev, offsets_dev, n_dev, batch, 0, n_max, opts, u, m_dev, s_dev, status_dev, ws,
                   kScratchBytes, stream, 0, -1, nullptr, &L);
}

expm_status_t expm_batched_stage(const void *A_dev, void *E_dev, const int64_t *offsets_dev,
                                 const int32_t *n_dev, int64_t batch, int64_t n_max,
                                 const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                                 int32_t *status_dev, void *ws_dev, size_t ws_bytes, void *stream,
                                 int32_t stage) {
  double u;
  expm_status_t st = check_opts(opts, &u);
  if (st != EXPM_OK) return st;
  if (!A_dev || !E_dev || !offsets_dev || !n_dev || !m_dev || !s_dev || batch < 1 || n_max < 1 ||
      A_dev == E_dev || stage < 0 || stage > 5)
    return EXPM_E_INVALID_ARG;
  if (real_order(opts, n_max) > kFusedNMax || tiled_only(opts) || opts->flags) return EXPM_E_UNSUPPORTED;
  return run_fused(A_dev, E_dev, offsets_dev, n_dev, batch, 0, n_max, opts, u, m_dev, s_dev,
                   status_dev, ws_dev, ws_bytes, stream, 0, stage);
}

expm_status_t expm_batched_uniform(const void *A_dev, void *E_dev, int64_t n, int64_t batch,
                                   const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                                   int32_t *status_dev, void *ws_dev, size_t ws_bytes, void *stream) {
  double u;
  expm_status_t st = check_opts(opts, &u);
  if (st != EXPM_OK) return st;
  if (!A_dev || !E_dev || !m_dev || !s_dev || batch < 1 || n < 1 || A_dev == E_dev) return EXPM_E_INVALID_ARG;
  if ((st = method_check(opts, n, u)) != EXPM_OK) return st;
  if (real_order(opts, n) > kFusedNMax || tiled_only(opts, n))
    return run_large_call(A_dev, E_dev, n, batch, opts, u, m_dev, s_dev, status_dev, ws_dev, ws_bytes, stream, 0);
  return run_fused(A_dev, E_dev, nullptr, nullptr, batch, n, n, opts, u, m_dev, s_dev, status_dev,
                   ws_dev, ws_bytes, stream, 0);
}

expm_status_t expm_magnus4_step(const double *S0_dev, const double *S1_dev, int64_t s_stride, const double *Y_in_dev,
                                double *Y_out_dev, const double *u1_dev, const double *u2_dev, int64_t n,
                                int64_t batch, double h, const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                                int32_t *status_dev, void *stream) {
  double u;
  expm_status_t st = check_opts(opts, &u);
  if (st != EXPM_OK) return st;
  if (!S0_dev || !S1_dev || !Y_in_dev || !Y_out_dev || !u1_dev || !u2_dev || !m_dev || !s_dev || n < 1 ||
      batch < 1 || s_stride < 0 || !isfinite(h))
    return EXPM_E_INVALID_ARG;
  if (opts->dtype != EXPM_F64 || tiled_only(opts) || opts->flags || opts->sel == EXPM_SEL_LEARNED || n > 16)
    return EXPM_E_UNSUPPORTED;
  Consts k;
  if (!make_consts(u, &k)) return EXPM_E_INVALID_ARG;
  const int grid = grid_for(K_TINY, batch);
  return launch_magnus4(S0_dev, S1_dev, s_stride, Y_in_dev, Y_out_dev, u1_dev, u2_dev, (int)n, batch, h, opts->sel,
                        k, m_dev, s_dev, status_dev, grid, (hipStream_t)stream) == hipSuccess
             ? EXPM_OK
             : EXPM_E_HIP;
}

expm_status_t expm_features(const void *A_dev, const int64_t *offsets_dev, const int32_t *n_dev, int64_t batch,
                            int64_t n_max, const expm_opts_t *opts, double *features_dev, int32_t *m_dev,
                            int32_t *s_dev, void *ws_dev, size_t ws_bytes, void *stream) {
  double u;
  expm_status_t st = check_opts(opts, &u);
  if (st != EXPM_OK) return st;
  if (!A_dev || !offsets_dev || !n_dev || !features_dev || !m_dev || !s_dev || batch < 1 || n_max < 1)
    return EXPM_E_INVALID_ARG;
  if (opts->dtype != EXPM_F64 || tiled_only(opts) || opts->flags || n_max > kFusedNMax) return EXPM_E_UNSUPPORTED;
  return run_fused(A_dev, nullptr, offsets_dev, n_dev, batch, 0, n_max, opts, u, m_dev, s_dev, nullptr, ws_dev,
                   ws_bytes, stream, 1, -1, features_dev);
}

expm_status_t expm_tune_set(const expm_tune_t *t) {
  if (!t) return EXPM_E_INVALID_ARG;
  for (int k = 0; k < 3; ++k)
    if (t->arrangement[k] < 0 || t->arrangement[k] > 3) return EXPM_E_INVALID_ARG;
  if (t->small_kernel < 0 || t->small_kernel > 2) return EXPM_E_INVALID_ARG;
  for (int k = 0; k < 6; ++k)
    if (t->per_cu[k] < 0 || t->per_cu[k] > 64) return EXPM_E_INVALID_ARG;
  for (int k = 0; k < 4; ++k)
    if (t->tiles_per_launch[k] < 0 || t->tiles_per_launch[k] > (1 << 20)) return EXPM_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune = *t;
  return EXPM_OK;
}

expm_status_t expm_tune_get(expm_tune_t *t) {
  if (!t) return EXPM_E_INVALID_ARG;
  *t = tune_now();
  return EXPM_OK;
}

expm_status_t expm_tune_limits(expm_tune_t *t) {
  if (!t) return EXPM_E_INVALID_ARG;
  memset(t, 0, sizeof(*t));
  const FusedCaps c = fused_caps();
  if (c.cus == 0) return EXPM_E_HIP;
  t->arrangement[0] = t->arrangement[1] = t->arrangement[2] = 3;
  t->small_kernel = 2;
  t->per_cu[K_FUSED4] = c.per4; t->per_cu[K_FUSED8] = c.per8; t->per_cu[K_RES4] = c.res4;
  t->per_cu[K_RES6] = c.res6; t->per_cu[K_RES8] = c.res8; t->per_cu[K_TINY] = c.tiny;
  for (int k = 0; k < 4; ++k) t->tiles_per_launch[k] = kDefaultTiles;
  return EXPM_OK;
}

size_t expm_mlp_scratch_bytes(int32_t batch) {
  return batch < 1 ? 0 : mlp_scratch_floats(batch) * sizeof(float);
}

int32_t expm_mlp_param_count(void) { return kMlpParams; }

expm_status_t expm_mlp_forward(const float *params_dev, const float *x_dev, int32_t batch, float *logits_dev,
                               void *scratch_dev, size_t scratch_bytes, void *stream) {
  if (!params_dev || !x_dev || !logits_dev || !scratch_dev || batch < 1) return EXPM_E_INVALID_ARG;
  if (scratch_bytes < expm_mlp_scratch_bytes(batch)) return EXPM_E_WORKSPACE;
  return mlp_forward(params_dev, x_dev, batch, (float *)scratch_dev, logits_dev, (hipStream_t)stream) == hipSuccess
             ? EXPM_OK : EXPM_E_HIP;
}

expm_status_t expm_mlp_grad(const float *params_dev, const float *x_dev, const int32_t *y_dev, int32_t batch,
                            float *grads_dev, float *loss_dev, void *scratch_dev, size_t scratch_bytes, void *stream) {
  if (!params_dev || !x_dev || !y_dev || !grads_dev || !loss_dev || !scratch_dev || batch < 1)
    return EXPM_E_INVALID_ARG;
  if (scratch_bytes < expm_mlp_scratch_bytes(batch)) return EXPM_E_WORKSPACE;
  return mlp_grad(params_dev, x_dev, y_dev, batch, (float *)scratch_dev, grads_dev, loss_dev, (hipStream_t)stream) ==
                 hipSuccess ? EXPM_OK : EXPM_E_HIP;
}

expm_status_t expm_mlp_adam(float *params_dev, const float *grads_dev, float *m_dev, float *v_dev, int32_t step,
                            float lr, void *stream) {
  if (!params_dev || !grads_dev || !m_dev || !v_dev || step < 1 || !(lr > 0.0f)) return EXPM_E_INVALID_ARG;
  return mlp_adam_step(params_dev, grads_dev, m_dev, v_dev, step, lr, (hipStream_t)stream) == hipSuccess ? EXPM_OK
                                                                                                   : EXPM_E_HIP;
}

expm_status_t expm_learned_set(const float *params_dev, const double *norm_host, void *stream) {
  if (!params_dev || !norm_host) return EXPM_E_INVALID_ARG;
  for (int k = 0; k < kMlpIn; ++k)
    if (!(norm_host[kMlpIn + k] > 0.0) || !isfinite(norm_host[k])) return EXPM_E_INVALID_ARG;
  return learned_set(params_dev, norm_host, (hipStream_t)stream) == hipSuccess ? EXPM_OK : EXPM_E_HIP;
}

expm_status_t expm_learned_counts(int64_t *accepted, int64_t *rejected) {
  if (!accepted || !rejected) return EXPM_E_INVALID_ARG;
  unsigned long long c[2];
  if (learned_counts(c) != hipSuccess) return EXPM_E_HIP;
  *accepted = (int64_t)c[0];
  *rejected = (int64_t)c[1];
  return EXPM_OK;
}

}  // extern "C"
