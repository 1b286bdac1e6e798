// Host-side handle definitions of libtrx (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "trx_internal.h"

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct trx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int n_cu = 256;
  char arch[64] = {0};
  DevBuf ws;    // per-model slabs
  DevBuf aws;   // native atmospheric depth
  DevBuf grad;  // gradient workspace
  DevBuf sched; // work order of the persistent launch
  // profiling (trx_profile)
  bool profile = false;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[TRX_KERNEL_CLASSES] = {0};
  int launches[TRX_KERNEL_CLASSES] = {0};
  bool capturing = false;
  bool no_events = false;   // trx_forward_noalloc: record no profiling events
};

struct trx_tables {
  trx_ctx* ctx = nullptr;
  trx::DevTables dev;
  std::vector<double> wn;     // host copy of the grid
  std::vector<void*> owned;
};

struct trx_bins {
  trx_ctx* ctx = nullptr;
  const trx_tables* tables = nullptr;
  int n_ch = 0;
  int32_t* i0 = nullptr;
  int32_t* i1 = nullptr;
  int64_t* off = nullptr;
  double* w = nullptr;
  // the same weights by native point: point i lies in the channels
  // pch[poff[i] .. poff[i+1]) (ascending) with weights pw
  int64_t* poff = nullptr;
  int32_t* pch = nullptr;
  double* pw = nullptr;
  std::vector<void*> owned;
};

namespace trx {

// Launch-shape choices of one run (the autotuner's search space).
struct RunConfig {
  int span_cols = kSpanCols;  // columns per (model, span) work item
  int nrb_max = 7;            // ray-block capacity of the matrix-core kernel
  int persistent = 1;         // 1: persistent grid with work queues
  int group = 0;              // models per item group of the persistent order (0: all)
  int span_group = 4;         // consecutive 64-column spans per work item
  int rbw = 0;                // matrix-core kernel: 32-ray blocks per wave (1 or 2; 0: 1 up to 128 rays)
  int occ = 3;                // workgroups per CU the persistent kernel is built for (4: 128
                              // registers, smaller staging batches, two ray blocks in two passes)
};

// Scheduling buffers of one launch (device memory).
struct SchedBufs {
  int32_t* mlay = nullptr;   // [B]
  int2* mspan = nullptr;     // [B]
  int32_t* order = nullptr;  // [B]
  int32_t* qcount = nullptr; // [kQueues]
  static size_t bytes(int B) { return (size_t)B * 16 + 256; }
  static SchedBufs carve(void* base, int B) {
    SchedBufs s;
    uint8_t* p = (uint8_t*)base;
    s.mspan = (int2*)p;
    s.mlay = (int32_t*)(p + (size_t)B * 8);
    s.order = (int32_t*)(p + (size_t)B * 12);
    s.qcount = (int32_t*)(p + (size_t)B * 16);
    return s;
  }
};

trx_status set_err(trx_ctx* c, trx_status s, const char* fmt, ...);

// Brackets a kernel launch with profiling events when profiling is on.
struct ProfScope {
  trx_ctx* c;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(trx_ctx* ctx, int k);
  ~ProfScope();
};
trx_status hip_err(trx_ctx* c, hipError_t e, const char* what);
trx_status ensure_buffer(trx_ctx* c, DevBuf& buf, size_t bytes, const char* what);
trx_status upload(trx_ctx* c, const double* host, int64_t n, double** d64, float** d32,
                  std::vector<void*>& owned, double scale32 = 1.0);
void launch_copy_status(const uint8_t* ws, int64_t slab, const int32_t* B_dev, int B, int32_t* out,
                        hipStream_t s);
trx_status check_batch(trx_ctx* c, const trx_tables* t, const trx_batch* bt, int precision);

// Emission inputs of one launch (a null pointer: transmission).
struct EmissionIn {
  const double* T_star;   // [B] device, K
  int n_mu;               // Gauss-Legendre angles, 1..TRX_MAX_MU
};
// Checks the emission arguments of a call (n_mu, star pointer, layer limit).
trx_status check_emission(trx_ctx* c, int precision, int max_layers, const double* T_star, int n_mu);
// n Gauss-Legendre abscissas and weights on [0, 1] (weights sum to 1).
void gauss_legendre01(int n, double* mu, double* w);
DevBatch dev_batch(const trx_batch* bt);
RunConfig default_config(int precision, int max_layers);
trx_status enqueue_forward(trx_ctx* c, const trx_tables* t, const DevBatch& db, int B, const int32_t* B_dev,
                           int max_layers, const trx_bins* bins, int precision, const RunConfig& rc,
                           uint8_t* ws, void* aws, const SchedBufs& sb, double* depth_native,
                           double* depth_binned, int32_t* status, bool grad_layout = false,
                           double* tau = nullptr, const EmissionIn* em = nullptr, bool regimes = false);

// Gradient workspace carved from one buffer (base null: sizes only).
struct GradScratch {
  double* acc;        // [B][G.n] per-model FP64 accumulators
  double* binned;     // [B][n_ch] binned depth when the caller asks for none
  double* coef;       // [B][n_ch] dchi2/dD_c over the channel's weight sum
  float* dbar;        // [B][n_wn] dchi2/dD_i
  float* part;        // [B][n_items][G.n] per-item partial sums
  size_t bytes;
};
GradScratch carve_grad_scratch(void* base, int B, int n_wn, int n_ch, int NP);
size_t grad_scratch_bytes(int B, int n_wn, int n_ch, int NP);
// Forward pass on the gradient layout, chi^2, and the adjoint kernels.
// alloc: grow the buffers as needed (false: they are already large enough).
trx_status enqueue_chi2_grad(trx_ctx* c, const trx_tables* t, const DevBatch& db, int B, const int32_t* B_dev,
                             int max_layers, const trx_bins* bins, int precision, const RunConfig& rc,
                             DevBuf& ws, DevBuf& aws, DevBuf& sched, DevBuf& grad, const double* obs,
                             const double* sigma, double* chi2, double* dT, double* dvmr, double* dRp,
                             double* depth_binned, int32_t* status, bool alloc = true);

}  // namespace trx
