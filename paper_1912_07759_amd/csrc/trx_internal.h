// Internal layout shared by the HIP sources of libtrx (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/trx.h"

namespace trx {

constexpr int kHdrBytes = 2048;    // per-model header block in the slab
// Word 3 of a raw 32-bit buffer resource (gfx9 family): the buffer loads of
// the table rows take the column as the per-lane offset, the row as the
// uniform offset.
constexpr int kRsrcWord3 = 0x00020000;
// CIA cross-sections (~1e-46 cm^5) are below the FP32 range and their layer
// weights 1e-10 rho^2 (up to ~1e42 m^-6) above it, so the FP32 copy of the
// CIA tables is stored multiplied by kCiaScale32 and the FP32 CIA weights
// divided by it.
constexpr double kCiaScale32 = 1e40;

// Per 16-layer block, the distinct table corners its layers interpolate
// between: at most 4 (T, P) corners of the cross-section grid and 2
// temperature nodes of the CIA grid per layer.
constexpr int kMaxU = 64;
constexpr int kMaxV = 32;
// Per model, the distinct corners of all its layers (ids sorted): kernels
// stage them once per work item when they fit their capacity.
constexpr int kMListU = 160;
constexpr int kMListV = 32;
struct alignas(16) MList {
  int32_t nU;            // distinct cross-section corners (may exceed kMListU)
  int32_t nV;            // distinct CIA nodes (may exceed kMListV)
  int32_t pad[2];
  int32_t ids[kMListU];
  int32_t tids[kMListV];
};
struct alignas(16) KBlk {
  int32_t nU;
  int32_t nV;
  int32_t ids[kMaxU];    // corner id iT * n_P + iP
  int32_t tids[kMaxV];   // CIA temperature node
  int32_t pad[2];
};
constexpr int kMaxSpecies = TRX_MAX_ABSORBERS + 2;
constexpr int kMaxRegimes = TRX_MAX_REGIMES;
// Slots of the matrix-core modes are tracked per 16-slot block in 64-bit
// masks: at most 1024 slots per model.
constexpr int kMaxSlots = 1024;

// Chemistry of one run of layers (two-layer profiles): mixing ratios of the
// absorbers, H2 and He, and the CIA pair weights chi_a chi_b.
struct alignas(16) RegChem {
  double chi_s[kMaxSpecies];
  double cia_w[TRX_MAX_CIA];
  float chi_s32[kMaxSpecies];
  float cia_w32[TRX_MAX_CIA];
};

// Per-model values written by the geometry kernel and read by every later
// kernel.  Lives at the start of each model's workspace slab.
struct ModelHdr {
  int32_t n;          // layers (0 when the model is invalid)
  int32_t status;     // TRX_MODEL_* bits
  int32_t lo, hi;     // window [lo, hi)
  int32_t nrb;        // 32-ray blocks = ceil(n / 32)
  int32_t nkb;        // 16-layer blocks = ceil(n / 16)
  int32_t span_lo, span_hi;  // spans covered by the window
  double Rp2_Rs2;     // (Rp/Rs)^2
  double inv_Rs2;     // 1/Rs^2
  double Rp, mu_kg;
  double chi_s[kMaxSpecies];        // absorbers, H2, He
  float chi_abs32[TRX_MAX_ABSORBERS];  // absorbers only, zero padded
  double cia_w[TRX_MAX_CIA];        // chi_a * chi_b per CIA pair
  float chi_s32[kMaxSpecies];
  float cia_w32[TRX_MAX_CIA];
  // matrix-core modes: bit kq of kq_mask[rb] is set when slot block kq of
  // ray block rb has a nonzero path x weight product (rays above every layer
  // of a slot block see none of it)
  uint64_t kq_mask[TRX_MAX_LAYERS_MFMA / 32];
  // 1 when a cloud deck adds optical depth to some ray; its per-ray depth
  // is then folded into the annulus weights (see the geometry kernel)
  int32_t cloud;
  // emission layouts: F_p/F_s = em_scale x (the flux ratio), em_scale =
  // (Rp/Rs)^2; em_star = c2 / T_star (so that h c nu / k_B T_star =
  // em_star x wavenumber)
  double em_scale;
  double em_star;
  // runs of one chemistry (two-layer layouts; 1 otherwise): their
  // chemistry is in the slab's RegChem records, run 0 (the deepest) also
  // in chi_s, cia_w and their FP32 copies above
  int32_t nreg;
};
static_assert(sizeof(ModelHdr) <= kHdrBytes, "header too large");

// Device copy of the tables.
struct DevTables {
  int32_t n_wn, n_T, n_P, n_abs, n_cia, n_Tcia;
  int32_t has_rayleigh;
  const double* wn;        // [n_wn]
  const double* T;         // [n_T]
  const double* logP;      // [n_P]
  const double* Tcia;      // [n_Tcia]
  const double* xsec64;    // [n_abs][n_T][n_P][n_wn]
  const float* xsec32;     // same layout in FP32
  const double* cia64;     // [n_cia][n_Tcia][n_wn]
  const float* cia32;      // same layout in FP32, times kCiaScale32
  const double* ray64;     // [n_abs+2][n_wn] (zeros when absent)
  const float* ray32;
  // exponential temperature scheme (t_exp = 1): per absorber [n_T][n_P][n_wn]
  // pairs (sigma, log2(sigma at the next T node / sigma)) in FP32, the ratio
  // NaN where the scheme falls back to linear
  int32_t t_exp;
  const float2* xexp32;
  double mass[kMaxSpecies];          // amu: absorbers, H2, He
  int32_t cia_pair[TRX_MAX_CIA][2];
};

// Per-model slab layout (byte offsets from the slab start).
struct Layout {
  int32_t NP;              // padded layer capacity (multiple of 32)
  int32_t NRB, NKB;        // NP/32, NP/16
  int32_t NKQ;             // 16-slot blocks of the opacity slots (matrix-core modes)
  int64_t off_z, off_A64, off_A32, off_lw64, off_lw32, off_lid, off_kblk, off_mlist, off_dl;
  int64_t off_sid;         // [16 NKQ] table row of each opacity slot (corners, then CIA nodes)
  int64_t off_aw;          // [NP] float2 (A_j/Rs^2, Rayleigh path weight of ray j)
  int64_t off_pr64;        // FP64 slot form: [NP] FP64 Rayleigh path weight of ray j
  int64_t off_pc64;        // [NP] FP64 optical depth of the cloud deck along ray j (+inf: opaque)
  // emission layouts: per layer l the records {c2/T_l, c2 (T_{l-1} - T_l)/(T_l T_{l-1}),
  // c2 (1/T_l - 1/T_star), vertical cloud optical depth down to the bottom of
  // shell l}, FP32 (float4) and FP64 (double4); c2 = 100 h c / k_B (K cm)
  int32_t em;
  int64_t off_em32, off_em64;
  // exponential temperature scheme (tables with t_exp): the absorber slots
  // are the layers themselves, top first (slot q = layer N-1-q, its mixed
  // cross-sections formed per column by the forward kernels), and per slot
  // its layer's record {u, w_P, w_T, 0}: the exponent of the ratio of the
  // two T nodes (u = w_T T2 / T), the log10 P weight and the linear T
  // weight of the fallback, FP32 (float4) and FP64 (double4)
  int32_t xt;
  int64_t off_xt32, off_xt64;
  // two-layer profiles (rg): the layers fall into runs of one chemistry
  // (at most kMaxRegimes, deepest first); the opacity slots are (run,
  // corner) and (run, CIA node) pairs and one Rayleigh slot per run, each
  // run's slots of one kind padded to a multiple of 8 (a staging group
  // mixes with one run's mixing ratios), ordered top run first; the slot
  // table entry of a slot is its row | run << 24.  RegChem records at
  // off_rg.
  int32_t rg;
  int64_t off_rg;
  int32_t slot64;          // FP64 mode in the slot form (models of at most TRX_MAX_LAYERS_MFMA layers)
  int64_t dl_bytes;        // mode-specific path-length storage
  // gradient layouts only (0 otherwise); the gradient takes models of at
  // most kKGM opacity slots:
  int64_t off_lwd64;       // [NP][8] FP64 d(record weight)/dT at fixed P
  int64_t off_pa;          // P (FP32), rows = rays: [NRB][kKGM/16][64][8], lane l, step i: k = 2 i + l/32
  int64_t off_pt;          // P^T as A fragments, rows = slots: [kKGM/32][NP/16][64][8]
  int32_t grad;
  int64_t slab;            // bytes per model (multiple of 256)
};

// Opacity slots the gradient supports per model (corners and CIA nodes),
// in chunks of kKG: a work item of the adjoint holds one chunk's rows and
// partial sums.
constexpr int kKG = 128;
constexpr int kKGM = 256;
constexpr int kGChunks = kKGM / kKG;

// Opacity slots of a model in the matrix-core modes: its distinct
// cross-section corners (at most 4 per layer, at most the grid's n_T n_P;
// one per layer in the exponential scheme) and its distinct CIA temperature
// nodes (at most 2 per layer).
inline int slot_capacity(const DevTables& t, int NP, bool rg = false) {
  if (rg) {
    const int R = kMaxRegimes, pad = 7 * kMaxRegimes;
    const int corners = (t.t_exp ? NP : std::min(4 * NP, R * t.n_T * t.n_P)) + pad;
    const int nodes = t.n_cia > 0 ? std::min(2 * NP, R * t.n_Tcia) + pad : 0;
    const int ray = t.has_rayleigh ? 8 : 0;
    return std::min(corners + nodes + ray, kMaxSlots);
  }
  const int corners = t.t_exp ? NP : std::min(4 * NP, t.n_T * t.n_P);
  const int nodes = t.n_cia > 0 ? std::min(2 * NP, t.n_Tcia) : 0;
  return corners + nodes;
}

// Number of stored pieces of the path-length products per mode.
inline int dl_pieces(int precision) {
  switch (precision) {
    case TRX_FP32: return 2;
    case TRX_BF16_SPLIT2: return 2;
    case TRX_BF16_SPLIT3: return 3;
    default: return 1;
  }
}

// Bytes of one (ray block, slot block) fragment piece: 64 lanes x 8 values.
inline int frag_piece_bytes(int precision) {
  return precision == TRX_FP32 ? 64 * 8 * 4 : 64 * 8 * 2;
}

inline Layout make_layout(int N_max, int precision, bool grad, const DevTables& t, bool emission = false,
                          bool regimes = false) {
  Layout L{};
  L.NP = ((N_max + 31) / 32) * 32;
  L.NRB = L.NP / 32;
  L.NKB = L.NP / 16;
  L.NKQ = (slot_capacity(t, L.NP, regimes) + 15) / 16;
  int64_t o = kHdrBytes;
  auto take = [&](int64_t bytes) { int64_t r = o; o += (bytes + 255) / 256 * 256; return r; };
  L.off_z = take(8LL * L.NP);
  L.off_A64 = take(8LL * L.NP);
  L.off_A32 = take(4LL * L.NP);
  L.off_pc64 = take(8LL * L.NP);
  L.off_lw64 = take(8LL * 8 * L.NP);
  L.off_lw32 = take(4LL * 8 * L.NP);
  // per layer: abs corner, CIA node, model-list slots (abs, CIA), block-list
  // slots (abs, CIA), 2 spare
  L.off_lid = take(4LL * 8 * L.NP);
  L.off_kblk = take((int64_t)sizeof(KBlk) * L.NKB);
  L.off_mlist = take((int64_t)sizeof(MList));
  if (emission) {
    L.em = 1;
    L.off_em32 = take(16LL * L.NP);
    L.off_em64 = take(32LL * L.NP);
  }
  if (t.t_exp) {
    L.xt = 1;
    // records by slot (two-layer layouts pad each run's layer slots)
    const int nslot = regimes ? 16 * L.NKQ : L.NP;
    L.off_xt32 = take(16LL * nslot);
    L.off_xt64 = take(32LL * nslot);
  }
  if (regimes) {
    L.rg = 1;
    L.off_rg = take((int64_t)sizeof(RegChem) * kMaxRegimes);
  }
  if (precision == TRX_FP64 && L.NP > TRX_MAX_LAYERS_MFMA) {
    L.dl_bytes = 8LL * L.NP * L.NP;  // dense transposed dlT[k][j]
  } else if (precision == TRX_FP64) {
    // P in FP64 as v_mfma_f64_16x16x4f64 A fragments [16-ray block][kq][lane][4]
    L.slot64 = 1;
    L.off_sid = take(4LL * 16 * L.NKQ);
    L.off_aw = take(8LL * L.NP);
    L.off_pr64 = take(8LL * L.NP);
    L.dl_bytes = (int64_t)(L.NP / 16) * L.NKQ * 64 * 4 * 8;
  } else {
    // P[j][q] = sum_l dl[j][l] W[l][q] in A-operand fragments [rb][kq][piece]
    L.off_sid = take(4LL * 16 * L.NKQ);
    L.off_aw = take(8LL * L.NP);
    L.dl_bytes = (int64_t)L.NRB * L.NKQ * dl_pieces(precision) * frag_piece_bytes(precision);
  }
  L.off_dl = take(L.dl_bytes);
  if (grad) {
    L.grad = 1;
    L.off_lwd64 = take(8LL * 8 * L.NP);
    L.off_pa = take(4LL * L.NRB * (kKGM / 16) * 64 * 8);
    L.off_pt = take(4LL * (kKGM / 32) * (L.NP / 16) * 64 * 8);
    if (L.off_sid == 0) {   // FP64 forward: the gradient still needs the slot table and ray weights
      L.off_sid = take(4LL * 16 * L.NKQ);
      L.off_aw = take(8LL * L.NP);
    }
  }
  L.slab = o;
  return L;
}

}  // namespace trx

namespace trx {

// Batch inputs as seen by the kernels (device pointers).
struct DevBatch {
  const int32_t* n_layers;
  const int64_t* layer_off;
  const double* T;
  const double* p_bot;
  const double* p_top;
  const double* log10_vmr;
  const double* Rp;
  const double* Rs;
  const double* GM;
  const int32_t* wn_lo;
  const int32_t* wn_hi;
  double he_h2, kB, amu;
  int32_t gravity;
  const double* cloud_sigma;   // [B] or null (then the next two are null too)
  const double* cloud_p1;
  const double* cloud_p2;
  const double* vmr_top;       // [B][n_abs] two-layer top values, or null (then vmr_sw too)
  const double* vmr_sw;        // [B][n_abs] switch pressures
};

struct GeomArgs {
  DevBatch bt;
  DevTables tab;
  Layout L;
  uint8_t* ws;            // slabs: model b at ws + b * L.slab
  const int32_t* B_dev;   // device model count (plans), or null
  int32_t B;              // host model count (used when B_dev is null)
  int32_t precision;
  int32_t n_limit;        // largest accepted layer count
  int32_t span_cols;      // columns per work span
  double* depth_native;   // [B][n_wn] or null: NaN written for invalid models
  int32_t* mlay;          // [B] layer count (0 for an invalid model)
  int2* mspan;            // [B] spans [lo, hi) of kSpanCols columns its window covers
  // emission (L.em): the path matrix takes the vertical shell thickness
  // instead of the chords, and the records of the Planck terms are written
  const double* T_star;   // [B] stellar temperature, K
  double c2;              // 100 h c / k_B, K cm
};

// Columns of one work item of the forward kernels.
constexpr int kSpanCols = 64;
// Work queues of the persistent launch (one per XCD of the MI355X).
constexpr int kQueues = 8;

__host__ __device__ inline ModelHdr* hdr_of(uint8_t* ws, const Layout& L, int b) {
  return reinterpret_cast<ModelHdr*>(ws + (int64_t)b * L.slab);
}

void launch_geom(const GeomArgs& a, int B_grid, hipStream_t s);
void launch_tau_cloud(const uint8_t* ws, const Layout& L, const int32_t* B_dev, int B, int max_layers, int W,
                      double* tau, hipStream_t s);

}  // namespace trx

namespace trx {

// Arguments of the opacity + optical depth + depth kernels.
struct FwdArgs {
  DevTables tab;
  Layout L;
  uint8_t* ws;
  const int32_t* B_dev;
  int32_t B;
  int32_t span_cols;      // columns per (model, span) work item
  int32_t n_spans;
  double* depth_native;   // [B][n_wn] or null
  void* aws;              // [B][n_wn] atmospheric part a/Rs^2 (double for FP64, else float)
  int32_t* model_status;  // [B]
  double* tau;            // [B][tau_ld] optical depth tau[b][j][column] (rows j < N, window columns), or null
  int64_t tau_ld;         // max_layers * n_wn
  // persistent scheduling: queue q holds the items (model, span) of the
  // spans s = q (mod kQueues); the models in order[] (layer count
  // descending) are taken in groups of `group`, each group over the queue's
  // spans in increasing order; workgroups pop chunks of items with atomics.
  const int32_t* order;   // [B] model indices, longest first
  const int2* mspan;      // [B] span range per model
  int32_t* qcount;        // [kQueues] item counters, zeroed by the schedule kernel
  int32_t persistent;     // 1: persistent grid, 0: one workgroup per (model, span)
  int32_t group;          // models per item group of the persistent order (0: all)
  int32_t span_group;     // consecutive spans per work item (matrix-core kernel)
  int32_t accurate;       // matrix-core modes: depth epilogue accurate per element (gradient's forward)
  // emission (L.em): Gauss-Legendre angles on [0, 1], n_mu of them:
  // em_k[i] = 1/mu_i, em_c[i] = 2 w_i mu_i (sum to 1)
  int32_t n_mu;
  float em_k32[TRX_MAX_MU];
  float em_c32[TRX_MAX_MU];
  double em_k64[TRX_MAX_MU];
  double em_c64[TRX_MAX_MU];
};

void launch_schedule(const int32_t* mlay, const int32_t* B_dev, int B, int32_t* order, int32_t* qcount,
                     hipStream_t s);

struct BinArgs {
  const uint8_t* ws;
  Layout L;
  const int32_t* B_dev;
  int32_t B;
  int32_t n_wn;
  int32_t n_ch;
  const int32_t* ch_i0;   // [n_ch] first native index overlapping channel c
  const int32_t* ch_i1;   // [n_ch] one past the last
  const int64_t* ch_off;  // [n_ch] offset of channel c's weights
  const double* ch_w;     // weights
  const void* aws;
  int32_t aws_f64;
  double* out;            // [B][n_ch]
};

// Per-model FP64 accumulators of the adjoint (offsets in doubles; the same
// offsets in floats for the work items' partial sums, whose slot adjoints
// cover one chunk: kp = kKG, against kp = kKGM for the model's sums).
struct GradAcc {
  int32_t NP, kp;
  int32_t o_A, o_z, o_h, o_T, o_Rp, o_S, o_chi, o_cw, o_PR, o_P, n;
};
__host__ __device__ inline GradAcc make_grad_acc(int NP, int kp = kKGM) {
  GradAcc g{};
  g.NP = NP;
  g.kp = kp;
  int o = 0;
  g.o_A = o; o += NP;          // dchi2/dA_j (A_j including 1/Rs^2)
  g.o_z = o; o += NP;          // dchi2/dz_j
  g.o_h = o; o += NP + 1;      // dchi2/dh_k, shell boundaries 0..N
  g.o_T = o; o += NP;          // dchi2/dT_l through the opacity
  g.o_Rp = o; o += 1;          // dchi2/dRp (explicit terms)
  g.o_S = o; o += 1;           // sum_i dchi2/dD_i (every point of the window)
  g.o_chi = o; o += kMaxSpecies;  // dchi2/dchi_s through the opacity
  g.o_cw = o; o += TRX_MAX_CIA;   // dchi2/d(chi_a chi_b) per CIA pair
  g.o_PR = o; o += NP;         // dchi2/dPR_j, Rayleigh path weight of ray j
  o = (o + 31) / 32 * 32;
  g.o_P = o; o += NP * kp;     // dchi2/dP[j][q], row j of kp slots
  g.n = (o + 31) / 32 * 32;
  return g;
}

// Arguments of the adjoint kernels.
struct AdjArgs {
  DevTables tab;
  Layout L;
  GradAcc G;              // the model's sums (acc)
  GradAcc Gp;             // a work item's partial sums (part): one slot chunk
  uint8_t* ws;
  DevBatch bt;
  const int32_t* B_dev;
  int32_t B;
  int32_t n_ch;
  const int32_t* ch_i0;
  const int32_t* ch_i1;
  const int64_t* ch_off;
  const double* ch_w;
  const int64_t* pt_off;  // [n_wn + 1] channels of native point i: pt_ch[pt_off[i] ..]
  const int32_t* pt_ch;
  const double* pt_w;     // their weights w_ci
  double* coef;           // [B][n_ch] dchi2/dD_c / sum_i w_ci
  const double* binned;   // [B][n_ch] forward result
  const double* obs;      // [B][n_ch]
  const double* sigma;    // [n_ch]
  double* chi2;           // [B]
  float* dbar;            // [B][n_wn] dchi2/dD_i inside the window
  double* acc;            // [B][G.n]
  float* part;            // [B][n_items][Gp.n] per-item partial sums
  int32_t n_spans;        // 64-column spans of the grid
  int32_t span_group;     // spans per backward work item
  int32_t n_items;        // work items per model: ceil(n_spans / span_group) span groups x kGChunks slot chunks
  double* dT;             // [layer_off[B]]
  double* dvmr;           // [B][n_abs]
  double* dRp;            // [B]
  int32_t* model_status;  // [B]
};
// spans per backward work item
constexpr int kAdjSpanGroup = 32;
size_t adj_item_lds_bytes(const Layout& L);
void launch_chi2_dbar(const AdjArgs& a, int B_grid, hipStream_t s);
hipError_t launch_adj_item(const AdjArgs& a, int B_grid, hipStream_t s);
void launch_adj_reduce(const AdjArgs& a, int B_grid, hipStream_t s);
void launch_adj_pmat(const AdjArgs& a, int B_grid, hipStream_t s);
void launch_adj_geom(const AdjArgs& a, int B_grid, hipStream_t s);

void launch_fwd64(const FwdArgs& a, int B_grid, hipStream_t s);
void launch_fwd_mfma(const FwdArgs& a, int precision, int nrb_max, int rbw, int occ, int B_grid, int n_cu,
                     hipStream_t s);
void launch_bin(const BinArgs& a, int B_grid, hipStream_t s);

}  // namespace trx
