// Matrix-core forward kernel for the FP32 and split-bf16 modes: opacity
// (a4), optical depth (a5) and depth (a6) of one (model, 64-column span) per
// workgroup of four waves.
//
// Staging.  At the start of a work item the workgroup stages in LDS, for its
// 64 columns, the mixed value M_q = sum_i chi_i sigma_i[q] of every distinct
// table corner q of the model (the tables share one (T, log10 P) grid, so the
// bilinear weights are common to all absorbers and the absorber sum is taken
// once per corner) and the CIA sums C_t = sum_pairs chi_a chi_b sigma_pair[t]
// at its temperature nodes.  Waves split the corners (corner ids are uniform
// scalar loads) and keep 16 table loads per lane in flight.  A model with
// more distinct corners than the staging capacity stages those of each
// 16-layer block instead.
//
// Per 16-layer block the workgroup then
//  1. computes the absorption coefficient of the block's layers, wave w taking
//     layers 4w..4w+3 with one column per lane:
//       kappa_l = sum_q w_lq M_q + w_R R + w_c0 C_0 + w_c1 C_1
//     (equations opt_dpth, cia_opt_dpth, contrib; Opacities section), the
//     weights (bilinear factors x 1e-4 rho, CIA factors x 1e-10 rho^2) and
//     corner slots being per-layer records of the geometry kernel read with
//     scalar loads, and writes kappa to LDS already in the B-operand layout
//     of the matrix instruction (split into bf16 pieces in the bf16 modes);
//  2. accumulates tau[ray, col] += dl[ray, layers of the block] x kappa on the
//     matrix cores: wave w owns the ray blocks w, w+4 (both 32-column blocks,
//     so each path-length fragment is read once), and a ray block only takes
//     the layer blocks at or above its first ray (the triangle).
//   FP32 mode: v_mfma_f32_32x32x2_f32, kappa in FP32, path lengths as two
//     FP32 pieces (hi + lo).
//   bf16 modes: v_mfma_f32_32x32x16_bf16 with both operands split into bf16
//     pieces x = x0 + x1 (+ x2); the products with piece-index sum < 2 (two
//     pieces: x0 y0 + x0 y1 + x1 y0) or < 3 (three pieces, six products) are
//     accumulated in FP32.
//
// Depth.  Each accumulator element is a (ray, column) optical depth; a wave
// adds (A_j/Rs^2)(1 - exp(-tau)) over the 32 rays of a block per column (two
// lanes per column, one cross-lane exchange) into a per-ray-block partial in
// LDS, and the partials are summed in ray-block order (same bits every run).
#include "trx_internal.h"
#include "stage.h"

namespace trx {

namespace {

using stage::kRsrcWord3;
using stage::stage_rows;
static_assert(stage::kWaves == 4 && stage::kCols == 64, "staging shape");

constexpr int kWaves = 4;
constexpr int kCols = 64;               // columns per workgroup
// staged rows: the cross-section corners, then the CIA nodes
constexpr int kRows = 96;
static_assert(kRows >= kMaxU + kMaxV, "block staging must fit");
static_assert(TRX_MAX_LAYERS_MFMA % 32 == 0 && TRX_MAX_LAYERS_MFMA <= 64 * kWaves,
              "a thread copies at most two record halves and one slot pair");
constexpr int kInFlight = 16;           // table loads per lane issued together
constexpr int kChunk = 8;               // items popped per atomic (persistent launch)

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int MODE>
struct Cfg {
  // bf16 pieces of each operand (FP32 mode: 1 kappa piece, 2 path pieces)
  static constexpr int npc = MODE == TRX_BF16_SPLIT3 ? 3 : (MODE == TRX_BF16_SPLIT2 ? 2 : 1);
  // dwords of the B-operand buffer: [piece][column block][lane][4] (bf16) or
  // [column block][step 0..7][lane] (FP32)
  static constexpr int frag_dw = MODE == TRX_FP32 ? 2 * 8 * 64 : npc * 2 * 64 * 4;
};

template <int MODE, int RBW>
struct Smem {
  float rows[kRows][kCols];
  // B-operand fragments of the current layer block; after the last block
  // the same space holds the per-ray-block depth partials
  union {
    __attribute__((aligned(16))) uint32_t frag[2][Cfg<MODE>::frag_dw];   // by layer-block parity
    float part[kWaves * RBW][kCols];
  };
  // per-item copies of the model's records (read with uniform LDS addresses)
  __attribute__((aligned(16))) float lw[TRX_MAX_LAYERS_MFMA][8];   // layer weights, [7] = A_l/Rs^2
  int2 sl[TRX_MAX_LAYERS_MFMA];                                     // corner slots
  int32_t ids[kRows];                                               // staged corner ids
  int32_t tids[kRows];                                              // staged CIA nodes
  float chi[TRX_MAX_ABSORBERS];
  float chis[kMaxSpecies];   // all species (Rayleigh)
  float ciaw[TRX_MAX_CIA];
  int32_t items[kChunk];
  int32_t spans[kChunk];
  int32_t base;
};

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// (a, b) rounded to bf16 (nearest even) and packed, a in the low half
__device__ inline uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ inline float bf16_lo_f(uint32_t p) { return __uint_as_float(p << 16); }
__device__ inline float bf16_hi_f(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

// Model-level staging of one span: the mixed corner rows, the CIA node
// rows and the Rayleigh sum of column `col`.  The loads of the CIA nodes
// (up to two pairs) and of eight Rayleigh species are issued ahead of the
// first corner batch, so their latency overlaps it.  Returns the Rayleigh sum.
template <int MODE, int RBW>
__device__ inline float stage_model(const DevTables& tb, const MList* ml, const Smem<MODE, RBW>& sm, float* rows,
                                    float* crows, int col, int wave, int lane) {
  const int W = tb.n_wn;
  const int nU = ml->nU, nV = ml->nV;
  const int voff = col * 4;
  const bool has_cia = tb.n_cia > 0;
  const int64_t cia_stride = (int64_t)tb.n_Tcia * W;
  const int crec = (int)(cia_stride * 4 < 0x7fffffff ? cia_stride * 4 : 0x7fffffff);
  constexpr int CG = 8;   // CIA nodes per wave (nV <= kMListV = kWaves * CG)
  static_assert(kMListV <= kWaves * CG, "one round covers the CIA nodes");
  float cv[2][CG];
  int npair = 0;
  if (has_cia && nV > 0) {
    npair = min(tb.n_cia, 2);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p < npair) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(tb.cia32 + (int64_t)p * cia_stride), (short)0, crec, kRsrcWord3);
#pragma unroll
        for (int g = 0; g < CG; ++g) {
          const int t = wave + kWaves * g < nV ? wave + kWaves * g : 0;
          cv[p][g] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
              r, voff, __builtin_amdgcn_readfirstlane(sm.tids[t]) * W * 4, 0));
        }
      }
    }
  }
  const int ns = tb.has_rayleigh ? tb.n_abs + 2 : 0;
  float rv[8];
  if (ns > 0) {
    const __amdgpu_buffer_rsrc_t rr =
        __builtin_amdgcn_make_buffer_rsrc((void*)tb.ray32, (short)0, ns * W * 4, kRsrcWord3);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      rv[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rr, voff, min(k, ns - 1) * W * 4, 0));
  }
  const int64_t abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  stage_rows(tb.xsec32, abs_stride, W, col, sm.ids, nU, sm.chi, tb.n_abs, rows, wave, lane);
  // CIA node rows: C_t = sum_p chi_a chi_b sigma_p[t]
  if (npair > 0) {
#pragma unroll
    for (int g = 0; g < CG; ++g) {
      const int t = wave + kWaves * g;
      if (t < nV) {
        float v = sm.ciaw[0] * cv[0][g];
        if (npair > 1) v = fmaf(sm.ciaw[1], cv[1][g], v);
        crows[t * kCols + lane] = v;
      }
    }
    if (tb.n_cia > 2) {
      // further pairs: added row by row
      for (int p = 2; p < tb.n_cia; ++p) {
        const float* tp = tb.cia32 + (int64_t)p * cia_stride;
        for (int t = wave; t < nV; t += kWaves)
          crows[t * kCols + lane] = fmaf(sm.ciaw[p], tp[(int64_t)sm.tids[t] * W + col], crows[t * kCols + lane]);
      }
    }
  }
  float R = 0.f;
  if (ns > 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < ns) R = fmaf(sm.chis[k], rv[k], R);
    for (int k = 8; k < ns; ++k) R = fmaf(sm.chis[k], tb.ray32[(int64_t)k * W + col], R);
  }
  return R;
}

// Ray block r (0..RBW-1) of a wave: w, then 7 - w, so that the long
// triangle rows (low ray blocks) and the short ones are dealt evenly.
template <int RBW>
__device__ __forceinline__ int own_rb(int wave, int r) {
  return r == 0 ? wave : 2 * kWaves - 1 - wave;
}
static_assert(TRX_MAX_LAYERS_MFMA <= 32 * 2 * kWaves, "two ray blocks per wave cover every ray");

// One work item: model b, columns [64 span, 64 span + 64).  Called by all
// threads of the workgroup (every early return is uniform).
// RBW: ray blocks per wave (ray blocks / 4, rounded up).
template <int MODE, int RBW>
__device__ __forceinline__ void process(const FwdArgs& a, int b_in, int s_first, int s_end, Smem<MODE, RBW>& sm) {
  using C = Cfg<MODE>;
  // the item is the same for the whole workgroup: keep it, and every address
  // derived from it, in scalar registers (scalar loads of the layer records)
  const int b = __builtin_amdgcn_readfirstlane(b_in);
  const Layout& L = a.L;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  const int N = hd->n;
  if (N == 0) return;
  const int lo = hd->lo, hi = hd->hi;
  // the item's spans that meet the model's window
  const int sp0 = __builtin_amdgcn_readfirstlane(max(s_first, lo / kCols));
  const int sp1 = __builtin_amdgcn_readfirstlane(min(s_end, (hi + kCols - 1) / kCols));
  if (sp0 >= sp1) return;
  // the wave index is uniform across the wave: keep it (and what derives
  // from it) in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const DevTables& tb = a.tab;
  const int W = tb.n_wn;
  const bool has_cia = tb.n_cia > 0;

  const float* lw = reinterpret_cast<const float*>(slab + L.off_lw32);
  const int32_t* lid = reinterpret_cast<const int32_t*>(slab + L.off_lid);
  const KBlk* kblk = reinterpret_cast<const KBlk*>(slab + L.off_kblk);
  const MList* ml = reinterpret_cast<const MList*>(slab + L.off_mlist);
  const uint8_t* frag = slab + L.off_dl;
  const int nkb = hd->nkb, nrb = hd->nrb;
  const int NKB = L.NKB;

  const int64_t abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  const int64_t cia_stride = (int64_t)tb.n_Tcia * W;
  float* rows = &sm.rows[0][0];
  float* crows = rows;   // CIA rows follow the staged corners
  const int tid = threadIdx.x;
  // copy the corner ids of the model (or of layer block kb) into LDS, then
  // stage the mixed rows
  auto stage = [&](const int32_t* ids, int nU, const int32_t* tids, int nV, int ccol) {
    for (int e = tid; e < nU; e += 64 * kWaves) sm.ids[e] = ids[e];
    for (int e = tid; e < nV; e += 64 * kWaves) sm.tids[e] = tids[e];
    __syncthreads();
    stage_rows(tb.xsec32, abs_stride, W, ccol, sm.ids, nU, sm.chi, tb.n_abs, rows, wave, lane);
    crows = rows + nU * kCols;
    if (has_cia) stage_rows(tb.cia32, cia_stride, W, ccol, sm.tids, nV, sm.ciaw, tb.n_cia, crows, wave, lane);
  };
  // whole-model staging when the distinct corners fit, else per layer block
  const bool mstage = ml->nU + ml->nV <= kRows && ml->nV <= kMListV;
  const int slot_off = mstage ? 2 : 4;
  // the model's records (and its corner lists) into LDS: all loads of a
  // thread are issued before its stores.  The 32 nrb >= N records copied
  // include the zero records of the padding layers, so every layer and ray
  // of the last blocks reads defined values.
  {
    const int nrec = 32 * nrb;
    const float4* src = reinterpret_cast<const float4*>(lw);
    float4* dst = reinterpret_cast<float4*>(&sm.lw[0][0]);
    const int n4 = 2 * nrec;
    const int e0 = tid, e1 = tid + 64 * kWaves;
    const float4 r0 = e0 < n4 ? src[e0] : float4{};
    const float4 r1 = e1 < n4 ? src[e1] : float4{};
    const int2 s0 = tid < nrec ? *reinterpret_cast<const int2*>(lid + 8 * tid + slot_off) : int2{};
    int u0 = 0, u1 = 0;
    if (mstage) {
      if (tid < ml->nU) u0 = ml->ids[tid];
      if (tid < ml->nV) u1 = ml->tids[tid];
    }
    if (e0 < n4) dst[e0] = r0;
    if (e1 < n4) dst[e1] = r1;
    if (tid < nrec) sm.sl[tid] = s0;
    if (mstage) {
      if (tid < ml->nU) sm.ids[tid] = u0;
      if (tid < ml->nV) sm.tids[tid] = u1;
    }
    if (tid < TRX_MAX_ABSORBERS) sm.chi[tid] = hd->chi_abs32[tid];
    if (tid < kMaxSpecies) sm.chis[tid] = hd->chi_s32[tid];
    if (tid < TRX_MAX_CIA) sm.ciaw[tid] = hd->cia_w32[tid];
  }
  __syncthreads();

  for (int span = sp0; span < sp1; ++span) {
  const int col0 = span * kCols;
  const int col = col0 + lane;
  const bool valid = col >= lo && col < hi;
  const int cc = valid ? col : lo;

  float R = 0.f;
  if (mstage) {
    crows = rows + ml->nU * kCols;
    R = stage_model(tb, ml, sm, rows, crows, cc, wave, lane);
  } else if (tb.has_rayleigh) {
    // Rayleigh sum over all species, eight loads in flight (species indexes
    // past the last are clamped and their terms skipped)
    const int ns = tb.n_abs + 2;
    const __amdgpu_buffer_rsrc_t rr =
        __builtin_amdgcn_make_buffer_rsrc((void*)tb.ray32, (short)0, ns * W * 4, kRsrcWord3);
    for (int s0 = 0; s0 < ns; s0 += 8) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        v[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rr, cc * 4, min(s0 + k, ns - 1) * W * 4, 0));
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (s0 + k < ns) R = fmaf(sm.chis[s0 + k], v[k], R);
    }
  }

  f32x16 acc[RBW][2];
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    acc[r][0] = f32x16{};
    acc[r][1] = f32x16{};
  }

  // path-length (A operand) fragments of this wave's ray blocks: those of
  // block kb + 1 are loaded right after the products of block kb, so their
  // latency overlaps the opacity of kb + 1
  constexpr int kAW = MODE == TRX_FP32 ? 4 : C::npc;   // 16-byte words per lane
  u32x4 Anx[RBW][kAW];
  auto load_A = [&](int kb) {
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      const int rb = own_rb<RBW>(wave, r);
      if (rb < nrb && kb >= 2 * rb) {
        if constexpr (MODE == TRX_FP32) {
          const u32x4* fp = reinterpret_cast<const u32x4*>(frag + ((int64_t)frag_index(rb, kb, NKB) * 2 * 512 +
                                                                   lane * 8) * 4);
          Anx[r][0] = fp[0];
          Anx[r][1] = fp[1];
          Anx[r][2] = fp[128];
          Anx[r][3] = fp[129];
        } else {
          const u32x4* fp = reinterpret_cast<const u32x4*>(
              frag + ((int64_t)frag_index(rb, kb, NKB) * C::npc * 512 + lane * 8) * 2);
#pragma unroll
          for (int p = 0; p < C::npc; ++p) Anx[r][p] = fp[p * 64];
        }
      }
    }
  };
  load_A(0);
  if (mstage) __syncthreads();   // staged rows visible

  for (int kb = 0; kb < nkb; ++kb) {
    if (!mstage) {
      // all waves are past the opacity of block kb - 1 (barrier below)
      const KBlk* kd = kblk + kb;
      stage(kd->ids, kd->nU, kd->tids, kd->nV, cc);
      __syncthreads();
    }
    uint32_t* fr = sm.frag[kb & 1];

    // 1. opacity of layers 16 kb + 4 wave + jj, one column per lane: the
    // slot words and weights of the wave's 4 layers first, then all their
    // row reads, then the arithmetic (two LDS round trips)
    float kap[4];
    {
      const int l0 = 16 * kb + 4 * wave;
      uint32_t sl[4], cl[4];
      float4 wa[4];
      float3 wb[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int2 t = sm.sl[l0 + jj];
        sl[jj] = __builtin_amdgcn_readfirstlane((uint32_t)t.x);
        cl[jj] = __builtin_amdgcn_readfirstlane((uint32_t)t.y);
        wa[jj] = *reinterpret_cast<const float4*>(&sm.lw[l0 + jj][0]);
        wb[jj] = *reinterpret_cast<const float3*>(&sm.lw[l0 + jj][4]);
      }
      float m[4][4], c[4][2];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        m[jj][0] = rows[(sl[jj] & 0xff) * kCols + lane];
        m[jj][1] = rows[((sl[jj] >> 8) & 0xff) * kCols + lane];
        m[jj][2] = rows[((sl[jj] >> 16) & 0xff) * kCols + lane];
        m[jj][3] = rows[(sl[jj] >> 24) * kCols + lane];
        if (has_cia) {
          c[jj][0] = crows[(cl[jj] & 0xff) * kCols + lane];
          c[jj][1] = crows[((cl[jj] >> 8) & 0xff) * kCols + lane];
        }
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        float k = wa[jj].x * m[jj][0];
        k = fmaf(wa[jj].y, m[jj][1], k);
        k = fmaf(wa[jj].z, m[jj][2], k);
        k = fmaf(wa[jj].w, m[jj][3], k);
        k = fmaf(wb[jj].x, R, k);
        if (has_cia) {
          k = fmaf(wb[jj].y, c[jj][0], k);
          k = fmaf(wb[jj].z, c[jj][1], k);
        }
        // layers past N have zero weights and slots (LDS rows are finite)
        kap[jj] = l0 + jj < N ? k : 0.f;
      }
    }
    const int cb = lane >> 5, lc = lane & 31;
    if constexpr (MODE == TRX_FP32) {
      // 32x32x2 step i holds layers 2i, 2i+1: lane 32 (k%2) + col%32
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int k = 4 * wave + jj;
        fr[(cb * 8 + (k >> 1)) * 64 + 32 * (k & 1) + lc] = __float_as_uint(kap[jj]);
      }
    } else {
      // 32x32x16: lane 32 (k/8) + col%32 holds layers 8 (k/8) .. +7 packed
      // by pairs; this wave's layers are k = 4 wave .. 4 wave + 3
      const int fl = 32 * (wave >> 1) + lc;
      const int d0 = 2 * (wave & 1);
      float x0 = kap[0], x1 = kap[1], x2 = kap[2], x3 = kap[3];
#pragma unroll
      for (int p = 0; p < C::npc; ++p) {
        const uint32_t q0 = bf16_pair(x0, x1), q1 = bf16_pair(x2, x3);
        uint32_t* dst = fr + ((p * 2 + cb) * 64 + fl) * 4 + d0;
        *reinterpret_cast<uint2*>(dst) = make_uint2(q0, q1);
        x0 -= bf16_lo_f(q0);
        x1 -= bf16_hi_f(q0);
        x2 -= bf16_lo_f(q1);
        x3 -= bf16_hi_f(q1);
      }
    }
    // one barrier per layer block: the fragments are double-buffered, and a
    // wave that rewrites this buffer (block kb + 2) has passed the barrier of
    // block kb + 1, which every wave reaches only after its products of kb
    __syncthreads();

    // 2. matrix products for this wave's ray blocks (B fragments read once
    // for both)
    bool any = false;
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      const int rb = own_rb<RBW>(wave, r);
      any |= rb < nrb && kb >= 2 * rb;
    }
    if (any) {
      if constexpr (MODE == TRX_FP32) {
        float bk[2][8];
#pragma unroll
        for (int tcb = 0; tcb < 2; ++tcb)
#pragma unroll
          for (int st = 0; st < 8; ++st) bk[tcb][st] = __uint_as_float(fr[(tcb * 8 + st) * 64 + lane]);
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          const int rb = own_rb<RBW>(wave, r);
          if (rb < nrb && kb >= 2 * rb) {
#pragma unroll
            for (int tcb = 0; tcb < 2; ++tcb) {
#pragma unroll
              for (int st = 0; st < 8; ++st) {
                const float ah = __uint_as_float(Anx[r][st >> 2][st & 3]);
                const float al = __uint_as_float(Anx[r][2 + (st >> 2)][st & 3]);
                acc[r][tcb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ah, bk[tcb][st], acc[r][tcb], 0, 0, 0);
                acc[r][tcb] = __builtin_amdgcn_mfma_f32_32x32x2f32(al, bk[tcb][st], acc[r][tcb], 0, 0, 0);
              }
            }
          }
        }
      } else {
        u32x4 Bp[2][C::npc];
#pragma unroll
        for (int tcb = 0; tcb < 2; ++tcb)
#pragma unroll
          for (int p = 0; p < C::npc; ++p)
            Bp[tcb][p] = *reinterpret_cast<const u32x4*>(fr + ((p * 2 + tcb) * 64 + lane) * 4);
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          const int rb = own_rb<RBW>(wave, r);
          if (rb < nrb && kb >= 2 * rb) {
#pragma unroll
            for (int tcb = 0; tcb < 2; ++tcb) {
#pragma unroll
              for (int pa = 0; pa < C::npc; ++pa) {
#pragma unroll
                for (int pb = 0; pb + pa < C::npc; ++pb)
                  acc[r][tcb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                      __builtin_bit_cast(bf16x8, Anx[r][pa]), __builtin_bit_cast(bf16x8, Bp[tcb][pb]),
                      acc[r][tcb], 0, 0, 0);
              }
            }
          }
        }
      }
    }
    if (kb + 1 < nkb) load_A(kb + 1);
  }
  (void)kblk;
  __syncthreads();   // the partials below reuse the fragment space

  // depth: accumulator register q holds ray 8 (q/4) + 4 (lane/32) + q%4
  const float nl2e = -1.4426950408889634f;
  const int hl = lane >> 5;
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = own_rb<RBW>(wave, r);
    if (rb < nrb) {
#pragma unroll
      for (int tcb = 0; tcb < 2; ++tcb) {
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const float A = sm.lw[32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3)][7];
          s = fmaf(A, 1.f - __builtin_amdgcn_exp2f(nl2e * acc[r][tcb][q]), s);
        }
        s += __shfl_xor(s, 32, 64);
        if (hl == 0) sm.part[rb][32 * tcb + (lane & 31)] = s;
      }
    }
  }
  __syncthreads();
  if (wave == 0 && valid) {
    float atm = 0.f;
    for (int rb = 0; rb < nrb; ++rb) atm += sm.part[rb][lane];
    const int64_t o = (int64_t)b * W + col;
    reinterpret_cast<float*>(a.aws)[o] = atm;
    if (a.depth_native) a.depth_native[o] = hd->Rp2_Rs2 + (double)atm;
    if (!isfinite(atm)) atomicOr(&a.model_status[b], TRX_MODEL_NONFINITE);
  }
  __syncthreads();   // rows, fragments and partials are rewritten by the next span
  }
}

// One workgroup per (model, span).
template <int MODE, int RBW>
__global__ __launch_bounds__(64 * kWaves) void k_fwd_mfma(FwdArgs a) {
  __shared__ Smem<MODE, RBW> sm;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if ((int)blockIdx.x >= B) return;
  const int S = a.span_group;
  process<MODE, RBW>(a, blockIdx.x, blockIdx.y * S, blockIdx.y * S + S, sm);
}

// Persistent: a fixed grid pops chunks of (span, model) items from kQueues
// queues, queue q holding the spans s = q (mod kQueues) in increasing order
// and, per span, the models longest first; a workgroup starts on the queue of
// its XCD (workgroups are dealt to the XCDs round-robin) so that the waves of
// one XCD share the table rows of few spans in its L2, and moves on to the
// other queues when its own is drained.  Every workgroup leaves once all
// queues are drained.
template <int MODE, int RBW>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(3))) void k_fwd_mfma_persist(FwdArgs a) {
  __shared__ Smem<MODE, RBW> sm;
  const int B = a.B_dev ? *a.B_dev : a.B;
  const int S = a.span_group;
  const int ngroups = ((a.tab.n_wn + kCols - 1) / kCols + S - 1) / S;
  const int q0 = blockIdx.x % kQueues;
  for (int k = 0; k < kQueues; ++k) {
    const int q = (q0 + k) % kQueues;
    const int nsq = q < ngroups ? (ngroups - q + kQueues - 1) / kQueues : 0;
    const int total = nsq * B;
    // items of queue q: model groups of G (in the order of order[]), within a
    // group the queue's span groups (S consecutive spans) in increasing
    // order, within a span group the group's models; G = B gives plain
    // span-major order
    const int G = a.group > 0 && a.group < B ? a.group : B;
    while (true) {
      if (threadIdx.x == 0) sm.base = total > 0 ? atomicAdd(&a.qcount[q], kChunk) : 0;
      __syncthreads();
      const int base = sm.base;
      if (threadIdx.x < kChunk) {
        const int i = base + threadIdx.x;
        int code = -1, sp = 0;
        if (i < total) {
          const int g = i / (nsq * G);
          const int rem = i - g * nsq * G;
          const int gm = min(G, B - g * G);
          const int ls = rem / gm;
          const int slot = g * G + (rem - ls * gm);
          sp = ls * kQueues + q;
          const int bm = a.order[slot];
          const int2 r = a.mspan[bm];
          if (r.x < (sp + 1) * S && r.y > sp * S) code = bm;
        }
        sm.items[threadIdx.x] = code;
        sm.spans[threadIdx.x] = sp;
      }
      __syncthreads();
      if (base >= total) break;
      for (int c = 0; c < kChunk; ++c) {
        const int bm = sm.items[c];
        if (bm >= 0) process<MODE, RBW>(a, bm, sm.spans[c] * S, sm.spans[c] * S + S, sm);
      }
      __syncthreads();
    }
  }
}

template <int MODE, int RBW>
int occupancy() {
  static int blocks = 0;
  if (!blocks) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_mfma_persist<MODE, RBW>, 64 * kWaves, 0) !=
            hipSuccess || nb < 1)
      nb = 1;
    blocks = nb;
  }
  return blocks;
}

template <int MODE, int RBW>
void launch_rbw(const FwdArgs& a, int B_grid, int n_cu, hipStream_t s) {
  if (a.persistent) {
    const int grid = n_cu * occupancy<MODE, RBW>();
    hipLaunchKernelGGL((k_fwd_mfma_persist<MODE, RBW>), dim3(grid), dim3(64 * kWaves), 0, s, a);
  } else {
    dim3 grid(B_grid, ((a.tab.n_wn + kCols - 1) / kCols + a.span_group - 1) / a.span_group);
    hipLaunchKernelGGL((k_fwd_mfma<MODE, RBW>), grid, dim3(64 * kWaves), 0, s, a);
  }
}

template <int MODE>
void launch_mode(const FwdArgs& a, int nrb, int B_grid, int n_cu, hipStream_t s) {
  if (nrb <= 4) launch_rbw<MODE, 1>(a, B_grid, n_cu, s);
  else launch_rbw<MODE, 2>(a, B_grid, n_cu, s);
}

}  // namespace

void launch_fwd_mfma(const FwdArgs& a, int precision, int nrb_max, int B_grid, int n_cu, hipStream_t s) {
  if (B_grid <= 0) return;
  switch (precision) {
    case TRX_FP32: launch_mode<TRX_FP32>(a, nrb_max, B_grid, n_cu, s); break;
    case TRX_BF16_SPLIT2: launch_mode<TRX_BF16_SPLIT2>(a, nrb_max, B_grid, n_cu, s); break;
    default: launch_mode<TRX_BF16_SPLIT3>(a, nrb_max, B_grid, n_cu, s); break;
  }
}

}  // namespace trx
