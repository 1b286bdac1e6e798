// Adjoint of chi^2 = sum_c ((D_c - O_c)/sigma_c)^2 (a8) with respect to the
// per-layer temperatures, the log10 mixing ratios and Rp, in recompute mode:
// the optical depth of the forward pass is not stored but recomputed per
// work item.
//
// The forward model in the slot form of the matrix-core kernels: per model
// and wavenumber column c,
//   tau_j = sum_q P[j][q] M_q + PR_j R,  P = dl W,  PR = dl w_R,
//   D = Rp^2/Rs^2 + sum_j A_j (1 - e^{-tau_j}),
// with M_q the mixed cross-section of opacity slot q (a table corner,
// sum_i chi_i sigma_i[q], or a CIA node, sum_p w_p sigma_p[t]), R the mixed
// Rayleigh cross-section, W[l][q] the interpolation x density weights of
// layer l and dl the chords (Forward Models section; equations opt_dpth,
// cia_opt_dpth, contrib, tot_opt_dpth).  Reverse, per model:
//   Dbar_c = 2 (D_c - O_c)/sigma_c^2, Dbar_i = sum_c Dbar_c w_ci / sum_i' w_ci'
//   (binning, Binning subsection);
//   taubar_j = Dbar A_j e^{-tau_j},  Abar_j = sum_i Dbar_i (1 - e^{-tau_j});
//   Mbar = P^T taubar,  Rbar = PR^T taubar                (per column)
//   Pbar = sum_c taubar M^T,  PRbar = sum_c taubar R      (over all columns)
//   chibar_i = sum_c sum_q Mbar_q sigma_i[q], the CIA weights and the
//   Rayleigh species likewise;
// and once per model in FP64, from Pbar:
//   Wbar = dl^T Pbar  ->  Tbar_l = sum_q Wbar[l][q] dW[l][q]/dT_l (bracket
//   slopes and d rho/dT at fixed P),
//   dlbar = Pbar W^T  ->  zbar_j, hbar_m, Rpbar through the chords
//   dl[j][l] = 2 (Q_{j,l+1} - Q_{j,l}), Q_{j,m} = sqrt((h_m - z_j)(2 Rp + h_m + z_j)).
// A last per-model kernel walks the annulus weights, the shell boundaries,
// the altitude recursion and the chemistry (fill gases follow the sum
// constraint; log10 parameters) in reverse, in FP64.
//
// The work item is one model over a group of consecutive 64-column spans;
// its products take FP32 operands (P rounded from FP64) split into three
// bf16 pieces on v_mfma_f32_32x32x16_bf16 (FP32 accuracy), Pbar is
// accumulated in registers over the item's spans and each
// item writes its partial sums once; a per-model kernel adds them in a
// fixed order in FP64.  The result is held to 1e-4 of the FP64 reference
// gradient.
#include "trx_internal.h"

namespace trx {

namespace {

constexpr int kWaves = 8;
constexpr int kCols = 64;
constexpr int kLd = 65;   // LDS row stride of the [row][column] tiles: transposed reads hit distinct banks
constexpr int kAS = 4;    // tables per load batch in the staging
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
static_assert(kKG % 32 == 0 && kKG <= 4 * 32, "slot blocks of the gradient: one Mbar tile per wave");
static_assert(TRX_MAX_LAYERS_MFMA <= 32 * kWaves, "one ray block per wave");
constexpr int kWavesL = 12;   // waves of the workgroups of layouts above 128 rays
static_assert((TRX_MAX_LAYERS_MFMA / 32) * (kKG / 32) <= 3 * kWavesL, "three Pbar tiles per wave of 12 cover every layout");

// v of another lane of the same 16-lane row (DPP lane move; CTRL is the
// data-parallel-primitive control: quad permutations, row mirrors)
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
// sum over each 16-lane row, in every lane of the row: pairs, quads, the
// two halves of the row, then the two mirrored halves
__device__ inline float row_sum(float v) {
  v += dpp_mov<0xB1>(v);    // quad permutation (1, 0, 3, 2)
  v += dpp_mov<0x4E>(v);    // quad permutation (2, 3, 0, 1)
  v += dpp_mov<0x141>(v);   // mirror within each half-row (lane 7 - i)
  v += dpp_mov<0x140>(v);   // mirror within the row (lane 15 - i)
  return v;
}
__device__ inline float wave_sum(float v) {
  v = row_sum(v);
  v += __shfl_xor(v, 16, 64);
  return v + __shfl_xor(v, 32, 64);
}
__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// sum over the 32 lanes of a half-wave
__device__ inline float half_sum(float v) {
  v = row_sum(v);
  return v + __shfl_xor(v, 16, 64);
}

// Products on v_mfma_f32_32x32x16_bf16 at FP32 accuracy: each operand is
// split into three bf16 pieces (x = hi + mid + lo to about 2^-24 of x) and
// the six piece products with index sum below three are accumulated (the
// dropped ones are below 2^-24 of the product).  Lane l supplies the same 8
// operand values as for eight v_mfma_f32_32x32x2f32 steps, k = 2 v + l/32
// for step v: the bf16 instruction reads them as k = 8 (l/32) + v, the same
// permutation of k on both operands, which leaves the sum unchanged.
__device__ inline void split3(const float (&x)[8], u32x4 (&p)[3]) {
  float r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = x[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // (r[2i], r[2i+1]) rounded to bf16 (nearest even), r[2i] in the low half
      const uint32_t q = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{r[2 * i], r[2 * i + 1]}, bf16x2));
      p[c][i] = q;
      if (c < 2) {
        r[2 * i] -= __uint_as_float(q << 16);
        r[2 * i + 1] -= __uint_as_float(q & 0xffff0000u);
      }
    }
  }
}
__device__ inline f32x16 mfma3(const u32x4 (&a)[3], const u32x4 (&b)[3], f32x16 c) {
  auto m = [](u32x4 x, u32x4 y, f32x16 z) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, x), __builtin_bit_cast(bf16x8, y), z,
                                                   0, 0, 0);
  };
  c = m(a[2], b[0], c);
  c = m(a[1], b[1], c);
  c = m(a[0], b[2], c);
  c = m(a[1], b[0], c);
  c = m(a[0], b[1], c);
  return m(a[0], b[0], c);
}
// acc += A B over one 16-deep block, from each lane's 8 values of A and B
__device__ inline f32x16 mfma_block(const float (&av)[8], const float (&bv)[8], f32x16 acc) {
  u32x4 ap[3], bp[3];
  split3(av, ap);
  split3(bv, bp);
  return mfma3(ap, bp, acc);
}

// ---- chi^2 and the per-point cotangent Dbar_i ---------------------------
// Dbar_c = 2 (D_c - O_c)/sigma_c^2 per channel; Dbar_i = sum_c Dbar_c w_ci /
// sum_i' w_ci' per native point, summed over the point's channels in
// ascending order (no atomics: the same bits every run).
__global__ __launch_bounds__(256) void k_chi2_dbar(AdjArgs a) {
  constexpr int kW = 4;   // waves of this kernel
  const int b = blockIdx.x;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const uint8_t* slab = a.ws + (int64_t)b * a.L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  double* acc = a.acc + (int64_t)b * a.G.n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < a.G.n; e += 256) acc[e] = 0.0;
  const int N = hd->n;
  if (N == 0) {
    if (tid == 0) a.chi2[b] = __builtin_nan("");
    return;
  }
  const int lo = hd->lo, hi = hd->hi, W = a.tab.n_wn;
  double* coef = a.coef + (int64_t)b * a.n_ch;
  __shared__ double s_part[2][kW];
  double c2 = 0.0, sd = 0.0;
  for (int c = wave; c < a.n_ch; c += kW) {
    const int c0 = a.ch_i0[c];
    const int i0 = max(c0, lo), i1 = min(a.ch_i1[c], hi);
    const double* w = a.ch_w + a.ch_off[c] - c0;
    double ws = 0.0;
    for (int i = i0 + lane; i < i1; i += 64) ws += w[i];
    ws = wave_sum_d(ws);
    const double sg = a.sigma[c];
    const double r = (a.binned[(int64_t)b * a.n_ch + c] - a.obs[(int64_t)b * a.n_ch + c]) / sg;
    const double db = 2.0 * r / sg;
    c2 += r * r;
    sd += db;
    if (lane == 0) coef[c] = ws > 0.0 ? db / ws : 0.0;
  }
  if (lane == 0) {
    s_part[0][wave] = c2;
    s_part[1][wave] = sd;
  }
  __syncthreads();   // coef of every channel written (workgroup-scope fence)
  float* dbar = a.dbar + (int64_t)b * W;
  for (int i = lo + tid; i < hi; i += 256) {
    double t = 0.0;
    for (int64_t k = a.pt_off[i]; k < a.pt_off[i + 1]; ++k) t = fma(coef[a.pt_ch[k]], a.pt_w[k], t);
    dbar[i] = (float)t;
  }
  if (tid == 0) {
    double t2 = 0.0, ts = 0.0;
    for (int w = 0; w < kW; ++w) {
      t2 += s_part[0][w];
      ts += s_part[1][w];
    }
    a.chi2[b] = t2;
    // D_i = (Rp/Rs)^2 + ...: sum_i Dbar_i = sum_c Dbar_c
    acc[a.G.o_Rp] = ts * 2.0 * hd->Rp * hd->inv_Rs2;
    acc[a.G.o_S] = ts;
  }
}

// ---- per (model, span group): recompute and backward --------------------
struct ItemLds {
  float* rows;   // [kKG][kLd] mixed slot rows M of the span, later their adjoints
  float* tbar;   // [NP][kLd] taubar of the span
  float2* aw;    // [NP] (A_j/Rs^2, PR_j)
  float* rpart;  // [waves][64] Rayleigh sums by wave
  float* rbp;    // [NRB][64] Rbar of the span by ray block
  int32_t* sid;  // [kKG] table row of each slot
  float* chi;    // [TRX_MAX_ABSORBERS]
  float* ciaw;   // [TRX_MAX_CIA]
  float* chis;   // [kMaxSpecies]
  // this item's partial sums, each element written by one lane only (the
  // same bits every run): Abar_j and PRbar_j by column block [2][NP],
  // chibar and the CIA-weight adjoints by wave [waves][kMaxSpecies],
  // [waves][TRX_MAX_CIA]
  float* abp;
  float* prp;
  float* chp;
  float* cwp;
};

__host__ __device__ inline size_t carve(const Layout& L, const GradAcc& G, int nw, unsigned char* base,
                                        ItemLds* out) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + o : nullptr;
    o += (bytes + 15) / 16 * 16;
    return p;
  };
  ItemLds s;
  s.rows = (float*)take((size_t)kKG * kLd * 4);
  s.tbar = (float*)take((size_t)L.NP * kLd * 4);
  s.aw = (float2*)take((size_t)L.NP * 8);
  s.rpart = (float*)take((size_t)nw * kCols * 4);
  s.rbp = (float*)take((size_t)L.NRB * kCols * 4);
  s.sid = (int32_t*)take(kKG * 4);
  s.chi = (float*)take(TRX_MAX_ABSORBERS * 4);
  s.ciaw = (float*)take(TRX_MAX_CIA * 4);
  s.chis = (float*)take(kMaxSpecies * 4);
  s.abp = (float*)take((size_t)2 * L.NP * 4);
  s.prp = (float*)take((size_t)2 * L.NP * 4);
  s.chp = (float*)take((size_t)nw * kMaxSpecies * 4);
  s.cwp = (float*)take((size_t)nw * TRX_MAX_CIA * 4);
  if (out) *out = s;
  return o;
}

// s[i] += sum_t wt[t] tab_t[rows[i]][col] for the slots i in [i0, i1) of a
// group of 8 (tables t < nt at tab + t stride); rows of the other slots are
// clamped into the range (their loads are in bounds, their values unused).
__device__ inline void mix_group(const float* tab, int64_t stride, int nt, const float* wt, const int32_t* rows,
                                 int i0, int i1, int W, int voff, float (&s)[8]) {
  const int rec = (int)(stride * 4 < 0x7fffffff ? stride * 4 : 0x7fffffff);
  int soff[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = i < i0 ? i0 : (i >= i1 ? i1 - 1 : i);
    soff[i] = __builtin_amdgcn_readfirstlane(rows[k]) * W * 4;
  }
  for (int t0 = 0; t0 < nt; t0 += kAS) {
    float v[kAS][8];
#pragma unroll
    for (int tt = 0; tt < kAS; ++tt) {
      if (t0 + tt < nt) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(tab + (int64_t)(t0 + tt) * stride), (short)0, rec, kRsrcWord3);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[tt][i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff[i], 0));
      }
    }
#pragma unroll
    for (int tt = 0; tt < kAS; ++tt) {
      if (t0 + tt < nt) {
        const float c = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(wt[t0 + tt])));
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (i >= i0 && i < i1) s[i] = fmaf(c, v[tt][i], s[i]);
      }
    }
  }
}

// PT Pbar tiles per wave, NW waves per workgroup: 8 waves of two tiles cover
// 128 rays x 128 slots in 128 registers, so that two workgroups share a CU
// (the LDS of a 128-ray layout allows it, four waves per SIMD); 12 waves of
// three tiles cover 224 rays in 168 registers, one workgroup per CU (its LDS
// takes about 100 KB), three waves per SIMD.  MULTI: the build for models
// of more than one slot chunk (one item per span group and chunk); the other
// build takes the models of one chunk (one item per span group) without the
// code of the chunk loop.
template <int PT, int NW, bool MULTI>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(PT == 2 ? 4 : 3)))
void k_adj_item(AdjArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  const int B = a.B_dev ? *a.B_dev : a.B;
  const int b = __builtin_amdgcn_readfirstlane(blockIdx.x);
  if (b >= B) return;
  // work item: span group g, slot chunk c (the item's P adjoints and its
  // rows' mixing-ratio adjoints cover the chunk's slots; the optical depth
  // is recomputed over every chunk)
  const int by = __builtin_amdgcn_readfirstlane(blockIdx.y);
  const int grp = MULTI ? by / kGChunks : by, c = MULTI ? by - grp * kGChunks : 0;
  const int item = grp * kGChunks + c;   // the slot of this item's partial sums
  const Layout& L = a.L;
  const GradAcc& G = a.Gp;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  const int N = hd->n;
  if (N == 0) return;
  const int lo = hd->lo, hi = hd->hi;
  const int S = a.span_group;
  const int sp0 = max(grp * S, lo / kCols), sp1 = min(grp * S + S, (hi + kCols - 1) / kCols);
  if (sp0 >= sp1) return;
  const MList* ml = reinterpret_cast<const MList*>(slab + L.off_mlist);
  const int nUm = ml->nU, Km = nUm + ml->nV;
  if (Km > kKGM) {
    // more opacity slots than the gradient's capacity: not built here
    if (threadIdx.x == 0) atomicOr(&a.model_status[b], TRX_MODEL_GRAD_UNSUPPORTED);
    return;
  }
  if (MULTI != (Km > kKG)) return;   // the other build's model
  const int nch = MULTI ? (Km + kKG - 1) / kKG : 1;
  if (c >= nch) return;
  // the slots of chunk k: [kKG k, kKG k + K_k), corners first
  auto chunk_K = [&](int k) { return min(Km - kKG * k, kKG); };
  auto chunk_nU = [&](int k) { return min(max(nUm - kKG * k, 0), kKG); };
  const int K = chunk_K(c), nU = chunk_nU(c);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int hl = lane >> 5, lc = lane & 31;
  const DevTables& tb = a.tab;
  const int W = tb.n_wn;
  const int nrb = hd->nrb, NR = 32 * nrb;
  const int nqb = (K + 31) / 32;                  // 32-slot blocks of the own chunk
  const int NJB = L.NP / 16;
  const int64_t abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  const int64_t cia_stride = (int64_t)tb.n_Tcia * W;
  const float* pa = reinterpret_cast<const float*>(slab + L.off_pa);
  const float* pt = reinterpret_cast<const float*>(slab + L.off_pt);
  ItemLds s;
  carve(L, G, NW, dyn, &s);
  const int32_t* sidg = reinterpret_cast<const int32_t*>(slab + L.off_sid);

  // records: ray weights (zero past N), slot rows, mixing ratios
  {
    const float2* awg = reinterpret_cast<const float2*>(slab + L.off_aw);
    if (tid < NR) s.aw[tid] = awg[tid];
    // one chunk: its slot rows for every span of the item
    if (nch == 1 && tid < K) s.sid[tid] = sidg[tid];
    if (tid < TRX_MAX_ABSORBERS) s.chi[tid] = hd->chi_abs32[tid];
    if (tid < TRX_MAX_CIA) s.ciaw[tid] = hd->cia_w32[tid];
    if (tid < kMaxSpecies) s.chis[tid] = hd->chi_s32[tid];
    for (int e = tid; e < 2 * L.NP; e += 64 * NW) {
      s.abp[e] = 0.f;
      s.prp[e] = 0.f;
    }
    for (int e = tid; e < NW * kMaxSpecies; e += 64 * NW) s.chp[e] = 0.f;
    for (int e = tid; e < NW * TRX_MAX_CIA; e += 64 * NW) s.cwp[e] = 0.f;
  }
  __syncthreads();
  float* chp = s.chp + wave * kMaxSpecies;   // this wave's chibar partials
  float* cwp = s.cwp + wave * TRX_MAX_CIA;

  // Pbar tiles (32 rays x 32 slots) of this wave, t = wave + 8 u, kept in
  // registers over the item's spans
  constexpr int kPT = PT;
  f32x16 pb[kPT];
#pragma unroll
  for (int u = 0; u < kPT; ++u) pb[u] = f32x16{};
  const int ns = tb.has_rayleigh ? tb.n_abs + 2 : 0;
  // the per-ray and Rayleigh adjoints are the first chunk's items' (they do
  // not depend on the slots)
  const bool first_chunk = c == 0;

  for (int span = sp0; span < sp1; ++span) {
    const int col0 = span * kCols;
    const int col = col0 + lane;
    const bool valid = col >= lo && col < hi;
    const int cc = valid ? col : lo;
    const int voff = cc * 4;

    // the Rayleigh sums
    {
      float rp = 0.f;
      for (int k = wave; k < ns; k += NW) rp = fmaf(s.chis[k], tb.ray32[(int64_t)k * W + cc], rp);
      s.rpart[wave * kCols + lane] = rp;
    }
    // tau = P M + PR R over the chunks, the own chunk last so that its rows
    // stay staged: M of chunk k's slots (zero past its end), then this
    // wave's tiles (32 rays x 32 columns) over the chunk's nonzero 16-slot
    // blocks; the sums over the other chunks wait in the taubar tile of
    // LDS (each tile is one wave's), the last chunk's go on to taubar, and
    // for the first chunk's items to Abar, PRbar and Rbar
    for (int kk = 0; kk < nch; ++kk) {
      const int k = (c + 1 + kk) % nch;
      const int Kk = chunk_K(k), nUk = chunk_nU(k);
      const bool last = kk == nch - 1;
      if (nch > 1) {
        if (kk > 0) __syncthreads();   // the previous chunk's rows are consumed
        if (tid < Kk) s.sid[tid] = sidg[kKG * k + tid];
        __syncthreads();
      }
      for (int g = wave; g < 4 * ((Kk + 31) / 32); g += NW) {
        const int s0 = 8 * g;
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = 0.f;
        const int nc = min(max(nUk - s0, 0), 8);
        if (nc > 0) mix_group(tb.xsec32, abs_stride, tb.n_abs, s.chi, s.sid + s0, 0, nc, W, voff, v);
        const int vb = min(max(Kk - s0, 0), 8);
        if (vb > nc) mix_group(tb.cia32, cia_stride, tb.n_cia, s.ciaw, s.sid + s0, nc, vb, W, voff, v);
#pragma unroll
        for (int i = 0; i < 8; ++i) s.rows[(s0 + i) * kLd + lane] = v[i];
      }
      __syncthreads();
      const int nkq = (Kk + 15) / 16;
      for (int t = wave; t < 2 * nrb; t += NW) {
        const int rb = t >> 1, tcb = t & 1;
        const int c2 = 32 * tcb + lc;
        // nonzero slot blocks of the ray block within the chunk (each
        // block's fragment loaded at its turn: prefetching the next one
        // costs more in spilled registers than it hides)
        uint64_t m = (hd->kq_mask[rb] >> ((kKG / 16) * k)) & ((1ull << nkq) - 1ull);
        f32x16 tau = f32x16{};
        if (kk > 0) {
#pragma unroll
          for (int q = 0; q < 16; ++q) tau[q] = s.tbar[(32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3)) * kLd + c2];
        }
        auto afrag = [&](int kq, u32x4& x0, u32x4& x1) {
          const u32x4* fp = reinterpret_cast<const u32x4*>(
              pa + (((int64_t)rb * (kKGM / 16) + (kKG / 16) * k + kq) * 64 + lane) * 8);
          x0 = fp[0];
          x1 = fp[1];
        };
        u32x4 a0{}, a1{};
        int kq = m ? __builtin_ctzll(m) : -1;
        while (kq >= 0) {
          m &= m - 1;
          const int kn = m ? __builtin_ctzll(m) : -1;
          afrag(kq, a0, a1);
          float av[8], bv[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            av[i] = __uint_as_float(i < 4 ? a0[i] : a1[i - 4]);
            bv[i] = s.rows[(16 * kq + 2 * i + hl) * kLd + 32 * tcb + lc];
          }
          tau = mfma_block(av, bv, tau);
          kq = kn;
        }
        if (!last) {
#pragma unroll
          for (int q = 0; q < 16; ++q) s.tbar[(32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3)) * kLd + c2] = tau[q];
          continue;
        }
        float Rc = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) Rc += s.rpart[w * kCols + c2];
        const int cg = col0 + c2;
        const float Db = (cg >= lo && cg < hi) ? a.dbar[(int64_t)b * W + cg] : 0.f;
        float rs = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int j = 32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3);
          const float2 w = s.aw[j];
          const float x = fmaf(w.y, Rc, tau[q]);
          const float tv = Db * w.x * __expf(-x);
          s.tbar[j * kLd + c2] = tv;
          if (first_chunk) {
            rs = fmaf(w.y, tv, rs);
            // column sums of the annulus and Rayleigh-path cotangents of ray j
            const float ab = half_sum(-Db * expm1f(-x));
            const float pr = half_sum(tv * Rc);
            if (lc == 0 && j < N) {
              s.abp[tcb * L.NP + j] += ab;
              s.prp[tcb * L.NP + j] += pr;
            }
          }
        }
        if (first_chunk) {
          rs += __shfl_xor(rs, 32, 64);
          if (hl == 0) s.rbp[rb * kCols + c2] = rs;
        }
      }
    }
    __syncthreads();

    // Pbar += taubar M^T over the span's 64 columns (tiles of nonzero P)
#pragma unroll
    for (int u = 0; u < kPT; ++u) {
      const int t = wave + NW * u;
      if (t < nrb * nqb) {
        const int rb = t / nqb, qb = t - rb * nqb;
        if ((hd->kq_mask[rb] >> ((kKG / 16) * c + 2 * qb)) & 3) {
          const float* ar = s.tbar + (32 * rb + lc) * kLd + hl;
          const float* br = s.rows + (32 * qb + lc) * kLd + hl;
#pragma unroll 1
          for (int k16 = 0; k16 < 4; ++k16) {
            float av[8], bv[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              av[v] = ar[2 * (8 * k16 + v)];
              bv[v] = br[2 * (8 * k16 + v)];
            }
            pb[u] = mfma_block(av, bv, pb[u]);
          }
        }
      }
    }
    // Mbar = P^T taubar: tile (32 slots x 32 columns) t = wave
    f32x16 mb = f32x16{};
    const bool has_mb = wave < 2 * nqb;
    if (has_mb) {
      const int qb = wave >> 1, tcb = wave & 1;
      // 16-ray blocks with a nonzero product
      uint32_t jm = 0;
      for (int jb = 0; jb < 2 * nrb; ++jb)
        if ((hd->kq_mask[jb >> 1] >> ((kKG / 16) * c + 2 * qb)) & 3) jm |= 1u << jb;
      auto tfrag = [&](int jb, u32x4& x0, u32x4& x1) {
        const u32x4* fp = reinterpret_cast<const u32x4*>(
            pt + (((int64_t)((kKG / 32) * c + qb) * NJB + jb) * 64 + lane) * 8);
        x0 = fp[0];
        x1 = fp[1];
      };
      u32x4 a0{}, a1{};
      int jb = jm ? __builtin_ctz(jm) : -1;
      while (jb >= 0) {
        jm &= jm - 1;
        const int jn = jm ? __builtin_ctz(jm) : -1;
        tfrag(jb, a0, a1);
        float av[8], bv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          av[i] = __uint_as_float(i < 4 ? a0[i] : a1[i - 4]);
          bv[i] = s.tbar[(16 * jb + 2 * i + hl) * kLd + 32 * tcb + lc];
        }
        mb = mfma_block(av, bv, mb);
        jb = jn;
      }
    }
    __syncthreads();   // M is no longer read: its rows take Mbar
    if (has_mb) {
      const int qb = wave >> 1, tcb = wave & 1;
#pragma unroll
      for (int q = 0; q < 16; ++q) s.rows[(32 * qb + 8 * (q >> 2) + 4 * hl + (q & 3)) * kLd + 32 * tcb + lc] = mb[q];
    }
    __syncthreads();

    // mixing-ratio adjoints: corner rows against each absorber's table,
    // CIA node rows against each pair's table, Rbar against each species'
    // Rayleigh row
    {
      const int rec = (int)(abs_stride * 4 < 0x7fffffff ? abs_stride * 4 : 0x7fffffff);
      // corners x absorbers in flight: the 8-wave kernel's 128 registers
      // spill with four absorbers per batch (11.2 vs 12.0 ms with two)
      constexpr int DG = 8, DA = NW == 8 ? 2 : 4;
      for (int i0 = 0; i0 < tb.n_abs; i0 += DA) {
        float acc_i[DA] = {};
        for (int u0 = wave; u0 < nU; u0 += NW * DG) {
          int soff[DG];
#pragma unroll
          for (int g = 0; g < DG; ++g) {
            const int u = u0 + NW * g < nU ? u0 + NW * g : u0;
            soff[g] = __builtin_amdgcn_readfirstlane(s.sid[u]) * W * 4;
          }
          float v[DA][DG];
#pragma unroll
          for (int ii = 0; ii < DA; ++ii) {
            if (i0 + ii < tb.n_abs) {
              const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                  (void*)(tb.xsec32 + (int64_t)(i0 + ii) * abs_stride), (short)0, rec, kRsrcWord3);
#pragma unroll
              for (int g = 0; g < DG; ++g)
                v[ii][g] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff[g], 0));
            }
          }
#pragma unroll
          for (int ii = 0; ii < DA; ++ii) {
            if (i0 + ii < tb.n_abs) {
#pragma unroll
              for (int g = 0; g < DG; ++g)
                if (u0 + NW * g < nU) acc_i[ii] = fmaf(s.rows[(u0 + NW * g) * kLd + lane], v[ii][g], acc_i[ii]);
            }
          }
        }
#pragma unroll
        for (int ii = 0; ii < DA; ++ii) {
          if (i0 + ii < tb.n_abs) {
            const float t = wave_sum(acc_i[ii]);
            if (lane == 0) chp[i0 + ii] += t;
          }
        }
      }
      // CIA: the wave's nodes t = nU + wave + 8 k (at most kCN) of every
      // pair, all loads issued before the sums
      constexpr int kCN = 4;
      for (int p0 = 0; p0 < tb.n_cia; p0 += 2) {
        float cv[2][kCN];
#pragma unroll
        for (int pp = 0; pp < 2; ++pp)
#pragma unroll
          for (int k = 0; k < kCN; ++k) {
            const int t = nU + wave + NW * k;
            cv[pp][k] = (p0 + pp < tb.n_cia && t < K)
                            ? tb.cia32[(int64_t)(p0 + pp) * cia_stride + (int64_t)s.sid[t] * W + cc]
                            : 0.f;
          }
#pragma unroll
        for (int pp = 0; pp < 2; ++pp) {
          if (p0 + pp < tb.n_cia) {
            float acc_p = 0.f;
#pragma unroll
            for (int k = 0; k < kCN; ++k) {
              const int t = nU + wave + NW * k;
              if (t < K) acc_p = fmaf(s.rows[t * kLd + lane], cv[pp][k], acc_p);
            }
            acc_p = wave_sum(acc_p);
            if (lane == 0) cwp[p0 + pp] += acc_p;
          }
        }
      }
      // nodes past kCN per wave (more than 32 CIA nodes)
      for (int p = 0; p < tb.n_cia; ++p) {
        const float* tp = tb.cia32 + (int64_t)p * cia_stride;
        float acc_p = 0.f;
        for (int t = nU + wave + NW * kCN; t < K; t += NW)
          acc_p = fmaf(s.rows[t * kLd + lane], tp[(int64_t)s.sid[t] * W + cc], acc_p);
        if (nU + wave + NW * kCN < K) {
          acc_p = wave_sum(acc_p);
          if (lane == 0) cwp[p] += acc_p;
        }
      }
      // Rayleigh: the wave's species q = wave + 8 k, loads first (first
      // chunk's items only)
      float rl = 0.f;
      const int nsr = first_chunk ? ns : 0;
      for (int rb = 0; rb < nrb; ++rb) rl += s.rbp[rb * kCols + lane];
      constexpr int kRS = (kMaxSpecies + NW - 1) / NW;
      float rv[kRS];
#pragma unroll
      for (int k = 0; k < kRS; ++k) {
        const int q = wave + NW * k;
        rv[k] = q < nsr ? tb.ray32[(int64_t)q * W + cc] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < kRS; ++k) {
        const int q = wave + NW * k;
        if (q < nsr) {
          const float t = wave_sum(rl * rv[k]);
          if (lane == 0) chp[q] += t;
        }
      }
    }
    __syncthreads();   // rows, tbar and rbar are rewritten by the next span
  }

  // this item's partial sums, reduced per model in a fixed order later
  float* dst = a.part + ((int64_t)b * a.n_items + item) * G.n;
  for (int e = tid; e < G.o_P; e += 64 * NW) {
    float v = 0.f;
    if (e >= G.o_A && e < G.o_A + L.NP) {
      v = s.abp[e - G.o_A] + s.abp[L.NP + e - G.o_A];
    } else if (e >= G.o_PR && e < G.o_PR + L.NP) {
      v = s.prp[e - G.o_PR] + s.prp[L.NP + e - G.o_PR];
    } else if (e >= G.o_chi && e < G.o_chi + kMaxSpecies) {
      for (int w = 0; w < NW; ++w) v += s.chp[w * kMaxSpecies + e - G.o_chi];
    } else if (e >= G.o_cw && e < G.o_cw + TRX_MAX_CIA) {
      for (int w = 0; w < NW; ++w) v += s.cwp[w * TRX_MAX_CIA + e - G.o_cw];
    }
    dst[e] = v;
  }
#pragma unroll
  for (int u = 0; u < kPT; ++u) {
    const int t = wave + NW * u;
    if (t < nrb * nqb) {
      const int rb = t / nqb, qb = t - rb * nqb;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int j = 32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3);
        dst[G.o_P + j * G.kp + 32 * qb + lc] = pb[u][q];
      }
    }
  }
}

// ---- per model: sum of the item partials over its spans (FP64) -----------
__global__ __launch_bounds__(256) void k_adj_reduce(AdjArgs a) {
  const int b = blockIdx.x;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const uint8_t* slab = a.ws + (int64_t)b * a.L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  if (hd->n == 0) return;
  const MList* ml = reinterpret_cast<const MList*>(slab + a.L.off_mlist);
  const int K = ml->nU + ml->nV;
  if (K > kKGM) return;   // flagged by the item kernel
  const GradAcc& G = a.G;
  const GradAcc& Gp = a.Gp;
  const int S = a.span_group;
  const int g0 = hd->span_lo / S, g1 = (hd->span_hi - 1) / S;   // span groups that meet the window
  const int nch = (K + kKG - 1) / kKG;
  const float* src = a.part + (int64_t)b * a.n_items * Gp.n;
  double* acc = a.acc + (int64_t)b * G.n;
  const int NR = 32 * hd->nrb;
  // the slot-independent sums over every item of the model (chunks past the
  // first add their chunk's mixing-ratio adjoints and zeros elsewhere) ...
  for (int e = threadIdx.x; e < Gp.o_P; e += 256) {
    double t = 0.0;
    for (int g = g0; g <= g1; ++g)
      for (int c = 0; c < nch; ++c) t += src[(int64_t)(g * kGChunks + c) * Gp.n + e];
    acc[e] += t;
  }
  // ... and the P adjoints of chunk c's slots from chunk c's items
  for (int e = threadIdx.x; e < NR * K; e += 256) {
    const int j = e / K, q = e - j * K, c = q / kKG, qc = q - c * kKG;
    double t = 0.0;
    for (int g = g0; g <= g1; ++g) t += src[(int64_t)(g * kGChunks + c) * Gp.n + Gp.o_P + j * Gp.kp + qc];
    acc[G.o_P + j * G.kp + q] += t;
  }
}

// ---- per model: the path x weight products in reverse (FP64) -------------
// Wbar[l][q] = sum_{j <= l} dl[j][l] Pbar[j][q] for the slots q of layer l
// gives Tbar_l through dW/dT; dlbar[j][l] = sum_q Pbar[j][q] W[l][q] +
// PRbar_j w_R,l gives the chord adjoints: with dl[j][l] = 2 (Q_{j,l+1} -
// Q_{j,l}) (Q_{j,j} = 0), dQ/dh_m = (Rp + h_m)/Q, dQ/dz_j = -(Rp + z_j)/Q,
// dQ/dRp = (h_m - z_j)/Q (a zero Q, the top ray at the top boundary, has no
// derivative).  A cloud deck (optical depth tc_j along ray j, folded into
// the ray's weight A'_j = A_j e^{-tc_j} and the constant sum_j A_j (1 -
// e^{-tc_j})) unfolds here: with S = sum_i Dbar_i, Abar_j = Abar'_j
// e^{-tc_j} + S (1 - e^{-tc_j}) and tcbar_j = A'_j (S - Abar'_j), and
// tc_j = sum_l dl[j][l] c_l with the layer weight c_l = sigma rho_l joins
// the chord and temperature sums like the Rayleigh weight.
constexpr int kPM = 256;
__global__ __launch_bounds__(kPM) void k_adj_pmat(AdjArgs a) {
  const int b = blockIdx.x;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const Layout& L = a.L;
  const GradAcc& G = a.G;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  const int N = hd->n;
  if (N == 0) return;
  const MList* ml = reinterpret_cast<const MList*>(slab + L.off_mlist);
  const int nU = ml->nU, nV = ml->nV;
  if (nU + nV > kKGM) return;
  const double* zs = reinterpret_cast<const double*>(slab + L.off_z);
  const double* lw64 = reinterpret_cast<const double*>(slab + L.off_lw64);
  const double* lwd = reinterpret_cast<const double*>(slab + L.off_lwd64);
  const int32_t* lid = reinterpret_cast<const int32_t*>(slab + L.off_lid);
  double* acc = a.acc + (int64_t)b * G.n;
  const double* Pb = acc + G.o_P;
  const double* PRb = acc + G.o_PR;
  const double Rp = hd->Rp;
  const int tid = threadIdx.x;

  __shared__ double sZ[TRX_MAX_LAYERS_MFMA];
  __shared__ double sH[TRX_MAX_LAYERS_MFMA + 1];
  __shared__ double sW[TRX_MAX_LAYERS_MFMA][8];   // 4 corners, 2 CIA nodes, Rayleigh, cloud
  __shared__ double sD[TRX_MAX_LAYERS_MFMA][8];   // their d/dT at fixed P
  __shared__ int sS[TRX_MAX_LAYERS_MFMA][6];      // their slots
  __shared__ double sHb[TRX_MAX_LAYERS_MFMA + 1];
  __shared__ double sRp[kPM / 64];
  __shared__ double sTcb[TRX_MAX_LAYERS_MFMA];    // tcbar_j (zero without a deck)
  const int nq = nV > 0 ? 6 : 4;
  for (int l = tid; l < N; l += kPM) {
    sZ[l] = zs[l];
    const int perm[8] = {0, 1, 2, 3, 5, 6, 4, 7};
    for (int q = 0; q < 8; ++q) {
      const double w = lw64[8 * l + perm[q]];
      sW[l][q] = (q == 4 || q == 5) ? w / kCiaScale32 : w;
      sD[l][q] = lwd[8 * l + perm[q]];
    }
    double tcb = 0.0;
    if (hd->cloud) {
      const double tc = reinterpret_cast<const double*>(slab + L.off_pc64)[l];
      const double Ap = reinterpret_cast<const double*>(slab + L.off_A64)[l];
      const double S = acc[G.o_S], Abp = acc[G.o_A + l];
      // an opaque ray (tc = inf) has A' = 0 and no tcbar
      tcb = isinf(tc) ? 0.0 : Ap * (S - Abp);
      acc[G.o_A + l] = Abp * exp(-tc) - S * expm1(-tc);
    }
    sTcb[l] = tcb;
    const uint32_t c01 = (uint32_t)lid[8 * l + 6], c23 = (uint32_t)lid[8 * l + 7];
    const uint32_t cw = (uint32_t)lid[8 * l + 3];
    sS[l][0] = c01 & 0xffff;
    sS[l][1] = c01 >> 16;
    sS[l][2] = c23 & 0xffff;
    sS[l][3] = c23 >> 16;
    sS[l][4] = nU + (cw & 0xff);
    sS[l][5] = nU + ((cw >> 8) & 0xff);
  }
  for (int m = tid; m <= N; m += kPM) sHb[m] = 0.0;
  __syncthreads();
  for (int m = tid; m <= N; m += kPM) sH[m] = m == 0 ? 0.0 : (m == N ? sZ[N - 1] : 0.5 * (sZ[m - 1] + sZ[m]));
  __syncthreads();
  auto qv = [&](double h, double z) { return sqrt(fmax((h - z) * (2.0 * Rp + h + z), 0.0)); };
  auto chord = [&](int j, int l) -> double {
    const double zj = sZ[j];
    const double h0 = sH[l], h1 = sH[l + 1];
    const double q1 = qv(h1, zj);
    if (l == j) return 2.0 * q1;
    return 2.0 * (h1 - h0) * (2.0 * Rp + h0 + h1) / (q1 + qv(h0, zj));
  };

  // dchi2/d dl[j][l]: the path x weight products, the Rayleigh path and the
  // deck's optical depth of ray j, each through layer l's weight
  auto dlbar = [&](int j, int l) -> double {
    const double* pr = Pb + (int64_t)j * G.kp;
    double d = PRb[j] * sW[l][6] + sTcb[j] * sW[l][7];
    for (int q = 0; q < nq; ++q) d += pr[sS[l][q]] * sW[l][q];
    return d;
  };

  // temperatures through the weights: thread per layer
  for (int l = tid; l < N; l += kPM) {
    double wb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j <= l; ++j) {
      const double d = chord(j, l);
      const double* pr = Pb + (int64_t)j * G.kp;
      for (int q = 0; q < nq; ++q) wb[q] += d * pr[sS[l][q]];
      wb[6] += d * PRb[j];
      wb[7] += d * sTcb[j];
    }
    double t = 0.0;
    for (int q = 0; q < nq; ++q) t += wb[q] * sD[l][q];
    t += wb[6] * sD[l][6];
    t += wb[7] * sD[l][7];
    acc[G.o_T + l] += t;
  }
  // chords: thread per ray
  double rpb = 0.0;
  for (int j = tid; j < N; j += kPM) {
    const double zj = sZ[j];
    double zb = 0.0;
    double q0 = 0.0;
    for (int l = j; l < N; ++l) {
      const double g = 2.0 * dlbar(j, l);
      const double h1 = sH[l + 1];
      const double q1 = qv(h1, zj);
      if (q1 > 0.0) {
        zb -= g * (Rp + zj) / q1;
        rpb += g * (h1 - zj) / q1;
      }
      if (l > j && q0 > 0.0) {
        const double h0 = sH[l];
        zb += g * (Rp + zj) / q0;
        rpb -= g * (h0 - zj) / q0;
      }
      q0 = q1;
    }
    acc[G.o_z + j] += zb;
  }
  // shell boundaries: thread per boundary m >= 1 (h_0 = 0 is fixed), over
  // the rays below it; boundary m is the outer edge of shell m - 1 and the
  // inner edge of shell m (for the rays below layer m)
  for (int m = tid + 1; m <= N; m += kPM) {
    const double hm = sH[m];
    double t = 0.0;
    for (int j = 0; j < m; ++j) {
      const double q = qv(hm, sZ[j]);
      if (q > 0.0) {
        double g = dlbar(j, m - 1);
        if (m < N) g -= dlbar(j, m);
        t += 2.0 * g / q;
      }
    }
    sHb[m] = t * (Rp + hm);
  }
  rpb = wave_sum_d(rpb);
  if ((tid & 63) == 0) sRp[tid >> 6] = rpb;
  __syncthreads();
  for (int m = tid; m <= N; m += kPM) acc[G.o_h + m] += sHb[m];
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < kPM / 64; ++w) t += sRp[w];
    acc[G.o_Rp] += t;
  }
}

// ---- per model: annulus weights, shell boundaries, altitude, chemistry ---
__global__ __launch_bounds__(64) void k_adj_geom(AdjArgs a) {
  const int b = blockIdx.x;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const Layout& L = a.L;
  const GradAcc& G = a.G;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  const int N = hd->n;
  const int nabs = a.tab.n_abs;
  const int64_t off = a.bt.layer_off[b];
  const int nl = a.bt.n_layers[b];
  const bool bad = N == 0 || (a.model_status[b] & (TRX_MODEL_NONFINITE | TRX_MODEL_GRAD_UNSUPPORTED)) ||
                   !isfinite(a.chi2[b]);
  if (bad) {
    const double nan = __builtin_nan("");
    for (int l = threadIdx.x; l < nl; l += 64) a.dT[off + l] = nan;
    for (int i = threadIdx.x; i < nabs; i += 64) a.dvmr[(int64_t)b * nabs + i] = nan;
    if (threadIdx.x == 0) a.dRp[b] = nan;
    return;
  }
  if (threadIdx.x != 0) return;   // one sequential FP64 sweep per model (N <= 224)
  double* acc = a.acc + (int64_t)b * G.n;
  double* Ab = acc + G.o_A;
  double* zb = acc + G.o_z;
  double* hb = acc + G.o_h;
  double* Tb = acc + G.o_T;
  const double* z = reinterpret_cast<const double*>(slab + L.off_z);
  const double Rp = hd->Rp, inv_Rs2 = hd->inv_Rs2, mu = hd->mu_kg;
  const double GM = a.bt.GM[b], kB = a.bt.kB;
  const double* T = a.bt.T + off;
  double Rpb = acc[G.o_Rp];
  auto hof = [&](int k) -> double { return k == 0 ? 0.0 : (k == N ? z[N - 1] : 0.5 * (z[k - 1] + z[k])); };
  // annulus weights A_j = 2 (Rp + z_j)(h_{j+1} - h_j)/Rs^2
  for (int j = 0; j < N; ++j) {
    const double dh = hof(j + 1) - hof(j);
    const double f = 2.0 * Ab[j] * inv_Rs2;
    zb[j] += f * dh;
    Rpb += f * dh;
    hb[j + 1] += f * (Rp + z[j]);
    hb[j] -= f * (Rp + z[j]);
  }
  // shell boundaries: h_k = (z_{k-1} + z_k)/2, h_N = z_{N-1} (h_0 = 0 fixed)
  for (int k = 1; k < N; ++k) {
    zb[k - 1] += 0.5 * hb[k];
    zb[k] += 0.5 * hb[k];
  }
  zb[N - 1] += hb[N];
  // altitude recursion z_l = z_{l-1} - sC_{l-1} f, sC = k_B T ln(P_l/P_{l-1})/mu,
  // f = (Rp + z_{l-1})^2/GM (or Rp^2/GM), in reverse
  const double xb = log10(a.bt.p_bot[b]), xt = log10(a.bt.p_top[b]);
  auto Pof = [&](int l) -> double {
    const double p0 = pow(10.0, xb + (xt - xb) * (double)l / (double)N);
    const double p1 = pow(10.0, xb + (xt - xb) * (double)(l + 1) / (double)N);
    return p0 * sqrt(p1 / p0);
  };
  double mub = 0.0;
  double Pl = Pof(N - 1);
  for (int l = N - 1; l >= 1; --l) {
    const double Pm = Pof(l - 1);
    const double sC = kB * T[l - 1] * log(Pl / Pm) / mu;
    const double g = zb[l];
    if (a.bt.gravity == 0) {
      const double rz = Rp + z[l - 1];
      const double f = rz * rz / GM;
      zb[l - 1] += g * (1.0 - 2.0 * sC * rz / GM);
      Rpb += g * (-2.0 * sC * rz / GM);
      Tb[l - 1] += g * (-sC * f / T[l - 1]);
      mub += g * (sC * f / mu);
    } else {
      const double f = Rp * Rp / GM;
      zb[l - 1] += g;
      Rpb += g * (-2.0 * sC * Rp / GM);
      Tb[l - 1] += g * (-sC * f / T[l - 1]);
      mub += g * (sC * f / mu);
    }
    Pl = Pm;
  }
  // chemistry: CIA weights chi_a chi_b, mu = amu sum chi_s m_s, fill gases
  // chi_H2 = (1 - S)/(1 + r), chi_He = r chi_H2, log10 parameters
  double cb[kMaxSpecies];
  for (int q = 0; q < nabs + 2; ++q) cb[q] = acc[G.o_chi + q] + mub * a.bt.amu * a.tab.mass[q];
  for (int p = 0; p < a.tab.n_cia; ++p) {
    const int sa = a.tab.cia_pair[p][0], sb = a.tab.cia_pair[p][1];
    const double w = acc[G.o_cw + p];
    cb[sa] += w * hd->chi_s[sb];
    cb[sb] += w * hd->chi_s[sa];
  }
  const double r = a.bt.he_h2;
  const double fb = (cb[nabs] + r * cb[nabs + 1]) / (1.0 + r);
  for (int i = 0; i < nabs; ++i)
    a.dvmr[(int64_t)b * nabs + i] = (cb[i] - fb) * hd->chi_s[i] * 2.302585092994045684;
  for (int l = 0; l < N; ++l) a.dT[off + l] = Tb[l];
  a.dRp[b] = Rpb;
}

}  // namespace

// the 8-wave variant takes layouts of at most 128 rays (its two Pbar tiles
// per wave cover 4 x 4 ray x slot blocks), the 12-wave one the others
static bool adj_small(const Layout& L) { return L.NRB * (kKG / 32) <= 2 * kWaves; }
size_t adj_item_lds_bytes(const Layout& L) {
  return carve(L, make_grad_acc(L.NP, kKG), adj_small(L) ? kWaves : kWavesL, nullptr, nullptr);
}

void launch_chi2_dbar(const AdjArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return;
  hipLaunchKernelGGL(k_chi2_dbar, dim3(B_grid), dim3(256), 0, s, a);
}

hipError_t launch_adj_item(const AdjArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return hipSuccess;
  const size_t lds = adj_item_lds_bytes(a.L);
  const bool small = adj_small(a.L);
  for (const void* fn : {small ? (const void*)k_adj_item<2, kWaves, false> : (const void*)k_adj_item<3, kWavesL, false>,
                         small ? (const void*)k_adj_item<2, kWaves, true> : (const void*)k_adj_item<3, kWavesL, true>}) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // the models of one chunk, one item per span group; then those of more
  // (their items exit at once in the first launch, the others' in the second)
  const int ng = a.n_items / kGChunks;
  if (small) {
    hipLaunchKernelGGL((k_adj_item<2, kWaves, false>), dim3(B_grid, ng), dim3(64 * kWaves), lds, s, a);
    hipLaunchKernelGGL((k_adj_item<2, kWaves, true>), dim3(B_grid, a.n_items), dim3(64 * kWaves), lds, s, a);
  } else {
    hipLaunchKernelGGL((k_adj_item<3, kWavesL, false>), dim3(B_grid, ng), dim3(64 * kWavesL), lds, s, a);
    hipLaunchKernelGGL((k_adj_item<3, kWavesL, true>), dim3(B_grid, a.n_items), dim3(64 * kWavesL), lds, s, a);
  }
  return hipGetLastError();
}

void launch_adj_reduce(const AdjArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return;
  hipLaunchKernelGGL(k_adj_reduce, dim3(B_grid), dim3(256), 0, s, a);
}

void launch_adj_pmat(const AdjArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return;
  hipLaunchKernelGGL(k_adj_pmat, dim3(B_grid), dim3(kPM), 0, s, a);
}

void launch_adj_geom(const AdjArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return;
  hipLaunchKernelGGL(k_adj_geom, dim3(B_grid), dim3(64), 0, s, a);
}

}  // namespace trx
