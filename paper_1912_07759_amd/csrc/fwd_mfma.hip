// Matrix-core forward kernel for the FP32 and split-bf16 modes: opacity
// (a4), optical depth (a5) and depth (a6) of one (model, 64-column span) per
// workgroup of four waves.
//
// Contraction over opacity slots.  The optical depth of ray j at column c is
//   tau_j = sum_l dl[j][l] kappa_l,  kappa_l = sum_q W[l][q] M_q + w_R,l R
// (equations opt_dpth, cia_opt_dpth, contrib; Opacities section), where the
// slots q of a model are its distinct cross-section corners, with the mixed
// cross-sections M_q = sum_i chi_i sigma_i[q] (the tables share one
// (T, log10 P) grid, so the bilinear weights are common to all absorbers),
// and its distinct CIA temperature nodes, with the CIA sums
// M_t = sum_pairs chi_a chi_b sigma_pair[t]; R is the mixed Rayleigh
// cross-section.  The layer sums P[j][q] = sum_l dl[j][l] W[l][q] and
// PR_j = sum_l dl[j][l] w_R,l are taken once per model by the geometry (in
// FP64), so per column
//   tau_j = sum_q P[j][q] M_q + PR_j R,
// a contraction over the model's slots (some 50-100) instead of its layers.
//
// Per work item the workgroup stages M of its 64 columns, split into the
// B-operand pieces of the matrix instruction, in LDS (wave w takes the
// 8-slot groups w, w+4, ...; a lane loads 8 slots x 5 tables per batch, the
// next batch issued before the current one is mixed), and wave w contracts
// the ray blocks w (and 7 - w) over all slot blocks, the A fragments (P)
// streamed from the model's workspace one batch of slot blocks ahead.
// Models with more slots than one staging chunk (kKC) take several chunks.
// Builds: three workgroups per CU (168 registers) or four (128 registers,
// smaller load batches; two ray blocks per wave in two passes), with or
// without the code of two-layer layouts.
//   FP32 mode: v_mfma_f32_32x32x2_f32, M in FP32, P as two FP32 pieces.
//   bf16 modes: v_mfma_f32_32x32x16_bf16 with both operands split into bf16
//     pieces x = x0 + x1 (+ x2); the products with piece-index sum < 2 (two
//     pieces: x0 y0 + x0 y1 + x1 y0) or < 3 (three pieces, six products) are
//     accumulated in FP32.
//
// Exponential temperature scheme (Opacities section: sigma = a e^{-b/T}
// through the two bracketing temperature nodes).  It is not linear in the
// table values, so corners cannot be mixed once per model: each layer is
// its own slot (P[j][l] = dl[j][l] 1e-4 rho_l; the top layer first, so that
// the FP32 accumulator of a ray takes its smallest terms first, as with
// the corner slots, which follow rising pressure) and its row is staged per
// column as sum_i chi_i [(1 - w_P) g_i(iP) + w_P g_i(iP + 1)] with
// g = sigma1 2^{u log2(sigma2/sigma1)}, u = w_T T2/T, from a table of
// (sigma1, log2 ratio) pairs (one 8-byte load and one exp2 per absorber and
// pressure node); CIA slots stay linear.
//
// Depth.  Each accumulator element is a (ray, column) optical depth; a wave
// adds the Rayleigh term, then (A_j/Rs^2)(1 - exp(-tau)) over the 32 rays of
// a block per column (two lanes per column, one cross-lane exchange) into a
// per-ray-block partial in LDS, and the partials are summed in ray-block
// order (same bits every run).  The fast epilogue takes the sum as the ray
// block's sum of A_j less sum_j A_j e^{-tau_j}; its FP32 rounding is about
// 1e-7 of the block's sum of A_j whatever tau, which is far inside the
// depth's tolerance but, being the same for every column, shows in chi^2
// gradients near the optimum (so does the FP32 sum over rays that are
// opaque at every column: its rounding is one constant per model).  The
// accurate epilogue (the forward pass of the gradient) forms each
// 1 - e^{-tau_j} to a relative error of a few FP32 units (a range-reduced
// expm1) and sums A_j/Rs^2 (1 - e^{-tau_j}) in FP64 with A_j in FP64, so
// that no rounding is shared by every column.
//
// Emission (Forward Models section, the emission intensity and its
// Gauss-Legendre flux).  The path matrix of an emission layout holds the
// vertical shell thicknesses, so that the accumulator of row l is the
// optical depth tau_l from the top down to the bottom of shell l (plus the
// deck's, from the records).  The layer sum of the formal solution,
// I(mu) = B_s e^{-tau_0/mu} + sum_l B_l (e^{-tau_{l+1}/mu} - e^{-tau_l/mu})
// with B_s = B_0, telescopes to I = B_{N-1} + sum_{l >= 1} (B_{l-1} - B_l)
// e^{-tau_l/mu}, so the flux ratio is a sum over rows of one term each:
//   F/F_s = (Rp/Rs)^2 [B_{N-1} + sum_{l>=1} (B_{l-1} - B_l) G(tau_l)] / B_*,
//   G(tau) = sum_i 2 w_i mu_i e^{-tau/mu_i}.
// Relative to the star, B_l/B_* = e^{x_* - x_l} w_* / w_l with x = h c nu /
// k_B T and w = 1 - e^{-x} (accurate expm1), and the difference of two
// neighbouring layers is formed without cancellation,
// B_{l-1}/B_* - B_l/B_* = e^{x_* - x_l} (e^{x_l - x_{l-1}} - 1) w_* /
// (w_{l-1} w_l), where x_l - x_{l-1} comes from (T_{l-1} - T_l)/(T_l T_{l-1})
// (the direct difference when |x_l - x_{l-1}| > 1).  Rows are summed in
// FP64.
#include "trx_internal.h"

#include <type_traits>

namespace trx {

namespace {


constexpr int kWaves = 4;
constexpr int kCols = 64;               // columns per workgroup
constexpr int kKC = 128;                // slots per staging chunk
constexpr int kChunk = 8;               // items popped per atomic (persistent launch)
static_assert(TRX_MAX_LAYERS_MFMA % 32 == 0 && TRX_MAX_LAYERS_MFMA <= 64 * kWaves,
              "a thread copies the record of one ray");
static_assert(kKC <= 64 * kWaves, "a thread copies one slot id");

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int MODE, int RBW>
struct Cfg {
  // bf16 pieces of each operand (FP32 mode: 1 M piece, 2 P pieces)
  static constexpr int npc = MODE == TRX_BF16_SPLIT3 ? 3 : (MODE == TRX_BF16_SPLIT2 ? 2 : 1);
  // 16-byte words per lane of one (ray block, slot block) A fragment
  static constexpr int kAW = MODE == TRX_FP32 ? 4 : npc;
  // slot blocks per A batch (register budget: 4 words per batch)
  static constexpr int KB = 4 / (RBW * kAW) > 0 ? 4 / (RBW * kAW) : 1;
  // double-buffered A batches when they fit the budget; otherwise the next
  // batch is loaded once the current batch's products are issued
  static constexpr bool PF = RBW * kAW <= 4;
  // dwords of the B-operand buffer of one chunk: bf16 [kq][piece][col block]
  // [lane][4], FP32 [kq][col block][lane][8 steps]
  static constexpr int bdw = MODE == TRX_FP32 ? kKC * 64 : kKC * npc * 32;
};

// Depth epilogues: fast transit, accurate transit, emission.
enum { kEpiFast = 0, kEpiAcc = 1, kEpiEm = 2 };

template <int MODE, int RBW, int EPI, bool XT>
struct Smem {
  // B operand of the staged slot chunk
  __attribute__((aligned(16))) uint32_t bfrag[Cfg<MODE, RBW>::bdw];
  float part[kWaves * RBW][kCols];  // per-ray-block depth partials
  float2 aw[TRX_MAX_LAYERS_MFMA];   // per ray: A_j/Rs^2, -PR_j / ln 2
  // accurate and emission epilogues: per ray A_j/Rs^2 in FP64 (accurate),
  // per-ray-block FP64 partials; emission: the layer records
  double a64[EPI == kEpiAcc ? TRX_MAX_LAYERS_MFMA : 1];
  double partd[EPI != kEpiFast ? kWaves * RBW : 1][EPI != kEpiFast ? kCols : 1];
  float4 em[EPI == kEpiEm ? TRX_MAX_LAYERS_MFMA : 1];
  double emz[EPI == kEpiEm ? TRX_MAX_LAYERS_MFMA : 1];   // c2 (1/T_l - 1/T_*) in FP64
  float rpart[kWaves][kCols];       // Rayleigh sums by wave
  int32_t sid[kKC];                 // table rows of the chunk's slots (| run << 24)
  float4 xr[XT ? kKC : 1];          // exponential scheme: records of the chunk's layer slots
  float chis[kMaxRegimes][kMaxSpecies];   // mixing ratios per run: absorbers, H2, He
  float ciaw[kMaxRegimes][TRX_MAX_CIA];   // CIA pair weights per run
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

constexpr float kNegLog2e32 = -1.4426950408889634f;   // -1 / ln 2

// 1 - 2^x for x = -tau / ln 2 to a relative error of a few FP32 units, with
// rounding errors that do not share a sign: 2^x = 2^-k e^y with k the
// integer nearest -x and y = (x + k) ln 2, |y| <= ln 2 / 2 (x + k is exact);
// e^y - 1 by its Taylor series to y^9 (truncation below 1e-11 relative);
// then 1 - 2^x = -(2^-k (e^y - 1) + (2^-k - 1)), one rounding, and for
// k = 0 the series itself (no cancellation for small tau).  tau is capped
// at 100, where 1 - e^{-tau} rounds to 1.
__device__ inline float one_minus_exp2(float x) {
  const float xc = fmaxf(x, -144.26950408889634f);
  const float kf = __builtin_rintf(-xc);
  const float y = (xc + kf) * 0.69314718055994531f;
  float p = 1.f / 362880.f;
  p = fmaf(y, p, 1.f / 40320.f);
  p = fmaf(y, p, 1.f / 5040.f);
  p = fmaf(y, p, 1.f / 720.f);
  p = fmaf(y, p, 1.f / 120.f);
  p = fmaf(y, p, 1.f / 24.f);
  p = fmaf(y, p, 1.f / 6.f);
  p = fmaf(y, p, 0.5f);
  p = fmaf(y, p, 1.f);
  const float em1 = y * p;                                      // e^y - 1
  const float sc = __builtin_amdgcn_ldexpf(1.f, -(int)kf);      // 2^-k
  return -fmaf(sc, em1, sc - 1.f);
}

// e^{-y} for an argument y >= 0 known in FP64, to a few FP32 units and in
// the FP64 range (a planet's flux relative to its star's reaches e^-100
// and below at short wavelengths, and an FP32 argument of ~100 would lose
// 1e-6 of the result): 2^{-y log2 e} split into an integer power of two and
// 2^f, |f| <= 1/2, in FP64; +inf gives 0.
__device__ inline double exp_neg_dd(double y) {
  const double t = -1.4426950408889634074 * fmin(y, 2000.0);
  const double n = __builtin_rint(t);
  return __builtin_amdgcn_ldexp((double)__builtin_amdgcn_exp2f((float)(t - n)), (int)n);
}

// One row's term of the emission flux ratio (before (Rp/Rs)^2):
// (B_{l-1} - B_l)/B_* G(tau_l), from the records e (layer l) with its
// x_l - x_* term zl and that of layer l - 1, zm, in FP64, w = 1 - e^{-x} of
// both layers (wl, wm), the accumulator x = -tau_gas/ln 2, the wavenumber
// nu and the star's 1 - e^{-x_*}.  The Planck difference is
// e^{-(x_b - x_*)} q with x_b the hotter of the two layers when they
// differ by more than 1 in x (then the direct difference), else the
// cancellation-free form; each angle's exponential is taken together with
// e^{-(x_b - x_*)} in FP64 range.  The quotients take the hardware
// reciprocal (1 ulp; w lies in (0, 1], away from zero at these
// wavenumbers and temperatures).
__device__ inline double emission_term(float4 e, double zl, double zm, float x, float nu, double nud, float wst,
                                       float wl, float wm, const FwdArgs& a) {
  constexpr float kL2e = 1.4426950408889634f;
  const float dx = nu * e.y;                                     // x_l - x_{l-1}
  double yb;
  float q;
  if (fabsf(dx) <= 1.f) {
    yb = nud * zl;
    q = -one_minus_exp2(kL2e * dx) * wst * __builtin_amdgcn_rcpf(wm * wl);   // (e^{dx} - 1) w_* / (w_{l-1} w_l)
  } else if (dx > 1.f) {
    yb = nud * zm;
    q = wst * (__builtin_amdgcn_rcpf(wm) - __builtin_amdgcn_exp2f(-kL2e * dx) * __builtin_amdgcn_rcpf(wl));
  } else {
    yb = nud * zl;
    q = wst * (__builtin_amdgcn_exp2f(kL2e * dx) * __builtin_amdgcn_rcpf(wm) - __builtin_amdgcn_rcpf(wl));
  }
  // tau/mu_i with the deck's part (x = -tau_gas / ln 2)
  const float tau = e.w - 0.69314718055994531f * x;
  double G = 0.0;
#pragma unroll 4
  for (int i = 0; i < a.n_mu; ++i) G = fma((double)a.em_c32[i], exp_neg_dd(yb + (double)(tau * a.em_k32[i])), G);
  return (double)q * G;
}

// Ray block r (0..RBW-1) of a wave: w, then 7 - w.
template <int RBW>
__device__ __forceinline__ int own_rb(int wave, int r) {
  return r == 0 ? wave : 2 * kWaves - 1 - wave;
}
static_assert(TRX_MAX_LAYERS_MFMA <= 32 * 2 * kWaves, "two ray blocks per wave cover every ray");

// s[i] += sum_t wt[t] tab_t[row_i][col] over the tables t < nt (table t at
// tab + t stride) for the slots i in [i0, i1) of a group of 8; rows of the
// slots outside are clamped into it (their loads are in range, their values
// unused).  Loads: 8 slots x SA tables per batch, buffer loads with the
// column as the per-lane offset and the slot's row as the uniform offset.
template <int SA>
__device__ inline void mix_group(const float* tab, int64_t stride, int nt, const float* wt, const int32_t* rows,
                                 int i0, int i1, int W, int voff, float* s) {
  const int rec = (int)(stride * 4 < 0x7fffffff ? stride * 4 : 0x7fffffff);
  int soff[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = i < i0 ? i0 : (i >= i1 ? i1 - 1 : i);
    soff[i] = (__builtin_amdgcn_readfirstlane(rows[k]) & 0xffffff) * W * 4;
  }
  for (int t0 = 0; t0 < nt; t0 += SA) {
    float v[SA][8];
#pragma unroll
    for (int tt = 0; tt < SA; ++tt) {
      if (t0 + tt < nt) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(tab + (int64_t)(t0 + tt) * stride), (short)0, rec, kRsrcWord3);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[tt][i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff[i], 0));
      }
    }
#pragma unroll
    for (int tt = 0; tt < SA; ++tt) {
      if (t0 + tt < nt) {
        const float c = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(wt[t0 + tt])));
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (i >= i0 && i < i1) s[i] = fmaf(c, v[tt][i], s[i]);
      }
    }
  }
}

// Rayleigh slots of two-layer layouts: s[i] += sum_k chis[run of slot i][k]
// ray_k[col] over the ns species for the slots i in [i0, i1) of a group
// (the run in bits 24.. of the slot entry); each species' row is loaded once
// for all the group's slots.
__device__ inline void mix_rayleigh(const float* ray, int ns, int W, const float (*chis)[kMaxSpecies],
                                    const int32_t* rows, int i0, int i1, int voff, float* s) {
  const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc((void*)ray, (short)0, ns * W * 4, kRsrcWord3);
  int run[8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
    run[i] = min((int)((uint32_t)__builtin_amdgcn_readfirstlane(rows[i < i1 ? i : i1 - 1]) >> 24), kMaxRegimes - 1);
  for (int k = 0; k < ns; ++k) {
    const float v = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rr, voff, k * W * 4, 0));
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i >= i0 && i < i1)
        s[i] = fmaf(__uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(chis[run[i]][k]))), v, s[i]);
  }
}

// Exponential temperature scheme: s[i] += sum_t wt[t] sigma_t(layer of slot
// i) for the slots i < i1 of a group of 8 (the others clamped into range,
// their values unused), with
//   sigma = (1 - w_P) g(iP) + w_P g(iP + 1),  g = sigma1 2^{u log2(sigma2/sigma1)}
// at the two pressure nodes (Opacities section), from the pair table
// (sigma1, log2 ratio) of the slot's row; a NaN ratio (a value that is not
// positive) takes the linear form sigma1 + w_T (sigma2 - sigma1) from the
// FP32 table.  rec[i] = {u, w_P, w_T, 0}.  Loads: 8-byte buffer loads of
// the two pressure nodes of each slot for SA tables per batch; consecutive
// slots (layers) often share their row, or step one pressure node down, and
// then reuse the previous slot's pairs (uniform branches on the row offsets).
template <int SA>
__device__ inline void mix_group_xt(const float2* pairs, const float* tab, int64_t stride, int nt, const float* wt,
                                    const int32_t* rows, const float4* rec, int i1, int W, int nP, int col,
                                    float* s) {
  const int rec8 = (int)(stride * 8 < 0x7fffffff ? stride * 8 : 0x7fffffff);
  const int rec4 = (int)(stride * 4 < 0x7fffffff ? stride * 4 : 0x7fffffff);
  const int rowP = W * 8;   // next pressure node
  int soff[8];
  float u[8], wp[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = i >= i1 ? i1 - 1 : i;
    soff[i] = (__builtin_amdgcn_readfirstlane(rows[k]) & 0xffffff) * W * 8;
    u[i] = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(rec[k].x)));
    wp[i] = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(rec[k].y)));
  }
  for (int t0 = 0; t0 < nt; t0 += SA) {
    u32x2 v[SA][8][2];
#pragma unroll
    for (int tt = 0; tt < SA; ++tt) {
      if (t0 + tt < nt) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(pairs + (int64_t)(t0 + tt) * stride), (short)0, rec8, kRsrcWord3);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int dr = i > 0 ? soff[i] - soff[i - 1] : -1;
          if (dr == 0) {
            v[tt][i][0] = v[tt][i - 1][0];
            v[tt][i][1] = v[tt][i - 1][1];
          } else if (dr == rowP) {
            v[tt][i][0] = v[tt][i - 1][1];
            v[tt][i][1] = __builtin_amdgcn_raw_buffer_load_b64(r, 8 * col, soff[i] + rowP, 0);
          } else {
            v[tt][i][0] = __builtin_amdgcn_raw_buffer_load_b64(r, 8 * col, soff[i], 0);
            v[tt][i][1] = __builtin_amdgcn_raw_buffer_load_b64(r, 8 * col, soff[i] + rowP, 0);
          }
        }
      }
    }
#pragma unroll
    for (int tt = 0; tt < SA; ++tt) {
      if (t0 + tt < nt) {
        const float c = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(wt[t0 + tt])));
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if (i < i1) {
            float g[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              const float s1 = __uint_as_float(v[tt][i][p].x);
              const float d = __uint_as_float(v[tt][i][p].y);
              if (d == d) {
                g[p] = s1 * __builtin_amdgcn_exp2f(u[i] * d);
              } else {
                const __amdgpu_buffer_rsrc_t r4 = __builtin_amdgcn_make_buffer_rsrc(
                    (void*)(tab + (int64_t)(t0 + tt) * stride), (short)0, rec4, kRsrcWord3);
                const int row4 = soff[i] / 2 + p * W * 4 + nP * W * 4;   // (iT + 1, iP + p)
                const float s2 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r4, 4 * col, row4, 0));
                const float wT = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(rec[i].z)));
                g[p] = fmaf(wT, s2 - s1, s1);
              }
            }
            s[i] = fmaf(c, fmaf(wp[i], g[1] - g[0], g[0]), s[i]);
          }
        }
      }
    }
  }
}

// Full corner groups (8 slots, all corners) in batches of SA absorber
// tables: issue_corners loads tables t0 .. t0 + SA - 1 of the 8 slot rows,
// mix_corners adds chi_t times them; a wave keeps two batches in flight.
template <int SA>
__device__ inline void issue_corners(const float* tab, int64_t stride, int nt, const int32_t* rows, int t0, int W,
                                     int voff, float (&v)[SA][8]) {
  const int rec = (int)(stride * 4 < 0x7fffffff ? stride * 4 : 0x7fffffff);
  int soff[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) soff[i] = (__builtin_amdgcn_readfirstlane(rows[i]) & 0xffffff) * W * 4;
#pragma unroll
  for (int tt = 0; tt < SA; ++tt) {
    if (t0 + tt < nt) {
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(tab + (int64_t)(t0 + tt) * stride), (short)0, rec, kRsrcWord3);
#pragma unroll
      for (int i = 0; i < 8; ++i) v[tt][i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff[i], 0));
    }
  }
}
template <int SA>
__device__ inline void mix_corners(const float* wt, int nt, int t0, const float (&v)[SA][8], float (&s)[8]) {
#pragma unroll
  for (int tt = 0; tt < SA; ++tt) {
    if (t0 + tt < nt) {
      const float c = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(wt[t0 + tt])));
#pragma unroll
      for (int i = 0; i < 8; ++i) s[i] = fmaf(c, v[tt][i], s[i]);
    }
  }
}

// One work item: model b, columns [64 s_first, 64 s_end) cut to its window.
// Called by all threads of the workgroup (every early return is uniform).
// TAU: also write the optical depth of every ray and column to a.tau (a
// separate instantiation: the stores cost the hot kernel registers).
// EPI: the depth epilogue (kEpiFast, kEpiAcc, kEpiEm).
// XT: the exponential temperature scheme (the absorber slots are layers).
// OCC: workgroups per CU the kernel is built for (4: smaller load batches
// in the staging, 128 registers; with two ray blocks per wave, the blocks
// are taken in two passes over the span with one set of accumulators, the
// staged slots serving both).
// RG: built for two-layer layouts (runs of one chemistry per model); the
// other builds leave their code out.
template <int MODE, int RBW, bool TAU, int EPI, bool XT, int OCC = 3, bool RG = false>
__device__ __forceinline__ void process(const FwdArgs& a, int b_in, int s_first, int s_end,
                                        Smem<MODE, RBW, EPI, XT>& sm) {
  constexpr bool PASS = OCC == 4 && RBW == 2;
  constexpr int RR = PASS ? 1 : RBW;   // ray blocks held in registers at a time
  using C = Cfg<MODE, RR>;
  constexpr int npc = C::npc, kAW = C::kAW, KB = C::KB;
  constexpr bool PF = C::PF;
  // the item is the same for the whole workgroup: keep it, and every address
  // derived from it, in scalar registers
  const int b = __builtin_amdgcn_readfirstlane(b_in);
  const Layout& L = a.L;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  const int N = hd->n;
  if (N == 0) return;
  const int lo = hd->lo, hi = hd->hi;
  const int sp0 = __builtin_amdgcn_readfirstlane(max(s_first, lo / kCols));
  const int sp1 = __builtin_amdgcn_readfirstlane(min(s_end, (hi + kCols - 1) / kCols));
  if (sp0 >= sp1) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  const DevTables& tb = a.tab;
  const int W = tb.n_wn;
  const MList* ml = reinterpret_cast<const MList*>(slab + L.off_mlist);
  const int nU = ml->nU, nV = tb.n_cia > 0 ? ml->nV : 0;
  // two-layer layouts: one Rayleigh slot per run after the node slots
  const bool rg = RG && L.rg;
  const int nR = rg ? ml->pad[0] : 0;
  const int K = nU + nV + nR;
  const int nrb = hd->nrb;
  const int NKQ = L.NKQ;
  // the ray blocks of this wave in registers (pass: which of the two in
  // the two-pass build)
  int pass = 0;
  auto orb = [&](int r) -> int { return PASS ? own_rb<2>(wave, pass) : own_rb<RBW>(wave, r); };
  // slot blocks with a nonzero product, per ray block of this wave
  uint64_t msk[RR];
  uint64_t any_msk = 0;
  auto set_masks = [&]() {
    any_msk = 0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      const int rb = orb(r);
      msk[r] = rb < nrb ? hd->kq_mask[rb] : 0ull;
      any_msk |= msk[r];
    }
  };
  set_masks();
  const int32_t* sid = reinterpret_cast<const int32_t*>(slab + L.off_sid);
  const float2* awg = reinterpret_cast<const float2*>(slab + L.off_aw);
  const u32x4* frag = reinterpret_cast<const u32x4*>(slab + L.off_dl);
  const int64_t abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  const int64_t cia_stride = (int64_t)tb.n_Tcia * W;

  // per-item records: ray weights (zero past N; the Rayleigh path weight
  // scaled like the fragments), slot rows, mixing ratios
  {
    const int nr = 32 * nrb;
    const float2 w = tid < nr ? awg[tid] : float2{};
    const int32_t r = K <= kKC && tid < K ? sid[tid] : 0;
    if (tid < nr) sm.aw[tid] = float2{w.x, kNegLog2e32 * w.y};
    if constexpr (EPI == kEpiAcc) {
      const double* A64 = reinterpret_cast<const double*>(slab + L.off_A64);
      if (tid < nr) sm.a64[tid] = A64[tid];
    }
    if constexpr (EPI == kEpiEm) {
      const float4* e32 = reinterpret_cast<const float4*>(slab + L.off_em32);
      const double4* e64 = reinterpret_cast<const double4*>(slab + L.off_em64);
      if (tid < nr) {
        sm.em[tid] = e32[tid];
        sm.emz[tid] = e64[tid].z;
      }
    }
    if (K <= kKC && tid < K) sm.sid[tid] = r;
    if constexpr (XT)
      if (K <= kKC && tid < nU) sm.xr[tid] = reinterpret_cast<const float4*>(slab + L.off_xt32)[tid];
    if (tid < kMaxSpecies) sm.chis[0][tid] = hd->chi_s32[tid];
    if (tid < TRX_MAX_CIA) sm.ciaw[0][tid] = hd->cia_w32[tid];
    if (rg && tid < kMaxSpecies) {
      // the other runs' mixing ratios (two-layer profiles)
      const RegChem* rc = reinterpret_cast<const RegChem*>(slab + L.off_rg);
      for (int r = 1; r < kMaxRegimes; ++r) {
        sm.chis[r][tid] = rc[r].chi_s32[tid];
        if (tid < TRX_MAX_CIA) sm.ciaw[r][tid] = rc[r].cia_w32[tid];
      }
    }
  }
  __syncthreads();

  // A fragments of slot blocks kq0 .. kq0 + KB - 1 (block-local < nq) of this
  // wave's ray blocks
  auto load_A = [&](u32x4 (&A)[RR][KB][kAW], int kq0, int kqa, int nq) {
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      const int rb = orb(r);
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        if (kq0 + kk < nq && ((msk[r] >> (kqa + kq0 + kk)) & 1)) {
          const int64_t f = (int64_t)rb * NKQ + kqa + kq0 + kk;
          if constexpr (MODE == TRX_FP32) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              A[r][kk][2 * p] = frag[((f * 2 + p) * 64 + lane) * 2];
              A[r][kk][2 * p + 1] = frag[((f * 2 + p) * 64 + lane) * 2 + 1];
            }
          } else {
#pragma unroll
            for (int p = 0; p < npc; ++p) A[r][kk][p] = frag[(f * npc + p) * 64 + lane];
          }
        }
      }
    }
  };

  // sum of A_j over each of the wave's ray blocks, in the order in which the
  // depth epilogue sums A_j e^{-tau_j}: where every e^{-tau_j} is 1 the two
  // agree to the bit and the block adds exactly zero
  const int hl = lane >> 5, lc = lane & 31;
  float awsum[RR];
  auto set_awsum = [&]() {
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int rb = orb(r);
    float t = 0.f;
    if (rb < nrb) {
#pragma unroll
      for (int q = 0; q < 16; ++q) t = fmaf(sm.aw[32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3)].x, 1.f, t);
    }
    awsum[r] = t + __shfl_xor(t, 32, 64);
  }
  };
  set_awsum();

  // Rayleigh by ray weights (two-layer layouts: by slots)
  const int ns = tb.has_rayleigh && !rg ? tb.n_abs + 2 : 0;
  for (int span = sp0; span < sp1; ++span) {
    const int col = span * kCols + lane;
    const bool valid = col >= lo && col < hi;
    const int cc = valid ? col : lo;
    const int voff = cc * 4;

    // Rayleigh: wave w takes the species w, w + 4, ...; the loads of the
    // first four are issued ahead of the staging
    float rv[4];
    {
      const __amdgpu_buffer_rsrc_t rr =
          __builtin_amdgcn_make_buffer_rsrc((void*)tb.ray32, (short)0, (ns > 0 ? ns : 1) * W * 4, kRsrcWord3);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = wave + kWaves * u;
        rv[u] = k < ns ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rr, voff, k * W * 4, 0)) : 0.f;
      }
    }

    // the run whose mixing ratios a staged group of 8 slots takes (its
    // first slot's; two-layer layouts pad each run's slots of one kind to
    // whole groups)
    auto run_of_group = [&](int g) -> int {
      return rg ? min((int)((uint32_t)__builtin_amdgcn_readfirstlane(sm.sid[8 * g]) >> 24), kMaxRegimes - 1) : 0;
    };

    // one staging chunk (slots c0 ..): stage, then contract; the first
    // chunk zeroes the accumulators after its staging (they are not live
    // during it)
    f32x16 acc[RR][2];
    // stage: stage the chunk (false: the second pass over a chunk that is
    // still staged)
    auto run_chunk = [&](const int c0, auto first_t, const bool stage) {
      constexpr bool first = decltype(first_t)::value;
      // tables per load batch (two batches in flight): 5 when the
      // accumulators are not live (6 spills registers), else 2; built for
      // four workgroups per CU, 2 and 1
      constexpr int SA = OCC == 4 ? (first ? 2 : 1) : (first ? 5 : 2);
      const int nq = (min(kKC, K - c0) + 15) >> 4;
      const int kqa = c0 >> 4;
      if (stage && K > kKC) {
        __syncthreads();   // the previous chunk's products are done with bfrag
        if (tid < kKC && c0 + tid < K) sm.sid[tid] = sid[c0 + tid];
        if constexpr (XT)
          if (tid < kKC && c0 + tid < nU) sm.xr[tid] = reinterpret_cast<const float4*>(slab + L.off_xt32)[c0 + tid];
        __syncthreads();
      }
      u32x4 A[RR][KB][kAW];
      load_A(A, 0, kqa, nq);   // in flight during the staging
      if (stage) {

      // staging: 8-slot groups g = wave, wave + 4, ... of the chunk's nq
      // blocks; corner slots are mixed over the absorbers, node slots over
      // the CIA pairs, slots past K are zero.  The full corner groups come
      // first, their loads in batches of SA tables with the next batch
      // issued before the current one is mixed (two register buffers); the
      // remaining groups (corners and nodes, padding) follow one by one.
      const int ng = 2 * nq;
      auto write_group = [&](int g, float (&s)[8]) {
        const int kq = g >> 1, h = g & 1;
        const int tcb = lane >> 5, n = lane & 31;
        if constexpr (MODE == TRX_FP32) {
          // [kq][col block][lane' = 32 (k%2) + n][step k/2], k = 8 h + i
          float* dst = reinterpret_cast<float*>(sm.bfrag) + ((kq * 2 + tcb) * 64 + n) * 8 + 4 * h;
          *reinterpret_cast<float4*>(dst) = make_float4(s[0], s[2], s[4], s[6]);
          *reinterpret_cast<float4*>(dst + 32 * 8) = make_float4(s[1], s[3], s[5], s[7]);
        } else {
          // [kq][piece][col block][lane' = 32 h + n][8 bf16], k = 8 h + i
#pragma unroll
          for (int p = 0; p < npc; ++p) {
            u32x4 q;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              q[i] = bf16_pair(s[2 * i], s[2 * i + 1]);
              s[2 * i] -= bf16_lo_f(q[i]);
              s[2 * i + 1] -= bf16_hi_f(q[i]);
            }
            *reinterpret_cast<u32x4*>(sm.bfrag + (((kq * npc + p) * 2 + tcb) * 64 + 32 * h + n) * 4) = q;
          }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] = 0.f;
      };
      // full corner groups: g < gf (none in the exponential scheme)
      const int gf = XT ? 0 : min(ng, max(nU - c0, 0) / 8);
      const int na = tb.n_abs;
      const int nta = na > 0 ? na : 1;
      {
        float va[SA][8], vb2[SA][8], s[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] = 0.f;
        int g = wave, t0 = 0;
        if (g < gf) issue_corners<SA>(tb.xsec32, abs_stride, na, sm.sid + 8 * g, t0, W, voff, va);
        auto step = [&](float (&cur)[SA][8], float (&nxt)[SA][8]) {
          int gn = g, tn = t0 + SA;
          if (tn >= nta) {
            gn = g + kWaves;
            tn = 0;
          }
          if (gn < gf) issue_corners<SA>(tb.xsec32, abs_stride, na, sm.sid + 8 * gn, tn, W, voff, nxt);
          mix_corners<SA>(sm.chis[run_of_group(g)], na, t0, cur, s);
          if (tn == 0) write_group(g, s);
          g = gn;
          t0 = tn;
        };
        while (g < gf) {
          step(va, vb2);
          if (g >= gf) break;
          step(vb2, va);
        }
      }
      // the other groups
      for (int g = gf + ((wave - gf) % kWaves + kWaves) % kWaves; g < ng; g += kWaves) {
        const int s0 = c0 + 8 * g;
        const int run = run_of_group(g);
        float s[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] = 0.f;
        const int nc = min(max(nU - s0, 0), 8);
        if (nc > 0) {
          if constexpr (XT)
            mix_group_xt<first ? 2 : 1>(tb.xexp32, tb.xsec32, abs_stride, tb.n_abs, sm.chis[run], sm.sid + 8 * g,
                                         sm.xr + 8 * g, nc, W, tb.n_P, cc, s);
          else
            mix_group<SA>(tb.xsec32, abs_stride, tb.n_abs, sm.chis[run], sm.sid + 8 * g, 0, nc, W, voff, s);
        }
        const int vb = min(max(nU + nV - s0, 0), 8);
        if (vb > nc)
          mix_group<SA>(tb.cia32, cia_stride, tb.n_cia, sm.ciaw[run], sm.sid + 8 * g, nc, vb, W, voff, s);
        const int vr = min(max(K - s0, 0), 8);
        if (RG && vr > vb) mix_rayleigh(tb.ray32, tb.n_abs + 2, W, sm.chis, sm.sid + 8 * g, vb, vr, voff, s);
        write_group(g, s);
      }
      if (c0 == 0 && pass == 0) {
        float rp = 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = wave + kWaves * u;
          if (k < ns) rp = fmaf(sm.chis[0][k], rv[u], rp);
        }
        for (int k = wave + 4 * kWaves; k < ns; k += kWaves) rp = fmaf(sm.chis[0][k], tb.ray32[(int64_t)k * W + cc], rp);
        sm.rpart[wave][lane] = rp;
      }
      __syncthreads();   // staged slots visible
      }
      if (first) {
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          acc[r][0] = f32x16{};
          acc[r][1] = f32x16{};
        }
      }

      // products: batches of KB slot blocks, the next batch's A fragments
      // loaded before the current batch's products (PF) or after them.  A
      // wave issues them at a raised priority, lowered again before the
      // depth epilogue (a model of several chunks also stages its later
      // chunks raised): the other waves on its SIMD are mostly staging,
      // whose loads wait on L2 anyway.  15.92 -> 15.82 ms on the 4096-model
      // batch; raising the priority of the staging's load issue instead
      // cost time, and raising it through the epilogue gained less
      __builtin_amdgcn_s_setprio(1);
      for (int kb0 = 0; kb0 < nq; kb0 += KB) {
        u32x4 An[RR][KB][kAW];
        if constexpr (PF)
          if (kb0 + KB < nq) load_A(An, kb0 + KB, kqa, nq);
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          const int kq = kb0 + kk;
          if (kq < nq && ((any_msk >> (kqa + kq)) & 1)) {
            if constexpr (MODE == TRX_FP32) {
              float bk[2][8];
#pragma unroll
              for (int tcb = 0; tcb < 2; ++tcb) {
                const float* src = reinterpret_cast<const float*>(sm.bfrag) + ((kq * 2 + tcb) * 64 + lane) * 8;
                const float4 x0 = *reinterpret_cast<const float4*>(src);
                const float4 x1 = *reinterpret_cast<const float4*>(src + 4);
                bk[tcb][0] = x0.x; bk[tcb][1] = x0.y; bk[tcb][2] = x0.z; bk[tcb][3] = x0.w;
                bk[tcb][4] = x1.x; bk[tcb][5] = x1.y; bk[tcb][6] = x1.z; bk[tcb][7] = x1.w;
              }
#pragma unroll
              for (int r = 0; r < RR; ++r) {
                if ((msk[r] >> (kqa + kq)) & 1) {
#pragma unroll
                  for (int tcb = 0; tcb < 2; ++tcb) {
#pragma unroll
                    for (int st = 0; st < 8; ++st) {
                      const float ah = __uint_as_float(A[r][kk][st >> 2][st & 3]);
                      const float al = __uint_as_float(A[r][kk][2 + (st >> 2)][st & 3]);
                      acc[r][tcb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ah, bk[tcb][st], acc[r][tcb], 0, 0, 0);
                      acc[r][tcb] = __builtin_amdgcn_mfma_f32_32x32x2f32(al, bk[tcb][st], acc[r][tcb], 0, 0, 0);
                    }
                  }
                }
              }
            } else {
              u32x4 Bp[2][npc];
#pragma unroll
              for (int tcb = 0; tcb < 2; ++tcb)
#pragma unroll
                for (int p = 0; p < npc; ++p)
                  Bp[tcb][p] = *reinterpret_cast<const u32x4*>(sm.bfrag + (((kq * npc + p) * 2 + tcb) * 64 + lane) * 4);
#pragma unroll
              for (int r = 0; r < RR; ++r) {
                if ((msk[r] >> (kqa + kq)) & 1) {
#pragma unroll
                  for (int tcb = 0; tcb < 2; ++tcb) {
#pragma unroll
                    for (int pa = 0; pa < npc; ++pa) {
#pragma unroll
                      for (int pb = 0; pb + pa < npc; ++pb)
                        acc[r][tcb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, A[r][kk][pa]), __builtin_bit_cast(bf16x8, Bp[tcb][pb]),
                            acc[r][tcb], 0, 0, 0);
                    }
                  }
                }
              }
            }
          }
        }
        if (kb0 + KB < nq) {
          if constexpr (PF) {
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
              for (int kk = 0; kk < KB; ++kk)
#pragma unroll
                for (int w = 0; w < kAW; ++w) A[r][kk][w] = An[r][kk][w];
          } else {
            load_A(A, kb0 + KB, kqa, nq);
          }
        }
      }
    };
    for (pass = 0; pass < (PASS ? 2 : 1); ++pass) {
    if constexpr (PASS) {
      // this pass's ray block (the previous span ended on the other one)
      set_masks();
      set_awsum();
    }
    run_chunk(0, std::true_type{}, pass == 0 || K > kKC);
    for (int c0 = kKC; c0 < K; c0 += kKC) run_chunk(c0, std::false_type{}, true);
    __builtin_amdgcn_s_setprio(0);

    // depth: accumulator register q holds ray 8 (q/4) + 4 (lane/32) + q%4
    // of column 32 (column block) + lane%32, as -tau_j / ln 2 less the
    // Rayleigh term; sum_j A_j (1 - e^{-tau_j}) is taken as the ray block's
    // sum of A_j less sum_j A_j e^{-tau_j}
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      const int rb = orb(r);
      if (rb < nrb) {
#pragma unroll
        for (int tcb = 0; tcb < 2; ++tcb) {
          const int cl = 32 * tcb + lc;
          const float Rc = sm.rpart[0][cl] + sm.rpart[1][cl] + sm.rpart[2][cl] + sm.rpart[3][cl];
          float s = 0.f;
          double sd = 0.0;
          // emission: the column's wavenumber and the star's 1 - e^{-x_*};
          // wp: 1 - e^{-x} of the lane's previous row (rows 4k .. 4k + 3 of
          // a lane are consecutive layers)
          float nu = 0.f, wst = 0.f, wp = 0.f;
          double nud = 0.0;
          if constexpr (EPI == kEpiEm) {
            const int cg = span * kCols + cl;
            nud = tb.wn[cg < W ? cg : W - 1];
            nu = (float)nud;
            wst = one_minus_exp2(-1.4426950408889634f * nu * (float)hd->em_star);
          }
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const float2 w = sm.aw[32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3)];
            const float x = fmaf(w.y, Rc, acc[r][tcb][q]);   // -tau / ln 2
            if constexpr (EPI == kEpiAcc) {
              sd = fma(sm.a64[32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3)], (double)one_minus_exp2(x), sd);
            } else if constexpr (EPI == kEpiEm) {
              const int j = 32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3);
              constexpr float kL2e = 1.4426950408889634f;
              const float4 e = sm.em[j];
              const float wl = one_minus_exp2(-kL2e * nu * e.x);
              const float wm = (q & 3) ? wp : (j >= 1 ? one_minus_exp2(-kL2e * nu * sm.em[j - 1].x) : 1.f);
              wp = wl;
              if (j >= 1 && j < N) sd += emission_term(e, sm.emz[j], sm.emz[j - 1], x, nu, nud, wst, wl, wm, a);
              // the top layer also carries B_{N-1}/B_* (e^{-tau_N/mu} = 1): added here,
              // before the span's barrier, not by the final sum, whose wave
              // may overlap the next item's loading of these records
              if (j == N - 1) sd += exp_neg_dd(nud * sm.emz[j]) * (double)(wst * __builtin_amdgcn_rcpf(wl));
            } else {
              s = fmaf(w.x, __builtin_amdgcn_exp2f(x), s);
            }
            if constexpr (TAU) {
              const int j = 32 * rb + 8 * (q >> 2) + 4 * hl + (q & 3);
              const int cg = span * kCols + cl;
              if (j < N && cg >= lo && cg < hi)
                a.tau[(int64_t)b * a.tau_ld + (int64_t)j * W + cg] = -0.69314718055994531 * (double)x;
            }
          }
          if constexpr (EPI != kEpiFast) {
            sd += __shfl_xor(sd, 32, 64);
            if (hl == 0) sm.partd[rb][cl] = sd;
          } else {
            s += __shfl_xor(s, 32, 64);
            if (hl == 0) sm.part[rb][cl] = awsum[r] - s;
          }
        }
      }
    }
    }   // passes
    // one barrier ends the span: past it every wave is done with the slot
    // buffer, the ray weights and the Rayleigh sums of this span, so the
    // next span's staging may start while wave 0 sums the partials (they
    // are rewritten only after the next span's staging barrier)
    __syncthreads();
    if (wave == 0 && valid) {
      const int64_t o = (int64_t)b * W + col;
      if constexpr (EPI != kEpiFast) {
        double atm = 0.0;
        for (int rb = 0; rb < nrb; ++rb) atm += sm.partd[rb][lane];
        if constexpr (EPI == kEpiEm) {
          // (Rp/Rs)^2; only the partials (rewritten after the next span's
          // staging barrier) and the model's header are read here
          atm *= hd->em_scale;
          reinterpret_cast<double*>(a.aws)[o] = atm;   // FP64: the flux ratio spans the FP64 range
        } else {
          reinterpret_cast<float*>(a.aws)[o] = (float)atm;
        }
        if (a.depth_native) a.depth_native[o] = hd->Rp2_Rs2 + atm;
        if (!isfinite(atm)) atomicOr(&a.model_status[b], TRX_MODEL_NONFINITE);
      } else {
        float atm = 0.f;
        for (int rb = 0; rb < nrb; ++rb) atm += sm.part[rb][lane];
        reinterpret_cast<float*>(a.aws)[o] = atm;
        if (a.depth_native) a.depth_native[o] = hd->Rp2_Rs2 + (double)atm;
        if (!isfinite(atm)) atomicOr(&a.model_status[b], TRX_MODEL_NONFINITE);
      }
    }
  }
}

// One workgroup per (model, span).
template <int MODE, int RBW, bool TAU, int EPI, bool XT, bool RG>
__global__ __launch_bounds__(64 * kWaves) void k_fwd_mfma(FwdArgs a) {
  __shared__ Smem<MODE, RBW, EPI, XT> sm;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if ((int)blockIdx.x >= B) return;
  const int S = a.span_group;
  process<MODE, RBW, TAU, EPI, XT, 3, RG>(a, blockIdx.x, blockIdx.y * S, blockIdx.y * S + S, sm);
}

// Persistent: a fixed grid pops chunks of (span, model) items from kQueues
// queues, queue q holding the spans s = q (mod kQueues) in increasing order
// and, per span, the models longest first; a workgroup starts on the queue of
// its XCD (workgroups are dealt to the XCDs round-robin) so that the waves of
// one XCD share the table rows of few spans in its L2, and moves on to the
// other queues when its own is drained.  Every workgroup leaves once all
// queues are drained.
template <int MODE, int RBW, int EPI, bool XT, int OCC = 3, bool RG = false>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(OCC))) void k_fwd_mfma_persist(FwdArgs a) {
  __shared__ Smem<MODE, RBW, EPI, XT> sm;
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
        if (bm >= 0) process<MODE, RBW, false, EPI, XT, OCC, RG>(a, bm, sm.spans[c] * S, sm.spans[c] * S + S, sm);
      }
      __syncthreads();
    }
  }
}

template <int MODE, int RBW, int EPI, bool XT, int OCC, bool RG>
int occupancy() {
  static int blocks = 0;
  if (!blocks) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_mfma_persist<MODE, RBW, EPI, XT, OCC, RG>, 64 * kWaves,
                                                     0) !=
            hipSuccess || nb < 1)
      nb = 1;
    blocks = nb;
  }
  return blocks;
}

// The optical-depth output always takes the one-workgroup-per-item kernel.
template <int MODE, int RBW, int EPI, bool XT, int OCC = 3, bool RG = false>
void launch_rbw_epi(const FwdArgs& a, int B_grid, int n_cu, hipStream_t s) {
  if (a.persistent && !a.tau) {
    const int grid = n_cu * occupancy<MODE, RBW, EPI, XT, OCC, RG>();
    hipLaunchKernelGGL((k_fwd_mfma_persist<MODE, RBW, EPI, XT, OCC, RG>), dim3(grid), dim3(64 * kWaves), 0, s, a);
  } else {
    dim3 grid(B_grid, ((a.tab.n_wn + kCols - 1) / kCols + a.span_group - 1) / a.span_group);
    if (a.tau)
      hipLaunchKernelGGL((k_fwd_mfma<MODE, RBW, true, kEpiFast, XT, RG>), grid, dim3(64 * kWaves), 0, s, a);
    else
      hipLaunchKernelGGL((k_fwd_mfma<MODE, RBW, false, EPI, XT, RG>), grid, dim3(64 * kWaves), 0, s, a);
  }
}

// The build for two-layer layouts or the one without their code.
template <int MODE, int RBW, int EPI, bool XT>
void launch_rg(const FwdArgs& a, int B_grid, int n_cu, hipStream_t s) {
  if (a.L.rg) launch_rbw_epi<MODE, RBW, EPI, XT, 3, true>(a, B_grid, n_cu, s);
  else launch_rbw_epi<MODE, RBW, EPI, XT, 3, false>(a, B_grid, n_cu, s);
}

// The optical-depth output (transmission only) takes the fast epilogue: it
// writes tau, not the depth's rounding.
template <int MODE, int RBW>
void launch_rbw(const FwdArgs& a, int B_grid, int n_cu, int occ, hipStream_t s) {
  // the four-workgroup build (fast transit epilogue): one ray block per
  // wave, or two in two passes
  if (occ == 4 && !a.L.xt && !a.L.em && !a.accurate && !a.L.rg) {
    launch_rbw_epi<MODE, RBW, kEpiFast, false, 4>(a, B_grid, n_cu, s);
    return;
  }
  // the exponential scheme has no gradient, so no accurate epilogue; nor
  // have two-layer layouts
  if (a.L.xt) {
    if (a.L.em) launch_rg<MODE, RBW, kEpiEm, true>(a, B_grid, n_cu, s);
    else launch_rg<MODE, RBW, kEpiFast, true>(a, B_grid, n_cu, s);
  } else if (a.L.em) {
    launch_rg<MODE, RBW, kEpiEm, false>(a, B_grid, n_cu, s);
  } else if (a.accurate && !a.tau && !a.L.rg) {
    launch_rbw_epi<MODE, RBW, kEpiAcc, false>(a, B_grid, n_cu, s);
  } else {
    launch_rg<MODE, RBW, kEpiFast, false>(a, B_grid, n_cu, s);
  }
}

// Ray blocks per wave: one (the waves own ray blocks 0-3) for models of at
// most 128 rays unless rbw asks for two, else two (0-3 and 7-4).
template <int MODE>
void launch_mode(const FwdArgs& a, int nrb, int rbw, int occ, int B_grid, int n_cu, hipStream_t s) {
  if (nrb <= 4 && rbw != 2) launch_rbw<MODE, 1>(a, B_grid, n_cu, occ, s);
  else launch_rbw<MODE, 2>(a, B_grid, n_cu, occ, s);
}

}  // namespace

void launch_fwd_mfma(const FwdArgs& a, int precision, int nrb_max, int rbw, int occ, int B_grid, int n_cu,
                     hipStream_t s) {
  if (B_grid <= 0) return;
  switch (precision) {
    case TRX_FP32: launch_mode<TRX_FP32>(a, nrb_max, rbw, occ, B_grid, n_cu, s); break;
    case TRX_BF16_SPLIT2: launch_mode<TRX_BF16_SPLIT2>(a, nrb_max, rbw, occ, B_grid, n_cu, s); break;
    default: launch_mode<TRX_BF16_SPLIT3>(a, nrb_max, rbw, occ, B_grid, n_cu, s); break;
  }
}

}  // namespace trx
