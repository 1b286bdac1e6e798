// FP64 forward kernel (the reference path): opacity (a4), optical depth
// (a5) and depth (a6) of one (model, 64-column span) per workgroup of four
// waves, with the same structure as the matrix-core kernel of the fast modes
// but FP64 throughout.
//
// The model's distinct (T, log10 P) corners are mixed over the absorbers,
// M_q = sum_i chi_i sigma_i[q], for the workgroup's 64 columns and staged in
// LDS (per 16-layer block when there are too many); so are the CIA sums.  Per
// 16-layer block each wave computes 4 layers of
//   kappa_l = sum_q w_lq M_q + w_R R + w_c0 C_0 + w_c1 C_1
// (equations opt_dpth, cia_opt_dpth, contrib; Opacities section) into LDS,
// and the optical depth tau[ray, col] += dl[ray, block] kappa[block, col] is
// accumulated on the FP64 matrix instruction v_mfma_f64_16x16x4_f64 with
// 16-ray x 16-column tiles: wave w owns the 16-ray blocks w, w+4, ... (all
// four column blocks), a ray block takes the layers at or above its first
// ray.  Models above 256 layers take several passes over the ray blocks.
// Depth: D = (Rp/Rs)^2 + sum_j (A_j/Rs^2)(-expm1(-tau_j)), the per-ray-block
// partials summed in a fixed order.
//
// Models of at most TRX_MAX_LAYERS_MFMA layers take the slot form instead
// (k_fwd64s): tau_j = sum_q P[j][q] M_q + PR_j R with P = dl W formed once
// per model by the geometry in FP64, so each span stages the mixed rows M
// of the model's opacity slots (table corners and CIA nodes) and contracts
// over them on the same FP64 instruction, skipping the slot blocks whose P
// is zero for a ray block; no per-layer opacity is formed.
//
// Tables in the exponential temperature scheme (Opacities section) have one
// absorber slot per layer: its row is the layer's own mixed cross-section,
// sum_i chi_i sigma_i with sigma_i = sigma1 e^{u ln(sigma2/sigma1)} at the two
// pressure nodes of the layer's bracket and linear in log10 P between them;
// the dense kernel forms the same per layer.
#include "trx_internal.h"

namespace trx {

namespace {

constexpr int kWaves = 4;
constexpr int kCols = 64;
constexpr int kRows = 96;                 // staged corner + CIA rows
static_assert(kRows >= kMaxU + kMaxV, "block staging must fit");
constexpr int kRBW = 4;                   // 16-ray blocks per wave per pass

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct Smem64 {
  double rows[kRows][kCols];
  double kap[16][kCols];
  double part[kWaves * kRBW][kCols];
  double atm[kCols];
  double lw[16][8];
  int2 sl[16];
  int32_t ids[kRows];
  int32_t tids[kRows];
};

// rows[u][lane] = sum_i chi[i] * tab[i][ids[u]][col] (FP64 table laid out
// [i][corner][W]), corners u = wave, wave + 4, ...; 8 corners' loads of one
// absorber are issued together.
__device__ inline void stage64(const double* tab, int64_t abs_stride, int W, int col, const int32_t* ids, int nU,
                               const double* chi, int nabs, double* rows, int wave, int lane) {
  constexpr int G = 8;
  for (int u0 = wave; u0 < nU; u0 += kWaves * G) {
    int64_t off[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int u = u0 + kWaves * g < nU ? u0 + kWaves * g : u0;
      off[g] = (int64_t)__builtin_amdgcn_readfirstlane(ids[u]) * W + col;
    }
    double s[G];
#pragma unroll
    for (int g = 0; g < G; ++g) s[g] = 0.0;
    for (int i = 0; i < nabs; ++i) {
      const double* p = tab + (int64_t)i * abs_stride;
      double v[G];
#pragma unroll
      for (int g = 0; g < G; ++g) v[g] = p[off[g]];
      const double c = chi[i];
#pragma unroll
      for (int g = 0; g < G; ++g) s[g] = fma(c, v[g], s[g]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (u0 + kWaves * g < nU) rows[(u0 + kWaves * g) * kCols + lane] = s[g];
  }
}

// Exponential temperature scheme in FP64 (Opacities section):
// sigma1 (sigma2/sigma1)^u = sigma1 e^{u ln(sigma2/sigma1)}, or the linear
// form where either node value is not positive.
__device__ inline double xt_sigma64(double s1, double s2, double u, double wT) {
  return (s1 > 0.0 && s2 > 0.0) ? s1 * exp(u * log(s2 / s1)) : fma(wT, s2 - s1, s1);
}
// sum_t wt[t] sigma_t at the layer of record r = {u, w_P, w_T, 0} whose
// lower corner (iT, iP) has row offset o (= (iT n_P + iP) W + column):
// the exponential form in T at both pressure nodes, then linear in log10 P.
__device__ inline double xt_mix64(const double* tab, int64_t stride, int nt, const double* wt, int64_t o,
                                  double4 r, int W, int nP) {
  double acc = 0.0;
  const int64_t dT = (int64_t)nP * W;
  for (int t = 0; t < nt; ++t) {
    const double* p = tab + (int64_t)t * stride + o;
    const double g0 = xt_sigma64(p[0], p[dT], r.x, r.z);
    const double g1 = xt_sigma64(p[W], p[dT + W], r.x, r.z);
    acc = fma(wt[t], fma(r.y, g1 - g0, g0), acc);
  }
  return acc;
}

// TAU: also write the optical depth of every ray and column to a.tau (a
// separate instantiation: the stores cost the kernel registers)
template <bool TAU>
__device__ void process64(const FwdArgs& a, int b_in, int span_in, Smem64& sm) {
  const int b = __builtin_amdgcn_readfirstlane(b_in);
  const int span = __builtin_amdgcn_readfirstlane(span_in);
  const Layout& L = a.L;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  const int N = hd->n;
  if (N == 0) return;
  const int lo = hd->lo, hi = hd->hi;
  const int col0 = span * kCols;
  if (col0 >= hi || col0 + kCols <= lo) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  const int col = col0 + lane;
  const bool valid = col >= lo && col < hi;
  const int cc = valid ? col : lo;
  const DevTables& tb = a.tab;
  const int W = tb.n_wn;
  const bool has_cia = tb.n_cia > 0;

  double R = 0.0;
  if (tb.has_rayleigh)
    for (int s = 0; s < tb.n_abs + 2; ++s) R = fma(hd->chi_s[s], tb.ray64[(int64_t)s * W + cc], R);

  const double* lw = reinterpret_cast<const double*>(slab + L.off_lw64);
  const int32_t* lid = reinterpret_cast<const int32_t*>(slab + L.off_lid);
  const KBlk* kblk = reinterpret_cast<const KBlk*>(slab + L.off_kblk);
  const MList* ml = reinterpret_cast<const MList*>(slab + L.off_mlist);
  const double* A = reinterpret_cast<const double*>(slab + L.off_A64);
  const double* dlT = reinterpret_cast<const double*>(slab + L.off_dl);
  const int NP = L.NP;
  const int nkb = (N + 15) / 16;
  const int64_t abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  const int64_t cia_stride = (int64_t)tb.n_Tcia * W;

  double* rows = &sm.rows[0][0];
  double* crows = rows;
  auto stage = [&](const int32_t* ids, int nU, const int32_t* tids, int nV) {
    for (int e = tid; e < nU; e += 64 * kWaves) sm.ids[e] = ids[e];
    for (int e = tid; e < nV; e += 64 * kWaves) sm.tids[e] = tids[e];
    __syncthreads();
    stage64(tb.xsec64, abs_stride, W, cc, sm.ids, nU, hd->chi_s, tb.n_abs, rows, wave, lane);
    crows = rows + nU * kCols;
    if (has_cia) stage64(tb.cia64, cia_stride, W, cc, sm.tids, nV, hd->cia_w, tb.n_cia, crows, wave, lane);
  };
  // the exponential scheme forms each layer's cross-sections directly: only
  // the CIA rows are staged
  const bool xt = L.xt != 0;
  const double4* xt64 = reinterpret_cast<const double4*>(slab + L.off_xt64);
  const int nUs = xt ? 0 : ml->nU;
  const bool mstage = nUs + ml->nV <= kRows && ml->nV <= kMListV;
  const int slot_off = mstage ? 2 : 4;
  if (mstage) stage(ml->ids, nUs, ml->tids, ml->nV);
  if (tid < kCols) sm.atm[tid] = 0.0;

  const int nrb16 = (N + 15) / 16;
  for (int p0 = 0; p0 < nrb16; p0 += kWaves * kRBW) {
    f64x4 acc[kRBW][4];
#pragma unroll
    for (int r = 0; r < kRBW; ++r)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[r][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
    // ray block p0 starts at ray 16 p0: layer blocks from p0 on
    for (int kb = p0; kb < nkb; ++kb) {
      if (!mstage) {
        const KBlk* kd = kblk + kb;
        stage(kd->ids, xt ? 0 : kd->nU, kd->tids, kd->nV);
      }
      if (tid < 16 * 8) {
        const int l = 16 * kb + tid / 8;
        sm.lw[tid / 8][tid % 8] = l < N ? lw[8 * l + tid % 8] : 0.0;
      }
      if (tid < 16) {
        const int l = 16 * kb + tid;
        sm.sl[tid] = l < N ? *reinterpret_cast<const int2*>(lid + 8 * l + slot_off) : make_int2(0, 0);
      }
      __syncthreads();
      // opacity of layers 16 kb + 4 wave + jj
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int k = 4 * wave + jj;
        const int l = 16 * kb + k;
        double kv = 0.0;
        if (l < N) {
          const double* w = sm.lw[k];
          if (xt) {
            const int64_t o = (int64_t)lid[8 * l] * W + cc;
            kv = w[0] * xt_mix64(tb.xsec64, abs_stride, tb.n_abs, hd->chi_s, o, xt64[N - 1 - l], W, tb.n_P);
          } else {
            const uint32_t sl = __builtin_amdgcn_readfirstlane((uint32_t)sm.sl[k].x);
            kv = w[0] * rows[(sl & 0xff) * kCols + lane];
            kv = fma(w[1], rows[((sl >> 8) & 0xff) * kCols + lane], kv);
            kv = fma(w[2], rows[((sl >> 16) & 0xff) * kCols + lane], kv);
            kv = fma(w[3], rows[(sl >> 24) * kCols + lane], kv);
          }
          kv = fma(w[4], R, kv);
          if (has_cia) {
            const uint32_t cl = __builtin_amdgcn_readfirstlane((uint32_t)sm.sl[k].y);
            kv = fma(w[5], crows[(cl & 0xff) * kCols + lane], kv);
            kv = fma(w[6], crows[((cl >> 8) & 0xff) * kCols + lane], kv);
          }
        }
        sm.kap[k][lane] = kv;
      }
      __syncthreads();
      // tau += dl x kappa on 16x16x4 FP64 tiles; A operand lane l holds
      // dl[16 rb + l%16][4 s + l/16], B operand kappa[4 s + l/16][16 cb + l%16]
#pragma unroll
      for (int r = 0; r < kRBW; ++r) {
        const int rb = p0 + wave + kWaves * r;
        if (rb < nrb16 && kb >= rb) {
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const int k = 4 * st + (lane >> 4);
            const double av = dlT[(int64_t)(16 * kb + k) * NP + 16 * rb + (lane & 15)];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
              const double bv = sm.kap[k][16 * cb + (lane & 15)];
              acc[r][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[r][cb], 0, 0, 0);
            }
          }
        }
      }
      __syncthreads();
    }
    // depth partials: accumulator element q of lane l is ray l/16 + 4 q of
    // the block (the FP64 instruction interleaves its output rows)
#pragma unroll
    for (int r = 0; r < kRBW; ++r) {
      const int rb = p0 + wave + kWaves * r;
      if (rb < nrb16) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = 16 * rb + (lane >> 4) + 4 * q;
            s = fma(A[j], -expm1(-acc[r][cb][q]), s);
            if constexpr (TAU) {
              const int cg = col0 + 16 * cb + (lane & 15);
              if (j < N && cg >= lo && cg < hi) a.tau[(int64_t)b * a.tau_ld + (int64_t)j * W + cg] = acc[r][cb][q];
            }
          }
          s += __shfl_xor(s, 16, 64);
          s += __shfl_xor(s, 32, 64);
          if (lane < 16) sm.part[wave + kWaves * r][16 * cb + lane] = s;
        }
      } else if (lane < 16) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) sm.part[wave + kWaves * r][16 * cb + lane] = 0.0;
      }
    }
    __syncthreads();
    if (tid < kCols) {
      // slot wave + 4 r holds ray block p0 + wave + 4 r: summed in ray order
      double s = sm.atm[tid];
      for (int i = 0; i < kWaves * kRBW; ++i) s += sm.part[i][tid];
      sm.atm[tid] = s;
    }
    __syncthreads();
  }
  if (tid < kCols && valid) {
    const double atm = sm.atm[tid];
    const int64_t o = (int64_t)b * W + col;
    reinterpret_cast<double*>(a.aws)[o] = atm;
    if (a.depth_native) a.depth_native[o] = hd->Rp2_Rs2 + atm;
    if (!isfinite(atm)) atomicOr(&a.model_status[b], TRX_MODEL_NONFINITE);
  }
  __syncthreads();
}

template <bool TAU>
__global__ __launch_bounds__(64 * kWaves) void k_fwd64(FwdArgs a) {
  __shared__ Smem64 sm;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if ((int)blockIdx.x >= B) return;
  process64<TAU>(a, blockIdx.x, blockIdx.y, sm);
}


// ---- slot form ------------------------------------------------------------
constexpr int kKC64 = 96;    // slots per staging chunk
constexpr int kLd64 = 66;    // LDS row stride (doubles): the four row groups of a read hit distinct banks
constexpr int kR16 = 2;      // 16-ray blocks per wave per pass
static_assert(TRX_MAX_LAYERS_MFMA % 16 == 0, "16-ray blocks");

template <bool EM>
struct Smem64s {
  double rows[kKC64][kLd64];                       // mixed slot rows of the chunk
  double part[TRX_MAX_LAYERS_MFMA / 16][kCols];    // per-16-ray-block depth partials
  double rpart[kWaves][kCols];                     // Rayleigh sums by wave
  double A[TRX_MAX_LAYERS_MFMA];                   // A_j/Rs^2
  double PR[TRX_MAX_LAYERS_MFMA];                  // Rayleigh path weights
  int32_t sid[kKC64];
  double chis[kMaxRegimes][kMaxSpecies];   // mixing ratios per run (two-layer profiles; else run 0)
  double ciaw[kMaxRegimes][TRX_MAX_CIA];   // CIA pair weights times kCiaScale32 (the scale of P's CIA columns)
  double4 em[EM ? TRX_MAX_LAYERS_MFMA : 1];        // emission: the layer records
};

// One row's term of the emission flux ratio in FP64 (before (Rp/Rs)^2):
// (B_{l-1} - B_l)/B_* G(tau_l), G(tau) = sum_i 2 w_i mu_i e^{-tau/mu_i},
// from the records e (layer l: c2/T_l, c2 (T_{l-1} - T_l)/(T_l T_{l-1}),
// c2 (1/T_l - 1/T_*), the deck's vertical optical depth) and em (layer
// l - 1), the gas optical depth tau, the wavenumber nu and 1 - e^{-x_*}.
// B/B_* = e^{x_* - x} (1 - e^{-x_*})/(1 - e^{-x}); neighbouring layers'
// difference without cancellation as in the matrix-core kernel.
__device__ inline double emission_term64(double4 e, double4 em, double tau, double nu, double wst,
                                         const FwdArgs& a) {
  const double tt = tau + e.w;
  double G = 0.0;
  for (int i = 0; i < a.n_mu; ++i) G = fma(a.em_c64[i], exp(-tt * a.em_k64[i]), G);
  const double wl = -expm1(-nu * e.x), wm = -expm1(-nu * em.x);
  const double rl = exp(-nu * e.z);
  const double dx = nu * e.y;
  const double dB = fabs(dx) <= 1.0 ? rl * expm1(dx) * wst / (wm * wl) : wst * (exp(-nu * em.z) / wm - rl / wl);
  return dB * G;
}

// s[i] += sum_t wt[t] tab_t[rows[i]][col] over the tables t < nt for the
// slots i in [i0, i1) of a group of 8 (rows of the others clamped into it).
__device__ inline void mix64(const double* tab, int64_t stride, int nt, const double* wt, const int32_t* rows, int i0,
                             int i1, int W, int col, double (&s)[8]) {
  int64_t off[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = i < i0 ? i0 : (i >= i1 ? i1 - 1 : i);
    off[i] = (int64_t)(__builtin_amdgcn_readfirstlane(rows[k]) & 0xffffff) * W + col;
  }
  for (int t0 = 0; t0 < nt; t0 += 2) {
    double v[2][8];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
      if (t0 + tt < nt) {
        const double* p = tab + (int64_t)(t0 + tt) * stride;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[tt][i] = p[off[i]];
      }
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
      if (t0 + tt < nt) {
        const double c = wt[t0 + tt];
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (i >= i0 && i < i1) s[i] = fma(c, v[tt][i], s[i]);
      }
  }
}

template <bool TAU, bool EM>
__device__ void process64s(const FwdArgs& a, int b_in, int s_first, int s_end, Smem64s<EM>& sm) {
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
  const int nR = L.rg ? ml->pad[0] : 0;   // Rayleigh slots, one per run (two-layer layouts)
  const int K = nU + nV + nR;
  const int nrb = hd->nrb, n16 = 2 * nrb;
  const int NKQ = L.NKQ;
  const int32_t* sid = reinterpret_cast<const int32_t*>(slab + L.off_sid);
  const double* P = reinterpret_cast<const double*>(slab + L.off_dl);
  const double* A64 = reinterpret_cast<const double*>(slab + L.off_A64);
  const double* PR64 = reinterpret_cast<const double*>(slab + L.off_pr64);
  const int64_t abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  const int64_t cia_stride = (int64_t)tb.n_Tcia * W;
  const int ns = tb.has_rayleigh && !L.rg ? tb.n_abs + 2 : 0;

  if (tid < 32 * nrb) {
    sm.A[tid] = tid < N ? A64[tid] : 0.0;
    sm.PR[tid] = tid < N ? PR64[tid] : 0.0;
    if constexpr (EM) sm.em[tid] = reinterpret_cast<const double4*>(slab + L.off_em64)[tid];
  }
  if (K <= kKC64 && tid < K) sm.sid[tid] = sid[tid];
  if (tid < kMaxSpecies) sm.chis[0][tid] = hd->chi_s[tid];
  if (tid < TRX_MAX_CIA) sm.ciaw[0][tid] = hd->cia_w[tid] * kCiaScale32;
  if (L.rg && tid < kMaxSpecies) {
    // the other runs' mixing ratios (two-layer profiles)
    const RegChem* rc = reinterpret_cast<const RegChem*>(slab + L.off_rg);
    for (int r = 1; r < kMaxRegimes; ++r) {
      sm.chis[r][tid] = rc[r].chi_s[tid];
      if (tid < TRX_MAX_CIA) sm.ciaw[r][tid] = rc[r].cia_w[tid] * kCiaScale32;
    }
  }
  __syncthreads();

  for (int span = sp0; span < sp1; ++span) {
    const int col0 = span * kCols;
    const int col = col0 + lane;
    const bool valid = col >= lo && col < hi;
    const int cc = valid ? col : lo;
    {
      double rp = 0.0;
      for (int k = wave; k < ns; k += kWaves) rp = fma(sm.chis[0][k], tb.ray64[(int64_t)k * W + cc], rp);
      sm.rpart[wave][lane] = rp;
    }
    // stage the slot chunk c0 .. (8-slot groups g = wave, wave + 4, ...)
    auto stage_chunk = [&](int c0) {
      const int kc = min(kKC64, K - c0);
      if (K > kKC64) {
        __syncthreads();
        if (tid < kc) sm.sid[tid] = sid[c0 + tid];
        __syncthreads();
      }
      const int ng = 2 * ((kc + 15) / 16);
      for (int g = wave; g < ng; g += kWaves) {
        const int s0 = c0 + 8 * g;
        // the run of the group (its first slot's; two-layer layouts pad
        // each run's slots of one kind to whole groups)
        const int rg = s0 < K ? min((int)((uint32_t)__builtin_amdgcn_readfirstlane(sm.sid[8 * g]) >> 24),
                                    kMaxRegimes - 1) : 0;
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = 0.0;
        const int nc = min(max(nU - s0, 0), 8);
        if (nc > 0 && L.xt) {
          // exponential scheme: layer slots (records by slot)
          const double4* xr = reinterpret_cast<const double4*>(slab + L.off_xt64) + s0;
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (i < nc)
              v[i] = xt_mix64(tb.xsec64, abs_stride, tb.n_abs, sm.chis[rg],
                              (int64_t)(__builtin_amdgcn_readfirstlane(sm.sid[8 * g + i]) & 0xffffff) * W + cc,
                              xr[i], W, tb.n_P);
        } else if (nc > 0) {
          mix64(tb.xsec64, abs_stride, tb.n_abs, sm.chis[rg], sm.sid + 8 * g, 0, nc, W, cc, v);
        }
        const int vb = min(max(nU + nV - s0, 0), 8);
        if (vb > nc) mix64(tb.cia64, cia_stride, tb.n_cia, sm.ciaw[rg], sm.sid + 8 * g, nc, vb, W, cc, v);
        // Rayleigh slots (two-layer layouts): each its own run's mix
        const int vr = min(max(K - s0, 0), 8);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if (i >= vb && i < vr) {
            const int r = min((int)((uint32_t)__builtin_amdgcn_readfirstlane(sm.sid[8 * g + i]) >> 24), kMaxRegimes - 1);
            double acc = 0.0;
            for (int k = 0; k < tb.n_abs + 2; ++k) acc = fma(sm.chis[r][k], tb.ray64[(int64_t)k * W + cc], acc);
            v[i] = acc;
          }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) sm.rows[8 * g + i][lane] = v[i];
      }
      __syncthreads();
    };
    if (K <= kKC64) stage_chunk(0);

    // passes over the 16-ray blocks: wave w takes blocks p0 + w + 4 r
    for (int p0 = 0; p0 < n16; p0 += kWaves * kR16) {
      f64x4 acc[kR16][4];
#pragma unroll
      for (int r = 0; r < kR16; ++r)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[r][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
      uint64_t msk[kR16];
#pragma unroll
      for (int r = 0; r < kR16; ++r) {
        const int r16 = p0 + wave + kWaves * r;
        msk[r] = r16 < n16 ? hd->kq_mask[r16 >> 1] : 0ull;
      }
      for (int c0 = 0; c0 < K; c0 += kKC64) {
        if (K > kKC64) stage_chunk(c0);
        const int nq = (min(kKC64, K - c0) + 15) >> 4;
        for (int kq = 0; kq < nq; ++kq) {
          const int kqa = (c0 >> 4) + kq;
          if (!(((msk[0] | msk[1]) >> kqa) & 1)) continue;
          double bv[4][4];
#pragma unroll
          for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
              bv[st][cb] = sm.rows[16 * kq + 4 * st + (lane >> 4)][16 * cb + (lane & 15)];
#pragma unroll
          for (int r = 0; r < kR16; ++r) {
            if ((msk[r] >> kqa) & 1) {
              const int r16 = p0 + wave + kWaves * r;
              const double4 av = *reinterpret_cast<const double4*>(P + (((int64_t)r16 * NKQ + kqa) * 64 + lane) * 4);
              const double avs[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
              for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                  acc[r][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(avs[st], bv[st][cb], acc[r][cb], 0, 0, 0);
            }
          }
        }
      }
      // depth partials: element q of lane l is ray 16 r16 + l/16 + 4 q
#pragma unroll
      for (int r = 0; r < kR16; ++r) {
        const int r16 = p0 + wave + kWaves * r;
        if (r16 < n16) {
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            const int c = 16 * cb + (lane & 15);
            double Rc = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) Rc += sm.rpart[w][c];
            if constexpr (EM) {
              // emission: the rows' terms of the flux ratio
              const int cg = col0 + c;
              const double nu = tb.wn[cg < W ? cg : W - 1];
              const double wst = -expm1(-nu * hd->em_star);
              double s = 0.0;
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int j = 16 * r16 + (lane >> 4) + 4 * q;
                if (j >= 1 && j < N)
                  s += emission_term64(sm.em[j], sm.em[j - 1], fma(sm.PR[j], Rc, acc[r][cb][q]), nu, wst, a);
              }
              s += __shfl_xor(s, 16, 64);
              s += __shfl_xor(s, 32, 64);
              if (lane < 16) sm.part[r16][c] = s;
              continue;
            }
            // sum_j A_j (1 - e^{-tau_j}) as the block's sum of A_j less
            // sum_j A_j e^{-tau_j}, the first summed in the same order (a
            // block with tau = 0 adds exactly zero); the difference loses
            // at most ~1e-16 of sum_j A_j, against expm1 per element
            double s = 0.0, sa = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int j = 16 * r16 + (lane >> 4) + 4 * q;
              const double tau = fma(sm.PR[j], Rc, acc[r][cb][q]);
              s = fma(sm.A[j], exp(-tau), s);
              sa = fma(sm.A[j], 1.0, sa);
              if constexpr (TAU) {
                const int cg = col0 + c;
                if (j < N && cg >= lo && cg < hi) a.tau[(int64_t)b * a.tau_ld + (int64_t)j * W + cg] = tau;
              }
            }
            s += __shfl_xor(s, 16, 64);
            s += __shfl_xor(s, 32, 64);
            sa += __shfl_xor(sa, 16, 64);
            sa += __shfl_xor(sa, 32, 64);
            if (lane < 16) sm.part[r16][c] = sa - s;
          }
        }
      }
    }
    __syncthreads();
    if (tid < kCols && valid) {
      double atm = 0.0;
      for (int r16 = 0; r16 < n16; ++r16) atm += sm.part[r16][tid];
      if constexpr (EM) {
        // the top layer's B_{N-1}/B_*, then (Rp/Rs)^2
        const double nu = tb.wn[col];
        const double4 e = sm.em[N - 1];
        atm = hd->em_scale * (atm + exp(-nu * e.z) * (-expm1(-nu * hd->em_star)) / (-expm1(-nu * e.x)));
      }
      const int64_t o = (int64_t)b * W + col;
      reinterpret_cast<double*>(a.aws)[o] = atm;
      if (a.depth_native) a.depth_native[o] = hd->Rp2_Rs2 + atm;
      if (!isfinite(atm)) atomicOr(&a.model_status[b], TRX_MODEL_NONFINITE);
    }
    __syncthreads();   // rows, partials and Rayleigh sums are rewritten by the next span
  }
}

template <bool TAU, bool EM>
__global__ __launch_bounds__(64 * kWaves) void k_fwd64s(FwdArgs a) {
  __shared__ Smem64s<EM> sm;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if ((int)blockIdx.x >= B) return;
  const int S = a.span_group;
  process64s<TAU, EM>(a, blockIdx.x, blockIdx.y * S, blockIdx.y * S + S, sm);
}

}  // namespace

void launch_fwd64(const FwdArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return;
  const int spans = (a.tab.n_wn + kCols - 1) / kCols;
  if (a.L.slot64) {
    const int S = a.span_group > 0 ? a.span_group : 1;
    const dim3 grid(B_grid, (spans + S - 1) / S);
    if (a.L.em)
      hipLaunchKernelGGL((k_fwd64s<false, true>), grid, dim3(64 * kWaves), 0, s, a);
    else if (a.tau)
      hipLaunchKernelGGL((k_fwd64s<true, false>), grid, dim3(64 * kWaves), 0, s, a);
    else
      hipLaunchKernelGGL((k_fwd64s<false, false>), grid, dim3(64 * kWaves), 0, s, a);
  } else if (a.tau) {
    hipLaunchKernelGGL(k_fwd64<true>, dim3(B_grid, spans), dim3(64 * kWaves), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_fwd64<false>, dim3(B_grid, spans), dim3(64 * kWaves), 0, s, a);
  }
}

}  // namespace trx
