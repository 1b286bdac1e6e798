// FP64 forward kernel: opacity (a4), optical depth (a5) and depth (a6) for
// one (model, 256-column span) per workgroup, one 64-column slice per wave.
//
// Each lane owns one wavenumber.  The absorption coefficient of layer k is
// (equations opt_dpth, cia_opt_dpth, contrib; Opacities section)
//   kappa_k = sum_q w_kq M_q + w_R R + w_c0 C_0 + w_c1 C_1,
// where M_q = sum_i chi_i sigma_i(corner q) are the mixing-ratio-weighted
// table values at the four (T, log10 P) corners of the layer's bracket,
// R = sum_s chi_s sigma_R,s and C = sum_pairs chi_a chi_b sigma_pair(T node):
// since every table shares the T and P grids, the bilinear weights are the
// same for all absorbers and the sum over absorbers can be taken once per
// corner instead of once per layer.  The weights (bilinear factors times
// 1e-4 rho, 1e-10 rho^2) are per-layer records written by the geometry
// kernel, identical for all lanes, so they come from scalar loads.
//
// The optical depth tau_j = sum_{k>=j} dl[j,k] kappa_k is accumulated for 32
// rays at a time in registers (FP64 FMA with the path lengths as scalar
// operands); kappa is recomputed for each 32-ray block.  The depth adds
// sum_j (A_j/Rs^2) (1 - exp(-tau_j)) with 1 - exp(-tau) = -expm1(-tau).
#include "trx_internal.h"

namespace trx {

namespace {

constexpr int kWaves = 1;
constexpr int kSpan = 64 * kWaves;

// Mixing-ratio-weighted table values of one column in FP64:
// M(c) = sum_i chi_i sigma_i[c] and C(t) = sum_p (chi chi')_p sigma_p[t].
struct Mixer64 {
  const double* xs;   // xsec64 + col
  const double* ci;   // cia64 + col
  int64_t abs_stride; // n_T * n_P * n_wn
  int64_t cia_stride; // n_Tcia * n_wn
  int W, nabs, ncia;
  const double* chi;  // header chi_s
  const double* ciaw; // header cia_w

  __device__ double corner(int c) const {
    double s = 0.0;
    const double* p = xs + (int64_t)c * W;
    for (int i = 0; i < nabs; ++i) s = fma(chi[i], p[i * abs_stride], s);
    return s;
  }
  __device__ double cia(int t) const {
    double s = 0.0;
    const double* p = ci + (int64_t)t * W;
    for (int q = 0; q < ncia; ++q) s = fma(ciaw[q], p[q * cia_stride], s);
    return s;
  }
};

constexpr int kRowsAbs = 80;
constexpr int kRowsCia = 32;
static_assert(kRowsAbs >= kMaxU && kRowsCia >= kMaxV, "block staging must fit");

__device__ inline void stage64(const Mixer64& m, const int32_t* ids, int nU, const int32_t* tids,
                               int nV, double* rows, double* crows, int lane) {
  for (int u0 = 0; u0 < nU; u0 += 16) {
    double s[16];
#pragma unroll
    for (int g = 0; g < 16; ++g) s[g] = 0.0;
    for (int i = 0; i < m.nabs; ++i) {
      const double x = m.chi[i];
      double v[16];
#pragma unroll
      for (int g = 0; g < 16; ++g) {
        const int u = u0 + g < nU ? u0 + g : nU - 1;
        v[g] = m.xs[(int64_t)ids[u] * m.W + i * m.abs_stride];
      }
#pragma unroll
      for (int g = 0; g < 16; ++g) s[g] = fma(x, v[g], s[g]);
    }
#pragma unroll
    for (int g = 0; g < 16; ++g)
      if (u0 + g < nU) rows[(u0 + g) * 64 + lane] = s[g];
  }
  for (int v = 0; v < nV; ++v) crows[v * 64 + lane] = m.cia(tids[v]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * kWaves) void k_fwd64(FwdArgs a) {
  __shared__ double s_rows[kWaves][kRowsAbs + kRowsCia][64];
  const int b = blockIdx.x;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const Layout& L = a.L;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* h = reinterpret_cast<const ModelHdr*>(slab);
  const int N = h->n;
  if (N == 0) return;
  const int lo = h->lo, hi = h->hi;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col0 = blockIdx.y * kSpan + wave * 64;
  if (col0 >= hi || col0 + 64 <= lo) return;
  const int col = col0 + lane;
  const bool valid = col >= lo && col < hi;
  const int cc = valid ? col : lo;
  const DevTables& tb = a.tab;
  const int W = tb.n_wn;

  Mixer64 m;
  m.xs = tb.xsec64 + cc;
  m.ci = tb.cia64 + cc;
  m.abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  m.cia_stride = (int64_t)tb.n_Tcia * W;
  m.W = W; m.nabs = tb.n_abs; m.ncia = tb.n_cia;
  m.chi = h->chi_s;
  m.ciaw = h->cia_w;
  const bool has_cia = tb.n_cia > 0;

  double R = 0.0;
  if (tb.has_rayleigh)
    for (int s = 0; s < tb.n_abs + 2; ++s) R = fma(h->chi_s[s], tb.ray64[(int64_t)s * W + cc], R);

  const double* lw = reinterpret_cast<const double*>(slab + L.off_lw64);
  const int32_t* lid = reinterpret_cast<const int32_t*>(slab + L.off_lid);
  const KBlk* kblk = reinterpret_cast<const KBlk*>(slab + L.off_kblk);
  const MList* ml = reinterpret_cast<const MList*>(slab + L.off_mlist);
  const double* A = reinterpret_cast<const double*>(slab + L.off_A64);
  const double* dlT = reinterpret_cast<const double*>(slab + L.off_dl);
  const int NP = L.NP;
  double* rows = &s_rows[wave][0][0];
  double* crows = rows + kRowsAbs * 64;

  // whole-model staging when the distinct corners fit, else per layer block
  const bool mstage = ml->nU <= kRowsAbs && ml->nV <= kRowsCia;
  const int slot_off = mstage ? 2 : 4;
  if (mstage) stage64(m, ml->ids, ml->nU, ml->tids, has_cia ? ml->nV : 0, rows, crows, lane);

  double atm = 0.0;
  const int nrb = (N + 31) / 32, nkb = (N + 15) / 16;
  for (int rb = 0; rb < nrb; ++rb) {
    double tau[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) tau[j] = 0.0;
    for (int kb = 2 * rb; kb < nkb; ++kb) {
      if (!mstage) {
        const KBlk* kd = kblk + kb;
        __builtin_amdgcn_wave_barrier();
        stage64(m, kd->ids, kd->nU, kd->tids, has_cia ? kd->nV : 0, rows, crows, lane);
      }
      double kap[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int l = 16 * kb + j;
        double k = 0.0;
        if (l < N) {
          const uint32_t sl = (uint32_t)lid[8 * l + slot_off];
          const double* w = lw + 8 * l;
          k = w[0] * rows[(sl & 0xff) * 64 + lane];
          k = fma(w[1], rows[((sl >> 8) & 0xff) * 64 + lane], k);
          k = fma(w[2], rows[((sl >> 16) & 0xff) * 64 + lane], k);
          k = fma(w[3], rows[(sl >> 24) * 64 + lane], k);
          k = fma(w[4], R, k);
          if (has_cia) {
            const uint32_t cl = (uint32_t)lid[8 * l + slot_off + 1];
            k = fma(w[5], crows[(cl & 0xff) * 64 + lane], k);
            k = fma(w[6], crows[((cl >> 8) & 0xff) * 64 + lane], k);
          }
        }
        kap[j] = k;
      }
      // tau_j += dl[j, l] kappa_l for the 32 rays of this block (dl = 0 for l < j)
#pragma unroll
      for (int jl = 0; jl < 16; ++jl) {
        const double* d = dlT + (int64_t)(16 * kb + jl) * NP + 32 * rb;
#pragma unroll
        for (int j = 0; j < 32; ++j) tau[j] = fma(d[j], kap[jl], tau[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) atm = fma(A[32 * rb + j], -expm1(-tau[j]), atm);
  }
  if (valid) {
    const int64_t o = (int64_t)b * W + col;
    reinterpret_cast<double*>(a.aws)[o] = atm;
    if (a.depth_native) a.depth_native[o] = h->Rp2_Rs2 + atm;
    if (!isfinite(atm)) atomicOr(&a.model_status[b], TRX_MODEL_NONFINITE);
  }
}

}  // namespace

void launch_fwd64(const FwdArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return;
  const int spans = (a.tab.n_wn + kSpan - 1) / kSpan;
  hipLaunchKernelGGL(k_fwd64, dim3(B_grid, spans), dim3(64 * kWaves), 0, s, a);
}

}  // namespace trx
