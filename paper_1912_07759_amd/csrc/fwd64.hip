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

constexpr int kWaves = 4;
constexpr int kSpan = 64 * kWaves;

struct Mixer64 {
  const double* xs;   // xsec64 + col
  const double* ci;   // cia64 + col
  int64_t abs_stride; // n_T * n_P * n_wn
  int64_t cia_stride; // n_Tcia * n_wn
  int W, nP, nabs, ncia;
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

// Corner values of the current layer's bracket, reused when consecutive
// layers share corners (the bracket index is uniform across the wave).
struct Corners64 {
  int base = -1 << 30, cbase = -1 << 30;
  double c00 = 0, c10 = 0, c01 = 0, c11 = 0, C0 = 0, C1 = 0;

  __device__ void update(const Mixer64& m, int nb, int ncb) {
    const int nP = m.nP;
    if (nb != base) {
      if (nb == base - 1) {            // one pressure node down (moving up)
        c01 = c00; c11 = c10;
        c00 = m.corner(nb); c10 = m.corner(nb + nP);
      } else if (nb == base + 1) {
        c00 = c01; c10 = c11;
        c01 = m.corner(nb + 1); c11 = m.corner(nb + nP + 1);
      } else if (nb == base + nP) {    // one temperature node up
        c00 = c10; c01 = c11;
        c10 = m.corner(nb + nP); c11 = m.corner(nb + nP + 1);
      } else if (nb == base - nP) {
        c10 = c00; c11 = c01;
        c00 = m.corner(nb); c01 = m.corner(nb + 1);
      } else {
        c00 = m.corner(nb); c10 = m.corner(nb + nP);
        c01 = m.corner(nb + 1); c11 = m.corner(nb + nP + 1);
      }
      base = nb;
    }
    if (m.ncia > 0 && ncb != cbase) {
      if (ncb == cbase + 1) { C0 = C1; C1 = m.cia(ncb + 1); }
      else if (ncb == cbase - 1) { C1 = C0; C0 = m.cia(ncb); }
      else { C0 = m.cia(ncb); C1 = m.cia(ncb + 1); }
      cbase = ncb;
    }
  }
};

__global__ __launch_bounds__(64 * kWaves) void k_fwd64(FwdArgs a) {
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
  m.W = W; m.nP = tb.n_P; m.nabs = tb.n_abs; m.ncia = tb.n_cia;
  m.chi = h->chi_s;
  m.ciaw = h->cia_w;

  double R = 0.0;
  if (tb.has_rayleigh)
    for (int s = 0; s < tb.n_abs + 2; ++s) R = fma(h->chi_s[s], tb.ray64[(int64_t)s * W + cc], R);

  const double* lw = reinterpret_cast<const double*>(slab + L.off_lw64);
  const int32_t* lid = reinterpret_cast<const int32_t*>(slab + L.off_lid);
  const double* A = reinterpret_cast<const double*>(slab + L.off_A64);
  const double* dlT = reinterpret_cast<const double*>(slab + L.off_dl);
  const int NP = L.NP;

  double atm = 0.0;
  const int nrb = (N + 31) / 32;
  for (int rb = 0; rb < nrb; ++rb) {
    double tau[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) tau[j] = 0.0;
    Corners64 cs;
    for (int k = 32 * rb; k < N; ++k) {
      cs.update(m, lid[2 * k], lid[2 * k + 1]);
      const double* w = lw + 8 * k;
      double kap = w[0] * cs.c00;
      kap = fma(w[1], cs.c10, kap);
      kap = fma(w[2], cs.c01, kap);
      kap = fma(w[3], cs.c11, kap);
      kap = fma(w[4], R, kap);
      kap = fma(w[5], cs.C0, kap);
      kap = fma(w[6], cs.C1, kap);
      const double* d = dlT + (int64_t)k * NP + 32 * rb;
#pragma unroll
      for (int j = 0; j < 32; ++j) tau[j] = fma(d[j], kap, tau[j]);
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
  if (B_grid <= 0 || a.n_spans <= 0) return;
  hipLaunchKernelGGL(k_fwd64, dim3(B_grid, a.n_spans), dim3(64 * kWaves), 0, s, a);
}

}  // namespace trx
