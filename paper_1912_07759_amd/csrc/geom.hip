// Geometry kernel (FP64): steps a1-a3 of the forward model for one model
// per workgroup, plus the per-layer interpolation records used by the
// opacity step (a4).
//
//  a1  Pressure Profiles subsection: N+1 log-spaced boundary pressures,
//      centres P_l = p_l sqrt(p_{l+1}/p_l).  Chemistry subsection: constant
//      absorbers, H2/He fill sharing the rest of the volume with He/H2 = r,
//      mean molecular weight over all species.  Number density P/(k_B T).
//  a2  Forward Models section, altitude equation: z_0 = 0,
//      z_l = z_{l-1} - H_{l-1} ln(P_l/P_{l-1}), H = k_B T / (mu g),
//      g = GM/(Rp + z)^2 (or GM/Rp^2); one lane runs the recurrence.
//  a3  Chord lengths of the ray at z_j through the shell between
//      h_k = (z_{k-1}+z_k)/2 and h_{k+1} (h_0 = 0, h_N = z_{N-1}), written
//      in the cancellation-free form
//        dl[j,j] = 2 q_j(h_{j+1}),
//        dl[j,k] = 2 (h_{k+1}-h_k)(2Rp+h_k+h_{k+1}) / (q_j(h_{k+1}) + q_j(h_k)),
//      q_j(h) = sqrt((h - z_j)(2Rp + h + z_j)); annulus weights
//      A_j = 2 (Rp + z_j)(h_{j+1} - h_j), stored divided by Rs^2.
//  a4  records: per layer the four bilinear corner weights on (T, log10 P)
//      times 1e-4 rho (cm^2 -> m^2), the Rayleigh weight 1e-4 rho, the two
//      CIA weights in T times 1e-10 rho^2 (cm^5 -> m^5), and the corner
//      indices.  Out-of-range T and log10 P clamp to the grid; T and P both
//      below the grid give zero cross-section (Opacities section).
//      The model's opacity slots: its distinct corners (ordered by pressure
//      node, then temperature node) and its distinct CIA temperature nodes.
//      Exponential temperature scheme: the layers are the absorber slots
//      (top layer first), each with weight 1e-4 rho, and each slot keeps
//      its layer's {u, w_P, w_T} with u = (1/T - 1/T1)/(1/T2 - 1/T1) =
//      w_T T2/T.
//
// The matrix-core modes then take, per model, the products of the chord
// lengths and the opacity weights (k_pmat below).
#include "trx_internal.h"

namespace trx {

namespace {

constexpr int kThreads = 256;

__device__ inline bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

// Lower-closed bracket with edge clamping: grid[i] <= x < grid[i+1];
// below the grid: i = 0, w = 0; at or above the top: i = n-2, w = 1.
__device__ inline void bracket(const double* g, int n, double x, int& i, double& w,
                               bool& below, bool& clamped) {
  below = false;
  clamped = false;
  if (x < g[0]) { i = 0; w = 0.0; below = true; clamped = true; return; }
  if (x >= g[n - 1]) { i = n - 2; w = 1.0; clamped = true; return; }
  int lo = 0, hi = n - 1;  // g[lo] <= x < g[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (g[mid] <= x) lo = mid; else hi = mid;
  }
  i = lo;
  w = (x - g[lo]) / (g[lo + 1] - g[lo]);
}

// Round a float to bf16 (nearest even) and return the bf16 bits.  Finite
// inputs only (the path lengths are finite and non-negative).
__device__ inline uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_to_double(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}

__global__ __launch_bounds__(kThreads) void k_geom(GeomArgs a) {
  const int b = blockIdx.x;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const Layout& L = a.L;
  const DevTables& tb = a.tab;
  uint8_t* slab = a.ws + (int64_t)b * L.slab;
  ModelHdr* h = reinterpret_cast<ModelHdr*>(slab);
  double* zs = reinterpret_cast<double*>(slab + L.off_z);
  double* A64 = reinterpret_cast<double*>(slab + L.off_A64);
  float* A32 = reinterpret_cast<float*>(slab + L.off_A32);
  double* lw64 = reinterpret_cast<double*>(slab + L.off_lw64);
  float* lw32 = reinterpret_cast<float*>(slab + L.off_lw32);
  int32_t* lid = reinterpret_cast<int32_t*>(slab + L.off_lid);

  __shared__ double sP[TRX_MAX_LAYERS_FP64];
  __shared__ double sZ[TRX_MAX_LAYERS_FP64];
  __shared__ double sC[TRX_MAX_LAYERS_FP64];   // kB T_l * ln(P_{l+1}/P_l), later the deck's terms
  __shared__ int s_status;
  __shared__ double s_mu[kMaxRegimes];
  __shared__ int s_cut[kMaxRegimes + 1];   // first layer of each run
  __shared__ int s_lsw[TRX_MAX_ABSORBERS];  // first layer where each absorber takes its top value
  __shared__ int s_nreg;

  const int tid = threadIdx.x;
  const int N = a.bt.n_layers[b];
  const int lo = a.bt.wn_lo[b], hi = a.bt.wn_hi[b];
  const int64_t off = a.bt.layer_off[b];
  const double Rp = a.bt.Rp[b], Rs = a.bt.Rs[b], GM = a.bt.GM[b];
  const double pb = a.bt.p_bot[b], pt = a.bt.p_top[b];
  const int nabs = tb.n_abs;

  if (tid == 0) {
    int st = 0;
    if (N < 2 || N > a.n_limit) st |= TRX_MODEL_BAD_PROFILE;
    if (!finite_pos(Rp) || !finite_pos(Rs) || !finite_pos(GM)) st |= TRX_MODEL_BAD_PROFILE;
    if (!finite_pos(pb) || !finite_pos(pt) || !(pb > pt)) st |= TRX_MODEL_BAD_PROFILE;
    if (!(lo >= 0 && hi <= tb.n_wn && hi > lo)) st |= TRX_MODEL_BAD_WINDOW;
    double S = 0.0;
    bool fin = true;
    for (int i = 0; i < nabs; ++i) {
      double x = a.bt.log10_vmr[(int64_t)b * nabs + i];
      fin = fin && isfinite(x);
      S += pow(10.0, x);
      if (a.bt.vmr_top) {
        fin = fin && isfinite(a.bt.vmr_top[(int64_t)b * nabs + i]);
        fin = fin && finite_pos(a.bt.vmr_sw[(int64_t)b * nabs + i]);
      }
    }
    // two-layer models: each run's sum is checked once the runs are known
    if (!fin || (!a.bt.vmr_top && !(S < 1.0))) st |= TRX_MODEL_BAD_CHEMISTRY;
    if (a.bt.cloud_sigma) {
      const double sg = a.bt.cloud_sigma[b];
      if (!(sg >= 0.0)) st |= TRX_MODEL_BAD_PROFILE;
      if (sg > 0.0 && !(finite_pos(a.bt.cloud_p1[b]) && finite_pos(a.bt.cloud_p2[b]))) st |= TRX_MODEL_BAD_PROFILE;
    }
    if (L.em && !finite_pos(a.T_star[b])) st |= TRX_MODEL_BAD_PROFILE;
    s_status = st;
  }
  __syncthreads();
  if ((s_status & TRX_MODEL_BAD_PROFILE) == 0) {
    for (int l = tid; l < N; l += kThreads) {
      double T = a.bt.T[off + l];
      if (!finite_pos(T)) atomicOr(&s_status, TRX_MODEL_BAD_PROFILE);
    }
  }
  __syncthreads();
  // an invalid model: status, no layers, NaN in its window
  auto reject = [&](int status) {
    if (tid == 0) {
      h->n = 0; h->status = status; h->lo = lo; h->hi = hi;
      h->nrb = 0; h->nkb = 0; h->span_lo = 0; h->span_hi = 0;
      h->cloud = 0;
      h->nreg = 0;
      if (a.mlay) a.mlay[b] = 0;
      if (a.mspan) a.mspan[b] = make_int2(0, 0);
    }
    if (a.depth_native && (status & TRX_MODEL_BAD_WINDOW) == 0) {
      for (int i = lo + tid; i < hi; i += kThreads)
        a.depth_native[(int64_t)b * tb.n_wn + i] = __builtin_nan("");
    }
  };
  if (s_status) {
    reject(s_status);
    return;
  }

  // a1: pressure grid (boundaries log-spaced, geometric centres)
  const double xb = log10(pb), xt = log10(pt);
  for (int l = tid; l < N; l += kThreads) {
    double p0 = pow(10.0, xb + (xt - xb) * (double)l / (double)N);
    double p1 = pow(10.0, xb + (xt - xb) * (double)(l + 1) / (double)N);
    sP[l] = p0 * sqrt(p1 / p0);
  }
  __syncthreads();
  // a1: chemistry.  Constant profiles: one run.  Two-layer profiles
  // (Chemistry subsection): absorber i takes its top value from the first
  // layer whose centre pressure is below its switch pressure, l_i; the
  // distinct l_i inside the model cut its layers into runs of one
  // chemistry (run r: layers from the r-th cut on), each with its own fill
  // gases and mean molecular weight.
  RegChem* rgc = L.rg ? reinterpret_cast<RegChem*>(slab + L.off_rg) : nullptr;
  // the switch layer of each absorber (N: surface value everywhere)
  for (int i = tid; i < nabs; i += kThreads) {
    int l = N;
    if (a.bt.vmr_top) {
      const double sw = a.bt.vmr_sw[(int64_t)b * nabs + i];
      l = 0;
      while (l < N && sP[l] >= sw) ++l;
    }
    s_lsw[i] = l;
  }
  __syncthreads();
  if (tid == 0) {
    int R = 1;
    s_cut[0] = 0;
    for (int i = 0; i < nabs; ++i) {
      const int l = s_lsw[i];
      if (l <= 0 || l >= N) continue;
      bool seen = false;
      for (int r = 1; r < R; ++r) seen = seen || s_cut[r] == l;
      if (seen) continue;
      if (R == kMaxRegimes) {
        R = kMaxRegimes + 1;   // too many runs
        break;
      }
      // insertion keeps the cuts ascending
      int r = R++;
      while (r > 1 && s_cut[r - 1] > l) { s_cut[r] = s_cut[r - 1]; --r; }
      s_cut[r] = l;
    }
    int st = 0;
    if (R > kMaxRegimes) st |= TRX_MODEL_UNSUPPORTED;
    for (int r = 0; r < R && !st; ++r) {
      const int lr = s_cut[r];   // first layer of run r
      double chi[kMaxSpecies];
      double S = 0.0, mu = 0.0;
      for (int i = 0; i < nabs; ++i) {
        const bool top = lr >= s_lsw[i];
        const double x = top ? a.bt.vmr_top[(int64_t)b * nabs + i] : a.bt.log10_vmr[(int64_t)b * nabs + i];
        chi[i] = pow(10.0, x);
        S += chi[i];
        mu += chi[i] * tb.mass[i];
      }
      if (!(S < 1.0)) {
        st |= TRX_MODEL_BAD_CHEMISTRY;
        break;
      }
      const double rr = a.bt.he_h2;
      chi[nabs] = (1.0 - S) / (1.0 + rr);
      chi[nabs + 1] = rr * chi[nabs];
      mu += chi[nabs] * tb.mass[nabs] + chi[nabs + 1] * tb.mass[nabs + 1];
      s_mu[r] = mu * a.bt.amu;
      double cw[TRX_MAX_CIA];
      for (int p = 0; p < TRX_MAX_CIA; ++p)
        cw[p] = p < tb.n_cia ? chi[tb.cia_pair[p][0]] * chi[tb.cia_pair[p][1]] : 0.0;
      if (rgc) {
        for (int k = 0; k < kMaxSpecies; ++k) {
          const double v = k < nabs + 2 ? chi[k] : 0.0;
          rgc[r].chi_s[k] = v;
          rgc[r].chi_s32[k] = (float)v;
        }
        for (int p = 0; p < TRX_MAX_CIA; ++p) {
          rgc[r].cia_w[p] = cw[p];
          rgc[r].cia_w32[p] = (float)cw[p];
        }
      }
      if (r == 0) {
        for (int i = 0; i < TRX_MAX_ABSORBERS; ++i) h->chi_abs32[i] = i < nabs ? (float)chi[i] : 0.0f;
        for (int k = 0; k < nabs + 2; ++k) {
          h->chi_s[k] = chi[k];
          h->chi_s32[k] = (float)chi[k];
        }
        for (int p = 0; p < TRX_MAX_CIA; ++p) {
          h->cia_w[p] = cw[p];
          h->cia_w32[p] = (float)cw[p];
        }
      }
    }
    s_nreg = R;
    s_status = st;
  }
  __syncthreads();
  if (s_status) {
    reject(s_status);
    return;
  }
  const int R = s_nreg;
  // run of layer l
  auto run_of = [&](int l) {
    int r = 0;
    for (int k = 1; k < R; ++k) r += l >= s_cut[k];
    return r;
  };
  for (int l = tid; l < N - 1; l += kThreads)
    sC[l] = a.bt.kB * a.bt.T[off + l] * log(sP[l + 1] / sP[l]) / s_mu[run_of(l)];
  __syncthreads();
  // a2: altitude recurrence, one lane
  if (tid == 0) {
    double z = 0.0;
    sZ[0] = 0.0;
    if (a.bt.gravity == 0) {
      const double invGM = 1.0 / GM;
      for (int l = 1; l < N; ++l) {
        const double rz = Rp + z;
        z = z - sC[l - 1] * rz * rz * invGM;   // H = kB T (Rp+z)^2 / (mu GM)
        sZ[l] = z;
      }
    } else {
      const double f = Rp * Rp / GM;
      for (int l = 1; l < N; ++l) {
        z = z - sC[l - 1] * f;
        sZ[l] = z;
      }
    }
    const int sc = a.span_cols;
    h->n = N; h->status = 0; h->lo = lo; h->hi = hi;
    h->nrb = (N + 31) / 32; h->nkb = (N + 15) / 16;
    h->span_lo = lo / sc; h->span_hi = (hi + sc - 1) / sc;
    if (a.mlay) a.mlay[b] = N;
    if (a.mspan) a.mspan[b] = make_int2(lo / kSpanCols, (hi + kSpanCols - 1) / kSpanCols);
    h->Rp2_Rs2 = (Rp / Rs) * (Rp / Rs);
    for (int r = 0; r < TRX_MAX_LAYERS_MFMA / 32; ++r) h->kq_mask[r] = 0ull;   // set by the path-matrix kernel
    h->inv_Rs2 = 1.0 / (Rs * Rs);
    h->Rp = Rp;
    h->mu_kg = s_mu[0];
    h->nreg = R;
  }
  __syncthreads();
  const double inv_Rs2 = 1.0 / (Rs * Rs);

  // a3: chord length of ray j through layer k
  auto dl_of = [&](int j, int k) -> double {
    if (j >= N || k >= N || k < j) return 0.0;
    const double zj = sZ[j];
    const double hk = (k == 0) ? 0.0 : 0.5 * (sZ[k - 1] + sZ[k]);
    const double hk1 = (k == N - 1) ? sZ[N - 1] : 0.5 * (sZ[k] + sZ[k + 1]);
    const double q1 = sqrt(fmax((hk1 - zj) * (2.0 * Rp + hk1 + zj), 0.0));
    if (k == j) return 2.0 * q1;
    const double q0 = sqrt((hk - zj) * (2.0 * Rp + hk + zj));
    return 2.0 * (hk1 - hk) * (2.0 * Rp + hk + hk1) / (q1 + q0);
  };
  // cloud deck (equation clouds): sigma rho on the layers whose centre
  // pressure lies in [min(p1, p2), max(p1, p2)], at every wavenumber.  Its
  // optical depth along ray j, tc_j = sum_k dl[j][k] sigma rho_k, does not
  // depend on the wavenumber, so A_j (1 - e^{-tau_j - tc_j}) = A_j (1 -
  // e^{-tc_j}) + A_j e^{-tc_j} (1 - e^{-tau_j}): the first term joins the
  // model's constant (Rp/Rs)^2 and the ray carries A_j e^{-tc_j} as its
  // annulus weight, so that every forward kernel runs unchanged.  An opaque
  // deck (sigma = +inf) has tc_j = +inf on the rays with a nonzero path
  // through it, 0 on the others.
  const double csig = a.bt.cloud_sigma ? a.bt.cloud_sigma[b] : 0.0;
  const double cp_lo = csig > 0.0 ? fmin(a.bt.cloud_p1[b], a.bt.cloud_p2[b]) : 0.0;
  const double cp_hi = csig > 0.0 ? fmax(a.bt.cloud_p1[b], a.bt.cloud_p2[b]) : -1.0;
  const bool copaque = isinf(csig);
  auto in_deck = [&](int k) { return sP[k] >= cp_lo && sP[k] <= cp_hi; };
  double* pc64 = reinterpret_cast<double*>(slab + L.off_pc64);
  // emission: shell thickness and the per-layer records of the Planck terms
  auto shell_dz = [&](int k) -> double {
    const double h0 = (k == 0) ? 0.0 : 0.5 * (sZ[k - 1] + sZ[k]);
    const double h1 = (k == N - 1) ? sZ[N - 1] : 0.5 * (sZ[k] + sZ[k + 1]);
    return h1 - h0;
  };
  const double Tstar = L.em ? a.T_star[b] : 1.0;

  // exponential scheme: each layer is an absorber slot, the top run's
  // layers first, each run top layer first and padded to a multiple of 8
  // slots in two-layer layouts (constant profiles: slot N-1-l); the
  // records are kept by slot, zero for the padding slots
  __shared__ int s_xb[kMaxRegimes];
  if (L.xt) {
    if (tid == 0) {
      int base = 0;
      for (int r = R - 1; r >= 0; --r) {
        s_xb[r] = base;
        const int n = (r == R - 1 ? N : s_cut[r + 1]) - s_cut[r];
        base += L.rg ? (n + 7) / 8 * 8 : n;
      }
    }
    const int nslot = L.rg ? 16 * L.NKQ : L.NP;
    for (int q = tid; q < nslot; q += kThreads) {
      reinterpret_cast<double4*>(slab + L.off_xt64)[q] = make_double4(0.0, 0.0, 0.0, 0.0);
      reinterpret_cast<float4*>(slab + L.off_xt32)[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
  }
  auto xt_slot = [&](int l) {
    const int r = run_of(l);
    const int last = (r == R - 1 ? N : s_cut[r + 1]) - 1;
    return s_xb[r] + (last - l);
  };

  // a3: annulus weights; a4: layer records
  const int NP = L.NP;
  for (int l = tid; l < NP; l += kThreads) {
    if (l < N) {
      const double z = sZ[l];
      const double hl = (l == 0) ? 0.0 : 0.5 * (sZ[l - 1] + z);
      const double hu = (l == N - 1) ? z : 0.5 * (z + sZ[l + 1]);
      const double A0 = 2.0 * (Rp + z) * (hu - hl) * inv_Rs2;
      // the deck's optical depth along ray j = l (emission: vertically,
      // from the top down to the bottom of shell l)
      double tc = 0.0;
      for (int k = l; k < N && csig > 0.0; ++k) {
        if (!in_deck(k)) continue;
        const double d = L.em ? shell_dz(k) : dl_of(l, k);
        if (copaque) {
          if (d > 0.0) {   // one path through an opaque deck blocks the ray
            tc = __builtin_inf();
            break;
          }
        } else {
          tc += d * (csig * sP[k] / (a.bt.kB * a.bt.T[off + k]));
        }
      }
      // transmission folds the deck into the annulus weights and the
      // constant term; emission keeps it per layer in its records
      const double A = L.em ? A0 : A0 * exp(-tc);
      sC[l] = L.em ? 0.0 : -A0 * expm1(-tc);   // this ray's share of the deck's constant term
      pc64[l] = tc;
      if (L.em) {
        const double Tl = a.bt.T[off + l];
        const double Tm = l > 0 ? a.bt.T[off + l - 1] : Tl;
        const double e0 = a.c2 / Tl;
        const double e1 = l > 0 ? a.c2 * ((Tm - Tl) / (Tl * Tm)) : 0.0;
        const double e2 = a.c2 * ((Tstar - Tl) / (Tl * Tstar));
        reinterpret_cast<double4*>(slab + L.off_em64)[l] = make_double4(e0, e1, e2, tc);
        reinterpret_cast<float4*>(slab + L.off_em32)[l] = make_float4((float)e0, (float)e1, (float)e2, (float)tc);
      }
      zs[l] = z;
      A64[l] = A;
      A32[l] = (float)A;
      const double T = a.bt.T[off + l];
      const double P = sP[l];
      const double n = P / (a.bt.kB * T);
      int iT, iP, iC;
      double wT, wP, wC;
      bool Tb, Pb, c0, c1, c2 = false;
      bracket(tb.T, tb.n_T, T, iT, wT, Tb, c0);
      bracket(tb.logP, tb.n_P, log10(P), iP, wP, Pb, c1);
      const bool Tb_abs = Tb;
      const double f1 = 1e-4 * n;
      double w[8];
      if (Tb && Pb) {
        w[0] = w[1] = w[2] = w[3] = 0.0;
      } else if (L.xt) {
        // exponential scheme: the layer is its own slot with weight 1e-4 rho
        w[0] = f1;
        w[1] = w[2] = w[3] = 0.0;
      } else {
        w[0] = f1 * (1.0 - wT) * (1.0 - wP);
        w[1] = f1 * wT * (1.0 - wP);
        w[2] = f1 * (1.0 - wT) * wP;
        w[3] = f1 * wT * wP;
      }
      if (L.xt) {
        // sigma1 (sigma2/sigma1)^u, u = (1/T - 1/T1)/(1/T2 - 1/T1) = w_T T2/T
        // (0 and 1 under the clamps, where T is taken at the edge node)
        const double u = c0 ? wT : wT * (tb.T[iT + 1] / T);
        const int q = xt_slot(l);
        reinterpret_cast<double4*>(slab + L.off_xt64)[q] = make_double4(u, wP, wT, 0.0);
        reinterpret_cast<float4*>(slab + L.off_xt32)[q] = make_float4((float)u, (float)wP, (float)wT, 0.f);
      }
      w[4] = tb.has_rayleigh ? f1 : 0.0;
      if (tb.n_cia > 0) {
        bracket(tb.Tcia, tb.n_Tcia, T, iC, wC, Tb, c2);
        const double f2 = 1e-10 * n * n;
        w[5] = f2 * (1.0 - wC);
        w[6] = f2 * wC;
      } else {
        iC = 0;
        w[5] = w[6] = 0.0;
      }
      // the deck's weight sigma rho of this layer (the gradient's chord and
      // temperature terms; zero outside the deck and for an opaque deck)
      const bool cl = csig > 0.0 && !copaque && in_deck(l);
      w[7] = cl ? csig * n : 0.0;
      for (int q = 0; q < 8; ++q) {
        lw64[8 * l + q] = w[q];
        lw32[8 * l + q] = (float)(q >= 5 ? w[q] / kCiaScale32 : w[q]);
      }
      lw32[8 * l + 7] = (float)A;   // FP32 records carry the ray's annulus weight
      // ray weights of the slot form; the path-matrix kernel adds PR_j
      if (L.off_aw) reinterpret_cast<float2*>(slab + L.off_aw)[l] = make_float2((float)A, 0.f);
      if (L.off_pr64) reinterpret_cast<double*>(slab + L.off_pr64)[l] = 0.0;
      if (L.grad) {
        // d(weight)/dT at fixed P: the bracket slope in T (zero where T is
        // clamped: one-sided at nodes, Opacities section rules) and the
        // number-density factor, d rho/dT = -rho/T (rho^2 for CIA)
        double* lwd = reinterpret_cast<double*>(slab + L.off_lwd64) + 8 * l;
        const double dwT = c0 ? 0.0 : 1.0 / (tb.T[iT + 1] - tb.T[iT]);
        double d[8];
        if (Tb_abs && Pb) {
          d[0] = d[1] = d[2] = d[3] = 0.0;
        } else {
          d[0] = -f1 * dwT * (1.0 - wP) - w[0] / T;
          d[1] = f1 * dwT * (1.0 - wP) - w[1] / T;
          d[2] = -f1 * dwT * wP - w[2] / T;
          d[3] = f1 * dwT * wP - w[3] / T;
        }
        d[4] = -w[4] / T;
        if (tb.n_cia > 0) {
          const double dwC = c2 ? 0.0 : 1.0 / (tb.Tcia[iC + 1] - tb.Tcia[iC]);
          const double f2 = 1e-10 * n * n;
          d[5] = -f2 * dwC - 2.0 * w[5] / T;
          d[6] = f2 * dwC - 2.0 * w[6] / T;
        } else {
          d[5] = d[6] = 0.0;
        }
        d[7] = -w[7] / T;
        for (int q = 0; q < 8; ++q) lwd[q] = q >= 5 && q < 7 ? d[q] / kCiaScale32 : d[q];
      }
      lid[8 * l] = iT * tb.n_P + iP;
      lid[8 * l + 1] = iC;
    } else {
      zs[l] = 0.0;
      A64[l] = 0.0;
      A32[l] = 0.0f;
      pc64[l] = 0.0;
      if (L.em) {
        reinterpret_cast<double4*>(slab + L.off_em64)[l] = make_double4(0.0, 0.0, 0.0, 0.0);
        reinterpret_cast<float4*>(slab + L.off_em32)[l] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      if (L.off_aw) reinterpret_cast<float2*>(slab + L.off_aw)[l] = make_float2(0.f, 0.f);
      if (L.off_pr64) reinterpret_cast<double*>(slab + L.off_pr64)[l] = 0.0;
      for (int q = 0; q < 8; ++q) { lw64[8 * l + q] = 0.0; lw32[8 * l + q] = 0.0f; }
      if (L.grad)
        for (int q = 0; q < 8; ++q) reinterpret_cast<double*>(slab + L.off_lwd64)[8 * l + q] = 0.0;
      for (int q = 0; q < 8; ++q) lid[8 * l + q] = 0;   // padding layer: zero weights
    }
  }
  __syncthreads();
  if (tid == 0) {
    // the deck's constant term, summed in layer order
    double s = 0.0;
    for (int l = 0; l < N && csig > 0.0; ++l) s += sC[l];
    h->Rp2_Rs2 = (Rp / Rs) * (Rp / Rs) + s;
    h->cloud = csig > 0.0 ? 1 : 0;
    h->em_scale = (Rp / Rs) * (Rp / Rs);
    h->em_star = a.c2 / Tstar;
    if (L.em) {
      // the emission output has no additive constant (its records carry
      // the deck)
      h->Rp2_Rs2 = 0.0;
      h->cloud = 0;
    }
  }

  // distinct corners of the whole model (bitmaps over the keys
  // iP n_T + iT, slots = rank of the key among the set bits, so that the
  // slots follow the pressure nodes and a run of slots is used by a run of
  // layers) and each layer's slots in them; in the exponential scheme the
  // absorber slots are the layers, top first (slot q: layer N-1-q, its row
  // id the corner (iT, iP) it interpolates from), so that a ray's optical
  // depth is accumulated from its smallest terms up, as the corner slots
  // are (rising pressure nodes)
  __shared__ int s_nu;
  __shared__ uint32_t s_bm[TRX_MAX_TGRID * TRX_MAX_PGRID / 32];
  __shared__ uint32_t s_pre[TRX_MAX_TGRID * TRX_MAX_PGRID / 32];
  __shared__ uint32_t s_cbm[TRX_MAX_TGRID / 32];
  __shared__ uint32_t s_cpre[TRX_MAX_TGRID / 32];
  if (!L.rg) {
    const bool xt = L.xt != 0;
    const int nwords = (tb.n_T * tb.n_P + 31) / 32;
    const int ncwords = (tb.n_Tcia + 31) / 32;
    for (int w = tid; w < nwords; w += kThreads) s_bm[w] = 0u;
    for (int w = tid; w < ncwords; w += kThreads) s_cbm[w] = 0u;
    __syncthreads();
    const int nT = tb.n_T, nP = tb.n_P;
    // keys of the corners (iT, iP), (iT+1, iP), (iT, iP+1), (iT+1, iP+1)
    auto corner_keys = [&](int base, int* ks) {
      const int k0 = (base % nP) * nT + base / nP;
      ks[0] = k0;
      ks[1] = k0 + 1;
      ks[2] = k0 + nT;
      ks[3] = k0 + nT + 1;
    };
    for (int l = tid; l < N; l += kThreads) {
      int cs[4];
      corner_keys(lid[8 * l], cs);
      for (int q = 0; q < 4 && !xt; ++q) atomicOr(&s_bm[cs[q] >> 5], 1u << (cs[q] & 31));
      if (tb.n_cia > 0) {
        const int t0 = lid[8 * l + 1];
        atomicOr(&s_cbm[t0 >> 5], 1u << (t0 & 31));
        atomicOr(&s_cbm[(t0 + 1) >> 5], 1u << ((t0 + 1) & 31));
      }
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t acc = 0;
      for (int w = 0; w < nwords; ++w) { s_pre[w] = acc; acc += __popc(s_bm[w]); }
      uint32_t cacc = 0;
      for (int w = 0; w < ncwords; ++w) { s_cpre[w] = cacc; cacc += __popc(s_cbm[w]); }
      MList* ml = reinterpret_cast<MList*>(slab + L.off_mlist);
      ml->nU = xt ? N : (int)acc;
      ml->nV = tb.n_cia > 0 ? (int)cacc : 0;
      s_nu = xt ? N : (int)acc;
    }
    __syncthreads();
    MList* ml = reinterpret_cast<MList*>(slab + L.off_mlist);
    // the slot lists: the first kMListU / kMListV in the model list, all of
    // them (table rows, corners then CIA nodes) in the slot table of the
    // matrix-core modes
    int32_t* sid = L.off_sid ? reinterpret_cast<int32_t*>(slab + L.off_sid) : nullptr;
    const int nu = s_nu;
    for (int q = tid; q < (xt ? N : 0); q += kThreads) {
      if (q < kMListU) ml->ids[q] = lid[8 * (N - 1 - q)];
      if (sid) sid[q] = lid[8 * (N - 1 - q)];
    }
    for (int w = tid; w < (xt ? 0 : nwords); w += kThreads) {
      uint32_t bits = s_bm[w];
      int slot = (int)s_pre[w];
      while (bits) {
        const int key = 32 * w + __ffs(bits) - 1;
        const int id = (key % nT) * nP + key / nT;
        if (slot < kMListU) ml->ids[slot] = id;
        if (sid) sid[slot] = id;
        ++slot;
        bits &= bits - 1;
      }
    }
    if (tb.n_cia > 0) {
      for (int w = tid; w < ncwords; w += kThreads) {
        uint32_t bits = s_cbm[w];
        int slot = (int)s_cpre[w];
        while (bits) {
          const int t = 32 * w + __ffs(bits) - 1;
          if (slot < kMListV) ml->tids[slot] = t;
          if (sid) sid[nu + slot] = t;
          ++slot;
          bits &= bits - 1;
        }
      }
    }
    auto rank_full = [&](const uint32_t* bm, const uint32_t* pre, int c) -> uint32_t {
      const uint32_t below = bm[c >> 5] & ((1u << (c & 31)) - 1u);
      return pre[c >> 5] + __popc(below);
    };
    auto rank = [&](const uint32_t* bm, const uint32_t* pre, int c) -> uint32_t {
      const uint32_t r = rank_full(bm, pre, c);
      return r > 255u ? 255u : r;
    };
    for (int l = tid; l < N; l += kThreads) {
      int cs[4];
      corner_keys(lid[8 * l], cs);
      uint32_t slots = 0;
      for (int q = 0; q < 4 && !xt; ++q) slots |= rank(s_bm, s_pre, cs[q]) << (8 * q);
      lid[8 * l + 2] = (int32_t)slots;
      // unclamped 16-bit slots of the four corners (the exponential scheme:
      // the layer's own slot, the other three weights being zero)
      if (xt) {
        const int q = N - 1 - l;
        lid[8 * l + 6] = (int32_t)(q | (q << 16));
        lid[8 * l + 7] = (int32_t)(q | (q << 16));
      } else {
        lid[8 * l + 6] = (int32_t)(rank_full(s_bm, s_pre, cs[0]) | (rank_full(s_bm, s_pre, cs[1]) << 16));
        lid[8 * l + 7] = (int32_t)(rank_full(s_bm, s_pre, cs[2]) | (rank_full(s_bm, s_pre, cs[3]) << 16));
      }
      uint32_t cslots = 0;
      if (tb.n_cia > 0) {
        const int t0 = lid[8 * l + 1];
        cslots = rank(s_cbm, s_cpre, t0) | (rank(s_cbm, s_cpre, t0 + 1) << 8);
      }
      lid[8 * l + 3] = (int32_t)cslots;
    }
  } else {
    // two-layer layouts: the same per run, top run first, each run's
    // corner slots and node slots padded to a multiple of 8 (padding slots
    // point at row 0 and have no weight); then one Rayleigh slot per run.
    // The slot table holds row | run << 24; per layer, lid[2] = its run,
    // lid[3] = its two node slots (16 bits each, counted from the first
    // node slot), lid[6], lid[7] = its four corner slots.
    const bool xt = L.xt != 0;
    const int nT = tb.n_T, nP = tb.n_P;
    const int nwords = (nT * nP + 31) / 32;
    const int ncwords = (tb.n_Tcia + 31) / 32;
    const int cap = 16 * L.NKQ;
    int32_t* sid = reinterpret_cast<int32_t*>(slab + L.off_sid);
    __shared__ int s_cu[kMaxRegimes], s_cv[kMaxRegimes], s_ub[kMaxRegimes], s_vb[kMaxRegimes];
    __shared__ int s_tot[3];   // corner, node and Rayleigh slots (padded)
    auto corner_keys = [&](int base, int* ks) {
      const int k0 = (base % nP) * nT + base / nP;
      ks[0] = k0;
      ks[1] = k0 + 1;
      ks[2] = k0 + nT;
      ks[3] = k0 + nT + 1;
    };
    // the bitmaps of run r: its layers' corners and CIA nodes
    auto mark_run = [&](int r) {
      for (int w = tid; w < nwords; w += kThreads) s_bm[w] = 0u;
      for (int w = tid; w < ncwords; w += kThreads) s_cbm[w] = 0u;
      __syncthreads();
      const int la = s_cut[r], lb = r == R - 1 ? N : s_cut[r + 1];
      for (int l = la + tid; l < lb; l += kThreads) {
        int cs[4];
        corner_keys(lid[8 * l], cs);
        for (int q = 0; q < 4 && !xt; ++q) atomicOr(&s_bm[cs[q] >> 5], 1u << (cs[q] & 31));
        if (tb.n_cia > 0) {
          const int t0 = lid[8 * l + 1];
          atomicOr(&s_cbm[t0 >> 5], 1u << (t0 & 31));
          atomicOr(&s_cbm[(t0 + 1) >> 5], 1u << ((t0 + 1) & 31));
        }
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < nwords; ++w) { s_pre[w] = acc; acc += __popc(s_bm[w]); }
        uint32_t cacc = 0;
        for (int w = 0; w < ncwords; ++w) { s_cpre[w] = cacc; cacc += __popc(s_cbm[w]); }
        s_cu[r] = xt ? lb - la : (int)acc;
        s_cv[r] = tb.n_cia > 0 ? (int)cacc : 0;
      }
      __syncthreads();
    };
    // pass 1: the slot counts of every run, then the bases
    for (int r = R - 1; r >= 0; --r) mark_run(r);
    if (tid == 0) {
      int u = 0, v = 0;
      for (int r = R - 1; r >= 0; --r) {
        s_ub[r] = u;
        s_vb[r] = v;
        u += (s_cu[r] + 7) / 8 * 8;
        v += (s_cv[r] + 7) / 8 * 8;
      }
      s_tot[0] = u;
      s_tot[1] = v;
      s_tot[2] = tb.has_rayleigh ? (R + 7) / 8 * 8 : 0;
      if (u + v + s_tot[2] > cap) s_status = TRX_MODEL_UNSUPPORTED;
      MList* ml = reinterpret_cast<MList*>(slab + L.off_mlist);
      ml->nU = u;
      ml->nV = v;
      ml->pad[0] = s_tot[2];
      ml->pad[1] = R;
    }
    __syncthreads();
    if (s_status) {
      reject(s_status);
      return;
    }
    const int nU = s_tot[0], nV = s_tot[1];
    auto rank_of = [&](const uint32_t* bm, const uint32_t* pre, int c) -> int {
      return (int)(pre[c >> 5] + __popc(bm[c >> 5] & ((1u << (c & 31)) - 1u)));
    };
    // pass 2: each run's slots
    for (int r = R - 1; r >= 0; --r) {
      mark_run(r);
      const int la = s_cut[r], lb = r == R - 1 ? N : s_cut[r + 1];
      const int ub = s_ub[r], vb = s_vb[r];
      const uint32_t tag = (uint32_t)r << 24;
      if (xt) {
        for (int l = la + tid; l < lb; l += kThreads) sid[ub + (lb - 1 - l)] = (int32_t)(lid[8 * l] | tag);
      } else {
        for (int w = tid; w < nwords; w += kThreads) {
          uint32_t bits = s_bm[w];
          int slot = ub + (int)s_pre[w];
          while (bits) {
            const int key = 32 * w + __ffs(bits) - 1;
            sid[slot++] = (int32_t)(((key % nT) * nP + key / nT) | tag);
            bits &= bits - 1;
          }
        }
      }
      for (int q = ub + s_cu[r] + tid; q < ub + (s_cu[r] + 7) / 8 * 8; q += kThreads) sid[q] = (int32_t)tag;
      if (tb.n_cia > 0) {
        for (int w = tid; w < ncwords; w += kThreads) {
          uint32_t bits = s_cbm[w];
          int slot = nU + vb + (int)s_cpre[w];
          while (bits) {
            sid[slot++] = (int32_t)((32 * w + __ffs(bits) - 1) | tag);
            bits &= bits - 1;
          }
        }
        for (int q = nU + vb + s_cv[r] + tid; q < nU + vb + (s_cv[r] + 7) / 8 * 8; q += kThreads)
          sid[q] = (int32_t)tag;
      }
      for (int l = la + tid; l < lb; l += kThreads) {
        lid[8 * l + 2] = r;
        if (xt) {
          const int q = ub + (lb - 1 - l);
          lid[8 * l + 6] = (int32_t)(q | (q << 16));
          lid[8 * l + 7] = (int32_t)(q | (q << 16));
        } else {
          int cs[4];
          corner_keys(lid[8 * l], cs);
          lid[8 * l + 6] = (int32_t)((ub + rank_of(s_bm, s_pre, cs[0])) | ((ub + rank_of(s_bm, s_pre, cs[1])) << 16));
          lid[8 * l + 7] = (int32_t)((ub + rank_of(s_bm, s_pre, cs[2])) | ((ub + rank_of(s_bm, s_pre, cs[3])) << 16));
        }
        uint32_t cslots = 0;
        if (tb.n_cia > 0) {
          const int t0 = lid[8 * l + 1];
          cslots = (uint32_t)(vb + rank_of(s_cbm, s_cpre, t0)) | ((uint32_t)(vb + rank_of(s_cbm, s_cpre, t0 + 1)) << 16);
        }
        lid[8 * l + 3] = (int32_t)cslots;
      }
      __syncthreads();
    }
    // Rayleigh slots: run r at nU + nV + (R - 1 - r), the padding after them
    for (int q = tid; q < s_tot[2]; q += kThreads) {
      const int r = q < R ? R - 1 - q : 0;
      sid[nU + nV + q] = (int32_t)((uint32_t)r << 24);
    }
  }
  __syncthreads();

  // distinct corners of each 16-layer block and each layer's slots in them
  // (the FP64 kernel stages them when a model's lists overflow)
  KBlk* kblk = reinterpret_cast<KBlk*>(slab + L.off_kblk);
  const int nkb = (N + 15) / 16;
  for (int kb = tid; kb < (a.precision == TRX_FP64 && !L.slot64 ? L.NKB : 0); kb += kThreads) {
    KBlk d;
    d.nU = 0;
    d.nV = 0;
    bool over = false;
    for (int j = 0; j < 16 && kb < nkb; ++j) {
      const int l = 16 * kb + j;
      if (l >= N) break;
      const int base = lid[8 * l];
      const int cs[4] = {base, base + tb.n_P, base + 1, base + tb.n_P + 1};
      uint32_t slots = 0;
      for (int q = 0; q < 4; ++q) {
        int u = 0;
        while (u < d.nU && d.ids[u] != cs[q]) ++u;
        if (u == d.nU) {
          if (d.nU == kMaxU) { over = true; u = 0; }
          else d.ids[d.nU++] = cs[q];
        }
        slots |= (uint32_t)u << (8 * q);
      }
      lid[8 * l + 4] = (int32_t)slots;
      uint32_t cslots = 0;
      if (tb.n_cia > 0) {
        const int t0 = lid[8 * l + 1];
        const int ts[2] = {t0, t0 + 1};
        for (int q = 0; q < 2; ++q) {
          int v = 0;
          while (v < d.nV && d.tids[v] != ts[q]) ++v;
          if (v == d.nV) {
            if (d.nV == kMaxV) { over = true; v = 0; }
            else d.tids[d.nV++] = ts[q];
          }
          cslots |= (uint32_t)v << (8 * q);
        }
      }
      lid[8 * l + 5] = (int32_t)cslots;
    }
    if (over) d.nU = -1;
    for (int u = d.nU < 0 ? 0 : d.nU; u < kMaxU; ++u) d.ids[u] = 0;
    for (int v = d.nV; v < kMaxV; ++v) d.tids[v] = 0;
    d.pad[0] = d.pad[1] = 0;
    kblk[kb] = d;
  }

  // a3: chord lengths (dl_of above)
  uint8_t* dst = slab + L.off_dl;
  if (a.precision == TRX_FP64 && !L.slot64) {
    double* dlT = reinterpret_cast<double*>(dst);
    for (int e = tid; e < NP * NP; e += kThreads) {
      const int k = e / NP, j = e % NP;
      dlT[e] = dl_of(j, k);
    }
  }
}

// Path-length x opacity-weight products of the matrix-core modes (steps a3
// and a4 combined).  With the opacity slots q of a model and W[l][q] the
// weight of slot q in the opacity of layer l (the bilinear corner weight
// x 1e-4 rho, the CIA node weight x 1e-10 rho^2 / kCiaScale32, zero where
// layer l does not use q), the optical depth of ray j at one wavenumber is
//   tau_j = sum_l dl[j][l] kappa_l = sum_q P[j][q] M_q + PR_j R,
//   P[j][q] = sum_{l >= j} dl[j][l] W[l][q],  PR_j = sum_{l >= j} dl[j][l] w_R,l,
// where M_q is the mixed cross-section of slot q (sum_i chi_i sigma_i at a
// corner, or the CIA sum at a node) and R the mixed Rayleigh cross-section:
// the layer sums are taken here once per model in FP64, and the forward
// kernel contracts over the slots.  One workgroup per model, one thread per
// ray; P is accumulated in LDS 16 slots at a time, each block of slots over
// the run of layers that use one of them, and stored as A-operand fragments
// of the matrix instruction: FP32 mode hi + lo pieces in the
// v_mfma_f32_32x32x2_f32 layout (lane l, step i: P[32 rb + l%32][16 kq + 2 i + l/32]),
// bf16 modes 2 or 3 bf16 pieces in the v_mfma_f32_32x32x16_bf16 layout
// (lane l: P[32 rb + l%32][16 kq + 8 (l/32) + v], v = 0..7).  These two
// store -P / ln 2, so that the forward kernel's accumulator is the base-2
// exponent of e^{-tau} (the FP64 and gradient fragments hold P itself).
constexpr int kPT = 256;
constexpr double kNegLog2e = -1.4426950408889634074;   // -1 / ln 2
constexpr int kMaxKQ = (4 * TRX_MAX_LAYERS_MFMA + TRX_MAX_TGRID + 15) / 16;
static_assert(TRX_MAX_LAYERS_MFMA <= kPT, "one thread per ray");

// Workgroups per model: a model's tasks (slot blocks and the Rayleigh
// weights) are dealt to kPG workgroups, so that a lone model is not one
// workgroup's serial work.
constexpr int kPG = 4;
// EM, RG: built for emission and for two-layer layouts (the other builds
// leave their branches out of the chord and slot loops).
template <bool EM, bool RG>
__global__ __launch_bounds__(kPT) void k_pmat(GeomArgs a) {
  const int b = blockIdx.x;
  const int grp = blockIdx.y;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const Layout& L = a.L;
  uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  const int N = hd->n;
  if (N == 0) return;   // invalid model: the forward kernel skips it
  ModelHdr* hw = reinterpret_cast<ModelHdr*>(slab);
  const MList* ml = reinterpret_cast<const MList*>(slab + L.off_mlist);
  const int nU = ml->nU, nV = ml->nV;
  // two-layer layouts: one Rayleigh slot per run after the node slots
  const bool rg = RG && L.rg != 0;
  const int nRay = rg ? ml->pad[0] : 0, nRun = rg ? ml->pad[1] : 1;
  const int nkq = (nU + nV + nRay + 15) / 16;
  static_assert(kMaxKQ <= 64, "slot-block masks are 64 bits");
  const double* zs = reinterpret_cast<const double*>(slab + L.off_z);
  const double* A64 = reinterpret_cast<const double*>(slab + L.off_A64);
  const double* lw64 = reinterpret_cast<const double*>(slab + L.off_lw64);
  const int32_t* lid = reinterpret_cast<const int32_t*>(slab + L.off_lid);
  float2* aw = reinterpret_cast<float2*>(slab + L.off_aw);
  const double Rp = hd->Rp;
  const int tid = threadIdx.x;
  const int nrb = (N + 31) / 32;

  __shared__ double sZ[TRX_MAX_LAYERS_MFMA];
  __shared__ double sH[TRX_MAX_LAYERS_MFMA + 1];
  __shared__ double sW[TRX_MAX_LAYERS_MFMA][7];   // 4 corners, 2 CIA nodes, Rayleigh
  __shared__ int4 sS[TRX_MAX_LAYERS_MFMA];        // slots: corners 0,1 | 2,3 | CIA 0,1 (16 bits each) | Rayleigh
  __shared__ int sLo[kMaxKQ], sHi[kMaxKQ];
  __shared__ double sAcc[16][kPT];

  for (int l = tid; l < N; l += kPT) {
    sZ[l] = zs[l];
    for (int q = 0; q < 4; ++q) sW[l][q] = lw64[8 * l + q];
    sW[l][4] = lw64[8 * l + 5] / kCiaScale32;
    sW[l][5] = lw64[8 * l + 6] / kCiaScale32;
    sW[l][6] = lw64[8 * l + 4];
    const uint32_t cw = (uint32_t)lid[8 * l + 3];
    int cs = -1;
    if (nV > 0)
      cs = rg ? (int)((nU + (cw & 0xffff)) | ((nU + (cw >> 16)) << 16))
              : (int)((nU + (cw & 0xff)) | ((nU + ((cw >> 8) & 0xff)) << 16));
    // the Rayleigh slot of the layer's run (two-layer layouts)
    const int rs = rg && nRay > 0 ? nU + nV + (nRun - 1 - lid[8 * l + 2]) : 0;
    sS[l] = make_int4(lid[8 * l + 6], lid[8 * l + 7], cs, rs);
  }
  for (int c = tid; c < nkq; c += kPT) {
    sLo[c] = N;
    sHi[c] = -1;
  }
  __syncthreads();
  for (int m = tid; m <= N; m += kPT) sH[m] = m == 0 ? 0.0 : (m == N ? sZ[N - 1] : 0.5 * (sZ[m - 1] + sZ[m]));
  // the run of layers of each slot block
  for (int l = tid; l < N; l += kPT) {
    const int4 ss = sS[l];
    const uint32_t sl[7] = {(uint32_t)ss.x & 0xffffu, (uint32_t)ss.x >> 16, (uint32_t)ss.y & 0xffffu,
                            (uint32_t)ss.y >> 16, (uint32_t)ss.z & 0xffffu, (uint32_t)ss.z >> 16,
                            (uint32_t)ss.w};
    for (int q = 0; q < 7; ++q) {
      if ((q >= 4 && q < 6 && nV == 0) || (q == 6 && nRay == 0)) continue;
      atomicMin(&sLo[sl[q] >> 4], l);
      atomicMax(&sHi[sl[q] >> 4], l);
    }
  }
  __syncthreads();

  // the rays of the padded ray blocks are replicated R times over the
  // threads; replica rep takes the tasks rep, rep + R, ...: the slot blocks
  // 0 .. nkq-1, then the Rayleigh path weights
  const int NR32 = 32 * nrb;
  const int R = kPT / NR32;
  const int rep = tid / NR32;
  const int j = tid - rep * NR32;
  const bool act = rep < R && j < N;
  const double zj = act ? sZ[j] : 0.0;
  // chord of ray j through layer l, carrying q_j(h_l) in q0 (Forward
  // Models section): dl = 2 (q_j(h_{l+1}) - q_j(h_l)).  In FP64 the
  // difference loses about log10(q/dl) <= 3 digits, far below what P is
  // rounded to, and spares a division per step.
  auto qj = [&](double h) { return sqrt(fmax((h - zj) * (2.0 * Rp + h + zj), 0.0)); };
  // emission layouts: the vertical path from the bottom of shell j up
  // through shell l >= j is the shell's thickness
  const bool em = EM && L.em != 0;
  auto chord = [&](int l, double& q0) -> double {
    if (em) return sH[l + 1] - sH[l];
    const double q1 = qj(sH[l + 1]);
    const double d = 2.0 * (q1 - q0);   // q0 = 0 at l = j
    q0 = q1;
    return d;
  };

  // the Rayleigh task completes the ray weights the geometry initialised
  double* pr64 = L.off_pr64 ? reinterpret_cast<double*>(slab + L.off_pr64) : nullptr;

  uint8_t* dst = slab + L.off_dl;
  const int np = a.precision == TRX_BF16_SPLIT3 ? 3 : 2;
  // tasks of this workgroup: grp, grp + kPG, ... <= nkq; round r0 holds the
  // tasks of replicas 0 .. R-1
  const int ntask = grp <= nkq ? (nkq - grp) / kPG + 1 : 0;
  for (int r0 = 0; r0 < ntask; r0 += R) {
    const int c = (r0 + rep) < ntask ? grp + kPG * (r0 + rep) : nkq + 1;
    for (int v = 0; v < 16; ++v) sAcc[v][tid] = 0.0;
    if (act && c < nkq) {
      const int la = sLo[c], lb = sHi[c];
      const int l0 = max(j, la);
      if (l0 <= lb) {
        double q0 = l0 == j ? 0.0 : qj(sH[l0]);
        for (int l = l0; l <= lb; ++l) {
          const double d = chord(l, q0);
          const int4 ss = sS[l];
          const uint32_t sl[7] = {(uint32_t)ss.x & 0xffffu, (uint32_t)ss.x >> 16, (uint32_t)ss.y & 0xffffu,
                                  (uint32_t)ss.y >> 16, (uint32_t)ss.z & 0xffffu, (uint32_t)ss.z >> 16,
                                  (uint32_t)ss.w};
#pragma unroll
          for (int q = 0; q < 7; ++q)
            if ((int)(sl[q] >> 4) == c && (q < 4 || (q < 6 && nV > 0) || (q == 6 && nRay > 0)))
              sAcc[sl[q] & 15][tid] += d * sW[l][q];
        }
      }
    } else if (act && c == nkq && a.tab.has_rayleigh && !rg) {
      double pr = 0.0, q0 = 0.0;
      for (int l = j; l < N; ++l) pr += chord(l, q0) * sW[l][6];
      aw[j] = make_float2((float)A64[j], (float)pr);
      if (pr64) pr64[j] = pr;
    }
    {
      // ray blocks with a nonzero product in this slot block (each thread
      // checks its own ray; a half-wave holds one ray block of one replica)
      bool nz = false;
      for (int v = 0; v < 16; ++v) nz |= sAcc[v][tid] != 0.0;
      const unsigned long long bal = __ballot(nz);
      if ((tid & 31) == 0 && rep < R && c < nkq) {
        const unsigned long long half = (tid & 32) ? bal >> 32 : bal & 0xffffffffull;
        if (half) atomicOr(reinterpret_cast<unsigned long long*>(&hw->kq_mask[j >> 5]), 1ull << c);
      }
    }
    __syncthreads();
    // the fragments of the round's slot blocks: replica cr holds task
    // grp + kPG (r0 + cr)
    const int nc = min(R, ntask - r0);
    auto task_of = [&](int cr) { return grp + kPG * (r0 + cr); };
    if (L.grad && nU + nV <= kKGM) {
      // gradient layouts: P hi in FP32 as A fragments (rows = rays) and as
      // P^T fragments (rows = slots): lane l, step i holds
      // P[16 jb + 2 i + l/32][32 qb + l%32]; each slot block c writes the
      // lanes of its 16 slots (the last one also zeroes its partner half)
      float* pa = reinterpret_cast<float*>(slab + L.off_pa);
      float* pt = reinterpret_cast<float*>(slab + L.off_pt);
      for (int e = tid; e < nc * 64 * nrb; e += kPT) {
        const int cr = e / (64 * nrb), rem = e - cr * 64 * nrb;
        const int rb = rem >> 6, lane = rem & 63;
        if (task_of(cr) >= nkq) continue;
        const int col = cr * NR32 + 32 * rb + (lane & 31);
        float* o = pa + (((int64_t)rb * (kKGM / 16) + task_of(cr)) * 64 + lane) * 8;
        for (int i = 0; i < 8; ++i) o[i] = (float)sAcc[2 * i + (lane >> 5)][col];
      }
      for (int e = tid; e < nc * 64 * 2 * nrb; e += kPT) {
        const int cr = e / (128 * nrb), rem = e - cr * 128 * nrb;
        const int jb = rem >> 6, lane = rem & 63;
        const int c = task_of(cr), qb = c >> 1, half = c & 1;
        if (c >= nkq) continue;
        const int v = (lane & 31) - 16 * half;
        const bool mine = v >= 0 && v < 16;
        const bool zero_partner = !mine && half == 0 && c == nkq - 1;
        if (!mine && !zero_partner) continue;
        float* o = pt + (((int64_t)qb * (L.NP / 16) + jb) * 64 + lane) * 8;
        for (int i = 0; i < 8; ++i) {
          const int j = 16 * jb + 2 * i + (lane >> 5);
          o[i] = mine ? (float)sAcc[v][cr * NR32 + j] : 0.f;
        }
      }
    }
    if (a.precision == TRX_FP64) {
      if (L.slot64) {
        // v_mfma_f64_16x16x4f64 A operand: lane l, step s holds
        // P[16 r16 + l%16][16 kq + 4 s + l/16]
        double* f = reinterpret_cast<double*>(dst);
        for (int e = tid; e < nc * 128 * nrb; e += kPT) {
          const int cr = e / (128 * nrb), rem = e - cr * 128 * nrb;
          const int r16 = rem >> 6, lane = rem & 63;
          if (task_of(cr) >= nkq) continue;
          const int col = cr * NR32 + 16 * r16 + (lane & 15);
          double* o = f + (((int64_t)r16 * L.NKQ + task_of(cr)) * 64 + lane) * 4;
          for (int st = 0; st < 4; ++st) o[st] = sAcc[4 * st + (lane >> 4)][col];
        }
      }
    } else if (a.precision == TRX_FP32) {
      float* f = reinterpret_cast<float*>(dst);
      for (int e = tid; e < nc * 64 * nrb; e += kPT) {
        const int cr = e / (64 * nrb), rem = e - cr * 64 * nrb;
        const int rb = rem >> 6, lane = rem & 63;
        if (task_of(cr) >= nkq) continue;
        const int col = cr * NR32 + 32 * rb + (lane & 31);
        float* o = f + (((int64_t)rb * L.NKQ + task_of(cr)) * 2 * 64 + lane) * 8;
        for (int i = 0; i < 8; ++i) {
          const double x = kNegLog2e * sAcc[2 * i + (lane >> 5)][col];
          const float hi32 = (float)x;
          o[i] = hi32;
          o[64 * 8 + i] = (float)(x - (double)hi32);
        }
      }
    } else {
      uint16_t* f = reinterpret_cast<uint16_t*>(dst);
      for (int e = tid; e < nc * 64 * nrb; e += kPT) {
        const int cr = e / (64 * nrb), rem = e - cr * 64 * nrb;
        const int rb = rem >> 6, lane = rem & 63;
        if (task_of(cr) >= nkq) continue;
        const int col = cr * NR32 + 32 * rb + (lane & 31);
        uint16_t* o = f + (((int64_t)rb * L.NKQ + task_of(cr)) * np * 64 + lane) * 8;
        for (int v = 0; v < 8; ++v) {
          const double x = kNegLog2e * sAcc[8 * (lane >> 5) + v][col];
          const uint16_t p0 = bf16_bits((float)x);
          const double r1 = x - bf16_to_double(p0);
          const uint16_t p1 = bf16_bits((float)r1);
          o[v] = p0;
          o[64 * 8 + v] = p1;
          if (np == 3) o[2 * 64 * 8 + v] = bf16_bits((float)(r1 - bf16_to_double(p1)));
        }
      }
    }
    __syncthreads();
  }
}

// Work order of the persistent launch: model indices sorted by layer count,
// longest first (counting sort), and the queue counters zeroed.
__global__ __launch_bounds__(1024) void k_schedule(const int32_t* mlay, const int32_t* B_dev, int B,
                                                   int32_t* order, int32_t* qcount) {
  __shared__ int32_t hist[TRX_MAX_LAYERS_FP64 + 1];
  const int nb = B_dev ? *B_dev : B;
  for (int i = threadIdx.x; i <= TRX_MAX_LAYERS_FP64; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x < kQueues) qcount[threadIdx.x] = 0;
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int n = min(max(mlay[b], 0), TRX_MAX_LAYERS_FP64);
    atomicAdd(&hist[n], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int n = TRX_MAX_LAYERS_FP64; n >= 0; --n) {
      const int c = hist[n];
      hist[n] = acc;
      acc += c;
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int n = min(max(mlay[b], 0), TRX_MAX_LAYERS_FP64);
    order[atomicAdd(&hist[n], 1)] = b;
  }
}

}  // namespace

void launch_schedule(const int32_t* mlay, const int32_t* B_dev, int B, int32_t* order, int32_t* qcount,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_schedule, dim3(1), dim3(1024), 0, s, mlay, B_dev, B, order, qcount);
}

// The cloud deck's optical depth tc_j is folded into the annulus weights,
// not into tau; the optical-depth output adds it back, per ray, over the
// model's window.
static __global__ __launch_bounds__(256) void k_tau_cloud(const uint8_t* ws, Layout L, const int32_t* B_dev, int B,
                                                  int64_t ld, int W, double* tau) {
  const int b = blockIdx.x;
  if (b >= (B_dev ? *B_dev : B)) return;
  const uint8_t* slab = ws + (int64_t)b * L.slab;
  const ModelHdr* h = reinterpret_cast<const ModelHdr*>(slab);
  const int j = blockIdx.y;
  if (h->n == 0 || h->cloud == 0 || j >= h->n) return;
  const double tc = reinterpret_cast<const double*>(slab + L.off_pc64)[j];
  if (tc == 0.0) return;
  double* row = tau + (int64_t)b * ld + (int64_t)j * W;
  for (int i = h->lo + (int)threadIdx.x; i < h->hi; i += 256) row[i] += tc;
}

void launch_geom(const GeomArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return;
  hipLaunchKernelGGL(k_geom, dim3(B_grid), dim3(kThreads), 0, s, a);
  if (a.precision != TRX_FP64 || a.L.grad || a.L.slot64) {
    if (a.L.em) {
      if (a.L.rg) hipLaunchKernelGGL((k_pmat<true, true>), dim3(B_grid, kPG), dim3(kPT), 0, s, a);
      else hipLaunchKernelGGL((k_pmat<true, false>), dim3(B_grid, kPG), dim3(kPT), 0, s, a);
    } else {
      if (a.L.rg) hipLaunchKernelGGL((k_pmat<false, true>), dim3(B_grid, kPG), dim3(kPT), 0, s, a);
      else hipLaunchKernelGGL((k_pmat<false, false>), dim3(B_grid, kPG), dim3(kPT), 0, s, a);
    }
  }
}

void launch_tau_cloud(const uint8_t* ws, const Layout& L, const int32_t* B_dev, int B, int max_layers, int W,
                      double* tau, hipStream_t s) {
  if (B <= 0 || max_layers <= 0) return;
  hipLaunchKernelGGL(k_tau_cloud, dim3(B, max_layers), dim3(256), 0, s, ws, L, B_dev, B,
                     (int64_t)max_layers * W, W, tau);
}

}  // namespace trx
