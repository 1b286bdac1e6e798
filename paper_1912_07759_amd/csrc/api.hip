// Host side of the C ABI declared in include/trx.h: argument validation,
// device copies of the tables and channel weights, workspace management and
// the launch sequence (geometry -> opacity/optical depth/depth -> binning).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "trx_internal.h"
#include "trx_host.h"

using namespace trx;

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------
trx_status trx::set_err(trx_ctx* c, trx_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

trx_status trx::hip_err(trx_ctx* c, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return set_err(c, TRX_E_OUT_OF_MEMORY, "%s: out of device memory", what);
  return set_err(c, TRX_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

trx_status trx::ensure_buffer(trx_ctx* c, DevBuf& buf, size_t bytes, const char* what) {
  if (buf.bytes >= bytes && buf.ptr) return TRX_OK;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_err(c, e, what);
  if (buf.ptr) hipFree(buf.ptr);
  buf.ptr = nullptr;
  buf.bytes = 0;
  size_t want = std::max(bytes, (size_t)256);
  e = hipMalloc(&buf.ptr, want);
  if (e != hipSuccess) { buf.ptr = nullptr; return hip_err(c, e, what); }
  buf.bytes = want;
  return TRX_OK;
}

static bool strictly_increasing(const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  for (int i = 1; i < n; ++i)
    if (!(x[i] > x[i - 1])) return false;
  return true;
}

namespace {

__global__ void k_to_f32(const double* __restrict__ s, float* __restrict__ d, int64_t n, double scale) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += st) d[i] = (float)(s[i] * scale);
}

// Exponential-T pairs: for every absorber, temperature node iT, pressure
// node and wavenumber, (sigma[iT], log2(sigma[iT+1] / sigma[iT])) in FP32 from
// the FP64 table; NaN as the ratio where either value is not positive (that
// point takes the linear scheme), 0 at the last temperature node (no
// interval above it).
__global__ void k_exp_pairs(const double* __restrict__ s, float2* __restrict__ d, int64_t n, int64_t row_T,
                            int64_t per_abs) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double s1 = s[i];
    const int64_t within = i % per_abs;   // index inside one absorber's [n_T][n_P][n_wn]
    double r = 0.0;
    if (within + row_T < per_abs) {
      const double s2 = s[i + row_T];
      r = (s1 > 0.0 && s2 > 0.0) ? log2(s2 / s1) : __builtin_nan("");
    }
    d[i] = make_float2((float)s1, (float)r);
  }
}

__global__ void k_copy_status(const uint8_t* ws, int64_t slab, const int32_t* B_dev, int B,
                              int32_t* out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  int nb = B_dev ? *B_dev : B;
  if (b < nb) out[b] = reinterpret_cast<const ModelHdr*>(ws + (int64_t)b * slab)->status;
}

// Workspace of trx_forward_noalloc: one fixed array that each device holds
// from the first use of this code object until the process ends.  In host
// code the name is a stand-in for the symbol, not a device address: its
// address on a device is taken once, with that device current, by
// scratch_address(), and only that address is handed to kernels.
__device__ __align__(256) uint8_t scratch[TRX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxScratchDevices];
hipError_t g_scratch_err[kMaxScratchDevices];
void* g_scratch_ptr[kMaxScratchDevices];

// Device address of `scratch` on `device`, which must be the current
// device; looked up on the first call per device and kept.
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    g_scratch_done[device] = true;
  }
  *out = g_scratch_ptr[device];
  return g_scratch_err[device];
}

}  // namespace

trx_status trx::upload(trx_ctx* c, const double* host, int64_t n, double** d64, float** d32,
                       std::vector<void*>& owned, double scale32) {
  *d64 = nullptr;
  *d32 = nullptr;
  if (n == 0) return TRX_OK;
  hipError_t e = hipMalloc(d64, n * sizeof(double));
  if (e != hipSuccess) return hip_err(c, e, "trx_tables_create");
  owned.push_back(*d64);
  e = hipMalloc(d32, n * sizeof(float));
  if (e != hipSuccess) return hip_err(c, e, "trx_tables_create");
  owned.push_back(*d32);
  e = hipMemcpy(*d64, host, n * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(c, e, "trx_tables_create");
  hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, (hipStream_t)0, *d64, *d32, n, scale32);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "trx_tables_create");
  return TRX_OK;
}

void trx::launch_copy_status(const uint8_t* ws, int64_t slab, const int32_t* B_dev, int B,
                             int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_status, dim3((B + 255) / 256), dim3(256), 0, s, ws, slab, B_dev, B,
                     out);
}

// --------------------------------------------------------------------------
// context
// --------------------------------------------------------------------------
extern "C" trx_status trx_create(int device, trx_ctx** out) {
  if (!out) return TRX_E_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TRX_E_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return TRX_E_DEVICE;
  trx_ctx* c = new trx_ctx();
  c->device = device;
  c->stream = nullptr;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->n_cu = prop.multiProcessorCount;
    snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
  }
  // the no-allocation workspace of this device (a failure is reported by
  // trx_forward_noalloc, the only user)
  void* sp = nullptr;
  (void)scratch_address(device, &sp);
  *out = c;
  return TRX_OK;
}

extern "C" trx_status trx_destroy(trx_ctx* c) {
  if (!c) return TRX_E_INVALID_ARG;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (DevBuf* b : {&c->ws, &c->aws, &c->grad, &c->sched})
    if (b->ptr) hipFree(b->ptr);
  for (auto& r : c->pending) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
  for (hipEvent_t e : c->pool) hipEventDestroy(e);
  delete c;
  return TRX_OK;
}

extern "C" const char* trx_last_error(const trx_ctx* c) { return c ? c->err.c_str() : ""; }

extern "C" trx_status trx_set_stream(trx_ctx* c, void* s) {
  if (!c) return TRX_E_INVALID_ARG;
  c->stream = (hipStream_t)s;
  return TRX_OK;
}

extern "C" trx_status trx_synchronize(trx_ctx* c) {
  if (!c) return TRX_E_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? TRX_OK : hip_err(c, e, "trx_synchronize");
}

// --------------------------------------------------------------------------
// tables
// --------------------------------------------------------------------------
extern "C" trx_status trx_tables_create(trx_ctx* c, const trx_tables_desc* d, trx_tables** out) {
  if (!c) return TRX_E_INVALID_ARG;
  c->err.clear();
  if (!d || !out) return set_err(c, TRX_E_INVALID_ARG, "trx_tables_create: null argument");
  *out = nullptr;
  if (d->n_wn < 2 || !d->wn_cm1 || !strictly_increasing(d->wn_cm1, d->n_wn))
    return set_err(c, TRX_E_INVALID_ARG, "wavenumber grid must have >= 2 strictly increasing finite points");
  if (d->n_T < 2 || d->n_T > TRX_MAX_TGRID || !d->T_K || !strictly_increasing(d->T_K, d->n_T) ||
      d->T_K[0] <= 0)
    return set_err(c, TRX_E_INVALID_ARG, "temperature grid must have 2..%d strictly increasing positive points",
                   TRX_MAX_TGRID);
  if (d->n_P < 2 || d->n_P > TRX_MAX_PGRID || !d->log10P_Pa || !strictly_increasing(d->log10P_Pa, d->n_P))
    return set_err(c, TRX_E_INVALID_ARG, "log10 pressure grid must have 2..%d strictly increasing points",
                   TRX_MAX_PGRID);
  if (d->t_interp != TRX_T_LINEAR && d->t_interp != TRX_T_EXP)
    return set_err(c, TRX_E_INVALID_ARG, "t_interp must be TRX_T_LINEAR or TRX_T_EXP");
  if (d->n_abs < 0 || d->n_abs > TRX_MAX_ABSORBERS)
    return set_err(c, TRX_E_INVALID_ARG, "n_abs must be in 0..%d", TRX_MAX_ABSORBERS);
  if (d->n_abs > 0 && (!d->xsec_cm2 || !d->abs_mass_amu))
    return set_err(c, TRX_E_INVALID_ARG, "xsec_cm2 and abs_mass_amu are required when n_abs > 0");
  for (int i = 0; i < d->n_abs; ++i)
    if (!(std::isfinite(d->abs_mass_amu[i]) && d->abs_mass_amu[i] > 0))
      return set_err(c, TRX_E_INVALID_ARG, "absorber mass %d must be positive", i);
  if (!(d->h2_mass_amu > 0) || !(d->he_mass_amu > 0))
    return set_err(c, TRX_E_INVALID_ARG, "H2 and He masses must be positive");
  if (d->n_cia < 0 || d->n_cia > TRX_MAX_CIA)
    return set_err(c, TRX_E_INVALID_ARG, "n_cia must be in 0..%d", TRX_MAX_CIA);
  if (d->n_cia > 0) {
    if (d->n_Tcia < 2 || d->n_Tcia > TRX_MAX_TGRID || !d->Tcia_K ||
        !strictly_increasing(d->Tcia_K, d->n_Tcia) || !d->cia_cm5 || !d->cia_pair)
      return set_err(c, TRX_E_INVALID_ARG, "CIA needs a strictly increasing T grid of 2..%d points, tables and pairs",
                     TRX_MAX_TGRID);
    for (int p = 0; p < 2 * d->n_cia; ++p)
      if (d->cia_pair[p] < 0 || d->cia_pair[p] >= d->n_abs + 2)
        return set_err(c, TRX_E_INVALID_ARG, "CIA species id out of range");
  }
  {
    const double lim = 2147483648.0;   // row offsets are 32-bit byte offsets
    const double wb = 4.0 * d->n_wn;
    const double wx = d->t_interp == TRX_T_EXP ? 2.0 * wb : wb;
    if (wx * d->n_T * d->n_P >= lim || (d->n_cia > 0 && wb * d->n_Tcia >= lim) || wb * (d->n_abs + 2) >= lim)
      return set_err(c, TRX_E_UNSUPPORTED, "an FP32 table of one absorber, CIA pair or the Rayleigh table reaches 2 GiB");
  }
  hipSetDevice(c->device);
  trx_tables* t = new trx_tables();
  t->ctx = c;
  DevTables& D = t->dev;
  memset(&D, 0, sizeof D);
  D.n_wn = d->n_wn; D.n_T = d->n_T; D.n_P = d->n_P; D.n_abs = d->n_abs;
  D.n_cia = d->n_cia; D.n_Tcia = d->n_cia > 0 ? d->n_Tcia : 0;
  D.has_rayleigh = d->rayleigh_cm2 ? 1 : 0;
  t->wn.assign(d->wn_cm1, d->wn_cm1 + d->n_wn);
  auto fail = [&](trx_status s) { for (void* p : t->owned) hipFree(p); delete t; return s; };
  float* f32 = nullptr;
  double* g = nullptr;
  trx_status s;
  if ((s = upload(c, d->wn_cm1, d->n_wn, &g, &f32, t->owned)) != TRX_OK) return fail(s);
  D.wn = g;
  if ((s = upload(c, d->T_K, d->n_T, &g, &f32, t->owned)) != TRX_OK) return fail(s);
  D.T = g;
  if ((s = upload(c, d->log10P_Pa, d->n_P, &g, &f32, t->owned)) != TRX_OK) return fail(s);
  D.logP = g;
  const int64_t nx = (int64_t)d->n_abs * d->n_T * d->n_P * d->n_wn;
  if ((s = upload(c, d->xsec_cm2, nx, &g, &f32, t->owned)) != TRX_OK) return fail(s);
  D.xsec64 = g; D.xsec32 = f32;
  if (d->t_interp == TRX_T_EXP) {
    D.t_exp = 1;
    if (nx > 0) {
      float2* px = nullptr;
      hipError_t e = hipMalloc(&px, nx * sizeof(float2));
      if (e != hipSuccess) return fail(hip_err(c, e, "trx_tables_create"));
      t->owned.push_back(px);
      const int64_t row_T = (int64_t)d->n_P * d->n_wn;
      hipLaunchKernelGGL(k_exp_pairs, dim3(1024), dim3(256), 0, (hipStream_t)0, D.xsec64, px, nx, row_T,
                         (int64_t)d->n_T * row_T);
      e = hipGetLastError();
      if (e != hipSuccess) return fail(hip_err(c, e, "trx_tables_create"));
      D.xexp32 = px;
    }
  }
  if (d->n_cia > 0) {
    if ((s = upload(c, d->Tcia_K, d->n_Tcia, &g, &f32, t->owned)) != TRX_OK) return fail(s);
    D.Tcia = g;
    const int64_t nc = (int64_t)d->n_cia * d->n_Tcia * d->n_wn;
    if ((s = upload(c, d->cia_cm5, nc, &g, &f32, t->owned, kCiaScale32)) != TRX_OK) return fail(s);
    D.cia64 = g; D.cia32 = f32;
    for (int p = 0; p < d->n_cia; ++p) {
      D.cia_pair[p][0] = d->cia_pair[2 * p];
      D.cia_pair[p][1] = d->cia_pair[2 * p + 1];
    }
  }
  if (d->rayleigh_cm2) {
    if ((s = upload(c, d->rayleigh_cm2, (int64_t)(d->n_abs + 2) * d->n_wn, &g, &f32, t->owned)) != TRX_OK)
      return fail(s);
    D.ray64 = g; D.ray32 = f32;
  }
  for (int i = 0; i < d->n_abs; ++i) D.mass[i] = d->abs_mass_amu[i];
  D.mass[d->n_abs] = d->h2_mass_amu;
  D.mass[d->n_abs + 1] = d->he_mass_amu;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(hip_err(c, e, "trx_tables_create"));
  *out = t;
  return TRX_OK;
}

extern "C" trx_status trx_tables_destroy(trx_tables* t) {
  if (!t) return TRX_E_INVALID_ARG;
  hipSetDevice(t->ctx->device);
  hipDeviceSynchronize();
  for (void* p : t->owned) hipFree(p);
  delete t;
  return TRX_OK;
}

// --------------------------------------------------------------------------
// channels
// --------------------------------------------------------------------------
extern "C" trx_status trx_bins_create(trx_ctx* c, const trx_tables* t, int32_t n_ch, const double* lo,
                                      const double* hi, trx_bins** out) {
  if (!c) return TRX_E_INVALID_ARG;
  c->err.clear();
  if (!t || !lo || !hi || !out || n_ch < 1)
    return set_err(c, TRX_E_INVALID_ARG, "trx_bins_create: null argument or n_ch < 1");
  *out = nullptr;
  for (int k = 0; k < n_ch; ++k)
    if (!(std::isfinite(lo[k]) && std::isfinite(hi[k]) && hi[k] > lo[k]))
      return set_err(c, TRX_E_INVALID_ARG, "channel %d must have finite edges lo < hi", k);
  const std::vector<double>& wn = t->wn;
  const int W = (int)wn.size();
  std::vector<double> elo(W), ehi(W);
  for (int i = 0; i + 1 < W; ++i) {
    double m = 0.5 * (wn[i] + wn[i + 1]);
    ehi[i] = m;
    elo[i + 1] = m;
  }
  elo[0] = wn[0] - (elo[1] - wn[0]);
  ehi[W - 1] = wn[W - 1] + (wn[W - 1] - ehi[W - 2]);
  std::vector<int32_t> i0(n_ch), i1(n_ch);
  std::vector<int64_t> off(n_ch);
  std::vector<double> w;
  for (int k = 0; k < n_ch; ++k) {
    // native bins overlapping [lo, hi): ehi > lo and elo < hi
    int a = (int)(std::upper_bound(ehi.begin(), ehi.end(), lo[k]) - ehi.begin());
    int b = (int)(std::lower_bound(elo.begin(), elo.end(), hi[k]) - elo.begin());
    if (b < a) b = a;
    i0[k] = a;
    i1[k] = b;
    off[k] = (int64_t)w.size();
    for (int i = a; i < b; ++i) {
      double ov = std::min(hi[k], ehi[i]) - std::max(lo[k], elo[i]);
      w.push_back(std::max(ov, 0.0) / (ehi[i] - elo[i]));
    }
  }
  // the same weights by native point, channels ascending
  std::vector<int64_t> poff(W + 1, 0);
  for (int k = 0; k < n_ch; ++k)
    for (int i = i0[k]; i < i1[k]; ++i) ++poff[i + 1];
  for (int i = 0; i < W; ++i) poff[i + 1] += poff[i];
  std::vector<int32_t> pch(std::max<int64_t>(poff[W], 1));
  std::vector<double> pw(std::max<int64_t>(poff[W], 1));
  {
    std::vector<int64_t> fill(poff.begin(), poff.end() - 1);
    for (int k = 0; k < n_ch; ++k)
      for (int i = i0[k]; i < i1[k]; ++i) {
        pch[fill[i]] = k;
        pw[fill[i]++] = w[off[k] + (i - i0[k])];
      }
  }
  if (w.empty()) w.push_back(0.0);
  hipSetDevice(c->device);
  trx_bins* bn = new trx_bins();
  bn->ctx = c;
  bn->tables = t;
  bn->n_ch = n_ch;
  hipError_t e = hipSuccess;
  auto put = [&](void** d, const void* h, size_t n) {
    if (e != hipSuccess) return;
    e = hipMalloc(d, n);
    if (e == hipSuccess) { bn->owned.push_back(*d); e = hipMemcpy(*d, h, n, hipMemcpyHostToDevice); }
  };
  put((void**)&bn->i0, i0.data(), n_ch * sizeof(int32_t));
  put((void**)&bn->i1, i1.data(), n_ch * sizeof(int32_t));
  put((void**)&bn->off, off.data(), n_ch * sizeof(int64_t));
  put((void**)&bn->w, w.data(), w.size() * sizeof(double));
  put((void**)&bn->poff, poff.data(), poff.size() * sizeof(int64_t));
  put((void**)&bn->pch, pch.data(), pch.size() * sizeof(int32_t));
  put((void**)&bn->pw, pw.data(), pw.size() * sizeof(double));
  if (e != hipSuccess) {
    for (void* p : bn->owned) hipFree(p);
    delete bn;
    return hip_err(c, e, "trx_bins_create");
  }
  *out = bn;
  return TRX_OK;
}

extern "C" trx_status trx_bins_destroy(trx_bins* b) {
  if (!b) return TRX_E_INVALID_ARG;
  hipSetDevice(b->ctx->device);
  hipDeviceSynchronize();
  for (void* p : b->owned) hipFree(p);
  delete b;
  return TRX_OK;
}

// --------------------------------------------------------------------------
// forward
// --------------------------------------------------------------------------
trx_status trx::check_batch(trx_ctx* c, const trx_tables* t, const trx_batch* bt, int precision) {
  if (!t) return set_err(c, TRX_E_INVALID_ARG, "tables handle is null");
  if (t->ctx != c) return set_err(c, TRX_E_INVALID_ARG, "tables belong to another context");
  if (!bt) return set_err(c, TRX_E_INVALID_ARG, "batch is null");
  if (bt->B < 1) return set_err(c, TRX_E_INVALID_ARG, "batch.B must be >= 1");
  if (precision < TRX_FP64 || precision > TRX_BF16_SPLIT3)
    return set_err(c, TRX_E_INVALID_ARG, "unknown precision %d", precision);
  if (bt->max_layers < 2) return set_err(c, TRX_E_INVALID_ARG, "batch.max_layers must be >= 2");
  const int limit = precision == TRX_FP64 ? TRX_MAX_LAYERS_FP64 : TRX_MAX_LAYERS_MFMA;
  if (bt->max_layers > limit)
    return set_err(c, TRX_E_UNSUPPORTED, "max_layers %d exceeds %d for this precision", bt->max_layers, limit);
  if (!bt->n_layers || !bt->layer_off || !bt->T_K || !bt->p_bot_Pa || !bt->p_top_Pa || !bt->Rp_m ||
      !bt->Rs_m || !bt->GM_m3s2 || !bt->wn_lo || !bt->wn_hi || (t->dev.n_abs > 0 && !bt->log10_vmr))
    return set_err(c, TRX_E_INVALID_ARG, "a batch array pointer is null");
  if (!(bt->he_h2_ratio >= 0) || !(bt->k_B > 0) || !(bt->amu_kg > 0))
    return set_err(c, TRX_E_INVALID_ARG, "he_h2_ratio must be >= 0 and k_B, amu_kg > 0");
  if (bt->gravity != 0 && bt->gravity != 1) return set_err(c, TRX_E_INVALID_ARG, "gravity must be 0 or 1");
  const int nc = !!bt->cloud_sigma_m2 + !!bt->cloud_p_top_Pa + !!bt->cloud_p_bottom_Pa;
  if (nc != 0 && nc != 3)
    return set_err(c, TRX_E_INVALID_ARG, "cloud deck arrays: all three or none");
  if (!bt->log10_vmr_top != !bt->vmr_switch_Pa)
    return set_err(c, TRX_E_INVALID_ARG, "two-layer arrays: log10_vmr_top and vmr_switch_Pa both or neither");
  if (bt->log10_vmr_top && precision == TRX_FP64 && bt->max_layers > TRX_MAX_LAYERS_MFMA)
    return set_err(c, TRX_E_UNSUPPORTED, "two-layer profiles take at most %d layers in TRX_FP64",
                   TRX_MAX_LAYERS_MFMA);
  return TRX_OK;
}

trx_status trx::check_emission(trx_ctx* c, int precision, int max_layers, const double* T_star, int n_mu) {
  if (n_mu < 1 || n_mu > TRX_MAX_MU)
    return set_err(c, TRX_E_INVALID_ARG, "n_mu must be in 1..%d", TRX_MAX_MU);
  if (!T_star) return set_err(c, TRX_E_INVALID_ARG, "the stellar temperatures are required");
  if (precision == TRX_FP64 && max_layers > TRX_MAX_LAYERS_MFMA)
    return set_err(c, TRX_E_UNSUPPORTED, "emission takes at most %d layers", TRX_MAX_LAYERS_MFMA);
  return TRX_OK;
}

// Gauss-Legendre rule on [-1, 1]: the roots x_i of the Legendre polynomial
// P_n by Newton's method from x = cos(pi (i + 3/4)/(n + 1/2)), with P_n and
// P_n' from the three-term recurrence (k P_k = (2k-1) x P_{k-1} - (k-1)
// P_{k-2}) and P_n' = n (x P_n - P_{n-1})/(x^2 - 1); weights 2/((1 - x^2)
// P_n'(x)^2).  Mapped to mu = (1 + x)/2 with weights w/2.
void trx::gauss_legendre01(int n, double* mu, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double x = cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    mu[i] = 0.5 * (1.0 + x);
    w[i] = 1.0 / ((1.0 - x * x) * dp * dp);   // half of 2 / ((1 - x^2) P_n'^2)
  }
}

DevBatch trx::dev_batch(const trx_batch* bt) {
  DevBatch d;
  d.n_layers = bt->n_layers; d.layer_off = bt->layer_off; d.T = bt->T_K;
  d.p_bot = bt->p_bot_Pa; d.p_top = bt->p_top_Pa; d.log10_vmr = bt->log10_vmr;
  d.Rp = bt->Rp_m; d.Rs = bt->Rs_m; d.GM = bt->GM_m3s2;
  d.wn_lo = bt->wn_lo; d.wn_hi = bt->wn_hi;
  d.he_h2 = bt->he_h2_ratio; d.kB = bt->k_B; d.amu = bt->amu_kg; d.gravity = bt->gravity;
  d.cloud_sigma = bt->cloud_sigma_m2; d.cloud_p1 = bt->cloud_p_top_Pa; d.cloud_p2 = bt->cloud_p_bottom_Pa;
  d.vmr_top = bt->log10_vmr_top; d.vmr_sw = bt->vmr_switch_Pa;
  return d;
}

trx_status trx::enqueue_forward(trx_ctx* c, const trx_tables* t, const DevBatch& db, int B,
                                const int32_t* B_dev, int max_layers, const trx_bins* bins,
                                int precision, const RunConfig& rc, uint8_t* ws, void* aws,
                                const SchedBufs& sb, double* depth_native, double* depth_binned,
                                int32_t* status, bool grad_layout, double* tau, const EmissionIn* em,
                                bool regimes) {
  const Layout L = make_layout(max_layers, precision, grad_layout, t->dev, em != nullptr, regimes);
  GeomArgs g;
  g.bt = db;
  g.tab = t->dev;
  g.L = L;
  g.ws = ws;
  g.B_dev = B_dev;
  g.B = B;
  g.precision = precision;
  g.n_limit = max_layers;
  g.span_cols = rc.span_cols;
  g.depth_native = depth_native;
  g.mlay = sb.mlay;
  g.mspan = sb.mspan;
  g.T_star = em ? em->T_star : nullptr;
  // h c / k_B in K cm (h and c exact SI, k_B as passed)
  g.c2 = 100.0 * 6.62607015e-34 * 299792458.0 / db.kB;
  {
    ProfScope ps(c, TRX_KERNEL_GEOMETRY);
    launch_geom(g, B, c->stream);
  }
  launch_copy_status(ws, L.slab, B_dev, B, status, c->stream);
  const bool persistent = rc.persistent && precision != TRX_FP64;
  if (persistent) {
    ProfScope ps(c, TRX_KERNEL_SCHEDULE);
    launch_schedule(sb.mlay, B_dev, B, sb.order, sb.qcount, c->stream);
  }

  FwdArgs f;
  memset(&f, 0, sizeof f);
  f.tab = t->dev;
  f.L = L;
  f.ws = ws;
  f.B_dev = B_dev;
  f.B = B;
  f.span_cols = rc.span_cols;
  f.n_spans = (t->dev.n_wn + rc.span_cols - 1) / rc.span_cols;
  f.depth_native = depth_native;
  f.aws = aws;
  f.model_status = status;
  f.tau = tau;
  f.tau_ld = (int64_t)max_layers * t->dev.n_wn;
  f.order = sb.order;
  f.mspan = sb.mspan;
  f.qcount = sb.qcount;
  f.persistent = persistent ? 1 : 0;
  f.group = rc.group;
  f.span_group = rc.span_group > 0 ? rc.span_group : 1;
  // the residual D - obs of a chi^2 gradient near the optimum is at the
  // noise level: its forward pass takes the accurate depth epilogue
  f.accurate = grad_layout ? 1 : 0;
  if (em) {
    double mu[TRX_MAX_MU], w[TRX_MAX_MU];
    gauss_legendre01(em->n_mu, mu, w);
    f.n_mu = em->n_mu;
    for (int i = 0; i < em->n_mu; ++i) {
      f.em_k64[i] = 1.0 / mu[i];
      f.em_c64[i] = 2.0 * w[i] * mu[i];
      f.em_k32[i] = (float)f.em_k64[i];
      f.em_c32[i] = (float)f.em_c64[i];
    }
  }
  {
    ProfScope ps(c, TRX_KERNEL_FORWARD);
    if (precision == TRX_FP64) {
      launch_fwd64(f, B, c->stream);
    } else {
      launch_fwd_mfma(f, precision, rc.nrb_max, rc.rbw, rc.occ, B, c->n_cu, c->stream);
    }
  }
  if (tau && db.cloud_sigma) launch_tau_cloud(ws, L, B_dev, B, max_layers, t->dev.n_wn, tau, c->stream);
  if (depth_binned) {
    BinArgs ba;
    ba.ws = ws; ba.L = L; ba.B_dev = B_dev; ba.B = B;
    ba.n_wn = t->dev.n_wn; ba.n_ch = bins->n_ch;
    ba.ch_i0 = bins->i0; ba.ch_i1 = bins->i1; ba.ch_off = bins->off; ba.ch_w = bins->w;
    ba.aws = aws; ba.aws_f64 = precision == TRX_FP64 || em != nullptr; ba.out = depth_binned;
    ProfScope ps(c, TRX_KERNEL_BINNING);
    launch_bin(ba, B, c->stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "kernel launch");
  return TRX_OK;
}

GradScratch trx::carve_grad_scratch(void* base, int B, int n_wn, int n_ch, int NP) {
  const GradAcc G = make_grad_acc(NP);
  const GradAcc Gp = make_grad_acc(NP, kKG);
  const size_t spans = (size_t)(n_wn + kSpanCols - 1) / kSpanCols;
  const size_t items = (spans + kAdjSpanGroup - 1) / kAdjSpanGroup * kGChunks;
  uint8_t* p = (uint8_t*)base;
  size_t o = 0;
  auto take = [&](size_t bytes) -> void* {
    void* r = p ? p + o : nullptr;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  GradScratch g;
  g.acc = (double*)take((size_t)B * G.n * 8);
  g.binned = (double*)take((size_t)B * n_ch * 8);
  g.coef = (double*)take((size_t)B * n_ch * 8);
  g.dbar = (float*)take((size_t)B * n_wn * 4);
  g.part = (float*)take((size_t)B * items * Gp.n * 4);
  g.bytes = o;
  return g;
}

size_t trx::grad_scratch_bytes(int B, int n_wn, int n_ch, int NP) {
  return carve_grad_scratch(nullptr, B, n_wn, n_ch, NP).bytes;
}

trx_status trx::enqueue_chi2_grad(trx_ctx* c, const trx_tables* t, const DevBatch& db, int B,
                                  const int32_t* B_dev, int max_layers, const trx_bins* bins, int precision,
                                  const RunConfig& rc, DevBuf& ws, DevBuf& aws, DevBuf& sched, DevBuf& grad,
                                  const double* obs, const double* sigma, double* chi2, double* dT,
                                  double* dvmr, double* dRp, double* depth_binned, int32_t* status,
                                  bool alloc) {
  const Layout L = make_layout(max_layers, precision, true, t->dev);
  const GradAcc G = make_grad_acc(L.NP);
  const int W = t->dev.n_wn;
  const size_t esz = precision == TRX_FP64 ? 8 : 4;
  if (alloc) {
    trx_status s;
    if ((s = ensure_buffer(c, ws, (size_t)B * L.slab, "workspace")) != TRX_OK) return s;
    if ((s = ensure_buffer(c, aws, (size_t)B * W * esz, "workspace")) != TRX_OK) return s;
    if ((s = ensure_buffer(c, sched, SchedBufs::bytes(B), "workspace")) != TRX_OK) return s;
    if ((s = ensure_buffer(c, grad, grad_scratch_bytes(B, W, bins->n_ch, L.NP), "workspace")) != TRX_OK)
      return s;
  }
  const GradScratch gs = carve_grad_scratch(grad.ptr, B, W, bins->n_ch, L.NP);
  double* binned = depth_binned ? depth_binned : gs.binned;
  trx_status s = enqueue_forward(c, t, db, B, B_dev, max_layers, bins, precision, rc, (uint8_t*)ws.ptr,
                                 aws.ptr, SchedBufs::carve(sched.ptr, B), nullptr, binned, status, true);
  if (s != TRX_OK) return s;
  AdjArgs a;
  memset(&a, 0, sizeof a);
  a.tab = t->dev;
  a.L = L;
  a.G = G;
  a.Gp = make_grad_acc(L.NP, kKG);
  a.ws = (uint8_t*)ws.ptr;
  a.bt = db;
  a.B_dev = B_dev;
  a.B = B;
  a.n_ch = bins->n_ch;
  a.ch_i0 = bins->i0; a.ch_i1 = bins->i1; a.ch_off = bins->off; a.ch_w = bins->w;
  a.pt_off = bins->poff; a.pt_ch = bins->pch; a.pt_w = bins->pw;
  a.coef = gs.coef;
  a.binned = binned;
  a.obs = obs;
  a.sigma = sigma;
  a.chi2 = chi2;
  a.dbar = gs.dbar;
  a.acc = gs.acc;
  a.part = gs.part;
  a.n_spans = (W + kSpanCols - 1) / kSpanCols;
  a.span_group = kAdjSpanGroup;
  a.n_items = (a.n_spans + kAdjSpanGroup - 1) / kAdjSpanGroup * kGChunks;
  a.dT = dT;
  a.dvmr = dvmr;
  a.dRp = dRp;
  a.model_status = status;
  {
    ProfScope ps(c, TRX_KERNEL_GEOM_ADJ);
    launch_chi2_dbar(a, B, c->stream);
  }
  {
    ProfScope ps(c, TRX_KERNEL_ADJOINT);
    hipError_t e = launch_adj_item(a, B, c->stream);
    if (e != hipSuccess) return hip_err(c, e, "adjoint launch");
  }
  {
    ProfScope ps(c, TRX_KERNEL_GEOM_ADJ);
    launch_adj_reduce(a, B, c->stream);
    launch_adj_pmat(a, B, c->stream);
    launch_adj_geom(a, B, c->stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "adjoint launch");
  return TRX_OK;
}

RunConfig trx::default_config(int precision, int max_layers) {
  RunConfig rc;
  rc.nrb_max = (max_layers + 31) / 32;
  rc.persistent = precision != TRX_FP64;
  return rc;
}

extern "C" trx_status trx_forward(trx_ctx* c, const trx_tables* t, const trx_batch* bt,
                                  const trx_bins* bins, trx_precision precision, double* depth_native,
                                  double* depth_binned, int32_t* model_status, double* tau) {
  if (!c) return TRX_E_INVALID_ARG;
  c->err.clear();
  trx_status s = check_batch(c, t, bt, precision);
  if (s != TRX_OK) return s;
  if (!model_status) return set_err(c, TRX_E_INVALID_ARG, "model_status is required");
  if (depth_binned && !bins) return set_err(c, TRX_E_INVALID_ARG, "depth_binned requires bins");
  if (bins && bins->tables != t) return set_err(c, TRX_E_INVALID_ARG, "bins were made for other tables");
  hipSetDevice(c->device);
  const bool rg = bt->log10_vmr_top != nullptr;
  const Layout L = make_layout(bt->max_layers, precision, false, t->dev, false, rg);
  if ((s = ensure_buffer(c, c->ws, (size_t)bt->B * L.slab, "workspace")) != TRX_OK) return s;
  const size_t esz = precision == TRX_FP64 ? 8 : 4;
  if ((s = ensure_buffer(c, c->aws, (size_t)bt->B * t->dev.n_wn * esz, "workspace")) != TRX_OK) return s;
  if ((s = ensure_buffer(c, c->sched, SchedBufs::bytes(bt->B), "workspace")) != TRX_OK) return s;
  RunConfig rc = default_config(precision, bt->max_layers);
  return enqueue_forward(c, t, dev_batch(bt), bt->B, nullptr, bt->max_layers, bins, precision, rc,
                         (uint8_t*)c->ws.ptr, c->aws.ptr, SchedBufs::carve(c->sched.ptr, bt->B),
                         depth_native, depth_binned, model_status, false, tau, nullptr, rg);
}

extern "C" trx_status trx_forward_noalloc(trx_ctx* c, const trx_tables* t, const trx_batch* bt,
                                          const trx_bins* bins, trx_precision precision,
                                          double* depth_native, double* depth_binned,
                                          int32_t* model_status) {
  if (!c) return TRX_E_INVALID_ARG;
  c->err.clear();
  trx_status s = check_batch(c, t, bt, precision);
  if (s != TRX_OK) return s;
  if (!model_status) return set_err(c, TRX_E_INVALID_ARG, "model_status is required");
  if (depth_binned && !bins) return set_err(c, TRX_E_INVALID_ARG, "depth_binned requires bins");
  if (bins && bins->tables != t) return set_err(c, TRX_E_INVALID_ARG, "bins were made for other tables");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_err(c, e, "trx_forward_noalloc");
  void* base = nullptr;
  e = scratch_address(c->device, &base);
  if (e != hipSuccess || !base)
    return set_err(c, TRX_E_DEVICE, "trx_forward_noalloc: no scratch array on device %d (%s)", c->device,
                   hipGetErrorString(e));
  // carve the workspace of trx_forward (slabs, atmospheric depth, work
  // order) from the array, each part 256-byte aligned
  const bool rg = bt->log10_vmr_top != nullptr;
  const Layout L = make_layout(bt->max_layers, precision, false, t->dev, false, rg);
  const size_t esz = precision == TRX_FP64 ? 8 : 4;
  size_t used = 0;
  auto take = [&](size_t bytes) { const size_t o = used; used += (bytes + 255) / 256 * 256; return o; };
  const size_t o_ws = take((size_t)bt->B * (size_t)L.slab);
  const size_t o_aws = take((size_t)bt->B * (size_t)t->dev.n_wn * esz);
  const size_t o_sched = take(SchedBufs::bytes(bt->B));
  if (used > (size_t)TRX_NOALLOC_SCRATCH_BYTES)
    return set_err(c, TRX_E_UNSUPPORTED,
                   "trx_forward_noalloc: %d models of up to %d layers on %d wavenumbers need %zu bytes of "
                   "workspace, more than the %zu bytes of the fixed scratch array; split the batch",
                   bt->B, bt->max_layers, t->dev.n_wn, used, (size_t)TRX_NOALLOC_SCRATCH_BYTES);
  uint8_t* p = (uint8_t*)base;
  // no profiling events either: creating them may allocate
  c->no_events = true;
  s = enqueue_forward(c, t, dev_batch(bt), bt->B, nullptr, bt->max_layers, bins, precision,
                      default_config(precision, bt->max_layers), p + o_ws, p + o_aws,
                      SchedBufs::carve(p + o_sched, bt->B), depth_native, depth_binned, model_status, false,
                      nullptr, nullptr, rg);
  c->no_events = false;
  return s;
}

extern "C" trx_status trx_emission(trx_ctx* c, const trx_tables* t, const trx_batch* bt, const trx_bins* bins,
                                   trx_precision precision, int32_t n_mu, const double* T_star_K,
                                   double* fpfs_native, double* fpfs_binned, int32_t* model_status) {
  if (!c) return TRX_E_INVALID_ARG;
  c->err.clear();
  trx_status s = check_batch(c, t, bt, precision);
  if (s != TRX_OK) return s;
  if ((s = check_emission(c, precision, bt->max_layers, T_star_K, n_mu)) != TRX_OK) return s;
  if (!model_status) return set_err(c, TRX_E_INVALID_ARG, "model_status is required");
  if (fpfs_binned && !bins) return set_err(c, TRX_E_INVALID_ARG, "fpfs_binned requires bins");
  if (bins && bins->tables != t) return set_err(c, TRX_E_INVALID_ARG, "bins were made for other tables");
  hipSetDevice(c->device);
  const bool rg = bt->log10_vmr_top != nullptr;
  const Layout L = make_layout(bt->max_layers, precision, false, t->dev, true, rg);
  if ((s = ensure_buffer(c, c->ws, (size_t)bt->B * L.slab, "workspace")) != TRX_OK) return s;
  const size_t esz = 8;   // the flux ratio per native point is kept in FP64 in every mode
  if ((s = ensure_buffer(c, c->aws, (size_t)bt->B * t->dev.n_wn * esz, "workspace")) != TRX_OK) return s;
  if ((s = ensure_buffer(c, c->sched, SchedBufs::bytes(bt->B), "workspace")) != TRX_OK) return s;
  RunConfig rc = default_config(precision, bt->max_layers);
  const EmissionIn em{T_star_K, n_mu};
  return enqueue_forward(c, t, dev_batch(bt), bt->B, nullptr, bt->max_layers, bins, precision, rc,
                         (uint8_t*)c->ws.ptr, c->aws.ptr, SchedBufs::carve(c->sched.ptr, bt->B), fpfs_native,
                         fpfs_binned, model_status, false, nullptr, &em, rg);
}

// --------------------------------------------------------------------------
// measurement
// --------------------------------------------------------------------------
static hipEvent_t take_event(trx_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

trx::ProfScope::ProfScope(trx_ctx* ctx, int k) : c(ctx), kind(k) {
  if (!c->profile || c->capturing || c->no_events) return;
  a = take_event(c);
  b = take_event(c);
  hipEventRecord(a, c->stream);
}

trx::ProfScope::~ProfScope() {
  if (!a) return;
  hipEventRecord(b, c->stream);
  c->pending.push_back({kind, a, b});
}

static void drain(trx_ctx* c) {
  for (auto& r : c->pending) {
    hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->total_ms[r.kind] += ms;
      c->launches[r.kind] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->pending.clear();
}

extern "C" trx_status trx_profile(trx_ctx* c, int32_t enable) {
  if (!c) return TRX_E_INVALID_ARG;
  drain(c);
  c->profile = enable != 0;
  if (enable)
    for (int k = 0; k < TRX_KERNEL_CLASSES; ++k) { c->total_ms[k] = 0; c->launches[k] = 0; }
  return TRX_OK;
}

extern "C" trx_status trx_profile_read(trx_ctx* c, int32_t kernel, double* total_ms, int32_t* launches) {
  if (!c) return TRX_E_INVALID_ARG;
  if (kernel < 0 || kernel >= TRX_KERNEL_CLASSES || !total_ms || !launches)
    return set_err(c, TRX_E_INVALID_ARG, "trx_profile_read: bad kernel class or null output");
  drain(c);
  *total_ms = c->total_ms[kernel];
  *launches = c->launches[kernel];
  return TRX_OK;
}

// --------------------------------------------------------------------------
// chi^2 and its gradient (recompute mode)
// --------------------------------------------------------------------------
extern "C" trx_status trx_chi2_grad(trx_ctx* c, const trx_tables* t, const trx_batch* bt,
                                    const trx_bins* bins, trx_precision precision, const double* obs,
                                    const double* sigma, int32_t recompute, double* chi2, double* dT,
                                    double* dlog10vmr, double* dRp, double* depth_binned,
                                    int32_t* model_status) {
  if (!c) return TRX_E_INVALID_ARG;
  c->err.clear();
  trx_status s = check_batch(c, t, bt, precision);
  if (s != TRX_OK) return s;
  if (!bins) return set_err(c, TRX_E_INVALID_ARG, "trx_chi2_grad needs channels (bins)");
  if (bins->tables != t) return set_err(c, TRX_E_INVALID_ARG, "bins were made for other tables");
  if (!obs || !sigma || !chi2 || !dT || !dRp || !model_status || (t->dev.n_abs > 0 && !dlog10vmr))
    return set_err(c, TRX_E_INVALID_ARG, "trx_chi2_grad: a required pointer is null");
  if (!recompute)
    return set_err(c, TRX_E_UNSUPPORTED, "only the recompute mode of the gradient is built");
  if (t->dev.t_exp)
    return set_err(c, TRX_E_UNSUPPORTED, "the gradient of the exponential temperature scheme is not built");
  if (bt->log10_vmr_top)
    return set_err(c, TRX_E_UNSUPPORTED, "the gradient of two-layer profiles is not built");
  if (bt->max_layers > TRX_MAX_LAYERS_MFMA)
    return set_err(c, TRX_E_UNSUPPORTED, "the gradient supports at most %d layers", TRX_MAX_LAYERS_MFMA);
  hipSetDevice(c->device);
  return enqueue_chi2_grad(c, t, dev_batch(bt), bt->B, nullptr, bt->max_layers, bins, precision,
                           default_config(precision, bt->max_layers), c->ws, c->aws, c->sched, c->grad,
                           obs, sigma, chi2, dT, dlog10vmr, dRp, depth_binned, model_status);
}
