// Plans (a9): a fixed-capacity batched launch over a ragged live-point set,
// optionally replayed from a captured HIP graph, and the variant autotuner.
//
// The graph holds the whole launch sequence of trx_forward with the kernels
// reading the model count from device memory; before each replay a one-thread
// kernel writes the caller's B there, so a new B alone needs no new capture.
// Nothing in the captured sequence is a memset: the work counters of the
// persistent kernel are cleared by the ordering kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "trx_host.h"
#include "trx_internal.h"

using namespace trx;

struct trx_plan {
  trx_ctx* ctx = nullptr;
  const trx_tables* t = nullptr;
  const trx_bins* bins = nullptr;
  int B_max = 0, N_max = 0, precision = 0, flags = 0;
  RunConfig rc;
  std::string desc;
  // owned inputs (trx_plan_batch)
  std::vector<void*> owned;
  trx_batch own{};
  int32_t* B_dev = nullptr;
  DevBuf ws, aws, sched, grad, tune_binned, tune_status;
  // graph state
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  trx_batch cap_batch{};
  double* cap_native = nullptr;
  double* cap_binned = nullptr;
  int32_t* cap_status = nullptr;
  const void* cap_grad[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // emission plans: the stellar temperatures and angles (trx_plan_set_star)
  const double* T_star = nullptr;
  int n_mu = 0;
};

// Outputs (and, for gradient plans, observation inputs) of one launch.
struct PlanIO {
  double* native;
  double* binned;
  int32_t* status;
  const double* obs;
  const double* sigma;
  double* chi2;
  double* dT;
  double* dvmr;
  double* dRp;
};

namespace {

__global__ void k_set_count(int32_t* dst, int32_t v) { *dst = v; }

void describe(trx_plan* p) {
  char buf[160];
  snprintf(buf, sizeof buf, "persistent=%d group=%d spans=%d rbw=%d occ=%d", p->rc.persistent, p->rc.group,
           p->rc.span_group, p->rc.rbw, p->rc.occ);
  p->desc = buf;
}

void drop_graph(trx_plan* p) {
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

bool same_batch(const trx_batch& a, const trx_batch& b) {
  return a.max_layers == b.max_layers && a.n_layers == b.n_layers && a.layer_off == b.layer_off &&
         a.T_K == b.T_K && a.p_bot_Pa == b.p_bot_Pa && a.p_top_Pa == b.p_top_Pa &&
         a.log10_vmr == b.log10_vmr && a.Rp_m == b.Rp_m && a.Rs_m == b.Rs_m && a.GM_m3s2 == b.GM_m3s2 &&
         a.wn_lo == b.wn_lo && a.wn_hi == b.wn_hi && a.he_h2_ratio == b.he_h2_ratio && a.k_B == b.k_B &&
         a.amu_kg == b.amu_kg && a.gravity == b.gravity && a.cloud_sigma_m2 == b.cloud_sigma_m2 &&
         a.cloud_p_top_Pa == b.cloud_p_top_Pa && a.cloud_p_bottom_Pa == b.cloud_p_bottom_Pa &&
         a.log10_vmr_top == b.log10_vmr_top && a.vmr_switch_Pa == b.vmr_switch_Pa;
}

// The launch sequence of one plan run on the context's current stream.
// B_dev != null: kernels size their work from *B_dev (graph capture, grid
// sized for B_max); otherwise from B.
trx_status enqueue(trx_plan* p, const trx_batch* bt, int B, const int32_t* B_dev, const RunConfig& rc,
                   double* native, double* binned, int32_t* status) {
  const EmissionIn em{p->T_star, p->n_mu};
  return enqueue_forward(p->ctx, p->t, dev_batch(bt), B, B_dev, p->N_max, p->bins, p->precision, rc,
                         (uint8_t*)p->ws.ptr, p->aws.ptr, SchedBufs::carve(p->sched.ptr, p->B_max), native,
                         binned, status, false, nullptr, (p->flags & TRX_PLAN_EMISSION) ? &em : nullptr,
                         (p->flags & TRX_PLAN_TWO_LAYER) != 0);
}

trx_status enqueue_io(trx_plan* p, const trx_batch* bt, int B, const int32_t* B_dev, const RunConfig& rc,
                      const PlanIO& io) {
  if (!(p->flags & TRX_PLAN_GRAD)) return enqueue(p, bt, B, B_dev, rc, io.native, io.binned, io.status);
  return enqueue_chi2_grad(p->ctx, p->t, dev_batch(bt), B, B_dev, p->N_max, p->bins, p->precision, rc, p->ws,
                           p->aws, p->sched, p->grad, io.obs, io.sigma, io.chi2, io.dT, io.dvmr, io.dRp,
                           io.binned, io.status, false);
}

trx_status check_launch(trx_plan* p, const trx_batch* bt, double* binned, const int32_t* status,
                        bool need_status) {
  trx_ctx* c = p->ctx;
  trx_status s = check_batch(c, p->t, bt, p->precision);
  if (s != TRX_OK) return s;
  if (bt->B > p->B_max) return set_err(c, TRX_E_INVALID_ARG, "batch.B %d exceeds the plan's B_max %d", bt->B, p->B_max);
  if (bt->max_layers > p->N_max)
    return set_err(c, TRX_E_INVALID_ARG, "batch.max_layers %d exceeds the plan's N_max %d", bt->max_layers, p->N_max);
  if (need_status && !status) return set_err(c, TRX_E_INVALID_ARG, "model_status is required");
  if (binned && !p->bins) return set_err(c, TRX_E_INVALID_ARG, "depth_binned requires a plan made with bins");
  if ((p->flags & TRX_PLAN_EMISSION) && !p->T_star)
    return set_err(c, TRX_E_INVALID_ARG, "an emission plan needs its star (trx_plan_set_star) before a launch");
  if (bt->log10_vmr_top && !(p->flags & TRX_PLAN_TWO_LAYER))
    return set_err(c, TRX_E_INVALID_ARG, "a batch with two-layer profiles needs a TRX_PLAN_TWO_LAYER plan");
  return TRX_OK;
}

// ---- tiny flat JSON object of strings: {"key": "value", ...} -------------
std::map<std::string, std::string> read_cache(const char* path) {
  std::map<std::string, std::string> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  std::vector<std::string> toks;
  for (size_t i = 0; i < s.size(); ++i) {
    if (s[i] != '"') continue;
    std::string tok;
    for (++i; i < s.size() && s[i] != '"'; ++i) {
      if (s[i] == '\\' && i + 1 < s.size()) ++i;
      tok.push_back(s[i]);
    }
    toks.push_back(tok);
  }
  for (size_t i = 0; i + 1 < toks.size(); i += 2) m[toks[i]] = toks[i + 1];
  return m;
}

bool write_cache(const char* path, const std::map<std::string, std::string>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "{\n";
    size_t k = 0;
    for (auto& kv : m) f << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++k < m.size() ? ",\n" : "\n");
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

int bucket(int v) {
  int b = 1;
  while (b < v) b <<= 1;
  return b;
}

const char* prec_name(int p) {
  switch (p) {
    case TRX_FP64: return "fp64";
    case TRX_FP32: return "fp32";
    case TRX_BF16_SPLIT2: return "bf16x2";
    default: return "bf16x3";
  }
}

// Why a parsed variant does not fit the plan, or null.
const char* variant_unfit(const trx_plan* p, const RunConfig& rc) {
  const int nrb = (p->N_max + 31) / 32;
  if (rc.rbw == 1 && nrb > 4) return "one ray block per wave takes at most 128 layers";
  if (rc.occ == 4 && (p->precision == TRX_FP64 || !rc.persistent ||
                      (p->flags & (TRX_PLAN_EMISSION | TRX_PLAN_GRAD | TRX_PLAN_TWO_LAYER)) || p->t->dev.t_exp))
    return "the four-workgroup build is the persistent transmission kernel of one-chemistry layouts";
  return nullptr;
}

bool parse_variant(const char* v, RunConfig& rc) {
  RunConfig r = rc;
  std::istringstream ss(v ? v : "");
  std::string kv;
  while (ss >> kv) {
    const size_t eq = kv.find('=');
    if (eq == std::string::npos) return false;
    const std::string k = kv.substr(0, eq);
    char* end = nullptr;
    const long x = strtol(kv.c_str() + eq + 1, &end, 10);
    if (*end != '\0') return false;
    if (k == "persistent" && (x == 0 || x == 1)) r.persistent = (int)x;
    else if (k == "group" && x >= 0 && x <= (1 << 24)) r.group = (int)x;
    else if (k == "spans" && x >= 1 && x <= 64) r.span_group = (int)x;
    else if (k == "rbw" && x >= 0 && x <= 2) r.rbw = (int)x;
    else if (k == "occ" && (x == 3 || x == 4)) r.occ = (int)x;
    else return false;
  }
  rc = r;
  return true;
}

}  // namespace

extern "C" trx_status trx_plan_create(trx_ctx* c, const trx_tables* t, const trx_bins* bins, int32_t B_max,
                                      int32_t N_max, trx_precision precision, int32_t flags, trx_plan** out) {
  if (!c) return TRX_E_INVALID_ARG;
  c->err.clear();
  if (!out) return set_err(c, TRX_E_INVALID_ARG, "trx_plan_create: null output");
  *out = nullptr;
  if (!t || t->ctx != c) return set_err(c, TRX_E_INVALID_ARG, "tables are null or belong to another context");
  if (bins && bins->tables != t) return set_err(c, TRX_E_INVALID_ARG, "bins were made for other tables");
  if (precision < TRX_FP64 || precision > TRX_BF16_SPLIT3)
    return set_err(c, TRX_E_INVALID_ARG, "unknown precision %d", (int)precision);
  if (B_max < 1) return set_err(c, TRX_E_INVALID_ARG, "B_max must be >= 1");
  const int limit = precision == TRX_FP64 ? TRX_MAX_LAYERS_FP64 : TRX_MAX_LAYERS_MFMA;
  if (N_max < 2) return set_err(c, TRX_E_INVALID_ARG, "N_max must be >= 2");
  if (N_max > limit) return set_err(c, TRX_E_UNSUPPORTED, "N_max %d exceeds %d for this precision", N_max, limit);
  if (flags & ~(TRX_PLAN_GRAPH | TRX_PLAN_PERSISTENT | TRX_PLAN_GRAD | TRX_PLAN_EMISSION | TRX_PLAN_TWO_LAYER))
    return set_err(c, TRX_E_INVALID_ARG, "unknown plan flags 0x%x", flags);
  const bool grad = (flags & TRX_PLAN_GRAD) != 0;
  const bool emission = (flags & TRX_PLAN_EMISSION) != 0;
  const bool two_layer = (flags & TRX_PLAN_TWO_LAYER) != 0;
  if (grad && two_layer) return set_err(c, TRX_E_UNSUPPORTED, "the gradient of two-layer profiles is not built");
  if (two_layer && precision == TRX_FP64 && N_max > TRX_MAX_LAYERS_MFMA)
    return set_err(c, TRX_E_UNSUPPORTED, "two-layer profiles take at most %d layers in TRX_FP64",
                   TRX_MAX_LAYERS_MFMA);
  if (grad && emission) return set_err(c, TRX_E_UNSUPPORTED, "the gradient of the emission model is not built");
  if (emission && precision == TRX_FP64 && N_max > TRX_MAX_LAYERS_MFMA)
    return set_err(c, TRX_E_UNSUPPORTED, "emission takes at most %d layers", TRX_MAX_LAYERS_MFMA);
  if (grad && t->dev.t_exp)
    return set_err(c, TRX_E_UNSUPPORTED, "the gradient of the exponential temperature scheme is not built");
  if (grad && !bins) return set_err(c, TRX_E_INVALID_ARG, "gradient plans need channels (bins)");
  if (grad && N_max > TRX_MAX_LAYERS_MFMA)
    return set_err(c, TRX_E_UNSUPPORTED, "the gradient supports at most %d layers", TRX_MAX_LAYERS_MFMA);
  hipSetDevice(c->device);
  trx_plan* p = new trx_plan();
  p->ctx = c; p->t = t; p->bins = bins;
  p->B_max = B_max; p->N_max = N_max; p->precision = precision; p->flags = flags;
  p->rc = default_config(precision, N_max);
  if (!(flags & TRX_PLAN_PERSISTENT)) p->rc.persistent = 0;
  describe(p);
  auto fail = [&](trx_status s) { trx_plan_destroy(p); return s; };
  const Layout L = make_layout(N_max, precision, grad, t->dev, emission, two_layer);
  trx_status s;
  if ((s = ensure_buffer(c, p->ws, (size_t)B_max * L.slab, "plan workspace")) != TRX_OK) return fail(s);
  if (grad && (s = ensure_buffer(c, p->grad, grad_scratch_bytes(B_max, t->dev.n_wn, bins->n_ch, L.NP),
                                 "plan workspace")) != TRX_OK)
    return fail(s);
  const size_t esz = (precision == TRX_FP64 || emission) ? 8 : 4;
  if ((s = ensure_buffer(c, p->aws, (size_t)B_max * t->dev.n_wn * esz, "plan workspace")) != TRX_OK)
    return fail(s);
  if ((s = ensure_buffer(c, p->sched, SchedBufs::bytes(B_max), "plan workspace")) != TRX_OK) return fail(s);
  hipError_t e = hipSuccess;
  auto take = [&](size_t bytes) -> void* {
    void* d = nullptr;
    if (e != hipSuccess) return nullptr;
    e = hipMalloc(&d, std::max(bytes, (size_t)8));
    if (e != hipSuccess) return nullptr;
    p->owned.push_back(d);
    return d;
  };
  trx_batch& b = p->own;
  b.B = B_max;
  b.max_layers = N_max;
  b.n_layers = (int32_t*)take(4 * (size_t)B_max);
  b.layer_off = (int64_t*)take(8 * ((size_t)B_max + 1));
  b.T_K = (double*)take(8 * (size_t)B_max * N_max);
  b.p_bot_Pa = (double*)take(8 * (size_t)B_max);
  b.p_top_Pa = (double*)take(8 * (size_t)B_max);
  b.log10_vmr = (double*)take(8 * (size_t)B_max * std::max(t->dev.n_abs, 1));
  b.Rp_m = (double*)take(8 * (size_t)B_max);
  b.Rs_m = (double*)take(8 * (size_t)B_max);
  b.GM_m3s2 = (double*)take(8 * (size_t)B_max);
  b.wn_lo = (int32_t*)take(4 * (size_t)B_max);
  b.wn_hi = (int32_t*)take(4 * (size_t)B_max);
  b.he_h2_ratio = 0.17;
  b.k_B = 1.380649e-23;
  b.amu_kg = 1.66053906660e-27;
  b.gravity = 0;
  // cloud decks: zero cross-sections (no decks) until the caller writes them
  b.cloud_sigma_m2 = (double*)take(8 * (size_t)B_max);
  b.cloud_p_top_Pa = (double*)take(8 * (size_t)B_max);
  b.cloud_p_bottom_Pa = (double*)take(8 * (size_t)B_max);
  // two-layer plans: top values and switch pressures; until the caller
  // writes them, a switch far below every layer (surface values everywhere)
  b.log10_vmr_top = nullptr;
  b.vmr_switch_Pa = nullptr;
  if (two_layer) {
    const size_t n = (size_t)B_max * std::max(t->dev.n_abs, 1);
    b.log10_vmr_top = (double*)take(8 * n);
    b.vmr_switch_Pa = (double*)take(8 * n);
    if (e == hipSuccess) e = hipMemset((void*)b.log10_vmr_top, 0, 8 * n);
    if (e == hipSuccess) {
      std::vector<double> low(n, 1e-300);
      e = hipMemcpy((void*)b.vmr_switch_Pa, low.data(), 8 * n, hipMemcpyHostToDevice);
    }
  }
  p->B_dev = (int32_t*)take(4);
  if (e == hipSuccess) e = hipMemset((void*)b.cloud_sigma_m2, 0, 8 * (size_t)B_max);
  if (e == hipSuccess) e = hipMemset((void*)b.cloud_p_top_Pa, 0, 8 * (size_t)B_max);
  if (e == hipSuccess) e = hipMemset((void*)b.cloud_p_bottom_Pa, 0, 8 * (size_t)B_max);
  if (e != hipSuccess) return fail(hip_err(c, e, "trx_plan_create"));
  if (flags & TRX_PLAN_GRAPH) {
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_err(c, e, "trx_plan_create"));
  }
  *out = p;
  return TRX_OK;
}

extern "C" trx_status trx_plan_destroy(trx_plan* p) {
  if (!p) return TRX_E_INVALID_ARG;
  trx_ctx* c = p->ctx;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  drop_graph(p);
  if (p->cap) hipStreamDestroy(p->cap);
  for (DevBuf* b : {&p->ws, &p->aws, &p->sched, &p->grad, &p->tune_binned, &p->tune_status})
    if (b->ptr) hipFree(b->ptr);
  for (void* d : p->owned) hipFree(d);
  delete p;
  return TRX_OK;
}

extern "C" trx_status trx_plan_batch(trx_plan* p, trx_batch* out) {
  if (!p) return TRX_E_INVALID_ARG;
  if (!out) return set_err(p->ctx, TRX_E_INVALID_ARG, "trx_plan_batch: null output");
  *out = p->own;
  return TRX_OK;
}

extern "C" trx_status trx_plan_launch(trx_plan* p, const trx_batch* bt, double* native, double* binned,
                                      int32_t* status, const double* obs, const double* sigma, double* chi2,
                                      double* dT, double* dlog10vmr, double* dRp) {
  if (!p) return TRX_E_INVALID_ARG;
  trx_ctx* c = p->ctx;
  c->err.clear();
  const bool grad = (p->flags & TRX_PLAN_GRAD) != 0;
  if (!grad && (obs || sigma || chi2 || dT || dlog10vmr || dRp))
    return set_err(c, TRX_E_INVALID_ARG, "gradient outputs need a TRX_PLAN_GRAD plan");
  if (grad && (!obs || !sigma || !chi2 || !dT || !dRp || (p->t->dev.n_abs > 0 && !dlog10vmr)))
    return set_err(c, TRX_E_INVALID_ARG, "a gradient plan needs obs, sigma, chi2, dT, dlog10vmr and dRp");
  if (grad && native)
    return set_err(c, TRX_E_INVALID_ARG, "gradient plans do not write the native depth");
  trx_status s = check_launch(p, bt, binned, status, true);
  if (s != TRX_OK) return s;
  hipSetDevice(c->device);
  const PlanIO io{native, binned, status, obs, sigma, chi2, dT, dlog10vmr, dRp};
  // eager launches for plans without a graph, and while profiling (the
  // per-kernel events cannot sit between the nodes of a replayed graph)
  if (!(p->flags & TRX_PLAN_GRAPH) || c->profile) return enqueue_io(p, bt, bt->B, nullptr, p->rc, io);

  const void* gio[6] = {obs, sigma, chi2, dT, dlog10vmr, dRp};
  bool same = p->exec && same_batch(*bt, p->cap_batch) && native == p->cap_native && binned == p->cap_binned &&
              status == p->cap_status;
  for (int k = 0; k < 6 && same; ++k) same = gio[k] == p->cap_grad[k];
  if (!same) {
    drop_graph(p);
    hipStream_t user = c->stream;
    c->stream = p->cap;
    c->capturing = true;
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      c->stream = user;
      c->capturing = false;
      return hip_err(c, e, "graph capture");
    }
    s = enqueue_io(p, bt, p->B_max, p->B_dev, p->rc, io);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap, &g);
    c->stream = user;
    c->capturing = false;
    if (s != TRX_OK) {
      if (g) hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_err(c, e, "graph capture");
    p->graph = g;
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(p);
      return hip_err(c, e, "graph instantiate");
    }
    p->cap_batch = *bt;
    p->cap_native = native;
    p->cap_binned = binned;
    p->cap_status = status;
    for (int k = 0; k < 6; ++k) p->cap_grad[k] = gio[k];
  }
  hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, c->stream, p->B_dev, bt->B);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "trx_plan_launch");
  e = hipGraphLaunch(p->exec, c->stream);
  if (e != hipSuccess) return hip_err(c, e, "graph launch");
  return TRX_OK;
}

extern "C" trx_status trx_plan_set_star(trx_plan* p, const double* T_star_K, int32_t n_mu) {
  if (!p) return TRX_E_INVALID_ARG;
  trx_ctx* c = p->ctx;
  c->err.clear();
  if (!(p->flags & TRX_PLAN_EMISSION)) return set_err(c, TRX_E_INVALID_ARG, "not an emission plan");
  trx_status s = check_emission(c, p->precision, p->N_max, T_star_K, n_mu);
  if (s != TRX_OK) return s;
  if (T_star_K != p->T_star || n_mu != p->n_mu) drop_graph(p);
  p->T_star = T_star_K;
  p->n_mu = n_mu;
  return TRX_OK;
}

extern "C" trx_status trx_plan_set_variant(trx_plan* p, const char* v) {
  if (!p) return TRX_E_INVALID_ARG;
  RunConfig rc = p->rc;
  if (!parse_variant(v, rc)) return set_err(p->ctx, TRX_E_INVALID_ARG, "bad variant string '%s'", v ? v : "");
  if (rc.persistent && !(p->flags & TRX_PLAN_PERSISTENT))
    return set_err(p->ctx, TRX_E_INVALID_ARG, "plan was made without TRX_PLAN_PERSISTENT");
  if (const char* why = variant_unfit(p, rc)) return set_err(p->ctx, TRX_E_INVALID_ARG, "variant '%s': %s", v, why);
  p->rc = rc;
  drop_graph(p);
  describe(p);
  return TRX_OK;
}

extern "C" trx_status trx_autotune(trx_plan* p, const trx_batch* bt, const char* cache_json) {
  if (!p) return TRX_E_INVALID_ARG;
  trx_ctx* c = p->ctx;
  c->err.clear();
  trx_status s = check_launch(p, bt, nullptr, nullptr, false);
  if (s != TRX_OK) return s;
  hipSetDevice(c->device);
  char key[256];
  snprintf(key, sizeof key, "%s/%s/B%d/N%d/W%d/abs%d/flags%d", c->arch, prec_name(p->precision), bucket(p->B_max),
           bucket(p->N_max), p->t->dev.n_wn, p->t->dev.n_abs,
           p->flags & (TRX_PLAN_PERSISTENT | TRX_PLAN_EMISSION | TRX_PLAN_TWO_LAYER));
  std::map<std::string, std::string> cache;
  if (cache_json) {
    cache = read_cache(cache_json);
    auto it = cache.find(key);
    if (it != cache.end()) {
      RunConfig rc = p->rc;
      if (parse_variant(it->second.c_str(), rc) && (!rc.persistent || (p->flags & TRX_PLAN_PERSISTENT)) &&
          !variant_unfit(p, rc)) {
        p->rc = rc;
        drop_graph(p);
        describe(p);
        return TRX_OK;
      }
    }
  }
  // the search: span groups x (one workgroup per item, or the persistent
  // queues in span-major order or model groups of 16 and 64); then, around
  // the best of those, the tile layouts: one or two ray blocks per wave and
  // the four-workgroup build (two ray blocks per wave in two passes)
  std::vector<RunConfig> cand;
  RunConfig base = default_config(p->precision, p->N_max);
  if (p->precision == TRX_FP64) {
    base.persistent = 0;
    for (int sg : {1, 2, 4, 8}) {
      RunConfig r = base;
      r.span_group = sg;
      cand.push_back(r);
    }
  } else {
    for (int sg : {1, 2, 4, 8}) {
      RunConfig r = base;
      r.span_group = sg;
      r.persistent = 0;
      cand.push_back(r);
      if (p->flags & TRX_PLAN_PERSISTENT) {
        for (int g : {0, 64, 16}) {
          r.persistent = 1;
          r.group = g;
          cand.push_back(r);
        }
      }
    }
  }
  if ((s = ensure_buffer(c, p->tune_binned, p->bins ? (size_t)bt->B * p->bins->n_ch * 8 : 8, "autotune")) != TRX_OK)
    return s;
  if ((s = ensure_buffer(c, p->tune_status, (size_t)bt->B * 4, "autotune")) != TRX_OK) return s;
  double* binned = p->bins ? (double*)p->tune_binned.ptr : nullptr;
  int32_t* status = (int32_t*)p->tune_status.ptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  double best = 1e300;
  RunConfig pick = cand[0];
  auto time_all = [&](const std::vector<RunConfig>& cs) {
    for (const RunConfig& rc : cs) {
      if ((s = enqueue(p, bt, bt->B, nullptr, rc, nullptr, binned, status)) != TRX_OK) return;
      hipEventRecord(e0, c->stream);
      for (int r = 0; r < 3 && s == TRX_OK; ++r) s = enqueue(p, bt, bt->B, nullptr, rc, nullptr, binned, status);
      hipEventRecord(e1, c->stream);
      if (s != TRX_OK) return;
      hipError_t e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) { s = hip_err(c, e, "autotune"); return; }
      if (ms < best) { best = ms; pick = rc; }
    }
  };
  time_all(cand);
  if (s == TRX_OK && p->precision != TRX_FP64) {
    std::vector<RunConfig> tiles;
    for (int rbw : {1, 2})
      for (int occ : {3, 4}) {
        RunConfig r = pick;
        r.rbw = rbw;
        r.occ = occ;
        const bool same = (r.rbw == pick.rbw || (pick.rbw == 0 && r.rbw == ((p->N_max + 31) / 32 <= 4 ? 1 : 2))) &&
                          r.occ == pick.occ;
        if (!same && !variant_unfit(p, r)) tiles.push_back(r);
      }
    time_all(tiles);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (s != TRX_OK) return s;
  p->rc = pick;
  drop_graph(p);
  describe(p);
  if (cache_json) {
    cache[key] = p->desc;
    if (!write_cache(cache_json, cache))
      return set_err(c, TRX_E_INVALID_ARG, "cannot write autotune cache '%s'", cache_json);
  }
  return TRX_OK;
}

extern "C" const char* trx_plan_describe(const trx_plan* p) { return p ? p->desc.c_str() : ""; }
