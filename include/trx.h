/*
 * trx.h - C ABI of the MI355X transmission forward-model library.
 *
 * The library evaluates the transit-depth forward model of TauREx 3
 * (Al-Refaie et al., arXiv:1912.07759) on one AMD Instinct MI355X (gfx950):
 *
 *   a1  pressure grid, free chemistry with H2/He fill, mean molecular weight
 *       (Pressure Profiles and Chemistry subsections);
 *   a2  hydrostatic altitude recursion (Forward Models section, altitude
 *       equation), FP64 on the GPU;
 *   a3  chord path-length triangle and annulus weights (transit-depth
 *       integrals of the Forward Models section), FP64 on the GPU;
 *   a4  per-layer absorption coefficient: bilinear (T, log10 P) interpolation
 *       of cross-section tables, Rayleigh and CIA, weighted by mixing ratio
 *       and number density and summed before the path integral
 *       (equations opt_dpth, cia_opt_dpth, contrib; Opacities section);
 *   a5  optical depth tau[ray, wn] = sum_k dl[ray, k] kappa[k, wn];
 *   a6  depth D = (Rp^2 + sum_j A_j (1 - exp(-tau_j))) / Rs^2;
 *   a7  binning to channels with overlap weights (Binning subsection);
 *   a8  chi^2 against an observation and its gradient with respect to the
 *       per-layer temperatures, log10 mixing ratios and Rp;
 *   a9  a batched form over a ragged live-point set run as one persistent,
 *       graph-captured launch (the plan API);
 *   and the emission (eclipse) spectrum of the same atmospheres (Forward
 *   Models section, emission intensity and its Gauss-Legendre flux).
 *
 * Conventions
 *  - Units are SI (Forward Models section) except: wavenumbers in cm^-1,
 *    cross-sections in cm^2/molecule, CIA in cm^5/molecule^2, masses in amu.
 *  - All profile arrays are bottom first (layer 0 at the highest pressure,
 *    where the planet radius is defined).
 *  - Host pointers are read during the call only.  Device pointers are
 *    borrowed until the work enqueued on the context's stream has finished;
 *    the caller owns every input and output buffer.
 *  - Errors: a call that returns a status other than TRX_OK has enqueued no
 *    work; trx_last_error() then returns a message.  Out-of-range T or P is
 *    not an error (the tables clamp, Opacities section).  An invalid model
 *    inside a batch never fails the call: its model_status entry is set
 *    (bit mask below) and its outputs are NaN, so a sampler can assign it
 *    the minimum likelihood (Model Rejection subsection).
 */
#ifndef TRX_H
#define TRX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct trx_ctx trx_ctx;
typedef struct trx_tables trx_tables;
typedef struct trx_bins trx_bins;
typedef struct trx_plan trx_plan;

typedef enum {
  TRX_OK = 0,
  TRX_E_INVALID_ARG = 1,   /* bad pointer, size, grid or handle */
  TRX_E_OUT_OF_MEMORY = 2, /* device allocation failed */
  TRX_E_DEVICE = 3,        /* a HIP runtime call failed */
  TRX_E_UNSUPPORTED = 4    /* valid request outside what is built */
} trx_status;

/* Arithmetic of the opacity, optical-depth and depth steps.  Pressure grid,
 * chemistry, altitudes and path lengths are FP64 in every mode, and so are
 * the per-model products P = dl x (interpolation weights) that the matrix
 * cores contract with the mixed cross-sections.
 *  TRX_FP64         FP64 tables, opacity, contraction and depth (reference).
 *  TRX_FP32         FP32 tables and mixing, FP32 matrix-core contraction with
 *                   P split into FP32 hi + lo parts; the annulus terms
 *                   A_j (1 - e^-tau_j) summed in FP32, added to (Rp/Rs)^2 in
 *                   FP64 (so for the two modes below).
 *  TRX_BF16_SPLIT2  FP32 mixing; P and the mixed cross-sections each split
 *                   into two bf16 parts, three bf16 matrix-core products
 *                   (hi*hi + hi*lo + lo*hi) with FP32 accumulation.
 *  TRX_BF16_SPLIT3  three bf16 parts each, six products (~FP32 accuracy). */
typedef enum {
  TRX_FP64 = 0,
  TRX_FP32 = 1,
  TRX_BF16_SPLIT2 = 2,
  TRX_BF16_SPLIT3 = 3
} trx_precision;

/* model_status bits */
enum {
  TRX_MODEL_OK = 0,
  TRX_MODEL_BAD_CHEMISTRY = 1, /* sum of absorber mixing ratios >= 1, or non-finite */
  TRX_MODEL_BAD_PROFILE = 2,   /* n_layers out of range, T <= 0, Rp/Rs/GM <= 0,
                                  p_bot <= p_top, non-finite input */
  TRX_MODEL_BAD_WINDOW = 4,    /* window empty or outside the grid */
  TRX_MODEL_NONFINITE = 8,     /* a non-finite value appeared in the outputs */
  TRX_MODEL_GRAD_UNSUPPORTED = 16, /* trx_chi2_grad: the model has more distinct
                                     table corners and CIA nodes than the
                                     gradient supports (256); its gradient
                                     outputs are NaN */
  TRX_MODEL_UNSUPPORTED = 32   /* two-layer profiles that cut the model's layers
                                  into more than TRX_MAX_REGIMES runs of one
                                  chemistry, or more than 1024 opacity slots
                                  in all; its outputs are NaN */
};

/* Limits of the library. */
#define TRX_MAX_LAYERS_FP64 1024 /* TRX_FP64 */
#define TRX_MAX_LAYERS_MFMA 224  /* the matrix-core modes */
#define TRX_MAX_ABSORBERS 32
#define TRX_MAX_CIA 8
#define TRX_MAX_TGRID 128
#define TRX_MAX_PGRID 128
#define TRX_MAX_MU 16           /* Gauss-Legendre angles of the emission flux */
#define TRX_MAX_REGIMES 4       /* runs of one chemistry per model (two-layer profiles) */

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`; work is enqueued on the default
 * stream until trx_set_stream is called. */
trx_status trx_create(int device, trx_ctx** out);
trx_status trx_destroy(trx_ctx* ctx);
/* Message of the last failing call on this context ("" if none).  The
 * string is owned by the context and valid until its next call. */
const char* trx_last_error(const trx_ctx* ctx);
/* Enqueue subsequent work on `hip_stream` (a hipStream_t; NULL = default). */
trx_status trx_set_stream(trx_ctx* ctx, void* hip_stream);
/* Block until all work enqueued by this context has finished. */
trx_status trx_synchronize(trx_ctx* ctx);

/* ---- opacity tables (Opacities section) ------------------------------- */

/* How the cross-sections are interpolated in temperature between the two
 * bracketing grid temperatures T1 < T2 (Opacities section); either way the
 * result is then interpolated linearly in log10 P, and CIA is linear in T.
 *  TRX_T_LINEAR  sigma = sigma1 + (sigma2 - sigma1)(T - T1)/(T2 - T1).
 *  TRX_T_EXP     sigma = a e^{-b/T} through both nodes, i.e.
 *                sigma1 (sigma2/sigma1)^u with u = (1/T - 1/T1)/(1/T2 - 1/T1);
 *                where sigma1 or sigma2 is not positive that point takes
 *                the linear scheme.  Out-of-range T clamps to the edge
 *                node as in the linear scheme.  The device keeps a second
 *                FP32 table of (sigma, log2 of the ratio to the next
 *                temperature node) pairs, twice the FP32 table's size.
 *                Not differentiated: trx_chi2_grad and gradient plans
 *                return TRX_E_UNSUPPORTED for such tables. */
typedef enum {
  TRX_T_LINEAR = 0,
  TRX_T_EXP = 1
} trx_t_interp;

/* All pointers are HOST pointers, read during the call.  Every table lives
 * on one shared wavenumber grid (the paper's "native" grid, resampling
 * done by the caller).  Species ids: 0..n_abs-1 absorbers, n_abs = H2,
 * n_abs+1 = He. */
typedef struct {
  int32_t n_wn;                 /* >= 2 */
  const double* wn_cm1;         /* [n_wn] strictly increasing */
  int32_t n_T;                  /* 2..TRX_MAX_TGRID */
  const double* T_K;            /* [n_T] strictly increasing */
  int32_t n_P;                  /* 2..TRX_MAX_PGRID */
  const double* log10P_Pa;      /* [n_P] strictly increasing */
  int32_t n_abs;                /* 0..TRX_MAX_ABSORBERS */
  const double* xsec_cm2;       /* [n_abs][n_T][n_P][n_wn] */
  const double* abs_mass_amu;   /* [n_abs] */
  double h2_mass_amu;
  double he_mass_amu;
  int32_t n_cia;                /* 0..TRX_MAX_CIA */
  int32_t n_Tcia;               /* 2..TRX_MAX_TGRID if n_cia > 0 */
  const double* Tcia_K;         /* [n_Tcia] strictly increasing */
  const double* cia_cm5;        /* [n_cia][n_Tcia][n_wn] */
  const int32_t* cia_pair;      /* [n_cia][2] species ids */
  const double* rayleigh_cm2;   /* [n_abs + 2][n_wn], or NULL for none */
  int32_t t_interp;             /* trx_t_interp: scheme of the cross-sections in T */
} trx_tables_desc;

/* Copy the tables to the device (FP64 and FP32 copies, wavenumber
 * contiguous).  The handle owns the device memory.  Returns
 * TRX_E_INVALID_ARG for a malformed description (t_interp included) and
 * TRX_E_UNSUPPORTED when the FP32 table of one absorber (n_T n_P n_wn
 * values; twice that for TRX_T_EXP), of one CIA pair (n_Tcia n_wn) or the
 * Rayleigh table ((n_abs + 2) n_wn) reaches 2 GiB: the matrix-core kernels
 * address a table row with a 32-bit byte offset. */
trx_status trx_tables_create(trx_ctx* ctx, const trx_tables_desc* desc, trx_tables** out);
trx_status trx_tables_destroy(trx_tables* t);

/* ---- channels (Binning subsection) ------------------------------------ */

/* n_ch channels [lo_c, hi_c) in cm^-1 (HOST pointers).  Native bin edges
 * are the midpoints of the table grid, end bins mirrored; the weight of
 * native point i in channel c is the overlap of the two bins divided by
 * the native bin width; a channel's value is the weighted mean over the
 * native points of a model's window (NaN if it has none). */
trx_status trx_bins_create(trx_ctx* ctx, const trx_tables* t, int32_t n_ch,
                           const double* lo_cm1, const double* hi_cm1, trx_bins** out);
trx_status trx_bins_destroy(trx_bins* b);

/* ---- a batch of models ------------------------------------------------ */

/* B models with their own layer counts and wavenumber windows.  Array
 * pointers are DEVICE pointers; scalars are host values. */
typedef struct {
  int32_t B;                    /* >= 1 */
  int32_t max_layers;           /* host upper bound on n_layers[b] */
  const int32_t* n_layers;      /* [B] >= 2 */
  const int64_t* layer_off;     /* [B+1] offsets into T_K, layer_off[0] = 0 */
  const double* T_K;            /* [layer_off[B]] per-layer temperature */
  const double* p_bot_Pa;       /* [B] boundary pressure at the bottom */
  const double* p_top_Pa;       /* [B] boundary pressure at the top */
  const double* log10_vmr;      /* [B][n_abs] constant absorber profiles */
  const double* Rp_m;           /* [B] planet radius at z = 0 */
  const double* Rs_m;           /* [B] stellar radius */
  const double* GM_m3s2;        /* [B] planet G*M */
  const int32_t* wn_lo;         /* [B] window start index (inclusive) */
  const int32_t* wn_hi;         /* [B] window end index (exclusive) */
  double he_h2_ratio;           /* He/H2 volume ratio of the fill */
  double k_B;                   /* Boltzmann constant, J/K */
  double amu_kg;                /* atomic mass unit, kg */
  int32_t gravity;              /* 0: g = GM/(Rp+z)^2, 1: g = GM/Rp^2 */
  /* Optional flat-opacity cloud deck per model (equation clouds, Forward
   * Models section): the cross-section sigma (m^2 per molecule) times the
   * number density is added to the opacity of every layer whose centre
   * pressure lies between the two deck pressures (bounds included, in
   * either order), at every wavenumber.  All three NULL: no decks; else all
   * three set.  sigma = 0: no deck for that model; sigma = +INFINITY: a
   * fully opaque deck (every ray with a nonzero path through it is
   * blocked).  sigma < 0 or NaN, or (sigma > 0 and) a deck pressure that is
   * not finite and positive flags the model TRX_MODEL_BAD_PROFILE.  The
   * gradient treats the deck's layers as fixed: the deck pressures are not
   * differentiated (the deck is a step in P). */
  const double* cloud_sigma_m2;   /* [B] */
  const double* cloud_p_top_Pa;   /* [B] */
  const double* cloud_p_bottom_Pa;/* [B] */
  /* Optional two-layer mixing profiles (Chemistry subsection: the two-layer
   * profile with a surface and a top mixing ratio).  Absorber i of model b
   * has log10_vmr[b][i] at the layers whose centre pressure is at or above
   * vmr_switch_Pa[b][i] and log10_vmr_top[b][i] at the layers above (lower
   * pressure): a step, no smoothing.  The fill gases and the mean molecular
   * weight follow layer by layer (each altitude step takes the lower
   * layer's).  A constant gas has equal values (or a switch pressure
   * outside the model).  Both NULL: constant profiles; else both set.  A
   * switch pressure that is not finite and positive, a top value that is
   * not finite, or a layer whose absorbers sum to 1 or more flags
   * TRX_MODEL_BAD_CHEMISTRY; switches that cut a model's layers into more
   * than TRX_MAX_REGIMES runs flag TRX_MODEL_UNSUPPORTED.  Not
   * differentiated: trx_chi2_grad returns TRX_E_UNSUPPORTED; TRX_FP64 takes
   * at most TRX_MAX_LAYERS_MFMA layers with them. */
  const double* log10_vmr_top;    /* [B][n_abs] */
  const double* vmr_switch_Pa;    /* [B][n_abs] */
} trx_batch;

/* Forward model for every model of the batch.
 *  depth_native  DEVICE [B][n_wn] or NULL: native depth; only the entries
 *                inside each model's window are written.
 *  depth_binned  DEVICE [B][n_ch] or NULL (requires bins).
 *  model_status  DEVICE [B], required.
 *  tau           DEVICE [B][max_layers][n_wn] or NULL: the optical depth
 *                tau[b][j][i] of the chord at impact altitude z_j (ray j,
 *                j < n_layers[b]) at native point i, total of all
 *                contributions (equation tot_opt_dpth), written for the
 *                points of each model's window only; FP64 in TRX_FP64, the
 *                FP32 accumulator of the matrix product in the other modes.
 * Returns TRX_E_UNSUPPORTED if max_layers exceeds the mode's limit. */
trx_status trx_forward(trx_ctx* ctx, const trx_tables* t, const trx_batch* batch,
                       const trx_bins* bins, trx_precision precision,
                       double* depth_native, double* depth_binned, int32_t* model_status,
                       double* tau);

/* Emission forward model (Forward Models section: the emission intensity,
 * its N-point Gauss-Legendre flux and F_p/F_s = I/I_s (Rp/Rs)^2) of every
 * model of the batch: the same atmosphere and opacity as trx_forward (steps
 * a1-a4, cloud decks included), seen as a plane-parallel slab.
 *  - tau_l is the vertical optical depth from the top down to the bottom of
 *    shell l (the transmission shells: h_0 = 0, midpoints, h_N = z_{N-1});
 *    each shell emits the Planck intensity of its layer's temperature, the
 *    surface that of the bottom layer (the temperature at maximum pressure):
 *      I(mu) = B(T_0) e^{-tau_0/mu} + sum_l B(T_l) (e^{-tau_{l+1}/mu} - e^{-tau_l/mu});
 *  - flux ratio 2 sum_i w_i mu_i I(mu_i) / B(T_star) (Rp/Rs)^2 with the
 *    n_mu-point Gauss-Legendre nodes mu_i and weights w_i on [0, 1], so that
 *    an isothermal planet at T_star gives (Rp/Rs)^2; B is Planck's law per
 *    unit wavenumber (h, c exact SI; the batch's k_B).
 *  n_mu        1..TRX_MAX_MU angles.
 *  T_star_K    DEVICE [B] blackbody temperature of each model's star (a
 *              non-positive or non-finite one flags TRX_MODEL_BAD_PROFILE).
 *  fpfs_native DEVICE [B][n_wn] or NULL: F_p/F_s on the model's window.
 *  fpfs_binned DEVICE [B][n_ch] or NULL (requires bins), binned as depths.
 *  model_status DEVICE [B], required.
 * Returns TRX_E_UNSUPPORTED for TRX_FP64 batches of more than
 * TRX_MAX_LAYERS_MFMA layers.  No gradient of this model is built.  In the
 * FP32 and split-bf16 modes a planet whose flux is below ~1e-38 of the
 * star's at some wavenumber underflows to zero there. */
trx_status trx_emission(trx_ctx* ctx, const trx_tables* t, const trx_batch* batch, const trx_bins* bins,
                        trx_precision precision, int32_t n_mu, const double* T_star_K,
                        double* fpfs_native, double* fpfs_binned, int32_t* model_status);

/* Bytes of the fixed device array that trx_forward_noalloc works in. */
#define TRX_NOALLOC_SCRATCH_BYTES (64u << 20)

/* trx_forward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, outputs and errors as in trx_forward (without the optical-depth
 * output).  The call allocates and frees nothing: its workspace (per-model
 * slabs, the atmospheric depth per native point, the work order) is carved
 * from one fixed array of TRX_NOALLOC_SCRATCH_BYTES that each device holds
 * from its first trx_create until the process ends.  A batch needing more
 * (about 0.5 MB per 100-layer model on a 40000-point grid in the matrix-core
 * modes) returns TRX_E_UNSUPPORTED with the byte count in trx_last_error and
 * enqueues nothing: split it.  Every call on a device shares that device's
 * array and leaves the last call's contents in it; calls on one stream are
 * ordered, but calls whose work overlaps on one device (other streams, other
 * contexts, other threads) race and must not be issued. */
trx_status trx_forward_noalloc(trx_ctx* ctx, const trx_tables* t, const trx_batch* batch,
                               const trx_bins* bins, trx_precision precision,
                               double* depth_native, double* depth_binned, int32_t* model_status);

/* chi^2 = sum_c ((D_c - obs_c)/sigma_c)^2 and its gradient, per model.
 *  obs        DEVICE [B][n_ch]; sigma DEVICE [n_ch] (> 0).
 *  chi2       DEVICE [B]
 *  dT         DEVICE [layer_off[B]]   d chi2 / d T_l
 *  dlog10vmr  DEVICE [B][n_abs]       d chi2 / d log10 chi_i (fill gases
 *                                     follow the sum constraint)
 *  dRp        DEVICE [B]              d chi2 / d Rp
 *  depth_binned DEVICE [B][n_ch] or NULL
 *  recompute  1: the opacity and optical depth are recomputed in the
 *             backward pass instead of stored (the only mode built).
 * `precision` is the arithmetic of the forward pass, i.e. of the residual
 * D - obs, which near the optimum is at the noise level: there the matrix-
 * core modes take an accurate depth epilogue (each 1 - e^-tau_j to a few
 * FP32 units, the annulus sum in FP64), so that TRX_FP32 holds the gradient
 * to 1e-4 of the FP64 reference like TRX_FP64 (TRX_BF16_SPLIT2 keeps the
 * 16-bit rounding of the path x weight products: about 4e-5).  The
 * backward contractions take FP32 operands split into bf16 pieces (FP32
 * accuracy) and the layer-level adjoints are FP64.  Every sum runs in a
 * fixed order: the same call gives the same bits.  A model with more than 256
 * opacity slots (distinct table corners it interpolates from, plus CIA
 * temperature nodes) is flagged TRX_MODEL_GRAD_UNSUPPORTED with NaN
 * gradient outputs; above 128 its work items run the recompute of the
 * optical depth once per 128-slot chunk.
 * Derivatives at table nodes and under clamps are one-sided (the lower
 * bracket's slope; zero under a clamp).  The binned spectrum must cover
 * every channel in each model's window, else that model's chi2 is NaN.
 * Tables with t_interp = TRX_T_EXP, or a batch with two-layer profiles:
 * TRX_E_UNSUPPORTED. */
trx_status trx_chi2_grad(trx_ctx* ctx, const trx_tables* t, const trx_batch* batch,
                         const trx_bins* bins, trx_precision precision,
                         const double* obs, const double* sigma, int32_t recompute,
                         double* chi2, double* dT, double* dlog10vmr, double* dRp,
                         double* depth_binned, int32_t* model_status);

/* ---- plans: fixed-capacity batched launches (a9) ------------------------ */

/* Plan flags. */
enum {
  TRX_PLAN_GRAPH = 1,       /* replay the launch sequence from a HIP graph */
  TRX_PLAN_PERSISTENT = 2,  /* allow the persistent work-queue kernel */
  TRX_PLAN_GRAD = 4,        /* plan computes chi^2 and its gradient */
  TRX_PLAN_EMISSION = 8,    /* plan computes the emission spectrum (trx_emission);
                               the native and binned outputs hold F_p/F_s */
  TRX_PLAN_TWO_LAYER = 16   /* plan accepts batches with two-layer profiles (its
                               workspace holds the per-run chemistry); without
                               it such a batch is refused at launch */
};

/* A plan owns the workspace for up to B_max models of at most N_max layers
 * and, for TRX_PLAN_GRAPH, the captured HIP graph of one launch: geometry,
 * work ordering, opacity/optical depth/depth and binning (and the gradient
 * kernels for TRX_PLAN_GRAD).  It replaces the sampler-level parallelism
 * over live points (Parallel/MPI discussion of the Benchmarks section) by
 * one launch over the whole live-point set.  bins may be NULL (then no
 * binned output).  Creating a plan allocates; launching one does not.
 * TRX_PLAN_GRAD with TRX_T_EXP tables or with TRX_PLAN_TWO_LAYER:
 * TRX_E_UNSUPPORTED. */
trx_status trx_plan_create(trx_ctx* ctx, const trx_tables* t, const trx_bins* bins,
                           int32_t B_max, int32_t N_max, trx_precision precision,
                           int32_t flags, trx_plan** out);
trx_status trx_plan_destroy(trx_plan* p);
/* The star of a TRX_PLAN_EMISSION plan: DEVICE [B_max] temperatures
 * (borrowed by every later launch) and the number of Gauss-Legendre angles,
 * as in trx_emission.  Required before the first launch of such a plan. */
trx_status trx_plan_set_star(trx_plan* p, const double* T_star_K, int32_t n_mu);
/* Fill `out` with device input buffers owned by the plan (B = B_max,
 * max_layers = N_max, layer_off sized for B_max * N_max layers; default
 * constants He/H2 0.17, CODATA k_B and atomic mass unit, gravity 0; cloud
 * deck arrays zeroed at creation, i.e. no decks; for TRX_PLAN_TWO_LAYER
 * plans the two-layer arrays, their switch pressures at 1e-300 Pa at
 * creation, i.e. surface values everywhere, otherwise NULL).  Their use is
 * optional: any batch with B <= B_max and max_layers <= N_max can be
 * launched. */
trx_status trx_plan_batch(trx_plan* p, trx_batch* out);
/* Run the plan on `batch` (batch->B models).  Outputs as in trx_forward and
 * trx_chi2_grad; obs, sigma and the gradient outputs only for TRX_PLAN_GRAD
 * plans (NULL otherwise).  A graph plan captures its graph on the first
 * launch and again whenever an array pointer, output pointer or constant of
 * the call differs from the captured one; batch->B travels through device
 * memory, so a new B alone replays the same graph.  While trx_profile is
 * enabled the same kernels are launched one by one instead, so that each
 * is timed.  A TRX_PLAN_GRAD plan needs obs, sigma, chi2, dT, dlog10vmr,
 * dRp (as in trx_chi2_grad) and does not write depth_native (NULL). */
trx_status trx_plan_launch(trx_plan* p, const trx_batch* batch, double* depth_native,
                           double* depth_binned, int32_t* model_status,
                           const double* obs, const double* sigma, double* chi2,
                           double* dT, double* dlog10vmr, double* dRp);

/* ---- measurement --------------------------------------------------------- */

/* Kernel classes timed by trx_profile. */
enum {
  TRX_KERNEL_GEOMETRY = 0,  /* a1-a3: profiles, altitude, path lengths */
  TRX_KERNEL_FORWARD = 1,   /* a4-a6: opacity, optical depth, depth */
  TRX_KERNEL_BINNING = 2,   /* a7 */
  TRX_KERNEL_ADJOINT = 3,   /* a8: opacity/optical-depth adjoint */
  TRX_KERNEL_GEOM_ADJ = 4,  /* a8: geometry and altitude adjoint */
  TRX_KERNEL_SCHEDULE = 5,  /* a9: work ordering of the batched launch */
  TRX_KERNEL_CLASSES = 6
};

/* enable = 1: reset the totals and record a HIP event pair around every
 * later kernel launch of this context that is not part of a graph;
 * enable = 0: stop recording. */
trx_status trx_profile(trx_ctx* ctx, int32_t enable);
/* Wait for the recorded launches and return, for one kernel class, the
 * summed GPU time between its event pairs (ms) and the number of launches. */
trx_status trx_profile_read(trx_ctx* ctx, int32_t kernel, double* total_ms, int32_t* launches);

/* ---- tuning ------------------------------------------------------------ */

/* Choose the plan's kernel variant (persistent or one workgroup per item;
 * the model-group size of the persistent work order) for batches like
 * `batch`.  If cache_json names a file holding a choice for this device,
 * precision and shape bucket (B_max, N_max, grid size, absorbers), that
 * choice is taken without timing; otherwise every variant is run on `batch`
 * (outside any graph, outputs discarded), the fastest mean of three timed
 * runs is kept and, if cache_json is not NULL, written to the file (a flat
 * JSON object of strings).  Synchronises the context's stream. */
trx_status trx_autotune(trx_plan* p, const trx_batch* batch, const char* cache_json);
/* Set the variant directly from a string as returned by trx_plan_describe
 * ("persistent=1 group=0 spans=8"; unknown keys are an error). */
trx_status trx_plan_set_variant(trx_plan* p, const char* variant);
/* Current variant of a plan as a short printable string (owned by the
 * plan, valid until the next call on it). */
const char* trx_plan_describe(const trx_plan* p);

#ifdef __cplusplus
}
#endif
#endif /* TRX_H */
