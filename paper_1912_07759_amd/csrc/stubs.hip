// Entry points not built yet.
#include "trx_host.h"

extern "C" trx_status trx_chi2_grad(trx_ctx* c, const trx_tables*, const trx_batch*, const trx_bins*,
                                    trx_precision, const double*, const double*, int32_t, double*, double*,
                                    double*, double*, double*, int32_t*) {
  return trx::set_err(c, TRX_E_UNSUPPORTED, "trx_chi2_grad: not built");
}
extern "C" trx_status trx_plan_create(trx_ctx* c, const trx_tables*, const trx_bins*, int32_t, int32_t,
                                      trx_precision, int32_t, trx_plan** out) {
  if (out) *out = nullptr;
  return trx::set_err(c, TRX_E_UNSUPPORTED, "trx_plan_create: not built");
}
extern "C" trx_status trx_plan_destroy(trx_plan*) { return TRX_E_UNSUPPORTED; }
extern "C" trx_status trx_plan_batch(trx_plan*, trx_batch*) { return TRX_E_UNSUPPORTED; }
extern "C" trx_status trx_plan_launch(trx_plan*, int32_t, double*, double*, int32_t*, const double*,
                                      const double*, double*, double*, double*, double*) {
  return TRX_E_UNSUPPORTED;
}
extern "C" trx_status trx_autotune(trx_plan*, int32_t, const char*) { return TRX_E_UNSUPPORTED; }
extern "C" const char* trx_plan_describe(const trx_plan*) { return ""; }
