// Entry points not built yet.
#include "trx_host.h"

extern "C" trx_status trx_chi2_grad(trx_ctx* c, const trx_tables*, const trx_batch*, const trx_bins*,
                                    trx_precision, const double*, const double*, int32_t, double*, double*,
                                    double*, double*, double*, int32_t*) {
  return trx::set_err(c, TRX_E_UNSUPPORTED, "trx_chi2_grad: not built");
}
