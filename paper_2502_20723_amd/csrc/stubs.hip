// Entry points whose kernels are not built yet return TDO_EUNSUPPORTED.
#include "common.h"

extern "C" {
int32_t tdo_sample(tdo_ctx_t*, const tdo_arch_t*, const float*, int32_t, int64_t, uint64_t*, float*, uint64_t,
                   uint64_t*, int32_t, float, tdo_prec_t, uint64_t*, hipStream_t) {
  return tdo::set_error(TDO_EUNSUPPORTED, "tdo_sample: not implemented yet");
}
}
