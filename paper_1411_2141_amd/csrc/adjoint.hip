// Reverse mode of the unrolled registration (gradient of the final MSD).
#include <hip/hip_runtime.h>

#include "../../include/meshreg.h"
#include "ctx.h"

int mr_ctx::backward(const double *, int32_t, int32_t, const double *, double *, double *, float *,
                     double *, hipStream_t) {
  return MR_ESTATE;
}
