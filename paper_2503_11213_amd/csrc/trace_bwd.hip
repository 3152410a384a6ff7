// Adjoint of the trace + splat (placeholder until the reverse sweep lands).
#include <hip/hip_runtime.h>

#include "../../include/sdirt.h"

namespace sdirt {
int trace_backward_impl(const sdirt_lens*, const sdirt_sensor*, const sdirt_psf_query*,
                        const float*, double*, hipStream_t) {
    return SDIRT_EUNSUPPORTED;
}
}  // namespace sdirt
