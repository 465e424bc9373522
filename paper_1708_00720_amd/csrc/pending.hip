// Entry points whose kernels are not built yet: they report "not supported".
#include <hip/hip_runtime.h>

#include "bfx_internal.h"

namespace bfx {

hipError_t launch_xengine_batched(bool, const void *, int64_t, const BatchUnit *, int32_t,
                                  const int32_t *, int64_t, int64_t, int32_t *, bool,
                                  hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_xengine_f16(const void *, int64_t, int32_t, int32_t, float *, bool,
                              hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_beamform(const void *, const void *, int32_t, int32_t, int32_t, int64_t,
                           int32_t, float *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace bfx
