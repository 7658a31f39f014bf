// FP32 direct-sum kernels for 3-dimensional CV spaces (see direct_sum_impl.h).
#include "direct_sum_impl.h"

namespace abp {
hipError_t dispatch_f32_d3(const DirectArgs& A, int mask, bool iso, bool kahan, hipStream_t stream) {
  return dispatch_f32<3>(A, mask, iso, kahan, stream);
}
}  // namespace abp
