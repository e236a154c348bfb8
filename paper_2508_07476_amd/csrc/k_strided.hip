// Dispatch of the strided-axis correlation to the translation unit holding the
// requested (input type, outputs, radius) instantiation.
#include "st_internal.h"

namespace st {

hipError_t launch_strided_u16d(int R, const StridedParams& p, hipStream_t stream);
hipError_t launch_strided_f32d(int R, const StridedParams& p, hipStream_t stream);
hipError_t launch_strided_f32_small(int R, const StridedParams& p, hipStream_t stream);
hipError_t launch_strided_f32_large(int R, const StridedParams& p, hipStream_t stream);

hipError_t launch_strided(int R, int in_dtype, bool with_d, const StridedParams& p,
                          hipStream_t stream) {
  if (in_dtype == ST_DTYPE_U16) return with_d ? launch_strided_u16d(R, p, stream) : hipErrorInvalidValue;
  if (with_d) return launch_strided_f32d(R, p, stream);
  return R <= 12 ? launch_strided_f32_small(R, p, stream) : launch_strided_f32_large(R, p, stream);
}

}  // namespace st
