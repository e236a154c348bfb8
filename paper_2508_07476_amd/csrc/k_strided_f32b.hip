// Instantiations of the strided-axis correlation kernel: float input, G output, radii 14 and up.
#include "k_strided_impl.h"

namespace st {

hipError_t launch_strided_f32_large(int R, const StridedParams& p, hipStream_t stream) {
#define ST_CASE(r) case r: return strided_impl::launch_r<float, false, r>(p, stream);
  switch (R) { ST_RADII_LARGE(ST_CASE) default: return hipErrorInvalidValue; }
#undef ST_CASE
}

}  // namespace st
