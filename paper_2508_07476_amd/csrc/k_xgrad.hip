// Instantiations of the x-axis gradient pass fused with the outer product.
#include "k_xpass_impl.h"

namespace st {

hipError_t launch_xgrad(int R, const XGradParams& p, hipStream_t stream) {
#define ST_CASE(r) case r: return xpass_impl::launch_xgrad_r<r>(p, stream);
  switch (R) { ST_RADII_SIGMA(ST_CASE) default: return hipErrorInvalidValue; }
#undef ST_CASE
}

}  // namespace st
