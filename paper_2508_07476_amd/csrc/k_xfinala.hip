// Instantiations of the x-axis integration pass fused with eigen, FA and angles.
#include "k_xpass_impl.h"

namespace st {

hipError_t launch_xfinal_small(int R, const XFinalParams& p, hipStream_t stream) {
#define ST_CASE(r) case r: return xpass_impl::launch_xfinal_r<r>(p, stream);
  switch (R) { ST_RADII_SIGMA_SMALL(ST_CASE) default: return hipErrorInvalidValue; }
#undef ST_CASE
}

hipError_t launch_xfinal_grouped_small(int R, int lanes, const XFinalGroup& p, int64_t blocks, hipStream_t stream) {
#define ST_CASE(r) case r: return xpass_impl::launch_xfinal_grouped_r<r>(lanes, p, blocks, stream);
  switch (R) { ST_RADII_SIGMA_SMALL(ST_CASE) default: return hipErrorInvalidValue; }
#undef ST_CASE
}

}  // namespace st
