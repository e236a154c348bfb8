// Instantiations of the strided-axis correlation kernel: uint16 input, G and D outputs.
#include "k_strided_impl.h"

namespace st {

hipError_t launch_strided_u16d(int R, const StridedParams& p, hipStream_t stream) {
#define ST_CASE(r) case r: return strided_impl::launch_r<uint16_t, true, r>(p, stream);
  switch (R) { ST_RADII_SIGMA(ST_CASE) default: return hipErrorInvalidValue; }
#undef ST_CASE
}

}  // namespace st
