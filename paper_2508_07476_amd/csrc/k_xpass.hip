// Dispatch of the x-axis final pass to the translation unit holding the radius.
#include "st_internal.h"

namespace st {

hipError_t launch_xfinal_small(int R, const XFinalParams& p, hipStream_t stream);
hipError_t launch_xfinal_large(int R, const XFinalParams& p, hipStream_t stream);

hipError_t launch_xfinal(int R, const XFinalParams& p, hipStream_t stream) {
  return R <= 12 ? launch_xfinal_small(R, p, stream) : launch_xfinal_large(R, p, stream);
}

}  // namespace st
