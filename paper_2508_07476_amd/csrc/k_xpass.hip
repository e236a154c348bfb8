// Dispatch of the x-axis final pass to the translation unit holding the radius.
#include "st_internal.h"

namespace st {

hipError_t launch_xfinal_small(int R, const XFinalParams& p, hipStream_t stream);
hipError_t launch_xfinal_large(int R, const XFinalParams& p, hipStream_t stream);

hipError_t launch_xfinal_grouped_small(int R, int lanes, const XFinalGroup& p, int64_t blocks, hipStream_t stream);
hipError_t launch_xfinal_grouped_large(int R, int lanes, const XFinalGroup& p, int64_t blocks, hipStream_t stream);

hipError_t launch_xfinal(int R, const XFinalParams& p, hipStream_t stream) {
  return R <= 12 ? launch_xfinal_small(R, p, stream) : launch_xfinal_large(R, p, stream);
}

hipError_t launch_xfinal_grouped(int R, int lanes, const XFinalGroup& p, int64_t blocks, hipStream_t stream) {
  if (blocks < 1) return hipSuccess;
  return R <= 12 ? launch_xfinal_grouped_small(R, lanes, p, blocks, stream)
                 : launch_xfinal_grouped_large(R, lanes, p, blocks, stream);
}

}  // namespace st
