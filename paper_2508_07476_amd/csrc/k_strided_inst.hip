// Instantiations of the strided-axis correlation kernel.  This file is
// compiled once per instantiation group (ST_STRIDED_GROUP, set by the build),
// so the large radii compile in parallel.
#include "k_strided_impl.h"

#ifndef ST_STRIDED_GROUP
#error "ST_STRIDED_GROUP must be defined by the build"
#endif

namespace st {

#define ST_DEFINE(tag, Tin, D, r)                                                \
  hipError_t strided_##tag##_##r(const StridedParams& p, hipStream_t stream) {  \
    return strided_impl::launch_r<Tin, D, r>(p, stream);                        \
  }
#define ST_U16(r) ST_DEFINE(u16d, uint16_t, true, r)
#define ST_F32D(r) ST_DEFINE(f32d, float, true, r)
#define ST_F32(r) ST_DEFINE(f32, float, false, r) \
  hipError_t strided_grouped_##r(const StridedGroup& p, int64_t blocks, hipStream_t stream) { \
    return strided_impl::launch_grouped_r<r>(p, blocks, stream);                               \
  }

#if ST_STRIDED_GROUP == 0
ST_RADII_SIGMA(ST_U16)
#elif ST_STRIDED_GROUP == 1
ST_RADII_SIGMA(ST_F32D)
#elif ST_STRIDED_GROUP == 2
ST_RADII_SIGMA_SMALL(ST_F32)
#elif ST_STRIDED_GROUP == 3
ST_F32(14)
ST_F32(16)
#elif ST_STRIDED_GROUP == 4
ST_F32(20)
#elif ST_STRIDED_GROUP == 5
ST_F32(24)
#elif ST_STRIDED_GROUP == 6
ST_F32(28)
#elif ST_STRIDED_GROUP == 7
ST_F32(32)
#endif

}  // namespace st
