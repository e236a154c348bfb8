// Dispatch of the strided-axis correlation to the instantiation for the
// requested (input type, outputs, radius); the instantiations live in
// k_strided_inst.hip, compiled once per group.
#include "st_internal.h"

namespace st {

#define ST_DECL(tag, r) hipError_t strided_##tag##_##r(const StridedParams& p, hipStream_t stream);
#define ST_DECL_U16(r) ST_DECL(u16d, r)
#define ST_DECL_F32D(r) ST_DECL(f32d, r)
#define ST_DECL_F32(r) ST_DECL(f32, r) \
  hipError_t strided_grouped_##r(const StridedGroup& p, int64_t blocks, hipStream_t stream);
ST_RADII_SIGMA(ST_DECL_U16)
ST_RADII_SIGMA(ST_DECL_F32D)
ST_RADII_RHO(ST_DECL_F32)

hipError_t launch_strided(int R, int in_dtype, bool with_d, const StridedParams& p,
                          hipStream_t stream) {
#define ST_CASE_U16(r) case r: return strided_u16d_##r(p, stream);
#define ST_CASE_F32D(r) case r: return strided_f32d_##r(p, stream);
#define ST_CASE_F32(r) case r: return strided_f32_##r(p, stream);
  if (in_dtype == ST_DTYPE_U16) {
    if (!with_d) return hipErrorInvalidValue;
    switch (R) { ST_RADII_SIGMA(ST_CASE_U16) default: return hipErrorInvalidValue; }
  }
  if (with_d) {
    switch (R) { ST_RADII_SIGMA(ST_CASE_F32D) default: return hipErrorInvalidValue; }
  }
  switch (R) { ST_RADII_RHO(ST_CASE_F32) default: return hipErrorInvalidValue; }
}

hipError_t launch_strided_grouped(int R, const StridedGroup& p, int64_t blocks, hipStream_t stream) {
  if (blocks < 1) return hipSuccess;
#define ST_CASE_G(r) case r: return strided_grouped_##r(p, blocks, stream);
  switch (R) { ST_RADII_RHO(ST_CASE_G) default: return hipErrorInvalidValue; }
#undef ST_CASE_G
}

}  // namespace st
