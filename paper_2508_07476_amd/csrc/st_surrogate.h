// Internal declarations of the learned orientation surrogate (kernels and host).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "st_internal.h"

namespace st {

constexpr int kSgChannels = 32;
constexpr int kSgLayers = 5;
// float32 weights blob offsets: in_scale, in_offset; W1 [32][1][27], b1 [32];
// W2..W5 [32][32][27], b [32] each; Wh [5][32], bh [5]
constexpr int64_t kSgOffW1 = 2;
constexpr int64_t kSgOffB1 = kSgOffW1 + kSgChannels * 27;
constexpr int64_t kSgOffW2 = kSgOffB1 + kSgChannels;
constexpr int64_t kSgLayerStride = kSgChannels * kSgChannels * 27 + kSgChannels;  // W then b
constexpr int64_t kSgOffHead = kSgOffW2 + 4 * kSgLayerStride;
constexpr int64_t kSgWeights = kSgOffHead + 5 * kSgChannels + 5;
static_assert(kSgWeights == ST_SURROGATE_WEIGHTS, "blob layout and the header constant agree");

struct SgConvParams {
  const void* vol;        // first layer: raw volume (u16 or f32)
  const __bf16* in;       // later layers: [N][32] bf16
  __bf16* out;            // non-last layers: [N][32] bf16
  const __bf16* w1;       // packed first-layer weights [32][32]
  const __bf16* w;        // packed weights of this layer [27][32][32]
  const float* bias;      // [32] (in the blob)
  const float* scale_offset;  // blob[0], blob[1]: input affine map
  const float* head_w;    // [5][32] (last layer)
  const float* head_b;    // [5]
  const uint8_t* mask;
  float* e3;
  float* fa;
  float* ha;
  float* ia;
  float* conf;
  int64_t n, nz, ny, nx;
  int64_t x_tiles, y_tiles, zchunk;
  int has_axis;
  double center[3];
  double dir[3];
};

struct SgMergeParams {
  const uint8_t* mask;
  const float* conf;
  float threshold;
  const float* pe3;
  const float* pfa;
  const float* pha;
  const float* pia;
  float* e3;
  float* fa;
  float* ha;
  float* ia;
  int64_t n;
};

hipError_t launch_sg_pack(const float* blob, __bf16* w1, __bf16* w25, hipStream_t stream);
// layer 1..5; dtype is the raw volume's (first layer only)
hipError_t launch_sg_conv(int layer, int dtype, const SgConvParams& p, hipStream_t stream);
hipError_t launch_sg_merge(const SgMergeParams& p, hipStream_t stream);

}  // namespace st
