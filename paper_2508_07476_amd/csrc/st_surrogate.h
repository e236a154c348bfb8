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
  const __bf16* prev;     // backward data pass: forward activation whose ReLU mask gates the output
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
  // z slab: output planes [z_lo, z_hi); `in` holds planes from in_z0 on (the
  // planes z_lo - 1 .. z_hi, clamped to the volume, must be there), `out` and
  // `prev` from out_z0 on.  The raw volume and the final outputs are whole.
  int64_t z_lo, z_hi, in_z0, out_z0;
  int has_axis;
  double center[3];
  double dir[3];
};

// Merge of a run of voxels [begin, begin + count) of the volume (n voxels):
// where the mask holds and the confidence is below the threshold, the outputs
// take the structure-tensor path's, read at voxel i - src_shift of a source of
// src_n voxels (e3 planes src_n apart).
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
  int64_t begin, count, src_shift, src_n;
};

hipError_t launch_sg_pack(const float* blob, __bf16* w1, __bf16* w25, hipStream_t stream);
// layer 1..5; dtype is the raw volume's (first layer only)
hipError_t launch_sg_conv(int layer, int dtype, const SgConvParams& p, hipStream_t stream);
hipError_t launch_sg_merge(const SgMergeParams& p, hipStream_t stream);

// ---- per-tile fallback (k_sg_fallback.hip) -----------------------------------
// Fallback tiles are cubes of edge 32, 64 or 128 voxels on the volume's grid
// (the last ones clipped).  A tile is flagged when one of its voxels inside
// the mask has confidence below the threshold; one pass flags all three tile
// grids (flags[k] of edge 32 << k, tiles indexed (tz * tiles_y + ty) * tiles_x + tx).
constexpr int kSgTileEdges = 3;
struct SgTileFlagParams {
  const float* conf;
  const uint8_t* mask;  // or NULL
  float threshold;
  int64_t nz, ny, nx;
  int* flags[kSgTileEdges];  // zeroed by launch_sg_tile_flags
  int64_t tiles[kSgTileEdges];  // entries of each grid
};
hipError_t launch_sg_tile_flags(const SgTileFlagParams& p, hipStream_t stream);

// One crop: a flagged tile with the path's halo, clipped to the volume.
struct SgBox {
  int64_t z0, y0, x0;         // crop origin in the volume
  int64_t cz, cy, cx;         // crop sizes
  int64_t off;                // first voxel of the crop in the crop stack
  int64_t tz0, ty0, tx0;      // tile interior (volume coordinates), half-open
  int64_t tz1, ty1, tx1;
};
// Copies every crop of the volume (and of the mask) into the crop stack; one
// block per crop row, rows numbered through the crops (first[c]: crop c's first).
struct SgGatherParams {
  const void* vol;
  const uint8_t* mask;  // or NULL
  void* cvol;
  uint8_t* cmask;       // NULL when mask is
  const SgBox* boxes;   // device
  const int64_t* first; // device, count entries
  int count;
  int64_t rows;         // rows of all crops
  int64_t ny, nx;
};
hipError_t launch_sg_gather(int dtype, const SgGatherParams& p, hipStream_t stream);
// Writes the crops' path outputs over the surrogate's at every voxel of a
// tile interior that lies in the mask with confidence below the threshold;
// one block per interior row (first[c]: tile c's first).  Crop c's outputs sit
// at its offset in the stacks (e3: three planes of the crop's voxels at 3 off).
struct SgTileMergeParams {
  const SgBox* boxes;
  const int64_t* first;
  int count;
  int64_t rows;
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
  int64_t n, ny, nx;
};
hipError_t launch_sg_tile_merge(const SgTileMergeParams& p, hipStream_t stream);
// Training: a hidden layer (bias, ReLU, bf16 output) for any layer, the first
// reading the raw volume; and the backward data pass of a 32 -> 32 layer
// (weights packed transposed and tap-flipped, output gated by p.prev > 0).
hipError_t launch_sg_conv_hidden(bool first, int dtype, const SgConvParams& p, hipStream_t stream);
hipError_t launch_sg_conv_bwd(const SgConvParams& p, hipStream_t stream);

// ---- training kernels (k_surrogate_train.hip) --------------------------------
// Stored activations and gradients are [N][32] bf16, channel-last.  Row r of a
// volume of nz x ny x nx voxels (nx <= 32) holds voxels r * nx .. r * nx + nx - 1.
constexpr int kSgTrainMaxX = 32;          // rows of at most 32 voxels (one MFMA K step)
constexpr int kSgWgradBlocks = 256;       // blocks of the weight-gradient kernels
constexpr int kSgHeadSums = 5 * kSgChannels + 5 + 6;  // head gradient (Wh, bh) and six loss sums
constexpr int kSgTrainStats = 8;          // dir, fa, conf, total loss, sum w, within, mean angle (deg), count

// Backward weights of layers 2..5, packed [layer - 2][tap'][co'][ci'] = W[ci'][co'][26 - tap'].
hipError_t launch_sg_pack_bwd(const float* blob, __bf16* w25t, hipStream_t stream);

struct SgHeadParams {
  const __bf16* x5;       // [N][32]
  const float* head_w;    // [5][32] (float32 weights)
  const float* head_b;    // [5]
  const float* target;    // [3][N] label directions
  const float* target_fa; // [N]
  const uint8_t* weight;  // [N] loss weight (0 or 1)
  __bf16* g5;             // [N][32]: (Wh^T dL/dh) * (x5 > 0), unnormalised
  float* partial;         // [blocks][kSgHeadSums]
  int64_t n;
  float w_conf;           // weight of the confidence term
};
hipError_t launch_sg_head_train(const SgHeadParams& p, int blocks, hipStream_t stream);

struct SgWgradParams {
  const __bf16* g;        // [N][32] gradient at the layer's pre-activation
  const __bf16* x;        // [N][32] the layer's input activation (layers 2..5)
  const void* vol;        // layer 1: raw volume (dtype), x0 = bf16(v * scale + offset)
  const float* scale_offset;
  float* partial;         // [blocks][27 * 32 * 32 + 32] (layers 2..5) or [blocks][32 * 27 + 32] (layer 1)
  int64_t nz, ny, nx;     // the stacked volume (nx <= kSgTrainMaxX)
  int64_t rows_per_block;
};
hipError_t launch_sg_wgrad(const SgWgradParams& p, int blocks, hipStream_t stream);
hipError_t launch_sg_wgrad1(int dtype, const SgWgradParams& p, int blocks, hipStream_t stream);

// out[dst(j)] = sum over blocks of partial[b][j] for j < len (fixed order).
// mode 0: dst(j) = j; mode 1 (layer weights): j = (tap * 32 + co) * 32 + ci goes to
// (co * 32 + ci) * 27 + tap, and j >= 27 * 1024 (the bias) to 32 * 32 * 27 + (j - 27 * 1024);
// mode 2 (layer 1): j = co * 27 + tap goes to itself, the bias after it.
hipError_t launch_sg_reduce(const float* partial, int blocks, int len, int mode, float* out, hipStream_t stream);
// grad[i] /= (sum of weights), grad[0..1] = 0 (in_scale, in_offset are not
// trained); raw = the six loss sums (dir, fa, conf, weights, within, angle);
// stats[0..7] = mean dir, fa, conf terms, total loss, sum of weights, voxels
// within 2 degrees, mean angle (degrees), sum of weights.
hipError_t launch_sg_finish(float* grad, int64_t n, const float* raw, float w_conf, float* stats, hipStream_t stream);
// Adam on float32 parameters (moments m, v; step >= 1), skipping the first `frozen` values.
hipError_t launch_sg_adam(float* params, const float* grad, float* m, float* v, int64_t n, int64_t frozen,
                          int64_t step, float lr, float beta1, float beta2, float eps, hipStream_t stream);

}  // namespace st
