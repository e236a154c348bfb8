// Learned orientation surrogate: a dense 3-D CNN (five 3x3x3 convolutions with
// 32 channels and ReLU, a 1x1x1 head with 5 outputs) evaluated on the bf16
// matrix cores, float32 accumulation.
//
// Activations are channel-last bf16 ([voxel][32], 64 bytes per voxel).  A
// convolution is an implicit GEMM per tap: out[co][voxel] += W[co][ci] * in[ci][voxel
// + tap] with M = output channel (two 16-blocks), N = 16 consecutive voxels
// along x, K = the 32 input channels of one tap, one v_mfma_f32_16x16x32_bf16
// per (tap, M-block, N-block).  Operand layout of that instruction on gfx950
// (probed): lane l holds A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16],
// i = 0..7, and receives D[4 (l / 16) + r][l % 16], r = 0..3 -- so each lane
// ends with 4 consecutive output channels of one voxel, an 8-byte channel-last
// store.
//
// Two kernels.  The first layer and the training passes stream their weights:
// a block of 8 waves owns 8 (y) x 32 (x) output voxels and marches through a
// chunk of z planes; the layer's weights are staged in LDS once per block (27 x
// 32 x 32 bf16, tap-major, output channel, input channel) and the input planes
// live in a ring of 3 LDS planes of 10 x 34 voxels (faces clamped), the next
// plane's loads issued before the current plane's matrix products.  The
// inference layers 2..5 keep their weights in registers (k_sg_conv_ws, below).
// The last layer's epilogue evaluates the head, the normalisation, FA,
// confidence, the mask and the helix / intrusion angles.
#include "st_device.h"
#include "st_surrogate.h"

namespace st {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int C = kSgChannels;
constexpr int TY = 8, TX = 32, RY = TY + 2, RX = TX + 2;
constexpr int NT = 64 * TY;         // threads per block: one wave per output row
constexpr int PLANE_VOX = RY * RX;  // voxels of one staged plane

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// Packs the float32 blob into bf16 operand layouts: layer 1 as [co][k] (k < 27 a
// tap, the rest 0), layers 2..5 as [tap][co][ci].
__global__ void k_sg_pack(const float* blob, __bf16* w1, __bf16* w25) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < C * 32) {
    const int co = static_cast<int>(i / 32), k = static_cast<int>(i % 32);
    w1[i] = static_cast<__bf16>(k < 27 ? blob[kSgOffW1 + co * 27 + k] : 0.f);
  }
  const int64_t per = 27 * C * C;
  if (i < 4 * per) {
    const int layer = static_cast<int>(i / per);  // 0 -> network layer 2
    const int64_t r = i % per;
    const int tap = static_cast<int>(r / (C * C)), co = static_cast<int>((r / C) % C),
              ci = static_cast<int>(r % C);
    w25[i] = static_cast<__bf16>(blob[kSgOffW2 + layer * kSgLayerStride + (co * C + ci) * 27 + tap]);
  }
}

// Outputs of one voxel from its five head values o = bh + Wh x5: unit fibre
// vector with the canonical sign, FA and confidence (sigmoids), the helix and
// intrusion angles; zeros outside the mask.
__device__ __forceinline__ void head_outputs(const SgConvParams& p, const float o[5], int64_t z, int64_t yo,
                                             int64_t xv) {
  const int64_t vox = (z * p.ny + yo) * p.nx + xv;
  const bool inside = p.mask == nullptr || p.mask[vox] != 0;
  float ez = 0.f, ey = 0.f, ex = 0.f, fa = 0.f, conf = 0.f, ha = 0.f, ia = 0.f;
  if (inside) {
    const float nn = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    if (nn > 0.f) {
      const float inv = 1.f / sqrtf(nn);
      ez = o[0] * inv; ey = o[1] * inv; ex = o[2] * inv;
    } else {
      ez = 1.f;
    }
    const float az = fabsf(ez), ay = fabsf(ey), ax = fabsf(ex);
    const float lead = (az >= ay && az >= ax) ? ez : (ay >= ax ? ey : ex);
    if (lead < 0.f) { ez = -ez; ey = -ey; ex = -ex; }
    fa = 1.f / (1.f + expf(-o[3]));
    conf = 1.f / (1.f + expf(-o[4]));
    if (p.has_axis)
      (void)fibre_angles(ez, ey, ex, p.center, p.dir, static_cast<double>(z), static_cast<double>(yo),
                         static_cast<double>(xv), ha, ia);
  }
  const int64_t nvox = p.n;
  if (p.e3) { p.e3[vox] = ez; p.e3[nvox + vox] = ey; p.e3[2 * nvox + vox] = ex; }
  if (p.fa) p.fa[vox] = fa;
  if (p.conf) p.conf[vox] = conf;
  if (p.ha) p.ha[vox] = ha;
  if (p.ia) p.ia[vox] = ia;
}

// Streaming-weights layer: the first layer (FIRST: input is the raw volume, one
// channel), and the training passes (hidden layers storing their activations;
// BWD, the backward data pass: no bias, and the output is multiplied by the
// ReLU mask of p.prev (the forward activation at the output voxel) instead of
// passing through ReLU).
template <bool FIRST, typename Tin, bool BWD = false>
__global__ __launch_bounds__(NT) void k_sg_conv(const SgConvParams p) {
  constexpr int WN = FIRST ? C * 32 : 27 * C * C;             // bf16 weights staged
  constexpr int AN = FIRST ? 3 * PLANE_VOX : 3 * PLANE_VOX * C;  // bf16 activations staged
  __shared__ __attribute__((aligned(16))) __bf16 wl[WN];
  __shared__ __attribute__((aligned(16))) __bf16 al[AN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t b = blockIdx.x;
  const int64_t xt = b % p.x_tiles;
  b /= p.x_tiles;
  const int64_t yt = b % p.y_tiles;
  const int64_t zc = b / p.y_tiles;
  const int64_t x0 = xt * TX, y0 = yt * TY;
  const int64_t nz = p.nz, ny = p.ny, nx = p.nx;
  const int64_t z0 = p.z_lo + zc * p.zchunk;
  const int64_t z1 = (z0 + p.zchunk) < p.z_hi ? (z0 + p.zchunk) : p.z_hi;

  // weights: 16-byte chunks
  {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(FIRST ? p.w1 : p.w);
    bf16x8* dst = reinterpret_cast<bf16x8*>(wl);
    for (int i = tid; i < WN / 8; i += NT) dst[i] = src[i];
  }

  const double in_scale = FIRST ? static_cast<double>(p.scale_offset[0]) : 0.0;
  const double in_offset = FIRST ? static_cast<double>(p.scale_offset[1]) : 0.0;

  // staging of one input plane (index zi, clamped) into ring slot s
  // FIRST: one value per voxel (normalised, bf16); else 4 chunks of 16 bytes per voxel
  constexpr int PER = FIRST ? (PLANE_VOX + NT - 1) / NT : (PLANE_VOX * 4 + NT - 1) / NT;
  // the raw volume is whole; `in` starts at plane in_z0
  auto plane_base = [&](int64_t zi) { return (clampi(zi, nz) - (FIRST ? 0 : p.in_z0)) * ny * nx; };
  auto load_plane = [&](int64_t zi, bf16x8 (&pf)[PER], float (&pv)[PER]) {
    const int64_t pb = plane_base(zi);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int c = tid + NT * j;
      if constexpr (FIRST) {
        const int vi = c < PLANE_VOX ? c : PLANE_VOX - 1;
        const int row = vi / RX, col = vi % RX;
        const int64_t g = pb + clampi(y0 - 1 + row, ny) * nx + clampi(x0 - 1 + col, nx);
        pv[j] = static_cast<float>(static_cast<const Tin*>(p.vol)[g]);
      } else {
        const int cc = c < PLANE_VOX * 4 ? c : PLANE_VOX * 4 - 1;
        const int vi = cc >> 2, part = cc & 3;
        const int row = vi / RX, col = vi % RX;
        const int64_t g = pb + clampi(y0 - 1 + row, ny) * nx + clampi(x0 - 1 + col, nx);
        pf[j] = reinterpret_cast<const bf16x8*>(p.in + g * C)[part];
      }
    }
  };
  auto store_plane = [&](int s, const bf16x8 (&pf)[PER], const float (&pv)[PER]) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int c = tid + NT * j;
      if constexpr (FIRST) {
        if (c < PLANE_VOX)  // float64 affine map (exact product, one rounding), then float32, then bf16
          al[s * PLANE_VOX + c] = static_cast<__bf16>(
              static_cast<float>(fma(static_cast<double>(pv[j]), in_scale, in_offset)));
      } else {
        if (c < PLANE_VOX * 4) reinterpret_cast<bf16x8*>(al)[s * PLANE_VOX * 4 + c] = pf[j];
      }
    }
  };

  bf16x8 pf[PER];
  float pv[PER];
  load_plane(z0 - 1, pf, pv);
  store_plane(0, pf, pv);
  load_plane(z0, pf, pv);
  store_plane(1, pf, pv);
  load_plane(z0 + 1, pf, pv);
  store_plane(2, pf, pv);
  __syncthreads();

  const int li = lane & 15, lk = lane >> 4;
  const int64_t yo = y0 + wave;
  const float* bias = p.bias;
#pragma unroll 1
  for (int64_t z = z0; z < z1; ++z) {
    // ring slot of input plane z + d is (z - z0 + 1 + d) mod 3
    const int s0 = static_cast<int>((z - z0) % 3);  // plane z - 1
    const bool more = z + 1 < z1;
    if (more) load_plane(z + 2, pf, pv);  // in flight during the products

    f32x4 acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    if constexpr (FIRST) {
      // K = 32 "taps" of the single input channel (27 real, 5 zero)
      bf16x8 bo[2];
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int k = 8 * lk + i;
          if (k < 27) {
            const int dz = k / 9, dy = (k / 3) % 3, dx = k % 3;  // offsets + 1
            const int s = (s0 + dz) % 3;
            bo[n][i] = al[s * PLANE_VOX + (wave + dy) * RX + 16 * n + li + dx];
          } else {
            bo[n][i] = static_cast<__bf16>(0.f);
          }
        }
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const bf16x8 a = reinterpret_cast<const bf16x8*>(wl)[(16 * m + li) * 4 + lk];
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bo[n], acc[m][n], 0, 0, 0);
      }
    } else {
      const bf16x8* a8 = reinterpret_cast<const bf16x8*>(al);
      const bf16x8* w8 = reinterpret_cast<const bf16x8*>(wl);
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        const int s = (s0 + dz) % 3;
        bf16x8 bo[2], ao[2];
#pragma unroll
        for (int n = 0; n < 2; ++n)
          bo[n] = a8[(s * PLANE_VOX + (wave + dy) * RX + 16 * n + li + dx) * 4 + lk];
#pragma unroll
        for (int m = 0; m < 2; ++m) ao[m] = w8[(t * C + 16 * m + li) * 4 + lk];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 2; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao[m], bo[n], acc[m][n], 0, 0, 0);
      }
    }

#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int64_t xv = x0 + 16 * n + li;
      if (yo < ny && xv < nx) {
        const int64_t vox = ((z - p.out_z0) * ny + yo) * nx + xv;  // in out and prev
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int co = 16 * m + 4 * lk;
          bf16x4 o;
          if constexpr (BWD) {
            const bf16x4 xm = *reinterpret_cast<const bf16x4*>(p.prev + vox * C + co);
#pragma unroll
            for (int r = 0; r < 4; ++r)
              o[r] = static_cast<__bf16>(static_cast<float>(xm[r]) > 0.f ? acc[m][n][r] : 0.f);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = static_cast<__bf16>(fmaxf(acc[m][n][r] + bias[co + r], 0.f));
          }
          *reinterpret_cast<bf16x4*>(p.out + vox * C + co) = o;
        }
      }
    }

    __syncthreads();  // every read of the ring slot about to be replaced is done
    if (more) {
      store_plane(s0, pf, pv);  // plane z + 2 replaces plane z - 1
      __syncthreads();
    }
  }
}

// Weight-stationary 32 -> 32 layer (inference, layers 2..5).  A block of 4
// waves (one per SIMD) owns 8 (y) x 64 (x) output voxels and marches through a
// chunk of z planes; wave w computes rows 2w and 2w + 1, i.e. eight 16-voxel N
// blocks.  Every lane holds its A operands of all 27 taps and both 16-channel M
// blocks in registers for the whole chunk (216 VGPRs: the layer's weights are
// read from memory once per block), so per tap the wave reads only its eight B
// operands from the LDS ring and issues 16 MFMAs: half the LDS bytes per MFMA
// of a kernel that streams the weights too.  The input planes live in a ring
// of 3 LDS planes of 10 x 66 voxels (faces clamped; 124 KB, one block per CU);
// the next plane's loads are issued before the current plane's products and
// stored into the ring right after them, before the epilogue.
// LAST: the head is three more MFMAs per N block: the layer's output and the
// head weights each split into a high and a low bf16 part (about 16 bits of
// each), all products but low x low.
constexpr int WS_TY = 8, WS_TX = 64, WS_RY = WS_TY + 2, WS_RX = WS_TX + 2;
constexpr int WS_NT = 256;
constexpr int WS_PLANE = WS_RY * WS_RX;
constexpr int WS_PER = (WS_PLANE * 4 + WS_NT - 1) / WS_NT;  // 16-byte chunks per thread per plane

template <bool LAST>
__global__ __launch_bounds__(WS_NT) void k_sg_conv_ws(const SgConvParams p) {
  __shared__ __attribute__((aligned(16))) __bf16 al[3 * WS_PLANE * C];
  __shared__ float hw[LAST ? 5 * C : 1];  // head weights (read by lane-dependent channel)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if constexpr (LAST) {
    if (tid < 5 * C) hw[tid] = p.head_w[tid];
  }
  const int64_t nz = p.nz, ny = p.ny, nx = p.nx;
  const int64_t x_tiles = (nx + WS_TX - 1) / WS_TX, y_tiles = (ny + WS_TY - 1) / WS_TY;
  int64_t b = blockIdx.x;
  const int64_t xt = b % x_tiles;
  b /= x_tiles;
  const int64_t yt = b % y_tiles;
  const int64_t zc = b / y_tiles;
  const int64_t x0 = xt * WS_TX, y0 = yt * WS_TY;
  const int64_t z0 = p.z_lo + zc * p.zchunk;
  const int64_t z1 = (z0 + p.zchunk) < p.z_hi ? (z0 + p.zchunk) : p.z_hi;

  // A operands: lane holds W[t][16 m + li][8 lk .. 8 lk + 7]
  bf16x8 wa[27][2];
  {
    const bf16x8* w8 = reinterpret_cast<const bf16x8*>(p.w);
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
      for (int m = 0; m < 2; ++m) wa[t][m] = w8[(t * C + 16 * m + li) * 4 + lk];
  }
  float bias[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[m][r] = p.bias[16 * m + 4 * lk + r];

  auto load_plane = [&](int64_t zi, bf16x8 (&pf)[WS_PER]) {
    const int64_t pb = (clampi(zi, nz) - p.in_z0) * ny * nx;
#pragma unroll
    for (int j = 0; j < WS_PER; ++j) {
      const int c = tid + WS_NT * j;
      const int cc = c < WS_PLANE * 4 ? c : WS_PLANE * 4 - 1;
      const int vi = cc >> 2, part = cc & 3;
      const int row = vi / WS_RX, col = vi % WS_RX;
      const int64_t g = pb + clampi(y0 - 1 + row, ny) * nx + clampi(x0 - 1 + col, nx);
      pf[j] = reinterpret_cast<const bf16x8*>(p.in + g * C)[part];
    }
  };
  auto store_plane = [&](int s, const bf16x8 (&pf)[WS_PER]) {
#pragma unroll
    for (int j = 0; j < WS_PER; ++j) {
      const int c = tid + WS_NT * j;
      if (c < WS_PLANE * 4) reinterpret_cast<bf16x8*>(al)[s * WS_PLANE * 4 + c] = pf[j];
    }
  };

  bf16x8 pf[WS_PER];
  load_plane(z0 - 1, pf);
  store_plane(0, pf);
  load_plane(z0, pf);
  store_plane(1, pf);
  load_plane(z0 + 1, pf);
  store_plane(2, pf);
  __syncthreads();

  // LAST: the head h = Wh x5 on the matrix cores, with Wh (rows 0..4 of a
  // 16-row A operand) split into a bf16 high and low part.  A lane's B operand
  // is its own eight channels of x5, so its K index 8 lk + i stands for
  // channel 16 (i / 4) + 4 lk + i % 4, and A's columns follow that order.
  bf16x8 wh_hi, wh_lo;
  if constexpr (LAST) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float wv = li < 5 ? hw[li * C + 16 * (i >> 2) + 4 * lk + (i & 3)] : 0.f;
      const __bf16 hi = static_cast<__bf16>(wv);
      wh_hi[i] = hi;
      wh_lo[i] = static_cast<__bf16>(wv - static_cast<float>(hi));
    }
  }

  const bf16x8* a8 = reinterpret_cast<const bf16x8*>(al);
#pragma unroll 1
  for (int64_t z = z0; z < z1; ++z) {
    const int s0 = static_cast<int>((z - z0) % 3);  // ring slot of plane z - 1
    const bool more = z + 1 < z1;
    if (more) load_plane(z + 2, pf);  // in flight during the products

    f32x4 acc[2][8];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 8; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    // this lane's operand in each ring plane (planes z - 1, z, z + 1); the tap
    // and N-block offsets below are compile-time constants
    const bf16x8* base[3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
      base[dz] = a8 + ((((s0 + dz) % 3) * WS_RY + 2 * wave) * WS_RX + li) * 4 + lk;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
      bf16x8 bo[8];
#pragma unroll
      for (int n = 0; n < 8; ++n) bo[n] = base[dz][(((n >> 2) + dy) * WS_RX + 16 * (n & 3) + dx) * 4];
#pragma unroll
      for (int n = 0; n < 8; ++n)
#pragma unroll
        for (int m = 0; m < 2; ++m)
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][m], bo[n], acc[m][n], 0, 0, 0);
    }
    // the prefetched plane goes into the ring before the epilogue, so its
    // registers are free there
    __syncthreads();  // every read of the ring slot about to be replaced is done
    if (more) store_plane(s0, pf);  // plane z + 2 replaces plane z - 1

    if constexpr (!LAST) {
#pragma unroll
      for (int n = 0; n < 8; ++n) {
        const int64_t yo = y0 + 2 * wave + (n >> 2), xv = x0 + 16 * (n & 3) + li;
        if (yo < ny && xv < nx) {
          const int64_t vox = ((z - p.out_z0) * ny + yo) * nx + xv;
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            bf16x4 o;
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = static_cast<__bf16>(fmaxf(acc[m][n][r] + bias[m][r], 0.f));
            *reinterpret_cast<bf16x4*>(p.out + vox * C + 16 * m + 4 * lk) = o;
          }
        }
      }
    } else {
      // head: x5 = relu(acc + b), split like Wh into a high and a low bf16
      // part, is the B operand as the lane holds it (the product of the two
      // low parts, below 2^-16 of a term, is left out); D row q, column li is
      // h[q] of voxel li (rows 0..3 in lanes 0..15, row 4 in lanes 16..31).
      // Lanes of group lk then finish the voxels of N blocks lk and lk + 4.
      float hs[2][5];
#pragma unroll
      for (int n = 0; n < 8; ++n) {
        bf16x8 xh, xl;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float v = fmaxf(acc[i >> 2][n][i & 3] + bias[i >> 2][i & 3], 0.f);
          xh[i] = static_cast<__bf16>(v);
          xl[i] = static_cast<__bf16>(v - static_cast<float>(xh[i]));
        }
        f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh_hi, xh, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh_hi, xl, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh_lo, xh, d, 0, 0, 0);
        float qv[5];
#pragma unroll
        for (int r = 0; r < 4; ++r) qv[r] = __shfl(d[r], li);
        qv[4] = __shfl(d[0], 16 + li);
        if ((n & 3) == lk) {
#pragma unroll
          for (int q = 0; q < 5; ++q) hs[n >> 2][q] = qv[q];
        }
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int64_t yo = y0 + 2 * wave + k, xv = x0 + 16 * lk + li;
        if (yo < ny && xv < nx) {
          float o[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) o[q] = p.head_b[q] + hs[k][q];
          head_outputs(p, o, z, yo, xv);
        }
      }
    }

    __syncthreads();  // the replaced slot is written before the next plane's products
  }
}

template <bool LAST>
hipError_t launch_conv_ws(const SgConvParams& p, hipStream_t stream) {
  const int64_t blocks = ((p.nx + WS_TX - 1) / WS_TX) * ((p.ny + WS_TY - 1) / WS_TY) *
                         ((p.z_hi - p.z_lo + p.zchunk - 1) / p.zchunk);
  hipLaunchKernelGGL(k_sg_conv_ws<LAST>, dim3(static_cast<unsigned>(blocks)), dim3(WS_NT), 0, stream, p);
  return hipGetLastError();
}

// Voxels inside the mask whose confidence is below the threshold take the
// structure-tensor path's outputs.
__global__ void k_sg_merge(const SgMergeParams p) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= p.count) return;
  const int64_t i = p.begin + t, j = i - p.src_shift;
  if (p.mask != nullptr && p.mask[i] == 0) return;
  if (!(p.conf[i] < p.threshold)) return;
  if (p.e3) { p.e3[i] = p.pe3[j]; p.e3[p.n + i] = p.pe3[p.src_n + j]; p.e3[2 * p.n + i] = p.pe3[2 * p.src_n + j]; }
  if (p.fa) p.fa[i] = p.pfa[j];
  if (p.ha) p.ha[i] = p.pha[j];
  if (p.ia) p.ia[i] = p.pia[j];
}

template <bool FIRST, bool BWD = false>
hipError_t launch_conv(const SgConvParams& p, int dtype, hipStream_t stream) {
  const int64_t blocks = p.x_tiles * p.y_tiles * ((p.z_hi - p.z_lo + p.zchunk - 1) / p.zchunk);
  if (dtype == ST_DTYPE_U16)
    hipLaunchKernelGGL((k_sg_conv<FIRST, uint16_t, BWD>), dim3(static_cast<unsigned>(blocks)), dim3(NT), 0,
                       stream, p);
  else
    hipLaunchKernelGGL((k_sg_conv<FIRST, float, BWD>), dim3(static_cast<unsigned>(blocks)), dim3(NT), 0,
                       stream, p);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sg_pack(const float* blob, __bf16* w1, __bf16* w25, hipStream_t stream) {
  const int64_t n = 4 * 27 * C * C;
  hipLaunchKernelGGL(k_sg_pack, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, blob, w1, w25);
  return hipGetLastError();
}

hipError_t launch_sg_conv(int layer, int dtype, const SgConvParams& p, hipStream_t stream) {
  if (layer == 1) return launch_conv<true>(p, dtype, stream);
  if (layer == kSgLayers) return launch_conv_ws<true>(p, stream);
  return launch_conv_ws<false>(p, stream);
}

hipError_t launch_sg_conv_hidden(bool first, int dtype, const SgConvParams& p, hipStream_t stream) {
  return first ? launch_conv<true>(p, dtype, stream) : launch_conv<false>(p, ST_DTYPE_F32, stream);
}

hipError_t launch_sg_conv_bwd(const SgConvParams& p, hipStream_t stream) {
  return launch_conv<false, true>(p, ST_DTYPE_F32, stream);
}

hipError_t launch_sg_merge(const SgMergeParams& p, hipStream_t stream) {
  if (p.count < 1 || (p.count + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sg_merge, dim3(static_cast<unsigned>((p.count + 255) / 256)), dim3(256), 0, stream, p);
  return hipGetLastError();
}

}  // namespace st
