// Per-tile fallback of the surrogate to the structure-tensor path: flag the
// tiles that hold low-confidence voxels, gather each flagged tile with the
// path's halo into a crop stack, and write the crops' path outputs back over
// the surrogate's where the confidence is low.  All three kernels are plain
// copies and compares, bound by HBM.
#include "st_device.h"
#include "st_surrogate.h"

namespace st {
namespace {

constexpr int kFlagWaves = 4;   // waves per block of the flag pass
constexpr int kRowThreads = 128;  // threads per crop row (gather, merge)

__device__ __forceinline__ void raise_flag(int* f) {
  if (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_sg_fill_zero(int* p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// One wave per 64-voxel row segment; segments start at multiples of 64, so a
// segment lies in one tile of edge 64 or 128 and in two of edge 32.
__global__ __launch_bounds__(64 * kFlagWaves) void k_sg_tile_flags(const SgTileFlagParams p) {
  const int lane = threadIdx.x & 63;
  const int64_t segs = (p.nx + 63) >> 6;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kFlagWaves + (threadIdx.x >> 6);
  if (g >= p.nz * p.ny * segs) return;  // uniform across the wave
  const int64_t row = g / segs, seg = g - row * segs;
  const int64_t z = row / p.ny, y = row - z * p.ny;
  const int64_t x = (seg << 6) + lane;
  bool low = false;
  if (x < p.nx) {
    const int64_t i = row * p.nx + x;
    low = (p.mask == nullptr || p.mask[i] != 0) && p.conf[i] < p.threshold;
  }
  const uint64_t b = __ballot(low);
  if (b == 0) return;
#pragma unroll
  for (int k = 0; k < kSgTileEdges; ++k) {
    const int s = 5 + k;
    const int64_t tyn = (p.ny + (int64_t(1) << s) - 1) >> s, txn = (p.nx + (int64_t(1) << s) - 1) >> s;
    int* f = p.flags[k] + ((z >> s) * tyn + (y >> s)) * txn;
    if (k == 0) {
      if (lane == 0 && (b & 0xffffffffull)) raise_flag(f + 2 * seg);
      if (lane == 32 && (b >> 32)) raise_flag(f + 2 * seg + 1);
    } else if (lane == 0) {
      raise_flag(f + (seg >> (k - 1)));
    }
  }
}

template <class T>
__global__ __launch_bounds__(kRowThreads) void k_sg_gather(const SgGatherParams p) {
  const int64_t r = blockIdx.x;
  const int c = group_entry(p.first, p.count, r);
  const SgBox bx = p.boxes[c];
  const int64_t lr = r - p.first[c];
  const int64_t zz = lr / bx.cy, yy = lr - zz * bx.cy;
  const int64_t src = ((bx.z0 + zz) * p.ny + (bx.y0 + yy)) * p.nx + bx.x0;
  const int64_t dst = bx.off + lr * bx.cx;
  const T* in = static_cast<const T*>(p.vol);
  T* out = static_cast<T*>(p.cvol);
  for (int64_t x = threadIdx.x; x < bx.cx; x += kRowThreads) {
    out[dst + x] = in[src + x];
    if (p.mask != nullptr) p.cmask[dst + x] = p.mask[src + x];
  }
}

__global__ __launch_bounds__(kRowThreads) void k_sg_tile_merge(const SgTileMergeParams p) {
  const int64_t r = blockIdx.x;
  const int c = group_entry(p.first, p.count, r);
  const SgBox bx = p.boxes[c];
  const int64_t lr = r - p.first[c];
  const int64_t th = bx.ty1 - bx.ty0;
  const int64_t zz = bx.tz0 + lr / th, yy = bx.ty0 + lr % th;
  const int64_t cv = bx.cz * bx.cy * bx.cx;
  const int64_t crow = ((zz - bx.z0) * bx.cy + (yy - bx.y0)) * bx.cx - bx.x0;  // + x: index in the crop
  const int64_t vrow = (zz * p.ny + yy) * p.nx;
  for (int64_t x = bx.tx0 + threadIdx.x; x < bx.tx1; x += kRowThreads) {
    const int64_t i = vrow + x;
    if (p.mask != nullptr && p.mask[i] == 0) continue;
    if (!(p.conf[i] < p.threshold)) continue;
    const int64_t j = crow + x;
    if (p.e3) {
      p.e3[i] = p.pe3[3 * bx.off + j];
      p.e3[p.n + i] = p.pe3[3 * bx.off + cv + j];
      p.e3[2 * p.n + i] = p.pe3[3 * bx.off + 2 * cv + j];
    }
    if (p.fa) p.fa[i] = p.pfa[bx.off + j];
    if (p.ha) p.ha[i] = p.pha[bx.off + j];
    if (p.ia) p.ia[i] = p.pia[bx.off + j];
  }
}

bool fits_grid(int64_t blocks) { return blocks >= 1 && blocks <= 0x7fffffff; }

}  // namespace

hipError_t launch_sg_tile_flags(const SgTileFlagParams& p, hipStream_t stream) {
  for (int k = 0; k < kSgTileEdges; ++k) {
    if (!fits_grid((p.tiles[k] + 255) / 256)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sg_fill_zero, dim3(static_cast<unsigned>((p.tiles[k] + 255) / 256)), dim3(256), 0, stream,
                       p.flags[k], p.tiles[k]);
  }
  const int64_t waves = p.nz * p.ny * ((p.nx + 63) >> 6);
  const int64_t blocks = (waves + kFlagWaves - 1) / kFlagWaves;
  if (!fits_grid(blocks)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sg_tile_flags, dim3(static_cast<unsigned>(blocks)), dim3(64 * kFlagWaves), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_sg_gather(int dtype, const SgGatherParams& p, hipStream_t stream) {
  if (!fits_grid(p.rows) || p.count < 1) return hipErrorInvalidValue;
  if (dtype == ST_DTYPE_U16)
    hipLaunchKernelGGL(k_sg_gather<uint16_t>, dim3(static_cast<unsigned>(p.rows)), dim3(kRowThreads), 0, stream, p);
  else
    hipLaunchKernelGGL(k_sg_gather<float>, dim3(static_cast<unsigned>(p.rows)), dim3(kRowThreads), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_sg_tile_merge(const SgTileMergeParams& p, hipStream_t stream) {
  if (!fits_grid(p.rows) || p.count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sg_tile_merge, dim3(static_cast<unsigned>(p.rows)), dim3(kRowThreads), 0, stream, p);
  return hipGetLastError();
}

}  // namespace st
