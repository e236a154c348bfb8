// Standalone helix / intrusion angles of a given fibre field about an axis.
// One lane per 4 consecutive x voxels of a row; a pure streaming map
// (12 bytes of e3 + 1 byte of mask in, 8 bytes of angles + 1 byte of flags out).
#include "st_device.h"

namespace st {
namespace {

__global__ __launch_bounds__(256) void k_angles(const AnglesParams p) {
  const int lane = threadIdx.x;
  const int64_t xt = blockIdx.x % p.x_tiles;
  const int64_t row = (blockIdx.x / p.x_tiles) * kRowsPerBlock + threadIdx.y;
  if (row >= p.nrows) return;
  const int64_t x = xt * kXTile + kXVec * lane;
  if (x >= p.nx) return;
  const int64_t base = row * p.nx;
  const double pz = static_cast<double>(row / p.ny);
  const double py = static_cast<double>(row % p.ny);
#pragma unroll
  for (int v = 0; v < kXVec; ++v) {
    if (x + v >= p.nx) break;
    const int64_t i = base + x + v;
    float ha = 0.f, ia = 0.f;
    uint32_t fl = 0;
    if (p.mask != nullptr && p.mask[i] == 0) {
      fl = ST_FLAG_OUTSIDE_MASK;
    } else {
      const double vz = p.e3[i], vy = p.e3[p.n + i], vx = p.e3[2 * p.n + i];
      if (fibre_angles(vz, vy, vx, p.center, p.dir, pz, py, static_cast<double>(x + v), ha, ia))
        fl = ST_FLAG_ON_AXIS;
    }
    if (p.ha) p.ha[i] = ha;
    if (p.ia) p.ia[i] = ia;
    if (p.flags) p.flags[i] = static_cast<uint8_t>(fl);
  }
}

}  // namespace

hipError_t launch_angles(const AnglesParams& p, hipStream_t stream) {
  const int64_t blocks = p.x_tiles * ((p.nrows + kRowsPerBlock - 1) / kRowsPerBlock);
  hipLaunchKernelGGL(k_angles, dim3(static_cast<unsigned>(blocks)), dim3(64, kRowsPerBlock), 0,
                     stream, p);
  return hipGetLastError();
}

}  // namespace st
