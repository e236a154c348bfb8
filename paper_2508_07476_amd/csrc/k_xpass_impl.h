// x-axis passes: the last gradient pass fused with the outer product, and the
// last integration pass fused with the eigen-decomposition, FA and angles.
//
// Each wave owns one (z, y) row segment of kXTile = 256 outputs.  It stages the
// segment plus a halo of R samples on each side in LDS (coalesced global
// loads, boundary reflection per lane), then every lane computes kXVec = 4
// consecutive outputs from a register copy of its 2R+4 window, read from LDS
// with 16-byte loads, so each LDS value feeds up to 4 outputs.
#pragma once
#include "st_device.h"

namespace st {
namespace xpass_impl {

constexpr int lds_row(int R) { return ((kXTile + 2 * R + 4 + 3) / 4) * 4; }

// Fill lds[0 .. kXTile + 2R) with row[reflect(x0 - R + i)].
template <int R>
__device__ __forceinline__ void stage_row(float* lds, const float* row, int64_t x0, int64_t nx,
                                          int lane) {
  const int n = static_cast<int>(nx);
#pragma unroll
  for (int i = lane; i < kXTile + 2 * R; i += 64) {
    const int gx = reflect_lane(static_cast<int>(x0) - R + i, n);
    lds[i] = row[gx];
  }
}

// out[v] = sum_k w[k] * lds[4 lane + v + k], v = 0..3
template <int R>
__device__ __forceinline__ void conv4(const float* lds, int lane, const Taps& w, float out[kXVec]) {
  constexpr int NV = (2 * R + kXVec + 3) / 4;
  float buf[4 * NV];
  const float4* src = reinterpret_cast<const float4*>(lds + 4 * lane);
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const float4 t = src[q];
    buf[4 * q + 0] = t.x;
    buf[4 * q + 1] = t.y;
    buf[4 * q + 2] = t.z;
    buf[4 * q + 3] = t.w;
  }
#pragma unroll
  for (int v = 0; v < kXVec; ++v) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 2 * R + 1; ++k) acc = fmaf(w.w[k], buf[v + k], acc);
    out[v] = acc;
  }
}

__device__ __forceinline__ void store4(float* dst, int64_t x, int64_t nx, bool vec_ok,
                                       const float v[kXVec]) {
  if (vec_ok && x + kXVec <= nx) {
    *reinterpret_cast<float4*>(dst + x) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int i = 0; i < kXVec; ++i)
      if (x + i < nx) dst[x + i] = v[i];
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_xgrad(const XGradParams p) {
  constexpr int LR = lds_row(R);
  __shared__ __attribute__((aligned(16))) float lds[kRowsPerBlock][3][LR];
  const int lane = threadIdx.x;
  const int wv = threadIdx.y;
  const int64_t xt = blockIdx.x % p.x_tiles;
  const int64_t row = (blockIdx.x / p.x_tiles) * kRowsPerBlock + wv;
  const bool row_ok = row < p.nrows;
  const int64_t rr = row_ok ? row : p.nrows - 1;
  const int64_t x0 = xt * kXTile;
  const int64_t base = rr * p.nx;

  stage_row<R>(lds[wv][0], p.gg + base, x0, p.nx, lane);
  stage_row<R>(lds[wv][1], p.dg + base, x0, p.nx, lane);
  stage_row<R>(lds[wv][2], p.gd + base, x0, p.nx, lane);
  __syncthreads();

  float gx[kXVec], gy[kXVec], gz[kXVec];
  conv4<R>(lds[wv][0], lane, p.wd, gx);
  conv4<R>(lds[wv][1], lane, p.wg, gy);
  conv4<R>(lds[wv][2], lane, p.wg, gz);
  if (!row_ok) return;

  const int64_t x = x0 + kXVec * lane;
  if (x >= p.nx) return;
  const bool vec_ok = p.vec_ok != 0;
  float t[kXVec];
#define ST_PROD(idx, A, B)                                        \
  for (int v = 0; v < kXVec; ++v) t[v] = A[v] * B[v];             \
  store4(p.prod[idx] + base, x, p.nx, vec_ok, t);
  ST_PROD(0, gz, gz)
  ST_PROD(1, gz, gy)
  ST_PROD(2, gz, gx)
  ST_PROD(3, gy, gy)
  ST_PROD(4, gy, gx)
  ST_PROD(5, gx, gx)
#undef ST_PROD
}

template <int R>
__global__ __launch_bounds__(256) void k_xfinal(const XFinalParams p) {
  constexpr int LR = lds_row(R);
  __shared__ __attribute__((aligned(16))) float lds[kRowsPerBlock][6][LR];
  const int lane = threadIdx.x;
  const int wv = threadIdx.y;
  const int64_t xt = blockIdx.x % p.x_tiles;
  const int64_t row = (blockIdx.x / p.x_tiles) * kRowsPerBlock + wv;
  const bool row_ok = row < p.nrows;
  const int64_t rr = row_ok ? row : p.nrows - 1;
  const int64_t x0 = xt * kXTile;
  const int64_t base = rr * p.nx;

#pragma unroll
  for (int c = 0; c < 6; ++c) stage_row<R>(lds[wv][c], p.s[c] + base, x0, p.nx, lane);
  __syncthreads();

  float s[6][kXVec];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    conv4<R>(lds[wv][c], lane, p.w, s[c]);
    __builtin_amdgcn_sched_barrier(0);  // keep one component's window live at a time
  }
  if (!row_ok) return;
  const int64_t x = x0 + kXVec * lane;
  if (x >= p.nx) return;

  const double pz = static_cast<double>(rr / p.ny);
  const double py = static_cast<double>(rr % p.ny);
  float e3[3][kXVec], ev[3][kXVec], fa[kXVec], ha[kXVec], ia[kXVec];
  uint32_t fl[kXVec];
#pragma unroll
  for (int v = 0; v < kXVec; ++v) {
    const int64_t xv = x + v < p.nx ? x + v : p.nx - 1;
    const bool inside = p.mask == nullptr || p.mask[base + xv] != 0;
    if (inside) {
      const float s6[6] = {s[0][v], s[1][v], s[2][v], s[3][v], s[4][v], s[5][v]};
      VoxelOut o;
      solve_voxel(s6, p.has_axis != 0, p.center, p.dir, pz, py, static_cast<double>(x + v), o);
      e3[0][v] = o.e3[0]; e3[1][v] = o.e3[1]; e3[2][v] = o.e3[2];
      ev[0][v] = o.ev[0]; ev[1][v] = o.ev[1]; ev[2][v] = o.ev[2];
      fa[v] = o.fa; ha[v] = o.ha; ia[v] = o.ia; fl[v] = o.flags;
    } else {
      e3[0][v] = e3[1][v] = e3[2][v] = 0.f;
      ev[0][v] = ev[1][v] = ev[2][v] = 0.f;
      fa[v] = ha[v] = ia[v] = 0.f;
      fl[v] = ST_FLAG_OUTSIDE_MASK;
    }
  }
  const bool vec_ok = p.vec_ok != 0;
  if (p.e3) {
    store4(p.e3 + base, x, p.nx, vec_ok, e3[0]);
    store4(p.e3 + p.n + base, x, p.nx, vec_ok, e3[1]);
    store4(p.e3 + 2 * p.n + base, x, p.nx, vec_ok, e3[2]);
  }
  if (p.evals) {
    store4(p.evals + base, x, p.nx, vec_ok, ev[0]);
    store4(p.evals + p.n + base, x, p.nx, vec_ok, ev[1]);
    store4(p.evals + 2 * p.n + base, x, p.nx, vec_ok, ev[2]);
  }
  if (p.fa) store4(p.fa + base, x, p.nx, vec_ok, fa);
  if (p.ha) store4(p.ha + base, x, p.nx, vec_ok, ha);
  if (p.ia) store4(p.ia + base, x, p.nx, vec_ok, ia);
  if (p.flags) {
    if (vec_ok && x + kXVec <= p.nx) {
      const uint32_t packed = fl[0] | (fl[1] << 8) | (fl[2] << 16) | (fl[3] << 24);
      *reinterpret_cast<uint32_t*>(p.flags + base + x) = packed;
    } else {
      for (int v = 0; v < kXVec; ++v)
        if (x + v < p.nx) p.flags[base + x + v] = static_cast<uint8_t>(fl[v]);
    }
  }
}

template <int R>
hipError_t launch_xgrad_r(const XGradParams& p, hipStream_t stream) {
  const int64_t blocks = p.x_tiles * ((p.nrows + kRowsPerBlock - 1) / kRowsPerBlock);
  hipLaunchKernelGGL((k_xgrad<R>), dim3(static_cast<unsigned>(blocks)), dim3(64, kRowsPerBlock), 0,
                     stream, p);
  return hipGetLastError();
}

template <int R>
hipError_t launch_xfinal_r(const XFinalParams& p, hipStream_t stream) {
  const int64_t blocks = p.x_tiles * ((p.nrows + kRowsPerBlock - 1) / kRowsPerBlock);
  hipLaunchKernelGGL((k_xfinal<R>), dim3(static_cast<unsigned>(blocks)), dim3(64, kRowsPerBlock), 0,
                     stream, p);
  return hipGetLastError();
}

}  // namespace xpass_impl
}  // namespace st
