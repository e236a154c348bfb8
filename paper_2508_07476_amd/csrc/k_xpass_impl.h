// x-axis passes: the last gradient pass fused with the outer product, and the
// last integration pass fused with the eigen-decomposition, FA and angles.
//
// Each block is one wave.  It owns one (z, y) row segment of kXTile = 256
// outputs, or (final pass, narrow rows) four segments of 64 outputs from
// consecutive rows.  It stages each segment plus a halo of R samples on each
// side in LDS (coalesced global loads, boundary reflection per lane only for
// segments that touch a face), then every lane computes kXVec = 4 consecutive
// outputs, streaming its 2R+4 window from LDS in 16-byte pieces: each value
// feeds up to 4 outputs.  Values are widened to float64 as the window streams
// by, or, in the final pass's 64-lane segments, once as they are staged (the
// rows of three components at a time, in the bytes of six float32 rows), since
// a staged value lies in the windows of up to R / 2 + 1 lanes.  Intermediate
// planes are read and written with the workspace row pitch; the caller's mask
// and outputs with rows of nx.
#pragma once
#include "st_device.h"

namespace st {
namespace xpass_impl {

// A row segment of TL lanes covers TL * kXVec outputs.  Its staging slots cover
// the segment and both halos, rounded up to whole 16-byte windows.
constexpr int stage_slots(int R, int TL = 64) { return (TL * kXVec + 2 * R + 4 + TL - 1) / TL; }
// LDS row length of a segment: every staging slot (TL per lane step) and the
// 16-byte reads of the last lane's window fit; a multiple of 4 floats.
constexpr int lds_row(int R, int TL = 64) {
  return TL * stage_slots(R, TL) > ((TL * kXVec + 2 * R + 4 + 3) / 4) * 4
             ? TL * stage_slots(R, TL)
             : ((TL * kXVec + 2 * R + 4 + 3) / 4) * 4;
}

// Row index of LDS slot i = l + TL j of a segment starting at x0 (global
// x = x0 - R + i, reflected into [0, nx)); l is the lane within the segment.
// Slots past the staged range repeat a valid index (their values are never
// read).  Computed once per lane and shared by every component.
template <int R, int TL = 64>
__device__ __forceinline__ void stage_index(int idx[stage_slots(R, TL)], int64_t x0, int64_t nx, int l) {
  const int n = static_cast<int>(nx);
  const int g0 = static_cast<int>(x0) - R;
  const bool interior = g0 >= 0 && g0 + TL * stage_slots(R, TL) <= n;  // wave-uniform
#pragma unroll
  for (int j = 0; j < stage_slots(R, TL); ++j) {
    const int g = g0 + l + TL * j;
    idx[j] = interior ? g : reflect_lane(g, n);
  }
}

// Branch-free staging: all loads of the row segment are issued before the first
// LDS write.
template <int R, int TL = 64>
__device__ __forceinline__ void stage_row(float* lds, const float* row, const int idx[stage_slots(R, TL)],
                                          int l) {
  float v[stage_slots(R, TL)];
#pragma unroll
  for (int j = 0; j < stage_slots(R, TL); ++j) v[j] = row[idx[j]];
#pragma unroll
  for (int j = 0; j < stage_slots(R, TL); ++j) lds[l + TL * j] = v[j];
}

// out[v] = sum_k w[k] * lds[4 lane + v + k], v = 0..3, in float64.  The
// window is streamed through in 16-byte pieces: each value is widened once and
// enters the (up to) four sums it belongs to, each sum taking its taps in
// ascending order.
// SYMMETRIC: the taps are symmetric about the centre (bit for bit, as the
// smoothing taps are built), so only taps 0..R are read and R + 1 of them
// occupy registers; derivative taps must use the general form.
template <int R, bool SYMMETRIC = false>
__device__ __forceinline__ void conv4(const float* lds, int lane, const Taps& w, double out[kXVec]) {
  constexpr int NV = (2 * R + kXVec + 3) / 4;
  const float4* src = reinterpret_cast<const float4*>(lds + 4 * lane);
#pragma unroll
  for (int v = 0; v < kXVec; ++v) out[v] = 0.0;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const float4 t = src[q];
    const float e[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = 4 * q + u;
      const double d = static_cast<double>(e[u]);
#pragma unroll
      for (int v = 0; v < kXVec; ++v) {
        const int k = j - v;
        const int kk = SYMMETRIC && k > R ? 2 * R - k : k;
        if (k >= 0 && k <= 2 * R) out[v] = fma(w.w[kk], d, out[v]);
      }
    }
  }
}

// conv4 over a window already widened to float64 in LDS (16-byte reads of two
// values); the same sums in the same order as conv4 on the float32 row.
template <int R, bool SYMMETRIC = false>
__device__ __forceinline__ void conv4_f64(const double* lds, int lane, const Taps& w, double out[kXVec]) {
  constexpr int NP = (2 * R + kXVec + 1) / 2;
  const double2* src = reinterpret_cast<const double2*>(lds + 4 * lane);
#pragma unroll
  for (int v = 0; v < kXVec; ++v) out[v] = 0.0;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const double2 t = src[q];
    const double e[2] = {t.x, t.y};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = 2 * q + u;
#pragma unroll
      for (int v = 0; v < kXVec; ++v) {
        const int k = j - v;
        const int kk = SYMMETRIC && k > R ? 2 * R - k : k;
        if (k >= 0 && k <= 2 * R) out[v] = fma(w.w[kk], e[u], out[v]);
      }
    }
  }
}

__device__ __forceinline__ void store4(float* dst, int x, int nx, bool vec_ok,
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
__global__ __launch_bounds__(64) void k_xgrad(const XGradParams p) {
  constexpr int LR = lds_row(R);
  __shared__ __attribute__((aligned(16))) float lds[3][LR];
  const int lane = threadIdx.x;
  const int64_t xt = blockIdx.x % p.x_tiles;
  const int64_t row = blockIdx.x / p.x_tiles;  // one wave per (row, x tile)
  const int64_t x0 = xt * kXTile;
  const int64_t base = row * p.pitch;  // inputs and products are workspace rows

  int idx[stage_slots(R)];
  stage_index<R>(idx, x0, p.nx, lane);
  stage_row<R>(lds[0], p.gg + base, idx, lane);
  stage_row<R>(lds[1], p.dg + base, idx, lane);
  stage_row<R>(lds[2], p.gd + base, idx, lane);
  __syncthreads();

  double gx[kXVec], gy[kXVec], gz[kXVec];
  conv4<R>(lds[0], lane, p.wd, gx);
  conv4<R>(lds[1], lane, p.wg, gy);
  conv4<R>(lds[2], lane, p.wg, gz);

  const int nxi = static_cast<int>(p.nx);  // x positions are 32-bit (nx < 2^31)
  const int x = static_cast<int>(x0) + kXVec * lane;
  if (x >= nxi) return;
  const bool vec_ok = p.vec_ok != 0;
  float t[kXVec];
#define ST_PROD(idx, A, B)                                        \
  for (int v = 0; v < kXVec; ++v) t[v] = static_cast<float>(A[v] * B[v]); \
  store4(p.prod[idx] + base, x, nxi, vec_ok, t);
  ST_PROD(0, gz, gz)
  ST_PROD(1, gz, gy)
  ST_PROD(2, gz, gx)
  ST_PROD(3, gy, gy)
  ST_PROD(4, gy, gx)
  ST_PROD(5, gx, gx)
#undef ST_PROD
}

// x integration of the six tensor components (float64, on the vector ALUs:
// the float64 matrix-core and vector paths share issue slots, and the banded
// form costs fewer operations on the vector path), then the per-voxel
// eigen-decomposition, FA and angles of the lane's kXVec consecutive voxels.
// A wave holds 64 / TL row segments of TL lanes (TL * kXVec outputs each): one
// segment of 256 outputs, or four of 64 for rows whose width would leave much
// of a 256-wide segment idle.  Results are parked in the staged rows (free once
// every window has been read) and leave as 16-byte stores.
// Block `blk` of the final pass over the volume described by p (taps w); lds
// holds the block's staged rows.
template <int R, int TL>
__device__ __forceinline__ void xfinal_block(const XFinalGeo& p, const Taps& w, int64_t blk,
                                             float (&lds)[6][(64 / TL) * lds_row(R, TL)]) {
  constexpr int LR = lds_row(R, TL);
  const int lane = threadIdx.x;
  // row segment of the lane and lane within it (0 and lane for one segment per
  // wave, which keeps the row wave-uniform)
  const int sub = TL == 64 ? 0 : lane / TL, l = TL == 64 ? lane : lane % TL;
  constexpr int RPW = 64 / TL;  // rows per wave
  const int64_t xt = blk % p.x_tiles;
  const int64_t row0 = (blk / p.x_tiles) * RPW;  // first row of the wave
  const int64_t row = row0 + sub;
  const bool row_ok = row < p.nrows;
  const int64_t rr = row_ok ? row : p.nrows - 1;  // loads of a missing row stay in range
  const int64_t x0 = xt * (TL * kXVec);
  const int64_t base = rr * p.nx;  // mask and outputs
  const int nxi = static_cast<int>(p.nx);  // x positions are 32-bit (nx < 2^31)
  const int x = static_cast<int>(x0) + kXVec * l;
  float* seg[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) seg[c] = &lds[c][sub * LR];

  // mask bytes of the lane's voxels, fetched first so the loads overlap the filtering
  uint32_t inside_bits = 0xFu;
  if (p.mask != nullptr) {
    inside_bits = 0u;
#pragma unroll
    for (int v = 0; v < kXVec; ++v) {
      const int xr = x + v < nxi ? x + v : nxi - 1;
      inside_bits |= (p.mask[base + xr] != 0 ? 1u : 0u) << v;
    }
  }
  double acc[6][kXVec];
  if constexpr (TL == 64) {
    // The six float32 rows' bytes hold three float64 rows: stage and integrate
    // the components in two halves of three, widening every staged value once
    // (it lies in the windows of up to R / 2 + 1 lanes).
    constexpr int NS = stage_slots(R, TL);
    double* drow = reinterpret_cast<double*>(&lds[0][0]);
    int idx[NS];
    stage_index<R, TL>(idx, x0, p.nx, l);
    const int64_t sbase = rr * p.pitch;  // integrated products: workspace rows
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float v[3][NS];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < NS; ++j) v[c][j] = p.s[3 * h + c][sbase + idx[j]];
      if (h == 1) __syncthreads();  // the first half's windows are read
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < NS; ++j) drow[c * LR + l + TL * j] = static_cast<double>(v[c][j]);
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 3; ++c) conv4_f64<R, true>(drow + c * LR, l, w, acc[3 * h + c]);
    }
  } else {
    int idx[stage_slots(R, TL)];
    stage_index<R, TL>(idx, x0, p.nx, l);
    const int64_t sbase = rr * p.pitch;  // integrated products: workspace rows
#pragma unroll
    for (int c = 0; c < 6; ++c) stage_row<R, TL>(seg[c], p.s[c] + sbase, idx, l);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 6; ++c) conv4<R, true>(seg[c], l, w, acc[c]);
  }
  __syncthreads();  // every window read before the rows receive results

  // (z, y) of the lane's row; with several rows per wave the wave's first row
  // is divided once and stepped (at most 64 / TL - 1 steps)
  double pz, py;
  if constexpr (TL == 64) {
    pz = static_cast<double>(row / p.ny);
    py = static_cast<double>(row % p.ny);
  } else {
    int64_t pzi = row0 / p.ny, pyi = row0 % p.ny + sub;
    while (pyi >= p.ny) { pyi -= p.ny; ++pzi; }
    pz = static_cast<double>(pzi);
    py = static_cast<double>(pyi);
  }
  const int64_t n = p.n;
  uint32_t flag_word = 0u;  // the lane's flag bytes, voxel v in byte v
#pragma unroll 1
  for (int v = 0; v < kXVec; ++v) {
    const int xv = x + v;
    const bool inside = (inside_bits >> v) & 1u;
    double s6[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {  // voxel v's tensor is always in slot 0: rotate the rest down
      s6[c] = acc[c][0];
      acc[c][0] = acc[c][1];
      acc[c][1] = acc[c][2];
      acc[c][2] = acc[c][3];
    }
    float res[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float l1 = 0.f, l2 = 0.f, l3 = 0.f;
    uint32_t fl = ST_FLAG_OUTSIDE_MASK;
    if (inside) {
      EigOut o;
      eig_smallest(s6, o);
      res[0] = static_cast<float>(o.vz);
      res[1] = static_cast<float>(o.vy);
      res[2] = static_cast<float>(o.vx);
      res[3] = o.fa;
      l1 = o.l1; l2 = o.l2; l3 = o.l3;
      fl = o.degenerate ? ST_FLAG_DEGENERATE : 0u;
      if (p.has_axis && fibre_angles(o.vz, o.vy, o.vx, p.center, p.dir, pz, py,
                                     static_cast<double>(xv), res[4], res[5]))
        fl |= ST_FLAG_ON_AXIS;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) seg[q][kXVec * l + v] = res[q];
    if (row_ok && xv < nxi && p.evals) {  // optional output: scalar stores
      const int64_t i = base + xv;
      p.evals[i] = l1; p.evals[n + i] = l2; p.evals[2 * n + i] = l3;
    }
    flag_word |= (fl & 0xffu) << (8 * v);
  }
  if (p.flags != nullptr && row_ok && x < nxi) {
    // the lane's four flag bytes as one aligned 32-bit store where they are
    // whole (x is a multiple of 4), else one byte at a time
    if (p.vec_ok != 0 && ((base + x) & 3) == 0 && x + kXVec <= nxi) {
      *reinterpret_cast<uint32_t*>(p.flags + base + x) = flag_word;
    } else {
#pragma unroll
      for (int v = 0; v < kXVec; ++v)
        if (x + v < nxi) p.flags[base + x + v] = static_cast<uint8_t>(flag_word >> (8 * v));
    }
  }
  if constexpr (TL == 64) {
    // One row per wave.  Where a destination row starts off a 16-byte boundary
    // (nx not a multiple of 4), each lane writes the aligned group of the row
    // that holds segment positions [4 l - k, 4 l - k + 4) (k: offset of the
    // segment's first element inside its group) from the parked results, and
    // lane 0 also the last k positions; groups cut by an end of the segment
    // are written one element at a time.  Every element is written once.
    const int64_t s0 = base + x0;
    const bool shifted = p.vec_ok != 0 &&
                         (((s0 & 3) != 0 && (p.fa || p.ha || p.ia)) ||
                          (p.e3 && (((s0 & 3) | ((n + s0) & 3) | ((2 * n + s0) & 3)) != 0)));
    if (shifted) {  // wave-uniform
      __syncthreads();  // every lane's parked results visible
      const int seglen = min(TL * kXVec, nxi - static_cast<int>(x0));
      auto put = [&](float* plane, int64_t off, const float* src) {
        float* dst = plane + off + x0;  // segment start
        const int k = static_cast<int>((off + x0) & 3);
        const int g = kXVec * l - k;
        if (g >= 0 && g + kXVec <= seglen) {
          *reinterpret_cast<float4*>(dst + g) = make_float4(src[g], src[g + 1], src[g + 2], src[g + 3]);
        } else {
#pragma unroll
          for (int i = 0; i < kXVec; ++i)
            if (g + i >= 0 && g + i < seglen) dst[g + i] = src[g + i];
        }
        if (l == 0) {
#pragma unroll
          for (int i = 0; i < kXVec - 1; ++i) {
            const int t = TL * kXVec - k + i;
            if (i < k && t < seglen) dst[t] = src[t];
          }
        }
      };
      if (p.e3) {
        put(p.e3, base, seg[0]);
        put(p.e3, n + base, seg[1]);
        put(p.e3, 2 * n + base, seg[2]);
      }
      if (p.fa) put(p.fa, base, seg[3]);
      if (p.ha) put(p.ha, base, seg[4]);
      if (p.ia) put(p.ia, base, seg[5]);
      return;
    }
  }
  if (!row_ok || x >= nxi) return;
  // the lane reads back only what it wrote: no barrier needed
  float o4[6][kXVec];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const float4 t = *reinterpret_cast<const float4*>(&seg[q][kXVec * l]);
    o4[q][0] = t.x; o4[q][1] = t.y; o4[q][2] = t.z; o4[q][3] = t.w;
  }
  // float4 stores where the row segment starts on 16 bytes (x is a multiple of 4)
  auto vec_at = [&](int64_t off) { return p.vec_ok != 0 && (off & 3) == 0; };
  if (p.e3) {
    store4(p.e3 + base, x, nxi, vec_at(base), o4[0]);
    store4(p.e3 + n + base, x, nxi, vec_at(n + base), o4[1]);
    store4(p.e3 + 2 * n + base, x, nxi, vec_at(2 * n + base), o4[2]);
  }
  const bool vec_row = vec_at(base);
  if (p.fa) store4(p.fa + base, x, nxi, vec_row, o4[3]);
  if (p.ha) store4(p.ha + base, x, nxi, vec_row, o4[4]);
  if (p.ia) store4(p.ia + base, x, nxi, vec_row, o4[5]);
}

template <int R, int TL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TL == 16 ? 4 : 1)))
void k_xfinal(const XFinalParams p) {
  __shared__ __attribute__((aligned(16))) float lds[6][(64 / TL) * lds_row(R, TL)];
  xfinal_block<R, TL>(p, p.w, blockIdx.x, lds);
}

// One launch over a table of volumes that share the taps and the segment width.
template <int R, int TL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TL == 16 ? 4 : 1)))
void k_xfinal_grouped(const XFinalGroup p) {
  __shared__ __attribute__((aligned(16))) float lds[6][(64 / TL) * lds_row(R, TL)];
  const int64_t b = blockIdx.x;
  const int e = group_entry(p.g.first, p.g.count, b);
  const XFinalGeo g = p.g.geo[e];
  const int64_t local = b - p.g.first[e];
  if (local >= g.x_tiles * (TL == 64 ? g.nrows : (g.nrows + 3) / 4)) return;  // block-uniform
  xfinal_block<R, TL>(g, p.w, local, lds);
}

template <int R>
hipError_t launch_xgrad_r(const XGradParams& p, hipStream_t stream) {
  const int64_t blocks = p.x_tiles * p.nrows;
  hipLaunchKernelGGL((k_xgrad<R>), dim3(static_cast<unsigned>(blocks)), dim3(64), 0, stream, p);
  return hipGetLastError();
}

// p.tile_lanes selects the segment width (64, or 16 for radii up to
// kXNarrowMaxRadius); p.x_tiles must be ceil(nx / (tile_lanes * kXVec)).
template <int R>
hipError_t launch_xfinal_r(const XFinalParams& p, hipStream_t stream) {
  if (p.tile_lanes == 64) {
    const int64_t blocks = p.x_tiles * p.nrows;
    hipLaunchKernelGGL((k_xfinal<R, 64>), dim3(static_cast<unsigned>(blocks)), dim3(64), 0, stream, p);
    return hipGetLastError();
  }
  if constexpr (R <= kXNarrowMaxRadius) {
    if (p.tile_lanes == 16) {
      const int64_t blocks = p.x_tiles * ((p.nrows + 3) / 4);
      hipLaunchKernelGGL((k_xfinal<R, 16>), dim3(static_cast<unsigned>(blocks)), dim3(64), 0, stream, p);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <int R>
hipError_t launch_xfinal_grouped_r(int lanes, const XFinalGroup& p, int64_t blocks, hipStream_t stream) {
  if (lanes == 64) {
    hipLaunchKernelGGL((k_xfinal_grouped<R, 64>), dim3(static_cast<unsigned>(blocks)), dim3(64), 0, stream, p);
    return hipGetLastError();
  }
  if constexpr (R <= kXNarrowMaxRadius) {
    if (lanes == 16) {
      hipLaunchKernelGGL((k_xfinal_grouped<R, 16>), dim3(static_cast<unsigned>(blocks)), dim3(64), 0, stream, p);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace xpass_impl
}  // namespace st
