// 1-D Gaussian / derivative-of-Gaussian correlation along a strided axis (z or y).
//
// Lanes of a wave own 64 consecutive x columns (coalesced loads and stores);
// every lane walks the filtered axis with a register window of 2R+1 samples.
// The window rotates by static register renaming: the output loop is expanded
// (by a fold over an index sequence, so the expansion never depends on the
// unroller's size limits) to the window length, and sample k of output j sits
// in register (j + k) mod (2R+1).  Each input sample is loaded once per chunk,
// one block of 2R+1 outputs ahead of its use, so every lane keeps 2R+1 loads
// in flight; the axis position is wave-uniform (boundary reflection runs on
// the scalar unit) and the taps are kernel arguments held in scalar registers.
#pragma once
#include <utility>

#include "st_device.h"

namespace st {
namespace strided_impl {

// SAME: the outputs have the inputs' strides (every pass but the gradient's
// z pass over the caller's volume); one stride pair then serves both, which
// keeps the scalar registers within budget.
// Block `blk` of the pass over the volume described by p (taps wg, wd).
template <int R, typename Tin, bool WITH_D, bool SAME>
__device__ __forceinline__ void strided_block(const StridedGeo& p, const Taps& wg, const Taps& wd, int64_t blk) {
  constexpr int W = 2 * R + 1;
  const int lane = threadIdx.x;  // 0..63, x within the tile
  // flattened block index: x tile fastest, then "other" tile, then chunk, then job
  int64_t b = blk;
  const int64_t xt = b % p.x_tiles;
  b /= p.x_tiles;
  const int64_t ot = b % p.o_tiles;
  b /= p.o_tiles;
  const int chunk_id = static_cast<int>(b % p.nchunks);
  const int job = static_cast<int>(b / p.nchunks);

  const int64_t o = ot * 4 + threadIdx.y;
  if (o >= p.n_other) return;  // wave-uniform
  const int64_t x0 = xt * 64;
  const bool active = x0 + lane < p.nx;
  const int lx = active ? lane : static_cast<int>(p.nx - 1 - x0);  // keep loads in range

  const Tin* in = static_cast<const Tin*>(p.job[job].in) + o * p.s_other + x0;
  const int64_t so = SAME ? p.s_other : p.so_other;
  float* og = p.job[job].out_g + o * so + x0;
  float* od = WITH_D ? p.job[job].out_d + o * so + x0 : nullptr;

  // axis positions fit in 32 bits (each size < 2^31), so their compares and the
  // reflection stay on the scalar unit; only the element offsets are 64-bit
  const int n = static_cast<int>(p.n_axis);
  const int64_t sa = p.s_axis;                     // input stride of the filtered axis
  const int64_t soa = SAME ? sa : p.so_axis;       // output stride
  const int a0 = chunk_id * static_cast<int>(p.chunk);
  const int len = (n - a0) < p.chunk ? (n - a0) : static_cast<int>(p.chunk);
  // relative sample i <-> axis index a0 - R + i (reflected into [0, n))
  // streaming (non-temporal) loads and stores: every sample is read once per
  // chunk and every output once, so neither should displace cached data
  auto sample = [&](int i) {
    return static_cast<float>(
        __builtin_nontemporal_load(in + static_cast<int64_t>(reflect_lane(a0 - R + i, n)) * sa + lx));
  };
  // window and accumulators in float64 (each sample is widened once, on entry)

  // win: the 2R+1 samples of the current output; pre: the newest sample of each
  // output of the current block of W outputs, loaded one block ahead so that W
  // loads per lane are always in flight.
  double win[W];
  float pre[W];
#pragma unroll
  for (int j = 0; j < 2 * R; ++j) win[j] = sample(j);
#pragma unroll
  for (int j = 0; j < W; ++j) pre[j] = sample(2 * R + j);

  for (int tb = 0; tb < len; tb += W) {
    auto step = [&]<int J>(std::integral_constant<int, J>) {
      const int t = tb + J;
      const double v = pre[J];
      if (t + W < len) pre[J] = sample(t + W + 2 * R);  // same step of the next block
      win[(J + 2 * R) % W] = v;
      if (t < len) {
        double g = 0.0, d = 0.0;
        // the smoothing taps are symmetric and the derivative taps antisymmetric
        // about the centre (bit for bit, as built): reading only taps 0..R keeps
        // R + 1 of them in scalar registers instead of 2R + 1, which no longer
        // fit at the largest radii
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const double u = win[(J + k) % W];
          g = fma(wg.w[k <= R ? k : 2 * R - k], u, g);
          if constexpr (WITH_D) d = fma(k <= R ? wd.w[k] : -wd.w[2 * R - k], u, d);
        }
        if (active) {
          const int64_t at = static_cast<int64_t>(a0 + t) * soa + lane;
          __builtin_nontemporal_store(static_cast<float>(g), og + at);
          if constexpr (WITH_D) __builtin_nontemporal_store(static_cast<float>(d), od + at);
        }
      }
    };
    [&]<int... J>(std::integer_sequence<int, J...>) {
      (step(std::integral_constant<int, J>{}), ...);
    }(std::make_integer_sequence<int, W>{});
  }
}

template <int R, typename Tin, bool WITH_D, bool SAME>
__global__ __launch_bounds__(256) void k_strided(const StridedParams p) {
  strided_block<R, Tin, WITH_D, SAME>(p, p.wg, p.wd, blockIdx.x);
}

// One launch over a table of volumes (integration: float32 in, smoothing taps,
// shared strides).
template <int R>
__global__ __launch_bounds__(256) void k_strided_grouped(const StridedGroup p) {
  const int64_t b = blockIdx.x;
  const int e = group_entry(p.g.first, p.g.count, b);
  const StridedGeo g = p.g.geo[e];
  const int64_t local = b - p.g.first[e];
  if (local >= g.x_tiles * g.o_tiles * g.nchunks * g.njobs) return;  // block-uniform
  strided_block<R, float, false, true>(g, p.wg, p.wg, local);
}

template <int R>
hipError_t launch_grouped_r(const StridedGroup& p, int64_t blocks, hipStream_t stream) {
  hipLaunchKernelGGL((k_strided_grouped<R>), dim3(static_cast<unsigned>(blocks)), dim3(64, 4), 0, stream, p);
  return hipGetLastError();
}

// Outputs with strides of their own are supported by the two-output variant
// only (the gradient's z pass); other variants reject them.
template <typename Tin, bool WITH_D, int R>
hipError_t launch_r(const StridedParams& p, hipStream_t stream) {
  const int64_t blocks = p.x_tiles * p.o_tiles * p.nchunks * p.njobs;
  if (p.so_axis == p.s_axis && p.so_other == p.s_other) {
    hipLaunchKernelGGL((k_strided<R, Tin, WITH_D, true>), dim3(static_cast<unsigned>(blocks)), dim3(64, 4),
                       0, stream, p);
    return hipGetLastError();
  }
  if constexpr (WITH_D) {
    hipLaunchKernelGGL((k_strided<R, Tin, WITH_D, false>), dim3(static_cast<unsigned>(blocks)), dim3(64, 4),
                       0, stream, p);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace strided_impl
}  // namespace st
