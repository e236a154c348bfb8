// Fused gradient pass: Gaussian-derivative gradient at scale sigma and the
// six-component outer product in one read of the input volume (filter
// arithmetic and products in float64, products stored as float32).
//
// Filter order per input plane: y (G and D), then x (three combinations), then
// z through per-column register windows, so that
//   g_z = Dz (Gx Gy V),  g_y = Gz (Gx Dy V),  g_x = Gz (Dx Gy V).
// A block of TY waves owns a TY (y) x 64 (x) tile of output columns and a chunk
// of z outputs (by default TY = 8 up to radius 6, where 8-row blocks still fit
// four waves per SIMD without spilling, else 4; a 4-row variant is also built
// up to radius 6 for the batch autotuner).  For every input plane (z halo of R on
// each side, reflected at the faces) the (TY + 2R) x (64 + 2R) input tile is
// staged in LDS, in two buffers used by alternate planes; the next plane's
// loads are issued before the current plane is filtered.  Each wave filters
// along y the 64 + 2R columns of its own tile row, which only it reads in the
// x filter, so one block barrier per plane (after the staging) suffices: a
// wave that writes plane j + 1's buffer has passed plane j's barrier, and one
// that would overwrite plane j's buffer (at j + 2) waits at plane j + 1's for
// every wave to finish reading it.  Each
// column's z window lives in registers; the plane loop is expanded to the window
// length (a fold over an index sequence), so every plane's results land in a
// register fixed at compile time and the window never moves.
// Products leave with non-temporal stores into workspace planes whose rows have
// the workspace pitch (the input volume has rows of nx).
#include <utility>
#include "st_device.h"

namespace st {
namespace {

// Block `blk` of the gradient pass over the volume described by p (taps wg, wd).
template <int R, typename Tin, int TY>
__device__ __forceinline__ void grad_fused_block(const GradGeo& p, const Taps& wg, const Taps& wd, int64_t blk) {
  constexpr int W = 2 * R + 1;
  constexpr int TX = kGradTX;
  constexpr int NT = TX * TY;  // threads: one per output column of the tile
  constexpr int RX = TX + 2 * R, RY = TY + 2 * R;
  constexpr int NSTAGE = (RX * RY + NT - 1) / NT;  // staged elements per thread
  // The smoothing taps are symmetric about the centre (bit for bit, as built):
  // only taps 0..R are read, so R + 1 of them occupy scalar registers.
  auto tg = [&](int k) { return wg.w[k <= R ? k : 2 * R - k]; };
  __shared__ float raw[2][RY * RX];   // input planes (exact in float32), alternating
  __shared__ double yb[2][TY * RX];   // y-filtered plane, float64

  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  // Blocks are dealt round-robin to the 8 XCDs (each with its own L2); give each
  // XCD a contiguous run of tiles so that tiles sharing halo rows meet in one L2.
  const int64_t nblk = p.x_tiles * p.y_tiles * p.nchunks;
  int64_t b = blk;
  if (nblk % 8 == 0) b = (b % 8) * (nblk / 8) + b / 8;
  const int64_t xt = b % p.x_tiles;
  b /= p.x_tiles;
  const int64_t yt = b % p.y_tiles;
  const int chunk_id = static_cast<int>(b / p.y_tiles);
  const int64_t x0 = xt * TX, y0 = yt * TY;
  const int64_t nz = p.nz, ny = p.ny, nx = p.nx;
  // z positions fit in 32 bits (each size < 2^31): their compares and the
  // reflection stay on the scalar unit; element offsets are 64-bit
  const int nzi = static_cast<int>(nz);
  const int z0 = chunk_id * static_cast<int>(p.chunk);
  const int len = (nzi - z0) < p.chunk ? (nzi - z0) : static_cast<int>(p.chunk);
  const int64_t plane = ny * nx;  // < 2^31 (checked by the host)
  const Tin* vol = static_cast<const Tin*>(p.vol);

  // in-plane offsets of this thread's staging slots (reflected at the faces)
  int off[NSTAGE];
#pragma unroll
  for (int j = 0; j < NSTAGE; ++j) {
    int s = tid + NT * j;
    if (s >= RX * RY) s = RX * RY - 1;  // padding slots repeat the last element
    const int row = s / RX, col = s - (s / RX) * RX;
    const int gy = reflect_lane(static_cast<int>(y0) - R + row, static_cast<int>(ny));
    const int gx = reflect_lane(static_cast<int>(x0) - R + col, static_cast<int>(nx));
    off[j] = gy * static_cast<int>(nx) + gx;
  }
  float pf[NSTAGE];
  auto fetch = [&](int zi) {  // loads of input plane zi into pf
    const Tin* src = vol + static_cast<int64_t>(reflect_lane(zi, nzi)) * plane;
#pragma unroll
    for (int j = 0; j < NSTAGE; ++j) pf[j] = static_cast<float>(src[off[j]]);  // halo re-read by neighbours: keep cached
  };

  // Stage plane step j (already fetched into pf) and filter it along y then x;
  // returns the three partial results of this thread's column, and prefetches
  // plane `next`.
  auto filter_plane = [&](int j, int next, bool has_next, double& a, double& bq, double& c) {
    float* rb = raw[j & 1];
#pragma unroll
    for (int t = 0; t < NSTAGE; ++t) {
      const int s = tid + NT * t;
      if (s < RX * RY) rb[s] = pf[t];
    }
    if (has_next) fetch(next);
    __syncthreads();
    // y filter of the wave's own row (columns tx and tx + 64 of RX): only this
    // wave reads it, so no block barrier separates it from the x filter
#pragma unroll
    for (int q = 0; q < (RX + 63) / 64; ++q) {
      const int col = tx + 64 * q;
      if (col < RX) {
        double g = 0.0, d = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const double v = rb[(ty + k) * RX + col];
          g = fma(tg(k), v, g);
          d = fma(wd.w[k], v, d);
        }
        yb[0][ty * RX + col] = g;
        yb[1][ty * RX + col] = d;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double ga = 0.0, gb = 0.0, dc = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double u = yb[0][ty * RX + tx + k];
      const double w = yb[1][ty * RX + tx + k];
      ga = fma(tg(k), u, ga);
      dc = fma(wd.w[k], u, dc);
      gb = fma(tg(k), w, gb);
    }
    // materialise the three results here: otherwise the compiler sinks these
    // sums towards their use in the z filter and keeps every LDS value alive
    asm volatile("" : "+v"(ga), "+v"(gb), "+v"(dc));
    a = ga;   // Gx Gy V   -> Dz gives g_z
    bq = gb;  // Gx Dy V   -> Gz gives g_y
    c = dc;   // Dx Gy V   -> Gz gives g_x
  };

  const bool active = (x0 + tx < nx) && (y0 + ty < ny);
  const int64_t out_col = (y0 + ty) * p.opitch + (x0 + tx);
  const int64_t out_plane = ny * p.opitch;

  // z windows: slot (j + k) mod W of w* holds the column's partial results of
  // input plane j - 2R + k at plane step j; the plane loop is expanded W times
  // so that every slot index is static (no register moves)
  double wa[W], wb[W], wc[W];
  fetch(z0 - R);
  const int nplanes = len + 2 * R;
#pragma unroll 1
  for (int jb = 0; jb < nplanes; jb += W) {  // block-uniform trip count
    auto step = [&]<int J>(std::integral_constant<int, J>) {
      const int j = jb + J;
      if (j < nplanes) {
        double a, bq, c;
        filter_plane(j, z0 - R + j + 1, j + 1 < nplanes, a, bq, c);
        constexpr int S = (J + 2 * R) % W;
        wa[S] = a;
        wb[S] = bq;
        wc[S] = c;
        if (j >= 2 * R && active) {
          double gz = 0.0, gy = 0.0, gx = 0.0;
#pragma unroll
          for (int k = 0; k < W; ++k) {
            gz = fma(wd.w[k], wa[(J + k) % W], gz);
            gy = fma(tg(k), wb[(J + k) % W], gy);
            gx = fma(tg(k), wc[(J + k) % W], gx);
          }
          const int64_t i = static_cast<int64_t>(z0 + j - 2 * R) * out_plane + out_col;
          __builtin_nontemporal_store(static_cast<float>(gz * gz), p.prod[0] + i);
          __builtin_nontemporal_store(static_cast<float>(gz * gy), p.prod[1] + i);
          __builtin_nontemporal_store(static_cast<float>(gz * gx), p.prod[2] + i);
          __builtin_nontemporal_store(static_cast<float>(gy * gy), p.prod[3] + i);
          __builtin_nontemporal_store(static_cast<float>(gy * gx), p.prod[4] + i);
          __builtin_nontemporal_store(static_cast<float>(gx * gx), p.prod[5] + i);
        }
      }
    };
    [&]<int... J>(std::integer_sequence<int, J...>) {
      (step(std::integral_constant<int, J>{}), ...);
    }(std::make_integer_sequence<int, W>{});
  }
}

template <int R, typename Tin, int TY = grad_tile_rows(R)>
__global__ __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(TY == 8 ? 4 : 1)))
void k_grad_fused(const GradFusedParams p) {
  grad_fused_block<R, Tin, TY>(p, p.wg, p.wd, blockIdx.x);
}

// One launch over a table of volumes.  Each entry's block range starts on a
// multiple of 8, so the XCD-aware remap inside a volume sees its own blocks
// dealt round-robin to the 8 XCDs as in a launch of its own.
template <int R, typename Tin, int TY>
__global__ __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(TY == 8 ? 4 : 1)))
void k_grad_fused_grouped(const GradFusedGroup p) {
  const int64_t b = blockIdx.x;
  const int e = group_entry(p.g.first, p.g.count, b);
  const GradGeo g = p.g.geo[e];
  const int64_t local = b - p.g.first[e];
  if (local >= g.x_tiles * g.y_tiles * g.nchunks) return;  // alignment padding (block-uniform)
  grad_fused_block<R, Tin, TY>(g, p.wg, p.wd, local);
}

template <typename Tin, int R>
hipError_t launch_r(const GradFusedParams& p, hipStream_t stream) {
  const int64_t blocks = p.x_tiles * p.y_tiles * p.nchunks;
  if (p.rows == grad_tile_rows(R)) {
    hipLaunchKernelGGL((k_grad_fused<R, Tin>), dim3(static_cast<unsigned>(blocks)), dim3(kGradTX, grad_tile_rows(R)),
                       0, stream, p);
    return hipGetLastError();
  }
  if constexpr (grad_rows_supported(R, 4) && grad_tile_rows(R) != 4) {
    if (p.rows == 4) {
      hipLaunchKernelGGL((k_grad_fused<R, Tin, 4>), dim3(static_cast<unsigned>(blocks)), dim3(kGradTX, 4), 0,
                         stream, p);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

template <typename Tin, int R>
hipError_t launch_grouped_r(int rows, const GradFusedGroup& p, int64_t blocks, hipStream_t stream) {
  if (rows == grad_tile_rows(R)) {
    hipLaunchKernelGGL((k_grad_fused_grouped<R, Tin, grad_tile_rows(R)>), dim3(static_cast<unsigned>(blocks)),
                       dim3(kGradTX, grad_tile_rows(R)), 0, stream, p);
    return hipGetLastError();
  }
  if constexpr (grad_rows_supported(R, 4) && grad_tile_rows(R) != 4) {
    if (rows == 4) {
      hipLaunchKernelGGL((k_grad_fused_grouped<R, Tin, 4>), dim3(static_cast<unsigned>(blocks)), dim3(kGradTX, 4), 0,
                         stream, p);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_grad_fused(int R, int in_dtype, const GradFusedParams& p, hipStream_t stream) {
#define ST_CASE(r) case r: return in_dtype == ST_DTYPE_U16 ? launch_r<uint16_t, r>(p, stream) \
                                                           : launch_r<float, r>(p, stream);
  switch (R) { ST_CASE(1) ST_CASE(2) ST_CASE(3) ST_CASE(4) ST_CASE(5) ST_CASE(6) ST_CASE(7) ST_CASE(8)
    default: return hipErrorInvalidValue; }
#undef ST_CASE
}

hipError_t launch_grad_fused_grouped(int R, int in_dtype, int rows, const GradFusedGroup& p, int64_t blocks,
                                     hipStream_t stream) {
  if (blocks < 1) return hipSuccess;
#define ST_CASE(r) case r: return in_dtype == ST_DTYPE_U16 ? launch_grouped_r<uint16_t, r>(rows, p, blocks, stream) \
                                                           : launch_grouped_r<float, r>(rows, p, blocks, stream);
  switch (R) { ST_CASE(1) ST_CASE(2) ST_CASE(3) ST_CASE(4) ST_CASE(5) ST_CASE(6) ST_CASE(7) ST_CASE(8)
    default: return hipErrorInvalidValue; }
#undef ST_CASE
}

}  // namespace st
