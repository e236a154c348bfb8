// C ABI of the learned orientation surrogate: validation, workspace, the layer
// sequence and the fallback to the structure-tensor path.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "st_host.h"
#include "st_surrogate.h"

using st::host::device_fail;
using st::host::fail;

namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" int st_surrogate_infer(const void* volume, int dtype, const uint8_t* mask, int64_t nz,
                                  int64_t ny, int64_t nx, const void* weights, size_t weights_bytes,
                                  double min_confidence, double sigma, double rho, double truncate,
                                  const double* axis_center, const double* axis_direction, float* e3,
                                  float* fa, float* ha, float* ia, float* confidence, void* stream_) {
  st::host::clear_error();
  // ---- host-only validation ----
  if (volume == nullptr) return fail(ST_ERR_INVALID_ARG, "volume is NULL");
  if (dtype != ST_DTYPE_U16 && dtype != ST_DTYPE_F32)
    return fail(ST_ERR_INVALID_ARG, "dtype %d is neither ST_DTYPE_U16 nor ST_DTYPE_F32", dtype);
  int64_t n = 0;
  int st = st::host::check_sizes(nz, ny, nx, &n);
  if (st != ST_OK) return st;
  if (weights == nullptr) return fail(ST_ERR_INVALID_ARG, "weights is NULL");
  const size_t wbytes = 4 * static_cast<size_t>(ST_SURROGATE_WEIGHTS);
  if (weights_bytes < wbytes)
    return fail(ST_ERR_INVALID_ARG, "weights_bytes %zu < %zu (ST_SURROGATE_WEIGHTS float32 values)",
                weights_bytes, wbytes);
  if (!std::isfinite(min_confidence) || min_confidence < 0.0 || min_confidence > 1.0)
    return fail(ST_ERR_INVALID_ARG, "min_confidence must lie in [0, 1]");
  // a fallback only matters when an output st_compute also produces is requested
  const bool fallback = min_confidence > 0.0 && (e3 || fa || ha || ia);
  if (min_confidence > 0.0 && (st = st::host::check_scales(sigma, rho, truncate)) != ST_OK) return st;
  double unit[3] = {0, 0, 0};
  if ((st = st::host::check_axis_args(axis_center, axis_direction, unit)) != ST_OK) return st;
  const bool has_axis = axis_center != nullptr;
  if (!has_axis && (ha != nullptr || ia != nullptr))
    return fail(ST_ERR_INVALID_ARG, "ha / ia need an axis (axis_center and axis_direction)");
  if (!e3 && !fa && !ha && !ia && !confidence) return fail(ST_ERR_INVALID_ARG, "no output requested");
  if (st::host::alloc_fault_injected())
    return fail(ST_ERR_OUT_OF_MEMORY, "surrogate workspace allocation failed (ST_FAULT_INJECT=alloc)");

  // ---- device buffer checks ----
  const size_t N = static_cast<size_t>(n);
  const size_t esz = dtype == ST_DTYPE_U16 ? 2 : 4;
  if ((st = st::host::check_device_buffer(volume, N * esz, "volume")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(mask, N, "mask")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(weights, wbytes, "weights")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(e3, 3 * N * 4, "e3")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(fa, N * 4, "fa")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(ha, N * 4, "ha")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(ia, N * 4, "ia")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(confidence, N * 4, "confidence")) != ST_OK) return st;
  if ((reinterpret_cast<uintptr_t>(volume) % esz) != 0)
    return fail(ST_ERR_INVALID_ARG, "volume is not aligned to its element size");
  for (const void* q : {static_cast<const void*>(weights), static_cast<const void*>(e3),
                        static_cast<const void*>(fa), static_cast<const void*>(ha),
                        static_cast<const void*>(ia), static_cast<const void*>(confidence)})
    if (q && (reinterpret_cast<uintptr_t>(q) % 4) != 0)
      return fail(ST_ERR_INVALID_ARG, "weights and float outputs must be 4-byte aligned");

  // ---- workspace: activations, packed weights, fallback buffers ----
  const int C = st::kSgChannels;
  const size_t act = align256(N * C * 2);
  const size_t w1b = align256(32 * 32 * 2);
  const size_t w25b = align256(4 * 27 * static_cast<size_t>(C) * C * 2);
  const bool own_conf = fallback && confidence == nullptr;
  const size_t confb = own_conf ? align256(N * 4) : 0;
  const size_t plainw = fallback ? st::host::path_workspace_bytes(nz, ny, nx) : 0;
  if (fallback && plainw == 0) return fail(ST_ERR_INVALID_ARG, "workspace size of the volume overflows");
  const size_t pe3b = fallback && e3 ? align256(3 * N * 4) : 0;
  const size_t pfab = fallback && fa ? align256(N * 4) : 0;
  const size_t phab = fallback && ha ? align256(N * 4) : 0;
  const size_t piab = fallback && ia ? align256(N * 4) : 0;
  const size_t total = 2 * act + w1b + w25b + confb + plainw + pe3b + pfab + phab + piab;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  char* ws = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&ws), total, stream);
  if (e != hipSuccess || ws == nullptr) {
    (void)hipGetLastError();
    return fail(ST_ERR_OUT_OF_MEMORY, "hipMallocAsync(%zu) failed: %s", total, hipGetErrorString(e));
  }
  char* q = ws;
  auto take = [&](size_t b) { char* r = b ? q : nullptr; q += b; return r; };
  __bf16* actA = reinterpret_cast<__bf16*>(take(act));
  __bf16* actB = reinterpret_cast<__bf16*>(take(act));
  __bf16* w1 = reinterpret_cast<__bf16*>(take(w1b));
  __bf16* w25 = reinterpret_cast<__bf16*>(take(w25b));
  float* conf = own_conf ? reinterpret_cast<float*>(take(confb)) : confidence;
  char* pws = take(plainw);
  float* pe3 = reinterpret_cast<float*>(take(pe3b));
  float* pfa = reinterpret_cast<float*>(take(pfab));
  float* pha = reinterpret_cast<float*>(take(phab));
  float* pia = reinterpret_cast<float*>(take(piab));

  const float* blob = static_cast<const float*>(weights);
  const char* stage = "surrogate_pack";
  do {
    e = st::host::timed_call("surrogate_pack", stream, [&] { return st::launch_sg_pack(blob, w1, w25, stream); });
    if (e != hipSuccess) break;
    st::SgConvParams p;
    std::memset(&p, 0, sizeof(p));
    p.vol = volume;
    p.w1 = w1;
    p.scale_offset = blob;
    p.head_w = blob + st::kSgOffHead;
    p.head_b = blob + st::kSgOffHead + 5 * C;
    p.mask = mask;
    p.e3 = e3; p.fa = fa; p.ha = ha; p.ia = ia; p.conf = conf;
    p.n = n; p.nz = nz; p.ny = ny; p.nx = nx;
    p.x_tiles = (nx + 31) / 32;
    p.y_tiles = (ny + 7) / 8;  // 8 output rows per block
    p.zchunk = 16;
    p.has_axis = has_axis;
    if (has_axis)
      for (int i = 0; i < 3; ++i) { p.center[i] = axis_center[i]; p.dir[i] = unit[i]; }
    const __bf16* in = nullptr;
    __bf16* bufs[2] = {actA, actB};
    for (int layer = 1; layer <= st::kSgLayers && e == hipSuccess; ++layer) {
      p.in = in;
      p.out = layer < st::kSgLayers ? bufs[(layer - 1) & 1] : nullptr;
      p.w = layer >= 2 ? w25 + static_cast<size_t>(layer - 2) * 27 * C * C : nullptr;
      p.bias = layer == 1 ? blob + st::kSgOffB1
                          : blob + st::kSgOffW2 + (layer - 2) * st::kSgLayerStride + C * C * 27;
      stage = layer == 1 ? "surrogate_conv1" : (layer == st::kSgLayers ? "surrogate_conv5_head" : "surrogate_conv");
      e = st::host::timed_call(stage, stream, [&] { return st::launch_sg_conv(layer, dtype, p, stream); });
      in = p.out;
    }
    if (e != hipSuccess || !fallback) break;
    // fallback: the structure-tensor path on the whole volume, then a per-voxel merge
    st::host::PathArgs pa;
    st = st::host::prepare_path(pa, volume, dtype, mask, nz, ny, nx, sigma, rho, truncate, axis_center,
                                axis_direction, pe3, nullptr, pfa, pha, pia, nullptr);
    if (st != ST_OK) {  // cannot happen: every argument was validated above
      e = hipErrorInvalidValue;
      stage = "fallback arguments";
      break;
    }
    e = st::host::enqueue_path(pa, pws, stream, st::host::LaunchShape{}, true, &stage);
    if (e != hipSuccess) break;
    st::SgMergeParams m;
    m.mask = mask; m.conf = conf; m.threshold = static_cast<float>(min_confidence);
    m.pe3 = pe3; m.pfa = pfa; m.pha = pha; m.pia = pia;
    m.e3 = e3; m.fa = fa; m.ha = ha; m.ia = ia; m.n = n;
    stage = "surrogate_merge";
    e = st::host::timed_call("surrogate_merge", stream, [&] { return st::launch_sg_merge(m, stream); });
  } while (false);
  hipError_t f = hipFreeAsync(ws, stream);
  if (e == hipSuccess && f != hipSuccess) { e = f; stage = "hipFreeAsync"; }
  if (e != hipSuccess) return device_fail(e, stage);
  return ST_OK;
}
