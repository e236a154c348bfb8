// C ABI of the learned orientation surrogate: validation, workspace, the layer
// sequence and the fallback to the structure-tensor path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "st_host.h"
#include "st_surrogate.h"

using st::host::device_fail;
using st::host::fail;

namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// The three tile grids of the fallback (edges 32, 64, 128), stored one after
// the other in one int array.
struct TileGrids {
  int64_t dims[st::kSgTileEdges][3];
  int64_t count[st::kSgTileEdges], start[st::kSgTileEdges];
  int64_t total = 0;
  TileGrids(int64_t nz, int64_t ny, int64_t nx) {
    for (int k = 0; k < st::kSgTileEdges; ++k) {
      const int64_t t = int64_t(32) << k;
      dims[k][0] = (nz + t - 1) / t; dims[k][1] = (ny + t - 1) / t; dims[k][2] = (nx + t - 1) / t;
      count[k] = dims[k][0] * dims[k][1] * dims[k][2];
      start[k] = total;
      total += count[k];
    }
  }
};

struct FallbackPlan {
  int mode = 0;  // 0: nothing falls back, 1: flagged tiles, 2: the whole volume
  int edge = 0;
  int64_t voxels = 0;  // voxels of the crops
  std::vector<st::SgBox> boxes;
};

// What the calling thread's last st_surrogate_infer did.
struct FallbackInfo {
  int mode = 0, tile_edge = 0;
  int64_t tiles = 0, voxels = 0;
};
thread_local FallbackInfo g_last;

// Per-chunk cost of a crop in voxel units: its launches' share of a grouped
// round and the idle tail of its small grids.
constexpr int64_t kCropCost = int64_t(1) << 16;

// Boxes of the flagged tiles of edge 32 << k, each with `halo` voxels of
// context clipped to the volume, laid out one after the other in a stack.
std::vector<st::SgBox> tile_boxes(const TileGrids& g, int k, const std::vector<int>& flags, int halo, int64_t nz,
                                  int64_t ny, int64_t nx, int64_t* voxels) {
  std::vector<st::SgBox> boxes;
  const int64_t t = int64_t(32) << k;
  const int64_t n[3] = {nz, ny, nx};
  int64_t off = 0;
  for (int64_t i = 0; i < g.count[k]; ++i) {
    if (flags[static_cast<size_t>(g.start[k] + i)] == 0) continue;
    const int64_t tc[3] = {i / (g.dims[k][1] * g.dims[k][2]), (i / g.dims[k][2]) % g.dims[k][1], i % g.dims[k][2]};
    int64_t lo[3], hi[3], c0[3], cs[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = tc[d] * t;
      hi[d] = std::min(n[d], lo[d] + t);
      c0[d] = std::max<int64_t>(0, lo[d] - halo);
      cs[d] = std::min(n[d], hi[d] + halo) - c0[d];
    }
    st::SgBox b;
    b.z0 = c0[0]; b.y0 = c0[1]; b.x0 = c0[2];
    b.cz = cs[0]; b.cy = cs[1]; b.cx = cs[2];
    b.off = off;
    b.tz0 = lo[0]; b.ty0 = lo[1]; b.tx0 = lo[2];
    b.tz1 = hi[0]; b.ty1 = hi[1]; b.tx1 = hi[2];
    off += cs[0] * cs[1] * cs[2];
    boxes.push_back(b);
  }
  *voxels = off;
  return boxes;
}

// The cheapest fallback: the flagged tiles of one edge with their halo, or
// the whole volume when the crops would cost as much.
FallbackPlan choose_fallback(const TileGrids& g, const std::vector<int>& flags, int halo, int64_t nz, int64_t ny,
                             int64_t nx) {
  FallbackPlan best;
  if (std::find(flags.begin(), flags.end(), 1) == flags.end()) return best;
  const int64_t whole = nz * ny * nx;
  best.mode = 2;
  int64_t best_cost = whole;
  for (int k = 0; k < st::kSgTileEdges; ++k) {
    int64_t vox = 0;
    std::vector<st::SgBox> boxes = tile_boxes(g, k, flags, halo, nz, ny, nx, &vox);
    const int64_t cost = vox + kCropCost * static_cast<int64_t>(boxes.size());
    if (!boxes.empty() && cost < best_cost) {
      best_cost = cost;
      best.mode = 1;
      best.edge = 32 << k;
      best.voxels = vox;
      best.boxes = std::move(boxes);
    }
  }
  return best;
}

struct Outputs {
  float *e3, *fa, *ha, *ia;
};

// Output planes per z slab of the network: as many as let the two activation
// buffers (a slab plus 4 planes on each side, 64 bytes per voxel) fit in the
// slab budget (16 GiB, or ST_SURROGATE_SLAB_BYTES), at least one.
int64_t slab_planes(int64_t nz, int64_t ny, int64_t nx) {
  size_t budget = size_t(16) << 30;
  if (const char* v = std::getenv("ST_SURROGATE_SLAB_BYTES")) {
    char* end = nullptr;
    const unsigned long long b = std::strtoull(v, &end, 10);
    if (end != v && *end == '\0' && b > 0) budget = static_cast<size_t>(b);
  }
  const size_t plane = static_cast<size_t>(ny) * static_cast<size_t>(nx) * st::kSgChannels * 2;
  const int64_t halo = 2 * (st::kSgLayers - 1);
  const int64_t fit = static_cast<int64_t>(budget / (2 * plane));
  return std::max<int64_t>(1, std::min<int64_t>(nz, fit - halo));
}

// The structure-tensor path over the whole volume, streamed in z slabs through
// `scratch` (the network's activation buffers, no longer needed): each slab's
// planes plus the path's reach on both sides (a contiguous sub-volume, whose
// interior planes come out bit for bit as in one pass over the volume) into
// temporary outputs, then a merge of the slab's own planes where the
// confidence is below the threshold.  One pass when the whole volume fits; a
// buffer of its own when the scratch cannot hold a useful slab.
int whole_fallback(const void* volume, int dtype, const uint8_t* mask, int64_t nz, int64_t ny, int64_t nx,
                   double sigma, double rho, double truncate, const double* axis_center,
                   const double* axis_direction, const float* conf, float threshold, const Outputs& o,
                   char* scratch, size_t scratch_bytes, hipStream_t stream) {
  const size_t plane = static_cast<size_t>(ny) * static_cast<size_t>(nx);
  const size_t esz = dtype == ST_DTYPE_U16 ? 2 : 4;
  const int halo = st::host::path_halo(sigma, rho, truncate);
  // bytes for a sub-volume of P planes: the path's workspace and the temporary outputs
  auto need = [&](int64_t P) -> size_t {
    const size_t w = st::host::path_workspace_bytes(P, ny, nx);
    if (w == 0) return SIZE_MAX;
    const size_t v = static_cast<size_t>(P) * plane;
    return align256(w) + (o.e3 ? align256(3 * v * 4) : 0) + (o.fa ? align256(v * 4) : 0) +
           (o.ha ? align256(v * 4) : 0) + (o.ia ? align256(v * 4) : 0);
  };
  int64_t P = 0;  // the most planes the scratch holds
  for (int64_t lo = 1, hi = nz; lo <= hi;) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (need(mid) <= scratch_bytes) { P = mid; lo = mid + 1; } else { hi = mid - 1; }
  }
  int64_t S = P == nz ? nz : P - 2 * static_cast<int64_t>(halo);  // output planes per slab
  char* base = scratch;
  char* own = nullptr;
  if (S < 16 && S < nz) {  // too thin to be worth it: a buffer of slabs of 64 planes
    P = std::min<int64_t>(nz, 64 + 2 * static_cast<int64_t>(halo));
    S = P == nz ? nz : 64;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&own), need(P), stream);
    if (e != hipSuccess || own == nullptr) {
      (void)hipGetLastError();
      return fail(ST_ERR_OUT_OF_MEMORY, "hipMallocAsync(%zu) failed: %s", need(P), hipGetErrorString(e));
    }
    base = own;
  }
  const size_t vP = static_cast<size_t>(P) * plane;
  char* q = base;
  auto take = [&](size_t b) { char* r = b ? q : nullptr; q += b; return r; };
  char* pws = take(align256(st::host::path_workspace_bytes(P, ny, nx)));
  float* pe3 = reinterpret_cast<float*>(take(o.e3 ? align256(3 * vP * 4) : 0));
  float* pfa = reinterpret_cast<float*>(take(o.fa ? align256(vP * 4) : 0));
  float* pha = reinterpret_cast<float*>(take(o.ha ? align256(vP * 4) : 0));
  float* pia = reinterpret_cast<float*>(take(o.ia ? align256(vP * 4) : 0));
  const char* stage = "fallback arguments";
  hipError_t e = hipSuccess;
  for (int64_t za = 0; za < nz && e == hipSuccess; za += S) {
    const int64_t zb = std::min(nz, za + S);
    const int64_t a = S == nz ? 0 : std::max<int64_t>(0, za - halo), b = S == nz ? nz : std::min(nz, zb + halo);
    double center[3];
    if (axis_center) {
      center[0] = axis_center[0] - static_cast<double>(a);
      center[1] = axis_center[1];
      center[2] = axis_center[2];
    }
    st::host::PathArgs pa;
    if (st::host::prepare_path(pa, static_cast<const char*>(volume) + static_cast<size_t>(a) * plane * esz, dtype,
                               mask ? mask + static_cast<size_t>(a) * plane : nullptr, b - a, ny, nx, sigma, rho,
                               truncate, axis_center ? center : nullptr, axis_direction, pe3, nullptr, pfa, pha, pia,
                               nullptr) != ST_OK) {
      e = hipErrorInvalidValue;  // cannot happen: every argument was validated
      break;
    }
    e = st::host::enqueue_path(pa, pws, stream, st::host::LaunchShape{}, true, &stage);
    if (e != hipSuccess) break;
    st::SgMergeParams m;
    m.mask = mask; m.conf = conf; m.threshold = threshold;
    m.pe3 = pe3; m.pfa = pfa; m.pha = pha; m.pia = pia;
    m.e3 = o.e3; m.fa = o.fa; m.ha = o.ha; m.ia = o.ia;
    m.n = nz * static_cast<int64_t>(plane);
    m.begin = za * static_cast<int64_t>(plane);
    m.count = (zb - za) * static_cast<int64_t>(plane);
    m.src_shift = a * static_cast<int64_t>(plane);
    m.src_n = (b - a) * static_cast<int64_t>(plane);
    stage = "surrogate_merge";
    e = st::host::timed_call(stage, stream, [&] { return st::launch_sg_merge(m, stream); });
  }
  hipError_t f = own ? hipFreeAsync(own, stream) : hipSuccess;
  if (e == hipSuccess && f != hipSuccess) { e = f; stage = "hipFreeAsync"; }
  return e == hipSuccess ? ST_OK : device_fail(e, stage);
}

// The structure-tensor path on the flagged tiles only: gather every tile with
// its halo into a crop stack, run the crops as one grouped chunk batch (chains
// when sigma's radius needs the three-pass gradient), and merge each tile's
// interior.  Synchronous: returns once the merge has finished.
int tile_fallback(const FallbackPlan& plan, const void* volume, int dtype, const uint8_t* mask, int64_t nz,
                  int64_t ny, int64_t nx, double sigma, double rho, double truncate, const double* axis_center,
                  const double* axis_direction, const float* conf, float threshold, const Outputs& o,
                  hipStream_t stream) {
  const int count = static_cast<int>(plan.boxes.size());
  const size_t V = static_cast<size_t>(plan.voxels);
  const size_t esz = dtype == ST_DTYPE_U16 ? 2 : 4;
  // host tables: first gathered row and first merged row of every crop
  std::vector<int64_t> gfirst(count), mfirst(count);
  int64_t grows = 0, mrows = 0;
  size_t pathws = 0;
  for (int c = 0; c < count; ++c) {
    const st::SgBox& b = plan.boxes[c];
    gfirst[c] = grows;
    mfirst[c] = mrows;
    grows += b.cz * b.cy;
    mrows += (b.tz1 - b.tz0) * (b.ty1 - b.ty0);
    pathws += align256(st::host::path_workspace_bytes(b.cz, b.cy, b.cx));
  }
  const size_t boxb = align256(count * sizeof(st::SgBox)), firstb = align256(count * sizeof(int64_t));
  const size_t volb = align256(V * esz), maskb = mask ? align256(V) : 0;
  const size_t e3b = o.e3 ? align256(3 * V * 4) : 0, fb = align256(V * 4);
  const size_t total = boxb + 2 * firstb + volb + maskb + e3b + (o.fa ? fb : 0) + (o.ha ? fb : 0) +
                       (o.ia ? fb : 0) + pathws;
  char* ws = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&ws), total);
  if (e != hipSuccess || ws == nullptr) {
    (void)hipGetLastError();
    return fail(ST_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) for the fallback crops failed: %s", total,
                hipGetErrorString(e));
  }
  char* q = ws;
  auto take = [&](size_t b) { char* r = b ? q : nullptr; q += b; return r; };
  st::SgBox* dbox = reinterpret_cast<st::SgBox*>(take(boxb));
  int64_t* dgfirst = reinterpret_cast<int64_t*>(take(firstb));
  int64_t* dmfirst = reinterpret_cast<int64_t*>(take(firstb));
  char* cvol = take(volb);
  uint8_t* cmask = reinterpret_cast<uint8_t*>(take(maskb));
  float* pe3 = reinterpret_cast<float*>(take(e3b));
  float* pfa = reinterpret_cast<float*>(take(o.fa ? fb : 0));
  float* pha = reinterpret_cast<float*>(take(o.ha ? fb : 0));
  float* pia = reinterpret_cast<float*>(take(o.ia ? fb : 0));
  char* pws = take(pathws);

  int status = ST_OK;
  const char* stage = "fallback tables";
  st_batch* batch = nullptr;
  do {
    e = hipMemcpyAsync(dbox, plan.boxes.data(), count * sizeof(st::SgBox), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dgfirst, gfirst.data(), count * sizeof(int64_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dmfirst, mfirst.data(), count * sizeof(int64_t), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) break;
    st::SgGatherParams gp;
    gp.vol = volume; gp.mask = mask; gp.cvol = cvol; gp.cmask = cmask;
    gp.boxes = dbox; gp.first = dgfirst; gp.count = count; gp.rows = grows; gp.ny = ny; gp.nx = nx;
    stage = "surrogate_gather";
    e = st::host::timed_call(stage, stream, [&] { return st::launch_sg_gather(dtype, gp, stream); });
    if (e != hipSuccess) break;
    std::vector<st_chunk> chunks(count);
    for (int c = 0; c < count; ++c) {
      const st::SgBox& b = plan.boxes[c];
      st_chunk& k = chunks[c];
      std::memset(&k, 0, sizeof(k));
      k.volume = cvol + static_cast<size_t>(b.off) * esz;
      k.dtype = dtype;
      k.mask = mask ? cmask + b.off : nullptr;
      k.nz = b.cz; k.ny = b.cy; k.nx = b.cx;
      k.rho = rho;
      k.origin[0] = static_cast<double>(b.z0);
      k.origin[1] = static_cast<double>(b.y0);
      k.origin[2] = static_cast<double>(b.x0);
      k.e3 = pe3 ? pe3 + 3 * b.off : nullptr;
      k.fa = pfa ? pfa + b.off : nullptr;
      k.ha = pha ? pha + b.off : nullptr;
      k.ia = pia ? pia + b.off : nullptr;
    }
    stage = nullptr;  // st_batch_* report their own errors
    status = st_batch_create(chunks.data(), count, sigma, truncate, axis_center, axis_direction, ST_BATCH_GROUPED,
                             pws, pathws, &batch);
    if (status == ST_ERR_UNSUPPORTED)
      status = st_batch_create(chunks.data(), count, sigma, truncate, axis_center, axis_direction, 0, nullptr, 0,
                               &batch);
    if (status != ST_OK) break;
    status = st_batch_launch(batch, stream);
    if (status != ST_OK) break;
    st::SgTileMergeParams mp;
    mp.boxes = dbox; mp.first = dmfirst; mp.count = count; mp.rows = mrows;
    mp.mask = mask; mp.conf = conf; mp.threshold = threshold;
    mp.pe3 = pe3; mp.pfa = pfa; mp.pha = pha; mp.pia = pia;
    mp.e3 = o.e3; mp.fa = o.fa; mp.ha = o.ha; mp.ia = o.ia;
    mp.n = nz * ny * nx; mp.ny = ny; mp.nx = nx;
    stage = "surrogate_tile_merge";
    e = st::host::timed_call(stage, stream, [&] { return st::launch_sg_tile_merge(mp, stream); });
    if (e != hipSuccess) break;
    stage = "fallback synchronize";
    e = hipStreamSynchronize(stream);
  } while (false);
  if (batch != nullptr) {
    const int d = st_batch_destroy(batch);
    if (status == ST_OK && e == hipSuccess && d != ST_OK) status = d;
  }
  // on an error, work already enqueued may still read or write the crops
  if (status != ST_OK || e != hipSuccess) (void)hipStreamSynchronize(stream);
  const hipError_t f = hipFree(ws);
  if (status != ST_OK) return status;
  if (e != hipSuccess) return device_fail(e, stage);
  if (f != hipSuccess) return device_fail(f, "hipFree");
  return ST_OK;
}

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

  // ---- workspace: activations of one z slab, packed weights, confidence, tile flags ----
  const int C = st::kSgChannels;
  const int64_t slab = slab_planes(nz, ny, nx);
  const size_t act = align256(static_cast<size_t>(std::min<int64_t>(nz, slab + 2 * (st::kSgLayers - 1))) * ny * nx *
                              C * 2);
  const size_t w1b = align256(32 * 32 * 2);
  const size_t w25b = align256(4 * 27 * static_cast<size_t>(C) * C * 2);
  const bool own_conf = fallback && confidence == nullptr;
  const size_t confb = own_conf ? align256(N * 4) : 0;
  TileGrids grids(nz, ny, nx);
  const size_t flagb = fallback ? align256(grids.total * 4) : 0;
  const size_t total = w1b + w25b + confb + flagb;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  // the activations (the bulk) serve a whole-volume fallback as its scratch
  char* acts = nullptr;
  char* ws = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&acts), 2 * act, stream);
  if (e == hipSuccess && acts != nullptr) {
    e = hipMallocAsync(reinterpret_cast<void**>(&ws), total, stream);
    if (e != hipSuccess || ws == nullptr) (void)hipFreeAsync(acts, stream);
  }
  if (e != hipSuccess || acts == nullptr || ws == nullptr) {
    (void)hipGetLastError();
    return fail(ST_ERR_OUT_OF_MEMORY, "hipMallocAsync(%zu + %zu) failed: %s", 2 * act, total,
                hipGetErrorString(e));
  }
  char* q = ws;
  auto take = [&](size_t b) { char* r = b ? q : nullptr; q += b; return r; };
  __bf16* actA = reinterpret_cast<__bf16*>(acts);
  __bf16* actB = reinterpret_cast<__bf16*>(acts + act);
  __bf16* w1 = reinterpret_cast<__bf16*>(take(w1b));
  __bf16* w25 = reinterpret_cast<__bf16*>(take(w25b));
  float* conf = own_conf ? reinterpret_cast<float*>(take(confb)) : confidence;
  int* dflags = reinterpret_cast<int*>(take(flagb));

  const float* blob = static_cast<const float*>(weights);
  const char* stage = "surrogate_pack";
  int status = ST_OK;
  g_last = FallbackInfo{};
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
    __bf16* bufs[2] = {actA, actB};
    // z slabs: for output planes [za, zb), layer l computes the planes within
    // 5 - l of them (each later layer needs one more plane on each side)
    for (int64_t za = 0; za < nz && e == hipSuccess; za += slab) {
      const int64_t zb = std::min(nz, za + slab);
      const __bf16* in = nullptr;
      int64_t in_z0 = 0;
      for (int layer = 1; layer <= st::kSgLayers && e == hipSuccess; ++layer) {
        const int64_t g = st::kSgLayers - layer;
        p.z_lo = std::max<int64_t>(0, za - g);
        p.z_hi = std::min(nz, zb + g);
        p.in = in;
        p.in_z0 = in_z0;
        p.out = layer < st::kSgLayers ? bufs[(layer - 1) & 1] : nullptr;
        p.out_z0 = p.z_lo;
        p.w = layer >= 2 ? w25 + static_cast<size_t>(layer - 2) * 27 * C * C : nullptr;
        p.bias = layer == 1 ? blob + st::kSgOffB1
                            : blob + st::kSgOffW2 + (layer - 2) * st::kSgLayerStride + C * C * 27;
        stage = layer == 1 ? "surrogate_conv1" : (layer == st::kSgLayers ? "surrogate_conv5_head" : "surrogate_conv");
        e = st::host::timed_call(stage, stream, [&] { return st::launch_sg_conv(layer, dtype, p, stream); });
        in = p.out;
        in_z0 = p.z_lo;
      }
    }
    if (e != hipSuccess || !fallback) break;
    // which tiles hold voxels below the threshold (the host needs the answer)
    st::SgTileFlagParams fp;
    fp.conf = conf; fp.mask = mask; fp.threshold = static_cast<float>(min_confidence);
    fp.nz = nz; fp.ny = ny; fp.nx = nx;
    for (int k = 0; k < st::kSgTileEdges; ++k) { fp.flags[k] = dflags + grids.start[k]; fp.tiles[k] = grids.count[k]; }
    stage = "surrogate_tile_flags";
    e = st::host::timed_call(stage, stream, [&] { return st::launch_sg_tile_flags(fp, stream); });
    if (e != hipSuccess) break;
    std::vector<int> flags(static_cast<size_t>(grids.total));
    stage = "tile flags to the host";
    e = hipMemcpyAsync(flags.data(), dflags, flags.size() * sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) break;
    const int halo = st::host::path_halo(sigma, rho, truncate);
    const FallbackPlan plan = choose_fallback(grids, flags, halo, nz, ny, nx);
    g_last.mode = plan.mode;
    g_last.tile_edge = plan.edge;
    g_last.tiles = static_cast<int64_t>(plan.boxes.size());
    g_last.voxels = plan.mode == 2 ? n : plan.voxels;
    if (plan.mode == 0) break;  // every voxel keeps the surrogate's outputs
    Outputs out{e3, fa, ha, ia};
    if (plan.mode == 2) {
      status = whole_fallback(volume, dtype, mask, nz, ny, nx, sigma, rho, truncate, axis_center, axis_direction,
                              conf, static_cast<float>(min_confidence), out, acts, 2 * act, stream);
    } else {
      status = tile_fallback(plan, volume, dtype, mask, nz, ny, nx, sigma, rho, truncate, axis_center,
                             axis_direction, conf, static_cast<float>(min_confidence), out, stream);
    }
  } while (false);
  hipError_t f = hipFreeAsync(ws, stream);
  if (acts != nullptr) (void)hipFreeAsync(acts, stream);
  if (status != ST_OK) return status;
  if (e == hipSuccess && f != hipSuccess) { e = f; stage = "hipFreeAsync"; }
  if (e != hipSuccess) return device_fail(e, stage);
  return ST_OK;
}

extern "C" int st_surrogate_fallback_info(int* mode, int* tile_edge, int64_t* tiles, int64_t* voxels) {
  if (mode) *mode = g_last.mode;
  if (tile_edge) *tile_edge = g_last.tile_edge;
  if (tiles) *tiles = g_last.tiles;
  if (voxels) *voxels = g_last.voxels;
  return ST_OK;
}

// ---- training: gradient of the objective on a stack of patches, and Adam ---------

namespace {

struct TrainPlan {
  int64_t n = 0;                // voxels of the stack
  size_t act = 0, w1 = 0, w25 = 0, wpart = 0, hpart = 0, stats = 0, total = 0;
  int head_blocks = 0;
};

bool train_plan(int64_t npatch, int64_t patch, TrainPlan* t) {
  if (npatch < 1 || patch < 1 || patch > st::kSgTrainMaxX) return false;
  int64_t n;
  if (__builtin_mul_overflow(npatch, patch * patch * patch, &n)) return false;
  if (n > (int64_t(1) << 31)) return false;
  const int C = st::kSgChannels;
  t->n = n;
  t->act = align256(static_cast<size_t>(n) * C * 2);
  t->w1 = align256(32 * 32 * 2);
  t->w25 = align256(4 * 27 * static_cast<size_t>(C) * C * 2);
  t->wpart = align256(static_cast<size_t>(st::kSgWgradBlocks) * (27 * C * C + C) * 4);
  t->head_blocks = static_cast<int>(std::min<int64_t>(1024, (n + 255) / 256));
  t->hpart = align256(static_cast<size_t>(t->head_blocks) * st::kSgHeadSums * 4);
  t->stats = align256(st::kSgHeadSums * 4);
  // x1..x5, two gradient buffers, forward and backward weights, partials, raw sums
  t->total = 7 * t->act + t->w1 + 2 * t->w25 + t->wpart + t->hpart + t->stats;
  return true;
}

}  // namespace

extern "C" size_t st_surrogate_grad_workspace_bytes(int64_t npatch, int64_t patch) {
  TrainPlan t;
  return train_plan(npatch, patch, &t) ? t.total : 0;
}

extern "C" int st_surrogate_grad(const void* patches, int dtype, int64_t npatch, int64_t patch,
                                 const float* target_e3, const float* target_fa, const uint8_t* weight,
                                 const float* params, double conf_weight, float* grad, float* stats,
                                 void* workspace, size_t workspace_bytes, void* stream_) {
  st::host::clear_error();
  if (patches == nullptr || target_e3 == nullptr || target_fa == nullptr || weight == nullptr ||
      params == nullptr || grad == nullptr || stats == nullptr)
    return fail(ST_ERR_INVALID_ARG, "st_surrogate_grad: a required pointer is NULL");
  if (!std::isfinite(conf_weight) || conf_weight < 0.0)
    return fail(ST_ERR_INVALID_ARG, "conf_weight must be finite and >= 0");
  if (dtype != ST_DTYPE_U16 && dtype != ST_DTYPE_F32)
    return fail(ST_ERR_INVALID_ARG, "dtype %d is neither ST_DTYPE_U16 nor ST_DTYPE_F32", dtype);
  TrainPlan t;
  if (!train_plan(npatch, patch, &t))
    return fail(ST_ERR_INVALID_ARG, "npatch %lld x patch %lld: need npatch >= 1, 1 <= patch <= %d",
                (long long)npatch, (long long)patch, st::kSgTrainMaxX);
  if (workspace == nullptr && workspace_bytes != 0)
    return fail(ST_ERR_INVALID_ARG, "workspace is NULL but workspace_bytes is %zu", workspace_bytes);
  if (workspace != nullptr && workspace_bytes < t.total)
    return fail(ST_ERR_INVALID_ARG, "workspace_bytes %zu < required %zu", workspace_bytes, t.total);
  if (workspace == nullptr && st::host::alloc_fault_injected())
    return fail(ST_ERR_OUT_OF_MEMORY, "training workspace allocation failed (ST_FAULT_INJECT=alloc)");
  const size_t N = static_cast<size_t>(t.n);
  const size_t esz = dtype == ST_DTYPE_U16 ? 2 : 4;
  const size_t wbytes = 4 * static_cast<size_t>(ST_SURROGATE_WEIGHTS);
  int st;
  if ((st = st::host::check_device_buffer(patches, N * esz, "patches")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(target_e3, 3 * N * 4, "target_e3")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(target_fa, N * 4, "target_fa")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(weight, N, "weight")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(params, wbytes, "params")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(grad, wbytes, "grad")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(stats, st::kSgTrainStats * 4, "stats")) != ST_OK) return st;
  if ((st = st::host::check_device_buffer(workspace, t.total, "workspace")) != ST_OK) return st;
  for (const void* q : {static_cast<const void*>(target_e3), static_cast<const void*>(target_fa),
                        static_cast<const void*>(params), static_cast<const void*>(grad),
                        static_cast<const void*>(stats)})
    if ((reinterpret_cast<uintptr_t>(q) % 4) != 0) return fail(ST_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
  if ((reinterpret_cast<uintptr_t>(patches) % esz) != 0)
    return fail(ST_ERR_INVALID_ARG, "patches are not aligned to their element size");

  hipStream_t stream = static_cast<hipStream_t>(stream_);
  char* ws = static_cast<char*>(workspace);
  bool owned = false;
  if (ws == nullptr) {
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&ws), t.total, stream);
    if (e != hipSuccess || ws == nullptr) {
      (void)hipGetLastError();
      return fail(ST_ERR_OUT_OF_MEMORY, "hipMallocAsync(%zu) failed: %s", t.total, hipGetErrorString(e));
    }
    owned = true;
  }
  char* q = ws;
  auto take = [&](size_t b) { char* r = q; q += b; return r; };
  __bf16* xact[6] = {nullptr};
  for (int l = 1; l <= 5; ++l) xact[l] = reinterpret_cast<__bf16*>(take(t.act));
  __bf16* gbuf[2] = {reinterpret_cast<__bf16*>(take(t.act)), reinterpret_cast<__bf16*>(take(t.act))};
  __bf16* w1 = reinterpret_cast<__bf16*>(take(t.w1));
  __bf16* w25 = reinterpret_cast<__bf16*>(take(t.w25));
  __bf16* w25t = reinterpret_cast<__bf16*>(take(t.w25));
  float* wpart = reinterpret_cast<float*>(take(t.wpart));
  float* hpart = reinterpret_cast<float*>(take(t.hpart));
  float* sums = reinterpret_cast<float*>(take(t.stats));  // head gradient (165) and loss sums (6)

  const int C = st::kSgChannels;
  const int64_t P = patch;
  const int64_t nz = npatch * P, ny = P, nx = P;
  const int64_t rows = nz * ny;
  const int wb = static_cast<int>(std::min<int64_t>(st::kSgWgradBlocks, rows));
  const float* blob = params;
  const char* stage = "surrogate_pack";
  hipError_t e = hipSuccess;
  do {
    if ((e = st::launch_sg_pack(blob, w1, w25, stream)) != hipSuccess) break;
    stage = "surrogate_pack_bwd";
    if ((e = st::launch_sg_pack_bwd(blob, w25t, stream)) != hipSuccess) break;
    // forward: every layer stores its bf16 activation
    st::SgConvParams p;
    std::memset(&p, 0, sizeof(p));
    p.vol = patches;
    p.w1 = w1;
    p.scale_offset = blob;
    p.n = t.n; p.nz = nz; p.ny = ny; p.nx = nx;
    p.x_tiles = (nx + 31) / 32;
    p.y_tiles = (ny + 7) / 8;
    p.zchunk = 16;
    p.z_lo = 0; p.z_hi = nz; p.in_z0 = 0; p.out_z0 = 0;  // whole-stack buffers
    for (int layer = 1; layer <= st::kSgLayers && e == hipSuccess; ++layer) {
      p.in = layer == 1 ? nullptr : xact[layer - 1];
      p.out = xact[layer];
      p.w = layer >= 2 ? w25 + static_cast<size_t>(layer - 2) * 27 * C * C : nullptr;
      p.bias = layer == 1 ? blob + st::kSgOffB1 : blob + st::kSgOffW2 + (layer - 2) * st::kSgLayerStride + C * C * 27;
      stage = "surrogate_train_forward";
      e = st::launch_sg_conv_hidden(layer == 1, dtype, p, stream);
    }
    if (e != hipSuccess) break;
    // head, loss, g5
    st::SgHeadParams h;
    h.x5 = xact[5];
    h.head_w = blob + st::kSgOffHead;
    h.head_b = blob + st::kSgOffHead + 5 * C;
    h.target = target_e3;
    h.target_fa = target_fa;
    h.weight = weight;
    h.g5 = gbuf[0];
    h.partial = hpart;
    h.n = t.n;
    h.w_conf = static_cast<float>(conf_weight);
    stage = "surrogate_train_head";
    if ((e = st::launch_sg_head_train(h, t.head_blocks, stream)) != hipSuccess) break;
    stage = "surrogate_train_reduce";
    if ((e = st::launch_sg_reduce(hpart, t.head_blocks, st::kSgHeadSums, 0, sums, stream)) != hipSuccess) break;
    // layers 5..2: weight gradient, then the backward data pass into layer - 1
    st::SgWgradParams wg;
    std::memset(&wg, 0, sizeof(wg));
    wg.partial = wpart;
    wg.nz = nz; wg.ny = ny; wg.nx = nx;
    wg.rows_per_block = (rows + wb - 1) / wb;
    int cur = 0;
    for (int layer = st::kSgLayers; layer >= 2 && e == hipSuccess; --layer) {
      wg.g = gbuf[cur];
      wg.x = xact[layer - 1];
      stage = "surrogate_train_wgrad";
      if ((e = st::launch_sg_wgrad(wg, wb, stream)) != hipSuccess) break;
      stage = "surrogate_train_reduce";
      if ((e = st::launch_sg_reduce(wpart, wb, 27 * C * C + C, 1, grad + st::kSgOffW2 + (layer - 2) * st::kSgLayerStride,
                                    stream)) != hipSuccess)
        break;
      p.in = gbuf[cur];
      p.prev = xact[layer - 1];
      p.out = gbuf[1 - cur];
      p.w = w25t + static_cast<size_t>(layer - 2) * 27 * C * C;
      p.bias = nullptr;
      stage = "surrogate_train_backward";
      if ((e = st::launch_sg_conv_bwd(p, stream)) != hipSuccess) break;
      cur = 1 - cur;
    }
    if (e != hipSuccess) break;
    wg.g = gbuf[cur];
    wg.x = nullptr;
    wg.vol = patches;
    wg.scale_offset = blob;
    stage = "surrogate_train_wgrad1";
    if ((e = st::launch_sg_wgrad1(dtype, wg, wb, stream)) != hipSuccess) break;
    stage = "surrogate_train_reduce";
    if ((e = st::launch_sg_reduce(wpart, wb, 27 * C + C, 0, grad + st::kSgOffW1, stream)) != hipSuccess) break;
    // the head gradient (Wh, bh) into place; everything divided by the weight sum
    if ((e = st::launch_sg_reduce(sums, 1, 5 * C + 5, 0, grad + st::kSgOffHead, stream)) != hipSuccess) break;
    stage = "surrogate_train_finish";
    e = st::launch_sg_finish(grad, ST_SURROGATE_WEIGHTS, sums + 5 * C + 5, static_cast<float>(conf_weight), stats,
                             stream);
  } while (false);
  if (owned) {
    hipError_t f = hipFreeAsync(ws, stream);
    if (e == hipSuccess && f != hipSuccess) { e = f; stage = "hipFreeAsync"; }
  }
  if (e != hipSuccess) return device_fail(e, stage);
  return ST_OK;
}

extern "C" int st_surrogate_adam(float* params, const float* grad, float* adam_m, float* adam_v, int64_t step,
                                 double lr, double beta1, double beta2, double eps, void* stream) {
  st::host::clear_error();
  if (params == nullptr || grad == nullptr || adam_m == nullptr || adam_v == nullptr)
    return fail(ST_ERR_INVALID_ARG, "st_surrogate_adam: a required pointer is NULL");
  if (step < 1) return fail(ST_ERR_INVALID_ARG, "step must be >= 1");
  if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return fail(ST_ERR_INVALID_ARG, "need lr >= 0, 0 <= beta1, beta2 < 1 and eps > 0");
  const size_t wbytes = 4 * static_cast<size_t>(ST_SURROGATE_WEIGHTS);
  int st;
  for (const void* q : {static_cast<const void*>(params), static_cast<const void*>(grad),
                        static_cast<const void*>(adam_m), static_cast<const void*>(adam_v)})
    if ((st = st::host::check_device_buffer(q, wbytes, "Adam buffer")) != ST_OK) return st;
  hipError_t e = st::launch_sg_adam(params, grad, adam_m, adam_v, ST_SURROGATE_WEIGHTS, 2, step,
                                    static_cast<float>(lr), static_cast<float>(beta1), static_cast<float>(beta2),
                                    static_cast<float>(eps), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "surrogate_adam");
  return ST_OK;
}
