// Chunk batches: many independent volumes through the structure-tensor path as
// one unit of work (the paper's chunk-based processing with padding,
// Implementation section), built for one GPU with a large HBM.
//
// Chunks are dealt to up to ST_BATCH_MAX_LANES chains, largest first and each to
// the chain with the least voxels so far (longest-processing-time order); each
// chain owns a workspace slot sized for the largest chunk and a stream of its
// own, so small chunks that cannot fill the chip alone run side by side.  The
// fork / join of the chains is recorded once into a HIP graph and replayed.
// Every output is computed by the same kernels with the same per-voxel
// summation order in every configuration, so results are bitwise independent
// of the chain count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <vector>

#include "st_host.h"

using st::host::device_fail;
using st::host::fail;

struct st_batch {
  std::vector<st::host::PathArgs> chunks;
  size_t slot_bytes = 0;  // workspace of the largest chunk
  int slots = 0;          // workspace slots (the largest chain count possible)
  char* ws = nullptr;
  bool owned = false;
  int device = 0;
  // configuration
  int lanes = 1;
  bool use_graph = true;
  st::host::LaunchShape shape;
  double best_ms = 0.0;
  // runtime objects
  hipStream_t cap = nullptr;  // origin of the captured fork / join
  hipStream_t lane_stream[ST_BATCH_MAX_LANES] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[ST_BATCH_MAX_LANES] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<std::vector<int>> plan;  // chunk indices of every chain, in launch order
};

namespace {

// Restores the caller's current device on scope exit.
struct DeviceScope {
  int saved = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int dev) {
    err = hipGetDevice(&saved);
    if (err == hipSuccess && saved != dev) err = hipSetDevice(dev);
  }
  ~DeviceScope() {
    int cur = -1;
    if (saved >= 0 && hipGetDevice(&cur) == hipSuccess && cur != saved) (void)hipSetDevice(saved);
  }
};

void make_plan(st_batch* b) {
  const int n = static_cast<int>(b->chunks.size());
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int i, int j) { return b->chunks[i].n > b->chunks[j].n; });
  b->plan.assign(b->lanes, {});
  std::vector<int64_t> load(b->lanes, 0);
  for (int i : order) {
    const int k = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    b->plan[k].push_back(i);
    load[k] += b->chunks[i].n;
  }
}

// Fork from `root` into the chains, enqueue every chunk, join back into `root`.
hipError_t enqueue_all(st_batch* b, hipStream_t root, const char** stage) {
  *stage = "fork";
  hipError_t e = hipEventRecord(b->fork, root);
  if (e != hipSuccess) return e;
  for (int k = 0; k < b->lanes; ++k) {
    if (b->plan[k].empty()) continue;
    hipStream_t s = b->lane_stream[k];
    if ((e = hipStreamWaitEvent(s, b->fork, 0)) != hipSuccess) return e;
    char* ws = b->ws + static_cast<size_t>(k) * b->slot_bytes;
    for (int i : b->plan[k])
      if ((e = st::host::enqueue_path(b->chunks[i], ws, s, b->shape, false, stage)) != hipSuccess) return e;
    *stage = "join";
    if ((e = hipEventRecord(b->join[k], s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(root, b->join[k], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

void drop_graph(st_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Re-plans for the current configuration and, in graph mode, captures the graph.
int rebuild(st_batch* b) {
  make_plan(b);
  drop_graph(b);
  if (!b->use_graph) return ST_OK;
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return device_fail(e, "hipStreamBeginCapture");
  const char* stage = "";
  hipError_t ee = enqueue_all(b, b->cap, &stage);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);  // always ends the capture, also after a failure
  if (ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return device_fail(ee, stage);
  }
  if (e != hipSuccess) return device_fail(e, "hipStreamEndCapture");
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return device_fail(e, "hipGraphInstantiate");
  }
  return ST_OK;
}

int launch(st_batch* b, hipStream_t stream) {
  if (b->use_graph) {
    hipError_t e = hipGraphLaunch(b->exec, stream);
    return e == hipSuccess ? ST_OK : device_fail(e, "hipGraphLaunch");
  }
  const char* stage = "";
  hipError_t e = enqueue_all(b, stream, &stage);
  return e == hipSuccess ? ST_OK : device_fail(e, stage);
}

void release(st_batch* b) {
  if (b == nullptr) return;
  drop_graph(b);
  for (int k = 0; k < ST_BATCH_MAX_LANES; ++k) {
    if (b->lane_stream[k]) (void)hipStreamDestroy(b->lane_stream[k]);
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
  }
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->owned && b->ws) (void)hipFree(b->ws);
  delete b;
}

bool slot_plan(const st_chunk* chunks, int nchunks, size_t* slot) {
  size_t m = 0;
  for (int i = 0; i < nchunks; ++i) {
    const st_chunk& c = chunks[i];
    int64_t n = 0;
    if (c.nz < 1 || c.ny < 1 || c.nx < 1 || __builtin_mul_overflow(c.nz, c.ny, &n) ||
        __builtin_mul_overflow(n, c.nx, &n))
      return false;
    const size_t w = st::host::path_workspace_bytes(c.nz, c.ny, c.nx);
    if (w == 0) return false;
    m = std::max(m, w);
  }
  *slot = m;
  return true;
}

}  // namespace

extern "C" {

size_t st_batch_workspace_bytes(const st_chunk* chunks, int nchunks, int lanes) {
  if (chunks == nullptr || nchunks < 1 || lanes < 0 || lanes > ST_BATCH_MAX_LANES) return 0;
  size_t slot = 0;
  if (!slot_plan(chunks, nchunks, &slot)) return 0;
  const size_t slots = lanes == 0 ? ST_BATCH_MAX_LANES : static_cast<size_t>(lanes);
  size_t total = 0;
  if (__builtin_mul_overflow(slot, slots, &total)) return 0;
  return total;
}

int st_batch_create(const st_chunk* chunks, int nchunks, double sigma, double truncate,
                    const double* axis_center, const double* axis_direction, int lanes,
                    void* workspace, size_t workspace_bytes, st_batch** out) {
  st::host::clear_error();
  // ---- host-only validation ----
  if (out == nullptr) return fail(ST_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (chunks == nullptr || nchunks < 1) return fail(ST_ERR_INVALID_ARG, "need at least one chunk");
  if (lanes < 0 || lanes > ST_BATCH_MAX_LANES)
    return fail(ST_ERR_INVALID_ARG, "lanes %d is outside 0..%d", lanes, ST_BATCH_MAX_LANES);
  if ((axis_center == nullptr) != (axis_direction == nullptr))
    return fail(ST_ERR_INVALID_ARG, "axis_center and axis_direction must both be given or both be NULL");
  std::vector<st::host::PathArgs> args(nchunks);
  for (int i = 0; i < nchunks; ++i) {
    const st_chunk& c = chunks[i];
    double center[3] = {0, 0, 0};
    if (axis_center) {
      for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(c.origin[d]))
          return fail(ST_ERR_INVALID_ARG, "chunk %d: origin must be finite", i);
        center[d] = axis_center[d] - c.origin[d];  // the axis in the chunk's own voxel coordinates
      }
    }
    int st = st::host::prepare_path(args[i], c.volume, c.dtype, c.mask, c.nz, c.ny, c.nx, sigma, c.rho,
                                    truncate, axis_center ? center : nullptr, axis_direction, c.e3,
                                    c.evals, c.fa, c.ha, c.ia, c.flags);
    if (st != ST_OK) return fail(st, "chunk %d: %s", i, st_last_error());
  }
  size_t slot = 0;
  if (!slot_plan(chunks, nchunks, &slot)) return fail(ST_ERR_INVALID_ARG, "chunk sizes out of range");
  const int slots = lanes == 0 ? ST_BATCH_MAX_LANES : lanes;
  const size_t need = slot * static_cast<size_t>(slots);
  if (workspace == nullptr && workspace_bytes != 0)
    return fail(ST_ERR_INVALID_ARG, "workspace is NULL but workspace_bytes is %zu", workspace_bytes);
  if (workspace != nullptr && workspace_bytes < need)
    return fail(ST_ERR_INVALID_ARG, "workspace_bytes %zu < required %zu", workspace_bytes, need);

  // ---- device checks ----
  for (int i = 0; i < nchunks; ++i) {
    int st = st::host::check_path_buffers(args[i]);
    if (st != ST_OK) return fail(st, "chunk %d: %s", i, st_last_error());
  }
  if (workspace != nullptr) {
    int st = st::host::check_device_buffer(workspace, need, "workspace");
    if (st != ST_OK) return st;
  }

  st_batch* b = new (std::nothrow) st_batch();
  if (b == nullptr) return fail(ST_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->chunks = std::move(args);
  b->slot_bytes = slot;
  b->slots = slots;
  b->lanes = lanes == 0 ? slots : lanes;
  if (b->lanes > 1) {
    // concurrent chains fill the chip together: split each chunk's passes a
    // quarter as far as a lone volume would be (fewer z halo planes)
    b->shape.grad_min_blocks /= 4;
    b->shape.strided_min_waves /= 4;
  }
  hipError_t e = hipGetDevice(&b->device);
  const char* what = "hipGetDevice";
  if (e == hipSuccess) {
    what = "hipStreamCreateWithFlags";
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (int k = 0; k < ST_BATCH_MAX_LANES && e == hipSuccess; ++k)
      e = hipStreamCreateWithFlags(&b->lane_stream[k], hipStreamNonBlocking);
  }
  if (e == hipSuccess) {
    what = "hipEventCreateWithFlags";
    e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int k = 0; k < ST_BATCH_MAX_LANES && e == hipSuccess; ++k)
      e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
  }
  if (e == hipSuccess && workspace == nullptr) {
    what = "hipMalloc (batch workspace)";
    e = hipMalloc(reinterpret_cast<void**>(&b->ws), need);
    if (e == hipSuccess) b->owned = true;
  } else if (e == hipSuccess) {
    b->ws = static_cast<char*>(workspace);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release(b);
    return e == hipErrorOutOfMemory ? fail(ST_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e))
                                    : device_fail(e, what);
  }
  int st = rebuild(b);
  if (st != ST_OK) {
    release(b);
    return st;
  }
  *out = b;
  return ST_OK;
}

int st_batch_launch(st_batch* b, void* stream) {
  st::host::clear_error();
  if (b == nullptr) return fail(ST_ERR_INVALID_ARG, "batch is NULL");
  DeviceScope dev(b->device);
  if (dev.err != hipSuccess) return device_fail(dev.err, "hipSetDevice");
  return launch(b, static_cast<hipStream_t>(stream));
}

// Switched off: repeated re-capture of the batch graph on the same streams and
// events, mixed with direct enqueues on those events, crashed the host process
// intermittently on the target machine and the cause is not identified.  The
// configuration it chose in every measured run (8 chains, graph replay, default
// split targets) is what lanes = 0 gives.
int st_batch_tune(st_batch* b, void*, int reps) {
  st::host::clear_error();
  if (b == nullptr) return fail(ST_ERR_INVALID_ARG, "batch is NULL");
  if (reps < 1) return fail(ST_ERR_INVALID_ARG, "reps must be >= 1");
  return fail(ST_ERR_UNSUPPORTED,
              "st_batch_tune is switched off in this build (an unexplained host crash during graph "
              "re-capture); lanes = 0 selects its measured choice, 8 chains with graph replay");
}

int st_batch_config(const st_batch* b, int* lanes, int* use_graph, int64_t* grad_min_blocks,
                    int64_t* strided_min_waves, double* best_ms) {
  st::host::clear_error();
  if (b == nullptr) return fail(ST_ERR_INVALID_ARG, "batch is NULL");
  if (lanes) *lanes = b->lanes;
  if (use_graph) *use_graph = b->use_graph ? 1 : 0;
  if (grad_min_blocks) *grad_min_blocks = b->shape.grad_min_blocks;
  if (strided_min_waves) *strided_min_waves = b->shape.strided_min_waves;
  if (best_ms) *best_ms = b->best_ms;
  return ST_OK;
}

int st_batch_destroy(st_batch* b) {
  st::host::clear_error();
  if (b == nullptr) return ST_OK;
  DeviceScope dev(b->device);
  hipError_t e = hipSuccess;
  for (int k = 0; k < ST_BATCH_MAX_LANES && e == hipSuccess; ++k)
    if (b->lane_stream[k]) e = hipStreamSynchronize(b->lane_stream[k]);
  release(b);
  return e == hipSuccess ? ST_OK : device_fail(e, "hipStreamSynchronize");
}

}  // extern "C"
