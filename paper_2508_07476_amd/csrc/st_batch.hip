// Chunk batches: many independent volumes through the structure-tensor path as
// one unit of work (the paper's chunk-based processing with padding,
// Implementation section), built for one GPU with a large HBM.
//
// Chunks are dealt to up to ST_BATCH_MAX_LANES chains, largest first and each to
// the chain with the least voxels so far (longest-processing-time order); each
// chain owns a workspace slot sized for the largest chunk and a stream of its
// own, so small chunks that cannot fill the chip alone run side by side.  The
// fork / join of the chains is recorded into a HIP graph and replayed.  Every
// output is computed by the same kernels with the same per-voxel summation
// order in every configuration (chain count, split targets, tile shapes,
// graph or direct enqueue), so results are bitwise independent of it.
//
// Lifetime rules, kept by construction:
//  - every capture gets fork / join events of its own, created with the graph
//    and destroyed with it; direct enqueue uses a separate set of events;
//  - each launch waits for the previous one (on whatever stream it ran) and
//    records `done` on its own stream, so `done` follows every launch so far;
//    a graph is destroyed only after `done` and every stream of the batch have
//    been waited for, so no destroyed graph or event can still be referenced
//    by queued work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "st_host.h"

using st::host::device_fail;
using st::host::fail;

namespace {

// One captured batch: the graph, its executable and the events used only by
// its capture.
struct Captured {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t fork = nullptr;
  hipEvent_t join[ST_BATCH_MAX_LANES] = {};
};

// Events that order a fork / join: a capture's own, or the direct-enqueue set.
struct ForkJoin {
  hipEvent_t fork;
  const hipEvent_t* join;
};

// One launch of the grouped mode: a pass over every chunk of a round that
// shares its radius, taps and tile shape; its tables live in the batch's table
// buffer.
struct GroupLaunch {
  int kind = 0;    // 0 gradient, 1 z integration, 2 y integration, 3 final pass, 4 completion mark
  int R = 0;       // compiled radius
  int shape = 0;   // gradient tile rows, or final-pass segment lanes
  int dtype = 0;   // input type (gradient)
  st::Taps w0{}, w1{};  // gradient: smoothing, derivative taps; integration: smoothing taps
  size_t geo = 0, first = 0;  // byte offsets of the entry table (mark: chunk ids) and the block table
  int count = 0;
  int64_t blocks = 0;
};

}  // namespace

struct st_batch {
  std::vector<st::host::PathArgs> chunks;
  std::vector<st::host::LaunchShape> tiles;  // per chunk: tile shapes (split targets unused)
  size_t slot_bytes = 0;  // workspace of the largest chunk
  int slots = 0;          // workspace slots (the largest chain count possible)
  size_t ws_bytes = 0;    // workspace bytes the grouped rounds may fill
  char* ws = nullptr;
  bool owned = false;
  int device = 0;
  // configuration
  int lanes = 1;
  bool use_graph = true;
  st::host::LaunchShape shape;  // split targets of every chunk
  double best_ms = 0.0;
  // runtime objects
  hipStream_t cap = nullptr;  // origin of captures
  hipStream_t lane_stream[ST_BATCH_MAX_LANES] = {};
  hipEvent_t dfork = nullptr;  // direct enqueue
  hipEvent_t djoin[ST_BATCH_MAX_LANES] = {};
  hipEvent_t done = nullptr;   // recorded on the launch stream after every launch
  bool launched = false;
  Captured* captured = nullptr;
  std::vector<std::vector<int>> plan;  // chunk indices of every chain, in launch order
  // grouped mode: rounds of chunks whose workspaces fit together, each pass of a
  // round one launch per (radius, taps, tile shape) over a device table
  bool grouped = false;
  int rounds = 0;
  std::vector<GroupLaunch> glaunch;
  char* tables = nullptr;  // device buffer of the entry and block tables (owned)
  // completion record: a device launch counter and one pinned host word per
  // chunk that takes the counter's value when the chunk's last pass is done
  uint64_t* seq = nullptr;
  uint64_t* progress = nullptr;
  int64_t launches = 0;
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

// The launch shape of chunk i: the batch's split targets with the chunk's tiles.
st::host::LaunchShape chunk_shape(const st_batch* b, int i) {
  st::host::LaunchShape s = b->shape;
  s.grad_rows = b->tiles[i].grad_rows;
  s.xfinal_lanes = b->tiles[i].xfinal_lanes;
  return s;
}

// ---- grouped mode -------------------------------------------------------------

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool same_taps(const st::Taps& a, const st::Taps& b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

// Plans the grouped mode for the current tile shapes and uploads its tables
// (synchronous; the batch must be idle).  Chunks go into rounds by first-fit
// decreasing on their workspace bytes within the batch's workspace; each chunk
// of a round gets its own workspace region and a share of the split targets
// in proportion to its voxels, so a round's launch splits as far as one
// volume of the round's size would.  ST_ERR_UNSUPPORTED if a chunk needs the
// three-pass gradient (sigma radius above the fused pass's).
int plan_grouped(st_batch* b) {
  const int n = static_cast<int>(b->chunks.size());
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return b->chunks[i].n > b->chunks[j].n; });
  const size_t budget = b->ws_bytes;
  struct Round {
    size_t used = 0;
    std::vector<std::pair<int, size_t>> chunk_off;
    int64_t voxels = 0;
  };
  std::vector<Round> rounds;
  for (int i : order) {
    const st::host::PathArgs& a = b->chunks[i];
    const size_t w = align_up(st::host::path_workspace_bytes(a.nz, a.ny, a.nx), 256);
    size_t r = 0;
    while (r < rounds.size() && rounds[r].used + w > budget) ++r;
    if (r == rounds.size()) rounds.emplace_back();
    rounds[r].chunk_off.emplace_back(i, rounds[r].used);
    rounds[r].used += w;
    rounds[r].voxels += a.n;
  }
  // launches and their tables (host copies)
  std::vector<GroupLaunch> launches;
  std::vector<std::vector<char>> geos;
  std::vector<std::vector<int64_t>> firsts;
  const st::host::LaunchShape base;
  for (const Round& rd : rounds) {
    std::vector<st::host::PathPlan> plans(rd.chunk_off.size());
    for (size_t k = 0; k < rd.chunk_off.size(); ++k) {
      const int i = rd.chunk_off[k].first;
      st::host::LaunchShape sh = chunk_shape(b, i);
      const double share = static_cast<double>(b->chunks[i].n) / static_cast<double>(rd.voxels);
      sh.grad_min_blocks = std::max<int64_t>(1, static_cast<int64_t>(base.grad_min_blocks * share));
      sh.strided_min_waves = std::max<int64_t>(1, static_cast<int64_t>(base.strided_min_waves * share));
      st::host::plan_path(b->chunks[i], b->ws + rd.chunk_off[k].second, sh, &plans[k]);
      if (!plans[k].fused_grad)
        return fail(ST_ERR_UNSUPPORTED, "grouped launches need the fused gradient pass (chunk %d)", i);
    }
    // one pass kind at a time, entries grouped by (radius, taps, tile shape, type)
    for (int kind = 0; kind < 4; ++kind) {
      std::vector<bool> done(plans.size(), false);
      for (size_t k0 = 0; k0 < plans.size(); ++k0) {
        if (done[k0]) continue;
        const st::host::PathPlan& p0 = plans[k0];
        GroupLaunch L;
        L.kind = kind;
        if (kind == 0) {
          L.R = p0.rs; L.shape = p0.grad.rows; L.dtype = b->chunks[rd.chunk_off[k0].first].dtype;
          L.w0 = p0.grad.wg; L.w1 = p0.grad.wd;
        } else if (kind < 3) {
          L.R = p0.rr; L.w0 = kind == 1 ? p0.int_z.wg : p0.int_y.wg;
        } else {
          L.R = p0.rr; L.shape = p0.fin.tile_lanes; L.w0 = p0.fin.w;
        }
        std::vector<char> geo;
        std::vector<int64_t> first{0};
        for (size_t k = k0; k < plans.size(); ++k) {
          if (done[k]) continue;
          const st::host::PathPlan& p = plans[k];
          int64_t nb = 0;
          const char* g = nullptr;
          size_t gsz = 0;
          if (kind == 0) {
            if (p.rs != L.R || p.grad.rows != L.shape || b->chunks[rd.chunk_off[k].first].dtype != L.dtype ||
                !same_taps(p.grad.wg, L.w0) || !same_taps(p.grad.wd, L.w1))
              continue;
            nb = align_up(static_cast<size_t>(st::grad_blocks(p.grad)), 8);  // XCD remap per volume
            g = reinterpret_cast<const char*>(static_cast<const st::GradGeo*>(&p.grad));
            gsz = sizeof(st::GradGeo);
          } else if (kind < 3) {
            const st::StridedParams& q = kind == 1 ? p.int_z : p.int_y;
            if (p.rr != L.R || !same_taps(q.wg, L.w0)) continue;
            nb = st::strided_blocks(q);
            g = reinterpret_cast<const char*>(static_cast<const st::StridedGeo*>(&q));
            gsz = sizeof(st::StridedGeo);
          } else {
            if (p.rr != L.R || p.fin.tile_lanes != L.shape || !same_taps(p.fin.w, L.w0)) continue;
            nb = st::xfinal_blocks(p.fin);
            g = reinterpret_cast<const char*>(static_cast<const st::XFinalGeo*>(&p.fin));
            gsz = sizeof(st::XFinalGeo);
          }
          done[k] = true;
          geo.insert(geo.end(), g, g + gsz);
          first.push_back(first.back() + nb);
        }
        L.count = static_cast<int>(first.size()) - 1;
        L.blocks = first.back();
        if (L.blocks > INT32_MAX)
          return fail(ST_ERR_UNSUPPORTED, "a grouped launch of %lld blocks exceeds the grid limit", (long long)L.blocks);
        launches.push_back(L);
        geos.push_back(std::move(geo));
        firsts.push_back(std::move(first));
      }
    }
    // the round's chunks are complete once its launches have run
    GroupLaunch M;
    M.kind = 4;
    M.count = static_cast<int>(rd.chunk_off.size());
    std::vector<char> ids(rd.chunk_off.size() * sizeof(int64_t));
    for (size_t k = 0; k < rd.chunk_off.size(); ++k) {
      const int64_t c = rd.chunk_off[k].first;
      std::memcpy(ids.data() + k * sizeof(int64_t), &c, sizeof(c));
    }
    launches.push_back(M);
    geos.push_back(std::move(ids));
    firsts.push_back(std::vector<int64_t>{0});
  }
  // one device buffer for every table, each 256-byte aligned
  size_t total = 0;
  for (size_t l = 0; l < launches.size(); ++l) {
    launches[l].geo = total;
    total = align_up(total + geos[l].size(), 256);
    launches[l].first = total;
    total = align_up(total + firsts[l].size() * sizeof(int64_t), 256);
  }
  std::vector<char> host(total, 0);
  for (size_t l = 0; l < launches.size(); ++l) {
    std::memcpy(host.data() + launches[l].geo, geos[l].data(), geos[l].size());
    std::memcpy(host.data() + launches[l].first, firsts[l].data(), firsts[l].size() * sizeof(int64_t));
  }
  if (b->tables) {
    (void)hipFree(b->tables);
    b->tables = nullptr;
  }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&b->tables), std::max<size_t>(total, 256));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b->tables = nullptr;
    return e == hipErrorOutOfMemory ? fail(ST_ERR_OUT_OF_MEMORY, "batch table allocation failed")
                                    : device_fail(e, "hipMalloc (batch tables)");
  }
  e = hipMemcpy(b->tables, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_fail(e, "hipMemcpy (batch tables)");
  b->glaunch = std::move(launches);
  b->rounds = static_cast<int>(rounds.size());
  return ST_OK;
}

// Enqueues the grouped launches on `stream`, round after round.
hipError_t enqueue_grouped(st_batch* b, hipStream_t stream, const char** stage) {
  for (const GroupLaunch& L : b->glaunch) {
    hipError_t e;
    if (L.kind == 0) {
      st::GradFusedGroup g;
      g.g.geo = reinterpret_cast<const st::GradGeo*>(b->tables + L.geo);
      g.g.first = reinterpret_cast<const int64_t*>(b->tables + L.first);
      g.g.count = L.count;
      g.wg = L.w0;
      g.wd = L.w1;
      *stage = "grad_fused (grouped)";
      e = st::launch_grad_fused_grouped(L.R, L.dtype, L.shape, g, L.blocks, stream);
    } else if (L.kind < 3) {
      st::StridedGroup g;
      g.g.geo = reinterpret_cast<const st::StridedGeo*>(b->tables + L.geo);
      g.g.first = reinterpret_cast<const int64_t*>(b->tables + L.first);
      g.g.count = L.count;
      g.wg = L.w0;
      *stage = L.kind == 1 ? "integrate_z (grouped)" : "integrate_y (grouped)";
      e = st::launch_strided_grouped(L.R, g, L.blocks, stream);
    } else if (L.kind == 4) {
      *stage = "completion mark";
      e = st::launch_batch_mark(b->seq, b->progress, reinterpret_cast<const int64_t*>(b->tables + L.geo), L.count, 0,
                                stream);
    } else {
      st::XFinalGroup g;
      g.g.geo = reinterpret_cast<const st::XFinalGeo*>(b->tables + L.geo);
      g.g.first = reinterpret_cast<const int64_t*>(b->tables + L.first);
      g.g.count = L.count;
      g.w = L.w0;
      *stage = "integrate_x_eigen (grouped)";
      e = st::launch_xfinal_grouped(L.R, L.shape, g, L.blocks, stream);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Fork from `root` into the chains, enqueue every chunk, join back into `root`.
hipError_t enqueue_all(st_batch* b, hipStream_t root, const ForkJoin& fj, const char** stage) {
  *stage = "fork";
  hipError_t e = hipEventRecord(fj.fork, root);
  if (e != hipSuccess) return e;
  for (int k = 0; k < b->lanes; ++k) {
    if (b->plan[k].empty()) continue;
    hipStream_t s = b->lane_stream[k];
    if ((e = hipStreamWaitEvent(s, fj.fork, 0)) != hipSuccess) return e;
    char* ws = b->ws + static_cast<size_t>(k) * b->slot_bytes;
    for (int i : b->plan[k]) {
      if ((e = st::host::enqueue_path(b->chunks[i], ws, s, chunk_shape(b, i), false, stage)) != hipSuccess)
        return e;
      *stage = "completion mark";
      if ((e = st::launch_batch_mark(b->seq, b->progress, nullptr, 1, i, s)) != hipSuccess) return e;
    }
    *stage = "join";
    if ((e = hipEventRecord(fj.join[k], s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(root, fj.join[k], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Waits for every launch of the batch and every stream it owns.
hipError_t wait_idle(st_batch* b) {
  hipError_t e = hipSuccess;
  if (b->launched && b->done) e = hipEventSynchronize(b->done);
  for (int k = 0; k < ST_BATCH_MAX_LANES && e == hipSuccess; ++k)
    if (b->lane_stream[k]) e = hipStreamSynchronize(b->lane_stream[k]);
  if (e == hipSuccess && b->cap) e = hipStreamSynchronize(b->cap);
  return e;
}

void destroy_captured(Captured* c) {
  if (c == nullptr) return;
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->fork) (void)hipEventDestroy(c->fork);
  for (hipEvent_t ev : c->join)
    if (ev) (void)hipEventDestroy(ev);
  delete c;
}

// Destroys the batch's graph; its launches must be known to be complete (wait_idle).
void drop_graph(st_batch* b) {
  destroy_captured(b->captured);
  b->captured = nullptr;
}

// Plans for the current configuration and captures it into a new graph with
// events of its own (the batch must hold no graph).
int capture(st_batch* b) {
  make_plan(b);
  Captured* c = new (std::nothrow) Captured();
  if (c == nullptr) return fail(ST_ERR_OUT_OF_MEMORY, "host allocation failed");
  hipError_t e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  for (int k = 0; k < b->lanes && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&c->join[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    destroy_captured(c);
    return device_fail(e, "hipEventCreateWithFlags");
  }
  e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    destroy_captured(c);
    return device_fail(e, "hipStreamBeginCapture");
  }
  const char* stage = "";
  hipError_t ee = b->grouped ? enqueue_grouped(b, b->cap, &stage)
                             : enqueue_all(b, b->cap, ForkJoin{c->fork, c->join}, &stage);
  e = hipStreamEndCapture(b->cap, &c->graph);  // always ends the capture, also after a failure
  if (ee != hipSuccess || e != hipSuccess) {
    destroy_captured(c);
    return ee != hipSuccess ? device_fail(ee, stage) : device_fail(e, "hipStreamEndCapture");
  }
  e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    destroy_captured(c);
    return device_fail(e, "hipGraphInstantiate");
  }
  b->captured = c;
  return ST_OK;
}

// Enqueues the batch on `stream` after the batch's previous launch, whichever
// stream that was on (replays share the workspace and the outputs), and
// records `done` after it, so `done` always follows every launch so far.
int launch(st_batch* b, hipStream_t stream) {
  hipError_t e = hipSuccess;
  const char* stage = "hipStreamWaitEvent";
  if (b->launched && (e = hipStreamWaitEvent(stream, b->done, 0)) != hipSuccess) return device_fail(e, stage);
  stage = "launch counter";
  if ((e = st::launch_batch_begin(b->seq, stream)) != hipSuccess) return device_fail(e, stage);
  stage = "hipGraphLaunch";
  if (b->use_graph) {
    e = hipGraphLaunch(b->captured->exec, stream);
  } else if (b->grouped) {
    e = enqueue_grouped(b, stream, &stage);
  } else {
    e = enqueue_all(b, stream, ForkJoin{b->dfork, b->djoin}, &stage);
  }
  if (e == hipSuccess) {
    stage = "hipEventRecord";
    e = hipEventRecord(b->done, stream);
  }
  // the counter was bumped: from here on the record refers to this launch
  b->launches += 1;
  if (e != hipSuccess) return device_fail(e, stage);
  b->launched = true;
  return ST_OK;
}

void release(st_batch* b) {
  if (b == nullptr) return;
  drop_graph(b);
  for (int k = 0; k < ST_BATCH_MAX_LANES; ++k) {
    if (b->lane_stream[k]) (void)hipStreamDestroy(b->lane_stream[k]);
    if (b->djoin[k]) (void)hipEventDestroy(b->djoin[k]);
  }
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->dfork) (void)hipEventDestroy(b->dfork);
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->owned && b->ws) (void)hipFree(b->ws);
  if (b->tables) (void)hipFree(b->tables);
  if (b->seq) (void)hipFree(b->seq);
  if (b->progress) (void)hipHostFree(b->progress);
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

// ---- autotuning ---------------------------------------------------------------

// Elapsed milliseconds per repetition of fn() on `stream` (one untimed run first).
template <class F>
int time_reps(hipStream_t stream, hipEvent_t t0, hipEvent_t t1, int reps, F&& fn, double* ms) {
  int st = fn();
  if (st != ST_OK) return st;
  hipError_t e = hipEventRecord(t0, stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    if ((st = fn()) != ST_OK) return st;
  if (e == hipSuccess) e = hipEventRecord(t1, stream);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, t0, t1);
  if (e != hipSuccess) return device_fail(e, "autotune timing");
  *ms = static_cast<double>(f) / reps;
  return ST_OK;
}

// Tile shapes worth timing for one chunk: gradient tile rows compiled for its
// sigma radius, and final-pass segment widths compiled for its rho radius.
void tile_candidates(const st::host::PathArgs& a, std::vector<int>* rows, std::vector<int>* lanes) {
  const int rs = st::padded_radius(static_cast<int>(std::floor(a.truncate * a.sigma + 0.5)), true);
  const int rr = st::padded_radius(static_cast<int>(std::floor(a.truncate * a.rho + 0.5)), false);
  rows->clear();
  lanes->clear();
  if (rs <= st::kGradMaxRadius && a.ny * a.nx <= INT32_MAX)
    for (int r : {8, 4})
      if (st::grad_rows_supported(rs, r)) rows->push_back(r);
  for (int l : {64, 16})
    if (st::xfinal_lanes_supported(rr, l)) lanes->push_back(l);
}

}  // namespace

extern "C" {

size_t st_batch_workspace_bytes(const st_chunk* chunks, int nchunks, int lanes) {
  if (chunks == nullptr || nchunks < 1 || lanes < ST_BATCH_GROUPED || lanes > ST_BATCH_MAX_LANES) return 0;
  size_t slot = 0;
  if (!slot_plan(chunks, nchunks, &slot)) return 0;
  const size_t slots = lanes <= 0 ? ST_BATCH_MAX_LANES : static_cast<size_t>(lanes);
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
  if (lanes < ST_BATCH_GROUPED || lanes > ST_BATCH_MAX_LANES)
    return fail(ST_ERR_INVALID_ARG, "lanes %d is outside %d..%d", lanes, ST_BATCH_GROUPED, ST_BATCH_MAX_LANES);
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
  // chains need one slot each; grouped launches need one slot and use all the
  // workspace they are given (less workspace, more rounds; more, fewer)
  int slots = lanes <= 0 ? ST_BATCH_MAX_LANES : lanes;
  if (lanes == ST_BATCH_GROUPED && workspace != nullptr && workspace_bytes >= slot)
    slots = static_cast<int>(std::min<size_t>(ST_BATCH_MAX_LANES, workspace_bytes / slot));
  const size_t need = slot * static_cast<size_t>(slots);
  const size_t ws_bytes = lanes == ST_BATCH_GROUPED && workspace != nullptr ? workspace_bytes : need;
  if (workspace == nullptr && workspace_bytes != 0)
    return fail(ST_ERR_INVALID_ARG, "workspace is NULL but workspace_bytes is %zu", workspace_bytes);
  if (workspace != nullptr && workspace_bytes < need)
    return fail(ST_ERR_INVALID_ARG, "workspace_bytes %zu < required %zu", workspace_bytes, need);
  if (workspace == nullptr && st::host::alloc_fault_injected())
    return fail(ST_ERR_OUT_OF_MEMORY, "batch workspace allocation of %zu bytes failed (ST_FAULT_INJECT=alloc)",
                need);

  // ---- device checks ----
  for (int i = 0; i < nchunks; ++i) {
    int st = st::host::check_path_buffers(args[i]);
    if (st != ST_OK) return fail(st, "chunk %d: %s", i, st_last_error());
  }
  if (workspace != nullptr) {
    int st = st::host::check_device_buffer(workspace, ws_bytes, "workspace");
    if (st != ST_OK) return st;
  }

  st_batch* b = new (std::nothrow) st_batch();
  if (b == nullptr) return fail(ST_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->chunks = std::move(args);
  b->tiles.assign(b->chunks.size(), st::host::LaunchShape{});
  b->slot_bytes = slot;
  b->slots = slots;
  b->ws_bytes = ws_bytes;
  b->lanes = lanes <= 0 ? slots : lanes;
  b->grouped = lanes == ST_BATCH_GROUPED;
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
    e = hipEventCreateWithFlags(&b->dfork, hipEventDisableTiming);
    for (int k = 0; k < ST_BATCH_MAX_LANES && e == hipSuccess; ++k)
      e = hipEventCreateWithFlags(&b->djoin[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  }
  if (e == hipSuccess && workspace == nullptr) {
    what = "hipMalloc (batch workspace)";
    e = hipMalloc(reinterpret_cast<void**>(&b->ws), need);
    if (e == hipSuccess) b->owned = true;
  } else if (e == hipSuccess) {
    b->ws = static_cast<char*>(workspace);
  }
  if (e == hipSuccess) {
    what = "hipMalloc (launch counter)";
    e = hipMalloc(reinterpret_cast<void**>(&b->seq), sizeof(uint64_t));
    const uint64_t zero = 0;
    if (e == hipSuccess) e = hipMemcpy(b->seq, &zero, sizeof(zero), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    what = "hipHostMalloc (completion record)";
    e = hipHostMalloc(reinterpret_cast<void**>(&b->progress), b->chunks.size() * sizeof(uint64_t),
                      hipHostMallocDefault);
    if (e == hipSuccess) std::memset(b->progress, 0, b->chunks.size() * sizeof(uint64_t));
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release(b);
    return e == hipErrorOutOfMemory ? fail(ST_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e))
                                    : device_fail(e, what);
  }
  int st = b->grouped ? plan_grouped(b) : ST_OK;
  if (st == ST_OK) st = capture(b);
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

int st_batch_tune(st_batch* b, void* stream_, int reps) {
  st::host::clear_error();
  if (b == nullptr) return fail(ST_ERR_INVALID_ARG, "batch is NULL");
  if (reps < 1) return fail(ST_ERR_INVALID_ARG, "reps must be >= 1");
  DeviceScope dev(b->device);
  if (dev.err != hipSuccess) return device_fail(dev.err, "hipSetDevice");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  // nothing of an earlier graph may survive: its launches finish first
  hipError_t e = wait_idle(b);
  if (e != hipSuccess) return device_fail(e, "waiting for the batch");
  drop_graph(b);
  b->use_graph = false;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return device_fail(e, "hipEventCreate");
  }
  int st = ST_OK;

  // 1. tile shapes, chunk by chunk (alone on the stream, workspace slot 0):
  // gradient tile rows first, then the final pass's segment width
  std::vector<int> rows, lanes;
  for (size_t i = 0; i < b->chunks.size() && st == ST_OK; ++i) {
    tile_candidates(b->chunks[i], &rows, &lanes);
    for (int which = 0; which < 2 && st == ST_OK; ++which) {
      const std::vector<int>& cand = which == 0 ? rows : lanes;
      if (cand.size() < 2) continue;
      double best = INFINITY;
      int pick = cand[0];
      for (int v : cand) {
        st::host::LaunchShape s = chunk_shape(b, static_cast<int>(i));
        (which == 0 ? s.grad_rows : s.xfinal_lanes) = v;
        double ms = 0.0;
        st = time_reps(stream, t0, t1, reps, [&]() -> int {
          const char* stage = "";
          hipError_t er = st::host::enqueue_path(b->chunks[i], b->ws, stream, s, false, &stage);
          return er == hipSuccess ? ST_OK : device_fail(er, stage);
        }, &ms);
        if (st != ST_OK) break;
        if (ms < best) { best = ms; pick = v; }
      }
      (which == 0 ? b->tiles[i].grad_rows : b->tiles[i].xfinal_lanes) = pick;
    }
  }

  // 2. chain count, then split targets: the whole batch, direct enqueue; then
  // the grouped launches (when every chunk has the fused gradient pass)
  const st::host::LaunchShape base;
  b->grouped = false;
  auto time_batch = [&](int nl, double factor, double* ms) -> int {
    b->lanes = nl;
    b->shape.grad_min_blocks = std::max<int64_t>(1, static_cast<int64_t>(base.grad_min_blocks * factor));
    b->shape.strided_min_waves = std::max<int64_t>(1, static_cast<int64_t>(base.strided_min_waves * factor));
    make_plan(b);
    return time_reps(stream, t0, t1, reps, [&] { return launch(b, stream); }, ms);
  };
  int best_lanes = 1;
  double best_factor = 1.0, best_ms = INFINITY;
  for (int nl : {1, 2, 4, 8}) {
    if (st != ST_OK || nl > b->slots) break;
    const double f = nl > 1 ? 0.25 : 1.0;
    double ms = 0.0;
    st = time_batch(nl, f, &ms);
    if (st == ST_OK && ms < best_ms) { best_ms = ms; best_lanes = nl; best_factor = f; }
  }
  const double f0 = best_factor;
  for (double f : {f0 / 4, f0 * 4}) {
    if (st != ST_OK) break;
    double ms = 0.0;
    st = time_batch(best_lanes, f, &ms);
    if (st == ST_OK && ms < best_ms) { best_ms = ms; best_factor = f; }
  }

  bool best_grouped = false;
  if (st == ST_OK) {
    b->grouped = true;
    double ms = 0.0;
    int gst = plan_grouped(b);
    if (gst == ST_OK) gst = time_reps(stream, t0, t1, reps, [&] { return launch(b, stream); }, &ms);
    if (gst == ST_OK && ms < best_ms) {
      best_ms = ms;
      best_grouped = true;
    } else if (gst != ST_OK && gst != ST_ERR_UNSUPPORTED) {
      st = gst;
    }
    b->grouped = false;
    st::host::clear_error();
  }

  // 3. the chosen configuration replayed from one graph, against direct enqueue
  if (st == ST_OK) {
    double direct_ms = 0.0, graph_ms = 0.0;
    if (best_grouped) {
      b->grouped = true;
      b->lanes = 1;
      st = time_reps(stream, t0, t1, reps, [&] { return launch(b, stream); }, &direct_ms);
    } else {
      st = time_batch(best_lanes, best_factor, &direct_ms);
    }
    if (st == ST_OK) st = capture(b);
    if (st == ST_OK) {
      b->use_graph = true;
      st = time_reps(stream, t0, t1, reps, [&] { return launch(b, stream); }, &graph_ms);
    }
    if (st == ST_OK) {
      b->best_ms = std::min(direct_ms, graph_ms);
      if (direct_ms < graph_ms) {
        e = wait_idle(b);
        if (e != hipSuccess) st = device_fail(e, "waiting for the batch");
        drop_graph(b);
        b->use_graph = false;
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st != ST_OK) {
    // leave a usable batch: direct enqueue of the chains with whatever configuration was set
    (void)wait_idle(b);
    drop_graph(b);
    b->use_graph = false;
    b->grouped = false;
    make_plan(b);
  }
  return st;
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

int st_batch_plan(const st_batch* b, int* grouped, int* rounds, int* kernels) {
  st::host::clear_error();
  if (b == nullptr) return fail(ST_ERR_INVALID_ARG, "batch is NULL");
  if (grouped) *grouped = b->grouped ? 1 : 0;
  if (rounds) *rounds = b->grouped ? b->rounds : 0;
  if (kernels) {
    int64_t k = 0;
    if (b->grouped) {
      for (const GroupLaunch& L : b->glaunch) k += L.kind < 4;
    } else {
      for (const st::host::PathArgs& a : b->chunks) {
        st::host::PathPlan pl;
        st::host::plan_path(a, b->ws, st::host::LaunchShape{}, &pl);
        k += pl.fused_grad ? 4 : 7;
      }
    }
    *kernels = static_cast<int>(k);
  }
  return ST_OK;
}

int st_batch_progress(const st_batch* b, uint8_t* done, int nchunks, int64_t* launches) {
  st::host::clear_error();
  if (b == nullptr) return fail(ST_ERR_INVALID_ARG, "batch is NULL");
  if (done != nullptr && nchunks != static_cast<int>(b->chunks.size()))
    return fail(ST_ERR_INVALID_ARG, "nchunks %d, the batch has %zu chunks", nchunks, b->chunks.size());
  const uint64_t want = static_cast<uint64_t>(b->launches);
  if (done != nullptr)
    for (int c = 0; c < nchunks; ++c)
      done[c] = want > 0 && __atomic_load_n(b->progress + c, __ATOMIC_ACQUIRE) == want ? 1 : 0;
  if (launches) *launches = b->launches;
  return ST_OK;
}

int st_batch_tiles(const st_batch* b, int chunk, int* grad_rows, int* final_lanes) {
  st::host::clear_error();
  if (b == nullptr) return fail(ST_ERR_INVALID_ARG, "batch is NULL");
  if (chunk < 0 || chunk >= static_cast<int>(b->chunks.size()))
    return fail(ST_ERR_INVALID_ARG, "chunk %d is outside 0..%d", chunk, static_cast<int>(b->chunks.size()) - 1);
  if (grad_rows) *grad_rows = b->tiles[chunk].grad_rows;
  if (final_lanes) *final_lanes = b->tiles[chunk].xfinal_lanes;
  return ST_OK;
}

int st_batch_destroy(st_batch* b) {
  st::host::clear_error();
  if (b == nullptr) return ST_OK;
  DeviceScope dev(b->device);
  hipError_t e = wait_idle(b);
  release(b);
  return e == hipSuccess ? ST_OK : device_fail(e, "waiting for the batch");
}

}  // extern "C"
