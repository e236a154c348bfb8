// Drives every entry point of the library's C ABI through the HIP stand-in
// (see hostcheck.h): single volumes of several shapes and radii (fused and
// three-pass gradients, the largest integration radius, widths on both sides
// of the workspace pitch), the library-allocated and caller workspaces, the
// no-allocation entry point, re-angling, the surrogate with and without
// fallback, kernel timing, forced allocation failures, and chunk batches:
// creation with 1, 3 and 8 chains, replays, repeated autotuning between
// replays (whose pseudo-random timings make it choose graph replay on some
// calls and direct enqueue on others), tuning a batch that has never been
// launched, and destroying batches with launches still queued.  Exits 0 and
// prints "hostcheck: OK" when every call returned what it should; the stub
// aborts on any broken rule, ASan / UBSan on any memory or undefined-behaviour
// error.
#include <string>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hostcheck.h"
#include "st.h"

namespace {

int g_checks = 0;

void expect(int got, int want, const char* what) {
  ++g_checks;
  if (got != want) {
    std::fprintf(stderr, "hostcheck FAIL: %s returned %d, expected %d (%s)\n", what, got, want, st_last_error());
    std::exit(1);
  }
}

void* dev(size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess || p == nullptr) {
    std::fprintf(stderr, "hostcheck FAIL: stub allocation of %zu bytes\n", bytes);
    std::exit(1);
  }
  return p;
}

struct Vol {
  int64_t nz, ny, nx, n;
  int dtype;
  void* v = nullptr;
  uint8_t* mask = nullptr;
  float *e3 = nullptr, *evals = nullptr, *fa = nullptr, *ha = nullptr, *ia = nullptr, *conf = nullptr;
  uint8_t* flags = nullptr;
  Vol(int64_t z, int64_t y, int64_t x, int dt, bool with_mask) : nz(z), ny(y), nx(x), n(z * y * x), dtype(dt) {
    v = dev(static_cast<size_t>(n) * (dt == ST_DTYPE_U16 ? 2 : 4));
    if (with_mask) mask = static_cast<uint8_t*>(dev(n));
    e3 = static_cast<float*>(dev(3 * n * 4));
    evals = static_cast<float*>(dev(3 * n * 4));
    fa = static_cast<float*>(dev(n * 4));
    ha = static_cast<float*>(dev(n * 4));
    ia = static_cast<float*>(dev(n * 4));
    conf = static_cast<float*>(dev(n * 4));
    flags = static_cast<uint8_t*>(dev(n));
  }
  ~Vol() {
    for (void* p : {v, (void*)mask, (void*)e3, (void*)evals, (void*)fa, (void*)ha, (void*)ia, (void*)conf,
                    (void*)flags})
      (void)hipFree(p);
  }
};

const double kC[3] = {10.5, 11.25, 19.5}, kD[3] = {1.0, 0.2, -0.1};

int compute(Vol& a, double sigma, double rho, bool axis, bool caller_ws, hipStream_t s) {
  void* ws = nullptr;
  size_t wsb = 0;
  if (caller_ws) {
    wsb = st_workspace_bytes(a.nz, a.ny, a.nx);
    ws = dev(wsb);
  }
  const int r = st_compute(a.v, a.dtype, a.mask, a.nz, a.ny, a.nx, sigma, rho, 4.0, axis ? kC : nullptr,
                           axis ? kD : nullptr, a.e3, a.evals, a.fa, axis ? a.ha : nullptr, axis ? a.ia : nullptr,
                           a.flags, ws, wsb, s);
  if (ws) (void)hipFree(ws);
  return r;
}

void single_volumes(hipStream_t s) {
  struct Case {
    int64_t nz, ny, nx;
    int dtype;
    bool mask;
    double sigma, rho;
  } cases[] = {
      {20, 24, 40, ST_DTYPE_U16, true, 1.0, 2.0},   // fused gradient, radius 4
      {9, 30, 33, ST_DTYPE_F32, false, 2.0, 3.0},   // fused gradient radius 8 (4-row tiles), pitch 64
      {12, 10, 300, ST_DTYPE_U16, true, 2.6, 8.0},  // three-pass gradient (radius 11 -> 12), radius 32
      {5, 7, 9, ST_DTYPE_F32, false, 1.0, 2.0},     // smaller than the filter radii
      {3, 2, 1, ST_DTYPE_U16, false, 1.5, 1.0},     // one column
      {64, 3, 256, ST_DTYPE_F32, true, 1.0, 6.0},   // 256-wide rows, radius 24
  };
  for (const Case& c : cases) {
    Vol a(c.nz, c.ny, c.nx, c.dtype, c.mask);
    for (bool axis : {true, false})
      for (bool caller_ws : {true, false}) expect(compute(a, c.sigma, c.rho, axis, caller_ws, s), ST_OK, "st_compute");
    expect(st_compute_noalloc(a.v, a.dtype, a.mask, a.nz, a.ny, a.nx, c.sigma, c.rho, 4.0, kC, kD, a.e3, nullptr,
                              a.fa, a.ha, a.ia, a.flags, s),
           ST_OK, "st_compute_noalloc");
    expect(st_angles(a.e3, a.mask, a.nz, a.ny, a.nx, kC, kD, a.ha, a.ia, a.flags, s), ST_OK, "st_angles");
  }
  // the no-allocation entry point refuses a volume beyond its scratch, before any work
  {
    Vol a(1, 1, 1, ST_DTYPE_F32, false);
    expect(st_compute_noalloc(a.v, a.dtype, nullptr, 160, 160, 160, 1.0, 2.0, 4.0, nullptr, nullptr, a.fa,
                              nullptr, nullptr, nullptr, nullptr, nullptr, s),
           ST_ERR_UNSUPPORTED, "st_compute_noalloc beyond the scratch");
  }
  // buffers smaller than the volume are refused
  {
    Vol a(8, 8, 8, ST_DTYPE_F32, false);
    float* small = static_cast<float*>(dev(100));
    expect(st_compute(a.v, a.dtype, nullptr, 8, 8, 8, 1.0, 2.0, 4.0, nullptr, nullptr, small, nullptr, nullptr,
                      nullptr, nullptr, nullptr, nullptr, 0, s),
           ST_ERR_INVALID_ARG, "st_compute with a short output");
    (void)hipFree(small);
  }
}

void surrogate(hipStream_t s) {
  std::vector<float> host(ST_SURROGATE_WEIGHTS, 0.01f);
  float* w = static_cast<float*>(dev(host.size() * 4));
  for (bool mask : {true, false}) {
    Vol a(18, 20, 45, ST_DTYPE_U16, mask);
    for (double minc : {0.0, 0.9}) {
      expect(st_surrogate_infer(a.v, a.dtype, a.mask, a.nz, a.ny, a.nx, w, host.size() * 4, minc, 1.0, 2.0, 4.0,
                                kC, kD, a.e3, a.fa, a.ha, a.ia, a.conf, s),
             ST_OK, "st_surrogate_infer");
      expect(st_surrogate_infer(a.v, a.dtype, a.mask, a.nz, a.ny, a.nx, w, host.size() * 4, minc, 1.0, 2.0, 4.0,
                                nullptr, nullptr, a.e3, nullptr, nullptr, nullptr, nullptr, s),
             ST_OK, "st_surrogate_infer (e3 only)");
    }
  }
  // slabs of 3 output planes (11-plane buffers), with and without a fallback
  setenv("ST_SURROGATE_SLAB_BYTES", std::to_string(2 * 11 * 90 * 150 * 64).c_str(), 1);
  {
    Vol c(25, 90, 150, ST_DTYPE_U16, true);
    for (double minc : {0.0, 0.9})
      expect(st_surrogate_infer(c.v, c.dtype, c.mask, c.nz, c.ny, c.nx, w, host.size() * 4, minc, 1.0, 2.0, 4.0, kC,
                                kD, c.e3, c.fa, c.ha, c.ia, c.conf, s),
             ST_OK, "st_surrogate_infer in slabs");
  }
  // a whole-volume fallback streamed in slabs through the activation buffers
  // (28-plane buffers of 40 x 60 planes: about 49 planes of the path per slab)
  setenv("ST_SURROGATE_SLAB_BYTES", std::to_string(2 * 28 * 40 * 60 * 64).c_str(), 1);
  setenv("HOSTCHECK_FLAGS", "all", 1);
  {
    Vol c(80, 40, 60, ST_DTYPE_F32, true);
    expect(st_surrogate_infer(c.v, c.dtype, c.mask, c.nz, c.ny, c.nx, w, host.size() * 4, 0.9, 1.0, 2.0, 4.0, kC, kD,
                              c.e3, c.fa, c.ha, c.ia, c.conf, s),
           ST_OK, "st_surrogate_infer with a streamed whole-volume fallback");
    int mode = -1;
    expect(st_surrogate_fallback_info(&mode, nullptr, nullptr, nullptr), ST_OK, "st_surrogate_fallback_info");
    if (mode != 2) hc::violation("streamed fallback: mode %d", mode);
  }
  unsetenv("HOSTCHECK_FLAGS");
  unsetenv("ST_SURROGATE_SLAB_BYTES");
  // the per-tile fallback: a crop (the last tile flagged), the whole volume
  // (every third or every tile flagged: the crops would cost more), nothing (no
  // tile flagged), and the chains batch for a sigma whose radius needs the
  // three-pass gradient
  Vol b(70, 90, 150, ST_DTYPE_U16, true);
  struct Case { const char* flags; double sigma; int mode; };
  for (const Case& c : {Case{"one", 1.0, 1}, Case{"third", 1.0, 2}, Case{"all", 1.0, 2}, Case{"none", 1.0, 0},
                        Case{"one", 2.6, 1}}) {
    setenv("HOSTCHECK_FLAGS", c.flags, 1);
    for (bool conf_out : {true, false}) {
      expect(st_surrogate_infer(b.v, b.dtype, b.mask, b.nz, b.ny, b.nx, w, host.size() * 4, 0.9, c.sigma, 2.0, 4.0,
                                kC, kD, b.e3, b.fa, b.ha, b.ia, conf_out ? b.conf : nullptr, s),
             ST_OK, "st_surrogate_infer with a tile fallback");
      int mode = -1, edge = 0;
      int64_t tiles = 0, voxels = 0;
      expect(st_surrogate_fallback_info(&mode, &edge, &tiles, &voxels), ST_OK, "st_surrogate_fallback_info");
      if (mode != c.mode) hc::violation("fallback mode %d with %s tiles flagged, expected %d", mode, c.flags, c.mode);
      if (mode == 1 && (tiles < 1 || voxels < 1 || voxels >= b.nz * b.ny * b.nx))
        hc::violation("tile fallback of %lld crops, %lld voxels", (long long)tiles, (long long)voxels);
    }
  }
  unsetenv("HOSTCHECK_FLAGS");
  (void)hipFree(w);
}

void training(hipStream_t s) {
  std::vector<float> host(ST_SURROGATE_WEIGHTS, 0.01f);
  for (int P : {12, 32}) {
    const int64_t npatch = 3, n = npatch * P * P * P;
    void* vol = dev(n * 2);
    float* t = static_cast<float*>(dev(3 * n * 4));
    float* fa = static_cast<float*>(dev(n * 4));
    uint8_t* w = static_cast<uint8_t*>(dev(n));
    float* params = static_cast<float*>(dev(host.size() * 4));
    float* grad = static_cast<float*>(dev(host.size() * 4));
    float* m = static_cast<float*>(dev(host.size() * 4));
    float* v = static_cast<float*>(dev(host.size() * 4));
    float* stats = static_cast<float*>(dev(8 * 4));
    const size_t wsb = st_surrogate_grad_workspace_bytes(npatch, P);
    void* ws = dev(wsb);
    for (int step = 1; step <= 2; ++step) {
      expect(st_surrogate_grad(vol, ST_DTYPE_U16, npatch, P, t, fa, w, params, 0.1 * step, grad, stats,
                               step == 1 ? ws : nullptr,
                               step == 1 ? wsb : 0, s),
             ST_OK, "st_surrogate_grad");
      expect(st_surrogate_adam(params, grad, m, v, step, 1e-3, 0.9, 0.999, 1e-8, s), ST_OK, "st_surrogate_adam");
    }
    expect(st_surrogate_grad(vol, ST_DTYPE_U16, npatch, 33, t, fa, w, params, 0.1, grad, stats, nullptr, 0, s),
           ST_ERR_INVALID_ARG, "st_surrogate_grad with 33-voxel patches");
    expect(st_surrogate_grad(vol, ST_DTYPE_U16, npatch, P, t, fa, w, params, -1.0, grad, stats, nullptr, 0, s),
           ST_ERR_INVALID_ARG, "st_surrogate_grad with a negative confidence weight");
    expect(st_surrogate_adam(params, grad, m, v, 0, 1e-3, 0.9, 0.999, 1e-8, s), ST_ERR_INVALID_ARG,
           "st_surrogate_adam step 0");
    for (void* q : {vol, (void*)t, (void*)fa, (void*)w, (void*)params, (void*)grad, (void*)m, (void*)v, (void*)stats,
                    ws})
      (void)hipFree(q);
  }
}

void profiling(hipStream_t s) {
  expect(st_profile_enable(1), ST_OK, "st_profile_enable");
  Vol a(16, 16, 70, ST_DTYPE_F32, true);
  for (int r = 0; r < 3; ++r) expect(compute(a, 1.0, 3.0, true, true, s), ST_OK, "st_compute (timed)");
  const int n = st_profile_read(-1, nullptr, 0, nullptr, nullptr);
  if (n < 4) {
    std::fprintf(stderr, "hostcheck FAIL: %d timed kernels\n", n);
    std::exit(1);
  }
  for (int i = 0; i < n; ++i) {
    char name[64];
    double ms = 0;
    int64_t launches = 0;
    st_profile_read(i, name, sizeof(name), &ms, &launches);
    if (launches != 3) {
      std::fprintf(stderr, "hostcheck FAIL: kernel %s timed %lld times\n", name, (long long)launches);
      std::exit(1);
    }
  }
  expect(st_profile_reset(), ST_OK, "st_profile_reset");
  expect(st_profile_enable(0), ST_OK, "st_profile_enable(0)");
}

void fault_injection(hipStream_t s) {
  setenv("ST_FAULT_INJECT", "alloc", 1);
  Vol a(8, 9, 10, ST_DTYPE_U16, false);
  expect(compute(a, 1.0, 2.0, false, false, s), ST_ERR_OUT_OF_MEMORY, "st_compute under ST_FAULT_INJECT");
  expect(compute(a, 1.0, 2.0, false, true, s), ST_OK, "st_compute with a caller workspace under ST_FAULT_INJECT");
  std::vector<float> host(ST_SURROGATE_WEIGHTS, 0.f);
  float* w = static_cast<float*>(dev(host.size() * 4));
  expect(st_surrogate_infer(a.v, a.dtype, nullptr, a.nz, a.ny, a.nx, w, host.size() * 4, 0.0, 1.0, 2.0, 4.0,
                            nullptr, nullptr, a.e3, nullptr, nullptr, nullptr, nullptr, s),
         ST_ERR_OUT_OF_MEMORY, "st_surrogate_infer under ST_FAULT_INJECT");
  st_chunk c{};
  c.volume = a.v; c.dtype = a.dtype; c.nz = a.nz; c.ny = a.ny; c.nx = a.nx; c.rho = 2.0; c.e3 = a.e3;
  st_batch* b = nullptr;
  expect(st_batch_create(&c, 1, 1.0, 4.0, nullptr, nullptr, 2, nullptr, 0, &b), ST_ERR_OUT_OF_MEMORY,
         "st_batch_create under ST_FAULT_INJECT");
  if (b != nullptr) {
    std::fprintf(stderr, "hostcheck FAIL: a batch was returned with an error\n");
    std::exit(1);
  }
  unsetenv("ST_FAULT_INJECT");
  (void)hipFree(w);
}

struct Chunks {
  std::vector<Vol*> vols;
  std::vector<st_chunk> desc;
  Chunks() {
    // (origin, shape, rho): uneven, one thinner than its filter radius, masks on every other chunk
    const int64_t spec[][7] = {{10, 20, 30, 20, 26, 18, 2}, {0, 0, 0, 32, 20, 24, 3}, {30, 5, 8, 17, 23, 35, 4},
                               {20, 30, 2, 25, 25, 25, 2}, {60, 40, 10, 14, 30, 22, 3}, {5, 60, 40, 36, 17, 15, 4},
                               {40, 70, 90, 6, 5, 18, 4}};
    int i = 0;
    for (const auto& q : spec) {
      Vol* v = new Vol(q[3], q[4], q[5], i % 3 == 2 ? ST_DTYPE_F32 : ST_DTYPE_U16, i % 2 == 0);
      vols.push_back(v);
      st_chunk c{};
      c.volume = v->v; c.dtype = v->dtype; c.mask = v->mask;
      c.nz = v->nz; c.ny = v->ny; c.nx = v->nx; c.rho = static_cast<double>(q[6]);
      for (int d = 0; d < 3; ++d) c.origin[d] = static_cast<double>(q[d]);
      c.e3 = v->e3; c.evals = v->evals; c.fa = v->fa; c.ha = v->ha; c.ia = v->ia; c.flags = v->flags;
      desc.push_back(c);
      ++i;
    }
  }
  ~Chunks() {
    for (Vol* v : vols) delete v;
  }
};

st_batch* create(Chunks& ch, int lanes, void* ws = nullptr, size_t wsb = 0) {
  st_batch* b = nullptr;
  expect(st_batch_create(ch.desc.data(), static_cast<int>(ch.desc.size()), 1.0, 4.0, kC, kD, lanes, ws, wsb, &b),
         ST_OK, "st_batch_create");
  return b;
}

void batches(hipStream_t s, hipStream_t other) {
  Chunks ch;
  const int n = static_cast<int>(ch.desc.size());
  for (int lanes : {0, 1, 3, ST_BATCH_GROUPED}) {
    st_batch* b = create(ch, lanes);
    {  // completion record: nothing done before the first launch, three launches counted
      std::vector<uint8_t> done(n, 7);
      int64_t launches = -1;
      expect(st_batch_progress(b, done.data(), n, &launches), ST_OK, "st_batch_progress");
      if (launches != 0 || std::count(done.begin(), done.end(), 0) != n)
        hc::violation("st_batch_progress before a launch: %lld launches", (long long)launches);
      for (int r = 0; r < 3; ++r) expect(st_batch_launch(b, s), ST_OK, "st_batch_launch");
      expect(st_batch_progress(b, nullptr, 0, &launches), ST_OK, "st_batch_progress (count only)");
      if (launches != 3) hc::violation("st_batch_progress after three launches: %lld", (long long)launches);
      expect(st_batch_progress(b, done.data(), n + 1, nullptr), ST_ERR_INVALID_ARG, "st_batch_progress size");
    }
    for (int t = 0; t < 6; ++t) {
      expect(st_batch_tune(b, t % 2 ? s : other, 1 + t % 2), ST_OK, "st_batch_tune");
      int l = 0, g = 0;
      int64_t gb = 0, sw = 0;
      double ms = 0;
      expect(st_batch_config(b, &l, &g, &gb, &sw, &ms), ST_OK, "st_batch_config");
      if (l < 1 || l > ST_BATCH_MAX_LANES || !(ms > 0)) {
        std::fprintf(stderr, "hostcheck FAIL: tuned config lanes %d best %g\n", l, ms);
        std::exit(1);
      }
      for (int i = 0; i < n; ++i) {
        int rows = -1, fl = -1;
        expect(st_batch_tiles(b, i, &rows, &fl), ST_OK, "st_batch_tiles");
        if ((rows != 4 && rows != 8) || (fl != 16 && fl != 64)) {
          std::fprintf(stderr, "hostcheck FAIL: chunk %d tiles %d / %d\n", i, rows, fl);
          std::exit(1);
        }
      }
      for (int r = 0; r < 2; ++r) expect(st_batch_launch(b, r ? other : s), ST_OK, "st_batch_launch (tuned)");
    }
    int grouped = -1, rounds = -1, kernels = -1;
    expect(st_batch_plan(b, &grouped, &rounds, &kernels), ST_OK, "st_batch_plan");
    if (grouped < 0 || kernels < 1 || (grouped && rounds < 1)) {
      std::fprintf(stderr, "hostcheck FAIL: plan %d %d %d\n", grouped, rounds, kernels);
      std::exit(1);
    }
    expect(st_batch_tiles(b, n, nullptr, nullptr), ST_ERR_INVALID_ARG, "st_batch_tiles out of range");
    expect(st_batch_progress(nullptr, nullptr, 0, nullptr), ST_ERR_INVALID_ARG, "st_batch_progress of NULL");
    expect(st_batch_tune(b, s, 0), ST_ERR_INVALID_ARG, "st_batch_tune reps 0");
    expect(st_batch_destroy(b), ST_OK, "st_batch_destroy with launches queued");
  }
  {  // tuned before its first launch, then destroyed without a launch
    st_batch* b = create(ch, 0);
    expect(st_batch_tune(b, s, 1), ST_OK, "st_batch_tune before a launch");
    expect(st_batch_destroy(b), ST_OK, "st_batch_destroy");
  }
  for (int slots : {1, ST_BATCH_MAX_LANES}) {  // grouped launches in a caller workspace: one slot, several rounds
    const size_t wsb = st_batch_workspace_bytes(ch.desc.data(), n, slots);
    void* ws = dev(wsb);
    st_batch* b = create(ch, ST_BATCH_GROUPED, ws, wsb);
    int grouped = 0, rounds = 0;
    expect(st_batch_plan(b, &grouped, &rounds, nullptr), ST_OK, "st_batch_plan");
    if (!grouped || rounds < 1 || (slots == 1 && rounds < 2)) {
      std::fprintf(stderr, "hostcheck FAIL: grouped plan %d / %d rounds in %d slots\n", grouped, rounds, slots);
      std::exit(1);
    }
    for (int r = 0; r < 2; ++r) expect(st_batch_launch(b, r ? other : s), ST_OK, "st_batch_launch (grouped)");
    expect(st_batch_destroy(b), ST_OK, "st_batch_destroy (grouped)");
    (void)hipFree(ws);
  }
  {  // a sigma whose radius needs the three-pass gradient cannot be grouped
    st_batch* b = nullptr;
    expect(st_batch_create(ch.desc.data(), n, 2.6, 4.0, kC, kD, ST_BATCH_GROUPED, nullptr, 0, &b),
           ST_ERR_UNSUPPORTED, "st_batch_create grouped with sigma 2.6");
  }
  {  // a caller workspace; launched and destroyed with the launch still queued
    const size_t wsb = st_batch_workspace_bytes(ch.desc.data(), n, 2);
    void* ws = dev(wsb);
    st_batch* b = create(ch, 2, ws, wsb);
    expect(st_batch_launch(b, other), ST_OK, "st_batch_launch");
    expect(st_batch_destroy(b), ST_OK, "st_batch_destroy");
    (void)hipFree(ws);
  }
}

}  // namespace

int main() {
  hipStream_t s = nullptr, other = nullptr;
  if (hipStreamCreateWithFlags(&s, 0) != hipSuccess || hipStreamCreateWithFlags(&other, 0) != hipSuccess) return 1;
  single_volumes(nullptr);
  single_volumes(s);
  surrogate(s);
  training(s);
  profiling(s);
  fault_injection(s);
  batches(s, other);
  (void)hipStreamDestroy(s);
  (void)hipStreamDestroy(other);
  const hc::Counts c = hc::counts();
  const long live = hc::live_objects();
  std::printf("hostcheck: %d checks; %ld kernel launches, %ld captured operations, %ld graphs, %ld graph launches, "
              "%ld allocations; %ld objects left\n",
              g_checks, c.launches, c.captured_nodes, c.graphs, c.graph_launches, c.allocations, live);
  if (live != 0) {
    std::printf("hostcheck: FAIL (objects leaked)\n");
    return 1;
  }
  std::printf("hostcheck: OK\n");
  return 0;
}
