// C ABI of the structure-tensor library: argument validation, workspace plan,
// filter taps, kernel sequence on the caller's stream, and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "st_host.h"

namespace {
thread_local std::string g_error;
}  // namespace

namespace st {
namespace host {

void clear_error() { g_error.clear(); }

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int device_fail(hipError_t e, const char* what) {
  return fail(ST_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool alloc_fault_injected() {
  const char* v = std::getenv("ST_FAULT_INJECT");
  return v != nullptr && std::strcmp(v, "alloc") == 0;
}

}  // namespace host
}  // namespace st

namespace {

using st::host::device_fail;
using st::host::fail;

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int radius_of(double scale, double truncate) {
  if (!finite_pos(scale) || !finite_pos(truncate)) return -1;
  const double r = std::floor(truncate * scale + 0.5);
  if (r > 1e6) return 1 << 20;
  return static_cast<int>(r);
}

// Normalised sampled Gaussian (w0) and derivative (w1 = k/s^2 w0) taps of
// radius R in double, stored centred in a window of radius Rpad >= R (the
// outer taps are exact zeros).
void make_taps(double s, int R, int Rpad, st::Taps& w0, st::Taps* w1) {
  double g[st::kMaxTaps];
  double sum = 0.0;
  for (int k = -R; k <= R; ++k) {
    g[k + R] = std::exp(-(double(k) * k) / (2.0 * s * s));
    sum += g[k + R];
  }
  std::memset(&w0, 0, sizeof(w0));
  if (w1) std::memset(w1, 0, sizeof(*w1));
  for (int k = -R; k <= R; ++k) {
    const double v = g[k + R] / sum;
    w0.w[k + Rpad] = v;
    if (w1) w1->w[k + Rpad] = (double(k) / (s * s)) * v;
  }
}

bool checked_count(int64_t nz, int64_t ny, int64_t nx, int64_t* n) {
  if (nz < 1 || ny < 1 || nx < 1) return false;
  if (nz > INT32_MAX || ny > INT32_MAX || nx > INT32_MAX) return false;
  int64_t a;
  if (__builtin_mul_overflow(nz, ny, &a)) return false;
  if (__builtin_mul_overflow(a, nx, n)) return false;
  // every byte count derived from n (12 float planes) must fit
  size_t b;
  if (__builtin_mul_overflow(static_cast<size_t>(*n), size_t(48), &b)) return false;
  return true;
}

size_t plane_bytes(int64_t n) { return ((static_cast<size_t>(n) * 4 + 255) / 256) * 256; }

// The buffer [p, p + bytes) must lie inside one device allocation.
int check_buffer(const void* p, size_t bytes, const char* name) {
  if (p == nullptr) return ST_OK;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  hipError_t e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
  if (e != hipSuccess || base == nullptr) {
    (void)hipGetLastError();
    return fail(ST_ERR_INVALID_ARG, "%s is not a device allocation (%s)", name, hipGetErrorString(e));
  }
  const uintptr_t lo = reinterpret_cast<uintptr_t>(base);
  const uintptr_t hi = lo + size;
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  if (a < lo || a + bytes > hi || a + bytes < a)
    return fail(ST_ERR_INVALID_ARG, "%s: %zu bytes needed past its address but the allocation ends sooner",
                name, bytes);
  return ST_OK;
}

int check_axis(const double* c, const double* d, double unit[3]) {
  if ((c == nullptr) != (d == nullptr))
    return fail(ST_ERR_INVALID_ARG, "axis_center and axis_direction must both be given or both be NULL");
  if (c == nullptr) return ST_OK;
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(c[i]) || !std::isfinite(d[i]))
      return fail(ST_ERR_INVALID_ARG, "axis_center / axis_direction must be finite");
  const double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (!(len > 0.0) || !std::isfinite(len))
    return fail(ST_ERR_INVALID_ARG, "axis_direction must have a non-zero finite length");
  for (int i = 0; i < 3; ++i) unit[i] = d[i] / len;
  return ST_OK;
}

// ---- kernel timing ----------------------------------------------------------
struct ProfEntry {
  std::string name;
  double total_ms = 0.0;
  int64_t launches = 0;
};
struct ProfPending {
  int entry;
  hipEvent_t start, stop;
};
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<ProfEntry> entries;
  std::vector<ProfPending> pending;
  std::vector<hipEvent_t> pool;
};
Profiler& prof() {
  static Profiler* p = new Profiler();  // intentionally leaked: used until process exit
  return *p;
}

hipEvent_t take_event() {
  Profiler& P = prof();
  if (!P.pool.empty()) {
    hipEvent_t e = P.pool.back();
    P.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch `fn` on `stream`, bracketed by timing events when profiling is on.
template <class F>
hipError_t timed(const char* name, hipStream_t stream, F&& fn) {
  Profiler& P = prof();
  if (!P.on) return fn();
  std::lock_guard<std::mutex> lk(P.mu);
  int idx = -1;
  for (size_t i = 0; i < P.entries.size(); ++i)
    if (P.entries[i].name == name) idx = static_cast<int>(i);
  if (idx < 0) {
    P.entries.push_back(ProfEntry{name, 0.0, 0});
    idx = static_cast<int>(P.entries.size()) - 1;
  }
  hipEvent_t a = take_event(), b = take_event();
  if (a == nullptr || b == nullptr) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, stream);
  if (e != hipSuccess) return e;
  e = fn();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, stream);
  if (e != hipSuccess) return e;
  P.pending.push_back(ProfPending{idx, a, b});
  return hipSuccess;
}

}  // namespace

namespace st {
namespace host {

int check_device_buffer(const void* p, size_t bytes, const char* name) {
  return check_buffer(p, bytes, name);
}

int check_sizes(int64_t nz, int64_t ny, int64_t nx, int64_t* n) {
  if (!checked_count(nz, ny, nx, n))
    return fail(ST_ERR_INVALID_ARG, "sizes (%lld, %lld, %lld) must be >= 1, < 2^31 each, and their byte counts must fit",
                (long long)nz, (long long)ny, (long long)nx);
  return ST_OK;
}

int check_scales(double sigma, double rho, double truncate) {
  if (!finite_pos(sigma) || !finite_pos(rho) || !finite_pos(truncate))
    return fail(ST_ERR_INVALID_ARG, "sigma, rho and truncate must be finite and > 0");
  const int rs = radius_of(sigma, truncate), rr = radius_of(rho, truncate);
  if (rs < 1 || rr < 1)
    return fail(ST_ERR_INVALID_ARG, "kernel radius floor(truncate*scale + 0.5) must be >= 1 (got %d, %d)", rs, rr);
  if (rs > ST_MAX_RADIUS_SIGMA || rr > ST_MAX_RADIUS_RHO)
    return fail(ST_ERR_UNSUPPORTED, "kernel radius %d (sigma) / %d (rho) exceeds %d / %d", rs, rr,
                ST_MAX_RADIUS_SIGMA, ST_MAX_RADIUS_RHO);
  return ST_OK;
}

int check_axis_args(const double* center, const double* direction, double unit[3]) {
  return check_axis(center, direction, unit);
}

hipError_t timed_call(const char* name, hipStream_t stream, const std::function<hipError_t()>& fn) {
  return ::timed(name, stream, fn);
}

int path_halo(double sigma, double rho, double truncate) {
  const int rs = radius_of(sigma, truncate), rr = radius_of(rho, truncate);
  if (rs < 0 || rr < 0) return -1;
  const int ps = padded_radius(rs, true), pr = padded_radius(rr, false);
  return (ps > 0 ? ps : rs) + (pr > 0 ? pr : rr);
}

size_t path_workspace_bytes(int64_t nz, int64_t ny, int64_t nx) {
  if (nz < 1 || ny < 1 || nx < 1) return 0;
  int64_t m;
  size_t b;
  if (__builtin_mul_overflow(nz, ny, &m) || __builtin_mul_overflow(m, ws_pitch(nx), &m) ||
      __builtin_mul_overflow(static_cast<size_t>(m), size_t(64), &b))
    return 0;
  return 12 * plane_bytes(m);
}

int prepare_path(PathArgs& a, const void* volume, int dtype, const uint8_t* mask, int64_t nz,
                 int64_t ny, int64_t nx, double sigma, double rho, double truncate,
                 const double* axis_center, const double* axis_direction, float* e3, float* evals,
                 float* fa, float* ha, float* ia, uint8_t* flags) {
  // ---- host-only validation (no HIP call before it passes) ----
  if (volume == nullptr) return fail(ST_ERR_INVALID_ARG, "volume is NULL");
  if (dtype != ST_DTYPE_U16 && dtype != ST_DTYPE_F32)
    return fail(ST_ERR_INVALID_ARG, "dtype %d is neither ST_DTYPE_U16 nor ST_DTYPE_F32", dtype);
  int64_t n;
  if (!checked_count(nz, ny, nx, &n))
    return fail(ST_ERR_INVALID_ARG, "sizes (%lld, %lld, %lld) must be >= 1, < 2^31 each, and their byte counts must fit",
                (long long)nz, (long long)ny, (long long)nx);
  if (!finite_pos(sigma) || !finite_pos(rho) || !finite_pos(truncate))
    return fail(ST_ERR_INVALID_ARG, "sigma, rho and truncate must be finite and > 0");
  const int rs = radius_of(sigma, truncate), rr = radius_of(rho, truncate);
  if (rs < 1 || rr < 1)
    return fail(ST_ERR_INVALID_ARG, "kernel radius floor(truncate*scale + 0.5) must be >= 1 (got %d, %d)", rs, rr);
  if (rs > ST_MAX_RADIUS_SIGMA || rr > ST_MAX_RADIUS_RHO)
    return fail(ST_ERR_UNSUPPORTED, "kernel radius %d (sigma) / %d (rho) exceeds %d / %d", rs, rr,
                ST_MAX_RADIUS_SIGMA, ST_MAX_RADIUS_RHO);
  double unit[3] = {0, 0, 0};
  int st = check_axis(axis_center, axis_direction, unit);
  if (st != ST_OK) return st;
  const bool has_axis = axis_center != nullptr;
  if (!has_axis && (ha != nullptr || ia != nullptr))
    return fail(ST_ERR_INVALID_ARG, "ha / ia need an axis (axis_center and axis_direction)");
  if (!e3 && !evals && !fa && !ha && !ia && !flags)
    return fail(ST_ERR_INVALID_ARG, "no output requested");

  a.volume = volume; a.dtype = dtype; a.mask = mask;
  a.nz = nz; a.ny = ny; a.nx = nx; a.n = n;
  a.sigma = sigma; a.rho = rho; a.truncate = truncate;
  a.has_axis = has_axis;
  for (int i = 0; i < 3; ++i) {
    a.center[i] = has_axis ? axis_center[i] : 0.0;
    a.unit[i] = unit[i];
  }
  a.e3 = e3; a.evals = evals; a.fa = fa; a.ha = ha; a.ia = ia; a.flags = flags;
  return ST_OK;
}

int check_path_buffers(const PathArgs& a) {
  const size_t N = static_cast<size_t>(a.n);
  const size_t esz = a.dtype == ST_DTYPE_U16 ? 2 : 4;
  int st;
  if ((st = check_buffer(a.volume, N * esz, "volume")) != ST_OK) return st;
  if ((st = check_buffer(a.mask, N, "mask")) != ST_OK) return st;
  if ((st = check_buffer(a.e3, 3 * N * 4, "e3")) != ST_OK) return st;
  if ((st = check_buffer(a.evals, 3 * N * 4, "evals")) != ST_OK) return st;
  if ((st = check_buffer(a.fa, N * 4, "fa")) != ST_OK) return st;
  if ((st = check_buffer(a.ha, N * 4, "ha")) != ST_OK) return st;
  if ((st = check_buffer(a.ia, N * 4, "ia")) != ST_OK) return st;
  if ((st = check_buffer(a.flags, N, "flags")) != ST_OK) return st;
  if ((reinterpret_cast<uintptr_t>(a.volume) % esz) != 0)
    return fail(ST_ERR_INVALID_ARG, "volume is not aligned to its element size");
  for (const void* q : {static_cast<const void*>(a.e3), static_cast<const void*>(a.evals),
                        static_cast<const void*>(a.fa), static_cast<const void*>(a.ha),
                        static_cast<const void*>(a.ia)})
    if (q && (reinterpret_cast<uintptr_t>(q) % 4) != 0)
      return fail(ST_ERR_INVALID_ARG, "float outputs must be 4-byte aligned");
  return ST_OK;
}

void plan_path(const PathArgs& a, char* ws, const LaunchShape& shape, PathPlan* plan) {
  const void* volume = a.volume;
  const int64_t nz = a.nz, ny = a.ny, nx = a.nx;
  // workspace planes: rows of `pitch` elements (the volume's rows are nx long)
  const int64_t pitch = ws_pitch(nx);
  const size_t pb = plane_bytes(nz * ny * pitch);
  float* A[6];
  float* B[6];
  for (int c = 0; c < 6; ++c) {
    A[c] = reinterpret_cast<float*>(ws + c * pb);
    B[c] = reinterpret_cast<float*>(ws + (6 + c) * pb);
  }

  // compiled radii: the next one up, taps zero-padded
  const int rs = radius_of(a.sigma, a.truncate), rr = radius_of(a.rho, a.truncate);
  const int ps = st::padded_radius(rs, true), pr = st::padded_radius(rr, false);
  plan->rs = ps;
  plan->rr = pr;
  st::Taps gs, ds, gr;
  make_taps(a.sigma, rs, ps, gs, &ds);
  make_taps(a.rho, rr, pr, gr, nullptr);

  // in_volume: the jobs read the caller's volume (rows of nx), else workspace
  // planes; outputs are always workspace planes
  auto strided = [&](st::StridedParams& p, bool zaxis, bool in_volume, int njobs, const st::StridedJob* jobs,
                     int R, const st::Taps& wg, const st::Taps* wd) {
    std::memset(&p, 0, sizeof(p));
    for (int j = 0; j < njobs; ++j) p.job[j] = jobs[j];
    p.njobs = njobs;
    p.nx = nx;
    const int64_t ip = in_volume ? nx : pitch;
    if (zaxis) {
      p.n_axis = nz; p.s_axis = ny * ip; p.n_other = ny; p.s_other = ip;
      p.so_axis = ny * pitch; p.so_other = pitch;
    } else {
      p.n_axis = ny; p.s_axis = ip; p.n_other = nz; p.s_other = ny * ip;
      p.so_axis = pitch; p.so_other = ny * pitch;
    }
    p.x_tiles = (nx + 63) / 64;
    p.o_tiles = (p.n_other + 3) / 4;
    // split the filtered axis until the launch has enough waves to fill the chip
    const int64_t waves = p.x_tiles * p.n_other * njobs;
    int nchunks = 1;
    const int64_t min_chunk = std::max<int64_t>(64, 4 * R);
    while (waves * nchunks < shape.strided_min_waves &&
           (p.n_axis + 2 * nchunks - 1) / (2 * nchunks) >= min_chunk)
      nchunks *= 2;
    p.nchunks = nchunks;
    p.chunk = (p.n_axis + nchunks - 1) / nchunks;
    p.nchunks = static_cast<int>((p.n_axis + p.chunk - 1) / p.chunk);
    p.wg = wg;
    if (wd) p.wd = *wd;
  };

  // gradient at sigma and outer product: one fused pass when the radius and the
  // plane size allow it, else z pass (G, D), y pass, x pass + outer product
  plan->fused_grad = ps <= st::kGradMaxRadius && ny * nx <= INT32_MAX;
  if (plan->fused_grad) {
    st::GradFusedParams& p = plan->grad;
    std::memset(&p, 0, sizeof(p));
    p.vol = volume;
    for (int c = 0; c < 6; ++c) p.prod[c] = B[c];
    p.nz = nz; p.ny = ny; p.nx = nx;
    p.opitch = pitch;
    p.x_tiles = (nx + st::kGradTX - 1) / st::kGradTX;
    const int64_t rows = shape.grad_rows ? shape.grad_rows : st::grad_tile_rows(ps);
    p.rows = static_cast<int>(rows);
    p.y_tiles = (ny + rows - 1) / rows;
    // split z until there are enough waves to fill the chip (grad_min_blocks
    // counts blocks of four waves), keeping chunks >= 8R
    const int64_t waves_per_block = rows;  // one wave per tile row
    int64_t nch = 1;
    while (p.x_tiles * p.y_tiles * nch * waves_per_block < 4 * shape.grad_min_blocks && nz / (2 * nch) >= 8 * ps)
      nch *= 2;
    p.chunk = (nz + nch - 1) / nch;
    p.nchunks = static_cast<int>((nz + p.chunk - 1) / p.chunk);
    p.wg = gs; p.wd = ds;
  } else {
    const st::StridedJob jz = {volume, B[0], B[1]}, jy0 = {B[0], A[0], A[1]}, jy1 = {B[1], A[2], nullptr};
    strided(plan->grad_z, true, true, 1, &jz, ps, gs, &ds);
    strided(plan->grad_y0, false, false, 1, &jy0, ps, gs, &ds);
    strided(plan->grad_y1, false, false, 1, &jy1, ps, gs, nullptr);
    st::XGradParams& p = plan->grad_x;
    std::memset(&p, 0, sizeof(p));
    p.gg = A[0]; p.dg = A[1]; p.gd = A[2];
    for (int c = 0; c < 6; ++c) p.prod[c] = B[c];
    p.nx = nx; p.pitch = pitch; p.nrows = nz * ny; p.x_tiles = (nx + st::kXTile - 1) / st::kXTile;
    p.vec_ok = 1;  // workspace rows: 16-byte aligned
    p.wg = gs; p.wd = ds;
  }
  // integration: z pass, y pass (6 components each)
  st::StridedJob j[6];
  for (int c = 0; c < 6; ++c) j[c] = st::StridedJob{B[c], A[c], nullptr};
  strided(plan->int_z, true, false, 6, j, pr, gr, nullptr);
  for (int c = 0; c < 6; ++c) j[c] = st::StridedJob{A[c], B[c], nullptr};
  strided(plan->int_y, false, false, 6, j, pr, gr, nullptr);
  // x integration fused with eigen, FA, angles
  st::XFinalParams& p = plan->fin;
  std::memset(&p, 0, sizeof(p));
  for (int c = 0; c < 6; ++c) p.s[c] = B[c];
  p.mask = a.mask; p.e3 = a.e3; p.evals = a.evals; p.fa = a.fa; p.ha = a.ha; p.ia = a.ia; p.flags = a.flags;
  p.n = a.n; p.nz = nz; p.ny = ny; p.nx = nx; p.pitch = pitch; p.nrows = nz * ny;
  // segments of 64 lanes (256 outputs), or of 16 (64 outputs, four rows per
  // wave) where that fills at least 5 % more of the lanes
  auto fill = [&](int64_t tl) {
    const int64_t t = tl * st::kXVec;
    return static_cast<double>(nx) / static_cast<double>(t * ((nx + t - 1) / t));
  };
  p.tile_lanes = shape.xfinal_lanes ? shape.xfinal_lanes
                                    : (pr <= st::kXNarrowMaxRadius && fill(16) >= fill(64) + 0.05) ? 16 : 64;
  p.x_tiles = (nx + p.tile_lanes * st::kXVec - 1) / (p.tile_lanes * st::kXVec);
  bool vec = true;  // the kernel also checks each row's and plane's offset
  for (const void* q : {static_cast<const void*>(a.e3), static_cast<const void*>(a.evals),
                        static_cast<const void*>(a.fa), static_cast<const void*>(a.ha),
                        static_cast<const void*>(a.ia)})
    if (q && (reinterpret_cast<uintptr_t>(q) % 16) != 0) vec = false;
  if (a.flags && (reinterpret_cast<uintptr_t>(a.flags) % 4) != 0) vec = false;
  p.vec_ok = vec;
  p.has_axis = a.has_axis;
  if (a.has_axis)
    for (int i = 0; i < 3; ++i) { p.center[i] = a.center[i]; p.dir[i] = a.unit[i]; }
  p.w = gr;
}

hipError_t enqueue_path(const PathArgs& a, char* ws, hipStream_t stream, const LaunchShape& shape,
                        bool profile, const char** stage_out) {
  auto timed = [&](const char* name, hipStream_t s, auto&& fn) -> hipError_t {
    return profile ? ::timed(name, s, fn) : fn();
  };
  PathPlan pl;
  plan_path(a, ws, shape, &pl);
  const int ps = pl.rs, pr = pl.rr;
  hipError_t e = hipSuccess;
  const char* stage = "";
  do {
    if (pl.fused_grad) {
      stage = "grad_fused";
      e = timed("grad_fused", stream, [&] { return st::launch_grad_fused(ps, a.dtype, pl.grad, stream); });
      if (e != hipSuccess) break;
    } else {
      stage = "grad_z";
      e = timed("grad_z", stream, [&] { return st::launch_strided(ps, a.dtype, true, pl.grad_z, stream); });
      if (e != hipSuccess) break;
      stage = "grad_y";
      e = timed("grad_y", stream, [&] { return st::launch_strided(ps, ST_DTYPE_F32, true, pl.grad_y0, stream); });
      if (e != hipSuccess) break;
      e = timed("grad_y", stream, [&] { return st::launch_strided(ps, ST_DTYPE_F32, false, pl.grad_y1, stream); });
      if (e != hipSuccess) break;
      stage = "grad_x_outer";
      e = timed("grad_x_outer", stream, [&] { return st::launch_xgrad(ps, pl.grad_x, stream); });
      if (e != hipSuccess) break;
    }
    stage = "integrate_z";
    e = timed("integrate_z", stream, [&] { return st::launch_strided(pr, ST_DTYPE_F32, false, pl.int_z, stream); });
    if (e != hipSuccess) break;
    stage = "integrate_y";
    e = timed("integrate_y", stream, [&] { return st::launch_strided(pr, ST_DTYPE_F32, false, pl.int_y, stream); });
    if (e != hipSuccess) break;
    stage = "integrate_x_eigen";
    e = timed("integrate_x_eigen", stream, [&] { return st::launch_xfinal(pr, pl.fin, stream); });
  } while (false);
  *stage_out = stage;
  return e;
}

}  // namespace host
}  // namespace st

extern "C" {

int st_version(void) { return 10000; }

const char* st_last_error(void) { return g_error.c_str(); }

int st_filter_radius(double scale, double truncate) { return radius_of(scale, truncate); }

size_t st_workspace_bytes(int64_t nz, int64_t ny, int64_t nx) {
  int64_t n;
  if (!checked_count(nz, ny, nx, &n)) return 0;
  return st::host::path_workspace_bytes(nz, ny, nx);
}

int st_compute(const void* volume, int dtype, const uint8_t* mask, int64_t nz, int64_t ny,
               int64_t nx, double sigma, double rho, double truncate, const double* axis_center,
               const double* axis_direction, float* e3, float* evals, float* fa, float* ha,
               float* ia, uint8_t* flags, void* workspace, size_t workspace_bytes, void* stream_) {
  g_error.clear();
  st::host::PathArgs a;
  int st = st::host::prepare_path(a, volume, dtype, mask, nz, ny, nx, sigma, rho, truncate,
                                  axis_center, axis_direction, e3, evals, fa, ha, ia, flags);
  if (st != ST_OK) return st;
  const size_t ws_need = st::host::path_workspace_bytes(a.nz, a.ny, a.nx);
  if (ws_need == 0) return fail(ST_ERR_INVALID_ARG, "workspace size of the volume overflows");
  if (workspace == nullptr && workspace_bytes != 0)
    return fail(ST_ERR_INVALID_ARG, "workspace is NULL but workspace_bytes is %zu", workspace_bytes);
  if (workspace != nullptr && workspace_bytes < ws_need)
    return fail(ST_ERR_INVALID_ARG, "workspace_bytes %zu < required %zu", workspace_bytes, ws_need);
  if (workspace == nullptr && st::host::alloc_fault_injected())
    return fail(ST_ERR_OUT_OF_MEMORY, "workspace allocation of %zu bytes failed (ST_FAULT_INJECT=alloc)", ws_need);
  if ((st = st::host::check_path_buffers(a)) != ST_OK) return st;
  if ((st = check_buffer(workspace, ws_need, "workspace")) != ST_OK) return st;

  hipStream_t stream = static_cast<hipStream_t>(stream_);
  char* ws = static_cast<char*>(workspace);
  bool owned = false;
  if (ws == nullptr) {
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&ws), ws_need, stream);
    if (e != hipSuccess || ws == nullptr) {
      (void)hipGetLastError();
      return fail(ST_ERR_OUT_OF_MEMORY, "hipMallocAsync(%zu) failed: %s", ws_need, hipGetErrorString(e));
    }
    owned = true;
  }
  const char* stage = "";
  hipError_t e = st::host::enqueue_path(a, ws, stream, st::host::LaunchShape{}, true, &stage);
  if (owned) {
    hipError_t f = hipFreeAsync(ws, stream);
    if (e == hipSuccess && f != hipSuccess) { e = f; stage = "hipFreeAsync"; }
  }
  if (e != hipSuccess) return device_fail(e, stage);
  return ST_OK;
}

int st_angles(const float* e3, const uint8_t* mask, int64_t nz, int64_t ny, int64_t nx,
              const double* axis_center, const double* axis_direction, float* ha, float* ia,
              uint8_t* flags, void* stream_) {
  g_error.clear();
  if (e3 == nullptr) return fail(ST_ERR_INVALID_ARG, "e3 is NULL");
  int64_t n;
  if (!checked_count(nz, ny, nx, &n))
    return fail(ST_ERR_INVALID_ARG, "sizes (%lld, %lld, %lld) must be >= 1, < 2^31 each, and their byte counts must fit",
                (long long)nz, (long long)ny, (long long)nx);
  if (axis_center == nullptr || axis_direction == nullptr)
    return fail(ST_ERR_INVALID_ARG, "st_angles needs axis_center and axis_direction");
  double unit[3];
  int st = check_axis(axis_center, axis_direction, unit);
  if (st != ST_OK) return st;
  if (!ha && !ia && !flags) return fail(ST_ERR_INVALID_ARG, "no output requested");
  const size_t N = static_cast<size_t>(n);
  if ((st = check_buffer(e3, 3 * N * 4, "e3")) != ST_OK) return st;
  if ((st = check_buffer(mask, N, "mask")) != ST_OK) return st;
  if ((st = check_buffer(ha, N * 4, "ha")) != ST_OK) return st;
  if ((st = check_buffer(ia, N * 4, "ia")) != ST_OK) return st;
  if ((st = check_buffer(flags, N, "flags")) != ST_OK) return st;
  for (const void* q : {static_cast<const void*>(e3), static_cast<const void*>(ha), static_cast<const void*>(ia)})
    if (q && (reinterpret_cast<uintptr_t>(q) % 4) != 0)
      return fail(ST_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");

  st::AnglesParams p;
  std::memset(&p, 0, sizeof(p));
  p.e3 = e3; p.mask = mask; p.ha = ha; p.ia = ia; p.flags = flags;
  p.n = n; p.ny = ny; p.nx = nx; p.nrows = nz * ny;
  p.x_tiles = (nx + st::kXTile - 1) / st::kXTile;
  p.vec_ok = 0;
  for (int i = 0; i < 3; ++i) { p.center[i] = axis_center[i]; p.dir[i] = unit[i]; }
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  hipError_t e = timed("angles", stream, [&] { return st::launch_angles(p, stream); });
  if (e != hipSuccess) return device_fail(e, "angles");
  return ST_OK;
}

int st_profile_enable(int on) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  P.on = on != 0;
  return ST_OK;
}

int st_profile_reset(void) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  for (auto& q : P.pending) {
    (void)hipEventSynchronize(q.stop);
    P.pool.push_back(q.start);
    P.pool.push_back(q.stop);
  }
  P.pending.clear();
  P.entries.clear();
  return ST_OK;
}

int st_profile_read(int index, char* name, size_t name_len, double* total_ms, int64_t* launches) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  for (auto& q : P.pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(q.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, q.start, q.stop);
    if (e != hipSuccess) return -device_fail(e, "st_profile_read");
    P.entries[q.entry].total_ms += ms;
    P.entries[q.entry].launches += 1;
    P.pool.push_back(q.start);
    P.pool.push_back(q.stop);
  }
  P.pending.clear();
  const int count = static_cast<int>(P.entries.size());
  if (index >= 0 && index < count) {
    const ProfEntry& en = P.entries[index];
    if (name && name_len) {
      std::strncpy(name, en.name.c_str(), name_len - 1);
      name[name_len - 1] = '\0';
    }
    if (total_ms) *total_ms = en.total_ms;
    if (launches) *launches = en.launches;
  }
  return count;
}

}  // extern "C"
