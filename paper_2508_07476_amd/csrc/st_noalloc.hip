// st_compute_noalloc: the st_compute path with its workspace in a device array
// the library holds, for callers that cannot allocate device memory.
//
// The array (`scratch`) is a file-scope __device__ variable: every device the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code the name is only a stand-in for the array; the device
// address comes from hipGetSymbolAddress, looked up once per device on the
// first call made with that device current, and only that address is handed
// to kernels.  Calls that overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "st_host.h"

using st::host::device_fail;
using st::host::fail;

namespace {

// Room for the 12 workspace planes of a volume up to 128^3 (rows of 128).
static __device__ __align__(256) char scratch[ST_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
int scratch_on_device(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(ST_ERR_UNSUPPORTED, "device ordinal %d is beyond the %d devices the scratch table covers",
                dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return device_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    }
    g_ptr[dev] = ptr;
  }
  *out = static_cast<char*>(g_ptr[dev]);
  return ST_OK;
}

}  // namespace

extern "C" int st_compute_noalloc(const void* volume, int dtype, const uint8_t* mask, int64_t nz,
                                  int64_t ny, int64_t nx, double sigma, double rho, double truncate,
                                  const double* axis_center, const double* axis_direction, float* e3,
                                  float* evals, float* fa, float* ha, float* ia, uint8_t* flags,
                                  void* stream) {
  st::host::clear_error();
  st::host::PathArgs a;
  int st = st::host::prepare_path(a, volume, dtype, mask, nz, ny, nx, sigma, rho, truncate, axis_center,
                                  axis_direction, e3, evals, fa, ha, ia, flags);
  if (st != ST_OK) return st;
  const size_t need = st::host::path_workspace_bytes(a.nz, a.ny, a.nx);
  if (need == 0 || need > static_cast<size_t>(ST_NOALLOC_SCRATCH_BYTES))
    return fail(ST_ERR_UNSUPPORTED,
                "st_compute_noalloc: a %lld x %lld x %lld volume needs %zu workspace bytes, more than the "
                "%lld-byte library scratch (use st_compute with a workspace instead)",
                (long long)nz, (long long)ny, (long long)nx, need, (long long)ST_NOALLOC_SCRATCH_BYTES);
  if ((st = st::host::check_path_buffers(a)) != ST_OK) return st;
  char* ws = nullptr;
  if ((st = scratch_on_device(&ws)) != ST_OK) return st;
  // Every workspace element a kernel reads is written earlier in the same call,
  // so nothing is cleared.  No timing events: the profiler may create them.
  const char* stage = "";
  hipError_t e = st::host::enqueue_path(a, ws, static_cast<hipStream_t>(stream), st::host::LaunchShape{},
                                        false, &stage);
  if (e != hipSuccess) return device_fail(e, stage);
  return ST_OK;
}
