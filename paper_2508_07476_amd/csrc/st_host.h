// Host-side pieces shared by the single-volume entry points and the chunk
// batch: error reporting, argument validation and the pass sequence.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

#include "st_internal.h"

namespace st {
namespace host {

// Sets the thread-local message returned by st_last_error() and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int device_fail(hipError_t e, const char* what);
void clear_error();
// True when the environment variable ST_FAULT_INJECT is "alloc": every library
// allocation of device memory is then reported as failed (ST_ERR_OUT_OF_MEMORY)
// before any HIP call, so tests can exercise that path on any machine.
bool alloc_fault_injected();

// One volume through the whole path, validated.
struct PathArgs {
  const void* volume;
  int dtype;
  const uint8_t* mask;
  int64_t nz, ny, nx, n;
  double sigma, rho, truncate;
  bool has_axis;
  double center[3];  // axis point in this volume's own voxel coordinates (z, y, x)
  double unit[3];    // unit axis direction (z, y, x)
  float* e3;
  float* evals;
  float* fa;
  float* ha;
  float* ia;
  uint8_t* flags;
};

// Launch shapes: how far each pass splits its filtered axis to fill the chip.
// The gradient pass splits z until it has at least 4 * grad_min_blocks waves
// (blocks of four waves' worth); the strided passes split until they have at
// least strided_min_waves waves (in both cases only while the pieces stay long
// against the filter radius).  Every gradient piece re-reads 2R halo planes, so
// the split stops at four waves per SIMD: a 512^3 volume's x-y tiles already
// fill the chip.  A batch of concurrent chains uses a quarter of both targets.
// Tile shapes: grad_rows (output rows per gradient block) and xfinal_lanes
// (lanes per row segment of the final pass); 0 takes the library's default for
// the radius and width, other values must be compiled for the radius
// (grad_rows_supported, xfinal_lanes_supported).
struct LaunchShape {
  int64_t grad_min_blocks = 1024;
  int64_t strided_min_waves = 16384;
  int grad_rows = 0;
  int xfinal_lanes = 0;
};

// Sizes each in [1, 2^31) with every byte count of the path fitting: *n is the
// voxel count.  Sets the error message on failure.
int check_sizes(int64_t nz, int64_t ny, int64_t nx, int64_t* n);
// sigma, rho, truncate finite and positive, with radii in [1, ST_MAX_RADIUS_*].
int check_scales(double sigma, double rho, double truncate);
// Axis given as both pointers or neither, finite, non-zero direction; the unit
// direction goes to unit[] (untouched without an axis).
int check_axis_args(const double* center, const double* direction, double unit[3]);
// Runs fn() bracketed by the library's timing events (when profiling is on).
hipError_t timed_call(const char* name, hipStream_t stream, const std::function<hipError_t()>& fn);

// Host-only validation of one volume's arguments (no HIP call); fills `a`.
// Returns ST_OK or an error code with the message set.
int prepare_path(PathArgs& a, const void* volume, int dtype, const uint8_t* mask, int64_t nz,
                 int64_t ny, int64_t nx, double sigma, double rho, double truncate,
                 const double* axis_center, const double* axis_direction, float* e3, float* evals,
                 float* fa, float* ha, float* ia, uint8_t* flags);

// The buffer [p, p + bytes) lies inside one device allocation (p NULL: ST_OK).
int check_device_buffer(const void* p, size_t bytes, const char* name);

// Every non-NULL buffer of `a` lies inside one device allocation of the size
// the path reads or writes, and is aligned to its element size.
int check_path_buffers(const PathArgs& a);

// Row pitch (elements) of the workspace planes: nx rounded up to a multiple of
// 32 floats (128 bytes) above 32, else of 4.  Every 64-column wave access to a
// workspace row then starts on a cache line whatever the volume's width, and
// every row is 16-byte aligned.
inline int64_t ws_pitch(int64_t nx) { return nx > 32 ? (nx + 31) / 32 * 32 : (nx + 3) / 4 * 4; }

// Workspace bytes of the pass sequence for an nz x ny x nx volume (12 float
// planes of nz * ny * ws_pitch(nx) elements, each 256-byte aligned); 0 if a size
// is out of range.
size_t path_workspace_bytes(int64_t nz, int64_t ny, int64_t nx);

// Reach of the pass sequence: an output depends on the input voxels within
// this Chebyshev distance (the gradient's and the integration's compiled
// radii), so a crop whose faces lie this far from a voxel, or on the volume's
// own faces, gives that voxel's outputs bit for bit; -1 for invalid scales.
int path_halo(double sigma, double rho, double truncate);

// The launches of the pass sequence of `a` with workspace `ws`: compiled radii,
// taps and geometry, exactly as enqueue_path launches them.
struct PathPlan {
  int rs, rr;                       // compiled gradient and integration radii
  bool fused_grad;                  // one fused gradient pass (else grad_z, grad_y0, grad_y1, grad_x)
  GradFusedParams grad;
  StridedParams grad_z, grad_y0, grad_y1;
  XGradParams grad_x;
  StridedParams int_z, int_y;       // integration along z and y
  XFinalParams fin;                 // x integration, eigen-decomposition, FA, angles
};
void plan_path(const PathArgs& a, char* ws, const LaunchShape& shape, PathPlan* plan);

// Enqueues the pass sequence of `a` on `stream` with workspace `ws`.  With
// `profile`, each launch is bracketed by the library's timing events (when
// profiling is enabled).  On failure returns the HIP error and names the pass
// in *stage.
hipError_t enqueue_path(const PathArgs& a, char* ws, hipStream_t stream, const LaunchShape& shape,
                        bool profile, const char** stage);

}  // namespace host
}  // namespace st
