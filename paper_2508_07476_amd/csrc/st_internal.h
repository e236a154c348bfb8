// Internal declarations shared by the host layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/st.h"

namespace st {

constexpr int kMaxTaps = 2 * ST_MAX_RADIUS_RHO + 1;

// Kernel radii compiled into the library.  A request for radius R runs the
// smallest compiled radius R' >= R with the taps zero-padded to 2R'+1: the
// extra terms are exact zeros, so the result equals the radius-R filter.
#define ST_RADII_SIGMA_SMALL(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12)
#define ST_RADII_SIGMA(X) ST_RADII_SIGMA_SMALL(X) X(14) X(16)
#define ST_RADII_LARGE(X) X(14) X(16) X(20) X(24) X(28) X(32)
#define ST_RADII_RHO(X) ST_RADII_SIGMA(X) X(20) X(24) X(28) X(32)

inline int padded_radius(int R, bool sigma) {
  static const int rs[] = {
#define ST_LIST(r) r,
      ST_RADII_SIGMA(ST_LIST)
  };
  static const int rr[] = {ST_RADII_RHO(ST_LIST)
#undef ST_LIST
  };
  const int* b = sigma ? rs : rr;
  const int cnt = sigma ? int(sizeof(rs) / sizeof(int)) : int(sizeof(rr) / sizeof(int));
  for (int i = 0; i < cnt; ++i)
    if (b[i] >= R) return b[i];
  return -1;
}

// Filter taps in float64, index m <-> offset k = m - R.  Passed by value as a
// kernel argument so every tap lives in scalar registers.  All filter
// arithmetic runs in float64 (an FMA of either width issues at the same rate);
// intermediate planes are stored in float32.
struct Taps {
  double w[kMaxTaps];
};

// ---- strided-axis correlation (z or y) -------------------------------------
// One job = one input plane set filtered into one or two outputs (G and, when
// out_d != nullptr, D) with the same register window.
struct StridedJob {
  const void* in;
  float* out_g;
  float* out_d;
};

// Geometry of one strided launch (per volume in a grouped launch).
struct StridedGeo {
  StridedJob job[6];
  int njobs;
  int nchunks;       // chunks along the filtered axis
  int64_t chunk;     // outputs per chunk along the filtered axis
  int64_t n_axis;    // length of the filtered axis
  int64_t s_axis;    // element stride of the filtered axis in the inputs
  int64_t n_other;   // length of the remaining non-x axis
  int64_t s_other;   // its element stride in the inputs
  int64_t so_axis;   // the same two strides in the outputs (pitched workspace rows)
  int64_t so_other;
  int64_t nx;
  int64_t x_tiles;   // ceil(nx / 64)
  int64_t o_tiles;   // ceil(n_other / 4)
};

struct StridedParams : StridedGeo {
  Taps wg;           // smoothing taps: symmetric about the centre (read as such)
  Taps wd;           // derivative taps: antisymmetric about the centre
};

// in_dtype: ST_DTYPE_U16 or ST_DTYPE_F32.  with_d selects the two-output variant.
hipError_t launch_strided(int R, int in_dtype, bool with_d, const StridedParams& p,
                          hipStream_t stream);

// ---- x-axis gradient pass fused with the outer product ----------------------
struct XGradParams {
  const float* gg;  // Gy Gz V  -> Dx gives g_x
  const float* dg;  // Dy Gz V  -> Gx gives g_y
  const float* gd;  // Gy Dz V  -> Gx gives g_z
  float* prod[6];   // zz, zy, zx, yy, yx, xx
  int64_t nx;
  int64_t pitch;    // row pitch (elements) of the inputs and outputs (workspace rows)
  int64_t nrows;    // nz * ny
  int64_t x_tiles;  // ceil(nx / kXTile)
  int vec_ok;       // rows and outputs 16-byte aligned: float4 stores
  Taps wg;
  Taps wd;
};

// ---- x-axis integration fused with eigen-decomposition, FA and angles ------
struct XFinalGeo {
  const float* s[6];  // z- and y-integrated products, (zz, zy, zx, yy, yx, xx)
  const uint8_t* mask;
  float* e3;          // [3][N] or null
  float* evals;       // [3][N] or null
  float* fa;
  float* ha;
  float* ia;
  uint8_t* flags;
  int64_t n;          // nz * ny * nx
  int64_t nz, ny, nx;
  int64_t pitch;      // row pitch (elements) of s[] (workspace rows); mask and outputs use nx
  int64_t nrows;
  int64_t x_tiles;    // ceil(nx / (tile_lanes * kXVec))
  int tile_lanes;     // lanes per row segment: 64 (one row per wave) or 16 (four)
  int vec_ok;         // every float output 16-byte aligned: float4 stores wherever
                      // the row's element offset is a multiple of 4
  int has_axis;
  double center[3];   // (z, y, x)
  double dir[3];      // unit (z, y, x)
};

struct XFinalParams : XFinalGeo {
  Taps w;
};

constexpr int kXVec = 4;                 // consecutive x outputs per lane
constexpr int kXTile = 64 * kXVec;       // x outputs per wave (one row segment of 64 lanes)
constexpr int kXNarrowMaxRadius = 16;    // radii with 16-lane segments of the final pass
// Lanes per row segment of the final pass compiled for radius R.
constexpr bool xfinal_lanes_supported(int R, int lanes) {
  return lanes == 64 || (lanes == 16 && R <= kXNarrowMaxRadius);
}
constexpr int kRowsPerBlock = 4;         // rows per block of the angle kernel (one per wave)

hipError_t launch_xgrad(int R, const XGradParams& p, hipStream_t stream);
hipError_t launch_xfinal(int R, const XFinalParams& p, hipStream_t stream);

// ---- fused gradient: Gaussian-derivative gradient at sigma and outer product ----
// One pass over the input: every block owns a 4 x 64 (y, x) column tile and a
// chunk of z; each input plane of the chunk (plus z halo) is staged in LDS,
// filtered along y and then x, and the three partial results of each column
// enter register windows that are filtered along z.
struct GradGeo {
  const void* vol;
  float* prod[6];     // zz, zy, zx, yy, yx, xx
  int64_t nz, ny, nx;
  int64_t opitch;     // row pitch (elements) of prod[] (workspace rows); plane ny * opitch
  int64_t x_tiles, y_tiles;
  int64_t chunk;      // z outputs per block
  int nchunks;
  int rows;           // output rows (y) per block, one wave each: grad_rows_supported(R, rows)
};

struct GradFusedParams : GradGeo {
  Taps wg;
  Taps wd;
};
constexpr int kGradTX = 64;
// Output rows per block (one wave per row) by default: 8 where the kernel fits
// four waves per SIMD without spilling, else 4.
constexpr int grad_tile_rows(int R) { return R <= 6 ? 8 : 4; }
// Tile rows compiled for radius R: the default, and 4 rows up to radius 6 too.
constexpr bool grad_rows_supported(int R, int rows) {
  return rows == grad_tile_rows(R) || (rows == 4 && R <= 6);
}
constexpr int kGradMaxRadius = 8;  // larger sigma radii use the three separate passes
hipError_t launch_grad_fused(int R, int in_dtype, const GradFusedParams& p, hipStream_t stream);

// ---- grouped launches: one launch over several volumes ---------------------
// Block b of a grouped launch works on table entry e with
// first[e] <= b < first[e + 1], as block b - first[e] of that volume alone
// (blocks past that volume's own grid return at once).  Every entry of one
// launch shares the taps, the radius and the tile shape.  The tables are
// device memory owned by the caller of the launch.
template <class Geo>
struct Grouped {
  const Geo* geo;        // [count]
  const int64_t* first;  // [count + 1], first[0] = 0, nondecreasing
  int count;
};

struct GradFusedGroup {
  Grouped<GradGeo> g;
  Taps wg;
  Taps wd;
};
struct StridedGroup {      // integration passes: float32 input, smoothing taps only
  Grouped<StridedGeo> g;
  Taps wg;
};
struct XFinalGroup {
  Grouped<XFinalGeo> g;
  Taps w;
};

// Blocks of one volume alone in each pass (what the entry's range must hold).
inline int64_t grad_blocks(const GradGeo& g) { return g.x_tiles * g.y_tiles * g.nchunks; }
inline int64_t strided_blocks(const StridedGeo& g) { return g.x_tiles * g.o_tiles * g.nchunks * g.njobs; }
inline int64_t xfinal_blocks(const XFinalGeo& g) {
  return g.x_tiles * (g.tile_lanes == 64 ? g.nrows : (g.nrows + 3) / 4);
}

// `blocks` = first[count] of the host copy of the table.  rows / lanes: the tile
// shape every entry uses.  Strided entries must have njobs = 6 and share input
// and output strides (SAME).
hipError_t launch_grad_fused_grouped(int R, int in_dtype, int rows, const GradFusedGroup& p, int64_t blocks,
                                     hipStream_t stream);
hipError_t launch_strided_grouped(int R, const StridedGroup& p, int64_t blocks, hipStream_t stream);
hipError_t launch_xfinal_grouped(int R, int lanes, const XFinalGroup& p, int64_t blocks, hipStream_t stream);

// Chunk-batch completion record (k_batch.hip): *seq += 1; and progress[c] = *seq
// for the `count` chunks c = ids[t] (ids NULL: the one chunk `one`).
hipError_t launch_batch_begin(uint64_t* seq, hipStream_t stream);
hipError_t launch_batch_mark(const uint64_t* seq, uint64_t* progress, const int64_t* ids, int count, int64_t one,
                             hipStream_t stream);

// ---- standalone angles ------------------------------------------------------
struct AnglesParams {
  const float* e3;
  const uint8_t* mask;
  float* ha;
  float* ia;
  uint8_t* flags;
  int64_t n, ny, nx, nrows, x_tiles;
  int vec_ok;
  double center[3];
  double dir[3];
};
hipError_t launch_angles(const AnglesParams& p, hipStream_t stream);

}  // namespace st
