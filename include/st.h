/*
 * st.h -- C ABI of the MI355X (gfx950) voxel-wise 3D structure-tensor library.
 *
 * The library computes, for every voxel of a 3-D intensity volume, the local
 * fibre orientation of the paper's orientation module (Architecture section;
 * Figure 1(a)-(c)): Gaussian-derivative gradients at scale sigma, the
 * six-component gradient outer product, Gaussian integration at scale rho,
 * a 3x3 symmetric eigen-decomposition whose smallest-eigenvalue vector e3 is
 * the fibre direction, fractional anisotropy (FA), and helix / intrusion
 * angles (HA, IA) in a cylindrical frame about a given left-ventricular axis.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays are C-order [nz][ny][nx] (x fastest), unit isotropic spacing.
 *    Vectors (e3, axis centre, axis direction) are in (z, y, x) order.
 *  - Every array pointer is a DEVICE pointer allocated by the caller, except
 *    axis_center / axis_direction, which are HOST pointers to 3 doubles.
 *    The caller owns all memory; the library never frees caller memory.
 *  - Work is only enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *    the default stream). Results are valid once the caller synchronises the
 *    stream; the library never synchronises the device.
 *  - Arguments are validated on the host before any HIP call; on error the
 *    function returns a non-zero status, enqueues nothing and leaves every
 *    output untouched. st_last_error() then returns a thread-local message.
 *  - Results are bitwise deterministic for a given device and arguments
 *    (no atomics, fixed summation order).
 *
 * Filters (reading of the paper, which names the structure tensor but prints
 * no formula): for scale s and `truncate` t the kernel radius is
 * R = floor(t*s + 0.5); taps w0(k) = exp(-k^2/(2 s^2)) / sum_j exp(-j^2/(2 s^2))
 * and w1(k) = (k/s^2) w0(k) for k in [-R, R], applied as 1-D correlations with
 * half-sample symmetric reflection at every face.  Filter arithmetic runs in
 * float64 with float32 intermediate planes; the eigen-decomposition, FA and
 * the frame run in float64 with float32 trigonometric steps.
 */
#ifndef ST_H_
#define ST_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every entry point. */
#define ST_OK 0
#define ST_ERR_INVALID_ARG 1   /* a pointer, size, scale or axis is invalid */
#define ST_ERR_UNSUPPORTED 2   /* valid request this build cannot serve (e.g. kernel radius > 32) */
#define ST_ERR_OUT_OF_MEMORY 3 /* the library could not allocate its workspace */
#define ST_ERR_DEVICE 4        /* a HIP call failed; st_last_error() holds hipGetErrorString */

/* Input element types. */
#define ST_DTYPE_U16 1
#define ST_DTYPE_F32 2

/* Bits of the per-voxel flags output. */
#define ST_FLAG_DEGENERATE 1   /* trace <= 0 or (lambda2 - lambda3)/trace < 1e-3 */
#define ST_FLAG_OUTSIDE_MASK 2 /* mask == 0: every other output of the voxel is 0 */
#define ST_FLAG_ON_AXIS 4      /* distance to the axis < 1e-9: HA = IA = 0 */

/* Largest kernel radius R = floor(truncate*scale + 0.5) served, for sigma and rho. */
#define ST_MAX_RADIUS_SIGMA 16
#define ST_MAX_RADIUS_RHO 32

/* Library version, 10000*major + 100*minor + patch. */
int st_version(void);

/* Message describing the last non-OK status returned on this thread ("" if none). */
const char* st_last_error(void);

/* Kernel radius floor(truncate*scale + 0.5), or -1 if scale/truncate are not finite and > 0. */
int st_filter_radius(double scale, double truncate);

/*
 * Bytes of device workspace st_compute needs for an nz*ny*nx volume: 12 float32
 * planes, each 256-byte aligned, of nz*ny rows of nx values padded to a
 * multiple of 32 (of 4 when nx <= 32), so that the intermediate planes' rows
 * start on 128-byte lines.  The layout is internal; callers only size the
 * buffer.  Returns 0 on invalid sizes (non-positive, or a byte count that
 * overflows size_t).
 */
size_t st_workspace_bytes(int64_t nz, int64_t ny, int64_t nx);

/*
 * st_compute -- the whole orientation path in one call (paper: Figure 1(a)-(c),
 * orientation module of the Architecture section).
 *
 *  volume          device, nz*ny*nx elements of `dtype` (ST_DTYPE_U16 or ST_DTYPE_F32)
 *  mask            device, nz*ny*nx uint8 (nonzero = tissue) or NULL (every voxel is tissue).
 *                  The tensor is computed from the raw intensities; the mask only
 *                  gates the outputs (outside: e3 = evals = FA = HA = IA = 0, flags = 2).
 *  nz, ny, nx      sizes, each >= 1
 *  sigma, rho      gradient and integration scales in voxels (> 0, finite)
 *  truncate        kernel half-width in units of the scale (> 0; 4.0 is customary);
 *                  radii above ST_MAX_RADIUS_SIGMA / ST_MAX_RADIUS_RHO -> ST_ERR_UNSUPPORTED
 *  axis_center     host double[3] (z, y, x) voxel coordinates of a point on the axis, or NULL
 *  axis_direction  host double[3] (z, y, x) axis direction (any non-zero length);
 *                  NULL iff axis_center is NULL.  Without an axis, ha and ia must be NULL.
 *  e3              device float[3][nz*ny*nx] (SoA: z, y, x planes), unit fibre vectors
 *                  with canonical sign (largest-|.| component positive, ties to z then y), or NULL
 *  evals           device float[3][nz*ny*nx], lambda1 >= lambda2 >= lambda3, or NULL
 *  fa, ha, ia      device float[nz*ny*nx] (HA, IA in radians, in [-pi/2, pi/2]), or NULL
 *  flags           device uint8[nz*ny*nx] (ST_FLAG_* bits), or NULL
 *  workspace       device scratch of at least st_workspace_bytes(nz, ny, nx) bytes, or NULL
 *                  with workspace_bytes == 0: the library then allocates it stream-ordered
 *                  (hipMallocAsync) and frees it after the last kernel (hipFreeAsync).
 *  stream          hipStream_t on which all work is enqueued
 *
 * HA = atan2(f_a sgn f_t, |f_t|) and IA = atan2(f_r sgn f_t, |f_t|) with f_* the
 * components of e3 on the frame e_r (radial), e_t = a x e_r (right-handed) and a
 * (axis), sgn(0) = +1.  Buffers must not overlap each other or the workspace.
 */
int st_compute(const void* volume, int dtype, const uint8_t* mask,
               int64_t nz, int64_t ny, int64_t nx,
               double sigma, double rho, double truncate,
               const double* axis_center, const double* axis_direction,
               float* e3, float* evals, float* fa, float* ha, float* ia, uint8_t* flags,
               void* workspace, size_t workspace_bytes, void* stream);

/*
 * st_compute_noalloc -- st_compute for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It allocates nothing.
 *
 * Arguments, outputs and results are those of st_compute (bitwise: the same
 * kernels and workspace layout), without workspace / workspace_bytes.  The
 * workspace is a device array of ST_NOALLOC_SCRATCH_BYTES bytes held by the
 * library; every device it runs on keeps its own copy until the process ends.
 * Volumes whose st_workspace_bytes(nz, ny, nx) exceeds that size (about 128^3
 * voxels) return ST_ERR_UNSUPPORTED before any work is enqueued.  Nothing in
 * the array needs to start at zero.  Every call on a device shares that
 * device's array: calls on one stream are ordered, but calls that may overlap
 * on one device (other streams, other threads) race and give wrong results.
 */
#define ST_NOALLOC_SCRATCH_BYTES (128LL * 1024 * 1024)
int st_compute_noalloc(const void* volume, int dtype, const uint8_t* mask,
                       int64_t nz, int64_t ny, int64_t nx,
                       double sigma, double rho, double truncate,
                       const double* axis_center, const double* axis_direction,
                       float* e3, float* evals, float* fa, float* ha, float* ia, uint8_t* flags,
                       void* stream);

/*
 * st_angles -- helix and intrusion angles of a given fibre field about a new
 * axis (paper: Figure 1(c), cylindrical coordinate rotation), without
 * recomputing the tensor.
 *
 *  e3              device float[3][nz*ny*nx] (SoA z, y, x); need not be normalised
 *                  (a zero vector gives HA = IA = 0)
 *  mask            device uint8[nz*ny*nx] or NULL; outside: HA = IA = 0
 *  axis_center, axis_direction   host double[3] each, required
 *  ha, ia          device float[nz*ny*nx] outputs (radians); either may be NULL
 *  flags           device uint8[nz*ny*nx] or NULL: receives ST_FLAG_OUTSIDE_MASK and
 *                  ST_FLAG_ON_AXIS only (never ST_FLAG_DEGENERATE)
 */
int st_angles(const float* e3, const uint8_t* mask,
              int64_t nz, int64_t ny, int64_t nx,
              const double* axis_center, const double* axis_direction,
              float* ha, float* ia, uint8_t* flags, void* stream);

/*
 * st_surrogate_infer -- learned orientation surrogate with fallback.  Not a
 * method of the paper: a dense 3-D CNN trained to approximate the fibre
 * direction and FA that st_compute derives from the structure tensor (the
 * orientation output of Figure 1(b)), evaluated on the bf16 matrix cores.
 *
 * Network (weights blob: ST_SURROGATE_WEIGHTS float32 values, in this order:
 * in_scale, in_offset; W1 [32][1][27], b1 [32]; W2..W5 [32][32][27], b [32]
 * each; Wh [5][32], bh [5]; tap t = 9 (dz+1) + 3 (dy+1) + (dx+1)):
 *   x0 = bf16(v * in_scale + in_offset)
 *   x_l = relu(b_l + sum_{c,t} bf16(W_l)[:, c, t] x_{l-1}[c, p + off(t)]), l = 1..5,
 *         3x3x3 correlation with indices clamped at every face, float32
 *         accumulation, rounded to bf16 for l < 5
 *   h = bh + Wh x_5;  e3 = h[0:3]/|h[0:3]| with the canonical sign ((1,0,0)
 *   when zero);  FA = sigmoid(h[3]);  confidence = sigmoid(h[4]).
 *
 *  volume, dtype, mask, nz, ny, nx, axis_center, axis_direction: as st_compute.
 *  weights         DEVICE pointer to the float32 blob; weights_bytes >= 4 * ST_SURROGATE_WEIGHTS
 *  min_confidence  in [0, 1]: inside the mask, voxels whose confidence is below
 *                  it take st_compute's outputs (sigma, rho, truncate: as
 *                  st_compute, validated only when min_confidence > 0)
 *  e3 [3][N], fa, ha, ia, confidence [N]: DEVICE outputs, each may be NULL, at
 *                  least one given; ha / ia need the axis.  Outside the mask
 *                  every output is 0.  confidence is the surrogate's.
 * Fallback (min_confidence > 0 and an output other than confidence): the
 * volume is cut into cubic tiles; a tile holding a voxel below the threshold
 * inside the mask is flagged.  The call then waits for the flags (it is
 * synchronous from here on) and takes the cheapest of: nothing (no tile
 * flagged); the flagged tiles of one edge (32, 64 or 128 voxels), each
 * gathered with the structure-tensor path's reach of context (its compiled
 * gradient and integration radii) into a crop, all crops run as one chunk
 * batch (st_batch_create, grouped launches where sigma allows); or the whole
 * volume.  A crop gives its tile st_compute's whole-volume outputs bit for
 * bit (its faces lie beyond the path's reach or on the volume's faces); ha /
 * ia also when every axis_center coordinate minus an integer is exact in
 * double (e.g. a multiple of 1/2 below 2^50).  st_surrogate_fallback_info
 * reports which was taken.
 * The network runs in z slabs: two bf16 activation buffers of a slab plus 4
 * planes on each side (64 bytes per voxel each; slabs as thick as keep both
 * within 16 GiB, or within the byte count in the environment variable
 * ST_SURROGATE_SLAB_BYTES, the whole volume when it fits), every layer
 * computing only the planes the next one needs.  Results do not depend on the
 * slab thickness (bit for bit).
 * Device workspace: the two activation buffers, taken with hipMallocAsync on
 * `stream` and released the same way at the end of the call; with a fallback,
 * the crops (hipMalloc, about 75 bytes per crop voxel and their batch) or,
 * for the whole volume, nothing more: the structure-tensor path streams z
 * slabs (each with the path's reach of context, so bit for bit as one pass)
 * through the activation buffers.
 */
#define ST_SURROGATE_WEIGHTS 111783
int st_surrogate_infer(const void* volume, int dtype, const uint8_t* mask,
                       int64_t nz, int64_t ny, int64_t nx,
                       const void* weights, size_t weights_bytes, double min_confidence,
                       double sigma, double rho, double truncate,
                       const double* axis_center, const double* axis_direction,
                       float* e3, float* fa, float* ha, float* ia, float* confidence,
                       void* stream);

/* What the calling thread's last st_surrogate_infer did for its fallback:
 * mode 0 (none: no fallback asked or no tile flagged), 1 (flagged tiles of
 * edge *tile_edge: *tiles crops of *voxels voxels in all) or 2 (the whole
 * volume: *voxels = N).  Any output pointer may be NULL. */
int st_surrogate_fallback_info(int* mode, int* tile_edge, int64_t* tiles, int64_t* voxels);

/*
 * Training of the surrogate's weights on the matrix cores.  The objective, per
 * voxel with loss weight w (0 or 1), u = h[0:3] / |h[0:3]|, label direction t
 * (unit) and label FA f:
 *   l_dir = 1 - (u . t)^2;  l_fa = (sigmoid(h[3]) - f)^2;
 *   l_conf = softplus(h[4]) - c h[4], c = [angle(u, t) < 2 degrees] (a target);
 *   L = sum w (l_dir + l_fa + conf_weight l_conf) / sum w  (conf_weight >= 0,
 *   finite; 0.1 is the trainer's default).
 * Training stores every activation in bf16 (the fifth layer's too, which
 * inference keeps in float32) and every gradient at a pre-activation in bf16;
 * weights enter both passes rounded to bf16 and are kept in float32.
 *
 * st_surrogate_grad: L and its gradient for a stack of npatch patches of
 * patch^3 voxels (1 <= patch <= 32), each its own volume with clamped faces.
 *  patches         device [npatch * patch][patch][patch] of dtype
 *  target_e3       device float[3][N] (N = npatch * patch^3), label directions (unit)
 *  target_fa       device float[N];  weight: device uint8[N], 1 where the loss applies.
 *                  Loss voxels must lie at least 5 voxels inside their patch
 *                  (the network's receptive radius), so no face enters the gradient.
 *  params          device float[ST_SURROGATE_WEIGHTS] (the weights blob)
 *  grad            device float[ST_SURROGATE_WEIGHTS]: dL/dparams (0 for in_scale, in_offset)
 *  stats           device float[8]: mean l_dir, l_fa, l_conf, L, sum w, weighted
 *                  voxels within 2 degrees, mean angle (degrees), sum w
 *  workspace       st_surrogate_grad_workspace_bytes(npatch, patch) device bytes, or
 *                  NULL with workspace_bytes 0 (then allocated stream-ordered)
 * st_surrogate_adam: one Adam step (bias-corrected, step >= 1) on every weight
 * but in_scale and in_offset: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * params -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  All
 * arrays device float[ST_SURROGATE_WEIGHTS].
 */
size_t st_surrogate_grad_workspace_bytes(int64_t npatch, int64_t patch);
int st_surrogate_grad(const void* patches, int dtype, int64_t npatch, int64_t patch,
                      const float* target_e3, const float* target_fa, const uint8_t* weight,
                      const float* params, double conf_weight, float* grad, float* stats,
                      void* workspace, size_t workspace_bytes, void* stream);
int st_surrogate_adam(float* params, const float* grad, float* adam_m, float* adam_v, int64_t step,
                      double lr, double beta1, double beta2, double eps, void* stream);

/*
 * Chunk batches (the paper's chunk-based processing with padding, Implementation
 * section): many independent volumes -- typically halo-padded crops of one
 * large scan -- run through the st_compute path as one unit of work.
 *
 * st_batch_create validates every chunk (as st_compute would), assigns the
 * chunks to `lanes` concurrent chains (largest first, each to the chain with
 * the least work so far), gives every chain its own workspace slot and
 * captures the whole batch into a HIP graph.  st_batch_launch replays it on
 * `stream`; replays recompute every output.  st_batch_tune times candidate
 * launch configurations on the real chunks and keeps the fastest: per chunk
 * the tile shapes (rows of a gradient tile, lanes of a final-pass row
 * segment), then for the whole batch the chain count, how far each pass
 * splits its filtered axis, and graph replay vs direct multi-stream enqueue.
 * Results do not depend on the configuration (bitwise).  The chunk buffers
 * must stay valid, and must not be written, while a launch may run; chunks may
 * not share output buffers.
 */
typedef struct st_chunk {
  const void* volume;     /* device [nz][ny][nx] of dtype */
  int dtype;              /* ST_DTYPE_U16 or ST_DTYPE_F32 */
  const uint8_t* mask;    /* device [nz][ny][nx] or NULL */
  int64_t nz, ny, nx;
  double rho;             /* integration scale of this chunk */
  double origin[3];       /* (z, y, x) of volume[0][0][0] in the axis' coordinates */
  float* e3;              /* outputs as in st_compute, device or NULL */
  float* evals;
  float* fa;
  float* ha;
  float* ia;
  uint8_t* flags;
} st_chunk;

typedef struct st_batch st_batch;  /* opaque */

/* Largest chain count of a batch. */
#define ST_BATCH_MAX_LANES 8
/* `lanes` value that selects grouped launches (see st_batch_create). */
#define ST_BATCH_GROUPED (-1)

/* Workspace bytes a batch of these chunks needs with `lanes` chains (0 or
 * ST_BATCH_GROUPED = room for ST_BATCH_MAX_LANES): one slot per chain, each
 * st_workspace_bytes of the largest chunk; 0 if a chunk's sizes are invalid. */
size_t st_batch_workspace_bytes(const st_chunk* chunks, int nchunks, int lanes);

/* Builds a batch.  chunks: HOST array of nchunks >= 1 descriptors (copied).
 * sigma, truncate: as in st_compute, shared by every chunk.  axis_center /
 * axis_direction: HOST (z, y, x) or both NULL (then ha / ia must be NULL).
 * lanes: 1..ST_BATCH_MAX_LANES concurrent chains, 0 for ST_BATCH_MAX_LANES
 * chains, or ST_BATCH_GROUPED for grouped launches: the chunks are packed into
 * rounds whose workspaces fit the batch's workspace (first-fit decreasing),
 * and each pass of a round is one kernel launch over all of the round's
 * chunks that share its radius, taps and tile shape, reading every chunk's
 * geometry from a device table (the batch allocates its small table buffer
 * even with a caller workspace); ST_ERR_UNSUPPORTED if sigma's radius needs
 * the three-pass gradient.  Grouped launches fill all of a caller workspace of
 * one slot or more (fewer bytes, more and smaller rounds; with the sum of the
 * chunks' st_workspace_bytes, rounded up to 256 each, one round); without one
 * the batch allocates ST_BATCH_MAX_LANES slots.
 * workspace: device buffer of st_batch_workspace_bytes(chunks, nchunks, lanes)
 * bytes, or NULL for the batch to allocate (and free in st_batch_destroy).
 * On success *out holds the batch (owned by the caller, release with
 * st_batch_destroy).  Synchronous: returns after the graph is built. */
int st_batch_create(const st_chunk* chunks, int nchunks, double sigma, double truncate,
                    const double* axis_center, const double* axis_direction, int lanes,
                    void* workspace, size_t workspace_bytes, st_batch** out);

/* Enqueues the whole batch on `stream`. */
int st_batch_launch(st_batch* batch, void* stream);

/* Autotuning, synchronous: waits for the batch's earlier launches, destroys
 * its graph, then times on `stream` (each candidate once untimed, then `reps`
 * times): for every chunk alone, the gradient tile rows and the final-pass
 * segment lanes compiled for its radii; for the whole batch in direct
 * enqueue, the chain count (1, 2, 4, 8 up to the workspace slots) and split
 * targets (x1/4, x1, x4 around the chain count's default), then the grouped
 * launches; finally the chosen configuration replayed from one newly
 * captured graph against direct enqueue.  Keeps the fastest (best_ms in st_batch_config).  On an error the
 * batch stays usable with direct enqueue.  reps >= 1. */
int st_batch_tune(st_batch* batch, void* stream, int reps);

/* Current configuration; any output pointer may be NULL.  lanes: chains in use;
 * use_graph: 1 if launches replay the captured graph; grad_min_blocks: the
 * gradient pass splits z until its launch holds at least 4 * grad_min_blocks
 * waves (one wave per tile row); strided_min_waves: the same target for the
 * integration passes (with more than one chain both are a quarter of a lone
 * st_compute's, since the chains fill the chip together); best_ms: the tuned
 * time per launch of the configuration st_batch_tune chose (0 before tuning). */
int st_batch_config(const st_batch* batch, int* lanes, int* use_graph, int64_t* grad_min_blocks,
                    int64_t* strided_min_waves, double* best_ms);

/* How the batch launches: grouped (1) or chains (0); the rounds of the grouped
 * mode (0 for chains); the compute kernel launches one st_batch_launch makes
 * (besides the completion record's one-thread kernels).  Any output pointer
 * may be NULL. */
int st_batch_plan(const st_batch* batch, int* grouped, int* rounds, int* kernels);

/* Completion record, for resuming an interrupted batch (the paper saves every
 * chunk's outputs as it finishes, so a run can resume by chunk).  After the
 * last pass of each chunk (grouped launches: of each round) the GPU writes the
 * batch's launch count into a pinned host word of that chunk.  This call reads
 * those words without waiting for the GPU: done[c] = 1 when chunk c's outputs
 * of the batch's latest launch are complete, else 0 (all 0 before the first
 * launch); *launches = launches so far (st_batch_launch calls and the timing
 * runs of st_batch_tune, which leave every chunk complete).  It may be called while a
 * launch runs, or after one failed: a new batch of the chunks with done[c] = 0
 * finishes the work.  done: HOST array of nchunks (the batch's chunk count)
 * or NULL; launches may be NULL. */
int st_batch_progress(const st_batch* batch, uint8_t* done, int nchunks, int64_t* launches);

/* Tile shapes of chunk `chunk` (0 <= chunk < nchunks): the rows of a gradient
 * tile and the lanes of a final-pass row segment; 0 means the library's
 * default for the chunk's radii and width (what an untuned batch uses).
 * Either output pointer may be NULL. */
int st_batch_tiles(const st_batch* batch, int chunk, int* grad_rows, int* final_lanes);

/* Releases the batch (waits for its work to finish). */
int st_batch_destroy(st_batch* batch);

/*
 * Kernel timing for measurement tools.  While enabled, every kernel launched
 * by st_compute / st_angles is bracketed by HIP events recorded on the same
 * stream.  st_profile_read() waits for those events (host-side), adds their
 * elapsed times into per-kernel totals and returns the number of distinct
 * kernels seen; entry i's name, total milliseconds and launch count are
 * written to the optional outputs.  Not thread-safe; off by default.
 */
int st_profile_enable(int on);
int st_profile_reset(void);
int st_profile_read(int index, char* name, size_t name_len, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* ST_H_ */
