// Training kernels of the learned orientation surrogate: the loss and the head's
// backward pass, the weight gradients of the five convolutions (layers 2..5 on
// the bf16 matrix cores, layer 1 on the vector ALUs), deterministic reductions
// of per-block partial sums, and Adam on the float32 weights.  The forward
// pass and the backward data pass reuse the inference convolution kernel.
//
// Training runs on a stack of P^3 patches, P <= 32, laid out as one volume of
// npatch * P planes of P x P voxels; a row of the stack (fixed z, y) holds the
// P voxels of one MFMA K step.  Activations x_l and gradients g_l (at the
// pre-activation of layer l) are channel-last bf16, [N][32].
#include "st_device.h"
#include "st_surrogate.h"

namespace st {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int C = kSgChannels;
constexpr int WX = kSgTrainMaxX;   // voxels of a staged row
constexpr float kConfDeg = 2.0f;   // confidence target: within this angle of the label

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// Backward weights of layers 2..5: [layer][tap'][a][b] = W[b][a][26 - tap'], so
// that the forward kernel, which reads its weights as [tap][out][in], computes
// dx[a](q) = sum_{b, tap} W[b][a][tap] g[b](q - off(tap)).
__global__ void k_sg_pack_bwd(const float* blob, __bf16* w25t) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = 27 * C * C;
  if (i >= 4 * per) return;
  const int layer = static_cast<int>(i / per);
  const int64_t r = i % per;
  const int tp = static_cast<int>(r / (C * C)), a = static_cast<int>((r / C) % C), b = static_cast<int>(r % C);
  w25t[i] = static_cast<__bf16>(blob[kSgOffW2 + layer * kSgLayerStride + (b * C + a) * 27 + (26 - tp)]);
}

// The head and the loss on every weighted voxel: h = bh + Wh x5, direction term
// 1 - (u.t)^2 with u = h[0:3] / |h[0:3]|, FA term (sigmoid(h3) - f)^2, confidence
// term softplus(h4) - c h4 with c = [angle(u, t) < 2 deg].  dL/dh (unnormalised)
// goes back through the head into g5; the head's weight gradient and six loss
// sums are reduced over the block's voxels (fixed order) into per-block partials.
__global__ __launch_bounds__(256) void k_sg_head_train(const SgHeadParams p) {
  __shared__ float xs[256][C + 1];
  __shared__ float ds[256][11];
  const int tid = threadIdx.x;
  float acc = 0.f;  // thread j < kSgHeadSums accumulates sum j
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * 256; base < p.n;
       base += static_cast<int64_t>(gridDim.x) * 256) {  // block-uniform trip count
    const int64_t v = base + tid;
    float x[C];
    float d[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) d[k] = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = 0.f;
    if (v < p.n) {
      bf16x8 g8[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) g8[q] = bf16x8{};
      if (p.weight[v] != 0) {
        const bf16x8* src = reinterpret_cast<const bf16x8*>(p.x5 + v * C);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bf16x8 t8 = src[q];
#pragma unroll
          for (int i = 0; i < 8; ++i) x[8 * q + i] = static_cast<float>(t8[i]);
        }
        float h[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          float s = p.head_b[q];
#pragma unroll
          for (int c = 0; c < C; ++c) s = fmaf(p.head_w[q * C + c], x[c], s);
          h[q] = s;
        }
        const float tz = p.target[v], ty = p.target[p.n + v], tx = p.target[2 * p.n + v];
        const float nrm = sqrtf(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
        const float inv = nrm > 0.f ? 1.f / nrm : 1.f;
        const float uz = h[0] * inv, uy = h[1] * inv, ux = h[2] * inv;
        const float dot = uz * tz + uy * ty + ux * tx;
        const float l_dir = 1.f - dot * dot;
        d[0] = -2.f * dot * (tz - dot * uz) * inv;
        d[1] = -2.f * dot * (ty - dot * uy) * inv;
        d[2] = -2.f * dot * (tx - dot * ux) * inv;
        const float s3 = 1.f / (1.f + expf(-h[3]));
        const float e = s3 - p.target_fa[v];
        d[3] = 2.f * e * s3 * (1.f - s3);
        const float cz = uy * tx - ux * ty, cy = ux * tz - uz * tx, cx = uz * ty - uy * tz;
        const float ang = atan2f(sqrtf(cz * cz + cy * cy + cx * cx), fabsf(dot)) * 57.29577951308232f;
        const float c = ang < kConfDeg ? 1.f : 0.f;
        const float s4 = 1.f / (1.f + expf(-h[4]));
        d[4] = p.w_conf * (s4 - c);
        d[5] = l_dir;
        d[6] = e * e;
        d[7] = fmaxf(h[4], 0.f) + log1pf(expf(-fabsf(h[4]))) - c * h[4];
        d[8] = 1.f;
        d[9] = c;
        d[10] = ang;
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          float gc = 0.f;
#pragma unroll
          for (int q = 0; q < 5; ++q) gc = fmaf(p.head_w[q * C + cc], d[q], gc);
          g8[cc / 8][cc % 8] = static_cast<__bf16>(x[cc] > 0.f ? gc : 0.f);
        }
      }
      bf16x8* dst = reinterpret_cast<bf16x8*>(p.g5 + v * C);
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[q] = g8[q];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) xs[tid][c] = x[c];
#pragma unroll
    for (int k = 0; k < 11; ++k) ds[tid][k] = d[k];
    __syncthreads();
    if (tid < 5 * C) {
      const int q = tid / C, c = tid % C;
      for (int i = 0; i < 256; ++i) acc = fmaf(ds[i][q], xs[i][c], acc);
    } else if (tid < kSgHeadSums) {
      const int k = tid - 5 * C;  // 0..4: dh (bias), 5..10: loss sums
      for (int i = 0; i < 256; ++i) acc += ds[i][k];
    }
    __syncthreads();
  }
  if (tid < kSgHeadSums) p.partial[static_cast<int64_t>(blockIdx.x) * kSgHeadSums + tid] = acc;
}

// Weight gradient of a 32 -> 32 layer: dW[co][ci][tap] = sum_p g(p)[co] x(p + off(tap))[ci]
// and db[co] = sum_p g(p)[co], for the rows of one block.  Per row, g is staged
// channel-major ([ch][x]) and the nine neighbouring rows of x in three copies
// shifted by dx = -1, 0, 1 (indices clamped at every face), so that every
// operand of v_mfma_f32_16x16x32_bf16 is one aligned 16-byte LDS read: A[co][k]
// = g at voxel k, B[k][ci] = x at voxel k + dx, K = the 32 voxels of the row
// (voxels past nx are zero).  Wave w accumulates taps w, w + 8, w + 16 (and
// w + 24 for w < 3), four 16 x 16 tiles each.
__global__ __launch_bounds__(512) void k_sg_wgrad(const SgWgradParams p) {
  __shared__ __attribute__((aligned(16))) __bf16 gT[C * WX];
  __shared__ __attribute__((aligned(16))) __bf16 xs[9 * 3 * C * WX];
  __shared__ float dbs[WX][C];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t nz = p.nz, ny = p.ny;
  const int nx = static_cast<int>(p.nx);
  const int64_t nrows = nz * ny;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * p.rows_per_block;
  const int64_t r1 = r0 + p.rows_per_block < nrows ? r0 + p.rows_per_block : nrows;
  const int ntap = wave < 3 ? 4 : 3;
  f32x4 acc[4][2][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n) acc[i][m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int sv = tid >> 4, sc = 2 * (tid & 15);  // g staging: voxel, channel pair
  float db0 = 0.f, db1 = 0.f;
  for (int64_t r = r0; r < r1; ++r) {  // block-uniform trip count
    const int64_t z = r / ny, y = r % ny;
    {
      __bf16 a = static_cast<__bf16>(0.f), b = static_cast<__bf16>(0.f);
      if (sv < nx) {
        const __bf16* src = p.g + (r * nx + sv) * C + sc;
        a = src[0];
        b = src[1];
      }
      gT[sc * WX + sv] = a;
      gT[(sc + 1) * WX + sv] = b;
      db0 += static_cast<float>(a);
      db1 += static_cast<float>(b);
    }
    for (int k = tid; k < 9 * 3 * WX * 16; k += 512) {
      const int cp = k & 15;
      int q = k >> 4;
      const int i = q % WX;
      q /= WX;
      const int s = q % 3, rr = q / 3;
      __bf16 a = static_cast<__bf16>(0.f), b = static_cast<__bf16>(0.f);
      if (i < nx) {
        const int64_t zz = clampi(z + rr / 3 - 1, nz), yy = clampi(y + rr % 3 - 1, ny);
        const int64_t xx = clampi(i + s - 1, nx);
        const __bf16* src = p.x + ((zz * ny + yy) * nx + xx) * C + 2 * cp;
        a = src[0];
        b = src[1];
      }
      xs[((rr * 3 + s) * C + 2 * cp) * WX + i] = a;
      xs[((rr * 3 + s) * C + 2 * cp + 1) * WX + i] = b;
    }
    __syncthreads();
    bf16x8 A[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) A[m] = *reinterpret_cast<const bf16x8*>(gT + (16 * m + li) * WX + 8 * lk);
#pragma unroll
    for (int ti = 0; ti < 4; ++ti) {
      if (ti < ntap) {  // wave-uniform
        const int t = wave + 8 * ti;
        const int rr = (t / 9) * 3 + (t / 3) % 3, s = t % 3;
        bf16x8 B[2];
#pragma unroll
        for (int n = 0; n < 2; ++n)
          B[n] = *reinterpret_cast<const bf16x8*>(xs + ((rr * 3 + s) * C + 16 * n + li) * WX + 8 * lk);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 2; ++n)
            acc[ti][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[m], B[n], acc[ti][m][n], 0, 0, 0);
      }
    }
    __syncthreads();  // the next row's staging overwrites gT and xs
  }
  float* out = p.partial + static_cast<int64_t>(blockIdx.x) * (27 * C * C + C);
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) {
    if (ti < ntap) {
      const int t = wave + 8 * ti;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int co = 16 * m + 4 * lk + q, ci = 16 * n + li;
            out[(t * C + co) * C + ci] = acc[ti][m][n][q];
          }
    }
  }
  dbs[sv][sc] = db0;
  dbs[sv][sc + 1] = db1;
  __syncthreads();
  if (tid < C) {
    float s = 0.f;
    for (int v = 0; v < WX; ++v) s += dbs[v][tid];
    out[27 * C * C + tid] = s;
  }
}

// Weight gradient of layer 1 (one input channel, on the vector ALUs):
// dW1[co][tap] = sum_p g1(p)[co] x0(p + off(tap)), db1[co] = sum_p g1(p)[co], with
// x0 = bf16(v * scale + offset) formed exactly as the first convolution forms it.
template <typename Tin>
__global__ __launch_bounds__(256) void k_sg_wgrad1(const SgWgradParams p) {
  __shared__ float gs[WX][C + 1];
  __shared__ float x0s[9][WX + 2];
  const int tid = threadIdx.x;
  const int64_t nz = p.nz, ny = p.ny;
  const int nx = static_cast<int>(p.nx);
  const int64_t nrows = nz * ny;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * p.rows_per_block;
  const int64_t r1 = r0 + p.rows_per_block < nrows ? r0 + p.rows_per_block : nrows;
  const double scale = static_cast<double>(p.scale_offset[0]), offset = static_cast<double>(p.scale_offset[1]);
  const Tin* vol = static_cast<const Tin*>(p.vol);
  constexpr int NJ = C * 27 + C;  // 864 weights, 32 biases
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int64_t r = r0; r < r1; ++r) {  // block-uniform trip count
    const int64_t z = r / ny, y = r % ny;
    for (int k = tid; k < WX * C; k += 256) {
      const int v = k / C, c = k % C;
      gs[v][c] = v < nx ? static_cast<float>(p.g[(r * nx + v) * C + c]) : 0.f;
    }
    for (int k = tid; k < 9 * (WX + 2); k += 256) {
      const int rr = k / (WX + 2), i = k % (WX + 2);
      const int64_t zz = clampi(z + rr / 3 - 1, nz), yy = clampi(y + rr % 3 - 1, ny);
      const int64_t xx = clampi(i - 1, nx);
      const float v = static_cast<float>(vol[(zz * ny + yy) * nx + xx]);
      x0s[rr][i] = static_cast<float>(static_cast<__bf16>(static_cast<float>(fma(static_cast<double>(v), scale, offset))));
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = tid + 256 * q;
      if (j < C * 27) {
        const int co = j / 27, t = j % 27;
        const int rr = (t / 9) * 3 + (t / 3) % 3, dx = t % 3;  // dx + 1
        float s = 0.f;
        for (int v = 0; v < nx; ++v) s = fmaf(gs[v][co], x0s[rr][v + dx], s);
        acc[q] += s;
      } else if (j < NJ) {
        const int co = j - C * 27;
        float s = 0.f;
        for (int v = 0; v < nx; ++v) s += gs[v][co];
        acc[q] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = tid + 256 * q;
    if (j < NJ) p.partial[static_cast<int64_t>(blockIdx.x) * NJ + j] = acc[q];
  }
}

__global__ void k_sg_reduce(const float* partial, int blocks, int len, int mode, float* out) {
  const int j = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= len) return;
  float s = 0.f;
  for (int b = 0; b < blocks; ++b) s += partial[static_cast<int64_t>(b) * len + j];
  int dst = j;
  if (mode == 1) {
    constexpr int NW = 27 * C * C;
    if (j < NW) {
      const int t = j / (C * C), co = (j / C) % C, ci = j % C;
      dst = (co * C + ci) * 27 + t;
    }
  }
  out[dst] = s;
}

// raw: the six loss sums (dir, fa, conf, weights, within, angle).
__global__ void k_sg_finish(float* grad, int64_t n, const float* raw) {
  const float wsum = raw[3];
  const float inv = wsum > 0.f ? 1.f / wsum : 0.f;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    grad[i] = i < 2 ? 0.f : grad[i] * inv;
}

__global__ void k_sg_stats(const float* raw, float w_conf, float* stats) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const float wsum = raw[3];
  const float inv = wsum > 0.f ? 1.f / wsum : 0.f;
  const float dir = raw[0] * inv, fa = raw[1] * inv, conf = raw[2] * inv;
  stats[0] = dir;
  stats[1] = fa;
  stats[2] = conf;
  stats[3] = dir + fa + w_conf * conf;
  stats[4] = wsum;
  stats[5] = raw[4];
  stats[6] = raw[5] * inv;
  stats[7] = wsum;
}

__global__ void k_sg_adam(float* w, const float* g, float* m, float* v, int64_t n, int64_t frozen, float lr,
                          float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < frozen || i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

hipError_t launch_sg_pack_bwd(const float* blob, __bf16* w25t, hipStream_t stream) {
  const int64_t n = 4 * 27 * C * C;
  hipLaunchKernelGGL(k_sg_pack_bwd, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, blob, w25t);
  return hipGetLastError();
}

hipError_t launch_sg_head_train(const SgHeadParams& p, int blocks, hipStream_t stream) {
  hipLaunchKernelGGL(k_sg_head_train, dim3(blocks), dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_sg_wgrad(const SgWgradParams& p, int blocks, hipStream_t stream) {
  if (p.nx < 1 || p.nx > WX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sg_wgrad, dim3(blocks), dim3(512), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_sg_wgrad1(int dtype, const SgWgradParams& p, int blocks, hipStream_t stream) {
  if (p.nx < 1 || p.nx > WX) return hipErrorInvalidValue;
  if (dtype == ST_DTYPE_U16)
    hipLaunchKernelGGL(k_sg_wgrad1<uint16_t>, dim3(blocks), dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL(k_sg_wgrad1<float>, dim3(blocks), dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_sg_reduce(const float* partial, int blocks, int len, int mode, float* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_sg_reduce, dim3(static_cast<unsigned>((len + 255) / 256)), dim3(256), 0, stream, partial,
                     blocks, len, mode, out);
  return hipGetLastError();
}

hipError_t launch_sg_finish(float* grad, int64_t n, const float* raw, float w_conf, float* stats, hipStream_t stream) {
  hipLaunchKernelGGL(k_sg_finish, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, grad, n, raw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sg_stats, dim3(1), dim3(64), 0, stream, raw, w_conf, stats);
  return hipGetLastError();
}

hipError_t launch_sg_adam(float* params, const float* grad, float* m, float* v, int64_t n, int64_t frozen,
                          int64_t step, float lr, float beta1, float beta2, float eps, hipStream_t stream) {
  const float c1 = 1.f - powf(beta1, static_cast<float>(step)), c2 = 1.f - powf(beta2, static_cast<float>(step));
  hipLaunchKernelGGL(k_sg_adam, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, params, grad, m,
                     v, n, frozen, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace st
