// Completion record of a chunk batch: a launch counter in device memory, bumped
// at the start of every launch, and one pinned host word per chunk that takes
// the counter's value once the chunk's last pass has finished.  The host reads
// the words without synchronising, so the record survives an interrupted launch.
#include "st_internal.h"

namespace st {
namespace {

__global__ void k_batch_begin(uint64_t* seq) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *seq += 1;
}

__global__ __launch_bounds__(256) void k_batch_mark(const uint64_t* seq, uint64_t* progress, const int64_t* ids,
                                                    int count, int64_t one) {
  const int t = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (t >= count) return;
  const int64_t c = ids != nullptr ? ids[t] : one;
  __hip_atomic_store(progress + c, *seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

hipError_t launch_batch_begin(uint64_t* seq, hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, stream, seq);
  return hipGetLastError();
}

hipError_t launch_batch_mark(const uint64_t* seq, uint64_t* progress, const int64_t* ids, int count, int64_t one,
                             hipStream_t stream) {
  if (count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_batch_mark, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, stream, seq,
                     progress, ids, count, one);
  return hipGetLastError();
}

}  // namespace st
