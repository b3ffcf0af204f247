// Counter-based block sampler: one thread per inner iteration (the sampling
// step of Alg. 1-4; the composition is documented with smp::sample_block).
#include "internal.h"

namespace cabcd {
namespace {

__global__ void sample_kernel(uint64_t seed, int64_t h0, int64_t count, int b,
                              int64_t range, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  smp::sample_block(seed, h0 + i, b, range, idx + i * (int64_t)b);
}

}  // namespace

hipError_t launch_sample(uint64_t seed, int64_t h0, int64_t count, int b, int64_t range,
                         int32_t* idx, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int threads = 64;
  const int64_t blocks = (count + threads - 1) / threads;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, seed, h0,
                     count, b, range, idx);
  return hipGetLastError();
}

}  // namespace cabcd
