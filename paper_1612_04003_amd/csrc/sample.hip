// Counter-based block sampler: b distinct coordinates per inner iteration,
// uniform without replacement (Section 1 footnote; Alg. 1-4 sampling step),
// keyed by (seed, h) only so that every consumer of the same seed draws the
// same blocks (Section 3.1, after eq. recur).
//
// Composition (integer-only, so any two implementations agree bit for bit):
//   SplitMix64 output t of a stream seeded with x: mix64(x + GAMMA*(t+1))
//     (Steele, Lea & Flood, OOPSLA 2014; finaliser constants of that paper)
//   key(h) = output h of the stream seeded with `seed`
//   word t = upper 32 bits of output t of the stream seeded with key(h)
//   bounded(range): Lemire's multiply-shift with rejection (TOMACS 2019)
//   block: Floyd's algorithm (Bentley & Floyd, CACM 1987), insertion order.
// One thread per iteration; the already-drawn list lives in the output row.
#include "internal.h"

namespace cabcd {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t stream_out(uint64_t seed, uint64_t t) {
  return mix64(seed + kGamma * (t + 1));
}

__global__ void sample_kernel(uint64_t seed, int64_t h0, int64_t count, int b,
                              int64_t range, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t key = stream_out(seed, (uint64_t)(h0 + i));
  uint64_t t = 0;
  int32_t* out = idx + i * (int64_t)b;
  int filled = 0;
  for (int64_t j = range - b; j < range; ++j) {
    const uint64_t m = (uint64_t)(j + 1);          // draw uniformly from [0, j]
    uint64_t x = stream_out(key, t++) >> 32;
    uint64_t prod = x * m;
    uint32_t low = (uint32_t)prod;
    if (low < m) {
      const uint32_t thr = (uint32_t)((0x100000000ull - m) % m);
      while (low < thr) {
        x = stream_out(key, t++) >> 32;
        prod = x * m;
        low = (uint32_t)prod;
      }
    }
    const int32_t v = (int32_t)(prod >> 32);
    bool seen = false;
    for (int q = 0; q < filled; ++q) seen |= (out[q] == v);
    out[filled++] = seen ? (int32_t)j : v;
  }
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
