// The fused solve kernel (one workgroup per outer step) and its launcher; the
// device code and its design notes are in solve_dev.h.
#include "solve_dev.h"

namespace cabcd {
namespace {

using namespace sdev;

template <int BP, int PF, int THREADS, int MAP>
__global__ __launch_bounds__(THREADS) void solve_kernel(SolveArgs a) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
  solve_block<BP, PF, THREADS, MAP>(a, sm);
}

template <int BP, int PF, int THREADS, int MAP>
hipError_t launch_b(const SolveArgs& a, hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(solve_kernel<BP, PF, THREADS, MAP>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSolveMaxLds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((solve_kernel<BP, PF, THREADS, MAP>), dim3(1), dim3(THREADS),
                     solve_lds_bytes(a.m, a.b), st, a);
  return hipGetLastError();
}

// The one-barrier block mapping (MAP 1) whenever s BP lanes fit the workgroup,
// in the smallest workgroup that holds them (cheaper barriers on the chain).
template <int BP, int PF>
hipError_t launch_t(const SolveArgs& a, hipStream_t st) {
  const int lanes = a.s * BP;
  if constexpr (BP <= 16) {
    if (lanes <= 256) return launch_b<BP, PF, 256, 1>(a, st);
    if (lanes <= 512) return launch_b<BP, PF, 512, 1>(a, st);
  }
  if (a.m <= 512) return launch_b<BP, PF, 512, 0>(a, st);
  if constexpr (BP <= 8) {
    if (lanes <= 1024) return launch_b<BP, 2, 1024, 1>(a, st);
    return launch_b<BP, 2, 1024, 0>(a, st);
  }
  if constexpr (BP == 16) {
    if (lanes <= 1024) return launch_b<BP, 1, 1024, 1>(a, st);
    return launch_b<BP, 1, 1024, 0>(a, st);
  }
  return hipErrorInvalidValue;   // b in (16, 32] never reaches m > 512 within the LDS bound
}

}  // namespace

size_t solve_lds_bytes(int m, int b) {
  const int bp = pow2_at_least(b);
  const int s = (m + b - 1) / b;
  const int slots = std::max(kHashMin, pow2_at_least(2 * m));
  const size_t gi = std::max((size_t)s * (bp * bp + 1), sdev::hash_doubles(m, slots));
  return sizeof(double) * (gi + (size_t)bp + (size_t)s * bp);
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t st) {
  if (a.m > kSolveMaxRows || a.b > kSolveMaxB || solve_lds_bytes(a.m, a.b) > kSolveMaxLds)
    return hipErrorInvalidValue;
  switch (pow2_at_least(a.b)) {
    case 1: return launch_t<1, 8>(a, st);
    case 2: return launch_t<2, 8>(a, st);
    case 4: return launch_t<4, 8>(a, st);
    case 8: return launch_t<8, 8>(a, st);
    case 16: return launch_t<16, 4>(a, st);
    default: return launch_t<32, 1>(a, st);
  }
}

}  // namespace cabcd
