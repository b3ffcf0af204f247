// The fused solve kernel (one workgroup per outer step) and its launcher; the
// device code and its design notes are in solve_dev.h.
#include "solve_dev.h"

namespace cabcd {
namespace {

using namespace sdev;

template <int BP, int PF, int THREADS, int MAP, bool PRE>
__global__ __launch_bounds__(THREADS) void solve_kernel(SolveArgs a) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
  solve_block<BP, PF, THREADS, MAP, PRE>(a, sm);
}

template <int BP, int PF, int THREADS, int MAP, bool PRE>
hipError_t launch_k(const SolveArgs& a, hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(solve_kernel<BP, PF, THREADS, MAP, PRE>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSolveMaxLds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((solve_kernel<BP, PF, THREADS, MAP, PRE>), dim3(1), dim3(THREADS),
                     solve_lds_bytes(a.m, a.b), st, a);
  return hipGetLastError();
}

// Diagonal blocks inverted ahead (a.pre_inverted) are taken by the one-barrier
// solves (s BP <= 512 lanes) only, the ones the drivers ask it for.
template <int BP, int PF, int THREADS, int MAP>
hipError_t launch_b(const SolveArgs& a, hipStream_t st) {
  if (!a.pre_inverted) return launch_k<BP, PF, THREADS, MAP, false>(a, st);
  if constexpr (THREADS <= 512 && MAP == 1) return launch_k<BP, PF, THREADS, MAP, true>(a, st);
  return hipErrorInvalidValue;
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

// The diagonal blocks of nsteps Grams inverted ahead of their solves, with the
// solve's own Gauss-Jordan code and padding: BP <= 8 one block per lane,
// BP = 16 four blocks per wave (one row per lane).
template <int BP>
__global__ __launch_bounds__(64) void invert_diag_kernel(double* G, int m, int b, int s,
                                                          int* status) {
  G += (int64_t)blockIdx.y * m * m;
  const int lane = threadIdx.x;
  bool bad = false;
  auto at = [&](int j, int u, int v) -> double& {
    return G[(int64_t)(j * b + u) * m + j * b + v];
  };
  if constexpr (BP <= 8) {
    const int j = blockIdx.x * 64 + lane;
    if (j < s) {
      double e[BP][BP];
#pragma unroll
      for (int u = 0; u < BP; ++u)
#pragma unroll
        for (int v = 0; v < BP; ++v) e[u][v] = u < b && v < b ? at(j, u, v) : (u == v ? 1.0 : 0.0);
      gj_lane<BP>(e, bad);
#pragma unroll
      for (int u = 0; u < BP; ++u)
#pragma unroll
        for (int v = 0; v < BP; ++v)
          if (u < b && v < b) at(j, u, v) = e[u][v];
    }
  } else if constexpr (BP == 16) {
    // every lane takes part in the row broadcasts; groups past the last
    // block invert the identity
    const int j = blockIdx.x * 4 + (lane >> 4);
    const int u = lane & 15;
    const bool live = j < s && u < b;
    double e[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) e[v] = live && v < b ? at(j, u, v) : (u == v ? 1.0 : 0.0);
    gj_rows16<0>(e, u, bad);
    if (live) {
#pragma unroll
      for (int v = 0; v < 16; ++v)
        if (v < b) at(j, u, v) = e[v];
    }
  } else {
    static_assert(BP <= 16, "blocks up to 16 x 16");
  }
  if (bad) raise_status(status, DEV_NOTSPD);
}

template <int BP>
hipError_t launch_inv(double* G, int nsteps, int m, int b, int s, int* status, hipStream_t st) {
  const int per = BP <= 8 ? 64 : 4;   // blocks per workgroup
  hipLaunchKernelGGL(invert_diag_kernel<BP>, dim3((unsigned)((s + per - 1) / per), (unsigned)nsteps),
                     dim3(64), 0, st, G, m, b, s, status);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_invert_diag(double* G, int nsteps, int m, int b, int* status, hipStream_t st) {
  if (nsteps < 1 || nsteps > 65535 || b < 1 || b > 16 || m % b != 0)
    return hipErrorInvalidValue;
  const int s = m / b;
  switch (pow2_at_least(b)) {
    case 1: return launch_inv<1>(G, nsteps, m, b, s, status, st);
    case 2: return launch_inv<2>(G, nsteps, m, b, s, status, st);
    case 4: return launch_inv<4>(G, nsteps, m, b, s, status, st);
    case 8: return launch_inv<8>(G, nsteps, m, b, s, status, st);
    default: return launch_inv<16>(G, nsteps, m, b, s, status, st);
  }
}

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
