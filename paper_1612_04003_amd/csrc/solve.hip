// The s inner b x b solves of one outer step, fused into one workgroup.
//
// Primal (Alg. 2, eq. recur): with G the s-step Gram and S_jt = I_j^T I_t,
//   dw_j = Gamma_j^{-1} ( c_j - sum_{t<j} (G_jt + lambda S_jt) dw_t ),
//   c = -lambda w_I - (1/n) Y (z - y),   Gamma_j = G_jj.
// Dual (Alg. 4): writing Theta_j = G'_jj and using (1/(lambda n)) Y_j^T Y_t =
// n G'_jt, the printed recurrence becomes
//   da_j = Theta_j^{-1} ( c_j - sum_{t<j} (G'_jt + (1/n) S_jt) da_t ),
//   c = (1/n) (Y^T w - a_I - y_I).
// Both are one block forward substitution with the lower block triangle of the
// overlap-augmented Gram Gov = scale Y Y^T + shift [idx_p == idx_q], which the
// Gram reduction writes (its diagonal blocks are exactly Gamma_j / Theta_j
// because indices within a block are distinct).
//
// Phases (one workgroup, thread p owns row p of the outer step):
//  1. c, and the s diagonal blocks copied to LDS;
//  2. all s blocks factorised in parallel (unpivoted Cholesky, row-parallel
//     right-looking) and inverted (L^{-1}, then L^{-T} L^{-1}); a pivot <= 0 or
//     NaN raises the device status;
//  3. the dependent chain over j: delta_j = Gamma_j^{-1} rhs_j, then every later
//     row subtracts its Gov row segment times delta_j.  Row segments of the
//     next PF blocks are prefetched into registers so the chain waits on LDS
//     and barriers only;
//  4. delta written out, and x[idx] += delta by the first occurrence of each
//     coordinate, adding the duplicates in block order (single writer).
#include "internal.h"

#include <algorithm>

namespace cabcd {
namespace {

constexpr int kSolveThreads = 256;

template <int BMAX, int PF>
__global__ __launch_bounds__(kSolveThreads) void solve_kernel(SolveArgs a) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
  const int m = a.m, b = a.b, s = a.s;
  double* D = sm;                   // s blocks b x b: Cholesky, then the inverse
  double* Li = D + m * b;           // s blocks b x b: L^{-1}
  double* R = Li + m * b;           // b: rhs of the current block
  double* Dl = R + BMAX;            // m: delta
  int* Ix = reinterpret_cast<int*>(Dl + m);   // m: indices

  const int p = threadIdx.x;
  const bool active = p < m;
  const int j_of = active ? p / b : -1;   // block of this row (-1: no row)
  const int u = active ? p - j_of * b : 0;
  double* Dj = D + (active ? j_of : 0) * b * b;
  double* Lj = Li + (active ? j_of : 0) * b * b;

  // ---- phase 1
  double rhs = 0.0;
  int ip = 0;
  if (active) {
    ip = a.idx[p];
    Ix[p] = ip;
    const double yu = a.Yu[p];
    const double xi = a.x[ip];
    rhs = a.mode == 0 ? (-a.lambda * xi - yu / a.n) : ((yu - xi - a.y[ip]) / a.n);
    const double* g = a.G + (int64_t)p * m + j_of * b;
    for (int v = 0; v <= u; ++v) Dj[u * b + v] = g[v];
  }

  // Prefetch ring of Gov row segments for the first PF blocks.
  double ring[PF][BMAX];
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    if (q < j_of) {
      const double* g = a.G + (int64_t)p * m + q * b;
#pragma unroll
      for (int v = 0; v < BMAX; ++v) ring[q][v] = v < b ? g[v] : 0.0;
    }
  }
  __syncthreads();

  // ---- phase 2: Cholesky of every diagonal block, row u of block j per thread
  // Every row of the block reads the pivot before the diagonal is overwritten.
  bool bad = false;
  for (int k = 0; k < b; ++k) {
    double lkk = 1.0;
    if (active && u >= k) {
      const double piv = Dj[k * b + k];
      bad |= !(piv > 0.0);
      lkk = sqrt(piv);
      if (u > k) Dj[u * b + k] /= lkk;
    }
    __syncthreads();
    if (active && u == k) Dj[k * b + k] = lkk;
    if (active && u > k) {
      const double luk = Dj[u * b + k];
      for (int v = k + 1; v <= u; ++v) Dj[u * b + v] -= luk * Dj[v * b + k];
    }
    __syncthreads();
  }
  // column u of L^{-1}: solve L x = e_u by forward substitution
  if (active) {
    for (int v = 0; v < u; ++v) Lj[v * b + u] = 0.0;
    Lj[u * b + u] = 1.0 / Dj[u * b + u];
    for (int v = u + 1; v < b; ++v) {
      double t = 0.0;
      for (int w = u; w < v; ++w) t += Dj[v * b + w] * Lj[w * b + u];
      Lj[v * b + u] = -t / Dj[v * b + v];
    }
  }
  __syncthreads();
  // row u of Gamma^{-1} = L^{-T} L^{-1}
  if (active) {
    for (int v = 0; v < b; ++v) {
      double t = 0.0;
      for (int w = std::max(u, v); w < b; ++w) t += Lj[w * b + u] * Lj[w * b + v];
      Dj[u * b + v] = t;
    }
  }
  if (bad) *a.status = DEV_NOTSPD;
  __syncthreads();

  // ---- phase 3: the dependent chain over the s blocks
  for (int j0 = 0; j0 < s; j0 += PF) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int j = j0 + q;
      if (j < s) {
        if (j_of == j) R[u] = rhs;
        __syncthreads();
        if (p < b) {
          const double* Gi = D + j * b * b + p * b;
          double t = 0.0;
          for (int v = 0; v < b; ++v) t += Gi[v] * R[v];
          Dl[j * b + p] = t;
        }
        __syncthreads();
        if (j_of > j) {
          const double* dj = Dl + j * b;
#pragma unroll
          for (int v = 0; v < BMAX; ++v)
            if (v < b) rhs -= ring[q][v] * dj[v];
          const int jn = j + PF;
          if (jn < j_of) {
            const double* g = a.G + (int64_t)p * m + jn * b;
#pragma unroll
            for (int v = 0; v < BMAX; ++v) ring[q][v] = v < b ? g[v] : 0.0;
          }
        }
      }
    }
  }

  // ---- phase 4: outputs
  if (active) {
    const double dp = Dl[p];
    a.delta[p] = dp;
    if (!isfinite(dp)) *a.status = DEV_NONFINITE;
    bool first = true;
    for (int q = 0; q < p; ++q) first &= (Ix[q] != ip);
    if (first) {
      double acc = a.x[ip];
      for (int q = p; q < m; ++q)
        if (Ix[q] == ip) acc += Dl[q];
      a.x[ip] = acc;
    }
  }
}

template <int BMAX, int PF>
hipError_t launch_b(const SolveArgs& a, hipStream_t st) {
  const size_t bytes = sizeof(double) * (2 * (size_t)a.m * a.b + BMAX + a.m) +
                       sizeof(int) * (size_t)a.m;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(solve_kernel<BMAX, PF>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((solve_kernel<BMAX, PF>), dim3(1), dim3(kSolveThreads), bytes, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_solve(const SolveArgs& a, hipStream_t st) {
  if (a.m > kSolveThreads || a.b > 32) return hipErrorInvalidValue;
  if (a.b <= 8) return launch_b<8, 4>(a, st);
  if (a.b <= 16) return launch_b<16, 4>(a, st);
  return launch_b<32, 2>(a, st);
}

}  // namespace cabcd
