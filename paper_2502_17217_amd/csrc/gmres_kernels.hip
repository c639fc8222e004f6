// Device side of the Arnoldi bookkeeping of GMRES (Section 3.2): the small
// per-segment Hessenberg least-squares problem lives in device memory and is
// updated by one tiny kernel per Arnoldi step, so that a run of steps can be
// enqueued (or replayed from a captured HIP graph) without the host reading
// anything in between.
//
// Per segment s (columns of H are stored contiguously, H[s][j][0..mr]):
//   after the two CGS passes, column j is h_i = h[s][i] + h2[s][i] (i <= j)
//   and h_{j+1} = |w|; the earlier Givens rotations are applied, a new one
//   annihilates h_{j+1}, and g (the rotated right-hand side beta e_1) gives
//   the residual estimate |g_{j+1}|.  The segment stops when that estimate
//   reaches its target, on happy breakdown (h_{j+1} <= 1e-14 |w before
//   orthogonalisation|), on NaN, or at the iteration limit.
#include "gmres_dev.h"
#include "gmres_step_dev.h"

namespace jfnk {

namespace {

constexpr int kB = 256;

__global__ __launch_bounds__(kB) void k_cycle_init(GmresDev G, int S, const double* __restrict__ stage) {
  // stage: [S] active flags (as doubles), [S] beta, [S] target
  __shared__ int count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < S; s += kB) {
    const int a = stage[s] != 0.0;
    if (a) atomicAdd(&count, 1);
    const double beta = stage[S + s];
    G.act[s] = a;
    G.ran[s] = a;
    G.kk[s] = 0;
    G.target[s] = stage[2 * S + s];
    G.g[size_t(s) * (G.mr + 1)] = beta;
    G.fac[s] = a ? 1.0 / beta : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) G.nact[0] = count;
}

__global__ __launch_bounds__(kB) void k_step_finish(GmresDev G, int S, int j, int max_it,
                                                    const double* __restrict__ h, const double* __restrict__ h2,
                                                    const double* __restrict__ nrm) {
  __shared__ int count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < S; s += kB)
    if (givens_update(G, s, j, max_it, h + size_t(s) * kMaxBasis, h2 + size_t(s) * kMaxBasis, nrm[4 * s],
                      nrm[4 * s + 1]))
      atomicAdd(&count, 1);
  __syncthreads();
  if (threadIdx.x == 0) G.nact[0] = count;
}

// y = R^{-1} g on the first kk[s] rows (zero beyond), for segments that ran.
__global__ __launch_bounds__(kB) void k_lsq(GmresDev G, int S, double* __restrict__ y) {
  const int mr = G.mr;
  for (int s = threadIdx.x; s < S; s += kB) {
    double* ys = y + size_t(s) * kMaxBasis;
    const int k = G.ran[s] ? G.kk[s] : 0;
    for (int i = k; i < mr; ++i) ys[i] = 0.0;
    const double* g = G.g + size_t(s) * (mr + 1);
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < k; ++l) t -= G.H[(size_t(s) * mr + l) * (mr + 1) + i] * ys[l];
      ys[i] = t / G.H[(size_t(s) * mr + i) * (mr + 1) + i];
    }
  }
}

__global__ __launch_bounds__(kB) void k_zero_counters(GmresDev G, int S) {
  for (int s = threadIdx.x; s < S; s += kB) {
    G.its[s] = 0;
    G.flag[s] = 0;
    G.kk[s] = 0;
  }
}

}  // namespace

void gmres_zero_counters(const GmresDev& G, int S, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(kB), 0, s, G, S);
  JFNK_HIP(hipGetLastError());
}

void gmres_cycle_init(const GmresDev& G, int S, const double* stage, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(kB), 0, s, G, S, stage);
  JFNK_HIP(hipGetLastError());
}

void gmres_step_finish(const GmresDev& G, int S, int j, int max_it, const double* h, const double* h2,
                       const double* nrm, hipStream_t s) {
  hipLaunchKernelGGL(k_step_finish, dim3(1), dim3(kB), 0, s, G, S, j, max_it, h, h2, nrm);
  JFNK_HIP(hipGetLastError());
}

void gmres_lsq(const GmresDev& G, int S, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_lsq, dim3(1), dim3(kB), 0, s, G, S, y);
  JFNK_HIP(hipGetLastError());
}

}  // namespace jfnk
