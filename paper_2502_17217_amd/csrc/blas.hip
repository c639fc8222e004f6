// Vector kernels for the Krylov solver and the J.v step size, gfx950.
//
// Reductions are deterministic: a fixed grid of kRedBlocks workgroups, a
// fixed element-to-thread assignment (grid stride), a fixed butterfly over
// the 64 lanes of a wavefront, a fixed order over the 4 wavefronts of a
// workgroup, and a second single-workgroup pass over the partial sums in a
// fixed order.  The result depends only on the vector length and values.
#include <cfloat>

#include "blas.h"
#include "internal.h"

namespace jfnk {

namespace {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum over a 256-thread workgroup; valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double* sh) {
  x = wave_sum(x);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}

// Two squared norms; each thread keeps four independent loads in flight per
// vector (fixed element assignment, so the result is deterministic).
__global__ __launch_bounds__(kBlock) void k_norm2_pair(const double* __restrict__ a,
                                                       const double* __restrict__ b, int64_t n,
                                                       double* __restrict__ partials) {
  __shared__ double sh[4];
  double sa[4] = {0, 0, 0, 0}, sb[4] = {0, 0, 0, 0};
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    double x[4], y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x[q] = a[i + q * stride];
      y[q] = b[i + q * stride];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sa[q] = fma(x[q], x[q], sa[q]);
      sb[q] = fma(y[q], y[q], sb[q]);
    }
  }
  for (int q = 0; i < n; i += stride, ++q) {
    const double x = a[i], y = b[i];
    sa[q & 3] = fma(x, x, sa[q & 3]);
    sb[q & 3] = fma(y, y, sb[q & 3]);
  }
  double ta = block_sum((sa[0] + sa[1]) + (sa[2] + sa[3]), sh);
  double tb = block_sum((sb[0] + sb[1]) + (sb[2] + sb[3]), sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = ta;
    partials[2 * blockIdx.x + 1] = tb;
  }
}

__global__ __launch_bounds__(kBlock) void k_eps_final(const double* __restrict__ partials, int nb,
                                                      double* __restrict__ d_eps) {
  __shared__ double sh[4];
  double sa = 0, sb = 0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    sa += partials[2 * i];
    sb += partials[2 * i + 1];
  }
  sa = block_sum(sa, sh);
  sb = block_sum(sb, sh);
  if (threadIdx.x == 0) {
    // sqrt(eps_mach) * sqrt(1 + |u|) / |v|  (zero v -> zero step, J v = 0)
    const double sqrt_eps = 1.4901161193847656e-08;
    d_eps[0] = sb > 0 ? sqrt_eps * sqrt(1.0 + sqrt(sa)) / sqrt(sb) : 0.0;
  }
}

__global__ void k_set(double* d, double v) { d[0] = v; }

// Interleaved input-order [cell][dim] <-> component-major internal-order [dim][cell].
__global__ __launch_bounds__(kBlock) void k_permute(const int32_t* __restrict__ old_of_new,
                                                    const double* __restrict__ in,
                                                    double* __restrict__ out, int64_t n_cells,
                                                    int dim, int to_internal) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n_cells) return;
  const int64_t o = old_of_new[i];
  for (int k = 0; k < dim; ++k) {
    if (to_internal)
      out[k * n_cells + i] = in[o * dim + k];
    else
      out[o * dim + k] = in[k * n_cells + i];
  }
}

// partials[b * ldp + k0 + k] = block b's share of V_{k0+k} . w, k < nv (nv <= 8)
__global__ __launch_bounds__(kBlock) void k_mdot8(const double* __restrict__ V, int64_t ldv, int k0,
                                                  int nv, const double* __restrict__ w, int64_t n,
                                                  double* __restrict__ partials, int ldp) {
  __shared__ double sh[4];
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < nv) acc[k] = fma(V[(k0 + k) * ldv + i], wi, acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < nv) {
      const double s = block_sum(acc[k], sh);
      if (threadIdx.x == 0) partials[int64_t(blockIdx.x) * ldp + k0 + k] = s;
    }
  }
}

// out[k] (+)= sum_b partials[b * ldp + k] for k < nk; one workgroup per k.
__global__ __launch_bounds__(kBlock) void k_reduce_cols(const double* __restrict__ partials, int nb,
                                                        int ldp, double* __restrict__ out,
                                                        int accumulate) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += kBlock) s += partials[int64_t(b) * ldp + k];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[k] = accumulate ? out[k] + s : s;
}

// w[i] -= sum_{k<nk} h[k] V_k[i]  (sign = -1) or y[i] += sum h[k] V_k[i] (sign = +1)
__global__ __launch_bounds__(kBlock) void k_combine(const double* __restrict__ V, int64_t ldv, int nk,
                                                    const double* __restrict__ h, double sign,
                                                    double* __restrict__ w, int64_t n) {
  __shared__ double hs[kMaxBasis];
  for (int k = threadIdx.x; k < nk; k += kBlock) hs[k] = h[k];
  __syncthreads();
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
    double s = 0;
    for (int k = 0; k < nk; ++k) s = fma(hs[k], V[k * ldv + i], s);
    w[i] = fma(sign, s, w[i]);
  }
}

// y = x * (1/ *d_scale), or y = x * *d_scale when invert == 0
__global__ __launch_bounds__(kBlock) void k_scale_dev(const double* __restrict__ x,
                                                      const double* __restrict__ d_scale, int invert,
                                                      double* __restrict__ y, int64_t n) {
  const double s = invert ? 1.0 / d_scale[0] : d_scale[0];
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) y[i] = x[i] * s;
}

__global__ __launch_bounds__(kBlock) void k_axpby(double a, const double* __restrict__ x, double b,
                                                  double* __restrict__ y, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride)
    y[i] = fma(a, x[i], b * y[i]);
}

// y = a * x + b * z (three-operand form, y may alias neither)
__global__ __launch_bounds__(kBlock) void k_lincomb(double a, const double* __restrict__ x, double b,
                                                    const double* __restrict__ z,
                                                    double* __restrict__ y, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride)
    y[i] = fma(a, x[i], b * z[i]);
}

// z[k][c] = dinv[c] * r[k][c]  (diagonal of the scalar approximate Jacobian,
// applied to every component of the component-major vector)
__global__ __launch_bounds__(kBlock) void k_jacobi(const double* __restrict__ dinv,
                                                   const double* __restrict__ r,
                                                   double* __restrict__ z, int64_t n_cells, int dim) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x; c < n_cells; c += stride) {
    const double s = dinv[c];
    for (int k = 0; k < dim; ++k) z[k * n_cells + c] = s * r[k * n_cells + c];
  }
}

inline int grid_stride_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return int(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

void launch_eps(const double* u, const double* v, int64_t n, double* partials, double* d_eps,
                hipStream_t s) {
  hipLaunchKernelGGL(k_norm2_pair, dim3(kRedBlocks), dim3(kBlock), 0, s, u, v, n, partials);
  hipLaunchKernelGGL(k_eps_final, dim3(1), dim3(kBlock), 0, s, partials, kRedBlocks, d_eps);
  JFNK_HIP(hipGetLastError());
}

void launch_set_scalar(double* d, double value, hipStream_t s) {
  hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, s, d, value);
  JFNK_HIP(hipGetLastError());
}

void launch_permute(const int32_t* old_of_new, const double* in, double* out, int64_t n_cells,
                    int dim, bool to_internal, hipStream_t s) {
  const int nb = int((n_cells + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_permute, dim3(nb), dim3(kBlock), 0, s, old_of_new, in, out, n_cells, dim,
                     to_internal ? 1 : 0);
  JFNK_HIP(hipGetLastError());
}

void blas_mdot(const double* V, int64_t ldv, int nk, const double* w, int64_t n, double* partials,
               double* out, bool accumulate, hipStream_t s) {
  for (int k0 = 0; k0 < nk; k0 += 8) {
    const int nv = nk - k0 < 8 ? nk - k0 : 8;
    hipLaunchKernelGGL(k_mdot8, dim3(kRedBlocks), dim3(kBlock), 0, s, V, ldv, k0, nv, w, n, partials,
                       kMaxBasis);
  }
  hipLaunchKernelGGL(k_reduce_cols, dim3(nk), dim3(kBlock), 0, s, partials, kRedBlocks, kMaxBasis, out,
                     accumulate ? 1 : 0);
  JFNK_HIP(hipGetLastError());
}

void blas_combine(const double* V, int64_t ldv, int nk, const double* d_h, double sign, double* w,
                  int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, s, V, ldv, nk, d_h, sign,
                     w, n);
  JFNK_HIP(hipGetLastError());
}

void blas_scale_dev(const double* x, const double* d_scale, bool invert, double* y, int64_t n,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_scale_dev, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, s, x, d_scale,
                     invert ? 1 : 0, y, n);
  JFNK_HIP(hipGetLastError());
}

void blas_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, s, a, x, b, y, n);
  JFNK_HIP(hipGetLastError());
}

void blas_lincomb(double a, const double* x, double b, const double* z, double* y, int64_t n,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, s, a, x, b, z, y, n);
  JFNK_HIP(hipGetLastError());
}

void blas_jacobi(const double* dinv, const double* r, double* z, int64_t n_cells, int dim,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_jacobi, dim3(grid_stride_blocks(n_cells)), dim3(kBlock), 0, s, dinv, r, z,
                     n_cells, dim);
  JFNK_HIP(hipGetLastError());
}

}  // namespace jfnk
