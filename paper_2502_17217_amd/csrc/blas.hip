// Vector kernels for the Krylov solver and the J.v step size, gfx950.
//
// Reductions are deterministic and per segment: one workgroup per tile of
// kFvBlock cells (fixed reduction over the 64 lanes of a wavefront, fixed
// order over the 4 wavefronts), then one workgroup per segment sums that
// segment's tile partials in a fixed order.  A segment's result depends only
// on its own values, not on the other segments of a batch.
#include <cfloat>

#include "blas.h"
#include "internal.h"
#include "reduce_dev.h"

namespace jfnk {

namespace {

__global__ void k_set_n(double* d, int n, const double* src) {
  const int i = threadIdx.x;
  if (i < n) d[i] = src[i];
}

// External interleaved [cell][dim] (concatenated meshes, input order) <->
// internal component-major [dim][cell] (union order, padding cells zero).
__global__ __launch_bounds__(kBlock) void k_permute(const int32_t* __restrict__ ext_of_int,
                                                    const double* __restrict__ in,
                                                    double* __restrict__ out, int64_t n_cells,
                                                    int dim, int to_internal) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n_cells) return;
  const int64_t e = ext_of_int[i];
  for (int k = 0; k < dim; ++k) {
    if (to_internal)
      out[k * n_cells + i] = e >= 0 ? in[e * dim + k] : 0.0;
    else if (e >= 0)
      out[e * dim + k] = in[k * n_cells + i];
  }
}

// partials[blk * ldp + k0 + k] = tile blk's share of V_{k0+k} . w, k < nv (nv <= 8)
__global__ __launch_bounds__(kBlock) void k_mdot8(SegLayout L, const double* __restrict__ V, int64_t ldv,
                                                  int k0, int nv, const double* __restrict__ w,
                                                  const int32_t* __restrict__ active,
                                                  double* __restrict__ partials, int ldp) {
  __shared__ double sh[4];
  const int blk = blockIdx.x;
  if (active != nullptr && active[L.seg_of_block[blk]] == 0) return;
  const int c = blk * kFvBlock + threadIdx.x;
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  if (c < L.n_cells) {
    for (int q = 0; q < L.dim; ++q) {
      const size_t o = size_t(q) * L.n_cells + c;
      const double wi = w[o];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < nv) acc[k] = fma(V[(k0 + k) * ldv + o], wi, acc[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < nv) {
      const double s = block_sum(acc[k], sh);
      if (threadIdx.x == 0) partials[size_t(blk) * ldp + k0 + k] = s;
    }
  }
}

// out[seg * ldo + k] (+)= sum of the segment's tile partials, in tile order.
__global__ __launch_bounds__(kBlock) void k_reduce_seg(SegLayout L, const double* __restrict__ partials,
                                                       int ldp, const int32_t* __restrict__ active,
                                                       double* __restrict__ out, int ldo, int accumulate) {
  __shared__ double sh[4];
  const int k = blockIdx.x, seg = blockIdx.y;
  if (active != nullptr && active[seg] == 0) return;
  double s = 0;
  for (int b = L.block_first[seg] + threadIdx.x; b < L.block_first[seg + 1]; b += kBlock)
    s += partials[size_t(b) * ldp + k];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    const size_t o = size_t(seg) * ldo + k;
    out[o] = accumulate ? out[o] + s : s;
  }
}

// w += sign * sum_{k<nk} h[seg * ldh + k] V_k on the tile's segment
// B: the basis element type (double, or float for an FP32 basis, each
// element taken exactly to FP64 before its product).
template <class B>
__global__ __launch_bounds__(kBlock) void k_combine(SegLayout L, const B* __restrict__ V, int64_t ldv,
                                                    int nk_all, const double* __restrict__ h, int ldh,
                                                    double sign, const int32_t* __restrict__ active,
                                                    const int32_t* __restrict__ nk_seg,
                                                    double* __restrict__ w) {
  __shared__ double hs[kMaxBasis];
  const int blk = blockIdx.x;
  const int seg = L.seg_of_block[blk];
  if (active != nullptr && active[seg] == 0) return;
  const int nk = nk_seg != nullptr ? min(nk_all, nk_seg[seg]) : nk_all;
  for (int k = threadIdx.x; k < nk; k += kBlock) hs[k] = h[size_t(seg) * ldh + k];
  __syncthreads();
  const int c = blk * kFvBlock + threadIdx.x;
  if (c >= L.n_cells) return;
  for (int q = 0; q < L.dim; ++q) {
    const size_t o = size_t(q) * L.n_cells + c;
    double s = 0;
    for (int k = 0; k < nk; ++k) s = fma(hs[k], double(V[k * ldv + o]), s);
    w[o] = fma(sign, s, w[o]);
  }
}

__global__ __launch_bounds__(kBlock) void k_scale_seg(SegLayout L, const double* __restrict__ x,
                                                      const double* __restrict__ scale,
                                                      const int32_t* __restrict__ active,
                                                      double* __restrict__ y) {
  const int blk = blockIdx.x;
  const int seg = L.seg_of_block[blk];
  if (active != nullptr && active[seg] == 0) return;
  const int c = blk * kFvBlock + threadIdx.x;
  if (c >= L.n_cells) return;
  const double f = scale[seg];
  for (int q = 0; q < L.dim; ++q) {
    const size_t o = size_t(q) * L.n_cells + c;
    y[o] = f * x[o];
  }
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
// applied to every component of the component-major vector), or
// dinv[k][c] * r[k][c] when per_comp (meshes with symmetry faces)
__global__ __launch_bounds__(kBlock) void k_jacobi(const double* __restrict__ dinv,
                                                   const double* __restrict__ r,
                                                   double* __restrict__ z, int64_t n_cells, int dim,
                                                   int per_comp, const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  const int64_t ds = per_comp ? n_cells : 0;
  for (int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x; c < n_cells; c += stride) {
    for (int k = 0; k < dim; ++k) z[k * n_cells + c] = dinv[k * ds + c] * r[k * n_cells + c];
  }
}

// zf = z rounded to FP32 (to nearest); back: also z = zf, so that both hold
// the same value.  Skipped when gate is given and *gate == 0.
__global__ __launch_bounds__(kBlock) void k_round_fp32(double* __restrict__ z, float* __restrict__ zf, int64_t n,
                                                       int back, const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
    const float f = float(z[i]);
    zf[i] = f;
    if (back) z[i] = double(f);
  }
}

// Central-difference step from the forward one: eps *= factor, eps_neg = -eps.
__global__ void k_central_eps(double* __restrict__ eps, double* __restrict__ eps_neg, int S, double factor) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  const double e = eps[i] * factor;
  eps[i] = e;
  eps_neg[i] = -e;
}

inline int grid_stride_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return int(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

void launch_set_scalars(double* d, const double* h_values, int n, hipStream_t s) {
  JFNK_HIP(hipMemcpyAsync(d, h_values, sizeof(double) * n, hipMemcpyHostToDevice, s));
}

void launch_permute(const int32_t* ext_of_int, const double* in, double* out, int64_t n_cells, int dim,
                    bool to_internal, hipStream_t s) {
  const int nb = int((n_cells + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_permute, dim3(nb), dim3(kBlock), 0, s, ext_of_int, in, out, n_cells, dim,
                     to_internal ? 1 : 0);
  JFNK_HIP(hipGetLastError());
}

void blas_mdot(const SegLayout& L, const double* V, int64_t ldv, int nk, const double* w, double* partials,
               double* out, int ldo, bool accumulate, const int32_t* active, hipStream_t s) {
  for (int k0 = 0; k0 < nk; k0 += 8) {
    const int nv = nk - k0 < 8 ? nk - k0 : 8;
    hipLaunchKernelGGL(k_mdot8, dim3(L.n_blocks), dim3(kBlock), 0, s, L, V, ldv, k0, nv, w, active, partials,
                       kMaxBasis);
  }
  hipLaunchKernelGGL(k_reduce_seg, dim3(nk, L.n_seg), dim3(kBlock), 0, s, L, partials, kMaxBasis, active, out,
                     ldo, accumulate ? 1 : 0);
  JFNK_HIP(hipGetLastError());
}

void blas_combine(const SegLayout& L, const double* V, int64_t ldv, int nk, const double* h, int ldh,
                  double sign, double* w, const int32_t* active, hipStream_t s, const int32_t* nk_seg) {
  hipLaunchKernelGGL(k_combine<double>, dim3(L.n_blocks), dim3(kBlock), 0, s, L, V, ldv, nk, h, ldh, sign,
                     active, nk_seg, w);
  JFNK_HIP(hipGetLastError());
}

void blas_combine(const SegLayout& L, const float* V, int64_t ldv, int nk, const double* h, int ldh,
                  double sign, double* w, const int32_t* active, hipStream_t s, const int32_t* nk_seg) {
  hipLaunchKernelGGL(k_combine<float>, dim3(L.n_blocks), dim3(kBlock), 0, s, L, V, ldv, nk, h, ldh, sign,
                     active, nk_seg, w);
  JFNK_HIP(hipGetLastError());
}

void blas_round_fp32(double* z, float* zf, int64_t n, bool back, hipStream_t s, const int32_t* gate) {
  hipLaunchKernelGGL(k_round_fp32, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, s, z, zf, n, back ? 1 : 0, gate);
  JFNK_HIP(hipGetLastError());
}

void blas_scale_seg(const SegLayout& L, const double* x, const double* scale, double* y,
                    const int32_t* active, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_seg, dim3(L.n_blocks), dim3(kBlock), 0, s, L, x, scale, active, y);
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

void blas_central_eps(double* eps, double* eps_neg, int S, double factor, hipStream_t s) {
  hipLaunchKernelGGL(k_central_eps, dim3((S + 255) / 256), dim3(256), 0, s, eps, eps_neg, S, factor);
  JFNK_HIP(hipGetLastError());
}

void blas_jacobi(const double* dinv, const double* r, double* z, int64_t n_cells, int dim, bool per_comp,
                 hipStream_t s, const int32_t* gate) {
  hipLaunchKernelGGL(k_jacobi, dim3(grid_stride_blocks(n_cells)), dim3(kBlock), 0, s, dinv, r, z,
                     n_cells, dim, per_comp ? 1 : 0, gate);
  JFNK_HIP(hipGetLastError());
}

}  // namespace jfnk
