// Launchers of the Krylov vector kernels (blas.hip).  All pointers are
// device pointers; all calls are asynchronous on stream s.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace jfnk {

constexpr int kMaxBasis = 256;  // max restart length + 1 supported by the kernels

// out[k] = V_k . w for k < nk (V_k = V + k*ldv); partials needs kRedBlocks*kMaxBasis doubles.
// accumulate: out[k] += instead of =.
void blas_mdot(const double* V, int64_t ldv, int nk, const double* w, int64_t n, double* partials,
               double* out, bool accumulate, hipStream_t s);
// w += sign * sum_{k<nk} h[k] V_k  (h on the device)
void blas_combine(const double* V, int64_t ldv, int nk, const double* d_h, double sign, double* w,
                  int64_t n, hipStream_t s);
// y = x / *d_scale (invert) or x * *d_scale
void blas_scale_dev(const double* x, const double* d_scale, bool invert, double* y, int64_t n,
                    hipStream_t s);
// y = a x + b y
void blas_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
// y = a x + b z
void blas_lincomb(double a, const double* x, double b, const double* z, double* y, int64_t n,
                  hipStream_t s);
// z = D^{-1} r with one scalar per cell applied to every component
void blas_jacobi(const double* dinv, const double* r, double* z, int64_t n_cells, int dim,
                 hipStream_t s);

}  // namespace jfnk
