// Smoothed-aggregation AMG for the compact-stencil approximate Jacobian,
// stored and applied in FP32 (or FP64 for the full-precision twin).
#pragma once

#include <vector>

#include "internal.h"

namespace jfnk {

// Host CSR matrix (FP64) used during setup.
struct HostCsr {
  int64_t n = 0, m = 0;              // rows, cols
  HostVec<int32_t> ptr, col;
  HostVec<double> val;
  int64_t nnz() const { return int64_t(col.size()); }
};

// Device CSR matrix (FP32 or FP64 values).
struct DevCsr {
  int32_t n = 0, m = 0;
  int32_t lanes = 1;      // lanes that share a row in the row kernels (power of two, <= 64)
  int64_t nnz = 0;
  DevBuf ptr, col, val;
  void upload(const HostCsr& h, bool fp64, hipStream_t s);
};

struct AmgLevel {
  int64_t n = 0;
  DevCsr A, P, R;         // operator; prolongation (n x n_next); restriction = P^T
  DevBuf dinv;            // inverse diagonal of A (the hierarchy's precision); [dim][n] when ecorr is set
  DevBuf ecorr;           // finest level of a mesh with symmetry faces: [dim][n] per-component
                          // diagonal added to A (A holds the component mean); empty otherwise
  double lmax = 2.0;      // largest eigenvalue estimate of D^{-1} A
  size_t off_x = 0, off_b = 0, off_r = 0, off_d0 = 0, off_d1 = 0;  // workspace offsets (floats)
};

struct AmgHierarchy {
  std::vector<AmgLevel> levels;      // last level is solved by the dense inverse (or its diagonal)
  bool fp64 = false;                 // values and work vectors in FP64 (else FP32)
  bool coarse_diag = false;          // coarsest rows uncoupled: coarse_inv holds D^{-1} only
  DevBuf coarse_inv;                 // [n_c][n_c] column-major, or [n_c] when coarse_diag
  int64_t n_coarse = 0;
  size_t off_part = 0;               // work offset of the chunked dense product's partial sums
  int dim = 3;
  size_t work_floats = 0;
  double op_complexity = 0;          // sum nnz(A_l) / nnz(A_0)
  double setup_ms = 0;
};

// The diagonal a smoothing kernel uses: the inverse diagonal, shared by the
// components (dstride 0) or per component (dstride n), and the optional
// per-component diagonal correction of the finest level.
template <class T>
struct AmgDiag {
  const T* dinv = nullptr;
  int dstride = 0;
  const T* ecorr = nullptr;
};

// ---- kernels (amg_kernels.hip), T = float or double; vectors are
// component-major [dim][n] ----
template <class T>
void amg_cast_in(const double* r, T* b, int64_t n, int dim, hipStream_t s, const int32_t* gate);
template <class T>
void amg_cast_out(const T* x, double* z, int64_t n, int dim, hipStream_t s, const int32_t* gate);
// Chebyshev start from x = 0: r = D^-1 b, d = r/theta, x = d; with r64
// given, b = (T) r64 first (the finest level's FP64 input)
template <class T>
void amg_cheb_start0(const DevCsr& A, const AmgDiag<T>& dg, T* b, T* x, T* r, T* d, T inv_theta, int dim,
                     hipStream_t s, const int32_t* gate, const double* r64 = nullptr);
// Chebyshev start from a given x: r = D^-1 (b - A x), d = r/theta, x += d
// (defer_axpy: the next step applies x += d; z64 given: also z = -x in FP64)
template <class T>
void amg_cheb_start(const DevCsr& A, const AmgDiag<T>& dg, const T* b, T* x, T* r, T* d, T inv_theta, int dim,
                    hipStream_t s, const int32_t* gate, bool defer_axpy = false, double* z64 = nullptr);
// one Chebyshev step: r -= D^-1 A d_in; d_out = c1 d_in + c2 r; x += d_out
// (pend: x += d_in first, the deferred start update; z64 given: z = -x in FP64)
template <class T>
void amg_cheb_step(const DevCsr& A, const AmgDiag<T>& dg, const T* d_in, T* d_out, T* r, T* x, T c1, T c2,
                   int dim, hipStream_t s, const int32_t* gate, bool pend = false, double* z64 = nullptr);
// r = b - A x
template <class T>
void amg_residual(const DevCsr& A, const AmgDiag<T>& dg, const T* b, const T* x, T* r, int dim, hipStream_t s,
                  const int32_t* gate);
// y = M x (restriction) or y += M x (prolongation, accumulate = true)
template <class T>
void amg_spmv(const DevCsr& M, const T* x, T* y, bool accumulate, int dim, hipStream_t s, const int32_t* gate);
// x = inv * b (dense, n x n)
template <class T>
void amg_dense(const T* inv, const T* b, T* x, int n, int dim, hipStream_t s, const int32_t* gate);
// the same for larger n in two passes: chunks of kDenseChunk columns into
// part ([ceil(n / kDenseChunk)][dim][n]), then their sum in chunk order
constexpr int kDenseChunk = 256;
template <class T>
void amg_dense_chunked(const T* inv, const T* b, T* x, T* part, int n, int dim, hipStream_t s,
                       const int32_t* gate);
// out (n x n, both triangles, T) from the lower triangle of a column-major FP64 matrix
template <class T>
void amg_sym_from_lower(const double* lo, T* out, int n, hipStream_t s);
// x = dinv * b (coarsest level of uncoupled rows)
template <class T>
void amg_diag_solve(const T* dinv, const T* b, T* x, int n, int dim, hipStream_t s, const int32_t* gate);

}  // namespace jfnk
