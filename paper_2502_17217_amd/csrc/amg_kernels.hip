// Kernels of the AMG V-cycle (gfx950), instantiated for FP32 (the
// preconditioner of the mixed-precision path) and FP64 (its full-precision
// twin).  One thread, or a group of lanes, per matrix row; every kernel
// handles all displacement components (component-major arrays [dim][n]) so
// that a matrix row is read once for the dim right-hand sides.
#include "amg.h"
#include "reduce_dev.h"

namespace jfnk {

namespace {

constexpr int kB = 256;

inline int blocks_for(int64_t n) { return int((n + kB - 1) / kB); }

// Row i of a CSR matrix times x (D components), shared by the G lanes of a
// group: lane `sub` takes nonzeros sub, sub + G, ..., then a fixed reduction
// over the group (group_sum) leaves the row's sums in every lane of it.
template <class T, int D, int G>
__device__ __forceinline__ void row_dot(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                        const T* __restrict__ val, const T* __restrict__ x,
                                        int m, int i, int sub, T (&s)[D]) {
#pragma unroll
  for (int q = 0; q < D; ++q) s[q] = T(0);
  const int a = ptr[i], b = ptr[i + 1];
  for (int k = a + sub; k < b; k += G) {
    const T v = val[k];
    const int j = col[k];
#pragma unroll
    for (int q = 0; q < D; ++q) s[q] = fma(v, x[size_t(q) * m + j], s[q]);
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int q = 0; q < D; ++q) s[q] = group_sum<G>(s[q]);
  }
}

// Finest level of a mesh with symmetry faces: component q's operator is the
// stored matrix plus the diagonal ecorr[q] (the per-component part of the
// symmetry blocks), s[q] += ecorr[q][i] x[q][i]; no-op when ecorr is null.
template <class T, int D>
__device__ __forceinline__ void diag_correct(const T* __restrict__ ecorr, const T* __restrict__ x, int n, int i,
                                             T (&s)[D]) {
  if (ecorr == nullptr) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * n + i;
    s[q] = fma(ecorr[o], x[o], s[q]);
  }
}

// Row and lane-in-group of this thread when G lanes share a row.
template <int G>
__device__ __forceinline__ int row_of(int& sub) {
  sub = threadIdx.x % G;
  return blockIdx.x * (kB / G) + threadIdx.x / G;
}

template <class T>
__global__ __launch_bounds__(kB) void k_cast_in(const double* __restrict__ r, T* __restrict__ b,
                                                int64_t total, const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x;
  if (i < total) b[i] = T(r[i]);
}

template <class T>
__global__ __launch_bounds__(kB) void k_cast_out(const T* __restrict__ x, double* __restrict__ z,
                                                 int64_t total, const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x;
  if (i < total) z[i] = -double(x[i]);   // J_tilde = -A
}

// r64 != null (finest level): the right-hand side arrives in FP64 and is
// rounded into b here (the cast that would otherwise be its own launch).
template <class T, int D>
__global__ __launch_bounds__(kB) void k_cheb_start0(int n, const T* __restrict__ dinv, int dstride,
                                                    T* __restrict__ b, T* __restrict__ x,
                                                    T* __restrict__ r, T* __restrict__ d,
                                                    T inv_theta, const double* __restrict__ r64,
                                                    const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * n + i;
    const T di = dinv[size_t(q) * dstride + i];
    T bo;
    if (r64 != nullptr) {
      bo = T(r64[o]);
      b[o] = bo;
    } else {
      bo = b[o];
    }
    const T ri = di * bo;
    const T dd = ri * inv_theta;
    r[o] = ri;
    d[o] = dd;
    x[o] = dd;
  }
}

template <class T, int D, int G>
__global__ __launch_bounds__(kB) void k_cheb_start(int n, const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col,
                                                   const T* __restrict__ val,
                                                   const T* __restrict__ dinv, int dstride,
                                                   const T* __restrict__ ecorr,
                                                   const T* __restrict__ b, const T* __restrict__ x,
                                                   T* __restrict__ r, T* __restrict__ d,
                                                   T inv_theta, const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  int sub;
  const int i = row_of<G>(sub);
  if (i >= n) return;
  T s[D];
  row_dot<T, D, G>(ptr, col, val, x, n, i, sub, s);
  if (sub != 0) return;
  diag_correct<T, D>(ecorr, x, n, i, s);
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * n + i;
    const T di = dinv[size_t(q) * dstride + i];
    const T ri = di * (b[o] - s[q]);
    r[o] = ri;
    d[o] = ri * inv_theta;
  }
}

// x += d; z64 != null: also z = -x in FP64 (finest level, J_tilde = -A).
template <class T, int D>
__global__ __launch_bounds__(kB) void k_axpy_inplace(int n, const T* __restrict__ d, T* __restrict__ x,
                                                     double* __restrict__ z64,
                                                     const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * n + i;
    const T xo = x[o] + d[o];
    x[o] = xo;
    if (z64 != nullptr) z64[o] = -double(xo);
  }
}

// pend != 0: the previous start's x += d_in is still to be applied (it is,
// first: x = (x + d_in) + dd); z64 != null: also z = -x in FP64.
template <class T, int D, int G>
__global__ __launch_bounds__(kB) void k_cheb_step(int n, const int32_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col,
                                                  const T* __restrict__ val,
                                                  const T* __restrict__ dinv, int dstride,
                                                  const T* __restrict__ ecorr,
                                                  const T* __restrict__ d_in, T* __restrict__ d_out,
                                                  T* __restrict__ r, T* __restrict__ x, T c1,
                                                  T c2, int pend, double* __restrict__ z64,
                                                  const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  int sub;
  const int i = row_of<G>(sub);
  if (i >= n) return;
  T s[D];
  row_dot<T, D, G>(ptr, col, val, d_in, n, i, sub, s);
  if (sub != 0) return;
  diag_correct<T, D>(ecorr, d_in, n, i, s);
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * n + i;
    const T di = dinv[size_t(q) * dstride + i];
    const T ri = r[o] - di * s[q];
    const T dd = fma(c1, d_in[o], c2 * ri);
    r[o] = ri;
    d_out[o] = dd;
    T xo = x[o];
    if (pend) xo += d_in[o];
    xo += dd;
    x[o] = xo;
    if (z64 != nullptr) z64[o] = -double(xo);
  }
}

template <class T, int D, int G>
__global__ __launch_bounds__(kB) void k_residual(int n, const int32_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col,
                                                 const T* __restrict__ val, const T* __restrict__ ecorr,
                                                 const T* __restrict__ b,
                                                 const T* __restrict__ x, T* __restrict__ r,
                                                 const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  int sub;
  const int i = row_of<G>(sub);
  if (i >= n) return;
  T s[D];
  row_dot<T, D, G>(ptr, col, val, x, n, i, sub, s);
  if (sub != 0) return;
  diag_correct<T, D>(ecorr, x, n, i, s);
#pragma unroll
  for (int q = 0; q < D; ++q) r[size_t(q) * n + i] = b[size_t(q) * n + i] - s[q];
}

template <class T, int D, int G>
__global__ __launch_bounds__(kB) void k_spmv(int n, int m, const int32_t* __restrict__ ptr,
                                             const int32_t* __restrict__ col, const T* __restrict__ val,
                                             const T* __restrict__ x, T* __restrict__ y, int accumulate,
                                             const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  int sub;
  const int i = row_of<G>(sub);
  if (i >= n) return;
  T s[D];
  row_dot<T, D, G>(ptr, col, val, x, m, i, sub, s);
  if (sub != 0) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * n + i;
    y[o] = accumulate ? y[o] + s[q] : s[q];
  }
}

// x = A_c^{-1} b on the coarsest level.  inv is column-major (column j
// contiguous), so the 64 lanes of a wave read consecutive rows of one column
// and b[j] is a broadcast; the four waves of a workgroup take every fourth
// column and their partial sums meet in LDS.
template <class T, int D>
__global__ __launch_bounds__(kB) void k_dense(const T* __restrict__ inv, const T* __restrict__ b,
                                              T* __restrict__ x, int n, const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  constexpr int kWaves = kB / 64;
  __shared__ T part[kWaves][D][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  T s[D];
#pragma unroll
  for (int q = 0; q < D; ++q) s[q] = T(0);
  if (i < n) {
    for (int j = wave; j < n; j += kWaves) {
      const T a = inv[size_t(j) * n + i];
#pragma unroll
      for (int q = 0; q < D; ++q) s[q] = fma(a, b[size_t(q) * n + j], s[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < D; ++q) part[wave][q][lane] = s[q];
  __syncthreads();
  if (wave == 0 && i < n) {
#pragma unroll
    for (int q = 0; q < D; ++q) {
      T t = part[0][q][lane];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) t += part[w][q][lane];
      x[size_t(q) * n + i] = t;
    }
  }
}

// Larger coarsest levels, first of two passes: workgroup (ib, jc) sums
// columns jc*kDenseChunk .. +kDenseChunk of rows ib*64 .. +63 (the four waves
// take every fourth column and meet in LDS in a fixed order) into
// part[jc][q][i]; the second pass adds the chunks in order.  Enough
// workgroups to stream the whole inverse at once.
template <class T, int D>
__global__ __launch_bounds__(kB) void k_dense_part(const T* __restrict__ inv, const T* __restrict__ b,
                                                   T* __restrict__ part, int n, const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  constexpr int kWaves = kB / 64;
  __shared__ T acc[kWaves][D][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int j0 = blockIdx.y * kDenseChunk, j1 = min(n, j0 + kDenseChunk);
  T s[D];
#pragma unroll
  for (int q = 0; q < D; ++q) s[q] = T(0);
  if (i < n) {
    // eight of this wave's columns loaded at a time, then added in order
    int j = j0 + wave;
    for (; j + 7 * kWaves < j1; j += 8 * kWaves) {
      T a[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = inv[size_t(j + k * kWaves) * n + i];
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int q = 0; q < D; ++q) s[q] = fma(a[k], b[size_t(q) * n + j + k * kWaves], s[q]);
    }
    for (; j < j1; j += kWaves) {
      const T a = inv[size_t(j) * n + i];
#pragma unroll
      for (int q = 0; q < D; ++q) s[q] = fma(a, b[size_t(q) * n + j], s[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < D; ++q) acc[wave][q][lane] = s[q];
  __syncthreads();
  if (wave == 0 && i < n) {
#pragma unroll
    for (int q = 0; q < D; ++q) {
      T t = acc[0][q][lane];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) t += acc[w][q][lane];
      part[(size_t(blockIdx.y) * D + q) * n + i] = t;
    }
  }
}

// Second pass: one thread per (row, component), the chunks' partial sums
// loaded eight at a time and added in chunk order.
template <class T, int D>
__global__ __launch_bounds__(kB) void k_dense_sum(const T* __restrict__ part, T* __restrict__ x, int n, int nc,
                                                  const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int t = blockIdx.x * kB + threadIdx.x;
  if (t >= D * n) return;
  const int q = t / n, i = t % n;
  T s = part[size_t(q) * n + i];
  int c = 1;
  for (; c + 8 <= nc; c += 8) {
    T v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = part[(size_t(c + k) * D + q) * n + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; c < nc; ++c) s += part[(size_t(c) * D + q) * n + i];
  x[size_t(q) * n + i] = s;
}

// Both triangles of the inverse from the lower triangle rocSOLVER leaves
// (column-major, FP64), in the hierarchy's precision.
template <class T>
__global__ __launch_bounds__(kB) void k_sym_from_lower(const double* __restrict__ lo, T* __restrict__ out, int n) {
  const int64_t t = int64_t(blockIdx.x) * kB + threadIdx.x;
  if (t >= int64_t(n) * n) return;
  const int j = int(t / n), i = int(t % n);
  out[t] = T(i >= j ? lo[size_t(j) * n + i] : lo[size_t(i) * n + j]);
}

// x = D^{-1} b: the coarsest level when no two of its rows are coupled.
template <class T, int D>
__global__ __launch_bounds__(kB) void k_diag_solve(const T* __restrict__ dinv, const T* __restrict__ b,
                                                   T* __restrict__ x, int n, const int32_t* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const T di = dinv[i];
#pragma unroll
  for (int q = 0; q < D; ++q) x[size_t(q) * n + i] = di * b[size_t(q) * n + i];
}

}  // namespace

#define JFNK_DIM_DISPATCH(dim, KERNEL, ...)                                        \
  do {                                                                             \
    if ((dim) == 3)                                                                \
      hipLaunchKernelGGL((KERNEL<T, 3>), __VA_ARGS__);                             \
    else                                                                           \
      hipLaunchKernelGGL((KERNEL<T, 2>), __VA_ARGS__);                             \
    JFNK_HIP(hipGetLastError());                                                   \
  } while (0)

// Row kernels: dimension and lanes per row (grid sized for lanes * n threads).
#define JFNK_ROW_CASE(D, G, KERNEL, n, s, ...)                                                           \
  case G:                                                                                               \
    hipLaunchKernelGGL((KERNEL<T, D, G>), dim3(blocks_for(int64_t(n) * G)), dim3(kB), 0, s, __VA_ARGS__); \
    break;
#define JFNK_ROW_DISPATCH_D(D, lanes, KERNEL, n, s, ...)   \
  switch (lanes) {                                        \
    JFNK_ROW_CASE(D, 1, KERNEL, n, s, __VA_ARGS__)        \
    JFNK_ROW_CASE(D, 2, KERNEL, n, s, __VA_ARGS__)        \
    JFNK_ROW_CASE(D, 4, KERNEL, n, s, __VA_ARGS__)        \
    JFNK_ROW_CASE(D, 8, KERNEL, n, s, __VA_ARGS__)        \
    JFNK_ROW_CASE(D, 16, KERNEL, n, s, __VA_ARGS__)       \
    JFNK_ROW_CASE(D, 32, KERNEL, n, s, __VA_ARGS__)       \
    default:                                              \
      JFNK_ROW_CASE(D, 64, KERNEL, n, s, __VA_ARGS__)     \
  }
#define JFNK_ROW_DISPATCH(dim, lanes, KERNEL, n, s, ...)                       \
  do {                                                                         \
    if ((dim) == 3) {                                                          \
      JFNK_ROW_DISPATCH_D(3, lanes, KERNEL, n, s, __VA_ARGS__)                 \
    } else {                                                                   \
      JFNK_ROW_DISPATCH_D(2, lanes, KERNEL, n, s, __VA_ARGS__)                 \
    }                                                                          \
    JFNK_HIP(hipGetLastError());                                               \
  } while (0)

template <class T>
void amg_cast_in(const double* r, T* b, int64_t n, int dim, hipStream_t s, const int32_t* gate) {
  const int64_t t = n * dim;
  hipLaunchKernelGGL(k_cast_in<T>, dim3(blocks_for(t)), dim3(kB), 0, s, r, b, t, gate);
  JFNK_HIP(hipGetLastError());
}

template <class T>
void amg_cast_out(const T* x, double* z, int64_t n, int dim, hipStream_t s, const int32_t* gate) {
  const int64_t t = n * dim;
  hipLaunchKernelGGL(k_cast_out<T>, dim3(blocks_for(t)), dim3(kB), 0, s, x, z, t, gate);
  JFNK_HIP(hipGetLastError());
}

template <class T>
void amg_cheb_start0(const DevCsr& A, const AmgDiag<T>& dg, T* b, T* x, T* r, T* d, T inv_theta, int dim,
                     hipStream_t s, const int32_t* gate, const double* r64) {
  JFNK_DIM_DISPATCH(dim, k_cheb_start0, dim3(blocks_for(A.n)), dim3(kB), 0, s, A.n, dg.dinv, dg.dstride, b, x,
                    r, d, inv_theta, r64, gate);
}

template <class T>
void amg_cheb_start(const DevCsr& A, const AmgDiag<T>& dg, const T* b, T* x, T* r, T* d, T inv_theta, int dim,
                    hipStream_t s, const int32_t* gate, bool defer_axpy, double* z64) {
  // r = D^-1 (b - A x), d = r / theta, then x += d in a second pass (x is read
  // by other rows' products in the first pass), or in the next step's launch
  JFNK_ROW_DISPATCH(dim, A.lanes, k_cheb_start, A.n, s, A.n, A.ptr.as<int32_t>(), A.col.as<int32_t>(),
                    A.val.as<T>(), dg.dinv, dg.dstride, dg.ecorr, b, x, r, d, inv_theta, gate);
  if (!defer_axpy)
    JFNK_DIM_DISPATCH(dim, k_axpy_inplace, dim3(blocks_for(A.n)), dim3(kB), 0, s, A.n, d, x, z64, gate);
}

template <class T>
void amg_cheb_step(const DevCsr& A, const AmgDiag<T>& dg, const T* d_in, T* d_out, T* r, T* x, T c1, T c2,
                   int dim, hipStream_t s, const int32_t* gate, bool pend, double* z64) {
  JFNK_ROW_DISPATCH(dim, A.lanes, k_cheb_step, A.n, s, A.n, A.ptr.as<int32_t>(), A.col.as<int32_t>(),
                    A.val.as<T>(), dg.dinv, dg.dstride, dg.ecorr, d_in, d_out, r, x, c1, c2, pend ? 1 : 0, z64,
                    gate);
}

template <class T>
void amg_residual(const DevCsr& A, const AmgDiag<T>& dg, const T* b, const T* x, T* r, int dim, hipStream_t s,
                  const int32_t* gate) {
  JFNK_ROW_DISPATCH(dim, A.lanes, k_residual, A.n, s, A.n, A.ptr.as<int32_t>(), A.col.as<int32_t>(),
                    A.val.as<T>(), dg.ecorr, b, x, r, gate);
}

template <class T>
void amg_spmv(const DevCsr& M, const T* x, T* y, bool accumulate, int dim, hipStream_t s, const int32_t* gate) {
  JFNK_ROW_DISPATCH(dim, M.lanes, k_spmv, M.n, s, M.n, M.m, M.ptr.as<int32_t>(), M.col.as<int32_t>(),
                    M.val.as<T>(), x, y, accumulate ? 1 : 0, gate);
}

template <class T>
void amg_dense(const T* inv, const T* b, T* x, int n, int dim, hipStream_t s, const int32_t* gate) {
  JFNK_DIM_DISPATCH(dim, k_dense, dim3((n + 63) / 64), dim3(kB), 0, s, inv, b, x, n, gate);
}

template <class T>
void amg_dense_chunked(const T* inv, const T* b, T* x, T* part, int n, int dim, hipStream_t s,
                       const int32_t* gate) {
  const int nc = (n + kDenseChunk - 1) / kDenseChunk;
  JFNK_DIM_DISPATCH(dim, k_dense_part, dim3((n + 63) / 64, nc), dim3(kB), 0, s, inv, b, part, n, gate);
  JFNK_DIM_DISPATCH(dim, k_dense_sum, dim3(blocks_for(int64_t(dim) * n)), dim3(kB), 0, s, part, x, n, nc, gate);
}

template <class T>
void amg_sym_from_lower(const double* lo, T* out, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_sym_from_lower<T>, dim3(blocks_for(int64_t(n) * n)), dim3(kB), 0, s, lo, out, n);
  JFNK_HIP(hipGetLastError());
}

template <class T>
void amg_diag_solve(const T* dinv, const T* b, T* x, int n, int dim, hipStream_t s, const int32_t* gate) {
  JFNK_DIM_DISPATCH(dim, k_diag_solve, dim3(blocks_for(n)), dim3(kB), 0, s, dinv, b, x, n, gate);
}

#define JFNK_AMG_INSTANTIATE(T)                                                                           \
  template void amg_cast_in<T>(const double*, T*, int64_t, int, hipStream_t, const int32_t*);             \
  template void amg_cast_out<T>(const T*, double*, int64_t, int, hipStream_t, const int32_t*);            \
  template void amg_cheb_start0<T>(const DevCsr&, const AmgDiag<T>&, T*, T*, T*, T*, T, int, hipStream_t, \
                                   const int32_t*, const double*);                                        \
  template void amg_cheb_start<T>(const DevCsr&, const AmgDiag<T>&, const T*, T*, T*, T*, T, int,         \
                                  hipStream_t, const int32_t*, bool, double*);                            \
  template void amg_cheb_step<T>(const DevCsr&, const AmgDiag<T>&, const T*, T*, T*, T*, T, T, int,       \
                                 hipStream_t, const int32_t*, bool, double*);                             \
  template void amg_residual<T>(const DevCsr&, const AmgDiag<T>&, const T*, const T*, T*, int,            \
                                hipStream_t, const int32_t*);                                             \
  template void amg_spmv<T>(const DevCsr&, const T*, T*, bool, int, hipStream_t, const int32_t*);         \
  template void amg_dense<T>(const T*, const T*, T*, int, int, hipStream_t, const int32_t*);              \
  template void amg_dense_chunked<T>(const T*, const T*, T*, T*, int, int, hipStream_t, const int32_t*);  \
  template void amg_sym_from_lower<T>(const double*, T*, int, hipStream_t);                               \
  template void amg_diag_solve<T>(const T*, const T*, T*, int, int, hipStream_t, const int32_t*);

JFNK_AMG_INSTANTIATE(float)
JFNK_AMG_INSTANTIATE(double)

}  // namespace jfnk
