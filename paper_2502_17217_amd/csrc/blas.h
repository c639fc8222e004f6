// Launchers of the Krylov vector kernels (blas.hip).  All pointers are
// device pointers; all calls are asynchronous on stream s.
//
// Vectors are internal vectors of a mesh or batch: component-major
// [dim][n_cells] over the union numbering.  Reductions are per segment:
// every workgroup sums one tile of kFvBlock cells (all components) in a
// fixed order, and one workgroup per segment then sums that segment's tiles
// in order, so a segment's result depends only on its own values.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace jfnk {

constexpr int kMaxBasis = 256;  // max restart length + 1 supported by the kernels

struct SegLayout {
  int32_t n_cells = 0;               // union cells (N); a vector has dim * N entries
  int32_t dim = 0;
  int32_t n_seg = 0;
  int32_t n_blocks = 0;              // tiles of kFvBlock cells
  const int32_t* seg_of_block = nullptr;
  const int32_t* block_first = nullptr;  // [n_seg + 1]
};

// out[s * ldo + k] (+)= V_k . w restricted to segment s, k < nk (V_k = V + k*ldv).
// partials: n_blocks * kMaxBasis doubles.  Segments with active[s] == 0 are skipped.
void blas_mdot(const SegLayout& L, const double* V, int64_t ldv, int nk, const double* w, double* partials,
               double* out, int ldo, bool accumulate, const int32_t* active, hipStream_t s);
// w += sign * sum_{k<nk} h[s * ldh + k] V_k on each segment s (k < min(nk, nk_seg[s]) when
// nk_seg is given)
void blas_combine(const SegLayout& L, const double* V, int64_t ldv, int nk, const double* h, int ldh,
                  double sign, double* w, const int32_t* active, hipStream_t s,
                  const int32_t* nk_seg = nullptr);
// the same over a basis stored in FP32
void blas_combine(const SegLayout& L, const float* V, int64_t ldv, int nk, const double* h, int ldh,
                  double sign, double* w, const int32_t* active, hipStream_t s,
                  const int32_t* nk_seg = nullptr);
// zf = z rounded to FP32 (to nearest); back: also z = double(zf).  Skipped
// entirely when gate is given and *gate == 0.
void blas_round_fp32(double* z, float* zf, int64_t n, bool back, hipStream_t s, const int32_t* gate = nullptr);
// y = scale[s] * x on each segment s
void blas_scale_seg(const SegLayout& L, const double* x, const double* scale, double* y,
                    const int32_t* active, hipStream_t s);
// y = a x + b y (all entries)
void blas_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
// y = a x + b z (all entries)
void blas_lincomb(double a, const double* x, double b, const double* z, double* y, int64_t n,
                  hipStream_t s);
// ---- fused reductions (cgs_kernels.hip) ----
void fill_int(int32_t* d, int n, int32_t v, hipStream_t s);
// One launch: tickets[0..nt) = 0 and load[0..S) = value.
void call_setup(int32_t* tickets, int nt, double* load, int S, double value, hipStream_t s);
// true if some segment has more tiles than the in-kernel finish handles
bool any_large_segment(const SegLayout& L, const int32_t* h_block_first);
// eps[s] = sqrt(eps_mach) sqrt(1 + |u_s|) / |v_s| per active segment; uu
// (may be null): |u_s|^2 already known, at uu[s * ldu] (u is then not read)
void launch_eps_fused(const SegLayout& L, bool any_large, const double* u, const double* uu, int ldu,
                      const double* v, const int32_t* act, double* partials, int32_t* tickets, double* eps,
                      hipStream_t s);
struct GmresDev;
// Both classical Gram-Schmidt passes of Arnoldi step j against V_0..V_{nk-1}
// and the device Givens update (h, h2: [n_seg][kMaxBasis], nrm: [n_seg][4]).
void cgs2_step(const SegLayout& L, bool any_large, const double* V, int64_t ldv, int nk, double* w,
               double* h, double* h2, double* nrm, double* partials, int32_t* tickets, int32_t* counters,
               const GmresDev& G, int j, int max_it, hipStream_t s);

// Arnoldi step j with delayed reorthogonalisation (DCGS2): V_j holds the
// previous step's vector orthogonalised once (unit computed norm), w = J z_j.
// Completes Hessenberg column j-1 (its Givens step included), writes the
// final v_j into V_j, orthogonalises w once against V_0..V_j (first-pass
// column j) and leaves 1/|w| in G.fac for scaling w into V_{j+1}.
// closing: only the completion of column j-1 (end of a cycle, j = restart).
// partials2: a second region of n_blocks * kMaxBasis doubles.
void dcgs_step(const SegLayout& L, bool any_large, double* V, int64_t ldv, int j, double* w, double* h, double* h2,
               double* nrm, double* partials, double* partials2, int32_t* tickets, const GmresDev& G, int max_it,
               bool closing, hipStream_t s);

// eps[s] *= factor, eps_neg[s] = -eps[s] (central-difference step)
void blas_central_eps(double* eps, double* eps_neg, int S, double factor, hipStream_t s);
// z = D^{-1} r with one scalar per cell applied to every component, or one
// per cell and component when per_comp (dinv [dim][n_cells]); skipped
// entirely when gate is given and *gate == 0
void blas_jacobi(const double* dinv, const double* r, double* z, int64_t n_cells, int dim, bool per_comp,
                 hipStream_t s, const int32_t* gate = nullptr);

}  // namespace jfnk
