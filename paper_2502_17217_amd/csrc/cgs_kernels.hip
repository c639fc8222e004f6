// Fused kernels of one Arnoldi step's classical Gram-Schmidt (applied twice)
// and of the J v step size (Section 3.2, Eq. JF), gfx950.
//
// One workgroup per tile of kFvBlock cells.  A pass computes its tile's
// partial sums and, for segments of at most kFuseTiles tiles, the last tile
// of the segment to finish adds the segment's partials (one tile per lane,
// fixed wavefront reduction) and writes the result, so a whole pass is one launch.  Larger segments leave
// their partials to a separate reduction launch (k_reduce_large), spread
// over one workgroup per (column, segment).  Which of the two a segment
// takes depends only on its own size, so a mesh gets the same bits alone
// and inside a batch.
//
//   pass 1: h = V^T w and |w|^2 (before orthogonalisation)
//   pass 2: w -= V h, then h2 = V^T w
//   pass 3: w -= V h2, then |w|^2, and (when every segment is small) the
//           device Givens update of each segment in its last tile.
// and the two passes of the delayed-reorthogonalisation variant (DCGS2).
#include "blas.h"
#include "gmres_step_dev.h"
#include "reduce_dev.h"

namespace jfnk {

namespace {

__device__ __forceinline__ bool small_segment(const SegLayout& L, int seg, int& first, int& n) {
  first = L.block_first[seg];
  n = L.block_first[seg + 1] - first;
  return n <= kFuseTiles;
}

// w -= sum_k coef[k] V_k on cell c of the tile (all D components at once;
// each component's sum runs over k in order)
template <int D>
__device__ __forceinline__ void combine_cell(const SegLayout& L, const double* __restrict__ V, int64_t ldv,
                                             int nk, const double* __restrict__ coef, double* __restrict__ w,
                                             int c) {
  double s[D];
#pragma unroll
  for (int q = 0; q < D; ++q) s[q] = 0.0;
  for (int k = 0; k < nk; ++k) {
    const double ck = coef[k];
#pragma unroll
    for (int q = 0; q < D; ++q) s[q] = fma(ck, V[k * ldv + size_t(q) * L.n_cells + c], s[q]);
  }
#pragma unroll
  for (int q = 0; q < D; ++q) w[size_t(q) * L.n_cells + c] -= s[q];
}

// Tile sums of V_k . w (k < nk): per-wavefront sums go to
// wsum[wave][k] (store_tile_sums adds the four wavefronts in fixed order).
template <int D>
__device__ __forceinline__ void tile_dots(const SegLayout& L, const double* __restrict__ V, int64_t ldv,
                                          int nk, const double* __restrict__ w, int c,
                                          double (*wsum)[kMaxBasis]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double wi[D];
#pragma unroll
  for (int q = 0; q < D; ++q) wi[q] = c < L.n_cells ? w[size_t(q) * L.n_cells + c] : 0.0;
  for (int k0 = 0; k0 < nk; k0 += 8) {
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0;
    if (c < L.n_cells) {
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const size_t o = size_t(q) * L.n_cells + c;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k0 + k < nk) acc[k] = fma(V[(k0 + k) * ldv + o], wi[q], acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k0 + k < nk) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) wsum[wave][k0 + k] = s;
      }
  }
}

// Tile partial sums are stored column-major, partials[col * n_blocks + tile],
// so that a segment's tiles of one column are contiguous.
__device__ __forceinline__ size_t pidx(const SegLayout& L, int col, int tile) {
  return size_t(col) * L.n_blocks + tile;
}

// Segment sum of partial column col over tiles first .. first+n-1 (n <= 64),
// one tile per lane and the fixed wavefront reduction; valid in every lane.
__device__ __forceinline__ double segment_column_sum(const SegLayout& L, const double* __restrict__ partials,
                                                     int first, int n, int col) {
  const int lane = threadIdx.x & 63;
  const double x = lane < n ? partials[pidx(L, col, first + lane)] : 0.0;
  return wave_sum(x);
}

// |w|^2 over the tile's cells: per-wavefront sums into wsum[wave][col].
template <int D>
__device__ __forceinline__ void tile_norm2(const SegLayout& L, const double* __restrict__ w, int c,
                                           double (*wsum)[kMaxBasis], int col) {
  double s = 0;
  if (c < L.n_cells) {
    double x[D];
#pragma unroll
    for (int q = 0; q < D; ++q) x[q] = w[size_t(q) * L.n_cells + c];
#pragma unroll
    for (int q = 0; q < D; ++q) s = fma(x[q], x[q], s);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6][col] = s;
}

// partials[blk][k] = fixed-order sum of the four wavefront sums, k < ncol
// (after a barrier).
__device__ __forceinline__ void store_tile_sums(const SegLayout& L, double (*wsum)[kMaxBasis], int ncol,
                                                double* __restrict__ partials, int blk) {
  __syncthreads();
  for (int k = threadIdx.x; k < ncol; k += kBlock)
    partials[pidx(L, k, blk)] = ((wsum[0][k] + wsum[1][k]) + wsum[2][k]) + wsum[3][k];
}

// Passes 1 and 2.  coef == nullptr: pass 1 (also |w|^2 into column nk,
// finished into nrm[4 seg + 1]); otherwise pass 2 (w -= V coef first).
template <int D>
__global__ __launch_bounds__(kBlock) void k_cgs_pass(SegLayout L, const double* __restrict__ V, int64_t ldv,
                                                     int nk, double* __restrict__ w,
                                                     const double* __restrict__ coef,
                                                     const int32_t* __restrict__ act,
                                                     double* __restrict__ partials, int32_t* __restrict__ tickets,
                                                     double* __restrict__ out, double* __restrict__ nrm) {
  __shared__ double wsum[4][kMaxBasis];
  const int blk = blockIdx.x;
  const int seg = L.seg_of_block[blk];
  if (act != nullptr && act[seg] == 0) return;
  const int c = blk * kFvBlock + threadIdx.x;
  if (coef != nullptr && c < L.n_cells) combine_cell<D>(L, V, ldv, nk, coef + size_t(seg) * kMaxBasis, w, c);
  tile_dots<D>(L, V, ldv, nk, w, c, wsum);
  const int ncol = coef == nullptr ? nk + 1 : nk;
  if (coef == nullptr) tile_norm2<D>(L, w, c, wsum, nk);
  store_tile_sums(L, wsum, ncol, partials, blk);
  int first, n;
  if (!small_segment(L, seg, first, n)) return;
  if (!last_tile_of_segment(tickets + seg, n)) return;
  // each wavefront finishes every fourth column
  const int wave = threadIdx.x >> 6;
  for (int k = wave; k < ncol; k += 4) {
    const double t = segment_column_sum(L, partials, first, n, k);
    if ((threadIdx.x & 63) == 0) {
      if (k < nk)
        out[size_t(seg) * kMaxBasis + k] = t;
      else
        nrm[4 * seg + 1] = t;
    }
  }
}

// Pass 3: w -= V h2, |w|^2 into nrm[4 seg]; with finish != 0 (every segment
// small) the last tile of each segment also takes the Givens step, and the
// last segment to finish publishes the count of segments still active.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cgs_last(SegLayout L, const double* __restrict__ V, int64_t ldv,
                                                     int nk, double* __restrict__ w,
                                                     const double* __restrict__ h1, const double* __restrict__ h2,
                                                     const int32_t* __restrict__ act_in,
                                                     double* __restrict__ partials, int32_t* __restrict__ tickets,
                                                     int32_t* __restrict__ counters, double* __restrict__ nrm,
                                                     GmresDev G, int j, int max_it, int finish) {
  __shared__ double wsum[4][kMaxBasis];
  const int blk = blockIdx.x;
  const int seg = L.seg_of_block[blk];
  if (act_in[seg] == 0) return;
  const int c = blk * kFvBlock + threadIdx.x;
  if (c < L.n_cells) combine_cell<D>(L, V, ldv, nk, h2 + size_t(seg) * kMaxBasis, w, c);
  tile_norm2<D>(L, w, c, wsum, 0);
  store_tile_sums(L, wsum, 1, partials, blk);
  int first, n;
  if (!small_segment(L, seg, first, n)) return;
  if (!last_tile_of_segment(tickets + seg, n)) return;
  if (threadIdx.x >= 64) return;
  const double t = segment_column_sum(L, partials, first, n, 0);
  if (threadIdx.x != 0) return;
  nrm[4 * seg] = t;
  if (!finish) return;
  // segments taking this step = the active count published by the previous step
  const int taking = G.nact[0];
  const int a = givens_update(G, seg, j, max_it, h1 + size_t(seg) * kMaxBasis, h2 + size_t(seg) * kMaxBasis,
                              t, nrm[4 * seg + 1]);
  atomicAdd(counters + 1, a);
  __threadfence();
  if (atomicAdd(counters, 1) == taking - 1) {
    G.nact[0] = atomicAdd(counters + 1, 0);
    counters[0] = 0;
    counters[1] = 0;
  }
}

// ---- Gram-Schmidt with delayed reorthogonalisation (DCGS2) ----
// Step j holds u = V_j, the basis vector of step j-1 orthogonalised once
// and scaled to unit computed norm, and w = J z_j.  One read of V_0..V_j
// gives the dots of both u and w against V_0..V_{j-1}; u's second
// orthogonalisation u = alpha v_j + V a then completes column j-1 of the
// Hessenberg matrix, and a second read forms v_j and w's first
// orthogonalisation together.  Two reads of the basis per step instead of
// four; the Givens step of column j-1 is taken in step j, and a closing
// pass (dots of V_m only) completes the last column of a cycle.

// Pass 1 of step j: tile sums of a_k = V_k . u and b_k = V_k . w (k < j),
// c = u . w, d = u . u and |w|^2, from one read of V_0..V_j.  Columns: a,
// then c, d, |w|^2 at j, j+1, j+2 of partials; b at 0..j-1 of partials2.
// The last tile of a small segment finishes them into h[seg] and h2[seg].
// w == null (closing pass): a and d only.
template <int D>
__global__ __launch_bounds__(kBlock) void k_dcgs_dots(SegLayout L, const double* __restrict__ V, int64_t ldv,
                                                      int j, const double* __restrict__ w,
                                                      const int32_t* __restrict__ act,
                                                      double* __restrict__ partials,
                                                      double* __restrict__ partials2,
                                                      int32_t* __restrict__ tickets, double* __restrict__ h,
                                                      double* __restrict__ h2) {
  __shared__ double wa[4][kMaxBasis];
  __shared__ double wb[4][kMaxBasis];
  const int blk = blockIdx.x;
  const int seg = L.seg_of_block[blk];
  if (act[seg] == 0) return;
  const int c = blk * kFvBlock + threadIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool in = c < L.n_cells;
  const bool has_w = w != nullptr;
  double ui[D], wi[D];
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * L.n_cells + c;
    ui[q] = in ? V[j * ldv + o] : 0.0;
    wi[q] = (in && has_w) ? w[o] : 0.0;
  }
  for (int k0 = 0; k0 < j; k0 += 8) {
    double aa[8], bb[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) aa[k] = bb[k] = 0.0;
    if (in) {
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const size_t o = size_t(q) * L.n_cells + c;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k0 + k < j) {
            const double x = V[(k0 + k) * ldv + o];
            aa[k] = fma(x, ui[q], aa[k]);
            bb[k] = fma(x, wi[q], bb[k]);
          }
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k0 + k < j) {
        const double sa = wave_sum(aa[k]);
        const double sb = has_w ? wave_sum(bb[k]) : 0.0;
        if (lane == 0) {
          wa[wave][k0 + k] = sa;
          wb[wave][k0 + k] = sb;
        }
      }
  }
  double cu = 0.0, du = 0.0, ww = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    cu = fma(ui[q], wi[q], cu);
    du = fma(ui[q], ui[q], du);
    ww = fma(wi[q], wi[q], ww);
  }
  cu = wave_sum(cu);
  du = wave_sum(du);
  ww = wave_sum(ww);
  if (lane == 0) {
    wa[wave][j] = cu;
    wa[wave][j + 1] = du;
    wa[wave][j + 2] = ww;
  }
  store_tile_sums(L, wa, j + 3, partials, blk);
  store_tile_sums(L, wb, j, partials2, blk);
  int first, n;
  if (!small_segment(L, seg, first, n)) return;
  if (!last_tile_of_segment(tickets + seg, n)) return;
  // each wavefront finishes every fourth column
  for (int k = wave; k < 2 * j + 3; k += 4) {
    const bool A = k < j + 3;
    const double t = segment_column_sum(L, A ? partials : partials2, first, n, A ? k : k - (j + 3));
    if (lane == 0) {
      if (A)
        h[size_t(seg) * kMaxBasis + k] = t;
      else
        h2[size_t(seg) * kMaxBasis + k - (j + 3)] = t;
    }
  }
}

// Step j, one wavefront per segment, from a, c, d, |w|^2 (h[s]) and b
// (h2[s]).  For j > 0: alpha = sqrt(d - |a|^2) completes column j-1 (rows
// += sigma a, subdiagonal sigma alpha, sigma its first-pass subdiagonal) and
// takes its Givens step; d <= |a|^2 means u lies in the span of the basis (a
// breakdown: subdiagonal 0, the segment stops).  Then, unless the segment
// stops or last (closing pass), the first-pass column j (rows b, diagonal
// h_jj = (c - a.b) / alpha), with alpha and h_jj kept in nrm[4s+2],
// nrm[4s+3] for the update pass.  Step 0 has nothing to complete: alpha = 1,
// h_00 = c.  The dot products |a|^2 and a.b are lane-strided sums reduced in
// the fixed wavefront order; the Givens rotations of column j-1 run in one
// lane on a copy in LDS.
__global__ __launch_bounds__(64) void k_dcgs_finalize(GmresDev G, int j, int max_it, const double* __restrict__ h,
                                                      const double* __restrict__ h2, double* __restrict__ nrm,
                                                      int last) {
  __shared__ double col[kMaxBasis + 1];
  __shared__ double cl[kMaxBasis], sl[kMaxBasis];
  __shared__ int go;
  const int s = blockIdx.x, lane = threadIdx.x;
  if (G.act[s] == 0) return;
  const int mr = G.mr;
  const double* a = h + size_t(s) * kMaxBasis;
  const double* b = h2 + size_t(s) * kMaxBasis;
  const double cu = a[j], du = a[j + 1], ww = a[j + 2];
  if (!isfinite(du) || (!last && (!isfinite(cu) || !isfinite(ww)))) {
    if (lane == 0) segment_stop(G, s, true);
    return;
  }
  double pa = 0.0, pb = 0.0;
  for (int i = lane; i < j; i += 64) {
    pa = fma(a[i], a[i], pa);
    pb = fma(a[i], b[i], pb);
  }
  const double aa = wave_sum(pa), ab = wave_sum(pb);
  double alpha = 1.0;
  if (j > 0) {
    const double rem = du - aa;
    const bool in_span = !(rem > 0.0);
    alpha = in_span ? 0.0 : sqrt(rem);
    double* Hp = G.H + (size_t(s) * mr + j - 1) * (mr + 1);
    const double sigma = Hp[j];
    for (int i = lane; i < j; i += 64) col[i] = fma(sigma, a[i], Hp[i]);
    for (int i = lane; i < j - 1; i += 64) {
      cl[i] = G.cs[size_t(s) * mr + i];
      sl[i] = G.sn[size_t(s) * mr + i];
    }
    if (lane == 0) col[j] = sigma * alpha;
    __syncthreads();
    if (lane == 0) {
      // the rotations of columns 0..j-2, then column j-1's own
      const int c0 = j - 1;
      for (int i = 0; i < c0; ++i) {
        const double t = cl[i] * col[i] + sl[i] * col[i + 1];
        col[i + 1] = -sl[i] * col[i] + cl[i] * col[i + 1];
        col[i] = t;
      }
      double* g = G.g + size_t(s) * (mr + 1);
      const double rr = hypot(col[c0], col[c0 + 1]);
      const double cn = col[c0] / rr, sn = col[c0 + 1] / rr;
      G.cs[size_t(s) * mr + c0] = cn;
      G.sn[size_t(s) * mr + c0] = sn;
      col[c0] = rr;
      col[c0 + 1] = 0.0;
      g[c0 + 1] = -sn * g[c0];
      g[c0] = cn * g[c0];
      G.its[s] += 1;
      G.kk[s] = c0 + 1;
      const bool more = !(fabs(g[c0 + 1]) <= G.target[s] || G.its[s] >= max_it);
      go = more && !in_span;
      if (!go) segment_stop(G, s, false);
    }
    __syncthreads();
    for (int i = lane; i <= j; i += 64) Hp[i] = col[i];
    if (!go) return;
  }
  if (last) return;
  const double hjj = (cu - ab) / alpha;
  double* Hj = G.H + (size_t(s) * mr + j) * (mr + 1);
  for (int i = lane; i < j; i += 64) Hj[i] = b[i];
  if (lane == 0) {
    Hj[j] = hjj;
    nrm[4 * s + 2] = alpha;
    nrm[4 * s + 3] = hjj;
  }
}

// Pass 2 of step j: v_j = (u - V a) / alpha into V_j and w = w - V b - h_jj v_j
// from one read of V_0..V_{j-1}, then the tile sums of |w|^2 (column 0),
// finished into nrm[4 seg] for a small segment.
template <int D>
__global__ __launch_bounds__(kBlock) void k_dcgs_update(SegLayout L, double* __restrict__ V, int64_t ldv, int j,
                                                        double* __restrict__ w, const double* __restrict__ h,
                                                        const double* __restrict__ h2,
                                                        double* __restrict__ nrm, const int32_t* __restrict__ act,
                                                        double* __restrict__ partials,
                                                        int32_t* __restrict__ tickets) {
  __shared__ double wsum[4][kMaxBasis];
  const int blk = blockIdx.x;
  const int seg = L.seg_of_block[blk];
  if (act[seg] == 0) return;
  const int c = blk * kFvBlock + threadIdx.x;
  if (c < L.n_cells) {
    const double* a = h + size_t(seg) * kMaxBasis;
    const double* b = h2 + size_t(seg) * kMaxBasis;
    double sa[D], sb[D];
#pragma unroll
    for (int q = 0; q < D; ++q) sa[q] = sb[q] = 0.0;
    for (int k = 0; k < j; ++k) {
      const double ak = a[k], bk = b[k];
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const double x = V[k * ldv + size_t(q) * L.n_cells + c];
        sa[q] = fma(ak, x, sa[q]);
        sb[q] = fma(bk, x, sb[q]);
      }
    }
    const double alpha = nrm[4 * seg + 2], hjj = nrm[4 * seg + 3];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const size_t o = size_t(q) * L.n_cells + c;
      const double v = (V[j * ldv + o] - sa[q]) / alpha;
      V[j * ldv + o] = v;
      w[o] = fma(-hjj, v, w[o] - sb[q]);
    }
  }
  tile_norm2<D>(L, w, c, wsum, 0);
  store_tile_sums(L, wsum, 1, partials, blk);
  int first, n;
  if (!small_segment(L, seg, first, n)) return;
  if (!last_tile_of_segment(tickets + seg, n)) return;
  if (threadIdx.x >= 64) return;
  const double t = segment_column_sum(L, partials, first, n, 0);
  if (threadIdx.x == 0) nrm[4 * seg] = t;
}

// End of step j per segment (one workgroup over all segments): sigma = |w|
// is the first-pass subdiagonal of column j (completed by step j + 1) and
// 1/sigma scales w into u_{j+1}; sigma negligible against |w| before the
// pass (a breakdown) completes column j as it stands and stops the segment.
// Publishes the count of segments still taking steps.
__global__ __launch_bounds__(kBlock) void k_dcgs_step_end(GmresDev G, int S, int j, int max_it,
                                                          const double* __restrict__ h,
                                                          const double* __restrict__ nrm) {
  __shared__ int count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  const int mr = G.mr;
  for (int s = threadIdx.x; s < S; s += kBlock) {
    if (G.act[s] == 0) {
      G.fac[s] = 0.0;
      continue;
    }
    const double sigma = sqrt(nrm[4 * s]);
    const double w0 = sqrt(h[size_t(s) * kMaxBasis + j + 2]);
    double* Hj = G.H + (size_t(s) * mr + j) * (mr + 1);
    Hj[j + 1] = sigma;
    if (!isfinite(sigma)) {
      segment_stop(G, s, true);
      continue;
    }
    if (sigma <= 1e-14 * fmax(w0, 1e-300)) {
      (void)givens_apply(G, s, j, max_it);
      segment_stop(G, s, false);
      continue;
    }
    G.fac[s] = 1.0 / sigma;
    atomicAdd(&count, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) G.nact[0] = count;
}

// Segment sums of partial columns col0 .. col0+ncol-1 for segments larger
// than kFuseTiles: out[seg * ldo + k].
// This thread's share of a large segment's column: tiles first + threadIdx.x,
// + kBlock, + 2 kBlock, ... added in that order; the loads of eight
// consecutive terms are issued together (the order of the additions is
// unchanged).
template <int B>
__device__ __forceinline__ double strided_column_sum(const SegLayout& L, const double* __restrict__ partials,
                                                     int col, int first, int n) {
  constexpr int kU = 8;
  double s = 0;
  int b = first + threadIdx.x;
  for (; b + (kU - 1) * B < first + n; b += kU * B) {
    double x[kU];
#pragma unroll
    for (int i = 0; i < kU; ++i) x[i] = partials[pidx(L, col, b + i * B)];
#pragma unroll
    for (int i = 0; i < kU; ++i) s += x[i];
  }
  for (; b < first + n; b += B) s += partials[pidx(L, col, b)];
  return s;
}

// Sum over a kWideBlock-thread workgroup (16 wavefronts in fixed order);
// valid in thread 0.
constexpr int kWideBlock = 1024;
__device__ __forceinline__ double wide_block_sum(double x, double* sh) {
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kWideBlock / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kWideBlock) void k_reduce_large(SegLayout L, const double* __restrict__ partials,
                                                             int col0, const int32_t* __restrict__ act,
                                                             double* __restrict__ out, int ldo) {
  __shared__ double sh[kWideBlock / 64];
  const int k = blockIdx.x, seg = blockIdx.y;
  if (act != nullptr && act[seg] == 0) return;
  int first, n;
  if (small_segment(L, seg, first, n)) return;
  double s = strided_column_sum<kWideBlock>(L, partials, col0 + k, first, n);
  s = wide_block_sum(s, sh);
  if (threadIdx.x == 0) out[size_t(seg) * ldo + k] = s;
}

// J v step size, fused: tile sums of |u|^2 and |v|^2 (columns 0 and 1 of the
// tile's partial row) and, for small segments, eps in the last tile:
// eps = sqrt(eps_mach) sqrt(1 + |u|) / |v| (0 when v = 0).
#ifndef JFNK_EPS_TILES
#define JFNK_EPS_TILES 4
#endif
constexpr int kEpsTiles = JFNK_EPS_TILES;  // tiles a workgroup of the step-size kernel sums at once

__device__ __forceinline__ double eps_of(double uu, double vv) {
  const double sqrt_eps = 1.4901161193847656e-08;
  return vv > 0 ? sqrt_eps * sqrt(1.0 + sqrt(uu)) / sqrt(vv) : 0.0;
}

// Step size of J v per segment (Eq. JF): tile partials of |u|^2 and |v|^2;
// for a small segment the last of its tiles to finish adds them (one tile
// per lane) and writes eps, a large one is finished by k_eps_large (no
// arrival counter shared by thousands of tiles).  A workgroup sums
// kEpsTiles tiles at once, every load issued before the first sum (each
// tile's partial formed as tile_norm2 forms it).  kCachedU: |u|^2 of each
// segment is given (uu[seg * ldu], u fixed over a linear solve) and u is not
// read.
template <int D, bool kCachedU>
__global__ __launch_bounds__(kBlock) void k_eps_tiles(SegLayout L, const double* __restrict__ u,
                                                      const double* __restrict__ uu, int ldu,
                                                      const double* __restrict__ v,
                                                      const int32_t* __restrict__ act,
                                                      double* __restrict__ partials, int32_t* __restrict__ tickets,
                                                      double* __restrict__ eps) {
  __shared__ double wsum[4][2 * kEpsTiles];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = L.n_cells;
  for (int b0 = blockIdx.x * kEpsTiles; b0 < L.n_blocks; b0 += gridDim.x * kEpsTiles) {
    double x[kEpsTiles][D], y[kEpsTiles][D];
#pragma unroll
    for (int j = 0; j < kEpsTiles; ++j) {
      const int blk = b0 + j;
      const int c = blk * kFvBlock + threadIdx.x;
      const bool on = blk < L.n_blocks && c < n && (act == nullptr || act[L.seg_of_block[blk]] != 0);
#pragma unroll
      for (int q = 0; q < D; ++q) {
        x[j][q] = (on && !kCachedU) ? u[size_t(q) * n + c] : 0.0;
        y[j][q] = on ? v[size_t(q) * n + c] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < kEpsTiles; ++j) {
      double su = 0.0, sv = 0.0;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        su = fma(x[j][q], x[j][q], su);
        sv = fma(y[j][q], y[j][q], sv);
      }
      su = wave_sum(su);
      sv = wave_sum(sv);
      if (lane == 0) {
        wsum[wave][2 * j] = su;
        wsum[wave][2 * j + 1] = sv;
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kEpsTiles) {
      const int j = threadIdx.x >> 1, blk = b0 + j;
      if (blk < L.n_blocks && (act == nullptr || act[L.seg_of_block[blk]] != 0))
        partials[pidx(L, threadIdx.x & 1, blk)] =
            ((wsum[0][threadIdx.x] + wsum[1][threadIdx.x]) + wsum[2][threadIdx.x]) + wsum[3][threadIdx.x];
    }
    for (int j = 0; j < kEpsTiles; ++j) {
      const int blk = b0 + j;
      if (blk >= L.n_blocks) break;
      const int seg = L.seg_of_block[blk];
      if (act != nullptr && act[seg] == 0) continue;
      int first, cnt;
      if (small_segment(L, seg, first, cnt) && last_tile_of_segment(tickets + seg, cnt) && threadIdx.x < 64) {
        const double tu = kCachedU ? uu[size_t(seg) * ldu] : segment_column_sum(L, partials, first, cnt, 0);
        const double tv = segment_column_sum(L, partials, first, cnt, 1);
        if (threadIdx.x == 0) eps[seg] = eps_of(tu, tv);
      }
    }
    __syncthreads();  // wsum is rewritten by the next round
  }
}

// Large segments, one workgroup of kWideBlock threads each: tile b to
// thread (b - first) mod kWideBlock, then a fixed tree.
__global__ __launch_bounds__(kWideBlock) void k_eps_large(SegLayout L, const double* __restrict__ partials,
                                                          const double* __restrict__ uu, int ldu,
                                                          const int32_t* __restrict__ act,
                                                          double* __restrict__ eps) {
  __shared__ double sh[kWideBlock / 64];
  const int seg = blockIdx.x;
  if (act != nullptr && act[seg] == 0) return;
  int first, n;
  if (small_segment(L, seg, first, n)) return;
  double su = uu != nullptr ? 0.0 : strided_column_sum<kWideBlock>(L, partials, 0, first, n);
  double sv = strided_column_sum<kWideBlock>(L, partials, 1, first, n);
  su = uu != nullptr ? uu[size_t(seg) * ldu] : wide_block_sum(su, sh);
  sv = wide_block_sum(sv, sh);
  if (threadIdx.x == 0) eps[seg] = eps_of(su, sv);
}

// Per-call set-up of a workspace: arrival counters to zero, the load factor
// of every segment.
__global__ void k_call_setup(int32_t* __restrict__ tickets, int nt, double* __restrict__ load, int S,
                             double value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nt) tickets[i] = 0;
  if (i < S) load[i] = value;
}

__global__ void k_fill_int(int32_t* d, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = v;
}

}  // namespace

bool any_large_segment(const SegLayout& L, const int32_t* h_block_first) {
  for (int s = 0; s < L.n_seg; ++s)
    if (h_block_first[s + 1] - h_block_first[s] > kFuseTiles) return true;
  return false;
}

void call_setup(int32_t* tickets, int nt, double* load, int S, double value, hipStream_t s) {
  const int n = nt > S ? nt : S;
  hipLaunchKernelGGL(k_call_setup, dim3((n + 255) / 256), dim3(256), 0, s, tickets, nt, load, S, value);
  JFNK_HIP(hipGetLastError());
}

void fill_int(int32_t* d, int n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, d, n, v);
  JFNK_HIP(hipGetLastError());
}

void launch_eps_fused(const SegLayout& L, bool any_large, const double* u, const double* uu, int ldu,
                      const double* v, const int32_t* act, double* partials, int32_t* tickets, double* eps,
                      hipStream_t s) {
  const int grid = (L.n_blocks + kEpsTiles - 1) / kEpsTiles;
  if (uu != nullptr) {
    if (L.dim == 3)
      hipLaunchKernelGGL((k_eps_tiles<3, true>), dim3(grid), dim3(kBlock), 0, s, L, u, uu, ldu, v, act, partials,
                         tickets, eps);
    else
      hipLaunchKernelGGL((k_eps_tiles<2, true>), dim3(grid), dim3(kBlock), 0, s, L, u, uu, ldu, v, act, partials,
                         tickets, eps);
  } else {
    if (L.dim == 3)
      hipLaunchKernelGGL((k_eps_tiles<3, false>), dim3(grid), dim3(kBlock), 0, s, L, u, uu, ldu, v, act, partials,
                         tickets, eps);
    else
      hipLaunchKernelGGL((k_eps_tiles<2, false>), dim3(grid), dim3(kBlock), 0, s, L, u, uu, ldu, v, act, partials,
                         tickets, eps);
  }
  if (any_large)
    hipLaunchKernelGGL(k_eps_large, dim3(L.n_seg), dim3(kWideBlock), 0, s, L, partials, uu, ldu, act, eps);
  JFNK_HIP(hipGetLastError());
}

void cgs2_step(const SegLayout& L, bool any_large, const double* V, int64_t ldv, int nk, double* w,
               double* h, double* h2, double* nrm, double* partials, int32_t* tickets, int32_t* counters,
               const GmresDev& G, int j, int max_it, hipStream_t s) {
  const int32_t* act = G.act;
  const dim3 g(L.n_blocks), b(kBlock), wide(kWideBlock);
  const bool d3 = L.dim == 3;
  // pass 1
  if (d3)
    hipLaunchKernelGGL(k_cgs_pass<3>, g, b, 0, s, L, V, ldv, nk, w, nullptr, act, partials, tickets, h, nrm);
  else
    hipLaunchKernelGGL(k_cgs_pass<2>, g, b, 0, s, L, V, ldv, nk, w, nullptr, act, partials, tickets, h, nrm);
  if (any_large) {
    hipLaunchKernelGGL(k_reduce_large, dim3(nk, L.n_seg), wide, 0, s, L, partials, 0, act, h, kMaxBasis);
    hipLaunchKernelGGL(k_reduce_large, dim3(1, L.n_seg), wide, 0, s, L, partials, nk, act, nrm + 1, 4);
  }
  // pass 2
  if (d3)
    hipLaunchKernelGGL(k_cgs_pass<3>, g, b, 0, s, L, V, ldv, nk, w, h, act, partials, tickets, h2, nrm);
  else
    hipLaunchKernelGGL(k_cgs_pass<2>, g, b, 0, s, L, V, ldv, nk, w, h, act, partials, tickets, h2, nrm);
  if (any_large)
    hipLaunchKernelGGL(k_reduce_large, dim3(nk, L.n_seg), wide, 0, s, L, partials, 0, act, h2, kMaxBasis);
  // pass 3 (+ Givens when every segment is small)
  if (d3)
    hipLaunchKernelGGL(k_cgs_last<3>, g, b, 0, s, L, V, ldv, nk, w, h, h2, act, partials, tickets, counters, nrm, G,
                       j, max_it, any_large ? 0 : 1);
  else
    hipLaunchKernelGGL(k_cgs_last<2>, g, b, 0, s, L, V, ldv, nk, w, h, h2, act, partials, tickets, counters, nrm, G,
                       j, max_it, any_large ? 0 : 1);
  if (any_large) {
    hipLaunchKernelGGL(k_reduce_large, dim3(1, L.n_seg), wide, 0, s, L, partials, 0, act, nrm, 4);
    gmres_step_finish(G, L.n_seg, j, max_it, h, h2, nrm, s);
  }
  JFNK_HIP(hipGetLastError());
}

void dcgs_step(const SegLayout& L, bool any_large, double* V, int64_t ldv, int j, double* w, double* h, double* h2,
               double* nrm, double* partials, double* partials2, int32_t* tickets, const GmresDev& G, int max_it,
               bool closing, hipStream_t s) {
  const int32_t* act = G.act;
  const dim3 g(L.n_blocks), b(kBlock), wide(kWideBlock);
  const bool d3 = L.dim == 3;
  const double* wd = closing ? nullptr : w;
  if (d3)
    hipLaunchKernelGGL(k_dcgs_dots<3>, g, b, 0, s, L, V, ldv, j, wd, act, partials, partials2, tickets, h, h2);
  else
    hipLaunchKernelGGL(k_dcgs_dots<2>, g, b, 0, s, L, V, ldv, j, wd, act, partials, partials2, tickets, h, h2);
  if (any_large) {
    hipLaunchKernelGGL(k_reduce_large, dim3(j + 3, L.n_seg), wide, 0, s, L, partials, 0, act, h, kMaxBasis);
    if (j > 0)
      hipLaunchKernelGGL(k_reduce_large, dim3(j, L.n_seg), wide, 0, s, L, partials2, 0, act, h2, kMaxBasis);
  }
  hipLaunchKernelGGL(k_dcgs_finalize, dim3(L.n_seg), dim3(64), 0, s, G, j, max_it, h, h2, nrm, closing ? 1 : 0);
  if (!closing) {
    if (d3)
      hipLaunchKernelGGL(k_dcgs_update<3>, g, b, 0, s, L, V, ldv, j, w, h, h2, nrm, act, partials, tickets);
    else
      hipLaunchKernelGGL(k_dcgs_update<2>, g, b, 0, s, L, V, ldv, j, w, h, h2, nrm, act, partials, tickets);
    if (any_large) hipLaunchKernelGGL(k_reduce_large, dim3(1, L.n_seg), wide, 0, s, L, partials, 0, act, nrm, 4);
    hipLaunchKernelGGL(k_dcgs_step_end, dim3(1), b, 0, s, G, L.n_seg, j, max_it, h, nrm);
  }
  JFNK_HIP(hipGetLastError());
}

}  // namespace jfnk
