// Residual and Jacobian-free J.v kernels for gfx950.
//
// Two passes over the cells, one lane per cell, gather-only (no atomics):
//   k_gradient: least-squares gradient of w = u + eps v (Eq. leastSquaresGrad,
//               weights omega_f = |Gamma_f| in both the sum and G_P).  G_P is
//               rebuilt from the cell centroids and face areas on the fly, so
//               no per-slot least-squares vectors are stored:
//               grad w_P = G_P^{-1} sum_f |Gamma|/(d.d) d (x) (w_N - w_P).
//               It writes the record {w, grad w} of every cell (component-
//               major arrays) for the second pass.
//   k_flux:     face forces (Eq. divStressDiscret) + Rhie-Chow stabilisation
//               (Eq. RhieChow) summed over the cell's faces in a fixed slot
//               order, then either R(w) or (R(w) - R(u))/eps (Eq. JF).
// Every internal face is evaluated from identical operands in owner
// orientation by both adjacent cells (operand selection, one code path), so
// the two contributions are exact negatives and the sum telescopes.
//
// Rhie-Chow, written in the jump form of Appendix D:
//   alpha K_bar [ |Delta| (w_N - w_P)/|d| - Delta . grad w_f ] |Gamma|
//     = alpha K_bar |Gamma|^2 / (d . Gamma) [ (w_N - w_P) - d . grad w_f ],
// since Delta = d/(d.n), |Delta|/|d| = 1/(d.n) and n = Gamma/|Gamma|.
//
// Data layout: vectors, centroids, face data and the per-cell record are
// component-major (one array of n values per component) so that the 64 lanes
// of a wavefront, which handle 64 consecutive cells, read consecutive
// addresses for their own cell and -- in a bandwidth-reduced cell order --
// nearly consecutive addresses for the same neighbour slot.
//
// Neo-Hookean total-Lagrangian face force (Appendix A/B): with a = cof(F) Gamma
// and F^T a = J Gamma, (a . sigma) simplifies to
//   mu J^{-2/3} F Gamma + [ kappa/2 (J - 1/J) - mu/3 J^{-5/3} tr(F F^T) ] a.
#include <algorithm>

#include "internal.h"

namespace jfnk {

namespace {

__device__ __forceinline__ int xcd_block(int bid, int nb_launch) {
  // Hardware hands consecutive workgroup ids to the 8 XCDs round-robin;
  // give each XCD one contiguous range of cell blocks so that neighbouring
  // cells (close in the bandwidth-reduced order) share an L2.
#if JFNK_XCD_REMAP
  const int per = nb_launch / kNumXcd;
  return (bid % kNumXcd) * per + bid / kNumXcd;
#else
  return bid;
#endif
}

template <int D>
__device__ __forceinline__ void load_w(const double* __restrict__ u, const double* __restrict__ v,
                                       double eps, int n, int c, double (&w)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double uk = u[size_t(k) * n + c];
    w[k] = v ? fma(eps, v[size_t(k) * n + c], uk) : uk;
  }
}

template <int D>
__device__ __forceinline__ void load_soa(const double* __restrict__ a, int n, int c, double (&x)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) x[k] = a[size_t(k) * n + c];
}

// Material constants of the segment a workgroup works on.
struct Law {
  double mu, lam, kappa, aK;
};

// ---------------------------------------------------------------- laws
template <int D>
__device__ __forceinline__ void traction_le(const Law& m, const double (&g)[D][D],
                                            const double (&G)[D], double (&t)[D]) {
  double tr = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) tr += g[k][k];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double s = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) s = fma(G[i], g[i][j] + g[j][i], s);
    t[j] = fma(m.mu, s, m.lam * tr * G[j]);
  }
}

__device__ __forceinline__ void traction_nh3(const Law& m, const double (&g)[3][3],
                                             const double (&G)[3], double (&t)[3]) {
  double F[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) F[a][b] = (a == b ? 1.0 : 0.0) + g[b][a];
  double C[3][3];
  C[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  C[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  C[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  C[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
  C[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
  C[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
  C[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
  C[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
  C[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  const double J = F[0][0] * C[0][0] + F[0][1] * C[0][1] + F[0][2] * C[0][2];
  double trb = 0, a[3], FG[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    a[i] = C[i][0] * G[0] + C[i][1] * G[1] + C[i][2] * G[2];
    FG[i] = F[i][0] * G[0] + F[i][1] * G[1] + F[i][2] * G[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) trb = fma(F[i][k], F[i][k], trb);
  }
  const double cj = cbrt(J);
  const double Jm23 = 1.0 / (cj * cj);
  const double invJ = 1.0 / J;
  const double ca = 0.5 * m.kappa * (J - invJ) - (m.mu / 3.0) * Jm23 * invJ * trb;
  const double cf = m.mu * Jm23;
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] = fma(cf, FG[i], ca * a[i]);
}

__device__ __forceinline__ void traction_nh2(const Law& m, const double (&g)[2][2],
                                             const double (&G)[2], double (&t)[2]) {
  // plane strain: F_zz = 1, out-of-plane terms vanish for an in-plane Gamma
  const double F00 = 1.0 + g[0][0], F01 = g[1][0], F10 = g[0][1], F11 = 1.0 + g[1][1];
  const double J = F00 * F11 - F01 * F10;
  const double a0 = F11 * G[0] - F10 * G[1];
  const double a1 = -F01 * G[0] + F00 * G[1];
  const double FG0 = F00 * G[0] + F01 * G[1];
  const double FG1 = F10 * G[0] + F11 * G[1];
  const double trb = F00 * F00 + F01 * F01 + F10 * F10 + F11 * F11 + 1.0;
  const double cj = cbrt(J);
  const double Jm23 = 1.0 / (cj * cj);
  const double invJ = 1.0 / J;
  const double ca = 0.5 * m.kappa * (J - invJ) - (m.mu / 3.0) * Jm23 * invJ * trb;
  const double cf = m.mu * Jm23;
  t[0] = fma(cf, FG0, ca * a0);
  t[1] = fma(cf, FG1, ca * a1);
}

template <int D, int LAW>
__device__ __forceinline__ void traction(const Law& m, const double (&g)[D][D],
                                         const double (&G)[D], double (&t)[D]) {
  if constexpr (LAW == JFNK_LINEAR_ELASTIC) {
    traction_le<D>(m, g, G, t);
  } else if constexpr (D == 3) {
    traction_nh3(m, g, G, t);
  } else {
    traction_nh2(m, g, G, t);
  }
}

// Force on the owner side of an internal face (owner A, neighbour B).
template <int D, int LAW>
__device__ __forceinline__ void internal_face_force(const Law& m, const double (&G)[D], double wf,
                                                    const double (&xA)[D], const double (&xB)[D],
                                                    const double (&wA)[D], const double (&wB)[D],
                                                    const double (&gA)[D][D], const double (&gB)[D][D],
                                                    double (&f)[D]) {
  double gf[D][D];
  const double wb = 1.0 - wf;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) gf[i][j] = fma(wf, gA[i][j], wb * gB[i][j]);
  traction<D, LAW>(m, gf, G, f);
  double d[D], dG = 0, GG = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    d[k] = xB[k] - xA[k];
    dG = fma(d[k], G[k], dG);
    GG = fma(G[k], G[k], GG);
  }
  const double coef = m.aK * GG / dG;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double dg = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) dg = fma(d[i], gf[i][j], dg);
    f[j] = fma(coef, (wB[j] - wA[j]) - dg, f[j]);
  }
}

// ---------------------------------------------------------------- kernels
// Slots are processed in unrolled chunks of kChunk: all slot indices of a
// chunk are loaded first, then all gathers are issued, so that a wavefront
// has many independent memory requests in flight.
#ifndef JFNK_CHUNK
#define JFNK_CHUNK 6
#endif
constexpr int kChunk = JFNK_CHUNK;

template <int D>
__device__ __forceinline__ void load_rec(const double* __restrict__ rec, int n, int c, double (&w)[D],
                                         double (&g)[D][D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) w[k] = rec[size_t(k) * n + c];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) g[i][j] = rec[size_t(D + i * D + j) * n + c];
}

// Neighbour data of the gradient pass: w = u + eps v and the centroid of
// cell j, either gathered from global memory (j = cell number) or read from
// the workgroup's LDS copy of its tile and halo (j = position in the copy).
template <int D>
struct GradGlobal {
  const double* u;
  const double* v;
  const double* xc;
  double eps;
  int n;
  __device__ __forceinline__ void get(int j, double (&w)[D], double (&x)[D]) const {
    load_w<D>(u, v, eps, n, j, w);
    load_soa<D>(xc, n, j, x);
  }
};

template <int D>
struct GradLds {
  const double* lds;  // [D][S] w, then [D][S] centroids
  int S;
  __device__ __forceinline__ void get(int j, double (&w)[D], double (&x)[D]) const {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      w[k] = lds[k * S + j];
      x[k] = lds[(D + k) * S + j];
    }
  }
};

// Least-squares gradient of cell c (Eq. leastSquaresGrad with the weight
// |Gamma_f| in the sum and in G_P) and its record {w, grad w}.  ids holds
// the neighbour ids of the slots in the source's numbering; self is c's id.
// Neighbour ids and |Gamma_f| of one chunk of a cell's slots.
struct GradChunk {
  int nb[kChunk];
  double mg[kChunk];
};

__device__ __forceinline__ void load_grad_chunk(const MeshDev& m, const int32_t* __restrict__ ids, int s0,
                                                int width, int lane, int k0, GradChunk& gc) {
  int fc[kChunk];
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int idx = s0 + (k0 + k) * kSlice + lane;
    gc.nb[k] = (k0 + k < width) ? ids[idx] : kSlotPad;
    fc[k] = (k0 + k < width) ? m.slot_fc[idx] : 0;
  }
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int f = fc[k] >= 0 ? fc[k] : ~fc[k];
    gc.mg[k] = gc.nb[k] >= 0 ? m.magG[f] : 0.0;
  }
}

template <int D, class Src>
__device__ __forceinline__ void gradient_cell(const MeshDev& m, const Src& src, const int32_t* __restrict__ ids,
                                              int self, int c, double* __restrict__ rec) {
  const int n = m.n_cells;
  double wP[D], xP[D];
  src.get(self, wP, xP);
  double Gs[D][D], M[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Gs[i][j] = M[i][j] = 0.0;
  const int slice = c / kSlice, lane = c % kSlice;
  const int s0 = m.slice_ptr[slice];
  const int width = (m.slice_ptr[slice + 1] - s0) / kSlice;
  for (int k0 = 0; k0 < width; k0 += kChunk) {
    GradChunk gc;
    load_grad_chunk(m, ids, s0, width, lane, k0, gc);
    const int* nb = gc.nb;
    const double* mg = gc.mg;
    double xN[kChunk][D], wN[kChunk][D];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const int nn = nb[k] >= 0 ? nb[k] : self;
      src.get(nn, wN[k], xN[k]);
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      if (nb[k] < 0) continue;
      double d[D], dd = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        d[q] = xN[k][q] - xP[q];
        dd = fma(d[q], d[q], dd);
      }
      const double wt = mg[k] / dd;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const double wd = wt * d[i];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          Gs[i][j] = fma(wd, d[j], Gs[i][j]);
          M[i][j] = fma(wd, wN[k][j] - wP[j], M[i][j]);
        }
      }
    }
  }
  double g[D][D];
  if constexpr (D == 3) {
    const double a00 = Gs[1][1] * Gs[2][2] - Gs[1][2] * Gs[1][2];
    const double a01 = Gs[0][2] * Gs[1][2] - Gs[0][1] * Gs[2][2];
    const double a02 = Gs[0][1] * Gs[1][2] - Gs[0][2] * Gs[1][1];
    const double a11 = Gs[0][0] * Gs[2][2] - Gs[0][2] * Gs[0][2];
    const double a12 = Gs[0][1] * Gs[0][2] - Gs[0][0] * Gs[1][2];
    const double a22 = Gs[0][0] * Gs[1][1] - Gs[0][1] * Gs[0][1];
    const double inv = 1.0 / (Gs[0][0] * a00 + Gs[0][1] * a01 + Gs[0][2] * a02);
    const double A[3][3] = {{a00, a01, a02}, {a01, a11, a12}, {a02, a12, a22}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) g[i][j] = (A[i][0] * M[0][j] + A[i][1] * M[1][j] + A[i][2] * M[2][j]) * inv;
  } else {
    const double inv = 1.0 / (Gs[0][0] * Gs[1][1] - Gs[0][1] * Gs[0][1]);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      g[0][j] = (Gs[1][1] * M[0][j] - Gs[0][1] * M[1][j]) * inv;
      g[1][j] = (-Gs[0][1] * M[0][j] + Gs[0][0] * M[1][j]) * inv;
    }
  }
#pragma unroll
  for (int k = 0; k < D; ++k) rec[size_t(k) * n + c] = wP[k];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) rec[size_t(D + i * D + j) * n + c] = g[i][j];
}

template <int D>
__device__ __forceinline__ void zero_rec(double* __restrict__ rec, int n, int c) {
#pragma unroll
  for (int k = 0; k < D + D * D; ++k) rec[size_t(k) * n + c] = 0.0;
}

// Every cell pass loops over the tiles it - blockIdx.x = 0, G, 2G, ... of a
// launch of G workgroups (G = one per tile, or a persistent grid chosen by
// the tuner; G is a multiple of the XCD count, so a workgroup stays on the
// tiles its XCD owns).
template <int D>
__global__ __launch_bounds__(kFvBlock, JFNK_FV_MINWAVES) void k_gradient(MeshDev m, const double* __restrict__ u,
                                                                           const double* __restrict__ v,
                                                                           SegScalars sc,
                                                                           double* __restrict__ rec, int nb_real,
                                                                           int nb_launch) {
  const int n = m.n_cells;
  for (int it = blockIdx.x; it < nb_launch; it += gridDim.x) {
    const int lb = xcd_block(it, nb_launch);
    if (lb >= nb_real) continue;
    const int seg = m.seg_of_block[lb];
    if (sc.active != nullptr && sc.active[seg] == 0) continue;
    const int c = lb * kFvBlock + threadIdx.x;
    if (c >= n) continue;
    if (c - m.seg[seg].cell_off >= m.seg[seg].n_cells) {  // alignment padding
      zero_rec<D>(rec, n, c);
      continue;
    }
    const GradGlobal<D> src{u, v, m.xc, (v != nullptr) ? sc.eps[seg] : 0.0, n};
    gradient_cell<D>(m, src, m.slot_nb, c, c, rec);
  }
}

// Tiled gradient pass: one workgroup per tile; w and the centroids of the
// tile's cells and halo are staged in LDS with all lanes active, then every
// neighbour is read from LDS.  Exits before the barrier are uniform over the
// workgroup.
template <int D>
__global__ __launch_bounds__(kFvBlock) void k_gradient_tiled(MeshDev m, const double* __restrict__ u,
                                                             const double* __restrict__ v, SegScalars sc,
                                                             double* __restrict__ rec, int nb_real, int nb_launch) {
  extern __shared__ double lds[];
  const int n = m.n_cells, S = m.halo_stride;
  for (int it = blockIdx.x; it < nb_launch; it += gridDim.x) {
    const int tile = xcd_block(it, nb_launch);
    if (tile >= nb_real) continue;
    const int seg = m.seg_of_block[tile];
    if (sc.active != nullptr && sc.active[seg] == 0) continue;
    const double eps = (v != nullptr) ? sc.eps[seg] : 0.0;
    const int base = tile * kFvBlock;
    const int h0 = m.halo_ptr[tile], nh = m.halo_ptr[tile + 1] - h0;
    const int c = base + threadIdx.x;
    for (int i = threadIdx.x; i < kFvBlock + nh; i += kFvBlock) {
      const int cg = i < kFvBlock ? base + i : m.halo_cells[h0 + i - kFvBlock];
      double w[D], x[D];
      if (cg < n) {
        load_w<D>(u, v, eps, n, cg, w);
        load_soa<D>(m.xc, n, cg, x);
      } else {
#pragma unroll
        for (int k = 0; k < D; ++k) w[k] = x[k] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        lds[k * S + i] = w[k];
        lds[(D + k) * S + i] = x[k];
      }
    }
    __syncthreads();
    if (c < n) {
      if (c - m.seg[seg].cell_off >= m.seg[seg].n_cells) {
        zero_rec<D>(rec, n, c);
      } else {
        const GradLds<D> src{lds, S};
        gradient_cell<D>(m, src, m.slot_loc, threadIdx.x, c, rec);
      }
    }
    __syncthreads();  // the LDS copy is rewritten for the next tile
  }
}

// Neighbour data of the flux pass: the record {w, grad w} and the centroid
// of cell j, gathered from global memory or read from the LDS copy.
template <int D>
struct FluxGlobal {
  const double* rec;
  const double* xc;
  int n;
  __device__ __forceinline__ void get(int j, double (&w)[D], double (&g)[D][D], double (&x)[D]) const {
    load_rec<D>(rec, n, j, w, g);
    load_soa<D>(xc, n, j, x);
  }
};

template <int D>
struct FluxLds {
  const double* lds;  // rows: w (D), grad w (D*D), centroid (D), each of length S
  int S;
  __device__ __forceinline__ void get(int j, double (&w)[D], double (&g)[D][D], double (&x)[D]) const {
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = lds[k * S + j];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) g[a][b] = lds[(D + a * D + b) * S + j];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = lds[(D + D * D + k) * S + j];
  }
};

// Boundary face bf of cell P added to R: displacement faces Gamma . sigma_P
// plus the Rhie-Chow term against load * u_bar; traction faces
// load |Gamma| T_bar and pressure faces -load p Gamma (stored pre-multiplied).
template <int D, int LAW>
__device__ __forceinline__ void boundary_force(const MeshDev& m, const Law& law, int bf, double load,
                                               const double (&wP)[D], const double (&gP)[D][D], double (&R)[D]) {
  const double* r = m.bface + size_t(bf) * kBfaceRec;
  const int type = int(r[9]);
  if (type == kBcDisp) {
    double G[D], db[D], ub[D], t[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      G[q] = r[q];
      db[q] = r[3 + q];
      ub[q] = load * r[6 + q];
    }
    traction<D, LAW>(law, gP, G, t);
    double dG = 0, GG = 0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      dG = fma(db[q], G[q], dG);
      GG = fma(G[q], G[q], GG);
    }
    const double coef = law.aK * GG / dG;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double dg = 0;
#pragma unroll
      for (int i = 0; i < D; ++i) dg = fma(db[i], gP[i][j], dg);
      R[j] += fma(coef, (ub[j] - wP[j]) - dg, t[j]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < D; ++q) R[q] = fma(load, r[6 + q], R[q]);
  }
}

// Sum of the face forces of cell c (Eq. divStressDiscret + Eq. RhieChow);
// ids holds the neighbour ids of the slots in the source's numbering and
// self is c's id.
template <int D, int LAW, class Src>
__device__ __forceinline__ void cell_forces(const MeshDev& m, const Law& law, const Src& src,
                                            const int32_t* __restrict__ ids, int self, int c, double load,
                                            double (&R)[D]) {
  double wP[D], xP[D], gP[D][D];
  src.get(self, wP, gP, xP);
#pragma unroll
  for (int k = 0; k < D; ++k) R[k] = 0.0;
  const int slice = c / kSlice, lane = c % kSlice;
  const int s0 = m.slice_ptr[slice];
  const int width = (m.slice_ptr[slice + 1] - s0) / kSlice;
  for (int k0 = 0; k0 < width; k0 += kChunk) {
    int nb[kChunk], fc[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const int idx = s0 + (k0 + k) * kSlice + lane;
      nb[k] = (k0 + k < width) ? ids[idx] : kSlotPad;
      fc[k] = (k0 + k < width) ? m.slot_fc[idx] : 0;
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      if (nb[k] >= 0) {
        const bool own = fc[k] >= 0;
        const int f = own ? fc[k] : ~fc[k];
        double G[D], xN[D], wN[D], gN[D][D];
        load_soa<D>(m.fG, m.n_int, f, G);
        const double wf = m.fw[f];
        src.get(nb[k], wN, gN, xN);
        // canonical operands: A = owner, B = neighbour of the face
        double xA[D], xB[D], wA[D], wB[D], gA[D][D], gB[D][D], fo[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          xA[i] = own ? xP[i] : xN[i];
          xB[i] = own ? xN[i] : xP[i];
          wA[i] = own ? wP[i] : wN[i];
          wB[i] = own ? wN[i] : wP[i];
#pragma unroll
          for (int j = 0; j < D; ++j) {
            gA[i][j] = own ? gP[i][j] : gN[i][j];
            gB[i][j] = own ? gN[i][j] : gP[i][j];
          }
        }
        internal_face_force<D, LAW>(law, G, wf, xA, xB, wA, wB, gA, gB, fo);
#pragma unroll
        for (int q = 0; q < D; ++q) R[q] += own ? fo[q] : -fo[q];
      } else if (nb[k] == kSlotBoundary) {
        boundary_force<D, LAW>(m, law, fc[k], load, wP, gP, R);
      }
    }
  }
}

constexpr int kLawMixed = -1;

// R(w), or (R(w) - R(u))/eps when Ru is given, of cell c (not padding).
template <int D, int LAWSEL, class Src>
__device__ __forceinline__ void flux_cell(const MeshDev& m, const SegInfo& si, const Src& src,
                                          const int32_t* __restrict__ ids, int self, int c, double load,
                                          double eps, const double* __restrict__ Ru, double* __restrict__ out) {
  const int n = m.n_cells;
  const Law law{si.mu, si.lam, si.kappa, si.aK};
  double R[D];
  if constexpr (LAWSEL == kLawMixed) {
    if (si.law == JFNK_NEO_HOOKEAN)
      cell_forces<D, JFNK_NEO_HOOKEAN>(m, law, src, ids, self, c, load, R);
    else
      cell_forces<D, JFNK_LINEAR_ELASTIC>(m, law, src, ids, self, c, load, R);
  } else {
    cell_forces<D, LAWSEL>(m, law, src, ids, self, c, load, R);
  }
  if (Ru != nullptr) {
    const double ie = eps != 0.0 ? 1.0 / eps : 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q)
      out[size_t(q) * n + c] = eps != 0.0 ? (R[q] - Ru[size_t(q) * n + c]) * ie : 0.0;
  } else {
#pragma unroll
    for (int q = 0; q < D; ++q) out[size_t(q) * n + c] = R[q];
  }
}

// LAWSEL: JFNK_LINEAR_ELASTIC, JFNK_NEO_HOOKEAN, or kLawMixed (law chosen per
// segment, i.e. per workgroup).
template <int D, int LAWSEL>
__global__ __launch_bounds__(kFvBlock, JFNK_FV_MINWAVES) void k_flux(MeshDev m, const double* __restrict__ rec,
                                                                       SegScalars sc,
                                                                       const double* __restrict__ Ru,
                                                                       double* __restrict__ out, int nb_real,
                                                                       int nb_launch) {
  const int n = m.n_cells;
  for (int it = blockIdx.x; it < nb_launch; it += gridDim.x) {
    const int lb = xcd_block(it, nb_launch);
    if (lb >= nb_real) continue;
    const int seg = m.seg_of_block[lb];
    if (sc.active != nullptr && sc.active[seg] == 0) continue;
    const int c = lb * kFvBlock + threadIdx.x;
    if (c >= n) continue;
    const SegInfo& si = m.seg[seg];
    if (c - si.cell_off >= si.n_cells) {  // alignment padding
#pragma unroll
      for (int q = 0; q < D; ++q) out[size_t(q) * n + c] = 0.0;
      continue;
    }
    const FluxGlobal<D> src{rec, m.xc, n};
    flux_cell<D, LAWSEL>(m, si, src, m.slot_nb, c, c, sc.load[seg], Ru ? sc.eps[seg] : 0.0, Ru, out);
  }
}

// Tiled flux pass.  The records and centroids of the tile's cells and halo
// are staged in LDS (rows of length halo_stride).  Phase A evaluates every
// internal face touching the tile once, spread evenly over the workgroup
// (owner first, the canonical operand order), into LDS; phase B sums each
// cell's slots in slot order (face forces from LDS with the sign of the
// side, boundary faces evaluated in place), the same sequence of operations
// as the gather pass, so both give the same bits.  Exits before a barrier
// are uniform over the workgroup.
// Face data of up to kEnt entries of the tile's face list (entries
// e = threadIdx.x + j * kFvBlock), loaded before the staging barrier so that
// every global load of the tile is in flight at once.
constexpr int kEnt = 4;
template <int D>
struct FaceBatch {
  int n = 0;
  int lo[kEnt], ln[kEnt];
  double G[kEnt][D], wf[kEnt];
};

template <int D>
__device__ __forceinline__ void load_faces(const MeshDev& m, int tile, int e0, FaceBatch<D>& fb) {
  const int f0 = m.fbeg[tile], n_own = m.fbeg[tile + 1] - f0;
  const int i0 = m.in_ptr[tile], n_ent = n_own + m.in_ptr[tile + 1] - i0;
  fb.n = 0;
#pragma unroll
  for (int j = 0; j < kEnt; ++j) {
    const int e = e0 + j * kFvBlock;
    if (e >= n_ent) break;
    const int f = e < n_own ? f0 + e : m.in_face[i0 + e - n_own];
    const int packed = e < n_own ? m.face_loc[f] : m.in_loc[i0 + e - n_own];
    fb.lo[j] = packed & 0xffff;
    fb.ln[j] = packed >> 16;
    load_soa<D>(m.fG, m.n_int, f, fb.G[j]);
    fb.wf[j] = m.fw[f];
    fb.n = j + 1;
  }
}

// Phase A: the loaded faces, owner first (the canonical operand order).
template <int D, int LAW>
__device__ __forceinline__ void face_forces(const SegInfo& si, const FluxLds<D>& src, int e0, const FaceBatch<D>& fb,
                                            double* __restrict__ ff, int fs) {
  const Law law{si.mu, si.lam, si.kappa, si.aK};
#pragma unroll
  for (int j = 0; j < kEnt; ++j) {
    if (j >= fb.n) break;
    double xA[D], xB[D], wA[D], wB[D], gA[D][D], gB[D][D], fo[D];
    src.get(fb.lo[j], wA, gA, xA);
    src.get(fb.ln[j], wB, gB, xB);
    internal_face_force<D, LAW>(law, fb.G[j], fb.wf[j], xA, xB, wA, wB, gA, gB, fo);
#pragma unroll
    for (int q = 0; q < D; ++q) ff[q * fs + e0 + j * kFvBlock] = fo[q];
  }
}

// Phase B: cell c sums its slots in slot order (face forces from LDS with
// the sign of its side, boundary faces evaluated in place).
// Slot metadata of one chunk of a cell's slots.
struct SlotChunk {
  int nb[kChunk], fc[kChunk], lf[kChunk];
};

__device__ __forceinline__ void load_slots(const MeshDev& m, int s0, int width, int lane, int k0, SlotChunk& sl) {
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int idx = s0 + (k0 + k) * kSlice + lane;
    const bool in = k0 + k < width;
    sl.nb[k] = in ? m.slot_loc[idx] : kSlotPad;
    sl.fc[k] = in ? m.slot_fc[idx] : 0;
    sl.lf[k] = in ? int(m.slot_lf[idx]) : 0;
  }
}

// first: the cell's first chunk of slots, loaded before the tile's barriers
template <int D, int LAW>
__device__ __forceinline__ void tile_cell_sum(const MeshDev& m, const SegInfo& si, const FluxLds<D>& src, int self,
                                              int c, double load, const double* __restrict__ ff, int fs,
                                              const SlotChunk& first, double (&R)[D]) {
  const Law law{si.mu, si.lam, si.kappa, si.aK};
  double wP[D], xP[D], gP[D][D];
  src.get(self, wP, gP, xP);
#pragma unroll
  for (int q = 0; q < D; ++q) R[q] = 0.0;
  const int slice = c / kSlice, lane = c % kSlice;
  const int s0 = m.slice_ptr[slice];
  const int width = (m.slice_ptr[slice + 1] - s0) / kSlice;
  for (int k0 = 0; k0 < width; k0 += kChunk) {
    SlotChunk cur;
    if (k0 == 0)
      cur = first;
    else
      load_slots(m, s0, width, lane, k0, cur);
    const int* nb = cur.nb;
    const int* fc = cur.fc;
    const int* lf = cur.lf;
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      if (nb[k] >= 0) {
        const bool own = fc[k] >= 0;
#pragma unroll
        for (int q = 0; q < D; ++q) R[q] += own ? ff[q * fs + lf[k]] : -ff[q * fs + lf[k]];
      } else if (nb[k] == kSlotBoundary) {
        boundary_force<D, LAW>(m, law, fc[k], load, wP, gP, R);
      }
    }
  }
}

// Tiled flux pass.  The records and centroids of the tile's cells and halo
// are staged in LDS (rows of length halo_stride).  Phase A evaluates every
// internal face touching the tile once, spread evenly over the workgroup
// (owner first, the canonical operand order), into LDS; phase B sums each
// cell's slots in slot order, the same sequence of operations as the
// gather pass, so both give the same bits.  Exits before a barrier are
// uniform over the workgroup.
template <int D, int LAWSEL>
__global__ __launch_bounds__(kFvBlock) void k_flux_tiled(MeshDev m, const double* __restrict__ rec,
                                                         SegScalars sc, const double* __restrict__ Ru,
                                                         double* __restrict__ out, int nb_real, int nb_launch) {
  extern __shared__ double lds[];
  const int n = m.n_cells, S = m.halo_stride, fs = m.face_stride;
  constexpr int kRows = 2 * D + D * D;
  double* ff = lds + kRows * S;
  for (int it = blockIdx.x; it < nb_launch; it += gridDim.x) {
    const int tile = xcd_block(it, nb_launch);
    if (tile >= nb_real) continue;
    const int seg = m.seg_of_block[tile];
    if (sc.active != nullptr && sc.active[seg] == 0) continue;
    const int base = tile * kFvBlock;
    const int h0 = m.halo_ptr[tile], nh = m.halo_ptr[tile + 1] - h0;
    const int n_ent = m.fbeg[tile + 1] - m.fbeg[tile] + m.in_ptr[tile + 1] - m.in_ptr[tile];
    FaceBatch<D> fb;
    load_faces<D>(m, tile, threadIdx.x, fb);
    // this cell's first chunk of slots and R(u), also ahead of the barriers
    const int c = base + threadIdx.x;
    SlotChunk first;
    double ru[D];
#pragma unroll
    for (int q = 0; q < D; ++q) ru[q] = 0.0;
    if (c < n) {
      const int s0 = m.slice_ptr[c / kSlice];
      load_slots(m, s0, (m.slice_ptr[c / kSlice + 1] - s0) / kSlice, c % kSlice, 0, first);
      if (Ru != nullptr)
#pragma unroll
        for (int q = 0; q < D; ++q) ru[q] = Ru[size_t(q) * n + c];
    }
    for (int i = threadIdx.x; i < kFvBlock + nh; i += kFvBlock) {
      const int cg = i < kFvBlock ? base + i : m.halo_cells[h0 + i - kFvBlock];
      if (cg < n) {
#pragma unroll
        for (int r = 0; r < D + D * D; ++r) lds[r * S + i] = rec[size_t(r) * n + cg];
#pragma unroll
        for (int k = 0; k < D; ++k) lds[(D + D * D + k) * S + i] = m.xc[size_t(k) * n + cg];
      } else {
#pragma unroll
        for (int r = 0; r < kRows; ++r) lds[r * S + i] = 0.0;
      }
    }
    __syncthreads();
    const SegInfo& si = m.seg[seg];
    const FluxLds<D> src{lds, S};
    // phase A, kEnt entries per thread per round (one round unless the tile
    // touches more than kEnt * kFvBlock faces)
    for (int e0 = threadIdx.x;; e0 += kEnt * kFvBlock) {
      if (e0 != threadIdx.x) load_faces<D>(m, tile, e0, fb);
      if constexpr (LAWSEL == kLawMixed) {
        if (si.law == JFNK_NEO_HOOKEAN)
          face_forces<D, JFNK_NEO_HOOKEAN>(si, src, e0, fb, ff, fs);
        else
          face_forces<D, JFNK_LINEAR_ELASTIC>(si, src, e0, fb, ff, fs);
      } else {
        face_forces<D, LAWSEL>(si, src, e0, fb, ff, fs);
      }
      if (e0 - int(threadIdx.x) + kEnt * kFvBlock >= n_ent) break;
    }
    __syncthreads();
    if (c < n) {
      if (c - si.cell_off < si.n_cells) {
        const double load = sc.load[seg];
        double R[D];
        if constexpr (LAWSEL == kLawMixed) {
          if (si.law == JFNK_NEO_HOOKEAN)
            tile_cell_sum<D, JFNK_NEO_HOOKEAN>(m, si, src, threadIdx.x, c, load, ff, fs, first, R);
          else
            tile_cell_sum<D, JFNK_LINEAR_ELASTIC>(m, si, src, threadIdx.x, c, load, ff, fs, first, R);
        } else {
          tile_cell_sum<D, LAWSEL>(m, si, src, threadIdx.x, c, load, ff, fs, first, R);
        }
        if (Ru != nullptr) {
          const double eps = sc.eps[seg];
          const double ie = eps != 0.0 ? 1.0 / eps : 0.0;
#pragma unroll
          for (int q = 0; q < D; ++q) out[size_t(q) * n + c] = eps != 0.0 ? (R[q] - ru[q]) * ie : 0.0;
        } else {
#pragma unroll
          for (int q = 0; q < D; ++q) out[size_t(q) * n + c] = R[q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < D; ++q) out[size_t(q) * n + c] = 0.0;  // alignment padding
      }
    }
    __syncthreads();  // the LDS copy is rewritten for the next tile
  }
}

// nb_real tiles, nb_launch = tiles rounded up to the XCD count, and the
// number of workgroups launched (persistent grid when the tuner set one).
inline void grid_for(const MeshDev& m, int& nb_real, int& nb_launch, int& grid) {
  nb_real = (m.n_cells + kFvBlock - 1) / kFvBlock;
  nb_launch = ((nb_real + kNumXcd - 1) / kNumXcd) * kNumXcd;
  grid = nb_launch;
  if (m.persist > 0) grid = std::min(nb_launch, ((m.persist + kNumXcd - 1) / kNumXcd) * kNumXcd);
}

}  // namespace

void launch_gradient(const MeshDev& m, const double* u, const double* v, const SegScalars& sc,
                     double* rec, hipStream_t s) {
  int nr, nl, g;
  grid_for(m, nr, nl, g);
  if (m.tiled && m.lds_kernels) {
    const size_t lds = sizeof(double) * 2 * m.dim * size_t(m.halo_stride);
    if (m.dim == 3)
      hipLaunchKernelGGL(k_gradient_tiled<3>, dim3(g), dim3(kFvBlock), lds, s, m, u, v, sc, rec, nr, nl);
    else
      hipLaunchKernelGGL(k_gradient_tiled<2>, dim3(g), dim3(kFvBlock), lds, s, m, u, v, sc, rec, nr, nl);
  } else if (m.dim == 3) {
    hipLaunchKernelGGL(k_gradient<3>, dim3(g), dim3(kFvBlock), 0, s, m, u, v, sc, rec, nr, nl);
  } else {
    hipLaunchKernelGGL(k_gradient<2>, dim3(g), dim3(kFvBlock), 0, s, m, u, v, sc, rec, nr, nl);
  }
  JFNK_HIP(hipGetLastError());
}

namespace {

template <int D, int LAWSEL>
void flux_launch(const MeshDev& m, const double* rec, const SegScalars& sc, const double* Ru, double* out,
                 hipStream_t s) {
  int nr, nl, g;
  grid_for(m, nr, nl, g);
  if (m.tiled && m.lds_kernels) {
    const size_t lds = flux_lds_bytes(D, m.halo_stride, m.face_stride);
    hipLaunchKernelGGL((k_flux_tiled<D, LAWSEL>), dim3(g), dim3(kFvBlock), lds, s, m, rec, sc, Ru, out, nr, nl);
  } else {
    hipLaunchKernelGGL((k_flux<D, LAWSEL>), dim3(g), dim3(kFvBlock), 0, s, m, rec, sc, Ru, out, nr, nl);
  }
}

}  // namespace

void launch_flux(const MeshDev& m, const double* rec, const SegScalars& sc, const double* Ru, double* out,
                 hipStream_t s) {
  const int mask = m.law_mask;
  if (m.dim == 3) {
    if (mask == 2)
      flux_launch<3, JFNK_NEO_HOOKEAN>(m, rec, sc, Ru, out, s);
    else if (mask == 1)
      flux_launch<3, JFNK_LINEAR_ELASTIC>(m, rec, sc, Ru, out, s);
    else
      flux_launch<3, kLawMixed>(m, rec, sc, Ru, out, s);
  } else {
    if (mask == 2)
      flux_launch<2, JFNK_NEO_HOOKEAN>(m, rec, sc, Ru, out, s);
    else if (mask == 1)
      flux_launch<2, JFNK_LINEAR_ELASTIC>(m, rec, sc, Ru, out, s);
    else
      flux_launch<2, kLawMixed>(m, rec, sc, Ru, out, s);
  }
  JFNK_HIP(hipGetLastError());
}

}  // namespace jfnk
