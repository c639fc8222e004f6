// Residual and Jacobian-free J.v kernels for gfx950.
//
// Two passes over the cells, one lane per cell, no atomics (gathered from
// global memory, or staged per tile of 256 cells in LDS; a third form fuses
// both passes per tile, see k_jv_fused):
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

// a * b + c is fused only within one source expression, as the front end
// reads it (besides the explicit fma() calls), never by the back end across
// statements: every pass (gathered, LDS-staged, fused, any chunk size or
// launch shape) then evaluates each expression with the same roundings and
// gives the same bits.
#pragma clang fp contract(on)

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

// Head of a tile's halo list for the gradient pass: the tile of loop
// position it, its halo range, and the id of this thread's cell among the
// first kFvBlock halo cells (n_cells when none).  A persistent workgroup
// loads the head of its next tile while it works on the current one, so the
// staging loads of the halo values need not wait for their ids.  (The flux
// pass loads its heads in place: with its larger register file the early
// load measured slower there.)
struct HaloHead {
  int tile, h0, nh, cg1;
};

__device__ __forceinline__ HaloHead halo_head(const MeshDev& m, int it, int nb_real, int nb_launch) {
  HaloHead hh{nb_real, 0, 0, m.n_cells};
  if (it < nb_launch) hh.tile = xcd_block(it, nb_launch);
  if (hh.tile < nb_real) {
    hh.h0 = m.halo_ptr[hh.tile];
    hh.nh = m.halo_ptr[hh.tile + 1] - hh.h0;
    if (int(threadIdx.x) < hh.nh) hh.cg1 = m.halo_cells[hh.h0 + threadIdx.x];
  }
  return hh;
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

// J^(-1/3) of the neo-Hookean laws: a single-precision seed 2^(-log2|J|/3)
// with the sign of J, then two Newton corrections in FP64,
// y <- y + y (1 - J y^3)/3, which leave y within about one ulp (quadratic
// convergence from ~22 correct bits); J^(-2/3) = y^2 and 1/J = y^3 then
// cost two products instead of a cube root and two divisions.
__device__ __forceinline__ double inv_cbrt(double J) {
  const float a = fabsf(float(J));
  double y = double(__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(a) * (1.0f / 3.0f)));
  y = J < 0.0 ? -y : y;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double y3 = (y * y) * y;
    const double r = fma(-J, y3, 1.0);
    y = fma(y, r * (1.0 / 3.0), y);
  }
  return y;
}

// Neo-Hookean face force (Appendix B, total Lagrangian form of Appendix A):
// with a = cof(F) Gamma the force is sigma a, sigma = mu/J dev(bbar) +
// kappa/2 (J - 1/J) I, bbar = J^(-2/3) F F^T.  It is evaluated through
// H = F - I = (grad w)^T so that no term of size mu |Gamma| cancels against
// another: near the reference state the stress is small next to mu, and
// forming F F^T and J and then subtracting I (or the trace) would leave
// rounding errors of size eps_mach mu |Gamma| in every face force, which the
// finite difference of J v divides by eps (about sqrt(eps_mach)).  The
// exact identities used (3 x 3):
//   J - 1    = tr H + (sum of the principal 2 x 2 minors of H) + det H
//   cof F    = (1 + tr H) I - H^T + cof H
//   J F G - a = (H + H^T - tr H I - cof H) G + (J - 1)(G + H G)  =: q
//   tr(F F^T) - 3 = 2 tr H + |H|^2
// so that  dev(bbar) a = J^(-2/3) (q - (tr(F F^T) - 3)/3 a)  and
//   sigma a = mu J^(-5/3) (q - (tr(F F^T) - 3)/3 a)
//             + kappa (J - 1)(1 + (J - 1)/2)/J a.
// Plane strain (F_zz = 1, H_zz = 0): cof H drops out of the in-plane
// components and J - 1 = tr H + det H.
__device__ __forceinline__ void traction_nh3(const Law& m, const double (&g)[3][3],
                                             const double (&G)[3], double (&t)[3]) {
  // H[a][b] = g[b][a]
  double C[3][3];   // cofactor matrix of H
  C[0][0] = g[1][1] * g[2][2] - g[2][1] * g[1][2];
  C[0][1] = g[2][1] * g[0][2] - g[0][1] * g[2][2];
  C[0][2] = g[0][1] * g[1][2] - g[1][1] * g[0][2];
  C[1][0] = g[2][0] * g[1][2] - g[1][0] * g[2][2];
  C[1][1] = g[0][0] * g[2][2] - g[2][0] * g[0][2];
  C[1][2] = g[1][0] * g[0][2] - g[0][0] * g[1][2];
  C[2][0] = g[1][0] * g[2][1] - g[2][0] * g[1][1];
  C[2][1] = g[2][0] * g[0][1] - g[0][0] * g[2][1];
  C[2][2] = g[0][0] * g[1][1] - g[1][0] * g[0][1];
  const double tr = g[0][0] + g[1][1] + g[2][2];
  const double detH = g[0][0] * C[0][0] + g[1][0] * C[0][1] + g[2][0] * C[0][2];
  const double Jm1 = tr + ((C[0][0] + C[1][1] + C[2][2]) + detH);
  const double J = 1.0 + Jm1;
  double a[3], q[3], hh = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double HG = g[0][i] * G[0] + g[1][i] * G[1] + g[2][i] * G[2];
    const double HtG = g[i][0] * G[0] + g[i][1] * G[1] + g[i][2] * G[2];
    const double CG = C[i][0] * G[0] + C[i][1] * G[1] + C[i][2] * G[2];
    a[i] = fma(tr, G[i], G[i]) - HtG + CG;
    q[i] = ((HG + HtG) - fma(tr, G[i], CG)) + Jm1 * (G[i] + HG);
#pragma unroll
    for (int k = 0; k < 3; ++k) hh = fma(g[i][k], g[i][k], hh);
  }
  const double trE = fma(2.0, tr, hh);
  const double y = inv_cbrt(J);
  const double Jm23 = y * y;
  const double invJ = Jm23 * y;
  const double cq = m.mu * (Jm23 * invJ);
  const double ca = m.kappa * Jm1 * fma(0.5, Jm1, 1.0) * invJ - cq * trE * (1.0 / 3.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] = fma(cq, q[i], ca * a[i]);
}

__device__ __forceinline__ void traction_nh2(const Law& m, const double (&g)[2][2],
                                             const double (&G)[2], double (&t)[2]) {
  // plane strain: F_zz = 1, out-of-plane terms vanish for an in-plane Gamma;
  // H00 = g00, H01 = g10, H10 = g01, H11 = g11
  const double tr = g[0][0] + g[1][1];
  const double detH = g[0][0] * g[1][1] - g[1][0] * g[0][1];
  const double Jm1 = tr + detH;
  const double J = 1.0 + Jm1;
  const double HG0 = g[0][0] * G[0] + g[1][0] * G[1];
  const double HG1 = g[0][1] * G[0] + g[1][1] * G[1];
  const double HtG0 = g[0][0] * G[0] + g[0][1] * G[1];
  const double HtG1 = g[1][0] * G[0] + g[1][1] * G[1];
  const double a0 = fma(tr, G[0], G[0]) - HtG0;
  const double a1 = fma(tr, G[1], G[1]) - HtG1;
  const double q0 = ((HG0 + HtG0) - tr * G[0]) + Jm1 * (G[0] + HG0);
  const double q1 = ((HG1 + HtG1) - tr * G[1]) + Jm1 * (G[1] + HG1);
  const double hh = g[0][0] * g[0][0] + g[0][1] * g[0][1] + g[1][0] * g[1][0] + g[1][1] * g[1][1];
  const double trE = fma(2.0, tr, hh);
  const double y = inv_cbrt(J);
  const double Jm23 = y * y;
  const double invJ = Jm23 * y;
  const double cq = m.mu * (Jm23 * invJ);
  const double ca = m.kappa * Jm1 * fma(0.5, Jm1, 1.0) * invJ - cq * trE * (1.0 / 3.0);
  t[0] = fma(cq, q0, ca * a0);
  t[1] = fma(cq, q1, ca * a1);
}

// St. Venant-Kirchhoff face force (Appendix B): S = 2 mu E + lambda tr(E) I
// with the Green strain E = (g + g^T + g g^T)/2, sigma = F S F^T / J (Eq.
// S2sigma); with a = cof(F) Gamma = J F^-T Gamma the force a . sigma is
// F S Gamma (F = I + g^T), which needs neither J nor the cofactor and has
// no cancellation against I.  Plane strain: E_zz = 0, in-plane terms only.
template <int D>
__device__ __forceinline__ void traction_svk(const Law& m, const double (&g)[D][D],
                                             const double (&G)[D], double (&t)[D]) {
  double E[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double gg = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) gg = fma(g[i][k], g[j][k], gg);
      E[i][j] = 0.5 * ((g[i][j] + g[j][i]) + gg);
    }
  double tr = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) tr += E[k][k];
  double SG[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double e = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) e = fma(E[i][j], G[j], e);
    SG[i] = fma(2.0 * m.mu, e, m.lam * tr * G[i]);
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double h = 0.0;   // (g^T S Gamma)_i = sum_k g[k][i] (S Gamma)_k
#pragma unroll
    for (int k = 0; k < D; ++k) h = fma(g[k][i], SG[k], h);
    t[i] = SG[i] + h;
  }
}

template <int D, int LAW>
__device__ __forceinline__ void traction(const Law& m, const double (&g)[D][D],
                                         const double (&G)[D], double (&t)[D]) {
  if constexpr (LAW == JFNK_LINEAR_ELASTIC) {
    traction_le<D>(m, g, G, t);
  } else if constexpr (LAW == JFNK_ST_VENANT_KIRCHHOFF) {
    traction_svk<D>(m, g, G, t);
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
// slots per chunk of the gradients read from the LDS copy of a tile
#ifndef JFNK_TILED_CHUNK
#define JFNK_TILED_CHUNK 3
#endif
constexpr int kTiledChunk = JFNK_TILED_CHUNK;

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

// Neighbour ids and |Gamma_f| of one chunk of CH of a cell's slots.
template <int CH>
struct GradChunk {
  int nb[CH];
  double mg[CH];
};

// Slots of cell c in its slice of the mesh's slot arrays (ids in the
// source's numbering); |Gamma_f| from the per-slot copy when mg is given,
// else gathered through the slot's face number.  bface(k): the boundary
// face of boundary slot k.
struct SliceSlots {
  const int32_t* ids;
  int s0, lane, width;
  const double* mg = nullptr;
  __device__ __forceinline__ int bface(const MeshDev& m, int k) const { return m.slot_fc[s0 + k * kSlice + lane]; }
  template <int CH>
  __device__ __forceinline__ void load(const MeshDev& m, int k0, GradChunk<CH>& gc) const {
    if (mg != nullptr) {
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int idx = s0 + (k0 + k) * kSlice + lane;
        gc.nb[k] = (k0 + k < width) ? ids[idx] : kSlotPad;
        gc.mg[k] = (k0 + k < width) ? mg[idx] : 0.0;
      }
      return;
    }
    int fc[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int idx = s0 + (k0 + k) * kSlice + lane;
      gc.nb[k] = (k0 + k < width) ? ids[idx] : kSlotPad;
      fc[k] = (k0 + k < width) ? m.slot_fc[idx] : 0;
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int f = fc[k] >= 0 ? fc[k] : ~fc[k];
      gc.mg[k] = gc.nb[k] >= 0 ? m.magG[f] : 0.0;
    }
  }
};

// Slots of halo cell i of a tile in the tile's lists (slot-major over the
// tile's nh halo cells: position in the tile's copy, |Gamma_f|), in the
// slot order of the cell's own slice.
struct HaloSlots {
  const int16_t* loc;
  const double* mg;
  int nh, i, width;
  const int32_t* fc;  // boundary faces of the boundary slots (meshes with symmetry faces)
  __device__ __forceinline__ int bface(const MeshDev&, int k) const { return fc[k * nh + i]; }
  template <int CH>
  __device__ __forceinline__ void load(const MeshDev&, int k0, GradChunk<CH>& gc) const {
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int idx = (k0 + k) * nh + i;
      gc.nb[k] = (k0 + k < width) ? int(loc[idx]) : kSlotPad;
      gc.mg[k] = (k0 + k < width) ? mg[idx] : 0.0;
    }
  }
};

// Symmetry face bf of a cell with value wP (Eq. leastSquaresGrad, its
// symmetry sum): the mirror image at d_s = 2 h n, h = d_b . n, with value
// R wP, so G_P += |Gamma| n n and the sum += -(|Gamma| / h) (n . wP) n n.
// Other boundary faces add nothing.
template <int D>
__device__ __forceinline__ void symmetry_lsq(const MeshDev& m, int bf, const double (&wP)[D], double (&Gs)[D][D],
                                             double (&M)[D][D]) {
  const double* r = m.bface + size_t(bf) * kBfaceRec;
  if (int(r[9]) != kBcSymm) return;
  double n[D], mg = 0, h = 0, wn = 0;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    n[q] = r[6 + q];
    mg = fma(r[q], n[q], mg);
    h = fma(r[3 + q], n[q], h);
    wn = fma(wP[q], n[q], wn);
  }
  const double a = -(mg / h) * wn;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      Gs[i][j] = fma(mg * n[i], n[j], Gs[i][j]);
      M[i][j] = fma(a * n[i], n[j], M[i][j]);
    }
}

// Least-squares gradient (Eq. leastSquaresGrad with the weight |Gamma_f| in
// the sum and in G_P) of the cell with id self in the source, its slots read
// from sl in slot order, CH at a time (the chunk size changes only how many
// loads are in flight, not the order of the sums).  Returns w_P and grad w_P.
template <int D, int CH = kChunk, class Src, class Slots>
__device__ __forceinline__ void lsq_gradient(const MeshDev& m, const Src& src, const Slots& sl, int self,
                                             double (&wP)[D], double (&g)[D][D]) {
  double xP[D];
  src.get(self, wP, xP);
  double Gs[D][D], M[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Gs[i][j] = M[i][j] = 0.0;
  for (int k0 = 0; k0 < sl.width; k0 += CH) {
    GradChunk<CH> gc;
    sl.template load<CH>(m, k0, gc);
    const int* nb = gc.nb;
    const double* mg = gc.mg;
    double xN[CH][D], wN[CH][D];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int nn = nb[k] >= 0 ? nb[k] : self;
      src.get(nn, wN[k], xN[k]);
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      if (nb[k] < 0) {
        if (m.has_symm && nb[k] == kSlotBoundary) symmetry_lsq<D>(m, sl.bface(m, k0 + k), wP, Gs, M);
        continue;
      }
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
}

// Gradient of cell c and its record {w, grad w}; ids holds the neighbour
// ids of the slots in the source's numbering and self is c's id.
template <int D, int CH = kChunk, class Src>
__device__ __forceinline__ void gradient_cell(const MeshDev& m, const Src& src, const int32_t* __restrict__ ids,
                                              int self, int c, double* __restrict__ rec,
                                              const double* __restrict__ mg = nullptr) {
  const int n = m.n_cells;
  const int slice = c / kSlice, lane = c % kSlice;
  const int s0 = m.slice_ptr[slice];
  const SliceSlots sl{ids, s0, lane, (m.slice_ptr[slice + 1] - s0) / kSlice, mg};
  double wP[D], g[D][D];
  lsq_gradient<D, CH>(m, src, sl, self, wP, g);
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
__global__ __launch_bounds__(kFvBlock, JFNK_TILED_MINWAVES) void k_gradient_tiled(MeshDev m, const double* __restrict__ u,
                                                             const double* __restrict__ v, SegScalars sc,
                                                             double* __restrict__ rec, int nb_real, int nb_launch) {
  extern __shared__ double lds[];
  const int n = m.n_cells, S = m.halo_stride;
  HaloHead next = halo_head(m, blockIdx.x, nb_real, nb_launch);
  for (int it = blockIdx.x; it < nb_launch; it += gridDim.x) {
    const HaloHead hh = next;
    next = halo_head(m, it + gridDim.x, nb_real, nb_launch);
    const int tile = hh.tile;
    if (tile >= nb_real) continue;
    const int seg = m.seg_of_block[tile];
    if (sc.active != nullptr && sc.active[seg] == 0) continue;
    const double eps = (v != nullptr) ? sc.eps[seg] : 0.0;
    const int base = tile * kFvBlock;
    const int h0 = hh.h0, nh = hh.nh;
    const int c = base + threadIdx.x;
    // the tile and the first kFvBlock halo cells in one round trip
    {
      const int cg0 = c, cg1 = hh.cg1;
      double w0[D], x0[D], w1[D], x1[D];
#pragma unroll
      for (int k = 0; k < D; ++k) w0[k] = x0[k] = w1[k] = x1[k] = 0.0;
      if (cg0 < n) {
        load_w<D>(u, v, eps, n, cg0, w0);
        load_soa<D>(m.xc, n, cg0, x0);
      }
      if (cg1 < n) {
        load_w<D>(u, v, eps, n, cg1, w1);
        load_soa<D>(m.xc, n, cg1, x1);
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        lds[k * S + threadIdx.x] = w0[k];
        lds[(D + k) * S + threadIdx.x] = x0[k];
      }
      if (threadIdx.x < nh)
#pragma unroll
        for (int k = 0; k < D; ++k) {
          lds[k * S + kFvBlock + threadIdx.x] = w1[k];
          lds[(D + k) * S + kFvBlock + threadIdx.x] = x1[k];
        }
    }
    for (int i = threadIdx.x + 2 * kFvBlock; i < kFvBlock + nh; i += kFvBlock) {
      const int cg = m.halo_cells[h0 + i - kFvBlock];
      double w[D], x[D];
      load_w<D>(u, v, eps, n, cg, w);
      load_soa<D>(m.xc, n, cg, x);
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
        gradient_cell<D, kTiledChunk>(m, src, m.slot_loc, threadIdx.x, c, rec, m.slot_mg);
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

// Record of boundary face bf: Gamma, d_b, value, type.
__device__ __forceinline__ void load_bface(const MeshDev& m, int bf, double (&r)[kBfaceRec]) {
  const double* p = m.bface + size_t(bf) * kBfaceRec;
#pragma unroll
  for (int k = 0; k < kBfaceRec; ++k) r[k] = p[k];
}

// Force on boundary face r of cell P: displacement faces Gamma . sigma_P
// plus the Rhie-Chow term against load * u_bar; symmetry faces the internal
// face force against the mirror image of P (Eq. symm: centroid x_P + 2 h n,
// value R wP, gradient R grad wP R, weight 1/2); traction faces
// load |Gamma| T_bar and pressure faces -load p Gamma (stored pre-multiplied).
template <int D, int LAW>
__device__ __forceinline__ void boundary_face_force(const Law& law, const double (&r)[kBfaceRec], double load,
                                                    const double (&wP)[D], const double (&gP)[D][D],
                                                    double (&f)[D]) {
  const int type = int(r[9]);
  if (type == kBcSymm) {
    double G[D], n[D], xA[D], xB[D], wB[D], gB[D][D], gn[D], ng[D];
    double h = 0, wn = 0, ngn = 0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      G[q] = r[q];
      n[q] = r[6 + q];
      h = fma(r[3 + q], n[q], h);
      wn = fma(wP[q], n[q], wn);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      gn[i] = 0;
      ng[i] = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        gn[i] = fma(gP[i][j], n[j], gn[i]);
        ng[i] = fma(n[j], gP[j][i], ng[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) ngn = fma(n[i], gn[i], ngn);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xA[i] = 0.0;
      xB[i] = 2.0 * h * n[i];
      wB[i] = fma(-2.0 * wn, n[i], wP[i]);
#pragma unroll
      for (int j = 0; j < D; ++j)
        gB[i][j] = gP[i][j] - 2.0 * gn[i] * n[j] - 2.0 * n[i] * ng[j] + 4.0 * ngn * n[i] * n[j];
    }
    internal_face_force<D, LAW>(law, G, 0.5, xA, xB, wP, wB, gP, gB, f);
  } else if (type == kBcDisp) {
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
      f[j] = fma(coef, (ub[j] - wP[j]) - dg, t[j]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < D; ++q) f[q] = load * r[6 + q];
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
        double r[kBfaceRec], f[D];
        load_bface(m, fc[k], r);
        boundary_face_force<D, LAW>(law, r, load, wP, gP, f);
#pragma unroll
        for (int q = 0; q < D; ++q) R[q] += f[q];
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
    else if (si.law == JFNK_ST_VENANT_KIRCHHOFF)
      cell_forces<D, JFNK_ST_VENANT_KIRCHHOFF>(m, law, src, ids, self, c, load, R);
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
    flux_cell<D, LAWSEL>(m, si, src, m.slot_nb, c, c, sc.load_at(seg), Ru ? sc.eps[seg] : 0.0, Ru, out);
  }
}

// Face-parallel evaluation in the LDS passes.
// Face data of up to kEnt entries of the tile's face list (entries
// e = threadIdx.x + j * kFvBlock), loaded before the staging barrier so that
// every global load of the tile is in flight at once.
constexpr int kEnt = 4;
template <int D>
struct FaceBatch {
  int n = 0;
  int pos[kEnt];  // LDS positions: owner (low 16 bits), neighbour (high 16 bits)
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
    fb.pos[j] = packed;
    load_soa<D>(m.fG, m.n_int, f, fb.G[j]);
    fb.wf[j] = m.fw[f];
    fb.n = j + 1;
  }
}

// Phase A: entry j of the loaded faces, owner first (the canonical operand
// order).
template <int D, int LAW, class Src>
__device__ __forceinline__ void one_face_force(const Law& law, const Src& src, const FaceBatch<D>& fb, int j,
                                               double (&fo)[D]) {
  double xA[D], xB[D], wA[D], wB[D], gA[D][D], gB[D][D];
  src.get(fb.pos[j] & 0xffff, wA, gA, xA);
  src.get(fb.pos[j] >> 16, wB, gB, xB);
  internal_face_force<D, LAW>(law, fb.G[j], fb.wf[j], xA, xB, wA, wB, gA, gB, fo);
#if JFNK_FACE_SCHED_BARRIER
  // one neo-Hookean face's operands live at a time: keeps the passes at
  // two waves per SIMD
  if constexpr (LAW == JFNK_NEO_HOOKEAN) __builtin_amdgcn_sched_barrier(0);
#endif
}

// All loaded faces into registers.
template <int D, int LAW, class Src>
__device__ __forceinline__ void face_forces_reg(const SegInfo& si, const Src& src, const FaceBatch<D>& fb,
                                                double (&fo)[kEnt][D]) {
  const Law law{si.mu, si.lam, si.kappa, si.aK};
#pragma unroll
  for (int j = 0; j < kEnt; ++j) {
    if (j >= fb.n) break;
    one_face_force<D, LAW>(law, src, fb, j, fo[j]);
  }
}

template <int D>
__device__ __forceinline__ void store_face_forces(const FaceBatch<D>& fb, const double (&fo)[kEnt][D], int e0,
                                                  double* __restrict__ ff, int fs) {
#pragma unroll
  for (int j = 0; j < kEnt; ++j) {
    if (j >= fb.n) break;
#pragma unroll
    for (int q = 0; q < D; ++q) ff[q * fs + e0 + j * kFvBlock] = fo[j][q];
  }
}

// All loaded faces into the face-force rows, each stored when computed.
template <int D, int LAW, class Src>
__device__ __forceinline__ void face_forces(const SegInfo& si, const Src& src, int e0, const FaceBatch<D>& fb,
                                            double* __restrict__ ff, int fs) {
  const Law law{si.mu, si.lam, si.kappa, si.aK};
#pragma unroll
  for (int j = 0; j < kEnt; ++j) {
    if (j >= fb.n) break;
    double fo[D];
    one_face_force<D, LAW>(law, src, fb, j, fo);
#pragma unroll
    for (int q = 0; q < D; ++q) ff[q * fs + e0 + j * kFvBlock] = fo[q];
  }
}

template <int D, int LAWSEL, class Src>
__device__ __forceinline__ void face_forces_sel(const SegInfo& si, const Src& src, const FaceBatch<D>& fb,
                                                double (&fo)[kEnt][D]) {
  if constexpr (LAWSEL == kLawMixed) {
    if (si.law == JFNK_NEO_HOOKEAN)
      face_forces_reg<D, JFNK_NEO_HOOKEAN>(si, src, fb, fo);
    else if (si.law == JFNK_ST_VENANT_KIRCHHOFF)
      face_forces_reg<D, JFNK_ST_VENANT_KIRCHHOFF>(si, src, fb, fo);
    else
      face_forces_reg<D, JFNK_LINEAR_ELASTIC>(si, src, fb, fo);
  } else {
    face_forces_reg<D, LAWSEL>(si, src, fb, fo);
  }
}

// Phase B: cell c sums its slots in slot order, every face force (internal
// with the sign of its side, boundary) read from LDS.
// Slot codes of one chunk of a cell's slots.
struct SlotChunk {
  int code[kChunk];
};

__device__ __forceinline__ void load_slots(const MeshDev& m, int s0, int width, int lane, int k0, SlotChunk& sl) {
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int idx = s0 + (k0 + k) * kSlice + lane;
    sl.code[k] = k0 + k < width ? m.slot_code[idx] : -1;
  }
}

// first: the cell's first chunk of slots, loaded before the tile's barriers.
template <int D>
__device__ __forceinline__ void tile_cell_sum(const MeshDev& m, int c, const double* __restrict__ ff, int fs,
                                              const SlotChunk& first, double (&R)[D]) {
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
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const int code = cur.code[k];
      if (code >= 0) {
        const int e = code >> 1;
#pragma unroll
        for (int q = 0; q < D; ++q) R[q] += (code & 1) ? -ff[q * fs + e] : ff[q * fs + e];
      }
    }
  }
}

// Phase B of cell c and its output: R(w), or (R(w) - R(u))/eps when jv.
template <int D>
__device__ __forceinline__ void cell_sum_out(const MeshDev& m, int c, const double* __restrict__ ff, int fs,
                                             const SlotChunk& first, double eps, bool jv, const double (&ru)[D],
                                             double* __restrict__ out) {
  const int n = m.n_cells;
  double R[D];
  tile_cell_sum<D>(m, c, ff, fs, first, R);
  if (jv) {
    const double ie = eps != 0.0 ? 1.0 / eps : 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) out[size_t(q) * n + c] = eps != 0.0 ? (R[q] - ru[q]) * ie : 0.0;
  } else {
#pragma unroll
    for (int q = 0; q < D; ++q) out[size_t(q) * n + c] = R[q];
  }
}

// Boundary faces of a tile in phase A: entry tid of the tile's boundary
// list (record loaded ahead of the barriers), the rest (lists longer than
// kFvBlock) loaded in place.
struct BndEntry {
  int loc = -1;
  double r[kBfaceRec];
};

__device__ __forceinline__ void load_bnd(const MeshDev& m, int tile, int eb, BndEntry& be) {
  const int b0 = m.bnd_ptr[tile];
  be.loc = -1;
  if (eb < m.bnd_ptr[tile + 1] - b0) {
    be.loc = m.bnd_loc[b0 + eb];
    load_bface(m, m.bnd_face[b0 + eb], be.r);
  }
}

template <int D, int LAW, class Src>
__device__ __forceinline__ void bnd_force(const SegInfo& si, const Src& src, const BndEntry& be, double load,
                                          double (&f)[D]) {
  const Law law{si.mu, si.lam, si.kappa, si.aK};
  double wP[D], gP[D][D], xP[D];
  src.get(be.loc, wP, gP, xP);
  boundary_face_force<D, LAW>(law, be.r, load, wP, gP, f);
}

template <int D, int LAWSEL, class Src>
__device__ __forceinline__ void bnd_force_sel(const SegInfo& si, const Src& src, const BndEntry& be, double load,
                                              double (&f)[D]) {
  if constexpr (LAWSEL == kLawMixed) {
    if (si.law == JFNK_NEO_HOOKEAN)
      bnd_force<D, JFNK_NEO_HOOKEAN>(si, src, be, load, f);
    else if (si.law == JFNK_ST_VENANT_KIRCHHOFF)
      bnd_force<D, JFNK_ST_VENANT_KIRCHHOFF>(si, src, be, load, f);
    else
      bnd_force<D, JFNK_LINEAR_ELASTIC>(si, src, be, load, f);
  } else {
    bnd_force<D, LAWSEL>(si, src, be, load, f);
  }
}

// Tiled flux pass.  The records and centroids of the tile's cells and halo
// are staged in LDS (rows of length halo_stride).  Phase A evaluates every
// face touching the tile once (its boundary faces, then its internal faces,
// owner first, the canonical operand order), spread evenly over the
// workgroup, into LDS; phase B sums each cell's slots in slot order, the
// same sequence of operations as the gather pass, so both give the same
// bits.  Exits before a barrier are uniform over the workgroup.
template <int D, int LAWSEL>
__global__ __launch_bounds__(kFvBlock, JFNK_TILED_MINWAVES) void k_flux_tiled(MeshDev m, const double* __restrict__ rec,
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
    const int n_bnd = m.bnd_ptr[tile + 1] - m.bnd_ptr[tile];
    FaceBatch<D> fb;
    load_faces<D>(m, tile, threadIdx.x, fb);
    // boundary entries from the last lane down: the first lanes also take the
    // last round of internal faces, so no lane gets more than its share
    const int eb0 = kFvBlock - 1 - int(threadIdx.x);
    BndEntry be;
    load_bnd(m, tile, eb0, be);
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
    // the tile and the first kFvBlock halo cells in one round trip
    {
      const int cg0 = c, cg1 = threadIdx.x < nh ? m.halo_cells[h0 + threadIdx.x] : n;
      double r0[kRows], r1[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) r0[r] = r1[r] = 0.0;
      if (cg0 < n) {
#pragma unroll
        for (int r = 0; r < D + D * D; ++r) r0[r] = rec[size_t(r) * n + cg0];
#pragma unroll
        for (int k = 0; k < D; ++k) r0[D + D * D + k] = m.xc[size_t(k) * n + cg0];
      }
      if (cg1 < n) {
#pragma unroll
        for (int r = 0; r < D + D * D; ++r) r1[r] = rec[size_t(r) * n + cg1];
#pragma unroll
        for (int k = 0; k < D; ++k) r1[D + D * D + k] = m.xc[size_t(k) * n + cg1];
      }
#pragma unroll
      for (int r = 0; r < kRows; ++r) lds[r * S + threadIdx.x] = r0[r];
      if (threadIdx.x < nh)
#pragma unroll
        for (int r = 0; r < kRows; ++r) lds[r * S + kFvBlock + threadIdx.x] = r1[r];
    }
    for (int i = threadIdx.x + 2 * kFvBlock; i < kFvBlock + nh; i += kFvBlock) {
      const int cg = m.halo_cells[h0 + i - kFvBlock];
#pragma unroll
      for (int r = 0; r < D + D * D; ++r) lds[r * S + i] = rec[size_t(r) * n + cg];
#pragma unroll
      for (int k = 0; k < D; ++k) lds[(D + D * D + k) * S + i] = m.xc[size_t(k) * n + cg];
    }
    __syncthreads();
    const SegInfo& si = m.seg[seg];
    const FluxLds<D> src{lds, S};
    // phase A: boundary faces (entries n_ent + eb), one per lane per round
    {
      const double load = sc.load_at(seg);
      for (int eb = eb0; eb < n_bnd; eb += kFvBlock) {
        if (eb != eb0) load_bnd(m, tile, eb, be);
        double f[D];
        bnd_force_sel<D, LAWSEL>(si, src, be, load, f);
#pragma unroll
        for (int q = 0; q < D; ++q) ff[q * fs + n_ent + eb] = f[q];
      }
    }
    // internal faces, kEnt entries per lane per round (one round unless the
    // tile touches more than kEnt * kFvBlock faces)
    for (int e0 = threadIdx.x;; e0 += kEnt * kFvBlock) {
      if (e0 != threadIdx.x) load_faces<D>(m, tile, e0, fb);
      if constexpr (LAWSEL == kLawMixed) {
        if (si.law == JFNK_NEO_HOOKEAN)
          face_forces<D, JFNK_NEO_HOOKEAN>(si, src, e0, fb, ff, fs);
        else if (si.law == JFNK_ST_VENANT_KIRCHHOFF)
          face_forces<D, JFNK_ST_VENANT_KIRCHHOFF>(si, src, e0, fb, ff, fs);
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
        cell_sum_out<D>(m, c, ff, fs, first, Ru ? sc.eps[seg] : 0.0, Ru != nullptr, ru, out);
      } else {
#pragma unroll
        for (int q = 0; q < D; ++q) out[size_t(q) * n + c] = 0.0;  // alignment padding
      }
    }
    __syncthreads();  // the LDS copy is rewritten for the next tile
  }
}

// Fused J v pass: one workgroup per tile, nothing but the result written.
// The tile, its halo and its second ring (the outside cells adjacent to the
// halo) are staged in LDS as w = u + eps v and centroids (rows of length
// ring_stride); the gradients of the tile's cells and of its halo cells are
// computed from that copy into LDS (rows of length halo_stride), in the
// same slot order as the gradient pass; then phase A and phase B of the
// tiled flux pass follow, the face forces overwriting the w/centroid rows
// once phase A has read them (boundary faces wait in a small row of their
// own until then).  Every cell's gradient and every face force
// is the same sequence of operations as in the two passes, so the result
// is the same bits.  Exits before a barrier are uniform over the workgroup.
template <int D>
struct FusedLds {
  const double* wx;  // [D][R] w, then [D][R] centroids
  const double* g;   // [D*D][S] gradients
  int R, S;
  __device__ __forceinline__ void get(int j, double (&w)[D], double (&gr)[D][D], double (&x)[D]) const {
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = wx[k * R + j];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) gr[a][b] = g[(a * D + b) * S + j];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = wx[(D + k) * R + j];
  }
};

constexpr int kStageRounds = 3;
#ifndef JFNK_FUSED_CHUNK
#define JFNK_FUSED_CHUNK 3
#endif
constexpr int kFusedChunk = JFNK_FUSED_CHUNK;  // slots per chunk of the LDS-sourced gradients

template <int D, int LAWSEL>
__global__ __launch_bounds__(kFvBlock, JFNK_FUSED_MINWAVES) void k_jv_fused(MeshDev m, const double* __restrict__ u,
                                                                            const double* __restrict__ v,
                                                                            SegScalars sc,
                                                                            const double* __restrict__ Ru,
                                                                            double* __restrict__ out, int nb_real,
                                                                            int nb_launch, int wx_size) {
  extern __shared__ double lds[];
  const int n = m.n_cells, R = m.ring_stride, S = m.halo_stride, fs = m.face_stride, W = m.h1_width;
  double* wx = lds;
  double* gl = lds + wx_size;
  double* bl = gl + D * D * S;  // boundary face forces until the face rows are free
  double* ff = lds;             // face forces, over the w/centroid rows
  for (int it = blockIdx.x; it < nb_launch; it += gridDim.x) {
    const int tile = xcd_block(it, nb_launch);
    if (tile >= nb_real) continue;
    const int seg = m.seg_of_block[tile];
    if (sc.active != nullptr && sc.active[seg] == 0) continue;
    const double eps = (v != nullptr) ? sc.eps[seg] : 0.0;
    const int base = tile * kFvBlock;
    const int h0 = m.halo_ptr[tile], nh = m.halo_ptr[tile + 1] - h0;
    const int r0 = m.h2_ptr[tile], n2 = m.h2_ptr[tile + 1] - r0;
    const int c = base + threadIdx.x;
    const SegInfo& si = m.seg[seg];
    const bool real = c < n && c - si.cell_off < si.n_cells;
    // Staging, three rounds of the copy at once: indices, then every load,
    // then the LDS writes, so that the copy waits for one round trip to
    // memory after its indices.
    const int total = kFvBlock + nh + n2;
    int cg[kStageRounds];
#pragma unroll
    for (int r = 0; r < kStageRounds; ++r) {
      const int i = threadIdx.x + r * kFvBlock;
      cg[r] = i < kFvBlock        ? base + i
              : i < kFvBlock + nh ? m.halo_cells[h0 + i - kFvBlock]
              : i < total         ? m.h2_cells[r0 + i - kFvBlock - nh]
                                  : n;
    }
    double sw[kStageRounds][D], sx[kStageRounds][D];
#pragma unroll
    for (int r = 0; r < kStageRounds; ++r) {
      if (cg[r] < n) {
        load_w<D>(u, v, eps, n, cg[r], sw[r]);
        load_soa<D>(m.xc, n, cg[r], sx[r]);
      } else {
#pragma unroll
        for (int k = 0; k < D; ++k) sw[r][k] = sx[r][k] = 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < kStageRounds; ++r) {
      const int i = threadIdx.x + r * kFvBlock;
      if (i < total) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
          wx[k * R + i] = sw[r][k];
          wx[(D + k) * R + i] = sx[r][k];
        }
      }
    }
    for (int i = threadIdx.x + kStageRounds * kFvBlock; i < total; i += kFvBlock) {
      const int cgi = i < kFvBlock + nh ? m.halo_cells[h0 + i - kFvBlock] : m.h2_cells[r0 + i - kFvBlock - nh];
      double w[D], x[D];
      load_w<D>(u, v, eps, n, cgi, w);
      load_soa<D>(m.xc, n, cgi, x);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        wx[k * R + i] = w[k];
        wx[(D + k) * R + i] = x[k];
      }
    }
    __syncthreads();
    // gradients of the tile's cells, then of its halo cells
    const GradLds<D> gsrc{wx, R};
    {
      double wP[D], gP[D][D];
      if (real) {
        const int s0 = m.slice_ptr[c / kSlice];
        const SliceSlots sl{m.slot_loc, s0, int(c % kSlice), (m.slice_ptr[c / kSlice + 1] - s0) / kSlice,
                            m.slot_mg};
        lsq_gradient<D, kFusedChunk>(m, gsrc, sl, threadIdx.x, wP, gP);
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          wP[a] = 0.0;
#pragma unroll
          for (int b = 0; b < D; ++b) gP[a][b] = 0.0;
        }
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) gl[(a * D + b) * S + threadIdx.x] = gP[a][b];
    }
    for (int i = threadIdx.x; i < nh; i += kFvBlock) {
      const HaloSlots hi{m.h1_loc + size_t(h0) * W, m.h1_mg + size_t(h0) * W, nh, i, W,
                         m.h1_fc != nullptr ? m.h1_fc + size_t(h0) * W : nullptr};
      double wH[D], gH[D][D];
      lsq_gradient<D, kFusedChunk>(m, gsrc, hi, kFvBlock + i, wH, gH);
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) gl[(a * D + b) * S + kFvBlock + i] = gH[a][b];
    }
    // this lane's faces, in flight while the slower lanes finish (a tile
    // has at most kEnt * kFvBlock internal and kFvBlock boundary faces)
    FaceBatch<D> fb;
    load_faces<D>(m, tile, threadIdx.x, fb);
    __syncthreads();
    // phase A into registers; the face forces replace the w/centroid rows
    // once every lane has read them.  Boundary entries go from the last
    // lane down (the first lanes also take the last round of internal faces).
    {
      const int eb0 = kFvBlock - 1 - int(threadIdx.x);
      BndEntry be;
      load_bnd(m, tile, eb0, be);
      const int n_ent = m.fbeg[tile + 1] - m.fbeg[tile] + m.in_ptr[tile + 1] - m.in_ptr[tile];
      const FusedLds<D> src{wx, gl, R, S};
      if (be.loc >= 0) {
        double f[D];
        bnd_force_sel<D, LAWSEL>(si, src, be, sc.load_at(seg), f);
#pragma unroll
        for (int q = 0; q < D; ++q) bl[q * kFvBlock + threadIdx.x] = f[q];
      }
      double fo[kEnt][D];
      face_forces_sel<D, LAWSEL>(si, src, fb, fo);
      __syncthreads();
      if (be.loc >= 0)
#pragma unroll
        for (int q = 0; q < D; ++q) ff[q * fs + n_ent + eb0] = bl[q * kFvBlock + threadIdx.x];
      store_face_forces<D>(fb, fo, threadIdx.x, ff, fs);
    }
    __syncthreads();
    if (c < n) {
      if (real) {
        const int s0 = m.slice_ptr[c / kSlice];
        SlotChunk first;
        load_slots(m, s0, (m.slice_ptr[c / kSlice + 1] - s0) / kSlice, c % kSlice, 0, first);
        double ru[D];
#pragma unroll
        for (int q = 0; q < D; ++q) ru[q] = Ru != nullptr ? Ru[size_t(q) * n + c] : 0.0;
        cell_sum_out<D>(m, c, ff, fs, first, Ru ? sc.eps[seg] : 0.0, Ru != nullptr, ru, out);
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

template <int D, int LAWSEL>
void fused_launch(const MeshDev& m, const double* u, const double* v, const SegScalars& sc, const double* Ru,
                  double* out, hipStream_t s) {
  int nr, nl, g;
  grid_for(m, nr, nl, g);
  const int wx = fused_wx_doubles(D, m.ring_stride, m.face_stride);
  const size_t lds = fused_lds_bytes(D, m.ring_stride, m.halo_stride, m.face_stride);
  hipLaunchKernelGGL((k_jv_fused<D, LAWSEL>), dim3(g), dim3(kFvBlock), lds, s, m, u, v, sc, Ru, out, nr, nl, wx);
}

}  // namespace

void launch_fused(const MeshDev& m, const double* u, const double* v, const SegScalars& sc, const double* Ru,
                  double* out, hipStream_t s) {
  const int mask = m.law_mask;
  if (m.dim == 3) {
    if (mask == 2)
      fused_launch<3, JFNK_NEO_HOOKEAN>(m, u, v, sc, Ru, out, s);
    else if (mask == 4)
      fused_launch<3, JFNK_ST_VENANT_KIRCHHOFF>(m, u, v, sc, Ru, out, s);
    else if (mask == 1)
      fused_launch<3, JFNK_LINEAR_ELASTIC>(m, u, v, sc, Ru, out, s);
    else
      fused_launch<3, kLawMixed>(m, u, v, sc, Ru, out, s);
  } else {
    if (mask == 2)
      fused_launch<2, JFNK_NEO_HOOKEAN>(m, u, v, sc, Ru, out, s);
    else if (mask == 4)
      fused_launch<2, JFNK_ST_VENANT_KIRCHHOFF>(m, u, v, sc, Ru, out, s);
    else if (mask == 1)
      fused_launch<2, JFNK_LINEAR_ELASTIC>(m, u, v, sc, Ru, out, s);
    else
      fused_launch<2, kLawMixed>(m, u, v, sc, Ru, out, s);
  }
  JFNK_HIP(hipGetLastError());
}

void launch_flux(const MeshDev& m, const double* rec, const SegScalars& sc, const double* Ru, double* out,
                 hipStream_t s) {
  const int mask = m.law_mask;
  if (m.dim == 3) {
    if (mask == 2)
      flux_launch<3, JFNK_NEO_HOOKEAN>(m, rec, sc, Ru, out, s);
    else if (mask == 4)
      flux_launch<3, JFNK_ST_VENANT_KIRCHHOFF>(m, rec, sc, Ru, out, s);
    else if (mask == 1)
      flux_launch<3, JFNK_LINEAR_ELASTIC>(m, rec, sc, Ru, out, s);
    else
      flux_launch<3, kLawMixed>(m, rec, sc, Ru, out, s);
  } else {
    if (mask == 2)
      flux_launch<2, JFNK_NEO_HOOKEAN>(m, rec, sc, Ru, out, s);
    else if (mask == 4)
      flux_launch<2, JFNK_ST_VENANT_KIRCHHOFF>(m, rec, sc, Ru, out, s);
    else if (mask == 1)
      flux_launch<2, JFNK_LINEAR_ELASTIC>(m, rec, sc, Ru, out, s);
    else
      flux_launch<2, kLawMixed>(m, rec, sc, Ru, out, s);
  }
  JFNK_HIP(hipGetLastError());
}

}  // namespace jfnk
