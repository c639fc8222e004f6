// Segregated solution procedure (Section 3.1): the quasi-Newton iteration
// J_tilde du = -R(u_k) of Eq. SegSys, each displacement component's system
// (Eq. SegSysX-Z) solved by preconditioned conjugate gradients on
// A = -J_tilde (symmetric positive definite) until its residual has fallen
// by the inner factor (Section 3.2 uses 0.9).  The paper's baseline for the
// Jacobian-free Newton-Krylov method, built on the same residual kernels and
// the same approximate Jacobian.  Single-mesh handles; the CG scalars of
// the components live on the device, one host read per CG iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "reduce_dev.h"
#include "solver.h"

namespace jfnk {

namespace {

constexpr int kB = 256;

inline int blocks_for(int64_t n) { return int((n + kB - 1) / kB); }

double wall_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// y = A x, A = -J_tilde: the diagonal ad[q * ds + c] (ds = 0: shared by the
// components) and the off-diagonal ao[f] of every internal face, gathered
// over the cell's slots.
template <int D>
__global__ __launch_bounds__(kB) void k_jt_apply(MeshDev m, const double* __restrict__ ad, int ds,
                                                 const double* __restrict__ ao, const double* __restrict__ x,
                                                 double* __restrict__ y) {
  const int n = m.n_cells;
  const int c = blockIdx.x * kB + threadIdx.x;
  if (c >= n) return;
  double s[D];
#pragma unroll
  for (int q = 0; q < D; ++q) s[q] = ad[size_t(q) * ds + c] * x[size_t(q) * n + c];
  const int slice = c / kSlice, lane = c % kSlice;
  const int s0 = m.slice_ptr[slice], width = (m.slice_ptr[slice + 1] - s0) / kSlice;
  for (int k = 0; k < width; ++k) {
    const int idx = s0 + k * kSlice + lane;
    const int nb = m.slot_nb[idx];
    if (nb < 0) continue;
    const int fc = m.slot_fc[idx];
    const double a = ao[fc >= 0 ? fc : ~fc];
#pragma unroll
    for (int q = 0; q < D; ++q) s[q] = fma(a, x[size_t(q) * n + nb], s[q]);
  }
#pragma unroll
  for (int q = 0; q < D; ++q) y[size_t(q) * n + c] = s[q];
}

// Per-component dot products over one workgroup's cells:
// part[blk * 2D + q] = a_q . b_q and, when c is given, part[blk * 2D + D + q] = c_q . d_q.
template <int D>
__global__ __launch_bounds__(kB) void k_dots(int n, const double* __restrict__ a, const double* __restrict__ b,
                                             const double* __restrict__ c, const double* __restrict__ d,
                                             double* __restrict__ part) {
  __shared__ double sh[4];
  const int i = blockIdx.x * kB + threadIdx.x;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * n + i;
    double t = block_sum(i < n ? a[o] * b[o] : 0.0, sh);
    if (threadIdx.x == 0) part[size_t(blockIdx.x) * 2 * D + q] = t;
    if (c != nullptr) {
      t = block_sum(i < n ? c[o] * d[o] : 0.0, sh);
      if (threadIdx.x == 0) part[size_t(blockIdx.x) * 2 * D + D + q] = t;
    }
  }
}

// out[j] = sum over the workgroups of part[blk * 2D + j], j < 2D, in a fixed
// order (one workgroup).
template <int D>
__global__ __launch_bounds__(kB) void k_dots_finish(int nblk, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double sh[4];
  for (int j = 0; j < 2 * D; ++j) {
    double x = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kB) x += part[size_t(b) * 2 * D + j];
    x = block_sum(x, sh);
    if (threadIdx.x == 0) out[j] = x;
  }
}

// CG scalars of the components, st[]: rz [0, D), rr0 [D, 2D), alpha [2D, 3D),
// beta [3D, 4D), active [4D, 5D), active count [5D]; dots: the latest k_dots
// result.
template <int D>
__global__ void k_cg_init(const double* __restrict__ dots, double* __restrict__ st) {
  if (threadIdx.x != 0) return;
  double cnt = 0;
  for (int q = 0; q < D; ++q) {
    st[q] = dots[q];                      // r . z
    st[D + q] = dots[D + q];              // r . r at the start
    st[2 * D + q] = st[3 * D + q] = 0.0;
    st[4 * D + q] = dots[D + q] > 0.0 ? 1.0 : 0.0;
    cnt += st[4 * D + q];
  }
  st[5 * D] = cnt;
}

template <int D>
__global__ void k_cg_alpha(const double* __restrict__ dots, double* __restrict__ st) {
  if (threadIdx.x != 0) return;
  for (int q = 0; q < D; ++q) {
    const double pq = dots[q];
    st[2 * D + q] = (st[4 * D + q] != 0.0 && pq > 0.0) ? st[q] / pq : 0.0;
  }
}

// after the new r . z and r . r: components whose residual fell below tol2
// times the start (squared) stop; beta for the others
template <int D>
__global__ void k_cg_beta(const double* __restrict__ dots, double tol2, double* __restrict__ st) {
  if (threadIdx.x != 0) return;
  double cnt = 0;
  for (int q = 0; q < D; ++q) {
    if (st[4 * D + q] == 0.0) continue;
    const double rz = dots[q], rr = dots[D + q];
    if (!(rr > tol2 * st[D + q]) || st[q] == 0.0) {
      st[4 * D + q] = 0.0;
      st[3 * D + q] = 0.0;
      continue;
    }
    st[3 * D + q] = rz / st[q];
    st[q] = rz;
    cnt += 1.0;
  }
  st[5 * D] = cnt;
}

// x_q += alpha_q p_q, r_q -= alpha_q w_q
template <int D>
__global__ __launch_bounds__(kB) void k_cg_update(int n, const double* __restrict__ st, const double* __restrict__ p,
                                                  const double* __restrict__ w, double* __restrict__ x,
                                                  double* __restrict__ r) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const double a = st[2 * D + q];
    const size_t o = size_t(q) * n + i;
    x[o] = fma(a, p[o], x[o]);
    r[o] = fma(-a, w[o], r[o]);
  }
}

// p_q = z_q + beta_q p_q for the components still iterating
template <int D>
__global__ __launch_bounds__(kB) void k_cg_direction(int n, const double* __restrict__ st,
                                                     const double* __restrict__ z, double* __restrict__ p) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    if (st[4 * D + q] == 0.0) continue;
    const size_t o = size_t(q) * n + i;
    p[o] = fma(st[3 * D + q], p[o], z[o]);
  }
}

#define JFNK_SEG_DISPATCH(dim, KERNEL, grid, ...)                                   \
  do {                                                                             \
    if ((dim) == 3)                                                                \
      hipLaunchKernelGGL((KERNEL<3>), grid, dim3(kB), 0, s, __VA_ARGS__);          \
    else                                                                           \
      hipLaunchKernelGGL((KERNEL<2>), grid, dim3(kB), 0, s, __VA_ARGS__);          \
    JFNK_HIP(hipGetLastError());                                                   \
  } while (0)

// A = -J_tilde on the device: the diagonal (with the inertia term of the
// current time step and, with symmetry faces, per component) and the
// off-diagonal of every internal face.
void ensure_jtilde(jfnk_mesh* m, hipStream_t s) {
  if (m->seg_jt_ready && m->seg_jt_dt == m->pc_dt) return;
  const HostMesh& h = m->host;
  const int D = h.dim;
  const int64_t N = h.n_cells;
  const std::vector<double>& diag = m->pc_diag_eff.empty() ? h.pc_diag : m->pc_diag_eff;
  std::vector<double> ad(h.pc_sym.empty() ? size_t(N) : size_t(N) * D);
  if (h.pc_sym.empty()) {
    for (int64_t c = 0; c < N; ++c) ad[c] = -diag[c];
  } else {
    for (int q = 0; q < D; ++q)
      for (int64_t c = 0; c < N; ++c) ad[size_t(q) * N + c] = -(diag[c] + h.pc_sym[size_t(c) * D + q]);
  }
  std::vector<double> ao(std::max<int64_t>(h.n_int, 1), 0.0);
  for (int64_t f = 0; f < h.n_int; ++f) ao[f] = -h.pc_off[f];
  for (auto [buf, v] : {std::pair<DevBuf*, const std::vector<double>*>{&m->b_seg_ad, &ad}, {&m->b_seg_ao, &ao}}) {
    if (buf->bytes < v->size() * sizeof(double)) buf->alloc(v->size() * sizeof(double));
    JFNK_HIP(hipMemcpyAsync(buf->p, v->data(), v->size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  JFNK_HIP(hipStreamSynchronize(s));
  m->seg_jt_ready = true;
  m->seg_jt_dt = m->pc_dt;
}

}  // namespace

void segregated_solve(jfnk_mesh* m, const jfnk_segregated_opts& o, double* u, FvWork& fw, KrylovWork& kw,
                      hipStream_t s, jfnk_stats& st, jfnk_status& status) {
  const double t0 = wall_ms();
  const int D = m->dev.dim;
  const int N = m->dev.n_cells;
  const int64_t n = int64_t(N) * D;
  const SegLayout L = layout_of(m);
  ensure_jtilde(m, s);
  precond_setup(m, o.precond, s);
  const double* ad = m->b_seg_ad.as<double>();
  const int ds = m->host.pc_sym.empty() ? 0 : N;
  const double* ao = m->b_seg_ao.as<double>();
  double* R = kw.R;
  double* du = kw.du;
  double* r = kw.r;
  double* z = kw.w;
  double* p = kw.b;
  double* w = kw.V;
  double* sc = kw.h;      // CG scalars (5D + 1)
  double* dots = kw.h2;   // latest dot products (2D)
  const int nblk = blocks_for(N);
  const dim3 grid(nblk);
  const double tol2 = o.inner_rtol * o.inner_rtol;
  auto dots2 = [&](const double* a, const double* b, const double* c, const double* d) {
    JFNK_SEG_DISPATCH(D, k_dots, grid, N, a, b, c, d, fw.partials);
    JFNK_SEG_DISPATCH(D, k_dots_finish, dim3(1), nblk, fw.partials, dots);
  };
  // z = -P^{-1} r: the preconditioner approximates J_tilde^{-1} = -A^{-1}
  auto precondition = [&]() {
    precond_apply(m, o.precond, o.cheb_degree, r, z, kw, s, false);
    blas_lincomb(-1.0, z, 0.0, z, z, n, s);
  };
  volatile double* host = m->pinned;
  st = jfnk_stats{};
  status = JFNK_OK;
  std::vector<double> nr;
  const int N_inc = o.n_increments;
  for (int k = 1; k <= N_inc && status == JFNK_OK; ++k) {
    fw.setup(s, double(k) / N_inc);
    fw.uniform = false;
    residual_into(m, u, R, fw, nullptr, s);
    seg_norms2(m, L, R, fw, kw, nullptr, s, nr);
    const double r0 = std::sqrt(nr[0]);
    st.res0 = r0;
    double rn = r0;
    int it = 0;
    while (true) {
      if (!std::isfinite(rn)) {
        status = JFNK_E_NAN;
        break;
      }
      if (rn <= std::max(o.rtol * r0, o.atol)) break;
      if (it >= o.max_outer_it) {
        status = JFNK_E_NOT_CONVERGED;
        break;
      }
      // A du = R from du = 0, each component to inner_rtol
      fill_device(du, n, 0.0, s);
      blas_lincomb(1.0, R, 0.0, R, r, n, s);
      precondition();
      blas_lincomb(1.0, z, 0.0, z, p, n, s);
      dots2(r, z, r, r);
      JFNK_SEG_DISPATCH(D, k_cg_init, dim3(1), dots, sc);
      for (int j = 0; j < o.max_inner_it; ++j) {
        JFNK_SEG_DISPATCH(D, k_jt_apply, grid, m->dev, ad, ds, ao, p, w);
        dots2(p, w, nullptr, nullptr);
        JFNK_SEG_DISPATCH(D, k_cg_alpha, dim3(1), dots, sc);
        JFNK_SEG_DISPATCH(D, k_cg_update, grid, N, sc, p, w, du, r);
        precondition();
        dots2(r, z, r, r);
        JFNK_SEG_DISPATCH(D, k_cg_beta, dim3(1), dots, tol2, sc);
        JFNK_HIP(hipMemcpyAsync((void*)host, sc + 5 * D, sizeof(double), hipMemcpyDeviceToHost, s));
        JFNK_HIP(hipStreamSynchronize(s));
        st.gmres_it++;
        if (host[0] == 0.0) break;
        JFNK_SEG_DISPATCH(D, k_cg_direction, grid, N, sc, z, p);
      }
      blas_axpby(1.0, du, 1.0, u, n, s);
      residual_into(m, u, R, fw, nullptr, s);
      seg_norms2(m, L, R, fw, kw, nullptr, s, nr);
      rn = std::sqrt(nr[0]);
      ++it;
      st.newton_it++;
    }
    st.res_final = rn;
  }
  st.t_ms[0] = wall_ms() - t0;
}

}  // namespace jfnk
