// GMRES and Newton drivers on the host for one mesh or a batch of meshes
// (segments) solved in lockstep; all vector work runs in the HIP kernels of
// fv_kernels.hip / blas.hip / amg_kernels.hip.
//
// GMRES (Section 3.2): restarted, right preconditioned; the preconditioned
// directions z_j = P^{-1} v_j are kept (flexible form), so a variable
// preconditioner such as the FP32 V-cycle is allowed.  Arnoldi uses
// classical Gram-Schmidt applied twice.  Every segment has its own
// Hessenberg matrix, Givens rotations, tolerance and convergence; the host
// receives the new Hessenberg columns of all segments with one strided copy
// per Arnoldi step and switches finished segments off through device flags,
// so their workgroups return at once.  Each restart cycle ends with the true
// residual b - J x.
//
// Newton (Eq. NewtonRaphson, s = 1) with equal load increments k/N per
// segment (N may differ between segments); convergence per increment when
// |R(u)| <= max(rtol |R(u_0)|, atol) (Section 3.3, Euclidean norm, stol = 0);
// linear solves to the relative tolerance eta.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "solver.h"

namespace jfnk {

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

__global__ void k_fill(double* d, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = v;
}

// Per-segment squared norms of x (device scratch kw.nrm, column 0).
void seg_norms2(jfnk_mesh* m, const SegLayout& L, const double* x, FvWork& fw, KrylovWork& kw,
                const int32_t* act, hipStream_t s, std::vector<double>& out) {
  const int S = m->n_seg();
  blas_mdot(L, x, 0, 1, x, fw.partials, kw.nrm, 4, false, act, s);
  JFNK_HIP(hipMemcpy2DAsync(m->pinned, sizeof(double), kw.nrm, 4 * sizeof(double), sizeof(double), S,
                            hipMemcpyDeviceToHost, s));
  JFNK_HIP(hipStreamSynchronize(s));
  out.assign(m->pinned, m->pinned + S);
}

// Host -> device through the second half of the pinned buffer; waits so the
// staging area can be reused.
void upload_flags(jfnk_mesh* m, const std::vector<char>& flag, int32_t* d_act, hipStream_t s) {
  int32_t* p = reinterpret_cast<int32_t*>(m->pinned + m->pinned_doubles / 2);
  for (size_t i = 0; i < flag.size(); ++i) p[i] = flag[i] ? 1 : 0;
  JFNK_HIP(hipMemcpyAsync(d_act, p, sizeof(int32_t) * flag.size(), hipMemcpyHostToDevice, s));
  JFNK_HIP(hipStreamSynchronize(s));
}

void upload_doubles(jfnk_mesh* m, const std::vector<double>& v, double* d, hipStream_t s) {
  double* p = m->pinned + m->pinned_doubles / 2;
  std::copy(v.begin(), v.end(), p);
  JFNK_HIP(hipMemcpyAsync(d, p, sizeof(double) * v.size(), hipMemcpyHostToDevice, s));
  JFNK_HIP(hipStreamSynchronize(s));
}

}  // namespace

SegLayout layout_of(const jfnk_mesh* m) {
  SegLayout L;
  L.n_cells = m->dev.n_cells;
  L.dim = m->dev.dim;
  L.n_seg = m->n_seg();
  L.n_blocks = int32_t(n_tiles(m));
  L.seg_of_block = m->dev.seg_of_block;
  L.block_first = m->b_block_first.as<int32_t>();
  return L;
}

void fill_device(double* d, int n, double value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, d, n, value);
  JFNK_HIP(hipGetLastError());
}

void residual_into(jfnk_mesh* m, const double* u, double* R, FvWork& fw, const int32_t* active,
                   hipStream_t s) {
  Profiler& p = m->prof;
  SegScalars sc{nullptr, fw.load, active};
  int t = p.on ? p.begin(1, s) : -1;
  launch_gradient(m->dev, u, nullptr, sc, fw.grad, s);
  if (t >= 0) p.end(t, s);
  t = p.on ? p.begin(2, s) : -1;
  launch_flux(m->dev, fw.grad, sc, nullptr, R, s);
  if (t >= 0) p.end(t, s);
}

void jv_into(jfnk_mesh* m, const double* u, const double* Ru, const double* v, double eps, double* Jv,
             FvWork& fw, const int32_t* active, hipStream_t s) {
  Profiler& p = m->prof;
  int t = p.on ? p.begin(0, s) : -1;
  if (eps > 0)
    fill_device(fw.eps, m->n_seg(), eps, s);
  else
    launch_eps(m->dev, m->b_block_first.as<int32_t>(), u, v, fw.partials, fw.eps, active, s);
  if (t >= 0) p.end(t, s);
  SegScalars sc{fw.eps, fw.load, active};
  t = p.on ? p.begin(1, s) : -1;
  launch_gradient(m->dev, u, v, sc, fw.grad, s);
  if (t >= 0) p.end(t, s);
  t = p.on ? p.begin(2, s) : -1;
  launch_flux(m->dev, fw.grad, sc, Ru, Jv, s);
  if (t >= 0) p.end(t, s);
}

void gmres_solve(jfnk_mesh* m, const double* u, const double* Ru, const double* b, double* x,
                 bool x_is_zero, const jfnk_gmres_opts& o, FvWork& fw, KrylovWork& kw, hipStream_t s,
                 const std::vector<char>& part_in, std::vector<GmresSeg>& out, double* t_ms) {
  const int S = m->n_seg();
  const int64_t n = int64_t(m->dev.n_cells) * m->dev.dim;
  const int mr = o.restart;
  const SegLayout L = layout_of(m);
  const double t0 = now_ms();
  std::vector<char> part = part_in.empty() ? std::vector<char>(S, 1) : part_in;
  out.assign(S, GmresSeg());
  upload_flags(m, part, kw.act, s);
  std::vector<double> v2;
  seg_norms2(m, L, b, fw, kw, kw.act, s, v2);
  std::vector<double> target(S), beta(S), prev(S);
  std::vector<int> stalls(S, 0);
  std::vector<char> done(S, 0);
  for (int g = 0; g < S; ++g) {
    out[g].bnorm = part[g] ? std::sqrt(v2[g]) : 0.0;
    target[g] = std::max(o.rtol * out[g].bnorm, o.atol);
    if (!part[g]) done[g] = 1;
    if (part[g] && !std::isfinite(out[g].bnorm)) {
      out[g].status = JFNK_E_NAN;
      done[g] = 1;
    }
  }
  // r = b - J x
  if (x_is_zero) {
    JFNK_HIP(hipMemcpyAsync(kw.r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  } else {
    jv_into(m, u, Ru, x, o.eps, kw.w, fw, kw.act, s);
    for (int g = 0; g < S; ++g) out[g].jv += part[g];
    blas_lincomb(1.0, b, -1.0, kw.w, kw.r, n, s);
  }
  seg_norms2(m, L, kw.r, fw, kw, kw.act, s, v2);
  for (int g = 0; g < S; ++g) {
    beta[g] = std::sqrt(v2[g]);
    prev[g] = beta[g];
    out[g].res_true = beta[g];
  }
  const size_t ldH = size_t(mr + 1);
  std::vector<double> H(size_t(S) * ldH * mr), cs(size_t(S) * mr), sn(size_t(S) * mr),
      gv(size_t(S) * (mr + 1));
  std::vector<double> yv(size_t(S) * kMaxBasis), fac(S);
  std::vector<int> kk(S);
  std::vector<char> act(S);
  while (true) {
    // which segments run a cycle
    bool any = false;
    for (int g = 0; g < S; ++g) {
      act[g] = 0;
      if (done[g]) continue;
      if (!std::isfinite(beta[g])) {
        out[g].status = JFNK_E_NAN;
        done[g] = 1;
      } else if (beta[g] <= target[g] || out[g].bnorm == 0.0) {
        out[g].status = JFNK_OK;
        done[g] = 1;
      } else if (out[g].iterations >= o.max_it) {
        out[g].status = JFNK_E_NOT_CONVERGED;
        done[g] = 1;
      } else {
        act[g] = 1;
        any = true;
      }
    }
    if (!any) break;
    std::vector<char> ran = act;
    upload_flags(m, act, kw.act, s);
    for (int g = 0; g < S; ++g) fac[g] = act[g] ? 1.0 / beta[g] : 0.0;
    upload_doubles(m, fac, kw.fac, s);
    blas_scale_seg(L, kw.r, kw.fac, kw.V, kw.act, s);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    std::fill(kk.begin(), kk.end(), 0);
    for (int g = 0; g < S; ++g) gv[size_t(g) * (mr + 1)] = beta[g];
    for (int j = 0; j < mr; ++j) {
      double* Vj = kw.V + size_t(j) * n;
      double* Zj = kw.Z + size_t(j) * n;
      const double tp = now_ms();
      if (o.precond == JFNK_PC_NONE)
        JFNK_HIP(hipMemcpyAsync(Zj, Vj, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      else
        precond_apply(m, o.precond, o.cheb_degree, Vj, Zj, kw, s);
      const double tj = now_ms();
      jv_into(m, u, Ru, Zj, o.eps, kw.w, fw, kw.act, s);
      const double tc = now_ms();
      // |w| before orthogonalisation (breakdown test), then CGS2
      blas_mdot(L, kw.w, 0, 1, kw.w, fw.partials, kw.nrm + 1, 4, false, kw.act, s);
      blas_mdot(L, kw.V, n, j + 1, kw.w, fw.partials, kw.h, kMaxBasis, false, kw.act, s);
      blas_combine(L, kw.V, n, j + 1, kw.h, kMaxBasis, -1.0, kw.w, kw.act, s);
      blas_mdot(L, kw.V, n, j + 1, kw.w, fw.partials, kw.h2, kMaxBasis, false, kw.act, s);
      blas_combine(L, kw.V, n, j + 1, kw.h2, kMaxBasis, -1.0, kw.w, kw.act, s);
      blas_mdot(L, kw.w, 0, 1, kw.w, fw.partials, kw.nrm, 4, false, kw.act, s);
      // Hessenberg columns of all segments: [S][j+1] twice, norms [S][4]
      double* ph = m->pinned;
      double* ph2 = ph + size_t(S) * (j + 1);
      double* pn = ph2 + size_t(S) * (j + 1);
      JFNK_HIP(hipMemcpy2DAsync(ph, sizeof(double) * (j + 1), kw.h, sizeof(double) * kMaxBasis,
                                sizeof(double) * (j + 1), S, hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipMemcpy2DAsync(ph2, sizeof(double) * (j + 1), kw.h2, sizeof(double) * kMaxBasis,
                                sizeof(double) * (j + 1), S, hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipMemcpyAsync(pn, kw.nrm, sizeof(double) * 4 * S, hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipStreamSynchronize(s));
      if (t_ms) {
        t_ms[3] += tj - tp;
        t_ms[1] += tc - tj;
        t_ms[2] += now_ms() - tc;
      }
      bool still = false;
      for (int g = 0; g < S; ++g) {
        fac[g] = 0.0;
        if (!act[g]) continue;
        out[g].jv++;
        const double hn = std::sqrt(pn[4 * g]);
        const double w0 = std::sqrt(pn[4 * g + 1]);
        double* Hj = &H[(size_t(g) * mr + j) * ldH];
        double* c = &cs[size_t(g) * mr];
        double* sg = &sn[size_t(g) * mr];
        double* gg = &gv[size_t(g) * (mr + 1)];
        for (int i = 0; i <= j; ++i) Hj[i] = ph[size_t(g) * (j + 1) + i] + ph2[size_t(g) * (j + 1) + i];
        Hj[j + 1] = hn;
        if (!std::isfinite(hn) || !std::isfinite(w0)) {
          out[g].status = JFNK_E_NAN;
          done[g] = 1;
          act[g] = 0;
          ran[g] = 0;
          continue;
        }
        for (int i = 0; i < j; ++i) {
          const double t = c[i] * Hj[i] + sg[i] * Hj[i + 1];
          Hj[i + 1] = -sg[i] * Hj[i] + c[i] * Hj[i + 1];
          Hj[i] = t;
        }
        const double rr = std::hypot(Hj[j], Hj[j + 1]);
        c[j] = Hj[j] / rr;
        sg[j] = Hj[j + 1] / rr;
        Hj[j] = rr;
        Hj[j + 1] = 0.0;
        gg[j + 1] = -sg[j] * gg[j];
        gg[j] = c[j] * gg[j];
        out[g].iterations++;
        kk[g] = j + 1;
        const bool breakdown = hn <= 1e-14 * std::max(w0, 1e-300);
        if (breakdown || std::fabs(gg[j + 1]) <= target[g] || out[g].iterations >= o.max_it) {
          act[g] = 0;
        } else {
          fac[g] = 1.0 / hn;
          still = true;
        }
      }
      if (!still || j + 1 == mr) break;
      upload_flags(m, act, kw.act, s);
      upload_doubles(m, fac, kw.fac, s);
      blas_scale_seg(L, kw.w, kw.fac, kw.V + size_t(j + 1) * n, kw.act, s);
    }
    // y = H^{-1} g per segment, x += Z y
    int kmax = 0;
    std::fill(yv.begin(), yv.end(), 0.0);
    for (int g = 0; g < S; ++g) {
      if (!ran[g]) continue;
      const int k = kk[g];
      kmax = std::max(kmax, k);
      const double* gg = &gv[size_t(g) * (mr + 1)];
      double* y = &yv[size_t(g) * kMaxBasis];
      for (int i = k - 1; i >= 0; --i) {
        double t = gg[i];
        for (int l = i + 1; l < k; ++l) t -= H[(size_t(g) * mr + l) * ldH + i] * y[l];
        y[i] = t / H[(size_t(g) * mr + i) * ldH + i];
      }
      out[g].restarts++;
    }
    if (kmax == 0) continue;
    upload_flags(m, ran, kw.act, s);
    upload_doubles(m, yv, kw.y, s);
    blas_combine(L, kw.Z, n, kmax, kw.y, kMaxBasis, 1.0, x, kw.act, s);
    // true residual
    jv_into(m, u, Ru, x, o.eps, kw.w, fw, kw.act, s);
    blas_lincomb(1.0, b, -1.0, kw.w, kw.r, n, s);
    seg_norms2(m, L, kw.r, fw, kw, kw.act, s, v2);
    for (int g = 0; g < S; ++g) {
      if (!ran[g]) continue;
      out[g].jv++;
      beta[g] = std::sqrt(v2[g]);
      out[g].res_true = beta[g];
      if (beta[g] > 0.999 * prev[g] && beta[g] > target[g]) {
        if (++stalls[g] >= 3) {
          out[g].status = JFNK_E_BREAKDOWN;
          done[g] = 1;
        }
      } else {
        stalls[g] = 0;
      }
      prev[g] = std::min(prev[g], beta[g]);
    }
  }
  if (t_ms) t_ms[0] += now_ms() - t0;
}

void newton_solve(jfnk_mesh* m, const std::vector<int>& n_inc, const jfnk_newton_opts& o, double* u,
                  FvWork& fw, KrylovWork& kw, hipStream_t s, std::vector<jfnk_stats>& stats,
                  std::vector<jfnk_status>& status) {
  const int S = m->n_seg();
  const int64_t n = int64_t(m->dev.n_cells) * m->dev.dim;
  const SegLayout L = layout_of(m);
  const double t0 = now_ms();
  stats.assign(S, jfnk_stats{});
  status.assign(S, JFNK_OK);
  jfnk_gmres_opts go = o.gmres;
  go.rtol = o.eta;
  go.atol = 0.0;
  std::vector<int> inc(S, 1), it_inc(S, 0);
  std::vector<char> done(S, 0), fresh(S, 1), part(S, 0);
  std::vector<double> load(S), r0(S, 0.0), rn(S), v2;
  for (int g = 0; g < S; ++g) load[g] = 1.0 / n_inc[g];
  std::vector<GmresSeg> gres;
  double t_ms[8] = {0};
  while (true) {
    upload_doubles(m, load, fw.load, s);
    std::vector<char> live(S);
    for (int g = 0; g < S; ++g) live[g] = !done[g];
    upload_flags(m, live, kw.act, s);
    const double tr = now_ms();
    residual_into(m, u, kw.R, fw, kw.act, s);
    seg_norms2(m, L, kw.R, fw, kw, kw.act, s, v2);
    t_ms[4] += now_ms() - tr;
    bool need_step = false, pending = false;
    for (int g = 0; g < S; ++g) {
      part[g] = 0;
      if (done[g]) continue;
      rn[g] = std::sqrt(v2[g]);
      if (fresh[g]) {
        r0[g] = rn[g];
        fresh[g] = 0;
        it_inc[g] = 0;
        stats[g].res0 = r0[g];
      }
      stats[g].res_final = rn[g];
      if (!std::isfinite(rn[g])) {
        status[g] = JFNK_E_NAN;
        done[g] = 1;
        continue;
      }
      if (rn[g] <= std::max(o.rtol * r0[g], o.atol)) {
        if (inc[g] >= n_inc[g]) {
          done[g] = 1;
        } else {
          ++inc[g];
          load[g] = double(inc[g]) / n_inc[g];
          fresh[g] = 1;
          pending = true;
        }
        continue;
      }
      if (it_inc[g] >= o.max_newton_it) {
        status[g] = JFNK_E_NOT_CONVERGED;
        done[g] = 1;
        continue;
      }
      if (rn[g] > 1e8 * std::max(r0[g], 1e-300)) {
        status[g] = JFNK_E_DIVERGED;
        done[g] = 1;
        continue;
      }
      part[g] = 1;
      need_step = true;
    }
    if (!need_step) {
      if (pending) continue;
      break;
    }
    // J du = -R on the segments that need a step (du = 0 elsewhere)
    blas_lincomb(-1.0, kw.R, 0.0, kw.R, kw.b, n, s);
    JFNK_HIP(hipMemsetAsync(kw.du, 0, sizeof(double) * n, s));
    gmres_solve(m, u, kw.R, kw.b, kw.du, true, go, fw, kw, s, part, gres, t_ms);
    for (int g = 0; g < S; ++g) {
      if (!part[g]) continue;
      stats[g].gmres_it += gres[g].iterations;
      stats[g].restarts += gres[g].restarts;
      stats[g].jv_evals += gres[g].jv;
      stats[g].newton_it++;
      it_inc[g]++;
      if (gres[g].status == JFNK_E_NAN) {
        status[g] = JFNK_E_NAN;
        done[g] = 1;
      }
    }
    blas_axpby(1.0, kw.du, 1.0, u, n, s);
  }
  t_ms[0] = now_ms() - t0;
  for (int g = 0; g < S; ++g)
    for (int k = 0; k < 8; ++k) stats[g].t_ms[k] = t_ms[k];
}

}  // namespace jfnk
