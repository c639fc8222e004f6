// GMRES and Newton drivers on the host; all vector work runs in the HIP
// kernels of fv_kernels.hip / blas.hip / precond.hip.
//
// GMRES (Section 3.2): restarted, right preconditioned; the preconditioned
// directions z_j = P^{-1} v_j are kept (flexible form), so a variable
// preconditioner such as an FP32 V-cycle is allowed.  Arnoldi uses
// classical Gram-Schmidt applied twice (two multi-dot + update passes).
// Givens rotations and the small triangular solve run on the host from one
// device-to-host copy of the new Hessenberg column per Arnoldi step.
// Each restart cycle ends with the true residual b - J x.
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

// Copy `count` device doubles to the mesh's pinned scalars and wait.
void read_scalars(jfnk_mesh* m, const double* d, int count, hipStream_t s) {
  JFNK_HIP(hipMemcpyAsync(m->pinned, d, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  JFNK_HIP(hipStreamSynchronize(s));
}

double dev_norm(jfnk_mesh* m, const double* x, int64_t n, FvWork& fw, double* slot, hipStream_t s) {
  blas_mdot(x, 0, 1, x, n, fw.partials, slot, false, s);
  read_scalars(m, slot, 1, s);
  return std::sqrt(m->pinned[0]);
}

}  // namespace

void residual_into(jfnk_mesh* m, double load, const double* u, double* R, FvWork& fw, hipStream_t s) {
  Profiler& p = m->prof;
  int t = p.on ? p.begin(1, s) : -1;
  launch_gradient(m->dev, u, nullptr, nullptr, fw.grad, s);
  if (t >= 0) p.end(t, s);
  t = p.on ? p.begin(2, s) : -1;
  launch_flux(m->dev, fw.grad, nullptr, nullptr, R, load, s);
  if (t >= 0) p.end(t, s);
}

void jv_into(jfnk_mesh* m, double load, const double* u, const double* Ru, const double* v,
             double eps, double* Jv, FvWork& fw, hipStream_t s) {
  Profiler& p = m->prof;
  double* d_eps = fw.scalars;
  int t = p.on ? p.begin(0, s) : -1;
  if (eps > 0)
    launch_set_scalar(d_eps, eps, s);
  else
    launch_eps(u, v, int64_t(m->dev.n_cells) * m->dev.dim, fw.partials, d_eps, s);
  if (t >= 0) p.end(t, s);
  t = p.on ? p.begin(1, s) : -1;
  launch_gradient(m->dev, u, v, d_eps, fw.grad, s);
  if (t >= 0) p.end(t, s);
  t = p.on ? p.begin(2, s) : -1;
  launch_flux(m->dev, fw.grad, d_eps, Ru, Jv, load, s);
  if (t >= 0) p.end(t, s);
}

GmresResult gmres_solve(jfnk_mesh* m, double load, const double* u, const double* Ru, const double* b,
                        double* x, bool x_is_zero, const jfnk_gmres_opts& o, FvWork& fw,
                        KrylovWork& kw, hipStream_t s, double* t_ms) {
  const int64_t n = int64_t(m->dev.n_cells) * m->dev.dim;
  const int mr = o.restart;
  GmresResult res;
  double t0 = now_ms();
  double* hs = kw.h;  // device: [0..j] Hessenberg column, [kMaxBasis..] scalars
  res.bnorm = dev_norm(m, b, n, fw, hs + kMaxBasis, s);
  JFNK_REQUIRE(std::isfinite(res.bnorm), JFNK_E_NAN, "gmres: right-hand side is not finite");
  const double target = std::max(o.rtol * res.bnorm, o.atol);
  // r = b - J x
  if (x_is_zero) {
    JFNK_HIP(hipMemcpyAsync(kw.r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  } else {
    jv_into(m, load, u, Ru, x, o.eps, kw.w, fw, s);
    res.jv++;
    blas_lincomb(1.0, b, -1.0, kw.w, kw.r, n, s);
  }
  double beta = dev_norm(m, kw.r, n, fw, hs + kMaxBasis, s);
  res.res_true = beta;
  std::vector<double> H(size_t(mr + 1) * mr), cs(mr), sn(mr), g(mr + 1), y(mr);
  double prev_cycle_beta = beta;
  int stalls = 0;
  while (true) {
    if (!std::isfinite(beta)) {
      res.status = JFNK_E_NAN;
      break;
    }
    if (beta <= target || res.bnorm == 0.0) {
      res.status = JFNK_OK;
      break;
    }
    if (res.iterations >= o.max_it) {
      res.status = JFNK_E_NOT_CONVERGED;
      break;
    }
    // v_0 = r / beta
    blas_lincomb(1.0 / beta, kw.r, 0.0, kw.r, kw.V, n, s);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool nan = false;
    for (int j = 0; j < mr; ++j) {
      double* Vj = kw.V + size_t(j) * n;
      double* Zj = kw.Z + size_t(j) * n;
      double tp = now_ms();
      if (o.precond == JFNK_PC_NONE) {
        JFNK_HIP(hipMemcpyAsync(Zj, Vj, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      } else {
        precond_apply(m, o.precond, o.cheb_degree, Vj, Zj, kw, s);
      }
      double tj = now_ms();
      jv_into(m, load, u, Ru, Zj, o.eps, kw.w, fw, s);
      res.jv++;
      double tc = now_ms();
      // |w| before orthogonalisation (breakdown test), then CGS2
      blas_mdot(kw.w, 0, 1, kw.w, n, fw.partials, hs + kMaxBasis + 1, false, s);
      blas_mdot(kw.V, n, j + 1, kw.w, n, fw.partials, hs, false, s);
      blas_combine(kw.V, n, j + 1, hs, -1.0, kw.w, n, s);
      blas_mdot(kw.V, n, j + 1, kw.w, n, fw.partials, kw.y, false, s);
      blas_combine(kw.V, n, j + 1, kw.y, -1.0, kw.w, n, s);
      blas_mdot(kw.w, 0, 1, kw.w, n, fw.partials, hs + kMaxBasis, false, s);
      // gather h + h2 and the two norms on the host
      JFNK_HIP(hipMemcpyAsync(m->pinned, hs, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipMemcpyAsync(m->pinned + kMaxBasis, kw.y, sizeof(double) * (j + 1),
                              hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipMemcpyAsync(m->pinned + 2 * kMaxBasis, hs + kMaxBasis, sizeof(double) * 2,
                              hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipStreamSynchronize(s));
      if (t_ms) {
        t_ms[3] += tj - tp;
        t_ms[1] += tc - tj;
        t_ms[2] += now_ms() - tc;
      }
      const double* ph = m->pinned;
      const double hn = std::sqrt(ph[2 * kMaxBasis]);
      const double w0 = std::sqrt(ph[2 * kMaxBasis + 1]);
      double* Hj = &H[size_t(j) * (mr + 1)];
      for (int i = 0; i <= j; ++i) Hj[i] = ph[i] + ph[kMaxBasis + i];
      Hj[j + 1] = hn;
      if (!std::isfinite(hn) || !std::isfinite(w0)) {
        nan = true;
        break;
      }
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t;
      }
      const double rr = std::hypot(Hj[j], Hj[j + 1]);
      cs[j] = Hj[j] / rr;
      sn[j] = Hj[j + 1] / rr;
      Hj[j] = rr;
      Hj[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      res.iterations++;
      k = j + 1;
      if (hn <= 1e-14 * std::max(w0, 1e-300)) break;  // happy breakdown
      blas_lincomb(1.0 / hn, kw.w, 0.0, kw.w, kw.V + size_t(j + 1) * n, n, s);
      if (std::fabs(g[j + 1]) <= target || res.iterations >= o.max_it) break;
    }
    if (nan) {
      res.status = JFNK_E_NAN;
      break;
    }
    // y = H^{-1} g (upper triangular), x += Z y
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < k; ++l) t -= H[size_t(l) * (mr + 1) + i] * y[l];
      y[i] = t / H[size_t(i) * (mr + 1) + i];
    }
    for (int i = 0; i < k; ++i) m->pinned[i] = y[i];
    JFNK_HIP(hipMemcpyAsync(kw.y, m->pinned, sizeof(double) * k, hipMemcpyHostToDevice, s));
    blas_combine(kw.Z, n, k, kw.y, 1.0, x, n, s);
    res.restarts++;
    // true residual
    jv_into(m, load, u, Ru, x, o.eps, kw.w, fw, s);
    res.jv++;
    blas_lincomb(1.0, b, -1.0, kw.w, kw.r, n, s);
    beta = dev_norm(m, kw.r, n, fw, hs + kMaxBasis, s);
    res.res_true = beta;
    if (beta > 0.999 * prev_cycle_beta && beta > target) {
      if (++stalls >= 3) {
        res.status = JFNK_E_BREAKDOWN;
        break;
      }
    } else {
      stalls = 0;
    }
    prev_cycle_beta = std::min(prev_cycle_beta, beta);
  }
  if (t_ms) t_ms[0] += now_ms() - t0;
  return res;
}

}  // namespace jfnk
