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
// Newton (Eq. NewtonRaphson) with equal load increments k/N per segment (N
// may differ between segments); convergence per increment when
// |R(u)| <= max(rtol |R(u_0)|, atol) (Section 3.3, Euclidean norm, stol = 0);
// linear solves to the relative tolerance eta.  The step length s is 1, or
// with the line search of Section 3.2 the first of 1, 1/2, 1/4, ... that
// decreases |R| (per segment).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <shared_mutex>
#include <vector>

#include "gmres_dev.h"
#include "solver.h"

namespace jfnk {

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

__global__ void k_fill(double* d, int64_t n, double v) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = v;
}

}  // namespace

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

void fill_device(double* d, int64_t n, double value, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill, dim3(unsigned(std::max<int64_t>(blocks, 1))), dim3(256), 0, s, d, n, value);
  JFNK_HIP(hipGetLastError());
}

void residual_into(jfnk_mesh* m, const double* u, double* R, FvWork& fw, const int32_t* active,
                   hipStream_t s) {
  Profiler& p = m->prof;
  SegScalars sc{nullptr, fw.load_ptr(), active, fw.load1};
  if (m->dev.lds_kernels == 2) {
    const int t = p.on ? p.begin(2, s) : -1;
    launch_fused(m->dev, u, nullptr, sc, nullptr, R, s);
    if (t >= 0) p.end(t, s);
    if (m->src.active()) launch_source(m, sc, u, R, R, true, s);
    return;
  }
  int t = p.on ? p.begin(1, s) : -1;
  launch_gradient(m->dev, u, nullptr, sc, fw.grad, s);
  if (t >= 0) p.end(t, s);
  t = p.on ? p.begin(2, s) : -1;
  launch_flux(m->dev, fw.grad, sc, nullptr, R, s);
  if (t >= 0) p.end(t, s);
  if (m->src.active()) launch_source(m, sc, u, R, R, true, s);
}

void jv_into(jfnk_mesh* m, const double* u, const double* Ru, const double* v, double eps, double* Jv,
             FvWork& fw, const int32_t* active, hipStream_t s, const double* uu, bool ru_surface,
             const CentralFd* cfd) {
  Profiler& p = m->prof;
  if (cfd != nullptr) {
    jv_central(m, u, v, eps, Jv, fw, active, s, uu, *cfd);
    return;
  }
  if (m->src.active() && !ru_surface) {
    // the finite difference runs on the surface terms only: the volume
    // terms are affine in u, their derivative is added exactly below
    launch_source(m, SegScalars{nullptr, fw.load_ptr(), active, fw.load1}, u, Ru, fw.ru_src, false, s);
    Ru = fw.ru_src;
  }
  int t = p.on ? p.begin(0, s) : -1;
  if (eps > 0)
    fill_device(fw.eps, m->n_seg(), eps, s);
  else
    launch_eps_fused(layout_of(m), m->any_large, u, uu, 1, v, active, fw.partials, fw.eps_tickets(), fw.eps, s);
  if (t >= 0) p.end(t, s);
  SegScalars sc{fw.eps, fw.load_ptr(), active, fw.load1};
  if (m->dev.lds_kernels == 2) {
    t = p.on ? p.begin(2, s) : -1;
    launch_fused(m->dev, u, v, sc, Ru, Jv, s);
    if (t >= 0) p.end(t, s);
  } else {
    t = p.on ? p.begin(1, s) : -1;
    launch_gradient(m->dev, u, v, sc, fw.grad, s);
    if (t >= 0) p.end(t, s);
    t = p.on ? p.begin(2, s) : -1;
    launch_flux(m->dev, fw.grad, sc, Ru, Jv, s);
    if (t >= 0) p.end(t, s);
  }
  if (m->src.dt > 0) launch_inertia_jv(m, sc, v, Jv, s);
}

// (R(u + eps v) - R(u - eps v)) / (2 eps) with the cube-root step: the
// forward-difference step times eps_mach^(-1/6), or eps as given.
void jv_central(jfnk_mesh* m, const double* u, const double* v, double eps, double* Jv, FvWork& fw,
                const int32_t* active, hipStream_t s, const double* uu, const CentralFd& cfd) {
  Profiler& p = m->prof;
  const int S = m->n_seg();
  int t = p.on ? p.begin(0, s) : -1;
  if (eps > 0) {
    fill_device(fw.eps, S, eps, s);
    blas_central_eps(fw.eps, cfd.eps_neg, S, 1.0, s);
  } else {
    launch_eps_fused(layout_of(m), m->any_large, u, uu, 1, v, active, fw.partials, fw.eps_tickets(), fw.eps, s);
    blas_central_eps(fw.eps, cfd.eps_neg, S, kCentralStepFactor, s);
  }
  if (t >= 0) p.end(t, s);
  // surface terms at u - eps v, then at u + eps v against them
  const SegScalars scm{cfd.eps_neg, fw.load_ptr(), active, fw.load1};
  const SegScalars scp{fw.eps, fw.load_ptr(), active, fw.load1};
  if (m->dev.lds_kernels == 2) {
    t = p.on ? p.begin(2, s) : -1;
    launch_fused(m->dev, u, v, scm, nullptr, cfd.rm, s);
    launch_fused(m->dev, u, v, scp, cfd.rm, Jv, s);
    if (t >= 0) p.end(t, s);
  } else {
    t = p.on ? p.begin(1, s) : -1;
    launch_gradient(m->dev, u, v, scm, fw.grad, s);
    if (t >= 0) p.end(t, s);
    t = p.on ? p.begin(2, s) : -1;
    launch_flux(m->dev, fw.grad, scm, nullptr, cfd.rm, s);
    if (t >= 0) p.end(t, s);
    t = p.on ? p.begin(1, s) : -1;
    launch_gradient(m->dev, u, v, scp, fw.grad, s);
    if (t >= 0) p.end(t, s);
    t = p.on ? p.begin(2, s) : -1;
    launch_flux(m->dev, fw.grad, scp, cfd.rm, Jv, s);
    if (t >= 0) p.end(t, s);
  }
  blas_lincomb(0.5, Jv, 0.0, Jv, Jv, int64_t(m->dev.n_cells) * m->dev.dim, s);
  if (m->src.dt > 0) launch_inertia_jv(m, scp, v, Jv, s);
}

void StepGraphs::clear() {
  for (hipGraphExec_t& e : exec)
    if (e) (void)hipGraphExecDestroy(e);
  exec.clear();
  work = nullptr;
}

namespace {

// Arnoldi steps j0 <= j < j1 for every active segment: z_j = P^{-1} v_j,
// w = J z_j (right preconditioning; with augmentation the last n_aug
// directions z_j are the stored corrections instead), or w = P^{-1} J v_j
// (left), then two classical Gram-Schmidt passes, |w|, the device-side
// Givens update, and v_{j+1} = w / h_{j+1,j}.  No host interaction:
// capturable.
void enqueue_steps(jfnk_mesh* m, const SegLayout& L, const double* u, const double* Ru, bool ru_surface,
                   const jfnk_gmres_opts& o, FvWork& fw, KrylovWork& kw, int j0, int j1, hipStream_t s,
                   int n_aug = 0) {
  const int64_t n = int64_t(m->dev.n_cells) * m->dev.dim;
  const CentralFd cfd{kw.rm, kw.eps_neg};
  const CentralFd* c = o.fd_central ? &cfd : nullptr;
  for (int j = j0; j < j1; ++j) {
    double* Vj = kw.V + size_t(j) * n;
    if (kw.z32) {
      // FP32 basis (right preconditioning, no augmentation): z_j is formed in
      // zd, rounded to FP32 into its slot, and J v takes the rounded value,
      // the same number the solution update reads back.  The AMG32 V-cycle
      // writes FP32 values already, so zd needs no rewrite then.
      precond_apply(m, o.precond, o.cheb_degree, Vj, kw.zd, kw, s);
      Profiler& p = m->prof;
      const int t = p.on ? p.begin(3, s) : -1;
      blas_round_fp32(kw.zd, kw.Zf + size_t(j) * n, n, pc_kind(o.precond) != JFNK_PC_AMG32, s, kw.gd.nact);
      if (t >= 0) p.end(t, s);
      jv_into(m, u, Ru, kw.zd, o.eps, kw.w, fw, kw.act, s, kw.uu, ru_surface, c);
    } else if (o.left) {
      double* Zj = kw.Z + size_t(j) * n;
      jv_into(m, u, Ru, Vj, o.eps, Zj, fw, kw.act, s, kw.uu, ru_surface, c);
      precond_apply(m, o.precond, o.cheb_degree, Zj, kw.w, kw, s);
    } else {
      double* Zj = kw.Z + size_t(j) * n;
      // augmentation directions occupy slots restart - augment .. of Z
      const int a = j - (o.restart - o.augment);
      if (a < 0 || a >= n_aug) precond_apply(m, o.precond, o.cheb_degree, Vj, Zj, kw, s);
      jv_into(m, u, Ru, Zj, o.eps, kw.w, fw, kw.act, s, kw.uu, ru_surface, c);
    }
    Profiler& p = m->prof;
    const int t = p.on ? p.begin(4, s) : -1;
    if (o.orth) {
      // V_{j+1} is kept at the end of a cycle too: the closing pass
      // reorthogonalises it to complete the cycle's last column
      dcgs_step(L, m->any_large, kw.V, n, j, kw.w, kw.h, kw.h2, kw.nrm, fw.partials, kw.partials2,
                fw.cgs_tickets(), kw.gd, o.max_it, false, s);
      blas_scale_seg(L, kw.w, kw.fac, kw.V + size_t(j + 1) * n, kw.act, s);
    } else {
      cgs2_step(L, m->any_large, kw.V, n, j + 1, kw.w, kw.h, kw.h2, kw.nrm, fw.partials, fw.cgs_tickets(),
                fw.step_counters(), kw.gd, j, o.max_it, s);
      if (j + 1 < o.restart) blas_scale_seg(L, kw.w, kw.fac, kw.V + size_t(j + 1) * n, kw.act, s);
    }
    if (t >= 0) p.end(t, s);
  }
}

hipEvent_t mesh_event(jfnk_mesh* m, int i) {
  if (!m->ev[i]) JFNK_HIP(hipEventCreateWithFlags(&m->ev[i], hipEventDisableTiming));
  return m->ev[i];
}

}  // namespace

void gmres_solve(jfnk_mesh* m, const double* u, const double* Ru, const double* b, double* x,
                 bool x_is_zero, const jfnk_gmres_opts& o_in, FvWork& fw, KrylovWork& kw, hipStream_t s,
                 const std::vector<char>& part_in, std::vector<GmresSeg>& out, double* t_ms) {
  // orth = 2: the handle's choice where DCGS2 applies
  jfnk_gmres_opts o = o_in;
  if (o.orth == 2) o.orth = (!o.left && o.restart <= kMaxDcgsRestart) ? m->tune.orth : 0;
  const int S = m->n_seg();
  const int64_t n = int64_t(m->dev.n_cells) * m->dev.dim;
  const int mr = o.restart;
  const SegLayout L = layout_of(m);
  const double t0 = now_ms();
  std::vector<char> part = part_in.empty() ? std::vector<char>(S, 1) : part_in;
  const CentralFd cfd{kw.rm, kw.eps_neg};
  JFNK_REQUIRE(kw.z32 == pc_z32(o.precond), JFNK_E_ARG, "gmres: workspace carved for another Z basis");
  JFNK_REQUIRE(!kw.z32 || (!o.left && o.augment == 0), JFNK_E_ARG,
               "gmres: the FP32 Z basis needs right preconditioning without augmentation");
  out.assign(S, GmresSeg());
  upload_flags(m, part, kw.act, s);
  // with volume terms the J v of every step differences the surface terms
  // only: their part of R(u) is formed once here
  const bool ru_surface = m->src.active();
  if (ru_surface) {
    launch_source(m, SegScalars{nullptr, fw.load_ptr(), kw.act, fw.load1}, u, Ru, fw.ru_src, false, s);
    Ru = fw.ru_src;
  }
  // |u|^2 per segment, once: u is fixed over the solve, so the automatic J v
  // step of every Arnoldi step needs only |v|
  if (o.eps <= 0) blas_mdot(L, u, 0, 1, u, fw.partials, kw.uu, 1, false, kw.act, s);
  std::vector<double> v2;
  // left preconditioning measures every residual after P^{-1}: the target
  // is rtol |P^{-1} b| (P^{-1} b formed in the first Z slot, free here)
  if (o.left) {
    precond_apply(m, o.precond, o.cheb_degree, b, kw.Z, kw, s, false);
    seg_norms2(m, L, kw.Z, fw, kw, kw.act, s, v2);
  } else {
    seg_norms2(m, L, b, fw, kw, kw.act, s, v2);
  }
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
  // r = b - J x, or P^{-1}(b - J x) with left preconditioning
  if (x_is_zero) {
    blas_lincomb(1.0, o.left ? kw.Z : b, 0.0, b, kw.r, n, s);
  } else {
    jv_into(m, u, Ru, x, o.eps, kw.w, fw, kw.act, s, kw.uu, ru_surface, o.fd_central ? &cfd : nullptr);
    for (int g = 0; g < S; ++g) out[g].jv += part[g];
    blas_lincomb(1.0, b, -1.0, kw.w, kw.r, n, s);
    if (o.left) {
      precond_apply(m, o.precond, o.cheb_degree, kw.r, kw.w, kw, s, false);
      blas_lincomb(1.0, kw.w, 0.0, kw.w, kw.r, n, s);
    }
  }
  seg_norms2(m, L, kw.r, fw, kw, kw.act, s, v2);
  for (int g = 0; g < S; ++g) {
    beta[g] = std::sqrt(v2[g]);
    prev[g] = beta[g];
    out[g].res_true = beta[g];
  }
  GmresDev& G = kw.gd;
  gmres_zero_counters(G, S, s);
  const int K = std::min(mr, o.step_chunk > 0 ? o.step_chunk : std::max(1, m->tune.step_chunk));
  const int n_chunks = (mr + K - 1) / K;
  // Graphs need a capturable stream and unchanged launch arguments.
  const int graphs = o.graphs == 2 ? m->tune.graphs : o.graphs;
  // augmentation changes the steps from cycle to cycle: direct launches
  const bool use_graphs = graphs != 0 && s != nullptr && !m->prof.on && o.augment == 0;
  if (use_graphs) {
    StepGraphs& sg = m->graphs;
    const void* work = static_cast<const void*>(kw.V);
    if (sg.work != work || sg.u != u || sg.Ru != Ru || sg.restart != mr || sg.precond != o.precond ||
        sg.cheb != o.cheb_degree || sg.chunk != K || sg.eps != o.eps || sg.max_it != o.max_it ||
        sg.left != o.left || sg.central != o.fd_central || sg.orth != o.orth) {
      sg.clear();
      sg.work = work;
      sg.u = u;
      sg.Ru = Ru;
      sg.restart = mr;
      sg.precond = o.precond;
      sg.cheb = o.cheb_degree;
      sg.chunk = K;
      sg.eps = o.eps;
      sg.max_it = o.max_it;
      sg.left = o.left;
      sg.central = o.fd_central;
      sg.orth = o.orth;
      sg.exec.assign(n_chunks, nullptr);
    }
  }
  // pinned host layout: [0, S) norms, then int32 its/kk/flag, then chunk flags
  double* pin = m->pinned;
  int32_t* pin_i = reinterpret_cast<int32_t*>(pin + S);
  int32_t* pin_nact = pin_i + 3 * S + 8;
  double* stage = m->pinned + m->pinned_doubles / 2;
  std::vector<int> its(S, 0);
  std::vector<char> act(S);
  int n_aug = 0;   // augmentation directions available (LGMRES)
  std::vector<double> dfac(S);
  while (true) {
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
      } else if (its[g] >= o.max_it) {
        out[g].status = JFNK_E_NOT_CONVERGED;
        done[g] = 1;
      } else {
        act[g] = 1;
        any = true;
      }
    }
    if (!any) break;
    // cycle start: flags, beta and targets in one upload (the staging area is
    // rewritten only after the synchronisation at the end of the cycle)
    for (int g = 0; g < S; ++g) {
      stage[g] = act[g] ? 1.0 : 0.0;
      stage[S + g] = beta[g];
      stage[2 * S + g] = target[g];
    }
    JFNK_HIP(hipMemcpyAsync(kw.stage, stage, sizeof(double) * 3 * S, hipMemcpyHostToDevice, s));
    gmres_cycle_init(G, S, kw.stage, s);
    blas_scale_seg(L, kw.r, kw.fac, kw.V, kw.act, s);
    const double ts = now_ms();
    // runs of K steps; while run c executes, the host waits for run c-1's
    // count of active segments and stops enqueueing when it is zero
    for (int c = 0; c < n_chunks; ++c) {
      const int j0 = c * K, j1 = std::min(mr, j0 + K);
      if (use_graphs) {
        hipGraphExec_t& ex = m->graphs.exec[c];
        if (!ex) {
          std::unique_lock<std::shared_mutex> lk(capture_mutex());
          hipGraph_t gr = nullptr;
          JFNK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
          try {
            enqueue_steps(m, L, u, Ru, ru_surface, o, fw, kw, j0, j1, s, n_aug);
          } catch (...) {
            (void)hipStreamEndCapture(s, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            throw;
          }
          JFNK_HIP(hipStreamEndCapture(s, &gr));
          const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          JFNK_HIP(e);
        }
        JFNK_HIP(hipGraphLaunch(ex, s));
      } else {
        enqueue_steps(m, L, u, Ru, ru_surface, o, fw, kw, j0, j1, s, n_aug);
      }
      JFNK_HIP(hipMemcpyAsync(pin_nact + (c & 63), G.nact, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipEventRecord(mesh_event(m, c & 1), s));
      if (c > 0) {
        JFNK_HIP(hipEventSynchronize(mesh_event(m, (c - 1) & 1)));
        if (pin_nact[(c - 1) & 63] == 0) break;
      }
    }
    // delayed reorthogonalisation: the segments still taking steps after the
    // cycle's last step complete its column with a closing pass
    if (o.orth) {
      Profiler& p = m->prof;
      const int t = p.on ? p.begin(4, s) : -1;
      dcgs_step(L, m->any_large, kw.V, n, mr, kw.w, kw.h, kw.h2, kw.nrm, fw.partials, kw.partials2,
                fw.cgs_tickets(), kw.gd, o.max_it, true, s);
      if (t >= 0) p.end(t, s);
    }
    const double te = now_ms();
    // x += Z y on the segments that ran, then the true residual
    {
      Profiler& p = m->prof;
      const int t = p.on ? p.begin(5, s) : -1;
      gmres_lsq(G, S, kw.y, s);
      if (o.left) {
        blas_combine(L, kw.V, n, mr, kw.y, kMaxBasis, 1.0, x, G.ran, s, G.kk);
      } else if (o.augment > 0) {
        // the cycle's correction delta = Z y goes to x and, normalised, to the
        // first augmentation slot; older corrections move one slot on
        fill_device(kw.r, n, 0.0, s);
        blas_combine(L, kw.Z, n, mr, kw.y, kMaxBasis, 1.0, kw.r, G.ran, s, G.kk);
        blas_axpby(1.0, kw.r, 1.0, x, n, s);
        const int a0 = mr - o.augment;
        for (int i = std::min(n_aug, o.augment - 1); i > 0; --i)
          blas_lincomb(1.0, kw.Z + size_t(a0 + i - 1) * n, 0.0, kw.Z, kw.Z + size_t(a0 + i) * n, n, s);
        std::vector<double> d2;
        seg_norms2(m, L, kw.r, fw, kw, G.ran, s, d2);
        for (int g = 0; g < S; ++g) dfac[g] = d2[g] > 0 ? 1.0 / std::sqrt(d2[g]) : 0.0;
        upload_doubles(m, dfac, kw.stage, s);
        blas_scale_seg(L, kw.r, kw.stage, kw.Z + size_t(a0) * n, G.ran, s);
        n_aug = std::min(n_aug + 1, o.augment);
      } else if (kw.z32) {
        blas_combine(L, kw.Zf, n, mr, kw.y, kMaxBasis, 1.0, x, G.ran, s, G.kk);
      } else {
        blas_combine(L, kw.Z, n, mr, kw.y, kMaxBasis, 1.0, x, G.ran, s, G.kk);
      }
      if (t >= 0) p.end(t, s);
    }
    jv_into(m, u, Ru, x, o.eps, kw.w, fw, G.ran, s, kw.uu, ru_surface, o.fd_central ? &cfd : nullptr);
    {
      Profiler& p = m->prof;
      const int t = p.on ? p.begin(5, s) : -1;
      blas_lincomb(1.0, b, -1.0, kw.w, kw.r, n, s);
      if (o.left) {
        precond_apply(m, o.precond, o.cheb_degree, kw.r, kw.w, kw, s, false);
        blas_lincomb(1.0, kw.w, 0.0, kw.w, kw.r, n, s);
      }
      blas_mdot(L, kw.r, 0, 1, kw.r, fw.partials, kw.nrm, 4, false, G.ran, s);
      if (t >= 0) p.end(t, s);
    }
    JFNK_HIP(hipMemcpy2DAsync(pin, sizeof(double), kw.nrm, 4 * sizeof(double), sizeof(double), S,
                              hipMemcpyDeviceToHost, s));
    JFNK_HIP(hipMemcpyAsync(pin_i, G.its, sizeof(int32_t) * S, hipMemcpyDeviceToHost, s));
    JFNK_HIP(hipMemcpyAsync(pin_i + S, G.kk, sizeof(int32_t) * S, hipMemcpyDeviceToHost, s));
    JFNK_HIP(hipMemcpyAsync(pin_i + 2 * S, G.flag, sizeof(int32_t) * S, hipMemcpyDeviceToHost, s));
    JFNK_HIP(hipStreamSynchronize(s));
    if (t_ms) {
      t_ms[2] += te - ts;
      t_ms[6] += now_ms() - te;
    }
    for (int g = 0; g < S; ++g) {
      if (!act[g]) continue;
      const int steps = pin_i[g] - its[g];
      its[g] = pin_i[g];
      out[g].iterations = its[g];
      out[g].jv += steps;
      if (pin_i[2 * S + g]) {
        out[g].status = JFNK_E_NAN;
        done[g] = 1;
        continue;
      }
      if (pin_i[S + g] > 0) out[g].restarts++;
      out[g].jv++;
      beta[g] = std::sqrt(pin[g]);
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
  std::vector<int> inc(S, 1), it_inc(S, 0), last(S);
  std::vector<char> done(S, 0), fresh(S, 1), part(S, 0);
  std::vector<double> load(S), r0(S, 0.0), rn(S), v2;
  for (int g = 0; g < S; ++g) {
    inc[g] = std::min(std::max(o.inc_begin, 1), n_inc[g]);
    last[g] = o.inc_end > 0 ? std::min(std::max(o.inc_end, inc[g]), n_inc[g]) : n_inc[g];
    load[g] = double(inc[g]) / n_inc[g];
  }
  std::vector<GmresSeg> gres;
  double t_ms[8] = {0};
  const double dtol = o.dtol > 0 ? o.dtol : 1e8;
  std::vector<double> step(S, 1.0);
  std::vector<char> trial(S, 0), small_step(S, 0);
  std::vector<double> du2, u2;
  // step test of Section 3.3: |s du| <= stol |u| after the update ends the
  // increment (checked at the next residual evaluation)
  auto check_step = [&](const std::vector<char>& took) {
    if (o.stol <= 0) return;
    upload_flags(m, took, kw.act, s);
    seg_norms2(m, L, kw.du, fw, kw, kw.act, s, du2);
    seg_norms2(m, L, u, fw, kw, kw.act, s, u2);
    for (int g = 0; g < S; ++g)
      if (took[g] && !done[g] && step[g] * std::sqrt(du2[g]) <= o.stol * std::sqrt(u2[g])) small_step[g] = 1;
  };
  const int max_bt = o.max_backtrack > 0 ? o.max_backtrack : 8;
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
      if (rn[g] <= std::max(o.rtol * r0[g], o.atol) || small_step[g]) {
        small_step[g] = 0;
        if (inc[g] >= last[g]) {
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
      if (rn[g] > dtol * std::max(r0[g], 1e-300)) {
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
    // central differences once some segment is within central_below of its target
    go.fd_central = o.gmres.fd_central;
    if (o.central_below > 0)
      for (int g = 0; g < S; ++g)
        if (part[g] && rn[g] <= o.central_below * r0[g]) go.fd_central = 1;
    // J du = -R on the segments that need a step (du = 0 elsewhere)
    blas_lincomb(-1.0, kw.R, 0.0, kw.R, kw.b, n, s);
    fill_device(kw.du, n, 0.0, s);
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
    for (int g = 0; g < S; ++g) step[g] = 1.0;
    if (!o.line_search) {
      blas_axpby(1.0, kw.du, 1.0, u, n, s);
      check_step(part);
      continue;
    }
    // Line search: u = u_old + s du per segment, u_old kept in kw.b (the
    // right-hand side is no longer needed); segments still searching have
    // their residual evaluated, the others keep their accepted step (their u
    // is recomputed with the same operands, so it does not change).
    blas_lincomb(1.0, u, 0.0, u, kw.b, n, s);
    for (int g = 0; g < S; ++g) {
      step[g] = 1.0;
      trial[g] = part[g] && !done[g];
    }
    const double tl = now_ms();
    for (int t = 0;; ++t) {
      upload_doubles(m, step, kw.fac, s);
      blas_scale_seg(L, kw.du, kw.fac, kw.w, nullptr, s);
      blas_lincomb(1.0, kw.b, 1.0, kw.w, u, n, s);
      bool any = false;
      for (int g = 0; g < S; ++g) any = any || trial[g];
      if (!any) break;
      upload_flags(m, trial, kw.act, s);
      residual_into(m, u, kw.R, fw, kw.act, s);
      seg_norms2(m, L, kw.R, fw, kw, kw.act, s, v2);
      for (int g = 0; g < S; ++g) {
        if (!trial[g]) continue;
        const double rt = std::sqrt(v2[g]);
        if (rt < rn[g] || t >= max_bt) {
          trial[g] = 0;   // accepted (a NaN never compares below)
        } else {
          step[g] *= 0.5;
        }
      }
      bool again = false;
      for (int g = 0; g < S; ++g) again = again || trial[g];
      if (!again) break;
    }
    t_ms[4] += now_ms() - tl;
    check_step(part);
  }
  t_ms[0] = now_ms() - t0;
  for (int g = 0; g < S; ++g)
    for (int k = 0; k < 8; ++k) stats[g].t_ms[k] = t_ms[k];
}

}  // namespace jfnk
