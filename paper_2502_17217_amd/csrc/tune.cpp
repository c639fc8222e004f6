// Launch-shape and schedule tuner for one mesh handle (a single mesh or a
// batch): every launch-shape and schedule candidate computes the same bits,
// so the choice is made on measured time only, on the handle's own mesh and
// state.
//
//   cell passes of J v: one fused pass per tile or LDS-staged gradient and
//     flux passes (when the mesh is tile-ordered), or direct gathers; one
//     workgroup per tile or a persistent grid of 2, 4 or 8 workgroups per
//     compute unit, each timed with HIP events over repeated J v products;
//   Arnoldi schedule: the number of steps enqueued between host checks and
//     whether runs are replayed from HIP graphs, each timed over the same
//     preconditioned GMRES solve of J x = -R(u);
//   orthogonalisation (for solves that leave it to the handle): Gram-Schmidt
//     twice or with delayed reorthogonalisation, timed on the same solve
//     under the chosen schedule.  The two differ in rounding, not in the
//     method; a solve that names one gets that one.
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

// Compute units of the current device (256 on MI355X), for the persistent
// grid sizes the tuner tries.
int compute_units() {
  int dev = 0, cu = 0;
  JFNK_HIP(hipGetDevice(&dev));
  JFNK_HIP(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
  return cu > 0 ? cu : 256;
}

}  // namespace

void autotune(jfnk_mesh* m, const jfnk_gmres_opts& o_in, const double* u, double load, void* work, hipStream_t s,
              jfnk_tune_report* rep) {
  const int S = m->n_seg();
  const int64_t n = int64_t(m->dev.n_cells) * m->dev.dim;
  jfnk_tune_report r{};
  Carver c(work);
  FvWork fw;
  fw.carve(c, m);
  fw.setup(s, load);
  KrylovWork kw;
  kw.carve(c, m, o_in.restart, precond_work_floats(m, o_in.precond), pc_z32(o_in.precond));
  precond_setup(m, o_in.precond, s);
  const bool prof = m->prof.on;
  m->prof.on = false;
  m->graphs.clear();
  // R(u) into kw.R; a fixed direction v = 1 in kw.r; J v into kw.w
  residual_into(m, u, kw.R, fw, nullptr, s);
  fill_device(kw.r, n, 1.0, s);
  hipEvent_t e0, e1;
  JFNK_HIP(hipEventCreate(&e0));
  JFNK_HIP(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  // ---- cell passes
  const int tiles = int((m->dev.n_cells + kFvBlock - 1) / kFvBlock);
  std::vector<int> lds_opts{0};
  if (m->dev.tiled) lds_opts = m->dev.fused ? std::vector<int>{2, 1, 0} : std::vector<int>{1, 0};
  std::vector<int> grid_opts{0};
  for (int k : {2, 4, 8})
    if (k * compute_units() < tiles) grid_opts.push_back(k * compute_units());
  const int reps = 10;
  double best = 1e300;
  int best_lds = m->dev.lds_kernels, best_grid = m->dev.persist;
  for (int lds : lds_opts)
    for (int grid : grid_opts) {
      m->dev.lds_kernels = lds;
      m->dev.persist = grid;
      for (int i = 0; i < 2; ++i) jv_into(m, u, kw.R, kw.r, o_in.eps, kw.w, fw, nullptr, s);
      JFNK_HIP(hipEventRecord(e0, s));
      for (int i = 0; i < reps; ++i) jv_into(m, u, kw.R, kw.r, o_in.eps, kw.w, fw, nullptr, s);
      JFNK_HIP(hipEventRecord(e1, s));
      JFNK_HIP(hipEventSynchronize(e1));
      float ms = 0;
      JFNK_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double per = double(ms) / reps;
      if (r.n_jv < 16) {
        r.jv_lds[r.n_jv] = lds;
        r.jv_persist[r.n_jv] = grid;
        r.jv_ms[r.n_jv] = per;
        r.n_jv++;
      }
      if (per < best) {
        best = per;
        best_lds = lds;
        best_grid = grid;
      }
    }
  m->dev.lds_kernels = best_lds;
  m->dev.persist = best_grid;
  r.lds_kernels = best_lds;
  r.persist = best_grid;
  // ---- Arnoldi schedule: the same solve J x = -R(u) under each candidate
  blas_lincomb(-1.0, kw.R, 0.0, kw.R, kw.b, n, s);
  const int chunks[] = {1, 1, 2, 4, 8};
  const int graphs[] = {0, 1, 1, 1, 1};
  best = 1e300;
  int best_chunk = m->tune.step_chunk, best_graphs = m->tune.graphs;
  for (int k = 0; k < 5; ++k) {
    if (chunks[k] > o_in.restart) continue;
    if (graphs[k] && s == nullptr) continue;
    jfnk_gmres_opts o = o_in;
    o.step_chunk = chunks[k];
    o.graphs = graphs[k];
    std::vector<GmresSeg> res;
    // a first, untimed run captures the graphs of this schedule
    for (int pass = 0; pass < 2; ++pass) {
      fill_device(kw.du, n, 0.0, s);
      JFNK_HIP(hipStreamSynchronize(s));
      const double t0 = now_ms();
      gmres_solve(m, u, kw.R, kw.b, kw.du, true, o, fw, kw, s, {}, res, nullptr);
      const double dt = now_ms() - t0;
      if (pass == 1) {
        if (r.n_solve < 8) {
          r.solve_chunk[r.n_solve] = chunks[k];
          r.solve_graphs[r.n_solve] = graphs[k];
          r.solve_ms[r.n_solve] = dt;
          r.n_solve++;
        }
        if (dt < best) {
          best = dt;
          best_chunk = chunks[k];
          best_graphs = graphs[k];
        }
      }
    }
  }
  m->tune.step_chunk = best_chunk;
  m->tune.graphs = best_graphs;
  r.step_chunk = best_chunk;
  r.graphs = best_graphs;
  // ---- orthogonalisation, under the chosen schedule (where DCGS2 applies)
  r.orth = m->tune.orth;
  if (!o_in.left && o_in.restart <= kMaxDcgsRestart) {
    double t_orth[2] = {0.0, 0.0};
    for (int orth = 0; orth < 2; ++orth) {
      jfnk_gmres_opts o = o_in;
      o.step_chunk = best_chunk;
      o.graphs = best_graphs;
      o.orth = orth;
      std::vector<GmresSeg> res;
      for (int pass = 0; pass < 2; ++pass) {
        fill_device(kw.du, n, 0.0, s);
        JFNK_HIP(hipStreamSynchronize(s));
        const double t0 = now_ms();
        gmres_solve(m, u, kw.R, kw.b, kw.du, true, o, fw, kw, s, {}, res, nullptr);
        if (pass == 1) t_orth[orth] = now_ms() - t0;
      }
      r.orth_ms[orth] = t_orth[orth];
    }
    m->tune.orth = t_orth[1] <= t_orth[0] ? 1 : 0;
    r.orth = m->tune.orth;
  }
  m->tune.tuned = 1;
  m->graphs.clear();
  m->prof.on = prof;
  if (rep) *rep = r;
}

}  // namespace jfnk
