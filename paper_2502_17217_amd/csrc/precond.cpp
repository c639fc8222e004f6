// Preconditioner dispatch (Section 3.2: the compact-stencil approximate
// Jacobian J_tilde of Section 3.1 as the preconditioning matrix P).
//   JACOBI : z = diag(J_tilde)^{-1} r in FP64 (block-Jacobi; the blocks are
//            scalar times identity).
//   AMG32  : aggregation-AMG V-cycle on the scalar J_tilde with Chebyshev
//            smoothing, stored and applied in FP32 (amg.cpp / amg_kernels.hip).
//   AMG64  : the same hierarchy and cycle in FP64.
#include "blas.h"
#include "solver.h"

namespace jfnk {

size_t amg_work_floats(const jfnk_mesh* m);
size_t amg_work_floats(int64_t n, int dim);
void amg_setup(jfnk_mesh* m, bool fp64, hipStream_t s);
void amg_apply(jfnk_mesh* m, bool fp64, int cheb_degree, const double* r, double* z, void* work,
               hipStream_t s, const int32_t* gate);

size_t precond_work_floats(int64_t n_cells, int dim, int precond) {
  precond = pc_kind(precond);
  if (precond == JFNK_PC_AMG32) return amg_work_floats(n_cells, dim);
  if (precond == JFNK_PC_AMG64) return 2 * amg_work_floats(n_cells, dim);
  return 0;
}

size_t precond_work_floats(const jfnk_mesh* m, int precond) {
  return precond_work_floats(m->host.n_cells, m->host.dim, precond);
}

void precond_setup(jfnk_mesh* m, int precond, hipStream_t s) {
  if (amg_precond(precond)) amg_setup(m, pc_kind(precond) == JFNK_PC_AMG64, s);
}

// The kernels return at once when gate (the count of segments still taking
// Arnoldi steps) is zero, so that steps enqueued past convergence cost only
// their launches.
void precond_apply(jfnk_mesh* m, int precond, int cheb_degree, const double* r, double* z,
                   KrylovWork& kw, hipStream_t s, bool gated) {
  const int64_t n = int64_t(m->dev.n_cells) * m->dev.dim;
  const int32_t* gate = gated ? kw.gd.nact : nullptr;
  precond = pc_kind(precond);
  if (precond == JFNK_PC_JACOBI) {
    blas_jacobi(m->b_pc_dinv.as<double>(), r, z, m->dev.n_cells, m->dev.dim, m->dev.has_symm != 0, s, gate);
  } else if (amg_precond(precond)) {
    amg_apply(m, precond == JFNK_PC_AMG64, cheb_degree, r, z, kw.pc, s, gate);
  } else {
    blas_lincomb(1.0, r, 0.0, r, z, n, s);   // a kernel copy (capturable in a graph)
  }
}

}  // namespace jfnk
