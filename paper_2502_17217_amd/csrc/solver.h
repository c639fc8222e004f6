// Host-side drivers: residual / J.v sequences, GMRES and Newton.
#pragma once

#include "internal.h"
#include "workspace.h"

namespace jfnk {

// R(u) into R (gradient pass + flux pass).
void residual_into(jfnk_mesh* m, double load, const double* u, double* R, FvWork& fw, hipStream_t s);

// J v into Jv using cached Ru; eps <= 0 selects the automatic step (device).
// Leaves the step used in fw.scalars[0].
void jv_into(jfnk_mesh* m, double load, const double* u, const double* Ru, const double* v,
             double eps, double* Jv, FvWork& fw, hipStream_t s);

struct GmresResult {
  jfnk_status status = JFNK_OK;
  int iterations = 0;
  int restarts = 0;
  int jv = 0;
  double bnorm = 0, res_true = 0;
};

// Right-preconditioned restarted (flexible) GMRES with CGS2 for J x = b.
// x_is_zero skips the initial J x product.
GmresResult gmres_solve(jfnk_mesh* m, double load, const double* u, const double* Ru, const double* b,
                        double* x, bool x_is_zero, const jfnk_gmres_opts& o, FvWork& fw,
                        KrylovWork& kw, hipStream_t s, double* t_ms);

size_t precond_work_floats(const jfnk_mesh* m, int precond);
void precond_setup(jfnk_mesh* m, int precond, hipStream_t s);
void precond_apply(jfnk_mesh* m, int precond, int cheb_degree, const double* r, double* z,
                   KrylovWork& kw, hipStream_t s);
void amg_destroy(AmgHierarchy* a);

}  // namespace jfnk
