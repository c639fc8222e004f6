// FP32 aggregation-AMG preconditioner (placeholder until the hierarchy is built).
#include "solver.h"

namespace jfnk {

struct AmgHierarchy {};

size_t amg_work_floats(const jfnk_mesh*) { return 0; }

void amg_setup(jfnk_mesh*, hipStream_t) {
  throw Error{JFNK_E_ARG, "AMG preconditioner is not available in this build"};
}

void amg_apply(jfnk_mesh*, int, const double*, double*, float*, hipStream_t) {
  throw Error{JFNK_E_ARG, "AMG preconditioner is not available in this build"};
}

void amg_destroy(AmgHierarchy* a) { delete a; }

}  // namespace jfnk
