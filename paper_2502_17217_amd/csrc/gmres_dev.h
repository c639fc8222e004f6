// Device-resident GMRES bookkeeping (gmres_kernels.hip): per-segment
// Hessenberg columns, Givens rotations, rotated right-hand side and step
// counters, so that Arnoldi steps need no host round trip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "blas.h"
#include "internal.h"

namespace jfnk {

struct GmresDev {
  int mr = 0;                // restart length
  double* H = nullptr;       // [S][mr][mr+1] rotated Hessenberg columns (R factor)
  double* cs = nullptr;      // [S][mr]
  double* sn = nullptr;      // [S][mr]
  double* g = nullptr;       // [S][mr+1] rotated beta e_1
  double* target = nullptr;  // [S] residual target of the segment
  double* fac = nullptr;     // [S] scale of the next basis vector (1/h_{j+1,j}, 0 when stopped)
  int32_t* act = nullptr;    // [S] 1 while the segment takes Arnoldi steps (read by every kernel)
  int32_t* ran = nullptr;    // [S] 1 if the segment started the current cycle (0 after NaN)
  int32_t* kk = nullptr;     // [S] steps taken in the current cycle
  int32_t* its = nullptr;    // [S] steps taken in this solve
  int32_t* flag = nullptr;   // [S] 1: NaN/Inf met
  int32_t* nact = nullptr;   // [1] segments still active after the last step
};

void gmres_zero_counters(const GmresDev& G, int S, hipStream_t s);
// stage (device): [S] active flags, [S] beta, [S] target
void gmres_cycle_init(const GmresDev& G, int S, const double* stage, hipStream_t s);
void gmres_step_finish(const GmresDev& G, int S, int j, int max_it, const double* h, const double* h2,
                       const double* nrm, hipStream_t s);
void gmres_lsq(const GmresDev& G, int S, double* y, hipStream_t s);

}  // namespace jfnk
