// Device-side Givens update of one segment's Hessenberg column (included
// by HIP sources only; see gmres_kernels.hip for the method).
#pragma once

#include "gmres_dev.h"

namespace jfnk {

// Column j of segment s (rows 0..j+1 already in G.H): the rotations of
// columns 0..j-1 applied to it, its own rotation formed, g and the step
// counts updated.  Returns 1 if the residual estimate is still above the
// target and the step limit not reached.
__device__ inline int givens_apply(const GmresDev& G, int s, int j, int max_it) {
  const int mr = G.mr;
  double* Hj = G.H + (size_t(s) * mr + j) * (mr + 1);
  double* c = G.cs + size_t(s) * mr;
  double* sn = G.sn + size_t(s) * mr;
  double* g = G.g + size_t(s) * (mr + 1);
  for (int i = 0; i < j; ++i) {
    const double t = c[i] * Hj[i] + sn[i] * Hj[i + 1];
    Hj[i + 1] = -sn[i] * Hj[i] + c[i] * Hj[i + 1];
    Hj[i] = t;
  }
  const double rr = hypot(Hj[j], Hj[j + 1]);
  c[j] = Hj[j] / rr;
  sn[j] = Hj[j + 1] / rr;
  Hj[j] = rr;
  Hj[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = c[j] * g[j];
  G.its[s] += 1;
  G.kk[s] = j + 1;
  return !(fabs(g[j + 1]) <= G.target[s] || G.its[s] >= max_it);
}

// A segment stops taking steps; nan: its values are not finite.
__device__ inline void segment_stop(const GmresDev& G, int s, bool nan) {
  if (nan) {
    G.flag[s] = 1;
    G.ran[s] = 0;
  }
  G.act[s] = 0;
  G.fac[s] = 0.0;
}

// Column j of segment s from the two Gram-Schmidt passes (coefficients
// h1[i] + h2[i], i <= j), |w|^2 after (hn2) and before (w02) the passes.
// Returns 1 if the segment takes another step.
__device__ inline int givens_update(const GmresDev& G, int s, int j, int max_it, const double* h1,
                                    const double* h2, double hn2, double w02) {
  const int mr = G.mr;
  if (G.act[s] == 0) {
    G.fac[s] = 0.0;
    return 0;
  }
  const double hn = sqrt(hn2);
  const double w0 = sqrt(w02);
  double* Hj = G.H + (size_t(s) * mr + j) * (mr + 1);
  for (int i = 0; i <= j; ++i) Hj[i] = h1[i] + h2[i];
  Hj[j + 1] = hn;
  if (!isfinite(hn) || !isfinite(w0)) {
    segment_stop(G, s, true);
    return 0;
  }
  const int more = givens_apply(G, s, j, max_it);
  const bool breakdown = hn <= 1e-14 * fmax(w0, 1e-300);
  if (breakdown || !more) {
    segment_stop(G, s, false);
    return 0;
  }
  G.fac[s] = 1.0 / hn;
  return 1;
}

}  // namespace jfnk
