// Volume terms of the residual (Section 2.3.1, midpoint rule per cell):
// the body force load * f_b,P Omega_P and the inertia -rho Omega_P a_P with
// the BDF2 acceleration of Eq. (inertia2)
//   a_P = [3 (3 u - 4 u^t + u^{t-1}) / (2 dt) - 4 v^t + v^{t-1}] / (2 dt),
// plus the element-wise updates of a transient step (Taylor predictor of
// Eq. (predictor), BDF2 velocity and acceleration).  One thread per cell,
// all components; padding cells of a batch are left untouched.
#include "solver.h"

namespace jfnk {

namespace {

constexpr int kB = 256;

struct SourceArgs {
  int n;                        // union cells
  const int32_t* seg_of_block;
  const SegInfo* seg;
  const double* vol;
  const double* body;           // [dim][n] or null
  double dt;                    // > 0: inertia
  const double* u_n;
  const double* u_nm1;
  const double* v_n;
  const double* v_nm1;
  const double* load;           // per segment, or null: load1
  double load1;
  const int32_t* active;        // per segment, or null
};

// Cell c of segment seg, or -1 for a padding cell / a switched-off segment.
__device__ __forceinline__ int cell_segment(const SourceArgs& a, int c) {
  const int seg = a.seg_of_block[c / kFvBlock];
  if (a.active != nullptr && a.active[seg] == 0) return -1;
  const SegInfo& g = a.seg[seg];
  return (c - g.cell_off < g.n_cells) ? seg : -1;
}

// mode 0: out = in + S(u)        (residual: surface terms + volume terms)
// mode 1: out = in - S(u)        (the surface part of a cached R(u))
template <int D>
__global__ __launch_bounds__(kB) void k_source(SourceArgs a, const double* __restrict__ u, const double* in,
                                               double* out, int mode) {
  const int c = blockIdx.x * kB + threadIdx.x;
  if (c >= a.n) return;
  const int seg = cell_segment(a, c);
  if (seg < 0) return;
  const double V = a.vol[c];
  const double ld = a.load != nullptr ? a.load[seg] : a.load1;
  const double rho = a.seg[seg].rho;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * a.n + c;
    double s = 0.0;
    if (a.body != nullptr) s = ld * a.body[o] * V;
    if (a.dt > 0.0 && rho > 0.0) {
      const double h = 0.5 / a.dt;
      const double vel = (3.0 * u[o] - 4.0 * a.u_n[o] + a.u_nm1[o]) * h;
      const double acc = (3.0 * vel - 4.0 * a.v_n[o] + a.v_nm1[o]) * h;
      s -= rho * V * acc;
    }
    out[o] = mode == 0 ? in[o] + s : in[o] - s;
  }
}

// Jv -= rho Omega 9/(4 dt^2) v: the inertia term's derivative (exact, the
// term is affine in u).
template <int D>
__global__ __launch_bounds__(kB) void k_inertia_jv(SourceArgs a, const double* __restrict__ v,
                                                   double* __restrict__ jv) {
  const int c = blockIdx.x * kB + threadIdx.x;
  if (c >= a.n) return;
  const int seg = cell_segment(a, c);
  if (seg < 0) return;
  const double k = 2.25 * a.seg[seg].rho * a.vol[c] / (a.dt * a.dt);
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = size_t(q) * a.n + c;
    jv[o] = fma(-k, v[o], jv[o]);
  }
}

// u = u^t + dt v^t + dt^2/2 a^t (Eq. predictor), or u = u^t.
__global__ __launch_bounds__(kB) void k_predict(int64_t total, double dt, int taylor, const double* __restrict__ un,
                                                const double* __restrict__ v, const double* __restrict__ acc,
                                                double* __restrict__ u) {
  const int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x;
  if (i >= total) return;
  u[i] = taylor ? fma(0.5 * dt * dt, acc[i], fma(dt, v[i], un[i])) : un[i];
}

// After a step: v^{t+1} = (3 u - 4 u^t + u^{t-1})/(2 dt),
// a^{t+1} = (3 v^{t+1} - 4 v^t + v^{t-1})/(2 dt); then the histories shift:
// u_prev <- u^t, v_prev <- v^t, v <- v^{t+1}, acc <- a^{t+1}.
__global__ __launch_bounds__(kB) void k_bdf2_update(int64_t total, double dt, const double* __restrict__ u,
                                                    const double* __restrict__ un, double* __restrict__ u_prev,
                                                    double* __restrict__ v, double* __restrict__ v_prev,
                                                    double* __restrict__ acc) {
  const int64_t i = int64_t(blockIdx.x) * kB + threadIdx.x;
  if (i >= total) return;
  const double h = 0.5 / dt;
  const double vn = v[i], vp = v_prev[i], u0 = un[i];
  const double vel = (3.0 * u[i] - 4.0 * u0 + u_prev[i]) * h;
  acc[i] = (3.0 * vel - 4.0 * vn + vp) * h;
  u_prev[i] = u0;
  v_prev[i] = vn;
  v[i] = vel;
}

SourceArgs args_of(const jfnk_mesh* m, const SegScalars& sc) {
  const VolumeSource& src = m->src;
  SourceArgs a;
  a.n = m->dev.n_cells;
  a.seg_of_block = m->dev.seg_of_block;
  a.seg = m->dev.seg;
  a.vol = m->b_vol.as<double>();
  a.body = src.has_body ? src.body.as<double>() : nullptr;
  a.dt = src.dt;
  a.u_n = src.u_n;
  a.u_nm1 = src.u_nm1;
  a.v_n = src.v_n;
  a.v_nm1 = src.v_nm1;
  a.load = sc.load;
  a.load1 = sc.load1;
  a.active = sc.active;
  return a;
}

inline int blocks_for(int64_t n) { return int((n + kB - 1) / kB); }

}  // namespace

void launch_source(const jfnk_mesh* m, const SegScalars& sc, const double* u, const double* in, double* out,
                   bool add, hipStream_t s) {
  const SourceArgs a = args_of(m, sc);
  if (m->dev.dim == 3)
    hipLaunchKernelGGL(k_source<3>, dim3(blocks_for(a.n)), dim3(kB), 0, s, a, u, in, out, add ? 0 : 1);
  else
    hipLaunchKernelGGL(k_source<2>, dim3(blocks_for(a.n)), dim3(kB), 0, s, a, u, in, out, add ? 0 : 1);
  JFNK_HIP(hipGetLastError());
}

void launch_inertia_jv(const jfnk_mesh* m, const SegScalars& sc, const double* v, double* jv, hipStream_t s) {
  const SourceArgs a = args_of(m, sc);
  if (m->dev.dim == 3)
    hipLaunchKernelGGL(k_inertia_jv<3>, dim3(blocks_for(a.n)), dim3(kB), 0, s, a, v, jv);
  else
    hipLaunchKernelGGL(k_inertia_jv<2>, dim3(blocks_for(a.n)), dim3(kB), 0, s, a, v, jv);
  JFNK_HIP(hipGetLastError());
}

void launch_predict(int64_t total, double dt, bool taylor, const double* un, const double* v, const double* acc,
                    double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_predict, dim3(blocks_for(total)), dim3(kB), 0, s, total, dt, taylor ? 1 : 0, un, v, acc, u);
  JFNK_HIP(hipGetLastError());
}

void launch_bdf2_update(int64_t total, double dt, const double* u, const double* un, double* u_prev, double* v,
                        double* v_prev, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_bdf2_update, dim3(blocks_for(total)), dim3(kB), 0, s, total, dt, u, un, u_prev, v, v_prev,
                     acc);
  JFNK_HIP(hipGetLastError());
}

}  // namespace jfnk
