// Host-side drivers: residual / J.v sequences, GMRES and Newton, for one
// mesh or a batch of meshes (segments) solved in lockstep.
#pragma once

#include <vector>

#include "internal.h"
#include "workspace.h"

namespace jfnk {

SegLayout layout_of(const jfnk_mesh* m);
void fill_device(double* d, int64_t n, double value, hipStream_t s);
// Per-segment squared norms of x, read back to the host (waits on s).
void seg_norms2(jfnk_mesh* m, const SegLayout& L, const double* x, FvWork& fw, KrylovWork& kw,
                const int32_t* act, hipStream_t s, std::vector<double>& out);
// Host values / flags to the device through the pinned staging area (waits on s).
void upload_flags(jfnk_mesh* m, const std::vector<char>& flag, int32_t* d_act, hipStream_t s);
void upload_doubles(jfnk_mesh* m, const std::vector<double>& v, double* d, hipStream_t s);

// R(u) into R with the per-segment load factors in fw.load (device).
void residual_into(jfnk_mesh* m, const double* u, double* R, FvWork& fw, const int32_t* active,
                   hipStream_t s);

// J v into Jv using cached Ru; eps <= 0 selects the automatic per-segment
// step (computed on the device into fw.eps), eps > 0 is used for every segment.
// uu (may be null): per-segment |u|^2, when already known.  With volume
// terms set on the mesh (body force, inertia), Ru is the full R(u) unless
// ru_surface is true, in which case it is R(u) without its volume terms.
// Central difference (R(u + eps v) - R(u - eps v)) / (2 eps): the regions
// it uses (R(u - eps v) and -eps per segment); Ru is then not used.
struct CentralFd {
  double* rm = nullptr;
  double* eps_neg = nullptr;
};
// eps_mach^(1/3) / eps_mach^(1/2): the automatic central step from the forward one
constexpr double kCentralStepFactor = 406.3746693038589;
void jv_into(jfnk_mesh* m, const double* u, const double* Ru, const double* v, double eps, double* Jv,
             FvWork& fw, const int32_t* active, hipStream_t s, const double* uu = nullptr,
             bool ru_surface = false, const CentralFd* cfd = nullptr);
void jv_central(jfnk_mesh* m, const double* u, const double* v, double eps, double* Jv, FvWork& fw,
                const int32_t* active, hipStream_t s, const double* uu, const CentralFd& cfd);

// ---- volume terms (source_kernels.hip) ----
// out = in + S(u) (add) or out = in - S(u): S = load f_b Omega - rho Omega a_BDF2(u)
void launch_source(const jfnk_mesh* m, const SegScalars& sc, const double* u, const double* in, double* out,
                   bool add, hipStream_t s);
// jv -= rho Omega 9/(4 dt^2) v
void launch_inertia_jv(const jfnk_mesh* m, const SegScalars& sc, const double* v, double* jv, hipStream_t s);
void launch_predict(int64_t total, double dt, bool taylor, const double* un, const double* v, const double* acc,
                    double* u, hipStream_t s);
void launch_bdf2_update(int64_t total, double dt, const double* u, const double* un, double* u_prev, double* v,
                        double* v_prev, double* acc, hipStream_t s);
// J_tilde's diagonal with the inertia term of time step dt (0: none): the
// Jacobi inverse is updated and AMG hierarchies built for another dt dropped.
void set_preconditioner_inertia(jfnk_mesh* m, double dt, hipStream_t s);

struct GmresSeg {
  jfnk_status status = JFNK_OK;
  int iterations = 0;
  int restarts = 0;
  int jv = 0;
  double bnorm = 0, res_true = 0;
};

// Right-preconditioned restarted (flexible) GMRES with CGS2 for J x = b on
// every segment s with part[s] != 0 (all segments when part is empty).
// x_is_zero skips the initial J x product.
void gmres_solve(jfnk_mesh* m, const double* u, const double* Ru, const double* b, double* x,
                 bool x_is_zero, const jfnk_gmres_opts& o, FvWork& fw, KrylovWork& kw, hipStream_t s,
                 const std::vector<char>& part, std::vector<GmresSeg>& out, double* t_ms);

// Segregated quasi-Newton iteration with J_tilde (single-mesh handles).
void segregated_solve(jfnk_mesh* m, const jfnk_segregated_opts& o, double* u, FvWork& fw, KrylovWork& kw,
                      hipStream_t s, jfnk_stats& st, jfnk_status& status);

// Newton-Raphson with per-segment load increments; per-segment stats.
void newton_solve(jfnk_mesh* m, const std::vector<int>& n_increments, const jfnk_newton_opts& o,
                  double* u, FvWork& fw, KrylovWork& kw, hipStream_t s, std::vector<jfnk_stats>& stats,
                  std::vector<jfnk_status>& status);

// Longest restart of the delayed-reorthogonalisation Arnoldi (its dots of
// step j take j + 3 partial columns, at most kMaxBasis).
constexpr int kMaxDcgsRestart = 250;

// The preconditioner of a precond value, and whether it carries the FP32
// Z-basis flag.
inline int pc_kind(int precond) { return precond & ~JFNK_PC_Z32; }
inline bool pc_z32(int precond) { return (precond & JFNK_PC_Z32) != 0; }
inline bool amg_precond(int precond) { return pc_kind(precond) == JFNK_PC_AMG32 || pc_kind(precond) == JFNK_PC_AMG64; }
// Preconditioner work region of a solve workspace, in floats (4-byte units).
size_t precond_work_floats(const jfnk_mesh* m, int precond);
size_t precond_work_floats(int64_t n_cells, int dim, int precond);
void precond_setup(jfnk_mesh* m, int precond, hipStream_t s);
// gated: the kernels skip when no segment is taking Arnoldi steps (inside a
// cycle); outside a cycle the application must not be gated.
void precond_apply(jfnk_mesh* m, int precond, int cheb_degree, const double* r, double* z,
                   KrylovWork& kw, hipStream_t s, bool gated = true);
void amg_destroy(AmgHierarchy* a);
// Device bytes held by a hierarchy (0 for null).
size_t amg_device_bytes(const AmgHierarchy* a);
void amg_describe(const AmgHierarchy& H, jfnk_amg_info& info);
void autotune(jfnk_mesh* m, const jfnk_gmres_opts& o, const double* u, double load, void* work, hipStream_t s,
              jfnk_tune_report* rep);

}  // namespace jfnk
