// Layout of the caller-provided device workspace.
#pragma once

#include <cstddef>
#include <cstdint>

#include "blas.h"
#include "gmres_dev.h"
#include "internal.h"

namespace jfnk {

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Carves named regions out of one device allocation (or only measures it
// when base == nullptr).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += align256(count * sizeof(T));
    return p;
  }
};

inline int64_t n_tiles(int64_t n_cells) { return (n_cells + kFvBlock - 1) / kFvBlock; }
inline int64_t n_tiles(const jfnk_mesh* m) { return n_tiles(m->host.n_cells); }

// Regions used by jfnk_residual / jfnk_jv.
struct FvWork {
  double* grad = nullptr;      // [rec_doubles(dim)][n_cells] per-cell {w, grad w}
  double* ru = nullptr;        // [n_dof] R(u) when not supplied
  double* ru_src = nullptr;    // [n_dof] R(u) without its volume terms (J v with body force / inertia)
  double* partials = nullptr;  // [n_tiles * kMaxBasis]
  double* eps = nullptr;       // [n_seg] J v step per segment
  double* load = nullptr;      // [n_seg] load factor per segment
  int32_t* tickets = nullptr;  // [2 n_seg + 8] arrival counters of the fused reductions (zero between launches)
  int S = 0;
  void carve(Carver& c, int64_t n, int dim, int S_) {
    S = S_;
    grad = c.take<double>(size_t(n) * rec_doubles(dim));
    ru = c.take<double>(size_t(n) * dim);
    ru_src = c.take<double>(size_t(n) * dim);
    partials = c.take<double>(size_t(n_tiles(n)) * kMaxBasis);
    eps = c.take<double>(S);
    load = c.take<double>(S);
    tickets = c.take<int32_t>(size_t(2) * S + 8);
  }
  int32_t* eps_tickets() const { return tickets; }
  int32_t* cgs_tickets() const { return tickets + S; }
  int32_t* step_counters() const { return tickets + 2 * S; }
  // The caller's workspace starts uninitialised: clear the counters once.
  void zero_counters(hipStream_t s) const { fill_int(tickets, 2 * S + 8, 0, s); }
  // zero_counters and the same load factor for every segment, in one launch
  void setup(hipStream_t s, double load_value) const { call_setup(tickets, 2 * S + 8, load, S, load_value, s); }
  // For one residual or J v with the same load factor everywhere: the factor
  // travels as a kernel argument, and the counters are cleared only when a
  // segment finishes its sums in-kernel (nothing to launch otherwise).
  bool uniform = false;
  double load1 = 0.0;
  void setup_uniform(hipStream_t s, double load_value, bool any_small) {
    uniform = true;
    load1 = load_value;
    if (any_small) zero_counters(s);
  }
  const double* load_ptr() const { return uniform ? nullptr : load; }
  void carve(Carver& c, const jfnk_mesh* m) { carve(c, m->host.n_cells, m->host.dim, m->n_seg()); }
};

// Additional regions used by the Krylov solver and Newton.
struct KrylovWork {
  double* V = nullptr;    // [(m+1)][n_dof] orthonormal basis
  double* Z = nullptr;    // [m][n_dof] preconditioned directions (flexible GMRES), or null:
  float* Zf = nullptr;    // [m][n_dof] the same in FP32 (Z-basis flag), with
  double* zd = nullptr;   // [n_dof] the direction being formed, in FP64
  bool z32 = false;       // the Z basis is Zf
  double* w = nullptr;    // [n_dof]
  double* r = nullptr;    // [n_dof]
  double* b = nullptr;    // [n_dof] Newton right-hand side
  double* du = nullptr;   // [n_dof] Newton correction
  double* R = nullptr;    // [n_dof] Newton residual R(u)
  double* h = nullptr;    // [n_seg][kMaxBasis] Hessenberg column, first pass
  double* h2 = nullptr;   // [n_seg][kMaxBasis] second pass
  double* nrm = nullptr;  // [n_seg][4] squared norms
  double* y = nullptr;    // [n_seg][kMaxBasis] least-squares solution
  double* fac = nullptr;  // [n_seg] per-segment factors
  int32_t* act = nullptr; // [n_seg] active flags
  double* stage = nullptr;  // [3 n_seg] per-cycle values uploaded by the host
  double* uu = nullptr;     // [n_seg] |u|^2 of the state of the current linear solve
  double* rm = nullptr;     // [n_dof] R(u - eps v) of a central-difference J v
  double* eps_neg = nullptr;  // [n_seg] -eps of a central-difference J v
  double* partials2 = nullptr;  // [n_tiles * kMaxBasis] second tile-sum region (DCGS2 dots)
  GmresDev gd;            // device Arnoldi bookkeeping (shares fac and act)
  float* pc = nullptr;    // preconditioner work (FP32)
  size_t pc_floats = 0;
  void carve(Carver& c, const jfnk_mesh* m, int restart, size_t pc_f, bool z32 = false) {
    carve(c, m->host.n_cells, m->host.dim, m->n_seg(), restart, pc_f, z32);
  }
  void carve(Carver& c, int64_t n_cells, int dim, int S, int restart, size_t pc_f, bool z32 = false) {
    const int64_t n_dof = n_cells * dim;
    V = c.take<double>(size_t(restart + 1) * n_dof);
    this->z32 = z32;
    if (z32) {
      Zf = c.take<float>(size_t(restart) * n_dof);
      zd = c.take<double>(n_dof);
    } else {
      Z = c.take<double>(size_t(restart) * n_dof);
    }
    w = c.take<double>(n_dof);
    r = c.take<double>(n_dof);
    b = c.take<double>(n_dof);
    du = c.take<double>(n_dof);
    R = c.take<double>(n_dof);
    h = c.take<double>(size_t(S) * kMaxBasis);
    h2 = c.take<double>(size_t(S) * kMaxBasis);
    nrm = c.take<double>(size_t(S) * 4);
    y = c.take<double>(size_t(S) * kMaxBasis);
    fac = c.take<double>(S);
    act = c.take<int32_t>(S);
    stage = c.take<double>(size_t(3) * S);
    uu = c.take<double>(S);
    rm = c.take<double>(n_dof);
    eps_neg = c.take<double>(S);
    partials2 = c.take<double>(size_t(n_tiles(n_cells)) * kMaxBasis);
    gd.mr = restart;
    gd.H = c.take<double>(size_t(S) * restart * (restart + 1));
    gd.cs = c.take<double>(size_t(S) * restart);
    gd.sn = c.take<double>(size_t(S) * restart);
    gd.g = c.take<double>(size_t(S) * (restart + 1));
    gd.target = c.take<double>(S);
    gd.fac = fac;
    gd.act = act;
    gd.ran = c.take<int32_t>(S);
    gd.kk = c.take<int32_t>(S);
    gd.its = c.take<int32_t>(S);
    gd.flag = c.take<int32_t>(S);
    gd.nact = c.take<int32_t>(4);
    pc_floats = pc_f;
    pc = pc_f ? c.take<float>(pc_f) : nullptr;
  }
};

// Workspace bytes of a solve (op 1) on n cells of dimension dim in S segments.
inline size_t solve_workspace_bytes(int64_t n, int dim, int S, int restart, size_t pc_floats, bool z32 = false) {
  Carver c(nullptr);
  FvWork fw;
  fw.carve(c, n, dim, S);
  KrylovWork kw;
  kw.carve(c, n, dim, S, restart, pc_floats, z32);
  return c.off;
}

}  // namespace jfnk
