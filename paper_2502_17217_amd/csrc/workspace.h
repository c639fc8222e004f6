// Layout of the caller-provided device workspace.
#pragma once

#include <cstddef>
#include <cstdint>

#include "blas.h"
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

// Regions used by jfnk_residual / jfnk_jv.
struct FvWork {
  double* grad = nullptr;      // [n_cells][rec_doubles(dim)] per-cell {w, x_c, grad w}
  double* ru = nullptr;        // [n_dof] R(u) when not supplied
  double* partials = nullptr;  // [kRedBlocks * kMaxBasis]
  double* scalars = nullptr;   // [64]: 0 eps, 1.. reserved
  void carve(Carver& c, int64_t n_cells, int dim) {
    grad = c.take<double>(size_t(n_cells) * rec_doubles(dim));
    ru = c.take<double>(size_t(n_cells) * dim);
    partials = c.take<double>(size_t(kRedBlocks) * kMaxBasis);
    scalars = c.take<double>(64);
  }
};

// Additional regions used by the Krylov solver and Newton.
struct KrylovWork {
  double* V = nullptr;    // [(m+1)][n_dof] orthonormal basis
  double* Z = nullptr;    // [m][n_dof] preconditioned directions (flexible GMRES)
  double* w = nullptr;    // [n_dof]
  double* r = nullptr;    // [n_dof]
  double* b = nullptr;    // [n_dof] Newton right-hand side
  double* du = nullptr;   // [n_dof] Newton correction
  double* R = nullptr;    // [n_dof] Newton residual R(u)
  double* h = nullptr;    // [kMaxBasis + 8] Hessenberg column / scalars
  double* y = nullptr;    // [kMaxBasis]
  float* pc = nullptr;    // preconditioner work (FP32)
  size_t pc_floats = 0;
  void carve(Carver& c, int64_t n_dof, int m, size_t pc_f) {
    V = c.take<double>(size_t(m + 1) * n_dof);
    Z = c.take<double>(size_t(m) * n_dof);
    w = c.take<double>(n_dof);
    r = c.take<double>(n_dof);
    b = c.take<double>(n_dof);
    du = c.take<double>(n_dof);
    R = c.take<double>(n_dof);
    h = c.take<double>(kMaxBasis + 8);
    y = c.take<double>(kMaxBasis);
    pc_floats = pc_f;
    pc = pc_f ? c.take<float>(pc_f) : nullptr;
  }
};

}  // namespace jfnk
