// Internal declarations shared by the host code and the HIP kernels of the
// JFNK library.  Nothing here is part of the public ABI (see include/jfnk.h).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "jfnk.h"

namespace jfnk {

// Error carried from the inside of the library to the C ABI, where it is
// turned into a status code and a thread-local message.
struct Error {
  jfnk_status status;
  std::string msg;
};

void set_last_error(const std::string& msg);

// Host threads for setup work: at most 16 and at most the hardware's; one
// for fewer than four items (starting threads would cost more than it saves).
inline int host_threads(int64_t items) {
  const int hw = int(std::thread::hardware_concurrency());
  if (items < 4) return 1;
  return int(std::max<int64_t>(1, std::min<int64_t>({items, int64_t(16), int64_t(hw > 0 ? hw : 1)})));
}

// Runs job(t) for t = 1 .. nt-1 on persistent host threads (and job(0) on
// the caller), returning when all have finished.  False when another host
// thread is using the pool (the caller then starts its own threads).
bool host_pool_run(int nt, const std::function<void(int)>& job);

// f(i, t) for i in [0, n) on host_threads(n) threads (indices handed out in
// turn, t = the calling thread's number for per-thread scratch); an
// exception is rethrown after every thread has finished (the one of the
// lowest index).
template <class F>
void parallel_for(int64_t n, F&& f) {
  const int nt = host_threads(n);
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i, 0);
    return;
  }
  std::atomic<int64_t> next{0};
  std::mutex mu;
  std::exception_ptr err;
  int64_t err_i = n;
  auto work = [&](int t) {
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= n) return;
      try {
        f(i, t);
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu);
        if (i < err_i) {
          err_i = i;
          err = std::current_exception();
        }
      }
    }
  };
  if (!host_pool_run(nt, work)) {
    std::vector<std::thread> pool;
    for (int k = 1; k < nt; ++k) pool.emplace_back(work, k);
    work(0);
    for (std::thread& th : pool) th.join();
  }
  if (err) std::rethrow_exception(err);
}

#define JFNK_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::jfnk::Error{JFNK_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define JFNK_REQUIRE(cond, status, msg)                  \
  do {                                                   \
    if (!(cond)) throw ::jfnk::Error{(status), (msg)};   \
  } while (0)

// Cells are processed one per lane; 64 consecutive cells (one wavefront)
// form an ELL slice whose slot arrays are stored [slot][lane].
constexpr int kSlice = 64;
constexpr int kBlock = 256;
constexpr int kNumXcd = 8;
// launch shape of the two cell passes (tuned on gfx950)
#ifndef JFNK_FV_MINWAVES
#define JFNK_FV_MINWAVES 1
#endif
// waves per SIMD the LDS-tiled cell passes are compiled for
#ifndef JFNK_TILED_MINWAVES
#define JFNK_TILED_MINWAVES 1
#endif
// waves per SIMD the fused J v pass is compiled for
#ifndef JFNK_FUSED_MINWAVES
#define JFNK_FUSED_MINWAVES 1
#endif
// scheduling barrier between the neo-Hookean face evaluations of a lane
#ifndef JFNK_FACE_SCHED_BARRIER
#define JFNK_FACE_SCHED_BARRIER 1
#endif
#ifndef JFNK_XCD_REMAP
#define JFNK_XCD_REMAP 1
#endif
// Cells of the two cell passes are processed in workgroups of kFvBlock
// consecutive cells; segments of a batch start on multiples of kSegAlign so
// that every workgroup belongs to exactly one segment.
constexpr int kFvBlock = 256;
constexpr int kSegAlign = kFvBlock;
// LDS budget of one workgroup of the tiled (LDS-staged) cell passes: the
// tile's kFvBlock cells plus its halo, (2 dim + dim^2) doubles per cell
constexpr int kTileLdsBytes = 64 * 1024;
inline int64_t tile_halo_limit(int dim) { return kTileLdsBytes / (8 * (2 * dim + dim * dim)) - kFvBlock; }
// LDS of one flux workgroup (staged tile + halo, then the in-tile face
// forces); at most this, so that two workgroups share a compute unit
constexpr int kFluxLdsBytes = 80 * 1024;
inline size_t flux_lds_bytes(int dim, int64_t halo_stride, int64_t face_stride) {
  return sizeof(double) * (size_t(2 * dim + dim * dim) * size_t(halo_stride) + size_t(dim) * size_t(face_stride));
}
// Face entries of one tile that a lane of the fused J v pass holds in
// registers between its phases (the pass needs faces_max <= this).
constexpr int kFusedFaceEntries = 4 * kFvBlock;
// LDS of the fused J v pass: w and centroids of tile, halo and second ring
// (later overwritten by the face forces), gradients of tile and halo, one
// row of boundary face forces
inline int fused_wx_doubles(int dim, int64_t ring_stride, int64_t face_stride) {
  return int(std::max<int64_t>(2 * dim * ring_stride, dim * face_stride));
}
inline size_t fused_lds_bytes(int dim, int64_t ring_stride, int64_t halo_stride, int64_t face_stride) {
  return sizeof(double) * (size_t(fused_wx_doubles(dim, ring_stride, face_stride)) +
                           size_t(dim * dim) * size_t(halo_stride) + size_t(dim) * kFvBlock);
}
// slot_nb values
constexpr int kSlotBoundary = -1;
constexpr int kSlotPad = -2;
// stride (doubles) of one internal-face record {Gamma, w} and of one
// boundary-face record {Gamma(3), d_b(3), value(3), type}
constexpr int kFaceRec = 4;
constexpr int kBfaceRec = 10;
// boundary type codes in the record (a symmetry record holds
// {Gamma, d_b, unit normal, type})
constexpr int kBcDisp = 1, kBcTrac = 2, kBcPres = 3, kBcSymm = 4;

// Per-segment constants (one segment = one mesh of a batch).
struct SegInfo {
  double mu, lam, kappa;     // law constants (Appendix B)
  double aK;                 // alpha_rc * K_bar, K_bar = 2 mu + lambda
  int32_t law;
  int32_t cell_off;          // first cell of the segment in the union numbering
  int32_t n_cells;           // cells of the segment (cells beyond are padding)
  int32_t pad_;
  double rho;                // density (inertia term only)
};

// Read-only device view of a mesh or a batch of meshes (the union of the
// segments, each renumbered internally and placed at an aligned offset),
// passed by value to kernels.  Cell and face arrays are component-major
// (structure of arrays) so that 64 lanes reading consecutive cells or faces
// touch consecutive addresses.
struct MeshDev {
  int32_t n_cells;           // union cells including alignment padding
  int32_t dim;
  int32_t n_slices;
  int32_t n_int;             // union internal faces
  int32_t n_seg;
  int32_t law_mask;          // bit 0: linear-elastic, bit 1: neo-Hookean, bit 2: St. Venant-Kirchhoff segment
  int32_t has_symm;          // some boundary face is a symmetry plane (its record type kBcSymm)
  int32_t pad_symm_;
  const int32_t* slice_ptr;  // [n_slices + 1], in slots (multiples of kSlice)
  const int32_t* slot_nb;    // neighbour cell, kSlotBoundary or kSlotPad
  const int32_t* slot_fc;    // internal: face (owner side) or ~face (neighbour side); boundary: bface
  const double* xc;          // [dim][n_cells] cell centroids
  const double* fG;          // [dim][n_int] Gamma_f, outward from the owner
  const double* fw;          // [n_int] interpolation weight w_f of the owner
  const double* magG;        // [n_int] |Gamma_f|
  const double* bface;       // [n_boundary][10] {Gamma, d_b, value, type}
  const int32_t* seg_of_block;  // [ceil(n_cells / kFvBlock)]
  const SegInfo* seg;        // [n_seg]
  // tiles (tiled != 0): slot_loc gives the neighbour's position in the
  // workgroup's LDS copy (0..kFvBlock-1: inside the tile, kFvBlock + h:
  // entry h of the tile's halo list) or the slot_nb code of other slots
  int32_t tiled;
  int32_t lds_kernels;       // tiled mesh: 1 LDS-staged passes, 2 fused single pass; 0 gathers (tuner's choice)
  int32_t persist;           // workgroups of a persistent cell-pass launch (0: one per tile)
  int32_t halo_stride;       // kFvBlock + largest halo: LDS row length
  const int32_t* slot_loc;   // [n_slots]
  const int32_t* halo_ptr;   // [n_tiles + 1]
  const int32_t* halo_cells; // [halo_ptr[n_tiles]] cell numbers
  // Face lists of the tiles for the LDS flux pass.  Tile t evaluates each
  // internal face touching it once: the faces its cells own (the contiguous
  // range fbeg[t] .. fbeg[t+1]-1, owner < neighbour) and the incoming faces
  // owned by an earlier tile (in_face[in_ptr[t] ..]); face_loc / in_loc pack
  // the LDS positions of owner (low 16 bits) and neighbour (high 16 bits).
  // After the internal faces (n_ent entries) come the tile's boundary faces
  // (bnd_face[bnd_ptr[t] ..]: boundary-face numbers, bnd_loc: the owner's
  // position in the tile).  slot_code gives, for every slot, the entry of
  // its face in the tile's list, 2 entry + 1 on the neighbour side of an
  // internal face and 2 entry otherwise, -1 for padding slots.
  const int32_t* fbeg;       // [n_tiles + 1]
  const int32_t* face_loc;   // [n_int]
  const int32_t* in_ptr;     // [n_tiles + 1]
  const int32_t* in_face;    // [in_ptr[n_tiles]]
  const int32_t* in_loc;     // [in_ptr[n_tiles]]
  const int32_t* bnd_ptr;    // [n_tiles + 1]
  const int32_t* bnd_face;   // [bnd_ptr[n_tiles]]
  const int32_t* bnd_loc;    // [bnd_ptr[n_tiles]]
  const int32_t* slot_code;  // [n_slots]
  const double* slot_mg;     // [n_slots] |Gamma_f| of the slot's face (0 for other slots)
  int32_t face_stride;       // largest face list of a tile (internal + boundary): LDS row length
  // Fused J v pass (fused != 0): a tile also stages its second ring (outside
  // cells adjacent to the halo, h2_cells[h2_ptr[t] ..]) and recomputes the
  // halo cells' gradients.  Halo cell i of tile t has its slots, in its own
  // slot order, at h1_loc/h1_mg[halo_ptr[t] * h1_width + k * n_halo + i]:
  // the neighbour's position in the tile's copy (tile, halo, second ring)
  // or a slot code, and |Gamma_f| of the slot's face.
  int32_t fused;
  int32_t h1_width;          // slots per halo cell in the lists (largest slice width)
  int32_t ring_stride;       // kFvBlock + largest halo + largest second ring
  const int32_t* h2_ptr;     // [n_tiles + 1]
  const int32_t* h2_cells;   // [h2_ptr[n_tiles]]
  const int16_t* h1_loc;     // [halo total * h1_width]
  const double* h1_mg;       // [halo total * h1_width]
  const int32_t* h1_fc;      // [halo total * h1_width] boundary face of a boundary slot (has_symm only)
};

// Per-call, per-segment device scalars.
// Segments with at most this many tiles finish their sums inside the
// producing kernel (in its last tile); larger ones use a separate reduction
// launch spread over many workgroups.
constexpr int kFuseTiles = 64;

struct SegScalars {
  const double* eps;         // [n_seg] J v step (null: residual evaluation)
  const double* load;        // [n_seg] load factor, or null: load1 for every segment
  const int32_t* active;     // [n_seg] or null: segments with 0 are skipped
  double load1 = 0.0;
  __host__ __device__ double load_at(int seg) const { return load != nullptr ? load[seg] : load1; }
};

// Host-side result of mesh preprocessing (all in internal numbering).
struct HostMesh {
  int dim = 0;
  int64_t n_cells = 0, n_int = 0, n_bnd = 0;
  std::vector<int32_t> old_of_new, new_of_old;
  std::vector<double> xc, vol;
  std::vector<double> face;         // n_int * kFaceRec
  std::vector<double> magG;         // n_int, |Gamma_f| (least-squares weights)
  std::vector<int32_t> fown, fnb;   // internal faces, owner < neighbour
  std::vector<double> bface;        // n_bnd * kBfaceRec
  std::vector<int32_t> bown;
  std::vector<int32_t> slice_ptr, slot_nb, slot_fc;
  std::vector<double> pc_diag;      // approximate Jacobian, scalar diagonal (alpha_pc)
  std::vector<double> pc_off;       // per internal face off-diagonal coefficient
  // symmetry faces: per-component addition to the diagonal, [n_cells][dim]
  // (the diagonal of the n n block); empty when the mesh has none
  std::vector<double> pc_sym;
  int64_t bandwidth = 0;
  bool tiled = false;               // cell order is in compact tiles whose halos fit the LDS budget
  int64_t tile_halo_max = 0;
};

struct Material {
  int law = JFNK_LINEAR_ELASTIC;
  double E = 0, nu = 0, alpha_rc = 1, alpha_pc = 1, rho = 0;
  double mu = 0, lam = 0, kappa = 0, Kbar = 0;
};

Material make_material(const jfnk_material& m);
void build_host_mesh(const jfnk_mesh_desc& d, const Material& mat, HostMesh& hm);
// Inverse of the approximate Jacobian's diagonal for the Jacobi
// preconditioner: [n] from the scalar diagonal, or [dim][n] when sym (the
// symmetry faces' per-component additions, [n][dim]) is not empty.
std::vector<double> jacobi_inverse(const std::vector<double>& diag, const std::vector<double>& sym, int dim);

// Host arrays of a batch union, ready for upload.
// Host vector whose resize leaves new elements of trivial type unset: large
// setup arrays that are written in full right after they are sized, by
// several threads, have their pages first touched in parallel rather than by
// one zero fill.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};
template <class T>
using HostVec = std::vector<T, NoInitAlloc<T>>;

struct UnionArrays {
  std::vector<int32_t> slice_ptr, slot_nb, slot_fc, ext, seg_of_block;
  std::vector<int32_t> slot_loc, halo_ptr, halo_cells, fbeg, face_loc, in_ptr, in_face, in_loc;
  std::vector<int16_t> h1_loc;
  std::vector<int32_t> h2_ptr, h2_cells, bnd_ptr, bnd_face, bnd_loc, slot_code;
  std::vector<double> h1_mg, slot_mg;
  std::vector<int32_t> h1_fc;
  // faces_max: largest internal face list of a tile; bnd_max: largest
  // boundary list; ent_max: largest internal + boundary list
  int64_t halo_max = 0, faces_max = 0, bnd_max = 0, ent_max = 0, h2_max = 0, h1_width = 0;
  HostVec<double> xc, face, magG, bface;  // sized without zero fill, written in full
  std::vector<double> vol;                  // cell volumes (0 on padding cells)
  std::vector<double> pc_dinv;              // [n] or, with symmetry faces, [dim][n]
  std::vector<SegInfo> seg;
};

// Allocation context of the calling thread: when `stream` is set (the
// request workers of the server), device buffers are allocated and freed
// stream-ordered on it, so that one request's allocations never wait for
// the work of requests running on other streams; `pinned` (if set) is a
// caller-owned pinned host buffer of `pinned_doubles` doubles that new mesh
// handles use instead of allocating their own.
struct AllocContext {
  hipStream_t stream = nullptr;
  double* pinned = nullptr;
  size_t pinned_doubles = 0;
};
AllocContext& alloc_context();

// HIP graph capture (exclusive) against allocation, free and other
// device-wide calls made by other threads (shared): the runtime may reject
// such calls while any stream of the process is being captured.
std::shared_mutex& capture_mutex();

// Device buffer with RAII.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;  // non-null: allocated with hipMallocAsync on this stream
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), stream(o.stream) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      stream = o.stream;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() noexcept;
  void alloc(size_t b);
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

struct AmgHierarchy;  // AMG preconditioner (amg.cpp)

// Volume terms of the residual (Section 2.3.1): a body force per unit volume
// and the BDF2 inertia of Eq. (inertia2) from caller-owned previous
// displacements and velocities (internal layout).
struct VolumeSource {
  DevBuf body;                 // [dim][n_cells] body force density (internal layout)
  bool has_body = false;
  double dt = 0;               // > 0: inertia included
  const double* u_n = nullptr;
  const double* u_nm1 = nullptr;
  const double* v_n = nullptr;
  const double* v_nm1 = nullptr;
  bool active() const { return has_body || dt > 0; }
};

// HIP-event timing of kernel classes (enabled per mesh for measurement).
struct Profiler {
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    int cls;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  static constexpr int kClasses = 6;
  double ms[kClasses] = {0, 0, 0, 0, 0, 0};
  int64_t calls[kClasses] = {0, 0, 0, 0, 0, 0};
  hipEvent_t get();
  // Record a start event; returns the index for end().
  int begin(int cls, hipStream_t s);
  void end(int idx, hipStream_t s);
  void collect();
  ~Profiler();
};

}  // namespace jfnk

namespace jfnk {
struct Segment {
  HostMesh host;             // the mesh in its own internal numbering
  Material mat;
  int64_t cell_off = 0;      // first union cell
  int64_t ext_off = 0;       // first cell in the concatenated external (input-order) layout
  int64_t face_off = 0, bface_off = 0;
};
}  // namespace jfnk

namespace jfnk {
// HIP graphs of runs of Arnoldi steps, captured once per set of launch
// arguments (workspace, state vectors, options) and replayed every cycle.
struct StepGraphs {
  const void* work = nullptr;
  const double* u = nullptr;
  const double* Ru = nullptr;
  int restart = 0, precond = -1, cheb = 0, chunk = 0, max_it = 0, left = -1, central = -1, orth = -1;
  double eps = 0;
  std::vector<hipGraphExec_t> exec;  // one per chunk of steps (null until captured)
  void clear();
};

// Launch choices made by the autotuner (jfnk_autotune) or the defaults.
struct Tuning {
  int step_chunk = 1;    // Arnoldi steps enqueued between host convergence checks
  int graphs = 1;        // replay runs of steps from HIP graphs
  int orth = 1;          // Arnoldi orthogonalisation where DCGS2 applies (1 DCGS2, 0 CGS2)
  int tuned = 0;         // 1 once jfnk_autotune has run
};
}  // namespace jfnk

// The opaque handle of the ABI: one mesh, or a batch of meshes solved
// together (segments).
struct jfnk_mesh {
  std::vector<jfnk::Segment> segs;
  jfnk::HostMesh host;              // union arrays (approximate Jacobian, faces) used by setup code
  int64_t n_ext_cells = 0;          // sum of segment cells
  std::vector<int32_t> block_first; // [n_seg + 1] first workgroup (kFvBlock cells) of each segment
  jfnk::MeshDev dev{};
  jfnk::DevBuf b_slice_ptr, b_slot_nb, b_slot_fc, b_xc, b_fG, b_fw, b_magG, b_bface, b_ext, b_pc_dinv,
      b_seg_of_block, b_seg, b_block_first, b_slot_loc, b_halo_ptr, b_halo_cells, b_slot_code, b_bnd_ptr, b_bnd_face, b_bnd_loc, b_fbeg,
      b_face_loc, b_in_ptr, b_in_face, b_in_loc, b_h2_ptr, b_h2_cells, b_h1_loc, b_h1_mg,
      b_slot_mg, b_h1_fc;
  double* pinned = nullptr;         // pinned host scalars for D2H reads
  size_t pinned_doubles = 0;
  bool pinned_owned = true;
  jfnk_mesh_info info{};
  jfnk::VolumeSource src;
  jfnk::DevBuf b_vol;                    // [n_cells] cell volumes (union; 0 on padding)
  double pc_dt = 0;                      // inertia time step included in the preconditioners (0: none)
  std::vector<double> pc_diag_eff;       // J_tilde diagonal with the inertia term (empty: host.pc_diag)
  jfnk::AmgHierarchy* amg = nullptr;     // FP32 hierarchy (JFNK_PC_AMG32)
  jfnk::AmgHierarchy* amg64 = nullptr;   // FP64 hierarchy (JFNK_PC_AMG64)
  jfnk::DevBuf b_seg_ad, b_seg_ao;       // -J_tilde for the segregated solver: diagonal, face off-diagonals
  bool seg_jt_ready = false;
  double seg_jt_dt = 0;                  // inertia time step included in b_seg_ad
  jfnk::Profiler prof;
  jfnk::StepGraphs graphs;
  jfnk::Tuning tune;
  hipStream_t solve_stream = nullptr;   // own stream for graph capture when the caller passes the null stream
  bool any_large = true;                // a segment has more tiles than the fused reductions finish in-kernel
  bool any_small = true;                // a segment is finished in-kernel (uses the arrival counters)
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  int n_seg() const { return int(segs.size()); }
  jfnk_mesh() = default;
  jfnk_mesh(const jfnk_mesh&) = delete;
  jfnk_mesh& operator=(const jfnk_mesh&) = delete;
  ~jfnk_mesh();   // releases graphs, events, the own stream, AMG and owned pinned memory
};

namespace jfnk {

// ---- kernel launchers (fv_kernels.hip, blas.hip) ----
// Per-cell record of w = u + eps*v (v may be null), written by the gradient
// pass and gathered by the flux pass: {w, grad w} stored component-major,
// rec_doubles(dim) arrays of n_cells doubles.
inline int rec_doubles(int dim) { return dim + dim * dim; }
void launch_gradient(const MeshDev& m, const double* u, const double* v, const SegScalars& sc,
                     double* rec, hipStream_t s);
// out = (R(w) - Ru)/eps if Ru != null else R(w) (per-segment eps and load).
// Fused single pass: R(w) (v = null, Ru = null) or (R(u + eps v) - R(u))/eps.
void launch_fused(const MeshDev& m, const double* u, const double* v, const SegScalars& sc, const double* Ru,
                  double* out, hipStream_t s);
void launch_flux(const MeshDev& m, const double* rec, const SegScalars& sc, const double* Ru, double* out,
                 hipStream_t s);
void launch_set_scalars(double* d, const double* h_values, int n, hipStream_t s);
void build_union(jfnk_mesh& m, UnionArrays& ua);
// The fused J v pass fits a tiled union: tile positions fit 16 bits, the
// face entries of a tile one register round (internal faces kEnt per lane,
// boundary faces one per lane), the copy a workgroup's LDS.
inline bool fused_fits(int dim, const UnionArrays& ua) {
  const int64_t ring = kFvBlock + ua.halo_max + ua.h2_max;
  return ring < 32768 && ua.faces_max <= kFusedFaceEntries && ua.bnd_max <= kFvBlock &&
         fused_lds_bytes(dim, ring, kFvBlock + ua.halo_max, std::max<int64_t>(ua.ent_max, 1)) <=
             size_t(kFluxLdsBytes) * 2;
}
// Upload the union of m's segments on stream s (mesh handle setup).
void finish_handle(jfnk_mesh& m, hipStream_t s, double t0);
size_t device_bytes_of(const HostMesh& h);

void launch_permute(const int32_t* ext_of_int, const double* in, double* out, int64_t n_cells, int dim,
                    bool to_internal, hipStream_t s);

}  // namespace jfnk
