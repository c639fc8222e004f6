// The C ABI of the library (include/jfnk.h): argument checking, error
// translation, mesh upload, and the Newton driver.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>

#include "solver.h"

namespace jfnk {

namespace {
thread_local std::string g_last_error;

template <class F>
jfnk_status guarded(F&& f) {
  try {
    f();
    return JFNK_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return JFNK_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return JFNK_E_ARG;
  }
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Transpose a row-major [rows][cols] host array (row stride `ld`) into
// component-major [cols][rows].
template <class V>
std::vector<double> to_soa(const V& a, int64_t rows, int cols, int ld) {
  std::vector<double> out(size_t(rows) * cols);
  for (int64_t r = 0; r < rows; ++r)
    for (int k = 0; k < cols; ++k) out[size_t(k) * rows + r] = a[size_t(r) * ld + k];
  return out;
}

template <class T, class A>
void upload(DevBuf& b, const std::vector<T, A>& v, hipStream_t s) {
  b.alloc(std::max<size_t>(v.size() * sizeof(T), 256));
  if (!v.empty())
    JFNK_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}


void check_mesh(const jfnk_mesh* m) {
  JFNK_REQUIRE(m != nullptr, JFNK_E_ARG, "null mesh handle");
}

void check_ptr(const void* p, const char* what) {
  JFNK_REQUIRE(p != nullptr, JFNK_E_ARG, std::string("null device pointer: ") + what);
}

void check_work(const void* w) {
  JFNK_REQUIRE(w != nullptr, JFNK_E_ARG, "null workspace");
  JFNK_REQUIRE((reinterpret_cast<uintptr_t>(w) & 255) == 0, JFNK_E_ARG,
               "workspace must be 256-byte aligned");
}

void check_opts(const jfnk_gmres_opts& o) {
  JFNK_REQUIRE(o.restart >= 1 && o.restart < kMaxBasis, JFNK_E_ARG, "gmres: restart out of range");
  JFNK_REQUIRE(o.max_it >= 1, JFNK_E_ARG, "gmres: max_it must be >= 1");
  JFNK_REQUIRE(o.rtol >= 0 && o.atol >= 0, JFNK_E_ARG, "gmres: negative tolerance");
  JFNK_REQUIRE(pc_kind(o.precond) >= JFNK_PC_NONE && pc_kind(o.precond) <= JFNK_PC_AMG64, JFNK_E_ARG,
               "gmres: unknown preconditioner");
  JFNK_REQUIRE(!pc_z32(o.precond) || (!o.left && !o.augment), JFNK_E_ARG,
               "gmres: the FP32 Z basis needs right preconditioning without augmentation");
  JFNK_REQUIRE(!amg_precond(o.precond) || (o.cheb_degree >= 1 && o.cheb_degree <= 16), JFNK_E_ARG,
               "gmres: cheb_degree must lie in [1, 16]");
  JFNK_REQUIRE(o.step_chunk >= 0 && o.step_chunk <= o.restart, JFNK_E_ARG,
               "gmres: step_chunk must lie in [0, restart]");
  JFNK_REQUIRE(o.graphs >= 0 && o.graphs <= 2, JFNK_E_ARG, "gmres: graphs must be 0, 1 or 2");
  JFNK_REQUIRE(o.left == 0 || o.left == 1, JFNK_E_ARG, "gmres: left must be 0 or 1");
  JFNK_REQUIRE(o.augment >= 0 && o.augment < o.restart, JFNK_E_ARG, "gmres: augment must lie in [0, restart)");
  JFNK_REQUIRE(!(o.left && o.augment), JFNK_E_ARG, "gmres: augmentation needs right preconditioning");
  JFNK_REQUIRE(o.fd_central == 0 || o.fd_central == 1, JFNK_E_ARG, "gmres: fd_central must be 0 or 1");
  JFNK_REQUIRE(o.orth >= 0 && o.orth <= 2, JFNK_E_ARG, "gmres: orth must be 0, 1 or 2");
  JFNK_REQUIRE(o.orth != 1 || (!o.left && o.restart <= kMaxDcgsRestart), JFNK_E_ARG,
               "gmres: orth = 1 needs right preconditioning and restart <= 250");
}

// Stream the solvers run on: the caller's, or, when the caller passes the
// null stream (which cannot be captured) and graphs are requested, the
// handle's own stream ordered after the caller's work.
hipStream_t solver_stream(jfnk_mesh* m, hipStream_t s, bool graphs) {
  if (s != nullptr || !graphs) return s;
  if (!m->solve_stream) JFNK_HIP(hipStreamCreateWithFlags(&m->solve_stream, hipStreamNonBlocking));
  if (!m->ev[2]) JFNK_HIP(hipEventCreateWithFlags(&m->ev[2], hipEventDisableTiming));
  JFNK_HIP(hipEventRecord(m->ev[2], s));
  JFNK_HIP(hipStreamWaitEvent(m->solve_stream, m->ev[2], 0));
  return m->solve_stream;
}

bool wants_graphs(const jfnk_mesh* m, const jfnk_gmres_opts& o) {
  return (o.graphs == 2 ? m->tune.graphs : o.graphs) != 0;
}

// The caller's stream waits for the solver's.
void join_stream(jfnk_mesh* m, hipStream_t caller, hipStream_t used) {
  if (used == caller) return;
  if (!m->ev[3]) JFNK_HIP(hipEventCreateWithFlags(&m->ev[3], hipEventDisableTiming));
  JFNK_HIP(hipEventRecord(m->ev[3], used));
  JFNK_HIP(hipStreamWaitEvent(caller, m->ev[3], 0));
}

}  // namespace

size_t device_bytes_of(const HostMesh& h) {
  auto b = [](size_t x) { return std::max<size_t>(x, 256); };
  return b(h.slice_ptr.size() * 4) + b(h.slot_nb.size() * 4) + b(h.slot_fc.size() * 4) +
         b(h.xc.size() * 8) + b(size_t(h.n_int) * h.dim * 8) + b(size_t(h.n_int) * 8) +
         b(h.magG.size() * 8) + b(h.bface.size() * 8) + b(h.old_of_new.size() * 4) +
         b(size_t(h.n_cells) * 8) + b(size_t(h.n_cells / kFvBlock + 1) * 4) + 3 * 256 +
         // tiles: slot_loc, slot_code, halo, incoming-face and boundary lists (at most one
         // entry per slot each), per-tile offsets, packed face positions
         (h.tiled ? 6 * b(h.slot_nb.size() * 4) + 5 * b(size_t(h.n_cells / kFvBlock + 2) * 4) +
                        b(size_t(h.n_int) * 4) +
                        // second ring (at most one entry per slot), the halo cells' slot lists,
                        // |Gamma_f| per slot
                        b(h.slot_nb.size() * 4) + b(h.slot_nb.size() * 10) + b(h.slot_nb.size() * 8)
                  : 0);
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

// Persistent worker threads for host setup passes.  Created on first use and
// kept for the life of the process (the object is never destroyed, so no
// thread is joined during static destruction).
class HostPool {
 public:
  explicit HostPool(int workers) {
    for (int k = 1; k <= workers; ++k)
      std::thread([this, k] { loop(k); }).detach();
  }
  bool run(int nt, const std::function<void(int)>& job) {
    std::unique_lock<std::mutex> busy(busy_, std::try_to_lock);
    if (!busy.owns_lock()) return false;
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &job;
      nt_ = nt;
      remaining_ = nt - 1;
      ++gen_;
    }
    start_.notify_all();
    job(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return remaining_ == 0; });
    job_ = nullptr;
    return true;
  }

 private:
  void loop(int k) {
    int64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* job;
      {
        std::unique_lock<std::mutex> lk(mu_);
        start_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        if (k >= nt_) continue;
        job = job_;
      }
      (*job)(k);
      std::lock_guard<std::mutex> lk(mu_);
      if (--remaining_ == 0) done_.notify_all();
    }
  }
  std::mutex busy_, mu_;
  std::condition_variable start_, done_;
  const std::function<void(int)>* job_ = nullptr;
  int nt_ = 0, remaining_ = 0;
  int64_t gen_ = 0;
};

}  // namespace

bool host_pool_run(int nt, const std::function<void(int)>& job) {
  static HostPool* pool = new HostPool(15);
  if (nt - 1 > 15) return false;
  return pool->run(nt, job);
}

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  JFNK_HIP(hipEventCreate(&e));
  return e;
}

int Profiler::begin(int cls, hipStream_t s) {
  Rec r{get(), get(), cls};
  JFNK_HIP(hipEventRecord(r.a, s));
  pending.push_back(r);
  return int(pending.size()) - 1;
}

void Profiler::end(int idx, hipStream_t s) { JFNK_HIP(hipEventRecord(pending[idx].b, s)); }

void Profiler::collect() {
  for (Rec& r : pending) {
    JFNK_HIP(hipEventSynchronize(r.b));
    float t = 0;
    JFNK_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.cls] += t;
    calls[r.cls] += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}

Profiler::~Profiler() {
  for (Rec& r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

AllocContext& alloc_context() {
  thread_local AllocContext ctx;
  return ctx;
}

std::shared_mutex& capture_mutex() {
  static std::shared_mutex mu;
  return mu;
}

void DevBuf::release() noexcept {
  if (p) {
    std::shared_lock<std::shared_mutex> lk(capture_mutex());
    if (stream)
      (void)hipFreeAsync(p, stream);
    else
      (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
}

void DevBuf::alloc(size_t b) {
  release();
  stream = alloc_context().stream;
  std::shared_lock<std::shared_mutex> lk(capture_mutex());
  hipError_t e = stream ? hipMallocAsync(&p, b, stream) : hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    throw Error{JFNK_E_OOM, "device allocation of " + std::to_string(b) + " bytes failed"};
  }
  bytes = b;
}

}  // namespace jfnk

using namespace jfnk;

jfnk_mesh::~jfnk_mesh() {
  if (amg) amg_destroy(amg);   // its buffers take the capture lock themselves
  if (amg64) amg_destroy(amg64);
  std::shared_lock<std::shared_mutex> lk(capture_mutex());
  graphs.clear();
  for (hipEvent_t& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (solve_stream) (void)hipStreamDestroy(solve_stream);
  if (pinned && pinned_owned) (void)hipHostFree(pinned);
}

namespace jfnk {

// Build the union of the handle's segments and upload it.
void finish_handle(jfnk_mesh& m, hipStream_t s, double t0) {
  UnionArrays ua;
  build_union(m, ua);
  const HostMesh& h = m.host;
  const int dim = h.dim;
  upload(m.b_slice_ptr, ua.slice_ptr, s);
  upload(m.b_slot_nb, ua.slot_nb, s);
  upload(m.b_slot_fc, ua.slot_fc, s);
  upload(m.b_xc, to_soa(ua.xc, h.n_cells, dim, dim), s);
  upload(m.b_vol, ua.vol, s);
  upload(m.b_fG, to_soa(ua.face, h.n_int, dim, kFaceRec), s);
  {
    std::vector<double> fw(h.n_int);
    for (int64_t j = 0; j < h.n_int; ++j) fw[j] = ua.face[j * kFaceRec + (dim == 3 ? 3 : 2)];
    upload(m.b_fw, fw, s);
  }
  upload(m.b_magG, ua.magG, s);
  upload(m.b_bface, ua.bface, s);
  upload(m.b_ext, ua.ext, s);
  upload(m.b_pc_dinv, ua.pc_dinv, s);
  upload(m.b_seg_of_block, ua.seg_of_block, s);
  upload(m.b_seg, ua.seg, s);
  upload(m.b_block_first, m.block_first, s);
  if (h.tiled) {
    upload(m.b_slot_loc, ua.slot_loc, s);
    upload(m.b_halo_ptr, ua.halo_ptr, s);
    upload(m.b_halo_cells, ua.halo_cells, s);
    upload(m.b_slot_code, ua.slot_code, s);
    upload(m.b_bnd_ptr, ua.bnd_ptr, s);
    upload(m.b_bnd_face, ua.bnd_face, s);
    upload(m.b_bnd_loc, ua.bnd_loc, s);
    upload(m.b_fbeg, ua.fbeg, s);
    upload(m.b_face_loc, ua.face_loc, s);
    upload(m.b_in_ptr, ua.in_ptr, s);
    upload(m.b_in_face, ua.in_face, s);
    upload(m.b_in_loc, ua.in_loc, s);
    upload(m.b_h2_ptr, ua.h2_ptr, s);
    upload(m.b_h2_cells, ua.h2_cells, s);
    upload(m.b_h1_loc, ua.h1_loc, s);
    upload(m.b_h1_mg, ua.h1_mg, s);
    if (!h.pc_sym.empty()) upload(m.b_h1_fc, ua.h1_fc, s);
    upload(m.b_slot_mg, ua.slot_mg, s);
  }
  JFNK_HIP(hipStreamSynchronize(s));
  const int S = m.n_seg();
  m.pinned_doubles = size_t(4 * kMaxBasis + 8) * size_t(std::max(S, 1)) + 64;
  AllocContext& ac = alloc_context();
  if (ac.pinned && ac.pinned_doubles >= m.pinned_doubles) {
    m.pinned = ac.pinned;
    m.pinned_owned = false;
  } else {
    std::shared_lock<std::shared_mutex> lk(capture_mutex());
    JFNK_HIP(hipHostMalloc(reinterpret_cast<void**>(&m.pinned), sizeof(double) * m.pinned_doubles,
                           hipHostMallocDefault));
  }
  MeshDev& d = m.dev;
  d.n_cells = int32_t(h.n_cells);
  d.dim = dim;
  d.n_slices = int32_t(ua.slice_ptr.size() - 1);
  d.n_int = int32_t(h.n_int);
  d.n_seg = S;
  d.law_mask = 0;
  for (const Segment& g : m.segs)
    d.law_mask |= g.mat.law == JFNK_NEO_HOOKEAN ? 2 : g.mat.law == JFNK_ST_VENANT_KIRCHHOFF ? 4 : 1;
  d.slice_ptr = m.b_slice_ptr.as<int32_t>();
  d.slot_nb = m.b_slot_nb.as<int32_t>();
  d.slot_fc = m.b_slot_fc.as<int32_t>();
  d.xc = m.b_xc.as<double>();
  d.fG = m.b_fG.as<double>();
  d.fw = m.b_fw.as<double>();
  d.magG = m.b_magG.as<double>();
  d.bface = m.b_bface.as<double>();
  d.seg_of_block = m.b_seg_of_block.as<int32_t>();
  d.seg = m.b_seg.as<SegInfo>();
  {
    SegLayout L;
    L.n_seg = S;
    m.any_large = any_large_segment(L, m.block_first.data());
    m.any_small = false;
    for (int k = 0; k < S; ++k) m.any_small = m.any_small || m.block_first[k + 1] - m.block_first[k] <= kFuseTiles;
  }
  d.tiled = h.tiled ? 1 : 0;
  d.lds_kernels = d.tiled;
  d.persist = 0;
  d.halo_stride = int32_t(kFvBlock + ua.halo_max);
  d.slot_loc = h.tiled ? m.b_slot_loc.as<int32_t>() : nullptr;
  d.halo_ptr = h.tiled ? m.b_halo_ptr.as<int32_t>() : nullptr;
  d.halo_cells = h.tiled ? m.b_halo_cells.as<int32_t>() : nullptr;
  d.slot_code = h.tiled ? m.b_slot_code.as<int32_t>() : nullptr;
  d.bnd_ptr = h.tiled ? m.b_bnd_ptr.as<int32_t>() : nullptr;
  d.bnd_face = h.tiled ? m.b_bnd_face.as<int32_t>() : nullptr;
  d.bnd_loc = h.tiled ? m.b_bnd_loc.as<int32_t>() : nullptr;
  d.fbeg = h.tiled ? m.b_fbeg.as<int32_t>() : nullptr;
  d.face_loc = h.tiled ? m.b_face_loc.as<int32_t>() : nullptr;
  d.in_ptr = h.tiled ? m.b_in_ptr.as<int32_t>() : nullptr;
  d.in_face = h.tiled ? m.b_in_face.as<int32_t>() : nullptr;
  d.in_loc = h.tiled ? m.b_in_loc.as<int32_t>() : nullptr;
  d.face_stride = int32_t(std::max<int64_t>(ua.ent_max, 1));
  // the deduplicating LDS flux pass needs its staged tile and face forces in LDS
  if (d.tiled && flux_lds_bytes(dim, d.halo_stride, d.face_stride) > size_t(kFluxLdsBytes) * 2) d.lds_kernels = 0;
  d.h1_width = int32_t(ua.h1_width);
  d.ring_stride = int32_t(kFvBlock + ua.halo_max + ua.h2_max);
  d.h2_ptr = h.tiled ? m.b_h2_ptr.as<int32_t>() : nullptr;
  d.h2_cells = h.tiled ? m.b_h2_cells.as<int32_t>() : nullptr;
  d.h1_loc = h.tiled ? m.b_h1_loc.as<int16_t>() : nullptr;
  d.h1_mg = h.tiled ? m.b_h1_mg.as<double>() : nullptr;
  d.has_symm = h.pc_sym.empty() ? 0 : 1;
  d.h1_fc = (h.tiled && d.has_symm) ? m.b_h1_fc.as<int32_t>() : nullptr;
  d.slot_mg = h.tiled ? m.b_slot_mg.as<double>() : nullptr;
  d.fused = (d.tiled && fused_fits(dim, ua)) ? 1 : 0;
  jfnk_mesh_info& in = m.info;
  in.n_cells = h.n_cells;
  in.dim = dim;
  in.n_dof = h.n_cells * dim;
  in.n_internal_faces = h.n_int;
  in.n_boundary_faces = h.n_bnd;
  in.bandwidth = h.bandwidth;
  in.device_bytes = int64_t(m.b_slice_ptr.bytes + m.b_slot_nb.bytes + m.b_slot_fc.bytes + m.b_xc.bytes +
                            m.b_fG.bytes + m.b_fw.bytes + m.b_magG.bytes + m.b_bface.bytes +
                            m.b_ext.bytes + m.b_pc_dinv.bytes + m.b_seg_of_block.bytes + m.b_seg.bytes +
                            m.b_block_first.bytes + m.b_slot_loc.bytes + m.b_halo_ptr.bytes +
                            m.b_halo_cells.bytes + m.b_slot_code.bytes + m.b_bnd_ptr.bytes +
                            m.b_bnd_face.bytes + m.b_bnd_loc.bytes + m.b_fbeg.bytes + m.b_face_loc.bytes +
                            m.b_in_ptr.bytes + m.b_in_face.bytes + m.b_in_loc.bytes + m.b_h2_ptr.bytes +
                            m.b_h2_cells.bytes + m.b_h1_loc.bytes + m.b_h1_mg.bytes +
                            m.b_slot_mg.bytes + m.b_h1_fc.bytes);
  in.n_slots = int64_t(ua.slot_nb.size());
  in.n_segments = S;
  in.n_dof_external = m.n_ext_cells * dim;
  in.tiled = d.tiled;
  in.tile_halo_max = int32_t(ua.halo_max);
  in.tile_halo_total = int64_t(ua.halo_cells.size());
  in.tile_incoming_total = int64_t(ua.in_face.size());
  in.tile_ring2_max = int32_t(ua.h2_max);
  in.tile_ring2_total = int64_t(ua.h2_cells.size());
  in.tile_faces_max = int32_t(ua.faces_max);
  in.tile_entries_max = int32_t(ua.ent_max);
  in.fused = d.fused;
  in.setup_ms = now_ms() - t0;
}

}  // namespace jfnk

extern "C" {

const char* jfnk_last_error(void) { return g_last_error.c_str(); }

jfnk_status jfnk_autotune(jfnk_mesh* mesh, const jfnk_gmres_opts* opts, const double* d_u, double load,
                          void* d_work, void* stream, jfnk_tune_report* report) {
  return guarded([&] {
    check_mesh(mesh);
    check_ptr(d_u, "u");
    check_work(d_work);
    JFNK_REQUIRE(opts, JFNK_E_ARG, "autotune: null options");
    check_opts(*opts);
    JFNK_REQUIRE(std::isfinite(load), JFNK_E_ARG, "autotune: load factor not finite");
    const hipStream_t caller = static_cast<hipStream_t>(stream);
    const hipStream_t s = solver_stream(mesh, caller, true);
    autotune(mesh, *opts, d_u, load, d_work, s, report);
    join_stream(mesh, caller, s);
  });
}

jfnk_status jfnk_set_cell_passes(jfnk_mesh* mesh, int32_t passes, int32_t persist) {
  return guarded([&] {
    check_mesh(mesh);
    JFNK_REQUIRE(passes >= 0 && passes <= 2, JFNK_E_ARG, "set_cell_passes: passes must be 0, 1 or 2");
    JFNK_REQUIRE(passes == 0 || mesh->dev.tiled, JFNK_E_ARG, "set_cell_passes: the mesh is not tile-ordered");
    JFNK_REQUIRE(passes < 2 || mesh->dev.fused, JFNK_E_ARG,
                 "set_cell_passes: the fused pass does not fit this mesh's tiles");
    JFNK_REQUIRE(persist >= 0, JFNK_E_ARG, "set_cell_passes: persist < 0");
    std::shared_lock<std::shared_mutex> lk(capture_mutex());
    mesh->graphs.clear();  // captured runs hold the old launches
    mesh->dev.lds_kernels = passes;
    mesh->dev.persist = persist;
  });
}

jfnk_status jfnk_amg_info_get(const jfnk_mesh* mesh, int32_t precond, jfnk_amg_info* info) {
  return guarded([&] {
    check_mesh(mesh);
    JFNK_REQUIRE(info != nullptr, JFNK_E_ARG, "amg_info: null output");
    JFNK_REQUIRE(precond == JFNK_PC_AMG32 || precond == JFNK_PC_AMG64, JFNK_E_ARG,
                 "amg_info: precond must be AMG32 or AMG64");
    const AmgHierarchy* H = precond == JFNK_PC_AMG64 ? mesh->amg64 : mesh->amg;
    JFNK_REQUIRE(H != nullptr, JFNK_E_ARG, "amg_info: hierarchy not built yet (run a solve or jfnk_autotune)");
    amg_describe(*H, *info);
  });
}

const char* jfnk_version(void) { return "jfnk-mi355x 0.1 (gfx950)"; }


jfnk_status jfnk_create_mesh(const jfnk_mesh_desc* desc, const jfnk_material* mat, void* stream,
                             jfnk_mesh** out) {
  return jfnk_create_batch(desc, mat, 1, stream, out);
}

jfnk_status jfnk_create_batch(const jfnk_mesh_desc* descs, const jfnk_material* mats, int32_t n,
                              void* stream, jfnk_mesh** out) {
  return guarded([&] {
    JFNK_REQUIRE(descs && mats && out && n >= 1, JFNK_E_ARG, "create: null argument or empty batch");
    *out = nullptr;
    const double t0 = now_ms();
    auto m = std::make_unique<jfnk_mesh>();
    m->segs.resize(n);
    // The meshes of a batch are independent: host threads take them in turn.
    // The error reported is that of the lowest-numbered failing mesh.
    std::vector<Error> errs(n);
    std::vector<char> failed(n, 0);
    std::atomic<int32_t> next{0};
    auto work = [&] {
      for (int32_t s; (s = next.fetch_add(1)) < n;) {
        try {
          m->segs[s].mat = make_material(mats[s]);
          build_host_mesh(descs[s], m->segs[s].mat, m->segs[s].host);
        } catch (Error& e) {
          errs[s] = e;
          failed[s] = 1;
        } catch (const std::bad_alloc&) {
          errs[s] = Error{JFNK_E_OOM, "host allocation failed"};
          failed[s] = 1;
        } catch (const std::exception& e) {
          errs[s] = Error{JFNK_E_ARG, e.what()};
          failed[s] = 1;
        }
      }
    };
    const int nt = std::max(1, std::min<int>(n, int(std::thread::hardware_concurrency()) > 0
                                                    ? std::min(16, int(std::thread::hardware_concurrency()))
                                                    : 1));
    std::vector<std::thread> pool;
    for (int k = 1; k < nt; ++k) pool.emplace_back(work);
    work();
    for (std::thread& t : pool) t.join();
    for (int32_t s = 0; s < n; ++s)
      if (failed[s]) {
        Error e = errs[s];
        if (n > 1) e.msg = "batch mesh " + std::to_string(s) + ": " + e.msg;
        throw e;
      }
    finish_handle(*m, static_cast<hipStream_t>(stream), t0);
    *out = m.release();
  });
}

jfnk_status jfnk_segment_info(const jfnk_mesh* mesh, int32_t seg, int64_t* cell_off, int64_t* n_cells,
                              int64_t* ext_off) {
  return guarded([&] {
    JFNK_REQUIRE(mesh != nullptr, JFNK_E_ARG, "null mesh handle");
    JFNK_REQUIRE(seg >= 0 && seg < mesh->n_seg(), JFNK_E_ARG, "segment index out of range");
    const Segment& g = mesh->segs[seg];
    if (cell_off) *cell_off = g.cell_off;
    if (n_cells) *n_cells = g.host.n_cells;
    if (ext_off) *ext_off = g.ext_off;
  });
}

jfnk_status jfnk_inspect_mesh(const jfnk_mesh_desc* desc, const jfnk_material* mat,
                              jfnk_mesh_info* info, double* xc_out, double* vol_out) {
  return guarded([&] {
    JFNK_REQUIRE(desc && mat && info, JFNK_E_ARG, "inspect_mesh: null argument");
    const double t0 = now_ms();
    Material mt = make_material(*mat);
    HostMesh h;
    build_host_mesh(*desc, mt, h);
    std::memset(info, 0, sizeof(*info));
    info->n_cells = h.n_cells;
    info->dim = h.dim;
    info->n_dof = h.n_cells * h.dim;
    info->n_internal_faces = h.n_int;
    info->n_boundary_faces = h.n_bnd;
    info->bandwidth = h.bandwidth;
    info->device_bytes = int64_t(device_bytes_of(h));
    info->setup_ms = now_ms() - t0;
    info->n_slots = int64_t(h.slot_nb.size());
    info->n_segments = 1;
    info->n_dof_external = h.n_cells * h.dim;
    info->tiled = h.tiled ? 1 : 0;
    info->tile_halo_max = int32_t(h.tile_halo_max);
    if (h.tiled) {
      // the tile lists the device handle would build, host side only
      jfnk_mesh tmp;
      tmp.segs.resize(1);
      tmp.segs[0].host = h;
      tmp.segs[0].mat = mt;
      UnionArrays ua;
      build_union(tmp, ua);
      info->tile_halo_total = int64_t(ua.halo_cells.size());
      info->tile_incoming_total = int64_t(ua.in_face.size());
      info->tile_ring2_max = int32_t(ua.h2_max);
      info->tile_ring2_total = int64_t(ua.h2_cells.size());
      info->tile_faces_max = int32_t(ua.faces_max);
      info->tile_entries_max = int32_t(ua.ent_max);
      info->fused = fused_fits(h.dim, ua) ? 1 : 0;
    }
    for (int64_t i = 0; i < h.n_cells; ++i) {
      const int64_t o = h.old_of_new[i];
      if (xc_out)
        for (int k = 0; k < h.dim; ++k) xc_out[o * h.dim + k] = h.xc[i * h.dim + k];
      if (vol_out) vol_out[o] = h.vol[i];
    }
  });
}

jfnk_status jfnk_destroy_mesh(jfnk_mesh* mesh) {
  return guarded([&] {
    if (!mesh) return;
    delete mesh;
  });
}

jfnk_status jfnk_profile_enable(jfnk_mesh* mesh, int32_t on) {
  return guarded([&] {
    check_mesh(mesh);
    mesh->prof.on = on != 0;
  });
}

jfnk_status jfnk_profile_read(jfnk_mesh* mesh, double* ms, int64_t* calls, int32_t reset) {
  return guarded([&] {
    check_mesh(mesh);
    mesh->prof.collect();
    for (int k = 0; k < Profiler::kClasses; ++k) {
      if (ms) ms[k] = mesh->prof.ms[k];
      if (calls) calls[k] = mesh->prof.calls[k];
      if (reset) {
        mesh->prof.ms[k] = 0;
        mesh->prof.calls[k] = 0;
      }
    }
  });
}

jfnk_status jfnk_get_mesh_info(const jfnk_mesh* mesh, jfnk_mesh_info* info) {
  return guarded([&] {
    check_mesh(mesh);
    JFNK_REQUIRE(info, JFNK_E_ARG, "null info");
    *info = mesh->info;
  });
}

jfnk_status jfnk_mesh_order(const jfnk_mesh* mesh, int32_t* old_of_new) {
  return guarded([&] {
    check_mesh(mesh);
    JFNK_REQUIRE(old_of_new, JFNK_E_ARG, "null output");
    // per segment, in segment order: input cell index (within the segment) of each internal cell
    int64_t o = 0;
    for (const Segment& g : mesh->segs) {
      std::memcpy(old_of_new + o, g.host.old_of_new.data(), sizeof(int32_t) * g.host.n_cells);
      o += g.host.n_cells;
    }
  });
}

jfnk_status jfnk_to_internal(const jfnk_mesh* mesh, const double* d_in, double* d_out, void* stream) {
  return guarded([&] {
    check_mesh(mesh);
    check_ptr(d_in, "in");
    check_ptr(d_out, "out");
    JFNK_REQUIRE(d_in != d_out, JFNK_E_ARG, "permutation cannot run in place");
    launch_permute(mesh->b_ext.as<int32_t>(), d_in, d_out, mesh->host.n_cells, mesh->host.dim, true,
                   static_cast<hipStream_t>(stream));
  });
}

jfnk_status jfnk_to_external(const jfnk_mesh* mesh, const double* d_in, double* d_out, void* stream) {
  return guarded([&] {
    check_mesh(mesh);
    check_ptr(d_in, "in");
    check_ptr(d_out, "out");
    JFNK_REQUIRE(d_in != d_out, JFNK_E_ARG, "permutation cannot run in place");
    launch_permute(mesh->b_ext.as<int32_t>(), d_in, d_out, mesh->host.n_cells, mesh->host.dim, false,
                   static_cast<hipStream_t>(stream));
  });
}

jfnk_status jfnk_workspace_size(const jfnk_mesh* mesh, int32_t op, int32_t restart, int32_t precond,
                                size_t* bytes) {
  return guarded([&] {
    check_mesh(mesh);
    JFNK_REQUIRE(bytes, JFNK_E_ARG, "null output");
    JFNK_REQUIRE(op >= 0 && op <= 3, JFNK_E_ARG, "workspace_size: op must be 0, 1, 2 or 3");
    Carver c(nullptr);
    FvWork fw;
    fw.carve(c, mesh);
    if (op == 3) {
      (void)c.take<double>(size_t(mesh->dev.n_cells) * mesh->dev.dim);   // R(u - eps v)
      (void)c.take<double>(mesh->n_seg());                                // -eps
    } else if (op >= 1) {
      JFNK_REQUIRE(restart >= 1 && restart < kMaxBasis, JFNK_E_ARG, "workspace_size: bad restart");
      JFNK_REQUIRE(pc_kind(precond) >= JFNK_PC_NONE && pc_kind(precond) <= JFNK_PC_AMG64, JFNK_E_ARG,
                   "workspace_size: unknown preconditioner");
      KrylovWork kw;
      kw.carve(c, mesh, restart, precond_work_floats(mesh, precond), pc_z32(precond));
      if (op == 2) (void)c.take<double>(size_t(mesh->dev.n_cells) * mesh->dev.dim);   // u^t of a transient step
    }
    *bytes = c.off;
  });
}

jfnk_status jfnk_residual(jfnk_mesh* mesh, double load, const double* d_u, double* d_R, void* d_work,
                          void* stream) {
  return guarded([&] {
    check_mesh(mesh);
    check_ptr(d_u, "u");
    check_ptr(d_R, "R");
    check_work(d_work);
    JFNK_REQUIRE(d_u != d_R, JFNK_E_ARG, "residual: R may not alias u");
    JFNK_REQUIRE(std::isfinite(load), JFNK_E_ARG, "residual: load factor not finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver c(d_work);
    FvWork fw;
    fw.carve(c, mesh);
    fw.setup_uniform(s, load, mesh->any_small);
    residual_into(mesh, d_u, d_R, fw, nullptr, s);
  });
}

jfnk_status jfnk_jv(jfnk_mesh* mesh, double load, const double* d_u, const double* d_Ru,
                    const double* d_v, double eps, double* d_Jv, double* eps_used, void* d_work,
                    void* stream) {
  return guarded([&] {
    check_mesh(mesh);
    check_ptr(d_u, "u");
    check_ptr(d_v, "v");
    check_ptr(d_Jv, "Jv");
    check_work(d_work);
    JFNK_REQUIRE(d_Jv != d_u && d_Jv != d_v && d_Jv != d_Ru, JFNK_E_ARG, "jv: output aliases an input");
    JFNK_REQUIRE(std::isfinite(eps) && std::isfinite(load), JFNK_E_ARG, "jv: eps/load not finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver c(d_work);
    FvWork fw;
    fw.carve(c, mesh);
    fw.setup_uniform(s, load, mesh->any_small);
    const double* Ru = d_Ru;
    if (!Ru) {
      residual_into(mesh, d_u, fw.ru, fw, nullptr, s);
      Ru = fw.ru;
    }
    jv_into(mesh, d_u, Ru, d_v, eps, d_Jv, fw, nullptr, s);
    if (eps_used) {
      JFNK_HIP(hipMemcpyAsync(mesh->pinned, fw.eps, sizeof(double) * mesh->n_seg(), hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipStreamSynchronize(s));
      std::memcpy(eps_used, mesh->pinned, sizeof(double) * mesh->n_seg());
    }
  });
}

jfnk_status jfnk_jv_central(jfnk_mesh* mesh, double load, const double* d_u, const double* d_v, double eps,
                            double* d_Jv, double* eps_used, void* d_work, void* stream) {
  return guarded([&] {
    check_mesh(mesh);
    check_ptr(d_u, "u");
    check_ptr(d_v, "v");
    check_ptr(d_Jv, "Jv");
    check_work(d_work);
    JFNK_REQUIRE(d_Jv != d_u && d_Jv != d_v, JFNK_E_ARG, "jv_central: output aliases an input");
    JFNK_REQUIRE(std::isfinite(eps) && std::isfinite(load), JFNK_E_ARG, "jv_central: eps/load not finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver c(d_work);
    FvWork fw;
    fw.carve(c, mesh);
    CentralFd cfd;
    cfd.rm = c.take<double>(size_t(mesh->dev.n_cells) * mesh->dev.dim);
    cfd.eps_neg = c.take<double>(mesh->n_seg());
    fw.setup_uniform(s, load, mesh->any_small);
    jv_into(mesh, d_u, nullptr, d_v, eps, d_Jv, fw, nullptr, s, nullptr, false, &cfd);
    if (eps_used) {
      JFNK_HIP(hipMemcpyAsync(mesh->pinned, fw.eps, sizeof(double) * mesh->n_seg(), hipMemcpyDeviceToHost, s));
      JFNK_HIP(hipStreamSynchronize(s));
      std::memcpy(eps_used, mesh->pinned, sizeof(double) * mesh->n_seg());
    }
  });
}

jfnk_status jfnk_gmres(jfnk_mesh* mesh, double load, const double* d_u, const double* d_Ru,
                       const double* d_b, double* d_x, const jfnk_gmres_opts* opts, jfnk_stats* stats,
                       void* d_work, void* stream) {
  jfnk_status st = JFNK_OK;
  jfnk_status g = guarded([&] {
    check_mesh(mesh);
    check_ptr(d_u, "u");
    check_ptr(d_Ru, "Ru");
    check_ptr(d_b, "b");
    check_ptr(d_x, "x");
    check_work(d_work);
    JFNK_REQUIRE(opts, JFNK_E_ARG, "gmres: null options");
    check_opts(*opts);
    JFNK_REQUIRE(std::isfinite(load), JFNK_E_ARG, "gmres: load factor not finite");
    const hipStream_t caller = static_cast<hipStream_t>(stream);
    const hipStream_t s = solver_stream(mesh, caller, wants_graphs(mesh, *opts));
    Carver c(d_work);
    FvWork fw;
    fw.carve(c, mesh);
    fw.setup(s, load);
    KrylovWork kw;
    kw.carve(c, mesh, opts->restart, precond_work_floats(mesh, opts->precond), pc_z32(opts->precond));
    precond_setup(mesh, opts->precond, s);
    double t_ms[8] = {0};
    std::vector<GmresSeg> r;
    gmres_solve(mesh, d_u, d_Ru, d_b, d_x, false, *opts, fw, kw, s, {}, r, t_ms);
    join_stream(mesh, caller, s);
    for (int k = 0; k < mesh->n_seg(); ++k) {
      if (stats) {
        jfnk_stats& o = stats[k];
        std::memset(&o, 0, sizeof(o));
        o.gmres_it = r[k].iterations;
        o.restarts = r[k].restarts;
        o.jv_evals = r[k].jv;
        o.res0 = r[k].bnorm;
        o.res_final = r[k].res_true;
        std::memcpy(o.t_ms, t_ms, sizeof(t_ms));
      }
      if (st == JFNK_OK && r[k].status != JFNK_OK) st = r[k].status;
    }
    if (st == JFNK_E_NOT_CONVERGED) set_last_error("gmres: iteration limit reached");
    if (st == JFNK_E_BREAKDOWN) set_last_error("gmres: stagnation (true residual not decreasing)");
    if (st == JFNK_E_NAN) set_last_error("gmres: NaN/Inf encountered");
  });
  return g != JFNK_OK ? g : st;
}

static jfnk_status newton_common(jfnk_mesh* mesh, const int32_t* n_increments, const jfnk_newton_opts* opts,
                                 double* d_u, jfnk_stats* stats, jfnk_status* seg_status, void* d_work,
                                 void* stream) {
  jfnk_status st = JFNK_OK;
  jfnk_status g = guarded([&] {
    check_mesh(mesh);
    check_ptr(d_u, "u");
    check_work(d_work);
    JFNK_REQUIRE(opts, JFNK_E_ARG, "newton: null options");
    JFNK_REQUIRE(opts->max_newton_it >= 1, JFNK_E_ARG, "newton: max_newton_it must be >= 1");
    JFNK_REQUIRE(opts->rtol >= 0 && opts->atol >= 0 && opts->eta > 0 && opts->stol >= 0, JFNK_E_ARG,
                 "newton: bad tolerance");
    JFNK_REQUIRE(opts->line_search == 0 || opts->line_search == 1, JFNK_E_ARG, "newton: line_search must be 0 or 1");
    JFNK_REQUIRE(opts->max_backtrack <= 60, JFNK_E_ARG, "newton: max_backtrack must be <= 60");
    JFNK_REQUIRE(opts->central_below >= 0 && std::isfinite(opts->central_below), JFNK_E_ARG,
                 "newton: central_below must be finite and >= 0");
    check_opts(opts->gmres);
    const int S = mesh->n_seg();
    std::vector<int> inc(S);
    for (int k = 0; k < S; ++k) {
      inc[k] = n_increments ? n_increments[k] : opts->n_increments;
      JFNK_REQUIRE(inc[k] >= 1, JFNK_E_ARG, "newton: n_increments must be >= 1");
    }
    const hipStream_t caller = static_cast<hipStream_t>(stream);
    const hipStream_t s = solver_stream(mesh, caller, wants_graphs(mesh, opts->gmres));
    Carver c(d_work);
    FvWork fw;
    fw.carve(c, mesh);
    fw.zero_counters(s);
    KrylovWork kw;
    kw.carve(c, mesh, opts->gmres.restart, precond_work_floats(mesh, opts->gmres.precond),
             pc_z32(opts->gmres.precond));
    set_preconditioner_inertia(mesh, mesh->src.dt, s);
    const double ts = now_ms();
    precond_setup(mesh, opts->gmres.precond, s);
    const double setup = now_ms() - ts;
    std::vector<jfnk_stats> sv;
    std::vector<jfnk_status> stv;
    newton_solve(mesh, inc, *opts, d_u, fw, kw, s, sv, stv);
    join_stream(mesh, caller, s);
    for (int k = 0; k < S; ++k) {
      sv[k].t_ms[5] = setup;
      if (stats) stats[k] = sv[k];
      if (seg_status) seg_status[k] = stv[k];
      if (st == JFNK_OK && stv[k] != JFNK_OK) st = stv[k];
    }
    if (st == JFNK_E_NOT_CONVERGED) set_last_error("newton: iteration limit reached");
    if (st == JFNK_E_DIVERGED) set_last_error("newton: residual diverged");
    if (st == JFNK_E_NAN) set_last_error("newton: residual became NaN/Inf");
  });
  return g != JFNK_OK ? g : st;
}

}  // extern "C"

namespace jfnk {

void set_preconditioner_inertia(jfnk_mesh* m, double dt, hipStream_t s) {
  if (dt == m->pc_dt) return;
  const HostMesh& h = m->host;
  std::vector<double> diag(h.pc_diag.begin(), h.pc_diag.end());
  if (dt > 0) {
    // -9/4 rho Omega / dt^2 on the block diagonal (Section 3.1); the volumes
    // and densities come from the segments in union numbering
    for (const Segment& g : m->segs)
      for (int64_t c = 0; c < g.host.n_cells; ++c)
        diag[g.cell_off + c] -= 2.25 * g.mat.rho * g.host.vol[c] / (dt * dt);
  }
  const std::vector<double> dinv = jacobi_inverse(diag, h.pc_sym, h.dim);
  JFNK_HIP(hipMemcpyAsync(m->b_pc_dinv.p, dinv.data(), dinv.size() * sizeof(double), hipMemcpyHostToDevice, s));
  JFNK_HIP(hipStreamSynchronize(s));
  m->pc_diag_eff = dt > 0 ? std::move(diag) : std::vector<double>();
  for (AmgHierarchy** a : {&m->amg, &m->amg64})
    if (*a) {
      amg_destroy(*a);
      *a = nullptr;
    }
  m->pc_dt = dt;
}

}  // namespace jfnk

extern "C" {

jfnk_status jfnk_set_body_force(jfnk_mesh* mesh, const double* h_body, void* stream) {
  return guarded([&] {
    check_mesh(mesh);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (!h_body) {
      mesh->src.has_body = false;
      mesh->src.body.release();
      return;
    }
    for (int64_t i = 0; i < mesh->n_ext_cells * mesh->host.dim; ++i)
      JFNK_REQUIRE(std::isfinite(h_body[i]), JFNK_E_ARG, "set_body_force: value not finite");
    const size_t bytes = sizeof(double) * size_t(mesh->n_ext_cells) * mesh->host.dim;
    DevBuf tmp;
    tmp.alloc(bytes);
    JFNK_HIP(hipMemcpyAsync(tmp.p, h_body, bytes, hipMemcpyHostToDevice, s));
    mesh->src.body.alloc(sizeof(double) * size_t(mesh->dev.n_cells) * mesh->dev.dim);
    JFNK_HIP(hipMemsetAsync(mesh->src.body.p, 0, mesh->src.body.bytes, s));   // padding cells
    launch_permute(mesh->b_ext.as<int32_t>(), tmp.as<double>(), mesh->src.body.as<double>(), mesh->dev.n_cells,
                   mesh->dev.dim, true, s);
    JFNK_HIP(hipStreamSynchronize(s));
    mesh->src.has_body = true;
  });
}

jfnk_status jfnk_set_inertia(jfnk_mesh* mesh, double dt, const double* d_u_n, const double* d_u_nm1,
                             const double* d_v_n, const double* d_v_nm1, void* stream) {
  return guarded([&] {
    check_mesh(mesh);
    JFNK_REQUIRE(std::isfinite(dt), JFNK_E_ARG, "set_inertia: dt not finite");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (dt <= 0) {
      mesh->src.dt = 0;
      mesh->src.u_n = mesh->src.u_nm1 = mesh->src.v_n = mesh->src.v_nm1 = nullptr;
      set_preconditioner_inertia(mesh, 0.0, s);
      return;
    }
    check_ptr(d_u_n, "u_n");
    check_ptr(d_u_nm1, "u_nm1");
    check_ptr(d_v_n, "v_n");
    check_ptr(d_v_nm1, "v_nm1");
    bool any_mass = false;
    for (const Segment& g : mesh->segs) any_mass = any_mass || g.mat.rho > 0;
    JFNK_REQUIRE(any_mass, JFNK_E_ARG, "set_inertia: no mesh of the handle has a density rho > 0");
    mesh->src.dt = dt;
    mesh->src.u_n = d_u_n;
    mesh->src.u_nm1 = d_u_nm1;
    mesh->src.v_n = d_v_n;
    mesh->src.v_nm1 = d_v_nm1;
    set_preconditioner_inertia(mesh, dt, s);
  });
}

jfnk_status jfnk_dynamic_step(jfnk_mesh* mesh, double dt, int32_t predictor, const jfnk_newton_opts* opts,
                              double* d_u, double* d_u_prev, double* d_v, double* d_v_prev, double* d_a,
                              jfnk_stats* stats, void* d_work, void* stream) {
  jfnk_status st = JFNK_OK;
  jfnk_status g = guarded([&] {
    check_mesh(mesh);
    check_ptr(d_u, "u");
    check_ptr(d_u_prev, "u_prev");
    check_ptr(d_v, "v");
    check_ptr(d_v_prev, "v_prev");
    check_ptr(d_a, "a");
    check_work(d_work);
    JFNK_REQUIRE(dt > 0 && std::isfinite(dt), JFNK_E_ARG, "dynamic_step: dt must be positive");
    JFNK_REQUIRE(opts, JFNK_E_ARG, "dynamic_step: null options");
    JFNK_REQUIRE(opts->max_newton_it >= 1 && opts->eta > 0 && opts->rtol >= 0 && opts->atol >= 0 &&
                     opts->stol >= 0,
                 JFNK_E_ARG, "dynamic_step: bad Newton options");
    check_opts(opts->gmres);
    const hipStream_t caller = static_cast<hipStream_t>(stream);
    const hipStream_t s = solver_stream(mesh, caller, wants_graphs(mesh, opts->gmres));
    const int64_t n = int64_t(mesh->dev.n_cells) * mesh->dev.dim;
    Carver c(d_work);
    FvWork fw;
    fw.carve(c, mesh);
    fw.zero_counters(s);
    KrylovWork kw;
    kw.carve(c, mesh, opts->gmres.restart, precond_work_floats(mesh, opts->gmres.precond),
             pc_z32(opts->gmres.precond));
    double* un = c.take<double>(size_t(n));
    // u^t aside; the unknown starts from the predictor
    blas_lincomb(1.0, d_u, 0.0, d_u, un, n, s);
    launch_predict(n, dt, predictor != 0, un, d_v, d_a, d_u, s);
    mesh->src.dt = dt;
    mesh->src.u_n = un;
    mesh->src.u_nm1 = d_u_prev;
    mesh->src.v_n = d_v;
    mesh->src.v_nm1 = d_v_prev;
    struct Clear {
      jfnk_mesh* m;
      ~Clear() {
        m->src.dt = 0;
        m->src.u_n = m->src.u_nm1 = m->src.v_n = m->src.v_nm1 = nullptr;
      }
    } clear{mesh};
    set_preconditioner_inertia(mesh, dt, s);
    const double ts = now_ms();
    precond_setup(mesh, opts->gmres.precond, s);
    const double setup = now_ms() - ts;
    jfnk_newton_opts o = *opts;
    o.n_increments = 1;
    o.inc_begin = o.inc_end = 0;
    std::vector<jfnk_stats> sv;
    std::vector<jfnk_status> stv;
    newton_solve(mesh, std::vector<int>(mesh->n_seg(), 1), o, d_u, fw, kw, s, sv, stv);
    for (jfnk_status x : stv)
      if (st == JFNK_OK && x != JFNK_OK) st = x;
    // velocity, acceleration and the shift of the histories
    launch_bdf2_update(n, dt, d_u, un, d_u_prev, d_v, d_v_prev, d_a, s);
    join_stream(mesh, caller, s);
    for (int k = 0; k < mesh->n_seg(); ++k) {
      sv[k].t_ms[5] = setup;
      if (stats) stats[k] = sv[k];
    }
    if (st == JFNK_E_NOT_CONVERGED) set_last_error("dynamic_step: Newton iteration limit reached");
    if (st == JFNK_E_DIVERGED) set_last_error("dynamic_step: residual diverged");
    if (st == JFNK_E_NAN) set_last_error("dynamic_step: residual became NaN/Inf");
  });
  return g != JFNK_OK ? g : st;
}

jfnk_status jfnk_newton_solve(jfnk_mesh* mesh, const jfnk_newton_opts* opts, double* d_u,
                              jfnk_stats* stats, void* d_work, void* stream) {
  if (opts && opts->n_increments < 1) {
    set_last_error("newton: n_increments must be >= 1");
    return JFNK_E_ARG;
  }
  return newton_common(mesh, nullptr, opts, d_u, stats, nullptr, d_work, stream);
}

jfnk_status jfnk_newton_solve_batch(jfnk_mesh* mesh, const int32_t* n_increments,
                                    const jfnk_newton_opts* opts, double* d_u, jfnk_stats* stats,
                                    jfnk_status* seg_status, void* d_work, void* stream) {
  return newton_common(mesh, n_increments, opts, d_u, stats, seg_status, d_work, stream);
}

jfnk_status jfnk_segregated_solve(jfnk_mesh* mesh, const jfnk_segregated_opts* opts, double* d_u,
                                  jfnk_stats* stats, void* d_work, void* stream) {
  jfnk_status st = JFNK_OK;
  jfnk_status g = guarded([&] {
    check_mesh(mesh);
    check_ptr(d_u, "u");
    check_work(d_work);
    JFNK_REQUIRE(opts, JFNK_E_ARG, "segregated: null options");
    JFNK_REQUIRE(mesh->n_seg() == 1, JFNK_E_ARG, "segregated: single-mesh handles only");
    JFNK_REQUIRE(opts->n_increments >= 1 && opts->max_outer_it >= 1 && opts->max_inner_it >= 1, JFNK_E_ARG,
                 "segregated: n_increments, max_outer_it and max_inner_it must be >= 1");
    JFNK_REQUIRE(opts->rtol >= 0 && opts->atol >= 0 && opts->inner_rtol > 0 && opts->inner_rtol < 1,
                 JFNK_E_ARG, "segregated: bad tolerance");
    JFNK_REQUIRE(!pc_z32(opts->precond) && (opts->precond == JFNK_PC_JACOBI || amg_precond(opts->precond)),
                 JFNK_E_ARG, "segregated: precond must be JACOBI, AMG32 or AMG64");
    JFNK_REQUIRE(!amg_precond(opts->precond) || (opts->cheb_degree >= 1 && opts->cheb_degree <= 16), JFNK_E_ARG,
                 "segregated: cheb_degree must lie in [1, 16]");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    Carver c(d_work);
    FvWork fw;
    fw.carve(c, mesh);
    fw.zero_counters(s);
    KrylovWork kw;
    kw.carve(c, mesh, 1, precond_work_floats(mesh, opts->precond));
    set_preconditioner_inertia(mesh, mesh->src.dt, s);
    jfnk_stats sv{};
    segregated_solve(mesh, *opts, d_u, fw, kw, s, sv, st);
    if (stats) *stats = sv;
    if (st == JFNK_E_NOT_CONVERGED) set_last_error("segregated: outer iteration limit reached");
    if (st == JFNK_E_NAN) set_last_error("segregated: residual became NaN/Inf");
  });
  return g != JFNK_OK ? g : st;
}

}  // extern "C"
