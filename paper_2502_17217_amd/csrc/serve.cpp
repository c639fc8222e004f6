// Request server: continuous admission of solves onto concurrent HIP streams
// with device-memory (HBM) admission control.  See the serving section of
// include/jfnk.h for the contract.
//
// Scheduling: requests wait in a FIFO queue.  Each worker owns a stream and
// a pinned host buffer; it takes the next request, does the host-only mesh
// preprocessing (no device memory), computes the exact device footprint of
// the solve, then waits for a reservation of that many bytes from the
// budget; reservations are granted strictly in the order they were asked
// for, so a large request is not starved by smaller ones behind it.  The
// device arrays are allocated and freed stream-ordered on the worker's
// stream, so no request waits for the work of another one.
#include <algorithm>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "solver.h"

namespace jfnk {

namespace {

double clock_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Owning copy of a jfnk_mesh_desc and its arrays.
struct DescCopy {
  std::vector<double> points;
  std::vector<int64_t> face_ptr;
  std::vector<int32_t> face_pts, owner, neighbour;
  std::vector<jfnk_patch> patches;
  std::vector<std::vector<double>> per_face;
  jfnk_mesh_desc d{};
  void copy(const jfnk_mesh_desc& s) {
    JFNK_REQUIRE(s.points && s.face_ptr && s.face_pts && s.owner && s.n_faces >= 0 && s.n_points >= 0 &&
                     (s.dim == 2 || s.dim == 3),
                 JFNK_E_ARG, "submit: invalid mesh description");
    points.assign(s.points, s.points + s.n_points * s.dim);
    face_ptr.assign(s.face_ptr, s.face_ptr + s.n_faces + 1);
    face_pts.assign(s.face_pts, s.face_pts + face_ptr.back());
    owner.assign(s.owner, s.owner + s.n_faces);
    if (s.n_internal > 0) neighbour.assign(s.neighbour, s.neighbour + s.n_internal);
    patches.assign(s.patches, s.patches + s.n_patches);
    per_face.resize(s.n_patches);
    for (int32_t p = 0; p < s.n_patches; ++p) {
      if (patches[p].per_face) {
        per_face[p].assign(patches[p].per_face, patches[p].per_face + patches[p].size * s.dim);
        patches[p].per_face = per_face[p].data();
      }
    }
    d = s;
    d.points = points.data();
    d.face_ptr = face_ptr.data();
    d.face_pts = face_pts.data();
    d.owner = owner.data();
    d.neighbour = neighbour.empty() ? nullptr : neighbour.data();
    d.patches = patches.empty() ? nullptr : patches.data();
  }
};

struct Request {
  uint64_t id = 0;
  DescCopy desc;
  jfnk_material mat{};
  jfnk_newton_opts opts{};
  double* u_out = nullptr;
  jfnk_request_info info{};
};

}  // namespace
}  // namespace jfnk

struct jfnk_server {
  jfnk_server_opts opts{};
  int device = 0;
  double t0 = 0;
  std::mutex mu;
  std::condition_variable cv_queue, cv_budget, cv_done;
  std::deque<jfnk::Request*> queue;
  std::map<uint64_t, std::unique_ptr<jfnk::Request>> all;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next_id = 1;
  size_t in_use = 0, peak = 0;
  uint64_t budget_next = 0, budget_serving = 0;   // FIFO tickets for reservations
  int64_t submitted = 0, completed = 0, rejected = 0, running = 0, cancelled = 0;
  double first_submit = -1, last_done = -1;
  std::vector<double> latencies;
};

namespace jfnk {

namespace {

// Wait for reservation turn `ticket`; then take `foot` bytes (waiting until
// they fit) or, with foot == 0, just pass the turn on.
// Waits for this ticket's turn and for foot bytes of budget; returns the
// server clock at the grant (taken under the lock, so grant times follow
// the ticket order).
double take_turn(jfnk_server* S, uint64_t ticket, size_t foot) {
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_budget.wait(lk, [&] { return S->budget_serving == ticket && S->in_use + foot <= S->opts.hbm_budget; });
  S->in_use += foot;
  S->peak = std::max(S->peak, S->in_use);
  S->budget_serving++;
  const double t = clock_ms() - S->t0;
  S->cv_budget.notify_all();
  return t;
}

void run_request(jfnk_server* S, Request* r, uint64_t ticket, hipStream_t stream, double* pinned,
                 size_t pinned_doubles) {
  jfnk_request_info& info = r->info;
  // host preprocessing (no device memory yet)
  auto m = std::make_unique<jfnk_mesh>();
  m->segs.resize(1);
  try {
    m->segs[0].mat = make_material(r->mat);
    build_host_mesh(r->desc.d, m->segs[0].mat, m->segs[0].host);
  } catch (...) {
    take_turn(S, ticket, 0);
    throw;
  }
  const HostMesh& h = m->segs[0].host;
  info.n_cells = h.n_cells;
  const jfnk_newton_opts& o = r->opts;
  const size_t pcf = precond_work_floats(h.n_cells, h.dim, o.gmres.precond);
  // AMG matrices: an estimate (about 60 B per fine row in FP32 on the meshes
  // measured, with margin); the hierarchy's actual bytes are checked after
  // its setup and any excess is added to the reservation
  const size_t amg_mats = amg_precond(o.gmres.precond)
                              ? size_t(h.n_cells) * (pc_kind(o.gmres.precond) == JFNK_PC_AMG64 ? 512 : 256)
                              : 0;
  const bool z32 = pc_z32(o.gmres.precond);
  const size_t foot = device_bytes_of(h) + solve_workspace_bytes(h.n_cells, h.dim, 1, o.gmres.restart, pcf, z32) +
                      amg_mats + size_t(h.n_cells) * h.dim * 16 + (size_t(1) << 20);
  info.footprint_bytes = int64_t(foot);
  if (foot > S->opts.hbm_budget) {
    take_turn(S, ticket, 0);
    throw Error{JFNK_E_OOM, "request footprint " + std::to_string(foot) + " exceeds the server's HBM budget"};
  }
  // reservation in request order
  const double t_grant = take_turn(S, ticket, foot);
  struct Release {
    jfnk_server* S;
    size_t foot;
    ~Release() {
      std::lock_guard<std::mutex> lk(S->mu);
      S->in_use -= foot;
      S->cv_budget.notify_all();
    }
  } release{S, foot};
  info.t_start_ms = t_grant;
  info.state = 1;
  if (S->opts.dry_run_us_per_kcell > 0) {
    std::this_thread::sleep_for(std::chrono::microseconds(
        int64_t(S->opts.dry_run_us_per_kcell * double(h.n_cells) / 1000.0)));
    if (r->u_out) std::fill(r->u_out, r->u_out + h.n_cells * h.dim, 0.0);
    info.status = JFNK_OK;
    return;
  }
  AllocContext& ac = alloc_context();
  ac.stream = stream;
  ac.pinned = pinned;
  ac.pinned_doubles = pinned_doubles;
  struct CtxReset {
    ~CtxReset() { alloc_context() = AllocContext(); }
  } ctx_reset;
  finish_handle(*m, stream, clock_ms());
  DevBuf work, u, ue;
  const size_t wbytes = solve_workspace_bytes(h.n_cells, h.dim, 1, o.gmres.restart, pcf, z32);
  work.alloc(wbytes);
  u.alloc(sizeof(double) * h.n_cells * h.dim);
  ue.alloc(sizeof(double) * h.n_cells * h.dim);
  JFNK_HIP(hipMemsetAsync(u.p, 0, u.bytes, stream));
  Carver c(work.p);
  FvWork fw;
  fw.carve(c, m.get());
  fw.zero_counters(stream);
  KrylovWork kw;
  kw.carve(c, m.get(), o.gmres.restart, pcf, z32);
  precond_setup(m.get(), o.gmres.precond, stream);
  const size_t amg_real = amg_device_bytes(m->amg) + amg_device_bytes(m->amg64);
  if (amg_real > amg_mats) {
    // the estimate was short: account for the excess (the hierarchy already
    // exists, so the budget may be exceeded by it until this request ends)
    const size_t extra = amg_real - amg_mats;
    std::lock_guard<std::mutex> lk(S->mu);
    S->in_use += extra;
    S->peak = std::max(S->peak, S->in_use);
    release.foot += extra;
    info.footprint_bytes += int64_t(extra);
  }
  std::vector<jfnk_stats> st;
  std::vector<jfnk_status> ss;
  newton_solve(m.get(), std::vector<int>(1, std::max(1, o.n_increments)), o, u.as<double>(), fw, kw, stream,
               st, ss);
  info.stats = st[0];
  info.status = ss[0];
  launch_permute(m->b_ext.as<int32_t>(), u.as<double>(), ue.as<double>(), h.n_cells, h.dim, false, stream);
  if (r->u_out)
    JFNK_HIP(hipMemcpyAsync(r->u_out, ue.p, ue.bytes, hipMemcpyDeviceToHost, stream));
  // free the device arrays stream-ordered, then wait for this stream only
  work.release();
  u.release();
  ue.release();
  for (AmgHierarchy** a : {&m->amg, &m->amg64})
    if (*a) {
      amg_destroy(*a);
      *a = nullptr;
    }
  m.reset();
  JFNK_HIP(hipStreamSynchronize(stream));
}

void worker_loop(jfnk_server* S) {
  hipStream_t stream = nullptr;
  double* pinned = nullptr;
  const size_t pinned_doubles = size_t(4 * kMaxBasis + 8) + 64;
  const bool gpu = S->opts.dry_run_us_per_kcell <= 0;
  if (gpu) {
    (void)hipSetDevice(S->device);
    std::shared_lock<std::shared_mutex> lk(capture_mutex());
    (void)hipStreamCreate(&stream);  // default priority
    (void)hipHostMalloc(reinterpret_cast<void**>(&pinned), sizeof(double) * pinned_doubles, hipHostMallocDefault);
  }
  while (true) {
    Request* r = nullptr;
    uint64_t ticket = 0;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_queue.wait(lk, [&] { return S->stop || !S->queue.empty(); });
      if (S->queue.empty()) break;  // stop requested and nothing left
      r = S->queue.front();
      S->queue.pop_front();
      S->running++;
      ticket = S->budget_next++;   // reservations are granted in dequeue (= arrival) order
    }
    try {
      if (gpu && (!stream || !pinned)) {
        take_turn(S, ticket, 0);
        throw Error{JFNK_E_HIP, "server worker could not create its stream"};
      }
      run_request(S, r, ticket, stream, pinned, pinned_doubles);
    } catch (const Error& e) {
      r->info.status = e.status;
      std::snprintf(r->info.error, sizeof(r->info.error), "%s", e.msg.c_str());
    } catch (const std::exception& e) {
      r->info.status = JFNK_E_ARG;
      std::snprintf(r->info.error, sizeof(r->info.error), "%s", e.what());
    } catch (...) {
      r->info.status = JFNK_E_ARG;
      std::snprintf(r->info.error, sizeof(r->info.error), "unknown failure");
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      r->info.t_done_ms = clock_ms() - S->t0;
      r->info.latency_ms = r->info.t_done_ms - r->info.t_submit_ms;
      r->info.state = 2;
      S->running--;
      if (r->info.status == JFNK_OK || r->info.status == JFNK_E_NOT_CONVERGED) {
        S->completed++;
        S->latencies.push_back(r->info.latency_ms);
        S->last_done = std::max(S->last_done, r->info.t_done_ms);
      } else {
        S->rejected++;
      }
    }
    S->cv_done.notify_all();
  }
  std::shared_lock<std::shared_mutex> lk(capture_mutex());
  if (stream) (void)hipStreamDestroy(stream);
  if (pinned) (void)hipHostFree(pinned);
}

}  // namespace
}  // namespace jfnk

using namespace jfnk;

namespace {
template <class F>
jfnk_status srv_guard(F&& f) {
  try {
    f();
    return JFNK_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return JFNK_E_OOM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return JFNK_E_ARG;
  }
}
}  // namespace

extern "C" {

jfnk_status jfnk_server_create(const jfnk_server_opts* opts, jfnk_server** out) {
  return srv_guard([&] {
    JFNK_REQUIRE(opts && out, JFNK_E_ARG, "server_create: null argument");
    JFNK_REQUIRE(opts->max_slots >= 1 && opts->max_slots <= 64, JFNK_E_ARG, "server: max_slots in [1, 64]");
    JFNK_REQUIRE(opts->max_queue >= 1, JFNK_E_ARG, "server: max_queue >= 1");
    JFNK_REQUIRE(opts->hbm_budget > 0, JFNK_E_ARG, "server: hbm_budget > 0");
    auto S = std::make_unique<jfnk_server>();
    S->opts = *opts;
    S->t0 = clock_ms();
    if (opts->dry_run_us_per_kcell <= 0) JFNK_HIP(hipGetDevice(&S->device));
    for (int i = 0; i < opts->max_slots; ++i) S->workers.emplace_back(worker_loop, S.get());
    *out = S.release();
  });
}

jfnk_status jfnk_server_submit(jfnk_server* S, const jfnk_mesh_desc* desc, const jfnk_material* mat,
                               const jfnk_newton_opts* opts, double* u_out, uint64_t* ticket) {
  return srv_guard([&] {
    JFNK_REQUIRE(S && desc && mat && opts && ticket, JFNK_E_ARG, "server_submit: null argument");
    JFNK_REQUIRE(opts->gmres.restart >= 1 && opts->gmres.restart < kMaxBasis && opts->n_increments >= 1 &&
                     opts->max_newton_it >= 1 && opts->eta > 0,
                 JFNK_E_ARG, "server_submit: bad options");
    {
      // a full queue refuses at once, before the description is copied
      std::lock_guard<std::mutex> lk(S->mu);
      JFNK_REQUIRE(int64_t(S->queue.size()) < S->opts.max_queue, JFNK_E_BUSY, "server_submit: queue full");
    }
    auto r = std::make_unique<Request>();
    r->desc.copy(*desc);
    r->mat = *mat;
    r->opts = *opts;
    r->u_out = u_out;
    std::lock_guard<std::mutex> lk(S->mu);
    JFNK_REQUIRE(!S->stop, JFNK_E_ARG, "server_submit: server is stopping");
    JFNK_REQUIRE(int64_t(S->queue.size()) < S->opts.max_queue, JFNK_E_BUSY, "server_submit: queue full");
    r->id = S->next_id++;
    r->info.state = 0;
    r->info.status = JFNK_OK;
    r->info.t_submit_ms = clock_ms() - S->t0;
    if (S->first_submit < 0) S->first_submit = r->info.t_submit_ms;
    *ticket = r->id;
    S->queue.push_back(r.get());
    S->all[r->id] = std::move(r);
    S->submitted++;
    S->cv_queue.notify_one();
  });
}

jfnk_status jfnk_server_poll(jfnk_server* S, uint64_t ticket, jfnk_request_info* info) {
  return srv_guard([&] {
    JFNK_REQUIRE(S && info, JFNK_E_ARG, "server_poll: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    JFNK_REQUIRE(it != S->all.end(), JFNK_E_ARG, "server_poll: unknown ticket");
    *info = it->second->info;
  });
}

jfnk_status jfnk_server_wait(jfnk_server* S, uint64_t ticket, jfnk_request_info* info) {
  return srv_guard([&] {
    JFNK_REQUIRE(S, JFNK_E_ARG, "server_wait: null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    JFNK_REQUIRE(it != S->all.end(), JFNK_E_ARG, "server_wait: unknown ticket");
    Request* r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->info.state == 2; });
    if (info) *info = r->info;
  });
}

jfnk_status jfnk_server_metrics_get(jfnk_server* S, jfnk_server_metrics* m) {
  return srv_guard([&] {
    JFNK_REQUIRE(S && m, JFNK_E_ARG, "server_metrics: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(m, 0, sizeof(*m));
    m->submitted = S->submitted;
    m->completed = S->completed;
    m->rejected = S->rejected;
    m->running = S->running;
    m->queued = int64_t(S->queue.size());
    m->cancelled = S->cancelled;
    m->hbm_in_use = int64_t(S->in_use);
    m->hbm_peak = int64_t(S->peak);
    std::vector<double> l = S->latencies;
    if (!l.empty()) {
      std::sort(l.begin(), l.end());
      auto pct = [&](double q) {
        const size_t i = size_t(std::ceil(q * double(l.size()))) - 1;
        return l[std::min(i, l.size() - 1)];
      };
      m->p50_ms = pct(0.50);
      m->p99_ms = pct(0.99);
      m->max_ms = l.back();
      double sum = 0;
      for (double x : l) sum += x;
      m->mean_ms = sum / double(l.size());
      const double span = S->last_done - S->first_submit;
      m->solves_per_s = span > 0 ? 1000.0 * double(S->completed) / span : 0.0;
    }
  });
}

jfnk_status jfnk_server_cancel_queued(jfnk_server* S, int64_t* n_cancelled) {
  return srv_guard([&] {
    JFNK_REQUIRE(S, JFNK_E_ARG, "server_cancel_queued: null server");
    int64_t n = 0;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const double t = clock_ms() - S->t0;
      for (Request* r : S->queue) {
        r->info.status = JFNK_E_BUSY;
        r->info.state = 2;
        r->info.t_done_ms = t;
        r->info.latency_ms = t - r->info.t_submit_ms;
        std::snprintf(r->info.error, sizeof(r->info.error), "cancelled before it started");
        ++n;
      }
      S->queue.clear();
      S->cancelled += n;
    }
    S->cv_done.notify_all();
    if (n_cancelled) *n_cancelled = n;
  });
}

jfnk_status jfnk_server_destroy(jfnk_server* S) {
  return srv_guard([&] {
    if (!S) return;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv_queue.notify_all();
    for (std::thread& t : S->workers) t.join();
    delete S;
  });
}

}  // extern "C"
