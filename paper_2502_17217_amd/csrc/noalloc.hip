// J v without any device allocation: jfnk_jv_noalloc.  For callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid it).  The per-call scratch of jfnk_jv (tile
// partial sums of the step size, per-segment eps, arrival counters, and the
// per-cell gradient record when the mesh does not run the fused single pass)
// lives in one file-scope device array of fixed size instead of a caller
// workspace; each GPU holds its own copy until the process ends.
#include <array>
#include <cmath>
#include <mutex>

#include "solver.h"

namespace jfnk {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

// The array itself.  Host code never uses this name as an address (on the
// host it is only a stand-in for the symbol): every use goes through the
// device address returned by hipGetSymbolAddress for the current device.
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
std::array<void*, kMaxDevices> g_ptr{};

// Device address of the current device's scratch array, looked up once per
// device with that device current.
void* scratch_ptr() {
  int dev = -1;
  JFNK_HIP(hipGetDevice(&dev));
  JFNK_REQUIRE(dev >= 0 && dev < kMaxDevices, JFNK_E_ARG, "jv_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[size_t(dev)] == nullptr) {
    void* p = nullptr;
    JFNK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    JFNK_REQUIRE(p != nullptr, JFNK_E_HIP, "jv_noalloc: no device address for the scratch array");
    g_ptr[size_t(dev)] = p;
  }
  return g_ptr[size_t(dev)];
}

// Regions of one call, carved from base (or only measured when base is null):
// the step-size partials need columns 0 and 1 of the tile partial layout.
size_t carve(Carver& c, const jfnk_mesh* m, bool need_ru, FvWork& fw) {
  const int64_t n = m->host.n_cells;
  const int dim = m->host.dim;
  const int S = m->n_seg();
  fw.S = S;
  fw.grad = m->dev.lds_kernels == 2 ? nullptr : c.take<double>(size_t(n) * rec_doubles(dim));
  fw.ru = need_ru ? c.take<double>(size_t(n) * dim) : nullptr;
  fw.partials = c.take<double>(size_t(2) * size_t(n_tiles(n)));
  fw.eps = c.take<double>(S);
  fw.load = c.take<double>(S);
  fw.tickets = c.take<int32_t>(size_t(2) * S + 8);
  return c.off;
}

}  // namespace

}  // namespace jfnk

using namespace jfnk;

extern "C" jfnk_status jfnk_jv_noalloc(jfnk_mesh* mesh, double load, const double* d_u, const double* d_Ru,
                                       const double* d_v, double eps, double* d_Jv, void* stream) {
  try {
    JFNK_REQUIRE(mesh != nullptr, JFNK_E_ARG, "null mesh handle");
    JFNK_REQUIRE(d_u && d_v && d_Jv, JFNK_E_ARG, "jv_noalloc: null device pointer");
    JFNK_REQUIRE(d_Jv != d_u && d_Jv != d_v && d_Jv != d_Ru, JFNK_E_ARG, "jv_noalloc: output aliases an input");
    JFNK_REQUIRE(std::isfinite(eps) && std::isfinite(load), JFNK_E_ARG, "jv_noalloc: eps/load not finite");
    JFNK_REQUIRE(!mesh->prof.on, JFNK_E_ARG, "jv_noalloc: kernel profiling is enabled on this mesh");
    FvWork fw;
    Carver measure(nullptr);
    const size_t need = carve(measure, mesh, d_Ru == nullptr, fw);
    JFNK_REQUIRE(need <= kScratchBytes, JFNK_E_ARG,
                 "jv_noalloc: this mesh needs " + std::to_string(need) + " bytes of scratch, more than the " +
                     std::to_string(kScratchBytes) + "-byte limit (pass R(u), or use jfnk_jv with a workspace)");
    Carver c(scratch_ptr());
    carve(c, mesh, d_Ru == nullptr, fw);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // the arrival counters must start at zero (a fill kernel, no memset node)
    fw.setup_uniform(s, load, mesh->any_small);
    const double* Ru = d_Ru;
    if (!Ru) {
      residual_into(mesh, d_u, fw.ru, fw, nullptr, s);
      Ru = fw.ru;
    }
    jv_into(mesh, d_u, Ru, d_v, eps, d_Jv, fw, nullptr, s);
    return JFNK_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return JFNK_E_ARG;
  }
}
