// pf_solve_noalloc: the LU Newton solve of pf_solve (Sec. II-A / II-B
// iteration tables, Sec. III-A inner solve) for callers that cannot allocate.
//
// Everything the solve needs beyond the case's resident storage lives in one
// file-scope device array, `pfn::scratch`, of kScratchBytes per device: the
// instance table and work items of the launch plan, the Newton-state gather,
// and the case's working storage (factor values, the dense block with its
// inverses and flags).  Host code never passes the array's name (a host-side
// stand-in) to a kernel or a copy: the device address, taken once per device
// with hipGetSymbolAddress when a context is created on it, is used instead.
// Calls on one device are serialised by a per-device lock, since they share
// the array; it keeps the last call's contents, and what must start at zero
// (the dense block's flags) is cleared by a fill kernel at every call.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace pfi {
pf_status start_batch(Batch* b, const pf_options* opt);  // newton.cpp
pf_status step_batch(Batch* b, const pf_options* opt);   // newton.cpp
}  // namespace pfi

using namespace pfi;

namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

// File-scope device array with external linkage: the code-object loader
// resolves device variables by name among global symbols only, so an
// internal-linkage (static) array would be invisible to hipGetSymbolAddress
// (the runtime stops the process when a registered variable cannot be
// found).  No device code names it; `used` keeps it in the code object.
namespace pfn {
__device__ __align__(256) __attribute__((used)) char scratch[kScratchBytes];
}  // namespace pfn

namespace {

std::mutex g_mu;                    // guards g_ptr and g_err
void* g_ptr[kMaxDevices] = {};      // device address of `scratch` per device
hipError_t g_err[kMaxDevices] = {}; // a failed lookup, reported by the solve
std::mutex g_dev_mu[kMaxDevices];   // one solve at a time per device

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace pfi {

// The device address of `scratch` on `device` (the device must be current).
pf_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("pf_ctx_create: device index out of range for the scratch table");
    return PF_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return PF_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(pfn::scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    g_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    return PF_E_DEVICE;
  }
  g_ptr[device] = p;
  return PF_OK;
}

}  // namespace pfi

extern "C" {

pf_status pf_solve_noalloc(pf_case* c, const pf_options* opt, pf_result* res, size_t* scratch_used) {
  if (!c || !res) {
    set_error("pf_solve_noalloc: NULL argument");
    return PF_E_INVALID;
  }
  if (c->busy.load()) {
    set_error("pf_solve_noalloc: case is queued or running");
    return PF_E_BUSY;
  }
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  pf_status st = check_opts(&o);
  if (st != PF_OK) return st;
  if (o.solver != PF_SOLVER_LU) {
    set_error("pf_solve_noalloc: only the LU inner solve runs without allocation");
    return PF_E_INVALID;
  }
  Ctx* ctx = c->ctx;
  const int dev = ctx->device;
  void* base = nullptr;
  hipError_t why = hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev >= 0 && dev < kMaxDevices) {
      base = g_ptr[dev];
      why = g_err[dev];
    }
  }
  if (!base) {
    set_error(std::string("pf_solve_noalloc: no scratch address for this device (") +
              (why != hipSuccess ? hipGetErrorName(why) : "no context was created on it") + ")");
    return PF_E_DEVICE;
  }
  std::lock_guard<std::mutex> dlk(g_dev_mu[dev]);
  std::lock_guard<std::mutex> lk(ctx->launch_mu);
  const auto t0 = std::chrono::steady_clock::now();
  std::memset(res, 0, sizeof *res);
  // plan on the host, then the layout in scratch: instance table and work
  // items | Newton-state gather | working storage
  Batch b;
  std::vector<int2> work;
  b.plan(ctx, {c}, &work);
  const size_t b_plan = al(b.plan_bytes(work.size()));
  const size_t b_red = al(sizeof(pfd::Red));
  const size_t need = b_plan + b_red + al(c->wbytes);
  if (scratch_used) *scratch_used = need;
  if (need > kScratchBytes) {
    set_error("pf_solve_noalloc: the case needs " + std::to_string(need) + " bytes of scratch, more than the " +
              std::to_string(kScratchBytes) + " the library holds per device");
    return PF_E_INVALID;
  }
  char* p = (char*)base;
  pfd::Red* d_red = (pfd::Red*)(p + b_plan);
  char* wmem = p + b_plan + b_red;
  if (!b.place(p, work)) {
    set_error("pf_solve_noalloc: upload of the launch plan failed");
    return PF_E_DEVICE;
  }
  // the case's own working storage (if any) steps aside for the call
  char* own = c->wown ? c->wbase : nullptr;
  attach_work(c, wmem, false, b.stream);
  ctx->prof_off = true;
  hipStream_t s = b.stream;
  st = start_batch(&b, &o);
  pfd::Red red;
  std::memset(&red, 0, sizeof red);
  for (int guard = 0; st == PF_OK && guard <= o.max_iter + 1; ++guard) {
    pfd::launch_gather_red(s, b.d_insts, 1, d_red);
    if (hipMemcpyAsync(&red, d_red, sizeof red, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("pf_solve_noalloc: device failure during the Newton iteration");
      st = PF_E_DEVICE;
      break;
    }
    if (red.timeout) {
      set_error("pf_solve_noalloc: an inter-work-group wait on the device timed out");
      st = PF_E_DEVICE;
      break;
    }
    if (!red.active) break;
    st = step_batch(&b, &o);
  }
  ctx->prof_off = false;
  (void)hipStreamSynchronize(s);
  // give the case back its own storage, or none
  c->wbase = nullptr;
  c->wown = false;
  if (own)
    attach_work(c, own, true, s);
  else
    detach_work(c);
  (void)hipStreamSynchronize(s);
  if (st != PF_OK) return st;
  res->status = red.status;
  res->iters = red.it;
  res->mismatch_inf = red.last_norm;
  res->max_step = red.last_step;
  res->device_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return PF_OK;
}

}  // extern "C"
