// mgwr_solve_static: mgwr_solve with the library's own file-scope device
// array as the plan's workspace, for callers that cannot allocate device
// memory (code under graph capture, tight serving loops).  Nothing here
// allocates: the array is part of the library's code object, and each device
// the library runs on holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "mgwr.h"
#include "plan_internal.h"

namespace mgwr {
void set_last_error(const std::string& msg);
}

namespace {

constexpr size_t kStaticBytes = MGWR_STATIC_WORKSPACE_BYTES;

// The workspace.  In host code this name is only a stand-in for the symbol:
// its device address comes from hipGetSymbolAddress (per device) and is the
// only form ever passed to the device.
__device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `dev`, looked up once per device with that
// device current (the caller's).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    mgwr::set_last_error("device ordinal beyond the static workspace table");
    return MGWR_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      mgwr::set_last_error(std::string("hipGetSymbolAddress(static workspace): ") + hipGetErrorString(e));
      return MGWR_ERR_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return MGWR_OK;
}

}  // namespace

extern "C" int mgwr_solve_static(mgwr_plan* plan, void* stream, const double* f_dev, const double* g_dev,
                                 double tol, double* u_dev, unsigned flags, mgwr_stats* stats) {
  if (!plan) {
    mgwr::set_last_error("null plan");
    return MGWR_ERR_INVALID_ARG;
  }
  if (flags & MGWR_WARM_START) {
    mgwr::set_last_error("mgwr_solve_static takes no warm start (the network's buffers are not in the static workspace)");
    return MGWR_ERR_INVALID_ARG;
  }
  const size_t need = mgwr::plan_workspace_bytes(plan);
  if (need > kStaticBytes) {
    mgwr::set_last_error("the plan needs " + std::to_string(need) + " bytes of workspace; the static workspace holds " +
                         std::to_string(kStaticBytes));
    return MGWR_ERR_INVALID_ARG;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    mgwr::set_last_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return MGWR_ERR_HIP;
  }
  void* ws = nullptr;
  int rc = scratch_address(dev, &ws);
  if (rc) return rc;
  const mgwr::PlanBinding saved = mgwr::plan_binding(plan);
  // bind to the array (uploads the packed H-matrix; every array a solve
  // reads before writing it, counters and flags included, is initialised by
  // the solve itself), solve, and point the plan back at its own binding
  rc = mgwr_plan_bind(plan, ws, kStaticBytes, stream);
  if (rc == MGWR_OK) {
    mgwr::detach_network(plan);
    rc = mgwr_solve(plan, f_dev, g_dev, tol, u_dev, flags, stats);
    e = hipStreamSynchronize((hipStream_t)stream);
    if (rc == MGWR_OK && e != hipSuccess) {
      mgwr::set_last_error(std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
      rc = MGWR_ERR_HIP;
    }
  }
  mgwr::restore_binding(plan, saved);
  return rc;
}
