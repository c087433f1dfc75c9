// aao_solve_no_alloc: aao_solve for callers that cannot allocate device
// memory.  The handle's workspace is placed in a file-scope device array
// (`scratch`, AAO_NO_ALLOC_SCRATCH_BYTES) that the library holds on every
// device it runs on until the process ends.  Calls on one device share that
// array and keep no state in it between calls: the constant tables are copied
// in and the counters cleared at the start of every call, so calls that
// overlap in time on one device race (they must be serialised by the caller).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "aao_internal.h"

namespace {

__device__ __align__(256) char scratch[AAO_NO_ALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};   // device address of `scratch`, per device

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current).  In host code the array's name is only
// a stand-in for the symbol; the address comes from hipGetSymbolAddress.
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int aao_solve_no_alloc(aao_problem* h, const double* rhs, double* x, aao_stats* st) {
  if (!h) return AAO_INVALID_ARG;
  if (!rhs || !x || rhs == x) {
    h->err = "rhs, x must be distinct device pointers";
    return AAO_INVALID_ARG;
  }
  if (h->ws_need > (size_t)AAO_NO_ALLOC_SCRATCH_BYTES) {
    h->err = "the workspace of this problem (" + std::to_string(h->ws_need) +
             " bytes) exceeds the static scratch of " + std::to_string((size_t)AAO_NO_ALLOC_SCRATCH_BYTES) +
             " bytes";
    return AAO_WORKSPACE_TOO_SMALL;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return aao::status_from_hip(h, e, "solve_no_alloc");
  if (dev < 0 || dev >= MAX_DEVICES) {
    h->err = "device index out of range";
    return AAO_INVALID_ARG;
  }
  void* ptr = nullptr;
  e = scratch_address(dev, &ptr);
  if (e != hipSuccess) return aao::status_from_hip(h, e, "scratch address");
  // run the ordinary solve in the scratch memory, then give the handle its
  // own workspace back (its graphs, which point there, stay valid)
  char* saved_ws = h->ws;
  const size_t saved_bytes = h->ws_bytes;
  h->ws = static_cast<char*>(ptr);
  h->ws_bytes = (size_t)AAO_NO_ALLOC_SCRATCH_BYTES;
  h->no_alloc = true;
  h->lds_budget = aao::mg_configure_lds();
  int rc;
  e = aao::upload_tables(h);
  if (e != hipSuccess) rc = aao::status_from_hip(h, e, "scratch upload");
  else rc = aao::solve(h, rhs, x, st, false);
  h->no_alloc = false;
  h->ws = saved_ws;
  h->ws_bytes = saved_bytes;
  return rc;
}
