// Allocation-free solve of libmgrit (mgrit_solve_static): the plan of
// mgrit_plan_create is built with every device array carved from one static
// per-device workspace, solved with mgrit_solve and released, so the call
// allocates no device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mgrit.h"
#include "plan.h"

namespace mgr {
namespace {

// The workspace.  In host code `scratch` names a host-side stand-in: only
// the device address from hipGetSymbolAddress may be handed to kernels or
// copies.
__device__ __align__(256) unsigned char scratch[MGRIT_STATIC_BYTES];

constexpr int kMaxDevices = 64;

struct DeviceSlot {
  std::once_flag once;
  int rc = MGRIT_EHIP;
  char* ptr = nullptr;  // device address of `scratch` on this device
  std::mutex busy;      // one call at a time per device
};
DeviceSlot g_slot[kMaxDevices];

// Resolve the device address of the workspace once per device, with that
// device current.
int workspace(int dev, char** out) {
  DeviceSlot& s = g_slot[dev];
  std::call_once(s.once, [&s] {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) {
      s.ptr = static_cast<char*>(p);
      s.rc = MGRIT_OK;
    } else {
      (void)hipGetLastError();
      s.rc = MGRIT_EHIP;
    }
  });
  *out = s.ptr;
  return s.rc;
}

struct ArenaScope {
  explicit ArenaScope(Arena* a) { set_thread_arena(a); }
  ~ArenaScope() { set_thread_arena(nullptr); }
};

}  // namespace
}  // namespace mgr

using namespace mgr;

extern "C" int mgrit_solve_static(int nx, int nt, double alpha, double cfl, int scheme, int m,
                                  int levels, const mgrit_taps* psi, int cycle, int relax,
                                  int precision, void* hip_stream, const double* u0,
                                  const double* uinit, double tol, int maxit, double* u_out,
                                  int out_kind, double* hist, int* iters) {
  // the argument checks of mgrit_solve, before anything is built
  if (!u0 || maxit < 0 || !(tol >= 0.0)) return MGRIT_EINVAL;
  if (out_kind < MGRIT_OUT_NONE || out_kind > MGRIT_OUT_ALL) return MGRIT_EINVAL;
  if (out_kind != MGRIT_OUT_NONE && !u_out) return MGRIT_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MGRIT_ENODEV;
  char* base = nullptr;
  int rc = workspace(dev, &base);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_slot[dev].busy);
  Arena arena;
  arena.base = base;
  arena.cap = MGRIT_STATIC_BYTES;
  ArenaScope scope(&arena);
  mgrit_plan_t plan = nullptr;
  rc = mgrit_plan_create(&plan, nx, nt, alpha, cfl, scheme, m, levels, psi, cycle, relax,
                         precision, hip_stream);
  if (rc) return arena.overflow ? MGRIT_ESCRATCH : rc;
  rc = mgrit_solve(plan, u0, uinit, tol, maxit, u_out, out_kind, hist, iters);
  mgrit_destroy(plan);  // waits for the stream; frees nothing of the workspace
  return rc;
}
