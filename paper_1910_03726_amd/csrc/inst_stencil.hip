// One shard of k_stencil instantiations: FP64 or FP32 (MGR_PREC 0/1) for one
// chunk length MGR_K and every window width of MGR_STENCIL_WIDTHS.
#include "registry.h"
#include "relax_kernels.h"

#ifndef MGR_PREC
#error "MGR_PREC must be defined"
#endif
#ifndef MGR_K
#error "MGR_K must be defined"
#endif

#define MGR_CAT3_(a, b, c) a##_##b##_##c
#define MGR_CAT3(a, b, c) MGR_CAT3_(a, b, c)

namespace mgr {
#if MGR_PREC == 0
typedef double StateT;
#else
typedef float StateT;
#endif

void MGR_CAT3(register_stencil, MGR_PREC, MGR_K)(KernelTable& t) {
  const int ki = k_index(MGR_K);
#define MGR_X(W)                                                                \
  t.stencil[MGR_PREC][ki][width_index(W)][0] = &k_stencil<StateT, MGR_K, W, false>;   \
  t.stencil[MGR_PREC][ki][width_index(W)][1] = &k_stencil<StateT, MGR_K, W, true>;    \
  t.stencil_b[MGR_PREC][ki][width_index(W)][0] = &k_stencil_b<StateT, MGR_K, W, false>; \
  t.stencil_b[MGR_PREC][ki][width_index(W)][1] = &k_stencil_b<StateT, MGR_K, W, true>;
  MGR_STENCIL_WIDTHS(MGR_X)
#undef MGR_X
}
}  // namespace mgr
