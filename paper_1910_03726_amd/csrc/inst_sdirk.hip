// k_sdirk and k_generic instantiations for one precision (MGR_PREC 0/1).
#include "registry.h"
#include "sdirk_kernels.h"

#ifndef MGR_PREC
#error "MGR_PREC must be defined"
#endif

#define MGR_CAT2_(a, b) a##_##b
#define MGR_CAT2(a, b) MGR_CAT2_(a, b)

namespace mgr {
#if MGR_PREC == 0
typedef double StateT;
#else
typedef float StateT;
#endif

void MGR_CAT2(register_sdirk, MGR_PREC)(KernelTable& t) {
#define MGR_S(K, S, NF)                                                                   \
  t.sdirk[MGR_PREC][sdirk_k_index(K)][sdirk_shape_index(S, NF)] = &k_sdirk<StateT, K, S, NF>; \
  t.sdirk_b[MGR_PREC][sdirk_k_index(K)][sdirk_shape_index(S, NF)] = &k_sdirk_b<StateT, K, S, NF>;
#define MGR_SK(K) MGR_S(K, 1, 1) MGR_S(K, 2, 1) MGR_S(K, 3, 2) MGR_S(K, 5, 3)
  MGR_SK(1) MGR_SK(2) MGR_SK(4) MGR_SK(8) MGR_SK(16)
#undef MGR_SK
#undef MGR_S
  t.generic[MGR_PREC] = &k_generic<StateT>;
  t.generic_b[MGR_PREC] = &k_generic_b<StateT>;
}
}  // namespace mgr
