// k_sdirk_pf instantiations for one precision (MGR_PREC 0/1).
#include "registry.h"
#include "sdirk_pf_kernels.h"

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

void MGR_CAT2(register_sdirk_pf, MGR_PREC)(KernelTable& t) {
#define MGR_P(K, S, NR, NB, NC)                                                        \
  t.sdirk_pf[MGR_PREC][sdirk_k_index(K)][sdirk_pf_shape_index(S, NR, NB, NC)] =        \
      &k_sdirk_pf<StateT, K, S, NR, NB, NC>;                                           \
  t.sdirk_pf_b[MGR_PREC][sdirk_k_index(K)][sdirk_pf_shape_index(S, NR, NB, NC)] =      \
      &k_sdirk_pf_b<StateT, K, S, NR, NB, NC>;
#define MGR_PK(K)                                                                       \
  MGR_P(K, 1, 1, 0, 0) MGR_P(K, 2, 2, 0, 0) MGR_P(K, 2, 0, 0, 1) MGR_P(K, 3, 3, 1, 0)   \
  MGR_P(K, 3, 1, 1, 1) MGR_P(K, 5, 4, 1, 0) MGR_P(K, 5, 2, 1, 1)
  MGR_PK(1) MGR_PK(2) MGR_PK(4) MGR_PK(8) MGR_PK(16)
#undef MGR_PK
#undef MGR_P
}
}  // namespace mgr
