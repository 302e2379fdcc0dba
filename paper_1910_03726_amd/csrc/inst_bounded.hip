// The bounded-interval relaxation kernel (FP64 state only).
#include "bounded_kernels.h"
#include "registry.h"

namespace mgr {
void register_bounded(KernelTable& t) {
  t.bounded = &k_bounded;
  t.bounded_b = &k_bounded_b;
}
}  // namespace mgr
