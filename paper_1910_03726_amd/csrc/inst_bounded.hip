// The bounded-interval relaxation kernels (FP64 state only).
#include "bounded_kernels.h"
#include "registry.h"

namespace mgr {
template <int W>
static void reg_tiled(KernelTable& t, int i) {
  static_assert(W > 0, "");
  t.bounded_tiled[0][i] = &k_bounded_tiled<bounded_k(W), W, false>;
  t.bounded_tiled_b[0][i] = &k_bounded_tiled_b<bounded_k(W), W, false>;
  t.bounded_tiled[1][i] = &k_bounded_tiled<bounded_k(W), W, true>;
  t.bounded_tiled_b[1][i] = &k_bounded_tiled_b<bounded_k(W), W, true>;
}

void register_bounded(KernelTable& t) {
  t.bounded = &k_bounded;
  t.bounded_b = &k_bounded_b;
  reg_tiled<4>(t, 0);
  reg_tiled<8>(t, 1);
  reg_tiled<12>(t, 2);
  reg_tiled<16>(t, 3);
  reg_tiled<24>(t, 4);
  reg_tiled<32>(t, 5);
  reg_tiled<48>(t, 6);
  reg_tiled<64>(t, 7);
}
}  // namespace mgr
