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

template <int I>
static void reg_lanes(KernelTable& t) {
  constexpr int K = kBoundedReg[I][0], HL = kBoundedReg[I][1], HR = kBoundedReg[I][2];
  t.bounded_reg[I] = &k_bounded_reg<K, HL, HR>;
  t.bounded_reg_b[I] = &k_bounded_reg_b<K, HL, HR>;
}

void register_bounded(KernelTable& t) {
  reg_lanes<0>(t);
  reg_lanes<1>(t);
  reg_lanes<2>(t);
  reg_lanes<3>(t);
  reg_lanes<4>(t);
  reg_lanes<5>(t);
  static_assert(kNumBoundedReg == 6, "");
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
