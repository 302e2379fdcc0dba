// Table of the compiled relaxation kernels (host side).
#pragma once

#include "common.h"

namespace mgr {

typedef void (*KernelFn)(RelaxArgs);
typedef void (*BatchFn)(BatchArgs);  // the same kernel over a merged grid

// Window widths W and chunk lengths K with a register-resident stencil
// kernel; other shapes use the generic LDS kernel.
#define MGR_STENCIL_WIDTHS(X) \
  X(2) X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64)
constexpr int kNumWidths = 13;
constexpr int kWidths[kNumWidths] = {2, 4, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64};
constexpr int kNumK = 6;
constexpr int kKs[kNumK] = {1, 2, 4, 8, 16, 32};

// SDIRK variants: chunk K and (stages S, recurrence factors NF)
constexpr int kNumSdirkK = 5;
constexpr int kSdirkKs[kNumSdirkK] = {1, 2, 4, 8, 16};
constexpr int kNumSdirkShapes = 4;
constexpr int kSdirkShapes[kNumSdirkShapes][2] = {{1, 1}, {2, 1}, {3, 2}, {5, 3}};

// SDIRK in partial fractions: (stages S, real terms NR, of which backward
// NB, complex terms NC); with U1-U4 at most one root of the stage matrix
// lies inside the unit circle, so the backward term is real
constexpr int kNumSdirkPfShapes = 7;
constexpr int kSdirkPfShapes[kNumSdirkPfShapes][4] = {
    {1, 1, 0, 0}, {2, 2, 0, 0}, {2, 0, 0, 1}, {3, 3, 1, 0}, {3, 1, 1, 1}, {5, 4, 1, 0},
    {5, 2, 1, 1}};

struct KernelTable {
  KernelFn stencil[2][kNumK][kNumWidths][2] = {};  // [prec][K][W][per-step IO]
  KernelFn sdirk[2][kNumSdirkK][kNumSdirkShapes] = {};
  KernelFn sdirk_pf[2][kNumSdirkK][kNumSdirkPfShapes] = {};
  KernelFn generic[2] = {};
  // batched entries of the same kernels, same indices
  BatchFn stencil_b[2][kNumK][kNumWidths][2] = {};
  BatchFn sdirk_b[2][kNumSdirkK][kNumSdirkShapes] = {};
  BatchFn sdirk_pf_b[2][kNumSdirkK][kNumSdirkPfShapes] = {};
  BatchFn generic_b[2] = {};
  // inflow/outflow boundaries (bounded_kernels.h), FP64 state: point by
  // point, and register-blocked (K = bounded_k(W) points per thread) for the
  // window widths kBoundedWidths
  KernelFn bounded = nullptr;
  BatchFn bounded_b = nullptr;
  // [right-hand side rows prefetched (coarse levels)][width]
  KernelFn bounded_tiled[2][8] = {};
  BatchFn bounded_tiled_b[2][8] = {};
  // fine levels: points held in registers (K, HL, HR of kBoundedReg)
  KernelFn bounded_reg[8] = {};
  BatchFn bounded_reg_b[8] = {};
};
// points per thread chunk (any window width): odd, so lanes K doubles apart
// hit distinct LDS banks
constexpr int bounded_k(int) { return 9; }
// inflow forcing rows the register-blocked kernel stages in LDS at a time
constexpr int kFRowsLds = 64;
constexpr int kNumBoundedWidths = 8;
constexpr int kBoundedWidths[kNumBoundedWidths] = {4, 8, 12, 16, 24, 32, 48, 64};
// lane-resident fine-level kernels: {K points per lane, HL upwind halo, HR
// downwind halo}; the windows of ERKp+Up for p = 1..3 (wider windows need
// more registers than three wavefronts per SIMD leave)
constexpr int kNumBoundedReg = 6;
constexpr int kBoundedReg[kNumBoundedReg][3] = {{8, 1, 0},  {8, 4, 0},  {8, 6, 3},
                                                {16, 1, 0}, {16, 4, 0}, {16, 6, 3}};


// Filled once on first use; prec 0 = FP64 state, 1 = FP32 state.
const KernelTable& kernel_table();

int width_index(int W);         // index into kWidths, -1 if absent
int k_index(int K);             // index into kKs, -1 if absent
int sdirk_k_index(int K);
int sdirk_shape_index(int S, int NF);
int sdirk_pf_shape_index(int S, int NR, int NB, int NC);  // -1 if absent

// Utility kernels (misc.hip).
void launch_norm_reduce(const double* partial, int n, double scale2, double* out,
                        void* stream);
void launch_axpy(double* y, const double* x, long long n, void* stream);
void launch_uniform_init(double* out, long long rows, int nx, unsigned long long seed,
                         void* stream);

// Spectral coarsest-level solve (spectral.hip): X rows 0..n of x^0 = 0,
// x^s = Psi x^s-1 + g^s for g rows 1..n, with S room for spectral_rows(n)
// x n_x complex values, mu the n_x eigenvalues of Psi and tw the twiddles
// e^{-2 pi i q/n_x}, q < n_x/2 (complex = two doubles).  n_x a power of two
// from 4 up to kSpectralMaxNx.  Returns 0, or -1 if the shape is not
// supported or a launch failed.
constexpr int kSpectralMaxNx = 8192;
bool spectral_supported(int nx);
size_t spectral_rows(int n);
int launch_spectral_solve(const double* g, double* X, void* S, const void* mu, const void* tw,
                          int nx, int n, void* stream);

}  // namespace mgr
