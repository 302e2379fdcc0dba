// Structures shared by the host planner and the gfx950 kernels of libmgrit.
//
// Layout in HBM: every space-time array is row-major [time level][n_x] FP64.
// A relaxation launch processes `nint` coarse intervals (the time-parallel
// dimension of MGRIT, Sec. 2.2), one workgroup per interval and spatial
// tile; the spatial state of a tile stays on-chip (registers or LDS) for
// all of its fine steps.
#pragma once

#include <stdint.h>

namespace mgr {

// What a relaxation launch writes (Sec. 2.2 terminology).
enum RelaxMode : int {
  MODE_FC = 0,   // F- then C-relaxation: out[j+out_off] = Phi^m start_j (+g)
  MODE_RES = 1,  // F-relaxation + C-point residual: out[j+1] = g + Phi^m start_j - ref[j+1]
  MODE_F = 2,    // F-relaxation writing every point: out[j*m + s], s = 0..m-1
                 // (the extra block j == nint writes its start state only)
  MODE_FW = 3,   // bounded kernel, a sweep of nint steps in chunks of m:
                 // block j steps from zero at row t0 = max(0, j*m - tile)
                 // up to row min((j+1)*m, nint), storing rows > j*m (and
                 // row 0 = 0 in block 0); exact when the operator vanishes
                 // after `tile` applications (truncated stencils whose
                 // offsets are all >= 1)
};

// How the right-hand side g of the level's system enters the steps.
enum RhsMode : int {
  RHS_NONE = 0,    // g = 0 (fine level)
  RHS_EVERY = 1,   // g^{jm+s} added after step s (rows of `rhs`, coarse levels)
  RHS_CPOINT = 2,  // g only at C-points: rhs[j+1] added after step m
};

struct RelaxArgs {
  // start state of interval j: in[j*in_stride] (+ corr[j*corr_stride]); zero if zero_in
  const double* in;
  long long in_stride;     // in rows
  const double* corr;
  long long corr_stride;   // in rows
  const double* sub;       // may be null: also subtract sub[j] and sub2[j]
  const double* sub2;      // (rows of n_x, stride 1) from the start state
  const double* rhs;
  const double* ref;       // MODE_RES: the C-points v being tested
  double* out;
  double* partial;         // sum of the squared outputs per workgroup (MODE_RES:
                           // of r, MODE_FC: of out[j+out_off]); may be null
  double* delta;           // MODE_FC, may be null: also delta[j+1] =
                           // out[j+out_off] - (in[j+1] + corr[j+1]), the
                           // update of C-point j+1 (row 0 set to 0)
  const double* taps;      // stencil: weights of the window offsets omin..omin+W-1
  const int* tap_off;      // generic kernel: offsets in [0, nx); bounded
                           // kernel: signed offsets
  const void* opdata;      // SDIRK kernel: device SdirkDev; bounded kernel:
                           // device BoundedDev
  int ntaps;               // generic / bounded kernel: number of taps
  int omin;                // stencil window start (frame shift per step), in
                           // [0, nx); bounded kernel: steps between the start
                           // times of consecutive blocks (inflow data rows)
  int mode, rhs_mode;
  int m;                   // fine steps per interval
  int nx;
  int nint;                // number of intervals (blocks of MODE_FC/MODE_RES)
  int zero_in;             // start from zero instead of `in`
  int write_row0;          // MODE_FC: block 0 also writes out[0] = start_0
  int out_off;             // MODE_FC: out row of interval j is j + out_off
  int write_last;          // MODE_F: also write the state after step m
  int skip_row0;           // MODE_F: the start row is already stored (chunked sweeps)
  int tile;                // stencil kernel: points per tile
  int tiles;               // stencil kernel: tiles per interval (block b: tile
                           // b % tiles of interval b / tiles)
  int preload;             // stencil kernel, RHS_EVERY: all m right-hand side
                           // rows staged in LDS before the first step
};

// Stencil kernels without per-step I/O whose halo comes by lane shifts
// (window W - 1 <= K) stage their start and end rows through LDS one half
// of the extent at a time: half the LDS, so more workgroups per CU.
constexpr bool kHalfStage = true;
constexpr bool stencil_half_stage(int K, int W, bool io) {
  return kHalfStage && !io && W - 1 <= K && K % 2 == 0;
}

// Inflow forcing values (steps x nf) the lane-resident bounded kernel stages
// in LDS at a time.
constexpr int kRegFCap = 256;
// Weights of one boundary row of that kernel (a multiple of 4).
constexpr int kRegLen = 24;
// The trailing values of lane b-1's chunk the right boundary rows may read:
// the stencil's upwind reach and the outflow extrapolation's (at most 4).
template <int K, int HL>
constexpr int kRegExportB() { return HL + 4 < K ? HL + 4 : K; }

// Several relaxation launches of the same kernel and launch shape merged
// into one grid (requests served together): member i owns blocks
// start[i] .. start[i+1]-1 (start[0] = 0) and runs with a[i] as if it had
// been launched alone.
constexpr int kMaxBatch = 8;
struct BatchArgs {
  RelaxArgs a[kMaxBatch];
  int start[kMaxBatch];
  int n;  // members, 1..kMaxBatch
};

// Operator of a level with inflow/outflow boundaries (Sec. 4.5), applied by
// the bounded kernel as
//   (Phi u)_i = sum_c lblk[i*ncl + c] u_c                 for i < nl,
//             = sum_c rblk[(i-nx+nr)*ncr + c] u_{nx-ncr+c}  for i >= nx - nr,
//             = sum_t taps[t] u_{i - off[t]} over 0 <= i - off[t] < nx
//                                                         otherwise,
// plus, on the fine level, the inflow forcing of the step from t_n:
// F[n*nf + i] added to rows i < nf (F: one row per fine step).
struct BoundedDev {
  int nl, ncl, nr, ncr, nf;
  int padl, padr;  // register-blocked kernel: zero points kept in LDS left
                   // and right of the state, so every window read is in
                   // bounds and reads 0 off the grid (the truncation)
  int pad_;
  const double* lblk;
  const double* rblk;
  const double* F;
  // lane-resident fine-level kernel (k_bounded_reg): region lanes [0, rg_a)
  // and [rg_b, rg_nla) of K points; the LDS window bu of rg_bu doubles per
  // step parity (left region and lane a's chunk in [0, rg_lw), then lane
  // b-1's chunk and the right region); rg_rows region rows, row r a window
  // of rg_len weights (rg_coef[r * rg_ls ..]) over bu from rg_cs[r], its
  // result stored at bu slot rg_dst[r]
  int rg_a, rg_b, rg_nla, rg_lw, rg_bu, rg_ls, rg_len, rg_rows;
  const double* rg_coef;
  const int* rg_cs;
  const int* rg_dst;
};

// One factor of a cyclic banded stage solve: a linear recurrence of order
// <= 2 run forward (dir = +1: y_i = x_i + a1 y_{i-1} + a2 y_{i-2}) or
// backward (dir = -1: y_i = x_i + a1 y_{i+1} + a2 y_{i+2}), periodic in i.
// The constants of its chunked scan over lanes (chunk length K, NL lanes):
// Hp[d] = H^(2^d) with H the 2x2 chunk transfer matrix, and
// Cinv = (I - H^NL)^{-1} (cyclic closure).  2x2 matrices are row-major.
constexpr int MAX_FACTORS = 4;
constexpr int MAX_STAGES = 6;
struct RecDev {
  int dir;
  int pad_;
  double a1, a2;
  double Hp[11][4];
  double Cinv[4];
};

// SDIRK step data (Appendix A, Table 8): stage matrix M = I - gamma dt L is
// applied as M^{-1} = scale * prod_f (factor f)^{-1}.
struct SdirkDev {
  int s;                 // stages
  int nf;                // recurrence factors
  int K;                 // chunk length the scan constants were built for
  int NL;                // lanes the scan constants were built for
  double A[MAX_STAGES][MAX_STAGES];
  double b[MAX_STAGES];
  double inv_gamma;      // 1/gamma: dt L Y_i = (Y_i - rhs_i)/gamma
  double scale;          // 1/K of the factorization
  RecDev f[MAX_FACTORS];
};

// The same stage solve in partial fractions: with the stage matrix's roots
// simple, M^{-1} = c0 I + sum_t A_t (I - q_t X_t)^{-1}, X_t = S (forward,
// dir = +1: y_i = x_i + q y_{i-1}) or S^{-1} (backward, dir = -1:
// y_i = x_i + q y_{i+1}), every term a first-order periodic recurrence on
// the same right-hand side, so that all terms of a stage share one local
// pass, one carry scan and one barrier.  Real roots give real terms; a
// conjugate pair gives one complex term contributing 2 Re(A y).  Scan
// constants as for RecDev, of the scalar (complex) chunk factor Q = q^K:
// Qp[d] = Q^(2^d) and close = (1 - Q^NL)^{-1}; complex values as (re, im).
constexpr int MAX_PF_TERMS = 4;
struct PfTermDev {
  int dir;
  int pad_;
  double q[2], a[2];
  double Qp[11][2];
  double close[2];
};
struct SdirkPfDev {
  int s;                  // stages
  int nr, nb, nc;         // real terms (the last nb of them backward), then
                          // complex terms (forward)
  int K, NL;
  double A[MAX_STAGES][MAX_STAGES];
  double inv_gamma;
  double c0;
  PfTermDev t[MAX_PF_TERMS];
};

}  // namespace mgr
