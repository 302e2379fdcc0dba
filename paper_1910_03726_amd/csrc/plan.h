// Internal plan structures of libmgrit (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mgrit.h"
#include "common.h"
#include "registry.h"
#include "setup.h"

namespace mgr {

enum OpKind { OP_STENCIL = 0, OP_GENERIC = 1, OP_SDIRK = 2, OP_BOUNDED = 3 };

// Fine-level residual passes write one partial sum per interval and tile.
constexpr int kMaxFineTiles = 16;

// Device memory of plans, from a per-device cache of released blocks (see
// plan.cpp); dev_free only once no queued work uses the block.
int dev_alloc(void** p, size_t bytes);
void dev_free(void* p);
void dev_trim();

// While a calling thread has an arena set, dev_alloc hands out 256-byte
// aligned pieces of [base, base + cap) instead of blocks of its own,
// dev_free leaves pointers inside it alone, and a plan's norm word is the
// arena's host_word: plans built that way allocate no device or pinned host
// memory (the allocation-free solve, static_solve.hip).
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool overflow = false;  // a request did not fit
  double host_word = 0.0;
};
void set_thread_arena(Arena* a);  // nullptr: back to the block cache

// One launch shape of the stencil kernel: `tiles` workgroups per interval,
// each of NL lanes x K points, writing `tile` points.  A tiled shape
// (tiles > 1) is valid for passes of at most `max_steps` steps (the tile's
// dependence cone must fit its extent); the untiled one for any count.
struct StencilShape {
  int K = 0, NL = 0, tiles = 1, tile = 0, max_steps = 0;
  int preload_rows = 0;                 // passes of <= this many steps stage
                                        // their right-hand side rows in LDS
  KernelFn fn[2] = {nullptr, nullptr};  // [FP64 state, FP32 state]
  BatchFn bfn[2] = {nullptr, nullptr};  // their batched entries
  size_t shmem[2] = {0, 0};
  double est_us = 0.0;                  // planner's launch-time estimate
};

// The relaxation operator of one level and the kernels that apply it.
struct OpDesc {
  int kind = OP_GENERIC;
  KernelFn fn[2] = {nullptr, nullptr};  // generic / SDIRK: [FP64 state, FP32 state]
  BatchFn bfn[2] = {nullptr, nullptr};
  size_t shmem[2] = {0, 0};             // dynamic LDS bytes per precision
  StencilShape whole[2], tiled[2];      // stencil: [no per-step IO, per-step IO]
  int seq_chunk = 0;                    // sequential sweeps: steps per launch
  double seq_us = 1e300;                // sequential sweeps: modelled time of one
  double* d_mu = nullptr;               // spectral solve: eigenvalues of the
  double* d_tw = nullptr;               // operator and twiddles (complex)
  int NL = 0, K = 0;                    // lanes per workgroup, points per lane
  int width = 0, Wbucket = 0, omin = 0; // stencil window, compiled width, start
  int ntaps = 0, nnz = 0;
  double flops_pps = 0.0;               // algorithmic flops per point and step
  double* d_taps = nullptr;
  int* d_off = nullptr;
  void* d_sdirk = nullptr;              // SDIRK: device SdirkPfDev (sdirk_terms > 0)
  int sdirk_terms = 0;                  // or SdirkDev (the factored form)
  void* d_bnd = nullptr;                // bounded kernel: device BoundedDev
  int reg_inst = -1, reg_rows = 0;      // bounded fine level: kBoundedReg entry of
                                        // the lane-resident kernel, its region rows
  int nilq = 0;                         // bounded coarse operator with every offset
                                        // >= 1: Psi^nilq = 0 (else 0)
  std::vector<void*> d_extra;           // bounded kernel: its blocks and forcing
  size_t bytes = 0;
  hipStream_t stream = nullptr;         // allocation and upload stream
  std::vector<std::vector<char>> staged;  // host sources of pending uploads

  // allocate `b` device bytes at *d and queue the upload of `h` (copied to
  // `staged`, dropped once the stream has drained)
  int upload(void** d, const void* h, size_t b);

  // steps: fine steps of one relaxation pass (m), or of the whole sweep
  // (seq); nblk: workgroup rows of a pass (intervals); max_tiles: bound on
  // tiles per interval
  int init_stencil(const Taps& t, int nx, int steps, int nblk, bool seq, int max_tiles,
                   std::string& err);
  int init_sdirk(const Tableau& t, double cfl, int nx, std::string& err);
  // inflow/outflow levels (Sec. 4.5): `interior` with signed offsets; the
  // fine level also brings its boundary rows and the forcing table F
  // (nt rows of fine->nf values); `stride`: fine steps between the start
  // times of consecutive blocks of a pass
  int init_bounded(const Taps& interior, const InflowOp* fine, const std::vector<double>* F,
                   int nx, int stride, std::string& err);
  void release();
  std::string describe() const;
};

struct Level {
  int n = 0;         // time steps on this level
  int nc = 0;        // coarse intervals (n / m), 0 on the coarsest level
  OpDesc op;         // relaxation operator (levels < L)
  OpDesc seq;        // coarsest level: single-workgroup sequential sweep
  double* X = nullptr;  // levels >= 2: all n+1 points (solution / correction)
  double* V = nullptr;  // levels >= 2 (not coarsest): relaxed C-points
  double* W = nullptr;  // the same, of a cycle started from corrected C-points
  double* R = nullptr;  // C-point residuals = right-hand side of level l+1
};

struct Plan;

// Relaxation launches of several plans recorded on one stream and issued
// together: launches of the same kernel, block size and LDS size (the same
// pass of requests with the same shape) become one batched launch over the
// concatenated grids; the others go out one by one.  A plan's launches keep
// their order.
struct Batch {
  struct Entry {
    KernelFn fn;
    BatchFn bfn;
    int nl;
    size_t lds;
    long long blocks;
    RelaxArgs args;
    Plan* owner;
  };
  hipStream_t stream = nullptr;
  std::vector<Entry> pending;
  long long launches = 0, merged = 0;  // kernels launched, entries merged into them
  int flush();
};

// What a profiled launch is: its level, pass (MGRIT_PASS_*), arithmetic
// precision and algorithmic HBM bytes and flops.
struct ProfTag {
  int level = 0, pass = 0, prec = 0;
  double bytes = 0.0, flops = 0.0;
};

struct ProfPending {
  int cls;
  hipEvent_t e0, e1;
  ProfTag tag;
};

struct Plan {
  int nx = 0, nt = 0, m = 0, scheme = 0;
  int cycle_kind = 0, relax_kind = 0, precision = 0;
  bool inflow = false;  // inflow/outflow boundaries (Sec. 4.5)
  double alpha = 1.0, cfl = 0.0, dx = 0.0, dt = 0.0, scale = 0.0;
  hipStream_t stream = nullptr;
  std::vector<Level> lev;
  double *Va = nullptr, *Vb = nullptr;      // fine C-point iterates (ping-pong)
  double *U = nullptr, *Rout = nullptr;     // FP64 refinement iterate and residual
  double *partial = nullptr, *d_norm = nullptr, *h_norm = nullptr;
  unsigned long long seed = 1;
  size_t bytes = 0;
  std::string description, description_levels;
  // coarsest level: spectral solve (possible if S is allocated, chosen if
  // `spectral`) or chunked sweeps
  int coarse_mode = MGRIT_COARSE_AUTO;
  bool spectral = false;
  // inflow plans: the coarsest sweep in overlapping chunks (nilpotent Psi)
  bool chunked = false;
  double* Sspec = nullptr;
  double spectral_us = 0.0;
  int set_coarse_mode(int mode);
  mgrit_stats stats = {};
  // profiling
  bool profiling = false;
  mgrit_profile prof = {};
  double fine_dof_steps = 0.0, prof_dof_base = 0.0;
  std::vector<ProfPending> pending;
  std::vector<hipEvent_t> event_pool;
  ProfTag tag;                            // of the next profiled launch
  std::vector<mgrit_prof_entry> detail;   // per (level, pass, precision)
  int parts = 0;  // partial sums written by the last residual launch
  Batch* batch = nullptr;  // set: relaxation launches are recorded there

  int launch(const OpDesc& op, int prec, const RelaxArgs& a, int grid, int cls);
  hipEvent_t take_event();
  void collect_profile();
  int mark_util(int cls, hipEvent_t& e0);
  void end_util(int cls, hipEvent_t e0);
  int relax(int l, int prec, int mode, const double* in, long long in_stride,
            const double* corr, const double* rhs, int rhs_mode, double* out,
            double* partial, int steps, double* delta = nullptr,
            const double* sub = nullptr, const double* sub2 = nullptr);
  int copy_cpoints(int l, int prec, const double* in, long long in_stride,
                   const double* corr, double* out);
  // one launch of the coarsest level's sequential sweep (steps s0..), or 1
  // in *last if it was the last one
  int sequential_chunk(int s0, const double* g, bool* last);
};

// MGRIT solves of n plans on one stream, step by step together, with their
// relaxation launches batched (solve.cpp); arguments as mgrit_solve, one
// entry per plan, status[i] its return code.
int solve_group(Plan* const* plans, int n, const double* const* u0, const double* const* uinit,
                const double* tol, const int* maxit, double* const* u_out, const int* out_kind,
                double* const* hist, int* iters, int* status);

}  // namespace mgr
