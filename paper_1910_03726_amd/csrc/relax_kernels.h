// Relaxation kernels of libmgrit for CDNA4 (gfx950).
//
// The time-parallel dimension of MGRIT (Sec. 2.2), the coarse intervals, is
// the grid: one workgroup per interval, or per spatial tile of an interval.
// Inside a workgroup the spatial values stay on-chip for all m fine steps
// (temporal blocking); only start states, the right-hand side rows of
// coarse levels and the outputs touch HBM.
//
// Kernel families sharing the launch arguments (RelaxArgs):
//   k_stencil<T,K,W,IO>  a periodic stencil of window W (the ERK stepper of
//                        Corollary 1 or a coarse operator Psi): lane l owns
//                        K contiguous points in registers; taps applied in
//                        a frame that moves with the window start omin each
//                        step, so every halo comes from the upwind (left)
//                        neighbour; optionally spatially tiled.
//   k_generic<T>         any n_x and any tap list; state in LDS.
//   k_sdirk<T,K,S,NF>    SDIRK stages (sdirk_kernels.h).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"

namespace mgr {

__device__ __forceinline__ int wrap_hi(int i, int n) { return i >= n ? i - n : i; }

__device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// For lane l > 0 the value v of lane l - 1 of the wavefront, for lane 0
// `old` (DPP wave_shr:1 without bound control: no LDS traffic).
__device__ __forceinline__ int shr1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ float shr1(float old, float v) {
  return __int_as_float(shr1(__float_as_int(old), __float_as_int(v)));
}
__device__ __forceinline__ double shr1(double old, double v) {
  return __hiloint2double(shr1(__double2hiint(old), __double2hiint(v)),
                          shr1(__double2loint(old), __double2loint(v)));
}

// Row element g of a row (g < 2^29): a 32-bit byte offset from the row's
// uniform base, which global loads/stores take as a scalar base plus a
// vector offset (no 64-bit address arithmetic per element).
__device__ __forceinline__ double ld_row(const double* row, unsigned g) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(row) + (g << 3));
}
__device__ __forceinline__ void st_row(double* row, unsigned g, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(row) + (g << 3)) = v;
}

// Wait for every outstanding vector-memory load of this wavefront
// (s_waitcnt vmcnt(0), other counters untouched).  Called once after values
// that stay in registers through a step loop are loaded: without it the
// wait for them is re-inserted at the loop head, where in every step it
// also drains the prefetches and stores of the step before.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The member of a batched launch that this workgroup belongs to (its
// arguments) and the workgroup's index within that member's own grid.
__device__ __forceinline__ RelaxArgs batch_member(const BatchArgs& b, int& blk) {
  const int x = (int)blockIdx.x;
  int r = 0;
#pragma unroll
  for (int i = 1; i < kMaxBatch; ++i) r += (i < b.n && x >= b.start[i]) ? 1 : 0;
  blk = x - b.start[r];
  return b.a[r];
}

// Deterministic block sum (fixed reduction order); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// ---------------------------------------------------------------------------
// Coalesced row traffic through LDS
// ---------------------------------------------------------------------------
// Lane l owns local points p = l*K .. l*K+K-1; local point p is the true
// point (p + sh) mod n_x (the frame shift of the stencil kernels).  Rows go
// between HBM and LDS with consecutive lanes on consecutive doubles (full
// cache lines per instruction) and between LDS and each lane's chunk with
// local point p at stg[p + p/K]: one pad slot per chunk makes the chunk
// reads and writes free of bank conflicts.
template <int K>
struct Stager {
  double* stg;
  int nx, NL, lane;
  __device__ __forceinline__ int slot(int p) const { return p + p / K; }
  __device__ __forceinline__ int local(int i, int sh) const {
    int p = i - sh;
    return p + ((p < 0) ? nx : 0);
  }
  // global -> registers in the coalesced layout (element q is true point
  // lane + q*NL); used to issue a row's loads early
  __device__ __forceinline__ void fetch(const double* row, double (&r)[K]) const {
#pragma unroll
    for (int q = 0; q < K; ++q) r[q] = row[lane + q * NL];
  }
  // coalesced registers -> this lane's chunk
  template <typename T>
  __device__ __forceinline__ void deliver(const double (&r)[K], int sh, T (&x)[K]) const {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) stg[slot(local(lane + q * NL, sh))] = r[q];
    __syncthreads();
    const int b = lane * (K + 1);
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = (T)stg[b + k];
  }
  template <typename T>
  __device__ __forceinline__ void load(const double* row, int sh, T (&x)[K]) const {
    double r[K];
    fetch(row, r);
    deliver(r, sh, x);
  }
  template <typename T>
  __device__ __forceinline__ void store(double* row, int sh, const T (&x)[K]) const {
    __syncthreads();
    const int b = lane * (K + 1);
#pragma unroll
    for (int k = 0; k < K; ++k) stg[b + k] = (double)x[k];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int i = lane + q * NL;
      row[i] = stg[slot(local(i, sh))];
    }
  }
};

// LDS doubles of the staging area for n_x points in chunks of K.
__host__ __device__ constexpr int stage_doubles(int nx, int K) { return nx + nx / K; }

// Start state of interval j in FP64 (staged, coalesced).
template <int K>
__device__ __forceinline__ void start_state(const RelaxArgs& a, int j, const Stager<K>& S,
                                            double (&v)[K]) {
  if (a.zero_in) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    return;
  }
  S.load(a.in + (long long)j * a.in_stride * a.nx, 0, v);
  __builtin_amdgcn_sched_barrier(0);  // one row in flight at a time
  if (a.corr) {
    double c[K];
    S.load(a.corr + (long long)j * a.corr_stride * a.nx, 0, c);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += c[k];
  }
  if (a.sub) {
    double c[K];
    S.load(a.sub + (long long)j * a.nx, 0, c);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] -= c[k];
  }
  if (a.sub2) {
    double c[K];
    S.load(a.sub2 + (long long)j * a.nx, 0, c);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] -= c[k];
  }
}

// Stores after the last step; `sh` is the frame shift of x.
template <typename T, int K>
__device__ __forceinline__ void finish(const RelaxArgs& a, int j, const Stager<K>& S, int sh,
                                       const T (&x)[K], double* red) {
  const int nx = a.nx;
  if (a.mode != MODE_FC && a.mode != MODE_RES) return;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = (double)x[k];
  if (a.rhs_mode == RHS_CPOINT) {
    double g[K];
    S.load(a.rhs + (long long)(j + 1) * nx, sh, g);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += g[k];
  }
  double ss = 0.0;
  if (a.mode == MODE_FC) {
    if (a.partial) {
#pragma unroll
      for (int k = 0; k < K; ++k) ss += v[k] * v[k];
    }
    S.store(a.out + (long long)(j + a.out_off) * nx, sh, v);
    if (a.delta) {
      // update of C-point j+1: out - (in + corr), row 0 = 0
      double u[K];
      if (a.zero_in) {
#pragma unroll
        for (int k = 0; k < K; ++k) u[k] = 0.0;
      } else {
        S.load(a.in + (long long)(j + 1) * a.in_stride * nx, sh, u);
      }
      if (a.corr) {
        double c[K];
        S.load(a.corr + (long long)(j + 1) * a.corr_stride * nx, sh, c);
#pragma unroll
        for (int k = 0; k < K; ++k) u[k] += c[k];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) u[k] = v[k] - u[k];
      S.store(a.delta + (long long)(j + 1) * nx, sh, u);
      if (j == 0) {
        for (int i = S.lane; i < nx; i += S.NL) a.delta[i] = 0.0;
      }
    }
  } else {
    double rf[K];
    S.load(a.ref + (long long)(j + 1) * nx, sh, rf);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v[k] -= rf[k];
      ss += v[k] * v[k];
    }
    S.store(a.out + (long long)(j + 1) * nx, sh, v);
    if (j == 0) {
      for (int i = S.lane; i < nx; i += S.NL) a.out[i] = 0.0;  // r^0 = 0
    }
  }
  if (a.partial) {
    const double s = block_sum(ss, red);
    if (threadIdx.x == 0) a.partial[j] = s;
  }
}

// Extent of a stencil workgroup: E = NL*K consecutive frame positions e
// (lane l owns e = l*K .. l*K+K-1).  Position e of a row whose frame shift
// is sh is the true point (f0 + e + sh) mod n_x.  Rows are staged through
// LDS with slot(e) = e + e/K: the coalesced order (e = lane + q*NL) and the
// chunk order are both free of bank conflicts.
template <int K>
struct Extent {
  int nx, NL, lane, E, f0;  // f0 in [0, n_x), E <= n_x
  __device__ __forceinline__ static int slot(int e) { return e + e / K; }
  // true point of position 0 at frame shift sh (sh in [0, n_x))
  __device__ __forceinline__ int first(int sh) const { return wrap_hi(f0 + sh, nx); }
  // true point of position e (b = first(sh)); unsigned, so that row
  // addresses are a uniform base plus a 32-bit lane offset
  __device__ __forceinline__ unsigned at(int b, int e) const {
    unsigned g = (unsigned)(b + e);
    return g >= (unsigned)nx ? g - (unsigned)nx : g;
  }
  // global -> registers, coalesced (element q is position lane + q*NL)
  __device__ __forceinline__ void fetch(const double* row, int sh, double (&r)[K]) const {
    const int b = first(sh);
#pragma unroll
    for (int q = 0; q < K; ++q) r[q] = ld_row(row, at(b, lane + q * NL));
  }
  __device__ __forceinline__ void put(double* stg, const double (&r)[K]) const {
#pragma unroll
    for (int q = 0; q < K; ++q) stg[slot(lane + q * NL)] = r[q];
  }
  // the same for half h of the extent (positions h E/2 + lane + q NL,
  // q < K/2) into a staging area of half the size
  __device__ __forceinline__ void fetch_half(const double* row, int h, double (&r)[K / 2]) const {
    const int b = first(0) + h * (E / 2);
#pragma unroll
    for (int q = 0; q < K / 2; ++q) r[q] = ld_row(row, at(b, lane + q * NL));
  }
  __device__ __forceinline__ void put_half(double* stg, const double (&r)[K / 2]) const {
#pragma unroll
    for (int q = 0; q < K / 2; ++q) stg[slot(lane + q * NL)] = r[q];
  }
  // this lane's chunk of a row, straight from global memory
  __device__ __forceinline__ void chunk(const double* row, int sh, double (&r)[K]) const {
    const int b = first(sh);
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = ld_row(row, at(b, lane * K + k));
  }
};

// Stores after the last step of a stencil workgroup (MODE_FC / MODE_RES):
// the tile's positions [eout, E) of the state x (frame shift sh), staged
// for coalesced access; residuals and their partial sum (one per
// workgroup, at partial[j * tiles + c], i.e. at its block index).  HALF:
// the staging area holds half the extent, so the lanes of each half stage
// their chunks in turn.
template <typename T, int K, bool HALF>
__device__ __forceinline__ void finish_extent(const RelaxArgs& a, int j, int blk, const Extent<K>& X,
                                              int eout, int sh, const T (&x)[K], double* stg,
                                              double* red) {
  if (a.mode != MODE_FC && a.mode != MODE_RES) return;
  const int nx = a.nx, NL = X.NL, lane = X.lane, E = X.E;
  const int bs = X.first(sh);
  const long long rj = (long long)(j + 1) * nx;
  const double* grow = a.rhs_mode == RHS_CPOINT ? a.rhs + rj : nullptr;
  const double* rrow = a.mode == MODE_RES ? a.ref + rj : nullptr;
  double* orow = a.out + (a.mode == MODE_FC ? (long long)(j + a.out_off) * nx : rj);
  // FC with delta: the current C-point j+1 (in + corr) and the update row
  const bool dl = a.mode == MODE_FC && a.delta;
  const double* urow = (dl && !a.zero_in) ? a.in + (long long)(j + 1) * a.in_stride * nx : nullptr;
  const double* crow = (dl && a.corr) ? a.corr + (long long)(j + 1) * a.corr_stride * nx : nullptr;
  double* drow = dl ? a.delta + rj : nullptr;
  double ss = 0.0;
  // position e of the extent, its staged value v
  auto emit = [&](int e, double v) __attribute__((always_inline)) {
    const unsigned g = X.at(bs, e);
    if (grow) v += ld_row(grow, g);
    if (rrow) v -= ld_row(rrow, g);
    ss += v * v;
    st_row(orow, g, v);
    if (dl) {
      double u = urow ? ld_row(urow, g) : 0.0;
      if (crow) u += ld_row(crow, g);
      st_row(drow, g, v - u);
    }
  };
  if constexpr (!HALF) {
    __syncthreads();  // the image / staging area is no longer read
    const int b = lane * (K + 1);
#pragma unroll
    for (int k = 0; k < K; ++k) stg[b + k] = (double)x[k];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int e = eout + lane + q * NL;
      if (e < E) emit(e, stg[Extent<K>::slot(e)]);
    }
  } else {
    // half h: lanes [h NL/2, (h+1) NL/2), positions [h E/2, (h+1) E/2)
    const int hl = NL / 2, EH = E / 2;
    for (int h = 0; h < 2; ++h) {
      __syncthreads();  // the staging area is no longer read
      if ((lane >= hl) == (h == 1)) {
        const int b = (lane - h * hl) * (K + 1);
#pragma unroll
        for (int k = 0; k < K; ++k) stg[b + k] = (double)x[k];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < K / 2; ++q) {
        const int e = lane + q * NL;  // within the half
        if (h * EH + e >= eout) emit(h * EH + e, stg[Extent<K>::slot(e)]);
      }
    }
  }
  // row 0: r^0 = 0 (MODE_RES), delta^0 = 0 (MODE_FC with delta)
  double* zrow = a.mode == MODE_RES ? a.out : (dl ? a.delta : nullptr);
  if (zrow && j == 0) {
    const int b0 = X.first(0);
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int e = eout + lane + q * NL;
      if (e < E) st_row(zrow, X.at(b0, e), 0.0);
    }
  }
  if (a.partial) {
    const double s = block_sum(ss, red);
    if (lane == 0) a.partial[blk] = s;
  }
}

// The stencil kernel.  Workgroup (c, j) -- block j*tiles + c of a 1-D grid
// -- advances interval j by m steps of
// a periodic window-W stencil (the ERK stepper of Corollary 1 or a coarse
// operator Psi) and writes the points of tile c: true frame positions
// [c*C, min((c+1)*C, n_x)) with C = a.tile.  With one tile (C = E = n_x)
// the extent is the whole periodic line.  With several tiles the extent
// ends at the tile's end and reaches m*(W-1) points upwind of it, the
// dependence cone of the tile over m steps: the points left of the cone
// are computed from wrapped neighbours and discarded (redundant work
// bought for parallelism across CUs without any inter-workgroup sync).
//
// IO = false: no per-step memory traffic (fine-level FC and residual
// passes); IO = true: a right-hand side row every step and/or every state
// stored (coarse levels, interpolation, sequential sweeps).  Per-step rows
// move between HBM and each lane's chunk directly; right-hand side rows are
// prefetched two steps ahead.
//
// Two ways to apply the stencil, chosen at compile time:
//  * W-1 <= K (halo within the left neighbour lane): in place, right to
//    left, halo values by a DPP lane shift inside the wavefront and, for
//    lane 0, from a 2*H-value LDS slot per wavefront;
//  * W-1 > K (wide coarse operators): the chunk image of every lane sits in
//    LDS (padded layout), each output accumulates while halo values stream
//    from LDS one at a time (registers ~2K instead of K+W).
//
// Dynamic LDS: with `preload` first the m right-hand side rows (staged
// layout, E + E/K doubles each), then the staging area (E + E/K doubles:
// start/end rows), which in the second case also holds the two chunk images (2*((E+M) + (E+M)/K)
// values of T, M = W-1 rounded up to a multiple of K), then 2*H slots per
// wavefront (first case only).
template <typename T, int K, int W, bool IO>
__device__ __forceinline__ void stencil_body(const RelaxArgs& a, const int blk) {
  constexpr bool kShfl = (W - 1 <= K);
  constexpr int H = (W - 1 < K) ? (W - 1) : K;
  constexpr int HW = (W > 1) ? (W - 1) : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];

  const int NL = blockDim.x, lane = threadIdx.x, nx = a.nx, m = a.m;
  const int c = (int)((unsigned)blk % (unsigned)a.tiles), j = (int)((unsigned)blk / (unsigned)a.tiles);
  const int wave = lane >> 6, lw = lane & 63, nwave = NL >> 6;
  const int E = NL * K;
  const int t0 = c * a.tile, t1 = min(t0 + a.tile, nx);
  const int eout = E - (t1 - t0);  // first position written
  int f0 = (t1 - E) % nx;
  f0 += (f0 < 0) ? nx : 0;
  const Extent<K> X{nx, NL, lane, E, f0};
  // start and end rows staged half the extent at a time
  constexpr bool HALF = stencil_half_stage(K, W, IO);
  const int nst = HALF ? E / 2 + E / 2 / K : E + E / K;  // doubles of the staging area
  const bool preload = IO && a.preload && a.rhs_mode == RHS_EVERY;
  double* ring = reinterpret_cast<double*>(smem_raw);  // preloaded rows 1..m
  unsigned char* lds = smem_raw + (preload ? sizeof(double) * (size_t)m * nst : 0);
  double* stg = reinterpret_cast<double*>(lds);
  T* sm = reinterpret_cast<T*>(lds + sizeof(double) * nst);  // halo slots
  // streaming case: two chunk images (steps alternate), position p at
  // slot(p + M), the M positions before 0 a copy of the last M (periodic
  // wrap, or discarded values of a tile), so that every halo address is
  // this lane's base plus a constant
  constexpr int M = ((W - 1 + K - 1) / K) * K;
  const int nimg = (E + M) + (E + M) / K;
  T* img0 = reinterpret_cast<T*>(stg);
  T* img1 = img0 + nimg;
  const int b = lane * (K + 1);
  const bool ghost = lane * K >= E - M;  // this chunk is also copied before 0
  // write x as the image of buffer im (and its ghost copy)
  auto put_image = [&](T* im, const T (&xv)[K]) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < K; ++k) im[b + (M + M / K) + k] = xv[k];
    if (ghost) {
#pragma unroll
      for (int k = 0; k < K; ++k) im[b + (M + M / K) + k - NL * (K + 1)] = xv[k];
    }
  };

  // start state (FP64, staged)
  const bool store0 = (a.mode == MODE_F && !a.skip_row0) ||
                      (a.mode == MODE_FC && a.write_row0 && j == 0);
  T x[K];
  if constexpr (HALF) {
    // each half fetched (coalesced), staged and taken by its lanes in turn:
    // half the LDS and half a row in registers
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      double v[K / 2];
      if (a.zero_in) {
#pragma unroll
        for (int q = 0; q < K / 2; ++q) v[q] = 0.0;
      } else {
        X.fetch_half(a.in + (long long)j * a.in_stride * nx, h, v);
        const double* adds[3] = {a.corr ? a.corr + (long long)j * a.corr_stride * nx : nullptr,
                                 a.sub ? a.sub + (long long)j * nx : nullptr,
                                 a.sub2 ? a.sub2 + (long long)j * nx : nullptr};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          if (!adds[r]) continue;
          double w[K / 2];
          X.fetch_half(adds[r], h, w);
#pragma unroll
          for (int q = 0; q < K / 2; ++q) v[q] += r == 0 ? w[q] : -w[q];
        }
      }
      if (store0) {
        double* row = a.out + (a.mode == MODE_F ? (long long)j * m * nx : 0LL);
        const int b0 = X.first(0) + h * (E / 2);
#pragma unroll
        for (int q = 0; q < K / 2; ++q)
          if (h * (E / 2) + lane + q * NL >= eout) st_row(row, X.at(b0, lane + q * NL), v[q]);
      }
      if (h == 1) __syncthreads();  // the first half has been taken
      X.put_half(stg, v);
      __syncthreads();
      if ((lane >= NL / 2) == (h == 1)) {
        const int bh = b - h * (NL / 2) * (K + 1);
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = (T)stg[bh + k];
      }
    }
  } else {
    double v[K];
    if (a.zero_in) {
#pragma unroll
      for (int q = 0; q < K; ++q) v[q] = 0.0;
    } else {
      X.fetch(a.in + (long long)j * a.in_stride * nx, 0, v);
      if (a.corr) {
        double cr[K];
        X.fetch(a.corr + (long long)j * a.corr_stride * nx, 0, cr);
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] += cr[q];
      }
      // one row at a time, like the correction, so that at most one row
      // beside v is held in registers
      if (a.sub) {
        double sr[K];
        X.fetch(a.sub + (long long)j * nx, 0, sr);
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] -= sr[q];
      }
      if (a.sub2) {
        double sr[K];
        X.fetch(a.sub2 + (long long)j * nx, 0, sr);
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] -= sr[q];
      }
    }
    X.put(stg, v);
    __syncthreads();
    if (store0) {
      double* row = a.out + (a.mode == MODE_F ? (long long)j * m * nx : 0LL);
      const int b0 = X.first(0);
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int e = eout + lane + q * NL;
        if (e < E) st_row(row, X.at(b0, e), stg[Extent<K>::slot(e)]);
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = (T)stg[b + k];
  }
  if (a.mode == MODE_F && j == a.nint) return;  // extra block: the last C-point
  // the taps through the scalar cache (read only): FP64 taps stay in
  // scalar registers, which the FMAs take as operands
  T tp[W];
  {
    typedef __attribute__((address_space(4))) const double cdouble;
    const cdouble* tq = (const cdouble*)a.taps;
#pragma unroll
    for (int t = 0; t < W; ++t) tp[t] = (T)tq[t];
  }
  wait_vmem();

  const bool every = IO && a.rhs_mode == RHS_EVERY;
  const bool store_steps = IO && a.mode == MODE_F;
  const long long row0 = (long long)j * m;
  // right-hand side chunks of the next two steps (ga: odd steps, gb: even)
  double ga[IO ? K : 1], gb[IO ? K : 1];
  if constexpr (IO) {
    if (preload) {
      // all right-hand side rows into LDS, up to 32/K rows in flight
      constexpr int B = (32 / K) > 0 ? 32 / K : 1;
      int shr = 0;
      for (int s0 = 1; s0 <= m; s0 += B) {
        double r[B][K];
#pragma unroll
        for (int i = 0; i < B; ++i) {
          shr = wrap_hi(shr + a.omin, nx);
          if (s0 + i <= m) X.fetch(a.rhs + (row0 + s0 + i) * nx, shr, r[i]);
        }
#pragma unroll
        for (int i = 0; i < B; ++i)
          if (s0 + i <= m) X.put(ring + (long long)(s0 + i - 1) * nst, r[i]);
      }
    } else if (every) {
      if (m >= 1) X.chunk(a.rhs + (row0 + 1) * nx, wrap_hi(a.omin, nx), ga);
      if (m >= 2)
        X.chunk(a.rhs + (row0 + 2) * nx, wrap_hi(wrap_hi(a.omin, nx) + a.omin, nx), gb);
    }
  }
  __syncthreads();  // staging area free (start row delivered and stored)
  if constexpr (!kShfl) {
    put_image(img0, x);
    __syncthreads();
  }

  int sh = 0;
  // one step: x <- taps * x (+ g); g is this step's right-hand side chunk
  auto step = [&](int s, double (&g)[IO ? K : 1], auto ev, auto pl)
                  __attribute__((always_inline)) {
    constexpr bool EV = decltype(ev)::value;  // right-hand side every step
    constexpr bool PL = decltype(pl)::value;  // ... preloaded in LDS
    if constexpr (kShfl) {
      if constexpr (W > 1) {
        T halo[HW];
        T* slot = sm + (s & 1) * nwave * H;
        if (lw == 63) {
#pragma unroll
          for (int e = 0; e < H; ++e) slot[wave * H + e] = x[K - H + e];
        }
        __syncthreads();
        const int pw = (wave + nwave - 1) % nwave;
        // halo[h]: the point W-1-h to the left of lane*K, element
        // K-(W-1-h) of the left neighbour lane: a DPP shift inside the
        // wavefront over the previous wavefront's edge value (read by all
        // lanes at one address), which lane 0 keeps
#pragma unroll
        for (int h = 0; h < W - 1; ++h)
          halo[h] = shr1(slot[pw * H + (h + H - (W - 1))], x[K - (W - 1 - h)]);
        // in place, right to left: x[k] <- sum_t tp[t] * x[k - t]
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
          T acc = (T)0;
#pragma unroll
          for (int t = 0; t < W; ++t) {
            const int idx = k - t;
            const T v = (idx >= 0) ? x[idx >= 0 ? idx : 0] : halo[idx < 0 ? W - 1 + idx : 0];
            acc = fma(tp[t], v, acc);
          }
          x[k] = acc;
        }
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] *= tp[0];
      }
    } else {
      // halo positions q = -(W-1)..-1 (relative to lane*K) from the image
      // of the previous step in batches of NB LDS reads, the next batch in
      // flight while the current one is consumed; then the own chunk
      const T* im = (s & 1) ? img0 : img1;
      constexpr int NB = 12;
      constexpr int NBAT = (W - 1 + NB - 1) / NB;
      T acc[K];
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = (T)0;
      T hv[2][NB];
      auto read_batch = [&](int bi, T (&h)[NB]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int q = -(W - 1) + bi * NB + i;
          if (q < 0) h[i] = im[b + ((q + M) + (q + M) / K)];
        }
      };
      read_batch(0, hv[0]);
#pragma unroll
      for (int bi = 0; bi < NBAT; ++bi) {
        if (bi + 1 < NBAT) read_batch(bi + 1, hv[(bi + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int q = -(W - 1) + bi * NB + i;
          if (q < 0) {
#pragma unroll
            for (int k = 0; k < K && k < q + W; ++k) acc[k] = fma(tp[k - q], hv[bi & 1][i], acc[k]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int q = 0; q < K; ++q) {
#pragma unroll
        for (int k = q; k < K && k < q + W; ++k) acc[k] = fma(tp[k - q], x[q], acc[k]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) x[k] = acc[k];
    }
    sh = wrap_hi(sh + a.omin, nx);
    if constexpr (IO) {
      if constexpr (EV && PL) {
        const double* rr = ring + (long long)(s - 1) * nst + b;  // (preloaded)
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] += (T)rr[k];
      } else if constexpr (EV) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] += (T)g[k];
        // prefetch the row of step s+2 (clamped to the last row) into the
        // registers just used: unconditional, so that they stay one
        // loop-carried value and the load is first waited for two steps on
        const int sh2 = wrap_hi(wrap_hi(sh + a.omin, nx) + a.omin, nx);
        X.chunk(a.rhs + (row0 + min(s + 2, m)) * nx, sh2, g);
      }
      if (kShfl && store_steps && (s < m || a.write_last)) {
        // no image: each lane stores its chunk
        double* row = a.out + (row0 + s) * nx;
        const int bs = X.first(sh);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int e = lane * K + k;
          if (e >= eout) st_row(row, X.at(bs, e), (double)x[k]);
        }
      }
    }
    if constexpr (!kShfl) {
      // the other buffer: its last readers (step s-1) passed the barrier
      // of step s-1 before anyone reaches this write
      T* im = (s & 1) ? img1 : img0;
      put_image(im, x);
      __syncthreads();
      if (store_steps && (s < m || a.write_last)) {
        // coalesced stores from the new image (overwritten two steps on)
        double* row = a.out + (row0 + s) * nx;
        const int bs = X.first(sh);
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const int e = lane + q * NL;
          if (e >= eout) st_row(row, X.at(bs, e), (double)im[(e + M) + (e + M) / K]);
        }
      }
    }
  };
  // with a right-hand side in registers, steps in pairs (odd steps use ga,
  // even ones gb); the loop is written once per source of the right-hand
  // side so that no register carries a value merged from two paths
  auto run = [&](auto ev, auto pl) __attribute__((always_inline)) {
    if constexpr (!decltype(ev)::value) {
      for (int s = 1; s <= m; ++s) step(s, ga, ev, pl);
    } else {
      int s = 1;
      for (; s + 1 <= m; s += 2) {
        step(s, ga, ev, pl);
        step(s + 1, gb, ev, pl);
      }
      if (s == m) step(s, ga, ev, pl);
    }
  };
  if (!every) run(std::false_type{}, std::false_type{});
  else if (preload) run(std::true_type{}, std::true_type{});
  else run(std::true_type{}, std::false_type{});
  finish_extent<T, K, HALF>(a, j, blk, X, eout, sh, x, stg, red);
}

template <typename T, int K, int W, bool IO>
__global__ void __launch_bounds__(512) k_stencil(RelaxArgs a) {
  stencil_body<T, K, W, IO>(a, (int)blockIdx.x);
}

template <typename T, int K, int W, bool IO>
__global__ void __launch_bounds__(512) k_stencil_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  stencil_body<T, K, W, IO>(a, blk);
}

// ---------------------------------------------------------------------------
// Generic: any n_x, any tap list (offsets in [0, n_x)); state in LDS
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void generic_body(const RelaxArgs& a, const int j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int nx = a.nx, m = a.m, NT = blockDim.x, tid = threadIdx.x;
  T* cur = reinterpret_cast<T*>(smem_raw);
  T* nxt = cur + nx;
  for (int p = tid; p < nx; p += NT) {
    double v = 0.0;
    if (!a.zero_in) {
      v = a.in[(long long)j * a.in_stride * nx + p];
      if (a.corr) v += a.corr[(long long)j * a.corr_stride * nx + p];
      if (a.sub) v -= a.sub[(long long)j * nx + p];
      if (a.sub2) v -= a.sub2[(long long)j * nx + p];
    }
    if (a.mode == MODE_F) a.out[(long long)j * m * nx + p] = v;
    else if (a.mode == MODE_FC && a.write_row0 && j == 0) a.out[p] = v;
    cur[p] = (T)v;
  }
  if (a.mode == MODE_F && j == a.nint) return;
  __syncthreads();
  for (int s = 1; s <= m; ++s) {
    const double* g = (a.rhs_mode == RHS_EVERY) ? a.rhs + ((long long)j * m + s) * nx : nullptr;
    for (int p = tid; p < nx; p += NT) {
      T acc = (T)0;
      for (int t = 0; t < a.ntaps; ++t) {
        int q = p - a.tap_off[t];
        q += (q < 0) ? nx : 0;
        acc = fma((T)a.taps[t], cur[q], acc);
      }
      if (g) acc += (T)g[p];
      nxt[p] = acc;
      if (a.mode == MODE_F && (s < m || a.write_last))
        a.out[((long long)j * m + s) * nx + p] = (double)acc;
    }
    __syncthreads();
    T* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (a.mode == MODE_FC) {
    const double* gc = (a.rhs_mode == RHS_CPOINT) ? a.rhs + (long long)(j + 1) * nx : nullptr;
    double ss = 0.0;
    for (int p = tid; p < nx; p += NT) {
      double v = (double)cur[p];
      if (gc) v += gc[p];
      a.out[(long long)(j + a.out_off) * nx + p] = v;
      ss += v * v;
      if (a.delta) {
        double u = a.zero_in ? 0.0 : a.in[(long long)(j + 1) * a.in_stride * nx + p];
        if (a.corr) u += a.corr[(long long)(j + 1) * a.corr_stride * nx + p];
        a.delta[(long long)(j + 1) * nx + p] = v - u;
        if (j == 0) a.delta[p] = 0.0;
      }
    }
    if (a.partial) {
      const double s = block_sum(ss, red);
      if (tid == 0) a.partial[j] = s;
    }
  } else if (a.mode == MODE_RES) {
    const double* gc = (a.rhs_mode == RHS_CPOINT) ? a.rhs + (long long)(j + 1) * nx : nullptr;
    double ss = 0.0;
    for (int p = tid; p < nx; p += NT) {
      double v = (double)cur[p];
      if (gc) v += gc[p];
      v -= a.ref[(long long)(j + 1) * nx + p];
      a.out[(long long)(j + 1) * nx + p] = v;
      if (j == 0) a.out[p] = 0.0;
      ss += v * v;
    }
    if (a.partial) {
      const double s = block_sum(ss, red);
      if (tid == 0) a.partial[j] = s;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_generic(RelaxArgs a) {
  generic_body<T>(a, (int)blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_generic_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  generic_body<T>(a, blk);
}

}  // namespace mgr
