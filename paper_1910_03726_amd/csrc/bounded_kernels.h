// Relaxation kernel for levels with inflow/outflow boundaries (Sec. 4.5).
//
// Phi is no longer circulant: rows near x = -1 and x = 1 carry the boundary
// closures, the coarse operators are the periodic Psi truncated to the
// interval, and every fine step adds the inflow forcing of its time.  The
// kernel keeps one interval's state in LDS (two n_x buffers, FP64) and
// applies the operator of BoundedDev (common.h) point by point: consecutive
// threads own consecutive points, so tap reads from LDS are conflict-free.
// Launch arguments and outputs are those of the periodic kernels
// (RelaxArgs, relax_kernels.h), with `opdata` the level's BoundedDev,
// signed offsets in `tap_off` and `omin` the fine steps between the start
// times of consecutive blocks.
#pragma once

#include "relax_kernels.h"

namespace mgr {

__device__ __forceinline__ double bounded_row(const BoundedDev& bd, const double* __restrict__ taps,
                                              const int* __restrict__ off, int ntaps,
                                              const double* cur, int p, int nx) {
  double acc = 0.0;
  if (p < bd.nl) {
    const double* row = bd.lblk + (long long)p * bd.ncl;
    for (int c = 0; c < bd.ncl; ++c) acc = fma(row[c], cur[c], acc);
  } else if (p >= nx - bd.nr) {
    const double* row = bd.rblk + (long long)(p - (nx - bd.nr)) * bd.ncr;
    const double* src = cur + (nx - bd.ncr);
    for (int c = 0; c < bd.ncr; ++c) acc = fma(row[c], src[c], acc);
  } else {
    for (int t = 0; t < ntaps; ++t) {
      const int q = p - off[t];
      if (q >= 0 && q < nx) acc = fma(taps[t], cur[q], acc);
    }
  }
  return acc;
}

__device__ __forceinline__ void bounded_body(const RelaxArgs& a, const int j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const BoundedDev bd = *reinterpret_cast<const BoundedDev*>(a.opdata);
  const int nx = a.nx, m = a.m, NT = blockDim.x, tid = threadIdx.x;
  double* cur = reinterpret_cast<double*>(smem_raw);
  double* nxt = cur + nx;
  for (int p = tid; p < nx; p += NT) {
    double v = 0.0;
    if (!a.zero_in) {
      v = a.in[(long long)j * a.in_stride * nx + p];
      if (a.corr) v += a.corr[(long long)j * a.corr_stride * nx + p];
    }
    if (a.mode == MODE_F) a.out[(long long)j * m * nx + p] = v;
    else if (a.mode == MODE_FC && a.write_row0 && j == 0) a.out[p] = v;
    cur[p] = v;
  }
  if (a.mode == MODE_F && j == a.nint) return;
  __syncthreads();
  for (int s = 1; s <= m; ++s) {
    const double* g = (a.rhs_mode == RHS_EVERY) ? a.rhs + ((long long)j * m + s) * nx : nullptr;
    const double* f = bd.F ? bd.F + ((long long)j * a.omin + s - 1) * bd.nf : nullptr;
    for (int p = tid; p < nx; p += NT) {
      double acc = bounded_row(bd, a.taps, a.tap_off, a.ntaps, cur, p, nx);
      if (f && p < bd.nf) acc += f[p];
      if (g) acc += g[p];
      nxt[p] = acc;
      if (a.mode == MODE_F && (s < m || a.write_last))
        a.out[((long long)j * m + s) * nx + p] = acc;
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (a.mode == MODE_FC) {
    const double* gc = (a.rhs_mode == RHS_CPOINT) ? a.rhs + (long long)(j + 1) * nx : nullptr;
    double ss = 0.0;
    for (int p = tid; p < nx; p += NT) {
      double v = cur[p];
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
      double v = cur[p];
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

// Register-blocked variant.  Thread t owns chunks of K consecutive points;
// the truncated stencil is a dense window of W weights, c[i] the weight of
// offset omax - i (tap_off[0] = omax, taps = the W weights), so
// out_{b+k} = sum_i c[i] u_{b - omax + k + i} with u = 0 off the grid (the
// truncation).  A chunk reads its K + W - 1 inputs from LDS once into
// registers (zero where the window leaves the grid).  K is odd, so lanes
// whose chunks start K doubles apart read distinct LDS banks.  The dense
// boundary rows of the fine level are staged in LDS at the start and
// computed one row per thread.  Right-hand side rows and the inflow
// forcing are loaded before the arithmetic that precedes their use.
// LDS: state and next state (2 n_x), then the left and right blocks.
template <int K, int W>
__device__ __forceinline__ void bounded_tiled_body(const RelaxArgs& a, const int j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const BoundedDev bd = *reinterpret_cast<const BoundedDev*>(a.opdata);
  const int nx = a.nx, m = a.m, NT = blockDim.x, tid = threadIdx.x;
  const int omax = a.tap_off[0];
  const int nch = (nx + K - 1) / K;
  double* cur = reinterpret_cast<double*>(smem_raw);
  double* nxt = cur + nx;
  double* lb = nxt + nx;
  double* rb = lb + bd.nl * bd.ncl;
  for (int q = tid; q < bd.nl * bd.ncl; q += NT) lb[q] = bd.lblk[q];
  for (int q = tid; q < bd.nr * bd.ncr; q += NT) rb[q] = bd.rblk[q];
  for (int p = tid; p < nx; p += NT) {
    double v = 0.0;
    if (!a.zero_in) {
      v = a.in[(long long)j * a.in_stride * nx + p];
      if (a.corr) v += a.corr[(long long)j * a.corr_stride * nx + p];
    }
    if (a.mode == MODE_F) a.out[(long long)j * m * nx + p] = v;
    else if (a.mode == MODE_FC && a.write_row0 && j == 0) a.out[p] = v;
    cur[p] = v;
  }
  if (a.mode == MODE_F && j == a.nint) return;
  __syncthreads();
  constexpr bool kHold = W <= 12;
  double c[kHold ? W : 1];
  if constexpr (kHold) {
#pragma unroll
    for (int i = 0; i < W; ++i) c[i] = a.taps[i];
  }
  // boundary row of this thread (fine level), or -1
  const int brow = tid < bd.nl ? tid : (tid < bd.nl + bd.nr ? nx - bd.nr + (tid - bd.nl) : -1);
  const double* Fb = bd.F ? bd.F + (long long)j * a.omin * bd.nf : nullptr;
  double fnext = (Fb && brow >= 0 && brow < bd.nf && m >= 1) ? Fb[brow] : 0.0;
  for (int s = 1; s <= m; ++s) {
    const double* g = (a.rhs_mode == RHS_EVERY) ? a.rhs + ((long long)j * m + s) * nx : nullptr;
    const bool store = a.mode == MODE_F && (s < m || a.write_last);
    double* orow = store ? a.out + ((long long)j * m + s) * nx : nullptr;
    const double fcur = fnext;
    if (Fb && brow >= 0 && brow < bd.nf && s < m) fnext = Fb[(long long)s * bd.nf + brow];
    for (int ch = tid; ch < nch; ch += NT) {
      const int b = ch * K;
      double gv[K];
#pragma unroll
      for (int k = 0; k < K; ++k) gv[k] = (g && b + k < nx) ? g[b + k] : 0.0;
      // stream the K + W - 1 window values: value i feeds out_k with
      // weight c[i - k]
      double acc[K];
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = 0.0;
      const int w0 = b - omax;
#pragma unroll
      for (int i = 0; i < K + W - 1; ++i) {
        const int q = w0 + i;
        const double v = (unsigned)q < (unsigned)nx ? cur[q] : 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (i - k >= 0 && i - k < W)
            acc[k] = fma(kHold ? c[kHold ? i - k : 0] : a.taps[i - k], v, acc[k]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int p = b + k;
        if (p < nx && p >= bd.nl && p < nx - bd.nr) {
          const double o = acc[k] + gv[k];
          nxt[p] = o;
          if (orow) orow[p] = o;
        }
      }
    }
    if (brow >= 0) {
      double acc = 0.0;
      if (brow < bd.nl) {
        const double* row = lb + brow * bd.ncl;
#pragma unroll 4
        for (int q = 0; q < bd.ncl; ++q) acc = fma(row[q], cur[q], acc);
      } else {
        const double* row = rb + (brow - (nx - bd.nr)) * bd.ncr;
        const double* src = cur + (nx - bd.ncr);
#pragma unroll 4
        for (int q = 0; q < bd.ncr; ++q) acc = fma(row[q], src[q], acc);
      }
      if (brow < bd.nf) acc += fcur;
      if (g) acc += g[brow];
      nxt[brow] = acc;
      if (orow) orow[brow] = acc;
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (a.mode == MODE_FC) {
    const double* gc = (a.rhs_mode == RHS_CPOINT) ? a.rhs + (long long)(j + 1) * nx : nullptr;
    double ss = 0.0;
    for (int p = tid; p < nx; p += NT) {
      double v = cur[p];
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
      double v = cur[p];
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

__global__ void __launch_bounds__(256) k_bounded(RelaxArgs a) { bounded_body(a, (int)blockIdx.x); }

__global__ void __launch_bounds__(256) k_bounded_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  bounded_body(a, blk);
}

template <int K, int W>
__global__ void __launch_bounds__(512) k_bounded_tiled(RelaxArgs a) {
  bounded_tiled_body<K, W>(a, (int)blockIdx.x);
}

template <int K, int W>
__global__ void __launch_bounds__(512) k_bounded_tiled_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  bounded_tiled_body<K, W>(a, blk);
}

}  // namespace mgr

