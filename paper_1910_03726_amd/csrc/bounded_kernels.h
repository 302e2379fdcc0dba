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

__global__ void __launch_bounds__(256) k_bounded(RelaxArgs a) { bounded_body(a, (int)blockIdx.x); }

__global__ void __launch_bounds__(256) k_bounded_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  bounded_body(a, blk);
}

}  // namespace mgr
