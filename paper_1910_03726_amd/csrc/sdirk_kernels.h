// SDIRK relaxation kernel of libmgrit for CDNA4 (gfx950): the stage
// matrices of an SDIRK stepper (Appendix A, Table 8) applied through cyclic
// linear recurrences evaluated by exact chunked scans over lanes.
#pragma once

#include "relax_kernels.h"

namespace mgr {

// ---------------------------------------------------------------------------
// SDIRK: cyclic banded stage solves by chunked recurrence scans
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mat2_mul_d(const double* a, const double* b, double* c) {
  const double r0 = a[0] * b[0] + a[1] * b[2], r1 = a[0] * b[1] + a[1] * b[3];
  const double r2 = a[2] * b[0] + a[3] * b[2], r3 = a[2] * b[1] + a[3] * b[3];
  c[0] = r0; c[1] = r1; c[2] = r2; c[3] = r3;
}

// H^e from the table Hp[d] = H^(2^d), e < 2048.
__device__ __forceinline__ void mat2_pow_tab(const RecDev& f, int e, double* out) {
  double r[4] = {1.0, 0.0, 0.0, 1.0};
  for (int d = 0; d < 11; ++d)
    if (e & (1 << d)) mat2_mul_d(r, f.Hp[d], r);
  out[0] = r[0]; out[1] = r[1]; out[2] = r[2]; out[3] = r[3];
}

// y <- (recurrence f)^{-1} y over the whole periodic line (K points per
// lane, NL lanes).  Pw = H^(lv+1) and Pl = H^v (I - H^NL)^{-1} for this
// lane's virtual index v (v = lane forward, NL-1-lane backward).
template <typename T, int K>
__device__ __forceinline__ void rec_apply(T (&y)[K], const RecDev& f, const T (&Pw)[4],
                                          const T (&Pl)[4], T* scan, int NL) {
  const int dir = f.dir;
  const int lane = threadIdx.x;
  const int v = dir > 0 ? lane : NL - 1 - lane;
  const int lv = v & 63, wv = v >> 6, nw = NL >> 6;
  const T a1 = (T)f.a1, a2 = (T)f.a2;
  // 1. zero-carry local pass: end state (y_last, y_last-1)
  T y1 = (T)0, y2 = (T)0;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int k = dir > 0 ? kk : K - 1 - kk;
    const T nv = y[k] + a1 * y1 + a2 * y2;
    y2 = y1;
    y1 = nv;
  }
  // 2. inclusive scan of the affine carries inside the wavefront
  T I1 = y1, I2 = y2;
#pragma unroll
  for (int dd = 0; dd < 6; ++dd) {
    const int d = 1 << dd;
    const int sv = lv >= d ? lv - d : lv;
    const int sp = dir > 0 ? sv : 63 - sv;
    const T o1 = __shfl(I1, sp, 64), o2 = __shfl(I2, sp, 64);
    if (lv >= d) {
      const double* H = f.Hp[dd];
      const T n1 = I1 + (T)H[0] * o1 + (T)H[1] * o2;
      const T n2 = I2 + (T)H[2] * o1 + (T)H[3] * o2;
      I1 = n1;
      I2 = n2;
    }
  }
  // 3. wavefront totals
  if (lv == 63) {
    scan[2 * wv] = I1;
    scan[2 * wv + 1] = I2;
  }
  __syncthreads();
  // 4. carry into this wavefront (Q) and the total over all lanes (Tt)
  const double* H64 = f.Hp[6];
  T Q1 = (T)0, Q2 = (T)0, T1 = (T)0, T2 = (T)0;
  for (int w = 0; w < nw; ++w) {
    if (w == wv) {
      Q1 = T1;
      Q2 = T2;
    }
    const T n1 = (T)H64[0] * T1 + (T)H64[1] * T2 + scan[2 * w];
    const T n2 = (T)H64[2] * T1 + (T)H64[3] * T2 + scan[2 * w + 1];
    T1 = n1;
    T2 = n2;
  }
  // 5. global inclusive value of this lane, 6. exclusive via the left lane
  const T G1 = I1 + Pw[0] * Q1 + Pw[1] * Q2;
  const T G2 = I2 + Pw[2] * Q1 + Pw[3] * Q2;
  const int sv = lv >= 1 ? lv - 1 : lv;
  const int sp = dir > 0 ? sv : 63 - sv;
  T P1 = __shfl(G1, sp, 64), P2 = __shfl(G2, sp, 64);
  if (lv == 0) {
    P1 = Q1;
    P2 = Q2;
  }
  // 7. periodic closure, 8. rerun the recurrence from the true carry
  y1 = P1 + Pl[0] * T1 + Pl[1] * T2;
  y2 = P2 + Pl[2] * T1 + Pl[3] * T2;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int k = dir > 0 ? kk : K - 1 - kk;
    const T nv = y[k] + a1 * y1 + a2 * y2;
    y2 = y1;
    y1 = nv;
    y[k] = nv;
  }
}

// Dynamic LDS: the staging area (stage_doubles(n_x, K) doubles).
template <typename T, int K, int S, int NF>
__device__ __forceinline__ void sdirk_body(const RelaxArgs& a, const int j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ T scan[2][32];
  __shared__ double red[16];
  const SdirkDev* sd = reinterpret_cast<const SdirkDev*>(a.sdirk);
  const int NL = blockDim.x, lane = threadIdx.x, nx = a.nx, m = a.m;
  const Stager<K> St{reinterpret_cast<double*>(smem_raw), nx, NL, lane};

  double v0[K];
  start_state<K>(a, j, St, v0);
  if (a.mode == MODE_F) {
    St.store(a.out + (long long)j * m * nx, 0, v0);
    if (j == a.nint) return;
  } else if (a.mode == MODE_FC && a.write_row0 && j == 0) {
    St.store(a.out, 0, v0);
  }
  // per-lane scan matrices of each factor
  T Pw[NF][4], Pl[NF][4];
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const RecDev& f = sd->f[q];
    const int v = f.dir > 0 ? lane : NL - 1 - lane;
    double hw[4], hv[4], pl[4];
    mat2_pow_tab(f, (v & 63) + 1, hw);
    mat2_pow_tab(f, v, hv);
    mat2_mul_d(hv, f.Cinv, pl);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Pw[q][i] = (T)hw[i];
      Pl[q][i] = (T)pl[i];
    }
  }
  const T scale = (T)sd->scale, ig = (T)sd->inv_gamma;
  T u[K];
#pragma unroll
  for (int k = 0; k < K; ++k) u[k] = (T)v0[k];
  T ks[S > 1 ? S - 1 : 1][K];
  int call = 0;
  for (int s = 1; s <= m; ++s) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      // stage i: rhs = u + sum_{l<i} a_il dt L Y_l;  Y = M^{-1} rhs
      T r[K], y[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        T acc = u[k];
#pragma unroll
        for (int l = 0; l < i; ++l) acc += (T)sd->A[i][l] * ks[l][k];
        r[k] = acc;
        y[k] = acc * scale;
      }
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        rec_apply<T, K>(y, sd->f[q], Pw[q], Pl[q], &scan[call & 1][0], NL);
        ++call;
      }
      if (i < S - 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) ks[i][k] = (y[k] - r[k]) * ig;  // dt L Y_i
      } else {
        // stiffly accurate (b = last row of A): u^{n+1} = Y_s
#pragma unroll
        for (int k = 0; k < K; ++k) u[k] = y[k];
      }
    }
    if (a.rhs_mode == RHS_EVERY) {
      T g[K];
      St.load(a.rhs + ((long long)j * m + s) * nx, 0, g);
#pragma unroll
      for (int k = 0; k < K; ++k) u[k] += g[k];
    }
    if (a.mode == MODE_F && (s < m || a.write_last))
      St.store(a.out + ((long long)j * m + s) * nx, 0, u);
  }
  finish<T, K>(a, j, St, 0, u, red);
}

template <typename T, int K, int S, int NF>
__global__ void __launch_bounds__(512) k_sdirk(RelaxArgs a) {
  sdirk_body<T, K, S, NF>(a, (int)blockIdx.x);
}

template <typename T, int K, int S, int NF>
__global__ void __launch_bounds__(512) k_sdirk_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  sdirk_body<T, K, S, NF>(a, blk);
}

}  // namespace mgr
