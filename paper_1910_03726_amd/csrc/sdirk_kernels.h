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

// DPP move of v by control CTRL (row / wave shifts); lanes without a
// source keep `old` (no bound control).
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float old, float v) {
  return __int_as_float(dpp_mov<CTRL>(__float_as_int(old), __float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double old, double v) {
  return __hiloint2double(dpp_mov<CTRL>(__double2hiint(old), __double2hiint(v)),
                          dpp_mov<CTRL>(__double2loint(old), __double2loint(v)));
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// One Hillis-Steele step of the affine carry scan inside 16-lane rows:
// combine with the value d lanes back in the recurrence's direction
// (row_shr for forward, row_shl for backward recurrences).
template <typename T, int D>
__device__ __forceinline__ void row_scan_step(T& I1, T& I2, bool fwd, int r16, const double* H) {
  const T o1 = fwd ? dpp_mov<0x110 + D>(I1, I1) : dpp_mov<0x100 + D>(I1, I1);
  const T o2 = fwd ? dpp_mov<0x110 + D>(I2, I2) : dpp_mov<0x100 + D>(I2, I2);
  if (r16 >= D) {
    const T n1 = I1 + (T)H[0] * o1 + (T)H[1] * o2;
    const T n2 = I2 + (T)H[2] * o1 + (T)H[3] * o2;
    I1 = n1;
    I2 = n2;
  }
}

// y <- (recurrence f)^{-1} y over the whole periodic line (K points per
// lane, NL lanes).  Pw = H^(lv+1), Pr = H^(r+1) (r: position in its 16-lane
// row) and Pl = H^v (I - H^NL)^{-1} for this lane's virtual index v (v =
// lane forward, NL-1-lane backward).  Inside a wavefront the carries are
// scanned with DPP row shifts and the row totals read from their lanes, so
// only the step across wavefronts goes through LDS.
template <typename T, int K>
__device__ __forceinline__ void rec_apply(T (&y)[K], const RecDev& f, const T (&Pw)[4],
                                          const T (&Pr)[4], const T (&Pl)[4], T* scan, int NL) {
  const int dir = f.dir;
  const bool fwd = dir > 0;
  const int lane = threadIdx.x;
  const int v = fwd ? lane : NL - 1 - lane;
  const int lv = v & 63, wv = v >> 6, nw = NL >> 6;
  const int r16 = lv & 15, q = lv >> 4;  // virtual position in its row, virtual row
  const T a1 = (T)f.a1, a2 = (T)f.a2;
  // 1. zero-carry local pass: end state (y_last, y_last-1)
  T y1 = (T)0, y2 = (T)0;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int k = fwd ? kk : K - 1 - kk;
    const T nv = y[k] + a1 * y1 + a2 * y2;
    y2 = y1;
    y1 = nv;
  }
  // 2. inclusive scan of the affine carries inside the wavefront: rows of
  // 16 lanes by DPP, then the totals of the rows before
  T I1 = y1, I2 = y2;
  row_scan_step<T, 1>(I1, I2, fwd, r16, f.Hp[0]);
  row_scan_step<T, 2>(I1, I2, fwd, r16, f.Hp[1]);
  row_scan_step<T, 4>(I1, I2, fwd, r16, f.Hp[2]);
  row_scan_step<T, 8>(I1, I2, fwd, r16, f.Hp[3]);
  {
    // virtual row t ends at lane 16 t + 15 (forward) or 48 - 16 t (backward)
    const T e01 = lane_value(I1, fwd ? 15 : 48), e02 = lane_value(I2, fwd ? 15 : 48);
    const T e11 = lane_value(I1, fwd ? 31 : 32), e12 = lane_value(I2, fwd ? 31 : 32);
    const T e21 = lane_value(I1, fwd ? 47 : 16), e22 = lane_value(I2, fwd ? 47 : 16);
    const double* H16 = f.Hp[4];
    // carries into rows 1, 2, 3
    const T c11 = e01, c12 = e02;
    const T c21 = e11 + (T)H16[0] * c11 + (T)H16[1] * c12;
    const T c22 = e12 + (T)H16[2] * c11 + (T)H16[3] * c12;
    const T c31 = e21 + (T)H16[0] * c21 + (T)H16[1] * c22;
    const T c32 = e22 + (T)H16[2] * c21 + (T)H16[3] * c22;
    if (q > 0) {
      const T C1 = q == 1 ? c11 : (q == 2 ? c21 : c31);
      const T C2 = q == 1 ? c12 : (q == 2 ? c22 : c32);
      const T n1 = I1 + Pr[0] * C1 + Pr[1] * C2;
      const T n2 = I2 + Pr[2] * C1 + Pr[3] * C2;
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
  // 5. global inclusive value of this lane, 6. exclusive via the previous
  // lane in the recurrence's direction (the first lane takes Q)
  const T G1 = I1 + Pw[0] * Q1 + Pw[1] * Q2;
  const T G2 = I2 + Pw[2] * Q1 + Pw[3] * Q2;
  const T P1 = fwd ? dpp_mov<0x138>(Q1, G1) : dpp_mov<0x130>(Q1, G1);
  const T P2 = fwd ? dpp_mov<0x138>(Q2, G2) : dpp_mov<0x130>(Q2, G2);
  // 7. periodic closure, 8. rerun the recurrence from the true carry
  y1 = P1 + Pl[0] * T1 + Pl[1] * T2;
  y2 = P2 + Pl[2] * T1 + Pl[3] * T2;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int k = fwd ? kk : K - 1 - kk;
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
  const SdirkDev* sd = reinterpret_cast<const SdirkDev*>(a.opdata);
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
  T Pw[NF][4], Pr[NF][4], Pl[NF][4];
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const RecDev& f = sd->f[q];
    const int v = f.dir > 0 ? lane : NL - 1 - lane;
    double hw[4], hr[4], hv[4], pl[4];
    mat2_pow_tab(f, (v & 63) + 1, hw);
    mat2_pow_tab(f, (v & 15) + 1, hr);
    mat2_pow_tab(f, v, hv);
    mat2_mul_d(hv, f.Cinv, pl);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Pw[q][i] = (T)hw[i];
      Pr[q][i] = (T)hr[i];
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
        rec_apply<T, K>(y, sd->f[q], Pw[q], Pr[q], Pl[q], &scan[call & 1][0], NL);
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
