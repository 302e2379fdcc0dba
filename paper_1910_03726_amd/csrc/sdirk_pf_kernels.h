// SDIRK relaxation kernel of libmgrit in partial-fraction form (SdirkPfDev,
// common.h): every stage solve M Y = rhs (Appendix A, Table 8; M = I -
// gamma dt L circulant, Corollary 1) is
//     Y = c0 rhs + sum_t A_t (I - q_t X_t)^{-1} rhs,
// a sum of first-order periodic recurrences on the same right-hand side.
// Each lane owns K consecutive points; per stage all terms run their
// zero-carry local pass, their chunk carries are scanned together (DPP
// row shifts inside the wavefront, one LDS exchange and one barrier across
// wavefronts), closed periodically, and each term is rerun from its true
// carry straight into the sum.  Compared with the factored form
// (sdirk_kernels.h) a stage costs one scan instead of one per factor, and
// every carry is a scalar (or a complex number for a conjugate pair)
// instead of a 2 x 2 transfer.
#pragma once

#include "sdirk_kernels.h"

namespace mgr {

// x + y * z for complex values held as (re, im) pairs
template <typename T>
__device__ __forceinline__ void cfma(T& xr, T& xi, T yr, T yi, T zr, T zi) {
  const T r = xr + yr * zr - yi * zi;
  const T i = xi + yr * zi + yi * zr;
  xr = r;
  xi = i;
}

// (re, im) of Q^e from the table Qp[d] = Q^(2^d), e < 2048, in FP64
__device__ __forceinline__ void cpow_tab(const double (*Qp)[2], int e, double& pr, double& pi) {
  double r = 1.0, i = 0.0;
#pragma unroll
  for (int d = 0; d < 11; ++d)
    if (e & (1 << d)) {
      const double nr = r * Qp[d][0] - i * Qp[d][1];
      const double ni = r * Qp[d][1] + i * Qp[d][0];
      r = nr;
      i = ni;
    }
  pr = r;
  pi = i;
}

// The value 2^d lanes back in term t's direction inside 16-lane rows (DPP
// row_shr for forward terms, row_shl for backward ones; lanes without a
// source get their own value, which the caller weights by zero).
template <typename T, int NR, int NB>
__device__ __forceinline__ T pf_row_shift(int t, int d, T v) {
  const bool fw = t < NR - NB || t >= NR;
  switch (d) {
    case 0: return fw ? dpp_mov<0x111>(v, v) : dpp_mov<0x101>(v, v);
    case 1: return fw ? dpp_mov<0x112>(v, v) : dpp_mov<0x102>(v, v);
    case 2: return fw ? dpp_mov<0x114>(v, v) : dpp_mov<0x104>(v, v);
    default: return fw ? dpp_mov<0x118>(v, v) : dpp_mov<0x108>(v, v);
  }
}

// Terms in the order the setup stores them: NR - NB forward real terms,
// NB backward real terms, NC forward complex terms (a conjugate pair each),
// so that every term's direction is known at compile time.
template <int NR, int NB>
__device__ __forceinline__ constexpr bool pf_fwd(int t) { return t < NR - NB || t >= NR; }

template <typename T, int K, int S, int NR, int NB, int NC>
__device__ __forceinline__ void sdirk_pf_body(const RelaxArgs& a, const int j) {
  constexpr int NT = NR + NC;       // terms
  constexpr int NV = NR + 2 * NC;   // carry values per lane
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ T scan[2][8][NV];      // wavefront totals, double buffered
  __shared__ double red[16];
  const SdirkPfDev* sd = reinterpret_cast<const SdirkPfDev*>(a.opdata);
  const int NL = blockDim.x, lane = threadIdx.x, nx = a.nx, m = a.m;
  const int nw = NL >> 6;
  const Stager<K> St{reinterpret_cast<double*>(smem_raw), nx, NL, lane};

  double v0[K];
  start_state<K>(a, j, St, v0);
  if (a.mode == MODE_F) {
    St.store(a.out + (long long)j * m * nx, 0, v0);
    if (j == a.nint) return;
  } else if (a.mode == MODE_FC && a.write_row0 && j == 0) {
    St.store(a.out, 0, v0);
  }
  // per-term lane constants: Pw = Q^(lv+1), Pr = Q^(r16+1), Pl = Q^v close
  // (v the lane's index in the term's direction, lv and r16 its position in
  // the wavefront and in its 16-lane row)
  T Pw[NT][2], Pr[NT][2], Pl[NT][2];
  bool fwd[NT];
  int r16[NT], rq[NT], lv[NT], wv[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const PfTermDev& f = sd->t[t];
    fwd[t] = pf_fwd<NR, NB>(t);
    const int v = fwd[t] ? lane : NL - 1 - lane;
    lv[t] = v & 63;
    wv[t] = v >> 6;
    r16[t] = v & 15;
    rq[t] = lv[t] >> 4;
    double pr, pi, hr, hi, wr, wi;
    cpow_tab(f.Qp, lv[t] + 1, wr, wi);
    cpow_tab(f.Qp, r16[t] + 1, hr, hi);
    cpow_tab(f.Qp, v, pr, pi);
    Pw[t][0] = (T)wr;
    Pw[t][1] = (T)wi;
    Pr[t][0] = (T)hr;
    Pr[t][1] = (T)hi;
    Pl[t][0] = (T)(pr * f.close[0] - pi * f.close[1]);
    Pl[t][1] = (T)(pr * f.close[1] + pi * f.close[0]);
  }
  // every constant of the step in registers before the step loop
  T cq[NT][2], ca[NT][2], cQ[NT][5][2], cH[NT][2];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const PfTermDev& f = sd->t[t];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      cq[t][c] = (T)f.q[c];
      ca[t][c] = (T)f.a[c];
      cH[t][c] = (T)f.Qp[6][c];  // Q^64
#pragma unroll
      for (int d = 0; d < 5; ++d) cQ[t][d][c] = (T)f.Qp[d][c];  // Q^(2^d)
    }
  }
  T cA[S][S];
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int l = 0; l < S; ++l) cA[i][l] = (T)sd->A[i][l];
  const T c0 = (T)sd->c0, ig = (T)sd->inv_gamma;
  T u[K];
#pragma unroll
  for (int k = 0; k < K; ++k) u[k] = (T)v0[k];
  T ks[S > 1 ? S - 1 : 1][K];
  int call = 0;
  for (int s = 1; s <= m; ++s) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      // stage i: rhs = u + sum_{l<i} a_il dt L Y_l;  Y = M^{-1} rhs
      T r[K], acc[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        T x = u[k];
#pragma unroll
        for (int l = 0; l < i; ++l) x += cA[i][l] * ks[l][k];
        r[k] = x;
        acc[k] = c0 * x;
      }
      // 1. zero-carry local passes of all terms, interleaved (independent
      // chains): each term's end value (I0, I1)
      T I0[NT], I1[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        I0[t] = (T)0;
        I1[t] = (T)0;
      }
#pragma unroll
      for (int kk = 0; kk < K; ++kk)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int k = pf_fwd<NR, NB>(t) ? kk : K - 1 - kk;
          if (t < NR) {
            I0[t] = r[k] + cq[t][0] * I0[t];
          } else {
            const T n0 = r[k] + cq[t][0] * I0[t] - cq[t][1] * I1[t];
            I1[t] = cq[t][0] * I1[t] + cq[t][1] * I0[t];
            I0[t] = n0;
          }
        }
      // 2. inclusive carry scan inside the wavefront: rows of 16 lanes by
      // DPP (lanes without a source D lanes back add nothing: a zero
      // coefficient, so no branch), then the totals of the rows before
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        T o0[NT], o1[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          o0[t] = pf_row_shift<T, NR, NB>(t, d, I0[t]);
          o1[t] = t >= NR ? pf_row_shift<T, NR, NB>(t, d, I1[t]) : (T)0;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const bool on = r16[t] >= (1 << d);
          const T m0 = on ? cQ[t][d][0] : (T)0;
          if (t < NR) {
            I0[t] = fma(m0, o0[t], I0[t]);
          } else {
            const T m1 = on ? cQ[t][d][1] : (T)0;
            cfma<T>(I0[t], I1[t], m0, m1, o0[t], o1[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bool fw = pf_fwd<NR, NB>(t);
        // virtual row b ends at lane 16 b + 15 (forward) or 48 - 16 b (backward)
        const T e00 = lane_value(I0[t], fw ? 15 : 48);
        const T e10 = lane_value(I0[t], fw ? 31 : 32);
        const T e20 = lane_value(I0[t], fw ? 47 : 16);
        const T h0 = cQ[t][4][0];
        const T pm0 = rq[t] > 0 ? Pr[t][0] : (T)0;  // row 0 takes no carry
        if (t >= NR) {
          const T e01 = lane_value(I1[t], fw ? 15 : 48);
          const T e11 = lane_value(I1[t], fw ? 31 : 32);
          const T e21 = lane_value(I1[t], fw ? 47 : 16);
          const T h1 = cQ[t][4][1];
          T c2r = e10, c2i = e11;
          cfma<T>(c2r, c2i, h0, h1, e00, e01);
          T c3r = e20, c3i = e21;
          cfma<T>(c3r, c3i, h0, h1, c2r, c2i);
          T Cr = e00, Ci = e01;
          Cr = rq[t] >= 2 ? c2r : Cr;
          Ci = rq[t] >= 2 ? c2i : Ci;
          Cr = rq[t] >= 3 ? c3r : Cr;
          Ci = rq[t] >= 3 ? c3i : Ci;
          const T pm1 = rq[t] > 0 ? Pr[t][1] : (T)0;
          cfma<T>(I0[t], I1[t], pm0, pm1, Cr, Ci);
        } else {
          const T c2 = e10 + h0 * e00;
          const T c3 = e20 + h0 * c2;
          T C = e00;
          C = rq[t] >= 2 ? c2 : C;
          C = rq[t] >= 3 ? c3 : C;
          I0[t] = fma(pm0, C, I0[t]);
        }
      }
      // 3. wavefront totals of every term through LDS, one barrier
      {
        T(*buf)[NV] = scan[call & 1];
        int vi = 0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if (lv[t] == 63) {
            buf[wv[t]][vi] = I0[t];
            if (t >= NR) buf[wv[t]][vi + 1] = I1[t];
          }
          vi += t >= NR ? 2 : 1;
        }
      }
      __syncthreads();
      // 4. carry into this wavefront (Q) and total over all lanes (Tt) of
      // every term, from the totals stored by virtual wavefront index (the
      // loop unrolled to the largest workgroup, 8 wavefronts, so that all
      // LDS reads issue together)
      T Q0[NT], Q1[NT], T0[NT], T1[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        Q0[t] = Q1[t] = T0[t] = T1[t] = (T)0;
      }
      {
        T(*buf)[NV] = scan[call & 1];
#pragma unroll
        for (int w = 0; w < 8; ++w) {
          if (w < nw) {
            T b[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) b[v] = buf[w][v];
            int vi = 0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              const bool mine = w == wv[t];
              Q0[t] = mine ? T0[t] : Q0[t];
              Q1[t] = mine ? T1[t] : Q1[t];
              if (t >= NR) {
                T n0 = b[vi], n1 = b[vi + 1];
                cfma<T>(n0, n1, cH[t][0], cH[t][1], T0[t], T1[t]);
                T0[t] = n0;
                T1[t] = n1;
              } else {
                T0[t] = b[vi] + cH[t][0] * T0[t];
              }
              vi += t >= NR ? 2 : 1;
            }
          }
        }
      }
      // 5. global inclusive value; 6. exclusive via the previous lane in the
      // term's direction (the first lane takes Q); 7. periodic closure
      T P0[NT], P1[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bool fw = pf_fwd<NR, NB>(t);
        T G0 = I0[t], G1 = I1[t];
        if (t >= NR) cfma<T>(G0, G1, Pw[t][0], Pw[t][1], Q0[t], Q1[t]);
        else G0 = fma(Pw[t][0], Q0[t], G0);
        P0[t] = fw ? dpp_mov<0x138>(Q0[t], G0) : dpp_mov<0x130>(Q0[t], G0);
        P1[t] = (T)0;
        if (t >= NR) P1[t] = fw ? dpp_mov<0x138>(Q1[t], G1) : dpp_mov<0x130>(Q1[t], G1);
        if (t >= NR) cfma<T>(P0[t], P1[t], Pl[t][0], Pl[t][1], T0[t], T1[t]);
        else P0[t] = fma(Pl[t][0], T0[t], P0[t]);
      }
      // 8. every term rerun from its true carry into the sum, interleaved
#pragma unroll
      for (int kk = 0; kk < K; ++kk)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int k = pf_fwd<NR, NB>(t) ? kk : K - 1 - kk;
          if (t < NR) {
            P0[t] = r[k] + cq[t][0] * P0[t];
            acc[k] = fma(ca[t][0], P0[t], acc[k]);
          } else {
            const T n0 = r[k] + cq[t][0] * P0[t] - cq[t][1] * P1[t];
            P1[t] = cq[t][0] * P1[t] + cq[t][1] * P0[t];
            P0[t] = n0;
            acc[k] += (T)2 * (ca[t][0] * P0[t] - ca[t][1] * P1[t]);
          }
        }
      ++call;
      if (i < S - 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) ks[i][k] = (acc[k] - r[k]) * ig;  // dt L Y_i
      } else {
        // stiffly accurate (b = last row of A): u^{n+1} = Y_s
#pragma unroll
        for (int k = 0; k < K; ++k) u[k] = acc[k];
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

template <typename T, int K, int S, int NR, int NB, int NC>
__global__ void __launch_bounds__(512) k_sdirk_pf(RelaxArgs a) {
  sdirk_pf_body<T, K, S, NR, NB, NC>(a, (int)blockIdx.x);
}

template <typename T, int K, int S, int NR, int NB, int NC>
__global__ void __launch_bounds__(512) k_sdirk_pf_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  sdirk_pf_body<T, K, S, NR, NB, NC>(a, blk);
}

}  // namespace mgr
