// Relaxation kernel for levels with inflow/outflow boundaries (Sec. 4.5).
//
// Phi is no longer circulant: rows near x = -1 and x = 1 carry the boundary
// closures, the coarse operators are the periodic Psi truncated to the
// interval, and every fine step adds the inflow forcing of its time.  Both
// kernels keep one interval's state in LDS (FP64) and apply the operator of
// BoundedDev (common.h): k_bounded point by point (any tap list; consecutive
// threads own consecutive points), k_bounded_tiled register-blocked over a
// dense window of up to 64 taps (below).
// Launch arguments and outputs are those of the periodic kernels
// (RelaxArgs, relax_kernels.h), with `opdata` the level's BoundedDev,
// signed offsets in `tap_off` and `omin` the fine steps between the start
// times of consecutive blocks.
#pragma once

#include "registry.h"
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

constexpr int kFRows = kFRowsLds;

// Barrier for LDS traffic only: release and acquire at workgroup scope on
// the local address space, so global loads issued for a later step stay in
// flight across it (a full __syncthreads waits for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Register-blocked variant.  Thread t owns chunks of K consecutive points;
// the truncated stencil is a dense window of W weights, c[i] the weight of
// offset omax - i (tap_off[0] = omax, taps = the W weights), so
// out_{b+k} = sum_i c[i] u_{b - omax + k + i} with u = 0 off the grid (the
// truncation).  A chunk reads its K + W - 1 inputs from LDS once into
// registers; the state buffers carry padl / padr zero points on either side
// (BoundedDev), so those reads need no bounds checks.  K is odd, so lanes
// whose chunks start K doubles apart read distinct LDS banks.  The dense
// boundary rows of the fine level are staged in LDS at the start; each is
// summed by four lanes (a quarter of the dependent chain).  The inflow forcing is staged in LDS for
// kFRows steps at a time; with PF (levels with a right-hand side every
// step) the right-hand side rows of a thread's first chunk are loaded at
// the end of the step before their use.  Steps are separated by LDS-only
// barriers, so those loads stay in flight across them.
// Also runs MODE_FW (common.h): the coarsest sweep in overlapping chunks.
// LDS: state and next state (each padl + n_x + padr), the left and right
// blocks, then kFRows forcing rows.
template <int K, int W, bool PF>
__device__ __forceinline__ void bounded_tiled_body(const RelaxArgs& a, const int j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const BoundedDev bd = *reinterpret_cast<const BoundedDev*>(a.opdata);
  const int nx = a.nx, m = a.m, NT = blockDim.x, tid = threadIdx.x;
  const int omax = a.tap_off[0];
  const int nch = (nx + K - 1) / K;
  // rows of this block: steps 1..nsteps write rows rbase + s
  const bool fw = a.mode == MODE_FW;
  const int t0 = fw ? max(0, j * m - a.tile) : 0;
  const int warm = fw ? j * m - t0 : 0;
  const int nsteps = fw ? warm + min(m, a.nint - j * m) : m;
  const long long rbase = fw ? (long long)t0 : (long long)j * m;
  const int span = bd.padl + nx + bd.padr;
  double* bufa = reinterpret_cast<double*>(smem_raw);
  double* cur = bufa + bd.padl;
  double* nxt = bufa + span + bd.padl;
  // boundary rows staged with odd row strides (distinct LDS banks per row)
  const int lst = bd.ncl | 1, rst = bd.ncr | 1;
  double* lb = bufa + 2 * span;
  double* rb = lb + bd.nl * lst;
  for (int q = tid; q < bd.padl; q += NT) bufa[q] = bufa[span + q] = 0.0;
  for (int q = tid; q < bd.padr; q += NT) cur[nx + q] = nxt[nx + q] = 0.0;
  for (int q = tid; q < bd.nl * bd.ncl; q += NT) lb[(q / bd.ncl) * lst + q % bd.ncl] = bd.lblk[q];
  for (int q = tid; q < bd.nr * bd.ncr; q += NT) rb[(q / bd.ncr) * rst + q % bd.ncr] = bd.rblk[q];
  // start state: loads issued in batches of BL per thread before their use
  constexpr int BL = 8;
  {
    const double* in = a.zero_in ? nullptr : a.in + (long long)j * a.in_stride * nx;
    const double* co = (a.zero_in || !a.corr) ? nullptr : a.corr + (long long)j * a.corr_stride * nx;
    double* o0 = a.mode == MODE_F ? a.out + (long long)j * m * nx
                                  : (((a.mode == MODE_FC && a.write_row0) || fw) && j == 0 ? a.out
                                                                                    : nullptr);
    for (int p0 = tid; p0 < nx; p0 += BL * NT) {
      double v[BL], c2[BL];
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = p0 + u * NT;
        v[u] = (in && p < nx) ? in[p] : 0.0;
        c2[u] = (co && p < nx) ? co[p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = p0 + u * NT;
        if (p < nx) {
          const double x = v[u] + c2[u];
          if (o0) o0[p] = x;
          cur[p] = x;
        }
      }
    }
  }
  if (a.mode == MODE_F && j == a.nint) return;
  __syncthreads();
  constexpr bool kHold = W <= 12;
  double c[kHold ? W : 1];
  if constexpr (kHold) {
#pragma unroll
    for (int i = 0; i < W; ++i) c[i] = a.taps[i];
  }
  // boundary rows (fine level): four consecutive threads share a row, each
  // summing every fourth column; brow is this thread's row or -1
  const int bq = tid >> 2, bpart = tid & 3;
  const int brow = bq < bd.nl ? bq : (bq < bd.nl + bd.nr ? nx - bd.nr + (bq - bd.nl) : -1);
  // inflow forcing rows, staged in LDS kFRows steps at a time
  double* fst = rb + bd.nr * rst;
  const double* Fb = bd.F ? bd.F + (long long)j * a.omin * bd.nf : nullptr;
  const bool has_g = a.rhs_mode == RHS_EVERY;
  const int b0 = tid * K;  // the thread's first chunk
  constexpr int KP = PF ? K : 1;
  double gnext[KP];
  if (PF && has_g) {
#pragma unroll
    for (int k = 0; k < KP; ++k)
      gnext[k] = (nsteps >= 1 && b0 + k < nx) ? a.rhs[(rbase + 1) * nx + b0 + k] : 0.0;
  }
  for (int s = 1; s <= nsteps; ++s) {
    const double* g = has_g ? a.rhs + (rbase + s) * nx : nullptr;
    const bool store = (a.mode == MODE_F && (s < m || a.write_last)) || (fw && s > warm);
    double* orow = store ? a.out + (rbase + s) * nx : nullptr;
    if (Fb && (s - 1) % kFRows == 0) {
      const int rows = min(kFRows, nsteps - (s - 1));
      for (int q = tid; q < rows * bd.nf; q += NT) fst[q] = Fb[(long long)(s - 1) * bd.nf + q];
      __syncthreads();
    }
    for (int ch = tid; ch < nch; ch += NT) {
      const int b = ch * K;
      // stream the K + W - 1 window values: value i feeds out_k with
      // weight c[i - k]
      double acc[K];
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = 0.0;
      const int w0 = b - omax;
#pragma unroll
      for (int i = 0; i < K + W - 1; ++i) {
        const double v = cur[w0 + i];
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (i - k >= 0 && i - k < W)
            acc[k] = fma(kHold ? c[kHold ? i - k : 0] : a.taps[i - k], v, acc[k]);
      }
      if (has_g) {  // uniform
        if (PF && ch == tid) {
#pragma unroll
          for (int k = 0; k < K; ++k) acc[k] += gnext[PF ? k : 0];
        } else {
#pragma unroll
          for (int k = 0; k < K; ++k) acc[k] += b + k < nx ? g[b + k] : 0.0;
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int p = b + k;
        if (p < nx && p >= bd.nl && p < nx - bd.nr) {
          nxt[p] = acc[k];
          if (orow) orow[p] = acc[k];
        }
      }
    }
    if (bd.nl + bd.nr > 0) {  // uniform: every lane takes part in the quad sums
      double acc = 0.0;
      if (brow >= 0 && brow < bd.nl) {
        const double* row = lb + brow * lst;
#pragma unroll 2
        for (int q = bpart; q < bd.ncl; q += 4) acc = fma(row[q], cur[q], acc);
      } else if (brow >= 0) {
        const double* row = rb + (brow - (nx - bd.nr)) * rst;
        const double* src = cur + (nx - bd.ncr);
#pragma unroll 2
        for (int q = bpart; q < bd.ncr; q += 4) acc = fma(row[q], src[q], acc);
      }
      // quad sum in a fixed order (lanes 4i..4i+3 of one wavefront)
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (brow >= 0 && bpart == 0) {
        if (Fb && brow < bd.nf) acc += fst[((s - 1) % kFRows) * bd.nf + brow];
        if (has_g) acc += g[brow];
        nxt[brow] = acc;
        if (orow) orow[brow] = acc;
      }
    }
    // next step's right-hand side for the first chunk, in flight across
    // the barrier
    if (PF && has_g && s < nsteps) {
#pragma unroll
      for (int k = 0; k < KP; ++k) gnext[k] = b0 + k < nx ? g[nx + b0 + k] : 0.0;
    }
    lds_barrier();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (a.mode == MODE_FC) {
    const double* gc = (a.rhs_mode == RHS_CPOINT) ? a.rhs + (long long)(j + 1) * nx : nullptr;
    const double* in1 = (a.delta && !a.zero_in) ? a.in + (long long)(j + 1) * a.in_stride * nx : nullptr;
    const double* co1 = (a.delta && a.corr) ? a.corr + (long long)(j + 1) * a.corr_stride * nx : nullptr;
    double* orow = a.out + (long long)(j + a.out_off) * nx;
    double ss = 0.0;
    for (int p0 = tid; p0 < nx; p0 += BL * NT) {
      double gv[BL], iv[BL], cv[BL];
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = p0 + u * NT;
        gv[u] = (gc && p < nx) ? gc[p] : 0.0;
        iv[u] = (in1 && p < nx) ? in1[p] : 0.0;
        cv[u] = (co1 && p < nx) ? co1[p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = p0 + u * NT;
        if (p < nx) {
          const double v = cur[p] + gv[u];
          orow[p] = v;
          ss += v * v;
          if (a.delta) {
            a.delta[(long long)(j + 1) * nx + p] = v - (iv[u] + cv[u]);
            if (j == 0) a.delta[p] = 0.0;
          }
        }
      }
    }
    if (a.partial) {
      const double s = block_sum(ss, red);
      if (tid == 0) a.partial[j] = s;
    }
  } else if (a.mode == MODE_RES) {
    const double* gc = (a.rhs_mode == RHS_CPOINT) ? a.rhs + (long long)(j + 1) * nx : nullptr;
    const double* ref = a.ref + (long long)(j + 1) * nx;
    double ss = 0.0;
    for (int p0 = tid; p0 < nx; p0 += BL * NT) {
      double gv[BL], rv[BL];
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = p0 + u * NT;
        gv[u] = (gc && p < nx) ? gc[p] : 0.0;
        rv[u] = p < nx ? ref[p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = p0 + u * NT;
        if (p < nx) {
          const double v = cur[p] + gv[u] - rv[u];
          a.out[(long long)(j + 1) * nx + p] = v;
          if (j == 0) a.out[p] = 0.0;
          ss += v * v;
        }
      }
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

// For lane l < 63 the value v of lane l + 1 of the wavefront, for lane 63
// `old` (DPP wave_shl:1 without bound control).
__device__ __forceinline__ double shl1(double old, double v) {
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), 0x130, 0xf,
                                             0xf, false);
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), 0x130, 0xf,
                                             0xf, false);
  return __hiloint2double(hi, lo);
}

// Lane-resident variant for the fine level: one interval per workgroup.
// Lanes 0..NL-1 (NL = blockDim.x - 64) own K consecutive points each in
// registers, lane l the points l*K .. l*K+K-1 (points from n_x on are
// zeros); the stencil is a dense window: out_p = sum_i c[i] u_{p-HL+i}, HL
// points upwind and HR downwind.  A step takes the halos from the neighbour
// lanes by DPP lane shifts and, at wavefront edges, from two LDS slots per
// wavefront; one LDS-only barrier per step, and no global memory access
// inside the step loop (with MODE_F the states are stored).
//
// The boundary rows are no stencil rows: lanes [0, a) and [b, nla) (the
// chunks that hold them; `region` lanes) hand their points to the last
// wavefront, which keeps those points' states in LDS (bu) and advances them
// row by row, each row a dense window of the level's Phi (the closures of
// Sec. 4.5 and, between them and the interior, stencil rows; at most
// kRegLen weights, held in registers) over bu.  bu
// holds, per step parity, the left region's points, lane a's chunk, lane
// b-1's chunk and the right region's points; lanes a and b-1 export their
// chunks there before the barrier.  Region lanes keep running the stencil
// on stale points (their results are discarded); after the barrier lane
// a-1 takes its last HL points and lane b its first HR points of the step
// from bu before the DPP shifts, so every non-region lane reads true
// values (a and b are no multiples of 64, so a region lane never feeds a
// non-region lane through a wavefront-edge slot), and every region lane
// takes all its points from bu after the last step.  With MODE_F the last
// wavefront stores the region points of every step.  The inflow forcing (rows
// < nf <= a*K) is added there too, staged in LDS before the first step (in
// blocks of kRegFCap / nf steps when m * nf exceeds kRegFCap).  The two
// kinds of wavefront run loops of their own with the same barriers.
//
// Modes FC (no update rows), RES and F, no right-hand side: the fine
// level's passes; the host refuses the rest.
//
// LDS: the staging area NL*(K+1) doubles (start and end rows, coalesced),
// the edge slots 2 * NL/64 * (HL+HR), bu 2 * rg_bu, the forcing kRegFCap:
// under 40 KB for n_x = 4096, four workgroups per CU.  Registers are held
// to six wavefronts per SIMD (76 VGPRs): a workgroup of five wavefronts
// places two on one SIMD, and at five per SIMD only three workgroups fit.
template <int K, int HL, int HR>
__device__ __forceinline__ void bounded_reg_body(const RelaxArgs& a, const int j) {
  constexpr int W = HL + HR + 1;
  constexpr int HE = HL + HR;  // doubles of one wavefront's edge slots
  constexpr int XB = kRegExportB<K, HL>();
  constexpr int BL = 10;       // loads per thread in flight (row traffic):
                               // more would not fit six wavefronts per SIMD
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const BoundedDev* bd = reinterpret_cast<const BoundedDev*>(a.opdata);
  const int nx = a.nx, m = a.m, NT = blockDim.x, tid = threadIdx.x;
  const int NL = NT - 64, nwi = NL >> 6, lw = tid & 63;
  // the wavefront index as a scalar: branches on it are uniform
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool bwave = wave >= nwi;
  const int BU = bd->rg_bu;
  const int np = NL * K;
  double* stg = reinterpret_cast<double*>(smem_raw);
  double* ed = stg + NL * (K + 1);
  double* bu = ed + 2 * nwi * HE;
  double* fst = bu + 2 * BU;
  const int nf = bd->nf;
  const double* const Fg = bd->F;
  // forcing steps staged in LDS at a time
  const int fr = nf > 0 ? kRegFCap / nf : 1;
  const bool store_steps = a.mode == MODE_F;
  const long long row0 = (long long)j * m;

  // start state, staged (coalesced reads, then each lane its chunk); the
  // last wavefront also stages the region rows, clears bu and stages the
  // first forcing block
  {
    const double* in = a.zero_in ? nullptr : a.in + (long long)j * a.in_stride * nx;
    const double* co =
        (a.zero_in || !a.corr) ? nullptr : a.corr + (long long)j * a.corr_stride * nx;
    const bool st0 = (a.mode == MODE_F && !a.skip_row0) ||
                     (a.mode == MODE_FC && a.write_row0 && j == 0);
    double* o0 = st0 ? a.out + (a.mode == MODE_F ? row0 * nx : 0LL) : nullptr;
    for (int q0 = tid; q0 < np; q0 += BL * NT) {
      double v[BL], c2[BL];
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = q0 + u * NT;
        v[u] = (in && p < nx) ? in[p] : 0.0;
        c2[u] = (co && p < nx) ? co[p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = q0 + u * NT;
        if (p < np) {
          const double x = v[u] + c2[u];
          if (o0 && p < nx) o0[p] = x;
          stg[p + p / K] = x;
        }
      }
    }
    if (bwave) {
      for (int q = lw; q < 2 * BU; q += 64) bu[q] = 0.0;
      if (Fg && j < a.nint) {
        const double* F0 = Fg + (long long)j * a.omin * nf;
        const int n0 = min(fr, m) * nf;
        for (int q = lw; q < n0; q += 64) fst[q] = F0[q];
      }
    }
  }
  if (a.mode == MODE_F && j == a.nint) return;  // extra block: the last C-point
  __syncthreads();
  const int ra = bd->rg_a, rb = bd->rg_b, nla = bd->rg_nla, LW = bd->rg_lw;
  double x[K];

  if (!bwave) {
    // ---- lanes -----------------------------------------------------------
    // bu slot of this lane's region points (-1: not a region lane, -2: zeros
    // past the last chunk); lanes a and b-1 export their chunks
    const int pslot =
        tid < ra ? tid * K : (tid >= rb ? (tid < nla ? LW + (tid - rb + 1) * K : -2) : -1);
    double c[W];
    {
      // through the scalar cache (read only): the taps stay in scalar
      // registers, which the FMAs take as operands
      typedef __attribute__((address_space(4))) const double cdouble;
      const cdouble* tq = (const cdouble*)a.taps;
#pragma unroll
      for (int i = 0; i < W; ++i) c[i] = tq[i];
    }
    const int eo = wave * HE;
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = stg[tid * (K + 1) + k];
    for (int s = 0; s < m; ++s) {
      const int par = s & 1;
      double* bcur = bu + par * BU;
      double* ecur = ed + par * nwi * HE;
      // exports of state s: wavefront edges, lanes a and b-1 (the last
      // wavefront reads HR values of lane a, at most XB of lane b-1)
      if (lw == 63) {
#pragma unroll
        for (int h = 0; h < HL; ++h) ecur[eo + h] = x[K - HL + h];
      }
      if (lw == 0) {
#pragma unroll
        for (int h = 0; h < HR; ++h) ecur[eo + HL + h] = x[h];
      }
      if (tid == ra) {
#pragma unroll
        for (int k = 0; k < HR; ++k) bcur[ra * K + k] = x[k];
      }
      if (tid == rb - 1) {
#pragma unroll
        for (int k = K - XB; k < K; ++k) bcur[LW + k] = x[k];
      }
      lds_barrier();
      // region lanes hold stale points between steps; only lane a-1's last
      // HL and lane b's first HR points reach other lanes (the DPP shifts),
      // so only those are taken from bu (the rest after the last step)
      if (tid == ra - 1) {
#pragma unroll
        for (int h = 0; h < HL; ++h) x[K - HL + h] = bcur[ra * K - HL + h];
      }
      if (tid == rb) {
#pragma unroll
        for (int h = 0; h < HR; ++h) x[h] = bcur[LW + K + h];
      }
      // state s (region points: stored by the last wavefront)
      if (store_steps && s >= 1 && pslot == -1) {
        double* orow = a.out + (row0 + s) * nx;
#pragma unroll
        for (int k = 0; k < K; ++k) orow[tid * K + k] = x[k];
      }
      double el[HL > 0 ? HL : 1], er[HR > 0 ? HR : 1];
#pragma unroll
      for (int h = 0; h < HL; ++h) el[h] = 0.0;
#pragma unroll
      for (int h = 0; h < HR; ++h) er[h] = 0.0;
      if (wave > 0) {
#pragma unroll
        for (int h = 0; h < HL; ++h) el[h] = ecur[eo - HE + h];
      }
      if (wave + 1 < nwi) {
#pragma unroll
        for (int h = 0; h < HR; ++h) er[h] = ecur[eo + HE + HL + h];
      }
      double hl[HL > 0 ? HL : 1], hr[HR > 0 ? HR : 1];
#pragma unroll
      for (int h = 0; h < HL; ++h) hl[h] = shr1(el[h], x[K - HL + h]);
#pragma unroll
      for (int h = 0; h < HR; ++h) hr[h] = shl1(er[h], x[h]);
      // in place, left to right: x[k] is overwritten by output k, its old
      // value kept for outputs k+1..k+HL in a ring of HL registers
      constexpr int HLa = HL > 0 ? HL : 1;
      double old[HLa];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const int q = k - HL + i;
          double u;
          if (q < 0)
            u = hl[q < 0 ? q + HL : 0];
          else if (q < k)
            u = old[q % HLa];
          else if (q < K)
            u = x[q < K ? q : 0];
          else
            u = hr[q >= K ? q - K : 0];
          acc = fma(c[i], u, acc);
        }
        if constexpr (HL > 0) old[k % HLa] = x[k];
        x[k] = acc;
      }
    }
    lds_barrier();
    if (pslot != -1) {
      const double* bcur = bu + (m & 1) * BU;
#pragma unroll
      for (int k = 0; k < K; ++k) x[k] = pslot >= 0 ? bcur[pslot + k] : 0.0;
    }
    if (store_steps && m >= 1 && a.write_last) {
      double* orow = a.out + (row0 + m) * nx;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (tid * K + k < nx) orow[tid * K + k] = x[k];
    }
    if (a.mode == MODE_FC || a.mode == MODE_RES) {
#pragma unroll
      for (int k = 0; k < K; ++k) stg[tid * (K + 1) + k] = x[k];
    }
  } else {
    // ---- the last wavefront: region row lw (< rg_rows) of point rp, a
    // window of kRegLen weights (in registers) over bu from rcs, the result
    // to slot rdst ----
    const bool act = lw < bd->rg_rows;
    int rcs = 0, rdst = 0, rp = nx;
    double cr[kRegLen];
#pragma unroll
    for (int t = 0; t < kRegLen; ++t) cr[t] = 0.0;
    if (act) {
      rcs = bd->rg_cs[lw];
      rdst = bd->rg_dst[lw];
      rp = lw < ra * K ? lw : rb * K + (lw - ra * K);
      const double* co = bd->rg_coef + lw * bd->rg_ls;
#pragma unroll
      for (int t = 0; t < kRegLen; ++t) cr[t] = co[t];
    }
    const bool rforce = act && Fg && rp < nf;
    for (int q = lw; q < ra * K; q += 64) bu[q] = stg[q + q / K];
    for (int q = lw; q < (nla - rb) * K; q += 64) {
      const int p = rb * K + q;
      bu[LW + K + q] = stg[p + p / K];
    }
    for (int s = 0; s < m; ++s) {
      const int par = s & 1;
      if (Fg && s > 0 && s % fr == 0) {
        // the next block of forcing steps (m * nf > kRegFCap only)
        const double* Fs = Fg + ((long long)j * a.omin + s) * nf;
        const int n = min(fr, m - s) * nf;
        for (int q = lw; q < n; q += 64) fst[q] = Fs[q];
      }
      lds_barrier();
      if (store_steps && s >= 1) {
        // state s of the region points
        double* orow = a.out + (row0 + s) * nx;
        const double* bc = bu + par * BU;
        for (int q = lw; q < ra * K; q += 64) orow[q] = bc[q];
        for (int q = lw; q < nx - rb * K; q += 64) orow[rb * K + q] = bc[LW + K + q];
      }
      if (act) {
        const double* ur = bu + par * BU + rcs;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        // in thirds: at most a third of the window's reads in registers
#pragma unroll
        for (int h = 0; h < 3; ++h) {
#pragma unroll
          for (int t = h * kRegLen / 3; t < (h + 1) * kRegLen / 3; t += 4) {
            s0 = fma(cr[t], ur[t], s0);
            s1 = fma(cr[t + 1], ur[t + 1], s1);
            s2 = fma(cr[t + 2], ur[t + 2], s2);
            s3 = fma(cr[t + 3], ur[t + 3], s3);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        double v = (s0 + s1) + (s2 + s3);
        if (rforce) v += fst[(s % fr) * nf + rp];
        bu[(par ^ 1) * BU + rdst] = v;
      }
    }
    lds_barrier();
  }
  if (a.mode != MODE_FC && a.mode != MODE_RES) return;
  // final state through the staging area, then coalesced row work
  __syncthreads();
  double ss = 0.0;
  if (a.mode == MODE_FC) {
    double* orow = a.out + (long long)(j + a.out_off) * nx;
    for (int p = tid; p < nx; p += NT) {
      const double v = stg[p + p / K];
      orow[p] = v;
      ss += v * v;
    }
  } else {
    const double* ref = a.ref + (long long)(j + 1) * nx;
    double* orow = a.out + (long long)(j + 1) * nx;
    for (int p0 = tid; p0 < nx; p0 += BL * NT) {
      double rv[BL];
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = p0 + u * NT;
        rv[u] = p < nx ? ref[p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int p = p0 + u * NT;
        if (p < nx) {
          const double v = stg[p + p / K] - rv[u];
          orow[p] = v;
          if (j == 0) a.out[p] = 0.0;
          ss += v * v;
        }
      }
    }
  }
  if (a.partial) {
    const double t = block_sum(ss, red);
    if (tid == 0) a.partial[j] = t;
  }
}

template <int K, int HL, int HR>
__global__ void __launch_bounds__(1024, 6) k_bounded_reg(RelaxArgs a) {
  bounded_reg_body<K, HL, HR>(a, (int)blockIdx.x);
}

template <int K, int HL, int HR>
__global__ void __launch_bounds__(1024, 6) k_bounded_reg_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  bounded_reg_body<K, HL, HR>(a, blk);
}

template <int K, int W, bool PF>
__global__ void __launch_bounds__(512) k_bounded_tiled(RelaxArgs a) {
  bounded_tiled_body<K, W, PF>(a, (int)blockIdx.x);
}

template <int K, int W, bool PF>
__global__ void __launch_bounds__(512) k_bounded_tiled_b(BatchArgs b) {
  int blk;
  const RelaxArgs a = batch_member(b, blk);
  bounded_tiled_body<K, W, PF>(a, blk);
}

}  // namespace mgr

