// libmgrit host runtime: plans, the MGRIT cycle driver and the C-ABI of
// include/mgrit.h.  Every step of a solve runs in the kernels of
// relax_kernels.h / misc.hip on the plan's HIP stream; this file only
// sequences launches, keeps the level hierarchy and reads back one FP64
// norm per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mgrit.h"
#include "plan.h"
#include "registry.h"
#include "setup.h"

namespace mgr {

// ---------------------------------------------------------------------------
// kernel selection
// ---------------------------------------------------------------------------
// LDS bytes of k_stencil for an extent of E points, chunk K, NL lanes,
// compiled width Wb, state element size el and per-step I/O io (the
// staging area holds half the extent when stencil_half_stage).
static size_t stencil_lds(int E, int K, int NL, int Wb, size_t el, bool io) {
  const int Es = stencil_half_stage(K, Wb, io) ? E / 2 : E;  // staged positions
  const size_t stage = sizeof(double) * (size_t)(Es + Es / K);
  if (Wb - 1 <= K) {
    const int H = std::min(Wb - 1, K);
    return stage + 2 * (size_t)(NL / 64) * std::max(H, 1) * el;
  }
  const int M = (Wb - 1 + K - 1) / K * K;
  const size_t img = (size_t)((E + M) + (E + M) / K) * el;
  return std::max(stage, 2 * img);
}

// Per-kernel facts from its code object, cached: whether it spills
// registers to scratch memory, and the dynamic LDS it may use, which is
// raised once to all of the CU's 160 KB not taken by static LDS (a limit,
// not a reservation; never lowered, so plans of any size can share it).
struct KernelInfo {
  bool spills = true;
  size_t max_lds = 0;
};

static KernelInfo kernel_info(KernelFn fn) {
  static std::mutex mu;
  static std::unordered_map<const void*, KernelInfo> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find((const void*)fn);
  if (it != cache.end()) return it->second;
  KernelInfo ki;
  hipFuncAttributes attr;
  std::memset(&attr, 0, sizeof attr);
  if (hipFuncGetAttributes(&attr, (const void*)fn) == hipSuccess) {
    ki.spills = attr.localSizeBytes > 0;
    const size_t want = 160 * 1024 - std::min<size_t>(attr.sharedSizeBytes, 160 * 1024);
    if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)want) == hipSuccess) {
      ki.max_lds = want;
    } else {
      (void)hipGetLastError();
      ki.max_lds = 64 * 1024;
    }
  } else {
    (void)hipGetLastError();
  }
  cache[(const void*)fn] = ki;
  return ki;
}

static bool spills(KernelFn fn) { return kernel_info(fn).spills; }

// Launch-time model of one stencil pass on the 256 CUs of the chip (2.4
// GHz): nwg workgroups of NL lanes x K points, S steps of Wb taps, occ
// workgroups resident per CU.  A step of the `conc` workgroups on one CU
// costs the larger of a latency floor (LDS round trip, barrier) and its
// FMA issue time (16 FP64/FP32 lanes per SIMD per clock, 4 SIMDs) plus,
// when the halo streams from LDS, its LDS traffic (128 B per clock); each
// round of resident workgroups adds the start and end row traffic, each
// launch a fixed cost.  Constants fitted to launch-shape sweeps on MI355X
// (the model's pick is within 2 % of the fastest measured shape on every
// swept level of the 4096 x 16384 ERK3 and 8192 x 65536 ERK5 workloads).
static double stencil_time_us(int nwg, int NL, int K, int Wb, int S, int occ) {
  const int kCU = 256;
  const double clk_us = 1.0 / 2400.0;
  occ = std::max(occ, 1);
  const int conc = std::min(occ, (nwg + kCU - 1) / kCU);
  const int nw = NL / 64;
  const double fma = std::ceil(conc * nw / 4.0) * K * Wb * 4.0;
  const double lds = (Wb - 1 <= K) ? 0.0 : conc * (double)NL * (Wb - 1 + K) * 8.0 / 128.0;
  const double step = std::max(600.0, 1.2 * fma + lds);
  const long long rounds = (nwg + (long long)kCU * occ - 1) / ((long long)kCU * occ);
  return rounds * (S * step + 4800.0) * clk_us + 1.5;
}

// Resident workgroups per CU, cached per (kernel, lanes, LDS bytes): the
// planner asks for hundreds of candidate shapes per plan.
static int occupancy(KernelFn fn, int NL, size_t lds) {
  struct Key {
    const void* fn;
    int NL;
    size_t lds;
    bool operator==(const Key& o) const { return fn == o.fn && NL == o.NL && lds == o.lds; }
  };
  struct Hash {
    size_t operator()(const Key& k) const {
      return std::hash<const void*>()(k.fn) ^ (std::hash<size_t>()(k.lds * 1024 + k.NL) << 1);
    }
  };
  static std::mutex mu;
  static std::unordered_map<Key, int, Hash> cache;
  const Key key{(const void*)fn, NL, lds};
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, NL, lds) !=
      hipSuccess) {
    (void)hipGetLastError();
    nb = 1;
  }
  if (nb < 1) nb = 1;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = nb;
  return nb;
}

static int pick_width(int W) {
  for (int i = 0; i < kNumWidths; ++i)
    if (kWidths[i] >= W) return kWidths[i];
  return -1;
}

// Fill the kernels and LDS sizes of shape `sh` (K, NL set); false if it
// does not fit the CU's 160 KB of LDS.
static bool finish_shape(StencilShape& sh, int E, int Wb, bool io) {
  const KernelTable& kt = kernel_table();
  const int ki = k_index(sh.K), wi = width_index(Wb);
  if (ki < 0 || wi < 0) return false;
  sh.shmem[0] = stencil_lds(E, sh.K, sh.NL, Wb, sizeof(double), io);
  sh.shmem[1] = stencil_lds(E, sh.K, sh.NL, Wb, sizeof(float), io);
  if (sh.shmem[0] > 160 * 1024) return false;
  for (int q = 0; q < 2; ++q) {
    sh.fn[q] = kt.stencil[q][ki][wi][io ? 1 : 0];
    sh.bfn[q] = kt.stencil_b[q][ki][wi][io ? 1 : 0];
    if (!sh.fn[q] || !sh.bfn[q]) return false;
  }
  return true;
}

// Right-hand side rows a pass may stage in LDS next to the shape's own
// LDS: up to the kernel's LDS limit when the launch has at most two
// workgroups per CU anyway, else within 64 KB (keeps two or more
// resident).  False if the shape itself does not fit.
static bool set_lds(StencilShape& sh, long long nwg, bool io) {
  const size_t lim = std::min(kernel_info(sh.fn[0]).max_lds, kernel_info(sh.fn[1]).max_lds);
  if (sh.shmem[0] > lim) return false;
  const size_t row = sizeof(double) * (size_t)sh.NL * (sh.K + 1);
  const size_t budget = nwg <= 2 * 256 ? lim : std::min<size_t>(lim, 64 * 1024);
  sh.preload_rows = (io && sh.shmem[0] < budget) ? (int)((budget - sh.shmem[0]) / row) : 0;
  return true;
}

// Untiled shape: NL = n_x/K lanes (a multiple of 64, at most 512) over the
// whole periodic line, the spill-free chunk with the lowest modelled time
// for S steps over nblk workgroups (if none is spill-free, the fastest
// modelled one).
static bool pick_whole(int nx, int Wb, int S, int nblk, bool io, StencilShape& out) {
  bool found = false, spill_free = false;
  for (int i = 0; i < kNumK; ++i) {
    StencilShape sh;
    sh.K = kKs[i];
    if (nx % sh.K) continue;
    sh.NL = nx / sh.K;
    if (sh.NL % 64 || sh.NL > 512 || sh.NL < 64 || Wb - 1 > nx) continue;
    if (!finish_shape(sh, nx, Wb, io)) continue;
    const bool sf = !spills(sh.fn[0]) && !spills(sh.fn[1]);
    if (found && spill_free && !sf) continue;
    sh.tiles = 1;
    sh.tile = nx;
    sh.max_steps = 1 << 30;
    if (!set_lds(sh, nblk, io)) continue;
    sh.est_us = stencil_time_us(nblk, sh.NL, sh.K, Wb, S, occupancy(sh.fn[0], sh.NL, sh.shmem[0]));
    if (!found || (sf && !spill_free) || sh.est_us < out.est_us) {
      out = sh;
      found = true;
      spill_free = sf;
    }
  }
  return found;
}

// Tiled shape for passes of S steps of a window of true width `width`:
// extent E = NL*K < n_x, tile C = E - S*(width-1) outputs, ceil(n_x/C)
// tiles; the spill-free shape with the lowest modelled time.
static bool pick_tiled(int nx, int width, int Wb, int S, int nblk, bool io, int max_tiles,
                       StencilShape& out) {
  const long long G = (long long)S * (width - 1);
  bool found = false;
  for (int i = 0; i < kNumK; ++i) {
    const int K = kKs[i];
    for (int NL = 64; NL <= 512; NL += 64) {
      const long long E = (long long)NL * K;
      if (E >= nx || E <= G) continue;
      StencilShape sh;
      sh.K = K;
      sh.NL = NL;
      sh.tile = (int)(E - G);
      sh.tiles = (nx + sh.tile - 1) / sh.tile;
      sh.max_steps = S;
      if (sh.tiles < 2 || sh.tiles > max_tiles) continue;
      if (!finish_shape(sh, (int)E, Wb, io) || spills(sh.fn[0]) || spills(sh.fn[1])) continue;
      if (!set_lds(sh, (long long)nblk * sh.tiles, io)) continue;
      sh.est_us = stencil_time_us((int)std::min<long long>((long long)nblk * sh.tiles, 1 << 30),
                                  NL, K, Wb, S, occupancy(sh.fn[0], NL, sh.shmem[0]));
      if (!found || sh.est_us < out.est_us) {
        out = sh;
        found = true;
      }
    }
  }
  return found;
}

int OpDesc::init_stencil(const Taps& t, int nx, int steps, int nblk, bool seq, int max_tiles,
                         std::string& err) {
  nnz = (int)t.off.size();
  flops_pps = 2.0 * nnz;
  std::vector<double> dense;
  int W = 1;
  tap_window(t, nx, omin, W, dense);
  width = W;
  const int Wb = pick_width(W);
  bool ok = Wb > 0;
  if (ok && seq) {
    // sequential sweep: steps per launch and shape with the lowest modelled
    // total time (launches run back to back on one stream)
    double best = 1e300;
    ok = pick_whole(nx, Wb, steps, 1, true, whole[1]) && pick_whole(nx, Wb, steps, 1, false, whole[0]);
    if (ok) {
      best = (spills(whole[1].fn[0]) || spills(whole[1].fn[1])) ? 1e300 : whole[1].est_us;
      seq_chunk = steps;
      for (int S = 4; S < steps; S *= 2) {
        StencilShape sh;
        if (!pick_tiled(nx, W, Wb, S, 1, true, max_tiles, sh)) continue;
        const double tot = ((steps + S - 1) / S) * sh.est_us;
        if (tot < best) {
          best = tot;
          seq_chunk = S;
          tiled[1] = sh;
        }
      }
      seq_us = best < 1e299 ? best : whole[1].est_us;
    }
  } else if (ok) {
    for (int io = 0; io < 2 && ok; ++io) {
      ok = pick_whole(nx, Wb, steps, nblk, io, whole[io]);
      StencilShape sh;
      const bool whole_spills = ok && (spills(whole[io].fn[0]) || spills(whole[io].fn[1]));
      if (ok && steps >= 1 && pick_tiled(nx, W, Wb, steps, nblk, io, max_tiles, sh) &&
          (whole_spills || sh.est_us < whole[io].est_us))
        tiled[io] = sh;
    }
  }
  if (ok) {
    kind = OP_STENCIL;
    K = whole[0].K;
    NL = whole[0].NL;
    Wbucket = Wb;
    dense.resize(Wb, 0.0);
    return upload((void**)&d_taps, dense.data(), dense.size() * sizeof(double));
  }
  // generic LDS kernel: state of 2 n_x values in LDS
  if ((size_t)2 * nx * sizeof(double) > 160 * 1024) {
    err = "n_x too large for the generic relaxation kernel";
    return MGRIT_EINVAL;
  }
  const KernelTable& kt = kernel_table();
  kind = OP_GENERIC;
  NL = 256;
  fn[0] = kt.generic[0];
  fn[1] = kt.generic[1];
  bfn[0] = kt.generic_b[0];
  bfn[1] = kt.generic_b[1];
  shmem[0] = (size_t)2 * nx * sizeof(double);
  shmem[1] = (size_t)2 * nx * sizeof(float);
  std::vector<int> off;
  std::vector<double> w;
  for (int q = 0; q < W; ++q)
    if (dense[q] != 0.0) {
      off.push_back((omin + q) % nx);
      w.push_back(dense[q]);
    }
  ntaps = (int)off.size();
  omin = 0;
  int rc = upload((void**)&d_taps, w.data(), w.size() * sizeof(double));
  if (!rc) rc = upload((void**)&d_off, off.data(), off.size() * sizeof(int));
  if (rc) return rc;
  for (int p = 0; p < 2; ++p)
    if (shmem[p] > kernel_info(fn[p]).max_lds) {
      err = "n_x too large for the generic relaxation kernel";
      return MGRIT_EINVAL;
    }
  return MGRIT_OK;
}

int OpDesc::init_sdirk(const Tableau& t, double cfl, int nx, std::string& err) {
  const KernelTable& kt = kernel_table();
  // lanes: NL = nx/K, multiple of 64, at most 512; prefer NL = 256
  int bestK = -1;
  double best = 1e30;
  for (int i = 0; i < kNumSdirkK; ++i) {
    const int k = kSdirkKs[i];
    if (nx % k) continue;
    const int nl = nx / k;
    if (nl % 64 || nl > 512) continue;
    const double score = std::fabs(std::log2((double)nl) - 8.0) + (nl > 256 ? 0.5 : 0.0);
    if (score < best) {
      best = score;
      bestK = k;
    }
  }
  if (bestK < 0) {
    err = "SDIRK plans need n_x a multiple of 64 with n_x/K <= 512 for K <= 16";
    return MGRIT_EINVAL;
  }
  K = bestK;
  NL = nx / K;
  SdirkDev sd;
  if (!sdirk_setup(t, cfl, K, NL, sd, err)) return MGRIT_EINVAL;
  // algorithmic flops per point and step, from the factored form: each
  // stage scales its right-hand side, runs the factors' recurrences (2 flops
  // per coefficient), combines the earlier stage derivatives (2 per non-zero
  // a_il) and, unless it is the last (stiffly accurate) stage, forms its
  // derivative (2)
  flops_pps = 0.0;
  for (int i = 0; i < sd.s; ++i) {
    flops_pps += 1.0;
    for (int q = 0; q < sd.nf; ++q) flops_pps += sd.f[q].a2 != 0.0 ? 4.0 : 2.0;
    for (int l = 0; l < i; ++l)
      if (sd.A[i][l] != 0.0) flops_pps += 2.0;
    if (i < sd.s - 1) flops_pps += 2.0;
  }
  kind = OP_SDIRK;
  nnz = 0;
  shmem[0] = shmem[1] = sizeof(double) * (size_t)(nx + nx / K);  // staging
  // the partial-fraction kernel when the roots allow it and it compiles
  // without spills, else the factored one
  SdirkPfDev pf;
  std::string pf_err;
  if (sdirk_setup_pf(t, cfl, K, NL, pf, pf_err)) {
    const int pi = sdirk_pf_shape_index(pf.s, pf.nr, pf.nb, pf.nc);
    const int ki = sdirk_k_index(K);
    if (pi >= 0 && ki >= 0 && kt.sdirk_pf[0][ki][pi] && kt.sdirk_pf[1][ki][pi] &&
        !spills(kt.sdirk_pf[0][ki][pi]) && !spills(kt.sdirk_pf[1][ki][pi]) &&
        shmem[0] <= kernel_info(kt.sdirk_pf[0][ki][pi]).max_lds &&
        shmem[1] <= kernel_info(kt.sdirk_pf[1][ki][pi]).max_lds) {
      fn[0] = kt.sdirk_pf[0][ki][pi];
      fn[1] = kt.sdirk_pf[1][ki][pi];
      bfn[0] = kt.sdirk_pf_b[0][ki][pi];
      bfn[1] = kt.sdirk_pf_b[1][ki][pi];
      sdirk_terms = pf.nr + pf.nc;
      return upload(&d_sdirk, &pf, sizeof(SdirkPfDev));
    }
  }
  const int si = sdirk_shape_index(sd.s, sd.nf);
  if (si < 0) {
    err = "no SDIRK kernel for this stage/factor count";
    return MGRIT_EINVAL;
  }
  fn[0] = kt.sdirk[0][sdirk_k_index(K)][si];
  fn[1] = kt.sdirk[1][sdirk_k_index(K)][si];
  bfn[0] = kt.sdirk_b[0][sdirk_k_index(K)][si];
  bfn[1] = kt.sdirk_b[1][sdirk_k_index(K)][si];
  for (int p = 0; p < 2; ++p)
    if (shmem[p] > kernel_info(fn[p]).max_lds) {
      err = "n_x too large for the SDIRK kernel's LDS staging";
      return MGRIT_EINVAL;
    }
  return upload(&d_sdirk, &sd, sizeof(SdirkDev));
}

// Region tables of the lane-resident fine-level kernel (k_bounded_reg,
// bounded_kernels.h) for entry `inst` of kBoundedReg: false if the window
// [omn, omx] of the interior stencil or the boundary rows do not fit it.
struct RegRegion {
  int K = 0, HL = 0, HR = 0, NT = 0;
  int a = 0, b = 0, nla = 0, lw = 0, bu = 0, ls = 0, len = 0, rows = 0;
  std::vector<double> coef;
  std::vector<int> cs, dst;
  size_t lds = 0;
};

static bool bounded_reg_region(const InflowOp& f, int nf, int nx, int inst, int omx, int omn,
                               RegRegion& R) {
  const int K = kBoundedReg[inst][0], HL = kBoundedReg[inst][1], HR = kBoundedReg[inst][2];
  if (omx > HL || -omn > HR || f.nl < 1 || f.nr < 1) return false;
  const int nla = (nx + K - 1) / K, NL = (nla + 63) / 64 * 64;
  if (NL + 64 > 1024) return false;
  // region lanes: [0, a) hold the left boundary rows, [b, nla) the right
  // ones; lanes a-1 and a (b-1 and b) share a wavefront
  int a = (f.nl + K - 1) / K;
  if (a % 64 == 0) ++a;
  int b = (nx - f.nr) / K;
  if (b % 64 == 0) --b;
  if (b <= a || nf > a * K) return false;
  const int rows = a * K + (nla - b) * K;
  if (rows > 64) return false;
  const int LW = (a + 1) * K, RW = (nla - b + 1) * K;
  // row r: point p; its nonzero columns and their bu slots
  std::vector<int> mn(rows), mx(rows);
  int len = 1;
  for (int r = 0; r < rows; ++r) {
    const int p = r < a * K ? r : b * K + (r - a * K);
    int lo = 1 << 30, hi = -1;
    if (p < nx) {
      int c0, c1;
      if (p < f.nl) {
        c0 = 0;
        c1 = f.ncl - 1;
      } else if (p >= nx - f.nr) {
        c0 = nx - f.ncr;
        c1 = nx - 1;
      } else {
        c0 = std::max(0, p - omx);
        c1 = std::min(nx - 1, p - omn);
      }
      for (int c = c0; c <= c1; ++c)
        if (inflow_entry(f, nx, p, c) != 0.0) {
          lo = std::min(lo, c);
          hi = std::max(hi, c);
        }
    }
    if (hi < 0) lo = hi = r < a * K ? 0 : b * K;  // a zero row
    // lane a exports its first HR values, lane b-1 its last XB
    const int XB = std::min(K, HL + 4);
    if (r < a * K ? hi >= a * K + HR : lo < b * K - XB) return false;
    mn[r] = lo;
    mx[r] = hi;
    len = std::max(len, hi - lo + 1);
  }
  len = (len + 3) / 4 * 4;
  if (len > kRegLen) return false;
  len = kRegLen;  // the kernel reads kRegLen weights (zeros past the row)
  R.K = K;
  R.HL = HL;
  R.HR = HR;
  R.NT = NL + 64;
  R.a = a;
  R.b = b;
  R.nla = nla;
  R.lw = LW;
  R.bu = LW + RW + len;
  R.len = len;
  R.ls = len + 1;
  R.rows = rows;
  R.coef.assign((size_t)rows * R.ls, 0.0);
  R.cs.assign(rows, 0);
  R.dst.assign(rows, 0);
  for (int r = 0; r < rows; ++r) {
    const bool left = r < a * K;
    const int p = left ? r : b * K + (r - a * K);
    const int slot0 = left ? 0 : LW - (b - 1) * K;  // bu slot of column c: c + slot0
    R.cs[r] = mn[r] + slot0;
    R.dst[r] = p + slot0;
    if (p < nx)
      for (int c = mn[r]; c <= mx[r]; ++c)
        R.coef[(size_t)r * R.ls + (c - mn[r])] = inflow_entry(f, nx, p, c);
  }
  R.lds = sizeof(double) * ((size_t)NL * (K + 1) + (size_t)2 * (NL / 64) * (HL + HR) +
                            (size_t)2 * R.bu + kRegFCap);
  return true;
}

int OpDesc::init_bounded(const Taps& interior, const InflowOp* fine,
                         const std::vector<double>* F, int nx, int stride, std::string& err) {
  const KernelTable& kt = kernel_table();
  kind = OP_BOUNDED;
  fn[1] = nullptr;  // FP64 state only
  bfn[1] = nullptr;
  nnz = (int)interior.off.size();
  flops_pps = 2.0 * nnz;
  omin = stride;
  // register-blocked kernel: the taps as one dense window of a compiled
  // width, chunks of bounded_k(width) points
  int omx = -(1 << 30), omn = 1 << 30;
  for (int o : interior.off) {
    omx = std::max(omx, o);
    omn = std::min(omn, o);
  }
  const int W = nnz ? omx - omn + 1 : 1;
  int wi = -1;
  for (int i = 0; i < kNumBoundedWidths && wi < 0; ++i)
    if (kBoundedWidths[i] >= W) wi = i;
  const int kb = wi >= 0 ? bounded_k(kBoundedWidths[wi]) : 1;
  const int nch = (nx + kb - 1) / kb;
  int rc;
  // (four threads per boundary row, the rows staged in LDS after the state;
  // zero padding around the state covers every window read)
  const int nbrows = fine ? fine->nl + fine->nr : 0;
  const int Wt = wi >= 0 ? kBoundedWidths[wi] : 0;
  const int padl = std::max(0, omx), padr = std::max(0, Wt - 1 - omx) + kb;
  const size_t tiled_lds =
      sizeof(double) * ((size_t)2 * (padl + nx + padr) +
                        (fine ? (size_t)fine->nl * (fine->ncl | 1) +
                                    (size_t)fine->nr * (fine->ncr | 1) +
                                    (size_t)kFRowsLds * fine->nf
                              : 0));
  const int pf = fine ? 0 : 1;  // coarse levels add a right-hand side row every step
  // fine level: the lane-resident kernel, chunks of 16 points from n_x =
  // 2048 on (else 8 where the halos fit), the smallest compiled window
  RegRegion R;
  bool lanes = false;
  if (fine && nnz) {
    const int nf = F ? fine->nf : 0;
    for (int pass = 0; pass < 2 && !lanes; ++pass) {
      const int Kw = (nx >= 2048) == (pass == 0) ? 16 : 8;
      for (int i = 0; i < kNumBoundedReg && !lanes; ++i) {
        if (kBoundedReg[i][0] != Kw || !kt.bounded_reg[i]) continue;
        if (!bounded_reg_region(*fine, nf, nx, i, omx, omn, R)) continue;
        if (R.lds > kernel_info(kt.bounded_reg[i]).max_lds || spills(kt.bounded_reg[i])) continue;
        lanes = true;
        reg_inst = i;
      }
    }
  }
  if (lanes) {
    const int Wr = R.HL + R.HR + 1;
    std::vector<double> dense(Wr, 0.0);
    for (size_t t = 0; t < interior.off.size(); ++t) dense[R.HL - interior.off[t]] += interior.w[t];
    fn[0] = kt.bounded_reg[reg_inst];
    bfn[0] = kt.bounded_reg_b[reg_inst];
    NL = R.NT;
    K = R.K;
    shmem[0] = shmem[1] = R.lds;
    ntaps = Wr;
    width = W;
    Wbucket = 0;
    reg_rows = R.rows;
    rc = upload((void**)&d_taps, dense.data(), dense.size() * sizeof(double));
    if (!rc) rc = upload((void**)&d_off, &R.HL, sizeof(int));
  } else if (nnz && wi >= 0 && kt.bounded_tiled[pf][wi] && 4 * nbrows <= 512 &&
      tiled_lds <= kernel_info(kt.bounded_tiled[pf][wi]).max_lds) {
    const int Wb = kBoundedWidths[wi];
    std::vector<double> dense(Wb, 0.0);
    for (size_t t = 0; t < interior.off.size(); ++t) dense[omx - interior.off[t]] += interior.w[t];
    const int one = omx;
    fn[0] = kt.bounded_tiled[pf][wi];
    bfn[0] = kt.bounded_tiled_b[pf][wi];
    NL = std::min(512, (std::max(nch, 4 * nbrows) + 63) / 64 * 64);
    shmem[0] = shmem[1] = tiled_lds;
    ntaps = Wb;
    width = W;
    Wbucket = Wb;
    rc = upload((void**)&d_taps, dense.data(), dense.size() * sizeof(double));
    if (!rc) rc = upload((void**)&d_off, &one, sizeof(int));
    // truncated, strictly lower triangular (every offset >= 1): nilpotent,
    // Psi^q = 0 once q * (smallest offset) >= n_x
    if (!fine && omn >= 1) nilq = (nx + omn - 1) / omn;
  } else {
    fn[0] = kt.bounded;
    bfn[0] = kt.bounded_b;
    NL = 256;
    shmem[0] = shmem[1] = (size_t)2 * nx * sizeof(double);
    ntaps = nnz;
    Wbucket = 0;
    rc = upload((void**)&d_taps, interior.w.data(), interior.w.size() * sizeof(double));
    if (!rc) rc = upload((void**)&d_off, interior.off.data(), interior.off.size() * sizeof(int));
  }
  if (!fn[0] || shmem[0] > kernel_info(fn[0]).max_lds) {
    err = "n_x too large for the bounded relaxation kernel";
    return MGRIT_EINVAL;
  }
  if (rc) return rc;
  BoundedDev bd;
  std::memset(&bd, 0, sizeof bd);
  if (Wbucket) {
    bd.padl = padl;
    bd.padr = padr;
  }
  auto put = [&](const std::vector<double>& h, const double** dst) {
    if (h.empty()) return (int)MGRIT_OK;  // an empty block stays NULL
    void* d = nullptr;
    const int r = upload(&d, h.data(), h.size() * sizeof(double));
    if (r) return r;
    d_extra.push_back(d);
    *dst = (const double*)d;
    return MGRIT_OK;
  };
  if (fine) {
    bd.nl = fine->nl;
    bd.ncl = fine->ncl;
    bd.nr = fine->nr;
    bd.ncr = fine->ncr;
    bd.nf = F ? fine->nf : 0;
    if ((rc = put(fine->lblk, &bd.lblk)) || (rc = put(fine->rblk, &bd.rblk))) return rc;
    if (bd.nf > 0 && (rc = put(*F, &bd.F))) return rc;
  }
  if (lanes) {
    bd.rg_a = R.a;
    bd.rg_b = R.b;
    bd.rg_nla = R.nla;
    bd.rg_lw = R.lw;
    bd.rg_bu = R.bu;
    bd.rg_ls = R.ls;
    bd.rg_len = R.len;
    bd.rg_rows = R.rows;
    if ((rc = put(R.coef, &bd.rg_coef))) return rc;
    void* d = nullptr;
    for (int t = 0; t < 2; ++t) {
      const std::vector<int>& h = t ? R.dst : R.cs;
      if ((rc = upload(&d, h.data(), h.size() * sizeof(int)))) return rc;
      d_extra.push_back(d);
      (t ? bd.rg_dst : bd.rg_cs) = (const int*)d;
    }
  }
  return upload(&d_bnd, &bd, sizeof bd);
}

int OpDesc::upload(void** d, const void* h, size_t b) {
  if (dev_alloc(d, b) != MGRIT_OK) return MGRIT_ENOMEM;
  bytes += b;
  if (b == 0) return MGRIT_OK;
  staged.emplace_back((const char*)h, (const char*)h + b);
  if (hipMemcpyAsync(*d, staged.back().data(), b, hipMemcpyHostToDevice, stream) != hipSuccess)
    return MGRIT_EHIP;
  return MGRIT_OK;
}

void OpDesc::release() {
  dev_free(d_taps);
  dev_free(d_off);
  dev_free(d_sdirk);
  dev_free(d_bnd);
  for (void* q : d_extra) dev_free(q);
  d_extra.clear();
  d_bnd = nullptr;
  dev_free(d_mu);
  dev_free(d_tw);
  d_mu = d_tw = nullptr;
  staged.clear();
  d_taps = nullptr;
  d_off = nullptr;
  d_sdirk = nullptr;
}

std::string OpDesc::describe() const {
  char buf[160];
  if (kind == OP_STENCIL) {
    std::string d;
    snprintf(buf, sizeof buf, "stencil<K=%d,W=%d(of %d)> NL=%d omin=%d nnz=%d", K, Wbucket,
             width, NL, omin, nnz);
    d = buf;
    for (int io = 0; io < 2; ++io)
      if (tiled[io].tiles > 1) {
        snprintf(buf, sizeof buf, " %s:%dx%d<K=%d>NL=%d/%d steps", io ? "io" : "plain",
                 tiled[io].tiles, tiled[io].tile, tiled[io].K, tiled[io].NL,
                 tiled[io].max_steps);
        d += buf;
      }
    return d;
  }
  else if (kind == OP_GENERIC)
    snprintf(buf, sizeof buf, "generic ntaps=%d NT=%d", ntaps, NL);
  else if (kind == OP_BOUNDED)
  {
    char kw[64] = "", nq[32] = "";
    if (Wbucket) snprintf(kw, sizeof kw, "<K=%d,W=%d>", bounded_k(Wbucket), Wbucket);
    if (reg_inst >= 0)
      snprintf(kw, sizeof kw, "_lanes<K=%d,HL=%d,HR=%d> rows=%d", kBoundedReg[reg_inst][0],
               kBoundedReg[reg_inst][1], kBoundedReg[reg_inst][2], reg_rows);
    if (nilq) snprintf(nq, sizeof nq, " nilpotent q=%d", nilq);
    snprintf(buf, sizeof buf, "bounded%s ntaps=%d NT=%d%s%s", kw, ntaps, NL,
             d_extra.empty() ? "" : " +boundary rows", nq);
  }
  else if (sdirk_terms)
    snprintf(buf, sizeof buf, "sdirk_pf<K=%d,terms=%d> NL=%d", K, sdirk_terms, NL);
  else
    snprintf(buf, sizeof buf, "sdirk<K=%d> NL=%d", K, NL);
  return buf;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
static RelaxArgs base_args(const Plan& P, const OpDesc& op) {
  RelaxArgs a;
  std::memset(&a, 0, sizeof a);
  a.taps = op.d_taps;
  a.tap_off = op.d_off;
  a.opdata = op.d_sdirk ? op.d_sdirk : op.d_bnd;
  a.ntaps = op.ntaps;
  a.omin = op.omin;
  a.nx = P.nx;
  a.in_stride = 1;
  a.corr_stride = 1;
  a.tile = P.nx;
  a.tiles = 1;
  return a;
}

int Plan::launch(const OpDesc& op, int prec, const RelaxArgs& a, int grid, int cls) {
  // stencil kernels come without per-step memory traffic unless the pass
  // adds a right-hand side every step or stores every state
  const bool io = a.rhs_mode == RHS_EVERY || a.mode == MODE_F;
  RelaxArgs args = a;
  KernelFn fn = op.fn[prec];
  BatchFn bfn = op.bfn[prec];
  int nl = op.NL;
  size_t lds = op.shmem[prec];
  long long blocks = grid;
  parts = grid;
  if (op.kind == OP_STENCIL) {
    const StencilShape* sh = &op.whole[io];
    if (op.tiled[io].tiles > 1 && a.m >= 1 && a.m <= op.tiled[io].max_steps)
      sh = &op.tiled[io];
    fn = sh->fn[prec];
    bfn = sh->bfn[prec];
    nl = sh->NL;
    lds = sh->shmem[prec];
    args.tile = sh->tile;
    args.tiles = sh->tiles;
    args.preload = 0;
    if (io && a.rhs_mode == RHS_EVERY && a.m >= 1 && a.m <= sh->preload_rows) {
      args.preload = 1;
      lds += sizeof(double) * (size_t)a.m * sh->NL * (sh->K + 1);
    }
    blocks = (long long)grid * sh->tiles;
    parts = (int)blocks;
  }
  if (!fn || blocks < 1 || blocks > 0x7fffffffLL) return MGRIT_EINVAL;
  // the lane-resident bounded kernel runs the fine level's passes only
  if (op.reg_inst >= 0 &&
      (a.rhs_mode != RHS_NONE || a.mode == MODE_FW || a.delta || a.sub || a.sub2))
    return MGRIT_EINVAL;
  if (batch) {
    batch->pending.push_back({fn, bfn, nl, lds, blocks, args, this});
    return MGRIT_OK;
  }
  void* kargs[] = {&args};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (profiling) {
    e0 = take_event();
    (void)hipEventRecord(e0, stream);
  }
  hipError_t st =
      hipLaunchKernel((const void*)fn, dim3((unsigned)blocks), dim3(nl), kargs, lds, stream);
  if (st != hipSuccess) return MGRIT_EHIP;
  if (profiling) {
    e1 = take_event();
    (void)hipEventRecord(e1, stream);
    pending.push_back({cls, e0, e1, tag});
  }
  return MGRIT_OK;
}

hipEvent_t Plan::take_event() {
  if (event_pool.empty()) {
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  hipEvent_t e = event_pool.back();
  event_pool.pop_back();
  return e;
}

void Plan::collect_profile() {
  for (auto& p : pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.e0, p.e1);
    prof.ms[p.cls] += ms;
    prof.launches[p.cls] += 1;
    mgrit_prof_entry* e = nullptr;
    for (auto& d : detail)
      if (d.level == p.tag.level && d.pass == p.tag.pass && d.precision == p.tag.prec) e = &d;
    if (!e) {
      mgrit_prof_entry z = {};
      z.level = p.tag.level;
      z.pass = p.tag.pass;
      z.precision = p.tag.prec;
      detail.push_back(z);
      e = &detail.back();
    }
    e->launches += 1;
    e->ms += ms;
    e->bytes += p.tag.bytes;
    e->flops += p.tag.flops;
    event_pool.push_back(p.e0);
    event_pool.push_back(p.e1);
  }
  pending.clear();
}

int Plan::mark_util(int cls, hipEvent_t& e0) {
  if (!profiling) return MGRIT_OK;
  e0 = take_event();
  (void)hipEventRecord(e0, stream);
  (void)cls;
  return MGRIT_OK;
}

void Plan::end_util(int cls, hipEvent_t e0) {
  if (!profiling) return;
  hipEvent_t e1 = take_event();
  (void)hipEventRecord(e1, stream);
  pending.push_back({cls, e0, e1, tag});
}

// Algorithmic HBM bytes and flops of a relaxation launch over `grid`
// workgroup rows: start rows (and corrections), right-hand side rows,
// reference rows, rows written; the operator's flops per point and step.
static ProfTag relax_tag(const OpDesc& op, const RelaxArgs& a, int grid, int level, int prec) {
  ProfTag t;
  t.level = level;
  t.prec = prec;
  t.pass = a.mode == MODE_FC ? MGRIT_PASS_FC : (a.mode == MODE_RES ? MGRIT_PASS_RES : MGRIT_PASS_F);
  const double nint = a.nint, m = a.m;
  double rows = 0.0;
  if (!a.zero_in) rows += grid;
  if (a.corr) rows += grid;
  if (a.sub) rows += grid;
  if (a.sub2) rows += grid;
  if (a.rhs_mode == RHS_EVERY) rows += nint * m;
  if (a.rhs_mode == RHS_CPOINT) rows += nint;
  if (a.mode == MODE_FC) {
    rows += nint + (a.write_row0 ? 1 : 0);
    if (a.delta) rows += (a.zero_in ? 0 : nint) + (a.corr ? nint : 0) + nint;
  } else if (a.mode == MODE_RES) {
    rows += 2.0 * nint + 1.0;  // reference rows read, residual rows (and row 0) written
  } else {
    rows += nint * m + (grid > a.nint ? 1 : 0) + (a.write_last ? nint : 0);
  }
  t.bytes = rows * a.nx * 8.0;
  t.flops = nint * m * a.nx * (op.flops_pps + (a.rhs_mode == RHS_EVERY ? 1.0 : 0.0));
  return t;
}

// Relaxation on level l (0 = fine).  mode: MODE_FC / MODE_RES / MODE_F.
int Plan::relax(int l, int prec, int mode, const double* in, long long in_stride,
                const double* corr, const double* rhs, int rhs_mode, double* out,
                double* partial, int steps, double* delta, const double* sub,
                const double* sub2) {
  Level& L = lev[l];
  const OpDesc& op = L.op;
  RelaxArgs a = base_args(*this, op);
  a.in = in;
  a.in_stride = in_stride;
  a.zero_in = in == nullptr;
  a.corr = corr;
  a.sub = sub;
  a.sub2 = sub2;
  a.rhs = rhs;
  a.rhs_mode = rhs ? rhs_mode : RHS_NONE;
  a.mode = mode;
  a.m = steps;
  a.nint = L.nc;
  a.out = out;
  a.partial = partial;
  if (mode == MODE_FC) {
    a.out_off = 1;
    a.write_row0 = 1;
    a.delta = delta;
  } else if (mode == MODE_RES) {
    a.ref = in;
  }
  const int grid = L.nc + (mode == MODE_F ? 1 : 0);
  if (l == 0) fine_dof_steps += (double)L.nc * steps * nx;
  if (profiling) {
    tag = relax_tag(op, a, grid, l, prec);
    // on coarse levels a homogeneous FC pass is the residual's propagation
    // of the FCF update (cycle() in solve.cpp)
    if (l > 0 && mode == MODE_FC && !rhs) tag.pass = MGRIT_PASS_RES;
  }
  return launch(op, prec, a, grid, l == 0 ? MGRIT_PROF_RELAX_FINE
                                          : (mode == MODE_F ? MGRIT_PROF_OTHER
                                                            : MGRIT_PROF_RELAX_COARSE));
}

// v^j = u^j (+ e^j) for j = 0..nc: the C-points of F-relaxation-only
// (Parareal) iterations, by a zero-step pass.
int Plan::copy_cpoints(int l, int prec, const double* in, long long in_stride,
                       const double* corr, double* out) {
  Level& L = lev[l];
  const OpDesc& op = L.op;
  RelaxArgs a = base_args(*this, op);
  a.in = in;
  a.in_stride = in_stride;
  a.zero_in = in == nullptr;
  a.corr = corr;
  a.mode = MODE_FC;
  a.m = 0;
  a.nint = L.nc + 1;
  a.out = out;
  a.out_off = 0;
  if (profiling) {
    tag = ProfTag();
    tag.level = l;
    tag.pass = MGRIT_PASS_COPY;
    tag.prec = prec;
    tag.bytes = (double)(L.nc + 1) * nx * 8.0 * ((in ? 1 : 0) + (corr ? 1 : 0) + 1);
    tag.flops = corr ? (double)(L.nc + 1) * nx : 0.0;
  }
  return launch(op, prec, a, L.nc + 1, MGRIT_PROF_OTHER);
}

// Coarsest level: x^0 = g^0 = 0, x^{n+1} = Phi_L x^n + g^{n+1}, all points.
// Always FP64 (the sequential coarse solve stays FP64 in every precision).
// The sweep runs in launches of op.seq_chunk steps, each starting from the
// last row the one before stored; this is the launch from step s0.
int Plan::sequential_chunk(int s0, const double* g, bool* last) {
  Level& L = lev.back();
  const OpDesc& op = L.seq;
  if (chunked && s0 == 0) {
    // nilpotent truncated Psi: a step depends on the states of the last
    // nilq steps only, so chunks of nilq steps run in parallel, each from
    // zero nilq steps before its first row (the same values bit for bit)
    RelaxArgs a = base_args(*this, op);
    a.zero_in = 1;
    a.rhs = g;
    a.rhs_mode = RHS_EVERY;
    a.mode = MODE_FW;
    a.m = op.nilq;
    a.tile = op.nilq;
    a.nint = L.n;
    a.out = L.X;
    *last = true;
    if (profiling) {
      tag = ProfTag();
      tag.level = (int)lev.size() - 1;
      tag.pass = MGRIT_PASS_SWEEP;
      tag.bytes = 2.0 * L.n * nx * 8.0;  // right-hand side rows in, solution rows out
      tag.flops = (double)L.n * nx * (op.flops_pps + 1.0);
    }
    return launch(op, 0, a, (L.n + op.nilq - 1) / op.nilq, MGRIT_PROF_COARSEST);
  }
  const int S = op.seq_chunk > 0 ? op.seq_chunk : L.n;
  RelaxArgs a = base_args(*this, op);
  if (s0 == 0) {
    a.zero_in = 1;
  } else {
    a.in = L.X + (long long)s0 * nx;
    a.skip_row0 = 1;
  }
  a.rhs = g + (long long)s0 * nx;
  a.rhs_mode = RHS_EVERY;
  a.mode = MODE_F;
  a.m = std::min(S, L.n - s0);
  a.nint = 1;
  a.write_last = 1;
  a.out = L.X + (long long)s0 * nx;
  *last = s0 + S >= L.n;
  if (profiling) {
    tag = ProfTag();
    tag.level = (int)lev.size() - 1;
    tag.pass = MGRIT_PASS_SWEEP;
    // start row (after the first launch), right-hand side rows, rows stored
    tag.bytes = ((s0 ? 1.0 : 0.0) + 2.0 * a.m + (s0 ? 0.0 : 1.0)) * nx * 8.0;
    tag.flops = (double)a.m * nx * (op.flops_pps + 1.0);
  }
  return launch(op, 0, a, 1, MGRIT_PROF_COARSEST);
}

int Batch::flush() {
  const size_t n = pending.size();
  std::vector<char> used(n, 0);
  int rc = MGRIT_OK;
  for (size_t i = 0; i < n && rc == MGRIT_OK; ++i) {
    if (used[i]) continue;
    const Entry& e = pending[i];
    // members joining entry i: same kernel and shape, at most one entry per
    // plan, and no earlier entry of their plan still waiting
    std::vector<size_t> grp(1, i);
    used[i] = 1;
    for (size_t k = i + 1; k < n && grp.size() < (size_t)kMaxBatch && e.bfn; ++k) {
      const Entry& f = pending[k];
      if (used[k] || f.fn != e.fn || f.nl != e.nl || f.lds != e.lds) continue;
      bool ok = true;
      for (size_t q = i; q < k && ok; ++q)
        if (pending[q].owner == f.owner && (!used[q] || std::find(grp.begin(), grp.end(), q) != grp.end()))
          ok = false;
      if (!ok) continue;
      grp.push_back(k);
      used[k] = 1;
    }
    hipError_t st;
    if (grp.size() == 1) {
      RelaxArgs args = e.args;
      void* kargs[] = {&args};
      st = hipLaunchKernel((const void*)e.fn, dim3((unsigned)e.blocks), dim3(e.nl), kargs, e.lds,
                           stream);
    } else {
      BatchArgs b;
      std::memset(&b, 0, sizeof b);
      long long total = 0;
      for (size_t q = 0; q < grp.size(); ++q) {
        b.a[q] = pending[grp[q]].args;
        b.start[q] = (int)total;
        total += pending[grp[q]].blocks;
        pending[grp[q]].owner->stats.batched_launches += 1;
      }
      b.n = (int)grp.size();
      if (total > 0x7fffffffLL || kernel_info((KernelFn)e.bfn).max_lds < e.lds) {
        rc = MGRIT_EINVAL;
        break;
      }
      void* kargs[] = {&b};
      st = hipLaunchKernel((const void*)e.bfn, dim3((unsigned)total), dim3(e.nl), kargs, e.lds,
                           stream);
      merged += (long long)grp.size();
    }
    if (st != hipSuccess) rc = MGRIT_EHIP;
    ++launches;
  }
  pending.clear();
  return rc;
}

}  // namespace mgr

namespace mgr {
// Device bytes of a plan's space-time arrays (everything but the taps).
size_t plan_state_bytes(int nx, int nt, int m, int levels, int precision) {
  const size_t row = (size_t)nx * sizeof(double);
  const long long nc = nt / m;
  size_t b = 3 * (size_t)(nc + 1) * row;                       // V_a, V_b, R_1
  if (precision != MGRIT_FP64) b += 2 * (size_t)(nc + 1) * row;  // U, R_out
  long long n = nt;
  for (int l = 1; l < levels; ++l) {
    n /= m;
    b += (size_t)(n + 1) * row;                                 // X_l
    if (l < levels - 1) b += 3 * (size_t)(n / m + 1) * row;     // V_l, W_l, R_l
  }
  b += ((size_t)(nc + 1) * kMaxFineTiles + 1) * sizeof(double);  // partials, norm
  if (spectral_supported(nx))  // spectral coarsest solve: rows, eigenvalues, twiddles
    b += spectral_rows((int)n) * nx * 16 + (size_t)nx * 16 + (size_t)(nx / 2) * 16;
  return b;
}

// Modelled time of one spectral coarsest-level solve of n steps (row
// transforms, mode recurrences, inverse transforms) on MI355X: a fixed part
// per row length (the three launches and the latency of one row's
// transforms, measured at each power of two from 512 up; 14 us below) plus
// 11 ps per point and step (the solve's 80 bytes of traffic per point and
// step at about 7 TB/s).  Fitted to 16 measured shapes, n_x = 512..8192 and
// n = 16..1024: within 20 %.
static double spectral_time_us(int nx, int n) {
  // fixed part at n_x = 2^8 .. 2^13
  static const double base[] = {14.0, 14.7, 16.2, 17.8, 20.0, 31.5};
  int lg = 0;
  while ((1 << lg) < nx) ++lg;
  const double b = base[std::min(std::max(lg, 8), 13) - 8];
  return b + 1.1e-5 * (double)(n + 1) * nx;
}

int Plan::set_coarse_mode(int mode) {
  if (mode != MGRIT_COARSE_AUTO && mode != MGRIT_COARSE_SWEEP && mode != MGRIT_COARSE_SPECTRAL)
    return MGRIT_EINVAL;
  if (mode == MGRIT_COARSE_SPECTRAL && !Sspec) return MGRIT_EINVAL;
  coarse_mode = mode;
  spectral = Sspec && (mode == MGRIT_COARSE_SPECTRAL ||
                       (mode == MGRIT_COARSE_AUTO && spectral_us < lev.back().seq.seq_us));
  const OpDesc& cs = lev.back().seq;
  chunked = mode == MGRIT_COARSE_AUTO && cs.kind == OP_BOUNDED && cs.nilq > 0 &&
            2 * cs.nilq < lev.back().n;
  description = description_levels + (spectral ? " (spectral solve)" : "") +
                (chunked ? " (chunked sweep)" : "");
  return MGRIT_OK;
}
}  // namespace mgr

using namespace mgr;

namespace mgr {

// The current device must be a gfx950; the answer is cached per device.
static int check_device() {
  static std::atomic<int> known[64];  // 0 unknown, 1 gfx950, 2 other
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return MGRIT_ENODEV;
  if (dev < 64 && known[dev].load() != 0) return known[dev].load() == 1 ? MGRIT_OK : MGRIT_ENODEV;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MGRIT_ENODEV;
  const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
  if (dev < 64) known[dev].store(ok ? 1 : 2);
  return ok ? MGRIT_OK : MGRIT_ENODEV;
}

// Device blocks of plans.  A released block is kept and handed to a later
// request of the same size class (four classes per power of two, so at most
// 25 % above the bytes asked for) on the same device: giving a block back to
// the driver costs up to several hundred microseconds and taking it again
// tens, which a server that builds and drops a plan per request would pay on
// every array.  Callers release a block only when no queued work uses it
// any more.  At most kCacheCap bytes are kept; dev_trim() frees them all.
namespace {
constexpr size_t kCacheCap = (size_t)16 << 30;
std::mutex g_blk_mu;
std::map<std::pair<int, size_t>, std::vector<void*>> g_blk_free;
std::unordered_map<void*, std::pair<int, size_t>> g_blk_live;
size_t g_blk_cached = 0;

size_t size_class(size_t b) {
  b = std::max<size_t>(b, 4096);
  int p = 63 - __builtin_clzll((unsigned long long)b);
  const size_t step = (size_t)1 << (p - 2);
  return (b + step - 1) / step * step;
}
}  // namespace

thread_local Arena* t_arena = nullptr;

void set_thread_arena(Arena* a) { t_arena = a; }

static bool in_arena(const void* p) {
  const Arena* a = t_arena;
  return a && (const char*)p >= a->base && (const char*)p < a->base + a->cap;
}

int dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (Arena* a = t_arena) {
    const size_t off = (a->used + 255) & ~(size_t)255;
    if (off > a->cap || bytes > a->cap - off) {
      a->overflow = true;
      return MGRIT_ENOMEM;
    }
    *p = a->base + off;
    a->used = off + bytes;
    return MGRIT_OK;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MGRIT_ENODEV;
  const size_t c = size_class(bytes);
  {
    std::lock_guard<std::mutex> lk(g_blk_mu);
    auto it = g_blk_free.find({dev, c});
    if (it != g_blk_free.end() && !it->second.empty()) {
      *p = it->second.back();
      it->second.pop_back();
      g_blk_cached -= c;
      g_blk_live[*p] = {dev, c};
      return MGRIT_OK;
    }
  }
  if (hipMalloc(p, c) != hipSuccess) {
    (void)hipGetLastError();
    dev_trim();
    if (hipMalloc(p, c) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return MGRIT_ENOMEM;
    }
  }
  std::lock_guard<std::mutex> lk(g_blk_mu);
  g_blk_live[*p] = {dev, c};
  return MGRIT_OK;
}

void dev_free(void* p) {
  if (!p || in_arena(p)) return;
  {
    std::lock_guard<std::mutex> lk(g_blk_mu);
    auto it = g_blk_live.find(p);
    if (it != g_blk_live.end()) {
      const auto key = it->second;
      g_blk_live.erase(it);
      if (g_blk_cached + key.second <= kCacheCap) {
        g_blk_free[key].push_back(p);
        g_blk_cached += key.second;
        return;
      }
    }
  }
  (void)hipFree(p);
}

void dev_trim() {
  std::vector<void*> all;
  {
    std::lock_guard<std::mutex> lk(g_blk_mu);
    for (auto& kv : g_blk_free)
      for (void* q : kv.second) all.push_back(q);
    g_blk_free.clear();
    g_blk_cached = 0;
  }
  for (void* q : all) (void)hipFree(q);
}

// Pinned host words that receive residual norms, one per plan.  They come
// from slabs kept until the process ends: releasing pinned memory waits for
// the whole device, which would stall every other stream at each plan's end.
std::mutex g_word_mu;
std::vector<double*> g_free_words;

static double* take_host_word() {
  if (t_arena) return &t_arena->host_word;
  std::lock_guard<std::mutex> lk(g_word_mu);
  if (g_free_words.empty()) {
    constexpr int kSlab = 1024;
    double* slab = nullptr;
    if (hipHostMalloc((void**)&slab, kSlab * sizeof(double)) != hipSuccess) return nullptr;
    for (int i = kSlab - 1; i >= 0; --i) g_free_words.push_back(slab + i);
  }
  double* w = g_free_words.back();
  g_free_words.pop_back();
  return w;
}

static void give_host_word(double* w) {
  if (!w || (t_arena && w == &t_arena->host_word)) return;
  std::lock_guard<std::mutex> lk(g_word_mu);
  g_free_words.push_back(w);
}

}  // namespace mgr

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

int mgrit_version(void) { return 100; }

const char* mgrit_strerror(int code) {
  switch (code) {
    case MGRIT_OK: return "success";
    case MGRIT_EINVAL: return "invalid argument or unsupported shape";
    case MGRIT_EUNSTABLE: return "Courant number above the CFL limit of the explicit scheme";
    case MGRIT_ENOMEM: return "allocation failed";
    case MGRIT_EHIP: return "HIP runtime error";
    case MGRIT_ENOTCONV: return "maximum iterations reached above tolerance";
    case MGRIT_EDIVERGED: return "non-finite residual norm";
    case MGRIT_EIMAG: return "least-squares solution has imaginary part above 1e-8";
    case MGRIT_ENODEV: return "no usable gfx950 device";
    case MGRIT_ECAPACITY: return "output arrays too small";
    case MGRIT_EBUSY: return "admission refused: HBM budget";
    case MGRIT_ESCRATCH: return "plan does not fit the static workspace of mgrit_solve_static";
    default: return "unknown error";
  }
}

int mgrit_max_amplification(int scheme, double cfl, double* amp) {
  Tableau t;
  if (!amp || !get_tableau(scheme, t) || !(cfl > 0.0)) return MGRIT_EINVAL;
  *amp = max_amplification(t, cfl);
  return MGRIT_OK;
}

int mgrit_phi_taps(int scheme, double cfl, int nx, int capacity, int* offsets,
                   double* weights, int* nnz) {
  Tableau t;
  if (!get_tableau(scheme, t) || nx < 1 || !nnz || !(cfl > 0.0)) return MGRIT_EINVAL;
  if (t.implicit) return MGRIT_EINVAL;
  Taps tp;
  erk_taps(t, cfl, nx, tp);
  *nnz = (int)tp.off.size();
  if ((int)tp.off.size() > capacity) return MGRIT_ECAPACITY;
  if (!offsets || !weights) return MGRIT_EINVAL;
  for (size_t i = 0; i < tp.off.size(); ++i) {
    offsets[i] = tp.off[i];
    weights[i] = tp.w[i];
  }
  return MGRIT_OK;
}

int mgrit_psi_optimize(int scheme, double cfl, int nx, int m, int levels, int rule,
                       const int* widths, double eta, mgrit_taps* out, double* max_imag) {
  if (!out) return MGRIT_EINVAL;
  std::vector<Taps> h;
  double mi = 0.0;
  int rc;
  try {
    rc = psi_hierarchy(scheme, cfl, nx, m, levels, rule, widths, eta, h, mi);
  } catch (...) {
    return MGRIT_ENOMEM;
  }
  if (rc != MGRIT_OK && rc != MGRIT_EIMAG) return rc;
  if (max_imag) *max_imag = mi;
  for (int l = 0; l < levels - 1; ++l) {
    const Taps& t = h[l];
    if ((int)t.off.size() > out[l].nnz || !out[l].offset || !out[l].weight) {
      out[l].nnz = (int)t.off.size();
      return MGRIT_ECAPACITY;
    }
    out[l].nnz = (int)t.off.size();
    for (size_t i = 0; i < t.off.size(); ++i) {
      out[l].offset[i] = t.off[i];
      out[l].weight[i] = t.w[i];
    }
  }
  return rc;
}

int mgrit_psi_optimize_bound(int scheme, double cfl, int nx, int nt, int m, int levels,
                             double target, mgrit_taps* out, double* bounds,
                             double* max_imag) {
  if (!out) return MGRIT_EINVAL;
  std::vector<Taps> h;
  std::vector<double> b;
  double mi = 0.0;
  int rc;
  try {
    rc = psi_hierarchy_bound(scheme, cfl, nx, nt, m, levels, target, MGRIT_PSI_BOUND_MAX_WIDTH, h,
                             b, mi);
  } catch (...) {
    return MGRIT_ENOMEM;
  }
  if (rc != MGRIT_OK && rc != MGRIT_EIMAG) return rc;
  if (max_imag) *max_imag = mi;
  for (int l = 0; l < levels - 1; ++l) {
    const Taps& t = h[l];
    if ((int)t.off.size() > out[l].nnz || !out[l].offset || !out[l].weight) {
      out[l].nnz = (int)t.off.size();
      return MGRIT_ECAPACITY;
    }
    out[l].nnz = (int)t.off.size();
    for (size_t i = 0; i < t.off.size(); ++i) {
      out[l].offset[i] = t.off[i];
      out[l].weight[i] = t.w[i];
    }
    if (bounds) bounds[l] = b[l];
  }
  return rc;
}


}  // extern "C"

namespace mgr {

// Plans of both problems: periodic (inflow == NULL) or with inflow/outflow
// boundaries and the inflow data rows of mgrit_plan_create_inflow.
static int plan_create(mgrit_plan_t* out, int nx, int nt, double alpha, double cfl,
                       int scheme, int m, int levels, const mgrit_taps* psi, int cycle,
                       int relax, int precision, void* hip_stream, const double* inflow,
                       int n_derivs) {
  if (!out) return MGRIT_EINVAL;
  *out = nullptr;
  Tableau t;
  if (!get_tableau(scheme, t) || nx < 2 || nt < 1 || m < 2 || levels < 2 ||
      !(alpha > 0.0) || !(cfl > 0.0) || !psi)
    return MGRIT_EINVAL;
  if (inflow && (t.implicit || precision != MGRIT_FP64 || n_derivs < t.p + 1))
    return MGRIT_EINVAL;
  if (cycle != MGRIT_CYCLE_V && cycle != MGRIT_CYCLE_F) return MGRIT_EINVAL;
  if (relax != MGRIT_RELAX_FCF && relax != MGRIT_RELAX_F) return MGRIT_EINVAL;
  if (precision != MGRIT_FP64 && precision != MGRIT_FP32_RELAX && precision != MGRIT_FP32_IR)
    return MGRIT_EINVAL;
  long long span = 1;
  for (int l = 1; l < levels; ++l) span *= m;
  if (span > nt || nt % span) return MGRIT_EINVAL;
  for (int l = 0; l < levels - 1; ++l)
    if (psi[l].nnz < 1 || !psi[l].offset || !psi[l].weight) return MGRIT_EINVAL;
  if (!t.implicit && max_amplification(t, cfl) > 1.0 + 1e-6) return MGRIT_EUNSTABLE;
  int rc = check_device();
  if (rc) return rc;

  Plan* P = new (std::nothrow) Plan();
  if (!P) return MGRIT_ENOMEM;
  P->nx = nx;
  P->nt = nt;
  P->m = m;
  P->scheme = scheme;
  P->alpha = alpha;
  P->cfl = cfl;
  P->cycle_kind = cycle;
  P->relax_kind = relax;
  P->precision = precision;
  P->inflow = inflow != nullptr;
  P->dx = 2.0 / nx;
  P->dt = cfl * P->dx / alpha;
  P->scale = std::sqrt(P->dx * P->dt);
  P->stream = (hipStream_t)hip_stream;
  std::string err;
  auto fail = [&](int code) {
    mgrit_destroy(reinterpret_cast<mgrit_plan_t>(P));
    return code;
  };
  try {
    P->lev.resize(levels);
    long long n = nt;
    for (int l = 0; l < levels; ++l) {
      Level& L = P->lev[l];
      L.op.stream = L.seq.stream = P->stream;
      L.n = (int)n;
      L.nc = (l < levels - 1) ? (int)(n / m) : 0;
      if (inflow && l == 0) {
        InflowOp fop;
        rc = inflow_setup(t, cfl, alpha, nx, fop, err);
        if (!rc) {
          // forcing of the step from t_n: row n = B g^(0..p)(t_n)
          std::vector<double> F((size_t)nt * fop.nf, 0.0);
          for (long long r = 0; r < nt; ++r)
            for (int i = 0; i < fop.nf; ++i) {
              double v = 0.0;
              for (int d = 0; d < fop.nd; ++d)
                v += fop.B[(size_t)i * fop.nd + d] * inflow[r * n_derivs + d];
              F[(size_t)r * fop.nf + i] = v;
            }
          rc = L.op.init_bounded(fop.interior, &fop, &F, nx, m, err);
        }
      } else if (inflow) {
        // the periodic Psi truncated to the interval (signed offsets)
        Taps f;
        for (int i = 0; i < psi[l - 1].nnz; ++i) {
          int o = ((psi[l - 1].offset[i] % nx) + nx) % nx;
          if (o > nx / 2) o -= nx;
          f.off.push_back(o);
          f.w.push_back(psi[l - 1].weight[i]);
        }
        if (l < levels - 1) rc = L.op.init_bounded(f, nullptr, nullptr, nx, m, err);
        else rc = L.seq.init_bounded(f, nullptr, nullptr, nx, m, err);
      } else if (l == 0) {
        if (t.implicit) rc = L.op.init_sdirk(t, cfl, nx, err);
        else {
          Taps f;
          erk_taps(t, cfl, nx, f);
          rc = L.op.init_stencil(f, nx, m, (int)(n / m), false, kMaxFineTiles, err);
        }
      } else {
        Taps f;
        f.off.assign(psi[l - 1].offset, psi[l - 1].offset + psi[l - 1].nnz);
        f.w.assign(psi[l - 1].weight, psi[l - 1].weight + psi[l - 1].nnz);
        if (l < levels - 1) rc = L.op.init_stencil(f, nx, m, (int)(n / m), false, 1 << 20, err);
        else rc = L.seq.init_stencil(f, nx, (int)n, 1, true, 1 << 20, err);
      }
      if (rc) return fail(rc);
      P->bytes += L.op.bytes + L.seq.bytes;
      n /= m;
    }
    // device buffers
    auto alloc = [&](double** p, long long rows) {
      size_t b = (size_t)rows * nx * sizeof(double);
      if (dev_alloc((void**)p, b) != MGRIT_OK) return false;
      P->bytes += b;
      return true;
    };
    const long long nc = nt / m;
    if (!alloc(&P->Va, nc + 1) || !alloc(&P->Vb, nc + 1) || !alloc(&P->lev[0].R, nc + 1))
      return fail(MGRIT_ENOMEM);
    if (precision != MGRIT_FP64 && (!alloc(&P->U, nc + 1) || !alloc(&P->Rout, nc + 1)))
      return fail(MGRIT_ENOMEM);
    for (int l = 1; l < levels; ++l) {
      Level& L = P->lev[l];
      if (!alloc(&L.X, L.n + 1)) return fail(MGRIT_ENOMEM);
      if (l < levels - 1 &&
          (!alloc(&L.V, L.nc + 1) || !alloc(&L.W, L.nc + 1) || !alloc(&L.R, L.nc + 1)))
        return fail(MGRIT_ENOMEM);
    }
    if (dev_alloc((void**)&P->partial, (size_t)(nc + 1) * kMaxFineTiles * sizeof(double)) !=
            MGRIT_OK ||
        dev_alloc((void**)&P->d_norm, sizeof(double)) != MGRIT_OK ||
        !(P->h_norm = take_host_word()))
      return fail(MGRIT_ENOMEM);
    P->bytes += ((size_t)(nc + 1) * kMaxFineTiles + 1) * sizeof(double);
    if (!inflow && spectral_supported(nx)) {
      // the coarsest stencil's eigenvalues and the transform's twiddles
      Level& C = P->lev.back();
      Taps f;
      f.off.assign(psi[levels - 2].offset, psi[levels - 2].offset + psi[levels - 2].nnz);
      f.w.assign(psi[levels - 2].weight, psi[levels - 2].weight + psi[levels - 2].nnz);
      std::vector<cd> mu, tw(nx / 2);
      taps_eigs(f, nx, mu);
      for (int q = 0; q < nx / 2; ++q) {
        const double a = -6.283185307179586476925286766559 * (double)q / (double)nx;
        tw[q] = cd(std::cos(a), std::sin(a));
      }
      const size_t before = C.seq.bytes;
      if (C.seq.upload((void**)&C.seq.d_mu, mu.data(), mu.size() * sizeof(cd)) ||
          C.seq.upload((void**)&C.seq.d_tw, tw.data(), tw.size() * sizeof(cd)) ||
          dev_alloc((void**)&P->Sspec, spectral_rows(C.n) * nx * sizeof(cd)) != MGRIT_OK)
        return fail(MGRIT_ENOMEM);
      P->bytes += C.seq.bytes - before + spectral_rows(C.n) * nx * sizeof(cd);
      P->spectral_us = spectral_time_us(nx, C.n);
    }
    std::string d;
    for (int l = 0; l < levels; ++l) {
      const OpDesc& o = (l == levels - 1) ? P->lev[l].seq : P->lev[l].op;
      char hdr[64];
      snprintf(hdr, sizeof hdr, "L%d n=%d: ", l + 1, P->lev[l].n);
      d += hdr + o.describe() + (l + 1 < levels ? "; " : "");
    }
    P->description_levels = d;
    (void)P->set_coarse_mode(MGRIT_COARSE_AUTO);
  } catch (...) {
    return fail(MGRIT_ENOMEM);
  }
  // allocations and uploads were queued on the plan's stream
  if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(MGRIT_EHIP);
  for (auto& L : P->lev) {
    L.op.staged.clear();
    L.seq.staged.clear();
  }
  *out = reinterpret_cast<mgrit_plan_t>(P);
  return MGRIT_OK;
}

}  // namespace mgr

extern "C" {

int mgrit_plan_create(mgrit_plan_t* out, int nx, int nt, double alpha, double cfl,
                      int scheme, int m, int levels, const mgrit_taps* psi, int cycle,
                      int relax, int precision, void* hip_stream) {
  return plan_create(out, nx, nt, alpha, cfl, scheme, m, levels, psi, cycle, relax, precision,
                     hip_stream, nullptr, 0);
}

int mgrit_plan_create_inflow(mgrit_plan_t* out, int nx, int nt, double alpha, double cfl,
                             int scheme, int m, int levels, const mgrit_taps* psi, int cycle,
                             int relax, const double* inflow, int n_derivs, void* hip_stream) {
  if (!inflow) return MGRIT_EINVAL;
  return plan_create(out, nx, nt, alpha, cfl, scheme, m, levels, psi, cycle, relax, MGRIT_FP64,
                     hip_stream, inflow, n_derivs);
}

int mgrit_inflow_operator(int scheme, double cfl, double alpha, int nx, double* phi, double* B,
                          int* n_derivs) {
  Tableau t;
  if (!get_tableau(scheme, t) || t.implicit || nx < 2 || !(cfl > 0.0) || !(alpha > 0.0) ||
      !n_derivs)
    return MGRIT_EINVAL;
  InflowOp op;
  std::string err;
  int rc;
  try {
    rc = inflow_setup(t, cfl, alpha, nx, op, err);
  } catch (...) {
    return MGRIT_ENOMEM;
  }
  if (rc) return rc;
  *n_derivs = op.nd;
  if (phi)
    for (int i = 0; i < nx; ++i)
      for (int c = 0; c < nx; ++c) phi[(size_t)i * nx + c] = inflow_entry(op, nx, i, c);
  if (B)
    for (int i = 0; i < nx; ++i)
      for (int d = 0; d < op.nd; ++d)
        B[(size_t)i * op.nd + d] = i < op.nf ? op.B[(size_t)i * op.nd + d] : 0.0;
  return MGRIT_OK;
}

void mgrit_destroy(mgrit_plan_t plan) {
  if (!plan) return;
  Plan* P = reinterpret_cast<Plan*>(plan);
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  else (void)hipDeviceSynchronize();
  for (auto& L : P->lev) {
    L.op.release();
    L.seq.release();
    dev_free(L.X);
    dev_free(L.V);
    dev_free(L.W);
    dev_free(L.R);
  }
  for (double* p : {P->Va, P->Vb, P->U, P->Rout, P->partial, P->d_norm, P->Sspec}) dev_free(p);
  give_host_word(P->h_norm);
  for (auto& p : P->pending) {
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
  }
  for (auto e : P->event_pool) (void)hipEventDestroy(e);
  delete P;
}

int mgrit_plan_estimate_bytes(int nx, int nt, int m, int levels, int precision,
                              size_t* bytes) {
  if (!bytes || nx < 1 || nt < 1 || m < 2 || levels < 2) return MGRIT_EINVAL;
  // space-time arrays plus a bound on the per-level taps and stage data
  *bytes = plan_state_bytes(nx, nt, m, levels, precision) + (size_t)levels * 64 * 1024;
  return MGRIT_OK;
}

int mgrit_plan_bytes(mgrit_plan_t plan, size_t* b) {
  if (!plan || !b) return MGRIT_EINVAL;
  *b = reinterpret_cast<Plan*>(plan)->bytes;
  return MGRIT_OK;
}

int mgrit_plan_set_seed(mgrit_plan_t plan, unsigned long long seed) {
  if (!plan) return MGRIT_EINVAL;
  reinterpret_cast<Plan*>(plan)->seed = seed;
  return MGRIT_OK;
}

int mgrit_plan_set_coarse_solver(mgrit_plan_t plan, int mode) {
  if (!plan) return MGRIT_EINVAL;
  return reinterpret_cast<Plan*>(plan)->set_coarse_mode(mode);
}

int mgrit_get_stats(mgrit_plan_t plan, mgrit_stats* s) {
  if (!plan || !s) return MGRIT_EINVAL;
  *s = reinterpret_cast<Plan*>(plan)->stats;
  return MGRIT_OK;
}

int mgrit_set_profiling(mgrit_plan_t plan, int enable) {
  if (!plan) return MGRIT_EINVAL;
  Plan* P = reinterpret_cast<Plan*>(plan);
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  else (void)hipDeviceSynchronize();
  P->collect_profile();
  P->profiling = enable != 0;
  if (enable) {
    std::memset(&P->prof, 0, sizeof P->prof);
    P->detail.clear();
    P->prof_dof_base = P->fine_dof_steps;
  }
  return MGRIT_OK;
}

int mgrit_get_profile(mgrit_plan_t plan, mgrit_profile* prof) {
  if (!plan || !prof) return MGRIT_EINVAL;
  Plan* P = reinterpret_cast<Plan*>(plan);
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  else (void)hipDeviceSynchronize();
  P->collect_profile();
  *prof = P->prof;
  prof->fine_dof_steps = P->fine_dof_steps - P->prof_dof_base;
  return MGRIT_OK;
}

int mgrit_get_profile_detail(mgrit_plan_t plan, mgrit_prof_entry* out, int capacity,
                             int* count) {
  if (!plan || !count || capacity < 0 || (capacity > 0 && !out)) return MGRIT_EINVAL;
  Plan* P = reinterpret_cast<Plan*>(plan);
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  else (void)hipDeviceSynchronize();
  P->collect_profile();
  std::vector<mgrit_prof_entry> d = P->detail;
  std::sort(d.begin(), d.end(), [](const mgrit_prof_entry& x, const mgrit_prof_entry& y) {
    if (x.level != y.level) return x.level < y.level;
    if (x.pass != y.pass) return x.pass < y.pass;
    return x.precision < y.precision;
  });
  *count = (int)d.size();
  for (int i = 0; i < capacity && i < (int)d.size(); ++i) out[i] = d[i];
  return MGRIT_OK;
}

int mgrit_operator_complexity(mgrit_plan_t plan, double* oc) {
  if (!plan || !oc) return MGRIT_EINVAL;
  Plan* P = reinterpret_cast<Plan*>(plan);
  // eq. (10); the fine SDIRK stepper has no finite nnz: report NaN
  const int L = (int)P->lev.size();
  double n1 = P->lev[0].op.nnz;
  if (n1 <= 0) {
    *oc = NAN;
    return MGRIT_OK;
  }
  double s = 0.0, f = 1.0;
  for (int l = 0; l < L; ++l) {
    const OpDesc& o = (l == L - 1) ? P->lev[l].seq : P->lev[l].op;
    s += f * o.nnz;
    f /= P->m;
  }
  *oc = s / n1;
  return MGRIT_OK;
}

const char* mgrit_plan_describe(mgrit_plan_t plan) {
  if (!plan) return "";
  return reinterpret_cast<Plan*>(plan)->description.c_str();
}

int phi_apply_batch(mgrit_plan_t plan, const double* in, double* out, int batch,
                    int ksteps) {
  if (!plan || batch < 0 || ksteps < 0) return MGRIT_EINVAL;
  if (batch == 0) return MGRIT_OK;  // nothing to do (the rows may be NULL)
  if (!in || !out) return MGRIT_EINVAL;
  Plan* P = reinterpret_cast<Plan*>(plan);
  const OpDesc& op = P->lev[0].op;
  RelaxArgs a = base_args(*P, op);
  a.in = in;
  a.mode = MODE_FC;
  a.m = ksteps;
  a.nint = batch;
  a.out = out;
  a.out_off = 0;
  if (op.kind == OP_BOUNDED) {
    // every row steps from t = 0 with the plan's inflow data (n_t rows)
    if (ksteps > P->nt) return MGRIT_EINVAL;
    a.omin = 0;
  }
  const int prec = P->precision != MGRIT_FP64 ? 1 : 0;
  if (P->profiling) P->tag = relax_tag(op, a, batch, 0, prec);
  return P->launch(op, prec, a, batch, MGRIT_PROF_RELAX_FINE);
}

}  // extern "C"
