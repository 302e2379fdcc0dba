// Spectral solve of the coarsest level's system x^0 = 0,
// x^{s} = Psi x^{s-1} + g^{s} (s = 1..n) for a periodic stencil Psi.
//
// Psi is circulant (Sec. 4.1), so the discrete Fourier transform
// diagonalises it: with hat(u)_k = sum_i u_i e^{-2 pi i k i / n_x} and
// mu_k = sum_t w_t e^{-2 pi i k o_t / n_x} (its eigenvalues),
// hat(Psi u)_k = mu_k hat(u)_k and every mode obeys its own scalar
// recurrence hat(x)^{s}_k = mu_k hat(x)^{s-1}_k + hat(g)^{s}_k.  The n steps
// that a sweep takes one after the other become: a transform of every row
// (all rows at once), one recurrence per mode (all modes at once), and an
// inverse transform of every row.  The result is the sweep's up to rounding.
//
// Transforms: one workgroup per row.  A real row x of n_x points is
// transformed as the N = n_x/2 complex points z_n = x_{2n} + i x_{2n+1}
// (the row's own memory read as complex values): with Z = DFT_N(z),
// E_k = (Z_k + conj Z_{N-k})/2 and O_k = (Z_k - conj Z_{N-k})/(2i) are the
// transforms of the even and odd points, and hat(x)_k = E_k + w^k O_k,
// w = e^{-2 pi i / n_x}.  Modes k = 0..N are kept; the others are their
// conjugates (the row is real), and so are those of every later row (Psi
// is real).  The inverse runs the same identities backwards.
//
// The N-point transform is radix-2 in passes of up to three stages held in
// registers.  The forward transform decimates in frequency (natural order
// in, bit-reversed order out) and the inverse in time (bit-reversed order
// in, natural order out), so neither touches global memory out of order:
// the first forward pass and the last inverse pass read and write rows
// coalesced, and the bit-reversed order lives only in LDS, where the
// even/odd split reads and writes it.  LDS holds the N points (one pad slot
// every 16 against bank conflicts) and the n_x/2 twiddles e^{-2 pi i q/n_x}
// (the N-point transform uses the even ones).
#include <hip/hip_runtime.h>

#include <mutex>

#include "registry.h"

namespace mgr {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

constexpr int kRadixLg = 3;   // stages per register pass
constexpr int kMaxLgN = 12;   // N = n_x/2 <= 4096

__device__ __forceinline__ int bitrev(int i, int lg) {
  return (int)(__builtin_bitreverse32((unsigned)i) >> (32 - lg));
}
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// Threads of a row transform of N = 2^LG complex points: one group of 2^R1
// points each in the first pass (R1 = min(LG, 3); every group has its
// thread), at least one wavefront.
template <int LG>
constexpr int fft_threads() {
  constexpr int R1 = LG < kRadixLg ? LG : kRadixLg;
  constexpr int t = (1 << LG) >> R1;
  static_assert(t <= 1024, "one first-pass group per thread");
  return t < 64 ? 64 : t;
}
// LDS: the N points (padded), then the n_x/2 = N twiddles
constexpr size_t fft_lds(int N) {
  return sizeof(double2) * ((size_t)N + N / 16 + 1 + (size_t)N);
}

// Decimation-in-frequency stages u = TOP .. TOP-R+1 (pairs 2^u apart) on the
// group base + m 2^LO (m < 2^R, LO = TOP-R+1; base has zero bits LO..TOP)
// held in registers.  The twiddle of pair (i, i + 2^u) is W_{2^(u+1)}^i =
// tl[i << (LG - u)].
template <int R, int LG, int TOP>
__device__ __forceinline__ void dif_butterflies(double2 (&v)[1 << R], int base,
                                                const double2* tl) {
  constexpr int LO = TOP - R + 1;
#pragma unroll
  for (int r = R - 1; r >= 0; --r) {
    const int u = LO + r;
    const int bl = base & ((1 << u) - 1);
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) {
      if (m & (1 << r)) continue;
      const int i = bl + ((m << LO) & ((1 << u) - 1));
      const double2 a = v[m], c = v[m + (1 << r)];
      v[m] = cadd(a, c);
      v[m + (1 << r)] = cmul(csub(a, c), tl[i << (LG - u)]);
    }
  }
}

// Decimation-in-time stages u = LO .. LO+R-1 of the inverse transform
// (conjugate twiddles) on the same kind of group.
template <int R, int LG, int LO>
__device__ __forceinline__ void dit_butterflies(double2 (&v)[1 << R], int base,
                                                const double2* tl) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int u = LO + r;
    const int bl = base & ((1 << u) - 1);
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) {
      if (m & (1 << r)) continue;
      const int i = bl + ((m << LO) & ((1 << u) - 1));
      const double2 t = cmulc(v[m + (1 << r)], tl[i << (LG - u)]);
      v[m + (1 << r)] = csub(v[m], t);
      v[m] = cadd(v[m], t);
    }
  }
}

// group g of a pass over bits LO..TOP: g with a zero field at LO..TOP
template <int LO, int TOP>
__device__ __forceinline__ int group_base(int g) {
  return (g & ((1 << LO) - 1)) | ((g >> LO) << (TOP + 1));
}

// Forward passes after the first, down to stage 0, in place in LDS; each
// ends with a barrier.
template <int LG, int TOP>
__device__ __forceinline__ void dif_rest(double2* x, const double2* tl) {
  if constexpr (TOP >= 0) {
    constexpr int R = TOP + 1 < kRadixLg ? TOP + 1 : kRadixLg;
    constexpr int LO = TOP - R + 1, T = fft_threads<LG>();
#pragma unroll
    for (int g0 = 0; g0 < ((1 << LG) >> R); g0 += T) {
      const int g = g0 + (int)threadIdx.x;
      if (((1 << LG) >> R) % T == 0 || g < ((1 << LG) >> R)) {
        const int base = group_base<LO, TOP>(g);
        double2 v[1 << R];
#pragma unroll
        for (int m = 0; m < (1 << R); ++m) v[m] = x[pad(base + (m << LO))];
        dif_butterflies<R, LG, TOP>(v, base, tl);
#pragma unroll
        for (int m = 0; m < (1 << R); ++m) x[pad(base + (m << LO))] = v[m];
      }
    }
    __syncthreads();
    dif_rest<LG, TOP - R>(x, tl);
  }
}

// Inverse passes from stage LO up, in place in LDS with a barrier after
// each; the last one writes the real row y (z_n = y_{2n} + i y_{2n+1})
// times 1/N.
template <int LG, int LO>
__device__ __forceinline__ void dit_rest(double2* x, const double2* tl, double2* y) {
  if constexpr (LO < LG) {
    constexpr int R = LG - LO < kRadixLg ? LG - LO : kRadixLg;
    constexpr int TOP = LO + R - 1, T = fft_threads<LG>();
    constexpr bool last = TOP == LG - 1;
    constexpr double scale = 1.0 / (double)(1 << LG);
#pragma unroll
    for (int g0 = 0; g0 < ((1 << LG) >> R); g0 += T) {
      const int g = g0 + (int)threadIdx.x;
      if (((1 << LG) >> R) % T == 0 || g < ((1 << LG) >> R)) {
        const int base = group_base<LO, TOP>(g);
        double2 v[1 << R];
#pragma unroll
        for (int m = 0; m < (1 << R); ++m) v[m] = x[pad(base + (m << LO))];
        dit_butterflies<R, LG, LO>(v, base, tl);
#pragma unroll
        for (int m = 0; m < (1 << R); ++m) {
          if (last) y[base + (m << LO)] = make_double2(v[m].x * scale, v[m].y * scale);
          else x[pad(base + (m << LO))] = v[m];
        }
      }
    }
    if (!last) {
      __syncthreads();
      dit_rest<LG, LO + R>(x, tl, y);
    }
  }
}

// S row r = modes 0..N of g row r, r = 1..n (block b: row b+1)
template <int LG>
__global__ void __launch_bounds__(fft_threads<LG>()) k_fft_rows_fwd(
    const double* __restrict__ g, double2* __restrict__ S, const double2* __restrict__ tw,
    int ld) {
  constexpr int N = 1 << LG, T = fft_threads<LG>();
  constexpr int R1 = LG < kRadixLg ? LG : kRadixLg, LO1 = LG - R1;
  extern __shared__ double2 lds[];
  double2* x = lds;
  double2* tl = lds + N + N / 16 + 1;
  const long long r = (long long)blockIdx.x + 1;
  const double2* z = reinterpret_cast<const double2*>(g + r * 2 * N);
  const int tid = threadIdx.x;
  // first pass (stages LG-1 .. LO1, group `tid`): its points are loaded
  // before the twiddles go to LDS, so both loads are in flight together
  const bool has = tid < (N >> R1);
  double2 v[1 << R1];
  if (has) {
#pragma unroll
    for (int m = 0; m < (1 << R1); ++m) v[m] = z[tid + (m << LO1)];
  }
#pragma unroll
  for (int q0 = 0; q0 < N; q0 += T)
    if (N % T == 0 || q0 + tid < N) tl[q0 + tid] = tw[q0 + tid];
  __syncthreads();
  if (has) {
    dif_butterflies<R1, LG, LG - 1>(v, tid, tl);
#pragma unroll
    for (int m = 0; m < (1 << R1); ++m) x[pad(tid + (m << LO1))] = v[m];
  }
  __syncthreads();
  dif_rest<LG, LO1 - 1>(x, tl);
  // even/odd split: Z_k sits at bitrev(k)
  double2* out = S + r * ld;
  for (int k = tid; k <= N / 2; k += T) {
    const double2 zk = x[pad(bitrev(k, LG))];
    const double2 zn = x[pad(bitrev((N - k) & (N - 1), LG))];
    if (k == 0) {
      out[0] = make_double2(zk.x + zk.y, 0.0);
      out[N] = make_double2(zk.x - zk.y, 0.0);
      continue;
    }
    const double2 E = make_double2(0.5 * (zk.x + zn.x), 0.5 * (zk.y - zn.y));
    const double2 O = make_double2(0.5 * (zk.y + zn.y), -0.5 * (zk.x - zn.x));
    const double2 wO = cmul(tl[k], O);
    out[k] = cadd(E, wO);
    out[N - k] = make_double2(E.x - wO.x, wO.y - E.y);  // conj(E - wO)
  }
}

// X row r = inverse transform of the modes 0..N of S row r, r = 1..n; block
// 0 writes X row 0 = 0
template <int LG>
__global__ void __launch_bounds__(fft_threads<LG>()) k_fft_rows_inv(
    const double2* __restrict__ S, double* __restrict__ X, const double2* __restrict__ tw,
    int ld) {
  constexpr int N = 1 << LG, T = fft_threads<LG>();
  extern __shared__ double2 lds[];
  double2* x = lds;
  double2* tl = lds + N + N / 16 + 1;
  const long long r = blockIdx.x;
  const int tid = threadIdx.x;
  double2* y = reinterpret_cast<double2*>(X + r * 2 * N);
  if (r == 0) {
    for (int i = tid; i < N; i += T) y[i] = make_double2(0.0, 0.0);
    return;
  }
#pragma unroll
  for (int q0 = 0; q0 < N; q0 += T)
    if (N % T == 0 || q0 + tid < N) tl[q0 + tid] = tw[q0 + tid];
  // Z_k = E_k + i O_k, E_k = (Y_k + conj Y_{N-k})/2,
  // O_k = (Y_k - conj Y_{N-k}) conj(w^k)/2; Z_{N-k} = conj E_k + i conj O_k;
  // modes 0 and N enter by their real parts (the row is real)
  const double2* Y = S + r * ld;
  for (int k = tid; k <= N / 2; k += T) {
    const double2 yk = Y[k], yn = Y[N - k];
    if (k == 0) {
      x[pad(0)] = make_double2(0.5 * (yk.x + yn.x), 0.5 * (yk.x - yn.x));
      continue;
    }
    const double2 E = make_double2(0.5 * (yk.x + yn.x), 0.5 * (yk.y - yn.y));
    const double2 O = cmulc(make_double2(0.5 * (yk.x - yn.x), 0.5 * (yk.y + yn.y)), tw[k]);
    x[pad(bitrev(k, LG))] = make_double2(E.x - O.y, E.y + O.x);
    x[pad(bitrev(N - k, LG))] = make_double2(E.x + O.y, O.x - E.y);
  }
  __syncthreads();
  dit_rest<LG, 0>(x, tl, y);
}

// Mode recurrences S[s][k] <- mu_k S[s-1][k] + S[s][k], s = 1..n, from 0,
// for modes k < nm.  A workgroup takes kScanModes consecutive modes and
// splits rows 1..n into kScanChunks chunks of L = ceil(n / kScanChunks)
// rows; thread (c, q) runs chunk c of mode q.  Each chunk first runs from
// zero, which gives its end value e_c and multiplier P_c = mu^(rows); the
// value entering chunk c is then the composition of the chunks before it
// (a_{c+1} = P_c a_c + e_c, from LDS), and the chunk reruns its recurrence
// from that value (from registers when L <= kScanRegs, else reloaded).
// Lanes of a wavefront take 16 consecutive modes of four chunks, so every
// row access is a contiguous 256 bytes.
constexpr int kScanModes = 16, kScanChunks = 64, kScanRegs = 8;
__global__ void __launch_bounds__(1024) k_mode_scan(double2* __restrict__ S,
                                                     const double2* __restrict__ mu, int nm,
                                                     int ld, int n) {
  __shared__ double2 Pc[kScanChunks][kScanModes], Ec[kScanChunks][kScanModes];
  const int q = threadIdx.x % kScanModes, c = threadIdx.x / kScanModes;
  const int k = blockIdx.x * kScanModes + q;
  const int L = (n + kScanChunks - 1) / kScanChunks;
  // rows s0 .. s0+len-1 of this chunk (len may be 0); none for modes >= nm
  const int s0 = 1 + c * L;
  const int len = k < nm ? max(0, min(L, n - s0 + 1)) : 0;
  const double2 m = k < nm ? mu[k] : make_double2(0.0, 0.0);
  double2* col = S + (long long)s0 * ld + k;
  double2 v[kScanRegs];
  double2 e = make_double2(0.0, 0.0), P = make_double2(1.0, 0.0);
  for (int t0 = 0; t0 < len; t0 += kScanRegs) {
#pragma unroll
    for (int t = 0; t < kScanRegs; ++t)
      if (t0 + t < len) v[t] = col[(long long)(t0 + t) * ld];
#pragma unroll
    for (int t = 0; t < kScanRegs; ++t)
      if (t0 + t < len) {
        e = cadd(cmul(m, e), v[t]);
        P = cmul(m, P);
      }
  }
  Pc[c][q] = P;
  Ec[c][q] = e;
  __syncthreads();
  double2 a = make_double2(0.0, 0.0);
  for (int b = 0; b < c; ++b) a = cadd(cmul(Pc[b][q], a), Ec[b][q]);
  for (int t0 = 0; t0 < len; t0 += kScanRegs) {
    if (L > kScanRegs) {
#pragma unroll
      for (int t = 0; t < kScanRegs; ++t)
        if (t0 + t < len) v[t] = col[(long long)(t0 + t) * ld];
    }
#pragma unroll
    for (int t = 0; t < kScanRegs; ++t)
      if (t0 + t < len) {
        a = cadd(cmul(m, a), v[t]);
        col[(long long)(t0 + t) * ld] = a;
      }
  }
}

size_t spectral_rows(int n) { return (size_t)n + 1; }

bool spectral_supported(int nx) {
  return nx >= 4 && nx <= kSpectralMaxNx && (nx & (nx - 1)) == 0;
}

// The transforms of every supported size, and their LDS limits (above 64 KB
// the kernels' limit is raised once per process).
struct FftKernels {
  const void* fwd;
  const void* inv;
  int threads;
  size_t lds;
};

template <int LG>
static FftKernels fft_kernels() {
  return {(const void*)k_fft_rows_fwd<LG>, (const void*)k_fft_rows_inv<LG>, fft_threads<LG>(),
          fft_lds(1 << LG)};
}

static const FftKernels* fft_table() {
  static std::once_flag once;
  static FftKernels t[kMaxLgN + 1];
  static bool ok = false;
  std::call_once(once, [] {
    t[1] = fft_kernels<1>();   t[2] = fft_kernels<2>();   t[3] = fft_kernels<3>();
    t[4] = fft_kernels<4>();   t[5] = fft_kernels<5>();   t[6] = fft_kernels<6>();
    t[7] = fft_kernels<7>();   t[8] = fft_kernels<8>();   t[9] = fft_kernels<9>();
    t[10] = fft_kernels<10>(); t[11] = fft_kernels<11>(); t[12] = fft_kernels<12>();
    ok = true;
    for (int lg = 1; lg <= kMaxLgN; ++lg)
      for (const void* f : {t[lg].fwd, t[lg].inv})
        ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)t[lg].lds) == hipSuccess;
    (void)hipGetLastError();
  });
  return ok ? t : nullptr;
}

int launch_spectral_solve(const double* g, double* X, void* S, const void* mu, const void* tw,
                          int nx, int n, void* stream) {
  static_assert(kSpectralMaxNx == 2 << kMaxLgN, "transform sizes");
  if (!spectral_supported(nx) || n < 1) return -1;
  const FftKernels* tab = fft_table();
  if (!tab) return -1;
  const int N = nx / 2;
  int lgN = 0;
  while ((1 << lgN) < N) ++lgN;
  const FftKernels& K = tab[lgN];
  hipStream_t s = (hipStream_t)stream;
  double2* Sp = (double2*)S;
  const double2* twp = (const double2*)tw;
  int ld = nx;  // S rows keep a stride of n_x complex values; modes 0..N are used
  {
    void* args[] = {(void*)&g, (void*)&Sp, (void*)&twp, (void*)&ld};
    if (hipLaunchKernel(K.fwd, dim3((unsigned)n), dim3(K.threads), args, K.lds, s) != hipSuccess)
      return -1;
  }
  k_mode_scan<<<dim3((unsigned)((N + kScanModes) / kScanModes)), dim3(kScanModes * kScanChunks),
                0, s>>>(Sp, (const double2*)mu, N + 1, nx, n);
  {
    const double2* Sc = Sp;
    void* args[] = {(void*)&Sc, (void*)&X, (void*)&twp, (void*)&ld};
    if (hipLaunchKernel(K.inv, dim3((unsigned)(n + 1)), dim3(K.threads), args, K.lds, s) !=
        hipSuccess)
      return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mgr
