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
// Transforms: one workgroup per row, radix-2 decimation in time grouped
// into passes of four stages in registers (below).
#include <hip/hip_runtime.h>

#include <mutex>

#include "registry.h"

namespace mgr {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// The transform of one row runs in passes of up to four radix-2 stages
// (decimation in time, input in bit-reversed order).  In a pass that does
// stages s0 .. s0+R-1 a thread owns groups of 2^R elements
// base + m 2^s0 (m < 2^R; base has zero bits s0 .. s0+R-1): every butterfly
// of those stages pairs two elements of one group, so a pass reads each
// element once, runs its R stages in registers and writes it once.  The
// first pass reads the row from global memory in bit-reversed order, the
// last one writes the result to global memory (consecutive lanes then own
// consecutive elements); passes in between go through LDS (16 n_x bytes).
// Twiddles e^{-2 pi i q / n_x} (q < n_x/2) come from a table in global
// memory (L2-resident), loaded before each group's arithmetic.
constexpr int kFftThreads = 256;

__device__ __forceinline__ int bitrev(int i, int lg) {
  return (int)(__builtin_bitreverse32((unsigned)i) >> (32 - lg));
}

// one pass: input from gin_re (real row) / gin (complex row) in bit-reversed
// order, or from LDS; output to gout (complex row) / gout_re (real part times
// scale), or to LDS
template <int R>
__device__ __forceinline__ void fft_pass(double2* lds, const double* gin_re, const double2* gin,
                                         double2* gout, double* gout_re, double scale,
                                         const double2* __restrict__ tw, int nx, int lg, int s0,
                                         bool inverse) {
  constexpr int G = 1 << R;
  const int ngroups = nx >> R;
  for (int grp = threadIdx.x; grp < ngroups; grp += blockDim.x) {
    const int lo = grp & ((1 << s0) - 1);
    const int base = lo + ((grp >> s0) << (s0 + R));
    double2 x[G];
#pragma unroll
    for (int m = 0; m < G; ++m) {
      const int idx = base + (m << s0);
      if (gin_re) x[m] = make_double2(gin_re[bitrev(idx, lg)], 0.0);
      else if (gin) x[m] = gin[bitrev(idx, lg)];
      else x[m] = lds[idx];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int half = 1 << (s0 + r);
      const int stride = nx / (2 * half);
#pragma unroll
      for (int m = 0; m < G; ++m) {
        if (m & (1 << r)) continue;
        const int k = (base + (m << s0)) & (half - 1);
        double2 w = tw[k * stride];
        if (inverse) w.y = -w.y;
        const double2 t = cmul(x[m + (1 << r)], w);
        x[m + (1 << r)] = make_double2(x[m].x - t.x, x[m].y - t.y);
        x[m] = make_double2(x[m].x + t.x, x[m].y + t.y);
      }
    }
#pragma unroll
    for (int m = 0; m < G; ++m) {
      const int idx = base + (m << s0);
      if (gout_re) gout_re[idx] = x[m].x * scale;
      else if (gout) gout[idx] = x[m];
      else lds[idx] = x[m];
    }
  }
}

// the whole transform of a row: input from in_re (real) or in (complex),
// output to out (complex) or out_re (real part times scale)
__device__ __forceinline__ void fft_row(double2* lds, const double* in_re, const double2* in,
                                        double2* out, double* out_re, double scale,
                                        const double2* __restrict__ tw, int nx, int lg,
                                        bool inverse) {
  for (int s0 = 0; s0 < lg; s0 += 4) {
    const int R = lg - s0 < 4 ? lg - s0 : 4;
    const bool first = s0 == 0, last = s0 + R >= lg;
    const double* ir = first ? in_re : nullptr;
    const double2* ic = first ? in : nullptr;
    double2* oc = last ? out : nullptr;
    double* orr = last ? out_re : nullptr;
    switch (R) {
      case 4: fft_pass<4>(lds, ir, ic, oc, orr, scale, tw, nx, lg, s0, inverse); break;
      case 3: fft_pass<3>(lds, ir, ic, oc, orr, scale, tw, nx, lg, s0, inverse); break;
      case 2: fft_pass<2>(lds, ir, ic, oc, orr, scale, tw, nx, lg, s0, inverse); break;
      default: fft_pass<1>(lds, ir, ic, oc, orr, scale, tw, nx, lg, s0, inverse); break;
    }
    if (!last) __syncthreads();
  }
}

// S row r = transform of g row r, r = 1..n (block b: row b+1)
__global__ void __launch_bounds__(kFftThreads) k_fft_rows_fwd(const double* __restrict__ g,
                                                               double2* __restrict__ S,
                                                               const double2* __restrict__ tw,
                                                               int nx, int lg) {
  extern __shared__ double2 a[];
  const long long r = (long long)blockIdx.x + 1;
  fft_row(a, g + r * nx, nullptr, S + r * nx, nullptr, 1.0, tw, nx, lg, false);
}

// X row r = real part of the inverse transform of S row r / n_x, r = 1..n;
// block 0 writes X row 0 = 0
__global__ void __launch_bounds__(kFftThreads) k_fft_rows_inv(const double2* __restrict__ S,
                                                               double* __restrict__ X,
                                                               const double2* __restrict__ tw,
                                                               int nx, int lg) {
  extern __shared__ double2 a[];
  const long long r = blockIdx.x;
  double* out = X + r * nx;
  if (r == 0) {
    for (int i = threadIdx.x; i < nx; i += blockDim.x) out[i] = 0.0;
    return;
  }
  fft_row(a, nullptr, S + r * nx, nullptr, out, 1.0 / nx, tw, nx, lg, true);
}

// per mode k: S[s][k] <- mu_k S[s-1][k] + S[s][k], s = 1..n, from 0; the
// loads of a batch of 16 rows are issued before its dependent updates
__global__ void __launch_bounds__(256) k_mode_scan(double2* __restrict__ S,
                                                    const double2* __restrict__ mu, int nx,
                                                    int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nx) return;
  const double2 m = mu[k];
  double2 acc = make_double2(0.0, 0.0);
  constexpr int B = 16;
  for (int s0 = 1; s0 <= n; s0 += B) {
    double2 v[B];
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (s0 + b <= n) v[b] = S[(long long)(s0 + b) * nx + k];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (s0 + b <= n) {
        const double2 p = cmul(m, acc);
        acc = make_double2(p.x + v[b].x, p.y + v[b].y);
        S[(long long)(s0 + b) * nx + k] = acc;
      }
    }
  }
}

size_t spectral_rows(int n) { return (size_t)n + 1; }

bool spectral_supported(int nx) {
  return nx >= 4 && nx <= kSpectralMaxNx && (nx & (nx - 1)) == 0;
}

// LDS above 64 KB needs the kernels' limit raised once per process.
static bool raise_lds_limit() {
  static std::once_flag once;
  static bool ok = false;
  std::call_once(once, [] {
    const int want = (int)(sizeof(double2) * kSpectralMaxNx);
    ok = hipFuncSetAttribute((const void*)k_fft_rows_fwd,
                             hipFuncAttributeMaxDynamicSharedMemorySize, want) == hipSuccess &&
         hipFuncSetAttribute((const void*)k_fft_rows_inv,
                             hipFuncAttributeMaxDynamicSharedMemorySize, want) == hipSuccess;
    (void)hipGetLastError();
  });
  return ok;
}

int launch_spectral_solve(const double* g, double* X, void* S, const void* mu, const void* tw,
                          int nx, int n, void* stream) {
  if (!spectral_supported(nx) || n < 1) return -1;
  if (!raise_lds_limit()) return -1;
  int lg = 0;
  while ((1 << lg) < nx) ++lg;
  const size_t lds = sizeof(double2) * (size_t)nx;
  hipStream_t s = (hipStream_t)stream;
  double2* Sp = (double2*)S;
  k_fft_rows_fwd<<<dim3((unsigned)n), dim3(kFftThreads), lds, s>>>(g, Sp, (const double2*)tw, nx,
                                                                   lg);
  k_mode_scan<<<dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s>>>(Sp, (const double2*)mu,
                                                                       nx, n);
  k_fft_rows_inv<<<dim3((unsigned)(n + 1)), dim3(kFftThreads), lds, s>>>(
      Sp, X, (const double2*)tw, nx, lg);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mgr
