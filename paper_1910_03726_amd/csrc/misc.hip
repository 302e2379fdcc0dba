// Small utility kernels and the kernel table of libmgrit.
#include <hip/hip_runtime.h>

#include "registry.h"
#include "relax_kernels.h"

namespace mgr {

// ---- kernel table --------------------------------------------------------
#define MGR_DECL_K(K) void register_stencil_0_##K(KernelTable&); \
                      void register_stencil_1_##K(KernelTable&);
MGR_DECL_K(1) MGR_DECL_K(2) MGR_DECL_K(4) MGR_DECL_K(8) MGR_DECL_K(16) MGR_DECL_K(32)
#undef MGR_DECL_K
void register_sdirk_0(KernelTable&);
void register_sdirk_1(KernelTable&);
void register_sdirk_pf_0(KernelTable&);
void register_sdirk_pf_1(KernelTable&);
void register_bounded(KernelTable&);

int width_index(int W) {
  for (int i = 0; i < kNumWidths; ++i)
    if (kWidths[i] == W) return i;
  return -1;
}
int k_index(int K) {
  for (int i = 0; i < kNumK; ++i)
    if (kKs[i] == K) return i;
  return -1;
}
int sdirk_k_index(int K) {
  for (int i = 0; i < kNumSdirkK; ++i)
    if (kSdirkKs[i] == K) return i;
  return -1;
}
int sdirk_shape_index(int S, int NF) {
  for (int i = 0; i < kNumSdirkShapes; ++i)
    if (kSdirkShapes[i][0] == S && kSdirkShapes[i][1] == NF) return i;
  return -1;
}

int sdirk_pf_shape_index(int S, int NR, int NB, int NC) {
  for (int i = 0; i < kNumSdirkPfShapes; ++i)
    if (kSdirkPfShapes[i][0] == S && kSdirkPfShapes[i][1] == NR &&
        kSdirkPfShapes[i][2] == NB && kSdirkPfShapes[i][3] == NC)
      return i;
  return -1;
}

static KernelTable build_table() {
  KernelTable t;
#define MGR_REG_K(K) register_stencil_0_##K(t); register_stencil_1_##K(t);
  MGR_REG_K(1) MGR_REG_K(2) MGR_REG_K(4) MGR_REG_K(8) MGR_REG_K(16) MGR_REG_K(32)
#undef MGR_REG_K
  register_sdirk_0(t);
  register_sdirk_1(t);
  register_sdirk_pf_0(t);
  register_sdirk_pf_1(t);
  register_bounded(t);
  return t;
}

const KernelTable& kernel_table() {
  static const KernelTable t = build_table();
  return t;
}

// ---- discrete L2 norm from per-interval partial sums ------------------------
// out[0] = sqrt(scale2 * sum_i partial[i]); fixed summation order.
__global__ void __launch_bounds__(256) k_norm_reduce(const double* partial, int n,
                                                      double scale2, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = sqrt(scale2 * s);
}

void launch_norm_reduce(const double* partial, int n, double scale2, double* out,
                        void* stream) {
  hipLaunchKernelGGL(k_norm_reduce, dim3(1), dim3(256), 0, (hipStream_t)stream, partial,
                     n, scale2, out);
}

// ---- y += x ---------------------------------------------------------------
__global__ void k_axpy(double* y, const double* x, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) y[i] += x[i];
}

void launch_axpy(double* y, const double* x, long long n, void* stream) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, y,
                     x, n);
}

// ---- seeded U[0,1) initial iterate -------------------------------------------
// Value i of the stream is splitmix64 (Steele, Lea & Flood, OOPSLA 2014) of
// the state seed + (i+1) * 0x9E3779B97F4A7C15, scaled by 2^-53 from its top
// 53 bits.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__global__ void k_uniform_init(double* out, long long n, unsigned long long seed) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const unsigned long long z =
        splitmix64(seed + (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ULL);
    out[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0);
  }
}

void launch_uniform_init(double* out, long long rows, int nx, unsigned long long seed,
                         void* stream) {
  const long long n = rows * (long long)nx;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_uniform_init, dim3((unsigned)blocks), dim3(256), 0,
                     (hipStream_t)stream, out, n, seed);
}

}  // namespace mgr
