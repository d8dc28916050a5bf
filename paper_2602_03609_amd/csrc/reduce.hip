// Deterministic FP64 reductions over points and the final likelihood assembly
// (Sec. "Estimation and prediction" for the Gaussian NLL; the Woodbury identity
// and the matrix determinant lemma for the VIF form):
//   nll = n/2 log(2 pi) + 1/2 (sum_i log D_i + log det M) + 1/2 (z'z - q' M^-1 q).
// Sums use a fixed grid and fixed-order trees, so repeated runs give identical bits.
#include <math.h>

#include "internal.hpp"

namespace vif {

namespace {

constexpr int kSumBlocks = 256;
constexpr int kSumThreads = 256;

__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kSumThreads) void sum_stage1(int64_t n, const double* __restrict__ x,
                                                          int squared, double* __restrict__ part) {
  __shared__ double sh[kSumThreads];
  const int64_t chunk = (n + kSumBlocks - 1) / kSumBlocks;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kSumThreads) {
    const double v = x[i];
    acc += squared ? v * v : v;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kSumThreads) void sum_stage2(const double* __restrict__ part,
                                                          double* __restrict__ out) {
  __shared__ double sh[kSumThreads];
  const double s = block_sum(part[threadIdx.x], sh);
  if (threadIdx.x == 0) *out = s;
}

// One workgroup: log det M from the diagonal of the Cholesky factor of the
// augmented Woodbury matrix (M in rows 0 .. k-1, q' in row k), and q' M^-1 q as
// the squared norm of the factor's row k, which is L_M^-1 q.
__global__ __launch_bounds__(1024) void finalize_kernel(int64_t n, int k, int kpad,
                                                        const double* __restrict__ LM,
                                                        const double* __restrict__ sum_logD,
                                                        const double* __restrict__ zz,
                                                        double* __restrict__ out) {
  __shared__ double sh[1024];
  const int tid = threadIdx.x;
  double logdet = 0.0, quad = 0.0;
  if (k > 0) {
    double acc = 0.0, qa = 0.0;
    for (int a = tid; a < k; a += 1024) {
      acc += log(LM[(int64_t)a * kpad + a]);
      const double v = LM[(int64_t)k * kpad + a];
      qa += v * v;
    }
    logdet = 2.0 * block_sum(acc, sh);
    __syncthreads();
    quad = block_sum(qa, sh);
  }
  if (tid == 0) {
    const double sl = *sum_logD, z2 = *zz;
    const double LOG2PI = 1.8378770664093454836;
    out[0] = 0.5 * (double)n * LOG2PI + 0.5 * (sl + logdet) + 0.5 * (z2 - quad);
    out[1] = sl;
    out[2] = z2;
    out[3] = logdet;
    out[4] = quad;
  }
}

__global__ void init_flags_kernel(unsigned long long* f) {
  const int t = threadIdx.x;
  if (t < 4) f[t] = ~0ull;
  if (t == 4) f[4] = 0ull;
}

}  // namespace

hipError_t launch_init_flags(void* flags, hipStream_t s) {
  hipLaunchKernelGGL(init_flags_kernel, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<unsigned long long*>(flags));
  return hipGetLastError();
}

hipError_t launch_sum(int64_t n, const double* x, int squared, double* partial, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(sum_stage1, dim3(kSumBlocks), dim3(kSumThreads), 0, s, n, x, squared,
                     partial);
  hipLaunchKernelGGL(sum_stage2, dim3(1), dim3(kSumThreads), 0, s, (const double*)partial, out);
  return hipGetLastError();
}

__global__ void copy_f64_kernel(const double* __restrict__ src, double* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

hipError_t launch_copy_f64(const double* src, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(copy_f64_kernel, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

hipError_t launch_finalize(int64_t n, int k, int kpad, const double* LM, const double* sum_logD,
                           const double* zz, double* out, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(1024), 0, s, n, k, kpad, LM, sum_logD, zz,
                     out);
  return hipGetLastError();
}

}  // namespace vif
