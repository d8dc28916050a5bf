// Correlation-based neighbor selection (Sec. "Correlation-based Vecchia neighbor
// selection", Alg. 2 semantics): exact top-m earlier points per query under a
// FP64 log-correlation key, ties to the lower index.
//
// Design (gfx950): one wavefront per query. Candidate slabs (all points sharing
// one integer time) are visited in increasing lag; within a slab, 64 candidates
// are keyed per step (coalesced SoA loads), candidates that beat the current
// m-th entry are found with a ballot and inserted one at a time into a sorted
// list held one entry per lane. The scan stops at the first lag whose bound
// (suffix maximum of -tab1) is strictly below the m-th key: no later slab can
// contain a better or tying candidate with a lower index.
#include <limits.h>
#include <math.h>

#include "internal.hpp"

namespace vif {

namespace {

__global__ void validate_times_kernel(int64_t n, const double* __restrict__ t,
                                      uint32_t* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ti = t[i];
  uint32_t bits = 0;
  if (!isfinite(ti)) bits |= 1u;
  else if (ti != rint(ti)) bits |= 2u;
  if (i > 0 && !(ti >= t[i - 1])) bits |= 4u;
  if (bits) atomicOr(flag, bits);
}

__global__ void slab_start_kernel(int64_t n, const double* __restrict__ t, double t0, int L,
                                  int32_t* __restrict__ slab_start) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  int cur = (i < n) ? (int)(t[i] - t0) : L + 1;
  int prev = (i == 0) ? -1 : (int)(t[i - 1] - t0);
  for (int s = prev + 1; s <= cur; ++s) slab_start[s] = (int32_t)i;
}

// Ranking keys. Fixed operation order and no contraction, so that any IEEE FP64
// implementation of the same sequence returns the same bits.
template <int MODE>
__device__ __forceinline__ double rank_key(double dx, double dy, double t1, double t2,
                                           const NbrArgs& A) {
#pragma clang fp contract(off)
  if (MODE == 1) {
    double u = dx * A.ir_s;
    double v = dy * A.ir_s;
    double s = u * u + v * v;
    return -(t1 + s);
  }
  double h2 = dx * dx + dy * dy;
  if (MODE == 0) {
    double g = sqrt(h2);
    return -(t1 + g * t2);
  }
  if (MODE == 2) {
    double g = pow(h2, A.gamma);
    return -(t1 + g * t2);
  }
  double x = sqrt(h2) * t2;
  double s = A.nu_code == 1 ? x - log1p(x) : x - log1p(x + x * x / 3.0);
  s = s > 0.0 ? s : 0.0;
  return -(t1 + s);
}

template <int MODE>
__global__ __launch_bounds__(256) void neighbors_wave_kernel(NbrArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= A.n) return;  // uniform per wave
  const int m = A.m;
  const double qx = A.sx[i], qy = A.sy[i];
  const int ti = (int)(A.t[i] - A.t0);
  double K = -INFINITY;
  int I = INT_MAX;
  int cnt = 0;
  double thr = -INFINITY;
  int thr_i = INT_MAX;
  for (int lag = 0; lag <= ti; ++lag) {
    if (cnt >= m && A.bnd[lag] < thr) break;
    const int slab = ti - lag;
    const int lo = A.slab_start[slab];
    const int hi = (lag == 0) ? (int)i : A.slab_start[slab + 1];
    const double t1 = A.tab1[lag], t2 = A.tab2[lag];
    for (int base = lo; base < hi; base += 64) {
      const int j = base + lane;
      const bool valid = j < hi;
      double key = -INFINITY;
      if (valid) key = rank_key<MODE>(A.sx[j] - qx, A.sy[j] - qy, t1, t2, A);
      const bool better = valid && (cnt < m || key > thr || (key == thr && j < thr_i));
      unsigned long long mask = __ballot(better);
      while (mask) {
        const int s = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        const double ck = __shfl(key, s);
        const int cj = __shfl(j, s);
        if (cnt >= m && !(ck > thr || (ck == thr && cj < thr_i))) continue;
        const bool before = lane < cnt && (K > ck || (K == ck && I < cj));
        const int pos = __popcll(__ballot(before));
        const double pK = __shfl_up(K, 1);
        const int pI = __shfl_up(I, 1);
        if (lane == pos) {
          K = ck;
          I = cj;
        } else if (lane > pos) {
          K = pK;
          I = pI;
        }
        if (cnt < m) ++cnt;
        if (cnt >= m) {
          thr = __shfl(K, m - 1);
          thr_i = __shfl(I, m - 1);
        }
      }
    }
  }
  if (lane < m) A.nbr[i * m + lane] = lane < cnt ? I : -1;
}

}  // namespace

hipError_t launch_validate_times(int64_t n, const double* t, uint32_t* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned grid = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(validate_times_kernel, dim3(grid), dim3(256), 0, s, n, t, flag);
  return hipGetLastError();
}

hipError_t launch_slab_start(int64_t n, const double* t, double t0, int L, int32_t* slab_start,
                             hipStream_t s) {
  unsigned grid = (unsigned)((n + 1 + 255) / 256);
  hipLaunchKernelGGL(slab_start_kernel, dim3(grid), dim3(256), 0, s, n, t, t0, L, slab_start);
  return hipGetLastError();
}

hipError_t launch_neighbors(const NbrArgs& a, hipStream_t s) {
  if (a.n <= 0 || a.m <= 0) return hipSuccess;
  unsigned grid = (unsigned)((a.n + 3) / 4);
  switch (a.mode) {
    case 0: hipLaunchKernelGGL(neighbors_wave_kernel<0>, dim3(grid), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(neighbors_wave_kernel<1>, dim3(grid), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(neighbors_wave_kernel<2>, dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(neighbors_wave_kernel<3>, dim3(grid), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace vif
