// Shared device helpers and the covariance functions of the library (gfx950 only).
//
// Covariance kinds (latent covariance, nugget added by the callers):
//   GNEITING          psi = a|dt|^(2 alpha) + 1,
//                     C = sigma2 psi^-tau exp(-c |ds|^(2 gamma) psi^-(beta gamma))
//   GNEITING_MATERN   Eq. (Gneiting) with d = 2: x = c|ds| psi^-(gamma/2),
//                     C = sigma2 psi^-(delta+gamma) g_nu(x), g_nu in closed form for
//                     nu in {1/2, 3/2, 5/2} (Sec. "GPU acceleration")
//   MATERN_ANISO      C = sigma2 g_nu(d), d = sqrt(|ds|^2/range_s^2 + dt^2/range_t^2)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vif {

constexpr int kWave = 64;

// Kernel hyperparameters in the form the device code uses (passed by value).
struct KernDev {
  int kind;
  int nu_code;        // 0: nu=1/2, 1: nu=3/2, 2: nu=5/2
  int gamma_half;     // GNEITING with gamma == 1/2 (spatial part is sqrt(h2))
  double sigma2, nugget, a, c, two_alpha, tau, bg, gamma, half_gamma, dpg, ir_s2, ir_t2;
};

// Normalised Matern correlation g_nu(x) in closed form.
template <typename T>
__device__ __forceinline__ T matern_poly(int nu_code, T x) {
  if (nu_code == 0) return T(1);
  if (nu_code == 1) return T(1) + x;
  return T(1) + x + x * x * T(1.0 / 3.0);
}

__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dexp(float x) { return __expf(x); }
__device__ __forceinline__ double dlog(double x) { return log(x); }
__device__ __forceinline__ float dlog(float x) { return __logf(x); }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float dsqrt(float x) { return __fsqrt_rn(x); }

// Latent covariance for coordinate differences. Differences are formed in FP64
// by the caller and converted to T afterwards.
template <typename T>
__device__ __forceinline__ T cov_eval(const KernDev& K, T dx, T dy, T dt) {
  T h2 = dx * dx + dy * dy;
  if (K.kind == 3) {
    T d = dsqrt(h2 * T(K.ir_s2) + dt * dt * T(K.ir_t2));
    return T(K.sigma2) * matern_poly<T>(K.nu_code, d) * dexp(-d);
  }
  T adt = dt < T(0) ? -dt : dt;
  T ta = adt > T(0) ? dexp(T(K.two_alpha) * dlog(adt)) : T(0);
  T lp = dlog(T(K.a) * ta + T(1));  // log psi
  if (K.kind == 1) {
    T g = K.gamma_half ? dsqrt(h2) : (h2 > T(0) ? dexp(T(K.gamma) * dlog(h2)) : T(0));
    return T(K.sigma2) * dexp(-T(K.tau) * lp - T(K.c) * g * dexp(-T(K.bg) * lp));
  }
  T x = T(K.c) * dsqrt(h2) * dexp(-T(K.half_gamma) * lp);
  return T(K.sigma2) * matern_poly<T>(K.nu_code, x) * dexp(-T(K.dpg) * lp - x);
}

// The stretched-exponential Gneiting kernel (kind 1) factored for many pairs at
// one time lag: gneiting_lag gives A = -tau log psi and e = exp(-beta gamma log psi)
// for |dt|, gneiting_pair the covariance from them, with the operations of
// cov_eval in the same order. The values agree with cov_eval to rounding: A is
// rounded on its own here, where cov_eval may fuse -tau log psi into the
// following subtraction.
template <typename T>
__device__ __forceinline__ void gneiting_lag(const KernDev& K, T dt, T& A, T& e) {
  T adt = dt < T(0) ? -dt : dt;
  T ta = adt > T(0) ? dexp(T(K.two_alpha) * dlog(adt)) : T(0);
  T lp = dlog(T(K.a) * ta + T(1));
  A = -T(K.tau) * lp;
  e = dexp(-T(K.bg) * lp);
}
template <typename T>
__device__ __forceinline__ T gneiting_pair(const KernDev& K, T dx, T dy, T A, T e) {
  T h2 = dx * dx + dy * dy;
  T g = K.gamma_half ? dsqrt(h2) : (h2 > T(0) ? dexp(T(K.gamma) * dlog(h2)) : T(0));
  return T(K.sigma2) * dexp(A - T(K.c) * g * e);
}

// Wave-local memory ordering for communication through LDS between lanes of
// one wavefront (LDS instructions of a wave execute in order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Accumulator layout of the 16x16 MFMA tiles: element e of `lane` holds
// D[row][lane % 16]. The FP32-accumulating forms stack four consecutive rows
// per lane group; the FP64 form interleaves them with stride 4.
__device__ __forceinline__ int mfma16_row_f32acc(int lane, int e) { return 4 * (lane >> 4) + e; }
__device__ __forceinline__ int mfma16_row_f64(int lane, int e) { return (lane >> 4) + 4 * e; }

// Record the smallest failing index (vector atomic on global memory).
__device__ __forceinline__ void flag_fail(unsigned long long* flag, long long idx) {
  atomicMin(flag, (unsigned long long)idx);
}

}  // namespace vif
