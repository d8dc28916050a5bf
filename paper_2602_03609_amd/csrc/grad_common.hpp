// Device helpers shared by the gradient kernels: wave reductions, lane reads,
// and the latent covariance with its derivatives in every hyperparameter.
#pragma once

#include <math.h>

#include "internal.hpp"

namespace vif {

__device__ __forceinline__ double rdl(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// Closed-form Matern correlation g(x) and x g'(x) for nu = 1/2, 3/2, 5/2.
__device__ __forceinline__ void matern_g_xdg(int nu_code, double x, double& g, double& xdg) {
  const double e = exp(-x);
  if (nu_code == 0) {
    g = e;
    xdg = -x * e;
  } else if (nu_code == 1) {
    g = (1.0 + x) * e;
    xdg = -x * x * e;
  } else {
    g = (1.0 + x + x * x * (1.0 / 3.0)) * e;
    xdg = -x * x * (1.0 + x) * e * (1.0 / 3.0);
  }
}

// Latent covariance and its derivatives in the parameter order of the
// gradient (GNEITING: sigma2, nugget, a, c, alpha, beta, gamma, tau;
// GNEITING_MATERN: sigma2, nugget, a, c, alpha, gamma, delta;
// MATERN_ANISO: sigma2, nugget, range_s, range_t); dC[1] (nugget) is zero and
// entries past the kind's count are zero.
__device__ __forceinline__ double cov_and_grad(const GradKern& G, double dx, double dy, double dt,
                                               double dC[kGradMaxParams]) {
  const double h2 = dx * dx + dy * dy;
  if (G.kind == 2) {
    // C = amp g(x), amp = sigma2 psi^-(delta + gamma), x = c |ds| psi^(-gamma/2);
    // with X = x g'(x): dC/dc = amp X / c, dC/dgamma = -C log psi - amp X log psi / 2,
    // dC/dpsi = (-(delta + gamma) C - gamma amp X / 2) / psi.
    const double adt = fabs(dt);
    const double ldt = adt > 0.0 ? log(adt) : 0.0;
    const double ta = adt > 0.0 ? exp(G.two_alpha * ldt) : 0.0;
    const double psi = G.a * ta + 1.0;
    const double lp = log(psi);
    const double amp = G.sigma2 * exp(-(G.delta + G.gamma) * lp);
    const double x = G.c * sqrt(h2) * exp(-0.5 * G.gamma * lp);
    double g, X;
    matern_g_xdg(G.nu_code, x, g, X);
    const double C = amp * g;
    const double dpsi = (-(G.delta + G.gamma) * C - 0.5 * G.gamma * amp * X) / psi;
    dC[0] = C / G.sigma2;
    dC[1] = 0.0;
    dC[2] = dpsi * ta;
    dC[3] = amp * X / G.c;
    dC[4] = dpsi * G.a * ta * 2.0 * ldt;
    dC[5] = -C * lp - 0.5 * amp * X * lp;
    dC[6] = -C * lp;
    dC[7] = 0.0;
    return C;
  }
  if (G.kind == 3) {
    const double d = sqrt(h2 * G.ir_s2 + dt * dt * G.ir_t2);
    const double e = exp(-d);
    double g, fp;
    if (G.nu_code == 0) {
      g = e;
      fp = -e;
    } else if (G.nu_code == 1) {
      g = (1.0 + d) * e;
      fp = -d * e;
    } else {
      g = (1.0 + d + d * d * (1.0 / 3.0)) * e;
      fp = -d * (1.0 + d) * e * (1.0 / 3.0);
    }
    const double C = G.sigma2 * g;
    const double inv_d = d > 0.0 ? 1.0 / d : 0.0;
    dC[0] = g;
    dC[1] = 0.0;
    dC[2] = G.sigma2 * fp * (-h2 * G.ir_s2 * G.inv_rs) * inv_d;
    dC[3] = G.sigma2 * fp * (-dt * dt * G.ir_t2 * G.inv_rt) * inv_d;
#pragma unroll
    for (int pp = 4; pp < kGradMaxParams; ++pp) dC[pp] = 0.0;
    return C;
  }
  const double adt = fabs(dt);
  const double ldt = adt > 0.0 ? log(adt) : 0.0;
  const double ta = adt > 0.0 ? exp(G.two_alpha * ldt) : 0.0;
  const double psi = G.a * ta + 1.0;
  const double lp = log(psi);
  const double E = exp(-G.bg * lp);
  const double lh2 = h2 > 0.0 ? log(h2) : 0.0;
  const double g = h2 > 0.0 ? exp(G.gamma * lh2) : 0.0;
  const double q = G.c * g * E;
  const double C = G.sigma2 * exp(-G.tau * lp - q);
  const double dlp = C * (-G.tau + G.bg * q) / psi;
  dC[0] = C / G.sigma2;
  dC[1] = 0.0;
  dC[2] = dlp * ta;
  dC[3] = -C * g * E;
  dC[4] = dlp * G.a * ta * 2.0 * ldt;
  dC[5] = C * q * G.gamma * lp;
  dC[6] = -C * q * (lh2 - G.beta * lp);
  dC[7] = -C * lp;
  return C;
}

// Lower-triangle pair e = r (r + 1) / 2 + s, s <= r.
__device__ __forceinline__ void pair_of(int e, int& r, int& s) {
  r = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= e) ++r;
  while (r * (r + 1) / 2 > e) --r;
  s = e - r * (r + 1) / 2;
}

}  // namespace vif
