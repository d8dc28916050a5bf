// Gradient of the Vecchia NLL with respect to the kernel hyperparameters (the
// quantity the paper's quasi-Newton fit needs, Sec. "Estimation and
// prediction"). Per point, with S = N(i) + {i} (i last), the NLL term is
// 1/2 [l(S) - l(N)], l(T) = log det Sigma~_TT + y_T' Sigma~_TT^-1 y_T, so its
// derivative is the difference of the Gaussian formula
//     dl(T) = tr(Sigma~_TT^-1 dSigma~_TT) - alpha_T' dSigma~_TT alpha_T
// on the two nested blocks. With L = chol(Sigma~_SS), the inverses differ by
// the rank-one term v v' (v = last row of L^-1 = (-A_i, 1) / sqrt(D_i)), and
// alpha_S = alpha_N + z_i v (z_i = (L^-1 y_S)_last, alpha_N = Sigma~_NN^-1 y_N
// padded with a zero), which gives
//     dNLL_i = 1/2 [(1 - z_i^2) v' dSigma~ v - 2 z_i v' dSigma~ alpha_N].
//
// gfx950 design: one wavefront per point, lane r holding row r of the block in
// registers (QMAX = 32 or 64 rows). The q(q+1)/2 covariance entries of the
// lower triangle are spread over the 64 lanes and land in the lanes' rows
// through LDS; the Cholesky factor (pivots and multipliers through readlane),
// the forward solve for L^-1 y, and the two backward solves (for v and
// alpha_N, whose column sums are wave reductions) stay in registers; the
// derivative matrices are never formed: the lower pairs are spread over the
// lanes again, each evaluating dC for every parameter and accumulating its
// share of v' dC v and v' dC alpha_N. Per-point results go to parameter-major
// arrays summed later in a fixed order (deterministic). For the Gneiting kernel
// with integer times, the quantities that depend on the time lag alone come
// from a per-lag table (the operations of the direct evaluation), leaving one
// logarithm and one or two exponentials per pair.
#include <math.h>

#include "grad_common.hpp"
#include "internal.hpp"

namespace vif {
namespace {

// Per-lag quantities of the Gneiting kernel: A = -tau log psi, e = psi^(-beta gamma),
// |dt|^(2 alpha), psi, log psi, log |dt|.
constexpr int kLagVals = kGradLagVals;

__global__ __launch_bounds__(256) void grad_lag_kernel(GradKern G, int nlag, double* __restrict__ tab) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= nlag) return;
  const double adt = (double)l;
  const double ldt = adt > 0.0 ? log(adt) : 0.0;
  const double ta = adt > 0.0 ? exp(G.two_alpha * ldt) : 0.0;
  const double psi = G.a * ta + 1.0;
  const double lp = log(psi);
  double* o = tab + (int64_t)kLagVals * l;
  o[0] = -G.tau * lp;
  o[1] = exp(-G.bg * lp);
  o[2] = ta;
  o[3] = psi;
  o[4] = lp;
  o[5] = ldt;
}

// cov_and_grad for the Gneiting kernel from a lag-table row (the same formulas).
__device__ __forceinline__ double cov_and_grad_lag(const GradKern& G, double dx, double dy,
                                                   const double* __restrict__ lt,
                                                   double dC[kGradMaxParams]) {
  const double h2 = dx * dx + dy * dy;
  const double ta = lt[2], psi = lt[3], lp = lt[4], ldt = lt[5], E = lt[1];
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

template <int QMAX>
struct GradLds {
  double x[64], y[64], t[64], v[64], al[64];
  double blk[QMAX][QMAX + 1];
};

template <int QMAX>
__global__ __launch_bounds__(256) void vecchia_grad_kernel(GradArgs A) {
  __shared__ GradLds<QMAX> sw[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  if (i >= A.n) return;  // whole wavefront; no workgroup barriers below
  const int m = A.m, P = A.P;
  const int r = lane;
  // ---- conditioning set: valid neighbors are earlier points forming a prefix ----
  int idx = -1;
  if (r < m) idx = A.nbr[i * m + r];
  const bool valid = r < m && idx >= 0 && (int64_t)idx < i;
  const unsigned long long vb = __ballot(valid);
  const unsigned long long mmask = m >= 64 ? ~0ull : ((1ull << m) - 1ull);
  const int p = (int)__builtin_ctzll(~(vb & mmask));
  const unsigned long long badb = __ballot(r < m && idx != -1 && !valid);
  if (r == 0 && m > 0 && ((badb & mmask) != 0ull || ((vb & mmask) >> p) != 0ull))
    flag_fail(A.bad_nbr, i);
  const int q = p + 1;  // block size, i last
  const int64_t row = r < p ? (int64_t)idx : i;  // lanes past the block: any valid row
  const double xr = A.sx[row], yr = A.sy[row], tr = A.t[row];
  const double yv = r < q ? A.y[row] : 0.0;
  // ---- block Sigma~_SS: the q(q+1)/2 lower entries spread over the lanes, through
  //      LDS into registers (lane r holds row r; identity beyond q) ----
  double* sx_ = sw[wave].x;
  double* sy_ = sw[wave].y;
  double* st_ = sw[wave].t;
  double(*blk)[QMAX + 1] = sw[wave].blk;
  sx_[r] = xr;
  sy_[r] = yr;
  st_[r] = tr;
  wave_lds_sync();
  const int npair = q * (q + 1) / 2;
  for (int e = r; e < npair; e += 64) {
    int rr, ss;
    pair_of(e, rr, ss);
    double c;
    if (A.lagtab) {
      const double* lt = A.lagtab + (int64_t)kLagVals * (int)fabs(st_[rr] - st_[ss]);
      c = gneiting_pair<double>(A.K, sx_[rr] - sx_[ss], sy_[rr] - sy_[ss], lt[0], lt[1]);
    } else {
      c = cov_eval<double>(A.K, sx_[rr] - sx_[ss], sy_[rr] - sy_[ss], st_[rr] - st_[ss]);
    }
    if (rr == ss) c += A.nugget;
    blk[rr][ss] = c;
  }
  wave_lds_sync();
  double a[QMAX];
#pragma unroll
  for (int s = 0; s < QMAX; ++s) a[s] = (r < q && s <= r) ? blk[r][s] : (r == s ? 1.0 : 0.0);
  // ---- Cholesky, pivots and multipliers through readlane ----
  bool okp = true;
#pragma unroll
  for (int kk = 0; kk < QMAX; ++kk) {
    const double d = rdl(a[kk], kk);
    const bool ok = d > 0.0 && d < INFINITY;
    okp = okp && ok;
    const double piv = ok ? sqrt(d) : 1.0;
    const double lm = r > kk ? a[kk] / piv : 0.0;
    if (r >= kk) a[kk] = r > kk ? lm : piv;
#pragma unroll
    for (int c = kk + 1; c < QMAX; ++c) a[c] -= lm * rdl(lm, c);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (r == 0 && !okp) flag_fail(A.fail, i);
  // ---- u = L^-1 y (forward) ----
  double u = 0.0, accf = 0.0;
#pragma unroll
  for (int k = 0; k < QMAX; ++k) {
    const double val = (yv - accf) / a[k];
    const double uk = rdl(val, k);
    if (r == k) u = uk;
    accf += r > k ? a[k] * uk : 0.0;
  }
  const double z = rdl(u, p);
  // ---- v = last row of L^-1: L' v = e_p (backward, column sums by reduction) ----
  double v = 0.0;
#pragma unroll
  for (int k = QMAX - 1; k >= 0; --k) {
    if (k <= p) {
      const double part = (r > k && r <= p) ? a[k] * v : 0.0;
      const double sum = wave_sum(part);
      const double lkk = rdl(a[k], k);
      const double vk = ((k == p) ? 1.0 : 0.0) - sum;
      if (r == k) v = vk / lkk;
    }
  }
  // ---- alpha_N = L_N^-T u_N (backward over the first p rows) ----
  double al = 0.0;
#pragma unroll
  for (int k = QMAX - 1; k >= 0; --k) {
    if (k < p) {
      const double part = (r > k && r < p) ? a[k] * al : 0.0;
      const double sum = wave_sum(part);
      const double lkk = rdl(a[k], k);
      const double uk = rdl(u, k);
      if (r == k) al = (uk - sum) / lkk;
    }
  }
  // ---- derivative forms v' dS v and v' dS alpha_N over the lower pairs (each
  //      off-diagonal pair stands for both (r, s) and (s, r)) ----
  sw[wave].v[r] = v;
  sw[wave].al[r] = al;
  wave_lds_sync();
  double t1[kGradMaxParams], t2[kGradMaxParams];
#pragma unroll
  for (int pp = 0; pp < kGradMaxParams; ++pp) t1[pp] = t2[pp] = 0.0;
  for (int e = r; e < npair; e += 64) {
    int rr, ss;
    pair_of(e, rr, ss);
    const double vr = sw[wave].v[rr], vs = sw[wave].v[ss];
    const double ar = sw[wave].al[rr], as = sw[wave].al[ss];
    double dC[kGradMaxParams];
    if (A.lagtab)
      cov_and_grad_lag(A.G, sx_[rr] - sx_[ss], sy_[rr] - sy_[ss],
                       A.lagtab + (int64_t)kLagVals * (int)fabs(st_[rr] - st_[ss]), dC);
    else
      cov_and_grad(A.G, sx_[rr] - sx_[ss], sy_[rr] - sy_[ss], st_[rr] - st_[ss], dC);
    const bool diag = rr == ss;
    const double wv = diag ? vr * vs : 2.0 * vr * vs;
    const double wa = diag ? vr * as : vr * as + vs * ar;
#pragma unroll
    for (int pp = 0; pp < kGradMaxParams; ++pp) {
      t1[pp] += dC[pp] * wv;
      t2[pp] += dC[pp] * wa;
    }
    if (diag) {  // nugget: dSigma~ = I
      t1[1] += wv;
      t2[1] += wa;
    }
  }
  // D_i = L_pp^2: log D_i = 2 log L_pp
  double lpiv = 0.0;
#pragma unroll
  for (int k = 0; k < QMAX; ++k)
    if (k == p) lpiv = rdl(a[k], k);
  for (int pp = 0; pp < P; ++pp) {
    const double s1 = wave_sum(t1[pp]);
    const double s2 = wave_sum(t2[pp]);
    if (r == 0) A.g[(int64_t)pp * A.n + i] = 0.5 * ((1.0 - z * z) * s1 - 2.0 * z * s2);
  }
  if (r == 0) {
    A.logD[i] = 2.0 * log(lpiv);
    A.z[i] = z;
  }
}

}  // namespace

hipError_t launch_grad_lags(const GradKern& G, int nlag, double* tab, hipStream_t s) {
  hipLaunchKernelGGL(grad_lag_kernel, dim3((unsigned)((nlag + 255) / 256)), dim3(256), 0, s, G,
                     nlag, tab);
  return hipGetLastError();
}

hipError_t launch_vecchia_grad(const GradArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + 3) / 4));
  if (a.m < 32)
    hipLaunchKernelGGL(vecchia_grad_kernel<32>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(vecchia_grad_kernel<64>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace vif
