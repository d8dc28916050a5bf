// Residual-correlation neighbors for VIF. The VIF factor is built on the
// residual of the low-rank part (Sec. "The Vecchia-inducing-point full-scale
// approximation"); its conditioning sets are chosen by the correlation metric
// of Sec. "Correlation-based Vecchia neighbor selection" applied to the latent
// residual r(p, q) = C(p, q) - U_p . U_q, U = C(X, Z) L_k^-T:
//     rho(i, j) = |r(i, j)| / sqrt(r(i, i) r(j, j)),
// ranked for query i over j < i by key(i, j) = r(i, j)^2 / r(j, j) (the same
// order; r(i, i) is common to the row), key -1 when r(j, j) <= 0, ties to the
// lower index, min(i, m) entries and -1 padding.
//
// gfx950 design: the exact search is a brute force over the lower triangle,
// n^2 k / 2 multiply-adds of U U', so it is a GEMM with a top-m epilogue. One
// workgroup owns 64 queries and walks the 64-wide candidate blocks up to its
// own: the 64 x 64 tile of U_I U_J' on FP64 MFMA (K staged through LDS 16 at a
// time), then the tile's keys (covariance in FP64, minus the Gram) into LDS,
// then one lane per query merges the 64 candidates into its sorted list in LDS
// (a candidate enters only if it beats the m-th key; blocks and columns are
// visited in increasing index, so ties keep the earlier index). Workgroups are
// launched heaviest (last) block first. The global loads of the next K stage
// are issued before the current stage's products. For the Gneiting kernel with
// integer times the factors that depend on the time lag alone come from a
// table per lag (gneiting_lag), and each entry costs one exponential
// (gneiting_pair performs the operations of cov_eval; the values agree to
// rounding).
#include <math.h>

#include "internal.hpp"

namespace vif {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int RB = 64;    // queries per workgroup and candidates per tile
constexpr int RBK = 16;   // K per LDS stage

__global__ __launch_bounds__(256) void resid_lag_kernel(KernDev K, int nlag, double* __restrict__ tab) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= nlag) return;
  double a, e;
  gneiting_lag<double>(K, (double)l, a, e);
  tab[2 * l] = a;
  tab[2 * l + 1] = e;
}

__global__ __launch_bounds__(256) void resid_var_kernel(int64_t n, int kpad, double sigma2,
                                                        const double* __restrict__ U,
                                                        double* __restrict__ d) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int l = lane; l < kpad; l += 64) {
    const double u = U[i * kpad + l];
    s += u * u;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) d[i] = sigma2 - s;
}

// MAXM: list capacity (32 when m <= 32, so that two workgroups fit in one CU's
// LDS; 64 otherwise).
template <int MAXM>
__global__ __launch_bounds__(256) void resid_topm_kernel(ResidArgs A) {
  __shared__ double As[RB][RBK + 1];
  __shared__ double Bs[RB][RBK + 1];
  __shared__ double keyT[RB][RB + 1];
  __shared__ double lk[RB][MAXM];
  __shared__ int32_t li[RB][MAXM];
  __shared__ int32_t cnt[RB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int nb = (int)((A.n + RB - 1) / RB);
  const int I = nb - 1 - (int)blockIdx.x;
  const int64_t I0 = (int64_t)I * RB;
  const int m = A.m;
  if (tid < RB) cnt[tid] = 0;
  const int lr = tid >> 2, lq = (tid & 3) * 4;  // loader: row, first k of the stage
  for (int J = 0; J <= I; ++J) {
    const int64_t J0 = (int64_t)J * RB;
    __syncthreads();  // the previous tile's merge has read keyT
    d4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
    // Stage k0's slice of U_I and U_J: 16 doubles per row, four per thread.
    double2 u0 = {0.0, 0.0}, u1 = {0.0, 0.0}, v0 = {0.0, 0.0}, v1 = {0.0, 0.0};
    auto fetch = [&](int k0) __attribute__((always_inline)) {
      if (I0 + lr < A.n) {
        const double2* src = reinterpret_cast<const double2*>(A.U + (I0 + lr) * A.kpad + k0 + lq);
        u0 = src[0];
        u1 = src[1];
      }
      if (J0 + lr < A.n) {
        const double2* src = reinterpret_cast<const double2*>(A.U + (J0 + lr) * A.kpad + k0 + lq);
        v0 = src[0];
        v1 = src[1];
      }
    };
    if (A.kpad > 0) fetch(0);
    for (int k0 = 0; k0 < A.kpad; k0 += RBK) {
      __syncthreads();
      As[lr][lq] = u0.x; As[lr][lq + 1] = u0.y; As[lr][lq + 2] = u1.x; As[lr][lq + 3] = u1.y;
      Bs[lr][lq] = v0.x; Bs[lr][lq + 1] = v0.y; Bs[lr][lq + 2] = v1.x; Bs[lr][lq + 3] = v1.y;
      __syncthreads();
      if (k0 + RBK < A.kpad) fetch(k0 + RBK);  // in flight during the products
#pragma unroll
      for (int ks = 0; ks < RBK / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        double av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = As[wr * 32 + a * 16 + (lane & 15)][kk];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Bs[wc * 32 + b * 16 + (lane & 15)][kk];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    // Keys of the tile: candidate j = J0 + col for query i = I0 + row, j < i.
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = wc * 32 + b * 16 + (lane & 15);
      const int64_t j = J0 + col;
      const bool jok = j < A.n;
      const double xj = jok ? A.sx[j] : 0.0, yj = jok ? A.sy[j] : 0.0, tj = jok ? A.t[j] : 0.0;
      const double dj = jok ? A.d[j] : 0.0;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = wr * 32 + a * 16 + mfma16_row_f64(lane, e);
          const int64_t i = I0 + row;
          double key = -INFINITY;  // not a candidate
          if (i < A.n && j < i) {
            const double ti = A.t[i];
            double c;
            if (A.lagtab) {
              const int lag = (int)fabs(ti - tj);
              c = gneiting_pair<double>(A.K, A.sx[i] - xj, A.sy[i] - yj, A.lagtab[2 * lag],
                                        A.lagtab[2 * lag + 1]);
            } else {
              c = cov_eval<double>(A.K, A.sx[i] - xj, A.sy[i] - yj, ti - tj);
            }
            const double r = c - acc[a][b][e];
            key = dj > 0.0 ? r * r / dj : -1.0;
          }
          keyT[row][col] = key;
        }
    }
    __syncthreads();
    if (tid < RB) {
      const int r = tid;
      int c0 = cnt[r];
      for (int c = 0; c < RB; ++c) {
        const double key = keyT[r][c];
        if (key == -INFINITY) continue;
        if (c0 == m && !(key > lk[r][m - 1])) continue;
        int pos = c0 < m ? c0 : m - 1;
        while (pos > 0 && lk[r][pos - 1] < key) {
          lk[r][pos] = lk[r][pos - 1];
          li[r][pos] = li[r][pos - 1];
          --pos;
        }
        lk[r][pos] = key;
        li[r][pos] = (int32_t)(J0 + c);
        if (c0 < m) ++c0;
      }
      cnt[r] = c0;
    }
  }
  __syncthreads();
  if (tid < RB && I0 + tid < A.n) {
    const int64_t i = I0 + tid;
    for (int q = 0; q < m; ++q) A.nbr[i * m + q] = q < cnt[tid] ? li[tid][q] : -1;
  }
}

}  // namespace

hipError_t launch_resid_var(int64_t n, int kpad, double sigma2, const double* U, double* d,
                            hipStream_t s) {
  hipLaunchKernelGGL(resid_var_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, kpad,
                     sigma2, U, d);
  return hipGetLastError();
}

hipError_t launch_resid_lags(const KernDev& K, int nlag, double* tab, hipStream_t s) {
  hipLaunchKernelGGL(resid_lag_kernel, dim3((unsigned)((nlag + 255) / 256)), dim3(256), 0, s, K,
                     nlag, tab);
  return hipGetLastError();
}

hipError_t launch_resid_topm(const ResidArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.n + RB - 1) / RB);
  if (a.m <= 32)
    hipLaunchKernelGGL(resid_topm_kernel<32>, dim3(nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(resid_topm_kernel<64>, dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace vif
