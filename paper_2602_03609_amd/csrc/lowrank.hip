// Low-rank part of the VIF approximation (Sec. "Low-rank inducing point
// approximations" and Sec. "The Vecchia-inducing-point full-scale
// approximation"): Sigma_k = C(Z,Z) (+ jitter I), L_k = chol(Sigma_k),
// U = Sigma_nk L_k^-T so that Sigma_nk Sigma_k^-1 Sigma_kn = U U', and the
// Woodbury matrix M = I + W'W with q = W'z for the likelihood assembly.
//
// gfx950 design:
//  * k x k factorisations (Sigma_k, M) in FP64: blocked right-looking Cholesky
//    with 64-wide panels (panel factor + TRSM kernel, trailing-update kernel);
//    triangular inverse by independent 64-column blocks.
//  * U: the cross-covariance is generated straight into U's buffer, then
//    multiplied in place by P' = L_k^-T one 64-row tile per workgroup, column
//    blocks right to left (block J needs C columns <= J only), on MFMA.
//  * M: split-K Gram of [W | z] over row chunks into FP64 partial tiles (MFMA),
//    reduced in a fixed order (deterministic; no floating-point atomics).
#include <math.h>

#include <type_traits>

#include "internal.hpp"

namespace vif {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int NB = 64;

// ---------------------------------------------------------------- Sigma_k ----
__global__ void cov_kk_kernel(LowRankArgs A, double* __restrict__ S) {
  const int a = blockIdx.y;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.kpad) return;
  double v;
  if (a < A.k && b < A.k) {
    v = cov_eval<double>(A.K, A.zx[a] - A.zx[b], A.zy[a] - A.zy[b], A.zt[a] - A.zt[b]);
    if (a == b) v += A.jitter;
  } else {
    v = (a == b) ? 1.0 : 0.0;
  }
  S[(int64_t)a * A.kpad + b] = v;
}

// ---------------------------------------------------------------- Cholesky ---
// Panel kernel: block w factors the diagonal block jb (redundantly) and, for
// w > 0, solves row block jb + w of the panel against it.
__global__ __launch_bounds__(256) void chol_panel_kernel(int N, double* __restrict__ A, int jb,
                                                         unsigned long long* fail,
                                                         double* __restrict__ dscr) {
  __shared__ double Ld[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int w = blockIdx.x;
  const int64_t d0 = (int64_t)jb * NB;
  if (tid == 0) bad = -1;
  for (int e = tid; e < NB * NB; e += 256) {
    int r = e / NB, c = e % NB;
    Ld[r][c] = (c <= r) ? A[(d0 + r) * N + d0 + c] : 0.0;
  }
  __syncthreads();
  for (int kk = 0; kk < NB; ++kk) {
    if (tid == 0) {
      double d = Ld[kk][kk];
      if (!(d > 0.0) || !(d < INFINITY)) {
        if (bad < 0) bad = kk;
        d = 1.0;
      }
      Ld[kk][kk] = sqrt(d);
    }
    __syncthreads();
    if (tid > kk && tid < NB) Ld[tid][kk] /= Ld[kk][kk];
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
      int r = e / NB, c = e % NB;
      if (c > kk && r >= c) Ld[r][c] -= Ld[r][kk] * Ld[c][kk];
    }
    __syncthreads();
  }
  if (w == 0) {
    // The other blocks of this launch still read the unfactored diagonal block,
    // so the factor goes to scratch; the update launch copies it into place.
    if (tid == 0 && bad >= 0) atomicMin(fail, (unsigned long long)(d0 + bad));
    for (int e = tid; e < NB * NB; e += 256) {
      int r = e / NB, c = e % NB;
      dscr[e] = (c <= r) ? Ld[r][c] : 0.0;
    }
    return;
  }
  const int64_t r0 = (int64_t)(jb + w) * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    int r = e / NB, c = e % NB;
    X[r][c] = A[(r0 + r) * N + d0 + c];
  }
  __syncthreads();
  // X L' = A_panel: row r independent; column c sequential.
  if (tid < NB) {
    const int r = tid;
    for (int c = 0; c < NB; ++c) {
      double s = X[r][c];
      for (int cp = 0; cp < c; ++cp) s -= X[r][cp] * Ld[c][cp];
      X[r][c] = s / Ld[c][c];
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    int r = e / NB, c = e % NB;
    A[(r0 + r) * N + d0 + c] = X[r][c];
  }
}

// Trailing update of tile (IB, JB), jb < JB <= IB: A_IJ -= L_I,jb L_J,jb'.
// The last block copies the factored diagonal block from scratch into A.
__global__ __launch_bounds__(256) void chol_update_kernel(int N, double* __restrict__ A, int jb,
                                                          const double* __restrict__ dscr) {
  __shared__ double La[NB][NB + 1];
  __shared__ double Lb[NB][NB + 1];
  if (blockIdx.x == gridDim.x - 1) {
    const int64_t d0 = (int64_t)jb * NB;
    for (int e = threadIdx.x; e < NB * NB; e += 256) A[(d0 + e / NB) * N + d0 + e % NB] = dscr[e];
    return;
  }
  // Map blockIdx.x to (IB, JB) over the lower triangle of the trailing blocks.
  int t = blockIdx.x, IB = jb + 1;
  while (t >= IB - jb) {
    t -= IB - jb;
    ++IB;
  }
  const int JB = jb + 1 + t;
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)jb * NB, ra = (int64_t)IB * NB, rb = (int64_t)JB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    int r = e / NB, c = e % NB;
    La[r][c] = A[(ra + r) * N + c0 + c];
    Lb[r][c] = A[(rb + r) * N + c0 + c];
  }
  __syncthreads();
  const int tr = tid / 16, tc = tid % 16;
  double acc[4][4] = {};
  for (int kk = 0; kk < NB; ++kk) {
    double av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) av[i] = La[tr + 16 * i][kk];
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = Lb[tc + 16 * j][kk];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) A[(ra + tr + 16 * i) * N + rb + tc + 16 * j] -= acc[i][j];
}

// ----------------------------------------------------------- triangular inverse
// Block cb computes column block cb of P = L^-1: for rb = cb.., P_rb,cb =
// L_rb,rb^-1 (delta I - sum_{cb<=j<rb} L_rb,j P_j,cb).
__global__ __launch_bounds__(256) void trinv_kernel(int N, const double* __restrict__ L,
                                                    double* __restrict__ P) {
  __shared__ double Ta[NB][NB + 1];
  __shared__ double Tb[NB][NB + 1];
  __shared__ double R[NB][NB + 1];
  const int cb = blockIdx.x;
  const int NT = N / NB;
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)cb * NB;
  for (int rb = 0; rb < cb; ++rb)
    for (int e = tid; e < NB * NB; e += 256) P[((int64_t)rb * NB + e / NB) * N + c0 + e % NB] = 0.0;
  const int tr = tid / 16, tc = tid % 16;
  for (int rb = cb; rb < NT; ++rb) {
    const int64_t r0 = (int64_t)rb * NB;
    double acc[4][4] = {};
    for (int j = cb; j < rb; ++j) {
      __syncthreads();
      for (int e = tid; e < NB * NB; e += 256) {
        int r = e / NB, c = e % NB;
        Ta[r][c] = L[(r0 + r) * N + (int64_t)j * NB + c];          // L_rb,j [r][c]
        Tb[r][c] = P[((int64_t)j * NB + r) * N + c0 + c];          // P_j,cb [r][c]
      }
      __syncthreads();
      for (int kk = 0; kk < NB; ++kk) {
        double av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = Ta[tr + 16 * i][kk];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) bv[jj] = Tb[kk][tc + 16 * jj];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) acc[i][jj] += av[i] * bv[jj];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        int r = tr + 16 * i, c = tc + 16 * jj;
        R[r][c] = ((rb == cb && r == c) ? 1.0 : 0.0) - acc[i][jj];
      }
    for (int e = tid; e < NB * NB; e += 256) {
      int r = e / NB, c = e % NB;
      Ta[r][c] = L[(r0 + r) * N + r0 + c];  // diagonal block
    }
    __syncthreads();
    // Forward substitution, one column per thread.
    if (tid < NB) {
      const int c = tid;
      for (int r = 0; r < NB; ++r) {
        double s = R[r][c];
        for (int rp = 0; rp < r; ++rp) s -= Ta[r][rp] * R[rp][c];
        R[r][c] = s / Ta[r][r];
      }
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
      int r = e / NB, c = e % NB;
      P[(r0 + r) * N + c0 + c] = R[r][c];
    }
  }
}

// --------------------------------------------------------------- U = C P' ----
template <typename UT>
__global__ __launch_bounds__(256) void crosscov_kernel(LowRankArgs A, UT* __restrict__ U) {
  const int64_t i = blockIdx.x;
  const int l = blockIdx.y * 256 + threadIdx.x;
  if (l >= A.kpad) return;
  UT v = UT(0);
  if (l < A.k) {
    const double dx = A.sx[i] - A.zx[l], dy = A.sy[i] - A.zy[l], dt = A.t[i] - A.zt[l];
    if (sizeof(UT) == 8)
      v = (UT)cov_eval<double>(A.K, dx, dy, dt);
    else
      v = (UT)cov_eval<float>(A.K, (float)dx, (float)dy, (float)dt);
  }
  U[i * A.kpad + l] = v;
}

// FP64: U[I, J] = sum_{l < (J+1)*64} C[I, l] P[J, l], in place, J right to left.
__global__ __launch_bounds__(256) void trmm_f64_kernel(int64_t n, int kpad,
                                                       double* __restrict__ U,
                                                       const double* __restrict__ P) {
  constexpr int BM = 64, BK = 16;
  __shared__ double As[BM][BK + 1];
  __shared__ double Bs[NB][BK + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t I0 = (int64_t)blockIdx.x * BM;
  const int NT = kpad / NB;
  const int lr = tid >> 2, lk = (tid & 3) * 4;  // loader: row, first k
  const bool row_ok = I0 + lr < n;
  for (int jb = NT - 1; jb >= 0; --jb) {
    const int J0 = jb * NB;
    d4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
    const int kend = J0 + NB;
    for (int k0 = 0; k0 < kend; k0 += BK) {
      __syncthreads();
      {
        double2 u0 = {0.0, 0.0}, u1 = {0.0, 0.0};
        if (row_ok) {
          const double2* src = reinterpret_cast<const double2*>(U + (I0 + lr) * kpad + k0 + lk);
          u0 = src[0];
          u1 = src[1];
        }
        As[lr][lk] = u0.x; As[lr][lk + 1] = u0.y; As[lr][lk + 2] = u1.x; As[lr][lk + 3] = u1.y;
        const double2* ps = reinterpret_cast<const double2*>(P + (int64_t)(J0 + lr) * kpad + k0 + lk);
        double2 p0 = ps[0], p1 = ps[1];
        Bs[lr][lk] = p0.x; Bs[lr][lk + 1] = p0.y; Bs[lr][lk + 2] = p1.x; Bs[lr][lk + 3] = p1.y;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
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
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = I0 + wr * 32 + a * 16 + mfma16_row_f64(lane, e);
          const int col = J0 + wc * 32 + b * 16 + (lane & 15);
          if (row < n) U[row * kpad + col] = acc[a][b][e];
        }
  }
}

// FP32 storage (FP32 and split-BF16 arithmetic): same in-place scheme; P is
// converted from FP64 on load.
template <bool BF16X3>
__global__ __launch_bounds__(256) void trmm_f32_kernel(int64_t n, int kpad, float* __restrict__ U,
                                                       const double* __restrict__ P) {
  constexpr int BM = 64, BK = 32;
  __shared__ float As[BM][BK + 4];
  __shared__ float Bs[NB][BK + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t I0 = (int64_t)blockIdx.x * BM;
  const int NT = kpad / NB;
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const bool row_ok = I0 + lr < n;
  for (int jb = NT - 1; jb >= 0; --jb) {
    const int J0 = jb * NB;
    f4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
    const int kend = J0 + NB;
    for (int k0 = 0; k0 < kend; k0 += BK) {
      __syncthreads();
      {
        float4 u0 = {0.f, 0.f, 0.f, 0.f}, u1 = {0.f, 0.f, 0.f, 0.f};
        if (row_ok) {
          const float4* src = reinterpret_cast<const float4*>(U + (I0 + lr) * kpad + k0 + lk);
          u0 = src[0];
          u1 = src[1];
        }
        As[lr][lk + 0] = u0.x; As[lr][lk + 1] = u0.y; As[lr][lk + 2] = u0.z; As[lr][lk + 3] = u0.w;
        As[lr][lk + 4] = u1.x; As[lr][lk + 5] = u1.y; As[lr][lk + 6] = u1.z; As[lr][lk + 7] = u1.w;
        const double* ps = P + (int64_t)(J0 + lr) * kpad + k0 + lk;
#pragma unroll
        for (int e = 0; e < 8; ++e) Bs[lr][lk + e] = (float)ps[e];
      }
      __syncthreads();
      if constexpr (!BF16X3) {
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
          const int kk = ks * 4 + (lane >> 4);
          float av[2], bv[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) av[a] = As[wr * 32 + a * 16 + (lane & 15)][kk];
#pragma unroll
          for (int b = 0; b < 2; ++b) bv[b] = Bs[wc * 32 + b * 16 + (lane & 15)][kk];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
      } else {
        const int kb = (lane >> 4) * 8;
        bf8v ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float x = As[wr * 32 + a * 16 + (lane & 15)][kb + e];
            __bf16 h = (__bf16)x;
            ah[a][e] = h;
            al[a][e] = (__bf16)(x - (float)h);
          }
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float x = Bs[wc * 32 + b * 16 + (lane & 15)][kb + e];
            __bf16 h = (__bf16)x;
            bh[b][e] = h;
            bl[b][e] = (__bf16)(x - (float)h);
          }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
          }
      }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = I0 + wr * 32 + a * 16 + mfma16_row_f32acc(lane, e);
          const int col = J0 + wc * 32 + b * 16 + (lane & 15);
          if (row < n) U[row * kpad + col] = acc[a][b][e];
        }
  }
}

// ------------------------------------------------------------------- SYRK ----
__device__ __forceinline__ void tile_of(int t, int& TI, int& TJ) {
  TI = 0;
  while (t > TI) {
    t -= TI + 1;
    ++TI;
  }
  TJ = t;
}

// part[c][t] = sum over the rows of chunk c of W[:, TI]' W[:, TJ] (64 x 64, FP64).
//
// Block b serves row chunk c = b % nchunk and tile pair t = b / nchunk. With
// nchunk = 8 and the round-robin dispatch of workgroups over the 8 XCDs, every
// tile pair of one chunk runs on the same XCD, so the chunk's W rows are read
// from HBM about once and then served by that XCD's L2 to all tile pairs.
// Staging through LDS is double-buffered: the next rows are loaded into
// registers while the MFMAs consume the current buffer.
template <int PREC>
__global__ __launch_bounds__(256) void syrk_kernel(int64_t n, int kpad, const void* __restrict__ Wv,
                                                   double* __restrict__ part, int nchunk,
                                                   int ntile) {
  constexpr int BK = PREC >= 2 ? 32 : 16;  // rows per step (the MFMA K)
  using UT = typename std::conditional<PREC == 0, double, float>::type;
  constexpr int EPT = BK * NB / 256;       // elements per thread per operand per step
  constexpr int VW = 16 / sizeof(UT);      // elements per 16-byte load
  __shared__ UT Wa[2][BK][NB + 4];
  __shared__ UT Wb[2][BK][NB + 4];
  const UT* W = reinterpret_cast<const UT*>(Wv);
  const int c = blockIdx.x % nchunk;
  const int t = blockIdx.x / nchunk;
  int TI, TJ;
  tile_of(t, TI, TJ);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t chunk = (n + nchunk - 1) / nchunk;
  const int64_t rbeg = (int64_t)c * chunk;
  const int64_t rend = rbeg + chunk < n ? rbeg + chunk : n;
  const int lrow = tid / (NB / EPT), lcol = (tid % (NB / EPT)) * EPT;
  using AccT = typename std::conditional<PREC == 0, d4v, f4v>::type;
  AccT acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b2 = 0; b2 < 2; ++b2) acc[a][b2] = AccT{0, 0, 0, 0};
  double accd[2][2][4] = {};
  int flush = 0;

  UT ra[EPT], rb[EPT];
  auto load = [&](int64_t r0) {
    const int64_t row = r0 + lrow;
    if (row < rend) {
      const UT* pa = W + row * kpad + TI * NB + lcol;
      const UT* pb = W + row * kpad + TJ * NB + lcol;
#pragma unroll
      for (int v = 0; v < EPT / VW; ++v) {
        const float4 xa = reinterpret_cast<const float4*>(pa)[v];
        const float4 xb = reinterpret_cast<const float4*>(pb)[v];
        *reinterpret_cast<float4*>(&ra[v * VW]) = xa;
        *reinterpret_cast<float4*>(&rb[v * VW]) = xb;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        ra[e] = UT(0);
        rb[e] = UT(0);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      Wa[buf][lrow][lcol + e] = ra[e];
      Wb[buf][lrow][lcol + e] = rb[e];
    }
  };

  const int64_t nsteps = (rend - rbeg + BK - 1) / BK;
  if (nsteps > 0) {
    load(rbeg);
    store(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < nsteps; ++st) {
    const int buf = (int)(st & 1);
    const bool more = st + 1 < nsteps;
    if (more) load(rbeg + (st + 1) * BK);
    if constexpr (PREC <= 1) {
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        UT av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = Wa[buf][kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) bv[b2] = Wb[buf][kk][wc * 32 + b2 * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b2 = 0; b2 < 2; ++b2) {
            if constexpr (PREC == 0)
              acc[a][b2] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b2], acc[a][b2], 0, 0, 0);
            else
              acc[a][b2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b2], acc[a][b2], 0, 0, 0);
          }
      }
    } else {
      // Split-BF16: 2 terms / 3 products (PREC 2) or 3 terms / 6 products (PREC 3).
      constexpr int NS = PREC == 3 ? 3 : 2;
      const int kb = (lane >> 4) * 8;
      bf8v pa[2][NS], pb[2][NS];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          float x = (float)Wa[buf][kb + e][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
          for (int sp = 0; sp < NS; ++sp) {
            const __bf16 h = (__bf16)x;
            pa[a][sp][e] = h;
            x -= (float)h;
          }
        }
#pragma unroll
      for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          float x = (float)Wb[buf][kb + e][wc * 32 + b2 * 16 + (lane & 15)];
#pragma unroll
          for (int sp = 0; sp < NS; ++sp) {
            const __bf16 h = (__bf16)x;
            pb[b2][sp][e] = h;
            x -= (float)h;
          }
        }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) {
          if constexpr (NS == 3) {
            acc[a][b2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[a][2], pb[b2][0], acc[a][b2], 0, 0, 0);
            acc[a][b2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[a][1], pb[b2][1], acc[a][b2], 0, 0, 0);
            acc[a][b2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[a][0], pb[b2][2], acc[a][b2], 0, 0, 0);
          }
          acc[a][b2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[a][1], pb[b2][0], acc[a][b2], 0, 0, 0);
          acc[a][b2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[a][0], pb[b2][1], acc[a][b2], 0, 0, 0);
          acc[a][b2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[a][0], pb[b2][0], acc[a][b2], 0, 0, 0);
        }
    }
    if constexpr (PREC != 0) {
      // FP32 accumulation inside tiles of 1024 rows, FP64 across them.
      if (++flush == 1024 / BK) {
        flush = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b2 = 0; b2 < 2; ++b2) {
#pragma unroll
            for (int e = 0; e < 4; ++e) accd[a][b2][e] += (double)acc[a][b2][e];
            acc[a][b2] = AccT{0, 0, 0, 0};
          }
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
  }
  double* out = part + ((int64_t)c * ntile + t) * (NB * NB);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wr * 32 + a * 16 +
                        (PREC == 0 ? mfma16_row_f64(lane, e) : mfma16_row_f32acc(lane, e));
        const int col = wc * 32 + b2 * 16 + (lane & 15);
        out[row * NB + col] = accd[a][b2][e] + (double)acc[a][b2][e];
      }
}

__global__ void syrk_reduce_kernel(int k, int kpad, const double* __restrict__ part, int splits,
                                   int ntile, double* __restrict__ M, double* __restrict__ q,
                                   double* __restrict__ zz) {
  const int t = blockIdx.x;
  int TI, TJ;
  tile_of(t, TI, TJ);
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += part[((int64_t)sp * ntile + t) * (NB * NB) + e];
    const int r = TI * NB + e / NB, c = TJ * NB + e % NB;
    double v = (r == c) ? 1.0 : 0.0;
    if (r < k && c < k) v += s;
    M[(int64_t)r * kpad + c] = v;
    if (r == k && c < k) q[c] = s;
    if (r == k && c == k) *zz = s;
  }
}

}  // namespace

hipError_t launch_cov_kk(const LowRankArgs& a, double* S, hipStream_t s) {
  dim3 grid((a.kpad + 255) / 256, a.kpad);
  hipLaunchKernelGGL(cov_kk_kernel, grid, dim3(256), 0, s, a, S);
  return hipGetLastError();
}

hipError_t launch_cholesky(int N, double* A, double* scratch, unsigned long long* fail,
                           hipStream_t s) {
  const int NT = N / NB;
  for (int jb = 0; jb < NT; ++jb) {
    hipLaunchKernelGGL(chol_panel_kernel, dim3(NT - jb), dim3(256), 0, s, N, A, jb, fail, scratch);
    const int nt = NT - jb - 1;
    hipLaunchKernelGGL(chol_update_kernel, dim3(nt * (nt + 1) / 2 + 1), dim3(256), 0, s, N, A, jb,
                       (const double*)scratch);
  }
  return hipGetLastError();
}

hipError_t launch_trinv(int N, const double* L, double* P, hipStream_t s) {
  hipLaunchKernelGGL(trinv_kernel, dim3(N / NB), dim3(256), 0, s, N, L, P);
  return hipGetLastError();
}

hipError_t launch_crosscov(const LowRankArgs& a, void* U, int prec, hipStream_t s) {
  dim3 g1((unsigned)a.n, (a.kpad + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL(crosscov_kernel<double>, g1, dim3(256), 0, s, a, (double*)U);
  else
    hipLaunchKernelGGL(crosscov_kernel<float>, g1, dim3(256), 0, s, a, (float*)U);
  return hipGetLastError();
}

hipError_t launch_trmm(const LowRankArgs& a, const double* P, void* U, int prec, hipStream_t s) {
  const unsigned g2 = (unsigned)((a.n + 63) / 64);
  if (prec == 0)
    hipLaunchKernelGGL(trmm_f64_kernel, dim3(g2), dim3(256), 0, s, a.n, a.kpad, (double*)U, P);
  else if (prec == 1)
    hipLaunchKernelGGL(trmm_f32_kernel<false>, dim3(g2), dim3(256), 0, s, a.n, a.kpad, (float*)U,
                       P);
  else
    hipLaunchKernelGGL(trmm_f32_kernel<true>, dim3(g2), dim3(256), 0, s, a.n, a.kpad, (float*)U,
                       P);
  return hipGetLastError();
}

int syrk_splits(int64_t, int) { return 8; }

hipError_t launch_syrk(int64_t n, int kpad, const void* W, int prec, double* part, int splits,
                       hipStream_t s) {
  const int nt = kpad / NB;
  const int ntile = nt * (nt + 1) / 2;
  dim3 grid(ntile * splits);
  if (prec == 0)
    hipLaunchKernelGGL(syrk_kernel<0>, grid, dim3(256), 0, s, n, kpad, W, part, splits, ntile);
  else if (prec == 1)
    hipLaunchKernelGGL(syrk_kernel<1>, grid, dim3(256), 0, s, n, kpad, W, part, splits, ntile);
  else if (prec == 2)
    hipLaunchKernelGGL(syrk_kernel<2>, grid, dim3(256), 0, s, n, kpad, W, part, splits, ntile);
  else
    hipLaunchKernelGGL(syrk_kernel<3>, grid, dim3(256), 0, s, n, kpad, W, part, splits, ntile);
  return hipGetLastError();
}

hipError_t launch_syrk_reduce(int k, int kpad, const double* part, int splits, double* M,
                              double* q, double* zz, hipStream_t s) {
  const int nt = kpad / NB;
  const int ntile = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(syrk_reduce_kernel, dim3(ntile), dim3(256), 0, s, k, kpad, part, splits,
                     ntile, M, q, zz);
  return hipGetLastError();
}

}  // namespace vif
