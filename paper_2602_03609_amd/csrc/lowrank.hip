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
//  * M: split-K Gram of [W | z] over row chunks into partial tiles on MFMA
//    (FP64 tiles for the FP64/FP32 modes; for the split-BF16 modes, 128 x 128
//    FP32 tiles over 4096-row chunks from operands split once at staging),
//    reduced in FP64 in a fixed order (deterministic; no floating-point atomics).
#include <math.h>

#include <atomic>
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
// Lane 4q + go's value to the four lanes 4q .. 4q + 3 (a DPP quad permutation;
// go is a compile-time constant where it is called).
__device__ __forceinline__ double quad_bcast(double x, int go) {
  const long long b = __double_as_longlong(x);
  int lo = (int)b, hi = (int)(b >> 32);
  switch (go) {
    case 0: lo = __builtin_amdgcn_update_dpp(lo, lo, 0x00, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(hi, hi, 0x00, 0xF, 0xF, false); break;
    case 1: lo = __builtin_amdgcn_update_dpp(lo, lo, 0x55, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(hi, hi, 0x55, 0xF, 0xF, false); break;
    case 2: lo = __builtin_amdgcn_update_dpp(lo, lo, 0xAA, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(hi, hi, 0xAA, 0xF, 0xF, false); break;
    default: lo = __builtin_amdgcn_update_dpp(lo, lo, 0xFF, 0xF, 0xF, false);
             hi = __builtin_amdgcn_update_dpp(hi, hi, 0xFF, 0xF, 0xF, false); break;
  }
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Solves T y = b (T lower triangular 64 x 64 in LDS, rd[r] = 1 / T[r][r] in LDS)
// for 64 right-hand sides at once, all in registers: lanes 4s..4s+3 hold
// right-hand side s, lane 4s + g holding entries g, g + 4, ..., g + 60 in v[].
// Column r of the elimination is broadcast from its owner lane within the quad
// by a DPP move (no LDS round trip on the serial chain); no barriers.
// Multiplying by the stored reciprocal keeps the division off the serial chain
// of the 64 columns. Every lane of the wavefront takes part.
__device__ __forceinline__ void tri_solve_regs(double v[16], const double (*T)[NB + 1],
                                               const double* rd, int g) {
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    const int go = r & 3, io = r >> 2;
    double y = v[io] * rd[r];
    y = quad_bcast(y, go);
    if (g == go) v[io] = y;
#pragma unroll
    for (int i = io; i < 16; ++i) {
      if (i > io || g > go) v[i] -= T[g + 4 * i][r] * y;
    }
  }
}

// x from lane `lane` of the wave (a uniform value, through scalar registers).
__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Panel step: block w factors the diagonal block jb (redundantly) and, for
// w > 0, solves row block jb + w of the panel against it.
__device__ __forceinline__ void chol_panel_body(int N, double* __restrict__ A, int jb,
                                                unsigned long long* fail,
                                                double* __restrict__ dscr, const int w) {
  __shared__ double Ld[NB][NB + 1];
  __shared__ double rd[NB];
  __shared__ __attribute__((aligned(16))) double sm[NB];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int64_t d0 = (int64_t)jb * NB;
  const int s = tid >> 2, g = tid & 3;
  // Right-looking factorisation of the diagonal block by wave 0 in registers:
  // lane r holds row r; the pivot is read from its owner lane with readlane
  // (scalar registers) and the multipliers l_c through LDS, with no
  // synchronisation until the factor is stored. Entries above the diagonal
  // are never touched: the multiplier of rows r <= kk is zero. The multipliers
  // are a[kk] / sqrt(d) formed as a[kk] * rs with rs = 1 / sqrt(d) from the
  // hardware estimate and two Newton steps (rs += rs (1 - d rs^2) / 2), which
  // keeps the serial chain from one column to the next short; the diagonal
  // itself is the correctly rounded sqrt(d), computed beside the chain.
  if (tid < NB) {
    const int r = tid;
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) a[c] = (c <= r) ? A[(d0 + r) * N + d0 + c] : 0.0;
    int badl = -1;
#pragma unroll
    for (int kk = 0; kk < NB; ++kk) {
      const double d = readlane_f64(a[kk], kk);
      const bool okp = d > 0.0 && d < INFINITY;
      const double piv = okp ? sqrt(d) : 1.0;
      double rs = __builtin_amdgcn_rsq(okp ? d : 1.0);
#pragma unroll
      for (int it = 0; it < 2; ++it) rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
      rs = okp ? rs : 1.0;
      if (!okp && badl < 0) badl = kk;
      const double lm = r > kk ? a[kk] * rs : 0.0;
      if (r >= kk) a[kk] = r > kk ? lm : piv;
      // The multipliers reach the other lanes through LDS, one broadcast read per
      // two columns (a wavefront's LDS operations complete in issue order, so the
      // reads see this step's writes and the next step's writes follow the reads;
      // the wavefront-scope fences keep the compiler from reordering them).
      sm[r] = lm;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int c2 = (kk + 1) & ~1; c2 < NB; c2 += 2) {
        const double2 p = *reinterpret_cast<const double2*>(&sm[c2]);
        if (c2 >= kk + 1) a[c2] -= lm * p.x;
        a[c2 + 1] -= lm * p.y;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_sched_barrier(0);  // one column at a time (bounded scalar live ranges)
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) Ld[r][c] = (c <= r) ? a[c] : 0.0;
    rd[r] = 1.0 / Ld[r][r];
    if (r == 0) bad = badl;
  }
  __syncthreads();
  if (w == 0) {
    // The other blocks of this launch still read the unfactored diagonal block,
    // so the factor goes to scratch; the update launch copies it into place.
    if (tid == 0 && bad >= 0) atomicMin(fail, (unsigned long long)(d0 + bad));
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, c = e % NB;
      dscr[e] = (c <= r) ? Ld[r][c] : 0.0;
    }
    return;
  }
  // X L' = A_panel, i.e. L x = a for each row a of the panel block: row s,
  // entries g + 4i.
  const int64_t r0 = (int64_t)(jb + w) * NB;
  double v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = A[(r0 + s) * N + d0 + g + 4 * i];
  tri_solve_regs(v, Ld, rd, g);
#pragma unroll
  for (int i = 0; i < 16; ++i) A[(r0 + s) * N + d0 + g + 4 * i] = v[i];
}

__global__ __launch_bounds__(256) void chol_panel_kernel(int N, double* __restrict__ A, int jb,
                                                         unsigned long long* fail,
                                                         double* __restrict__ dscr) {
  chol_panel_body(N, A, jb, fail, dscr, blockIdx.x);
}

// Trailing update of tile (IB, JB), jb < JB <= IB: A_IJ -= L_I,jb L_J,jb'.
// The last block copies the factored diagonal block from scratch into A.
// Update step: block b < nblk - 1 updates one lower trailing block; the last one
// copies the factored diagonal block into place.
__device__ __forceinline__ void chol_update_body(int N, double* __restrict__ A, int jb,
                                                 const double* __restrict__ dscr, const int b,
                                                 const int nblk) {
  __shared__ double La[NB][NB + 1];
  __shared__ double Lb[NB][NB + 1];
  if (b == nblk - 1) {
    const int64_t d0 = (int64_t)jb * NB;
    for (int e = threadIdx.x; e < NB * NB; e += 256) A[(d0 + e / NB) * N + d0 + e % NB] = dscr[e];
    return;
  }
  // Map b to (IB, JB) over the lower triangle of the trailing blocks.
  int t = b, IB = jb + 1;
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

__global__ __launch_bounds__(256) void chol_update_kernel(int N, double* __restrict__ A, int jb,
                                                          const double* __restrict__ dscr) {
  chol_update_body(N, A, jb, dscr, blockIdx.x, gridDim.x);
}

// One panel or update step of the blocked Cholesky for a set of matrices at once:
// the launch's blocks are dealt to the matrices by the prefix pre[] (matrix p
// takes blocks pre[p] .. pre[p + 1] - 1), so independent factorisations share
// the step's launch instead of queueing their own.
__device__ __forceinline__ int cholset_member(const CholSet& S, int b) {
  int p = 0;
  while (p + 1 < S.count && b >= S.pre[p + 1]) ++p;
  return p;
}

__global__ __launch_bounds__(256) void chol_panel_set_kernel(CholSet S) {
  const int p = cholset_member(S, blockIdx.x);
  chol_panel_body(S.N[p], S.A[p], S.jb, S.fail[p], S.dscr[p], blockIdx.x - S.pre[p]);
}

__global__ __launch_bounds__(256) void chol_update_set_kernel(CholSet S) {
  const int p = cholset_member(S, blockIdx.x);
  chol_update_body(S.N[p], S.A[p], S.jb, S.dscr[p], blockIdx.x - S.pre[p], S.pre[p + 1] - S.pre[p]);
}

// ----------------------------------------------------------- triangular inverse
// P = L^-1 by doubling: the 64 x 64 diagonal blocks are inverted first; then,
// for block sizes b = 64, 128, 256, ..., each pair of adjacent inverted blocks
// A (upper left) and C (lower right) is joined by X = -C^-1 L_CA A^-1, the
// lower-left block of the inverse of [[L_A, 0], [L_CA, L_C]]. Each level is two
// launches of 64 x 64 FP64 tile products (T = L_CA A^-1 into scratch, then
// X = -C^-1 T), with as many workgroups as the level has output tiles, instead
// of one serial chain per column block.

// Block t: P_tt = L_tt^-1 (64 right-hand sides of the identity solved in
// registers) and the tiles of P above the diagonal in row block t set to zero.
__global__ __launch_bounds__(256) void trinv_diag_kernel(int N, const double* __restrict__ L,
                                                         double* __restrict__ P) {
  __shared__ double Ta[NB][NB + 1];
  __shared__ double rd[NB];
  const int t = blockIdx.x;
  const int NT = N / NB;
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)t * NB;
  for (int cb = t + 1; cb < NT; ++cb)
    for (int e = tid; e < NB * NB; e += 256) P[(r0 + e / NB) * N + (int64_t)cb * NB + e % NB] = 0.0;
  for (int e = tid; e < NB * NB; e += 256) Ta[e / NB][e % NB] = L[(r0 + e / NB) * N + r0 + e % NB];
  __syncthreads();
  if (tid < NB) rd[tid] = 1.0 / Ta[tid][tid];
  __syncthreads();
  const int sc = tid >> 2, g = tid & 3;
  double v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = (g + 4 * i == sc) ? 1.0 : 0.0;
  tri_solve_regs(v, Ta, rd, g);
#pragma unroll
  for (int i = 0; i < 16; ++i) P[(r0 + g + 4 * i) * N + r0 + sc] = v[i];
}

// acc (4 x 4 per thread, rows tr + 16 i, columns tc + 16 j of a 64 x 64 tile)
// += X_tile * Y_tile for row-major 64 x 64 tiles at x and y (leading dims lx, ly).
__device__ __forceinline__ void tile_fma(double (*Xs)[NB + 1], double (*Ys)[NB + 1],
                                         const double* __restrict__ x, int64_t lx,
                                         const double* __restrict__ y, int64_t ly,
                                         double acc[4][4]) {
  const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    Xs[e / NB][e % NB] = x[(int64_t)(e / NB) * lx + e % NB];
    Ys[e / NB][e % NB] = y[(int64_t)(e / NB) * ly + e % NB];
  }
  __syncthreads();
  for (int kk = 0; kk < NB; ++kk) {
    double av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) av[i] = Xs[tr + 16 * i][kk];
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = Ys[kk][tc + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
  }
}

// One level of the doubling, block size bt tiles. Workgroup -> (pair p, output
// tile (Il, Jl)); the pair's A block is tiles [s, s + bt), its C block tiles
// [s + bt, min(s + 2 bt, NT)), s = 2 p bt. PHASE 0: T[Il][Jl] = sum_{K >= J}
// L[I][K] P[K][J] (A^-1 is lower triangular); PHASE 1: P[I][J] = -sum_{K <= I}
// P[I][K] T[K][Jl] over the C block.
template <int PHASE>
__global__ __launch_bounds__(256) void trinv_level_kernel(int N, const double* __restrict__ L,
                                                          double* __restrict__ P,
                                                          double* __restrict__ T, int bt) {
  __shared__ double Xs[NB][NB + 1];
  __shared__ double Ys[NB][NB + 1];
  const int NT = N / NB;
  const int per = bt * bt;
  const int p = blockIdx.x / per, rem = blockIdx.x - p * per;
  const int Il = rem / bt, Jl = rem - (rem / bt) * bt;
  const int s = 2 * p * bt, c0 = s + bt;
  const int I = c0 + Il, J = s + Jl;
  if (I >= NT) return;  // ragged last C block: whole workgroup, before any barrier
  double* Tp = T + (int64_t)p * per * NB * NB;
  double acc[4][4] = {};
  if (PHASE == 0) {
    for (int K = J; K < c0; ++K)
      tile_fma(Xs, Ys, L + (int64_t)I * NB * N + (int64_t)K * NB, N,
               P + (int64_t)K * NB * N + (int64_t)J * NB, N, acc);
  } else {
    for (int K = c0; K <= I; ++K)
      tile_fma(Xs, Ys, P + (int64_t)I * NB * N + (int64_t)K * NB, N,
               Tp + (int64_t)((K - c0) * bt + Jl) * NB * NB, NB, acc);
  }
  const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (PHASE == 0)
        Tp[(int64_t)(Il * bt + Jl) * NB * NB + (tr + 16 * i) * NB + tc + 16 * j] = acc[i][j];
      else
        P[((int64_t)I * NB + tr + 16 * i) * N + (int64_t)J * NB + tc + 16 * j] = -acc[i][j];
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

// ------------------------------------------- U = C(X, Z) P' fused (split-BF16) ----
// P = L_k^-1 rounded to FP32 and split into NS bfloat16 terms, plane p at
// Pb + p * total: two terms keep its leading 16 significant bits, three all 24.
// Each plane is stored in the order the U kernel reads it: tiles of 16 rows x
// 32 columns (row j, column l at offset j * 32 + l % 32 in the tile), the tile
// of rows 16 t .. 16 t + 15 and columns 32 s .. 32 s + 31 at index
// ((t / 2) * (kpad / 32) + s) * 2 + t % 2; one wave's fragment load of a step
// is then one contiguous kilobyte.
template <int NS>
__global__ __launch_bounds__(256) void split_p_kernel(int64_t total, int kpad,
                                                      const double* __restrict__ P,
                                                      __bf16* __restrict__ Pb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int row = (int)(e / kpad), col = (int)(e - (int64_t)row * kpad);
  const int t = row >> 4, sl = col >> 5;
  const int64_t o =
      ((((int64_t)(t >> 1) * (kpad >> 5) + sl) * 2 + (t & 1)) * 16 + (row & 15)) * 32 + (col & 31);
  float x = (float)P[e];
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    const __bf16 h = (__bf16)x;
    Pb[p * total + o] = h;
    x -= (float)h;  // exact: h holds the leading bits of x
  }
}

// One block per 32 rows of X: the rows' cross-covariances C(x_i, z_l) are
// evaluated into LDS as NS bfloat16 terms, then U_i,j = sum_{l <= j} C_i,l P_j,l
// for all j on MFMA, P (split the same way) streamed from L2. C never goes to
// HBM; U is written once.
constexpr int URB = 32;
constexpr int UPAD = 8;

// The ROWS rows' coordinates into LDS (one load per row, all in flight at once),
// so that the row loop of fill_c_planes reads no global memory. Ends with a
// barrier.
template <int ROWS>
__device__ __forceinline__ void stage_rows(const LowRankArgs& A, int64_t i0, double* sRow) {
  const int tid = threadIdx.x;
  if (tid < 3 * ROWS) {
    const int row = tid / 3, c = tid - 3 * (tid / 3);
    const int64_t i = i0 + row;
    const double* src = c == 0 ? A.sx : (c == 1 ? A.sy : A.t);
    sRow[tid] = i < A.n ? src[i] : 0.0;
  }
  __syncthreads();
}

// C(x_i, z_l) for the ROWS rows from i0 and the columns lbeg .. lbeg + ncol - 1
// (ncol a multiple of 8) into NS bfloat16 planes of LDS (plane stride pst, row
// stride ldc, column l at l - lbeg): the FP32 value split into NS terms, each
// the bfloat16 rounding of what the previous ones leave. Rows past n and
// columns past k hold zeros. One thread per 8 consecutive columns x 8 rows.
// sRow: the rows' (x, y, t), staged in LDS by stage_rows.
template <int NS, int ROWS>
__device__ __forceinline__ void fill_c_planes(const LowRankArgs& A, int64_t i0, const double* sRow,
                                              int lbeg, int ncol, __bf16* C0, int pst, int ldc) {
  const int tid = threadIdx.x;
  const int ncg = ncol / 8;  // column groups
  for (int task = tid; task < ncg * (ROWS / 8); task += (int)blockDim.x) {
    const int cg = task % ncg, rg = task / ncg;
    double zx[8], zy[8], zt[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int l = lbeg + cg * 8 + c;
      const bool ok = l < A.k;
      zx[c] = ok ? A.zx[l] : 0.0;
      zy[c] = ok ? A.zy[l] : 0.0;
      zt[c] = ok ? A.zt[l] : 0.0;
    }
    // Gneiting: the lag factors depend on (t_i, z_l) only, and consecutive
    // points mostly share their time, so they are reused across rows.
    const bool fac = A.K.kind == 1;
    float fa[8], fe[8];
    double tcache = NAN;
#pragma unroll 1
    for (int rr = 0; rr < 8; ++rr) {
      const int row = rg * 8 + rr;
      const int64_t i = i0 + row;
      bf8v pl[NS];
      if (i < A.n) {
        const double xi = sRow[3 * row], yi = sRow[3 * row + 1], ti = sRow[3 * row + 2];
        if (fac && !(ti == tcache)) {
          tcache = ti;
#pragma unroll
          for (int c = 0; c < 8; ++c) gneiting_lag<float>(A.K, (float)(ti - zt[c]), fa[c], fe[c]);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int l = lbeg + cg * 8 + c;
          float v = 0.f;
          if (l < A.k) {
            if (fac)
              v = gneiting_pair<float>(A.K, (float)(xi - zx[c]), (float)(yi - zy[c]), fa[c], fe[c]);
            else
              v = cov_eval<float>(A.K, (float)(xi - zx[c]), (float)(yi - zy[c]),
                                  (float)(ti - zt[c]));
          }
#pragma unroll
          for (int p = 0; p < NS; ++p) {
            const __bf16 h = (__bf16)v;
            pl[p][c] = h;
            v -= (float)h;
          }
        }
      } else {
#pragma unroll
        for (int p = 0; p < NS; ++p)
#pragma unroll
          for (int c = 0; c < 8; ++c) pl[p][c] = (__bf16)0.f;
      }
#pragma unroll
      for (int p = 0; p < NS; ++p)
        *reinterpret_cast<bf8v*>(C0 + p * pst + row * ldc + cg * 8) = pl[p];
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

// Split-BF16 Gram of W over 4096-row chunks, FP32 partial tiles of 128 x 128.
//
// W arrives as its bfloat16 terms (x = h + m [+ l]) in 8-row blocks, so that one
// 16-byte piece is one lane's MFMA operand (8 consecutive rows of one column; the
// K order inside a 32-row step is the same for both operands, which is all a
// Gram needs). Pieces are copied to LDS unchanged, loads one step ahead in
// registers; one 48 KB buffer, so that two workgroups share a CU. Products of the terms (3 for NS = 2, 6 for NS = 3), smallest
// first, accumulate in FP32 over the chunk; the partials are summed in FP64 by
// syrk_split_reduce_kernel. Blocks are dealt to the 8 XCDs round-robin; XCD x
// runs the tiles of chunks x, x + 8, ... one chunk after the other, so that the
// tiles sharing a chunk's rows run together and find them in that XCD's L2.
constexpr int TB = 128;    // output tile
constexpr int SBK = 32;    // rows per step (the bf16 MFMA K)

template <int NS>
__global__ __launch_bounds__(256, 2) void syrk_split_kernel(int64_t nrows, int kpad,
                                                         const __bf16* __restrict__ Wp,
                                                         float* __restrict__ part, int nchunk,
                                                         int ntile, int chunk_blocks) {
  constexpr int PPS = NS * (SBK / 8) * TB / 256;  // 16-byte pieces per thread and strip
  __shared__ bf8v sP[1][2][NS][SBK / 8][TB];
  const int x = blockIdx.x & 7;
  const int l = blockIdx.x >> 3;
  const int c = (l / ntile) * 8 + x;
  const int t = l - (l / ntile) * ntile;
  if (c >= nchunk) return;  // whole block, before any barrier
  int TI, TJ;
  tile_of(t, TI, TJ);
  const bool diag = TI == TJ;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  // On a diagonal tile the upper-right quarter is the transpose of the lower-left.
  const bool skip = diag && wr < wc;
  const int64_t wrb = nrows / 8;
  const int64_t bbeg = (int64_t)c * chunk_blocks;
  const int64_t bend = bbeg + chunk_blocks < wrb ? bbeg + chunk_blocks : wrb;
  bf8v ra[PPS], rb[PPS];
  // Unconditional loads (out-of-range pieces re-read a valid one and are zeroed
  // at the store), so that each store waits for its own loads only.
  auto load = [&](int64_t b0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < PPS; ++i) {
      const int pc = tid + 256 * i;
      const int col = pc & (TB - 1), gq = (pc / TB) & 3, sp = pc / (TB * 4);
      int64_t blk = b0 + gq;
      blk = blk < bend ? blk : bend - 1;
      const int ca = min(TI * TB + col, kpad - 1), cb = min(TJ * TB + col, kpad - 1);
      ra[i] = *reinterpret_cast<const bf8v*>(Wp + ((sp * wrb + blk) * kpad + ca) * 8);
      rb[i] = *reinterpret_cast<const bf8v*>(Wp + ((sp * wrb + blk) * kpad + cb) * 8);
    }
  };
  auto store = [&](int buf, int64_t b0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < PPS; ++i) {
      const int pc = tid + 256 * i;
      const int col = pc & (TB - 1), gq = (pc / TB) & 3, sp = pc / (TB * 4);
      const bool okr = b0 + gq < bend;
      sP[buf][0][sp][gq][col] = (okr && TI * TB + col < kpad) ? ra[i] : bf8v{};
      sP[buf][1][sp][gq][col] = (okr && TJ * TB + col < kpad) ? rb[i] : bf8v{};
    }
  };

  f4v acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
  const int g = lane >> 4, j = lane & 15;
  const int nsteps = bend > bbeg ? (int)((bend - bbeg + 3) / 4) : 0;
  if (nsteps > 0) {
    load(bbeg);
    store(0, bbeg);
  }
  __syncthreads();
  for (int st = 0; st < nsteps; ++st) {
    const int buf = 0;
    const bool more = st + 1 < nsteps;
    const int64_t bnext = bbeg + (int64_t)(st + 1) * 4;
    if (more) load(bnext);
    if (!skip) {
      bf8v av[4][NS], bv[4][NS];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) av[a][sp] = sP[buf][0][sp][g][wr * 64 + a * 16 + j];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) bv[b][sp] = sP[buf][1][sp][g][wc * 64 + b * 16 + j];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if constexpr (NS == 3) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][2], bv[b][0], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][1], bv[b][1], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][0], bv[b][2], acc[a][b], 0, 0, 0);
          } else if (diag) {
            // Diagonal tiles keep the low-by-low product: on the diagonal it
            // is a sum of squares, so dropping it would bias every column
            // norm of W low.
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][1], bv[b][1], acc[a][b], 0, 0, 0);
          }
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][1], bv[b][0], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][0], bv[b][1], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][0], bv[b][0], acc[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
    if (more) {
      store(0, bnext);
      __syncthreads();
    }
  }
  if (skip) return;
  float* out = part + ((int64_t)c * ntile + t) * (TB * TB);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wr * 64 + a * 16 + mfma16_row_f32acc(lane, e);
        const int col = wc * 64 + b * 16 + j;
        out[row * TB + col] = acc[a][b][e];
      }
}

// Two-term (BF16X3) Gram in 256 x 256 tiles: one workgroup of eight wavefronts
// per CU (each 64 x 128 of the tile, 4 x 8 MFMA tiles), so each staged 16-byte
// piece of W feeds twice the products of a 128 x 128 tile and the CU asks its L2
// for half the bytes per product; two 64 KB stage buffers. Same chunking, XCD
// mapping, piece layout and product order as syrk_split_kernel<2>; a diagonal
// tile stages one block and the two wavefronts whose part lies wholly above the
// diagonal stay idle.
constexpr int TB2 = 256;

__global__ __launch_bounds__(512, 1) void syrk_split256_kernel(int64_t nrows, int kpad,
                                                              const __bf16* __restrict__ Wp,
                                                              float* __restrict__ part, int nchunk,
                                                              int ntile, int chunk_blocks) {
  constexpr int NS = 2;
  constexpr int PPS = NS * (SBK / 8) * TB2 / 512;  // 16-byte pieces per thread and block
  __shared__ bf8v sP[2][2][NS][SBK / 8][TB2];  // [stage buffer][block][term][row group][column]
  const int x = blockIdx.x & 7;
  const int l = blockIdx.x >> 3;
  const int c = (l / ntile) * 8 + x;
  const int t = l - (l / ntile) * ntile;
  if (c >= nchunk) return;  // whole block, before any barrier
  int TI, TJ;
  tile_of(t, TI, TJ);
  const bool diag = TI == TJ;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // rows wr * 64 .. + 63, columns wc * 128 .. + 127
  const bool skip = diag && wc * 128 >= wr * 64 + 64;
  const int64_t wrb = nrows / 8;
  const int64_t bbeg = (int64_t)c * chunk_blocks;
  const int64_t bend = bbeg + chunk_blocks < wrb ? bbeg + chunk_blocks : wrb;
  bf8v ra[PPS], rb[PPS];
  auto load = [&](int64_t b0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < PPS; ++i) {
      const int pc = tid + 512 * i;
      const int col = pc & (TB2 - 1), gq = (pc / TB2) & 3, sp = pc / (TB2 * 4);
      int64_t blk = b0 + gq;
      blk = blk < bend ? blk : bend - 1;
      const int ca = min(TI * TB2 + col, kpad - 1), cb = min(TJ * TB2 + col, kpad - 1);
      ra[i] = *reinterpret_cast<const bf8v*>(Wp + ((sp * wrb + blk) * kpad + ca) * 8);
      if (!diag) rb[i] = *reinterpret_cast<const bf8v*>(Wp + ((sp * wrb + blk) * kpad + cb) * 8);
    }
  };
  auto store = [&](int buf, int64_t b0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < PPS; ++i) {
      const int pc = tid + 512 * i;
      const int col = pc & (TB2 - 1), gq = (pc / TB2) & 3, sp = pc / (TB2 * 4);
      const bool okr = b0 + gq < bend;
      sP[buf][0][sp][gq][col] = (okr && TI * TB2 + col < kpad) ? ra[i] : bf8v{};
      if (!diag) sP[buf][1][sp][gq][col] = (okr && TJ * TB2 + col < kpad) ? rb[i] : bf8v{};
    }
  };
  const int sb = diag ? 0 : 1;
  f4v acc[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
  const int g = lane >> 4, j = lane & 15;
  const int nsteps = bend > bbeg ? (int)((bend - bbeg + 3) / 4) : 0;
  if (nsteps > 0) {
    load(bbeg);
    store(0, bbeg);
  }
  __syncthreads();
  // Two stage buffers: step st computes from buffer st & 1 while the next step's
  // pieces go to the other one, so each step needs one barrier.
  for (int st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    const bool more = st + 1 < nsteps;
    const int64_t bnext = bbeg + (int64_t)(st + 1) * 4;
    if (more) load(bnext);
    if (!skip) {
      bf8v bv[8][NS];
#pragma unroll
      for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) bv[b][sp] = sP[buf][sb][sp][g][wc * 128 + b * 16 + j];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        bf8v av[NS];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) av[sp] = sP[buf][0][sp][g][wr * 64 + a * 16 + j];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          if (diag) {
            // the low-by-low product on the diagonal tiles (sums of squares there)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], bv[b][1], acc[a][b], 0, 0, 0);
          }
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], bv[b][0], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], bv[b][1], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], bv[b][0], acc[a][b], 0, 0, 0);
        }
      }
    }
    if (more) store(buf ^ 1, bnext);
    __syncthreads();
  }
  if (skip) return;
  float* out = part + ((int64_t)c * ntile + t) * (TB2 * TB2);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wr * 64 + a * 16 + mfma16_row_f32acc(lane, e);
        const int col = wc * 128 + b * 16 + j;
        out[row * TB2 + col] = acc[a][b][e];
      }
}

// M = I + sum over chunks (FP64, fixed order) of the lower tiles, q = row k, zz = (k, k).
// Entry (r, c) of the matrix whose Cholesky factor gives both terms of the
// Woodbury assembly: rows and columns 0 .. k-1 hold M = I + W'W, row k holds
// q' = (W'z)' and, on the diagonal, 2 z'z + 1, rows past k the identity. Its
// factor is [[L_M, 0], [v', d]] with v = L_M^-1 q, so q' M^-1 q = |v|^2 with no
// separate triangular solve; the last pivot 2 z'z + 1 - q' M^-1 q exceeds z'z
// + 1 (q' M^-1 q <= z'z), so the factorisation cannot fail there. s is the
// Gram entry of [W z].
__device__ __forceinline__ double augmented_entry(int r, int c, int k, double s) {
  if (r < k && c < k) return (r == c ? 1.0 : 0.0) + s;
  if (r == k && c < k) return s;
  if (c == k && r < k) return s;
  if (r == k && c == k) return 2.0 * s + 1.0;
  return r == c ? 1.0 : 0.0;
}

template <int TT>
__global__ __launch_bounds__(256) void syrk_split_reduce_kernel(int k, int kpad,
                                                                const float* __restrict__ part,
                                                                int nchunk, int ntile,
                                                                double* __restrict__ M,
                                                                double* __restrict__ q,
                                                                double* __restrict__ zz) {
  constexpr int PER = TT * TT / 256;  // blocks per tile
  const int t = blockIdx.x / PER;
  const int e = (blockIdx.x - t * PER) * 256 + threadIdx.x;
  int TI, TJ;
  tile_of(t, TI, TJ);
  const int er = e / TT, ec = e - (e / TT) * TT;
  // A diagonal tile's upper triangle (parts of it are not computed) is
  // written by the thread of the mirrored lower entry, so every thread reads its
  // own entry's partials, contiguous across the block.
  const bool diag = TI == TJ;
  if (diag && er < ec) return;
  const float* src = part + (int64_t)t * (TT * TT) + e;
  const int64_t stride = (int64_t)ntile * (TT * TT);
  double s = 0.0;
#pragma unroll 8
  for (int cc = 0; cc < nchunk; ++cc) s += (double)src[cc * stride];
  const int r = TI * TT + er, col = TJ * TT + ec;
  if (r < kpad && col < kpad) {
    M[(int64_t)r * kpad + col] = augmented_entry(r, col, k, s);
    if (diag && er > ec) M[(int64_t)col * kpad + r] = augmented_entry(col, r, k, s);
  }
  if (r == k && col < k) q[col] = s;
  if (r == k && col == k) *zz = s;
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
    M[(int64_t)r * kpad + c] = augmented_entry(r, c, k, s);
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

hipError_t launch_cholesky_set(int count, double* const* A, const int* N, double* const* scratch,
                               unsigned long long* const* fail, hipStream_t s) {
  int maxnt = 0;
  for (int i = 0; i < count; ++i) maxnt = N[i] / NB > maxnt ? N[i] / NB : maxnt;
  for (int jb = 0; jb < maxnt; ++jb) {
    for (int phase = 0; phase < 2; ++phase) {
      // the matrices still factoring at this step, kCholSet per launch
      CholSet S{};
      S.jb = jb;
      auto flush = [&]() {
        if (S.count == 0) return hipSuccess;
        if (phase == 0)
          hipLaunchKernelGGL(chol_panel_set_kernel, dim3((unsigned)S.pre[S.count]), dim3(256), 0, s, S);
        else
          hipLaunchKernelGGL(chol_update_set_kernel, dim3((unsigned)S.pre[S.count]), dim3(256), 0, s, S);
        const hipError_t e = hipGetLastError();
        S.count = 0;
        S.pre[0] = 0;
        return e;
      };
      S.pre[0] = 0;
      for (int i = 0; i < count; ++i) {
        const int NT = N[i] / NB;
        if (NT <= jb) continue;
        const int nt = NT - jb - 1;
        const int nblk = phase == 0 ? NT - jb : nt * (nt + 1) / 2 + 1;
        S.A[S.count] = A[i];
        S.N[S.count] = N[i];
        S.dscr[S.count] = scratch[i];
        S.fail[S.count] = fail[i];
        S.pre[S.count + 1] = S.pre[S.count] + nblk;
        ++S.count;
        if (S.count == kCholSet) {
          const hipError_t e = flush();
          if (e != hipSuccess) return e;
        }
      }
      const hipError_t e = flush();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

size_t trinv_scratch_bytes(int N) {
  const int NT = N / NB;
  size_t tiles = 0;
  for (int bt = 1; bt < NT; bt *= 2) {
    const size_t pairs = (size_t)(NT + 2 * bt - 1) / (2 * bt);
    tiles = tiles > pairs * bt * bt ? tiles : pairs * bt * bt;
  }
  return tiles * NB * NB * sizeof(double);
}

hipError_t launch_trinv(int N, const double* L, double* P, double* T, hipStream_t s) {
  const int NT = N / NB;
  hipLaunchKernelGGL(trinv_diag_kernel, dim3(NT), dim3(256), 0, s, N, L, P);
  for (int bt = 1; bt < NT; bt *= 2) {
    const unsigned pairs = (unsigned)((NT + 2 * bt - 1) / (2 * bt));
    const dim3 grid(pairs * bt * bt);
    hipLaunchKernelGGL(trinv_level_kernel<0>, grid, dim3(256), 0, s, N, L, P, T, bt);
    hipLaunchKernelGGL(trinv_level_kernel<1>, grid, dim3(256), 0, s, N, L, P, T, bt);
  }
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

// NS = 2 terms keep 16 significant bits of C and P (three products per step:
// lh, hl, hh); NS = 3 keep all 24 (FP32-accurate U; six products: lh, mm, hl,
// mh, hm, hh), smallest first. A wave takes 32 output columns at a time (two
// 16-column blocks sharing the k range, since P_j,l = 0 for l > j), so each A
// fragment read from LDS feeds 2 NS products. The columns l of C are taken in
// two halves (three planes of 32 rows do not fit in LDS for the full k).
// Output columns j < kpad / 2 need only the first half: they are finished and
// written in the first phase. The upper columns keep their accumulators in
// registers across the phases and are written after the second.
// RT row tiles of 16 (ROWS = 16 RT rows per workgroup); MAXHI upper 32-column
// blocks per wave (kpad <= 2 * NWV * 32 * MAXHI). More rows per workgroup feed
// each P fragment read from L2 to more products (the L2 reads of P per row
// halve from 32 to 64 rows).
template <int NS, int NWV, int RT, int MAXHI>
__global__ __launch_bounds__(64 * NWV) void lowrank_u_kernel(LowRankArgs A, const __bf16* __restrict__ Pb,
                                                        float* __restrict__ U) {
  constexpr int ROWS = 16 * RT;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int kpad = A.kpad;
  const int kh = kpad / 2;  // kpad is a multiple of 64, so kh is one of 32
  const int ldc = kh + UPAD;
  const int pst = ROWS * ldc;
  __bf16* C0 = reinterpret_cast<__bf16*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * ROWS;
  const int64_t kk = (int64_t)kpad * kpad;
  const int nlo = kpad / 64;  // 32-column blocks below kh; as many above
  const int g = lane >> 4, j = lane & 15;

  // acc[r][c] += C[r * 16 + .., k0 .. k0 + 31] P[pb * 32 + c * 16 + .., k0 .. k0 + 31]'
  // for k0 = kb, kb + 32, .. < ke; C columns of this phase start at lbeg. Two
  // register sets alternate (steps unrolled by two), so that the P fragments
  // of the next step load while this one computes with no copy between sets.
  auto contract = [&](int pb, int lbeg, int kb, int ke, f4v (*acc)[2]) __attribute__((always_inline)) {
    // P in 16 x 32 tiles (split_p_kernel<NS>): the fragment of column
    // block c at step k0 is the kilobyte at ((pb * kpad / 32 + k0 / 32) * 2 + c) * 512.
    const __bf16* p0 = Pb + (int64_t)pb * kpad * 32 + j * 32 + 8 * g;
    auto load = [&](bf8v (*b)[NS], int k0) __attribute__((always_inline)) {
      const __bf16* q = p0 + k0 * 32;
#pragma unroll
      for (int p = 0; p < NS; ++p) {
        b[0][p] = *reinterpret_cast<const bf8v*>(q + p * kk);
        b[1][p] = *reinterpret_cast<const bf8v*>(q + p * kk + 512);
      }
    };
    auto step = [&](bf8v (*b)[NS], int k0) __attribute__((always_inline)) {
      const int ko = k0 - lbeg + 8 * g;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const __bf16* cp = C0 + (r * 16 + j) * ldc + ko;
        bf8v a[NS];
#pragma unroll
        for (int p = 0; p < NS; ++p) a[p] = *reinterpret_cast<const bf8v*>(cp + p * pst);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          f4v x = acc[r][c];
          if constexpr (NS == 3) {
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[c][0], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[c][1], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[c][2], x, 0, 0, 0);
          }
          x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[c][0], x, 0, 0, 0);
          x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[c][1], x, 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[c][0], x, 0, 0, 0);
        }
      }
    };
    bf8v x[2][NS], y[2][NS];
    load(x, kb);
    int k0 = kb;
    for (; k0 + 32 < ke; k0 += 64) {
      load(y, k0 + 32);
      __builtin_amdgcn_sched_barrier(0);  // issued before the step that hides them
      step(x, k0);
      load(x, k0 + 64 < ke ? k0 + 64 : k0 + 32);  // past the end: re-read (unconditional)
      __builtin_amdgcn_sched_barrier(0);
      step(y, k0 + 32);
    }
    if (k0 < ke) step(x, k0);  // odd step count
  };
  auto store = [&](int pb, f4v (*acc)[2]) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int jcol = pb * 32 + c * 16 + j;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = mfma16_row_f32acc(lane, e);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const int64_t ia = i0 + rt * 16 + r;
          if (ia < A.n) U[ia * kpad + jcol] = acc[rt][c][e];
        }
      }
    }
  };

  // ---- first half of the columns of C ----
  __shared__ double sRow[3 * ROWS];
  stage_rows<ROWS>(A, i0, sRow);
  fill_c_planes<NS, ROWS>(A, i0, sRow, 0, kh, C0, pst, ldc);
  __syncthreads();
  for (int pass = 0; pass * NWV < nlo; ++pass) {  // lower blocks, snake order for balance
    const int pb = pass * NWV + ((pass & 1) ? NWV - 1 - wave : wave);
    if (pb >= nlo) continue;
    f4v acc[RT][2];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r][0] = acc[r][1] = f4v{0.f, 0.f, 0.f, 0.f};
    contract(pb, 0, 0, pb * 32 + 32, acc);
    store(pb, acc);
  }
  f4v hi[MAXHI][RT][2];
#pragma unroll
  for (int q = 0; q < MAXHI; ++q) {
#pragma unroll
    for (int r = 0; r < RT; ++r) hi[q][r][0] = hi[q][r][1] = f4v{0.f, 0.f, 0.f, 0.f};
    const int hb = q * NWV + ((q & 1) ? NWV - 1 - wave : wave);
    if (hb < nlo) contract(nlo + hb, 0, 0, kh, hi[q]);
  }
  __syncthreads();  // every read of the first half is done

  // ---- second half ----
  fill_c_planes<NS, ROWS>(A, i0, sRow, kh, kh, C0, pst, ldc);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXHI; ++q) {
    const int hb = q * NWV + ((q & 1) ? NWV - 1 - wave : wave);
    if (hb >= nlo) continue;
    const int pb = nlo + hb;
    contract(pb, kh, kh, pb * 32 + 32, hi[q]);
    store(pb, hi[q]);
  }
}

namespace {
// Rows per workgroup: 64 for two terms up to kpad = 1024 (eight wavefronts, one
// workgroup per CU, 133 KB of LDS at kpad = 1024), else 32.
int lowrank_rows(int kpad, int prec) { return (prec == 2 && kpad <= 2 * 8 * 32 * 2) ? 64 : URB; }
}  // namespace

size_t lowrank_fused_lds(int kpad, int prec) {
  return (size_t)(prec == 3 ? 3 : 2) * lowrank_rows(kpad, prec) * (kpad / 2 + UPAD) * sizeof(__bf16);
}

bool lowrank_fused_ok(int kpad, int prec) {
  if (kpad > 2 * 8 * 32 * 4) return false;  // the eight-wavefront launch
  return lowrank_fused_lds(kpad, prec) + 3 * lowrank_rows(kpad, prec) * sizeof(double) <= 160 * 1024;
}

hipError_t prepare_lowrank_fused() {
  // The dynamic-LDS limit is raised to the largest size once per device.
  static std::atomic<int> attr_dev[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev >= 0 && dev < 64 && attr_dev[dev].load(std::memory_order_acquire)) return hipSuccess;
  // beside the static row stage of each variant
  const int dyn32 = 160 * 1024 - 3 * 32 * (int)sizeof(double);
  const int dyn64 = 160 * 1024 - 3 * 64 * (int)sizeof(double);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)lowrank_u_kernel<2, 8, 2, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, dyn32);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)lowrank_u_kernel<3, 8, 2, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, dyn32);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)lowrank_u_kernel<2, 8, 4, 2>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, dyn64);
  if (e == hipSuccess && dev >= 0 && dev < 64) attr_dev[dev].store(1, std::memory_order_release);
  return e;
}

hipError_t launch_lowrank_fused(const LowRankArgs& a, const double* P, void* Pb, float* U, int prec,
                                hipStream_t s) {
  const int64_t kk = (int64_t)a.kpad * a.kpad;
  __bf16* Ph = reinterpret_cast<__bf16*>(Pb);
  hipError_t e = prepare_lowrank_fused();
  if (e != hipSuccess) return e;
  const dim3 gs((unsigned)((kk + 255) / 256));
  const size_t lds = lowrank_fused_lds(a.kpad, prec);
  const int rows = lowrank_rows(a.kpad, prec);
  const unsigned grid = (unsigned)((a.n + rows - 1) / rows);
  if (prec == 3) {
    hipLaunchKernelGGL(split_p_kernel<3>, gs, dim3(256), 0, s, kk, a.kpad, P, Ph);
    hipLaunchKernelGGL((lowrank_u_kernel<3, 8, 2, 4>), dim3(grid), dim3(512), lds, s, a, (const __bf16*)Ph, U);
  } else {
    hipLaunchKernelGGL(split_p_kernel<2>, gs, dim3(256), 0, s, kk, a.kpad, P, Ph);
    if (rows == 64)
      hipLaunchKernelGGL((lowrank_u_kernel<2, 8, 4, 2>), dim3(grid), dim3(512), lds, s, a, (const __bf16*)Ph, U);
    else
      hipLaunchKernelGGL((lowrank_u_kernel<2, 8, 2, 4>), dim3(grid), dim3(512), lds, s, a, (const __bf16*)Ph, U);
  }
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

namespace {
int syrk_ntile(int kpad, int tb) {
  const int nt = (kpad + tb - 1) / tb;
  return nt * (nt + 1) / 2;
}
}  // namespace

// Output tile of the split-BF16 Gram: 256 for two terms when the 256-wide tiles
// are at least half real columns, else 128.
int syrk_split_tb(int kpad, int prec) { return (prec == 2 && kpad >= 512) ? TB2 : TB; }

int syrk_chunks(int64_t n, int, int prec, int chunk_rows) {
  if (prec <= 1) return 8;
  const int64_t c = (n + chunk_rows - 1) / chunk_rows;
  return (int)(((c + 7) / 8) * 8);
}

size_t syrk_part_bytes(int64_t n, int kpad, int prec, int chunk_rows) {
  const size_t c = (size_t)syrk_chunks(n, kpad, prec, chunk_rows);
  if (prec <= 1) return sizeof(double) * c * syrk_ntile(kpad, NB) * NB * NB;
  const int tb = syrk_split_tb(kpad, prec);
  return sizeof(float) * c * syrk_ntile(kpad, tb) * tb * tb;
}

hipError_t launch_syrk(int64_t n, int kpad, const void* W, int prec, void* part, int nchunk,
                       hipStream_t s, int chunk_rows) {
  if (prec >= 2) {
    const int tb = syrk_split_tb(kpad, prec);
    const int ntile = syrk_ntile(kpad, tb);
    dim3 grid((unsigned)(ntile * nchunk));
    if (tb == TB2)
      hipLaunchKernelGGL(syrk_split256_kernel, grid, dim3(512), 0, s, n, kpad, (const __bf16*)W,
                         (float*)part, nchunk, ntile, chunk_rows / 8);
    else if (prec == 2)
      hipLaunchKernelGGL(syrk_split_kernel<2>, grid, dim3(256), 0, s, n, kpad,
                         (const __bf16*)W, (float*)part, nchunk, ntile, chunk_rows / 8);
    else
      hipLaunchKernelGGL(syrk_split_kernel<3>, grid, dim3(256), 0, s, n, kpad,
                         (const __bf16*)W, (float*)part, nchunk, ntile, chunk_rows / 8);
    return hipGetLastError();
  }
  const int ntile = syrk_ntile(kpad, NB);
  dim3 grid(ntile * nchunk);
  double* pd = (double*)part;
  if (prec == 0)
    hipLaunchKernelGGL(syrk_kernel<0>, grid, dim3(256), 0, s, n, kpad, W, pd, nchunk, ntile);
  else
    hipLaunchKernelGGL(syrk_kernel<1>, grid, dim3(256), 0, s, n, kpad, W, pd, nchunk, ntile);
  return hipGetLastError();
}

hipError_t launch_syrk_reduce(int k, int kpad, const void* part, int prec, int nchunk, double* M,
                              double* q, double* zz, hipStream_t s) {
  if (prec >= 2) {
    const int tb = syrk_split_tb(kpad, prec);
    const int ntile = syrk_ntile(kpad, tb);
    if (tb == TB2)
      hipLaunchKernelGGL(syrk_split_reduce_kernel<TB2>, dim3((unsigned)(ntile * (TB2 * TB2 / 256))),
                         dim3(256), 0, s, k, kpad, (const float*)part, nchunk, ntile, M, q, zz);
    else
      hipLaunchKernelGGL(syrk_split_reduce_kernel<TB>, dim3((unsigned)(ntile * (TB * TB / 256))),
                         dim3(256), 0, s, k, kpad, (const float*)part, nchunk, ntile, M, q, zz);
    return hipGetLastError();
  }
  const int ntile = syrk_ntile(kpad, NB);
  hipLaunchKernelGGL(syrk_reduce_kernel, dim3(ntile), dim3(256), 0, s, k, kpad,
                     (const double*)part, nchunk, ntile, M, q, zz);
  return hipGetLastError();
}

}  // namespace vif
