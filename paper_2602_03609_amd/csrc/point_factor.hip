// Per-point Vecchia factor (Sec. "Vecchia approximation") and VIF residual
// factor (Sec. "The Vecchia-inducing-point full-scale approximation").
//
// For point i with conditioning set S = N(i) u {i} (i last, q = |S| <= 64):
//   G   = C(S,S) + nugget I                       (plain Vecchia)
//   G   = C(S,S) + nugget I - U_S U_S'            (VIF residual, U_S gathered rows)
//   G   = L L' (Cholesky),  w = L^-1 y_S
//   D_i = L_pp^2,  z_i = w_p = (y_i - A_i y_N)/sqrt(D_i),  A_i' = L_N^-T l_p
//   W_i = (U_i - A_i U_N) / sqrt(D_i)             (VIF; row i of D^-1/2 B U)
//
// gfx950 layout: a segment of ROWS lanes (ROWS = 16, 32 or 64, >= q) owns one
// point; lane r holds row r of G in registers (fully unrolled). Covariance
// entries are spread evenly over the segment and exchanged through LDS; the
// Cholesky broadcasts each new column through a double-buffered LDS vector and
// pivots through cross-lane permutes. The VIF Gram U_S U_S' runs on MFMA with
// the whole wavefront per point (FP64 16x16x4 MFMA, FP32 16x16x4 MFMA, or
// split-BF16 16x16x32 MFMA with FP32 accumulation, 3 or 6 products).
#include <math.h>

#include "internal.hpp"

namespace vif {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

template <int PREC> struct PrecT;
template <> struct PrecT<0> { using T = double; using UT = double; };
template <> struct PrecT<1> { using T = float; using UT = float; };
template <> struct PrecT<2> { using T = float; using UT = float; };
template <> struct PrecT<3> { using T = float; using UT = float; };

// ---- Gram U_S U_S' on MFMA, whole wave, result (full symmetric) into G[ROWS*ROWS] ----
template <int ROWS>
__device__ void gram_mfma_f64(const double* __restrict__ U, int ldu, const int* sidx, double* G,
                              int lane) {
  constexpr int NT = ROWS / 16;
  constexpr int NTT = NT * (NT + 1) / 2;
  const int rr = lane & 15, kq = lane >> 4;
  d4v acc[NTT];
#pragma unroll
  for (int t = 0; t < NTT; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
  const double* rowp[NT];
#pragma unroll
  for (int ti = 0; ti < NT; ++ti) {
    int s = sidx[ti * 16 + rr];
    rowp[ti] = s >= 0 ? U + (int64_t)s * ldu + kq * 4 : nullptr;
  }
  for (int kb = 0; kb < ldu; kb += 16) {
    double v[NT][4];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) {
      if (rowp[ti]) {
        const double2* p2 = reinterpret_cast<const double2*>(rowp[ti] + kb);
        double2 x0 = p2[0], x1 = p2[1];
        v[ti][0] = x0.x; v[ti][1] = x0.y; v[ti][2] = x1.x; v[ti][3] = x1.y;
      } else {
        v[ti][0] = v[ti][1] = v[ti][2] = v[ti][3] = 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj <= ti; ++tj) {
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[ti][c], v[tj][c], acc[t], 0, 0, 0);
          ++t;
        }
    }
  }
  int t = 0;
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj <= ti; ++tj) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int row = ti * 16 + mfma16_row_f64(lane, e), col = tj * 16 + rr;
        G[row * ROWS + col] = acc[t][e];
        if (ti != tj) G[col * ROWS + row] = acc[t][e];
      }
      ++t;
    }
}

template <int ROWS>
__device__ void gram_mfma_f32(const float* __restrict__ U, int ldu, const int* sidx, float* G,
                              int lane) {
  constexpr int NT = ROWS / 16;
  constexpr int NTT = NT * (NT + 1) / 2;
  const int rr = lane & 15, kq = lane >> 4;
  f4v acc[NTT];
#pragma unroll
  for (int t = 0; t < NTT; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  const float* rowp[NT];
#pragma unroll
  for (int ti = 0; ti < NT; ++ti) {
    int s = sidx[ti * 16 + rr];
    rowp[ti] = s >= 0 ? U + (int64_t)s * ldu + kq * 4 : nullptr;
  }
  for (int kb = 0; kb < ldu; kb += 16) {
    float v[NT][4];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) {
      if (rowp[ti]) {
        float4 x = *reinterpret_cast<const float4*>(rowp[ti] + kb);
        v[ti][0] = x.x; v[ti][1] = x.y; v[ti][2] = x.z; v[ti][3] = x.w;
      } else {
        v[ti][0] = v[ti][1] = v[ti][2] = v[ti][3] = 0.f;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj <= ti; ++tj) {
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[ti][c], v[tj][c], acc[t], 0, 0, 0);
          ++t;
        }
    }
  }
  int t = 0;
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj <= ti; ++tj) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int row = ti * 16 + mfma16_row_f32acc(lane, e), col = tj * 16 + rr;
        G[row * ROWS + col] = acc[t][e];
        if (ti != tj) G[col * ROWS + row] = acc[t][e];
      }
      ++t;
    }
}

// Split-BF16 products with FP32 accumulation. NPROD = 3: x = h + l (two bf16
// terms), products h*h + h*l + l*h (about 16 significant bits). NPROD = 6:
// x = h + m + l (three terms), products down to the 2^-24 level:
// h*h + (h*m + m*h) + (h*l + m*m + l*h), smallest issued first.
template <int ROWS, int NPROD>
__device__ void gram_mfma_bf16(const float* __restrict__ U, int ldu, const int* sidx, float* G,
                               int lane) {
  constexpr int NT = ROWS / 16;
  constexpr int NTT = NT * (NT + 1) / 2;
  constexpr int NS = NPROD == 3 ? 2 : 3;
  const int rr = lane & 15, kq = lane >> 4;
  f4v acc[NTT];
#pragma unroll
  for (int t = 0; t < NTT; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  const float* rowp[NT];
#pragma unroll
  for (int ti = 0; ti < NT; ++ti) {
    int s = sidx[ti * 16 + rr];
    rowp[ti] = s >= 0 ? U + (int64_t)s * ldu + kq * 8 : nullptr;
  }
  for (int kb = 0; kb < ldu; kb += 32) {
    bf8v part[NT][NS];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) {
      float x[8];
      if (rowp[ti]) {
        const float4* p4 = reinterpret_cast<const float4*>(rowp[ti] + kb);
        float4 a0 = p4[0], a1 = p4[1];
        x[0] = a0.x; x[1] = a0.y; x[2] = a0.z; x[3] = a0.w;
        x[4] = a1.x; x[5] = a1.y; x[6] = a1.z; x[7] = a1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = 0.f;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float r = x[e];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
          const __bf16 h = (__bf16)r;
          part[ti][sp][e] = h;
          r -= (float)h;
        }
      }
    }
    int t = 0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int tj = 0; tj <= ti; ++tj) {
        if constexpr (NPROD == 6) {
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][2], part[tj][0], acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][1], part[tj][1], acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][2], acc[t], 0, 0, 0);
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][1], part[tj][0], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][1], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][0], acc[t], 0, 0, 0);
        ++t;
      }
  }
  int t = 0;
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj <= ti; ++tj) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int row = ti * 16 + mfma16_row_f32acc(lane, e), col = tj * 16 + rr;
        G[row * ROWS + col] = acc[t][e];
        if (ti != tj) G[col * ROWS + row] = acc[t][e];
      }
      ++t;
    }
}

// Cholesky of the segment's ROWS x ROWS matrix, lane r holding row r in a[] (only
// a[j], j <= r, meaningful), with the forward solve of y carried along.
// On return a[j] = L[r][j] (j <= r), diag = L[r][r] and yv = (L^-1 y)[r]. Returns false on a
// nonpositive or non-finite pivot.
template <int ROWS, typename T>
__device__ __forceinline__ bool seg_cholesky(T (&a)[ROWS], T& yv, T& diag, const int r,
                                             const int sb, T* col2) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    T* col = col2 + (k & 1) * 2 * (ROWS + 1);
    const T piv0 = __shfl(a[k], sb + k);
    // A failed pivot is replaced by 1 so that the rest of the segment stays finite.
    const bool good = (piv0 > T(0)) && (piv0 < T(INFINITY));
    ok = ok && good;
    const T piv = good ? piv0 : T(1);
    const T rs = T(1) / dsqrt(piv);
    // Branch-free step: every lane stores its column entry and its scaled y value;
    // lane k's pair is the new diagonal and w_k = (L^-1 y)_k.
    const T lk = (r == k) ? piv * rs : a[k] * rs;
    diag = (r == k) ? lk : diag;
    a[k] = lk;
    col[r] = lk;
    col[ROWS + 1 + r] = yv * rs;
    wave_lds_sync();
    const T wk = col[ROWS + 1 + k];
    yv = (r == k) ? wk : ((r > k) ? yv - lk * wk : yv);
#pragma unroll
    for (int j = k + 1; j < ROWS; ++j) a[j] -= lk * col[j];
    // Keep the steps apart: overlapping them only raises register pressure.
    __builtin_amdgcn_sched_barrier(0);
  }
  return ok;
}

// Wavefronts per block: keeps the per-block LDS (one ROWS x ROWS matrix per
// point) at 32 KB in FP64.
template <int ROWS> constexpr int wpb() { return ROWS == 16 ? 4 : (ROWS == 32 ? 2 : 1); }

template <int ROWS, bool VIF, bool WANT_B, int PREC>
__global__ __launch_bounds__(64 * wpb<ROWS>()) void point_factor_kernel(FactorArgs A) {
  constexpr int kWPB = wpb<ROWS>();
  using T = typename PrecT<PREC>::T;
  using UT = typename PrecT<PREC>::UT;
  constexpr int PPW = 64 / ROWS;
  __shared__ T sM[kWPB][PPW][ROWS * ROWS];
  __shared__ T sCol[kWPB][PPW][4 * (ROWS + 1)];
  __shared__ double sX[kWPB][PPW][ROWS], sY[kWPB][PPW][ROWS], sT[kWPB][PPW][ROWS];
  __shared__ int sIdx[kWPB][PPW][ROWS];
  __shared__ T sB[kWPB][PPW][ROWS];

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int seg = lane / ROWS;
  const int r = lane % ROWS;
  const int sb = seg * ROWS;
  const int64_t i = ((int64_t)blockIdx.x * kWPB + wave) * PPW + seg;
  const bool active = i < A.n;
  const int m = A.m;

  int idx = -1;
  if (active && r < m) idx = A.nbr[i * m + r];
  // Valid neighbors are earlier points; they must form a prefix of the row.
  const bool valid = active && r < m && idx >= 0 && (int64_t)idx < i;
  const unsigned long long vb = __ballot(valid);
  const unsigned long long mmask = (1ull << m) - 1ull;
  const unsigned long long bits = (vb >> sb) & mmask;
  const int p = (int)__builtin_ctzll(~bits);
  const unsigned long long badb = __ballot(active && r < m && idx != -1 && !valid);
  if (active && r == 0 && m > 0) {
    const bool bad_entry = ((badb >> sb) & mmask) != 0ull;
    if (bad_entry || (bits >> p) != 0ull) flag_fail(A.bad_nbr, i);
  }
  const int q = p + 1;
  const int64_t srow = !active ? -1 : (r < p ? (int64_t)idx : (r == p ? i : -1));

  double xr = 0.0, yr = 0.0, tr = 0.0;
  T yv = T(0);
  if (srow >= 0) {
    xr = A.sx[srow];
    yr = A.sy[srow];
    tr = A.t[srow];
    if (A.y) yv = (T)A.y[srow];
  }
  sX[wave][seg][r] = xr;
  sY[wave][seg][r] = yr;
  sT[wave][seg][r] = tr;
  sIdx[wave][seg][r] = (int)srow;
  wave_lds_sync();

  T* M = sM[wave][seg];
  if constexpr (VIF) {
    // Gram of the gathered U rows, one point at a time with the whole wave.
#pragma unroll
    for (int s2 = 0; s2 < PPW; ++s2) {
      if (PREC == 0)
        gram_mfma_f64<ROWS>(reinterpret_cast<const double*>(A.U), A.ldu, sIdx[wave][s2],
                            reinterpret_cast<double*>(sM[wave][s2]), lane);
      else if (PREC == 1)
        gram_mfma_f32<ROWS>(reinterpret_cast<const float*>(A.U), A.ldu, sIdx[wave][s2],
                            reinterpret_cast<float*>(sM[wave][s2]), lane);
      else
        gram_mfma_bf16<ROWS, PREC == 3 ? 6 : 3>(reinterpret_cast<const float*>(A.U), A.ldu,
                                                 sIdx[wave][s2],
                                                 reinterpret_cast<float*>(sM[wave][s2]), lane);
    }
    wave_lds_sync();
  }

  // Strictly lower entries, balanced: lanes r and r + ROWS/2 share the row pair
  // (r', ROWS-1-r'), whose ROWS-1 entries they split by parity.
  {
    const int h = (r >= ROWS / 2) ? 1 : 0;
    const int rp = r - h * (ROWS / 2);
    const int R = ROWS - 1 - rp;
#pragma unroll 1
    for (int tt = 0; tt < ROWS / 2; ++tt) {
      const int e = h + 2 * tt;
      if (e < ROWS - 1) {
        const int row = (e < rp) ? rp : R;
        const int col = (e < rp) ? e : e - rp;
        T val = T(0);
        if (row < q) {
          const double dx = sX[wave][seg][row] - sX[wave][seg][col];
          const double dy = sY[wave][seg][row] - sY[wave][seg][col];
          const double dt = sT[wave][seg][row] - sT[wave][seg][col];
          val = cov_eval<T>(A.K, (T)dx, (T)dy, (T)dt);
          if constexpr (VIF) val -= M[row * ROWS + col];
        }
        M[row * ROWS + col] = val;
        M[col * ROWS + row] = val;
      }
    }
    T dg = T(1);
    if (r < q) {
      dg = T(A.K.sigma2 + A.K.nugget);
      if constexpr (VIF) dg -= M[r * ROWS + r];
    }
    M[r * ROWS + r] = dg;
  }
  wave_lds_sync();

  T a[ROWS];
#pragma unroll
  for (int j = 0; j < ROWS; ++j) a[j] = M[j * ROWS + r];

  T Ldiag = T(1);
  const bool ok = seg_cholesky<ROWS, T>(a, yv, Ldiag, r, sb, sCol[wave][seg]);
  if (active && r == 0 && !ok) flag_fail(A.fail, i);

  // Lane p now holds L_pp = sqrt(D_i) and z_i.
  const T Lpp_b = __shfl(Ldiag, sb + p);
  const T zi = __shfl(yv, sb + p);

  constexpr bool NEED_A = WANT_B || VIF;
  T x = T(0);
  if constexpr (NEED_A) {
    // L into LDS (row r from lane r), then back-solve L_N' x = l_p.
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < ROWS; ++j) M[r * ROWS + j] = (j <= r) ? a[j] : T(0);
    wave_lds_sync();
    T acc = (r < p) ? M[p * ROWS + r] : T(0);
    const T inv_diag = T(1) / Ldiag;
#pragma unroll
    for (int rr = ROWS - 1; rr >= 0; --rr) {
      const T xr_local = acc * inv_diag;
      const T xb = __shfl(xr_local, sb + rr);
      if (r == rr) x = xb;
      if (r < rr) acc -= M[rr * ROWS + r] * xb;
    }
    if (r >= p) x = T(0);
  }

  if constexpr (WANT_B) {
    if (active) {
      if (r < m) A.B[i * m + r] = (r < p) ? -(double)x : 0.0;
      if (r == 0) A.D[i] = (double)Lpp_b * (double)Lpp_b;
    }
  } else {
    if (active && r == 0) {
      A.logD[i] = 2.0 * log((double)Lpp_b);
      // VIF stores z_i in column k of W instead (it feeds q = W'z).
      if constexpr (!VIF) A.z[i] = (double)zi;
    }
  }

  if constexpr (VIF && !WANT_B) {
    // b_r = -x_r / L_pp (r < p), b_p = 1 / L_pp;  W_i = sum_r b_r U_{S_r}.
    const T inv = T(1) / Lpp_b;
    sB[wave][seg][r] = (r < p) ? -x * inv : (r == p ? inv : T(0));
    wave_lds_sync();
    const UT* U = reinterpret_cast<const UT*>(A.U);
    UT* W = reinterpret_cast<UT*>(A.W);
#pragma unroll
    for (int s2 = 0; s2 < PPW; ++s2) {
      const int64_t ip = ((int64_t)blockIdx.x * kWPB + wave) * PPW + s2;
      if (ip >= A.n) break;
      const int* S = sIdx[wave][s2];
      const T* bb = sB[wave][s2];
      const T zs = __shfl(zi, s2 * ROWS);
      for (int c = lane; c < A.ldu; c += 64) {
        T accw = T(0);
#pragma unroll 4
        for (int rr = 0; rr < ROWS; ++rr) {
          const int srr = S[rr];
          if (srr < 0) break;
          accw += bb[rr] * (T)U[(int64_t)srr * A.ldu + c];
        }
        W[ip * A.ldu + c] = (c == A.k) ? (UT)zs : (UT)accw;
      }
    }
  }
}

template <int ROWS, int PREC>
hipError_t launch_rows(const FactorArgs& a, int mode, bool vif, hipStream_t s) {
  constexpr int PPW = 64 / ROWS;
  constexpr int kWPB = wpb<ROWS>();
  const int64_t per_block = (int64_t)kWPB * PPW;
  const unsigned grid = (unsigned)((a.n + per_block - 1) / per_block);
  if (vif) {
    if (mode == 1)
      hipLaunchKernelGGL((point_factor_kernel<ROWS, true, true, PREC>), dim3(grid),
                         dim3(64 * kWPB), 0, s, a);
    else
      hipLaunchKernelGGL((point_factor_kernel<ROWS, true, false, PREC>), dim3(grid),
                         dim3(64 * kWPB), 0, s, a);
  } else {
    if (mode == 1)
      hipLaunchKernelGGL((point_factor_kernel<ROWS, false, true, PREC>), dim3(grid),
                         dim3(64 * kWPB), 0, s, a);
    else
      hipLaunchKernelGGL((point_factor_kernel<ROWS, false, false, PREC>), dim3(grid),
                         dim3(64 * kWPB), 0, s, a);
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_prec(const FactorArgs& a, int mode, hipStream_t s) {
  const bool vif = a.k > 0;
  const int q = a.m + 1;
  if (q <= 16) return launch_rows<16, PREC>(a, mode, vif, s);
  if (q <= 32) return launch_rows<32, PREC>(a, mode, vif, s);
  return launch_rows<64, PREC>(a, mode, vif, s);
}

}  // namespace

hipError_t launch_point_factor(const FactorArgs& a, int mode, int prec, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (prec == 0) return launch_prec<0>(a, mode, s);
  if (prec == 1) return launch_prec<1>(a, mode, s);
  if (prec == 2) return launch_prec<2>(a, mode, s);
  return launch_prec<3>(a, mode, s);
}

}  // namespace vif
