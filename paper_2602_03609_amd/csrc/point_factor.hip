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
// pivots through cross-lane permutes. Plain Vecchia uses point_factor_kernel;
// VIF uses vif_group_kernel, which shares the conditioning rows of a group of
// spatially adjacent points through LDS and forms the Grams U_S U_S' on MFMA
// (FP64 16x16x4, FP32 16x16x4, or split-BF16 16x16x32 with FP32 accumulation).
#include <limits.h>
#include <math.h>

#include <type_traits>

#include "internal.hpp"

namespace vif {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));

// One bfloat16 term of four values: returns bf16(rem) and leaves rem - that term
// in rem (the term's float values taken from its bits, so that the packed
// conversion is not repeated per value).
__device__ __forceinline__ bf4v bf16_term(f4v& rem) {
  bf4v hv;
#pragma unroll
  for (int c = 0; c < 4; ++c) hv[c] = (__bf16)rem[c];
  const uint2 u = __builtin_bit_cast(uint2, hv);
  rem[0] -= __uint_as_float(u.x << 16);
  rem[1] -= __uint_as_float(u.x & 0xffff0000u);
  rem[2] -= __uint_as_float(u.y << 16);
  rem[3] -= __uint_as_float(u.y & 0xffff0000u);
  return hv;
}

// LDS byte address of a pointer into a __shared__ array.
__device__ __forceinline__ unsigned lds_addr(const void* p) {
  return (unsigned)(size_t)(const __attribute__((address_space(3))) void*)p;
}
// LDS reads and writes for the direct-load staging loops, written out so that the
// compiler does not order them behind the direct loads in flight (which fill the
// other buffer); each block waits for its own LDS operations before it ends.
__device__ __forceinline__ void lds_read4(f4v& a, f4v& b, f4v& c, f4v& d, unsigned oa, unsigned ob,
                                          unsigned oc, unsigned od) {
  asm volatile(
      "ds_read_b128 %0, %4\n\tds_read_b128 %1, %5\n\tds_read_b128 %2, %6\n\tds_read_b128 %3, %7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(d)
      : "v"(oa), "v"(ob), "v"(oc), "v"(od)
      : "memory");
}
__device__ __forceinline__ void lds_write16(unsigned o, f4v v) {
  asm volatile("ds_write_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : : "v"(o), "v"(v) : "memory");
}

// v from the lane whose index differs in bit 0 (CTRL 0xB1) or bit 1 (CTRL 0x4E) of
// the quad, as a DPP move (no LDS traffic).
template <int CTRL>
__device__ __forceinline__ float quad_xor(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_xor(double v) {
  const int2 h = __builtin_bit_cast(int2, v);
  int2 o;
  o.x = __builtin_amdgcn_update_dpp(0, h.x, CTRL, 0xF, 0xF, false);
  o.y = __builtin_amdgcn_update_dpp(0, h.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, o);
}

template <int PREC> struct PrecT;
template <> struct PrecT<0> { using T = double; using UT = double; };
template <> struct PrecT<1> { using T = float; using UT = float; };
template <> struct PrecT<2> { using T = float; using UT = float; };
template <> struct PrecT<3> { using T = float; using UT = float; };

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

// Gauss-Jordan sweep over the first p columns of the segment's SPD matrix G
// (lane r holding row r in a[]; the point's own row p last, q = p + 1), with y
// carried as one more column. Step k eliminates column k from every other row
// (not only the rows below), so the regression coefficients come out with no
// back-substitution: afterwards lane r < p holds x_r = (G_NN^-1 G_Ni)_r in xo,
// and lane p holds d = G_ii - G_iN G_NN^-1 G_Ni (D_i) in xo and
// y_i - G_iN G_NN^-1 y_N in yv. The trailing block stays the symmetric Schur
// complement of a Cholesky step, so row k's entries past k are column k's, and
// each step is one LDS round trip: every lane writes its column-k entry (and
// its y), then reads the pivot row. Rows past q are the identity. Returns false
// on a nonpositive or non-finite pivot (p pivots and d).
template <int ROWS, typename T>
__device__ __forceinline__ bool seg_gauss_jordan(T (&a)[ROWS], T& yv, T& xo, const int r,
                                                 const int p, const int kmax, T* col2) {
  bool ok = true;
  T pivr = T(1);
#pragma unroll
  for (int k = 0; k < ROWS - 1; ++k) {
    if (k < kmax) {  // wave-uniform: the larger p of the wave's segments
      // column k and y, in 16-byte aligned halves (col2 holds 4 (ROWS + 4) values)
      T* col = col2 + (k & 1) * 2 * (ROWS + 4);
      col[r] = a[k];
      col[ROWS + 4 + r] = yv;
      wave_lds_sync();
      const bool act = k < p;
      const T piv0 = col[k];
      const bool good = !act || ((piv0 > T(0)) && (piv0 < T(INFINITY)));
      ok = ok && good;
      const T piv = (act && good) ? piv0 : T(1);
      // the hardware reciprocal and one Newton step instead of a division
      T inv = __builtin_amdgcn_rcpf(piv);
      inv = inv * (T(2) - piv * inv);
      const T f = (act && r != k) ? a[k] * inv : T(0);
      if (r == k) pivr = piv;
      yv -= f * col[ROWS + 4 + k];
#pragma unroll
      for (int j = k + 1; j < ROWS; ++j) a[j] -= f * col[j];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  T ap = T(0);
#pragma unroll
  for (int j = 0; j < ROWS; ++j) ap = (j == p) ? a[j] : ap;
  if (r == p) {
    ok = ok && (ap > T(0)) && (ap < T(INFINITY));
    xo = ap;
  } else {
    xo = (r < p) ? ap / pivr : T(0);
  }
  return ok;
}

// Wavefronts per block: keeps the per-block LDS (one ROWS x ROWS matrix per
// point) at 32 KB in FP64.
template <int ROWS> constexpr int wpb() { return ROWS == 16 ? 4 : (ROWS == 32 ? 2 : 1); }

// Plain Vecchia per-point factor (no low-rank part).
template <int ROWS, bool WANT_B, int PREC>
__global__ __launch_bounds__(64 * wpb<ROWS>()) void point_factor_kernel(FactorArgs A) {
  constexpr bool VIF = false;
  constexpr int kWPB = wpb<ROWS>();
  using T = typename PrecT<PREC>::T;
  using UT = typename PrecT<PREC>::UT;
  constexpr int PPW = 64 / ROWS;
  __shared__ T sM[kWPB][PPW][ROWS * ROWS];
  __shared__ T sCol[kWPB][PPW][4 * (ROWS + 1)];
  __shared__ double sX[kWPB][PPW][ROWS], sY[kWPB][PPW][ROWS], sT[kWPB][PPW][ROWS];
  __shared__ int sIdx[kWPB][PPW][ROWS];

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int seg = lane / ROWS;
  const int r = lane % ROWS;
  const int sb = seg * ROWS;
  // Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD walks a
  // contiguous range of the processing order (its L2 then holds the U rows
  // that spatially adjacent points share).
  const int64_t nblk = (A.n + (int64_t)kWPB * PPW - 1) / ((int64_t)kWPB * PPW);
  const int64_t per = (nblk + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (lb >= nblk) return;  // whole block
  const int64_t pos = (lb * kWPB + wave) * PPW + seg;
  const bool active = pos < A.n;
  const int64_t i = active ? (A.ord ? (int64_t)A.ord[pos] : pos) : A.n;
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

}

// ---------------------------------------------------------------------------
// VIF per-point factor, grouped. A workgroup takes GP consecutive points of the
// processing order (spatially adjacent points of one time slab). Their
// conditioning rows are merged into one sorted union (bitonic sort in LDS, then
// deduplicated); the union's rows of U are streamed through LDS in 128-byte
// column chunks, each chunk feeding the MFMA Grams of all GP points and, in a
// second pass, their W rows. Every U row is thus fetched once per group
// instead of once per point that uses it.
template <int ROWS, int PREC>
struct GroupShape {
  using T = typename PrecT<PREC>::T;
  static constexpr int PPW = 64 / ROWS;
  static constexpr int NW0 = (int)(65536 / (PPW * ROWS * ROWS * sizeof(T)));
  static constexpr int NW1 = NW0 > 8 ? 8 : NW0;
  // At most 16 points: the W product runs the group as the 16 rows of an MFMA tile.
  // At 32 rows per point, 8 points (4 wavefronts) per workgroup keep the LDS under
  // 80 KB, so two workgroups share a CU and one's Gram or W pass overlaps the
  // other's per-point phase (measured faster than 16 points in one workgroup,
  // despite the larger unions).
  static constexpr int NW = ROWS == 32 ? 4 : (NW1 * PPW > 16 ? 16 / PPW : NW1);  // wavefronts per workgroup
  static constexpr int GP = NW * PPW;            // points per workgroup
  static constexpr int NSLOT = GP * ROWS;        // conditioning rows (union upper bound)
};

// DMA (BF16X3 NLL, 32 rows): both passes stage the union's FP32 rows with direct
// global-to-LDS loads into two alternating buffers (chunks of 64 columns, 32 for
// unions of more than 64 rows), the loads of the next chunk in flight while the
// current one is used; the Gram pass splits its fragments into bfloat16 terms as
// it reads them.
template <int ROWS, bool WANT_B, int PREC, bool DMA = false>
__global__ __launch_bounds__((64 * GroupShape<ROWS, PREC>::NW), (DMA ? 3 : (ROWS == 32 ? 2 : 1))) void vif_group_kernel(FactorArgs A) {
  static_assert(!DMA || (ROWS == 32 && PREC >= 1 && !WANT_B),
                "direct-load staging: FP32 and split-BF16 NLL, 32 rows");
  using Sh = GroupShape<ROWS, PREC>;
  using T = typename PrecT<PREC>::T;
  using UT = typename PrecT<PREC>::UT;
  constexpr int PPW = Sh::PPW, NW = Sh::NW, GP = Sh::GP, NSLOT = Sh::NSLOT;
  constexpr int NTH = 64 * NW;
  constexpr int KC = 128 / (int)sizeof(UT);   // columns per staged chunk
  constexpr int VPE = 16 / (int)sizeof(UT);   // elements per 16-byte piece
  constexpr int SLD = KC + VPE;               // LDS row stride (elements), 16-byte aligned
  constexpr int NT = ROWS / 16;
  constexpr int NTT = NT * (NT + 1) / 2;
  // Shared area: union-row staging (Gram and W passes), the per-point matrices, and
  // in the W pass the 16 x union selection matrix beside the staged rows.
  constexpr size_t STAGE_B = (size_t)NSLOT * SLD * sizeof(UT);
  constexpr size_t MAT_B = (size_t)GP * ROWS * ROWS * sizeof(T);
  constexpr size_t SEL_B = (size_t)16 * (NSLOT + 8) * sizeof(UT);
  // Split-BF16 modes stage the Gram pass as NSP bfloat16 terms per value.
  constexpr bool SPLIT = PREC >= 2;
  constexpr int NSP = PREC == 3 ? 3 : 2;
  constexpr int BPAD = 8;  // bf16 row padding (16 bytes)
  constexpr int ZROW = 4 * KC;
  constexpr size_t SPL_B = SPLIT ? ((size_t)NSLOT * NSP * (KC + BPAD) + ZROW) * 2 : 0;
  constexpr size_t B1 = STAGE_B + SEL_B > MAT_B ? STAGE_B + SEL_B : MAT_B;
  // Direct-load staging: a 32 KB area (the union bitmap, then the chunk buffers, the
  // per-point matrices between the passes) holding two 16 KB buffers, or one of
  // 32 KB for the largest unions, then a zero segment read for empty slots; two W
  // result tiles (GP rows of 64 + 4 floats). About 52 KB in all: three workgroups
  // share a CU.
  constexpr int PBUF0 = 32 * 1024, PBUF1 = 16 * 1024;
  constexpr int PTILE = GP * (64 + 4) * 4;
  static_assert(!DMA || (size_t)PBUF0 >= MAT_B, "direct-load layout");
  constexpr size_t BIG_B = DMA ? (size_t)PBUF0 + 256 : (SPL_B > B1 ? SPL_B : B1);
  __shared__ __attribute__((aligned(16))) unsigned char sBig[DMA ? 16 : BIG_B];
  __shared__ __attribute__((aligned(16))) unsigned char sB0[DMA ? BIG_B : 16];
  __shared__ __attribute__((aligned(16))) unsigned char sTile[DMA ? 2 * PTILE : 16];
  __shared__ int sIdx[GP][ROWS];
  __shared__ int sSlot[GP][ROWS];
  __shared__ int sSort[NSLOT];
  __shared__ int sUniq[NSLOT];
  __shared__ int sNU;
  __shared__ int sLoHi[2];
  __shared__ double sX[GP][ROWS], sY[GP][ROWS], sT[GP][ROWS];
  __shared__ __attribute__((aligned(16))) T sCol[GP][4 * (ROWS + 4)];
  __shared__ T sBv[GP][ROWS];
  __shared__ T sZ[GP];
  __shared__ int64_t sI[GP];
  unsigned char* const sArea = DMA ? sB0 : sBig;  // the shared area (BIG_B bytes)
  UT* stage = reinterpret_cast<UT*>(sArea);
  T* sM = reinterpret_cast<T*>(sArea);

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int seg = lane / ROWS;
  const int r = lane % ROWS;
  const int sb = seg * ROWS;
  const int pl = wave * PPW + seg;  // point slot in the group
  // Workgroups are dealt round-robin to the 8 XCDs; each XCD walks a
  // contiguous range of groups so that its L2 holds the rows they share.
  // In the split-BF16 NLL modes the groups also cover the zero padding rows of
  // the W planes; those groups only write zeros.
  const int64_t ngrp = (SPLIT && !WANT_B) ? A.wrb * 8 / GP : (A.n + GP - 1) / GP;
  const int64_t per = (ngrp + 7) / 8;
  const int64_t g = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (g >= ngrp) return;  // whole block, before any barrier
  if constexpr (SPLIT && !WANT_B) {
    if (g * GP >= A.n) {
      __bf16* Wp = reinterpret_cast<__bf16*>(A.W);
      const bf4v zero = bf4v{};
      for (int e = tid; e < NSP * A.ldu * (GP / 4); e += NTH) {
        const int quad = e % (GP / 4), rest = e / (GP / 4);
        const int col = rest % A.ldu, sp = rest / A.ldu;
        const int64_t row0 = g * GP + 4 * quad;
        *reinterpret_cast<bf4v*>(Wp + ((sp * A.wrb + (row0 >> 3)) * A.ldu + col) * 8 +
                                 (row0 & 7)) = zero;
      }
      return;
    }
  }
  const int64_t pos = g * GP + pl;
  const bool active = pos < A.n;
  const int64_t i = active ? (A.ord ? (int64_t)A.ord[pos] : pos) : A.n;
  const int m = A.m;
  const UT* U = reinterpret_cast<const UT*>(A.U);

  // ---- conditioning rows and neighbor-row validation (per segment) ----
  int idx = -1;
  if (active && r < m) idx = A.nbr[i * m + r];
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
  sX[pl][r] = xr;
  sY[pl][r] = yr;
  sT[pl][r] = tr;
  sIdx[pl][r] = (int)srow;
  sSort[pl * ROWS + r] = srow >= 0 ? (int)srow : INT_MAX;
  if (r == 0) sI[pl] = active ? i : -1;
  if (tid == 0) {
    sLoHi[0] = INT_MAX;
    sLoHi[1] = -1;
  }
  __syncthreads();

  // ---- union of the group's conditioning rows, sorted, and each row's slot ----
  // The rows of a group lie in one or two time slabs, so their index range is
  // usually narrow: a bitmap over [lo, hi] marks them, and a prefix count over its
  // words gives the sorted union and every row's slot in a few barriers. Wider
  // ranges take a bitonic sort of the NSLOT entries and a binary search.
  {
    int vmin = srow >= 0 ? (int)srow : INT_MAX, vmax = srow >= 0 ? (int)srow : -1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      vmin = min(vmin, __shfl_xor(vmin, o));
      vmax = max(vmax, __shfl_xor(vmax, o));
    }
    if (lane == 0) {
      atomicMin(&sLoHi[0], vmin);
      atomicMax(&sLoHi[1], vmax);
    }
  }
  __syncthreads();
  constexpr int BMW = 512;  // bitmap words (16384 rows of index range)
  static_assert(BMW % NTH == 0 && 2 * BMW * sizeof(int) <= BIG_B, "bitmap in the staging area");
  constexpr int WPT = BMW / NTH;
  const int ulo = sLoHi[0], uhi = sLoHi[1];
  const bool use_bm = uhi < ulo || uhi - ulo < BMW * 32;
  if (use_bm) {
    unsigned* bm = reinterpret_cast<unsigned*>(sArea);
    int* pre = reinterpret_cast<int*>(sArea) + BMW;
    for (int w = tid; w < BMW; w += NTH) bm[w] = 0u;
    __syncthreads();
    if (srow >= 0) {
      const int off = (int)srow - ulo;
      atomicOr(&bm[off >> 5], 1u << (off & 31));
    }
    __syncthreads();
    // block-wide exclusive prefix of the word counts (WPT consecutive words per thread)
    unsigned wv[WPT];
    int cnt = 0;
#pragma unroll
    for (int e = 0; e < WPT; ++e) {
      wv[e] = bm[tid * WPT + e];
      cnt += __popc(wv[e]);
    }
    int inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int up = __shfl_up(inc, o);
      if (lane >= o) inc += up;
    }
    if (lane == 63) sSort[wave] = inc;  // wave totals (sSort is free on this path)
    __syncthreads();
    int base = inc - cnt;
    for (int w2 = 0; w2 < wave; ++w2) base += sSort[w2];
    if (tid == NTH - 1) sNU = base + cnt;
#pragma unroll
    for (int e = 0; e < WPT; ++e) {
      const int wi = tid * WPT + e;
      pre[wi] = base;
      unsigned b = wv[e];
      while (b) {
        const int bit = __builtin_ctz(b);
        b &= b - 1u;
        sUniq[base++] = ulo + wi * 32 + bit;
      }
    }
    __syncthreads();
    int slot = -1;
    if (srow >= 0) {
      const int off = (int)srow - ulo;
      slot = pre[off >> 5] + __popc(bm[off >> 5] & ((1u << (off & 31)) - 1u));
    }
    sSlot[pl][r] = slot;
    __syncthreads();
  }
  if (!use_bm) {
    for (int kk = 2; kk <= NSLOT; kk <<= 1) {
      for (int jj = kk >> 1; jj > 0; jj >>= 1) {
        for (int e = tid; e < NSLOT; e += NTH) {
          const int ptn = e ^ jj;
          if (ptn > e) {
            const int a0 = sSort[e], a1 = sSort[ptn];
            const bool up = (e & kk) == 0;
            if ((a0 > a1) == up) {
              sSort[e] = a1;
              sSort[ptn] = a0;
            }
          }
        }
        __syncthreads();
      }
    }
    if (wave == 0) {
      int base = 0;
      for (int c0 = 0; c0 < NSLOT; c0 += 64) {
        const int e = c0 + lane;
        const int v = sSort[e];
        const bool f = v != INT_MAX && (e == 0 || sSort[e - 1] != v);
        const unsigned long long bm = __ballot(f);
        const int at = base + __popcll(bm & ((1ull << lane) - 1ull));
        if (f) sUniq[at] = v;
        base += __popcll(bm);
      }
      if (lane == 0) sNU = base;
    }
    __syncthreads();
    for (int e = tid; e < NSLOT; e += NTH) {
      const int v = sIdx[e / ROWS][e % ROWS];
      int slot = -1;
      if (v >= 0) {
        int lo = 0, hi = sNU - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (sUniq[mid] < v) lo = mid + 1; else hi = mid;
        }
        slot = lo;
      }
      sSlot[e / ROWS][e % ROWS] = slot;
    }
    __syncthreads();
  }
  const int nu = sNU;

  // Staged chunk width: as many columns as the union size allows in the staging
  // area (wider chunks mean fewer barriers), and a divisor of the row length.
  constexpr int CAPB = (int)(BIG_B / sizeof(UT));          // elements of UT in sBig
  constexpr int MAXP0 = (CAPB / VPE + NTH - 1) / NTH;
  constexpr int MAXP = MAXP0 < 10 ? MAXP0 : 10;             // 16-byte pieces per thread
  // FP32/FP64 staging: nu rows of (width + VPE) elements.
  auto pick_width = [&](int cap, int rows) {
    cap = min(cap, MAXP * NTH * VPE);
    if (rows * (4 * KC + VPE) <= cap && A.ldu % (8 * KC) == 0) return 4 * KC;
    if (rows * (2 * KC + VPE) <= cap && A.ldu % (4 * KC) == 0) return 2 * KC;
    return KC;  // rows <= NSLOT + 15 always fits; ldu is a multiple of 64 >= 2 KC
  };
  // Split staging: NSP planes of nu rows of (width + BPAD) bfloat16, plane-major. A
  // row is an odd number of 16-byte units long, so the 16 rows one fragment read
  // gathers fall on different LDS banks unless their slots coincide modulo 16
  // (rows of interleaved planes, an even number of units apart, collided modulo 8).
  auto pick_width_split = [&]() {
    const int capb = (int)(BIG_B / 2) - ZROW;
    const int capp = MAXP * NTH * VPE;
    for (int w = 4 * KC; w > KC; w >>= 1)
      if (nu * NSP * (w + BPAD) <= capb && nu * w <= capp && A.ldu % (2 * w) == 0) return w;
    return KC;
  };
  bool split_stage = SPLIT;            // Gram pass; the W pass stages FP32
  int cw = SPLIT ? pick_width_split() : pick_width(CAPB, nu);
  int sld = SPLIT ? cw + BPAD : cw + VPE;  // row stride (bf16 per plane, or UT)
  int lppr = __builtin_ctz(cw / VPE);  // log2 of the 16-byte pieces per row and chunk
  int npieces = nu << lppr;
  __bf16* splane = reinterpret_cast<__bf16*>(sArea);
  // Two register sets of staged pieces: the loads of a chunk are issued two chunk
  // periods before its data go to LDS.
  f4v preA[MAXP], preB[MAXP];
  // Loads are unconditional (surplus lanes re-read the last piece) so that the
  // compiler can count them exactly and wait for one register set only. The
  // addresses of a thread's pieces at column 0 are set once per pass; a chunk's
  // load then adds its column.
  const UT* pptr[MAXP];
  auto set_ptrs = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < MAXP; ++j) {
      const int e = min(tid + j * NTH, npieces - 1);
      const int row = e >> lppr, piece = e & ((1 << lppr) - 1);
      pptr[j] = U + (int64_t)sUniq[row] * A.ldu + piece * VPE;
    }
  };
  auto load_into = [&](f4v (&pre)[MAXP], int kc) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < MAXP; ++j) pre[j] = *reinterpret_cast<const f4v*>(pptr[j] + kc);
  };
  auto store_from = [&](f4v (&pre)[MAXP]) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < MAXP; ++j) {
      const int e = tid + j * NTH;
      if (e < npieces) {
        const int row = e >> lppr, piece = e & ((1 << lppr) - 1);
        if (SPLIT && split_stage) {
          // x = t_0 + t_1 (+ t_2), each term the bfloat16 rounding of the remainder.
          f4v rem = pre[j];
#pragma unroll
          for (int sp = 0; sp < NSP; ++sp)
            *reinterpret_cast<bf4v*>(splane + (sp * nu + row) * sld + piece * 4) = bf16_term(rem);
        } else {
          *reinterpret_cast<f4v*>(stage + row * sld + piece * VPE) = pre[j];
        }
      }
    }
  };
  // One pass over the row in chunks of cw columns (an even number of them);
  // compute(kc) consumes the staged chunk kc. With first_issued, preA already
  // holds the loads of chunk 0. The loop body is free of conditional loads, so
  // each store waits for exactly the register set it writes out.
  auto run_pass = [&](auto&& compute, bool first_issued) __attribute__((always_inline)) {
    if (!first_issued) load_into(preA, 0);
    load_into(preB, cw);
    store_from(preA);
    __syncthreads();
    int kc = 0;
    for (; kc + 2 * cw < A.ldu; kc += 2 * cw) {
      load_into(preA, kc + 2 * cw);
      compute(kc);
      __syncthreads();
      store_from(preB);
      __syncthreads();
      load_into(preB, kc + 3 * cw);
      compute(kc + cw);
      __syncthreads();
      store_from(preA);
      __syncthreads();
    }
    compute(kc);
    __syncthreads();
    store_from(preB);
    __syncthreads();
    compute(kc + cw);
    __syncthreads();
  };

  // Direct-load geometry: a chunk is pcw columns of every union row, one segment of
  // 4 pcw bytes per row, its 16-byte units XOR-swizzled by the slot (2^lpu units).
  // A direct load moves 1 KB (64 lanes x 16 bytes) to consecutive LDS; pinst loads
  // fill a chunk, taken by the wavefronts in turn.
  [[maybe_unused]] int pcw = 64, lpu = 4, pinst = 0, pnbuf = 2;
  [[maybe_unused]] const char* gp[8];
  [[maybe_unused]] const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  if constexpr (DMA) {
    pcw = nu <= 64 ? 64 : 32;
    lpu = nu <= 64 ? 4 : 3;
    pinst = (nu + (64 >> lpu) - 1) >> (6 - lpu);
    pnbuf = pinst * 1024 <= PBUF1 ? 2 : 1;  // a single buffer (the whole area) holds 32 loads
  }
  // Each lane's source for its share of every load of a chunk, at column 0.
  [[maybe_unused]] auto dma_ptrs = [&]() __attribute__((always_inline)) {
    const int pu16 = 1 << lpu;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int inst = wave_u + i * NW;
      const int sg = min((inst << (6 - lpu)) + (lane >> lpu), nu - 1);
      const int u = (lane & (pu16 - 1)) ^ (sg & (pu16 - 1));
      gp[i] = reinterpret_cast<const char*>(U + (int64_t)sUniq[sg] * A.ldu + u * 4);
    }
  };
  // Loads of the chunk at column kc into buffer b (completion: vmcnt).
  [[maybe_unused]] auto dma_issue = [&](int kc, int b) __attribute__((always_inline)) {
    const int64_t koff = (int64_t)kc * 4;
    auto into = [&](unsigned char* base) __attribute__((always_inline)) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int inst = wave_u + i * NW;
        if (inst < pinst)
          __builtin_amdgcn_global_load_lds(gp[i] + koff,
                                           (__attribute__((address_space(3))) void*)(base + inst * 1024),
                                           16, 0, 0);
      }
    };
    into(sB0 + b * PBUF1);
  };
  // Start of a chunk: this wave's loads are in LDS, then every wave's.
  [[maybe_unused]] auto dma_wait = [&]() __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
  };

  // ---- Grams on MFMA from the staged union rows ----
  using AccT = typename std::conditional<PREC == 0, d4v, f4v>::type;
  AccT acc[PPW][NTT];
#pragma unroll
  for (int s2 = 0; s2 < PPW; ++s2)
#pragma unroll
    for (int t = 0; t < NTT; ++t) acc[s2][t] = AccT{0, 0, 0, 0};
  const int rr16 = lane & 15, kq = lane >> 4;
  auto gram_chunk = [&](int) __attribute__((always_inline)) {
    for (int sub = 0; sub < cw; sub += KC) {
#pragma unroll
    for (int s2 = 0; s2 < PPW; ++s2) {
      const int pp = wave * PPW + s2;
      if constexpr (PREC == 0) {
        // 16 doubles per step: lane group kq holds elements 4kq..4kq+3 (K = 4 per MFMA).
        double v[NT][4];
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
          const int sl = sSlot[pp][ti * 16 + rr16];
          if (sl >= 0) {
            const double2* src = reinterpret_cast<const double2*>(stage + sl * sld + sub + kq * 4);
            const double2 x0 = src[0], x1 = src[1];
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
              acc[s2][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[ti][c], v[tj][c], acc[s2][t], 0, 0, 0);
              ++t;
            }
        }
      } else {
        if constexpr (PREC == 1) {
          // 32 floats per step: lane group kq holds elements 8kq..8kq+7.
          float x[NT][8];
#pragma unroll
          for (int ti = 0; ti < NT; ++ti) {
            const int sl = sSlot[pp][ti * 16 + rr16];
            if (sl >= 0) {
              const float4* src = reinterpret_cast<const float4*>(stage + sl * sld + sub + kq * 8);
              const float4 a0 = src[0], a1 = src[1];
              x[ti][0] = a0.x; x[ti][1] = a0.y; x[ti][2] = a0.z; x[ti][3] = a0.w;
              x[ti][4] = a1.x; x[ti][5] = a1.y; x[ti][6] = a1.z; x[ti][7] = a1.w;
            } else {
#pragma unroll
              for (int e = 0; e < 8; ++e) x[ti][e] = 0.f;
            }
          }
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            int t = 0;
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
              for (int tj = 0; tj <= ti; ++tj) {
                acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti][c], x[tj][c], acc[s2][t], 0, 0, 0);
                ++t;
              }
          }
        } else {
          // Pre-split terms: lane group kq holds elements 8kq..8kq+7 of each plane.
          constexpr int NS = NSP;
          bf8v part[NT][NS];
#pragma unroll
          for (int ti = 0; ti < NT; ++ti) {
            const int sl = sSlot[pp][ti * 16 + rr16];
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
              if (sl >= 0)
                part[ti][sp] = *reinterpret_cast<const bf8v*>(splane + (sp * nu + sl) * sld + sub + kq * 8);
              else
                part[ti][sp] = bf8v{};
            }
          }
          int t = 0;
#pragma unroll
          for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int tj = 0; tj <= ti; ++tj) {
              if constexpr (NS == 3) {
                acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][2], part[tj][0], acc[s2][t], 0, 0, 0);
                acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][1], part[tj][1], acc[s2][t], 0, 0, 0);
                acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][2], acc[s2][t], 0, 0, 0);
              } else if (ti == tj) {
                // The dropped low-by-low product is a sum of squares on the
                // diagonal (it would bias every |U_r|^2 low by about 2^-18
                // relative, and with it every residual variance high); the
                // diagonal tiles keep it, so their entries are (h + l)(h + l).
                acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][1], part[tj][1], acc[s2][t], 0, 0, 0);
              }
              acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][1], part[tj][0], acc[s2][t], 0, 0, 0);
              acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][1], acc[s2][t], 0, 0, 0);
              acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][0], acc[s2][t], 0, 0, 0);
              ++t;
            }
        }
      }
    }
    }
  };
  if constexpr (DMA) {
    // Fragment addresses: lane (rr16, kq) of tile ti reads the two 16-byte units
    // 2 kq and 2 kq + 1 (columns 8 kq .. 8 kq + 7 of a 32-column step) of its
    // slot's segment, at (unit ^ (slot mod 2^lpu)); the second step of a
    // 64-column chunk flips bit 7 of the offset. Empty slots read zeros.
    if (tid < 16) reinterpret_cast<f4v*>(sB0 + PBUF0)[tid] = f4v{0.f, 0.f, 0.f, 0.f};
    const int pu16 = 1 << lpu;
    int fr[PPW][NT][2];  // byte offsets within a buffer; -1: empty slot
#pragma unroll
    for (int s2 = 0; s2 < PPW; ++s2)
#pragma unroll
      for (int ti = 0; ti < NT; ++ti) {
        const int sl = sSlot[wave * PPW + s2][ti * 16 + rr16];
#pragma unroll
        for (int h = 0; h < 2; ++h)
          fr[s2][ti][h] = sl >= 0 ? sl * 4 * pcw + (((2 * kq + h) ^ (sl & (pu16 - 1))) << 4) : -1;
      }
    const unsigned ab0 = lds_addr(sB0), ab1 = ab0 + PBUF1, abz = ab0 + PBUF0;
    // one pair's fragments (eight FP32 values per tile and lane), from buffer base ab
    auto frag = [&](f4v (&x)[NT][2], int s2, int sub, unsigned ab, unsigned az)
                    __attribute__((always_inline)) {
      const int sx = sub ? 128 : 0;
      unsigned ad[NT][2];
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          ad[ti][h] = fr[s2][ti][h] >= 0 ? ab + (unsigned)(fr[s2][ti][h] ^ sx) : az + 16 * h;
      lds_read4(x[0][0], x[0][1], x[1][0], x[1][1], ad[0][0], ad[0][1], ad[1][0], ad[1][1]);
    };
    // One pair's products. BF16X3: the fragments split into their two bfloat16
    // terms, three products per tile and the low-by-low product on the diagonal
    // tiles (as in the register-staged pass). BF16X6: three terms, the six products
    // whose term orders sum to at most two. FP32: eight K = 4 products per tile,
    // lane group kq holding columns 8 kq .. 8 kq + 7.
    auto pairmm = [&](f4v (&x)[NT][2], AccT (&ac)[NTT]) __attribute__((always_inline)) {
      if constexpr (PREC == 2) {
        bf8v pt[NT][2];
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
          const bf4v h0 = bf16_term(x[ti][0]), h1 = bf16_term(x[ti][1]);
          bf4v l0, l1;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            l0[c] = (__bf16)x[ti][0][c];
            l1[c] = (__bf16)x[ti][1][c];
          }
          pt[ti][0] = __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7);
          pt[ti][1] = __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7);
        }
        int t = 0;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
          for (int tj = 0; tj <= ti; ++tj) {
            if (ti == tj)
              ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][1], pt[tj][1], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][1], pt[tj][0], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][0], pt[tj][1], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][0], pt[tj][0], ac[t], 0, 0, 0);
            ++t;
          }
      } else if constexpr (PREC == 3) {
        bf8v pt[NT][3];
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
          const bf4v a0 = bf16_term(x[ti][0]), b0 = bf16_term(x[ti][1]);
          const bf4v a1 = bf16_term(x[ti][0]), b1 = bf16_term(x[ti][1]);
          bf4v a2, b2;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            a2[c] = (__bf16)x[ti][0][c];
            b2[c] = (__bf16)x[ti][1][c];
          }
          pt[ti][0] = __builtin_shufflevector(a0, b0, 0, 1, 2, 3, 4, 5, 6, 7);
          pt[ti][1] = __builtin_shufflevector(a1, b1, 0, 1, 2, 3, 4, 5, 6, 7);
          pt[ti][2] = __builtin_shufflevector(a2, b2, 0, 1, 2, 3, 4, 5, 6, 7);
        }
        int t = 0;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
          for (int tj = 0; tj <= ti; ++tj) {
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][2], pt[tj][0], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][1], pt[tj][1], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][0], pt[tj][2], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][1], pt[tj][0], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][0], pt[tj][1], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pt[ti][0], pt[tj][0], ac[t], 0, 0, 0);
            ++t;
          }
      } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          int t = 0;
#pragma unroll
          for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int tj = 0; tj <= ti; ++tj) {
              ac[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti][c >> 2][c & 3], x[tj][c >> 2][c & 3],
                                                           ac[t], 0, 0, 0);
              ++t;
            }
        }
      }
    };
    // One chunk of NSUB 32-column steps: each pair's products are issued before
    // the next pair's fragments are read.
    auto gram_dma = [&](auto nsub_c, unsigned ab, unsigned az) __attribute__((always_inline)) {
      constexpr int NSUB = decltype(nsub_c)::value;
      constexpr int NP = NSUB * PPW;
      f4v xs[2][NT][2];
      frag(xs[0], 0, 0, ab, az);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        pairmm(xs[q & 1], acc[q % PPW]);
        __builtin_amdgcn_sched_barrier(0);
        if (q + 1 < NP) frag(xs[(q + 1) & 1], (q + 1) % PPW, (q + 1) / PPW, ab, az);
      }
    };
    auto gram_chunk = [&](int b) __attribute__((always_inline)) {
      const unsigned ab = b ? ab1 : ab0, az = abz;
      if (pcw == 64)
        gram_dma(std::integral_constant<int, 2>{}, ab, az);
      else
        gram_dma(std::integral_constant<int, 1>{}, ab, az);
    };
    dma_ptrs();
    dma_issue(0, 0);
    const int nc = A.ldu / pcw;
    for (int c = 0; c < nc; ++c) {
      const int b = pnbuf == 2 ? (c & 1) : 0;
      dma_wait();
      if (pnbuf == 2 && c + 1 < nc) dma_issue((c + 1) * pcw, b ^ 1);
      gram_chunk(b);
      if (pnbuf == 1) {
        __syncthreads();
        if (c + 1 < nc) dma_issue((c + 1) * pcw, 0);
      }
    }
    __syncthreads();
  } else if constexpr (SPLIT && PPW > 1 && NSP == 2) {
    // BF16X3 with two or more points per wave: each (sub-step, point) pair's
    // fragments load while the previous pair's products run, from offsets fixed
    // for the pass; empty slots read the zero block (no masked loads).
    const int zoff = (int)(BIG_B / 2) - ZROW;
    for (int e = tid; e < ZROW; e += NTH) splane[zoff + e] = (__bf16)0.f;
    int fo[PPW][NT][NSP];
#pragma unroll
    for (int s2 = 0; s2 < PPW; ++s2)
#pragma unroll
      for (int ti = 0; ti < NT; ++ti) {
        const int sl = sSlot[wave * PPW + s2][ti * 16 + rr16];
#pragma unroll
        for (int sp = 0; sp < NSP; ++sp) fo[s2][ti][sp] = (sl >= 0 ? (sp * nu + sl) * sld : zoff) + kq * 8;
      }
    auto ld = [&](bf8v (&pt)[NT][NSP], const int (&o)[NT][NSP], int sub) __attribute__((always_inline)) {
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int sp = 0; sp < NSP; ++sp)
          pt[ti][sp] = *reinterpret_cast<const bf8v*>(splane + o[ti][sp] + sub);
    };
    auto mm = [&](const bf8v (&part)[NT][NSP], AccT (&ac)[NTT]) __attribute__((always_inline)) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj <= ti; ++tj) {
          if constexpr (NSP == 3) {
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][2], part[tj][0], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][1], part[tj][1], ac[t], 0, 0, 0);
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][2], ac[t], 0, 0, 0);
          } else if (ti == tj) {
            // low-by-low product on the diagonal tiles (a sum of squares there)
            ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][1], part[tj][1], ac[t], 0, 0, 0);
          }
          ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][1], part[tj][0], ac[t], 0, 0, 0);
          ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][1], ac[t], 0, 0, 0);
          ac[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part[ti][0], part[tj][0], ac[t], 0, 0, 0);
          ++t;
        }
    };
    [[maybe_unused]] auto gram_chunk_split = [&](int) __attribute__((always_inline)) {
      bf8v buf[2][NT][NSP];
      ld(buf[0], fo[0], 0);
      for (int sub = 0; sub < cw; sub += KC) {
        const int nx = sub + KC < cw ? sub + KC : sub;  // past the end: re-read (unused)
#pragma unroll
        for (int s2 = 0; s2 < PPW; ++s2) {
          if (s2 + 1 < PPW)
            ld(buf[(s2 + 1) & 1], fo[s2 + 1], sub);
          else
            ld(buf[0], fo[0], nx);
          mm(buf[s2 & 1], acc[s2]);
        }
      }
    };
    set_ptrs();
    run_pass(gram_chunk_split, false);
  } else {
    set_ptrs();
    run_pass(gram_chunk, false);
  }
  // Grams into LDS (the staging area is free now), full symmetric matrices.
#pragma unroll
  for (int s2 = 0; s2 < PPW; ++s2) {
    T* G = sM + (wave * PPW + s2) * ROWS * ROWS;
    int t = 0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int tj = 0; tj <= ti; ++tj) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = ti * 16 + (PREC == 0 ? mfma16_row_f64(lane, e) : mfma16_row_f32acc(lane, e));
          const int col = tj * 16 + rr16;
          G[row * ROWS + col] = acc[s2][t][e];
          if (ti != tj) G[col * ROWS + row] = acc[s2][t][e];
        }
        ++t;
      }
  }
  __syncthreads();

  // W-pass geometry (FP32 staging after the result tile of the split modes) and
  // the loads of its first chunk, in flight during the per-point phase.
  UT* wt = reinterpret_cast<UT*>(sArea);
  if constexpr (!WANT_B && !DMA) {
    split_stage = false;
    stage = wt + ((GP * (4 * KC + VPE) + VPE - 1) / VPE) * VPE;
    cw = pick_width(CAPB - (int)(stage - wt), nu);
    sld = cw + VPE;
    lppr = __builtin_ctz(cw / VPE);
    npieces = nu << lppr;
    set_ptrs();
    load_into(preA, 0);
  }

  // ---- per-point residual block, Cholesky, back-substitution (segment) ----
  T* M = sM + pl * ROWS * ROWS;
  const T* lag_tab = reinterpret_cast<const T*>(A.lagtab);
  {
    // Lane r takes the pairs (rp, e) for e < rp and (R, e - rp) otherwise, e = h + 2 tt:
    // every lane gets ROWS / 2 pairs of the lower triangle.
    const int h = (r >= ROWS / 2) ? 1 : 0;
    const int rp = r - h * (ROWS / 2);
    const int R = ROWS - 1 - rp;
    auto pair_of = [&](int tt, int& row, int& col) __attribute__((always_inline)) {
      const int e = h + 2 * tt;
      row = (e < rp) ? rp : R;
      col = (e < rp) ? e : e - rp;
      return e < ROWS - 1;
    };
    auto put = [&](int row, int col, T val) __attribute__((always_inline)) {
      M[row * ROWS + col] = val;
      M[col * ROWS + row] = val;
    };
    if (sizeof(T) == 4 && lag_tab) {
      // The lag factors of PB pairs are loaded together, then their covariances
      // formed with the operations of cov_eval (the lag-only factors from the table).
      constexpr int PB = ROWS / 2 < 8 ? ROWS / 2 : 8;
#pragma unroll 1
      for (int t0 = 0; t0 < ROWS / 2; t0 += PB) {
        T la[PB], le[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          int row, col;
          const bool on = pair_of(t0 + b, row, col) && row < q;
          const int lg = on ? (int)fabs(sT[pl][row] - sT[pl][col]) : 0;
          la[b] = lag_tab[2 * lg];
          le[b] = lag_tab[2 * lg + 1];
        }
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          int row, col;
          if (pair_of(t0 + b, row, col)) {
            T val = T(0);
            if (row < q) {
              const double dx = sX[pl][row] - sX[pl][col];
              const double dy = sY[pl][row] - sY[pl][col];
              val = gneiting_pair<T>(A.K, (T)dx, (T)dy, la[b], le[b]) - M[row * ROWS + col];
            }
            put(row, col, val);
          }
        }
      }
    } else {
#pragma unroll 1
      for (int tt = 0; tt < ROWS / 2; ++tt) {
        const int e = h + 2 * tt;
        if (e < ROWS - 1) {
          const int row = (e < rp) ? rp : R;
          const int col = (e < rp) ? e : e - rp;
          T val = T(0);
          if (row < q) {
            const double dx = sX[pl][row] - sX[pl][col];
            const double dy = sY[pl][row] - sY[pl][col];
            const double dt = sT[pl][row] - sT[pl][col];
            if (lag_tab) {
              const int lg = (int)fabs(dt);
              val = gneiting_pair<T>(A.K, (T)dx, (T)dy, lag_tab[2 * lg], lag_tab[2 * lg + 1]);
            } else {
              val = cov_eval<T>(A.K, (T)dx, (T)dy, (T)dt);
            }
            val -= M[row * ROWS + col];
          }
          M[row * ROWS + col] = val;
          M[col * ROWS + row] = val;
        }
      }
    }
    T dg = T(1);
    if (r < q) dg = T(A.K.sigma2 + A.K.nugget) - M[r * ROWS + r];
    M[r * ROWS + r] = dg;
  }
  wave_lds_sync();
  T a[ROWS];
#pragma unroll
  for (int j = 0; j < ROWS; ++j) a[j] = M[j * ROWS + r];
  if constexpr (DMA) {
    // Once every wave holds its blocks in registers, the first W chunk's loads go to
    // buffer 1 during the per-point phase; a chunk too large for it waits for the
    // whole area after that phase.
    __syncthreads();
    dma_ptrs();
    if (pnbuf == 2) dma_issue(0, 1);
  }
  // x_r = (G_NN^-1 G_Ni)_r (r < p), L_pp = sqrt(D_i), z_i = (y_i - x' y_N) / L_pp.
  T x = T(0), Lpp_b, zi;
  if constexpr (PREC == 0) {
    // FP64: Cholesky (its factor is kept for the gradient) and back-substitution.
    T Ldiag = T(1);
    const bool ok = seg_cholesky<ROWS, T>(a, yv, Ldiag, r, sb, sCol[pl]);
    if (active && r == 0 && !ok) flag_fail(A.fail, i);
    Lpp_b = __shfl(Ldiag, sb + p);
    zi = __shfl(yv, sb + p);
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < ROWS; ++j) M[r * ROWS + j] = (j <= r) ? a[j] : T(0);
    wave_lds_sync();
    T accb = (r < p) ? M[p * ROWS + r] : T(0);
    const T inv_diag = T(1) / Ldiag;
#pragma unroll
    for (int rr = ROWS - 1; rr >= 0; --rr) {
      const T xr_local = accb * inv_diag;
      const T xb = __shfl(xr_local, sb + rr);
      if (r == rr) x = xb;
      if (r < rr) accb -= M[rr * ROWS + r] * xb;
    }
    if (r >= p) x = T(0);
  } else {
    // FP32: one Gauss-Jordan sweep (no back-substitution).
    int kmax = p;
#pragma unroll
    for (int o = 32; o >= ROWS; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
    // uniform across the wave: a scalar, so the sweep's step guard is a scalar branch
    kmax = __builtin_amdgcn_readfirstlane(kmax);
    T xo = T(0);
    const bool ok = seg_gauss_jordan<ROWS, T>(a, yv, xo, r, p, kmax, sCol[pl]);
    const T d = __shfl(xo, sb + p);
    Lpp_b = dsqrt(d > T(0) ? d : T(1));
    zi = __shfl(yv, sb + p) / Lpp_b;
    x = (r < p) ? xo : T(0);
    const unsigned long long bad = __ballot(!ok);
    if (active && r == 0 && ((bad >> sb) & ((ROWS == 64) ? ~0ull : ((1ull << ROWS) - 1ull))) != 0ull)
      flag_fail(A.fail, i);
  }
  if constexpr (WANT_B) {
    if (active) {
      if (r < m) A.B[i * m + r] = (r < p) ? -(double)x : 0.0;
      if (r == 0) A.D[i] = (double)Lpp_b * (double)Lpp_b;
    }
    return;
  } else {
    if (active && r == 0) {
      A.logD[i] = 2.0 * log((double)Lpp_b);
      A.z[i] = (double)zi;
    }
    if constexpr (PREC == 0) {
      // the factor of the residual block, kept for the gradient (FP64 only)
      if (A.Lout && active) {
        double* lo = A.Lout + ((int64_t)i * ROWS + r) * ROWS;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) lo[j] = (j <= r) ? (double)a[j] : 0.0;
      }
    }
    // b_r = -x_r / L_pp (r < p), b_p = 1 / L_pp;  W_i = sum_r b_r U_{S_r}.
    const T inv = T(1) / Lpp_b;
    sBv[pl][r] = (r < p) ? -x * inv : (r == p ? inv : T(0));
    if (r == 0) sZ[pl] = active ? zi : T(0);
    __syncthreads();

    // ---- W rows: W_i = sum_r b_r U_{S_r}, gathered from the staged union rows ----
    if constexpr (DMA) {
      // An item is one point and one 16-byte piece of a chunk, its rows split over
      // 2^hs adjacent lanes (partial sums added across the quad). Each lane keeps its
      // rows' addresses within a buffer and their b_r in registers for the pass. The
      // items' results go to a tile, written out as W terms at the start of the next
      // chunk, before that chunk's loads are issued (two tiles alternate).
      const int nqp = pcw / 4;
      const int items = GP * nqp;  // 128 or 64: 2^hs lanes each fill the workgroup
      const int hs = 4 * items <= NTH ? 2 : 1;
      const int rpl = ROWS >> hs;  // 16 or 8
      const int it = tid >> hs;
      const int pp = it / nqp, cq = it - pp * nqp;
      const int part = tid & ((1 << hs) - 1);
      const int pu16 = 1 << lpu;
      float wb[16];
      unsigned wo[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int rr = part * rpl + e;
        const int sl = (it < items && e < rpl) ? sSlot[pp][rr] : -1;
        wb[e] = sl >= 0 ? (float)sBv[pp][rr] : 0.f;
        wo[e] = sl >= 0 ? (unsigned)(sl * 4 * pcw + ((cq ^ (sl & (pu16 - 1))) << 4)) : 0u;
      }
      const int wst = pcw + 4;
      const float* tiles = reinterpret_cast<const float*>(sTile);
      const unsigned at0 = lds_addr(sTile) + (unsigned)((pp * wst + cq * 4) * 4);
      // FP32: rows go to W directly (by point index), column k receiving z_i
      [[maybe_unused]] const int64_t ipw = sI[pp];
      [[maybe_unused]] const float zvw = (float)sZ[pp];
      [[maybe_unused]] float* Wf = reinterpret_cast<float*>(A.W);
      const unsigned ab0 = lds_addr(sB0), ab1 = ab0 + PBUF1;
      __bf16* Wp = reinterpret_cast<__bf16*>(A.W);
      // Rows 4h .. 4h + 3 of one column from a tile: one 8-byte piece per term plane
      // in the 8-row blocks of the W planes (rows in processing order).
      auto planes = [&](int kc, int t) __attribute__((always_inline)) {
        const float* wt = tiles + t * (PTILE / 4);
        for (int e = tid; e < pcw * (GP / 4); e += NTH) {
          const int col = e & (pcw - 1), h = e >> (lpu + 2);
          const int64_t row0 = g * GP + 4 * h;
          f4v v;
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4)
            v[q4] = (kc + col == A.k) ? (float)sZ[4 * h + q4] : wt[(4 * h + q4) * wst + col];
#pragma unroll
          for (int sp = 0; sp < NSP; ++sp)
            *reinterpret_cast<bf4v*>(
                Wp + ((sp * A.wrb + (row0 >> 3)) * A.ldu + kc + col) * 8 + (row0 & 7)) = bf16_term(v);
        }
      };
      auto gather = [&](unsigned ab, int t, int kc) __attribute__((always_inline)) {
        if (it < items) {
          f4v acc = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int r0 = 0; r0 < 16; r0 += 4) {
            if (r0 < rpl) {
              f4v v[4];
              lds_read4(v[0], v[1], v[2], v[3], ab + wo[r0], ab + wo[r0 + 1], ab + wo[r0 + 2], ab + wo[r0 + 3]);
#pragma unroll
              for (int e = 0; e < 4; ++e) acc += wb[r0 + e] * v[e];
            }
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[e] += quad_xor<0xB1>(acc[e]);
          if (hs >= 2) {
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] += quad_xor<0x4E>(acc[e]);
          }
          if (part == 0) {
            if constexpr (SPLIT) {
              lds_write16(at0 + (unsigned)(t * PTILE), acc);
            } else if (ipw >= 0) {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (kc + cq * 4 + e == A.k) acc[e] = zvw;
              *reinterpret_cast<f4v*>(Wf + ipw * A.ldu + kc + cq * 4) = acc;
            }
          }
        }
      };
      const int nc = A.ldu / pcw;  // chunk c in buffer (c + 1) mod 2, or all in buffer 0
      if (pnbuf == 1) dma_issue(0, 0);
      for (int c = 0; c < nc; ++c) {
        const int b = pnbuf == 2 ? ((c + 1) & 1) : 0;
        dma_wait();
        if constexpr (SPLIT) {
          if (c > 0) planes((c - 1) * pcw, (c - 1) & 1);
        }
        if (pnbuf == 2 && c + 1 < nc) dma_issue((c + 1) * pcw, b ^ 1);
        gather(b ? ab1 : ab0, c & 1, c * pcw);
        if (pnbuf == 1) {
          __syncthreads();
          if (c + 1 < nc) dma_issue((c + 1) * pcw, 0);
        }
      }
      if constexpr (SPLIT) {
        __syncthreads();
        planes((nc - 1) * pcw, (nc - 1) & 1);
      }
      return;
    }
    // An item is one point and one 16-byte piece of the staged chunk; each term is
    // one LDS read of a staged piece and VPE fused multiply-adds in the precision
    // of U (no products with the zeros of a dense selection matrix). The term's
    // row offset and b_r are read from LDS (the same address for the lanes of one
    // point); rows a point does not use have b_r = 0 and offset 0.
    constexpr int JI = (GP * (4 * KC / VPE) + NTH - 1) / NTH;  // items per thread, widest chunk
    typedef UT piece_t __attribute__((ext_vector_type(VPE)));
    const int nq = cw / VPE;
    const int items = GP * nq;
    // With fewer items than threads, an item's rows are split over 2^hs adjacent
    // lanes of a quad, whose partial sums are then added across the quad.
    const int hs = (ROWS >= 32 && 4 * items <= NTH) ? 2 : ((ROWS >= 16 && 2 * items <= NTH) ? 1 : 0);
    const int rpl = ROWS >> hs;  // rows per lane, a multiple of 8
    {
      const int sl = sSlot[pl][r];
      sSlot[pl][r] = sl >= 0 ? sl * sld : 0;
      if (sl < 0) sBv[pl][r] = T(0);
    }
    __syncthreads();
    UT* W = reinterpret_cast<UT*>(A.W);
    const int wst = cw + VPE;  // row stride of the result tile
    auto w_chunk = [&](int kc) __attribute__((always_inline)) {
#pragma unroll
      for (int j = 0; j < JI; ++j) {
        const int t2 = tid + j * NTH;
        const int it = t2 >> hs;
        if (it < items) {
          const int pp = it / nq, cq = it - pp * nq;
          const int sub = t2 & ((1 << hs) - 1);
          const int rb = sub * rpl;
          piece_t acc = piece_t{};
          const UT* src = stage + cq * VPE;
          // eight terms at a time: their reads in flight together
          for (int r0 = rb; r0 < rb + rpl; r0 += 8) {
            piece_t v[8];
            UT bb[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              v[e] = *reinterpret_cast<const piece_t*>(src + sSlot[pp][r0 + e]);
              bb[e] = (UT)sBv[pp][r0 + e];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) acc += bb[e] * v[e];
          }
          if (hs >= 1) {
#pragma unroll
            for (int e = 0; e < VPE; ++e) acc[e] += quad_xor<0xB1>(acc[e]);
          }
          if (hs >= 2) {
#pragma unroll
            for (int e = 0; e < VPE; ++e) acc[e] += quad_xor<0x4E>(acc[e]);
          }
          if (sub != 0) continue;
          if constexpr (SPLIT) {
            *reinterpret_cast<piece_t*>(wt + pp * wst + cq * VPE) = acc;
          } else {
            const int64_t ip = sI[pp];
            if (ip >= 0) {
#pragma unroll
              for (int e = 0; e < VPE; ++e)
                if (kc + cq * VPE + e == A.k) acc[e] = (UT)sZ[pp];
              *reinterpret_cast<piece_t*>(W + ip * A.ldu + kc + cq * VPE) = acc;
            }
          }
        }
      }
      if constexpr (SPLIT) {
        // Rows 4h .. 4h + 3 of one column from the tile: one 8-byte piece per term plane
        // in the 8-row blocks of the W planes (rows in processing order).
        __syncthreads();
        __bf16* Wp = reinterpret_cast<__bf16*>(A.W);
        for (int e = tid; e < cw * (GP / 4); e += NTH) {
          const int col = e % cw, h = e / cw;
          const int64_t row0 = g * GP + 4 * h;
          f4v v;
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4)
            v[q4] = (kc + col == A.k) ? (float)sZ[4 * h + q4] : (float)wt[(4 * h + q4) * wst + col];
#pragma unroll
          for (int sp = 0; sp < NSP; ++sp)
            *reinterpret_cast<bf4v*>(
                Wp + ((sp * A.wrb + (row0 >> 3)) * A.ldu + kc + col) * 8 + (row0 & 7)) = bf16_term(v);
        }
      }
    };
    run_pass(w_chunk, true);
  }
}

template <int ROWS, int PREC>
hipError_t launch_group(const FactorArgs& a, int mode, hipStream_t s) {
  using Sh = GroupShape<ROWS, PREC>;
  const int64_t ngrp =
      (PREC >= 2 && mode != 1) ? a.wrb * 8 / Sh::GP : (a.n + Sh::GP - 1) / Sh::GP;
  const unsigned grid = (unsigned)(((ngrp + 7) / 8) * 8);
  if constexpr (ROWS == 32 && PREC >= 1) {
    if (mode != 1) {
      hipLaunchKernelGGL((vif_group_kernel<32, false, PREC, true>), dim3(grid), dim3(64 * Sh::NW), 0, s, a);
      return hipGetLastError();
    }
  }
  if (mode == 1)
    hipLaunchKernelGGL((vif_group_kernel<ROWS, true, PREC>), dim3(grid), dim3(64 * Sh::NW), 0, s,
                       a);
  else
    hipLaunchKernelGGL((vif_group_kernel<ROWS, false, PREC>), dim3(grid), dim3(64 * Sh::NW), 0,
                       s, a);
  return hipGetLastError();
}

template <int ROWS, int PREC>
hipError_t launch_rows(const FactorArgs& a, int mode, hipStream_t s) {
  constexpr int PPW = 64 / ROWS;
  constexpr int kWPB = wpb<ROWS>();
  const int64_t per_block = (int64_t)kWPB * PPW;
  const int64_t nblk = (a.n + per_block - 1) / per_block;
  const unsigned grid = (unsigned)(((nblk + 7) / 8) * 8);
  if (mode == 1)
    hipLaunchKernelGGL((point_factor_kernel<ROWS, true, PREC>), dim3(grid), dim3(64 * kWPB), 0, s,
                       a);
  else
    hipLaunchKernelGGL((point_factor_kernel<ROWS, false, PREC>), dim3(grid), dim3(64 * kWPB), 0,
                       s, a);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_prec(const FactorArgs& a, int mode, hipStream_t s) {
  const int q = a.m + 1;
  if (a.k > 0) {
    if (q <= 16) return launch_group<16, PREC>(a, mode, s);
    if (q <= 32) return launch_group<32, PREC>(a, mode, s);
    return launch_group<64, PREC>(a, mode, s);
  }
  if (q <= 16) return launch_rows<16, PREC>(a, mode, s);
  if (q <= 32) return launch_rows<32, PREC>(a, mode, s);
  return launch_rows<64, PREC>(a, mode, s);
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void lag_table_kernel(KernDev K, int nlag, T* __restrict__ tab) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= nlag) return;
  T a, e;
  gneiting_lag<T>(K, (T)l, a, e);
  tab[2 * l] = a;
  tab[2 * l + 1] = e;
}

hipError_t launch_lag_table(const KernDev& K, int nlag, int prec, void* tab, hipStream_t s) {
  const dim3 grid((unsigned)((nlag + 255) / 256));
  if (prec == 0)
    hipLaunchKernelGGL(lag_table_kernel<double>, grid, dim3(256), 0, s, K, nlag, (double*)tab);
  else
    hipLaunchKernelGGL(lag_table_kernel<float>, grid, dim3(256), 0, s, K, nlag, (float*)tab);
  return hipGetLastError();
}

hipError_t launch_point_factor(const FactorArgs& a, int mode, int prec, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (prec == 0) return launch_prec<0>(a, mode, s);
  if (prec == 1) return launch_prec<1>(a, mode, s);
  if (prec == 2) return launch_prec<2>(a, mode, s);
  return launch_prec<3>(a, mode, s);
}

}  // namespace vif
