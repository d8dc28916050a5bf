// Gradient of the VIF NLL with respect to the kernel hyperparameters (the fit of
// Sec. "Estimation and prediction" for the approximation of Sec. "The
// Vecchia-inducing-point full-scale approximation").
//
// With W = D^-1/2 B U, z = D^-1/2 B y, M = I + W'W, q = W'z the NLL is
//   1/2 [sum log D_i + log det M + z'z - q'M^-1 q] + n/2 log 2pi.
// Writing v = M^-1 q, e = z - W v and h_i = M^-1 W_i' - e_i v (row i of
// H = W M^-1 - e v'), its derivative is
//   dNLL = sum_i [1/2 d log D_i + e_i dz_i + h_i . dW_i].
// Per point, with L L' = R_S the residual block (i last), b = last row of L^-1,
// z_i = b . y_S and W_i = b' U_S; d log D_i = b' dR b and db = -b' dR R^-1 +
// 1/2 (b' dR b) b', so the point's terms through its block are <Lambda_i, dR_S>
// with g_i = e_i y_S + U_S h_i, w_i = R_S^-1 g_i and
//   Lambda_i = 1/2 (1 + b . g_i) b b' - 1/2 (b w_i' + w_i b').
// dR_S = dC_S + dnugget I - d(U_S U_S'), and with the U-terms of dW_i this
// leaves sum_j Gamma_j . dU_j, Gamma_j = sum over (i, r) with S_ir = j of
//   b_r h_i - 2 (Lambda_i U_S)_r.
// U = C_nk L_k^-T gives dU = dC_nk L_k^-T - U Phi', Phi the lower triangle (half
// diagonal) of L_k^-1 dSigma_k L_k^-T, so
//   dNLL = sum_i <Lambda_i, dC_S + dnugget I> + <Gamma L_k^-1, dC_nk>
//          - <Phi(L_k^-1 dSigma_k L_k^-T), Gamma' U>.
//
// Lambda_i has rank two, so row r of b h_i' - 2 Lambda_i U_S is
//   b_r phi_i + w_r W_i,   phi_i = h_i - (1 + b . g_i) W_i + U_S' w_i,
// and Gamma_j sums these over the slots (i, r) with S_ir = j.
//
// gfx950 pieces: an FP64 MFMA GEMM (H, Gamma L_k^-1, Gamma' U by split K, and
// the k x k products); one wavefront per point for Lambda_i, its contraction with
// the block derivatives, and phi_i (written over h_i) with the slot weights
// (b_r, w_r); Gamma by rows, each row gathering its slots (listed by a count,
// scan and fill) in increasing slot order, so there are no floating-point
// atomics and repeated runs agree bit for bit; a reduction over the n x k
// cross-covariance derivatives.
#include <math.h>

#include "grad_common.hpp"
#include "internal.hpp"

namespace vif {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- FP64 GEMM --
// C[M x N] = alpha op(A) op(B) (+ gamma eu[i] ev[j]); row-major operands:
// op(A)[i][l] = ta ? A[l * lda + i] : A[i * lda + l], op(B)[l][j] likewise with tb.
// Split K: blockIdx.y picks the K range [y kchunk, (y + 1) kchunk) and the output
// C + y cstride (partials summed by gemm_splitk_reduce in a fixed order).
// Tile 128 x 128 per workgroup (four wavefronts, 64 x 64 each as 4 x 4 MFMA
// tiles of 16 x 16), K staged 16 at a time through LDS; the global loads of the
// next stage are in flight (in registers) while the MFMAs consume the current one.
// Workgroups are dealt round-robin to the 8 XCDs; each XCD takes a contiguous
// range of tiles, so the tiles that share a block row of op(A) share an L2.
constexpr int GBM = 128, GBN = 128, GBK = 16, GLD = GBM + 1;
constexpr int GLA = (GBM * GBK) / 256, GLB = (GBN * GBK) / 256;  // loads per thread and stage

__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmF64 g) {
  __shared__ double sA[GBK][GLD];
  __shared__ double sB[GBK][GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ntn = (g.N + GBN - 1) / GBN;
  const int64_t ntiles = ((g.M + GBM - 1) / GBM) * ntn;
  const int64_t per = (ntiles + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= ntiles) return;  // whole workgroup, before any barrier
  const int64_t bm = (t / ntn) * GBM;
  const int bn = (int)(t % ntn) * GBN;
  if (g.c_lower && bn >= bm + GBM) return;
  int64_t kb = (int64_t)blockIdx.y * g.kchunk;
  const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
  if (g.b_lower && kb < bn) kb = bn;  // op(B)[l][j] = 0 for l < j <= bn + ...: start at bn
  double* C = g.C + (int64_t)blockIdx.y * g.cstride;
  const int wr = wave >> 1, wc = wave & 1;
  d4v acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
  const int fr = lane & 15, fk = lane >> 4;
  // this thread's staging coordinates (fixed over the K loop)
  int amm[GLA], akk[GLA], bnn[GLB], bkk[GLB];
#pragma unroll
  for (int j = 0; j < GLA; ++j) {
    const int e = tid + 256 * j;
    if (g.ta) { akk[j] = e / GBM; amm[j] = e % GBM; } else { amm[j] = e / GBK; akk[j] = e % GBK; }
  }
#pragma unroll
  for (int j = 0; j < GLB; ++j) {
    const int e = tid + 256 * j;
    if (g.tb) { bnn[j] = e / GBK; bkk[j] = e % GBK; } else { bkk[j] = e / GBN; bnn[j] = e % GBN; }
  }
  double ra[GLA], rb[GLB];
  auto load = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < GLA; ++j) {
      const int64_t gi = bm + amm[j], gl = k0 + akk[j];
      ra[j] = (gi < g.M && gl < ke) ? (g.ta ? g.A[gl * g.lda + gi] : g.A[gi * g.lda + gl]) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < GLB; ++j) {
      const int gj = bn + bnn[j];
      const int64_t gl = k0 + bkk[j];
      rb[j] = (gj < g.N && gl < ke) ? (g.tb ? g.B[(int64_t)gj * g.ldb + gl] : g.B[gl * g.ldb + gj]) : 0.0;
    }
  };
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += GBK) {
#pragma unroll
    for (int j = 0; j < GLA; ++j) sA[akk[j]][amm[j]] = ra[j];
#pragma unroll
    for (int j = 0; j < GLB; ++j) sB[bkk[j]][bnn[j]] = rb[j];
    __syncthreads();
    if (k0 + GBK < ke) load(k0 + GBK);
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = sA[ks + fk][wr * 64 + a * 16 + fr];
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = sB[ks + fk][wc * 64 + b * 16 + fr];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = bm + wr * 64 + a * 16 + mfma16_row_f64(lane, e);
        const int j = bn + wc * 64 + b * 16 + fr;
        if (i < g.M && j < g.N) {
          double v = g.alpha * acc[a][b][e];
          if (g.eu) v += g.gamma * g.eu[i] * g.ev[j];
          C[i * g.ldc + j] = v;
        }
      }
}

__global__ __launch_bounds__(256) void gemm_splitk_reduce(int64_t count, int splits, int64_t stride,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  double s = 0.0;
  for (int sp = 0; sp < splits; ++sp) s += part[sp * stride + e];
  out[e] = s;
}

// ------------------------------------------------------------- small pieces --
__global__ __launch_bounds__(256) void fill_f64_kernel(double* __restrict__ p, int64_t cnt, double v) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < cnt) p[e] = v;
}

// Lout = the leading k x k block of the (augmented) factor, identity elsewhere.
__global__ __launch_bounds__(256) void lead_block_kernel(int k, int kpad, const double* __restrict__ F,
                                                         double* __restrict__ Lo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)kpad * kpad) return;
  const int r = (int)(e / kpad), c = (int)(e % kpad);
  Lo[e] = (r < k && c < k) ? (c <= r ? F[e] : 0.0) : (r == c ? 1.0 : 0.0);
}

// Rows and columns past k set to zero.
__global__ __launch_bounds__(256) void clip_kk_kernel(int k, int kpad, double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)kpad * kpad) return;
  const int r = (int)(e / kpad), c = (int)(e % kpad);
  if (r >= k || c >= k) X[e] = 0.0;
}

// y = X x for a kpad x kpad matrix, one wavefront per row.
__global__ __launch_bounds__(256) void matvec_kernel(int kpad, const double* __restrict__ X,
                                                     const double* __restrict__ x, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= kpad) return;
  double s = 0.0;
  for (int c = lane; c < kpad; c += 64) s += X[(int64_t)r * kpad + c] * x[c];
  s = wave_sum(s);
  if (lane == 0) y[r] = s;
}

// e_i = z_i - W_i . v over the first k columns, one wavefront per row.
__global__ __launch_bounds__(256) void resid_e_kernel(int64_t n, int k, int ldw, const double* __restrict__ W,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ v, double* __restrict__ e) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int c = lane; c < k; c += 64) s += W[i * ldw + c] * v[c];
  s = wave_sum(s);
  if (lane == 0) e[i] = z[i] - s;
}

// dSk[p][a][b] = d C(z_a, z_b) / d theta_p for a, b < k, zero elsewhere.
__global__ __launch_bounds__(256) void kk_deriv_kernel(GradKern G, int P, int k, int kpad,
                                                       const double* __restrict__ zx,
                                                       const double* __restrict__ zy,
                                                       const double* __restrict__ zt,
                                                       double* __restrict__ dSk) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t kk = (int64_t)kpad * kpad;
  if (e >= kk) return;
  const int a = (int)(e / kpad), b = (int)(e % kpad);
  double dC[kGradMaxParams];
#pragma unroll
  for (int p = 0; p < kGradMaxParams; ++p) dC[p] = 0.0;
  if (a < k && b < k) cov_and_grad(G, zx[a] - zx[b], zy[a] - zy[b], zt[a] - zt[b], dC);
  for (int p = 0; p < P; ++p) dSk[p * kk + e] = dC[p];
}

// out[p * nb + block] = sum over the block's entries of Phi(X_p) .* Psi, Phi the
// lower triangle of X_p with half its diagonal (entries past k are zero); Psi is
// read on and below the diagonal only.
__global__ __launch_bounds__(256) void phi_dot_kernel(int kpad, int P, const double* __restrict__ X,
                                                      const double* __restrict__ Psi,
                                                      double* __restrict__ out) {
  __shared__ double red[4][kGradMaxParams];
  const int64_t kk = (int64_t)kpad * kpad;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double t[kGradMaxParams];
#pragma unroll
  for (int p = 0; p < kGradMaxParams; ++p) t[p] = 0.0;
  if (e < kk) {
    const int a = (int)(e / kpad), b = (int)(e % kpad);
    if (a >= b) {
      const double w = a > b ? 1.0 : 0.5;
      for (int p = 0; p < P; ++p) t[p] = w * X[p * kk + e] * Psi[e];
    }
  }
  for (int p = 0; p < P; ++p) {
    const double s = wave_sum(t[p]);
    if (lane == 0) red[wave][p] = s;
  }
  __syncthreads();
  if (threadIdx.x < P)
    out[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// crossd[p][j] = sum_l Gt[j][l] dC(x_j, z_l)/dtheta_p over l < k, one wavefront per row j.
__global__ __launch_bounds__(256) void cross_deriv_kernel(GradKern G, int P, int64_t n, int k, int ldg,
                                                          const double* __restrict__ sx,
                                                          const double* __restrict__ sy,
                                                          const double* __restrict__ st,
                                                          const double* __restrict__ zx,
                                                          const double* __restrict__ zy,
                                                          const double* __restrict__ zt,
                                                          const double* __restrict__ Gt,
                                                          double* __restrict__ crossd) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const double xj = sx[j], yj = sy[j], tj = st[j];
  double t[kGradMaxParams];
#pragma unroll
  for (int p = 0; p < kGradMaxParams; ++p) t[p] = 0.0;
  for (int l = lane; l < k; l += 64) {
    const double w = Gt[j * ldg + l];
    double dC[kGradMaxParams];
    cov_and_grad(G, xj - zx[l], yj - zy[l], tj - zt[l], dC);
#pragma unroll
    for (int p = 0; p < kGradMaxParams; ++p) t[p] += w * dC[p];
  }
  for (int p = 0; p < P; ++p) {
    const double s = wave_sum(t[p]);
    if (lane == 0) crossd[(int64_t)p * n + j] = s;
  }
}

// ------------------------------------------------------- per-point terms ----
template <int QMAX>
struct VgLds {
  double x[64], y[64], t[64], b[64], w[64], g[64];
  int sidx[64];
  double lam[QMAX][QMAX + 1];
};

template <int QMAX>
constexpr int vg_waves() { return QMAX == 32 ? 4 : 2; }

template <int QMAX>
__global__ __launch_bounds__(64 * vg_waves<QMAX>()) void vif_grad_point_kernel(VifGradArgs A) {
  constexpr int NWV = vg_waves<QMAX>();
  __shared__ VgLds<QMAX> sw[NWV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * NWV + wave;
  if (i >= A.n) return;  // whole wavefront; no workgroup barriers below
  const int m = A.m, P = A.P, k = A.k, kpad = A.kpad;
  const int r = lane;
  VgLds<QMAX>& L = sw[wave];
  // ---- conditioning set (rows checked by the forward pass) ----
  int idx = -1;
  if (r < m) idx = A.nbr[i * m + r];
  const bool valid = r < m && idx >= 0 && (int64_t)idx < i;
  const unsigned long long vb = __ballot(valid);
  const unsigned long long mmask = m >= 64 ? ~0ull : ((1ull << m) - 1ull);
  const int p = (int)__builtin_ctzll(~(vb & mmask));
  const int q = p + 1;
  const int64_t row = r < p ? (int64_t)idx : i;
  L.x[r] = A.sx[row];
  L.y[r] = A.sy[row];
  L.t[r] = A.st[row];
  L.sidx[r] = r < q ? (int)row : -1;
  const double yv = r < q ? A.y[row] : 0.0;
  // ---- L rows (the forward pass's factor of R_S), identity past q ----
  double a[QMAX];
  {
    const int lr = A.lrows;
    const double* lo = A.Lfac + ((int64_t)i * lr + (r < q ? r : 0)) * lr;
#pragma unroll
    for (int s = 0; s < QMAX; ++s)
      a[s] = (r < q && s <= r) ? lo[s] : ((r == s) ? 1.0 : 0.0);
  }
  wave_lds_sync();
  // ---- b = last row of L^-1: L' b = e_p ----
  double bv = 0.0;
#pragma unroll
  for (int kk = QMAX - 1; kk >= 0; --kk) {
    if (kk <= p) {
      const double part = (r > kk && r <= p) ? a[kk] * bv : 0.0;
      const double sum = wave_sum(part);
      const double lkk = rdl(a[kk], kk);
      const double vk = ((kk == p) ? 1.0 : 0.0) - sum;
      if (r == kk) bv = vk / lkk;
    }
  }
  // ---- g = e_i y_S + U_S h_i (eight rows at a time, lanes over the columns; the
  // eight wave sums are independent, so their shuffles overlap) ----
  const double ei = A.e[i];
  const double* hrow = A.H + i * (int64_t)kpad;
  double gv = r < q ? ei * yv : 0.0;
  for (int r0 = 0; r0 < q; r0 += 8) {
    const double* urow[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) urow[e] = A.U + (int64_t)L.sidx[r0 + e < q ? r0 + e : r0] * kpad;
    double part[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) part[e] = 0.0;
    for (int c = lane; c < k; c += 64) {
      const double hc = hrow[c];
#pragma unroll
      for (int e = 0; e < 8; ++e) part[e] += urow[e][c] * hc;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const double t = wave_sum(part[e]);
      if (r == r0 + e && r0 + e < q) gv += t;
    }
  }
  // ---- w = R_S^-1 g: forward then backward solve ----
  double f = 0.0, accf = 0.0;
#pragma unroll
  for (int kk = 0; kk < QMAX; ++kk) {
    const double val = (gv - accf) / a[kk];
    const double fk = rdl(val, kk);
    if (r == kk) f = fk;
    accf += r > kk ? a[kk] * fk : 0.0;
  }
  double wv = 0.0;
#pragma unroll
  for (int kk = QMAX - 1; kk >= 0; --kk) {
    if (kk < q) {
      const double part = (r > kk && r < q) ? a[kk] * wv : 0.0;
      const double sum = wave_sum(part);
      const double lkk = rdl(a[kk], kk);
      const double fk = rdl(f, kk);
      if (r == kk) wv = (fk - sum) / lkk;
    }
  }
  if (r >= q) {
    bv = 0.0;
    wv = 0.0;
    gv = 0.0;
  }
  const double bg = wave_sum(bv * gv);
  const double c1 = 0.5 * (1.0 + bg);
  L.b[r] = bv;
  L.w[r] = wv;
  wave_lds_sync();
  // Lambda (full symmetric q x q, zero past q) into LDS
  for (int e = lane; e < QMAX * QMAX; e += 64) {
    const int rr = e / QMAX, ss = e % QMAX;
    L.lam[rr][ss] = c1 * L.b[rr] * L.b[ss] - 0.5 * (L.b[rr] * L.w[ss] + L.w[rr] * L.b[ss]);
  }
  wave_lds_sync();
  // ---- <Lambda, dC_S + dnugget I> over the lower pairs ----
  double tp[kGradMaxParams];
#pragma unroll
  for (int pp = 0; pp < kGradMaxParams; ++pp) tp[pp] = 0.0;
  const int npair = q * (q + 1) / 2;
  for (int e = lane; e < npair; e += 64) {
    int rr, ss;
    pair_of(e, rr, ss);
    double dC[kGradMaxParams];
    cov_and_grad(A.G, L.x[rr] - L.x[ss], L.y[rr] - L.y[ss], L.t[rr] - L.t[ss], dC);
    const bool diag = rr == ss;
    const double wl = diag ? L.lam[rr][ss] : 2.0 * L.lam[rr][ss];
#pragma unroll
    for (int pp = 0; pp < kGradMaxParams; ++pp) tp[pp] += wl * dC[pp];
    if (diag) tp[1] += wl;  // nugget
  }
  for (int pp = 0; pp < P; ++pp) {
    const double s = wave_sum(tp[pp]);
    if (lane == 0) A.blk[(int64_t)pp * A.n + i] = s;
  }
  // ---- Gamma's terms: Lambda is rank two, so row r of b h_i' - 2 Lambda U_S is
  // b_r phi_i + w_r W_i with phi_i = h_i - 2 c1 W_i + U_S' w (W_i = b' U_S) ----
  double* hw = A.H + i * (int64_t)kpad;
  const double* wrow = A.W + i * (int64_t)kpad;
  for (int c = lane; c < k; c += 64) {
    double v = 0.0;
    for (int rr = 0; rr < q; ++rr) v += L.w[rr] * A.U[(int64_t)L.sidx[rr] * kpad + c];
    hw[c] = hw[c] - 2.0 * c1 * wrow[c] + v;
  }
  if (r < QMAX) {
    const int64_t sl = i * QMAX + r;
    A.bw[2 * sl] = bv;
    A.bw[2 * sl + 1] = wv;
    A.key[sl] = r < q ? L.sidx[r] : -1;
    if (r < q) atomicAdd(A.cnt + L.sidx[r], 1);
  }
}

__global__ __launch_bounds__(256) void slot_fill_kernel(int64_t nslots, const int32_t* __restrict__ key,
                                                        const int32_t* __restrict__ off,
                                                        int32_t* __restrict__ fill,
                                                        int32_t* __restrict__ list) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nslots) return;
  const int j = key[e];
  if (j < 0) return;
  list[off[j] + atomicAdd(fill + j, 1)] = (int32_t)e;
}

// One wavefront per row j of Gamma. The row's slots are put in increasing order
// (rank by counting, in LDS; lists longer than GMAX are summed in list order),
// then summed term by term, lanes over the columns.
constexpr int GMAX = 512;

__global__ __launch_bounds__(256) void gamma_gather_kernel(GammaArgs A) {
  __shared__ int32_t sraw[4][GMAX], ssort[4][GMAX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 4 + wave;
  if (j >= A.n) return;  // whole wavefront; no workgroup barriers below
  const int beg = A.off[j], len = A.off[j + 1] - beg;
  const bool sorted = len <= GMAX;
  if (sorted) {
    for (int t = lane; t < len; t += 64) sraw[wave][t] = A.list[beg + t];
    wave_lds_sync();
    for (int t = lane; t < len; t += 64) {
      const int32_t me = sraw[wave][t];
      int rank = 0;
      for (int u = 0; u < len; ++u) rank += sraw[wave][u] < me ? 1 : 0;
      ssort[wave][rank] = me;  // slots are distinct
    }
    wave_lds_sync();
  }
  double* out = A.Gam + j * (int64_t)A.kpad;
  constexpr int CW = 8;  // columns per lane and pass
  for (int c0 = 0; c0 < A.kpad; c0 += 64 * CW) {
    double acc[CW];
#pragma unroll
    for (int t = 0; t < CW; ++t) acc[t] = 0.0;
    // two slots at a time: their row loads in flight together
    for (int u = 0; u < len; u += 2) {
      const bool two = u + 1 < len;
      const int32_t e0 = sorted ? ssort[wave][u] : A.list[beg + u];
      const int32_t e1 = two ? (sorted ? ssort[wave][u + 1] : A.list[beg + u + 1]) : e0;
      const double b0 = A.bw[2 * (int64_t)e0], w0 = A.bw[2 * (int64_t)e0 + 1];
      const double b1 = two ? A.bw[2 * (int64_t)e1] : 0.0, w1 = two ? A.bw[2 * (int64_t)e1 + 1] : 0.0;
      const double* p0 = A.phi + (int64_t)(e0 / A.qmax) * A.kpad;
      const double* q0 = A.W + (int64_t)(e0 / A.qmax) * A.kpad;
      const double* p1 = A.phi + (int64_t)(e1 / A.qmax) * A.kpad;
      const double* q1 = A.W + (int64_t)(e1 / A.qmax) * A.kpad;
#pragma unroll
      for (int t = 0; t < CW; ++t) {
        const int c = c0 + t * 64 + lane;
        if (c < A.k) acc[t] += (b0 * p0[c] + w0 * q0[c]) + (b1 * p1[c] + w1 * q1[c]);
      }
    }
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int c = c0 + t * 64 + lane;
      if (c < A.kpad) out[c] = acc[t];
    }
  }
}

}  // namespace

hipError_t launch_gemm_f64(const GemmF64& g, int splits, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int64_t tiles = ((g.M + GBM - 1) / GBM) * ((g.N + GBN - 1) / GBN);
  const int64_t grid = (tiles + 7) / 8 * 8;
  hipLaunchKernelGGL(gemm_f64_kernel, dim3((unsigned)grid, (unsigned)splits), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_splitk_reduce(int64_t count, int splits, int64_t stride, const double* part,
                                double* out, hipStream_t s) {
  hipLaunchKernelGGL(gemm_splitk_reduce, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     count, splits, stride, part, out);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t cnt, double v, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, cnt, v);
  return hipGetLastError();
}

hipError_t launch_lead_block(int k, int kpad, const double* F, double* Lo, hipStream_t s) {
  const int64_t cnt = (int64_t)kpad * kpad;
  hipLaunchKernelGGL(lead_block_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, k, kpad, F, Lo);
  return hipGetLastError();
}

hipError_t launch_clip_kk(int k, int kpad, double* X, hipStream_t s) {
  const int64_t cnt = (int64_t)kpad * kpad;
  hipLaunchKernelGGL(clip_kk_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, k, kpad, X);
  return hipGetLastError();
}

hipError_t launch_matvec(int kpad, const double* X, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(matvec_kernel, dim3((unsigned)((kpad + 3) / 4)), dim3(256), 0, s, kpad, X, x, y);
  return hipGetLastError();
}

hipError_t launch_resid_e(int64_t n, int k, int ldw, const double* W, const double* z,
                          const double* v, double* e, hipStream_t s) {
  hipLaunchKernelGGL(resid_e_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, k, ldw, W, z, v, e);
  return hipGetLastError();
}

hipError_t launch_kk_deriv(const GradKern& G, int P, int k, int kpad, const double* zx,
                           const double* zy, const double* zt, double* dSk, hipStream_t s) {
  const int64_t cnt = (int64_t)kpad * kpad;
  hipLaunchKernelGGL(kk_deriv_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, G, P, k,
                     kpad, zx, zy, zt, dSk);
  return hipGetLastError();
}

int phi_dot_blocks(int kpad) { return (int)(((int64_t)kpad * kpad + 255) / 256); }

hipError_t launch_phi_dot(int kpad, int P, const double* X, const double* Psi, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(phi_dot_kernel, dim3((unsigned)phi_dot_blocks(kpad)), dim3(256), 0, s, kpad, P, X,
                     Psi, out);
  return hipGetLastError();
}

hipError_t launch_cross_deriv(const GradKern& G, int P, int64_t n, int k, int ldg, const double* sx,
                              const double* sy, const double* st, const double* zx, const double* zy,
                              const double* zt, const double* Gt, double* crossd, hipStream_t s) {
  hipLaunchKernelGGL(cross_deriv_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, G, P, n, k,
                     ldg, sx, sy, st, zx, zy, zt, Gt, crossd);
  return hipGetLastError();
}

hipError_t launch_slot_fill(int64_t nslots, const int32_t* key, const int32_t* off, int32_t* fill,
                            int32_t* list, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(slot_fill_kernel, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, s, nslots,
                     key, off, fill, list);
  return hipGetLastError();
}

hipError_t launch_gamma_gather(const GammaArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_gather_kernel, dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_vif_grad_points(const VifGradArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  // the slot arrays (bw, key) hold 32 slots per point for m < 32, else 64
  if (a.m < 32) {
    hipLaunchKernelGGL(vif_grad_point_kernel<32>, dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(vif_grad_point_kernel<64>, dim3((unsigned)((a.n + 1) / 2)), dim3(128), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace vif
