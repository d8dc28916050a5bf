// Internal launch interface between the host C ABI (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace vif {

// Records `msg` as the calling thread's last error (vif_last_error) and returns code.
int32_t report_error(int32_t code, const char* msg);

// ---- neighbor search --------------------------------------------------------
// Key modes: 0 = -(tab1 + sqrt(h2)*tab2) (GNEITING gamma=1/2, GNEITING_MATERN nu=1/2)
//            1 = -(tab1 + (u*u + v*v))     (MATERN_ANISO, u = dx/range_s)
//            2 = -(tab1 + h2^gamma*tab2)   (GNEITING, general gamma)
//            3 = -(tab1 + s(x))            (GNEITING_MATERN nu in {3/2, 5/2})
struct NbrArgs {
  int64_t n;
  int m;
  int mode;
  int nu_code;
  double ir_s, gamma, t0;
  // Real-valued times (general = 1): slabs are time bins of width 1 / islab, the
  // tables hold the bin-lag bounds, and each pair's lag factors are computed from
  // its own lag l = t_i - t_j: psi = a l^(2 alpha) + 1, f1 = c1 log psi,
  // f2 = c * psi^e2 (GNEITING: c1 = tau, e2 = -(beta gamma); GNEITING_MATERN:
  // c1 = delta + gamma, e2 = -(gamma / 2)); MATERN_ANISO: f1 = (l ir_t)^2.
  int general;
  double islab, a, two_alpha, c1, c, e2, ir_t;
  const double *sx, *sy, *t;
  const double *tab1, *tab2, *bnd;
  int32_t* nbr;
  const int32_t* qlist;  // when set, query w of the launch is point qlist[w] (n = list length)
};

// Uniform spatial grid shared by all time slabs; cell (cx, cy) of slab l holds
// the points of time t0 + l whose coordinates fall in it, stored contiguously
// (CSR over key = l * ncell + cy * gx + cx).
struct GridArgs {
  int gx, gy, ncell, nslab;
  int morton;                           // 1: cells numbered in Z order (gx = gy = 2^b)
  double islab = 1.0;                   // slab of t: min((t - t0) * islab, nslab - 1)
  double xmin, ymin, cw, ch, icw, ich;  // cell sizes and their inverses
  double margin;                        // absolute slack on distance bounds
  const int32_t* off;                   // [nslab * ncell + 1]
  const double *px, *py;                // coordinates in CSR order
  const int32_t* pidx;                  // original index in CSR order
};

constexpr int kMaxCells = 1 << 22;  // nslab * ncell

// Candidate proposal (learned embedding or spatial distance) + exact rerank.
struct ProposeArgs {
  int ncand;            // candidates kept for the exact rerank (<= 128)
  int lags;             // window: slabs t_i - lags .. t_i
  int wmin, rmax;       // window radius: smallest r in 1..rmax with >= wmin points, else rmax
  int cmax;             // larger windows fall back to the exact search (<= kProposeCmax)
  const float* E;       // [n, 16] embeddings, or NULL: spatial distance
  const float* Ecsr;    // the embeddings permuted into the grid's CSR order
  int32_t* fallback;    // [n] 1 where the row must come from the exact search
};
constexpr int kProposeCmax = 1024;
hipError_t launch_propose(const NbrArgs& a, const GridArgs& g, const ProposeArgs& pa,
                          hipStream_t s);
// out[pos] = E[pidx[pos]] for 16-float rows.
hipError_t launch_permute16(int64_t n, const int32_t* pidx, const float* E, float* out,
                            hipStream_t s);
// p[0 .. cnt) = 0.
hipError_t launch_zero_i32(int32_t* p, int64_t cnt, hipStream_t s);
// Compacts i with flag[i] != 0 into list, count into *count (device, zeroed first).
hipError_t launch_compact(int64_t n, const int32_t* flag, int32_t* list, int32_t* count,
                          hipStream_t s);

// ---- learned proposal network (learn.hip) -------------------------------------
struct FeatArgs {
  double cx, cy, ct, ss, st;  // coordinate centre and scales
  double hyper[5];            // log a, log c, log alpha, log beta, log gamma minus centres
};
hipError_t launch_features(int64_t n, const double* sx, const double* sy, const double* t,
                           const FeatArgs& f, float* X, hipStream_t s);
hipError_t launch_mlp_forward(int64_t rows, const float* params, const float* X, float* E,
                              float* H, hipStream_t s);
int64_t mlp_backward_blocks(int64_t rows);
hipError_t launch_mlp_backward(int64_t rows, const float* params, const float* X, const float* H,
                               const float* dE, float* part, float* grad, hipStream_t s);
hipError_t launch_pair_loss(int64_t groups, int npos, int nneg, float tau, const float* E,
                            float* dE, float* loss, hipStream_t s);
hipError_t launch_adam(int64_t count, float* p, const float* g, float* m, float* v, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_batch(int64_t nq, const int32_t* queries, const int32_t* nbr_ext, int m_ext,
                        int npos, int nhard, int nrand, const uint32_t* rnd, int rand_window,
                        const float* X, float* Xb, hipStream_t s);

// Checks finite, integer-valued, nondecreasing times; sets bits in *flag.
hipError_t launch_validate_times(int64_t n, const double* t, uint32_t* flag, hipStream_t s);
// out[0..3] = min sx, max sx, min sy, max sy (partial: 4 * 256 doubles of scratch).
hipError_t launch_bbox(int64_t n, const double* sx, const double* sy, double* partial,
                       double* out, hipStream_t s);
// In-place exclusive scan of a[0 .. len); bsum: (len + 1023) / 1024 entries of scratch.
hipError_t launch_exclusive_scan(int32_t* a, int64_t len, int32_t* bsum, hipStream_t s);
// Builds the CSR grid: counts/fill [nslab*ncell + 1], bsum [scan scratch], key [n].
hipError_t launch_grid_build(int64_t n, const double* sx, const double* sy, const double* t,
                             double t0, const GridArgs& g, int32_t* counts, int32_t* fill,
                             int32_t* bsum, int32_t* key, double* px, double* py, int32_t* pidx,
                             hipStream_t s);
hipError_t launch_neighbors(const NbrArgs& a, const GridArgs& g, hipStream_t s);

// ---- per-point factor ---------------------------------------------------------
struct FactorArgs {
  int64_t n;
  int m;
  int k;    // inducing points (0 = plain Vecchia)
  int ldu;  // row stride of U and W (elements)
  KernDev K;
  const double *sx, *sy, *t, *y;
  const int32_t* nbr;
  const void* U;  // [n, ldu], FP64 or FP32 by precision
  void* W;        // [n, ldu]; column k receives z_i. Split-BF16 modes: see w_planes below.
  // Split-BF16 modes (prec 2, 3): W is written as its bfloat16 terms (2 or 3 planes),
  // rows in processing order, padded to wrb * 8 rows, in 8-row blocks: the term sp of
  // W[row][col] sits at ((sp * wrb + row / 8) * ldu + col) * 8 + row % 8.
  int64_t wrb;
  double *B, *D;  // factor outputs
  double *logD, *z;  // NLL outputs (per point)
  const int32_t* ord;           // processing order (a permutation of 0..n-1) or NULL
  // GNEITING with integer, nondecreasing times: (A, e) of gneiting_lag per lag, in the
  // precision of the covariance entries (launch_lag_table); NULL: direct evaluation.
  const void* lagtab;
  unsigned long long* fail;     // smallest point index with a non-positive-definite block
  unsigned long long* bad_nbr;  // smallest point index with an invalid neighbor row
  // FP64 VIF NLL only, optional: the Cholesky factor of each point's residual block,
  // [n, rows, rows] row-major (rows = 16 for m < 16, 32 for m < 32, else 64), zero above
  // the diagonal, the identity past the point's block.
  double* Lout;
};

// tab[2 l], tab[2 l + 1] = gneiting_lag(K, l) for l < nlag, in FP64 (prec 0) or FP32.
hipError_t launch_lag_table(const KernDev& K, int nlag, int prec, void* tab, hipStream_t s);
// mode: 0 = NLL terms, 1 = factor (B, D). prec: 0 FP64, 1 FP32, 2 BF16X3.
hipError_t launch_point_factor(const FactorArgs& a, int mode, int prec, hipStream_t s);

// ---- low-rank part ----------------------------------------------------------
struct LowRankArgs {
  int64_t n;
  int k, kpad;
  KernDev K;
  double jitter;
  const double *sx, *sy, *t;     // data points
  const double *zx, *zy, *zt;    // inducing points
};

// S = C(Z,Z) + jitter I on the leading k x k block, identity on the padding.
hipError_t launch_cov_kk(const LowRankArgs& a, double* S, hipStream_t s);
// In-place lower Cholesky of an N x N FP64 matrix (N multiple of 64; upper part of
// the diagonal blocks zeroed, other upper blocks untouched). scratch: 64*64 doubles.
hipError_t launch_cholesky(int N, double* A, double* scratch, unsigned long long* fail,
                           hipStream_t s);
// P = L^-1 (N a multiple of 64, both N x N row-major FP64, zeros above the
// diagonal); T: scratch of trinv_scratch_bytes(N).
size_t trinv_scratch_bytes(int N);
hipError_t launch_trinv(int N, const double* L, double* P, double* T, hipStream_t s);
// The blocked Cholesky of `count` matrices (each N[i] x N[i], N[i] a multiple of
// 64, in place, scratch[i] and fail[i] as for launch_cholesky) with one panel and
// one update launch per step for all of them (up to kCholSet per launch).
constexpr int kCholSet = 32;
struct CholSet {
  int count, jb;
  int pre[kCholSet + 1];
  double* A[kCholSet];
  double* dscr[kCholSet];
  unsigned long long* fail[kCholSet];
  int N[kCholSet];
};
hipError_t launch_cholesky_set(int count, double* const* A, const int* N, double* const* scratch,
                               unsigned long long* const* fail, hipStream_t s);
// U[i, l] = C(x_i, z_l) for l < k, 0 for k <= l < kpad; FP64 (prec 0) or FP32 (prec >= 1).
hipError_t launch_crosscov(const LowRankArgs& a, void* U, int prec, hipStream_t s);
// In place: U[i, :] <- U[i, :] P^T with P lower triangular (U = C(X,Z) L_k^-T).
hipError_t launch_trmm(const LowRankArgs& a, const double* P, void* U, int prec, hipStream_t s);
// Split-BF16 modes, kpad small enough for 32 rows of C in LDS (lowrank_fused_ok):
// U = C(X, Z) P' in one pass, C evaluated on chip, with C and P split into two
// bfloat16 terms (prec 2) or three (prec 3, FP32-accurate); Pb: 2 * kpad^2
// (prec 2) or 3 * kpad^2 (prec 3) bfloat16 scratch.
bool lowrank_fused_ok(int kpad, int prec);
// Raises the fused kernel's dynamic-LDS limit on the current device (once per
// device; called by launch_lowrank_fused, and before graph capture).
hipError_t prepare_lowrank_fused();
hipError_t launch_lowrank_fused(const LowRankArgs& a, const double* P, void* Pb, float* U, int prec,
                                hipStream_t s);
// Partial Gram of W over row chunks: part[c][tile] = sum over the rows of chunk c
// of W_I' W_J (FP64 64 x 64 tiles for prec 0/1, FP32 128 x 128 tiles for the
// split-BF16 modes). syrk_chunks gives the chunk count, syrk_part_bytes the size
// of part.
// For the split-BF16 modes, n is the padded row count of the W planes (wrb * 8).
// chunk_rows (a multiple of 8) sets the rows per FP32 partial in the split-BF16 modes.
int syrk_chunks(int64_t n, int kpad, int prec, int chunk_rows = 4096);
size_t syrk_part_bytes(int64_t n, int kpad, int prec, int chunk_rows = 4096);
hipError_t launch_syrk(int64_t n, int kpad, const void* W, int prec, void* part, int nchunk,
                       hipStream_t s, int chunk_rows = 4096);
// Rows of W (processing order, padded) in the split-BF16 plane layout.
inline int64_t w_plane_rows(int64_t n) { return (n + 15) / 16 * 16; }
// From G = sum_c part[c], the Gram of [W z]: M = the augmented Woodbury matrix
// (I + G[0:k,0:k], row and column k = q = G[k,0:k], entry (k,k) = 2 G[k,k] + 1,
// identity padding); q = G[k,0:k]; zz = G[k,k].
hipError_t launch_syrk_reduce(int k, int kpad, const void* part, int prec, int nchunk, double* M,
                              double* q, double* zz, hipStream_t s);

// ---- reductions and final assembly ------------------------------------------
// flags[0..3] = ~0 (no failure recorded), flags[4] = 0 (time checks).
hipError_t launch_init_flags(void* flags, hipStream_t s);
// Deterministic sum of x[0..n) into *out (two-level tree, fixed order). partial: [256] scratch.
hipError_t launch_sum(int64_t n, const double* x, int squared, double* partial, double* out,
                      hipStream_t s);
// *dst = *src (device scalars).
hipError_t launch_copy_f64(const double* src, double* dst, hipStream_t s);
// out[0] = nll, out[1..4] = terms. For k > 0, LM is the Cholesky factor of the
// augmented Woodbury matrix written by launch_syrk_reduce: log det M from its
// first k pivots, q' M^-1 q from its row k.
hipError_t launch_finalize(int64_t n, int k, int kpad, const double* LM, const double* sum_logD,
                           const double* zz, double* out, hipStream_t s);


// Residual-correlation neighbors (residual.hip).
struct ResidArgs {
  int64_t n;
  int m, kpad;
  KernDev K;
  const double *sx, *sy, *t;
  const double* U;  // [n, kpad] FP64 (NULL when kpad = 0)
  const double* d;  // residual variances [n]
  const double* lagtab;  // GNEITING with integer times: (A, e) per lag (gneiting_lag), else NULL
  int32_t* nbr;     // [n, m]
};
// tab[2 l], tab[2 l + 1] = gneiting_lag(K, l) for l < nlag.
hipError_t launch_resid_lags(const KernDev& K, int nlag, double* tab, hipStream_t s);
// d[i] = sigma2 - |U_i|^2.
hipError_t launch_resid_var(int64_t n, int kpad, double sigma2, const double* U, double* d,
                            hipStream_t s);
hipError_t launch_resid_topm(const ResidArgs& a, hipStream_t s);

// Vecchia NLL gradient (gradient.hip).
constexpr int kGradMaxParams = 8;
struct GradKern {  // hyperparameters in the form the derivative code uses
  int kind, nu_code;
  double sigma2, a, c, two_alpha, beta, gamma, bg, tau, delta, ir_s2, ir_t2, inv_rs, inv_rt;
};
struct GradArgs {
  int64_t n;
  int m, P;
  KernDev K;
  GradKern G;
  double nugget;
  const double *sx, *sy, *t, *y;
  const int32_t* nbr;
  double* g;     // [P, n] per-point gradient terms
  double* logD;  // [n]
  double* z;     // [n]
  const double* lagtab;  // GNEITING with integer times: launch_grad_lags table, else NULL
  unsigned long long* fail;
  unsigned long long* bad_nbr;
};
// Six values per lag l < nlag (see gradient.hip) for the Gneiting kernel.
constexpr int kGradLagVals = 6;
hipError_t launch_grad_lags(const GradKern& G, int nlag, double* tab, hipStream_t s);
hipError_t launch_vecchia_grad(const GradArgs& a, hipStream_t s);

// ---- VIF gradient (grad_vif.hip) ----------------------------------------------
// C[M x N] = alpha op(A) op(B) (+ gamma eu[i] ev[j] when eu != NULL), FP64,
// row-major; split K over blockIdx.y (kchunk per split, outputs cstride apart).
struct GemmF64 {
  int64_t M;
  int N;
  int64_t K;
  const double* A;
  int64_t lda;
  int ta;
  const double* B;
  int64_t ldb;
  int tb;
  double* C;
  int64_t ldc;
  double alpha;
  const double* eu;
  const double* ev;
  double gamma;
  // Structure that lets tiles or K steps be skipped: b_lower = op(B) is lower
  // triangular (op(B)[l][j] = 0 for l < j), so column block j needs l >= j only;
  // c_lower = only C[i][j] with i >= j is wanted (tiles wholly above the diagonal
  // are not computed and their entries are left unwritten).
  int b_lower, c_lower;
  int64_t kchunk;
  int64_t cstride;
};
hipError_t launch_gemm_f64(const GemmF64& g, int splits, hipStream_t s);
hipError_t launch_splitk_reduce(int64_t count, int splits, int64_t stride, const double* part,
                                double* out, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t cnt, double v, hipStream_t s);
hipError_t launch_lead_block(int k, int kpad, const double* F, double* Lo, hipStream_t s);
hipError_t launch_clip_kk(int k, int kpad, double* X, hipStream_t s);
hipError_t launch_matvec(int kpad, const double* X, const double* x, double* y, hipStream_t s);
hipError_t launch_resid_e(int64_t n, int k, int ldw, const double* W, const double* z,
                          const double* v, double* e, hipStream_t s);
hipError_t launch_kk_deriv(const GradKern& G, int P, int k, int kpad, const double* zx,
                           const double* zy, const double* zt, double* dSk, hipStream_t s);
int phi_dot_blocks(int kpad);
hipError_t launch_phi_dot(int kpad, int P, const double* X, const double* Psi, double* out,
                          hipStream_t s);
hipError_t launch_cross_deriv(const GradKern& G, int P, int64_t n, int k, int ldg, const double* sx,
                              const double* sy, const double* st, const double* zx, const double* zy,
                              const double* zt, const double* Gt, double* crossd, hipStream_t s);
struct VifGradArgs {
  int64_t n;
  int m, k, kpad, P;
  int lrows;           // row stride of Lfac: 16, 32 or 64, the per-point kernel's block width
  GradKern G;
  const double *sx, *sy, *st, *y;
  const int32_t* nbr;
  const double* Lfac;  // [n, lrows, lrows] residual-block factors, lower triangle by rows
  const double* U;     // [n, kpad]
  const double* W;     // [n, kpad]: the forward pass's W (FP64; column k holds z)
  double* H;           // [n, kpad]: W M^-1 - e v' on entry; phi on return (below)
  const double* e;     // [n]: z - W v
  double* blk;         // [P, n] per-point <Lambda_i, dC_S + dnugget I>
  // Gamma's terms per conditioning slot: row i of Gamma's sum over (i, r) is
  // b_ir phi_i + w_ir W_i (phi_i = h_i - (1 + b.g) W_i + U_S' w_i, written over H);
  // bw[(i * QMAX + r) * 2 + {0, 1}] = (b_ir, w_ir), key[i * QMAX + r] = S_ir (-1 past q),
  // cnt[j] += the number of slots with S_ir = j (zeroed by the caller).
  double* bw;
  int32_t* key;
  int32_t* cnt;
};
// Gamma_j = sum over slots (i, r) with S_ir = j of b_ir phi_i + w_ir W_i, from the
// slots listed by j (CSR off/list, each list summed in increasing slot order).
struct GammaArgs {
  int64_t n;
  int k, kpad, qmax;
  const double* phi;   // [n, kpad]
  const double* W;     // [n, kpad]
  const double* bw;    // [n * qmax, 2]
  const int32_t* off;  // [n + 1]
  const int32_t* list; // slots
  double* Gam;         // [n, kpad], written whole (zero past k)
};
hipError_t launch_vif_grad_points(const VifGradArgs& a, hipStream_t s);
// list[off[j] + ..] = slots with key = j (fill zeroed by the caller; any order).
hipError_t launch_slot_fill(int64_t nslots, const int32_t* key, const int32_t* off, int32_t* fill,
                            int32_t* list, hipStream_t s);
hipError_t launch_gamma_gather(const GammaArgs& a, hipStream_t s);

}  // namespace vif
