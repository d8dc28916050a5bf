/*
 * vif.h -- C ABI of the MI355X (gfx950) library that evaluates the Vecchia and
 * Vecchia-inducing-point full-scale (VIF) approximate negative log-likelihood of
 * a non-separable space-time Gaussian process (arXiv 2602.03609).
 *
 * Problem statement (Sec. "Spatio-temporal Gaussian process model"): points
 * (s_i, t_i) with s_i in R^2 and t_i in R, observations y (the residual after
 * the mean), a covariance c((s_i,t_i),(s_j,t_j)) with hyperparameters theta, a
 * nugget, m Vecchia neighbors per point and k inducing points.
 *
 * Conventions shared by every entry point
 *  - All array pointers are DEVICE pointers owned by the caller (e.g. torch
 *    tensors) unless marked HOST. Inputs are read only. The library allocates
 *    no device memory: every call takes a caller-owned workspace of at least
 *    vif_workspace_bytes(...) bytes (any alignment >= 256 bytes).
 *  - Points are passed as structure-of-arrays (sx, sy, t), FP64, length n.
 *    Index order is the Vecchia order; t must be nondecreasing in index (the
 *    time-stratified ordering of Sec. "Correlation-based Vecchia neighbor
 *    selection" guarantees it).
 *  - Work is enqueued on `hip_stream` (a hipStream_t; NULL = default stream).
 *    Every entry point returns after its results are complete on that stream.
 *  - Return value: VIF_OK or an error code; nothing is thrown across the ABI.
 *    vif_last_error() gives a message for the calling thread. Argument errors
 *    are detected before any launch. VIF_E_NOT_PD names the first point (or
 *    matrix) whose factorisation failed. After an error the contents of the
 *    output arrays are unspecified.
 *  - Not re-entrant on one workspace; distinct workspaces may be used from
 *    several host threads.
 */
#ifndef VIF_H
#define VIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  VIF_OK = 0,
  VIF_E_ARG = 1,          /* invalid argument (sizes, hyperparameters, time order) */
  VIF_E_NOT_PD = 2,       /* a covariance block, Sigma_k or M is not positive definite */
  VIF_E_DEVICE = 3,       /* HIP runtime error */
  VIF_E_WORKSPACE = 4,    /* workspace smaller than vif_workspace_bytes() */
  VIF_E_UNSUPPORTED = 5   /* valid request outside what this build implements */
};

/* Covariance kernels (latent covariance; the nugget is added separately).
 *
 * VIF_KERNEL_GNEITING: Gneiting-class kernel with stretched-exponential spatial
 *   part, psi = a|dt|^(2 alpha) + 1,
 *   C = sigma2 psi^-tau exp(-c |ds|^(2 gamma) / psi^(beta gamma)).
 *   Equals Eq. (Gneiting) at Matern smoothness 1/2 with paper gamma = 2 beta gamma,
 *   delta = tau - 2 beta gamma. Uses sigma2, a, c, alpha, beta, gamma, tau.
 *   Requires a, c, sigma2 > 0, alpha in (0,1], gamma in (0,1], beta in [0,1], tau >= 0.
 * VIF_KERNEL_GNEITING_MATERN: Eq. (Gneiting) with d = 2,
 *   x = c|ds| / psi^(gamma/2), C = sigma2 psi^-(delta+gamma) g_nu(x), where
 *   g_nu is the normalised Matern correlation in its closed form for
 *   nu in {0.5, 1.5, 2.5} (Sec. "GPU acceleration"). Uses sigma2, a, c, alpha,
 *   gamma (in [0,1]), delta (>= 0), nu.
 * VIF_KERNEL_MATERN_ANISO: C = sigma2 g_nu(d), d = sqrt(|ds|^2/range_s^2 + dt^2/range_t^2).
 *   Uses sigma2, range_s, range_t, nu.
 */
enum { VIF_KERNEL_GNEITING = 1, VIF_KERNEL_GNEITING_MATERN = 2, VIF_KERNEL_MATERN_ANISO = 3 };

/* Arithmetic of the per-point factors and the low-rank contractions.
 * FP64: everything in FP64 (FP64 MFMA for the contractions).
 * FP32: covariance entries and per-point Cholesky in FP32; U, the per-point
 *   Gram U_S U_S' and M = I + W'W on FP32 MFMA; U and W stored in FP32.
 * BF16X3: as FP32, but the three contractions run on BF16 MFMA with each FP32
 *   operand split in two bf16 terms, x = h + l, and the products
 *   h*h + h*l + l*h accumulated in FP32 (about 16 significant bits per product).
 *   The diagonal 16x16 tiles of the Gram U_S U_S' and the diagonal tiles of M
 *   add l*l: on a diagonal it is a sum of squares, and dropping it would bias
 *   every squared row norm low and every residual variance high.
 * BF16X6: as BF16X3 for U; the Gram and M, whose results enter the likelihood
 *   through cancellation (C - U_S U_S' and z'z - q'M^-1 q), split each operand
 *   in three bf16 terms and accumulate the six products down to 2^-24.
 * In every mode Sigma_k and its factor, the M factor, log-determinants,
 * quadratic forms and sums over points are FP64, and the FP32 partial sums of
 * M are combined in FP64 every 1024 rows. */
enum { VIF_PREC_FP64 = 0, VIF_PREC_FP32 = 1, VIF_PREC_BF16X3 = 2, VIF_PREC_BF16X6 = 3 };

enum { VIF_OP_NEIGHBORS = 0, VIF_OP_FACTOR = 1, VIF_OP_NLL = 2, VIF_OP_NEIGHBORS_NLL = 3 };

/* Hyperparameters (HOST struct; fields a kernel kind does not use are ignored).
 * nugget >= 0 is the noise variance of Eq. (Model). jitter >= 0 is added to the
 * diagonal of Sigma_k (0 = none). */
typedef struct {
  int32_t kind;
  double sigma2, nugget, a, c, alpha, beta, gamma, tau, nu, delta, range_s, range_t, jitter;
} vif_kernel;

/* n points, SoA device arrays of length n (FP64). */
typedef struct {
  int64_t n;
  const double* sx;
  const double* sy;
  const double* t;
} vif_points;

/* Upper bound on the number of distinct integer time lags (t[n-1] - t[0] + 1)
 * accepted by vif_neighbors. */
#define VIF_MAX_LAGS 65536
/* Largest neighbor count m (one wavefront holds one neighbor list). */
#define VIF_MAX_M 63
/* Largest number of inducing points k. */
#define VIF_MAX_K 4096

/* Bytes of workspace needed by operation `op` (VIF_OP_*) for n points, m
 * neighbors, k inducing points (0 = plain Vecchia) and precision `prec`.
 * Returns 0 for invalid arguments. */
size_t vif_workspace_bytes(int64_t n, int32_t m, int32_t k, int32_t prec, int32_t op);

/* Correlation-based neighbor selection (Sec. "Correlation-based Vecchia
 * neighbor selection", Alg. 2): for each i, the min(i, m) earlier points j < i
 * of largest correlation under the latent kernel (nugget excluded), ties to
 * the lower index. Output nbr: int32 [n*m] row-major, row i sorted by
 * decreasing correlation then increasing index, padded with -1.
 * Times must be integer-valued and nondecreasing with t[n-1]-t[0] < VIF_MAX_LAGS.
 * Ranking key: FP64 log-correlation with a fixed operation order (per-lag
 * factors from the host C math library, IEEE add/mul/sqrt per pair), which is
 * bit-reproducible for GNEITING with gamma = 1/2, GNEITING_MATERN with nu = 1/2
 * and MATERN_ANISO; other settings rank with device pow/log1p and may differ
 * from another implementation at near-ties. */
int32_t vif_neighbors(const vif_points* p, const vif_kernel* kern, int32_t m, int32_t* nbr,
                      void* ws, size_t ws_bytes, void* hip_stream);

/* Per-point Vecchia factor (Sec. "Vecchia approximation") or, when ind != NULL
 * and ind->n > 0, the VIF residual factor (Sec. "The Vecchia-inducing-point
 * full-scale approximation"), on the response covariance Sigma + nugget I.
 * nbr: int32 [n*m] as produced by vif_neighbors (any earlier indices, -1
 * padding at the end of a row). Outputs: B [n*m] FP64 with B[i*m+r] = -A_i[r]
 * paired with nbr[i*m+r] (0 where nbr is -1), so that B is the unit
 * lower-triangular factor with Cov ~ B^-1 D B^-T; D [n] FP64. */
int32_t vif_factor(const vif_points* p, const vif_kernel* kern, int32_t m, const int32_t* nbr,
                   const vif_points* ind, int32_t prec, double* B, double* D, void* ws,
                   size_t ws_bytes, void* hip_stream);

/* Negative log-likelihood (Sec. "Estimation and prediction") under the
 * Vecchia (ind == NULL or ind->n == 0) or VIF approximation. y: FP64 [n].
 * Result written to *nll (HOST). */
int32_t vif_nll(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                const int32_t* nbr, const vif_points* ind, int32_t prec, double* nll, void* ws,
                size_t ws_bytes, void* hip_stream);

/* As vif_nll, and also returns its four terms (HOST double[4]):
 * terms[0] = sum_i log D_i, terms[1] = z'z, terms[2] = log det M,
 * terms[3] = q' M^-1 q (the last two are 0 for plain Vecchia), so that
 * nll = n/2 log(2 pi) + (terms[0] + terms[2])/2 + (terms[1] - terms[3])/2. */
int32_t vif_nll_terms(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                      const int32_t* nbr, const vif_points* ind, int32_t prec, double* nll,
                      double* terms, void* ws, size_t ws_bytes, void* hip_stream);

/* vif_neighbors followed by vif_nll on its output, in one call: the neighbor
 * search (Alg. 2) runs on a library-owned stream of hip_stream's device (default
 * priority, restricted to all but 32 of the device's compute units) while
 * hip_stream builds Sigma_k, whose small launches take the CUs left free, and U;
 * the per-point stage waits for the search. When hip_stream is the null stream,
 * the NLL's work runs on a library-owned non-blocking stream ordered after the
 * null stream's earlier work. nbr (DEVICE int32 [n*m], written) and the NLL are
 * bit-identical to the two separate calls. Workspace:
 * vif_workspace_bytes(n, m, k, prec, VIF_OP_NEIGHBORS_NLL). Returns after every
 * stream it used has drained, also on error. Calls on one device from several
 * host threads run one at a time (they share those streams). */
int32_t vif_neighbors_nll(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                          int32_t* nbr, const vif_points* ind, int32_t prec, double* nll, void* ws,
                          size_t ws_bytes, void* hip_stream);

/* Bytes of the device array that vif_neighbors_noalloc uses as its workspace
 * (64 MiB; enough for the neighbor search of about 1.3 million points). */
#define VIF_NOALLOC_SCRATCH_BYTES (64u << 20)

/* vif_neighbors without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same arguments, result and errors as
 * vif_neighbors, bit-identical output. Its workspace is a file-scope device
 * array of VIF_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds
 * from the first call on that GPU until the process ends; the call allocates
 * nothing. Returns VIF_E_WORKSPACE, before any launch, when
 * vif_workspace_bytes(n, m, 0, VIF_PREC_FP64, VIF_OP_NEIGHBORS) exceeds that
 * size. All calls on one GPU share the array: calls that overlap in time on
 * one GPU (several host threads, or several streams) race and must not be
 * issued. */
int32_t vif_neighbors_noalloc(const vif_points* p, const vif_kernel* kern, int32_t m, int32_t* nbr,
                              void* hip_stream);

/* Message for the last error on the calling thread ("" after success). The
 * pointer stays valid until the next call on this thread. */
const char* vif_last_error(void);

/* Stage timing (instrumentation, not part of the method). When enabled, each
 * entry point records a pair of HIP events on its stream around every stage
 * below and, after its final synchronisation, adds the elapsed time to a
 * process-wide total. Not thread-safe: profile from one host thread. */
enum {
  VIF_STAGE_NEIGHBORS = 0,     /* slab table + neighbor search kernels */
  VIF_STAGE_SIGMA_K = 1,       /* Sigma_k, its Cholesky factor and inverse */
  VIF_STAGE_CROSSCOV = 2,      /* cross-covariance C(X,Z) into U's buffer */
  VIF_STAGE_TRMM = 3,          /* U = C(X,Z) L_k^-T, in place */
  VIF_STAGE_POINT_FACTOR = 4,  /* per-point factor (and W for the VIF NLL) */
  VIF_STAGE_SYRK = 5,          /* partial sums of [W z]'[W z] */
  VIF_STAGE_ASSEMBLY = 6,      /* reduction, chol(M), sums, final assembly */
  VIF_NSTAGES = 7
};
/* enable != 0 turns timing on, 0 turns it off; both reset the totals. */
int32_t vif_profile(int32_t enable);
/* Copies min(cap, VIF_NSTAGES) totals (ms) and call counts into the HOST
 * arrays; VIF_E_ARG for NULL outputs. */
int32_t vif_profile_read(double* total_ms, int32_t* calls, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* VIF_H */
