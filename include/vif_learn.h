/* vif_learn.h -- learned neighbor proposal for the correlation-based Vecchia
 * neighbor search (C ABI of libvif.so, next to vif.h).
 *
 * The paper ranks neighbors by correlation under the current kernel (Sec.
 * "Correlation-based Vecchia neighbor selection") and observes that this
 * metric has no exact Euclidean embedding for the Gneiting class, so it
 * searches the metric itself with a cover tree. This interface adds a learned
 * shortcut: a small network embeds each point, embedding distances propose
 * candidates inside a space-time window, and the exact correlation key of
 * vif_neighbors reranks them. The exact search stays the fallback and the
 * judge (recall against it).
 *
 * Conventions as in vif.h: arrays are DEVICE pointers owned by the caller,
 * work is enqueued on the caller's HIP stream, every function returns a VIF_*
 * status, vif_last_error() describes the last failure, and argument errors are
 * found before any launch. FP32 arrays are row-major.
 */
#ifndef VIF_LEARN_H
#define VIF_LEARN_H

#include <stddef.h>
#include <stdint.h>

#include "vif.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Network: VIF_MLP_IN -> 64 -> 64 -> 64 -> VIF_MLP_OUT, ReLU on hidden layers.
 * Parameters (FP32, VIF_MLP_PARAMS values) are packed as W1[8][64], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[64][16], b4[16]; a layer computes
 * h_out = h_in W + b. */
#define VIF_MLP_IN 8
#define VIF_MLP_HIDDEN 64
#define VIF_MLP_OUT 16
#define VIF_MLP_PARAMS 9936

/* Input features X [n, 8]: (sx - c[0]) / c[3], (sy - c[1]) / c[3],
 * (t - c[2]) / c[4], then log a - c[5], log c - c[6], log alpha - c[7],
 * log beta - c[8], log gamma - c[9] (the five parameters that shape the
 * Gneiting correlation; sigma2 and the nugget cannot change neighbor sets).
 * centre: HOST array of 10 doubles. Requires kern->kind == VIF_KERNEL_GNEITING. */
int32_t vif_mlp_features(const vif_points* points, const vif_kernel* kern,
                         const double* centre, float* X, void* hip_stream);

/* E [rows, 16] = network(X [rows, 8]); H [rows, 3, 64] receives the three
 * post-ReLU hidden layers when not NULL (needed by vif_mlp_backward). */
int32_t vif_mlp_forward(const float* params, const float* X, int64_t rows, float* E, float* H,
                        void* hip_stream);

/* Workspace bytes for vif_mlp_backward over `rows` rows. */
size_t vif_mlp_backward_ws(int64_t rows);

/* grad [VIF_MLP_PARAMS] = d/dparams of sum(dE * E) over the rows, from the
 * forward pass's X and H. Sums are taken per block of 64 rows and then in FP64
 * in block order, so the result is deterministic. */
int32_t vif_mlp_backward(const float* params, const float* X, const float* H, const float* dE,
                         int64_t rows, float* grad, void* ws, size_t ws_bytes, void* hip_stream);

/* Contrastive loss over `groups` groups of G = 1 + npos + nneg consecutive rows
 * of E: the query, npos exact neighbors, nneg non-neighbors. With
 * d_j = |e_q - e_j|^2, a group's loss is the mean over (p, n) of
 * softplus((d_p - d_n) / tau). Writes loss [groups] and dE [groups * G, 16],
 * the gradient of the summed loss. npos, nneg >= 1, npos + nneg <= 128, tau > 0. */
int32_t vif_mlp_pair_loss(const float* E, int64_t groups, int32_t npos, int32_t nneg, float tau,
                          float* dE, float* loss, void* hip_stream);

/* One Adam step (step counts from 1) on `count` FP32 values. */
int32_t vif_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t count,
                     int32_t step, float lr, float beta1, float beta2, float eps,
                     void* hip_stream);

/* Training rows: for each query q = queries[b] (int32 [nq]), rows
 * [q, nbr_ext[q][0 .. npos-1] (exact neighbors), nbr_ext[q][npos .. npos+nhard-1]
 * (the next ranks, hard non-neighbors), nrand earlier points q - 1 - (rnd % w)
 * with w = min(q, rand_window)]; a random draw equal to one of the listed
 * points is replaced by the last hard one. nbr_ext: int32 [n, m_ext] exact
 * rows with m_ext >= npos + nhard and no padding for the chosen queries;
 * rnd: uint32 [nq, nrand]; Xb [nq * G, 8] receives the rows' features from
 * X [n, 8]. */
int32_t vif_mlp_batch(const float* X, const int32_t* queries, int64_t nq, const int32_t* nbr_ext,
                      int32_t m_ext, int32_t npos, int32_t nhard, int32_t nrand,
                      const uint32_t* rnd, int32_t rand_window, float* Xb, void* hip_stream);

/* Workspace bytes for vif_propose_neighbors. */
size_t vif_propose_ws(int64_t n);

/* Proposal search. For point i, the window is every earlier point of the time
 * slabs t_i - lags .. t_i whose grid cell (square side `cell`, origin at the
 * minimum coordinates, cell index = trunc((x - min) / cell) clamped) is within
 * r cells of the query's in x and in y, r the smallest radius in 1..rmax whose
 * cells hold at least wmin points of those slabs (the query's whole slab
 * counted), else rmax; (lags + 1)(2 rmax + 1) <= 256. The ncand (<= 128) window
 * points of
 * smallest |e_i - e_j|^2 (FP32, summed in dimension order, no fused
 * multiply-add), or of smallest squared spatial distance (FP64) when E is
 * NULL, ties to the lower index, are reranked by the exact key of
 * vif_neighbors; nbr [n, m] receives the best m (key descending, index
 * ascending, -1 padding). Rows whose window holds fewer than min(i, m) points
 * or more than cmax (<= 1024) take the exact search instead; *n_fallback (HOST,
 * may be NULL) receives their count. E: FP32 [n, 16] (16-byte aligned) or
 * NULL. Synchronises the stream. */
int32_t vif_propose_neighbors(const vif_points* points, const vif_kernel* kern, int32_t m,
                              const float* E, int32_t ncand, double cell, int32_t lags,
                              int32_t wmin, int32_t rmax, int32_t cmax, int32_t* nbr,
                              int64_t* n_fallback, void* ws, size_t ws_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* VIF_LEARN_H */
