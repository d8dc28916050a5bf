/* vif_residual.h -- residual-correlation neighbors for VIF (C ABI of libvif.so).
 *
 * The VIF approximation builds its Vecchia factor on the residual of the
 * low-rank part (Sec. "The Vecchia-inducing-point full-scale approximation");
 * its conditioning sets are chosen by the correlation metric of Sec.
 * "Correlation-based Vecchia neighbor selection" applied to the residual
 * covariance of the latent process,
 *     r(p, q) = C(p, q) - U_p . U_q,   U = C(X, Z) L_k^-T,
 *     rho(i, j) = |r(i, j)| / sqrt(r(i, i) r(j, j)).
 * Row i of nbr lists the min(i, m) earlier points of largest rho (computed as
 * key r(i, j)^2 / r(j, j) in FP64, the same order; a point with r(j, j) <= 0
 * ranks after all others), ties to the lower index, -1 padding: the layout
 * vif_factor and vif_nll take. With ind->n = 0 (or ind NULL) the residual is the
 * covariance itself and the sets are those of vif_neighbors up to near-ties
 * (this search forms keys differently).
 *
 * The search is exact and brute force (n^2 k / 2 multiply-adds on FP64 MFMA);
 * it suits n up to a few hundred thousand.
 *
 * Conventions as in vif.h: DEVICE arrays owned by the caller, work on the
 * caller's HIP stream, VIF_* status, argument errors found before any launch,
 * vif_last_error() for the message.
 */
#ifndef VIF_RESIDUAL_H
#define VIF_RESIDUAL_H

#include <stddef.h>
#include <stdint.h>

#include "vif.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace bytes for vif_residual_neighbors (0 for invalid sizes). */
size_t vif_residual_ws(int64_t n, int32_t k);

/* nbr [n, m] (1 <= m <= VIF_MAX_M). ind: inducing points (may be NULL); L_k is
 * factored in FP64 with kern->jitter added; a Sigma_k that is not positive
 * definite returns VIF_E_NOT_PD. Synchronises the stream. */
int32_t vif_residual_neighbors(const vif_points* points, const vif_kernel* kern, int32_t m,
                               const vif_points* ind, int32_t* nbr, void* ws, size_t ws_bytes,
                               void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* VIF_RESIDUAL_H */
