/* vif_grad.h -- gradient of the Vecchia NLL in the kernel hyperparameters
 * (C ABI of libvif.so).
 *
 * The paper fits the hyperparameters by minimising the NLL with a quasi-Newton
 * method that uses its gradient (Sec. "Estimation and prediction"). For the
 * plain Vecchia approximation on Sigma + nugget I (the likelihood of vif_nll
 * with ind = NULL) the NLL is a sum over points of 1/2 [l(S_i) - l(N_i)],
 * l(T) = log det Sigma~_TT + y_T' Sigma~_TT^-1 y_T, S_i = N(i) + {i}; its
 * gradient is the sum of the Gaussian formula
 *     1/2 [tr(Sigma~_T^-1 dSigma~_T) - alpha_T' dSigma~_T alpha_T]
 * over the two nested blocks of every point.
 *
 * Parameters, in this order (the gradient array holds vif_grad_params(kind)):
 *   VIF_KERNEL_GNEITING:        sigma2, nugget, a, c, alpha, beta, gamma, tau
 *   VIF_KERNEL_GNEITING_MATERN: sigma2, nugget, a, c, alpha, gamma, delta   (nu fixed)
 *   VIF_KERNEL_MATERN_ANISO:    sigma2, nugget, range_s, range_t   (nu fixed)
 * vif_nll_grad covers plain Vecchia; vif_nll_grad_vif the VIF approximation
 * (inducing points).
 *
 * Conventions as in vif.h: DEVICE arrays owned by the caller, work on the
 * caller's HIP stream, VIF_* status, argument errors found before any launch.
 */
#ifndef VIF_GRAD_H
#define VIF_GRAD_H

#include <stddef.h>
#include <stdint.h>

#include "vif.h"

#ifdef __cplusplus
extern "C" {
#endif

#define VIF_GRAD_MAX_PARAMS 8

/* Number of gradient entries for a kernel kind (0 if not supported). */
int32_t vif_grad_params(int32_t kind);

/* Workspace bytes for vif_nll_grad (0 for invalid sizes). */
size_t vif_grad_ws(int64_t n);

/* *nll (HOST) and grad (HOST, vif_grad_params(kern->kind) values) of the
 * Vecchia NLL, nbr as for vif_nll (m <= VIF_MAX_M). Per-point terms are summed
 * in FP64 in a fixed order (repeatable bits). Synchronises the stream. */
int32_t vif_nll_grad(const vif_points* points, const double* y, const vif_kernel* kern, int32_t m,
                     const int32_t* nbr, double* nll, double* grad, void* ws, size_t ws_bytes,
                     void* hip_stream);

/* Workspace bytes for vif_nll_grad_vif (0 for invalid sizes; k >= 1). */
size_t vif_grad_vif_ws(int64_t n, int32_t m, int32_t k);

/* *nll (HOST) and grad (HOST, vif_grad_params(kern->kind) values, the order
 * above) of the VIF NLL (Sec. "The Vecchia-inducing-point full-scale
 * approximation"; the fit of Sec. "Estimation and prediction"), in FP64, for
 * neighbor rows nbr (as for vif_nll) and k = ind->n >= 1 inducing points; the
 * NLL equals vif_nll's in VIF_PREC_FP64. With W = D^-1/2 B U, z = D^-1/2 B y,
 * M = I + W'W, v = M^-1 W'z, e = z - W v and H = W M^-1 - e v', the derivative
 * is the sum over points of <Lambda_i, dC_S + dnugget I> (Lambda_i from the
 * point's residual-block factor, b = last row of its inverse, g_i = e_i y_S +
 * U_S H_i, w_i = R_S^-1 g_i: 1/2 (1 + b.g_i) b b' - 1/2 (b w_i' + w_i b')), plus
 * <Gamma L_k^-1, dC_nk> - <Phi(L_k^-1 dSigma_k L_k^-T), Gamma' U>, where Gamma
 * gathers b_r H_i - 2 (Lambda_i U_S)_r on the rows of U and Phi takes the lower
 * triangle with half the diagonal. Gamma is accumulated with FP64 atomics, so
 * the last bits can vary between calls. Workspace: vif_grad_vif_ws(n, m, k)
 * (about 5 n kpad + n q^2 doubles, kpad = k + 1 rounded up to 64, q = 32 for
 * m < 32, else 64). Synchronises the stream. */
int32_t vif_nll_grad_vif(const vif_points* points, const double* y, const vif_kernel* kern,
                         int32_t m, const int32_t* nbr, const vif_points* ind, double* nll,
                         double* grad, void* ws, size_t ws_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* VIF_GRAD_H */
