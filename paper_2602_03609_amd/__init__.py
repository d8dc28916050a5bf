"""MI355X (gfx950) library for the Vecchia / VIF approximate negative
log-likelihood of non-separable space-time Gaussian processes (arXiv 2602.03609).

The compute path is the HIP library libvif.so (C ABI in include/vif.h); this
package holds its build script and a thin ctypes binding with the same names.
"""
from ._lib import (  # noqa: F401
    Batch,
    VIF_E_ARG,
    VIF_E_NOT_PD,
    VIF_OK,
    VifError,
    VIF_KERNEL_GNEITING,
    VIF_KERNEL_GNEITING_MATERN,
    VIF_KERNEL_MATERN_ANISO,
    VIF_OP_FACTOR,
    VIF_OP_NEIGHBORS,
    VIF_OP_NEIGHBORS_NLL,
    VIF_OP_NLL,
    VIF_PREC_BF16X3,
    VIF_PREC_BF16X6,
    VIF_PREC_FP32,
    VIF_PREC_FP64,
    load,
    release_workspaces,
    vif_factor,
    vif_mlp_adam,
    vif_mlp_backward,
    vif_mlp_batch,
    vif_mlp_features,
    vif_mlp_forward,
    vif_mlp_pair_loss,
    vif_neighbors,
    vif_neighbors_nll,
    vif_neighbors_noalloc,
    vif_nll,
    vif_nll_grad,
    vif_nll_terms,
    vif_profile,
    vif_profile_read,
    vif_propose_neighbors,
    vif_residual_neighbors,
    vif_workspace_bytes,
)
