"""MI355X (gfx950) solver for 2-D TE scattering by the domain-integral-equation
method of Zouros & Budko: FFT-speed products with the discretised operator A and
its regularizer A_R, and restarted GMRES (optionally regularized and deflated)
driving them, and a U-Net that proposes GMRES initial guesses.  Every step runs
in the HIP library libdie_te.so; this module only marshals PyTorch device
tensors into its C ABI (include/die_te.h, include/die_te_learn.h).
"""
from __future__ import annotations

from .api import (  # noqa: F401
    Solver,
    die_te_setup,
    die_te_setup_multi,
    die_te_matvec,
    die_te_matvec_noalloc,
    die_te_regularize,
    die_te_solve,
    die_te_apply_deflation,
    die_te_deflation_info,
    die_te_operator_dense,
    die_te_spectrum,
    die_te_fft2,
    die_te_destroy,
    die_te_deflation_radius,
    die_te_plan_memory,
    die_te_profile,
    die_te_profile_read,
    die_te_profile_mem,
    die_te_last_error,
    UNet,
    die_te_unet_create,
    die_te_unet_num_params,
    die_te_unet_get_params,
    die_te_unet_set_params,
    die_te_unet_get_grads,
    die_te_unet_forward,
    die_te_unet_loss_grad,
    die_te_unet_adam,
    die_te_unet_train_step,
    die_te_unet_pack_inputs,
    die_te_unet_pack_targets,
    die_te_warm_start,
    die_te_unet_destroy,
)
from ._lib import DieTeError, load  # noqa: F401
