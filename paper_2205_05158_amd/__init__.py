"""MI355X-native TDNN DPD -> GMP PA cascade (arXiv 2205.05158): HIP kernels for
gfx950 behind the C ABI of include/dpdmi.h, a ctypes binding and a
torch.autograd.Function for direct-learning training steps."""
from ._lib import (DPD_BF16, DPD_ERR_NONFINITE, DPD_FP32, DPD_IMPL_PLAIN, DPD_IMPL_TUNED, DPD_NMSE_FIELDS,
                   DPD_OK, EXPORTS, LIB_PATH, Batch, dpd_nmse_status, dpd_symbol_mse,
                   dpd_symbol_mse_workspace_size,
                   GmpDesc, TdnnDesc, cascade_acpr, cascade_nmse, dpd_acpr_workspace_size,
                   dpd_adam_step, dpd_autotune, dpd_backward, dpd_cascade, dpd_cascade_clip, dpd_forward,
                   dpd_gmp_coeff_count, dpd_profile_enable, dpd_profile_report, dpd_tdnn_param_count, dpd_tune_get,
                   dpd_tune_set, dpd_version, dpd_workspace_size, fdcnn_backward, fdcnn_forward,
                   fdcnn_param_count, fdcnn_workspace_size, gmp_desc, gmp_ls_fit,
                   gmp_ls_workspace_size, lib, make_batch, pa_clip_forward, pa_gmp_forward, status_string,
                   tdnn_desc)
from .cascade import Cascade, CascadeFn, ClipCascade
from .ila import GmpIla
from .fdcnn import FdCnn, FdCnnFn
from .downlink import (Downlink, FdNn, FdNnFn, receiver_loss_grad, receiver_loss_grad_fdcnn,
                       train_receiver)

__all__ = [
    "DPD_BF16", "DPD_ERR_NONFINITE", "DPD_FP32", "DPD_IMPL_PLAIN", "DPD_IMPL_TUNED", "DPD_NMSE_FIELDS",
    "DPD_OK", "EXPORTS", "LIB_PATH", "Batch", "dpd_nmse_status", "dpd_symbol_mse",
    "dpd_symbol_mse_workspace_size",
    "GmpDesc", "TdnnDesc", "cascade_acpr", "cascade_nmse", "dpd_acpr_workspace_size",
    "dpd_adam_step", "dpd_autotune", "dpd_backward", "dpd_cascade", "dpd_cascade_clip", "dpd_forward", "dpd_gmp_coeff_count",
    "dpd_tdnn_param_count", "dpd_tune_get", "dpd_tune_set", "dpd_profile_enable", "dpd_profile_report",
    "dpd_version", "dpd_workspace_size", "fdcnn_backward", "fdcnn_forward", "fdcnn_param_count",
    "fdcnn_workspace_size", "gmp_desc", "gmp_ls_fit", "gmp_ls_workspace_size", "lib",
    "make_batch", "pa_clip_forward", "pa_gmp_forward", "status_string", "tdnn_desc", "Cascade",
    "CascadeFn", "ClipCascade", "GmpIla",
    "FdCnn", "FdCnnFn", "Downlink", "FdNn", "FdNnFn", "receiver_loss_grad",
    "receiver_loss_grad_fdcnn", "train_receiver",
]
