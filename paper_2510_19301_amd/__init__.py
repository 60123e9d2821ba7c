"""FLASH Viterbi decoding on MI355X (gfx950): HIP kernels behind a C ABI.

The compute path lives in libflashviterbi.so (built from csrc/ by
``paper_2510_19301_amd.build.build()``); this package only marshals torch
tensors into its C entry points.
"""
from ._lib import (FV_OK, FV_E_INVALID_ARG, FV_E_UNSUPPORTED, FV_E_WORKSPACE, FV_E_DEVICE,
                   FV_E_INFEASIBLE, FV_W_BEAM_FALLBACK, FvError, lib)
from .decode import (Batch, CsrModel, GaussEmission, decode, decode_batch, dense_model, model_descriptor,
                     workspace_bytes, workspace_bytes_models)
from .autograd import ViterbiScore, backward_workspace_bytes, viterbi_backward
from .tune import best_parallelism, tune

__all__ = ["FV_OK", "FV_E_INVALID_ARG", "FV_E_UNSUPPORTED", "FV_E_WORKSPACE", "FV_E_DEVICE",
           "FV_E_INFEASIBLE", "FV_W_BEAM_FALLBACK", "FvError", "lib", "Batch", "CsrModel", "GaussEmission",
           "decode", "decode_batch", "dense_model", "model_descriptor", "workspace_bytes", "workspace_bytes_models",
           "ViterbiScore", "viterbi_backward", "backward_workspace_bytes", "best_parallelism", "tune"]
