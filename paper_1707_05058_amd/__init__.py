"""MI355X-native chordal-decomposed primal ADMM for sparse SDPs.

The solver (Algorithm 1 of Zheng, Fantuzzi, Papachristodoulou, Goulart and
Wynn, "Chordal decomposition in operator-splitting methods for sparse
semidefinite programs") runs entirely in hand-written HIP kernels for gfx950
behind the C ABI of include/sdp.h; this package is its thin Python binding.
"""
from ._native import (A_CSR, A_DENSE, ALG_DUAL, ALG_HSDE, ALG_PRIMAL, DTYPE_FP32, DTYPE_FP64,
                      DUAL_INFEASIBLE, EXPORTS, PRIMAL_INFEASIBLE,
                      FP32_EIG, FP64,
                      SdpError, Solver, default_options, lib, make_options, pack_blocks,
                      projection_default_variant, projection_variant_kind, projection_variant_two_level,
                      projection_variants, psd_project_batched,
                      sdp_result, setup_status, sign_schedule,
                      unpack_blocks)
from .preprocess import (ChordalPattern, InstanceData, Scaling, chordal_extension,
                         extend_instance, scale_instance)

__all__ = ["Solver", "SdpError", "psd_project_batched", "projection_variants",
           "projection_default_variant", "sign_schedule",
           "projection_variant_kind", "projection_variant_two_level", "setup_status",
           "make_options",
           "default_options", "pack_blocks", "unpack_blocks", "lib", "EXPORTS", "FP64",
           "FP32_EIG", "DTYPE_FP32", "DTYPE_FP64", "A_DENSE", "A_CSR", "ALG_PRIMAL", "ALG_DUAL", "ALG_HSDE",
           "PRIMAL_INFEASIBLE", "DUAL_INFEASIBLE",
           "sdp_result", "ChordalPattern", "InstanceData", "Scaling", "chordal_extension",
           "extend_instance", "scale_instance"]
