"""MI355X-native negacyclic NTT library (forward NTT, inverse NTT, pointwise
product) over word-size primes, batched over RNS limbs and polynomials.

The compute path is libntt.so (hand-written HIP for gfx950, C ABI in
include/ntt.h); this package only marshals arguments to it.
"""
from .ntt import (  # noqa: F401
    NTT_BATCH_NO_GRAPH,
    NTT_JOB_FORWARD,
    NTT_JOB_INVERSE,
    Batch,
    ntt_autotune,
    ntt_plan_get_variant_for,
    ntt_tune_clear,
    ntt_tune_load,
    ntt_tune_save,
    NTT_ORDER_BITREV,
    NTT_PATH_AUTO,
    NTT_PATH_FOURSTEP,
    NTT_PATH_LDS,
    NTT_PATH_TINY,
    NTT_WORD32,
    NttError,
    Plan,
    lib,
    library_path,
    ntt_forward,
    ntt_forward_stage,
    ntt_inverse,
    ntt_inverse_stage,
    ntt_last_error,
    ntt_plan_create,
    ntt_plan_create_ex,
    ntt_plan_destroy,
    ntt_plan_get_psi,
    ntt_plan_get_variant,
    ntt_plan_set_quotient,
    ntt_plan_set_variant,
    ntt_pointwise_mul,
    ntt_pointwise_mul_inverse,
    ntt_pointwise_mul_inverse_stage,
    ntt_strerror,
    ntt_workspace_bytes,
)
