"""MI355X-native NTT and Groth16 quotient library (Python binding).

The compute path is the HIP library ``libzkntt.so`` built from ``csrc/``
(``python -m paper_2509_22684_amd.build``).  This package only marshals
arguments to its C ABI (``include/zkntt.h``): torch tensors supply device
memory and streams, and every step of every transform runs in the library's
kernels.  There is no fallback: if the library is missing, importing the
binding raises.
"""
from ._lib import (  # noqa: F401
    FIELDS,
    Batch,
    MsmBases,
    ntt_batch_create,
    ntt_batch_create_jobs,
    ntt_batch_destroy,
    ntt_batch_forward,
    ntt_batch_launch,
    ntt_batch_launch_eager,
    ntt_batch_set_spin_limit,
    ntt_batch_status,
    ntt_batch_workspace_bytes,
    Plan,
    ZkError,
    ZK_FLAG_FFMUL_FP64,
    ZK_FLAG_VALIDATE,
    lib,
    ntt_coset_forward,
    ntt_coset_inverse,
    ntt_forward,
    ntt_inverse,
    ntt_plan_create,
    ntt_plan_destroy,
    ntt_plan_get_opts,
    ntt_plan_resolve_opts,
    ntt_plan_table_bytes,
    ntt_tuning_clear,
    ntt_tuning_register,
    register_tuning_db,
    ntt_plan_device_bytes,
    ntt_plan_passes,
    ntt_profile_passes,
    ntt_workspace_bytes,
    quotient_coset_evals,
    quotient_poly,
    quotient_pointwise,
    quotient_workspace_bytes,
    zk_copy_to_host,
    zk_microbench,
    zk_field_mul,
    ntt_forward_noalloc,
    zk_last_error,
)
