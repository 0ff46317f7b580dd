"""librotseq: sequences of plane rotations applied to a matrix on MI355X.

The compute path is the HIP library ``librotseq.so`` (built by
``python -m paper_2412_01852_amd.build``); this package only marshals
arguments to its C ABI (``include/rotseq.h``).  Importing the package loads
nothing; the first call does, and fails loudly if the library is missing.
"""
from ._lib import (  # noqa: F401
    RotseqError, Options, ARITH_AUTO, ARITH_EXACT, ARITH_FMA, ARITH_LIFT,
    KERNEL_AUTO, KERNEL_MULTIPASS, KERNEL_CHAIN, KERNEL_MFMA,
    rotseq, rotseq_noalloc, reflseq, refl3seq, refl3_workspace_bytes, check_args, workspace_bytes, strerror, version, library_path,
    device_colmajor, host_colmajor, profile_enable, profile_read, device_status,
    STATUS_NOT_ORTHOGONAL, test_set_waits, fp64_ceiling, launch_describe,
    Problem, BatchInfo, Batch, batched, Server, ServerConfig, ServerStats, SweepInfo,
)
