"""FP64 CPU oracle for the direct-summation N-body hot path.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg to check and time the GPU library, never by the
GPU library itself. It shares no code with it.
"""

from .oracle import (accel, accel_sampled, kdk, diag, vjp, vjp_sampled, jvp, adjoint, diffusion3d,
                     num_threads, set_num_threads, DIAG_FIELDS)

__all__ = ["accel", "accel_sampled", "kdk", "diag", "vjp", "vjp_sampled", "jvp", "adjoint", "diffusion3d",
           "num_threads", "set_num_threads", "DIAG_FIELDS"]
