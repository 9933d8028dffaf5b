"""MI355X (gfx950) direct-summation N-body library: the softened pairwise
gravity of Eq. (1) inside a kick-drift-kick leapfrog, with precision
policies, FP64 diagnostics and a hand-written adjoint.

The compute path is libnbody.so (hand-written HIP kernels behind the C ABI
of include/nbody.h); this package is its thin Python binding. Importing it
does not load the library; the first call does, and raises if it is not
built.
"""

from ._lib import PREC, NBodyError, nb_launch  # noqa: F401
from .api import (accel, step, step_adjoint, diag, diag_dict, device_info, graph_cache_clear,  # noqa: F401
                  pass_info,
                  workspace_size, pos_dtype, mass_dtype, DIAG_FIELDS)
from .autograd import NBodyRollout, rollout  # noqa: F401
