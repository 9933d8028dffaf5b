"""The tuner's sweep contains the library's own choice (host-side: the
library's shape rules through nbody_pass_info, which needs no device, and
the tuner's candidate list), for every policy with a symmetric pass, both
pair passes and sizes across every threshold of the rules."""

import pytest

import paper_2411_18889_amd as nb
from paper_2411_18889_amd import tune

SIZES = (12288, 20000, 24576, 40077, 49152, 65536, 81920, 98304, 131072, 163840, 1 << 18,
         1 << 20, 1 << 22)


@pytest.mark.parametrize("prec", tune.SYM_PRECS)
@pytest.mark.parametrize("op", ("force", "adjoint"))
def test_sweep_contains_the_library_shape(op, prec):
    code = 1 if op == "force" else 2
    for n in SIZES:
        info = nb.pass_info(code, n, prec)
        assert info["symmetric"] == 1, (op, prec, n)
        lib = {"i_per_lane": info["i_per_lane"], "block": info["block"], "split": 0,
               "symmetric": 1}
        assert lib in tune.candidate_shapes(op, n, prec, True), (op, prec, n, lib)
