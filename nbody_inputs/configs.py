"""The five synthetic N-body workloads and their seeded inputs.

Every constant that is not an integer (1/N for N a power of two, the
softening eps and the step dt) is a power of two, so none of them is rounded
when it is handed to FP32 or FP64 code.

Readings where the workload description is silent:

* ``scale-2^20`` and ``subcluster-262144`` give no step size; dt = eps / 2,
  the ratio used by the other three workloads, is taken.
* ``subcluster-262144`` counts 262144 particles in total: 26214 (10 %) in the
  subcluster, 235930 in the main sphere, all of mass 1/262144.
* ``adjoint-16384`` targets are the end positions of an FP64 run of the same
  number of steps from the initial state perturbed by N(0, 1e-3) in every
  position and velocity component (seed 44; masses unperturbed). The targets
  are produced by whoever needs them (the tests use the CPU oracle); this
  module only draws the perturbation.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .plummer import plummer_sphere, plummer_with_subcluster


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    seed: int
    eps: float
    dt: float
    steps: int
    precisions: tuple
    G: float = 1.0
    ckpt_every: int = 0          # adjoint checkpoint interval (0: no adjoint)
    perturb_seed: int = 0
    perturb_sigma: float = 0.0
    sub_seed: int = 0            # subcluster seed (0: plain Plummer sphere)
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "fp64-1024": Workload("fp64-1024", 1024, 1, 2.0 ** -6, 2.0 ** -7, 10, ("f64",)),
    "fp32-65536": Workload("fp32-65536", 65536, 2, 2.0 ** -8, 2.0 ** -9, 100, ("f32",)),
    "subcluster-262144": Workload("subcluster-262144", 262144, 3, 2.0 ** -9, 2.0 ** -10, 20,
                                  ("mix_acc32", "mix_kahan", "mix_acc64", "mix_tilec"),
                                  sub_seed=33),
    "adjoint-16384": Workload("adjoint-16384", 16384, 4, 2.0 ** -7, 2.0 ** -8, 200,
                              ("mix_tilec",), ckpt_every=20, perturb_seed=44,
                              perturb_sigma=1e-3),
    "scale-2^20": Workload("scale-2^20", 1 << 20, 5, 2.0 ** -10, 2.0 ** -11, 10,
                           ("mix_tilec",), ckpt_every=20),
}


def make_state(w: Workload | str, n: int | None = None):
    """Initial (x, v, m) for a workload; ``n`` overrides the particle count
    (same seed and recipe) for scaled-down test cases."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    n = w.n if n is None else int(n)
    if w.sub_seed:
        return plummer_with_subcluster(n, w.seed, w.sub_seed)
    return plummer_sphere(n, w.seed)


def perturb_state(x, v, seed: int, sigma: float):
    """x, v plus independent N(0, sigma^2) noise in every component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dx = rng.normal(0.0, sigma, size=x.shape)
    dv = rng.normal(0.0, sigma, size=v.shape)
    return x + dx, v + dv


def random_unit_vectors(shape, seed: int):
    """A seeded random array of the given shape, scaled to unit 2-norm."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.normal(size=shape)
    return u / np.linalg.norm(u)
