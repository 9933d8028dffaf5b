"""Helpers shared by the GPU tests: device tensors from the seeded numpy
inputs, the relative-error metrics and the oracle sampling."""

import numpy as np
import torch

import paper_2411_18889_amd as nb

DEV = torch.device("cuda:0")

# tolerances from the accuracy targets: relative acceleration error (global
# 2-norm over all components) of 1e-5 for the FP32 pair arithmetic and 1e-12
# for FP64
TOL = {"f64": 1e-12, "f32": 1e-5, "mix_acc32": 1e-5, "mix_kahan": 1e-5, "mix_acc64": 1e-5,
       "mix_tilec": 1e-5}
PRECS = ("f64", "f32", "mix_acc32", "mix_kahan", "mix_acc64", "mix_tilec")


def to_dev(x, v, m, prec):
    pdt, mdt = nb.pos_dtype(prec), nb.mass_dtype(prec)
    return (torch.tensor(x, dtype=pdt, device=DEV), torch.tensor(v, dtype=pdt, device=DEV),
            torch.tensor(m, dtype=mdt, device=DEV))


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    nb_ = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb_) if nb_ > 0 else float(np.linalg.norm(a - b))


def per_particle(a, b):
    """median, p99 and max of |a_i - b_i| / |b_i|."""
    e = np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)
    return float(np.median(e)), float(np.quantile(e, 0.99)), float(e.max())


def sample_indices(x, count, central, seed, centres=()):
    """`count` seeded random particles plus the `central` ones nearest the
    centre of mass (where |a| is smallest and the relative error largest)
    and the `central` ones nearest each extra point of `centres` (a cluster
    core, where close pairs are densest)."""
    n = x.shape[1]
    rng = np.random.default_rng(seed)
    idx = rng.choice(n, size=min(count, n), replace=False)
    parts = [idx]
    for c in [x.mean(axis=1)] + [np.asarray(c, dtype=np.float64) for c in centres]:
        r = np.linalg.norm(x - c[:, None], axis=0)
        parts.append(np.argsort(r)[:central])
    return np.unique(np.concatenate(parts))


def cluster_centres(name, x):
    """Cluster cores of a workload beyond its centre of mass: for the
    subcluster workload, the centroid of the subcluster (its particles come
    last, round(n / 10) of them)."""
    from nbody_inputs import WORKLOADS
    if not WORKLOADS[name].sub_seed:
        return ()
    n = x.shape[1]
    n_sub = int(round(0.1 * n))
    return (x[:, n - n_sub:].mean(axis=1),)
