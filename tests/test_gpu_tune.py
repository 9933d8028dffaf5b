"""The launch-shape tuner (the paper's per-machine NTHREADS survey,
generalised): on a small set of shapes it times each one, checks each
against the library's own result, and reports the fastest."""

import pytest

from paper_2411_18889_amd import tune

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ("mix_tilec", "f64"))
def test_tuner_reports_the_fastest_checked_shape(prec):
    shapes = [(1, 256, 1), (2, 128, 4), (1, 64, 16)]
    r = tune.tune(4096, prec, shapes=shapes, reps=3)
    assert r["n"] == 4096 and r["prec"] == prec
    best = (r["best"]["i_per_lane"], r["best"]["block"], r["best"]["split"])
    assert best in shapes
    assert r["best_ms"] > 0 and r["library_ms"] > 0
    assert r["best_ms"] == min(row["ms"] for row in r["top5"])
    assert len(r["top5"]) == len(shapes)
