"""The learned selector against the method without it, on a small instance
of the evaluation pipeline: RoundRobin-profiled training runs, GPU
training, an exhaustive held-out table.  The trained network must beat the
untrained one and the static default, and selecting must cost at least 10x
less than timing every variant."""
import pytest

pytestmark = pytest.mark.gpu


def test_learned_selector_gain():
    # shapes up to 160 per side: large enough that the fastest variant
    # depends on the shape (small grids alone are launch-bound, where every
    # GPU variant times alike and the comparison would measure noise)
    from paper_2303_08873_amd import evaluate
    r = evaluate.run(n_train=160, n_test=80, max_dim=160, reps=5, epochs=200)
    learned, untrained, static = r["learned"], r["untrained_net"], r["static_default"]
    assert learned["geomean_regret_pct"] <= untrained["geomean_regret_pct"]
    assert learned["geomean_regret_pct"] <= static["geomean_regret_pct"] + 1.0
    assert learned["geomean_regret_pct"] <= 25.0
    assert r["selection_cost_ratio_median"] >= 10.0
