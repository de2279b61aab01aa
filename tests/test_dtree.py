"""The decision-tree comparator (the paper's own model): oracle pins, then
the library's host CART against the oracle on the same records (no GPU)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import synth


def test_oracle_single_threshold_by_hand(orc):
    X = [[float(x)] for x in range(10)]
    y = [0 if x < 5 else 1 for x in range(10)]
    t = orc.dtree_fit(X, y, 2, 2)
    assert t["feature"] == 0 and t["threshold"] == 4.5
    assert t["left"]["counts"] == [5, 0] and t["right"]["counts"] == [0, 5]
    assert orc.dtree_predict(t, [4.4]) == 0 and orc.dtree_predict(t, [4.6]) == 1


def test_oracle_xor_needs_depth_two(orc):
    X = [[a, b] for a in (0.0, 1.0) for b in (0.0, 1.0) for _ in range(3)]
    y = [int(a) ^ int(b) for a, b in X]
    deep = orc.dtree_fit(X, y, 2, 2)
    assert all(orc.dtree_predict(deep, x) == t for x, t in zip(X, y))
    stump = orc.dtree_fit(X, y, 1, 2)
    acc = np.mean([orc.dtree_predict(stump, x) == t for x, t in zip(X, y)])
    assert acc == 0.5


def test_oracle_stump_is_brute_force_optimal(orc):
    # every (feature, threshold) split, impurity from class proportions
    X = (synth.u01(5, 30 * 3).reshape(30, 3) * 8).round(1).tolist()
    y = (synth.u01(6, 30) * 3).astype(int).tolist()
    t = orc.dtree_fit(X, y, 1, 3)

    def imp(part):
        if not part:
            return Fraction(0)
        return 1 - sum(Fraction(part.count(k), len(part)) ** 2 for k in range(3))
    best = None
    for f in range(3):
        for thr in sorted(set(r[f] for r in X)):
            L = [c for r, c in zip(X, y) if r[f] <= thr]
            R = [c for r, c in zip(X, y) if r[f] > thr]
            if not L or not R:
                continue
            g = Fraction(len(L), 30) * imp(L) + Fraction(len(R), 30) * imp(R)
            best = g if best is None else min(best, g)
    L = [c for r, c in zip(X, y) if r[t["feature"]] <= t["threshold"]]
    R = [c for r, c in zip(X, y) if r[t["feature"]] > t["threshold"]]
    assert Fraction(len(L), 30) * imp(L) + Fraction(len(R), 30) * imp(R) == best


def test_label_records_median_and_ties(orc):
    recs = [([1.0], 0, 3.0), ([1.0], 1, 2.0), ([1.0], 1, 9.0), ([1.0], 1, 1.0), ([1.0], 2, 2.0),
            ([2.0], 0, 1.0), ([2.0], 1, 1.0)]
    X, y = orc.label_records(recs, 3)
    assert X == [[1.0], [2.0]] and y == [1, 0]   # medians 3, 2, 2 -> 1 ; tie 1 vs 1 -> 0


@pytest.mark.parametrize("seed,depth", [(11, 2), (12, 2), (13, 3), (14, 1)])
def test_library_tree_matches_oracle(orc, seed, depth):
    import paper_2303_08873_amd as ao
    V = 5
    n = 60
    F = synth.u01(seed, n * 3).reshape(n, 3)
    F = np.round(F * 6, 1)                     # repeated values -> ties in splits
    recs = []
    for q in range(n):
        f = [float(F[q, 0]), float(F[q, 1]), float(F[q, 2]), 1.0, 2.0, 0.0]
        base = np.array([F[q, 0], 6 - F[q, 0], F[q, 1], 3.0, 1.0 + F[q, 2]])
        noise = synth.u01(seed * 100 + q, V)
        for v in range(V):
            recs.append((f, v, float(math.exp(0.3 * base[v] + 0.2 * noise[v]))))
    mt = "dtree" if depth == 2 else f"dtree,{depth}"
    h = ao.region_declare_variants(f"dt_{seed}_{depth}", ao.AO_JACOBI7_F64,
                                   ao.jacobi_sweep_host(), min_train_data=10 ** 6,
                                   model_type=mt)
    for f, v, t in recs:
        ao.region_record(h, f, v, t)
    err = ao.selector_train(h)
    X, y = orc.label_records(recs, V)
    tree = orc.dtree_fit(X, y, depth, V)
    train_err = np.mean([orc.dtree_predict(tree, x) != t for x, t in zip(X, y)])
    assert err == pytest.approx(train_err, abs=1e-12)
    Q = (synth.u01(seed + 7, 200 * 3).reshape(200, 3) * 6.4 - 0.2).tolist()
    queries = [[a, b, c, 1.0, 2.0, 0.0] for a, b, c in Q] + X
    rc, ids = ao.selector_select(h, queries)
    assert rc == 0
    assert ids == [orc.dtree_predict(tree, qv) for qv in queries]
    ao.region_destroy(h)
