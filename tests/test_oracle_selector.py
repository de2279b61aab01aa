"""Pins of the selector-side oracle: variant ranges against the paper's
examples, the RoundRobin/train-trigger state machine, the exhaustive
selector, the region features, and the FP64 MLP (finite differences, a
hand-computed sparse network, a hand Adam step, fitting a known cost)."""
import math

import numpy as np
import pytest


# ---- variants clause ranges (Sec. 3.1; Sec. 3.2 examples) -----------------

def test_range_examples_from_paper(orc):
    # [10:20:2] is the paper's own example: 10, 12, 14, 16, 18, 20
    assert orc.expand_range(10, 20, 2) == [10, 12, 14, 16, 18, 20]
    # GPU threads use case: [64:1024:64] -> 16 policies, GPU_THREADS = 64 + policy*64
    r = orc.expand_range(64, 1024, 64)
    assert len(r) == 16 and all(r[p] == 64 + p * 64 for p in range(16))
    # co-scheduling use case: [0.0:1.0:0.1] -> 11 policies, GPU_FRAC = 0.0 + policy*0.1
    f = orc.expand_range(0.0, 1.0, 0.1)
    assert len(f) == 11 and f[0] == 0.0 and f[10] == 1.0
    assert all(f[p] == 0.0 + p * 0.1 for p in range(11))
    with pytest.raises(ValueError):
        orc.expand_range(1, 0, 1)


# ---- RoundRobin exploration and train trigger ----------------------------

def test_roundrobin_cycles_and_trigger_at_num_variants(orc):
    ex = orc.RoundRobinExplorer(3)          # min_train unspecified -> V (Sec. 3.1)
    feats = [1.0, 2.0]
    assert ex.step(feats) == (0, False)
    assert ex.step(feats) == (1, False)
    assert ex.step(feats) == (2, True)      # third unique (features, variant)


def test_duplicates_do_not_count(orc):
    ex = orc.RoundRobinExplorer(3, min_train=5)
    out = [ex.step([7.0]) for _ in range(9)]
    assert [v for v, _ in out] == [0, 1, 2, 0, 1, 2, 0, 1, 2]
    assert not any(f for _, f in out)       # only 3 unique pairs ever


def test_trigger_counts_new_features(orc):
    ex = orc.RoundRobinExplorer(2, min_train=4)
    seq = [([1.0], (0, False)), ([1.0], (1, False)), ([1.0], (0, False)), ([2.0], (1, False)),
           ([2.0], (0, True))]
    for f, want in seq:
        assert ex.step(f) == want


# ---- exhaustive selector -------------------------------------------------

def test_exhaustive_median_argmin_and_ties(orc):
    t = [[3.0, 1.0, 2.0], [1.5, 9.0, 1.5], [1.5, 1.5, 100.0]]
    best, med = orc.exhaustive_select(t)
    assert med == [2.0, 1.5, 1.5] and best == 1      # tie 1 vs 2 -> lowest id
    best, _ = orc.exhaustive_select([[math.nan], [2.0], [1.0]])
    assert best == 2
    assert orc.regret(1.1, 1.0) == pytest.approx(0.1)


# ---- features ------------------------------------------------------------

def test_stencil_features_hand(orc):
    f = orc.stencil_features(64, 32, 16, 10, 1)
    nbytes = 16 * 64 * 32 * 16 * 10
    assert f.dtype == np.float32
    assert list(f) == [6.0, 5.0, 4.0, 10.0, np.float32(math.log2(nbytes)), 1.0]


def test_csr_features_hand(orc):
    rp = np.array([0, 2, 2, 8, 9], dtype=np.int32)   # lengths 2, 0, 6, 1
    f = orc.csr_features(rp)
    # mean 9/4, variance (0.25^2 + 2.25^2 + 3.75^2 + 1.25^2) / 4 = 20.75 / 4 = 5.1875
    assert f[0] == 2.0 and f[1] == np.float32(math.log2(9)) and f[2] == np.float32(2.25)
    assert f[3] == np.float32(math.log2(6.1875)) and f[4] == np.float32(math.log2(6))


# ---- MLP ------------------------------------------------------------------

def _toy_data(seed, B=7):
    import synth
    X = synth.u01(seed, B * 6).reshape(B, 6) * 2 - 1
    y = synth.u01(seed + 1, B) - 0.5
    v = (synth.u01(seed + 2, B) * 12).astype(int)
    mask = np.zeros((B, 12))
    mask[np.arange(B), v] = 1
    return X, y, mask


def test_param_count(orc):
    assert orc.N_PARAMS == 6 * 64 + 64 + 64 * 64 + 64 + 64 * 12 + 12 == 5388


def test_gradient_matches_central_differences(orc):
    theta = orc.mlp_init(5)
    X, y, mask = _toy_data(100)
    g, _ = orc.mlp_grad(theta, X, y, mask)
    rng_idx = np.unique(np.concatenate([np.arange(0, orc.N_PARAMS, 37), [orc.N_PARAMS - 1]]))
    h = 1e-6
    num = []
    for i in rng_idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        num.append((orc.mlp_loss(tp, X, y, mask) - orc.mlp_loss(tm, X, y, mask)) / (2 * h))
    num = np.array(num)
    rel = np.linalg.norm(num - g[rng_idx]) / np.linalg.norm(num)
    assert rel < 1e-7


def test_hand_computed_sparse_network(orc):
    # One active path: z1_0 = 2*x0 - 1 = 1, h2_0 = 3*h1_0 = 3, o_0 = 0.5*3 + 0.25 = 1.75.
    p = {k: np.zeros(s) for k, s in orc.SHAPES.items()}
    p["W1"][0, 0], p["b1"][0] = 2.0, -1.0
    p["W2"][0, 0] = 3.0
    p["W3"][0, 0], p["b3"][0] = 0.5, 0.25
    theta = orc.mlp_flatten(p)
    X = np.zeros((1, 6)); X[0, 0] = 1.0
    mask = np.zeros((1, 12)); mask[0, 0] = 1.0
    o, _ = orc.mlp_forward(theta, X)
    assert o[0, 0] == 1.75 and np.all(o[0, 1:] == 0.0)
    assert orc.mlp_loss(theta, X, [1.0], mask) == 0.5 * 0.75 ** 2
    g = orc.mlp_unflatten(orc.mlp_grad(theta, X, [1.0], mask)[0])
    # dO = 0.75; dW3 = dO*h2 = 2.25; dh2 = dO*0.5 = 0.375 -> dW2 = 0.375*h1 = 0.375;
    # dh1 = 0.375*3 = 1.125 -> dW1 = 1.125*x0; units with z = 0 pass no gradient.
    assert g["W3"][0, 0] == 2.25 and g["b3"][0] == 0.75
    assert g["W2"][0, 0] == 0.375 and g["b2"][0] == 0.375
    assert g["W1"][0, 0] == 1.125 and g["b1"][0] == 1.125
    assert np.count_nonzero(orc.mlp_flatten(g)) == 6


def test_first_adam_step_is_signed_lr(orc):
    # Step 1: m_hat = g, v_hat = g^2, so the update is lr * g / (|g| + eps).
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    th, m, v = orc.adam_step(theta, g, np.zeros(3), np.zeros(3), 1)
    assert np.allclose(th, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_fits_known_cost_and_selects_its_argmin(orc):
    # ln t = a_v + b_v * s for variants v = 0..2 on one feature s: the trained
    # model must rank variants as the true cost does.
    recs = []
    a = [0.0, 1.0, 2.0]
    b = [1.0, 0.5, 0.0]
    for s in np.linspace(0.0, 4.0, 41):
        for v in range(3):
            recs.append(([float(s)], v, math.exp(a[v] + b[v] * s)))
    ds = orc.build_dataset(recs, 3)
    theta, loss = orc.mlp_train(ds, seed=3, epochs=300, batch=32, lr=3e-3)
    assert loss < 1e-3
    for s in (0.5, 1.2, 2.7, 3.6):
        truth = int(np.argmin([a[v] + b[v] * s for v in range(3)]))
        assert orc.mlp_select(theta, ds, [s], 3) == truth


def test_dataset_merges_duplicates_by_median(orc):
    recs = [([1.0], 0, 1.0), ([1.0], 0, 3.0), ([1.0], 0, 2.0), ([2.0], 1, 4.0)]
    ds = orc.build_dataset(recs, 2)
    assert list(ds["seconds"]) == [2.0, 4.0] and list(ds["variant"]) == [0, 1]
    assert ds["y"].sum() == pytest.approx(0.0)


def test_adam_constant_gradient_every_step(orc):
    # Under a constant gradient g the moments are geometric sums:
    # m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the bias-corrected
    # m_hat = g and v_hat = g^2 at every t and each step moves theta by
    # lr * g / (|g| + eps).  A bias correction with b*t in place of b^t, or a
    # moment recursion with the weights swapped, already differs at t = 2.
    theta0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 1e-3, 2.5])
    step = 1e-3 * g / (np.abs(g) + 1e-8)
    theta, m, v = theta0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, 41):
        theta, m, v = orc.adam_step(theta, g, m, v, t)
        assert np.allclose(m, (1.0 - 0.9 ** t) * g, rtol=1e-13, atol=0)
        assert np.allclose(v, (1.0 - 0.999 ** t) * g * g, rtol=1e-12, atol=0)
        assert np.allclose(theta, theta0 - t * step, rtol=0, atol=1e-13 * t)


def test_adam_step_is_invariant_to_gradient_scale(orc):
    # m_hat scales with c and sqrt(v_hat) with |c|, so for c > 0 the update
    # is the same up to eps: a v built from g rather than g^2 breaks this.
    import synth
    theta0 = synth.u01(31, 8) - 0.5
    gs = [synth.u01(32 + k, 8) - 0.5 for k in range(5)]
    runs = []
    for c in (1.0, 64.0):
        th, m, v = theta0.copy(), np.zeros(8), np.zeros(8)
        for t, g in enumerate(gs, start=1):
            th, m, v = orc.adam_step(th, c * g, m, v, t)
        runs.append(th)
    assert np.allclose(runs[0], runs[1], rtol=0, atol=1e-9)
    assert not np.allclose(runs[0], theta0, rtol=0, atol=1e-4)


def test_dataset_zscore_and_std_floor(orc):
    # Three records on two features: feature 0 = 1, 2, 3 (mean 2, population
    # std sqrt(2/3)); feature 1 constant 10 (std 0, floored at 1e-6, so it
    # normalises to 0); the unused feature slots 2..5 are 0 and stay 0.
    recs = [([1.0, 10.0], 0, math.exp(1.0)), ([2.0, 10.0], 1, math.exp(2.0)),
            ([3.0, 10.0], 0, math.exp(3.0))]
    ds = orc.build_dataset(recs, 2)
    s = math.sqrt(2.0 / 3.0)
    assert np.allclose(ds["X"][:, 0], [-1.0 / s, 0.0, 1.0 / s], rtol=1e-15, atol=0)
    assert np.all(ds["X"][:, 1:] == 0.0)
    assert list(ds["mu"][:2]) == [2.0, 10.0] and ds["sd"][0] == pytest.approx(s, rel=1e-15)
    assert np.all(ds["sd"][1:] == 1e-6)
    assert np.allclose(ds["y"], [-1.0, 0.0, 1.0], rtol=0, atol=1e-15)
    assert ds["y_mean"] == pytest.approx(2.0, rel=1e-15)
    assert ds["mask"].tolist() == [[1.0 if v == w else 0.0 for v in range(12)] for w in (0, 1, 0)]
    # a spread below the floor: 0, 2^-24, 2^-23 have population std
    # 2^-24 * sqrt(2/3) < 1e-6, so they divide by the floor
    tiny = [([0.0], 0, 1.0), ([2.0 ** -24], 0, 1.0), ([2.0 ** -23], 0, 1.0)]
    X = orc.build_dataset(tiny, 1)["X"][:, 0]
    assert np.allclose(X, [-2.0 ** -24 / 1e-6, 0.0, 2.0 ** -24 / 1e-6], rtol=1e-14, atol=0)


def test_mlp_init_he_uniform(orc):
    # He-uniform: W ~ U(-sqrt(6/fan_in), +sqrt(6/fan_in)) with fan_in the
    # layer's input width (6, 64, 64), variance 2/fan_in; biases zero.
    p = orc.mlp_unflatten(orc.mlp_init(11))
    for w, fan_in in (("W1", 6), ("W2", 64), ("W3", 64)):
        bound = math.sqrt(6.0 / fan_in)
        a = p[w].reshape(-1)
        assert np.all(np.abs(a) < bound)
        assert np.max(np.abs(a)) > 0.9 * bound          # the draws fill the interval
        assert abs(np.var(a) / (2.0 / fan_in) - 1.0) < 0.15
        assert abs(np.mean(a)) < 0.15 * bound
    for b in ("b1", "b2", "b3"):
        assert np.all(p[b] == 0.0)
    assert not np.array_equal(orc.mlp_init(11), orc.mlp_init(12))
    assert np.array_equal(orc.mlp_init(11), orc.mlp_init(11))
