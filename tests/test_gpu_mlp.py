"""GPU cost-model kernels against the FP64 oracle MLP, through the C ABI:
forward, gradient (normwise relative <= 1e-4), one Adam step, and the
learned selector trained on the GPU from profile records of a known cost."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2303_08873_amd as ao
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda:0")
    return ao, torch, dev, torch.cuda.current_stream(dev)


def _data(B, seed):
    X = (synth.u01(seed, B * 6).reshape(B, 6) * 4 - 2)
    y = synth.u01(seed + 1, B) * 2 - 1
    v = (synth.u01(seed + 2, B) * 12).astype(np.int64)
    mask = np.zeros((B, 12))
    mask[np.arange(B), v] = 1.0
    return X, y, mask


def _f32(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


@pytest.mark.parametrize("B", [1, 17, 64, 200, 256])
def test_forward_matches_oracle(env, orc, B):
    ao, torch, dev, st = env
    theta = orc.mlp_init(11).astype(np.float32).astype(np.float64)
    X, _, _ = _data(B, 5 + B)
    X = X.astype(np.float32).astype(np.float64)
    want, _ = orc.mlp_forward(theta, X)
    out = torch.empty(B * 12, dtype=torch.float32, device=dev)
    ao.ao_mlp_forward(_f32(torch, dev, theta), _f32(torch, dev, X), B, out, stream=st)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(B, 12).astype(np.float64)
    assert np.linalg.norm(got - want) <= 1e-5 * np.linalg.norm(want)


@pytest.mark.parametrize("B", [1, 40, 64, 130, 256])
def test_gradient_matches_oracle(env, orc, B):
    ao, torch, dev, st = env
    theta = orc.mlp_init(21).astype(np.float32).astype(np.float64)
    X, y, mask = _data(B, 100 + B)
    X = X.astype(np.float32).astype(np.float64)
    y = y.astype(np.float32).astype(np.float64)
    want_g, want_loss = orc.mlp_grad(theta, X, y, mask)
    grad = torch.full((ao.AO_MLP_PARAMS,), float("nan"), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ao.ao_mlp_grad(_f32(torch, dev, theta), _f32(torch, dev, X), _f32(torch, dev, y),
                   _f32(torch, dev, mask), B, grad, loss, stream=st)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(g)), "every parameter gradient must be written"
    assert np.linalg.norm(g - want_g) <= 1e-4 * np.linalg.norm(want_g)
    assert abs(float(loss.item()) - want_loss) <= 1e-4 * abs(want_loss)
    # per-layer check: a transposed or misplaced block would show here
    for k, sl in _slices(orc).items():
        ref = want_g[sl]
        if np.linalg.norm(ref) > 0:
            assert np.linalg.norm(g[sl] - ref) <= 1e-4 * np.linalg.norm(ref), k


def _slices(orc):
    out, o = {}, 0
    for k, s in orc.SHAPES.items():
        n = int(np.prod(s))
        out[k] = slice(o, o + n)
        o += n
    return out


def test_adam_step_matches_oracle(env, orc):
    ao, torch, dev, st = env
    theta = orc.mlp_init(3).astype(np.float32).astype(np.float64)
    X, y, mask = _data(64, 7)
    g, _ = orc.mlp_grad(theta, X, y, mask)
    g = g.astype(np.float32).astype(np.float64)
    m0 = (synth.u01(40, theta.size) * 0.01).astype(np.float32).astype(np.float64)
    v0 = (synth.u01(41, theta.size) * 1e-4).astype(np.float32).astype(np.float64)
    want, wm, wv = orc.adam_step(theta, g, m0, v0, 5, lr=1e-3)
    p = _f32(torch, dev, theta)
    m = _f32(torch, dev, m0)
    v = _f32(torch, dev, v0)
    ao.ao_mlp_adam(p, m, v, _f32(torch, dev, g), 5, 1e-3, stream=st)
    torch.cuda.synchronize()
    assert np.linalg.norm(p.cpu().numpy() - want) <= 1e-4 * np.linalg.norm(want - theta) + 1e-7
    # normwise: 0.9 m + 0.1 g cancels for some entries, so single elements of
    # the FP32 result can carry a large relative error
    assert np.linalg.norm(m.cpu().numpy() - wm) <= 1e-5 * np.linalg.norm(wm)
    assert np.linalg.norm(v.cpu().numpy() - wv) <= 1e-5 * np.linalg.norm(wv)


def _known_cost(f):
    # ln t of 4 variants, linear in two features: crossovers inside the range
    a = np.array([0.0, 1.0, 2.0, 0.5])
    b = np.array([1.0, 0.5, 0.0, 0.8])
    c = np.array([0.0, 0.3, -0.2, 0.6])
    return a + b * f[0] + c * f[1]


def test_selector_learns_known_cost(env, orc):
    ao, torch, dev, st = env
    h = ao.region_declare_variants("gpu_sel", ao.AO_JACOBI7_F64, ao.jacobi_variants_sweep()[:4],
                                   min_train_data=100000)
    recs = []
    grid = np.linspace(0.0, 4.0, 21)
    for f0 in grid:
        for f1 in grid[::2]:
            f = [float(f0), float(f1), 0, 0, 0, 0]
            lt = _known_cost(f)
            for v in range(4):
                ao.region_record(h, f, v, float(math.exp(lt[v])))
                recs.append((f, v, float(math.exp(lt[v]))))
    loss = ao.selector_train(h, epochs=300, batch=64, lr=3e-3, seed=3)
    assert loss < 5e-3
    st_ = ao.region_stats(h)
    assert st_.trained == 1 and st_.trainings == 1
    test = [[float(x), float(y), 0, 0, 0, 0] for x, y in
            zip(synth.u01(77, 300) * 4, synth.u01(78, 300) * 4)]
    rc, ids = ao.selector_select(h, test)
    assert rc == 0
    t_sel = np.array([math.exp(_known_cost(f)[i]) for f, i in zip(test, ids)])
    t_best = np.array([math.exp(_known_cost(f).min()) for f in test])
    regret_gpu = float(np.exp(np.mean(np.log(t_sel / t_best))) - 1)
    # the FP64 oracle trained on the same records
    ds = orc.build_dataset(recs, 4)
    theta, _ = orc.mlp_train(ds, seed=3, epochs=300, batch=64, lr=3e-3)
    ids_o = [orc.mlp_select(theta, ds, f, 4) for f in test]
    t_o = np.array([math.exp(_known_cost(f)[i]) for f, i in zip(test, ids_o)])
    regret_orc = float(np.exp(np.mean(np.log(t_o / t_best))) - 1)
    assert regret_gpu <= 0.02
    assert abs(regret_gpu - regret_orc) <= 0.01
    # batch of one and memo-free repeat give the same ids
    for f, i in list(zip(test, ids))[:10]:
        assert ao.selector_select(h, [f])[1] == [i]
    ao.region_destroy(h)
