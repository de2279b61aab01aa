"""Runtime paths that need the GPU: the train trigger firing inside
region_run, the trained model's round trip through save/load, the
out-of-range fallback, the exhaustive producer, and lazily harvested
timings."""
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


def _grid(torch, dev, n, seed):
    u0 = synth.grid_u01_torch(n, n, n, seed=seed, device=dev)
    return u0, torch.empty_like(u0)


def test_trigger_trains_inside_region_run_and_model_takes_over(env, orc):
    ao, torch, dev, st = env
    vs = ao.jacobi_variants_blocks()
    h = ao.region_declare_variants("rt_trigger", ao.AO_JACOBI7_F64, vs)  # min_train = 3
    grids = {n: _grid(torch, dev, n, 10 + n) for n in (16, 24, 32)}
    ex = orc.RoundRobinExplorer(3)
    fired = None
    for k, n in enumerate([16, 16, 16, 24, 24]):
        u0, out = grids[n]
        rc, v = ao.region_run(h, ao.jacobi_args(u0, out, n, n, n, 3), stream=st)
        f = orc.stencil_features(n, n, n, 3, 1)
        if fired is None:
            want_v, fire = ex.step(f)
            assert v == want_v and rc == ao.AO_NOTE_UNTRAINED
            if fire:
                fired = k
                assert ao.region_stats(h).trained == 1
        else:
            assert rc in (ao.AO_OK, ao.AO_NOTE_FALLBACK)
    assert fired == 2
    torch.cuda.synchronize()
    u0, out = grids[24]
    assert np.array_equal(out.cpu().numpy(), orc.jacobi7(u0.cpu().numpy(), 24, 24, 24, 3))
    _, seconds = ao.region_records(h)[1:]
    assert all(math.isfinite(s) and s > 0 for s in seconds)   # lazily harvested timings
    ao.region_destroy(h)


def test_save_load_trained_model_same_choices(env, tmp_path):
    ao, torch, dev, st = env
    vs = ao.jacobi_variants_sweep()[:4]
    h = ao.region_declare_variants("rt_persist", ao.AO_JACOBI7_F64, vs, min_train_data=10 ** 6)
    for x in np.linspace(0, 4, 30):
        for v in range(4):
            ao.region_record(h, [float(x), 1.0, 0, 0, 0, 0], v, math.exp((v - 1.5) * (x - 2.0)))
    ao.selector_train(h, epochs=100, batch=32, lr=3e-3)
    q = [[float(x), 1.0, 0, 0, 0, 0] for x in np.linspace(-0.2, 4.2, 37)]
    _, ids = ao.selector_select(h, q)
    path = str(tmp_path / "model.bin")
    ao.region_save(h, path)
    h2 = ao.region_declare_variants("rt_persist2", ao.AO_JACOBI7_F64, vs, min_train_data=10 ** 6)
    assert ao.region_stats(h2).trained == 0
    ao.region_load(h2, path)
    assert ao.region_stats(h2).trained == 1
    assert ao.selector_select(h2, q)[1] == ids
    ao.region_destroy(h)
    ao.region_destroy(h2)


def test_out_of_range_features_fall_back_to_timing(env, orc):
    ao, torch, dev, st = env
    vs = ao.jacobi_variants_blocks()
    h = ao.region_declare_variants("rt_ood", ao.AO_JACOBI7_F64, vs, min_train_data=10 ** 6)
    for x in np.linspace(4, 5, 8):
        for v in range(3):
            ao.region_record(h, [x, x, x, 3.0, 20.0, 1.0], v, 1e-4 * (1 + v))
    ao.selector_train(h, epochs=20)
    u0, out = _grid(torch, dev, 64, 77)        # log2 64 = 6: outside [4, 5] by > 25%
    rc, v = ao.region_run(h, ao.jacobi_args(u0, out, 64, 64, 64, 3), stream=st)
    assert rc == ao.AO_NOTE_FALLBACK and 0 <= v < 3
    st_ = ao.region_stats(h)
    assert st_.fallbacks == 1 and st_.memo_size == 1
    rc2, v2 = ao.region_run(h, ao.jacobi_args(u0, out, 64, 64, 64, 3), stream=st)
    assert rc2 == ao.AO_OK and v2 == v                     # memoised choice
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), orc.jacobi7(u0.cpu().numpy(), 64, 64, 64, 3))
    ao.region_destroy(h)


def test_exhaustive_producer_picks_the_profiled_minimum(env):
    ao, torch, dev, st = env
    vs = ao.jacobi_variants_sweep()
    h = ao.region_declare_variants("rt_exh", ao.AO_JACOBI7_F64, vs, model_type="exhaustive")
    u0, out = _grid(torch, dev, 96, 5)
    a = ao.jacobi_args(u0, out, 96, 96, 96, 4)
    rc, v = ao.region_run(h, a, stream=st)
    assert rc == ao.AO_OK
    feats, variants, seconds = ao.region_records(h)
    per = {}
    for var, s in zip(variants[:-1], seconds[:-1]):   # the profiling runs, then the run itself
        per.setdefault(var, []).append(s)
    med = {k: float(np.median(x)) for k, x in per.items()}
    assert v == min(med, key=lambda k: (med[k], k))
    # a device-resident 96^3 grid is faster on the GPU than on the host
    assert ao.jacobi_variants_sweep()[v].target == ao.AO_TARGET_GPU
    ao.region_destroy(h)
