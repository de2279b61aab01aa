"""The allocation-free entry point against region_run: for every GPU
variant of the size-sweep table, region_run_noalloc (ping-pong array from
the library's static device array) gives the same bits as region_run of
the same variant (ping-pong array from the region's own scratch), on two
calls in a row, the second with a smaller grid and an odd sweep count; a
grid whose execution needs more scratch than the static array holds is
refused before anything is enqueued, and a single-launch execution of such
a grid needs no scratch and runs."""
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


def _pair(ao, torch, dev, st, reg, v, shape, S, seed):
    nx, ny, nz = shape
    u0 = synth.grid_u01_torch(nx, ny, nz, seed=seed, device=dev)
    want = torch.full_like(u0, float("nan"))
    got = torch.full_like(u0, float("nan"))
    ao.region_run(reg, ao.jacobi_args(u0, want, nx, ny, nz, S), stream=st, variant=v)
    rc = ao.region_run_noalloc(reg, ao.jacobi_args(u0, got, nx, ny, nz, S), v, stream=st)
    torch.cuda.synchronize()
    assert rc == ao.AO_OK
    return u0, want, got


def test_noalloc_matches_region_run_every_gpu_variant(env):
    import oracle
    ao, torch, dev, st = env
    variants = ao.jacobi_variants_sweep()
    reg = ao.region_declare_variants("noalloc_sweep", ao.AO_JACOBI7_F64, variants,
                                     model_type="roundrobin")
    gpu = [v for v, x in enumerate(variants) if x.target == ao.AO_TARGET_GPU]
    assert gpu
    for v in gpu:
        # first call: 100 x 90 x 80 (720,000 points), 20 sweeps
        print(f"noalloc variant {v}: 100x90x80, 20 sweeps", flush=True)
        _, want, got = _pair(ao, torch, dev, st, reg, v, (100, 90, 80), 20, 11)
        assert torch.equal(want.view(torch.int64), got.view(torch.int64)), v
        # second call, smaller grid, odd sweep count: the array keeps the
        # first call's values, which must not leak into the result
        print(f"noalloc variant {v}: 37x29x23, 7 sweeps", flush=True)
        u0, want, got = _pair(ao, torch, dev, st, reg, v, (37, 29, 23), 7, 12)
        assert torch.equal(want.view(torch.int64), got.view(torch.int64)), v
        ref = oracle.jacobi7(u0.cpu().numpy(), 37, 29, 23, 7)
        assert np.array_equal(got.cpu().numpy(), ref), v
    ao.region_destroy(reg)


def test_noalloc_refuses_grids_beyond_the_array(env):
    ao, torch, dev, st = env
    variants = ao.jacobi_variants_sweep()
    reg = ao.region_declare_variants("noalloc_limit", ao.AO_JACOBI7_F64, variants,
                                     model_type="roundrobin")
    nx, ny, nz = 256, 256, 129  # 8,454,144 points: 67.6 MB of scratch
    assert nx * ny * nz * 8 > 67108864
    u0 = synth.grid_u01_torch(nx, ny, nz, seed=13, device=dev)
    out = torch.full_like(u0, float("nan"))
    with pytest.raises(ao.AdaptError) as ei:
        ao.region_run_noalloc(reg, ao.jacobi_args(u0, out, nx, ny, nz, 20), 0, stream=st)
    assert "static array" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.isnan(out).all()  # nothing was enqueued
    # one launch needs no scratch: a variant fusing four sweeps runs four
    t4 = next(v for v, x in enumerate(variants) if x.family == ao.FAM_JACOBI_ZREG_T4)
    want = torch.empty_like(u0)
    ao.region_run(reg, ao.jacobi_args(u0, want, nx, ny, nz, 4), stream=st, variant=t4)
    ao.region_run_noalloc(reg, ao.jacobi_args(u0, out, nx, ny, nz, 4), t4, stream=st)
    torch.cuda.synchronize()
    assert torch.equal(want.view(torch.int64), out.view(torch.int64))
    # host variants and host-resident data are refused
    host = next(v for v, x in enumerate(variants) if x.target == ao.AO_TARGET_HOST)
    with pytest.raises(ao.AdaptError):
        ao.region_run_noalloc(reg, ao.jacobi_args(u0, out, nx, ny, nz, 4), host, stream=st)
    ao.region_destroy(reg)
