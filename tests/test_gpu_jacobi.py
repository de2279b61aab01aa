"""GPU parity of the Jacobi region variants against the CPU oracle, through
the C ABI: every variant bit-identical to every other and to the oracle
(which sums in the same order; the bound is elementwise |g-o| <= 1e-12|o|,
met here with zero error), on ragged shapes, both residencies, edge cases,
and the full 512^3 x 20 workload on every point."""
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


def _check(got, want):
    assert got.shape == want.shape
    if not np.array_equal(got, want):
        rel = np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300))
        bad = int(np.sum(got != want))
        assert rel <= 1e-12, f"{bad} elements differ, max rel {rel:g}"
        pytest.fail(f"{bad} elements differ from the oracle (max rel {rel:g}, within 1e-12 "
                    "but the variants promise bit identity)")


def test_config_blocks_64cubed(env, orc):
    # 64^3 grid, 10 sweeps, u0 ~ U[0,1) seed 1, variants 64 / 256 / 1024 threads
    ao, torch, dev, st = env
    n, S = 64, 10
    u0_h = synth.grid_u01(n, n, n, seed=1)
    want = orc.jacobi7(u0_h, n, n, n, S)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    h = ao.region_declare_variants("gpu_c1", ao.AO_JACOBI7_F64, ao.jacobi_variants_blocks(),
                                   model_type="exhaustive")
    a = ao.jacobi_args(u0, out, n, n, n, S)
    for v in range(3):
        out.fill_(-1.0)
        ao.region_run(h, a, stream=st, variant=v)
        torch.cuda.synchronize()
        _check(out.cpu().numpy(), want)
    med = ao.region_profile(h, a, warmup=2, reps=5, stream=st)
    assert all(math.isfinite(t) and t > 0 for t in med)
    rc, chosen = ao.region_run(h, a, stream=st)   # exhaustive producer
    torch.cuda.synchronize()
    assert 0 <= chosen < 3
    _check(out.cpu().numpy(), want)
    assert torch.equal(u0.cpu(), torch.from_numpy(u0_h))  # u0 untouched
    ao.region_destroy(h)


SHAPES = [((37, 29, 13), 3), ((1, 1, 50), 2), ((65, 3, 7), 1), ((5, 130, 2), 4),
          ((129, 9, 33), 2), ((64, 64, 1), 5), ((3, 3, 3), 7)]


@pytest.mark.parametrize("shape,S", SHAPES)
@pytest.mark.parametrize("resident", [1, 0])
def test_sweep_variants_ragged(env, orc, shape, S, resident):
    ao, torch, dev, st = env
    nx, ny, nz = shape
    u0_h = synth.grid_u01(nx, ny, nz, seed=2000 + nx)
    want = orc.jacobi7(u0_h, nx, ny, nz, S)
    if resident:
        u0 = torch.from_numpy(u0_h).to(dev)
        out = torch.empty_like(u0)
    else:
        u0 = torch.from_numpy(u0_h).pin_memory()
        out = torch.empty(u0.shape, dtype=torch.float64).pin_memory()
    h = ao.region_declare_variants("gpu_c2", ao.AO_JACOBI7_F64, ao.jacobi_variants_sweep(),
                                   model_type="roundrobin")
    a = ao.jacobi_args(u0, out, nx, ny, nz, S, resident=resident)
    for v in range(10):
        out.fill_(-1.0)
        ao.region_run(h, a, stream=st, variant=v)
        torch.cuda.synchronize()
        _check(out.cpu().numpy(), want)


def test_nontemporal_and_zmarch_shapes(env, orc):
    ao, torch, dev, st = env
    nx, ny, nz, S = 70, 21, 45, 3
    u0_h = synth.grid_u01(nx, ny, nz, seed=9)
    want = orc.jacobi7(u0_h, nx, ny, nz, S)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    vs = [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_DIRECT, 64, 4, 1, ao.AO_VF_NT_STORE),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZMARCH, 64, 4, 7, ao.AO_VF_NT_STORE),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZMARCH, 128, 8, 1, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZMARCH, 16, 4, 100, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_DIRECT, 256, 4, 1, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZREG, 64, 1, 5, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZREG, 64, 8, 64, ao.AO_VF_NT_STORE),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZREG, 128, 2, 16, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZREG, 128, 4, 3, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZREG, 128, 8, 100, 0)]
    h = ao.region_declare_variants("gpu_shapes", ao.AO_JACOBI7_F64, vs, model_type="roundrobin")
    a = ao.jacobi_args(u0, out, nx, ny, nz, S)
    for v in range(len(vs)):
        out.fill_(-1.0)
        ao.region_run(h, a, stream=st, variant=v)
        torch.cuda.synchronize()
        _check(out.cpu().numpy(), want)


ZREG = [(64, 1, 1, 0), (64, 2, 7, 0), (64, 4, 64, 0), (64, 8, 3, 0), (128, 1, 2, 0), (128, 2, 9, 0),
        (128, 4, 5, 0), (128, 8, 64, 0), (64, 1, 1, 2), (64, 4, 24, 3), (128, 2, 9, 2), (64, 8, 5, 2)]


@pytest.mark.parametrize("shape,S", [((130, 37, 11), 3), ((1, 1, 9), 2), ((2, 33, 5), 2),
                                     ((257, 3, 4), 1), ((64, 32, 16), 2), ((6, 6, 6), 5)])
def test_zreg_all_shapes(env, orc, shape, S):
    # register z-march: every strip width / rows-per-wave / plane count,
    # ragged in every direction (odd nx refuses the 128-wide strip, which
    # loads pairs, and masks it)
    ao, torch, dev, st = env
    nx, ny, nz = shape
    u0_h = synth.grid_u01(nx, ny, nz, seed=31 + nx)
    want = orc.jacobi7(u0_h, nx, ny, nz, S)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    # flags: 1 streaming stores, 2 halo prefetch
    vs = [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZREG, bx, by, bz, fl) for bx, by, bz, fl in ZREG]
    h = ao.region_declare_variants(f"gpu_zreg_{nx}_{ny}_{nz}", ao.AO_JACOBI7_F64, vs,
                                   model_type="roundrobin")
    a = ao.jacobi_args(u0, out, nx, ny, nz, S)
    for v, (bx, by, bz, _) in enumerate(ZREG):
        out.fill_(-1.0)
        if bx == 128 and nx % 2:
            with pytest.raises(ao.AdaptError):
                ao.region_run(h, a, stream=st, variant=v)
            continue
        ao.region_run(h, a, stream=st, variant=v)
        torch.cuda.synchronize()
        _check(out.cpu().numpy(), want)


# (rows per wave, planes per block, flags: 1 streaming stores, 4 register cap)
T2 = [(1, 1, 0), (1, 3, 1), (2, 16, 0), (2, 5, 1), (4, 64, 0), (4, 2, 1), (2, 100, 0), (1, 7, 0),
      (3, 9, 0), (3, 4, 5), (4, 32, 5), (4, 7, 4)]
# rows 6 and 8, and the prefetching form (flag 2) with every other flag
T2_MORE = [(6, 1, 0), (6, 5, 1), (8, 3, 0), (8, 32, 1), (1, 1, 2), (2, 3, 3), (3, 16, 2),
           (4, 32, 3), (4, 2, 7), (6, 9, 2), (8, 7, 3), (3, 5, 6)]
T2_BIG = [(10, 1, 0), (12, 3, 1), (16, 5, 0), (10, 32, 3), (12, 7, 2), (16, 2, 1), (12, 33, 4)]


@pytest.mark.parametrize("shape,S", [((130, 37, 11), 3), ((1, 1, 9), 2), ((2, 33, 5), 4),
                                     ((257, 3, 4), 1), ((64, 32, 16), 2), ((6, 6, 6), 5),
                                     ((63, 5, 7), 6), ((125, 18, 33), 8)])
def test_two_sweep_family_all_shapes(env, orc, shape, S):
    # temporal blocking: two sweeps fused per pass (plus one single sweep when
    # S is odd), bit-identical to S separate sweeps
    ao, torch, dev, st = env
    nx, ny, nz = shape
    u0_h = synth.grid_u01(nx, ny, nz, seed=61 + nx + S)
    want = orc.jacobi7(u0_h, nx, ny, nz, S)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    for tag, lst in (("a", T2), ("b", T2_MORE), ("c", T2_BIG)):
        vs = [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_ZREG_T2, 64, r, bz, fl)
              for r, bz, fl in lst]
        h = ao.region_declare_variants(f"gpu_t2{tag}_{nx}_{ny}_{nz}_{S}", ao.AO_JACOBI7_F64, vs,
                                       model_type="roundrobin")
        for resident in (1, 0):
            if resident:
                a = ao.jacobi_args(u0, out, nx, ny, nz, S)
            else:
                uh = torch.from_numpy(u0_h).pin_memory()
                oh = torch.empty(uh.shape, dtype=torch.float64).pin_memory()
                a = ao.jacobi_args(uh, oh, nx, ny, nz, S, resident=0)
            for v in range(len(lst)):
                (out if resident else oh).fill_(-1.0)
                ao.region_run(h, a, stream=st, variant=v)
                torch.cuda.synchronize()
                _check((out if resident else oh).cpu().numpy(), want)
        ao.region_destroy(h)


T3 = [(1, 1, 0), (1, 5, 1), (2, 3, 0), (2, 16, 1), (3, 7, 0), (3, 32, 1), (4, 2, 0), (4, 16, 1),
      (6, 9, 0), (6, 1, 1), (8, 4, 0), (5, 11, 1)]
T4 = [(1, 1, 0), (1, 6, 1), (2, 3, 0), (2, 16, 1), (3, 7, 0), (3, 32, 1), (4, 2, 0), (4, 16, 1),
      (4, 5, 1), (2, 1, 0), (5, 3, 0), (5, 64, 1)]
# the same families with the early next-plane loads (flag 2, with and without
# streaming stores)
T3_PF = [(1, 1, 2), (1, 5, 3), (2, 3, 2), (2, 16, 3), (3, 7, 2), (5, 32, 3), (4, 2, 2),
         (4, 16, 3), (6, 9, 2), (6, 1, 3), (8, 4, 2), (8, 32, 3)]
T4_PF = [(1, 1, 2), (1, 6, 3), (2, 3, 2), (2, 16, 3), (3, 7, 2), (3, 32, 3), (4, 2, 2),
         (4, 16, 3), (4, 5, 3), (2, 1, 2), (5, 9, 2), (5, 64, 3)]
# level 0 staged through LDS for waves inside the grid (flag 8, with and
# without streaming stores)
T3_ST = [(1, 1, 8), (1, 5, 9), (2, 3, 8), (2, 16, 9), (3, 7, 8), (4, 2, 9), (4, 16, 8),
         (5, 11, 9), (6, 9, 8), (6, 1, 9), (8, 4, 8), (8, 32, 9)]
T4_ST = [(1, 1, 8), (1, 6, 9), (2, 3, 8), (2, 16, 9), (3, 7, 8), (3, 32, 9), (4, 2, 8),
         (4, 16, 9), (5, 5, 9), (5, 64, 9), (5, 3, 8), (2, 1, 8)]


@pytest.mark.parametrize("shape,S", [((130, 37, 11), 3), ((1, 1, 9), 2), ((2, 33, 5), 4),
                                     ((257, 3, 4), 1), ((64, 32, 16), 6), ((6, 6, 6), 5),
                                     ((61, 5, 7), 7), ((125, 18, 33), 9), ((60, 60, 3), 8),
                                     ((190, 41, 19), 8)])
def test_three_and_four_sweep_families_all_shapes(env, orc, shape, S):
    # three / four sweeps fused per pass (the S mod T remaining sweeps first as
    # one shorter pass), bit-identical to S separate sweeps; the wider shapes
    # have waves whose columns and rows lie inside the grid (the march
    # without per-lane selects) beside waves on the boundary
    ao, torch, dev, st = env
    nx, ny, nz = shape
    u0_h = synth.grid_u01(nx, ny, nz, seed=71 + nx + S)
    want = orc.jacobi7(u0_h, nx, ny, nz, S)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    for tag, fam, lst in (("", ao.FAM_JACOBI_ZREG_T3, T3), ("", ao.FAM_JACOBI_ZREG_T4, T4),
                          ("pf", ao.FAM_JACOBI_ZREG_T3, T3_PF),
                          ("pf", ao.FAM_JACOBI_ZREG_T4, T4_PF),
                          ("st", ao.FAM_JACOBI_ZREG_T3, T3_ST),
                          ("st", ao.FAM_JACOBI_ZREG_T4, T4_ST)):
        vs = [ao.Variant(ao.AO_TARGET_GPU, fam, 64, r, bz, fl) for r, bz, fl in lst]
        h = ao.region_declare_variants(f"gpu_tb{tag}{fam}_{nx}_{ny}_{nz}_{S}", ao.AO_JACOBI7_F64,
                                       vs, model_type="roundrobin")
        for resident in (1, 0):
            if resident:
                a = ao.jacobi_args(u0, out, nx, ny, nz, S)
            else:
                uh = torch.from_numpy(u0_h).pin_memory()
                oh = torch.empty(uh.shape, dtype=torch.float64).pin_memory()
                a = ao.jacobi_args(uh, oh, nx, ny, nz, S, resident=0)
            for v in range(len(lst)):
                (out if resident else oh).fill_(-1.0)
                ao.region_run(h, a, stream=st, variant=v)
                torch.cuda.synchronize()
                _check((out if resident else oh).cpu().numpy(), want)
        ao.region_destroy(h)


@pytest.mark.parametrize("shape,S", [((130, 37, 11), 3), ((64, 32, 16), 2), ((7, 5, 1), 2),
                                     ((33, 65, 10), 5), ((20, 20, 3), 0), ((70, 9, 2), 1)])
def test_cosched_every_fraction_both_residencies(env, orc, shape, S):
    # CPU+GPU co-scheduling: the host's share of z-planes in tenths 0..10,
    # one halo plane exchanged each way per sweep; bit-identical to S sweeps
    ao, torch, dev, st = env
    nx, ny, nz = shape
    u0_h = synth.grid_u01(nx, ny, nz, seed=81 + nz + S)
    want = orc.jacobi7(u0_h, nx, ny, nz, S)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    vs = [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_COSCHED, f, 0, 0, f % 2) for f in range(11)]
    h = ao.region_declare_variants(f"gpu_cosched_{nx}_{ny}_{nz}_{S}", ao.AO_JACOBI7_F64, vs,
                                   model_type="roundrobin")
    for resident in (1, 0):
        if resident:
            a = ao.jacobi_args(u0, out, nx, ny, nz, S)
        else:
            uh = torch.from_numpy(u0_h).pin_memory()
            oh = torch.empty(uh.shape, dtype=torch.float64).pin_memory()
            a = ao.jacobi_args(uh, oh, nx, ny, nz, S, resident=0)
        for v in range(len(vs)):
            (out if resident else oh).fill_(-1.0)
            ao.region_run(h, a, stream=st, variant=v)
            torch.cuda.synchronize()
            _check((out if resident else oh).cpu().numpy(), want)
        if not resident:
            assert np.array_equal(uh.numpy(), u0_h)   # the input is untouched
    ao.region_destroy(h)


def test_hbm_copy_probe(env):
    ao, torch, dev, st = env
    for n in (0, 1, 5, 4096, 1000003):
        src = torch.arange(n, dtype=torch.float64, device=dev)
        dst = torch.full((n,), -1.0, dtype=torch.float64, device=dev)
        ao.ao_hbm_copy(src, dst, n, nontemporal=(n % 2 == 1), stream=st)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)


def test_edge_cases(env, orc):
    ao, torch, dev, st = env
    h = ao.region_declare_variants("gpu_edges", ao.AO_JACOBI7_F64, ao.jacobi_variants_sweep(),
                                   model_type="roundrobin")
    # zero sweeps: out = u0
    u0_h = synth.grid_u01(9, 8, 7, seed=4)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    for v in (0, 3, 5):
        out.fill_(-1.0)
        ao.region_run(h, ao.jacobi_args(u0, out, 9, 8, 7, 0), stream=st, variant=v)
        torch.cuda.synchronize()
        assert torch.equal(out, u0)
    # empty grid: nothing to do, no error
    e = torch.empty(0, dtype=torch.float64, device=dev)
    ao.region_run(h, ao.jacobi_args(e, e, 0, 4, 4, 3), stream=st, variant=0)
    # launch failure: a 64x32 block (2048 threads) is refused on the host and masked
    bad = [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_DIRECT, 64, 32, 1, 0),
           ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_DIRECT, 64, 4, 1, 0)]
    hb = ao.region_declare_variants("gpu_badlaunch", ao.AO_JACOBI7_F64, bad, model_type="roundrobin")
    a = ao.jacobi_args(u0, out, 9, 8, 7, 2)
    with pytest.raises(ao.AdaptError) as err:
        ao.region_run(hb, a, stream=st, variant=0)
    assert err.value.code == -7
    assert ao.region_stats(hb).failed_mask == 1
    for _ in range(3):
        rc, v = ao.region_run(hb, a, stream=st)
        assert v == 1
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), orc.jacobi7(u0_h, 9, 8, 7, 2))
    med = ao.region_profile(hb, a, warmup=1, reps=2, stream=st)
    assert math.isinf(med[0]) and math.isfinite(med[1])


def test_full_size_512_every_variant_against_the_oracle(env, orc):
    # 512^3, 20 sweeps, device-resident: the whole output grid of every GPU
    # variant of the size sweep compared element by element with one run of
    # the serial oracle (about 4 s of host time)
    ao, torch, dev, st = env
    n, S = 512, 20
    u0 = synth.grid_u01_torch(n, n, n, seed=2009, device=dev)
    want = torch.from_numpy(orc.jacobi7(u0.cpu().numpy(), n, n, n, S)).to(dev)
    out = torch.empty_like(u0)
    gpu = ao.jacobi_sweep_gpu()
    h = ao.region_declare_variants("gpu_full", ao.AO_JACOBI7_F64, gpu, model_type="roundrobin")
    a = ao.jacobi_args(u0, out, n, n, n, S)
    for v in range(len(gpu)):
        out.fill_(-1.0)
        ao.region_run(h, a, stream=st, variant=v)
        torch.cuda.synchronize()
        if not torch.equal(out, want):
            bad = int((out != want).sum())
            rel = float(((out - want).abs() / want.abs().clamp_min(1e-300)).max())
            pytest.fail(f"variant {v}: {bad} of {n ** 3} points differ from the oracle "
                        f"(max rel {rel:g})")
    ao.region_destroy(h)


@pytest.mark.parametrize("shape,S", [((16, 16, 32), 7), ((8193, 1, 1), 2), ((1, 8192, 1), 3),
                                     ((20, 20, 20), 1), ((3, 5, 7), 20), ((16, 16, 33), 2)])
def test_direct_family_small_grids_in_lds(env, orc, shape, S):
    # with the all-sweeps-in-LDS flag, grids of at most 8192 points run all
    # sweeps in one workgroup's LDS (16x16x32, 1x8192x1, 20^3, 3x5x7);
    # 8193x1x1 and 16x16x33 just past the limit, and every grid without the
    # flag, take the per-sweep launches of the block shape; both
    # residencies, bit-identical to the oracle
    ao, torch, dev, st = env
    nx, ny, nz = shape
    u0_h = synth.grid_u01(nx, ny, nz, seed=91 + nz + S)
    want = orc.jacobi7(u0_h, nx, ny, nz, S)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    vs = [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_DIRECT, bx, by, 1, fl)
          for fl in (0, ao.AO_VF_LDS_SWEEPS) for bx, by in ((64, 4), (32, 8), (64, 16))]
    h = ao.region_declare_variants(f"gpu_lds_{nx}_{ny}_{nz}_{S}", ao.AO_JACOBI7_F64, vs,
                                   model_type="roundrobin")
    for resident in (1, 0):
        if resident:
            a = ao.jacobi_args(u0, out, nx, ny, nz, S)
        else:
            uh = torch.from_numpy(u0_h).pin_memory()
            oh = torch.empty(uh.shape, dtype=torch.float64).pin_memory()
            a = ao.jacobi_args(uh, oh, nx, ny, nz, S, resident=0)
        for v in range(len(vs)):
            (out if resident else oh).fill_(-1.0)
            ao.region_run(h, a, stream=st, variant=v)
            torch.cuda.synchronize()
            _check((out if resident else oh).cpu().numpy(), want)
    ao.region_destroy(h)


# (family, rows per wave, planes bound, flags: 1 streaming stores, 2 early
# next-plane loads, 8 staged level 0)
FILL = [("ZREG", 4, 32, 0), ("ZREG", 1, 9, 1), ("T2", 4, 32, 0), ("T2", 2, 17, 2),
        ("T3", 4, 22, 8), ("T3", 1, 8, 0), ("T4", 4, 74, 9), ("T4", 2, 16, 2), ("T4", 5, 40, 8)]


@pytest.mark.parametrize("shape,S", [((200, 300, 100), 10), ((130, 37, 41), 7), ((64, 64, 64), 5),
                                     ((257, 65, 33), 9), ((62, 6, 1), 3), ((3, 2, 130), 4)])
def test_fill_z_every_family(env, orc, shape, S):
    # AO_VF_FILL_Z: each launch cuts z into the chunks that fill the device
    # (at most bz planes each); the result stays bit-identical to the oracle
    # for every register z-march family, with the S mod T remaining sweeps
    # first (their launch fills the device the same way)
    ao, torch, dev, st = env
    fams = {"ZREG": ao.FAM_JACOBI_ZREG, "T2": ao.FAM_JACOBI_ZREG_T2,
            "T3": ao.FAM_JACOBI_ZREG_T3, "T4": ao.FAM_JACOBI_ZREG_T4}
    nx, ny, nz = shape
    u0_h = synth.grid_u01(nx, ny, nz, seed=91 + nx + S)
    want = orc.jacobi7(u0_h, nx, ny, nz, S)
    u0 = torch.from_numpy(u0_h).to(dev)
    out = torch.empty_like(u0)
    vs = [ao.Variant(ao.AO_TARGET_GPU, fams[f], 64, r, bz, fl | ao.AO_VF_FILL_Z)
          for f, r, bz, fl in FILL]
    h = ao.region_declare_variants(f"gpu_fill_{nx}_{ny}_{nz}_{S}", ao.AO_JACOBI7_F64, vs,
                                   model_type="roundrobin")
    a = ao.jacobi_args(u0, out, nx, ny, nz, S)
    for v, var in enumerate(vs):
        planes = ao.ao_jacobi_planes(var, nx, ny, nz)
        assert 1 <= planes <= min(var.bz, nz)
        out.fill_(-1.0)
        ao.region_run(h, a, stream=st, variant=v)
        torch.cuda.synchronize()
        _check(out.cpu().numpy(), want)
    ao.region_destroy(h)


def test_fill_z_device_picks(env):
    # the device's own residency: two four-sweep workgroups (239 VGPRs, 56
    # KB of LDS) per CU on 256 CUs keep 512^3 at 74 planes per block and cut
    # 256^3 into 6 chunks of 43 (480 blocks, two on most CUs)
    ao, torch, dev, st = env
    v3 = ao.jacobi_variants_sweep()[3]
    assert v3.flags & ao.AO_VF_FILL_Z
    cus = ao.ao_device_cus()
    got = {n: ao.ao_jacobi_planes(v3, n, n, n) for n in (64, 128, 256, 512)}
    print("CUs", cus, "planes of the four-sweep variant", got, flush=True)
    for n, p in got.items():
        assert 1 <= p <= min(74, n)
    if cus == 256:
        assert got[512] == 74 and got[256] == 43
