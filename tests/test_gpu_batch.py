"""Batched persistent execution of many uneven Jacobi instances: every
instance bit-identical to a standalone region run (and to the oracle on
small ones), before and after autotuning, eager and as a replayed graph."""
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


def _instances(ao, torch, dev, shapes, sweeps, seed0):
    ins, bufs = [], []
    for q, ((nx, ny, nz), s) in enumerate(zip(shapes, sweeps)):
        u0 = synth.grid_u01_torch(int(nx), int(ny), int(nz), seed=seed0 + q, device=dev)
        out = torch.full_like(u0, float("nan"))
        bufs.append((u0, out))
        ins.append(ao.jacobi_args(u0, out, int(nx), int(ny), int(nz), int(s)))
    return ins, bufs


def _reference(ao, torch, st, ins, bufs):
    h = ao.region_declare_variants("batch_ref", ao.AO_JACOBI7_F64,
                                   [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_JACOBI_DIRECT, 64, 4, 1, 0)],
                                   model_type="roundrobin")
    refs = []
    for a, (u0, out) in zip(ins, bufs):
        r = torch.empty_like(u0)
        ra = ao.jacobi_args(u0, r, a.nx, a.ny, a.nz, a.sweeps)
        ao.region_run(h, ra, stream=st, variant=0)
        refs.append(r)
    torch.cuda.synchronize()
    return refs


def _check(torch, bufs, refs, tag):
    for q, ((u0, out), r) in enumerate(zip(bufs, refs)):
        assert torch.equal(out, r), f"{tag}: instance {q} differs from its reference"


def test_batch_small_mixed_against_oracle(env, orc):
    ao, torch, dev, st = env
    shapes = [(8, 8, 8), (5, 17, 3), (70, 9, 40), (1, 1, 30), (33, 65, 2), (130, 20, 11),
              (16, 16, 16), (3, 200, 4)]
    sweeps = [5, 1, 4, 3, 0, 2, 7, 5]
    ins, bufs = _instances(ao, torch, dev, shapes, sweeps, 900)
    b = ao.batch_create(ins)
    ao.batch_run(b, stream=st, use_graph=False)
    torch.cuda.synchronize()
    for (u0, out), (nx, ny, nz), s in zip(bufs, shapes, sweeps):
        want = orc.jacobi7(u0.cpu().numpy(), nx, ny, nz, s)
        assert np.array_equal(out.cpu().numpy(), want), (nx, ny, nz, s)
    ao.batch_destroy(b)


def _oracle_refs(torch, orc, bufs, shapes, sweeps):
    refs = []
    for (u0, _), (nx, ny, nz), s in zip(bufs, shapes, sweeps):
        want = orc.jacobi7(u0.cpu().numpy(), int(nx), int(ny), int(nz), int(s))
        refs.append(torch.from_numpy(want).to(u0.device))
    return refs


def test_batch_256_uneven_graph_and_autotune(env, orc):
    # 256 grids, each dimension log-uniform in [8, 256] (seed 3), 5 sweeps:
    # every grid compared with the serial oracle, eager, after autotuning and
    # on every graph replay
    ao, torch, dev, st = env
    shapes = synth.batch_shapes(256, 8, 256, seed=3)
    ins, bufs = _instances(ao, torch, dev, shapes, [5] * 256, 3000)
    refs = _oracle_refs(torch, orc, bufs, shapes, [5] * 256)
    b = ao.batch_create(ins)
    inst, items, tiles = ao.batch_info(b)
    assert sum(inst) == 256 and all(i > 0 for i, c in zip(items, inst) if c > 0)
    ao.batch_run(b, stream=st, use_graph=False)
    torch.cuda.synchronize()
    _check(torch, bufs, refs, "eager")
    chosen = ao.batch_autotune(b, stream=st, warmup=1, reps=3)
    assert all((c >= 0) == (n > 0) for c, n in zip(chosen, inst))
    # graph replays with eager work in between, each replay checked
    for rep in range(3):
        for _, out in bufs:
            out.fill_(float("nan"))
        ao.batch_run(b, stream=st, use_graph=True)
        torch.cuda.synchronize()
        _check(torch, bufs, refs, f"graph replay {rep}")
        junk = torch.ones(1 << 20, device=dev) * rep   # eager work between replays
        torch.cuda.synchronize()
        del junk
    ao.batch_destroy(b)


def test_every_tile_candidate_bit_identical(env, orc):
    # every tile of the autotuner's table (single-sweep, fused two- and
    # three-sweep) forced on every bucket: instances of all sizes, sweep
    # counts 0..7 (every remainder of the fused passes)
    ao, torch, dev, st = env
    shapes = [(8, 8, 8), (5, 17, 3), (70, 9, 40), (1, 1, 30), (33, 65, 2), (130, 20, 11),
              (16, 16, 16), (3, 200, 4), (63, 62, 5), (125, 7, 64), (62, 1, 1), (124, 33, 9)]
    sweeps = [5, 1, 4, 3, 0, 2, 7, 5, 6, 1, 3, 4]
    ins, bufs = _instances(ao, torch, dev, shapes, sweeps, 1700)
    refs = _reference(ao, torch, st, ins, bufs)
    for q in (0, 1, 3, 10):   # standalone runs pinned to the oracle on small instances
        nx, ny, nz = shapes[q]
        want = orc.jacobi7(bufs[q][0].cpu().numpy(), nx, ny, nz, sweeps[q])
        assert np.array_equal(refs[q].cpu().numpy(), want)
    b = ao.batch_create(ins)
    cands = ao.batch_candidates()
    assert any(k > 10 for k, *_ in cands) and any(k == 0 for k, *_ in cands)
    for c, tile in enumerate(cands):
        ao.batch_set_tiles(b, [c] * 5)
        assert all(t == tuple(tile[1:]) for t in ao.batch_info(b)[2])
        for use_graph in (False, True):
            for _, out in bufs:
                out.fill_(float("nan"))
            ao.batch_run(b, stream=st, use_graph=use_graph)
            torch.cuda.synchronize()
            _check(torch, bufs, refs, f"candidate {c} {tile} graph={use_graph}")
    ao.batch_destroy(b)


def test_three_sweep_tiles_of_different_rows_across_buckets(env, orc):
    # the waves of one block run items of different (T, R) back to back:
    # three-sweep tiles with 1, 2 and 4 rows per wave on neighbouring buckets,
    # sweep counts whose remainders mix one-, two- and three-sweep first
    # passes, and grids whose upper waves have no rows (they skip the item at
    # once); every instance compared with the oracle, eager and on graph
    # replays
    ao, torch, dev, st = env
    shapes = [(12, 5, 9), (16, 13, 3), (30, 6, 17), (24, 31, 8), (60, 9, 33), (64, 3, 20),
              (100, 7, 12), (128, 19, 5), (130, 11, 6), (200, 37, 4), (61, 2, 40), (121, 5, 9)]
    sweeps = [5, 4, 6, 7, 5, 2, 4, 3, 5, 7, 1, 6]
    ins, bufs = _instances(ao, torch, dev, shapes, sweeps, 2400)
    refs = _oracle_refs(torch, orc, bufs, shapes, sweeps)
    b = ao.batch_create(ins)
    cands = ao.batch_candidates()
    tri = {r: [c for c, t in enumerate(cands) if t[0] == 20 + r] for r in (1, 2, 4)}
    assert all(tri[r] for r in (1, 2, 4))
    plans = [[tri[1][0], tri[2][0], tri[4][0], tri[2][-1], tri[1][-1]],
             [tri[4][0], tri[1][0], tri[2][0], tri[1][-1], tri[4][-1]],
             [tri[2][0], tri[4][-1], tri[1][-1], tri[4][0], tri[2][-1]]]
    for plan in plans:
        ao.batch_set_tiles(b, plan)
        for use_graph in (False, True, True):
            for _, out in bufs:
                out.fill_(float("nan"))
            ao.batch_run(b, stream=st, use_graph=use_graph)
            torch.cuda.synchronize()
            _check(torch, bufs, refs, f"tiles {plan} graph={use_graph}")
    ao.batch_destroy(b)


def test_min_traffic_counts_passes(env):
    # 16 B per point per pass: one-point-per-thread tiles take S passes,
    # three-sweep tiles ceil(S / 3) (the first pass takes S mod 3 sweeps)
    ao, torch, dev, st = env
    shapes = [(9, 10, 11), (40, 33, 20)]
    sweeps = [5, 7]
    ins, bufs = _instances(ao, torch, dev, shapes, sweeps, 900)
    b = ao.batch_create(ins)
    cands = ao.batch_candidates()
    direct = next(c for c, t in enumerate(cands) if t[0] == 0)
    tri = next(c for c, t in enumerate(cands) if t[0] in (21, 22, 24))
    pts = [nx * ny * nz for nx, ny, nz in shapes]
    ao.batch_set_tiles(b, [direct] * 5)
    assert ao.batch_min_traffic(b) == 16.0 * (pts[0] * 5 + pts[1] * 7)
    ao.batch_set_tiles(b, [tri] * 5)
    assert ao.batch_min_traffic(b) == 16.0 * (pts[0] * 2 + pts[1] * 3)
    ao.batch_destroy(b)
