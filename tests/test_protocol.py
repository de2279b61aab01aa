"""The evaluation protocol of Sec. 4: K-fold subset construction (oracle
pins and the package against the oracle) and the Online comparator's
explore -> train -> exploit loop run through the library on host variants
(decision-tree model, trained on the host)."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("count,seed", [(7, 1), (100, 40), (1001, 3), (4, 9)])
def test_oracle_kfold_groups_partition(orc, count, seed):
    for r in range(3):
        groups = orc.kfold_groups(count, 4, seed, r)
        flat = sorted(i for g in groups for i in g)
        assert flat == list(range(count))                      # a partition
        sizes = [len(g) for g in groups]
        assert max(sizes) - min(sizes) <= 1 and sum(sizes) == count
    # reshuffles differ (for more than a handful of inputs)
    if count >= 100:
        assert orc.kfold_groups(count, 4, seed, 0) != orc.kfold_groups(count, 4, seed, 1)


def test_oracle_rotations_cover_train_and_test(orc):
    K = 4
    for m in (1, 2, 3):
        rots = orc.rotations(K, m)
        assert len(rots) == K and all(len(r) == m for r in rots)
        for g in range(K):
            assert any(g in r for r in rots)          # trained on at least once
            assert any(g not in r for r in rots)      # tested at least once
    assert orc.rotations(4, 2) == [[0, 1], [1, 2], [2, 3], [0, 3]]


def test_package_protocol_splits_match_oracle(orc):
    from paper_2303_08873_amd import protocol
    for count, seed in ((7, 1), (1000, 40), (333, 5)):
        for r in range(4):
            got = protocol.kfold_groups(count, 4, seed, r)
            want = orc.kfold_groups(count, 4, seed, r)
            assert [list(map(int, g)) for g in got] == want
    for m in (1, 2, 3):
        assert protocol.rotations(4, m) == orc.rotations(4, m)


def test_online_loop_explores_then_exploits_on_host(orc):
    # an untrained region of the 5 host variants (min_train_data = 5): the
    # first 5 runs explore RoundRobin, the 5th trains, the rest use the
    # fastest explored variant; every output equals the oracle
    import paper_2303_08873_amd as ao
    vs = ao.jacobi_sweep_host()
    h = ao.region_declare_variants("online_host", ao.AO_JACOBI7_F64, vs, model_type="dtree")
    nx, ny, nz, S = 24, 20, 18, 3
    u0 = synth.grid_u01(nx, ny, nz, seed=11)
    want = orc.jacobi7(u0, nx, ny, nz, S)
    out = np.zeros_like(u0)
    a = ao.jacobi_args(u0, out, nx, ny, nz, S, resident=0)
    chosen = []
    for it in range(12):
        out.fill(-1.0)
        rc, v = ao.region_run(h, a, variant=-1)
        chosen.append(v)
        assert np.array_equal(out, want)
        if it == 4:
            assert ao.region_stats(h).trained == 1
    _, variants, seconds = ao.region_records(h)
    assert chosen[:5] == [0, 1, 2, 3, 4] and variants[:5] == [0, 1, 2, 3, 4]
    pick = orc.online_choice(seconds[:5])
    assert all(v == pick for v in chosen[5:])
    ao.region_destroy(h)
