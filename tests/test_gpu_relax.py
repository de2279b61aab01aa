"""GPU parity of the weighted-Jacobi relaxation region (AMGMk relax,
Table 3): every SpMV variant family with the fused update bit-identical to
the oracle, for several sweep counts and weights, on Pareto-row systems,
long (merge-path-split) rows, diagonal-only rows, and the full 2^22-row
system; relaxation features = SpMV features + sweeps."""
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


def _variants(ao):
    vs = ao.spmv_variants(blocks=(64, 256, 1024))
    vs.append(ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_MERGE_PATH, 128, 0, 1, 0))
    vs.append(ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_XSLICE, 0, 14, 1, 0))
    vs.append(ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_XSLICE, 0, 13, 1, 0))
    return vs


def _to(torch, dev, m):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in m.items()}


def _check_all(ao, torch, dev, st, orc, m, cases, name, variants=None):
    n = m["row_ptr"].size - 1
    t = _to(torch, dev, m)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    vs = variants if variants is not None else _variants(ao)
    hs = [ao.region_declare_variants(f"{name}_{c0}", ao.AO_CSR_RELAX_F64, vs[c0:c0 + 12],
                                     model_type="roundrobin") for c0 in range(0, len(vs), 12)]
    for omega, S in cases:
        want = orc.relax(m["row_ptr"], m["col"], m["val"], m["x"], m["b"], m["d"], omega, S)
        a = ao.relax_args(t["row_ptr"], t["col"], t["val"], t["x"], y, t["b"], t["d"], omega, S,
                          n, int(m["col"].size))
        for v in range(len(vs)):
            y.fill_(float("nan"))
            ao.region_run(hs[v // 12], a, stream=st, variant=v % 12)
            torch.cuda.synchronize()
            got = y.cpu().numpy()
            assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (name, omega, S, v)
        assert torch.equal(t["x"].cpu(), torch.from_numpy(m["x"]))  # x untouched
    for h in hs:
        ao.region_destroy(h)


CASES = [(2.0 / 3.0, 1), (1.0, 2), (0.8, 5), (0.5, 0), (1.3, 3)]


@pytest.mark.parametrize("n,tail,max_len,seed", [(5000, 1.5, 4096, 31), (3, 1.5, 4096, 32),
                                                  (777, 3.0, 64, 33)])
def test_pareto_systems(env, orc, n, tail, max_len, seed):
    ao, torch, dev, st = env
    m = synth.relax_system(n, seed, tail=tail, max_len=max_len)
    _check_all(ao, torch, dev, st, orc, m, CASES, f"gpu_relax_{n}_{seed}")


def test_long_rows_split_by_merge_path(env, orc):
    # rows of up to 4096 entries: merge-path splits them over workgroups and
    # finishes them in the fix-up kernel, where the update is applied too
    ao, torch, dev, st = env
    m = synth.relax_system(20000, 34, tail=1.1, mean=40.0, max_len=4096)
    lens = np.diff(m["row_ptr"])
    assert lens.max() >= 1024
    _check_all(ao, torch, dev, st, orc, m, [(2.0 / 3.0, 2), (1.0, 3)], "gpu_relax_long")


def test_diagonal_only_rows(env, orc):
    # mean row length 1: most rows hold only their diagonal entry
    ao, torch, dev, st = env
    m = synth.relax_system(4096, 35, mean=1.0, max_len=8)
    _check_all(ao, torch, dev, st, orc, m, [(1.0, 1), (0.7, 4)], "gpu_relax_diag")


def test_features_are_spmv_features_and_sweeps(env, orc):
    ao, torch, dev, st = env
    m = synth.relax_system(6000, 36)
    n = m["row_ptr"].size - 1
    t = _to(torch, dev, m)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    h = ao.region_declare_variants("gpu_relax_feat", ao.AO_CSR_RELAX_F64, _variants(ao))
    a = ao.relax_args(t["row_ptr"], t["col"], t["val"], t["x"], y, t["b"], t["d"], 0.9, 7, n,
                      int(m["col"].size))
    f = ao.region_features(h, a, stream=st)
    want = orc.csr_features(m["row_ptr"])
    assert np.allclose(f[:5], want[:5], rtol=1e-6, atol=1e-6) and f[5] == 7.0
    ao.region_destroy(h)


def test_full_size_2_22(env, orc):
    # the relaxation workload at its full size: n = 2^22 (about 71 M
    # nonzeros with the diagonal), 2 sweeps, one variant per family
    ao, torch, dev, st = env
    m = synth.relax_system(1 << 22, 5)
    vs = [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_THREAD_ROW, 256, 0, 1, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_WAVE_ROW, 256, 0, 1, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_MERGE_PATH, 1024, 0, 1, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_XSLICE, 0, 14, 1, 0)]
    _check_all(ao, torch, dev, st, orc, m, [(2.0 / 3.0, 2)], "gpu_relax_full", variants=vs)
