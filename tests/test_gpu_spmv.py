"""GPU parity of the SpMV region variants: every variant bit-identical to
the canonical-order oracle (and within 1e-12 * sum|a x| of the plain
left-to-right oracle), on Pareto-row matrices, empty and long rows, special
matrices, and the full 2^22-row workload; the GPU row-length features
against the oracle's."""
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


def _variants(ao):
    vs = ao.spmv_variants(blocks=(64, 256, 1024))
    for w in (1, 2, 4, 8, 16, 32):
        vs.append(ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_WAVE_ROW, 256, w, 1, 0))
    for b in (128, 512):
        vs.append(ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_MERGE_PATH, b, 0, 1, 0))
    for swl in (13, 14, 0):
        vs.append(ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_XSLICE, 0, swl, 1, 0))
    return vs


def _run_all(ao, torch, dev, st, m, name):
    n = m["row_ptr"].size - 1
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in m.items()}
    y = torch.empty(n, dtype=torch.float64, device=dev)
    a = ao.spmv_args(t["row_ptr"], t["col"], t["val"], t["x"], y, n, int(m["col"].size))
    vs = _variants(ao)
    outs = []
    for c0 in range(0, len(vs), 12):
        h = ao.region_declare_variants(f"{name}_{c0}", ao.AO_CSR_SPMV_F64, vs[c0:c0 + 12],
                                       model_type="roundrobin")
        for v in range(len(vs[c0:c0 + 12])):
            y.fill_(float("nan"))
            ao.region_run(h, a, stream=st, variant=v)
            torch.cuda.synchronize()
            outs.append((vs[c0 + v], y.cpu().numpy().copy()))
        ao.region_destroy(h)
    return outs


def _check_all(outs, want, want_plain, scale):
    for var, got in outs:
        assert not np.any(np.isnan(got)), f"{var}: rows not written"
        if not np.array_equal(got, want) or not np.array_equal(np.signbit(got), np.signbit(want)):
            bad = int(np.sum(got != want))
            pytest.fail(f"{var}: {bad} rows differ from the canonical oracle")
        assert np.all(np.abs(got - want_plain) <= 1e-12 * scale), var


def _scale(m):
    """sum_k |val_k x_col_k| per row (the scale of the plain-order tolerance)."""
    rp, col, val, x = m["row_ptr"], m["col"], m["val"], m["x"]
    cs = np.concatenate([[0.0], np.cumsum(np.abs(val * x[col]))])
    return cs[rp[1:].astype(np.int64)] - cs[rp[:-1].astype(np.int64)]


# (the last case: mostly one-nonzero rows, so an x-slice row block holds
# more units than its workgroup has threads)
@pytest.mark.parametrize("n,mean,max_len,seed", [(3000, 16.0, 300, 50), (700, 4.0, 700, 51),
                                                 (5000, 64.0, 4096, 52), (257, 16.0, 257, 53),
                                                 (40000, 1.5, 40, 54)])
def test_pareto_matrices(env, orc, n, mean, max_len, seed):
    ao, torch, dev, st = env
    m = synth.csr_matrix(n, seed, mean=mean, max_len=max_len)
    want = orc.spmv_canonical(m["row_ptr"], m["col"], m["val"], m["x"])
    plain = orc.spmv_plain(m["row_ptr"], m["col"], m["val"], m["x"])
    _check_all(_run_all(ao, torch, dev, st, m, f"par{seed}"), want, plain, _scale(m))


def test_empty_long_and_signed_zero_rows(env, orc):
    ao, torch, dev, st = env
    # rows: empty, 1, 64, 65, 4096 (ones), empty, 130, 7 (-0.0 products), empty
    lens = [0, 1, 64, 65, 4096, 0, 130, 7, 0]
    n = 5000
    rp, col = synth.csr_structure(len(lens), n, np.array(lens), 61)
    val = synth.normal_values(col.size, 61)
    x = synth.dense_vector_pm1(n, 61)
    s = rp[4]
    col[s:s + 4096] = np.arange(4096)   # row 4: 4096 ones times ones
    val[s:s + 4096] = 1.0
    x[:4096] = 1.0
    z0 = rp[7]
    col[z0:z0 + 7] = np.arange(4096, 4103)
    val[z0:z0 + 7] = -1.0
    x[4096:4103] = 0.0                  # products -1 * +0 = -0.0 -> the row sums to -0.0
    m = {"row_ptr": rp, "col": col, "val": val, "x": x}
    # 9 rows over 5000 columns: x is longer than y
    want = orc.spmv_canonical(rp, col, val, x)
    assert want[4] == 4096.0 and np.signbit(want[7]) and want[0] == 0 and not np.signbit(want[0])
    plain = orc.spmv_plain(rp, col, val, x)
    _check_all(_run_all(ao, torch, dev, st, m, "edge"), want, plain, _scale(m))


def test_special_matrices_exact(env, orc):
    ao, torch, dev, st = env
    n = 1000
    x = synth.dense_vector_pm1(n, 71)
    perm = np.argsort(synth.splitmix64(72, n)).astype(np.int32)
    for name, col, val in (("ident", np.arange(n, dtype=np.int32), np.ones(n)),
                           ("perm", perm, np.ones(n)),
                           ("diag", np.arange(n, dtype=np.int32), 2.0 ** (np.arange(n) % 7 - 3))):
        m = {"row_ptr": np.arange(n + 1, dtype=np.int32), "col": col, "val": val, "x": x}
        for var, got in _run_all(ao, torch, dev, st, m, name):
            assert np.array_equal(got, val * x[col]), (name, var)


def test_features_match_oracle(env, orc):
    ao, torch, dev, st = env
    m = synth.csr_matrix(20000, 81, mean=16.0, max_len=4096)
    n = 20000
    t = {k: torch.from_numpy(v).to(dev) for k, v in m.items()}
    y = torch.empty(n, dtype=torch.float64, device=dev)
    h = ao.region_declare_variants("feat", ao.AO_CSR_SPMV_F64, ao.spmv_variants()[:1],
                                   model_type="roundrobin")
    ao.region_run(h, ao.spmv_args(t["row_ptr"], t["col"], t["val"], t["x"], y, n,
                                  int(m["col"].size)), stream=st)
    f, _, _ = ao.region_records(h)
    want = orc.csr_features(m["row_ptr"])
    assert np.allclose(np.array(f[0][:5]), want, rtol=1e-6, atol=0)
    assert f[0][5] == 0.0
    ao.region_destroy(h)


def test_full_size_2_22(env, orc):
    # n = 2^22 rows, Pareto tail 1.5, mean 16, max 4096, seed 5: all variants
    # bit-identical to the canonical oracle on every row
    ao, torch, dev, st = env
    m = synth.csr_matrix(1 << 22, 5)
    want = orc.spmv_canonical(m["row_ptr"], m["col"], m["val"], m["x"])
    n = 1 << 22
    t = {k: torch.from_numpy(v).to(dev) for k, v in m.items()}
    y = torch.empty(n, dtype=torch.float64, device=dev)
    vs = ao.spmv_variants(xslice=(13, 14))
    h = ao.region_declare_variants("full22", ao.AO_CSR_SPMV_F64, vs, model_type="roundrobin")
    a = ao.spmv_args(t["row_ptr"], t["col"], t["val"], t["x"], y, n, int(m["col"].size),
                     values_id=1)
    for v in list(range(len(vs))) + [9, 10]:  # the x-slice ones again: reordered values reused
        y.fill_(float("nan"))
        ao.region_run(h, a, stream=st, variant=v)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        assert np.array_equal(got, want), f"variant {v}: {int(np.sum(got != want))} rows differ"
    ao.region_destroy(h)


def test_reused_buffers_same_n_and_nnz(env, orc):
    # Regression: two matrices with equal n and nnz placed one after the other
    # in the same device buffers must not share the per-matrix plan (each
    # spmv_args call carries a fresh structure id).
    ao, torch, dev, st = env
    n = 1 << 14
    ma = synth.csr_matrix(n, 54, mean=16.0, tail=1.5)
    mb = synth.csr_matrix(n, 57, mean=16.0, tail=2.0)
    assert ma["col"].size == mb["col"].size and not np.array_equal(ma["row_ptr"], mb["row_ptr"])
    t = {k: torch.from_numpy(v).to(dev) for k, v in ma.items()}
    y = torch.empty(n, dtype=torch.float64, device=dev)
    vs = ao.spmv_variants(xslice=(13, 14))
    h = ao.region_declare_variants("reuse", ao.AO_CSR_SPMV_F64, vs, model_type="roundrobin")
    for q, m in enumerate((ma, mb)):
        for k, v in m.items():
            t[k].copy_(torch.from_numpy(v))
        a = ao.spmv_args(t["row_ptr"], t["col"], t["val"], t["x"], y, n, int(m["col"].size),
                         values_id=q + 1)
        want = orc.spmv_canonical(m["row_ptr"], m["col"], m["val"], m["x"])
        for v in range(len(vs)):
            y.fill_(float("nan"))
            ao.region_run(h, a, stream=st, variant=v)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy(), want), v
    ao.region_destroy(h)


def test_gather_probe_sums(env):
    # the probe's per-wave sums against the same gathers summed on the host:
    # wave w of workgroup g covers entries 2048 g + 64 w' + 256 u (u = 0..7,
    # w' = lane group of wave w); order differs, so compare within rounding
    ao, torch, dev, st = env
    n, m = 5000, 2048 * 3 + 700
    rng = np.random.default_rng(3)
    idx = rng.integers(-5, n + 5, size=m).astype(np.int32)  # a few out of range: read x[0]
    x = rng.standard_normal(n)
    out = torch.full((ao.gather_probe_out_len(m),), float("nan"), dtype=torch.float64, device=dev)
    ti, tx = torch.from_numpy(idx).to(dev), torch.from_numpy(x).to(dev)
    ao.ao_gather_probe(ti, tx, m, n, out, stream=st)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ic = np.where((idx >= 0) & (idx < n), idx, 0)
    want = np.zeros(got.size)
    for k in range(m):
        g, t = divmod(k, 2048)
        want[4 * g + (t % 256) // 64] += x[ic[k]]
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_xslice_values_id(env, orc):
    # The x-slice family keeps the values in its own order: with values id 0
    # the copy is refreshed every call; a nonzero id lets calls reuse it, and
    # changed values under a new id are picked up
    ao, torch, dev, st = env
    n = 20000
    m = synth.csr_matrix(n, 91, mean=16.0, max_len=2000)
    t = {k: torch.from_numpy(v).to(dev) for k, v in m.items()}
    y = torch.empty(n, dtype=torch.float64, device=dev)
    h = ao.region_declare_variants("xs_values", ao.AO_CSR_SPMV_F64,
                                   [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_XSLICE, 0, 13, 1, 0)],
                                   model_type="roundrobin")
    sid = 424242

    def run(vid):
        y.fill_(float("nan"))
        ao.region_run(h, ao.spmv_args(t["row_ptr"], t["col"], t["val"], t["x"], y, n,
                                      int(m["col"].size), structure_id=sid, values_id=vid),
                      stream=st, variant=0)
        torch.cuda.synchronize()
        return y.cpu().numpy()

    want = orc.spmv_canonical(m["row_ptr"], m["col"], m["val"], m["x"])
    assert np.array_equal(run(5), want)
    assert np.array_equal(run(5), want)        # reordered values reused
    val2 = m["val"] * -0.5
    t["val"].copy_(torch.from_numpy(val2))
    want2 = orc.spmv_canonical(m["row_ptr"], m["col"], val2, m["x"])
    assert np.array_equal(run(6), want2)       # new id: values reordered again
    assert np.array_equal(run(0), want2)       # id 0: reordered on every call
    t["val"].copy_(torch.from_numpy(m["val"]))
    assert np.array_equal(run(0), want)
    ao.region_destroy(h)


def test_xslice_refuses_rows_above_its_limit(env, orc):
    # a row of 5000 nonzeros is above the family's 4608 limit: its variant
    # fails to launch and is masked, the others still run
    ao, torch, dev, st = env
    lens = np.full(300, 3, dtype=np.int64)
    lens[17] = 5000
    n = 8000
    rp, col = synth.csr_structure(lens.size, n, lens, 95)
    val = synth.normal_values(col.size, 95)
    x = synth.dense_vector_pm1(n, 95)
    t = {k: torch.from_numpy(v).to(dev) for k, v in
         {"row_ptr": rp, "col": col, "val": val, "x": x}.items()}
    y = torch.empty(lens.size, dtype=torch.float64, device=dev)
    vs = [ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_XSLICE, 0, 14, 1, 0),
          ao.Variant(ao.AO_TARGET_GPU, ao.FAM_SPMV_MERGE_PATH, 256, 0, 1, 0)]
    h = ao.region_declare_variants("xs_limit", ao.AO_CSR_SPMV_F64, vs, model_type="roundrobin")
    a = ao.spmv_args(t["row_ptr"], t["col"], t["val"], t["x"], y, lens.size, int(col.size))
    with pytest.raises(ao.AdaptError) as ei:
        ao.region_run(h, a, stream=st, variant=0)
    assert ei.value.code == -7 or "cannot launch" in str(ei.value)
    ao.region_run(h, a, stream=st, variant=1)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), orc.spmv_canonical(rp, col, val, x))
    ao.region_destroy(h)
