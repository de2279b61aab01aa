"""Host-side checks of the C-ABI library that need no GPU: every declared
symbol is exported, the host-CPU Jacobi variants are bit-exact against the
oracle, and the runtime's state machine (RoundRobin, train trigger,
persistence, argument errors) follows the oracle's explorer."""
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adaptomp.h")


@pytest.fixture(scope="module")
def ao():
    import paper_2303_08873_amd as ao
    return ao


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_symbols_exported(ao):
    names = _declared_functions()
    assert "region_declare_variants" in names and "selector_train" in names
    for n in names:
        assert hasattr(ao.lib, n), f"{n} declared in adaptomp.h but not exported"


def _host_region(ao, name, model_type="roundrobin", min_train=0):
    vs = ao.jacobi_sweep_host()
    return ao.region_declare_variants(name, ao.AO_JACOBI7_F64, vs, min_train, model_type)


@pytest.mark.parametrize("shape,S", [((20, 17, 9), 3), ((1, 1, 40), 2), ((65, 3, 7), 1),
                                     ((5, 130, 2), 4), ((2, 2, 2), 0)])
def test_host_variants_bit_exact(ao, orc, shape, S):
    nx, ny, nz = shape
    u0 = synth.grid_u01(nx, ny, nz, seed=7)
    want = orc.jacobi7(u0, nx, ny, nz, S)
    h = _host_region(ao, f"host_exact_{nx}_{ny}_{nz}_{S}")
    out = np.zeros_like(u0)
    a = ao.jacobi_args(u0, out, nx, ny, nz, S, resident=0)
    for v in range(5):
        out[:] = -1.0
        ao.region_run(h, a, variant=v)
        assert np.array_equal(out, want), v
    ao.region_destroy(h)


def test_roundrobin_and_trigger_follow_oracle(ao, orc):
    # mlp model type: the trigger attempts training when the oracle explorer
    # says so; with no GPU here the training fails, which region_stats counts.
    h = _host_region(ao, "rr_trigger", model_type="mlp", min_train=7)
    ex = orc.RoundRobinExplorer(5, min_train=7)
    u0 = synth.grid_u01(6, 5, 4, seed=3)
    out = np.zeros_like(u0)
    a = ao.jacobi_args(u0, out, 6, 5, 4, 1, resident=0)
    feats = [[1.0, 0, 0, 0, 0, 0], [1.0, 0, 0, 0, 0, 0], [2.0, 0, 0, 0, 0, 0]]
    fired_at = None
    for k in range(9):
        f = feats[min(k // 3, 2)] if k < 6 else [float(k), 0, 0, 0, 0, 0]
        rc, v = ao.region_run(h, a, features=f)
        want_v, fire = ex.step(f)
        assert v == want_v and rc == ao.AO_NOTE_UNTRAINED
        st = ao.region_stats(h)
        if fire:
            fired_at = k
        assert st.unique == len(ex.unique)
        if ao.ao_device_cus() == 0:
            assert st.train_failures == (1 if fired_at is not None else 0)
            if fired_at is not None:
                ex.trained = False  # the library keeps exploring after a failed training
        elif fire:
            assert st.trained == 1 and st.trainings == 1
            break
    assert fired_at is not None
    ao.region_destroy(h)


def test_declare_idempotent_and_conflict(ao):
    vs = ao.jacobi_sweep_host()
    h1 = ao.region_declare_variants("idem", ao.AO_JACOBI7_F64, vs)
    h2 = ao.region_declare_variants("idem", ao.AO_JACOBI7_F64, vs)
    assert h1.value == h2.value
    with pytest.raises(ao.AdaptError) as e:
        ao.region_declare_variants("idem", ao.AO_JACOBI7_F64, vs[:3])
    assert e.value.code == -5
    ao.region_destroy(h1)


def test_argument_errors(ao):
    h = _host_region(ao, "argerr")
    u0 = np.zeros(8)
    out = np.zeros(8)
    with pytest.raises(ao.AdaptError) as e:
        ao.region_run(h, ao.jacobi_args(u0, u0, 2, 2, 2, 1, resident=0), variant=0)
    assert e.value.code == -1  # u0 and out overlap
    with pytest.raises(ao.AdaptError):
        ao.region_run(h, ao.jacobi_args(u0, out, 2, 2, 2, 1, resident=0), variant=5)
    with pytest.raises(ao.AdaptError):
        ao.region_run(h, ao.jacobi_args(u0, out, -1, 2, 2, 1, resident=0), variant=0)
    with pytest.raises(ao.AdaptError):  # rows longer than 2^28 (checked before any access)
        ao.region_run(h, ao.jacobi_args(u0, out, (1 << 28) + 1, 1, 1, 1, resident=0), variant=0)
    bad = ao.Variant(ao.AO_TARGET_HOST, ao.FAM_JACOBI_DIRECT, 64, 1, 1, 0)
    with pytest.raises(ao.AdaptError):
        ao.region_declare_variants("badvar", ao.AO_JACOBI7_F64, [bad])
    with pytest.raises(ao.AdaptError):
        ao.region_declare_variants("badtype", ao.AO_JACOBI7_F64, [ao.jacobi_sweep_host()[0]],
                                   model_type="forest")
    with pytest.raises(ao.AdaptError):
        ao.region_declare_variants("toomany", ao.AO_JACOBI7_F64, ao.jacobi_variants_sweep() * 2)
    # z-march families accept only the row counts they are compiled for
    G = ao.AO_TARGET_GPU
    for fam, rows in ((ao.FAM_JACOBI_ZREG, (3, 16)), (ao.FAM_JACOBI_ZREG_T2, (5, 7, 9, 32)),
                      (ao.FAM_JACOBI_ZREG_T3, (7, 10, 12, 16)), (ao.FAM_JACOBI_ZREG_T4, (6, 8))):
        for r in rows:
            with pytest.raises(ao.AdaptError):
                ao.region_declare_variants(f"rows_{fam}_{r}", ao.AO_JACOBI7_F64,
                                           [ao.Variant(G, fam, 64, r, 8, 0)])
        with pytest.raises(ao.AdaptError):  # strip width other than 64
            ao.region_declare_variants(f"width_{fam}", ao.AO_JACOBI7_F64,
                                       [ao.Variant(G, fam, 32, 2, 8, 0)])
        with pytest.raises(ao.AdaptError):  # no planes per block
            ao.region_declare_variants(f"bz_{fam}", ao.AO_JACOBI7_F64,
                                       [ao.Variant(G, fam, 64, 2, 0, 0)])
    ok = [ao.Variant(G, ao.FAM_JACOBI_ZREG_T2, 64, r, 8, 0) for r in (1, 2, 3, 4, 6, 8, 10, 12, 16)]
    ao.region_destroy(ao.region_declare_variants("t2rows", ao.AO_JACOBI7_F64, ok))
    ok = [ao.Variant(G, ao.FAM_JACOBI_ZREG_T3, 64, r, 8, 1) for r in (1, 2, 3, 4, 5, 6, 8)]
    ao.region_destroy(ao.region_declare_variants("t3rows", ao.AO_JACOBI7_F64, ok))
    ok = [ao.Variant(G, ao.FAM_JACOBI_ZREG_T4, 64, r, 8, 1) for r in (1, 2, 3, 4, 5)]
    ao.region_destroy(ao.region_declare_variants("t4rows", ao.AO_JACOBI7_F64, ok))
    ok = [ao.Variant(G, fam, 64, 4, 16, fl) for fam in (ao.FAM_JACOBI_ZREG_T3, ao.FAM_JACOBI_ZREG_T4)
          for fl in (ao.AO_VF_STAGED, ao.AO_VF_STAGED | ao.AO_VF_NT_STORE)]
    ao.region_destroy(ao.region_declare_variants("staged_ok", ao.AO_JACOBI7_F64, ok))
    for fam, fl in ((ao.FAM_JACOBI_ZREG_T2, ao.AO_VF_STAGED), (ao.FAM_JACOBI_ZREG, ao.AO_VF_STAGED),
                    (ao.FAM_JACOBI_ZREG_T4, ao.AO_VF_STAGED | ao.AO_VF_HALO_PREFETCH)):
        with pytest.raises(ao.AdaptError):  # staging only for the three- and four-sweep marches
            ao.region_declare_variants(f"staged_bad_{fam}_{fl}", ao.AO_JACOBI7_F64,
                                       [ao.Variant(G, fam, 64, 4, 16, fl)])
    ok = [ao.Variant(G, ao.FAM_JACOBI_COSCHED, f, 0, 0, 0) for f in range(11)]
    ao.region_destroy(ao.region_declare_variants("cosched_ok", ao.AO_JACOBI7_F64, ok))
    for bad in ((11, 0, 0), (-1, 0, 0), (5, 1, 0), (5, 0, 2)):
        with pytest.raises(ao.AdaptError):
            ao.region_declare_variants(f"cosched_bad_{bad}", ao.AO_JACOBI7_F64,
                                       [ao.Variant(G, ao.FAM_JACOBI_COSCHED, *bad, 0)])
    ao.region_destroy(h)


def test_save_load_roundtrip_and_corruption(ao, tmp_path):
    h = _host_region(ao, "persist")
    u0 = synth.grid_u01(5, 4, 3, seed=2)
    out = np.zeros_like(u0)
    a = ao.jacobi_args(u0, out, 5, 4, 3, 2, resident=0)
    for _ in range(7):
        ao.region_run(h, a)
    ao.region_record(h, [3.0, 1, 1, 1, 1, 0], 2, 0.5)
    f0, v0, s0 = ao.region_records(h)
    path = str(tmp_path / "db.bin")
    ao.region_save(h, path)
    h2 = _host_region(ao, "persist2")
    ao.region_load(h2, path)
    f1, v1, s1 = ao.region_records(h2)
    assert f0 == f1 and v0 == v1 and s0 == s1 and len(v0) == 8
    assert ao.region_stats(h2).unique == ao.region_stats(h).unique
    raw = bytearray(open(path, "rb").read())
    raw[40] ^= 0xFF
    bad = str(tmp_path / "bad.bin")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(ao.AdaptError) as e:
        ao.region_load(h2, bad)
    assert e.value.code == -6
    assert ao.region_records(h2)[1] == v0  # unchanged after a failed load
    with pytest.raises(ao.AdaptError):
        ao.region_load(h2, str(tmp_path / "missing.bin"))
    other = ao.region_declare_variants("persist_other", ao.AO_JACOBI7_F64,
                                       ao.jacobi_sweep_host()[:3])
    with pytest.raises(ao.AdaptError):
        ao.region_load(other, path)
    for x in (h, h2, other):
        ao.region_destroy(x)


def test_record_validation(ao):
    h = _host_region(ao, "recval")
    with pytest.raises(ao.AdaptError):
        ao.region_record(h, [1, 2, 3, 4, 5, 6], 9, 1.0)
    with pytest.raises(ao.AdaptError):
        ao.region_record(h, [1, 2, 3, 4, 5, 6], 1, -1.0)
    ao.region_record(h, [1, 2, 3, 4, 5, 6], 1, 1e-3)
    assert ao.region_stats(h).records == 1
    ao.region_destroy(h)


def test_selector_select_untrained_returns_exploration_id(ao):
    h = _host_region(ao, "seluntrained")
    rc, ids = ao.selector_select(h, [[1, 2, 3, 4, 5, 6]] * 3)
    assert rc == ao.AO_NOTE_UNTRAINED and ids == [0, 0, 0]
    ao.region_destroy(h)


def test_batch_candidate_table_and_tile_errors(ao):
    cands = ao.batch_candidates()
    assert len(cands) == ao.lib.batch_candidates(None) >= 16
    for kind, tx, ty, tz in cands:
        assert kind in (0, 1, 2, 4, 11, 12, 14, 21, 22, 24) and tz >= 1
        if kind in (1, 2, 4):
            assert (tx, ty) == (64, 4 * kind)
        if 10 < kind < 20:
            assert (tx, ty) == (62, 4 * (kind - 10))
        if kind > 20:
            assert (tx, ty) == (60, 4 * (kind - 20))
    assert {k for k, *_ in cands} >= {0, 1, 11, 21}
    with pytest.raises(ao.AdaptError):
        ao.batch_set_tiles(None, [0] * 5)


def test_args_and_variant_layout_match_the_header(ao, tmp_path):
    # the ctypes mirrors of ao_args / ao_variant / ao_train_opts / ao_stats
    # must match the C layout field by field
    import ctypes
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"ao_args": ao.Args, "ao_variant": ao.Variant, "ao_train_opts": ao.TrainOpts,
               "ao_stats": ao.Stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "adaptomp.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_relax_argument_errors(ao):
    # argument checks run before any device work
    import numpy as np
    vs = ao.spmv_variants(blocks=(256,))
    h = ao.region_declare_variants("relax_args_cpu", ao.AO_CSR_RELAX_F64, vs)
    n = 16
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    val = np.ones(n)
    x, y, b, d = np.zeros(n), np.zeros(n), np.ones(n), np.ones(n)
    bad = [ao.relax_args(rp, col, val, x, x, b, d, 1.0, 2, n, n),        # y is x
           ao.relax_args(rp, col, val, x, y, None, d, 1.0, 2, n, n),     # no b
           ao.relax_args(rp, col, val, x, y, b, None, 1.0, 2, n, n),     # no diag
           ao.relax_args(rp, col, val, x, y, b, d, float("inf"), 2, n, n),
           ao.relax_args(rp, col, val, x, y, b, d, 1.0, -1, n, n),
           ao.relax_args(rp, col, val, x, b, b, d, 1.0, 2, n, n)]       # y is b
    host = ao.relax_args(rp, col, val, x, y, b, d, 1.0, 2, n, n)
    host.resident = 0                                                  # device only
    bad.append(host)
    for a in bad:
        with pytest.raises(ao.AdaptError) as e:
            ao.region_run(h, a, variant=0)
        assert e.value.code == -1
    ao.region_destroy(h)
    with pytest.raises(ao.AdaptError):   # relaxation variants run on the GPU
        ao.region_declare_variants("relax_host", ao.AO_CSR_RELAX_F64,
                                   [ao.jacobi_sweep_host()[0]])


def test_xslice_spmv_variant_validation(ao):
    G = ao.AO_TARGET_GPU
    ok = [ao.Variant(G, ao.FAM_SPMV_XSLICE, 0, swl, 1, 0) for swl in (0, 13, 14)]
    for kind in (ao.AO_CSR_SPMV_F64, ao.AO_CSR_RELAX_F64):
        ao.region_destroy(ao.region_declare_variants(f"xslice_ok_{kind}", kind, ok))
    for b, swl in ((256, 14), (0, 12), (0, 15), (0, 16)):
        with pytest.raises(ao.AdaptError):
            ao.region_declare_variants(f"xslice_bad_{b}_{swl}", ao.AO_CSR_SPMV_F64,
                                       [ao.Variant(G, ao.FAM_SPMV_XSLICE, b, swl, 1, 0)])


@pytest.mark.parametrize("resident", [0, 1])
def test_stencil_features_match_oracle(ao, orc, resident):
    # The feature vector the runtime feeds the cost model for a Jacobi region
    # (Sec. 3.1 features clause) equals the oracle's, for ragged, degenerate
    # (extent 0 or 1) and large shapes and sweep counts.  Host arithmetic:
    # no GPU is needed and the buffer addresses are never dereferenced.
    h = ao.region_declare_variants(f"feat_stencil_{resident}", ao.AO_JACOBI7_F64,
                                   ao.jacobi_variants_blocks(), model_type="roundrobin")
    shapes = [(64, 32, 16, 10), (1, 1, 1, 1), (0, 5, 7, 3), (5, 0, 7, 20), (7, 5, 0, 5),
              (37, 29, 13, 3), (512, 512, 512, 20), (8, 512, 100, 5), (3, 1, 1000, 0),
              (1 << 20, 1, 1, 2), (160, 160, 160, 7), (2, 3, 1, 1)]
    for nx, ny, nz, S in shapes:
        a = ao.Args()
        a.kind, a.resident = ao.AO_JACOBI7_F64, resident
        a.nx, a.ny, a.nz, a.sweeps = nx, ny, nz, S
        n = nx * ny * nz
        if n > 0:
            a.u0, a.out = 1 << 20, (1 << 20) + 8 * n + 64
        got = np.asarray(ao.region_features(h, a), dtype=np.float32)
        want = orc.stencil_features(nx, ny, nz, S, resident)
        assert got.tobytes() == want.tobytes(), ((nx, ny, nz, S), got, want)
    ao.region_destroy(h)


def test_lds_sweeps_flag_only_on_the_direct_family(ao):
    G = ao.AO_TARGET_GPU
    ok = ao.region_declare_variants("lds_flag_ok", ao.AO_JACOBI7_F64,
                                    [ao.Variant(G, ao.FAM_JACOBI_DIRECT, 64, 16, 1,
                                                ao.AO_VF_LDS_SWEEPS)])
    ao.region_destroy(ok)
    with pytest.raises(ao.AdaptError):
        ao.region_declare_variants("lds_flag_bad", ao.AO_JACOBI7_F64,
                                   [ao.Variant(G, ao.FAM_JACOBI_ZREG_T3, 64, 4, 4,
                                               ao.AO_VF_LDS_SWEEPS)])
    # the size-sweep table: the static default is the plain 256-thread kernel
    vs = ao.jacobi_variants_sweep()
    from paper_2303_08873_amd.variants import STATIC_DEFAULT
    d = vs[STATIC_DEFAULT]
    assert (d.family, d.bx * d.by, d.flags) == (ao.FAM_JACOBI_DIRECT, 256, 0)
    assert len(ao.jacobi_sweep_gpu()) + len(ao.jacobi_sweep_host()) == len(vs)
    assert all(v.target == G for v in ao.jacobi_sweep_gpu())
    assert all(v.target == ao.AO_TARGET_HOST for v in ao.jacobi_sweep_host())
