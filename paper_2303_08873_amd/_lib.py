"""ctypes binding of libadaptomp.so: one Python function per C entry point,
same names, argument marshalling only."""
from __future__ import annotations

import ctypes
import itertools
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libadaptomp.so")

AO_OK, AO_NOTE_UNTRAINED, AO_NOTE_FALLBACK = 0, 1, 2
AO_MAX_VARIANTS, AO_MAX_FEATURES, AO_MLP_PARAMS = 12, 6, 5388
AO_JACOBI7_F64, AO_CSR_SPMV_F64, AO_CSR_RELAX_F64 = 0, 1, 2
AO_TARGET_GPU, AO_TARGET_HOST = 0, 1
FAM_JACOBI_DIRECT, FAM_JACOBI_ZMARCH, FAM_JACOBI_HOST, FAM_JACOBI_ZREG = 0, 1, 2, 3
FAM_JACOBI_ZREG_T2 = 4
FAM_JACOBI_ZREG_T3 = 5
FAM_JACOBI_ZREG_T4 = 6
FAM_JACOBI_COSCHED = 7
FAM_SPMV_THREAD_ROW, FAM_SPMV_WAVE_ROW, FAM_SPMV_MERGE_PATH, FAM_SPMV_XSLICE = 10, 11, 12, 13
AO_VF_NT_STORE = 1
AO_VF_HALO_PREFETCH = 2
AO_VF_OCCUPANCY = 4
AO_VF_STAGED = 8
AO_VF_LDS_SWEEPS = 16
AO_VF_FILL_Z = 32
AO_PROFILE_RECORD = 1

_STATUS = {-1: "AO_EINVAL", -2: "AO_ENOMEM", -3: "AO_EHIP", -4: "AO_ESTATE", -5: "AO_EEXIST",
           -6: "AO_EIO", -7: "AO_ELAUNCH"}


class AdaptError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Variant(ctypes.Structure):
    _fields_ = [("target", ctypes.c_int32), ("family", ctypes.c_int32), ("bx", ctypes.c_int32),
                ("by", ctypes.c_int32), ("bz", ctypes.c_int32), ("flags", ctypes.c_int32)]

    def __repr__(self):
        return (f"Variant(target={self.target}, family={self.family}, bx={self.bx}, by={self.by}, "
                f"bz={self.bz}, flags={self.flags})")


class Args(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("resident", ctypes.c_int32),
                ("u0", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("sweeps", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("structure_id", ctypes.c_uint64), ("values_id", ctypes.c_uint64),
                ("b", ctypes.c_void_p), ("diag", ctypes.c_void_p), ("omega", ctypes.c_double)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("records", ctypes.c_int64), ("unique", ctypes.c_int64),
                ("trained", ctypes.c_int32), ("num_variants", ctypes.c_int32),
                ("explore_next", ctypes.c_int64), ("trainings", ctypes.c_int64),
                ("fallbacks", ctypes.c_int64), ("failed_mask", ctypes.c_int32),
                ("min_train", ctypes.c_int32), ("memo_size", ctypes.c_int64),
                ("last_train_seconds", ctypes.c_double), ("train_failures", ctypes.c_int64)]


def _load():
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one.  Loading torch first makes this library bind to that runtime, so
    # the process holds a single HIP runtime whose device pointers and
    # streams both sides share.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(lib_path):
        raise ImportError(f"{lib_path} is not built; run `python paper_2303_08873_amd/build.py` "
                          "(the package has no fallback path)")
    L = ctypes.CDLL(lib_path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    sig = {
        "region_declare_variants": [ctypes.c_char_p, I, P, I, I, ctypes.c_char_p, P],
        "region_run": [P, P, P, P, I, P],
        "region_record": [P, P, I, ctypes.c_double],
        "region_run_noalloc": [P, P, P, I],
        "region_features": [P, P, P, P],
        "region_profile": [P, P, P, I, I, I, P, I, P],
        "selector_train": [P, P, P],
        "selector_select": [P, P, I, P],
        "batch_create": [P, I, P],
        "batch_autotune": [P, P, I, I, P],
        "batch_run": [P, P, I],
        "batch_info": [P, P, P, P],
        "batch_candidates": [P],
        "batch_min_traffic": [P, P],
        "batch_set_tiles": [P, P],
        "batch_destroy": [P],
        "ao_mlp_forward": [P, P, I, P, P],
        "ao_mlp_grad": [P, P, P, P, I, P, P, P],
        "ao_mlp_adam": [P, P, P, P, I, ctypes.c_float, P],
        "region_stats": [P, P],
        "region_records": [P, P, P, P, I],
        "region_save": [P, ctypes.c_char_p],
        "region_load": [P, ctypes.c_char_p],
        "region_clear_memo": [P],
        "region_destroy": [P],
        "ao_device_cus": [],
        "ao_jacobi_planes": [P, I, I, I, I, I, P],
        "ao_hbm_copy": [P, P, ctypes.c_int64, I, P],
        "ao_gather_probe": [P, P, ctypes.c_int64, ctypes.c_int64, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.ao_last_error.argtypes = []
    L.ao_last_error.restype = ctypes.c_char_p
    return L


lib = _load()


def ao_last_error() -> str:
    return lib.ao_last_error().decode(errors="replace")


def _check(rc: int) -> int:
    if rc < 0:
        raise AdaptError(rc, ao_last_error())
    return rc


def _ptr(x):
    """Address of a torch tensor, numpy array, ctypes object or int (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    return ctypes.addressof(x)


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def region_declare_variants(model_name: str, kind: int, variants, min_train_data: int = 0,
                            model_type: str | None = None):
    arr = (Variant * len(variants))(*variants)
    h = ctypes.c_void_p()
    _check(lib.region_declare_variants(model_name.encode(), kind, arr, len(variants),
                                       min_train_data,
                                       model_type.encode() if model_type else None,
                                       ctypes.byref(h)))
    return h


def region_run(region, args: Args, features=None, stream=None, variant: int = -1):
    """Returns (status, chosen variant id)."""
    chosen = ctypes.c_int(-1)
    fbuf = None
    if features is not None:
        fbuf = (ctypes.c_float * AO_MAX_FEATURES)(*[float(v) for v in list(features)[:AO_MAX_FEATURES]])
    rc = _check(lib.region_run(region, ctypes.byref(args), fbuf, _stream(stream), variant,
                               ctypes.byref(chosen)))
    return rc, chosen.value


def region_run_noalloc(region, args: Args, variant: int, stream=None) -> int:
    """Run GPU variant `variant` without allocating (the library's static
    scratch array); returns the status."""
    return _check(lib.region_run_noalloc(region, ctypes.byref(args), _stream(stream), variant))


def region_features(region, args: Args, stream=None) -> list:
    out = (ctypes.c_float * AO_MAX_FEATURES)()
    _check(lib.region_features(region, ctypes.byref(args), _stream(stream), out))
    return list(out)


def region_record(region, features, variant: int, seconds: float) -> None:
    fbuf = (ctypes.c_float * AO_MAX_FEATURES)(*[float(v) for v in list(features)[:AO_MAX_FEATURES]])
    _check(lib.region_record(region, fbuf, variant, seconds))


def region_profile(region, args: Args, variant: int = -1, warmup: int = 3, reps: int = 10,
                   stream=None, record: bool = False, features=None, num_variants: int | None = None):
    """Median seconds per variant (list of num_variants, or one float)."""
    nv = 1 if variant >= 0 else (num_variants or region_stats(region).num_variants)
    out = (ctypes.c_double * nv)()
    fbuf = None
    if features is not None:
        fbuf = (ctypes.c_float * AO_MAX_FEATURES)(*[float(v) for v in list(features)[:AO_MAX_FEATURES]])
    _check(lib.region_profile(region, ctypes.byref(args), fbuf, variant, warmup, reps,
                              _stream(stream), AO_PROFILE_RECORD if record else 0, out))
    return out[0] if variant >= 0 else list(out)


def selector_train(region, epochs: int = 200, batch: int = 256, lr: float = 1e-3, seed: int = 7):
    opts = TrainOpts(epochs, batch, lr, seed)
    loss = ctypes.c_double(float("nan"))
    _check(lib.selector_train(region, ctypes.byref(opts), ctypes.byref(loss)))
    return loss.value


def selector_select(region, features):
    """features: [batch][6] floats -> (status, list of ids)."""
    rows = [list(map(float, r)) + [0.0] * (AO_MAX_FEATURES - len(r)) for r in features]
    n = len(rows)
    fbuf = (ctypes.c_float * (n * AO_MAX_FEATURES))(*[v for r in rows for v in r])
    out = (ctypes.c_int * max(n, 1))()
    rc = _check(lib.selector_select(region, fbuf, n, out))
    return rc, list(out)[:n]


def region_stats(region) -> Stats:
    st = Stats()
    _check(lib.region_stats(region, ctypes.byref(st)))
    return st


def region_records(region, max_records: int | None = None):
    """(features [n][6], variants [n], seconds [n]) as Python lists."""
    if max_records is None:
        max_records = region_stats(region).records
    f = (ctypes.c_float * (max_records * AO_MAX_FEATURES + 1))()
    v = (ctypes.c_int * (max_records + 1))()
    s = (ctypes.c_double * (max_records + 1))()
    n = _check(lib.region_records(region, f, v, s, max_records))
    feats = [list(f[i * AO_MAX_FEATURES:(i + 1) * AO_MAX_FEATURES]) for i in range(n)]
    return feats, list(v)[:n], list(s)[:n]


def region_save(region, path: str) -> None:
    _check(lib.region_save(region, path.encode()))


def region_load(region, path: str) -> None:
    _check(lib.region_load(region, path.encode()))


def region_clear_memo(region) -> None:
    _check(lib.region_clear_memo(region))


def region_destroy(region) -> None:
    _check(lib.region_destroy(region))


def ao_hbm_copy(src, dst, n: int, nontemporal: bool = False, stream=None) -> None:
    _check(lib.ao_hbm_copy(_ptr(src), _ptr(dst), n, 1 if nontemporal else 0, _stream(stream)))


def gather_probe_out_len(m: int) -> int:
    """Doubles ao_gather_probe writes for m indices."""
    return 4 * ((m + 2047) // 2048)


def ao_gather_probe(idx, x, m: int, nx: int, out, stream=None) -> None:
    _check(lib.ao_gather_probe(_ptr(idx), _ptr(x), m, nx, _ptr(out), _stream(stream)))


def ao_device_cus() -> int:
    return lib.ao_device_cus()


def ao_jacobi_planes(variant: Variant, nx: int, ny: int, nz: int, cus: int = 0,
                     blocks_per_cu: int = 0) -> int:
    """Planes per block one launch of a register z-march variant uses on an
    nx x ny x nz grid (for `cus` CUs holding `blocks_per_cu` workgroups
    each; cus = 0: the current device and the kernel's occupancy)."""
    out = ctypes.c_int32()
    _check(lib.ao_jacobi_planes(ctypes.byref(variant), nx, ny, nz, cus, blocks_per_cu,
                                ctypes.byref(out)))
    return out.value


def batch_create(instances):
    arr = (Args * len(instances))(*instances)
    h = ctypes.c_void_p()
    _check(lib.batch_create(arr, len(instances), ctypes.byref(h)))
    return h


def batch_autotune(batch, stream=None, warmup: int = 2, reps: int = 5):
    chosen = (ctypes.c_int * 5)()
    _check(lib.batch_autotune(batch, _stream(stream), warmup, reps, chosen))
    return list(chosen)


def batch_run(batch, stream=None, use_graph: bool = True) -> None:
    _check(lib.batch_run(batch, _stream(stream), 1 if use_graph else 0))


def batch_info(batch):
    inst = (ctypes.c_int * 5)()
    items = (ctypes.c_int * 5)()
    tiles = (ctypes.c_int * 15)()
    _check(lib.batch_info(batch, inst, items, tiles))
    return list(inst), list(items), [tuple(tiles[3 * b:3 * b + 3]) for b in range(5)]


def batch_min_traffic(batch) -> float:
    """Least HBM bytes one batch_run moves with the tiles in use."""
    out = ctypes.c_double(0.0)
    _check(lib.batch_min_traffic(batch, ctypes.byref(out)))
    return out.value


def batch_candidates():
    n = lib.batch_candidates(None)
    tiles = (ctypes.c_int * (4 * n))()
    lib.batch_candidates(tiles)
    return [tuple(tiles[4 * c:4 * c + 4]) for c in range(n)]


def batch_set_tiles(batch, cand) -> None:
    arr = (ctypes.c_int * 5)(*cand)
    _check(lib.batch_set_tiles(batch, arr))


def batch_destroy(batch) -> None:
    _check(lib.batch_destroy(batch))


def ao_mlp_forward(params, x, batch: int, out, stream=None) -> None:
    _check(lib.ao_mlp_forward(_ptr(params), _ptr(x), batch, _ptr(out), _stream(stream)))


def ao_mlp_grad(params, x, y, mask, batch: int, grad, loss=None, stream=None) -> None:
    _check(lib.ao_mlp_grad(_ptr(params), _ptr(x), _ptr(y), _ptr(mask), batch, _ptr(grad),
                           _ptr(loss), _stream(stream)))


def ao_mlp_adam(params, m, v, grad, t: int, lr: float = 1e-3, stream=None) -> None:
    _check(lib.ao_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), t, lr, _stream(stream)))


def jacobi_args(u0, out, nx: int, ny: int, nz: int, sweeps: int, resident: int = 1) -> Args:
    a = Args()
    a.kind = AO_JACOBI7_F64
    a.resident = resident
    a.u0 = _ptr(u0)
    a.out = _ptr(out)
    a.nx, a.ny, a.nz, a.sweeps = nx, ny, nz, sweeps
    return a


_structure_ids = itertools.count(1)


def spmv_args(row_ptr, col, val, x, y, n: int, nnz: int, structure_id: int | None = None,
              values_id: int = 0) -> Args:
    """Arguments of one SpMV execution.  Unless given, every call issues a
    fresh structure id, so the library's per-matrix plan is shared by the
    executions that reuse this Args object and never by another matrix.
    values_id (0 = unknown) names the contents of val: a nonzero id lets
    the x-slice family reuse its reordered copy of the values while the id
    stays the same; give changed values a new id."""
    a = Args()
    a.structure_id = next(_structure_ids) if structure_id is None else structure_id
    a.values_id = int(values_id)
    a.kind = AO_CSR_SPMV_F64
    a.resident = 1
    a.row_ptr, a.col, a.val, a.x, a.y = _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y)
    a.n, a.nnz = n, nnz
    return a


def relax_args(row_ptr, col, val, x, y, b, diag, omega: float, sweeps: int, n: int, nnz: int,
               structure_id: int | None = None, values_id: int = 0) -> Args:
    """Arguments of one weighted-Jacobi relaxation execution (S sweeps of
    x <- x + omega (b - A x) / diag from x into y); structure and values
    ids as for spmv_args."""
    a = spmv_args(row_ptr, col, val, x, y, n, nnz, structure_id, values_id)
    a.kind = AO_CSR_RELAX_F64
    a.b, a.diag, a.omega, a.sweeps = _ptr(b), _ptr(diag), float(omega), int(sweeps)
    return a
