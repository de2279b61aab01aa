"""Seeded synthetic inputs for the adaptive-region workloads.

This module is shared by the CPU oracle tests and the HIP path.  It holds
none of the method's arithmetic: only random draws and the shapes, value
distributions and sparsity structure of the workloads.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used counter-style: output i
(1-based) of the stream seeded with s is mix(s + i * 0x9E3779B97F4A7C15)
where mix is the published finaliser (xor-shift 30, multiply
0xBF58476D1CE4E5B9, xor-shift 27, multiply 0x94D049BB133111EB, xor-shift 31).

Independent quantities of one workload use sub-streams: the seed of
sub-stream ``tag`` of seed ``s`` is mix((s << 8) | tag) (64-bit wrap).
"""
from __future__ import annotations

import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1
_CHUNK = 1 << 24


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def mix64(v: int) -> int:
    """The SplitMix64 finaliser of one 64-bit integer."""
    return int(_mix(np.array([v & _MASK64], dtype=np.uint64))[0])


def substream(seed: int, tag: int) -> int:
    """Seed of sub-stream ``tag`` (0..255) of ``seed``."""
    return mix64(((seed << 8) | (tag & 0xFF)) & _MASK64)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start+1 .. start+count of SplitMix64(seed), as uint64."""
    out = np.empty(count, dtype=np.uint64)
    s = np.uint64(seed & _MASK64)
    for lo in range(0, count, _CHUNK):
        hi = min(count, lo + _CHUNK)
        i = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            out[lo:hi] = _mix(s + i * _GAMMA)
    return out


def u01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1): (z >> 11) * 2^-53, each exactly representable."""
    out = np.empty(count, dtype=np.float64)
    for lo in range(0, count, _CHUNK):
        hi = min(count, lo + _CHUNK)
        z = splitmix64(seed, hi - lo, start + lo)
        out[lo:hi] = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return out


def u01_open0(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in (0, 1]: ((z >> 11) + 1) * 2^-53."""
    z = splitmix64(seed, count, start)
    return ((z >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------
# Structured grids
# --------------------------------------------------------------------------

def grid_u01(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """Initial field u0 ~ U[0,1) of an nx*ny*nz grid, x fastest:
    element (i, j, k) sits at flat index (k*ny + j)*nx + i and takes draw
    number that index (0-based) of SplitMix64(seed)."""
    return u01(seed, nx * ny * nz)


def _log_uniform_int(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    u = u01(seed, count)
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def batch_shapes(count: int = 256, lo: int = 8, hi: int = 256, seed: int = 3) -> np.ndarray:
    """[count, 3] grid shapes (nx, ny, nz), each dimension
    round(exp(U[ln lo, ln hi])); draws are taken nx, ny, nz per instance."""
    return _log_uniform_int(substream(seed, 1), 3 * count, lo, hi).reshape(count, 3)


def selector_shapes(count: int, seed: int, lo: int = 8, hi: int = 512,
                    sweeps=(5, 10, 20)):
    """Shapes of the cost-model workload: per-axis dims log-uniform in
    [lo, hi], sweeps drawn uniformly from ``sweeps``, residency 50/50
    (1 = device memory, 0 = pinned host memory).

    Returns (dims [count,3] int64, sweeps [count] int64, resident [count] int64).
    """
    dims = _log_uniform_int(substream(seed, 1), 3 * count, lo, hi).reshape(count, 3)
    k = np.minimum((u01(substream(seed, 2), count) * len(sweeps)).astype(np.int64), len(sweeps) - 1)
    s = np.asarray(sweeps, dtype=np.int64)[k]
    res = (u01(substream(seed, 3), count) < 0.5).astype(np.int64)
    return dims, s, res


# --------------------------------------------------------------------------
# Sparse matrices (CSR, int32 indices, float64 values)
# --------------------------------------------------------------------------

def pareto_row_lengths(n: int, seed: int, mean: float = 16.0, tail: float = 1.5,
                       max_len: int = 4096) -> np.ndarray:
    """Row lengths L = min(max_len, ceil(scale * U^(-1/tail))), U in (0,1],
    scale = mean*(tail-1)/tail (so the untruncated Pareto mean is ``mean``)."""
    scale = mean * (tail - 1.0) / tail
    u = u01_open0(substream(seed, 1), n)
    lengths = np.ceil(scale * np.power(u, -1.0 / tail))
    return np.minimum(lengths, float(max_len)).astype(np.int64)


def csr_structure(n_rows: int, n_cols: int, lengths: np.ndarray, seed: int):
    """row_ptr (int32, n_rows+1) and col (int32, nnz): row i holds lengths[i]
    distinct columns drawn uniformly from [0, n_cols), stored ascending.
    Duplicates within a row are redrawn from further sub-streams
    (tags 16, 17, ...) until none remain.  A row longer than n_cols / 4
    instead takes the first lengths[i] columns of a random order of all
    columns (SplitMix64 keys of sub-stream 15 xor the row index)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.size and int(lengths.max()) > n_cols:
        raise ValueError("a row cannot hold more distinct columns than the matrix has")
    row_ptr64 = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr64[1:])
    nnz = int(row_ptr64[-1])
    if nnz >= 2 ** 31:
        raise ValueError("nnz must fit int32 indices")
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), lengths)
    cols = np.floor(u01(substream(seed, 2), nnz) * n_cols).astype(np.int64)
    for r in np.nonzero(lengths > n_cols // 4)[0]:
        order = np.argsort(splitmix64(substream(seed, 15) ^ int(r), n_cols), kind="stable")
        cols[row_ptr64[r]:row_ptr64[r + 1]] = order[:lengths[r]]
    key = rows * n_cols + cols
    key.sort()
    rnd = 0
    while True:
        dup = np.nonzero(key[1:] == key[:-1])[0] + 1
        if dup.size == 0:
            break
        r = key[dup] // n_cols
        fresh = np.floor(u01(substream(seed, 16 + rnd), dup.size) * n_cols).astype(np.int64)
        key[dup] = r * n_cols + fresh
        key.sort()
        rnd += 1
        if rnd > 200:
            raise RuntimeError("column de-duplication did not converge")
    col = (key - rows * n_cols).astype(np.int32)
    return row_ptr64.astype(np.int32), col


def normal_values(count: int, seed: int) -> np.ndarray:
    """N(0,1) by Box-Muller: sqrt(-2 ln u1) * cos(2 pi u2), u1 in (0,1], u2 in [0,1)."""
    u1 = u01_open0(substream(seed, 3), count)
    u2 = u01(substream(seed, 4), count)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def dense_vector_pm1(count: int, seed: int) -> np.ndarray:
    """x ~ U[-1, 1): 2u - 1 with u from u01 (exact)."""
    return 2.0 * u01(substream(seed, 5), count) - 1.0


def csr_matrix(n: int, seed: int, mean: float = 16.0, tail: float = 1.5, max_len: int = 4096):
    """The irregular-region workload: an n x n CSR matrix with Pareto-tailed
    row lengths, uniform distinct sorted columns, N(0,1) values, and a
    right-hand side x ~ U[-1,1).

    Returns dict(row_ptr int32[n+1], col int32[nnz], val f64[nnz], x f64[n])."""
    lengths = pareto_row_lengths(n, seed, mean=mean, tail=tail, max_len=min(max_len, n))
    row_ptr, col = csr_structure(n, n, lengths, seed)
    val = normal_values(col.size, seed)
    x = dense_vector_pm1(n, seed)
    return {"row_ptr": row_ptr, "col": col, "val": val, "x": x}


def relax_system(n: int, seed: int, mean: float = 16.0, tail: float = 1.5, max_len: int = 4096):
    """A linear system for the weighted-Jacobi relaxation workload: the
    csr_matrix(n, seed) off-diagonal pattern and values (an entry that falls
    on the diagonal is dropped) plus a diagonal entry in every row, d_i = 1 +
    sum_j |a_ij| over the row's off-diagonal entries (strict diagonal
    dominance), stored in column order; b ~ U[-1,1) and a starting vector
    x ~ U[-1,1) from their own substreams.

    Returns dict(row_ptr, col, val, d f64[n], b f64[n], x f64[n])."""
    m = csr_matrix(n, seed, mean=mean, tail=tail, max_len=max_len)
    row_ptr, col, val = m["row_ptr"], m["col"], m["val"]
    lengths = np.diff(row_ptr.astype(np.int64))
    rows = np.repeat(np.arange(n, dtype=np.int64), lengths)
    keep = col.astype(np.int64) != rows
    rows, col, val = rows[keep], col[keep], val[keep]
    kept = np.bincount(rows, minlength=n)
    d = 1.0 + np.bincount(rows, weights=np.abs(val), minlength=n)
    keys = rows * n + col.astype(np.int64)
    diag = np.arange(n, dtype=np.int64)
    at = np.searchsorted(keys, diag * n + diag)
    col = np.insert(col, at, diag.astype(np.int32))
    val = np.insert(val, at, d)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(kept + 1).astype(np.int32)
    b = 2.0 * u01(substream(seed, 6), n) - 1.0
    x = 2.0 * u01(substream(seed, 7), n) - 1.0
    return {"row_ptr": row_ptr, "col": col.astype(np.int32), "val": val, "d": d, "b": b, "x": x}


# --------------------------------------------------------------------------
# The same streams drawn on a torch device (int64 two's-complement wrap
# equals the uint64 arithmetic above; right shifts are made logical).
# --------------------------------------------------------------------------

def _s64(v: int) -> int:
    v &= _MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _lsr(z, k: int):
    return (z >> k) & ((1 << (64 - k)) - 1)


def u01_torch(seed: int, count: int, device, start: int = 0):
    """u01(seed, count, start) computed on a torch device."""
    import torch
    out = torch.empty(count, dtype=torch.float64, device=device)
    g, m1, m2, s = _s64(0x9E3779B97F4A7C15), _s64(0xBF58476D1CE4E5B9), _s64(0x94D049BB133111EB), _s64(seed)
    step = 1 << 25
    for lo in range(0, count, step):
        hi = min(count, lo + step)
        z = torch.arange(start + lo + 1, start + hi + 1, dtype=torch.int64, device=device) * g + s
        z = (z ^ _lsr(z, 30)) * m1
        z = (z ^ _lsr(z, 27)) * m2
        z = z ^ _lsr(z, 31)
        out[lo:hi] = _lsr(z, 11).to(torch.float64) * (2.0 ** -53)
    return out


def grid_u01_torch(nx: int, ny: int, nz: int, seed: int, device):
    """grid_u01 drawn directly in device memory (same values)."""
    return u01_torch(seed, nx * ny * nz, device)
