"""Pins of the SpMV oracle (plain and canonical order) to facts fixed outside
the oracle: exact special matrices, hand-derived canonical sums, the
pairwise-summation error bound against exact rationals."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "spmv_canonical_rows.txt")
U = 2.0 ** -53
B = 2.0 ** 53


def _val(tok):
    tok = tok.strip()
    if tok.startswith("-B"):
        return -B
    if tok.startswith("B"):
        return B + (float(tok[2:]) if "+" in tok else 0.0)
    return float(tok)


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.rstrip("\n")
        if not line.strip() or line.lstrip().startswith("#"):
            continue
        name, prods, canon, plain = [s.strip() for s in line.split("|")]
        rows.append((name, [_val(t) for t in prods.split()], _val(canon), _val(plain)))
    return rows


def _single_row(products):
    n = len(products)
    rp = np.array([0, n], dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    x = np.ones(max(n, 1))
    return rp, col, np.array(products, dtype=np.float64), x


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: r[0])
def test_hand_derived_rows(orc, row):
    name, prods, canon, plain = row
    a = _single_row(prods)
    yc = orc.spmv_canonical(*a)[0]
    yp = orc.spmv_plain(*a)[0]
    assert yc == canon and math.copysign(1, yc) == math.copysign(1, canon), name
    assert yp == plain and math.copysign(1, yp) == math.copysign(1, plain), name


def _rand_csr(n, seed, mean=4.0, tail=1.5, max_len=64):
    lengths = synth.pareto_row_lengths(n, seed, mean=mean, tail=tail, max_len=min(max_len, n))
    rp, col = synth.csr_structure(n, n, lengths, seed)
    return rp, col, synth.normal_values(col.size, seed), synth.dense_vector_pm1(n, seed)


def test_identity_diagonal_permutation_exact(orc):
    n = 37
    rp = np.arange(n + 1, dtype=np.int32)
    x = synth.dense_vector_pm1(n, 3)
    eye = np.arange(n, dtype=np.int32)
    for f in (orc.spmv_plain, orc.spmv_canonical):
        assert np.array_equal(f(rp, eye, np.ones(n), x), x)
        d = 2.0 ** np.arange(-5, n - 5)
        assert np.array_equal(f(rp, eye, d, x), d * x)
        perm = np.array(synth.splitmix64(9, n).argsort(), dtype=np.int32)
        assert np.array_equal(f(rp, perm, np.ones(n), x), x[perm])


def test_integer_matrix_exact_any_order(orc):
    n = 50
    rp, col, _, _ = _rand_csr(n, 21, mean=8.0, max_len=40)
    val = np.floor(synth.normal_values(col.size, 22) * 100)
    x = np.floor(synth.dense_vector_pm1(n, 23) * 1000)
    exact = np.array([sum(int(val[k]) * int(x[col[k]]) for k in range(rp[i], rp[i + 1]))
                      for i in range(n)], dtype=np.float64)
    assert np.array_equal(orc.spmv_plain(rp, col, val, x), exact)
    assert np.array_equal(orc.spmv_canonical(rp, col, val, x), exact)


def test_long_row_of_ones(orc):
    n = 4096
    rp = np.array([0, n], dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    for f in (orc.spmv_plain, orc.spmv_canonical):
        assert f(rp, col, np.ones(n), np.ones(n))[0] == 4096.0


def test_empty_rows_are_positive_zero(orc):
    rp = np.array([0, 0, 2, 2], dtype=np.int32)
    col = np.array([0, 2], dtype=np.int32)
    val = np.array([1.0, 2.0])
    x = np.array([1.0, 5.0, 3.0])
    for f in (orc.spmv_plain, orc.spmv_canonical):
        y = f(rp, col, val, x)
        assert y[0] == 0.0 and not np.signbit(y[0]) and y[1] == 7.0 and not np.signbit(y[2])


def test_pairwise_error_bound_against_exact(orc):
    # Higham: pairwise summation of L products has error <= gamma_{ceil(log2 L)+1} sum|p|
    # (the +1 covers the rounding of each product), gamma_k = k u / (1 - k u).
    rp, col, val, x = _rand_csr(300, 31, mean=12.0, max_len=200)
    y = orc.spmv_canonical(rp, col, val, x)
    yp = orc.spmv_plain(rp, col, val, x)
    for i in range(300):
        ks = range(rp[i], rp[i + 1])
        L = len(ks)
        if L == 0:
            continue
        exact = sum(Fraction(float(val[k])) * Fraction(float(x[col[k]])) for k in ks)
        absum = sum(abs(Fraction(float(val[k])) * Fraction(float(x[col[k]]))) for k in ks)
        kk = math.ceil(math.log2(L)) + 1 if L > 1 else 1
        gamma = Fraction(kk) * Fraction(U) / (1 - Fraction(kk) * Fraction(U))
        assert abs(Fraction(float(y[i])) - exact) <= gamma * absum
        gl = Fraction(L) * Fraction(U) / (1 - Fraction(L) * Fraction(U))
        assert abs(Fraction(float(yp[i])) - exact) <= gl * absum


def test_plain_and_canonical_agree_within_scaled_tolerance(orc):
    rp, col, val, x = _rand_csr(2000, 41, mean=16.0, max_len=512)
    y = orc.spmv_canonical(rp, col, val, x)
    yp = orc.spmv_plain(rp, col, val, x)
    scale = np.zeros(2000)
    for i in range(2000):
        ks = slice(rp[i], rp[i + 1])
        scale[i] = np.sum(np.abs(val[ks] * x[col[ks]]))
    assert np.all(np.abs(y - yp) <= 1e-12 * scale)


def test_generator_structure():
    # Sorted, distinct, in-range columns; Pareto lengths >= ceil(scale) and capped.
    n = 5000
    rp, col, val, x = _rand_csr(n, 51, mean=16.0, max_len=300)
    L = np.diff(rp)
    assert L.min() >= math.ceil(16.0 / 3.0) and L.max() <= 300
    for i in range(n):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < n
    assert np.all(x >= -1.0) and np.all(x < 1.0)


def test_byte_counts_are_the_arrays_touched_once(orc):
    # One SpMV reads row_ptr, col, val and x once and writes y once; one
    # relaxation sweep also reads b and diag once; one Jacobi sweep reads
    # and writes the grid once.  Counted from the arrays themselves.
    import synth
    for n, seed in ((1, 3), (257, 4), (4000, 5)):
        m = synth.csr_matrix(n, seed=seed, mean=6.0, max_len=50)
        y = np.empty(n)
        arrays = (m["row_ptr"], m["col"], m["val"], m["x"], y)
        assert orc.spmv_bytes(n, int(m["col"].size)) == sum(a.nbytes for a in arrays)
        b, d = np.empty(n), np.empty(n)
        assert orc.relax_bytes(n, int(m["col"].size)) == sum(a.nbytes for a in arrays + (b, d))
    for shape, S in (((3, 4, 5), 1), ((17, 1, 9), 7), ((0, 4, 4), 3)):
        u = synth.grid_u01(*shape, seed=1)
        assert orc.jacobi_bytes(*shape, S) == S * 2 * u.nbytes
