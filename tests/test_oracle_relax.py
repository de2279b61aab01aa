"""Pins of the weighted-Jacobi relaxation oracle (AMGMk relax, Table 3):
x <- x + (omega * (b - A x)) / d with A x in the canonical order."""
import numpy as np
import pytest

import synth


def _dense(row_ptr, col, val, n):
    A = np.zeros((n, n))
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            A[i, col[k]] += val[k]
    return A


def test_diagonal_system_gives_b_over_d_exactly(orc):
    # A = D with power-of-two diagonal, x0 = 0, omega = 1: one sweep is
    # exactly b / d, and b / d is a fixed point of every later sweep
    n = 64
    d = 2.0 ** np.arange(-8, 8, 0.25).round().astype(float)[:n]
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    b = synth.dense_vector_pm1(n, 3)
    x0 = np.zeros(n)
    for S in (1, 2, 5):
        got = orc.relax(row_ptr, col, d, x0, b, d, 1.0, S)
        assert np.array_equal(got, b / d)


def test_sweeps_zero_is_a_copy(orc):
    m = synth.relax_system(300, 4)
    got = orc.relax(m["row_ptr"], m["col"], m["val"], m["x"], m["b"], m["d"], 0.7, 0)
    assert np.array_equal(got, m["x"])


@pytest.mark.parametrize("omega", [1.0, 2.0 / 3.0, 0.3])
def test_exact_solution_is_a_fixed_point(orc, omega):
    # b = A x* summed in the canonical order makes every residual exactly 0
    m = synth.relax_system(2000, 5, tail=1.2, max_len=300)
    xs = synth.dense_vector_pm1(2000, 77)
    b = orc.spmv_canonical(m["row_ptr"], m["col"], m["val"], xs)
    got = orc.relax(m["row_ptr"], m["col"], m["val"], xs, b, m["d"], omega, 4)
    assert np.array_equal(got, xs)


@pytest.mark.parametrize("omega", [1.0, 2.0 / 3.0])
def test_contraction_towards_the_solution(orc, omega):
    # strict diagonal dominance: the error contracts in the max norm by
    # q = (1 - omega) + omega * rho per sweep, rho = max_i sum_{j!=i}|a_ij|/d_i
    n = 80
    m = synth.relax_system(n, 9, mean=6.0, max_len=40)
    A = _dense(m["row_ptr"], m["col"], m["val"], n)
    xs = np.linalg.solve(A, m["b"])
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    rho = float(np.max(off / m["d"]))
    assert rho < 1.0 and np.array_equal(np.diag(A), m["d"])
    q = (1.0 - omega) + omega * rho
    e0 = np.max(np.abs(m["x"] - xs))
    for S in (1, 5, 20):
        got = orc.relax(m["row_ptr"], m["col"], m["val"], m["x"], m["b"], m["d"], omega, S)
        assert np.max(np.abs(got - xs)) <= q ** S * e0 + S * 1e-13


def test_matches_the_plain_definition_within_rounding(orc):
    # the update written with numpy (dense product, another summation order)
    n = 500
    m = synth.relax_system(n, 12, tail=1.5, max_len=200)
    A = _dense(m["row_ptr"], m["col"], m["val"], n)
    omega, S = 0.8, 3
    x = m["x"].copy()
    for _ in range(S):
        x = x + omega * (m["b"] - A @ x) / m["d"]
    got = orc.relax(m["row_ptr"], m["col"], m["val"], m["x"], m["b"], m["d"], omega, S)
    scale = (np.abs(A) @ np.abs(x) + np.abs(m["b"])) / m["d"] + np.abs(x)
    assert np.all(np.abs(got - x) <= 1e-12 * scale)


def test_relax_system_structure():
    m = synth.relax_system(3000, 21)
    rp, col, val, d = m["row_ptr"], m["col"], m["val"], m["d"]
    for i in range(0, 3000, 7):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
        k = int(np.where(c == i)[0][0])
        v = val[rp[i]:rp[i + 1]]
        assert v[k] == d[i] and d[i] > np.abs(np.delete(v, k)).sum()
