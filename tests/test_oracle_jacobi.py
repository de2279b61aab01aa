"""Pins of the Jacobi oracle to facts fixed outside the oracle itself:
hand values, a closed-form eigenvector, exact invariants and an exact
rational evaluation within the rounding-error bound."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "jacobi_hand_values.txt")
C = 1.0 / 6.0
U = 2.0 ** -53  # unit roundoff of binary64


def _idx(nx, ny, i, j, k):
    return (k * ny + j) * nx + i


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = [s.strip() for s in line.split("|")]
        out[int(k)] = float.fromhex(v)
    return out


def test_constant_field_hand_values(orc):
    g = _golden()
    n = 5
    out = orc.jacobi7(np.ones(n ** 3), n, n, n, 1).reshape(n, n, n)
    for k in range(n):
        for j in range(n):
            for i in range(n):
                cnt = sum(1 for a, lim in ((i, n), (j, n), (k, n)) for d in (-1, 1) if 0 <= a + d < lim)
                assert out[k, j, i] == g[cnt], (i, j, k, cnt)


def test_constant_field_hand_values_by_exact_rounding():
    # fl(k * C) for k neighbours, by exact rational arithmetic (correct rounding
    # of Fraction -> float), independent of both the golden file and the oracle.
    g = _golden()
    for k, v in g.items():
        assert float(k * Fraction(C)) == v


def test_delta_at_centre(orc):
    n = 5
    u0 = np.zeros(n ** 3)
    u0[_idx(n, n, 2, 2, 2)] = 1.0
    out = orc.jacobi7(u0, n, n, n, 1)
    nb = {_idx(n, n, 2 + d[0], 2 + d[1], 2 + d[2]) for d in
          ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))}
    for p in range(n ** 3):
        assert out[p] == (C if p in nb else 0.0)


def test_add_order_hand_value(orc):
    # Centre of a 3^3 grid with xm = 2^53, xp = 1, ym = 1, other neighbours 0:
    # ((2^53 + 1) + 1) = 2^53 (two ties to even), so the centre is 2^53 * C
    # exactly = 0x1.5555555555555p+50.  Summing xp+ym first would give
    # (2^53 + 2) * C, which differs.
    n = 3
    u0 = np.zeros(27)
    u0[_idx(n, n, 0, 1, 1)] = 2.0 ** 53
    u0[_idx(n, n, 2, 1, 1)] = 1.0
    u0[_idx(n, n, 1, 0, 1)] = 1.0
    out = orc.jacobi7(u0, n, n, n, 1)
    assert out[_idx(n, n, 1, 1, 1)] == float.fromhex("0x1.5555555555555p+50")
    assert float.fromhex("0x1.5555555555555p+50") != (2.0 ** 53 + 2.0) * C


@pytest.mark.parametrize("n,s", [(8, 1), (9, 5), (12, 20)])
def test_eigenvector_closed_form(orc, n, s):
    # sin(pi (i+1) h) sin(pi (j+1) h) sin(pi (k+1) h), h = 1/(n+1), vanishes on
    # the ghost layer; the 6-neighbour average maps it to cos(pi h) times itself.
    h = 1.0 / (n + 1)
    a = np.sin(np.pi * (np.arange(n) + 1) * h)
    u0 = (a[:, None, None] * a[None, :, None] * a[None, None, :]).reshape(-1)
    out = orc.jacobi7(u0, n, n, n, s)
    exact = math.cos(math.pi * h) ** s * u0
    rel = np.max(np.abs(out - exact)) / np.max(np.abs(exact))
    assert rel < 12 * s * U + 8 * U


def test_eigenvector_rejects_fixed_boundary_reading(orc):
    # Under a fixed-outer-layer reading the eigenvector would use h = 1/(n-1);
    # the ghost-zero oracle must not reproduce that eigenvalue.
    n, s = 8, 3
    h = 1.0 / (n - 1)
    a = np.sin(np.pi * np.arange(n) * h)
    u0 = (a[:, None, None] * a[None, :, None] * a[None, None, :]).reshape(-1)
    out = orc.jacobi7(u0, n, n, n, s)
    assert np.max(np.abs(out - math.cos(math.pi * h) ** s * u0)) > 1e-3


def test_power_of_two_scaling_is_exact(orc):
    nx, ny, nz = 7, 5, 6
    u0 = synth.grid_u01(nx, ny, nz, seed=11)
    a = orc.jacobi7(u0, nx, ny, nz, 4)
    b = orc.jacobi7(u0 * 2.0 ** 10, nx, ny, nz, 4)
    assert np.array_equal(a * 2.0 ** 10, b)


def test_x_mirror_is_exact(orc):
    nx, ny, nz = 9, 4, 5
    u0 = synth.grid_u01(nx, ny, nz, seed=12).reshape(nz, ny, nx)
    a = orc.jacobi7(u0, nx, ny, nz, 6).reshape(nz, ny, nx)
    b = orc.jacobi7(np.ascontiguousarray(u0[:, :, ::-1]), nx, ny, nz, 6).reshape(nz, ny, nx)
    assert np.array_equal(a[:, :, ::-1], b)


def test_exact_rational_within_rounding_bound(orc):
    # Exact rational S-sweep result (true 1/6) vs the oracle: all values are
    # >= 0; a sweep rounds 5 additions of nonnegative terms, the constant
    # fl(1/6) and one multiply, so its relative error is at most
    # (1 + u)^7 - 1 < 8u, and errors of nonnegative inputs propagate with
    # weights summing to <= 1: (1 + 8u)^S - 1 bounds S sweeps (u = 2^-53).
    n, s = 4, 3
    u0 = synth.grid_u01(n, n, n, seed=13)
    cur = [Fraction(float(v)) for v in u0]
    sixth = Fraction(1, 6)

    def at(arr, i, j, k):
        if 0 <= i < n and 0 <= j < n and 0 <= k < n:
            return arr[_idx(n, n, i, j, k)]
        return Fraction(0)

    for _ in range(s):
        nxt = [Fraction(0)] * n ** 3
        for k in range(n):
            for j in range(n):
                for i in range(n):
                    nxt[_idx(n, n, i, j, k)] = sixth * (
                        at(cur, i - 1, j, k) + at(cur, i + 1, j, k) + at(cur, i, j - 1, k)
                        + at(cur, i, j + 1, k) + at(cur, i, j, k - 1) + at(cur, i, j, k + 1))
        cur = nxt
    out = orc.jacobi7(u0, n, n, n, s)
    bound = (1 + 8 * U) ** s - 1
    for p in range(n ** 3):
        ex = cur[p]
        assert abs(Fraction(float(out[p])) - ex) <= Fraction(bound) * ex


def test_zero_sweeps_and_empty(orc):
    u0 = synth.grid_u01(3, 3, 3, seed=1)
    assert np.array_equal(orc.jacobi7(u0, 3, 3, 3, 0), u0)
    assert orc.jacobi7(np.zeros(0), 0, 3, 3, 2).size == 0


def test_one_dimensional_line_matches_1d_stencil_by_hand(orc):
    # 1x1xn: only z neighbours exist; u = [1, 2, 4] -> [(0+2)C, (1+4)C, (2+0)C]
    out = orc.jacobi7(np.array([1.0, 2.0, 4.0]), 1, 1, 3, 1)
    assert out[0] == 2.0 * C and out[1] == 5.0 * C and out[2] == 2.0 * C
