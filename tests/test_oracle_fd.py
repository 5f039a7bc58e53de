"""Pins of the oracle's finite-difference weights against the conditions that
define central differences (exactness on polynomials up to the order) and
against the analytic derivative of a smooth periodic function."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import fd


def _solve_exact(rows, rhs):
    """Gaussian elimination over the rationals."""
    n = len(rows)
    m = [list(map(Fraction, r)) + [Fraction(b)] for r, b in zip(rows, rhs)]
    for c in range(n):
        p = next(i for i in range(c, n) if m[i][c] != 0)
        m[c], m[p] = m[p], m[c]
        for i in range(n):
            if i != c and m[i][c] != 0:
                f = m[i][c] / m[c][c]
                m[i] = [a - f * b for a, b in zip(m[i], m[c])]
    return [m[i][n] / m[i][i] for i in range(n)]


@pytest.mark.parametrize("order", [2, 4, 6])
def test_second_derivative_weights_solve_taylor_conditions(order):
    r = order // 2
    # sum_m c_m m^(2j) = [j == 1] for j = 1..r, c0 = -2 sum c_m
    rows = [[m ** (2 * j) for m in range(1, r + 1)] for j in range(1, r + 1)]
    rhs = [1 if j == 1 else 0 for j in range(1, r + 1)]
    c = _solve_exact(rows, rhs)
    expect = [-2 * sum(c)] + c
    assert list(fd.SECOND[order]) == expect


@pytest.mark.parametrize("order", [2, 4, 6])
def test_first_derivative_weights_solve_taylor_conditions(order):
    r = order // 2
    # 2 sum_m a_m m^(2j+1) = [j == 0] for j = 0..r-1
    rows = [[2 * m ** (2 * j + 1) for m in range(1, r + 1)] for j in range(r)]
    rhs = [1 if j == 0 else 0 for j in range(r)]
    assert list(fd.FIRST[order]) == _solve_exact(rows, rhs)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_convergence_order_on_sine(order):
    """Errors on sin(x) fall as h^order."""
    errs = []
    for n in (32, 64):
        h = 2 * np.pi / n
        x = h * np.arange(n)
        f = np.sin(x)
        c, a = fd.second(order), fd.first(order)
        d2 = c[0] * f + sum(c[m] * (np.roll(f, -m) + np.roll(f, m)) for m in range(1, len(c)))
        d1 = sum(a[m - 1] * (np.roll(f, -m) - np.roll(f, m)) for m in range(1, len(a) + 1))
        errs.append((np.abs(d2 / h ** 2 + f).max(), np.abs(d1 / h - np.cos(x)).max()))
    for i in range(2):
        rate = np.log2(errs[0][i] / errs[1][i])
        assert abs(rate - order) < 0.15, (order, i, rate)


def test_unsupported_order_rejected():
    with pytest.raises(ValueError):
        fd.radius(8)
