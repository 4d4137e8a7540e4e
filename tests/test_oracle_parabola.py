"""Pins of the oracle's local parabola (Sec. 2.1, Steps 1-5) and of the
parabola averages used by both Riemann problems (Sec. 2.4, the q(-nu t) and
q(+nu t) formulas).  Expected values come from hand-worked examples and from
closed forms of polynomials, not from the oracle."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ppm_worked_examples.txt")


def _cases():
    out = []
    with open(GOLD) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("|")
            q = [float(Fraction(t)) for t in lhs.split()]
            e = [float(Fraction(t)) for t in rhs.split()]
            out.append((q, e))
    return out


@pytest.mark.parametrize("q,expect", _cases())
def test_worked_examples(q, expect):
    got = oracle.parabola(q)
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-14)


def test_uniform_is_exact():
    for c in (0.0, 1.0, -3.7, 1e-9):
        np.testing.assert_array_equal(oracle.parabola([c] * 5), [c, c, 0.0, 0.0])


def test_full_cell_average_is_the_cell_value():
    # averaging the parabola over the whole cell returns q_i (conservation, Sec. 2.1)
    rng = np.random.default_rng(0)
    for _ in range(500):
        q = rng.normal(size=5) * rng.choice([1e-3, 1.0, 1e3])
        par = oracle.parabola(q)
        assert abs(oracle.avg_right(par, 1.0) - q[2]) <= 1e-14 * max(1.0, np.abs(q).max())
        assert abs(oracle.avg_left(par, 1.0) - q[2]) <= 1e-14 * max(1.0, np.abs(q).max())
        # and the parameters satisfy dq = qR - qL
        assert par[2] == par[1] - par[0]


def test_no_new_extrema_on_monotone_data():
    rng = np.random.default_rng(1)
    for _ in range(2000):
        steps = rng.exponential(size=4) * rng.choice([-1.0, 1.0])
        q = np.concatenate([[0.0], np.cumsum(steps)]) + rng.normal()
        par = oracle.parabola(q)
        lo = min(q[1], q[3])
        hi = max(q[1], q[3])
        tol = 1e-12 * (1.0 + np.abs(q).max())
        assert lo - tol <= par[0] <= hi + tol
        assert lo - tol <= par[1] <= hi + tol
        # the parabola itself stays within the neighbour range on the cell
        xi = np.linspace(0.0, 1.0, 21)
        vals = par[0] + xi * (par[2] + par[3] * (1.0 - xi))
        assert vals.min() >= lo - tol and vals.max() <= hi + tol


def test_partial_averages_of_exact_quadratic():
    # q(x) = x^2 + 4x on the cell [-1/2, 1/2]; averages over [1/2 - y, 1/2] and [-1/2, -1/2 + y]
    q = [-47 / 12, -35 / 12, 1 / 12, 61 / 12, 145 / 12]
    par = oracle.parabola(q)

    def prim(x):
        return x ** 3 / 3.0 + 2.0 * x * x

    for y in (0.05, 0.3, 0.77, 1.0):
        right = (prim(0.5) - prim(0.5 - y)) / y
        left = (prim(-0.5 + y) - prim(-0.5)) / y
        assert abs(oracle.avg_right(par, y) - right) < 1e-13
        assert abs(oracle.avg_left(par, y) - left) < 1e-13


def test_zero_width_average_is_the_edge_value():
    par = oracle.parabola([0.1, 0.4, 0.5, 0.9, 1.3])
    assert oracle.avg_right(par, 0.0) == par[1]
    assert oracle.avg_left(par, 0.0) == par[0]


def test_fourth_order_interface_on_cubic():
    # cell averages of x^3 + 3x: the interface value at x = 1/2 is exact (1/8 + 3/2)
    def avg(i):
        return i ** 3 + i / 4.0 + 3.0 * i

    q = [avg(i) for i in (-2, -1, 0, 1, 2)]
    par = oracle.parabola(q)
    assert abs(par[1] - 1.625) < 1e-14
    assert abs(par[0] + 1.625) < 1e-14
