"""Pins of the oracle's H/H2 chemistry step (Sec. 2.7 and the rate appendix).

* The piecewise fits of k2 and k3 are continuous at their switch temperatures
  (7390 K, 7291 K) to the 4-5 digits the coefficients carry: a wrong exponent
  or constant in either branch breaks this.
* The semi-implicit update n' = n + tau (C - D n) / (1 + tau D) has the fixed
  point C / D, contracts the distance to it by exactly 1 / (1 + tau D), tends
  to C / D as tau -> infinity, and stays within [0, all hydrogen molecular].
"""
import numpy as np

import oracle


def test_k2_continuous_at_switch():
    lo = oracle.k_rates(7390.0)[1]
    hi = oracle.k_rates(np.nextafter(7390.0, 1e9))[1]
    assert abs(lo - hi) / lo < 2e-4
    assert 1.15e-15 < lo < 1.17e-15


def test_k3_continuous_at_switch():
    lo = oracle.k_rates(7291.0)[2]
    hi = oracle.k_rates(np.nextafter(7291.0, 1e9))[2]
    assert abs(lo - hi) / lo < 2e-4
    assert 6.2e-16 < lo < 6.4e-16


def test_k1_closed_form_at_100K():
    # at T = 100 K every sqrt(T/100) and T/100 is 1: 3e-17 / (1 + 0.4 + 0.2 + 0.08)
    assert abs(oracle.k_rates(100.0)[0] - 3e-17 / 1.68) < 1e-30


def test_k4_optically_thin():
    assert abs(oracle.k_rates(1000.0)[3] - 5.61e-11) < 1e-24


def _P():
    return oracle.make_params((1, 1, 1))


def test_fixed_point_and_contraction():
    P = _P()
    rng = np.random.default_rng(7)
    for _ in range(200):
        rho = rng.uniform(0.1, 10)
        e = rng.uniform(0.05, 20)
        h2 = rho * 10 ** rng.uniform(-6, -0.5)
        dt = 10 ** rng.uniform(-6, -2)
        h2n, r = oracle.chem_cell(P, rho, e, h2, dt)
        C, D = r["C"], r["D"]
        ts = dt * P.t_unit
        n = P.n_unit * h2 / 2.0
        nn = P.n_unit * h2n / 2.0
        nstar = C / D
        # (n' - n*) (1 + tau D) = n - n*   (unless clamped)
        if 0.0 < nn < P.n_unit * rho / 2.0:
            lhs = (nn - nstar) * (1.0 + ts * D)
            assert abs(lhs - (n - nstar)) <= 1e-9 * (abs(n) + abs(nstar)) + 1e-300


def test_large_tau_limit_is_equilibrium():
    P = _P()
    rho, e, h2 = 1.0, 1.5, 1e-3
    for dt in (1e3, 1e9):
        h2n, r = oracle.chem_cell(P, rho, e, h2, dt)
        nstar = r["C"] / r["D"]
        n0 = P.n_unit * h2 / 2.0
        tD = dt * P.t_unit * r["D"]
        # distance to equilibrium shrinks as 1 / (1 + tau D)
        assert abs(P.n_unit * h2n / 2.0 - nstar) <= abs(n0 - nstar) / tD * (1 + 1e-6) + 1e-12 * nstar


def test_temperature_unit_map():
    # p = (gamma - 1) e, T = T_u mu p / rho with mu = 1 / (1 - x_H2 / 2)
    P = _P()
    _, r = oracle.chem_cell(P, 2.0, 3.0, 0.0, 1e-5)
    assert abs(r["T"] - P.T_unit * (2.0 / 3.0) * 3.0 / 2.0) < 1e-9
    _, r = oracle.chem_cell(P, 2.0, 3.0, 2.0, 1e-5)   # fully molecular: mu = 2
    assert abs(r["T"] - 2.0 * P.T_unit * (2.0 / 3.0) * 3.0 / 2.0) < 1e-9


def test_bounds_and_positivity():
    P = _P()
    rng = np.random.default_rng(8)
    for _ in range(500):
        rho = 10 ** rng.uniform(-3, 2)
        e = 10 ** rng.uniform(-4, 3)
        h2 = rho * rng.uniform(0, 1)
        dt = 10 ** rng.uniform(-8, 2)
        h2n, _ = oracle.chem_cell(P, rho, e, h2, dt)
        assert 0.0 <= h2n <= rho * (1 + 1e-15)


def test_stiff_step_is_stable():
    # tau D ~ 1e6: one step lands on the equilibrium without overshoot
    P = _P()
    h2n, r = oracle.chem_cell(P, 1.0, 1.5, 0.5, 1e6 / (5.61e-11 * P.t_unit))
    assert abs(P.n_unit * h2n / 2.0 - r["C"] / r["D"]) < 1e-6 * P.n_unit * 0.25


def test_chemistry_changes_only_h2():
    P = oracle.make_params((4, 4, 4))
    from paper_1608_08748_amd import inputs
    W = inputs.c1(n=4)
    U = oracle.prim_to_cons(P, W)
    V = U.copy()
    oracle.chemistry(P, V, 1e-3)
    np.testing.assert_array_equal(V[:9], U[:9])
    assert not np.array_equal(V[9], U[9])
