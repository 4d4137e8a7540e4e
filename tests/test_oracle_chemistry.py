"""Pins of the oracle's H/H2 chemistry step (Sec. 2.7 and the rate appendix).

* The piecewise fits of k2 and k3 are continuous at their switch temperatures
  (7390 K, 7291 K) to the 4-5 digits the coefficients carry: a wrong exponent
  or constant in either branch breaks this.
* The semi-implicit update n' = n + tau (C - D n) / (1 + tau D) has the fixed
  point C / D, contracts the distance to it by exactly 1 / (1 + tau D), tends
  to C / D as tau -> infinity, and stays within [0, all hydrogen molecular].
"""
import numpy as np
import pytest

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


# ---- composition of C and D (Sec. 2.7 with reactions 1-4 of the rate appendix)
#
# The rates k1'..k4 are pinned above; these tests pin how the step combines
# them with the species densities: n_H = n_u (rho - rho_H2), n_H2 = n_u rho_H2
# / 2, C = k1' n n_H (k1 carries the printed n / n_H factor), D = k2 n_H + k3
# n_H2 + k4, then one semi-implicit update.  The expected new density is
# composed here from the species densities of the chosen state and checked
# against the returned density (not against the oracle's own C and D), at
# one temperature in each combination of the k2 / k3 branches; each case
# also checks that a swap of k2 and k3, or of n_H and n_H2, would move the
# result far beyond the tolerance.

def _e_for_T(P, rho, h2, T, hp=0.0, gam=None):
    # T = T_u mu p / rho with p = (gamma - 1) e and mu = 1 / (1 - x_H2 / 2 + x_H+)
    mu = 1.0 / (1.0 - 0.5 * h2 / rho + hp / rho)
    g = P.gamma if gam is None else gam
    return T * rho / (P.T_unit * mu * (g - 1.0))


def _semi_implicit(n, C, D, ts):
    return n + ts * (C - D * n) / (1.0 + ts * D)


# (T, which branches): 5000 K both low; 7340 K k3 high, k2 low; 9000 K both high
@pytest.mark.parametrize("T", [5000.0, 7340.0, 9000.0])
def test_h2_update_composition(T):
    P = _P()
    rho, h2 = 2.0, 0.6
    e = _e_for_T(P, rho, h2, T)
    k1b, k2, k3, k4 = oracle.k_rates(T)
    nH = P.n_unit * (rho - h2)
    nH2 = P.n_unit * h2 / 2.0
    n = nH + nH2
    assert nH != nH2 and abs(k2 - k3) > 0.05 * max(k2, k3)
    # a step with tau D of order one, so C and D both shape the result
    D = k2 * nH + k3 * nH2 + k4
    dt = 1.0 / (D * P.t_unit)
    ts = dt * P.t_unit
    want = 2.0 * _semi_implicit(nH2, k1b * n * nH, D, ts) / P.n_unit
    got, r = oracle.chem_cell(P, rho, e, h2, dt)
    assert abs(r["T"] - T) < 1e-9 * T
    assert abs(got - want) <= 1e-12 * want
    # the test discriminates: swapped rates or swapped species move the result
    for Dx, Cx in ((k3 * nH + k2 * nH2 + k4, k1b * n * nH), (k2 * nH2 + k3 * nH + k4, k1b * n * nH2)):
        other = 2.0 * _semi_implicit(nH2, Cx, Dx, ts) / P.n_unit
        assert abs(other - want) > 1e-6 * want


@pytest.mark.parametrize("T", [5000.0, 7340.0, 9000.0])
def test_h2_and_hplus_update_composition_with_ions(T):
    # reactions 1-8: n_H = n_u (rho - rho_H2 - rho_H+), n_e = n_H+ = n_u rho_H+,
    # n = n_H + n_H2 + n_H+; H2 as above with the H+ clamp n_H2 <= n_u (rho -
    # rho_H+) / 2; H+ with C = k5 n_H + k6 n_H n_e, D = (k7 + k8) n_e
    P = oracle.make_params((1, 1, 1), ionisation=True)
    rho, h2, hp = 2.0, 0.6, 0.3
    nH = P.n_unit * (rho - h2 - hp)
    nH2 = P.n_unit * h2 / 2.0
    ne = P.n_unit * hp
    gam = (5 * nH + 5 * ne + 7 * nH2) / (3 * nH + 3 * ne + 5 * nH2)
    e = _e_for_T(P, rho, h2, T, hp=hp, gam=gam)
    k1b, k2, k3, k4 = oracle.k_rates(T)
    k5, k6, k7, k8 = oracle.ion_rates(T)
    n = nH + nH2 + ne
    D = k2 * nH + k3 * nH2 + k4
    dt = 1.0 / (D * P.t_unit)
    ts = dt * P.t_unit
    m2 = min(_semi_implicit(nH2, k1b * n * nH, D, ts), P.n_unit * (rho - hp) / 2.0)
    h2_want = 2.0 * m2 / P.n_unit
    mi = _semi_implicit(ne, k5 * nH + k6 * nH * ne, (k7 + k8) * ne, ts)
    mi = min(max(mi, 0.0), P.n_unit * (rho - h2_want))
    hp_want = mi / P.n_unit
    h2n, hpn, r = oracle.chem_cell_ion(P, rho, e, h2, hp, dt)
    assert abs(r["T"] - T) < 1e-9 * T
    assert abs(h2n - h2_want) <= 1e-12 * h2_want
    assert abs(hpn - hp_want) <= 1e-12 * hp_want
    for Dx, Cx in ((k3 * nH + k2 * nH2 + k4, k1b * n * nH), (k2 * nH2 + k3 * nH + k4, k1b * n * nH2)):
        other = 2.0 * _semi_implicit(nH2, Cx, Dx, ts) / P.n_unit
        assert abs(other - h2_want) > 1e-6 * h2_want


def test_ion_network_without_ions_reduces_to_h2_network():
    # with no H+ the H2 half of the eight-reaction update is the four-reaction
    # update at the cell's gamma_eff (two separately written oracle functions)
    rng = np.random.default_rng(11)
    for _ in range(50):
        rho = rng.uniform(0.2, 5.0)
        h2 = rho * rng.uniform(0.0, 0.9)
        e = rng.uniform(0.1, 10.0)
        dt = 10 ** rng.uniform(-5, -1)
        Pi = oracle.make_params((1, 1, 1), ionisation=True)
        gam = oracle.gamma_cell(Pi, rho, h2, 0.0)
        Pg = oracle.make_params((1, 1, 1), gamma=gam)
        h2i, hpi, _ = oracle.chem_cell_ion(Pi, rho, e, h2, 0.0, dt)
        h2g, _ = oracle.chem_cell(Pg, rho, e, h2, dt)
        assert abs(h2i - h2g) <= 1e-13 * max(h2g, 1e-300)
