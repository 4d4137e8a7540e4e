"""Pins of the oracle's ionisation network (reactions 5-8 with H+ and e-, the
effective adiabatic index of Sec. 4.3).

* gamma_eff reduces to 5/3 for atomic or fully ionised hydrogen and to 7/5 for
  molecular hydrogen; without the network it is the constant gamma.
* The printed collisional-ionisation fit, read with ln(T in eV), gives
  4.4e-22 cm^3/s at 5000 K and 7.4e-16 at 1e4 K; the printed recombination fit
  read with log10 gives about 7.4e-11 at 5000 K.
* The semi-implicit H+ update has the fixed point C / D, contracts the distance
  to it by exactly 1 / (1 + tau D), tends to it as tau -> infinity, and keeps
  H2 + H+ within the hydrogen present.
* The temperature uses the mean mass 1 / (1 - x_H2/2 + x_H+): fully ionised gas
  at the same p / rho is half as hot as atomic gas.
* In the step: H+ is advected conservatively (its total is constant through
  the NONADV and ADV stages), a uniform ionised state stays bitwise uniform,
  primitive -> conserved -> primitive recovers p with gamma_eff, and with the
  network off the H+ field stays zero.
"""
import numpy as np

import oracle


def _P(shape=(1, 1, 1), **kw):
    return oracle.make_params(shape, ionisation=True, **kw)


def test_gamma_eff_limits():
    P = _P()
    assert abs(oracle.gamma_cell(P, 1.0, 0.0, 0.0) - 5.0 / 3.0) < 1e-15
    assert abs(oracle.gamma_cell(P, 1.0, 1.0, 0.0) - 7.0 / 5.0) < 1e-15
    assert abs(oracle.gamma_cell(P, 1.0, 0.0, 1.0) - 5.0 / 3.0) < 1e-15
    # a mixture lies between the molecular and atomic values
    g = oracle.gamma_cell(P, 1.0, 0.4, 0.2)
    assert 7.0 / 5.0 < g < 5.0 / 3.0
    P0 = oracle.make_params((1, 1, 1), gamma=1.4)
    assert oracle.gamma_cell(P0, 1.0, 0.4, 0.2) == 1.4


def test_k6_values():
    assert abs(oracle.ion_rates(5000.0)[1] / 4.4e-22 - 1.0) < 0.02
    assert abs(oracle.ion_rates(1e4)[1] / 7.4e-16 - 1.0) < 0.02
    # strongly rising with temperature
    assert oracle.ion_rates(2e4)[1] > 100 * oracle.ion_rates(1e4)[1]


def test_k7_k8_values():
    k5, k6, k7, k8 = oracle.ion_rates(5000.0)
    assert k5 == 6e-18
    assert 7.0e-11 < k7 < 8.0e-11
    assert 1.0e-13 < k8 < 1.3e-13


def _e_at(P, T, rho, h2, hp):
    mu = 1.0 / (1.0 - 0.5 * h2 / rho + hp / rho)
    return T * rho / (P.T_unit * mu * (oracle.gamma_cell(P, rho, h2, hp) - 1.0))


def test_semi_implicit_h_plus_update():
    P = _P()
    rho, h2, hp, T = 1.0, 0.1, 0.05, 8000.0
    e = _e_at(P, T, rho, h2, hp)
    dts = (1e-6, 1e-4, 1e-2)
    for dt in dts:
        h2n, hpn, r = oracle.chem_cell_ion(P, rho, e, h2, hp, dt)
        assert abs(r["T"] - T) < 1e-9 * T
        nu = P.n_unit
        nH, ne = nu * (rho - h2 - hp), nu * hp
        C = r["k5"] * nH + r["k6"] * nH * ne
        D = (r["k7"] + r["k8"]) * ne
        nstar = C / D
        ts = dt * P.t_unit
        lhs = (nu * hpn - nstar) * (1.0 + ts * D)
        assert abs(lhs - (ne - nstar)) <= 1e-12 * max(abs(ne - nstar), ne)
        assert 0.0 <= hpn and h2n + hpn <= rho
    # tau -> infinity: the fixed point (clamped to the hydrogen left)
    h2n, hpn, r = oracle.chem_cell_ion(P, rho, e, h2, hp, 1e12)
    nu = P.n_unit
    nH, ne = nu * (rho - h2 - hp), nu * hp
    nstar = (r["k5"] * nH + r["k6"] * nH * ne) / ((r["k7"] + r["k8"]) * ne)
    assert abs(nu * hpn - min(nstar, nu * (rho - h2n))) <= 1e-6 * nstar


def test_temperature_uses_ion_mean_mass():
    P = _P()
    rho = 1.0
    p = 0.8
    g = oracle.gamma_cell(P, rho, 0.0, 0.0)
    _, _, ra = oracle.chem_cell_ion(P, rho, p / (g - 1.0), 0.0, 0.0, 1e-9)
    g = oracle.gamma_cell(P, rho, 0.0, 1.0)
    _, _, ri = oracle.chem_cell_ion(P, rho, p / (g - 1.0), 0.0, 1.0, 1e-9)
    assert abs(ri["T"] / ra["T"] - 0.5) < 1e-14


def _ionised_state(shape, seed):
    rng = np.random.default_rng(seed)
    W = np.zeros((10,) + shape)
    W[0] = rng.uniform(0.5, 2.0, shape)
    W[1:4] = rng.normal(0, 0.3, (3,) + shape)
    W[4] = rng.uniform(0.5, 1.5, shape)
    W[5:8] = rng.normal(0, 0.3, (3,) + shape)
    W[8] = rng.uniform(0.0, 0.3, shape)
    W[9] = rng.uniform(0.0, 0.5, shape)
    return W


def test_prim_roundtrip_with_gamma_eff():
    shape = (4, 5, 6)
    W = _ionised_state(shape, 1)
    P = _P(shape)
    U = oracle.prim_to_cons(P, W)
    g = np.vectorize(lambda r, a, b: oracle.gamma_cell(P, r, a, b))(U[0], U[9], U[10])
    assert np.abs((g - 1.0) * U[5] - W[4]).max() <= 1e-14 * np.abs(W[4]).max()
    assert np.array_equal(U[10], W[9] * W[0])


def test_h_plus_advected_conservatively():
    shape = (6, 8, 10)
    W = _ionised_state(shape, 2)
    P = _P(shape, chemistry=False)
    U = oracle.prim_to_cons(P, W)
    t0 = U[10].sum()
    dt = oracle.cfl_dt(P, U)
    oracle.nonadv_stage(P, U, dt)
    assert U[10].sum() == t0          # NONADV does not touch it
    oracle.adv_stage(P, U, dt)
    assert abs(U[10].sum() - t0) <= 1e-13 * np.abs(U[10]).sum()
    assert np.abs(U[10] - oracle.prim_to_cons(P, W)[10]).max() > 0   # it moved


def test_uniform_ionised_state_stays_uniform():
    shape = (4, 4, 4)
    W = np.zeros((10,) + shape)
    W[0], W[1], W[2], W[3], W[4] = 1.2, 0.3, -0.2, 0.1, 0.9
    W[5], W[6], W[7], W[8], W[9] = 0.4, 0.2, -0.3, 0.2, 0.3
    P = _P(shape, chemistry=False)
    U = oracle.prim_to_cons(P, W)
    U0 = U.copy()
    oracle.step(P, U, 1e-3)
    for f in range(oracle.NF):
        assert np.all(U[f] == U[f].ravel()[0]), f
    assert np.array_equal(U[10], U0[10])


def test_network_off_leaves_h_plus_zero():
    shape = (4, 6, 8)
    W = _ionised_state(shape, 3)
    W[9] = 0.0
    P = oracle.make_params(shape)
    U = oracle.prim_to_cons(P, W)
    for _ in range(2):
        oracle.step(P, U, oracle.cfl_dt(P, U))
    assert not U[10].any()
