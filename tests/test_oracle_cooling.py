"""Pins of the oracle's heating/cooling stage (Sec. 2 stage 5, Sec. 2.8 and the
appendix heating/cooling of reactions 1-4).

* Transcription: the two-branch fits of Lambda2's L_H and L_L meet at their
  switch temperatures (1087 K, 4031 K) to the 2-3 digits the printed
  coefficients carry, which also fixes x = log10(T / 1e4).
* The critical density of Gamma1 is 10^4 cm^-3 at T = 1e4 K (x = 0), so Gamma1
  there is 7.2e-12 erg times the formation rate of reaction 1 over
  (1 + 1e4 / n), with k1 in closed form.
* Lambda = n_H2 L_H / (1 + L_H / L_L) tends to n_H2 L_H at high density and to
  n_H2 L_L at low density.
* Gas without H2 is heated by H2 formation only.
* The stage is an explicit Euler step with frozen rates: the change of e is
  linear in tau; E takes exactly the change of e; nothing else moves; the
  temperature change equals (gamma - 1) tau (Gamma - Lambda) / (n k_B) in cgs,
  an independent check of the code energy unit; strong cooling stops at 10 K.
"""
import numpy as np

import oracle

KB = 1.380649e-16


def _P(n_unit=None, shape=(1, 1, 1), cooling=True):
    nu, Tu, tu = oracle.default_units()
    if n_unit is not None:
        nu = n_unit
    return oracle.make_params(shape, units=(nu, Tu, tu), cooling=cooling)


def _e_at(P, T, rho=1.0, h2=0.0):
    mu = 1.0 / (1.0 - 0.5 * h2 / rho)
    return T * rho / (P.T_unit * mu * (P.gamma - 1.0))


def test_lambda2_lh_continuous_at_1087K():
    L = oracle.lib()
    lo = L.orc_lh2(1087.0)
    hi = L.orc_lh2(np.nextafter(1087.0, 1e9))
    assert abs(lo - hi) / lo < 5e-3
    assert 1.39e-21 < lo < 1.41e-21


def test_lambda2_ll_continuous_at_4031K():
    L = oracle.lib()
    lo = L.orc_ll2(4031.0, 1.0, 0.0)
    hi = L.orc_ll2(np.nextafter(4031.0, 1e9), 1.0, 0.0)
    assert abs(lo - hi) / lo < 2e-2
    # density factor n_H2^0.77 + 1.2 n_H^0.77
    assert abs(L.orc_ll2(5000.0, 2.0, 3.0) / L.orc_ll2(5000.0, 1.0, 0.0) - (3.0 ** 0.77 + 1.2 * 2.0 ** 0.77) / 1.2) < 1e-12


def test_ncrit_at_1e4K():
    assert abs(oracle.lib().orc_ncrit(1e4) - 1e4) < 1e-9


def test_gamma1_closed_form_at_1e4K():
    P = _P()
    rho = 2.0
    e = _e_at(P, 1e4, rho=rho)
    _, t = oracle.heat_cool(P, rho, e, 0.0)
    assert abs(t[4] - 1e4) < 1e-8
    n = P.n_unit * rho
    k1 = 3e-17 * 10.0 / (1.0 + 4.0 + 20.0 + 800.0)   # sqrt(T/100) = 10, T/100 = 100
    want = 7.2e-12 * k1 * n * n / (1.0 + 1e4 / n)
    assert abs(t[0] - want) / want < 1e-12


def test_no_h2_heats_only():
    P = _P()
    r, t = oracle.heat_cool(P, 1.0, 1.5, 0.0)
    assert t[0] > 0.0 and t[1] == 0.0 and t[2] == 0.0 and t[3] == 0.0
    assert r == t[0]


def test_lambda2_density_limits():
    L = oracle.lib()
    T = 3000.0
    for nu, which in ((1e12, "high"), (1e-8, "low")):
        P = _P(n_unit=nu)
        rho, h2 = 1.0, 0.2
        e = _e_at(P, T, rho, h2)
        _, t = oracle.heat_cool(P, rho, e, h2)
        nH, nH2 = nu * (rho - h2), nu * h2 / 2
        T_ = t[4]
        lim = nH2 * (L.orc_lh2(T_) if which == "high" else L.orc_ll2(T_, nH, nH2))
        assert abs(t[2] / lim - 1.0) < 1e-3, (which, t[2], lim)


def test_lambda3_density_limits():
    L = oracle.lib()
    T = 6000.0
    for nu, which in ((1e30, "high"), (1e-8, "low")):
        P = _P(n_unit=nu)
        rho, h2 = 1.0, 0.2
        e = _e_at(P, T, rho, h2)
        _, t = oracle.heat_cool(P, rho, e, h2)
        nH2 = nu * h2 / 2
        n = nu * (rho - h2) + nH2
        T_ = t[4]
        lh = 1.1e-13 * np.exp(-6744.0 / T_)
        lim = nH2 * (lh if which == "high" else np.exp(L.orc_ln_ll3(T_, n)))
        assert abs(t[3] / lim - 1.0) < 1e-3, (which, t[3], lim)


def _state(seed, n=6):
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    P = oracle.make_params(shape, cooling=True)
    W = np.zeros((10,) + shape)
    W[0] = rng.uniform(0.5, 2.0, shape)
    W[1:4] = rng.normal(0, 0.3, (3,) + shape)
    W[4] = rng.uniform(0.05, 3.0, shape)          # T from about 150 K to 9000 K
    W[5:8] = rng.normal(0, 0.5, (3,) + shape)
    W[8] = rng.uniform(0.0, 0.5, shape)
    return P, oracle.prim_to_cons(P, W)


def test_energy_budget_and_untouched_fields():
    P, U = _state(1)
    U0 = U.copy()
    oracle.cooling(P, U, 1e-2)
    dE = U[4] - U0[4]
    de = U[5] - U0[5]
    assert np.all(np.abs(dE - de) <= 4 * np.spacing(np.abs(U0[4]) + np.abs(U[4])))
    assert abs(dE.sum() - de.sum()) <= 1e-13 * np.abs(U0[4]).sum()
    for f in (0, 1, 2, 3, 6, 7, 8, 9):
        assert np.array_equal(U[f], U0[f])
    assert np.any(de != 0.0)


def test_euler_step_is_linear_in_tau():
    P, U0 = _state(2)
    U1, U2 = U0.copy(), U0.copy()
    tau = 1e-7      # well below the shortest cooling time of this state (about 3e-5)
    oracle.cooling(P, U1, tau)
    oracle.cooling(P, U2, 2 * tau)
    d1 = U1[5] - U0[5]
    d2 = U2[5] - U0[5]
    assert np.all(np.abs(d1) < 0.05 * U0[5])   # no cell reaches the floor
    assert np.all(np.abs(d2 - 2 * d1) <= 1e-9 * np.abs(d1) + 4e-16 * np.abs(U0[5]))


def test_temperature_change_in_cgs():
    # Delta T = (gamma - 1) Delta(rho eps)_cgs / (n_particles k_B), n_particles = n_u rho / mu
    P = _P(shape=(1, 1, 1))
    rho, h2 = 1.3, 0.26
    e = _e_at(P, 2500.0, rho, h2)
    U = np.zeros((oracle.NF, 1, 1, 1))
    U[0], U[4], U[5], U[9] = rho, e, e, h2
    r, t = oracle.heat_cool(P, rho, e, h2)
    tau = 1e-6      # far from the floor: the cooling time of this cell is about 1e-4
    oracle.cooling(P, U, tau)
    mu = 1.0 / (1.0 - 0.5 * h2 / rho)
    T1 = P.T_unit * mu * (P.gamma - 1.0) * U[5, 0, 0, 0] / rho
    dT = (P.gamma - 1.0) * tau * P.t_unit * r / (P.n_unit * rho / mu * KB)
    assert abs((T1 - t[4]) - dT) <= 1e-9 * abs(dT)
    assert dT != 0.0


def test_strong_cooling_stops_at_10K():
    P = _P(n_unit=5e4, shape=(1, 1, 1))
    rho, h2 = 1.0, 0.5
    U = np.zeros((oracle.NF, 1, 1, 1))
    e = _e_at(P, 3000.0, rho, h2)
    U[0], U[4], U[5], U[9] = rho, e + 7.0, e, h2
    r, _ = oracle.heat_cool(P, rho, e, h2)
    assert r < 0.0
    oracle.cooling(P, U, 1e3)
    assert abs(U[5, 0, 0, 0] - _e_at(P, 10.0, rho, h2)) <= 1e-15 * e
    assert abs(U[4, 0, 0, 0] - (U[5, 0, 0, 0] + 7.0)) <= 1e-14 * (e + 7.0)


def test_step_runs_cooling_between_chemistry_and_regularisation():
    P, U0 = _state(3)
    Pn = oracle.make_params(U0.shape[1:], cooling=False)
    dt = 1e-3
    Ua, Ub = U0.copy(), U0.copy()
    oracle.step(P, Ua, dt)
    oracle.nonadv_stage(Pn, Ub, dt)
    oracle.adv_stage(Pn, Ub, dt)
    oracle.clamp_h2(Pn, Ub)
    oracle.chemistry(Pn, Ub, dt)
    oracle.cooling(P, Ub, dt)
    oracle.regularise(Pn, Ub)
    assert np.array_equal(Ua, Ub)
