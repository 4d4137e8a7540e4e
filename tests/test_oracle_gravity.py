"""Pins of the oracle's self-gravity (Sec. 2 equations, Sec. 2.4 central
differences, Sec. 2.9 Poisson solve in harmonic space).

* The potential satisfies the 27-point discrete Poisson equation in real space:
  (6 / h^2) (A Phi - Phi) = 4 pi G (rho - mean rho), A the tensor product of
  (1, 4, 1) / 6 along each axis, applied here with numpy rolls (independent of
  the harmonic-space solve); this fixes the sign and the scale of the printed
  Green's function.
* A single Fourier mode has the closed-form potential, and it tends to the
  continuum -4 pi G eps / k^2 at second order in h.
* The potential has zero mean and moves with the density (translation).
* The gravity sources are -rho grad(Phi) on m and -m . grad(Phi) on E, and
  their momentum sum vanishes (Newton's third law holds for the discrete
  operators, both circulant).
* Gravity pulls gas towards density peaks: from rest at uniform pressure, the
  momentum after one NONADV stage points to the peak.
"""
import numpy as np

import oracle


def _roll_avg(f, ax):
    return (4.0 * f + np.roll(f, 1, ax) + np.roll(f, -1, ax)) / 6.0


def _lap27(phi, h):
    A = _roll_avg(_roll_avg(_roll_avg(phi, 0), 1), 2)
    return 6.0 / (h * h) * (A - phi)


def test_potential_solves_27_point_poisson_equation():
    shape = (8, 12, 16)      # (nz, ny, nx); cubic cells of side 1/nx
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.2, 3.0, shape)
    G = 0.7
    P = oracle.make_params(shape, grav_G=G)
    phi = oracle.potential(P, rho)
    h = 1.0 / shape[2]
    res = _lap27(phi, h) - 4.0 * np.pi * G * (rho - rho.mean())
    assert np.abs(res).max() <= 1e-12 * 4.0 * np.pi * G * np.abs(rho - rho.mean()).max()
    assert abs(phi.mean()) <= 1e-15 * np.abs(phi).max()


def test_single_mode_closed_form_and_continuum_limit():
    G, eps, m = 1.3, 1e-2, 3
    errs = []
    for n in (16, 32, 64):
        shape = (1, 1, n)
        x = np.arange(n)
        rho = (1.0 + eps * np.cos(2 * np.pi * m * x / n)).reshape(shape)
        P = oracle.make_params(shape, grav_G=G)
        phi = oracle.potential(P, rho).ravel()
        h = 1.0 / n
        a = (3.0 - 2.0 * np.sin(np.pi * m / n) ** 2) / 3.0
        want = -(2.0 / 3.0) * np.pi * G * h * h * eps / (1.0 - a) * np.cos(2 * np.pi * m * x / n)
        # rounding scale: the potential of the whole density (mean 1), not of the eps mode
        assert np.abs(phi - want).max() <= 1e-13 * np.abs(want).max() / eps
        k = 2 * np.pi * m
        cont = -4.0 * np.pi * G * eps / k ** 2
        errs.append(abs(np.abs(phi).max() / abs(cont) - 1.0))
    # second order: the error falls about 4x per doubling
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5


def test_potential_translates_with_density():
    shape = (6, 10, 8)
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.5, 2.0, shape)
    P = oracle.make_params(shape, grav_G=1.0)
    phi = oracle.potential(P, rho)
    phi_s = oracle.potential(P, np.roll(rho, (2, -3, 5), (0, 1, 2)))
    assert np.abs(phi_s - np.roll(phi, (2, -3, 5), (0, 1, 2))).max() <= 1e-13 * np.abs(phi).max()


def _state(shape, seed):
    rng = np.random.default_rng(seed)
    W = np.zeros((10,) + shape)
    W[0] = rng.uniform(0.5, 2.0, shape)
    W[1:4] = rng.normal(0, 0.3, (3,) + shape)
    W[4] = rng.uniform(0.5, 1.5, shape)
    W[5:8] = rng.normal(0, 0.3, (3,) + shape)
    W[8] = 1e-3
    return W


def test_gravity_sources_in_nonadv_rhs():
    shape = (6, 8, 10)
    W = _state(shape, 5)
    G, dt = 0.9, 1e-3
    Pg = oracle.make_params(shape, grav_G=G)
    P0 = oracle.make_params(shape)
    U = oracle.prim_to_cons(P0, W)
    d = oracle.nonadv_rhs(Pg, U, dt) - oracle.nonadv_rhs(P0, U, dt)
    phi = oracle.potential(Pg, U[0])
    h = 1.0 / shape[2]
    g = [(np.roll(phi, -1, ax) - np.roll(phi, 1, ax)) / (2 * h) for ax in (2, 1, 0)]   # x, y, z
    for a in range(3):
        want = -dt * U[0] * g[a]
        assert np.abs(d[1 + a] - want).max() <= 1e-13 * np.abs(want).max()
    wE = -dt * (U[1] * g[0] + U[2] * g[1] + U[3] * g[2])
    assert np.abs(d[4] - wE).max() <= 1e-13 * np.abs(wE).max()
    for f in (0, 5, 6, 7, 8, 9):
        assert np.abs(d[f]).max() <= 1e-16 * np.abs(U[f]).max() + 1e-300
    # total gravitational momentum source vanishes
    for a in range(3):
        assert abs(d[1 + a].sum()) <= 1e-12 * np.abs(d[1 + a]).sum()


def test_gravity_pulls_towards_density_peak():
    n = 32
    shape = (1, 1, n)
    x = (np.arange(n) + 0.5) / n
    W = np.zeros((10,) + shape)
    W[0] = (1.0 + 0.1 * np.cos(2 * np.pi * x)).reshape(shape)
    W[4] = 1.0          # uniform pressure: no pressure force
    P = oracle.make_params(shape, grav_G=1.0, chemistry=False)
    U = oracle.prim_to_cons(P, W)
    oracle.nonadv_stage(P, U, 1e-3)
    mx = U[1].ravel()
    s = np.sin(2 * np.pi * x)
    inner = np.abs(s) > 0.2
    assert np.all(np.sign(mx[inner]) == -np.sign(s[inner]))   # towards the peak at x = 0
