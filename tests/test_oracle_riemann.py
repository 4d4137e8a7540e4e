"""Pins of the oracle's NONADV face Riemann solver (Sec. 2.4 and the
eigenvector appendix).

* The Jacobian of the non-advective 1D system, written from the governing
  equations of Sec. 2 (the matrix printed in Sec. 2.4), must equal R Omega L,
  and L R = I: a closed-form invariant that any transposed or mis-signed entry
  of the eigenvectors breaks.
* B = 0 with piecewise-constant data reduces to the linear acoustic Riemann
  problem about the averaged state (textbook primitive-variable solution).
* A uniform state is returned unchanged.
"""
import numpy as np
import pytest

import oracle

G = 5.0 / 3.0


def jacobian(rho, p, bn, bt1, bt2, g=G):
    # d q/dt + B dq/dx = 0 for q = (vn, vt1, vt2, Bt1, Bt2, p), no advection
    return np.array([
        [0, 0, 0, bt1 / rho, bt2 / rho, 1 / rho],
        [0, 0, 0, -bn / rho, 0, 0],
        [0, 0, 0, 0, -bn / rho, 0],
        [bt1, -bn, 0, 0, 0, 0],
        [bt2, 0, -bn, 0, 0, 0],
        [g * p, 0, 0, 0, 0, 0],
    ], dtype=float)


def _states(rng, count):
    for _ in range(count):
        rho = rng.uniform(0.05, 5.0)
        p = rng.uniform(0.01, 5.0)
        b = rng.normal(size=3) * rng.choice([0.1, 1.0, 3.0])
        yield rho, p, b[0], b[1], b[2]


def test_eigen_decomposition_diagonalises_the_jacobian():
    rng = np.random.default_rng(3)
    for rho, p, bn, bt1, bt2 in _states(rng, 300):
        lam, R, L = oracle.eigen(rho, p, bn, bt1, bt2)
        A = jacobian(rho, p, bn, bt1, bt2)
        scale = np.abs(A).max() + np.abs(lam).max() ** 2
        assert np.abs(L @ R - np.eye(6)).max() < 1e-12
        assert np.abs(R @ np.diag(lam) @ L - A).max() < 1e-11 * scale
        # eigenvalue ordering of Sec. 2.4: (cf, -cf, cs, -cs, ca, -ca)
        assert lam[0] >= lam[2] >= 0 and lam[0] >= lam[4] >= 0
        np.testing.assert_allclose(lam[1::2], -lam[0::2])
        assert abs(lam[4] - abs(bn) / np.sqrt(rho)) < 1e-13 * (1 + lam[4])


def test_eigen_degenerate_cases_stay_finite_and_exact():
    # field along the normal (Bt = 0), no field at all, and the triple point gamma p = Bn^2
    for rho, p, bn, bt1, bt2 in [(1.0, 0.6, 2.0, 0.0, 0.0), (1.0, 0.6, 0.0, 0.0, 0.0),
                                 (1.0, 0.6, 1.0, 0.0, 0.0), (2.0, 1.2, -np.sqrt(2.0), 0.0, 0.0),
                                 (1.0, 0.6, 0.0, 0.5, -0.2)]:
        lam, R, L = oracle.eigen(rho, p, bn, bt1, bt2)
        assert np.isfinite(R).all() and np.isfinite(L).all()
        assert np.abs(L @ R - np.eye(6)).max() < 1e-12
        A = jacobian(rho, p, bn, bt1, bt2)
        assert np.abs(R @ np.diag(lam) @ L - A).max() < 1e-12 * (1 + np.abs(A).max())


def _flat(v):
    return np.array([[x, x, 0.0, 0.0] for x in v])


def test_uniform_state_is_returned():
    rng = np.random.default_rng(4)
    for _ in range(100):
        rho = rng.uniform(0.1, 3)
        v = rng.normal(size=3)
        bt = rng.normal(size=2)
        p = rng.uniform(0.1, 3)
        bn = rng.normal()
        c = np.array([rho, v[0], v[1], v[2], bt[0], bt[1], p])
        par = _flat(c[1:])
        out = oracle.riemann_face(c, c, par, par, bn, ydx=rng.uniform(0, 3))
        np.testing.assert_allclose(out, c[1:], rtol=1e-13, atol=1e-13)


def test_b_zero_reduces_to_linear_acoustics():
    rng = np.random.default_rng(5)
    for _ in range(100):
        rl, rr = rng.uniform(0.1, 3, size=2)
        pl, pr = rng.uniform(0.1, 3, size=2)
        vnl, vnr = rng.normal(size=2)
        vt = rng.normal(size=2)          # same transverse velocity on both sides
        cl = np.array([rl, vnl, vt[0], vt[1], 0.0, 0.0, pl])
        cr = np.array([rr, vnr, vt[0], vt[1], 0.0, 0.0, pr])
        out = oracle.riemann_face(cl, cr, _flat(cl[1:]), _flat(cr[1:]), 0.0, ydx=0.7)
        sl, sr = np.sqrt(rl), np.sqrt(rr)
        rho = (sl * rl + sr * rr) / (sl + sr)
        p = (sl * pl + sr * pr) / (sl + sr)
        c = np.sqrt(G * p / rho)
        vn = 0.5 * (vnl + vnr) + (pl - pr) / (2 * rho * c)
        pf = 0.5 * (pl + pr) + 0.5 * rho * c * (vnl - vnr)
        np.testing.assert_allclose(out, [vn, vt[0], vt[1], 0.0, 0.0, pf], rtol=1e-12, atol=1e-13)


def test_b_zero_shear_gives_the_weak_field_alfven_state():
    # With Bn = 0 (sign taken +1) and a transverse velocity jump, the zero-speed
    # Alfven/slow pairs return the intermediate state of the rotational fan:
    # Vt = mean, Bt = -(sqrt(rho)/2) (vt_L - vt_R).
    rl, rr, p = 1.0, 4.0, 1.0
    cl = np.array([rl, 0.0, 0.3, -0.1, 0.0, 0.0, p])
    cr = np.array([rr, 0.0, -0.5, 0.2, 0.0, 0.0, p])
    out = oracle.riemann_face(cl, cr, _flat(cl[1:]), _flat(cr[1:]), 0.0, ydx=0.2)
    sl, sr = 1.0, 2.0
    rho = (sl * rl + sr * rr) / (sl + sr)
    np.testing.assert_allclose(out[1:3], [-0.1, 0.05], atol=1e-14)
    np.testing.assert_allclose(out[3:5], -0.5 * np.sqrt(rho) * np.array([0.8, -0.3]), atol=1e-13)


def test_mirror_symmetry():
    # reflecting x -> -x swaps the cells, flips vn and Bn, and flips the face vn
    rng = np.random.default_rng(6)
    for _ in range(50):
        cl = np.concatenate([[rng.uniform(0.2, 2)], rng.normal(size=5), [rng.uniform(0.2, 2)]])
        cr = np.concatenate([[rng.uniform(0.2, 2)], rng.normal(size=5), [rng.uniform(0.2, 2)]])
        bn = rng.normal()
        a = oracle.riemann_face(cl, cr, _flat(cl[1:]), _flat(cr[1:]), bn, ydx=0.4)
        ml, mr = cr.copy(), cl.copy()
        ml[1] *= -1
        mr[1] *= -1
        b = oracle.riemann_face(ml, mr, _flat(ml[1:]), _flat(mr[1:]), -bn, ydx=0.4)
        np.testing.assert_allclose(b, [-a[0], a[1], a[2], a[3], a[4], a[5]], rtol=1e-11, atol=1e-12)
