"""Degenerate cases of the method on the GPU against the oracle at the FP64
bar (tests/tolerance.py): the rate switches of reactions 2 and 3 (Sec. 2.7,
rate appendix), where the branch a cell takes is decided in FP64 from the
same temperature on both sides; fully atomic and fully molecular gas; a
zero field in 3D (every face takes the degenerate eigenvector normalisations
of Sec. 2.4); gas at rest (every ADV face velocity exactly zero)."""
import numpy as np
import pytest

import oracle
from paper_1608_08748_amd import binding, inputs
from tolerance import FLOOR, field_error, within

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _close(G, U, what):
    bad = []
    for f in range(binding.NFIELDS):
        rel, err, own, vec, mx = field_error(G, U, f, FLOOR["f64"])
        if not within(err, own, vec, TOL64, FLOOR["f64"]):
            bad.append("%s %.2e" % (binding.FIELDS[f], rel))
    assert not bad, what + ": " + ", ".join(bad)


def _steps(W, steps, **kw):
    shape = W.shape[1:]
    box = binding.Box(shape, **kw)
    box.init_state(W)
    P = oracle.make_params(shape, **kw)
    U = oracle.prim_to_cons(P, W)
    for _ in range(steps):
        dt = oracle.cfl_dt(P, U)
        assert abs(box.cfl_dt() - dt) <= 1e-13 * dt
        box.step(dt)
        oracle.step(P, U, dt)
    return box.get_state(), U, box.totals(), oracle.totals(P, U)


def test_chemistry_at_the_rate_switch_temperatures():
    # temperatures across the switches at 7291 K (k3) and 7390 K (k2), the
    # switch values themselves among them, at H2 mass fractions 0, 1e-3,
    # 0.3 and 1 (no atomic hydrogen left); gas at rest, so the tail stage
    # sees exactly these cells
    nx = 40
    T = np.concatenate([np.linspace(7200.0, 7480.0, nx - 4), [7291.0, 7390.0, 7291.0 * (1 + 1e-15), 7390.0 * (1 - 1e-15)]])
    xs = np.array([0.0, 1e-3, 0.3, 1.0])
    shape = (2, len(xs), nx)
    W = inputs.uniform(shape, rho=1.0, B=(0.1, 0.0, 0.0))
    rho = 1.0 + 0.25 * np.sin(np.arange(nx) * 0.7)
    W[0] = rho[None, None, :]
    W[8] = xs[None, :, None]
    Tu = oracle.default_units()[1]
    mu = 1.0 / (1.0 - 0.5 * W[8])
    W[4] = T[None, None, :] * W[0] / (Tu * mu)
    P = oracle.make_params(shape)
    U = oracle.prim_to_cons(P, W)
    Tcell = Tu * (1.0 / (1.0 - 0.5 * U[9] / U[0])) * (P.gamma - 1.0) * U[5] / U[0]
    assert (Tcell > 7390.0).any() and (Tcell <= 7390.0).any() and (Tcell > 7291.0).any() and (Tcell <= 7291.0).any()
    for dt in (1e-4, 3e-3):
        V = U.copy()
        oracle.clamp_h2(P, V)
        oracle.chemistry(P, V, dt)
        oracle.regularise(P, V)
        box = binding.Box(shape)
        box.set_state(U)
        box.debug_stage(binding.STAGE_TAIL, dt)
        G = box.get_state()
        box.close()
        _close(G, V, "tail at dt %g" % dt)
        assert np.any(np.abs(V[9] - U[9]) > 1e-6 * np.abs(U[9]).max())   # the chemistry acts


def test_fully_atomic_and_fully_molecular_gas():
    W = inputs.turbulence(20, seed=81, mach=4.0, beta=1.0, x_h2=1e-3)
    W[8, :, :, :10] = 0.0
    W[8, :, :, 10:] = 1.0
    G, U, tg, to = _steps(W, 3)
    _close(G, U, "x_H2 0 and 1")
    absq = np.abs(U).reshape(binding.NFIELDS, -1).sum(axis=1)
    assert np.all(np.abs(tg - to) <= TOL64 * absq)


def test_zero_field_in_three_dimensions():
    # B = 0 everywhere: every face takes alpha_f = 1, alpha_s = 0 and
    # beta = (1, 1) / sqrt(2); the zero-speed Alfven and slow pairs of a face
    # with a transverse velocity jump return the weak-field fan state (face
    # Bt = -(sqrt(rho) / 2) (vt_L - vt_R), pinned on the CPU), so the edge
    # fields grow a field from the shear, divergence-free
    W = inputs.turbulence(24, seed=82, mach=3.0, beta=1.0, x_h2=1e-3)
    W[5:8] = 0.0
    G, U, tg, to = _steps(W, 3)
    _close(G, U, "B = 0")
    assert np.abs(G[6:9]).max() > 1e-3
    P = oracle.make_params(G.shape[1:])
    assert oracle.max_divb(P, G) <= 1e-13 * np.abs(G[6:9]).max()


def test_gas_at_rest():
    W = inputs.uniform((6, 8, 10), rho=1.2, p=0.8, B=(0.2, -0.1, 0.3), x_h2=0.05)
    G, U, tg, to = _steps(W, 3)
    _close(G, U, "at rest")
    # only the chemistry (and e through nothing else) changes: the flow stays at rest
    assert np.all(G[1:4] == 0.0)
    for f in (0, 6, 7, 8):
        assert np.all(G[f] == G[f].flat[0])
