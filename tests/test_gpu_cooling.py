"""GPU parity of the heating/cooling stage (Sec. 2 stage 5, Sec. 2.8; appendix
heating/cooling of reactions 1-4) against the FP64 oracle, through the C ABI.

Tolerance as for the rest of the FP64 path: per-field L1 difference <= 1e-12
of the field's L1 norm.  The rates use exp, log, pow and sqrt on both sides
(device and host math libraries, each within an ulp or two), so the cooling
terms differ by a few ulps, far inside the tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_1608_08748_amd import binding, inputs, serving

from test_gpu_parity import TOL64, assert_fields_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _units(n_unit):
    nu, Tu, tu = binding.DEFAULT_UNITS
    return (n_unit, Tu, tu)


def _warm_molecular_state(shape, seed):
    """Random flow with temperatures from about 150 K to 9000 K and H2 mass
    fractions up to 0.5, so every heating and cooling term and both branches of
    the Lambda2 fits are exercised."""
    rng = np.random.default_rng(seed)
    W = np.zeros((10,) + shape)
    W[0] = rng.uniform(0.5, 2.0, shape)
    W[1:4] = rng.normal(0, 0.3, (3,) + shape)
    W[4] = rng.uniform(0.05, 3.0, shape)
    W[5:8] = rng.normal(0, 0.5, (3,) + shape)
    W[8] = rng.uniform(0.0, 0.5, shape)
    return W


@pytest.mark.parametrize("n_unit,dt", [(5.0, 1e-6), (5.0, 1e-2), (5e-3, 1e-3)])
def test_tail_stage_with_cooling(n_unit, dt):
    # n_unit = 5, dt = 1e-2: most cells cool to the 10 K floor in one step;
    # dt = 1e-6 and the dilute case: no cell reaches it
    shape = (10, 12, 14)
    W = _warm_molecular_state(shape, seed=61)
    units = _units(n_unit)
    P = oracle.make_params(shape, units=units, cooling=True)
    U = oracle.prim_to_cons(P, W)
    V = U.copy()
    oracle.clamp_h2(P, V)
    oracle.chemistry(P, V, dt)
    oracle.cooling(P, V, dt)
    oracle.regularise(P, V)
    box = binding.Box(shape, units=units, cooling=True)
    box.set_state(U)
    box.debug_stage(binding.STAGE_TAIL, dt)
    G = box.get_state()
    assert_fields_close(G, V, TOL64, "tail+cooling n_u=%g dt=%g" % (n_unit, dt))
    # the stage changed the energies (it is not a no-op)
    assert np.abs(G[5] - U[5]).max() > 1e-6 * np.abs(U[5]).max()


def test_steps_with_cooling_fp64():
    # C1-type flow, H2 fraction 0.02, dilute units: a few per cent of e per step
    shape = (20, 20, 20)
    W = inputs.c1(n=20)
    W[8] = 0.02
    units = _units(5e-3)
    P = oracle.make_params(shape, units=units, cooling=True)
    U = oracle.prim_to_cons(P, W)
    box = binding.Box(shape, units=units, cooling=True)
    box.init_state(W)
    Pn = oracle.make_params(shape, units=units, cooling=False)
    Un = U.copy()
    for _ in range(8):
        dt = oracle.cfl_dt(P, U)
        box.step(dt)
        oracle.step(P, U, dt)
        oracle.step(Pn, Un, dt)
    assert_fields_close(box.get_state(), U, TOL64, "cooling steps")
    # the stage matters here: the internal energy differs from the run without it
    assert abs(U[5].sum() - Un[5].sum()) > 1e-3 * Un[5].sum()


def test_serving_with_cooling_matches_single_box():
    W = _warm_molecular_state((12, 12, 12), seed=62)
    W[4] = 1.0
    units = _units(5e-3)
    sv = binding.Server(1 << 28, max_slots=4, precision=binding.FP64, units=units, cooling=True)
    out = serving.run(sv, [W, inputs.turbulence(16, seed=63, mach=2.0, beta=1.0, x_h2=0.1)], 3, keep_state=True)
    res = sv.result(out["records"][0]["id"])
    sv.close()
    box = binding.Box(W.shape[1:], precision=binding.FP64, units=units, cooling=True)
    box.init_state(W)
    for _ in range(3):
        box.step_cfl()
    np.testing.assert_array_equal(box.get_state(), res)
