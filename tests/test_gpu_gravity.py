"""GPU parity of self-gravity (Sec. 2 equations, Sec. 2.4, Sec. 2.9) against
the FP64 oracle through the C ABI: the potential from the on-device FFT
Poisson solve, the NONADV right-hand side with the gravity sources, and full
steps.  Tolerance as for the rest of the FP64 path (1e-12 relative L1); the
FFT and the oracle's plain transform differ by rounding of order log2(n) ulps.
"""
import numpy as np
import pytest

import oracle
from paper_1608_08748_amd import binding, inputs

from test_gpu_parity import TOL64, assert_fields_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _self_gravitating_state(shape, seed):
    rng = np.random.default_rng(seed)
    W = inputs.white_noise(shape, seed=seed, sigma=0.2, B=(0.1, 0.05, 0.0), x_h2=1e-3)
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx,
                          indexing="ij")
    W[0] = 1.0 + 0.3 * np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.1 * rng.uniform(-1, 1, shape)
    return W


@pytest.mark.parametrize("shape", [(16, 16, 16), (8, 4, 32), (1, 16, 64), (32, 1, 1)])
def test_potential_matches_oracle(shape):
    W = _self_gravitating_state(shape, 71)
    G = binding.gravity_G()
    box = binding.Box(shape, grav_G=G)
    box.init_state(W)
    P = oracle.make_params(shape, grav_G=G)
    U = oracle.prim_to_cons(P, W)
    ref = oracle.potential(P, U[0])
    got = box.potential()
    scale = np.abs(ref).sum()
    assert np.abs(got - ref).sum() <= TOL64 * scale, np.abs(got - ref).max()
    assert abs(got.mean()) <= 1e-14 * np.abs(ref).max()


def test_nonadv_rhs_with_gravity():
    shape = (8, 16, 16)
    W = _self_gravitating_state(shape, 72)
    G = 2.0
    P = oracle.make_params(shape, grav_G=G)
    U = oracle.prim_to_cons(P, W)
    dt = oracle.cfl_dt(P, U)
    ref = oracle.nonadv_rhs(P, U, dt)
    box = binding.Box(shape, grav_G=G)
    box.set_state(U)
    box.debug_stage(binding.STAGE_NONADV_RHS, dt)
    G_ = box.get_state()
    for f in range(binding.NFIELDS):
        scale = max(np.abs(ref[f]).sum(), 1e-300)
        assert np.abs(G_[f] - ref[f]).sum() <= TOL64 * scale + 1e-300, binding.FIELDS[f]


@pytest.mark.parametrize("shape", [(16, 16, 16), (8, 16, 32)])
def test_steps_with_gravity_fp64(shape):
    W = _self_gravitating_state(shape, 73)
    G = binding.gravity_G()
    P = oracle.make_params(shape, grav_G=G)
    U = oracle.prim_to_cons(P, W)
    box = binding.Box(shape, grav_G=G)
    box.init_state(W)
    for _ in range(6):
        dt = oracle.cfl_dt(P, U)
        box.step(dt)
        oracle.step(P, U, dt)
    assert_fields_close(box.get_state(), U, TOL64, "gravity steps %s" % (shape,))


def test_gravity_fp32_totals_close_to_fp64():
    shape = (32, 32, 32)
    W = _self_gravitating_state(shape, 74)
    G = binding.gravity_G()
    tots, dts = [], []
    for prec in (binding.FP64, binding.FP32_MIXED):
        box = binding.Box(shape, precision=prec, grav_G=G)
        box.init_state(W)
        for s in range(10):
            if prec == binding.FP64:
                dts.append(box.cfl_dt())     # the FP32 run replays the FP64 steps
            box.step(dts[s])
        tots.append(box.totals())
        if prec == binding.FP64:
            absq = np.abs(box.get_state()).reshape(binding.NFIELDS, -1).sum(axis=1)
    used = absq > 0          # the H+ field is zero without the ionisation network
    err = np.abs(tots[1] - tots[0])[used] / absq[used]
    assert err.max() <= 1e-5, err
