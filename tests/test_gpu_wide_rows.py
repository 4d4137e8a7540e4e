"""GPU parity of the path for boxes whose x rows do not fit one block (nx above
512 in FP64, above 1024 in FP32): x faces one per thread, then the full update
of all eight fields from the stored face outputs.  The default boxes take the
x-row kernel, which also updates m, E, e; these cases check the other path with
every optional term it carries (the network's gamma_eff in the face solve and
in the p dV work, the gravity sources, the tau R(U) debug stage), against the
FP64 oracle at the FP64 tolerance, and the FP32-state form of it against the
FP64 run at the totals gate.
"""
import numpy as np
import pytest

import oracle
from paper_1608_08748_amd import binding, inputs

from test_gpu_parity import TOL64, assert_fields_close, rel_l1
from test_gpu_ionisation import _ionised_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _pair(W, **kw):
    shape = W.shape[1:]
    box = binding.Box(shape, precision=binding.FP64, **kw)
    box.init_state(W)
    P = oracle.make_params(shape, **kw)
    U = oracle.prim_to_cons(P, W)
    return box, P, U


def _steps(box, P, U, n):
    for _ in range(n):
        dt = oracle.cfl_dt(P, U)
        box.step(dt)
        oracle.step(P, U, dt)


def test_wide_rows_with_ionisation():
    W = _ionised_state((2, 3, 520), 91)
    box, P, U = _pair(W, ionisation=True)
    _steps(box, P, U, 2)
    assert_fields_close(box.get_state(), U, TOL64, "wide rows, ionisation")


def test_wide_rows_with_gravity():
    # every axis a power of two, nx = 1024 above the FP64 row-block limit
    shape = (2, 2, 1024)
    W = inputs.white_noise(shape, seed=92, sigma=0.3, B=(0.2, -0.3, 0.1))
    x = (np.arange(shape[2]) + 0.5) / shape[2]
    W[0] = (1.0 + 0.4 * np.cos(2 * np.pi * 3 * x))[None, None, :] * np.ones(shape)
    box, P, U = _pair(W, grav_G=binding.gravity_G())
    _steps(box, P, U, 2)
    assert_fields_close(box.get_state(), U, TOL64, "wide rows, gravity")


@pytest.mark.parametrize("ion", [False, True])
def test_wide_rows_nonadv_rhs(ion):
    shape = (2, 3, 520)
    if ion:
        W = _ionised_state(shape, 93)
    else:
        W = inputs.white_noise(shape, seed=93, sigma=0.4, B=(0.2, 0.3, -0.1))
    P = oracle.make_params(shape, ionisation=ion)
    U = oracle.prim_to_cons(P, W)
    dt = oracle.cfl_dt(P, U)
    ref = oracle.nonadv_rhs(P, U, dt)
    box = binding.Box(shape, ionisation=ion)
    box.set_state(U)
    box.debug_stage(binding.STAGE_NONADV_RHS, dt)
    G = box.get_state()
    for f in range(binding.NFIELDS):
        scale = max(np.abs(ref[f]).sum(), 1e-300)
        assert np.abs(G[f] - ref[f]).sum() <= TOL64 * scale + 1e-300, binding.FIELDS[f]


def test_wide_rows_fp32_against_fp64():
    # nx = 1040: above the FP32 row-block limit too
    shape = (2, 3, 1040)
    W = inputs.white_noise(shape, seed=94, sigma=0.3, B=(0.2, -0.3, 0.1))
    a = binding.Box(shape, precision=binding.FP64)
    b = binding.Box(shape, precision=binding.FP32_MIXED)
    a.init_state(W)
    b.init_state(W)
    P = oracle.make_params(shape)
    U = oracle.prim_to_cons(P, W)
    for _ in range(4):
        dt = a.cfl_dt()
        a.step(dt)
        b.step(dt)
        oracle.step(P, U, dt)
    A, B = a.get_state(), b.get_state()
    assert_fields_close(A, U, TOL64, "wide rows fp64")
    ta, tb = a.totals(), b.totals()
    absq = np.abs(A).reshape(binding.NFIELDS, -1).sum(axis=1)
    for f in range(binding.NFIELDS):
        if absq[f] > 0:
            assert abs(ta[f] - tb[f]) <= 1e-5 * absq[f], (binding.FIELDS[f], abs(ta[f] - tb[f]) / absq[f])
    assert max(rel_l1(B[f], A[f]) for f in range(9)) < 1e-3
