"""Parity at the full size of the 512^3 workload, in the launch configuration
the bench times there (512-thread x-row blocks and fused ADV updates, FP64
x rows at four waves per SIMD).  The oracle cannot run 512^3 whole, so the
substage right-hand sides are compared at sampled cells, each against the
oracle on a 13^3 window around it (tests/window.py; the method is checked
against whole-box oracle runs on the CPU); whole steps are checked through
the conserved totals, which hold at any size.

At 512^3 a substage's increment tau R is about 1e-5 of the fluxes it is a
difference of (smooth fields, small dt / h), so the rounding of the fluxes
shows in it at 1e-11 of its own size in FP64 and 1e-3 in FP32.  The bars are
therefore on the substage result U + tau R, the quantity a step compares at
its tolerance (1e-12 FP64; 1e-5 FP32), and, for FP64, also on the increment
itself at 1e-9 of its own L1 norm (a wrong term of relative size above that
fails even where it is small against U).

On the 512^3 workload's seeded state (rms Mach 5, beta 0.3), at 12 x 125
sampled cells, NONADV and ADV right-hand sides:
  * FP64: U + tau R within 1e-12 in L1 per field, tau R within 1e-9 of its
    own L1 norm (each plus the FP64 rounding floor of its vector);
  * FP32 state: U + tau R within 1e-5 per field (the increment's own-norm
    error printed); then two steps at the FP64 run's dt: every total, e and
    rho_H2 included, within 1e-5 of the FP64 run's (relative to sum |q|),
    and the FP64 run's conserved totals unchanged to 1e-12 (mass, momentum,
    energy, face field).
"""
import numpy as np
import pytest

import oracle
from paper_1608_08748_amd import binding, inputs
from tolerance import FLOOR, field_error, within
from window import core_of_box, window_rhs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def c3_state():
    print("generating the 512^3 state", flush=True)
    W = inputs.c3()
    shape = W.shape[1:]
    P = oracle.make_params(shape)
    U = oracle.prim_to_cons(P, W)
    del W
    dt = oracle.cfl_dt(P, U)
    rng = np.random.default_rng(11)
    centres = [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(12)]
    print("state ready, dt %.6e" % dt, flush=True)
    return shape, P, U, dt, centres


def _sampled(box, U, stage, fn, dt, centres):
    """(GPU tau R, oracle tau R, U) at the sampled cells, fields first."""
    box.set_state(U)
    box.debug_stage(stage, dt)
    G = box.get_state()
    Gs = np.concatenate([core_of_box(G, c).reshape(binding.NFIELDS, -1) for c in centres], axis=1)
    del G
    Rs = np.concatenate([window_rhs(fn, U, c, dt).reshape(binding.NFIELDS, -1) for c in centres], axis=1)
    Us = np.concatenate([core_of_box(U, c).reshape(binding.NFIELDS, -1) for c in centres], axis=1)
    return Gs, Rs, Us


def _check(Gs, Rs, Us, what, tol_state, floor, tol_own=None):
    """U + tau R per field at tol_state; tau R against its own norm at tol_own
    (printed only when None)."""
    rows = []
    for f in range(binding.NFIELDS - 1):
        rel, err, own, vec, mx = field_error(Us + Gs, Us + Rs, f, floor)
        assert within(err, own, vec, tol_state, floor), (what, binding.FIELDS[f], "U + tau R", rel)
        rel_i, err_i, own_i, vec_i, _ = field_error(Gs, Rs, f, floor)
        if tol_own is not None:
            assert within(err_i, own_i, vec_i, tol_own, floor), (what, binding.FIELDS[f], "tau R", rel_i)
        rows.append("%s %.1e/%.1e" % (binding.FIELDS[f], rel, rel_i))
    print("%s at %d cells, L1 rel of U + tau R / of tau R:" % (what, Gs.shape[1]), rows, flush=True)


STAGES = ((binding.STAGE_NONADV_RHS, oracle.nonadv_rhs), (binding.STAGE_ADV_RHS, oracle.adv_rhs))


@pytest.mark.timeout(900)
def test_c3_full_size_fp64_rhs_at_sampled_cells(c3_state):
    shape, P, U, dt, centres = c3_state
    box = binding.Box(shape, precision=binding.FP64)
    box.set_state(U)
    assert abs(box.cfl_dt() - dt) <= 1e-13 * dt
    for stage, fn in STAGES:
        print("FP64 stage", fn.__name__, flush=True)
        Gs, Rs, Us = _sampled(box, U, stage, fn, dt, centres)
        _check(Gs, Rs, Us, "FP64 " + fn.__name__, 1e-12, FLOOR["f64"], tol_own=1e-9)
    box.close()


@pytest.mark.timeout(900)
def test_c3_full_size_fp32_rhs_and_totals(c3_state):
    shape, P, U, dt, centres = c3_state
    b32 = binding.Box(shape, precision=binding.FP32_MIXED)
    for stage, fn in STAGES:
        print("FP32 stage", fn.__name__, flush=True)
        Gs, Rs, Us = _sampled(b32, U, stage, fn, dt, centres)
        _check(Gs, Rs, Us, "FP32 " + fn.__name__, 1e-5, FLOOR["f32"])
    # two whole steps of each form at the FP64 run's dt
    b64 = binding.Box(shape, precision=binding.FP64)
    b64.set_state(U)
    b32.set_state(U)
    t0 = b64.totals()
    for s in range(2):
        d = b64.cfl_dt()
        b64.step(d)
        b32.step(d)
        print("step %d done" % (s + 1), flush=True)
    t64, t32 = b64.totals(), b32.totals()
    # sum |q| of the FP64 run's state after the steps (b_y, b_z start at zero)
    absq = np.abs(b64.get_state()).reshape(binding.NFIELDS, -1).sum(axis=1)
    rel = np.abs(t32 - t64) / np.maximum(absq, 1e-300)
    print("FP32 vs FP64 totals after 2 steps:", ["%s %.1e" % (binding.FIELDS[f], rel[f]) for f in range(9 + 1)],
          flush=True)
    assert np.all(rel[:binding.NFIELDS - 1] <= 1e-5)
    conserved = [0, 1, 2, 3, 4, 6, 7, 8]
    drift = np.abs(t64 - t0)[conserved] / absq[conserved]
    print("FP64 conserved totals drift over 2 steps:", ["%.1e" % v for v in drift], flush=True)
    assert np.all(drift <= 1e-12)
    b32.close()
    b64.close()
