"""The FP32 precision form where its x-row kernels run at the 512^3 and
1024^3 workloads: x rows of 512 and 1024 cells, one block per row (the FP32
state takes rows up to 1024 threads, the FP64 state up to 512).  Thin boxes
(2-3 cells across, every row carrying the same smooth data along x) keep the
oracle fast while every x row is full length.

Per case, on the same seeded turbulence-recipe state and the same dt sequence
(the oracle's CFL steps):
  * the FP64 GPU path against the oracle: fields L1 <= 1e-12 per field (plus
    the FP64 rounding floor of its vector),
    totals <= 1e-12 of sum |q| (the FP64 bar);
  * the FP32 path against the FP64 path: every total, e and rho_H2 included,
    within 1e-5 of sum |q| after every step (the precision form's bar on
    totals); after one step every field within 1e-5 in L1 plus the FP32
    rounding floor of its vector (tests/tolerance.py), before the flow has
    amplified rounding; after the last step the field L1 and L-inf
    errors are printed, not gated (supersonic turbulence amplifies rounding
    differences, so field errors grow with time).
"""
import numpy as np
import pytest

import oracle
from paper_1608_08748_amd import binding, inputs
from tolerance import FLOOR, field_error, within

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _norms(A, B, f):
    d = np.abs(A[f] - B[f])
    l1 = float(d.sum() / max(np.abs(B[f]).sum(), 1e-300))
    linf = float(d.max() / max(np.abs(B[f]).max(), 1e-300))
    return l1, linf


# (shape (nz, ny, nx), recipe, ionisation network)
CASES = [
    ((3, 2, 512), "c3", False),     # 512-thread FP32 rows; FP64 512-thread rows
    ((2, 3, 1024), "c4", False),    # 1024-thread FP32 rows; FP64 one face per thread
    ((2, 2, 1024), "c4", True),     # 1024-thread FP32 rows with the ionisation network
]


@pytest.mark.parametrize("shape,recipe,ion", CASES)
def test_fp32_rows_against_fp64_and_oracle(shape, recipe, ion):
    # the recipe's fields along x (wavenumbers 1-8 of the row), the same in
    # every row: smooth data, so FP32 and FP64 take the same limiter
    # decisions and the differences are rounding (a thin box's transverse
    # axes would only hold grid-scale modes, shocks from the first step)
    row = (1, 1, shape[2])
    if recipe == "c3":
        W = inputs.turbulence(row, seed=3, mach=5.0, beta=0.3, x_h2=1e-3)
    else:
        W = inputs.turbulence(row, seed=4, mach=10.0, beta=0.1, x_h2=1e-2, lognormal_sigma=1.0)
    W = np.ascontiguousarray(np.broadcast_to(W, (W.shape[0],) + tuple(shape)))
    if ion:
        W[9] = 1e-3
    print("case", shape, recipe, "ion" if ion else "", flush=True)
    P = oracle.make_params(shape, ionisation=ion)
    U = oracle.prim_to_cons(P, W)
    a = binding.Box(shape, precision=binding.FP64, ionisation=ion)
    b = binding.Box(shape, precision=binding.FP32_MIXED, ionisation=ion)
    a.init_state(W)
    b.init_state(W)
    nf = binding.NFIELDS if ion else binding.NFIELDS - 1
    steps = 6
    for s in range(steps):
        dt = oracle.cfl_dt(P, U)
        assert abs(a.cfl_dt() - dt) <= 1e-13 * dt
        assert abs(b.cfl_dt() - dt) <= 1e-5 * dt
        a.step(dt)
        b.step(dt)
        oracle.step(P, U, dt)
        A, B = a.get_state(), b.get_state()
        ta, tb = a.totals(), b.totals()
        absq = np.abs(A).reshape(binding.NFIELDS, -1).sum(axis=1)
        terr = [abs(ta[f] - tb[f]) / max(absq[f], 1e-300) for f in range(nf)]
        print("step %d fp32 totals rel" % (s + 1), ["%s %.1e" % (binding.FIELDS[f], terr[f]) for f in range(nf)],
              flush=True)
        for f in range(nf):
            assert terr[f] <= TOL32, (s, binding.FIELDS[f], terr[f])
        if s == 0:
            rows, bad = [], []
            for f in range(nf):
                rel, err, own, vec, _ = field_error(B, A, f, FLOOR["f32"])
                rows.append("%s %.1e (vector %.1e)" % (binding.FIELDS[f], rel, err / max(vec, 1e-300)))
                if not within(err, own, vec, TOL32, FLOOR["f32"]):
                    bad.append(binding.FIELDS[f])
            print("fp32 after 1 step, field L1 rel (and against the vector's norm)", rows, flush=True)
            assert not bad, bad
    # FP64 GPU against the oracle
    worst = 0.0
    for f in range(binding.NFIELDS):
        rel, err, own, vec, _ = field_error(A, U, f, FLOOR["f64"])
        assert within(err, own, vec, TOL64, FLOOR["f64"]), (binding.FIELDS[f], rel)
        worst = max(worst, rel if own > 0 else 0.0)
    to = oracle.totals(P, U)
    absq = np.abs(U).reshape(binding.NFIELDS, -1).sum(axis=1)
    assert np.all(np.abs(ta - to) <= TOL64 * absq)
    print("fp64 vs oracle after %d steps: worst field L1 rel %.1e" % (steps, worst), flush=True)
    tot = ["%s %.1e" % (binding.FIELDS[f], abs(ta[f] - tb[f]) / max(absq[f], 1e-300)) for f in range(nf)]
    fe = ["%s %.1e/%.1e" % ((binding.FIELDS[f],) + _norms(B, A, f)) for f in range(nf)]
    print("fp32 vs fp64 after %d steps: totals rel %s; fields L1/Linf rel %s" % (steps, tot, fe), flush=True)
