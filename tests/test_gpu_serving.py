"""Serving on the GPU: merged multi-box launches (persistent: a resident grid
claims the union of the boxes' tiles; the binding's default) give every box
exactly the bits it gets alone (and the same bits as the single-box API),
launches of one workgroup per tile the same bits again, served FP64
boxes of several sizes in one mix match the oracle, admission keeps the pool
within the HBM budget, and a faulty request does not disturb the others."""
import numpy as np
import pytest

from paper_1608_08748_amd import binding, inputs, serving

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _states():
    return [inputs.turbulence(16, seed=31, mach=3.0, beta=1.0, x_h2=1e-3),
            inputs.white_noise((8, 12, 20), seed=32, sigma=0.3, B=(0.2, 0.1, 0.0)),
            inputs.turbulence(24, seed=33, mach=6.0, beta=0.3, x_h2=1e-2)]


def _serve(states, precision, steps=3, budget=1 << 30, max_slots=8, **launch):
    sv = binding.Server(budget, max_slots=max_slots, precision=precision, **launch)
    out = serving.run(sv, states, steps, keep_state=True)
    res = [sv.result(sv_id) for sv_id in [r["id"] for r in out["records"]]]
    sv.close()
    return out, res


@pytest.mark.parametrize("precision", [binding.FP64, binding.FP32_MIXED])
def test_alone_equals_mix_equals_single_box(precision):
    states = _states()
    mix, mix_res = _serve(states, precision)
    assert mix["max_active"] == 3
    for i, W in enumerate(states):
        alone, alone_res = _serve([W], precision)
        np.testing.assert_array_equal(alone_res[0], mix_res[i])
        box = binding.Box(W.shape[1:], precision=precision)
        box.init_state(W)
        for _ in range(3):
            box.step_cfl()
        np.testing.assert_array_equal(box.get_state(), mix_res[i])
        np.testing.assert_array_equal(box.totals(), mix["records"][i]["totals"])


def test_merged_launch_with_a_grid_of_another_boxs_row_count():
    # A (32^3: 8 rows of 32 cells per x-row block, 128 blocks for 1024 rows)
    # and B (256-cell rows, 896 blocks) in one merged FP32 launch of 1024
    # workgroups, the row count of A: the XCD-band renumbering of the x rows
    # applies to one-row-per-block boxes only, so A's blocks stay its own
    A = inputs.turbulence(32, seed=51, mach=3.0, beta=1.0, x_h2=1e-3)
    B = inputs.white_noise((32, 28, 256), seed=52, sigma=0.3, B=(0.2, -0.1, 0.1))
    mix, mix_res = _serve([A, B], binding.FP32_MIXED)
    assert mix["max_active"] == 2
    for i, W in enumerate([A, B]):
        box = binding.Box(W.shape[1:], precision=binding.FP32_MIXED)
        box.init_state(W)
        for _ in range(3):
            box.step_cfl()
        np.testing.assert_array_equal(box.get_state(), mix_res[i])
        box.close()


def test_budget_limits_boxes_in_flight():
    states = [inputs.turbulence(16, seed=40 + k, mach=2.0, beta=1.0, x_h2=1e-3) for k in range(6)]
    p = binding.server_params(precision=binding.FP32_MIXED)
    per_box = binding.server_box_bytes(p, (16, 16, 16))
    sv = binding.Server(2 * per_box + 1024, max_slots=8, precision=binding.FP32_MIXED)
    out = serving.run(sv, states, 4)
    used, peak, cap = sv.memory()
    sv.close()
    assert out["statuses"] == [0]
    assert out["max_active"] == 2
    assert peak <= cap and peak == 2 * per_box and used == 0


def test_faulty_request_is_isolated():
    states = _states()
    bad = states[1].copy()
    bad[0, 2, 3, 4] = np.nan
    mix, mix_res = _serve([states[0], bad, states[2]], binding.FP64)
    assert mix["records"][1]["status"] == binding.MHD_ENONPHYS
    assert mix["records"][0]["status"] == 0 and mix["records"][2]["status"] == 0
    clean, clean_res = _serve([states[0], states[2]], binding.FP64)
    np.testing.assert_array_equal(clean_res[0], mix_res[0])
    np.testing.assert_array_equal(clean_res[1], mix_res[2])


def test_poisson_arrivals_complete():
    states = [inputs.turbulence(n, seed=50 + n, mach=4.0, beta=0.5, x_h2=1e-3) for n in (16, 24, 32, 16, 24)]
    sv = binding.Server(1 << 30, max_slots=3, precision=binding.FP32_MIXED)
    out = serving.run(sv, states, 5, arrivals=serving.poisson_arrivals(len(states), 50.0, seed=5))
    sv.close()
    assert out["statuses"] == [0]
    assert out["max_active"] <= 3
    assert out["latency_p99"] >= out["latency_p50"] > 0


@pytest.mark.parametrize("pinned", [False, True])
def test_borrowed_states_equal_copied(pinned):
    # lending the request states (pageable or pinned host memory) instead of
    # copying them at submission gives the same bits; the binding holds each
    # lent array until its completion has been polled
    import torch
    states = _states()
    if pinned:
        lent = []
        for W in states:
            P = torch.empty(W.shape, dtype=torch.float64, pin_memory=True).numpy()
            P[...] = W
            lent.append(P)
    else:
        lent = [W.copy() for W in states]
    ref, ref_res = _serve(states, binding.FP32_MIXED)
    sv = binding.Server(1 << 30, max_slots=2, precision=binding.FP32_MIXED)
    out = serving.run(sv, lent, 3, keep_state=True, borrow=True)
    assert not sv.held
    res = [sv.result(r["id"]) for r in out["records"]]
    sv.close()
    assert out["statuses"] == [0]
    for a, b in zip(ref_res, res):
        np.testing.assert_array_equal(a, b)


def test_bad_borrow_flag_rejected():
    sv = binding.Server(1 << 28, max_slots=2, precision=binding.FP32_MIXED)
    W = _states()[0]
    r = binding.Request()
    r.n[0], r.n[1], r.n[2] = W.shape[3], W.shape[2], W.shape[1]
    r.steps, r.keep_state, r.borrow = 1, 0, 2
    import ctypes
    rid = ctypes.c_uint64()
    W = np.ascontiguousarray(W)
    st = binding.lib().mhd_server_submit(sv.h, ctypes.byref(r), W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         ctypes.byref(rid))
    sv.close()
    assert st == binding.MHD_EINVAL


def test_close_with_rounds_in_flight():
    # a server closed while boxes are still stepping and others have just
    # finished (their completion not yet reported) releases everything; a new
    # server on the same device then serves the same request bit for bit
    states = _states()
    sv = binding.Server(1 << 30, max_slots=3, precision=binding.FP32_MIXED)
    for k, W in enumerate(states):
        sv.submit(W, 2 + 3 * k, keep_state=True, borrow=bool(k % 2))
    for _ in range(3):
        sv.progress()
    sv.close()
    assert not sv.held
    ref, ref_res = _serve(states[:1], binding.FP32_MIXED)
    again, again_res = _serve(states[:1], binding.FP32_MIXED)
    np.testing.assert_array_equal(ref_res[0], again_res[0])


def test_progress_reports_each_request_once():
    # pipelined rounds: every request is reported exactly once, after its
    # last step, and progress keeps returning once the queue is empty
    states = _states()
    sv = binding.Server(1 << 30, max_slots=2, precision=binding.FP64)
    ids = [sv.submit(W, 2) for W in states]
    seen = []
    for _ in range(20):
        na, npend = sv.progress()
        seen += [c["id"] for c in sv.poll()]
    sv.close()
    assert sorted(seen) == sorted(ids)
    assert (na, npend) == (0, 0)


def test_served_fp64_boxes_match_oracle():
    # boxes of three sizes served together in FP64 (each at its own device
    # CFL step) against the oracle run on each box alone at its CFL steps:
    # fields L1 and totals at the FP64 bar
    import oracle
    from tolerance import FLOOR, field_error, within
    states = [inputs.turbulence(16, seed=61, mach=3.0, beta=1.0, x_h2=1e-3),
              inputs.turbulence(24, seed=62, mach=6.0, beta=0.3, x_h2=1e-2),
              inputs.white_noise((8, 12, 20), seed=63, sigma=0.3, B=(0.2, 0.1, 0.0))]
    steps = 3
    mix, res = _serve(states, binding.FP64, steps=steps)
    assert mix["max_active"] == 3
    for W, G, rec in zip(states, res, mix["records"]):
        P = oracle.make_params(W.shape[1:])
        U = oracle.prim_to_cons(P, W)
        for _ in range(steps):
            oracle.step(P, U, oracle.cfl_dt(P, U))
        worst = 0.0
        for f in range(binding.NFIELDS):
            rel, err, own, vec, _ = field_error(G, U, f, FLOOR["f64"])
            assert within(err, own, vec, 1e-12, FLOOR["f64"]), (W.shape, binding.FIELDS[f], rel)
            worst = max(worst, rel if own > 0 else 0.0)
        to = oracle.totals(P, U)
        absq = np.abs(U).reshape(binding.NFIELDS, -1).sum(axis=1)
        assert np.all(np.abs(np.asarray(rec["totals"]) - to) <= 1e-12 * absq)
        print("served box %s vs oracle: worst field L1 rel %.1e" % (W.shape[1:], worst), flush=True)


@pytest.mark.parametrize("precision", [binding.FP64, binding.FP32_MIXED])
@pytest.mark.parametrize("max_workgroups", [0, 1, 3, 7])
def test_persistent_launches_equal_merged(precision, max_workgroups):
    # a resident grid of at most max_workgroups workgroups (0: what the chip
    # holds) walks the union of the boxes' tiles: a few workgroups take many
    # tiles each, across box boundaries, with the LDS reused tile after tile
    states = _states()
    merged, merged_res = _serve(states, precision, persistent=False)
    pers, pers_res = _serve(states, precision, persistent=True, max_workgroups=max_workgroups)
    assert pers["max_active"] == 3
    for i in range(len(states)):
        np.testing.assert_array_equal(pers_res[i], merged_res[i])
        np.testing.assert_array_equal(pers["records"][i]["totals"], merged["records"][i]["totals"])
        assert pers["records"][i]["status"] == 0


def test_persistent_launches_with_uneven_boxes_and_arrivals():
    # boxes of five sizes arriving over time, so the mix (and the tile list)
    # changes from round to round; each result equals its single-box run
    states = [inputs.turbulence(n, seed=70 + n, mach=4.0, beta=0.5, x_h2=1e-3) for n in (8, 12, 16, 20, 24)]
    sv = binding.Server(1 << 30, max_slots=3, precision=binding.FP32_MIXED, persistent=True, max_workgroups=5)
    out = serving.run(sv, states, 4, arrivals=[0.0, 0.0, 0.01, 0.02, 0.02], keep_state=True)
    res = [sv.result(r["id"]) for r in out["records"]]
    sv.close()
    for W, G in zip(states, res):
        box = binding.Box(W.shape[1:], precision=binding.FP32_MIXED)
        box.init_state(W)
        for _ in range(4):
            box.step_cfl()
        np.testing.assert_array_equal(box.get_state(), G)


def test_persistent_flags_rejected():
    import ctypes
    import torch
    for kw in ({"persistent": True, "max_workgroups": -1},):
        with pytest.raises(binding.MhdError):
            binding.Server(1 << 28, max_slots=2, precision=binding.FP32_MIXED, **kw)
    # a persistent flag other than 0 or 1, through the C ABI
    p = binding.server_params(precision=binding.FP32_MIXED, max_slots=2)
    p.persistent = 2
    total = (1 << 28) + binding.lib().mhd_server_reserved_bytes()
    ws = torch.empty(total, dtype=torch.uint8, device="cuda")
    p.stream = torch.cuda.current_stream().cuda_stream
    p.workspace = ws.data_ptr()
    p.workspace_bytes = total
    h = ctypes.c_void_p()
    assert binding.lib().mhd_server_create(ctypes.byref(p), ctypes.byref(h)) == binding.MHD_EINVAL
    assert not h.value
