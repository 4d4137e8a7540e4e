"""Benchmark of the operator-split MHD + H2 chemistry step on one MI355X.

    python bench.py [--config c2] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one full pass of the method over the box: NONADV stage (3 RK
substages: face Riemann solves along y, z, then x fused with the update of
m, E, e, then the face-field update from edge fields), ADV stage (3 RK
substages: face fluxes along y, then the update by field group with its x
faces (exchanged through LDS within whole x rows) and z faces (marched)),
the tail (H2 clamp, FP64 chemistry, FP64 regularisation, CFL speed) and the
CFL reduction.  The timed region is K steps, each at the CFL dt the
previous step's reduction left on the device (mhd_step_cfl), with the state
resident in HBM, bracketed by device synchronisation.  The FP32 forms'
errors against their FP64 run come from a second, untimed FP32 run that
replays the FP64 dt sequence (each dt held to the FP32 state's CFL bound).

Workloads (synthetic, seeded; see paper_1608_08748_amd/inputs.py):
  c2  256^3 FP64, rms Mach 5, beta 1, x_H2 1e-3, seed 2   (default)
  c3  512^3 FP32 state (FP64 chemistry / reductions), rms Mach 5, beta 0.3,
      seed 3, with the FP64 run of the same seed for the error
  c1  32^3 FP64 white-noise box (the oracle's own configuration)
  c4  1024^3 FP32 single box (about 237 GB of HBM), conservation over the run
  c5  serving: 256 boxes of {32..128}^3 with Poisson arrivals, p50/p99 latency

The default line (c2) also carries two legs of the metric: the FP32 form on
the same 256^3 state with its total and field errors against the FP64 run
(`fp32_leg`), and the serving workload with p50/p99 latency and
served-FP32-vs-FP64 errors for a sample of requests (`serving_leg`);
--no-legs leaves them out.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s FP64 vs FP32 @≤1e-5 rel err; p50/p99 batched-solve latency"
HBM_PEAK_GBS = 8000.0

# algorithmic HBM bytes per cell for one launch of each kernel class, in
# stored values (x 8 B for FP64, x 4 B for FP32): the fields the kernel must
# read once and write once, with neighbour re-reads excluded
# NONADV face class, per launch averaged over its three launches: the y and z
# face kernels read rho, m(3), e, 2 transverse b and the face b_n and write 7
# face outputs; the x-row kernel also updates m, E, e: it reads those 8 fields,
# the y and z face fluxes (5 each), E and Q0 of m, E, e (6), and writes m, E, e
# and the two edge-field components of its faces
ALG_VALUES = {
    "nonadv_face": ((8 + 5 + 5 + 6) + (5 + 2) + 2 * (8 + 7)) / 3,
    "nonadv_update": 6 + 3 + 3 + 3,    # 6 edge-field components, b and Q0 of b (3 each) -> b
    "adv_face": 7 + 7,        # the y march: 7 advected fields -> 7 fluxes
    # the two z-marching update launches that also form the x faces: rho, m
    # (U, Q0, y fluxes -> 4 fields: 16) and E, e, rho_H2 (the same 15 with
    # rho, mx, mz for the face velocities); per launch, averaged
    "adv_update": (16 + 15) / 2,
    "tail": 10 + 2,           # state -> h2, e
}


def _config(name, n=None):
    from paper_1608_08748_amd import binding, inputs
    if name == "c4r":
        n = n or 256
        return dict(desc="c4 recipe at %d^3: lognormal density sigma 1, rms Mach 10, beta 0.1, x_H2 1e-2, FP32 state/"
                         "fluxes, FP64 chemistry/regularisation/CFL/totals, with its FP64 run" % n,
                    n=n, gen=lambda: inputs.c4(n=n), precision=binding.FP32_MIXED, steps=50, dtype="f32+f64")
    if n is not None and name in ("c2", "c3"):
        base = _config(name)
        gen = {"c2": inputs.c2, "c3": inputs.c3}[name]
        base.update(n=n, gen=lambda: gen(n=n), desc=base["desc"].replace("%d^3" % base["n"], "%d^3" % n, 1))
        return base
    if name == "c1":
        return dict(desc="c1: 32^3 periodic box, white-noise velocity sigma 0.1, B=(0.1,0,0), FP64",
                    n=32, gen=lambda: inputs.c1(), precision=binding.FP64, steps=10, dtype="f64")
    if name == "c2":
        return dict(desc="c2: 256^3 periodic supersonic MHD turbulence, rms Mach 5, beta 1, x_H2 1e-3, FP64",
                    n=256, gen=lambda: inputs.c2(), precision=binding.FP64, steps=100, dtype="f64")
    if name == "c3":
        return dict(desc="c3: 512^3 periodic MHD turbulence, rms Mach 5, beta 0.3, FP32 state/fluxes, "
                         "FP64 chemistry/regularisation/CFL/totals",
                    n=512, gen=lambda: inputs.c3(), precision=binding.FP32_MIXED, steps=200, dtype="f32+f64")
    raise SystemExit("unknown config " + name)


def _copy_calibration(nbytes=1 << 30):
    """One device-to-device copy of a known size: its FETCH_SIZE / WRITE_SIZE
    counters calibrate the HBM-traffic counters of the step kernels."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def _timed_run(box, steps, dts=None, record=False):
    """K steps: with the given dt sequence, else each at its CFL dt.  Without
    `record` the CFL dt stays on the device (mhd_step_cfl, no host round trip
    per step); with it every dt is read back and returned."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    used = []
    for s in range(steps):
        if dts is not None:
            box.step(dts[s])
        elif record:
            dt = box.cfl_dt()
            box.step(dt)
            used.append(dt)
        else:
            box.step_cfl()
    box.cfl_dt()            # waits for the last step
    torch.cuda.synchronize()
    return time.perf_counter() - t0, used


# algorithmic floating-point operations per face of the NONADV face kernels,
# counted on the formulas with every add, subtract, multiply, divide, square
# root, min, max and comparison as one: per parabola variable (six) one
# limited slope (11), one interface value (5) and the Steps 2-5 finish (70);
# then the face solve: averaged state 20, eigen-structure 55, the 32 parabola
# averages the waves read 140, characteristic amplitudes 97, projector sum 49,
# fluxes and edge-field terms 24.  The x launch also updates m, E, e: 15 flux
# differences, 17 for the increments and the p dV term, 25 for the
# Runge-Kutta combination of five fields; the class figure is per launch,
# averaged over its three launches.
FACE_FLOPS = 6 * (11 + 5 + 70) + (20 + 55 + 140 + 97 + 49 + 24)
ALG_FLOPS = {"nonadv_face": (3 * FACE_FLOPS + (15 + 17 + 25)) / 3}
# published MI355X vector peaks (TFLOP/s) and HBM peak
VALU_PEAK_TF = {8: 78.6, 4: 157.3}

# HBM traffic of the dominant kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs, keyed by (workload, precision, kernel) and by a hash of
# the kernel sources at the time the counters were taken; FETCH_SIZE is scaled
# by 2 and WRITE_SIZE by 1, the factors that make a 1 GiB device copy read and
# write 1 GiB
TRAFFIC = {
    # average of the x-row (with the m, E, e update), y-march and z-march
    # face kernels, bytes per launch
    ("c2", 8, "nonadv_face"): ("2f1f983544ad1a06", 2868160284),
}


def _kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("mhd_math.hpp", "mhd_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1608_08748_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _roofline(timing, ncell, esz, workload):
    name, (ms, cnt) = max(((k, v) for k, v in timing.items() if k in ALG_VALUES), key=lambda kv: kv[1][0])
    avg_s = ms / cnt / 1e3
    alg_bytes = int(round(ALG_VALUES[name] * esz * ncell))
    gbs = alg_bytes / avg_s / 1e9
    tr = TRAFFIC.get((workload, esz, name))
    traffic = tr[1] if tr is not None and tr[0] == _kernel_source_hash() else None
    out = {"kernel": name, "avg_launch_ms": round(ms / cnt, 4), "launches": cnt, "traffic": traffic,
           "alg_bytes_per_launch": alg_bytes, "hbm_achieved_gbs": round(gbs, 1),
           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    if name in ALG_FLOPS:
        # one face per cell per launch
        tf = ALG_FLOPS[name] * ncell / avg_s / 1e12
        out.update({"bound": "alu", "achieved": round(tf, 2), "peak": VALU_PEAK_TF[esz], "unit": "TFLOP/s",
                    "frac": round(tf / VALU_PEAK_TF[esz], 4), "alg_flops_per_launch": int(round(ALG_FLOPS[name] * ncell))})
    else:
        out.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4)})
    return out


# minimum HBM traffic of a whole step: each of the six Runge-Kutta substages
# reads its inputs and the stage-start state once and writes its outputs once,
# and the tail reads the face fields: 126 field passes per cell-update
STEP_FIELD_PASSES = 126


def _step_roofline(cell_updates_per_s, esz):
    """The whole step's throughput as a fraction of the HBM roofline, against
    the minimum traffic per cell-update (126 field passes of esz bytes)."""
    per_cell = STEP_FIELD_PASSES * esz
    gbs = cell_updates_per_s * per_cell / 1e9
    return {"alg_bytes_per_cell_update": per_cell, "achieved_gbs": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "roofline_cell_updates_per_s": round(HBM_PEAK_GBS * 1e9 / per_cell, 1)}


def _gate_stats(U, gamma=5.0 / 3.0):
    """The two gates of the dual-energy sync (Sec. 2.8 with the pressure
    gate): over the cells of a state after a step, the fractions where the
    sync e := E - K - M ran (both gates open), where the pressure gate
    (gamma - 1)(E - K - M) > B^2/2 kept e, and where the 1e-3 gate kept it;
    and, over the cells the pressure gate kept, the internal energy that
    total-energy conservation would have given minus the one the scheme
    carries, relative to the total internal energy.  Host FP64 from the
    stored values; constant gamma."""
    import numpy as np
    rho, E, e = U[0], U[4], U[5]
    K = 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho
    M = 0.0
    for d in range(3):
        bf = U[6 + d]
        M = M + 0.125 * (bf + np.roll(bf, -1, axis=2 - d)) ** 2
    ei = E - K - M
    g1 = ei >= 1e-3 * E
    g2 = (gamma - 1.0) * ei > M
    kept_p = g1 & ~g2
    n = float(rho.size)
    return {"sync_fraction": float(np.count_nonzero(g1 & g2) / n),
            "kept_by_pressure_gate_fraction": float(np.count_nonzero(kept_p) / n),
            "kept_by_1e-3_gate_fraction": float(np.count_nonzero(~g1) / n),
            "pressure_gate_energy_gap_rel": float((ei[kept_p] - e[kept_p]).sum() / e.sum()),
            "pressure_gate_cells_mean_abs_gap_rel": float(np.mean(np.abs(ei[kept_p] - e[kept_p]) / e[kept_p]))
            if kept_p.any() else 0.0}


def _cpu_baseline(n=192, steps=3, cooling=False, grav_G=0.0, ionisation=False):
    import oracle
    from paper_1608_08748_amd import inputs
    oracle.build(force=False)
    if grav_G > 0:
        n, steps = 64, 2      # the oracle's Poisson solve is a plain O(n^4) transform
    W = inputs.c2(n=n)
    P = oracle.make_params(W.shape[1:], cooling=cooling, grav_G=grav_G, ionisation=ionisation)
    U = oracle.prim_to_cons(P, W)
    t0 = time.perf_counter()
    oracle.run(P, U, steps)
    el = time.perf_counter() - t0
    return {"value": round(n ** 3 * steps / el, 1), "unit": "cell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": "c2 recipe (rms Mach 5, beta 1, seed 2)%s%s%s at %d^3, %d steps, %.1f s"
            % (" with heating/cooling" if cooling else "", " with self-gravity" if grav_G > 0 else "",
               " with the ionisation network" if ionisation else "", n, steps, el)}


def _field_errors(A, B, nf):
    """Per-field L1 and L-inf differences of state A against reference B, each
    relative to the reference field's L1 norm and max-abs value."""
    import numpy as np
    from paper_1608_08748_amd import binding
    out = {}
    for f in range(nf):
        d = np.abs(A[f] - B[f])
        out[binding.FIELDS[f]] = {"l1": float(d.sum() / max(np.abs(B[f]).sum(), 1e-300)),
                                  "linf": float(d.max() / max(np.abs(B[f]).max(), 1e-300))}
    return out


def _total_errors(ta, tb, absq, nf):
    """|total(A) - total(B)| / sum |q_B| per field."""
    from paper_1608_08748_amd import binding
    return {binding.FIELDS[f]: float(abs(ta[f] - tb[f]) / absq[f]) for f in range(nf) if absq[f] > 0}


def _serving(requests, steps, budget_run=False, sample=4, persistent=True):
    """c5: requests with sizes {32,48,64,96,128}^3, rms Mach U[1,10], beta
    U[0.1,10], x_H2 log-uniform [1e-4,1e-1], `steps` steps each, FP32 state
    with FP64 chemistry; saturated run (all at t = 0) for the capacity, then
    Poisson arrivals at 0.8 of it for the latencies (and, with budget_run, a
    2 GB HBM budget).  Request states sit in pinned host memory and are lent
    to the server (no copy at submission; one DMA each at admission).  The
    merged launches are persistent (a resident grid claims the union of the
    boxes' tiles) unless persistent=False; the saturated run is repeated with
    the other launch form for comparison.  For `sample` requests of distinct
    sizes the served FP32 result is compared with the plain FP64 step of the
    same request on the same GPU (each at its own CFL steps)."""
    import numpy as np
    import torch
    from paper_1608_08748_amd import binding, inputs, serving
    torch.cuda.set_device(0)
    reqs = inputs.serving_requests(count=requests, seed=5)
    t = time.perf_counter()
    states = [inputs.request_state(r) for r in reqs]
    gen_s = time.perf_counter() - t
    t = time.perf_counter()
    pinned = []
    for W in states:
        P = torch.empty(W.shape, dtype=torch.float64, pin_memory=True).numpy()
        P[...] = W
        pinned.append(P)
    states = pinned
    pin_s = time.perf_counter() - t
    mean_cells = float(np.mean([r["n"] ** 3 for r in reqs]))
    # the first request of each size, smallest sizes first
    first = {}
    for i, r in enumerate(reqs):
        first.setdefault(r["n"], i)
    keep = [first[n] for n in sorted(first)][:sample]

    def one(budget, slots, arrivals, keep_idx=(), pers=persistent):
        sv = binding.Server(budget, max_slots=slots, precision=binding.FP32_MIXED, persistent=pers)
        out = serving.run(sv, states, steps, arrivals=arrivals, borrow=True, keep_state=set(keep_idx))
        kept = {i: sv.result(out["records"][i]["id"]) for i in keep_idx}
        _, peak, cap = sv.memory()
        sv.close()
        torch.cuda.empty_cache()
        out["kept"] = kept
        out["peak_pool_bytes"] = peak
        out["pool_bytes"] = cap
        return out

    # warm-up: a few requests through the merged kernels of both forms
    for pers in (False, True):
        sv = binding.Server(4 << 30, max_slots=8, precision=binding.FP32_MIXED, persistent=pers)
        serving.run(sv, states[:4], 2, borrow=True)
        sv.close()
    budget, slots = 64 << 30, 128
    sat = one(budget, slots, None)
    sat_other = one(budget, slots, None, pers=not persistent)
    req_rate = 0.8 * sat["throughput"] / (mean_cells * steps)
    arr = serving.poisson_arrivals(len(states), req_rate, seed=5)
    poi = one(budget, slots, arr, keep)
    # served FP32 against the plain FP64 step of the same requests, run as a
    # single FP64 box at its own CFL steps (each form at the dt sequence its
    # own state chooses: over 50 steps of Mach-10 turbulence the two states
    # part far enough that one form's dt can exceed the other's CFL bound);
    # an FP32 single box at its own CFL steps reproduces the served bits
    def errs(G, t, R, tR):
        absq = np.abs(R).reshape(binding.NFIELDS, -1).sum(axis=1)
        te = _total_errors(t, tR, absq, binding.NFIELDS - 1)
        fe = _field_errors(G, R, binding.NFIELDS - 1)
        return {"max_total_rel_err": max(te.values()), "total_rel_err": te,
                "max_field_l1_rel": max(v["l1"] for v in fe.values()),
                "max_field_linf_rel": max(v["linf"] for v in fe.values())}

    def single(W, precision):
        b = binding.Box(W.shape[1:], precision=precision)
        b.init_state(W)
        for _ in range(steps):
            b.step_cfl()
        G, t = b.get_state(), b.totals()
        b.close()
        return G, t, None

    cmp = []
    for i in keep:
        W = states[i]
        G32 = poi["kept"][i]
        t32 = np.asarray(poi["records"][i]["totals"])
        G64, t64, _ = single(W, binding.FP64)
        S32, _, _ = single(W, binding.FP32_MIXED)
        row = {"request": i, "n": reqs[i]["n"], "mach": round(reqs[i]["mach"], 3), "beta": round(reqs[i]["beta"], 3),
               "served_equals_single_box": bool(np.array_equal(S32, G32))}
        row.update(errs(G32, t32, G64, t64))
        cmp.append(row)
    torch.cuda.empty_cache()
    keys = ("throughput", "span_s", "rounds", "max_active", "statuses", "latency_p50", "latency_p99",
            "latency_mean", "peak_pool_bytes")
    res = {
        "value": round(poi["throughput"], 1), "unit": "cell-updates/s", "requests": len(states), "steps": steps,
        "latency_p50_s": round(poi["latency_p50"], 4), "latency_p99_s": round(poi["latency_p99"], 4),
        "arrival_rate_per_s": round(req_rate, 3), "hbm_budget_bytes": budget, "max_slots": slots,
        "launches": "persistent" if persistent else "one workgroup per tile",
        "poisson": {k: poi[k] for k in keys},
        "saturated": {k: sat[k] for k in keys},
        ("saturated_one_workgroup_per_tile" if persistent else "saturated_persistent"):
            {k: sat_other[k] for k in keys},
        "fp32_vs_fp64": {"what": "served FP32 result after %d steps against the plain FP64 step of the same "
                                 "request (single box, FP64 state), each at the CFL steps of its own state; an "
                                 "FP32 single box reproduces the served bits (served_equals_single_box); totals "
                                 "relative to sum |q|, fields L1 relative to the field's L1 norm, L-inf to its "
                                 "max" % steps,
                         "gate_total_rel": 1e-5,
                         "max_conserved_total_rel_err": max(
                             max(c["total_rel_err"][f] for f in CONSERVED) for c in cmp) if cmp else None,
                         "requests": cmp},
        "ic_generation_s": round(gen_s, 1), "pinning_s": round(pin_s, 1),
    }
    if budget_run:
        small = one(2 << 30, slots, None)
        res["budget_2GB"] = {k: small[k] for k in keys + ("pool_bytes",)}
    return res


def _serving_bench(args):
    """The serving workload as the line's headline."""
    steps = args.steps if args.steps is not None else 50
    sv = _serving(args.requests, steps, budget_run=True, persistent=args.launch == "persistent")
    return {
        "metric": METRIC, "value": sv["value"], "unit": "cell-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "c5: %d requests, boxes {32,48,64,96,128}^3, rms Mach U[1,10], beta U[0.1,10], "
                               "x_H2 log-uniform [1e-4,1e-1], %d steps each, FP32 state + FP64 chemistry, "
                               "Poisson arrivals at 0.8 x saturated capacity" % (sv["requests"], steps),
                   "hbm_budget_bytes": sv["hbm_budget_bytes"], "max_slots": sv["max_slots"],
                   "request_states": "pinned host memory, lent",
                   "parallelism": "single GPU, %s multi-box launches" % sv["launches"]},
        "serving": sv,
    }


def _largest_box_bench(args):
    """c4: one 1024^3 FP32 box (three state copies of 11 fields = 142 GB plus
    scratch, about 237 GB of HBM), lognormal density, rms Mach 10, beta 0.1.
    There is no FP64 twin at this size (it would need twice the memory); the
    full-size checks are the properties that hold at any size: conservation of
    mass, momentum, energy and face flux over the run, finiteness and
    positivity (latched faults)."""
    import numpy as np
    import torch
    from paper_1608_08748_amd import binding, inputs
    steps = args.steps if args.steps is not None else 50
    n = 1024
    torch.cuda.set_device(0)

    def log(msg):
        print("c4: " + msg, file=sys.stderr, flush=True)

    # warm-up on a small box (kernel loading)
    wb = binding.Box((64, 64, 64), precision=binding.FP32_MIXED)
    wb.init_state(inputs.c4(n=64))
    for _ in range(max(args.warmup, 1)):
        wb.step(wb.cfl_dt())
    wb.close()
    del wb
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    log("device memory free %.1f GB of %.1f GB" % (free / 1e9, total / 1e9))
    t = time.perf_counter()
    W = inputs.c4(n=n, log=log)
    log("initial condition generated in %.1f s" % (time.perf_counter() - t))
    box = binding.Box((n, n, n), precision=binding.FP32_MIXED)
    log("workspace %.1f GB" % (box.ws.numel() / 1e9))
    box.init_state(W)
    del W
    t0 = box.totals()
    box.set_timing(True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for s in range(steps):
        box.step_cfl()
        if s % 10 == 9:
            box.cfl_dt()    # waits, so the progress line follows the device
            log("step %d" % (s + 1))
    box.cfl_dt()
    torch.cuda.synchronize()
    el = time.perf_counter() - ts
    timing = box.get_timing()
    box.set_timing(False)
    t1 = box.totals()
    ncell = n ** 3
    drift = {binding.FIELDS[f]: float(abs(t1[f] - t0[f]) / max(abs(t0[f]), 1e-300)) for f in (0, 4, 6)}
    for f in (1, 2, 3, 7, 8):   # zero-mean fields: relative to the cell count
        drift[binding.FIELDS[f]] = float(abs(t1[f] - t0[f]) / ncell)
    return {
        "metric": METRIC, "value": round(ncell * steps / el, 1), "unit": "cell-updates/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(el / steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "c4: 1024^3 periodic MHD turbulence, lognormal density sigma 1, rms Mach 10, "
                               "beta 0.1, x_H2 1e-2, FP32 state/fluxes, FP64 chemistry/regularisation/CFL/totals",
                   "cells": ncell, "grid": [n, n, n], "workspace_bytes": int(box.ws.numel()),
                   "parallelism": "single GPU"},
        "roofline": _roofline(timing, ncell, 4, "c4"),
        "step_roofline": _step_roofline(ncell * steps / el, 4),
        "kernel_ms_per_step": {k: round(v[0] / steps, 3) for k, v in timing.items()},
        "conservation_drift": drift,
    }


# totals the flux form conserves (e has its p dV source, rho_H2 its chemistry)
CONSERVED = ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")


def _precision_leg(W, shape, steps, warmup, dts, G64, t64, phys, workload, gate=False):
    """FP32 state on the workload's state.  Timed: `steps` steps at the FP32
    state's own CFL dt (device-resident, as the FP64 line).  Errors: the FP64
    run's dt sequence replayed on the FP32 state, each dt held to the FP32
    state's own CFL bound (the two states drift apart, and after tens of
    steps the FP64 dt can exceed the FP32 bound by 1e-3), against that FP64
    run: every total and field."""
    import numpy as np
    import torch
    from paper_1608_08748_amd import binding
    box = binding.Box(shape, precision=binding.FP32_MIXED, **phys)
    box.init_state(W)
    for s in range(warmup):
        box.step_cfl()
    box.init_state(W)
    box.set_timing(True)
    el, _ = _timed_run(box, steps)
    timing = box.get_timing()
    box.set_timing(False)
    box.init_state(W)
    held, t_ref, t_run = [], 0.0, 0.0
    for s in range(steps):
        own = box.cfl_dt()
        dt = dts[s]
        if dt > own:
            held.append(dt / own - 1.0)
            dt = own
        box.step(dt)
        t_ref += dts[s]
        t_run += dt
    box.cfl_dt()
    t32 = box.totals()
    G32 = box.get_state()
    box.close()
    del box
    torch.cuda.empty_cache()
    nf = binding.NFIELDS if phys.get("ionisation") else binding.NFIELDS - 1
    ncell = int(np.prod(shape))
    absq = np.abs(G64).reshape(binding.NFIELDS, -1).sum(axis=1)
    te = _total_errors(t32, t64, absq, nf)
    fe = _field_errors(G32, G64, nf)
    gates = _gate_stats(G32) if gate else None
    del G32
    return {
        "value": round(ncell * steps / el, 1), "unit": "cell-updates/s", "ms_per_step": round(el / steps * 1e3, 3),
        "dtype": "f32+f64", "steps": steps,
        "what": "FP32 state and fluxes with FP64 chemistry, regularisation, CFL and totals, on the same initial "
                "state; timed at its own CFL dt; errors from a second run replaying the FP64 run's dt sequence "
                "(each dt held to the FP32 state's CFL bound) against that FP64 run: totals relative to sum |q|, "
                "fields L1 relative to the field's L1 norm and L-inf relative to its max",
        "dt_held_steps": len(held),
        "dt_held_max_rel": max(held) if held else 0.0,
        "elapsed_time_rel_diff": (t_ref - t_run) / t_ref,
        "roofline": _roofline(timing, ncell, 4, workload),
        "step_roofline": _step_roofline(ncell * steps / el, 4),
        "kernel_ms_per_step": {k: round(v[0] / steps, 3) for k, v in timing.items()},
        "gate_total_rel": 1e-5,
        "max_total_rel_err": max(te.values()),
        "max_conserved_total_rel_err": max(te[f] for f in CONSERVED if f in te),
        "total_rel_err": te,
        "fp32_field_err": fe,
        **({"regularisation_gates": gates} if gate else {}),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c4r", "c5"])
    ap.add_argument("--n", type=int, default=None, help="c2, c3, c4r: cells per axis (other than the configured)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--launch", default="persistent", choices=["persistent", "tile"],
                    help="serving: persistent multi-box launches, or one workgroup per tile")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="c2: leave out the FP32 and serving legs of the line")
    ap.add_argument("--cpu-only", action="store_true",
                    help="time only the oracle on the c2 recipe (--cpu-n, --cpu-steps; threads from "
                         "OMP_NUM_THREADS) and print its cpu_baseline object")
    ap.add_argument("--cpu-n", type=int, default=192)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--gate-stats", action="store_true",
                    help="c2, c3: add the regularisation gate statistics of the FP64 reference state")
    ap.add_argument("--cooling", action="store_true",
                    help="c1-c3: add the heating/cooling stage (Sec. 2 stage 5) after chemistry")
    ap.add_argument("--gravity", action="store_true",
                    help="c1-c3: add self-gravity (FFT Poisson solve each step, sources in NONADV)")
    ap.add_argument("--ionisation", action="store_true",
                    help="c1-c3: add the ionisation network (reactions 5-8, H+ field, gamma_eff)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this implementation runs one box on one GPU; --gpus %d is not supported "
              "(multi-GPU sharding is a design note only)" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)
    if args.cpu_only:
        print(json.dumps({"cpu_baseline": _cpu_baseline(n=args.cpu_n, steps=args.cpu_steps)}), flush=True)
        return

    import numpy as np
    import torch
    from paper_1608_08748_amd import binding

    def log(msg):
        print("bench: " + msg, file=sys.stderr, flush=True)

    if args.config == "c5":
        print(json.dumps(_serving_bench(args)), flush=True)
        return
    if args.config == "c4":
        print(json.dumps(_largest_box_bench(args)), flush=True)
        return

    cfg = _config(args.config, args.n)
    steps = args.steps if args.steps is not None else cfg["steps"]
    W = cfg["gen"]()
    log("initial condition %s generated" % (W.shape[1:],))
    shape = W.shape[1:]
    ncell = int(np.prod(shape))
    torch.cuda.set_device(0)
    cool = bool(args.cooling)
    if cool:
        cfg["desc"] += " + heating/cooling stage"
    gG = binding.gravity_G() if args.gravity else 0.0
    if gG > 0:
        cfg["desc"] += " + self-gravity (G = %.4f code units)" % gG
    ion = bool(args.ionisation)
    if ion:
        cfg["desc"] += " + ionisation network (H+ from zero)"
    phys = dict(cooling=cool, grav_G=gG, ionisation=ion)
    workload = args.config + ("+gravity" if gG > 0 else "") + ("+ionisation" if ion else "")
    esz = 8 if cfg["precision"] == binding.FP64 else 4
    legs = args.config in ("c3", "c4r") or (args.config == "c2" and not args.no_legs)

    # the FP64 run with its dt sequence read back each step: the reference of
    # the FP32 errors (c3's FP64 figure is this run's rate)
    ref_dts = G64 = t64 = None
    extra = {}
    if legs:
        ref = binding.Box(shape, precision=binding.FP64, **phys)
        ref.init_state(W)
        for _ in range(args.warmup):
            ref.step(ref.cfl_dt())
        ref.init_state(W)
        el64, ref_dts = _timed_run(ref, steps, record=True)
        t64 = ref.totals()
        G64 = ref.get_state()
        if args.gate_stats:
            extra["regularisation_gates"] = _gate_stats(G64)
        ref.close()
        del ref
        torch.cuda.empty_cache()
        log("FP64 reference run: %d steps, %.3f s" % (steps, el64))
        if args.config in ("c3", "c4r"):
            extra["fp64_same_seed"] = {"value": round(ncell * steps / el64, 1),
                                       "ms_per_step": round(el64 / steps * 1e3, 3)}

    if args.config in ("c3", "c4r"):
        leg = _precision_leg(W, shape, steps, args.warmup, ref_dts, G64, t64, phys, workload, gate=args.gate_stats)
        del G64
        out = {
            "metric": METRIC, "value": leg["value"], "unit": "cell-updates/s",
            "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": leg["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": cfg["dtype"],
            "data": "synthetic",
            "config": {"workload": cfg["desc"], "cells": ncell, "grid": list(shape)[::-1], "cfl": 0.3,
                       "gamma": 5.0 / 3.0, "theta": 1.0, "heating_cooling": cool, "self_gravity": gG > 0,
                       "ionisation": ion, "parallelism": "single GPU"},
        }
        for k in ("roofline", "step_roofline", "kernel_ms_per_step", "gate_total_rel", "max_total_rel_err",
                  "max_conserved_total_rel_err"):
            out[k] = leg[k]
        out["fp32_total_rel_err"] = leg["total_rel_err"]
        out["fp32_field_err"] = leg["fp32_field_err"]
        out.update(extra)
        if args.gate_stats:
            out["regularisation_gates"] = {"fp64": extra["regularisation_gates"], "fp32": leg["regularisation_gates"]}
    else:
        box = binding.Box(shape, precision=cfg["precision"], **phys)
        box.init_state(W)
        for _ in range(args.warmup):
            box.step(box.cfl_dt())
        box.init_state(W)      # timed run starts from the initial condition
        _copy_calibration()
        box.set_timing(True)
        el, _ = _timed_run(box, steps)
        timing = box.get_timing()
        box.set_timing(False)
        tot = box.totals()
        box.close()
        del box
        torch.cuda.empty_cache()
        log("timed run: %d steps, %.3f s" % (steps, el))
        out = {
            "metric": METRIC, "value": round(ncell * steps / el, 1), "unit": "cell-updates/s",
            "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": round(el / steps * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": cfg["dtype"],
            "data": "synthetic",
            "config": {"workload": cfg["desc"], "cells": ncell, "grid": list(shape)[::-1], "cfl": 0.3,
                       "gamma": 5.0 / 3.0, "theta": 1.0, "heating_cooling": cool, "self_gravity": gG > 0,
                       "ionisation": ion, "parallelism": "single GPU"},
            # counters are keyed by workload: self-gravity and the ionisation
            # network change the face kernels, heating/cooling only the tail
            "roofline": _roofline(timing, ncell, esz, workload),
            "step_roofline": _step_roofline(ncell * steps / el, esz),
            "kernel_ms_per_step": {k: round(v[0] / steps, 3) for k, v in timing.items()},
            "totals_end": [float(x) for x in tot],
        }
        if legs:
            # the timed run (device-resident dt) and the reference run (dt read
            # back) compute the same bits
            out["reference_run_bitwise"] = bool(np.array_equal(tot, t64))
            out.update(extra)
            out["fp32_leg"] = _precision_leg(W, shape, steps, args.warmup, ref_dts, G64, t64, phys, workload)
            del G64
            log("FP32 leg done")
            out["serving_leg"] = _serving(args.requests, 50, persistent=args.launch == "persistent")
            log("serving leg done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(cooling=cool, grav_G=gG, ionisation=ion)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
