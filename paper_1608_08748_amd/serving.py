"""Serving loop: requests arrive (Poisson process or all at once), are
submitted to a ``binding.Server`` as they arrive, and the host loop calls
``progress`` (admission + one merged step of every box in flight, pipelined
one round deep) until all requests have completed.  Latency is arrival to completion on the host clock;
throughput is total cell-updates over the span from the first arrival to the
last completion."""
import time

import numpy as np


def run(server, states, steps, arrivals=None, keep_state=False, borrow=False):
    """states: list of primitive arrays; arrivals: seconds after start for each
    request (None = all at t = 0); keep_state: True for every request, or a
    collection of request indices whose final state the server keeps for
    ``server.result``; borrow: lend the arrays to the server instead of
    copying them at submission.  Returns a dict of per-request records and
    aggregate statistics."""
    nreq = len(states)
    arr = np.zeros(nreq) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    order = np.argsort(arr, kind="stable")
    t0 = time.perf_counter()
    nxt = 0
    sid_of = {}
    rec = {}
    rounds = 0
    max_active = 0
    while len(rec) < nreq:
        now = time.perf_counter() - t0
        while nxt < nreq and arr[order[nxt]] <= now:
            i = int(order[nxt])
            keep = keep_state if isinstance(keep_state, bool) else i in keep_state
            sid = server.submit(states[i], steps, keep_state=keep, borrow=borrow)
            sid_of[sid] = i
            nxt += 1
        na, npend = server.progress()
        rounds += 1
        max_active = max(max_active, na)
        t_poll = time.perf_counter() - t0
        for c in server.poll():
            i = sid_of[c["id"]]
            c["index"] = i
            c["t_arrive"] = float(arr[i])
            c["t_complete"] = t_poll
            c["latency"] = t_poll - float(arr[i])
            rec[i] = c
        # idle until the next arrival only once every submitted request has
        # been reported (the last round's completions come with the next call)
        if na == 0 and npend == 0 and nxt < nreq and len(rec) == nxt:
            wait = arr[order[nxt]] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
    lat = np.array([rec[i]["latency"] for i in range(nreq)])
    cells = sum(int(rec[i]["cells"]) for i in range(nreq)) * steps
    span = max(rec[i]["t_complete"] for i in range(nreq)) - float(arr.min())
    return dict(records=[rec[i] for i in range(nreq)], latency_p50=float(np.percentile(lat, 50)),
                latency_p99=float(np.percentile(lat, 99)), latency_mean=float(lat.mean()),
                cell_updates=cells, span_s=span, throughput=cells / span, rounds=rounds, max_active=max_active,
                statuses=sorted(set(int(rec[i]["status"]) for i in range(nreq))))


def poisson_arrivals(n, rate, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
