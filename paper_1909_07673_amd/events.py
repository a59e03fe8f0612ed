"""Discrete-event replay of tenant requests on one data center, the
evaluation procedure of section VI-A: requests arrive at given events and
run for a given number of events; at every event the departures due give
their resources back, the arrivals join a waiting queue, and every waiting
request is submitted again in FCFS order; the ones that do not fit (all or
nothing) wait for the next event.

Host orchestration only: every placement, rejection and release is a call
into the library (dc_submit_request, dc_schedule, dc_release); the
fragmentation shares and utilities are read from the library's state
(dc_get_state) and allocations (dc_get_alloc)."""
from __future__ import annotations

import numpy as np

from .binding import RESULT_DTYPE


def unit_steps(req, status: int, failed_at: int) -> int:
    """Scoring steps a request took: one per pod (a container without a pod
    is a pod of its own), in the order of each pod's first container."""
    pod = getattr(req, "pod", None)
    if status == 0 and failed_at >= req.n:      # every pod placed, links did not fit
        status = 1
    if pod is None:
        return req.n if status == 1 else failed_at + 1
    seen, unit = {}, []
    for i, p in enumerate(pod):
        key = ("p", int(p)) if p >= 0 else ("c", i)
        seen.setdefault(key, len(seen))
        unit.append(seen[key])
    return len(seen) if status == 1 else unit[failed_at] + 1


def fragmentation(state: np.ndarray, link_caps) -> tuple:
    """Server and link fragmentation of section II-B: F(N^s), the share of
    servers hosting a container, and F(E^s), the share of links carrying
    traffic (available bandwidth below capacity).  state is dc_get_state's
    [6][N]; link_caps the three per-level capacities."""
    st = np.asarray(state, np.int64)
    caps = np.asarray(link_caps, np.int64)[:, None]
    return float((st[2] > 0).mean()), float((st[3:] < caps).mean())


def utilities(req, cpu_a, ram_a, bw_a) -> tuple:
    """U(i) per container (mean over CPU and RAM of allocated / maximum) and
    U(ij) per edge (allocated / maximum bandwidth), Eqs. (1)-(2)."""
    cx = req.cpu if req.cpu_max is None else req.cpu_max
    rx = req.ram if req.ram_max is None else req.ram_max
    bx = req.edges[:, 2] if req.bw_max is None else req.bw_max
    return (cpu_a / cx + ram_a / rx) / 2, bw_a / bx


def replay(sched, reqs, arrive, dur, link_caps, on_event=None) -> dict:
    """Replays requests reqs arriving at events arrive[q] (non-decreasing)
    and running dur[q] events once placed, on `sched` (a plain-form
    Scheduler of one data center), until every request is placed.  A
    request whose single pod cannot fit an empty data center would wait for
    ever; the caller's workload must not contain one.

    on_event(ev, submitted, results): optional callback after each event's
    schedule call with the submitted request indices and their results.

    Returns: placed[q] (event placed), rid[q] (the accepted attempt's id),
    events, steps (scoring steps), submissions, frag_s / frag_l (per
    event, after its submissions), delay[q]."""
    n = len(reqs)
    buf = np.zeros(max(n, 1), RESULT_DTYPE)
    placed = np.full(n, -1)
    acc_id = np.full(n, -1, np.int64)
    queue, ends = [], {}
    nxt = ev = steps = tries = 0
    frag_s, frag_l = [], []
    while nxt < n or queue:
        for rid in ends.pop(ev, []):
            rc = sched.release(rid)
            if rc != 0:
                raise RuntimeError(f"release of request {rid} failed ({rc})")
        while nxt < n and arrive[nxt] <= ev:
            queue.append(nxt)
            nxt += 1
        if queue:
            ids = [sched.submit(reqs[q]) for q in queue]
            res = sched.schedule_array(buf[:len(queue)])
            tries += len(queue)
            still = []
            for q, rid, r in zip(queue, ids, res):
                steps += unit_steps(reqs[q], int(r["status"]), int(r["failed_at"]))
                if r["status"] == 1:
                    placed[q] = ev
                    acc_id[q] = rid
                    ends.setdefault(ev + int(dur[q]), []).append(rid)
                else:
                    still.append(q)
            if on_event is not None:
                on_event(ev, list(queue), res.copy())
            queue = still
        fs, fl = fragmentation(sched.state(0), link_caps)
        frag_s.append(fs)
        frag_l.append(fl)
        ev += 1
    return dict(placed=placed, rid=acc_id, events=int(placed.max()) + 1 if n else 0, steps=steps,
                submissions=tries, frag_s=frag_s, frag_l=frag_l, delay=placed - np.asarray(arrive))
