#!/usr/bin/env python3
"""Throughput benchmark of the container-scheduling hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic requests:
the data-center state is rewound to its initial (background-loaded) state
and every request is scheduled in FCFS order -- per container: path stage,
criteria, scoring, selection, commit -- with the results copied back.  The
requests are uploaded to HBM before the timed region.

Default workload (one JSON line): k=16 fat-tree (1024 hosts), 40 Gbps host
links, 100 Gbps edge-aggregation / aggregation-core links, 0-70 %
background load, 2,000 FCFS requests of 2-32 containers, TOPSIS over (CPU,
RAM, active, path bandwidth), plain form: one kernel launch per container
step.  Other workloads (--workload) measure the batched form (256
instances), the large AHP case and the serving form on a Poisson trace.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "host-scores/sec (containers×hosts/s) at 1 GPU; p50/p99 per-request latency"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per host score of the fused step kernel: the six int32
# state arrays (CPU, RAM, placed count, uplink, edge-aggregation and
# aggregation-core residuals) read once per scored host.
BYTES_PER_HOST_SCORE = 24
# FP32 vector peak of MI355X, 157.3 TFLOP/s (256 CUs x 2.4 GHz x 128 FMA
# lanes per clock), as VALU lane-instructions per second: one lane-FMA per
# issue slot.  The Saaty passes are mostly compares and selects, which do not
# pack, so this peak is generous to them.
VALU_LANE_OPS = 157.3e12 / 2

WORKLOADS = {
    "plain": dict(preset="plain", mode="plain", method="topsis",
                  text="k=16 fat-tree (1024 hosts), 2000 FCFS requests of 2-32 containers, 0-70% background, "
                       "TOPSIS on CPU/RAM/active/path-bw, plain form (one launch per container step)"),
    "batched": dict(preset="batched", mode="batched", method="topsis",
                    text="256 independent k=16 fat-trees (1024 hosts each), 64-512 requests of 2-48 containers "
                         "per instance, TOPSIS, batched form (one persistent launch)"),
    "ahp": dict(preset="ahp", mode="plain", method="ahp",
                text="k=32 fat-tree (8192 hosts), 500 FCFS requests of 8-64 containers, 0-70% background, AHP "
                     "(Saaty 1-9) on CPU/RAM/uplink/path-bw/hops(cost), seven launches per container step"),
    "pods": dict(preset="pods", mode="plain", method="topsis",
                 text="k=16 fat-tree (1024 hosts), 2000 FCFS requests of 2-32 containers with up to half of each "
                      "request's containers in pods of 2-4 (one placement per pod), 0-70% background, TOPSIS, "
                      "plain form (one launch per pod step)"),
    "route_end": dict(preset="plain", mode="plain", method="topsis", routing=1,
                      text="k=16 fat-tree (1024 hosts), 2000 FCFS requests of 2-32 containers, 0-70% background, "
                           "TOPSIS, links routed after each request's last container (one wave per pair on the "
                           "residuals the placement left), plain form (one launch per container step)"),
    "ranges": dict(preset="ranges", mode="plain", method="topsis",
                   text="k=16 fat-tree (1024 hosts), 2000 FCFS requests of 2-32 containers with up to half in pods "
                        "and demands as [min, 2 x min] intervals (each placement given up to the maximum), 0-70% "
                        "background, TOPSIS, plain form (one launch per pod step)"),
    "paper_e2": dict(preset=None, mode="events", method="topsis",
                     text="the paper's GPU evaluation shape (section VI-A): k=20 fat-tree (2000 servers of 24 cores / "
                          "256 GB, 1 Gbps links), 6000 requests of 4 containers (up to half in pods, demands as "
                          "intervals up to 2 cores, 4 GB and 50 Mbps per pair) arriving over 250 of 500 events and "
                          "running 1-250 events; discrete-event replay, waiting requests retried in FCFS order at "
                          "every event; TOPSIS (Flat), plain form"),
    "paper_e2_ahp": dict(preset=None, mode="events", method="ahp",
                         text="as paper_e2 with AHP (Saaty 1-9, Flat weights)"),
    "tiles": dict(preset=None, mode="tiles", method="topsis",
                  text="TOPSIS scoring + selection alone (dc_topsis_tiles) over 32,768 materialised 4 x 1024 "
                       "integer decision matrices (512 MiB, the batched shape: 256 instances x 128 steps), "
                       "best server and score per matrix"),
    "serving": dict(preset="serving", mode="serving", method="topsis",
                    text="k=48 fat-tree (27648 hosts), 0-70% background, Poisson arrivals at 5000 req/s of 2-64 "
                         "containers, exponential lifetimes (mean 60 s) releasing their resources, TOPSIS, "
                         "serving form (persistent kernel) against the plain form on the same trace"),
}


def step_count(results):
    return sum(r.n if r.status == 1 else r.failed_at + 1 for r in results)


def _pod_steps(req, status, failed_at):
    """Steps a request took: one per pod (a container without a pod is a pod
    of its own), in the order of each pod's first container."""
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


def step_count_array(res, reqs=None):
    """Scoring steps in a RESULT_DTYPE record array (one per container, or
    one per pod when the requests, in result order, carry pods)."""
    import numpy as np
    if reqs is None:
        return int(np.where(res["status"] == 1, res["n"], res["failed_at"] + 1).sum())
    return sum(_pod_steps(q, int(r["status"]), int(r["failed_at"])) for q, r in zip(reqs, res))


def host_cpu():
    """The host's CPU model and the logical CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {len(os.sched_getaffinity(0))} logical CPUs available"


def cpu_baseline(insts, reqs, budget_s, meth):
    """The FP64 oracle, as it stands, on a bounded prefix of the same
    workload (single thread): the requests of instance 0 in FCFS order, then
    those of the next instances, until the time budget is spent."""
    import oracle
    steps = n_req = n_inst = 0
    t0 = time.perf_counter()
    for inst, rl in zip(insts, reqs):
        o = oracle.Oracle(inst, meth)
        n_inst += 1
        for req in rl:
            res = o.run_request(req)
            steps += _pod_steps(req, res["status"], res["failed_at"])
            n_req += 1
            if time.perf_counter() - t0 > budget_s:
                break
        o.close()
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    N = insts[0].n_hosts
    where = "the same workload" if n_inst == 1 else f"the first {n_inst} instances of the same workload"
    return dict(value=steps * N / dt, unit="host-scores/s", cores=1, kind="oracle",
                sample=f"first {n_req} requests ({steps} scoring steps) of {where} on one host "
                       f"thread, {dt:.1f} s", host=host_cpu())


def percentiles(x):
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99))} if x.size else None


def run_batch(args, wl):
    """Plain / batched / AHP: rewind + schedule all requests per step."""
    import numpy as np
    import torch
    import oracle
    import paper_1909_07673_amd as dc
    from workloads import make_config

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    insts, reqs = make_config(wl["preset"], seed=0)
    N = insts[0].n_hosts
    kw = {}
    if wl["method"] == "ahp":
        kw = dict(method=dc.DC_AHP, crit=(dc.DC_CRIT_CPU, dc.DC_CRIT_RAM, dc.DC_CRIT_UPLINK, dc.DC_CRIT_PATHBW,
                                          dc.DC_CRIT_HOPS), cost=(0, 0, 0, 0, 1))
    mode = dc.DC_MODE_BATCHED if wl["mode"] == "batched" else dc.DC_MODE_PLAIN
    s = dc.Scheduler(insts, mode=mode, stream=stream, grid=args.grid, graph=args.graph, block=args.block,
                     routing=wl.get("routing", 0), **kw)
    for i, rl in enumerate(reqs):
        for r in rl:
            s.submit(r, instance=i)
    s.rewind()                      # uploads the requests; they stay resident in HBM
    # the batched form autotunes its workgroup size; the plain form keeps the
    # library's size for its server count (1,024 threads from 257 servers on,
    # which the autotuner also picks there), so a profiled run times the same
    # kernel as an unprofiled one
    if args.block:
        tuned = args.block
    elif mode == dc.DC_MODE_BATCHED and wl["method"] == "topsis":
        tuned = s.autotune()
    else:
        tuned = 64 if N <= 64 else 256 if N <= 256 else 1024
    torch.cuda.synchronize()
    buf = np.zeros(s.pending(), dc.RESULT_DTYPE)
    for _ in range(args.warmup):
        s.rewind()
        s.schedule_array(buf)
    torch.cuda.synchronize()
    kern_ms, launches, results = 0.0, 0, None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.rewind()
        results = s.schedule_array(buf)
        ms, la, _ = s.last_timing()
        kern_ms += ms
        launches += la
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert len(results) == len(buf), "every queued request is decided in a step"
    flat = [q for rl in reqs for q in rl]       # submission order = result (request id) order
    with_pods = any(getattr(q, "pod", None) is not None for q in flat)
    steps = step_count_array(results, flat if with_pods else None)
    per_inst = np.bincount(results["instance"], weights=[
        _pod_steps(q, int(r["status"]), int(r["failed_at"])) for q, r in zip(flat, results)],
        minlength=len(insts))
    hs = steps * N
    value = hs * args.steps / wall
    lat = s.latency_us()
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    per_step_launches = max(launches // args.steps, 1)
    out = {
        "metric": METRIC, "value": value, "unit": "host-scores/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["text"], "k": insts[0].k, "hosts": N, "instances": len(insts),
                   "requests": sum(len(r) for r in reqs), "container_steps": steps,
                   "form": wl["mode"], "method": wl["method"], "block": tuned, "grid": args.grid,
                   "graph": args.graph,
                   "steps_per_instance": {"mean": float(per_inst.mean()), "max": int(per_inst.max())}},
        "latency_us": dict(percentiles(lat), kind="service (first step start to decision), device clock"),
    }
    if wl["method"] == "topsis":
        kname = ("k_topsis_batched" if mode == dc.DC_MODE_BATCHED else
                 "k_topsis_grid" if args.grid == 2 else "k_topsis_plain")
        bytes_per_launch = BYTES_PER_HOST_SCORE * hs / per_step_launches
        achieved = bytes_per_launch / avg_launch_s / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "avg_launch_us": avg_launch_s * 1e6, "launches_per_step": per_step_launches,
                           "bytes_per_launch": bytes_per_launch}
        meth = oracle.method(kind=oracle.TOPSIS, route_end=bool(wl.get("routing", 0)))
        if not args.no_scoring_kernel:
            # the scoring stage alone, streaming resident matrices (HBM-bound)
            out["scoring_kernel_roofline"] = dict(
                tile_timing(20, 2)[3], workload=WORKLOADS["tiles"]["text"])
    else:
        C = 5
        if N <= AHP_SORT_MAX:
            # AHP on the 1-9 scale through the sorted passes: the only
            # O(C N^2) work is the rank count, one compare per pair and
            # criterion at RANK_OPS VALU lane-instructions; the rate is taken
            # over the whole step's kernel time (all seven launches)
            pairs, ops, kname, unit = 1.0 * C * N * N * steps, AHP_RANK_OPS, "k_ahp_rank", "pair-compares/s"
        else:
            # pairwise passes: 2*C*N^2 Saaty evaluations per container step
            pairs, ops, kname, unit = 2.0 * C * N * N * steps, AHP_PAIR_OPS, "k_ahp_colsum+k_ahp_rowsum", "pair-evals/s"
        rate = pairs * args.steps / (kern_ms / 1e3)
        out["roofline"] = {"bound": "alu", "kernel": kname, "unit": unit, "achieved": rate,
                           "peak": VALU_LANE_OPS / ops, "frac": rate / (VALU_LANE_OPS / ops),
                           "traffic": None, "pair_ops": ops, "basis": "whole AHP step kernel time",
                           "avg_launch_us": avg_launch_s * 1e6, "launches_per_step": per_step_launches}
        meth = oracle.method(kind=oracle.AHP, crit=(oracle.CRIT_CPU, oracle.CRIT_RAM, oracle.CRIT_UPLINK,
                                                   oracle.CRIT_PATHBW, oracle.CRIT_HOPS), cost=[0, 0, 0, 0, 1])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(insts, reqs, args.cpu_budget, meth)
        out["cpu_baseline"]["vs_gpu"] = value / out["cpu_baseline"]["value"]
    s.close()
    return out


# VALU instructions per Saaty pair evaluation in the pairwise AHP passes,
# counted in the compiled inner loops (18.75 in k_ahp_colsum, 18.1 in
# k_ahp_rowsum), and per compare in the rank pass of the sorted form (33 per
# 16 values), which the 1-9 scale takes up to AHP_SORT_MAX servers.
AHP_PAIR_OPS = 18.4
AHP_RANK_OPS = 33 / 16
AHP_SORT_MAX = 8192


TILE_T, TILE_C, TILE_N = 32768, 4, 1024

# HBM traffic of the scoring kernel per launch at the shape above, from two
# rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
# `bench.py --workload tiles --copy-ref`, each scaled by what the same
# counter reads for the run's plain 512 MiB device copy.  Valid only for the
# kernel sources the counters were taken on (their SHA-256 below); reported
# as null once those sources change.
TILE_TRAFFIC = {
    "sources": ("paper_1909_07673_amd/csrc/dc_tiles.hpp", "paper_1909_07673_amd/csrc/dc_step.hpp"),
    "sha256": "fe44d0a139b0563055380f40dd70c609f189bdd011f6626bfd62dd65cebe8c27",
    "fetch_kib": 262216.77, "fetch_copy_kib": 262161.44,     # copy reads 524288 KiB
    "write_kib": 517.37, "write_copy_kib": 524288.0,         # copy writes 524288 KiB
}


def tile_traffic():
    """Scaled HBM bytes per launch of the scoring kernel, or None when its
    sources differ from those the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in TILE_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TILE_TRAFFIC["sha256"]:
        return None
    t = TILE_TRAFFIC
    fetch = t["fetch_kib"] * (524288.0 / t["fetch_copy_kib"])
    write = t["write_kib"] * (524288.0 / t["write_copy_kib"])
    return (fetch + write) * 1024.0


def tile_timing(steps, warmup, copy_ref=False):
    """Times dc_topsis_tiles over TILE_T resident matrices: returns (host
    matrices, average launch seconds from HIP events on the launch stream,
    wall seconds of the timed launches, roofline dict)."""
    import torch
    import paper_1909_07673_amd as dc
    from workloads import make_tiles

    T, C, N = TILE_T, TILE_C, TILE_N
    xh, _ = make_tiles(seed=2024, T=T, N=N, C=C)
    x = torch.from_numpy(xh).cuda()
    w = [1.0 / C] * C
    stream = torch.cuda.current_stream()
    for _ in range(max(warmup, 1)):
        dc.topsis_tiles(x, w, stream=stream)
    torch.cuda.synchronize()
    if copy_ref:
        # a plain device copy of the same bytes, for scaling HBM counters
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del y
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        dc.topsis_tiles(x, w, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_s = e0.elapsed_time(e1) / 1e3 / steps
    bytes_per_launch = 4 * C * N * T + 8 * T          # criteria read once, best + score written
    achieved = bytes_per_launch / launch_s / 1e9
    roof = {"bound": "hbm", "kernel": "k_topsis_tiles_wave<4,4>", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": tile_traffic(),
            "avg_launch_us": launch_s * 1e6, "bytes_per_launch": bytes_per_launch}
    del x
    return xh, launch_s, wall, roof


def run_tiles(args, wl):
    """Kernel roofline of TOPSIS scoring: one launch scores every server of
    every matrix and selects the best; the matrices are resident in HBM and
    larger than the 256 MiB last-level cache, so each launch streams them."""
    import numpy as np
    import torch

    torch.cuda.set_device(0)
    T, C, N = TILE_T, TILE_C, TILE_N
    w = [1.0 / C] * C
    xh, launch_s, wall, roof = tile_timing(args.steps, args.warmup, args.copy_ref)
    hs = T * N
    out = {
        "metric": METRIC, "value": hs * args.steps / wall, "unit": "host-scores/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["text"], "matrices": T, "criteria": C, "hosts": N, "form": "tiles",
                   "method": "topsis"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        done = 0
        while time.perf_counter() - t1 < args.cpu_budget and done < T:
            oracle.topsis(xh[done].astype(np.float64), w)
            done += 1
        el = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": done * N / el, "unit": "host-scores/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {done} of the {T} matrices, FP64 oracle TOPSIS, one thread",
                               "host": host_cpu()}
        out["cpu_baseline"]["vs_gpu"] = out["value"] / out["cpu_baseline"]["value"]
    return out


# Table V of the paper (TOPSIS / AHP, Flat weights): runtime for the whole
# 6000-request workload on its (unnamed) GPU, and simulation events needed.
PAPER_TABLE5 = {"topsis": {"runtime_s": 3.67, "events": 894, "U_ij": 1.0, "U_i": 0.9885},
                "ahp": {"runtime_s": 9.45, "events": 949, "U_ij": 1.0, "U_i": 0.9822}}


def run_events(args, wl):
    """Discrete-event replay: at every event the departures due release
    their resources, the arrivals join the waiting queue, and every waiting
    request is submitted in FCFS order; the ones that do not fit wait for
    the next event.  Reports the events needed to place every request, the
    provisioning delay, the server / link fragmentation (share of active
    servers and of links carrying traffic) averaged over the events, and the
    mean utilities U(i), U(ij) (Eqs. (1)-(2)) of what the requests were
    given, read after the timed replay."""
    import numpy as np
    import torch
    import paper_1909_07673_amd as dc
    from workloads import make_event_workload

    torch.cuda.set_device(0)
    inst, reqs, arrive, dur = make_event_workload(seed=0)
    N = inst.n_hosts
    kw = dict(method=dc.DC_AHP) if wl["method"] == "ahp" else {}
    s = dc.Scheduler([inst], **kw)
    cap_links = np.array([inst.bw_host_edge, inst.bw_edge_agg, inst.bw_agg_core], np.int64)[:, None]
    buf = np.zeros(len(reqs), dc.RESULT_DTYPE)
    placed = np.full(len(reqs), -1)
    acc_id = np.full(len(reqs), -1, np.int64)
    queue, ends = [], {}
    nxt = ev = steps = tries = 0
    frag_s, frag_l = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while nxt < len(reqs) or queue:
        for rid in ends.pop(ev, []):
            s.release(rid)
        while nxt < len(reqs) and arrive[nxt] <= ev:
            queue.append(nxt)
            nxt += 1
        if queue:
            ids = [s.submit(reqs[q]) for q in queue]
            res = s.schedule_array(buf[:len(queue)])
            tries += len(queue)
            still = []
            for q, rid, r in zip(queue, ids, res):
                steps += _pod_steps(reqs[q], int(r["status"]), int(r["failed_at"]))
                if r["status"] == 1:
                    placed[q] = ev
                    acc_id[q] = rid
                    ends.setdefault(ev + int(dur[q]), []).append(rid)
                else:
                    still.append(q)
            queue = still
        st = s.state(0).astype(np.int64)
        frag_s.append(float((st[2] > 0).mean()))
        frag_l.append(float((st[3:] < cap_links).mean()))
        ev += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    delay = placed - arrive
    u_i, u_ij = [], []
    for q, req in enumerate(reqs):
        ca, ra, ba = s.alloc(int(acc_id[q]), req.n, req.m)
        cx = req.cpu if req.cpu_max is None else req.cpu_max
        rx = req.ram if req.ram_max is None else req.ram_max
        bx = req.edges[:, 2] if req.bw_max is None else req.bw_max
        u_i.extend(((ca / cx + ra / rx) / 2).tolist())
        u_ij.extend((ba / bx).tolist())
    s.close()
    out = {
        "metric": METRIC, "value": steps * N / wall, "unit": "host-scores/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["text"], "k": inst.k, "hosts": N, "requests": len(reqs), "form": "plain",
                   "method": wl["method"]},
        "events": int(placed.max()) + 1, "runtime_s": wall, "scoring_steps": steps, "submissions": tries,
        "delay_events": {"mean": float(delay.mean()), "p99": float(np.percentile(delay, 99)),
                         "max": int(delay.max())},
        "fragmentation": {"servers": float(np.mean(frag_s)), "links": float(np.mean(frag_l))},
        "utility": {"U_i": float(np.mean(u_i)), "U_ij": float(np.mean(u_ij)),
                    "note": "mean over containers / container pairs of allocated over maximum"},
        "paper_table5": dict(PAPER_TABLE5[wl["method"]], hardware="unnamed GPU, CUDA 10.1; runtime includes "
                                                                   "the paper's simulator"),
    }
    return out


def replay(s, dc, reqs, arr, dep, serving, horizon_s):
    """Replays a Poisson trace in real time: request t is submitted at
    arr[t] (or as soon as admitted), departs at dep[t] if it was accepted.
    Returns per-request (status, steps, sojourn seconds) and the wall time."""
    import heapq
    n = len(reqs)
    ids = [None] * n
    done = {}
    arrival = {}
    sojourn = {}
    events = [(arr[t], 0, t) for t in range(n)]
    heapq.heapify(events)
    backlog = []            # arrivals waiting for admission (FCFS)
    t0 = time.perf_counter()
    id2t = {}

    def absorb(results):
        now = time.perf_counter() - t0
        for r in results:
            t = id2t[r.req_id]
            done[t] = r
            sojourn[t] = now - arr[t]
            if r.status == 1 and dep[t] < horizon_s:
                heapq.heappush(events, (dep[t], 1, t))

    while events or backlog or len(done) < n:
        now = time.perf_counter() - t0
        while events and events[0][0] <= now:
            when, kind, t = heapq.heappop(events)
            if kind == 0:
                backlog.append(t)
            elif s.release(ids[t]) not in (dc.DC_OK,):
                heapq.heappush(events, (now + 1e-4, 1, t))
        # the plain form takes the whole backlog in one blocking schedule
        # call; the serving form admits what fits and keeps polling
        while backlog:
            t = backlog[0]
            rid = s.try_submit(reqs[t]) if serving else s.submit(reqs[t])
            if rid is None:
                break
            ids[t] = rid
            id2t[rid] = t
            backlog.pop(0)
        absorb(s.schedule())
        if not events and not backlog and len(done) == n:
            break
        if not backlog and (not events or events[0][0] > now + 2e-4):
            time.sleep(5e-5)
    wall = time.perf_counter() - t0
    return done, sojourn, wall


def run_serving(args, wl):
    import numpy as np
    import torch
    import paper_1909_07673_amd as dc
    from workloads import make_config, make_trace

    torch.cuda.set_device(0)
    insts, _ = make_config("serving", seed=0, n_req=1)
    N = insts[0].n_hosts
    reqs, arr, dep = make_trace(seed=0, duration_s=args.trace_s)
    forms = {}
    # serving: the cooperative persistent kernel (the default at this size);
    # plain: one launch per container step on one workgroup (the default);
    # the other two variants for comparison
    variants = (("serving", dc.DC_MODE_SERVING, 0), ("plain", dc.DC_MODE_PLAIN, 0),
                ("serving_1wg", dc.DC_MODE_SERVING, 1), ("plain_grid", dc.DC_MODE_PLAIN, 2))
    for name, mode, grid in variants:
        s = dc.Scheduler(insts, mode=mode, grid=grid)
        done, soj, wall = replay(s, dc, reqs, arr, dep, mode == dc.DC_MODE_SERVING, args.trace_s)
        if mode == dc.DC_MODE_SERVING:
            s.drain()
        steps = step_count(done.values())
        lat = s.latency_us()
        forms[name] = {
            "host_scores_per_s": steps * N / wall, "wall_s": wall, "container_steps": steps,
            "accepted": int(sum(r.status for r in done.values())), "requests": len(reqs),
            "achieved_req_per_s": len(reqs) / wall, "offered_req_per_s": len(reqs) / args.trace_s,
            "service_us": percentiles(lat), "sojourn_ms": percentiles(np.array(list(soj.values())) * 1e3),
        }
        s.close()
    sv = forms["serving"]
    return {
        "metric": METRIC, "value": sv["host_scores_per_s"], "unit": "host-scores/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": sv["wall_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["text"], "k": 48, "hosts": N, "trace_s": args.trace_s,
                   "requests": len(reqs), "form": "serving", "method": "topsis"},
        "latency_us": dict(sv["service_us"], kind="service (admission to decision), device clock"),
        "forms": forms,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="plain", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--trace-s", type=float, default=2.0, help="serving: seconds of Poisson arrivals")
    ap.add_argument("--grid", type=int, default=0, choices=(0, 1, 2),
                    help="TOPSIS step: 0 automatic, 1 one workgroup, 2 one cooperative workgroup per pod")
    ap.add_argument("--block", type=int, default=0, choices=(0, 256, 512, 1024),
                    help="plain/batched TOPSIS: workgroup size (0 = autotuned)")
    ap.add_argument("--no-scoring-kernel", action="store_true",
                    help="plain/batched: skip the separate roofline of the scoring stage alone")
    ap.add_argument("--copy-ref", action="store_true",
                    help="tiles: also run one plain copy of the matrices (reference for HBM byte counters)")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1, 2),
                    help="batched form: 0 automatic (graph), 1 direct launch, 2 HIP graph")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the scheduler runs on one GPU only (asked for {args.gpus}); "
              "a data center's container steps are sequential and are not sharded across GPUs", file=sys.stderr)
        sys.exit(2)
    wl = WORKLOADS[args.workload]
    if wl["mode"] == "serving":
        out = run_serving(args, wl)
    elif wl["mode"] == "tiles":
        out = run_tiles(args, wl)
    elif wl["mode"] == "events":
        out = run_events(args, wl)
    else:
        out = run_batch(args, wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
