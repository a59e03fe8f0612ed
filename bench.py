#!/usr/bin/env python3
"""Throughput benchmark of the container-scheduling hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic requests:
the data-center state is rewound to its initial (background-loaded) state
and every request is scheduled in FCFS order -- per container: path stage,
criteria, scoring, selection, commit -- with the results copied back.  The
requests are uploaded to HBM before the timed region.

Default workload (one JSON line): 256 independent k=16 fat-trees (1,024
hosts each, 40 Gbps host links, 100 Gbps edge-aggregation /
aggregation-core links, 0-70 % background load), each with 64-512 FCFS
requests of 2-48 containers, TOPSIS over (CPU, RAM, active, path
bandwidth), batched form: one persistent launch per step, replayed from a
HIP graph, with the autotuned launch shape.  The line also carries the
plain form on one k=16 data center (one launch per container step), the
serving form against the plain form on a k=48 Poisson trace, and the
scoring stage alone over resident matrices.  Other workloads (--workload)
measure the plain form, the large AHP case, the serving form and the
paper's event-replay shape on their own.
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
# VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13
# lane-instructions per second without packing.  The AHP passes are compares,
# selects and integer adds, which do not pack; the published FP32 peak, 157.3
# TFLOP/s, counts two lanes per packed instruction and two FLOPs per FMA, so
# it is four times this rate in FLOPs (twice it in lane-instructions).
VALU_LANE_OPS = 256 * 64 * 2.4e9
VALU_LANE_OPS_PACKED = 157.3e12 / 2

WORKLOADS = {
    "plain": dict(preset="plain", mode="plain", method="topsis",
                  text="k=16 fat-tree (1024 hosts), 2000 FCFS requests of 2-32 containers, 0-70% background, "
                       "TOPSIS on CPU/RAM/active/path-bw, plain form (one launch per container step)"),
    "batched": dict(preset="batched", mode="batched", method="topsis",
                    text="256 independent k=16 fat-trees (1024 hosts each), 64-512 requests of 2-48 containers "
                         "per instance, TOPSIS, batched form (one persistent launch)"),
    "ahp": dict(preset="ahp", mode="plain", method="ahp",
                text="k=32 fat-tree (8192 hosts), 500 FCFS requests of 8-64 containers, 0-70% background, AHP "
                     "(Saaty 1-9) on CPU/RAM/uplink/path-bw/hops(cost), seven launches per container step "
                     "(criteria, run sort, run merge, column sums, row sums, global priority, select)"),
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
    from paper_1909_07673_amd.events import unit_steps
    return unit_steps(req, status, failed_at)


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


def _oracle_prefix(insts, reqs, meth, budget_s, which):
    """Runs the FP64 oracle, as it stands, over instances `which` in order
    (each instance's requests in FCFS order) until budget_s seconds have
    passed.  Returns (scoring steps, requests, instances touched)."""
    import oracle
    steps = n_req = n_inst = 0
    t0 = time.perf_counter()
    for i in which:
        o = oracle.Oracle(insts[i], meth)
        n_inst += 1
        for req in reqs[i]:
            res = o.run_request(req)
            steps += _pod_steps(req, res["status"], res["failed_at"])
            n_req += 1
            if time.perf_counter() - t0 > budget_s:
                break
        o.close()
        if time.perf_counter() - t0 > budget_s:
            break
    return steps, n_req, n_inst


_POOL_ARGS = None


def _pool_worker(w):
    insts, reqs, meth, budget_s, nw = _POOL_ARGS
    return _oracle_prefix(insts, reqs, meth, budget_s, range(w, len(insts), nw))


def cpu_baseline(insts, reqs, budget_s, meth, all_cores=False):
    """The FP64 oracle timed on this host: one thread on a prefix of the
    workload (instance 0 first), and with all_cores, one process per
    logical CPU this process may use, worker w taking instances w, w + W, ...
    (independent data centers, the fair CPU counterpart of the batched
    form).  Must run before this process touches the GPU: the workers are
    forked."""
    import oracle
    oracle.set_threads(1)
    N = insts[0].n_hosts
    t0 = time.perf_counter()
    steps, n_req, n_inst = _oracle_prefix(insts, reqs, meth, budget_s, range(len(insts)))
    dt = time.perf_counter() - t0
    where = "the same workload" if n_inst == 1 else f"the first {n_inst} instance(s) of the same workload"
    one = dict(value=steps * N / dt, unit="host-scores/s", cores=1, kind="oracle",
               sample=f"first {n_req} requests ({steps} scoring steps) of {where} on one host thread, {dt:.1f} s",
               host=host_cpu())
    if not all_cores or len(insts) < 2:
        return one
    import multiprocessing as mp
    global _POOL_ARGS
    nw = min(len(os.sched_getaffinity(0)), len(insts))
    _POOL_ARGS = (insts, reqs, meth, budget_s, nw)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(nw) as pool:
        parts = pool.map(_pool_worker, range(nw))
    dt = time.perf_counter() - t0
    _POOL_ARGS = None
    steps = sum(p[0] for p in parts)
    out = dict(value=steps * N / dt, unit="host-scores/s", cores=nw, kind="oracle",
               sample=f"{nw} processes, one per logical CPU, each running the oracle over its share of the "
                      f"{len(insts)} instances (instance w, w + {nw}, ...) in FCFS order for {budget_s:.0f} s: "
                      f"{sum(p[1] for p in parts)} requests, {steps} scoring steps in {dt:.1f} s",
               host=host_cpu(), one_thread=one)
    return out


def percentiles(x):
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99))} if x.size else None


def run_batch(args, wl, insts, reqs):
    """Plain / batched / AHP: rewind + schedule all requests per step."""
    import numpy as np
    import torch
    import paper_1909_07673_amd as dc

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
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
    # the batched form takes its launch shape from the autotuner (through its
    # cache, so a profiled run times the same kernel as an unprofiled one);
    # the plain form keeps the library's workgroup size for its server count
    # (1,024 threads from 257 servers on, which the autotuner also picks)
    tune = None
    if mode == dc.DC_MODE_BATCHED and not args.block:
        tune = s.autotune_cached(args.tune_cache or None)
    shape = s.shape()
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
                   "form": wl["mode"], "method": wl["method"], "shape": shape, "grid": args.grid,
                   "graph": args.graph,
                   "steps_per_instance": {"mean": float(per_inst.mean()), "max": int(per_inst.max())}},
        "latency_us": dict(percentiles(lat), kind="service (first step start to decision), device clock"),
    }
    if tune is not None:
        out["config"]["autotune"] = tune
    if wl["method"] == "topsis":
        kname = ("k_topsis_batched" if mode == dc.DC_MODE_BATCHED else
                 "k_topsis_grid" if args.grid == 2 else "k_topsis_plain")
        bytes_per_launch = BYTES_PER_HOST_SCORE * hs / per_step_launches
        achieved = bytes_per_launch / avg_launch_s / 1e9
        traffic = counter_traffic(BATCHED_TRAFFIC, shape) if kname == "k_topsis_batched" else None
        out["roofline"] = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "avg_launch_us": avg_launch_s * 1e6, "launches_per_step": per_step_launches,
                           "bytes_per_launch": bytes_per_launch,
                           "bytes_basis": "24 B per host-score: the six int32 state words of each scored server"}
    else:
        C = 5
        # the column and row sums take 2*C*N^2 Saaty evaluations per
        # container step by definition; the pairwise passes make them all,
        # at AHP_PAIR_OPS VALU lane-instructions each, so their ceiling is
        # the VALU lane rate / AHP_PAIR_OPS.  The sorted passes (the 1-9
        # scale up to AHP_SORT_MAX servers) reach the same sums in
        # O(C N log N) work: their rate is the equivalent evaluations per
        # second, which can exceed that ceiling (frac > 1).  Either rate is
        # taken over the whole step's kernel time.
        pairs, ops = 2.0 * C * N * N * steps, AHP_PAIR_OPS
        if N <= AHP_SORT_MAX:
            kname, unit = "AHP step, sorted passes", "pair-evals/s (equivalent)"
        else:
            kname, unit = "k_ahp_colsum+k_ahp_rowsum", "pair-evals/s"
        rate = pairs * args.steps / (kern_ms / 1e3)
        out["roofline"] = {"bound": "alu", "kernel": kname, "unit": unit, "achieved": rate,
                           "peak": VALU_LANE_OPS / ops, "frac": rate / (VALU_LANE_OPS / ops),
                           "frac_of_packed_fp32_peak": rate / (VALU_LANE_OPS_PACKED / ops),
                           "traffic": None, "pair_ops": ops, "basis": "whole AHP step kernel time",
                           "peak_basis": "256 CUs x 64 lanes x 2.4 GHz VALU lane-instructions/s (no packing)",
                           "avg_launch_us": avg_launch_s * 1e6, "launches_per_step": per_step_launches}
    s.close()
    return out


def oracle_method(wl):
    import oracle
    if wl["method"] == "ahp":
        return oracle.method(kind=oracle.AHP, crit=(oracle.CRIT_CPU, oracle.CRIT_RAM, oracle.CRIT_UPLINK,
                                                   oracle.CRIT_PATHBW, oracle.CRIT_HOPS), cost=[0, 0, 0, 0, 1])
    return oracle.method(kind=oracle.TOPSIS, route_end=bool(wl.get("routing", 0)))


# VALU instructions per Saaty pair evaluation in the pairwise AHP passes,
# counted in the compiled inner loops (18.75 in k_ahp_colsum, 18.1 in
# k_ahp_rowsum); the 1-9 scale takes the sorted passes up to AHP_SORT_MAX
# servers.
AHP_PAIR_OPS = 18.4
AHP_SORT_MAX = 8192


TILE_T, TILE_C, TILE_N = 32768, 4, 1024

# HBM traffic per launch from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads
# for the run's plain device copy of copy_kib KiB (which reads and writes
# copy_kib).  Valid only for the kernel sources the counters were taken on
# (their SHA-256); reported as null otherwise.
TILE_TRAFFIC = {
    "sources": ('paper_1909_07673_amd/csrc/dc_tiles.hpp', 'paper_1909_07673_amd/csrc/dc_step.hpp'),
    "sha256": "08556909eae8570b3b7579798445f363612b5a483a503d8710709e86ecb2d892",
    "copy_kib": 524288.0,
    "fetch_kib": 262212.31, "fetch_copy_kib": 262162.13,
    "write_kib": 517.64, "write_copy_kib": 524288.0,
}
# the batched kernel at the default workload (taken with
# `bench.py --workload batched --no-extras --no-cpu-baseline --steps 1
# --warmup 0 --copy-ref`, one pass per counter); its HBM traffic is the
# staging of each instance's state and the requests and results, which the
# launch shape (workgroup size, servers per thread, peer chunk) does not change
BATCHED_TRAFFIC = {
    "sources": ('paper_1909_07673_amd/csrc/dc_kernels.hpp', 'paper_1909_07673_amd/csrc/dc_step.hpp'),
    "sha256": "ca7aa44e0890ffe041a6034f91d4e5c7c362a0e19566e8175c74f09c93c173b4",
    "copy_kib": 524288.0,
    "fetch_kib": 119050.13, "fetch_copy_kib": 262161.5,
    "write_kib": 39380.88, "write_copy_kib": 524288.0,
}


def _sources_sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(t, shape=None):
    """Scaled HBM bytes per launch from the counters in t, or None when the
    sources (or the launch shape) differ from those they were taken on."""
    if t is None or _sources_sha(t["sources"]) != t["sha256"]:
        return None
    if shape is not None and t.get("shape") not in (None, shape):
        return None
    fetch = t["fetch_kib"] * (t["copy_kib"] / t["fetch_copy_kib"])
    write = t["write_kib"] * (t["copy_kib"] / t["write_copy_kib"])
    return (fetch + write) * 1024.0


def tile_traffic():
    return counter_traffic(TILE_TRAFFIC)


def copy_reference(nbytes=512 << 20):
    """One plain device-to-device copy of nbytes (a reference of known size
    for scaling HBM byte counters)."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y


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
        copy_reference(x.numel() * 4)
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
    """Discrete-event replay (paper_1909_07673_amd.events): at every event
    the departures due release their resources, the arrivals join the
    waiting queue, and every waiting request is submitted in FCFS order;
    the ones that do not fit wait for the next event.  Reports the events
    needed to place every request, the provisioning delay, the server / link
    fragmentation F(N^s), F(E^s) averaged over the events, and the mean
    utilities U(i), U(ij) (section II-B, Eqs. (1)-(2)) of what the requests
    were given, read after the timed replay."""
    import numpy as np
    import torch
    import paper_1909_07673_amd as dc
    from paper_1909_07673_amd import events
    from workloads import make_event_workload

    torch.cuda.set_device(0)
    inst, reqs, arrive, dur = make_event_workload(seed=0)
    N = inst.n_hosts
    kw = dict(method=dc.DC_AHP) if wl["method"] == "ahp" else {}
    s = dc.Scheduler([inst], **kw)
    caps = (inst.bw_host_edge, inst.bw_edge_agg, inst.bw_agg_core)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = events.replay(s, reqs, arrive, dur, caps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    u_i, u_ij = [], []
    for q, req in enumerate(reqs):
        ui, uij = events.utilities(req, *s.alloc(int(rep["rid"][q]), req.n, req.m))
        u_i.extend(ui.tolist())
        u_ij.extend(uij.tolist())
    s.close()
    delay = rep["delay"]
    out = {
        "metric": METRIC, "value": rep["steps"] * N / wall, "unit": "host-scores/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["text"], "k": inst.k, "hosts": N, "requests": len(reqs), "form": "plain",
                   "method": wl["method"]},
        "events": rep["events"], "runtime_s": wall, "scoring_steps": rep["steps"],
        "submissions": rep["submissions"],
        "delay_events": {"mean": float(delay.mean()), "p99": float(np.percentile(delay, 99)),
                         "max": int(delay.max())},
        "fragmentation": {"servers": float(np.mean(rep["frag_s"])), "links": float(np.mean(rep["frag_l"]))},
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


def run_serving(args, wl, variants_all=True):
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
    if not variants_all:
        variants = variants[:2]
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


def summary(out):
    """The keys of a workload's line that go into another line as an extra."""
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "config", "latency_us", "roofline")
    return {k: out[k] for k in keep if k in out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle work per cpu_baseline leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="batched: only the batched form (no plain, serving or scoring-stage extras)")
    ap.add_argument("--trace-s", type=float, default=2.0, help="serving: seconds of Poisson arrivals")
    ap.add_argument("--grid", type=int, default=0, choices=(0, 1, 2),
                    help="TOPSIS step: 0 automatic, 1 one workgroup, 2 one cooperative workgroup per pod")
    ap.add_argument("--block", type=int, default=0, choices=(0, 256, 512, 1024),
                    help="plain/batched TOPSIS: workgroup size (0 = library default / autotuned)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1909_07673_amd", "tune_cache.jsonl"),
                    help="batched: autotuner cache file ('' = tune every run)")
    ap.add_argument("--no-scoring-kernel", action="store_true",
                    help="plain/batched: skip the separate roofline of the scoring stage alone")
    ap.add_argument("--copy-ref", action="store_true",
                    help="tiles, batched: also run one plain device copy (reference for HBM byte counters)")
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
        from workloads import make_config
        insts, reqs = make_config(wl["preset"], seed=0)
        cpu = None
        if not args.no_cpu_baseline:
            # before the GPU is touched: the all-cores leg forks its workers
            cpu = cpu_baseline(insts, reqs, args.cpu_budget, oracle_method(wl), all_cores=wl["mode"] == "batched")
        out = run_batch(args, wl, insts, reqs)
        if cpu is not None:
            cpu["vs_gpu"] = out["value"] / cpu["value"]
            if "one_thread" in cpu:
                cpu["one_thread"]["vs_gpu"] = out["value"] / cpu["one_thread"]["value"]
            out["cpu_baseline"] = cpu
        if args.copy_ref:
            copy_reference()
        if args.workload == "batched" and not args.no_extras:
            # the plain per-container-launch path on one k=16 data center
            # (2,000 requests), the serving form against the plain form on
            # the k=48 Poisson trace, and the scoring stage alone
            pa = argparse.Namespace(**vars(args))
            pa.steps, pa.warmup, pa.block = 3, 1, 0
            pi, pr = make_config("plain", seed=0)
            plain = summary(run_batch(pa, WORKLOADS["plain"], pi, pr))
            out["plain_form"] = plain
            out["batched_vs_plain"] = {
                "host_scores_per_s": out["value"] / plain["value"],
                "p99_service_us": {"batched": out["latency_us"]["p99"], "plain": plain["latency_us"]["p99"]}}
            sv = run_serving(args, WORKLOADS["serving"], variants_all=False)
            out["serving_vs_plain_k48"] = {"config": sv["config"], "forms": sv["forms"]}
            if not args.no_scoring_kernel:
                out["scoring_kernel_roofline"] = dict(tile_timing(20, 2)[3], workload=WORKLOADS["tiles"]["text"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
