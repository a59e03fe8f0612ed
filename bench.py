#!/usr/bin/env python3
"""Throughput benchmark of the container-scheduling hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic requests:
the data-center state is rewound to its initial (background-loaded) state
and every request is scheduled in FCFS order -- per container: path stage,
criteria, scoring, selection, commit -- with the results copied back.  The
requests are uploaded to HBM before the timed region.

Default workload: k=16 fat-tree (1024 hosts), 40 Gbps host links, 100 Gbps
edge-aggregation / aggregation-core links, 0-70 % background load, 2,000
FCFS requests of 2-32 containers, TOPSIS over (CPU, RAM, active, path
bandwidth), plain form: one kernel launch per container step.

Prints one JSON line.
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

WORKLOADS = {
    "plain": dict(preset="plain", mode="plain", method="topsis",
                  text="k=16 fat-tree (1024 hosts), 2000 FCFS requests of 2-32 containers, 0-70% background, "
                       "TOPSIS on CPU/RAM/active/path-bw, plain form (one launch per container step)"),
    "batched": dict(preset="batched", mode="batched", method="topsis",
                    text="256 independent k=16 fat-trees (1024 hosts each), 64-512 requests of 2-48 containers "
                         "per instance, TOPSIS, batched form (one persistent launch)"),
}


def host_scores(results, N):
    steps = 0
    for r in results:
        steps += r.n if r.status == 1 else r.failed_at + 1
    return steps, steps * N


def cpu_baseline(insts, reqs, budget_s):
    """The FP64 oracle, as it stands, on a bounded prefix of the same
    workload (single thread)."""
    import oracle
    steps = 0
    t0 = time.perf_counter()
    n_req = 0
    o = oracle.Oracle(insts[0], oracle.method(kind=oracle.TOPSIS))
    for req in reqs[0]:
        res = o.run_request(req)
        steps += req.n if res["status"] == 1 else res["failed_at"] + 1
        n_req += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    N = insts[0].k ** 3 // 4
    return dict(value=steps * N / dt, unit="host-scores/s", cores=1, kind="oracle",
                sample=f"first {n_req} requests ({steps} container steps) of the same workload on one host "
                       f"thread, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="plain", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "a data center's container steps are sequential and are not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1909_07673_amd as dc
    from workloads import make_config

    wl = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    insts, reqs = make_config(wl["preset"], seed=0)
    N = insts[0].n_hosts
    mode = dc.DC_MODE_BATCHED if wl["mode"] == "batched" else dc.DC_MODE_PLAIN
    s = dc.Scheduler(insts, mode=mode, stream=stream)
    for i, rl in enumerate(reqs):
        for r in rl:
            s.submit(r, instance=i)
    s.rewind()                      # uploads the requests; they stay resident in HBM
    tuned = s.autotune()            # workgroup size picked by timing the candidates
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        s.rewind()
        s.schedule()
    torch.cuda.synchronize()
    kern_ms = 0.0
    launches = 0
    results = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.rewind()
        results = s.schedule()
        ms, la, _ = s.last_timing()
        kern_ms += ms
        launches += la
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    steps, hs = host_scores(results, N)
    value = hs * args.steps / wall
    lat = s.latency_us()
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    bytes_per_launch = BYTES_PER_HOST_SCORE * hs / max(launches // args.steps, 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9
    kname = "k_topsis_batched" if mode == dc.DC_MODE_BATCHED else "k_topsis_plain"
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "host-scores/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["text"], "k": insts[0].k, "hosts": N, "instances": len(insts),
                   "requests": sum(len(r) for r in reqs), "container_steps": steps,
                   "form": wl["mode"], "method": wl["method"], "block": tuned},
        "latency_us": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "kind": "service (first step start to decision), device clock"},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_us": avg_launch_s * 1e6, "launches_per_step": launches // args.steps,
                     "bytes_per_launch": bytes_per_launch},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(insts, reqs, args.cpu_budget)
        out["cpu_baseline"]["vs_gpu"] = value / out["cpu_baseline"]["value"]
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
