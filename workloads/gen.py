"""Seeded generators: fat-tree instances, tenant requests and serving traces.

Random streams are numpy PCG64 generators spawned from one SeedSequence per
configuration, so instance i of a batch always sees the same numbers no
matter how many instances are drawn.  Units are integers throughout:
CPU in cores, RAM in GB, bandwidth in Mbps.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class FatTree:
    """Sizes of a k-ary fat-tree (k even): k^3/4 hosts, k^2/2 edge and
    aggregation switches, k^2/4 core switches, and k^3/4 links per level."""
    k: int

    def __post_init__(self):
        if self.k < 2 or self.k % 2:
            raise ValueError("fat-tree arity k must be even and >= 2")

    @property
    def half(self) -> int:
        return self.k // 2

    @property
    def n_hosts(self) -> int:
        return self.k ** 3 // 4

    @property
    def n_edge(self) -> int:
        return self.k * self.k // 2

    @property
    def n_agg(self) -> int:
        return self.k * self.k // 2

    @property
    def n_core(self) -> int:
        return self.k * self.k // 4

    @property
    def n_links(self) -> int:
        return 3 * self.n_hosts


@dataclasses.dataclass
class Instance:
    """One data center: capacities plus background load already consumed."""
    k: int
    host_cpu: int
    host_ram: int
    bw_host_edge: int
    bw_edge_agg: int
    bw_agg_core: int
    host_used: Optional[np.ndarray] = None   # int32 [2][N]
    link_used: Optional[np.ndarray] = None   # int32 [3][N]

    @property
    def tree(self) -> FatTree:
        return FatTree(self.k)

    @property
    def n_hosts(self) -> int:
        return self.tree.n_hosts


@dataclasses.dataclass
class Request:
    """A tenant request: n containers with CPU/RAM demands, undirected
    communication edges (i, j, bw) with i < j, and optionally the pod of
    each container (pod[i] >= 0: its pod id; -1: no pod).  With demand
    intervals (section II-A) cpu, ram and the edges' bw are the minima and
    cpu_max, ram_max, bw_max (per edge) the maxima; None means max = min."""
    cpu: np.ndarray     # int32 [n]
    ram: np.ndarray     # int32 [n]
    edges: np.ndarray   # int32 [m][3]
    pod: Optional[np.ndarray] = None   # int32 [n] or None
    cpu_max: Optional[np.ndarray] = None   # int32 [n] or None
    ram_max: Optional[np.ndarray] = None   # int32 [n] or None
    bw_max: Optional[np.ndarray] = None    # int32 [m] or None

    @property
    def n(self) -> int:
        return int(self.cpu.shape[0])

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])


def _rng(seed_seq: np.random.SeedSequence) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_seq))


def make_instance(k: int, host_cpu: int, host_ram: int, bw_host_edge: int,
                  bw_edge_agg: int, bw_agg_core: int,
                  background: float = 0.0,
                  rng: Optional[np.random.Generator] = None) -> Instance:
    """Fat-tree with homogeneous hosts and per-level link capacities.

    With background > 0 every host resource and every link independently
    has floor(U[0, background) * capacity) already in use."""
    inst = Instance(k, host_cpu, host_ram, bw_host_edge, bw_edge_agg, bw_agg_core)
    if background > 0.0:
        assert rng is not None
        n = inst.n_hosts
        hu = np.empty((2, n), dtype=np.int32)
        hu[0] = np.floor(rng.uniform(0.0, background, n) * host_cpu).astype(np.int32)
        hu[1] = np.floor(rng.uniform(0.0, background, n) * host_ram).astype(np.int32)
        lu = np.empty((3, n), dtype=np.int32)
        for lvl, cap in enumerate((bw_host_edge, bw_edge_agg, bw_agg_core)):
            lu[lvl] = np.floor(rng.uniform(0.0, background, n) * cap).astype(np.int32)
        inst.host_used, inst.link_used = hu, lu
    return inst


def _random_connected_edges(n: int, density: float, rng: np.random.Generator,
                            bw_lo: int, bw_hi: int) -> np.ndarray:
    """Random connected graph: a random spanning tree (node t joins a uniform
    earlier node) plus uniformly drawn extra pairs up to
    max(n-1, ceil(density * n(n-1)/2)) edges; bandwidth uniform in
    [bw_lo, bw_hi]."""
    if n < 2:
        return np.zeros((0, 3), dtype=np.int32)
    target = max(n - 1, int(math.ceil(density * n * (n - 1) / 2)))
    parent = rng.integers(0, np.arange(1, n)).astype(np.int64)   # node t joins a uniform earlier node
    pi, pj = parent, np.arange(1, n, dtype=np.int64)
    if target > n - 1:
        # the pairs (i < j) not in the tree, in row-major order
        iu, ju = np.triu_indices(n, 1)
        in_tree = np.zeros((n, n), dtype=bool)
        in_tree[pi, pj] = True
        keep = ~in_tree[iu, ju]
        ri, rj = iu[keep], ju[keep]
        pick = np.sort(rng.choice(ri.shape[0], size=target - (n - 1), replace=False))
        pi, pj = np.concatenate([pi, ri[pick]]), np.concatenate([pj, rj[pick]])
    bw = rng.integers(bw_lo, bw_hi + 1, size=pi.shape[0])
    return np.stack([pi, pj, bw], axis=1).astype(np.int32)


def _random_pods(n: int, frac: float, rng: np.random.Generator) -> np.ndarray:
    """Up to floor(frac * n) containers (a uniform count, uniform choice)
    grouped into pods of 2-4 containers; the others get no pod (-1)."""
    pod = np.full(n, -1, dtype=np.int32)
    g = int(rng.integers(0, int(frac * n) + 1))
    if g < 2:
        return pod
    members = rng.permutation(n)[:g]
    pid, at = 0, 0
    while at < g:
        size = int(rng.integers(2, 5))
        if g - (at + size) == 1:        # no pod of one container
            size += 1
        pod[members[at:at + size]] = pid
        pid += 1
        at += size
    return pod


def make_requests(count: int, rng: np.random.Generator, n_lo: int, n_hi: int,
                  cpu_lo: int = 1, cpu_hi: int = 8, ram_lo: int = 1, ram_hi: int = 32,
                  bw_lo: int = 100, bw_hi: int = 2000, density: float = 0.5,
                  pod_frac: float = 0.0, ranges: Optional[str] = None) -> List[Request]:
    """ranges: None (fixed demands); "widen": the drawn demands are the
    minima and each maximum is min + U{0..min}; "lower": the drawn demands
    are the maxima and each minimum is U{1..max}."""
    reqs = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        cpu = rng.integers(cpu_lo, cpu_hi + 1, size=n).astype(np.int32)
        ram = rng.integers(ram_lo, ram_hi + 1, size=n).astype(np.int32)
        edges = _random_connected_edges(n, density, rng, bw_lo, bw_hi)
        pod = _random_pods(n, pod_frac, rng) if pod_frac > 0 else None
        req = Request(cpu, ram, edges, pod)
        if ranges == "widen":
            req.cpu_max = (cpu + rng.integers(0, cpu.astype(np.int64) + 1)).astype(np.int32)
            req.ram_max = (ram + rng.integers(0, ram.astype(np.int64) + 1)).astype(np.int32)
            bw = edges[:, 2].astype(np.int64)
            req.bw_max = (bw + rng.integers(0, bw + 1)).astype(np.int32)
        elif ranges == "lower":
            req.cpu_max, req.ram_max = cpu, ram
            req.cpu = rng.integers(1, cpu.astype(np.int64) + 1).astype(np.int32)
            req.ram = rng.integers(1, ram.astype(np.int64) + 1).astype(np.int32)
            req.bw_max = edges[:, 2].copy()
            req.edges = edges.copy()
            req.edges[:, 2] = rng.integers(1, edges[:, 2].astype(np.int64) + 1)
        elif ranges is not None:
            raise ValueError(f"unknown ranges mode {ranges!r}")
        reqs.append(req)
    return reqs


def pack_requests(reqs: Sequence[Request]):
    """Flatten requests into CSR arrays: container offsets, cpu, ram, edge
    offsets and edges [m][3]."""
    coff = np.zeros(len(reqs) + 1, dtype=np.int64)
    eoff = np.zeros(len(reqs) + 1, dtype=np.int64)
    for r, q in enumerate(reqs):
        coff[r + 1] = coff[r] + q.n
        eoff[r + 1] = eoff[r] + q.m
    cpu = np.concatenate([q.cpu for q in reqs]).astype(np.int32) if reqs else np.zeros(0, np.int32)
    ram = np.concatenate([q.ram for q in reqs]).astype(np.int32) if reqs else np.zeros(0, np.int32)
    edges = (np.concatenate([q.edges for q in reqs]).astype(np.int32)
             if reqs else np.zeros((0, 3), np.int32)).reshape(-1, 3)
    return coff, cpu, ram, eoff, edges


# --------------------------------------------------------------------------
# Workload presets.  Capacities: 32 cores / 256 GB per host.  The small
# case uses 10 Gbps everywhere and no background; the large ones use
# 40 Gbps host links, 100 Gbps edge-aggregation and aggregation-core links
# and a uniform 0-70 % background load on every host resource and link.
# --------------------------------------------------------------------------

CONFIGS = {
    "tiny":    dict(k=4,  caps=(32, 256, 10000, 10000, 10000), background=0.0,
                    n_req=(20, 20), n=(2, 6), instances=1),
    "plain":   dict(k=16, caps=(32, 256, 40000, 100000, 100000), background=0.7,
                    n_req=(2000, 2000), n=(2, 32), instances=1),
    "ahp":     dict(k=32, caps=(32, 256, 40000, 100000, 100000), background=0.7,
                    n_req=(500, 500), n=(8, 64), instances=1),
    "batched": dict(k=16, caps=(32, 256, 40000, 100000, 100000), background=0.7,
                    n_req=(64, 512), n=(2, 48), instances=256),
    "serving": dict(k=48, caps=(32, 256, 40000, 100000, 100000), background=0.7,
                    n_req=None, n=(2, 64), instances=1),
    # requests with pods: up to half of each request's containers grouped
    # into pods of 2-4 (the share the paper's second workload uses)
    "tiny_pods": dict(k=4, caps=(32, 256, 10000, 10000, 10000), background=0.0,
                      n_req=(20, 20), n=(2, 6), instances=1, pod_frac=0.5),
    "pods":    dict(k=16, caps=(32, 256, 40000, 100000, 100000), background=0.7,
                    n_req=(2000, 2000), n=(2, 32), instances=1, pod_frac=0.5),
    # demand intervals: each drawn demand is a minimum and its maximum is up
    # to twice it; 5 Gbps links at k = 4 so that paths, too, run short of
    # the maxima
    "tiny_ranges": dict(k=4, caps=(32, 256, 5000, 5000, 5000), background=0.0,
                        n_req=(20, 20), n=(2, 6), instances=1, ranges="widen"),
    "tiny_ranges_pods": dict(k=4, caps=(32, 256, 5000, 5000, 5000), background=0.0,
                             n_req=(20, 20), n=(2, 6), instances=1, pod_frac=0.5, ranges="widen"),
    "ranges":  dict(k=16, caps=(32, 256, 40000, 100000, 100000), background=0.7,
                    n_req=(2000, 2000), n=(2, 32), instances=1, pod_frac=0.5, ranges="widen"),
}


def make_config(name: str, seed: int = 0, instances: Optional[int] = None,
                n_req: Optional[int] = None, k: Optional[int] = None):
    """Return (instances, requests_per_instance) for a named preset.

    `instances`, `n_req` and `k` override the preset (smaller test cases of
    the same shape); instance i draws from SeedSequence(seed).spawn()[i]."""
    cfg = CONFIGS[name]
    n_inst = cfg["instances"] if instances is None else instances
    kk = cfg["k"] if k is None else k
    kids = np.random.SeedSequence(seed).spawn(n_inst)
    insts, reqs = [], []
    for i in range(n_inst):
        rng = _rng(kids[i])
        inst = make_instance(kk, *cfg["caps"], background=cfg["background"], rng=rng)
        if n_req is not None:
            cnt = n_req
        else:
            lo, hi = cfg["n_req"] if cfg["n_req"] else (100, 100)
            cnt = int(rng.integers(lo, hi + 1))
        reqs.append(make_requests(cnt, rng, *cfg["n"], pod_frac=cfg.get("pod_frac", 0.0),
                                  ranges=cfg.get("ranges")))
        insts.append(inst)
    return insts, reqs


def make_event_workload(seed: int, k: int = 20, n_req: int = 6000, n: int = 4, total_events: int = 500,
                        span: int = 250, ranges: Optional[str] = "lower", cpu_hi: int = 2, ram_hi: int = 4,
                        bw_hi: int = 50):
    """The shape of the paper's GPU evaluation (section VI-A): a k-ary
    fat-tree of 24-core / 256 GB servers with 1 Gbps links and no other
    load; n_req requests of n containers, up to half of them in pods, up to
    50 Mbps between a pair of containers, CPU up to 2 cores and RAM up to 4
    GB per container.  Each request arrives at a uniform event in
    [0, span) and runs for a uniform 1..span events of a total_events run.
    Demands are intervals by default (ranges="lower": those bounds are the
    maxima, the minima uniform below them).  cpu_hi, ram_hi, bw_hi: the
    upper bounds (heavier requests make requests wait on a small k).
    Returns (instance, requests, arrival events, durations)."""
    rng = _rng(np.random.SeedSequence([seed, 6]))
    inst = make_instance(k, 24, 256, 1000, 1000, 1000)
    reqs = make_requests(n_req, rng, n, n, cpu_lo=1, cpu_hi=cpu_hi, ram_lo=1, ram_hi=ram_hi, bw_lo=1, bw_hi=bw_hi,
                         pod_frac=0.5, ranges=ranges)
    arrive = np.sort(rng.integers(0, span, size=n_req))
    dur = rng.integers(1, span + 1, size=n_req)
    assert total_events >= 2 * span
    return inst, reqs, arrive, dur


def make_trace(seed: int, duration_s: float, rate_per_s: float = 5000.0,
               mean_life_s: float = 60.0, n_lo: int = 2, n_hi: int = 64):
    """Poisson arrivals (exponential inter-arrival, mean 1/rate) with
    exponential lifetimes on a simulated clock.  Returns (requests,
    arrival_times, departure_times); a departure after the end of the trace
    is reported as +inf."""
    rng = _rng(np.random.SeedSequence([seed, 5]))
    t, arr = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t >= duration_s:
            break
        arr.append(t)
    arr = np.asarray(arr)
    life = rng.exponential(mean_life_s, size=arr.shape[0])
    dep = arr + life
    dep[dep >= duration_s] = np.inf
    reqs = make_requests(arr.shape[0], rng, n_lo, n_hi)
    return reqs, arr, dep


# Value ranges of decision-matrix columns for standalone scoring: residual
# CPU cores, residual RAM GB, placed-container flag, path bandwidth (Mbps),
# summed hop count, then wider columns for extra criteria.
TILE_RANGES = ((0, 32), (0, 256), (0, 1), (0, 40000), (0, 384), (0, 100000), (0, 10), (0, (1 << 22) - 1))


def make_tiles(seed: int, T: int, N: int, C: int = 4, feasible_p: Optional[float] = None):
    """T integer decision matrices, criterion-major int32 [T][C][N], with the
    column ranges above, and (when feasible_p is given) a uint8 [T][N]
    feasibility mask drawn Bernoulli(feasible_p)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    x = np.empty((T, C, N), np.int32)
    for c in range(C):
        lo, hi = TILE_RANGES[c % len(TILE_RANGES)]
        x[:, c, :] = rng.integers(lo, hi + 1, size=(T, N), dtype=np.int32)
    feas = None
    if feasible_p is not None:
        feas = (rng.random((T, N)) < feasible_p).astype(np.uint8)
    return x, feas
