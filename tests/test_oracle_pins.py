"""Pins for the FP64 oracle: hand-worked examples, closed forms, invariants
and brute force.  Everything here runs on the CPU."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from workloads import make_instance, make_requests, Request

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- TOPSIS
@pytest.mark.parametrize("case", _load("topsis_hand.json")["cases"], ids=lambda c: c["name"][:40])
def test_topsis_hand_cases(oracle_lib, case):
    got = O.topsis(np.array(case["X"], float), case["w"], case["cost"])
    np.testing.assert_allclose(got, case["rank"], rtol=0, atol=1e-15)


def test_topsis_exact_tie_is_bitwise(oracle_lib):
    got = O.topsis(np.array([[3, 4, 0], [4, 3, 0]], float), [0.5, 0.5])
    assert got[0] == got[1]


def test_topsis_invariants(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(50):
        C, N = int(rng.integers(1, 6)), int(rng.integers(2, 40))
        X = rng.integers(0, 50, size=(C, N)).astype(float)
        w = rng.uniform(0.1, 1.0, C)
        w /= w.sum()
        cost = rng.integers(0, 2, C).astype(np.int32)
        r = O.topsis(X, w, cost)
        assert np.all(r >= 0) and np.all(r <= 1 + 1e-15)
        # positive column scaling leaves the closeness unchanged
        s = rng.uniform(0.5, 20.0, C)
        np.testing.assert_allclose(O.topsis(X * s[:, None], w, cost), r, rtol=1e-12, atol=1e-12)
        # permuting servers permutes the closeness
        perm = rng.permutation(N)
        np.testing.assert_allclose(O.topsis(X[:, perm], w, cost), r[perm], rtol=1e-12, atol=1e-12)
    # a server at the ideal on every criterion scores 1, one at the anti-ideal 0
    X = np.array([[5, 1, 3], [9, 2, 4]], float)
    r = O.topsis(X, [0.5, 0.5])
    assert r[0] == 1.0 and r[1] == 0.0
    # an all-zero criterion contributes nothing
    X0 = np.array([[5, 1, 3], [0, 0, 0]], float)
    np.testing.assert_allclose(O.topsis(X0, [0.5, 0.5]), O.topsis(X0[:1], [1.0]), atol=1e-15)


# ---------------------------------------------------------------- AHP
@pytest.mark.parametrize("case", _load("ahp_hand.json")["cases"], ids=lambda c: c["name"][:40])
def test_ahp_hand_cases(oracle_lib, case):
    scale = O.RATIO if case["scale"] == "ratio" else O.SAATY9
    got = O.ahp(np.array(case["X"], float), case["w"], case["cost"], scale=scale)
    want = [a / b for a, b in case["pg"]]
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-16)


def _saaty_def(p, q):
    """Saaty 1-9 comparison from the definition: ratio rounded half up,
    clamped to [1, 9], zero denominator scores 9, reverse is reciprocal."""
    if p == q:
        return Fraction(1)
    if p < q:
        return 1 / _saaty_def(q, p)
    if q == 0:
        return Fraction(9)
    r = Fraction(p, q) + Fraction(1, 2)
    s = r.numerator // r.denominator
    return Fraction(min(9, max(1, s)))


def test_saaty_table_exhaustive_cpu_ram(oracle_lib):
    for top in (32, 256):
        rng = range(top + 1)
        for p in rng:
            for q in rng:
                if top == 256 and (p % 3 and q % 5):   # RAM: a dense third of the table
                    continue
                assert O.saaty(p, q) == float(_saaty_def(p, q)), (p, q)


def test_saaty_half_boundaries_bandwidth(oracle_lib):
    rng = np.random.default_rng(7)
    for q in list(rng.integers(1, 20000, 400) * 2) + [2, 4, 40000]:
        q = int(q)
        for n in range(1, 10):
            for p in (n * q + q // 2 - 1, n * q + q // 2, n * q + q // 2 + 1):
                assert O.saaty(p, q) == float(_saaty_def(p, q)), (p, q)
                assert O.saaty(q, p) == float(_saaty_def(q, p)), (q, p)


def test_ahp_invariants(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(30):
        C, N = int(rng.integers(1, 5)), int(rng.integers(2, 30))
        X = rng.integers(0, 40, size=(C, N)).astype(float)
        w = rng.uniform(0.1, 1.0, C)
        w /= w.sum()
        cost = rng.integers(0, 2, C).astype(np.int32)
        pg, p1, p2 = O.ahp(X, w, cost, return_levels=True)
        np.testing.assert_allclose(p2.sum(axis=1), 1.0, rtol=1e-13)   # each local rank sums to 1
        np.testing.assert_allclose(p1, w, rtol=1e-13)                  # consistent weight matrix
        np.testing.assert_allclose(pg.sum(), w.sum(), rtol=1e-13)
        perm = rng.permutation(N)
        np.testing.assert_allclose(O.ahp(X[:, perm], w, cost), pg[perm], rtol=1e-13)
    # all-equal values: every server 1/N
    np.testing.assert_allclose(O.ahp(np.full((2, 7), 5.0), [0.5, 0.5]), 1 / 7, rtol=1e-15)
    # ratio scale: priorities equal v / sum(v)
    for _ in range(20):
        v = rng.integers(1, 1000, size=int(rng.integers(2, 50))).astype(float)
        np.testing.assert_allclose(O.ahp(v[None], [1.0], scale=O.RATIO), v / v.sum(), rtol=1e-13)


# ---------------------------------------------------------------- paths
def _ft_links(k):
    """Link endpoints of a k-ary fat-tree, written from the index
    conventions of the input format (independent of the oracle)."""
    h, N = k // 2, k ** 3 // 4
    ends = {}
    for u in range(N):
        ends[u] = (("h", u), ("e", u // h))
    for eg in range(k * k // 2):
        for a in range(h):
            ends[N + eg * h + a] = (("e", eg), ("a", (eg // h) * h + a))
    for ag in range(k * k // 2):
        for j in range(h):
            ends[2 * N + ag * h + j] = (("a", ag), ("c", (ag % h) * h + j))
    adj = {}
    for l, (x, y) in ends.items():
        adj.setdefault(x, []).append((y, l))
        adj.setdefault(y, []).append((x, l))
    return ends, adj


def _all_shortest(adj, u, v, maxlen=6):
    """Every simple path from host u to host v with at most maxlen links,
    keeping only the shortest ones (brute-force DFS)."""
    src, dst = ("h", u), ("h", v)
    if u == v:
        return [[]]
    found = []

    def go(x, seen, links):
        if len(links) > maxlen:
            return
        if x == dst:
            found.append(list(links))
            return
        for y, l in adj[x]:
            if y not in seen:
                seen.add(y)
                links.append(l)
                go(y, seen, links)
                links.pop()
                seen.discard(y)

    go(src, {src}, [])
    m = min(len(p) for p in found)
    return [p for p in found if len(p) == m]


@pytest.mark.parametrize("k", [4, 6])
def test_minimum_hop_paths_brute_force(oracle_lib, k):
    inst = make_instance(k, 32, 256, 10000, 10000, 10000)
    o = O.Oracle(inst)
    ends, adj = _ft_links(k)
    rng = np.random.default_rng(k)
    res = rng.integers(0, 6, size=3 * inst.n_hosts)      # small range: many ties
    for l, r in enumerate(res):
        o.set_link(l, int(r))
    h, N = k // 2, inst.n_hosts
    pairs = [(u, v) for u in range(N) for v in range(N)]
    if k > 4:
        pairs = [pairs[int(i)] for i in rng.choice(len(pairs), 300, replace=False)]
    widest_cache = {}
    for u, v in pairs:
        paths = _all_shortest(adj, u, v)
        hops = len(paths[0])
        same_edge, same_pod = u // h == v // h, u // (h * h) == v // (h * h)
        want_hops = 0 if u == v else 2 if same_edge else 4 if same_pod else 6
        want_cnt = 1 if hops <= 2 else h if hops == 4 else h * h
        assert hops == want_hops and len(paths) == want_cnt, (u, v)
        best = max((min(res[l] for l in p) if p else np.iinfo(np.int64).max) for p in paths)
        cnt, b, hp, links = o.widest_enum(u, v)
        assert (cnt, hp, b) == (len(paths), hops, best), (u, v)
        if hops:
            # tie-break: the first widest path when aggregation then core index ascend
            def key(p):
                aggs = sorted({l for l in p if N <= l < 2 * N})
                cores = [l for l in p if l >= 2 * N]
                return (min(l % h for l in aggs) if aggs else -1, min(l % h for l in cores) if cores else -1)
            first = min((p for p in paths if min(res[l] for l in p) == best), key=key)
            assert sorted(links.tolist()) == sorted(first), (u, v)
        if v not in widest_cache:
            widest_cache[v] = o.widest_from(v)
        W, H = widest_cache[v]
        assert H[u] == hops and (u == v or W[u] == best), (u, v)


# ---------------------------------------------------------------- criteria
def test_criteria_hand_case(oracle_lib):
    """k=4 data center (2 hosts per edge switch, 4 per pod), one placed peer
    on host 0 wanting 300 Mbps.  Expected criteria worked out by hand."""
    inst = make_instance(4, 32, 256, 1000, 1000, 1000)
    o = O.Oracle(inst)
    N = 16
    # residuals: uplinks 0..15 -> 1000 - 10*u ; one edge-agg link of edge 0 low
    for u in range(N):
        o.set_link(u, 1000 - 10 * u)
    o.set_link(N + 0 * 2 + 0, 200)      # edge 0 - agg (pod 0, a=0)
    o.set_link(N + 0 * 2 + 1, 700)      # edge 0 - agg (pod 0, a=1)
    o.set_link(2 * N + 1 * 2 + 0, 50)   # agg (pod 0, a=1) - core 2
    m = O.method(O.TOPSIS, crit=(O.CRIT_CPU, O.CRIT_RAM, O.CRIT_ACTIVE, O.CRIT_PATHBW,
                                 O.CRIT_UPLINK, O.CRIT_HOPS), cost=[0, 0, 0, 0, 0, 1],
                 weight=[1 / 6] * 6)
    o.m = m
    X, feas, _ = o.step_scores(4, 8, [0], [300])
    up = 1000 - 10 * np.arange(N)
    # host 0: co-located with the peer -> path bw = own uplink, 0 hops
    assert X[3][0] == up[0] and X[5][0] == 0
    # host 1: same edge switch -> min(up1, up0), 2 hops
    assert X[3][1] == min(up[1], up[0]) and X[5][1] == 2
    # hosts 2,3: same pod via agg a=0 (200) or a=1 (700) -> 700 bottleneck is min(up, 700)
    assert X[3][2] == min(up[2], 700) and X[5][2] == 4
    # hosts in other pods: via a=0 limited by 200, via a=1: core 2 link 50, core 3 link 1000 -> 700
    for u in range(4, N):
        assert X[3][u] == min(up[u], 700) and X[5][u] == 6
    assert np.all(X[4] == up) and np.all(X[0] == 32) and np.all(X[1] == 256) and np.all(X[2] == 0)
    assert feas.all()
    # 800 Mbps: host 0 (co-located) and host 1 (two uplinks of 1000 and 990)
    # stay feasible; every other path is capped at 700
    X, feas, _ = o.step_scores(4, 8, [0], [800])
    assert feas[0] and feas[1] and not feas[2:].any()
    # demand above the server's CPU
    X, feas, _ = o.step_scores(33, 8, [], [])
    assert not feas.any()


def test_uplink_sum_feasibility(oracle_lib):
    """Two remote peers each fit alone but not together on the uplink."""
    inst = make_instance(4, 32, 256, 1000, 10000, 10000)
    o = O.Oracle(inst)
    o.set_link(5, 500)
    _, feas, _ = o.step_scores(1, 1, [0, 1], [300, 300])
    assert not feas[5] and feas[4] and feas[0] and feas[1]


# ---------------------------------------------------------------- placement soundness
def _verify_solution(inst_k, before, after, req, hosts, links, bws):
    """Check an accepted placement against Eqs. (4)-(5), single hosting and
    path connectivity, using link endpoints written independently."""
    N = inst_k ** 3 // 4
    ends, _ = _ft_links(inst_k)
    use_cpu = np.zeros(N, np.int64)
    use_ram = np.zeros(N, np.int64)
    for i in range(req.n):
        use_cpu[hosts[i]] += req.cpu[i]
        use_ram[hosts[i]] += req.ram[i]
    assert np.all(use_cpu <= before[0]) and np.all(use_ram <= before[1])
    link_use = np.zeros(3 * N, np.int64)
    q = 0
    peers = {}
    for a, b, bw in req.edges:
        peers.setdefault(max(a, b), []).append((min(a, b), bw))
    for i in range(req.n):
        for j, bw in sorted(peers.get(i, [])):
            path = [l for l in links[q] if l >= 0]
            assert bws[q] == bw
            # path must walk from host(i) to host(j)
            cur = ("h", hosts[i])
            for l in path:
                x, y = ends[l]
                assert cur in (x, y)
                cur = y if cur == x else x
            assert cur == ("h", hosts[j])
            for l in path:
                link_use[l] += bw
            q += 1
    assert q == len(links)
    assert np.all(link_use <= before[3:].reshape(-1))
    np.testing.assert_array_equal(after[0], before[0] - use_cpu)
    np.testing.assert_array_equal(after[1], before[1] - use_ram)
    np.testing.assert_array_equal(after[3:].reshape(-1), before[3:].reshape(-1) - link_use)


def _brute_feasible(k, state, req):
    """Exists a placement plus a choice of minimum-hop paths satisfying the
    capacity and bandwidth constraints (tiny n only)."""
    N = k ** 3 // 4
    _, adj = _ft_links(k)
    pair_paths = {}
    edges = [(int(a), int(b), int(bw)) for a, b, bw in req.edges]
    for hosts in itertools.product(range(N), repeat=req.n):
        cpu = np.zeros(N, np.int64)
        ram = np.zeros(N, np.int64)
        for i, u in enumerate(hosts):
            cpu[u] += req.cpu[i]
            ram[u] += req.ram[i]
        if np.any(cpu > state[0]) or np.any(ram > state[1]):
            continue
        choices = []
        for a, b, bw in edges:
            key = (hosts[a], hosts[b])
            if key not in pair_paths:
                pair_paths[key] = _all_shortest(adj, *key)
            choices.append(pair_paths[key])
        for pick in itertools.product(*choices):
            use = np.zeros(3 * N, np.int64)
            for (a, b, bw), p in zip(edges, pick):
                for l in p:
                    use[l] += bw
            if np.all(use <= state[3:].reshape(-1)):
                return True
    return False


@pytest.mark.parametrize("kind", [O.TOPSIS, O.AHP])
def test_placement_soundness_brute_force(oracle_lib, kind):
    rng = np.random.default_rng(11 + kind)
    inst = make_instance(4, 32, 256, 3000, 3000, 3000, background=0.9, rng=rng)
    o = O.Oracle(inst, O.method(kind))
    n_acc = n_rej = 0
    for t in range(60):
        n = int(rng.integers(1, 4))
        req = make_requests(1, rng, n, n, cpu_lo=1, cpu_hi=14, ram_lo=1, ram_hi=90,
                            bw_lo=100, bw_hi=2500)[0]
        before = o.state().astype(np.int64)
        res = o.run_request(req)
        after = o.state().astype(np.int64)
        assert np.all(after >= 0)
        if res["status"] == 1:
            n_acc += 1
            links, bws = o.paths(res["rec_id"])
            _verify_solution(4, before, after, req, res["hosts"], links, bws)
            assert np.all(after[2] - before[2] == np.bincount(res["hosts"], minlength=16))
        else:
            n_rej += 1
            assert res["status"] == 0
            np.testing.assert_array_equal(after, before)
            if n == 1:
                # a single container is rejected only when nothing fits
                assert not _brute_feasible(4, before, req)
        if res["status"] == 1 and n == 1:
            assert _brute_feasible(4, before, req)
    assert n_acc >= 10 and n_rej >= 10


def test_release_restores_state(oracle_lib):
    rng = np.random.default_rng(5)
    inst = make_instance(6, 32, 256, 5000, 8000, 8000, background=0.5, rng=rng)
    o = O.Oracle(inst)
    s0 = o.state().copy()
    reqs = make_requests(60, rng, 2, 8)
    acc = []
    total_bw_hops = 0
    for r in reqs:
        res = o.run_request(r)
        assert np.all(o.state() >= 0)
        if res["status"] == 1:
            acc.append(res["rec_id"])
            links, bws = o.paths(res["rec_id"])
            total_bw_hops += int(sum(int(b) * int((l >= 0).sum()) for l, b in zip(links, bws)))
    assert len(acc) > 5
    used = (s0[3:].astype(np.int64) - o.state()[3:]).sum()
    assert used == total_bw_hops            # link usage = sum of bw x hops over routed pairs
    for rid in rng.permutation(acc):
        assert o.release(int(rid)) == 0
    np.testing.assert_array_equal(o.state(), s0)
    assert o.release(int(acc[0])) == -1      # second release of the same request


def test_invalid_requests_rejected(oracle_lib):
    inst = make_instance(4, 32, 256, 1000, 1000, 1000)
    o = O.Oracle(inst)
    bad = Request(np.array([1, 1], np.int32), np.array([1, 1], np.int32),
                  np.array([[0, 0, 5]], np.int32))
    assert o.run_request(bad)["status"] == -1
    dup = Request(np.array([1, 1], np.int32), np.array([1, 1], np.int32),
                  np.array([[0, 1, 5], [1, 0, 5]], np.int32))
    assert o.run_request(dup)["status"] == -1


# ---------------------------------------------------------------- pods (Eq. (8))
def _pods_of(n, pod):
    """Pods in the order of their first container, computed here from the
    definition: (unit of each container, containers of each pod)."""
    unit, groups, seen = [], [], {}
    for i in range(n):
        key = ("c", i) if pod is None or pod[i] < 0 else ("p", int(pod[i]))
        if key not in seen:
            seen[key] = len(groups)
            groups.append([])
        unit.append(seen[key])
        groups[seen[key]].append(i)
    return unit, groups


def test_pods_of_singletons_equal_no_pods(oracle_lib):
    """A request whose pods all hold one container schedules exactly as the
    same request without pods (same servers, scores, paths and state)."""
    rng = np.random.default_rng(21)
    inst = make_instance(6, 32, 256, 5000, 8000, 8000, background=0.5, rng=rng)
    a, b, c = O.Oracle(inst), O.Oracle(inst), O.Oracle(inst)
    for r in make_requests(40, rng, 2, 8):
        n = r.n
        ra = a.run_request(r)
        rb = b.run_request(Request(r.cpu, r.ram, r.edges, np.full(n, -1, np.int32)))
        rc = c.run_request(Request(r.cpu, r.ram, r.edges, np.arange(n, dtype=np.int32) * 7))
        for x in (rb, rc):
            assert x["status"] == ra["status"] and x["failed_at"] == ra["failed_at"]
            np.testing.assert_array_equal(x["hosts"], ra["hosts"])
            np.testing.assert_array_equal(x["scores"], ra["scores"])
        if ra["status"] == 1:
            for o2, x in ((b, rb), (c, rc)):
                pa, pb = a.paths(ra["rec_id"]), o2.paths(x["rec_id"])
                np.testing.assert_array_equal(pa[0], pb[0])
    np.testing.assert_array_equal(a.state(), b.state())
    np.testing.assert_array_equal(a.state(), c.state())


def test_one_pod_is_one_container(oracle_lib):
    """All containers in one pod: placed like one container with the summed
    demand, whatever traffic they exchange (it stays on the server)."""
    rng = np.random.default_rng(22)
    inst = make_instance(4, 32, 256, 10000, 10000, 10000, background=0.6, rng=rng)
    a, b = O.Oracle(inst), O.Oracle(inst)
    for r in make_requests(30, rng, 2, 4, cpu_hi=6, ram_hi=40):
        ra = a.run_request(Request(r.cpu, r.ram, r.edges, np.zeros(r.n, np.int32)))
        one = Request(np.array([r.cpu.sum()], np.int32), np.array([r.ram.sum()], np.int32),
                      np.zeros((0, 3), np.int32))
        rb = b.run_request(one)
        assert ra["status"] == rb["status"]
        if ra["status"] == 1:
            assert np.all(ra["hosts"] == rb["hosts"][0])
            assert np.all(ra["scores"] == rb["scores"][0])
            assert a.paths(ra["rec_id"])[0].shape[0] == 0
        else:
            assert ra["failed_at"] == 0
    np.testing.assert_array_equal(a.state(), b.state())


@pytest.mark.parametrize("kind", [O.TOPSIS, O.AHP])
def test_pod_placements_sound(oracle_lib, kind):
    """k=4, loaded: every accepted request with pods keeps each pod on one
    server (Eq. (8)), fits CPU and RAM (Eq. (4)) and routes the summed
    traffic between two pods on a path joining their servers within the
    link residuals (Eq. (5)); a rejected one changes nothing; a request that
    is one pod is rejected only when no server fits its summed demand."""
    rng = np.random.default_rng(31 + kind)
    inst = make_instance(4, 32, 256, 4000, 4000, 4000, background=0.8, rng=rng)
    o = O.Oracle(inst, O.method(kind))
    ends, _ = _ft_links(4)
    n_acc = n_rej = 0
    for t in range(80):
        n = int(rng.integers(2, 6))
        req = make_requests(1, rng, n, n, cpu_lo=1, cpu_hi=10, ram_lo=1, ram_hi=60, bw_lo=100,
                            bw_hi=1500, pod_frac=1.0)[0]
        unit, groups = _pods_of(n, req.pod)
        before = o.state().astype(np.int64)
        res = o.run_request(req)
        after = o.state().astype(np.int64)
        assert np.all(after >= 0)
        if res["status"] != 1:
            n_rej += 1
            assert res["status"] == 0 and res["failed_at"] == groups[unit[res["failed_at"]]][0]
            np.testing.assert_array_equal(after, before)
            if len(groups) == 1:
                fits = (before[0] >= req.cpu.sum()) & (before[1] >= req.ram.sum())
                assert not fits.any()
            continue
        n_acc += 1
        hosts = res["hosts"]
        for g in groups:
            assert len(set(hosts[g].tolist())) == 1          # Eq. (8)
        use_cpu = np.bincount(hosts, weights=req.cpu, minlength=16)
        use_ram = np.bincount(hosts, weights=req.ram, minlength=16)
        assert np.all(use_cpu <= before[0]) and np.all(use_ram <= before[1])
        # summed traffic between pods, expected in pod order then earlier pod
        dem = {}
        for a, b, bw in req.edges:
            ua, ub = unit[a], unit[b]
            if ua != ub:
                key = (max(ua, ub), min(ua, ub))
                dem[key] = dem.get(key, 0) + int(bw)
        links, bws = o.paths(res["rec_id"])
        keys = sorted(dem)
        assert len(keys) == len(links)
        link_use = np.zeros(48, np.int64)
        for (g, h), path, bw in zip(keys, links, bws):
            assert int(bw) == dem[(g, h)]
            cur = ("h", int(hosts[groups[g][0]]))
            for l in path[path >= 0]:
                x, y = ends[l]
                assert cur in (x, y)
                cur = y if cur == x else x
                link_use[l] += bw
            assert cur == ("h", int(hosts[groups[h][0]]))
        np.testing.assert_array_equal(after[0], before[0] - use_cpu)
        np.testing.assert_array_equal(after[1], before[1] - use_ram)
        np.testing.assert_array_equal(after[3:].reshape(-1), before[3:].reshape(-1) - link_use)
    assert n_acc >= 10 and n_rej >= 5


# ---------------------------------------------------------------- routing at the end of a request (section V-D)
def test_route_end_pairs_share_the_pre_routing_residuals(oracle_lib):
    """Hand case, k=4: containers 1 and 2 on server 4 (pod 1) each send
    1000 Mbps to container 0 on server 0 (pod 0).  The aggregation-core
    links of core (0, 0) hold 1500, every other one 1000.  Routed at each
    placement, the second pair sees 500 left on core (0, 0) and takes core
    (0, 1): accepted.  Routed at the end, both pairs pick core (0, 0) on the
    residuals the placement left and overdraw it: rejected, failed_at = n,
    nothing taken."""
    inst = make_instance(4, 32, 256, 40000, 10000, 1000)
    req = Request(np.ones(3, np.int32), np.ones(3, np.int32), np.array([[0, 1, 1000], [0, 2, 1000]], np.int32))
    out = {}
    for end in (False, True):
        o = O.Oracle(inst, O.method(route_end=end))
        o.set_link(2 * 16 + 0, 1500)       # pod 0, aggregation 0, core 0
        o.set_link(2 * 16 + 4, 1500)       # pod 1, aggregation 0, core 0
        s0 = o.state().copy()
        res = o.run_request(req, follow=np.array([0, 4, 4], np.int32))
        out[end] = (o, s0, res)
    o, s0, res = out[False]
    assert res["status"] == 1
    links, bws = o.paths(res["rec_id"])
    got = [sorted(int(l) for l in p if l >= 0) for p in links]
    assert got == [[0, 4, 16, 20, 32, 36], [0, 4, 16, 20, 33, 37]]
    o, s0, res = out[True]
    assert res["status"] == 0 and res["failed_at"] == 3
    np.testing.assert_array_equal(o.state(), s0)


def test_route_end_without_links_equals_route_each(oracle_lib):
    """Requests without traffic between containers schedule identically
    whichever way links are routed."""
    rng = np.random.default_rng(41)
    inst = make_instance(6, 32, 256, 5000, 8000, 8000, background=0.5, rng=rng)
    a, b = O.Oracle(inst), O.Oracle(inst, O.method(route_end=True))
    for r in make_requests(40, rng, 1, 8):
        r = Request(r.cpu, r.ram, np.zeros((0, 3), np.int32))
        ra, rb = a.run_request(r), b.run_request(r)
        assert ra["status"] == rb["status"]
        np.testing.assert_array_equal(ra["hosts"], rb["hosts"])
    np.testing.assert_array_equal(a.state(), b.state())


@pytest.mark.parametrize("kind", [O.TOPSIS, O.AHP])
def test_route_end_sound(oracle_lib, kind):
    """Routing at the end on a loaded k=4: an accepted request's pairs each
    run on a path joining their servers and the residuals absorb all of them
    (link usage = sum of demand x hops); a rejected one changes nothing."""
    rng = np.random.default_rng(51 + kind)
    inst = make_instance(4, 32, 256, 3000, 3000, 3000, background=0.8, rng=rng)
    o = O.Oracle(inst, O.method(kind, route_end=True))
    ends, _ = _ft_links(4)
    n_acc = n_rej = n_route = 0
    for t in range(80):
        n = int(rng.integers(2, 5))
        req = make_requests(1, rng, n, n, cpu_lo=1, cpu_hi=10, ram_lo=1, ram_hi=60, bw_lo=200, bw_hi=1500)[0]
        before = o.state().astype(np.int64)
        res = o.run_request(req)
        after = o.state().astype(np.int64)
        assert np.all(after >= 0)
        if res["status"] != 1:
            n_rej += 1
            n_route += res["failed_at"] == n
            np.testing.assert_array_equal(after, before)
            continue
        n_acc += 1
        _verify_solution(4, before, after, req, res["hosts"], *o.paths(res["rec_id"]))
    assert n_acc >= 10 and n_rej >= 5 and n_route >= 1
