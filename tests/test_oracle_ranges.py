"""Pins for the oracle's demand intervals (section II-A: every container and
container pair asks for a minimum and a maximum; the utilities U(i), U(ij)
of Eqs. (1)-(2) measure what it is given).  Reading: feasibility and every
capacity check use the minima; once the minima fit, a placement gives as
much as the chosen server has left, up to the maximum, and tops each routed
path up in peer order the same way.  Everything here runs on the
CPU and checks the oracle against hand cases, the reduction to fixed demands
and invariants computed independently of it."""
import numpy as np
import pytest

import oracle as O
from workloads import make_instance, make_requests, Request

from test_oracle_pins import _ft_links, _pods_of


def _req(cpu, ram, edges, cpu_max=None, ram_max=None, bw_max=None, pod=None):
    a = lambda x: None if x is None else np.asarray(x, np.int32)
    e = np.asarray(edges, np.int32).reshape(-1, 3)
    return Request(a(cpu), a(ram), e, a(pod), a(cpu_max), a(ram_max), a(bw_max))


def utilities(req, res):
    """U(i) per container (mean over CPU and RAM of allocated / maximum) and
    U(ij) per edge (allocated / maximum), Eqs. (1)-(2)."""
    cx = req.cpu if req.cpu_max is None else req.cpu_max
    rx = req.ram if req.ram_max is None else req.ram_max
    bx = req.edges[:, 2] if req.bw_max is None else req.bw_max
    ui = (res["cpu_a"] / np.maximum(cx, 1) + res["ram_a"] / np.maximum(rx, 1)) / 2
    uij = res["bw_a"] / np.maximum(bx, 1)
    return ui, uij


def test_equal_bounds_are_fixed_demands(oracle_lib):
    """max = min everywhere schedules exactly as fixed demands (servers,
    scores, paths, state), and every allocation is the demand."""
    rng = np.random.default_rng(61)
    inst = make_instance(6, 32, 256, 5000, 8000, 8000, background=0.5, rng=rng)
    for route_end in (False, True):
        a, b = O.Oracle(inst, O.method(route_end=route_end)), O.Oracle(inst, O.method(route_end=route_end))
        n_acc = 0
        for r in make_requests(40, rng, 2, 8, pod_frac=0.5):
            ra = a.run_request(r)
            rb = b.run_request(Request(r.cpu, r.ram, r.edges, r.pod, r.cpu.copy(), r.ram.copy(),
                                       r.edges[:, 2].copy()))
            assert ra["status"] == rb["status"] and ra["failed_at"] == rb["failed_at"]
            np.testing.assert_array_equal(ra["hosts"], rb["hosts"])
            np.testing.assert_array_equal(ra["scores"], rb["scores"])
            if ra["status"] == 1:
                n_acc += 1
                np.testing.assert_array_equal(a.paths(ra["rec_id"])[0], b.paths(rb["rec_id"])[0])
                np.testing.assert_array_equal(a.paths(ra["rec_id"])[1], b.paths(rb["rec_id"])[1])
                for x in (ra, rb):
                    np.testing.assert_array_equal(x["cpu_a"], r.cpu)
                    np.testing.assert_array_equal(x["ram_a"], r.ram)
                    np.testing.assert_array_equal(x["bw_a"], r.edges[:, 2])
        np.testing.assert_array_equal(a.state(), b.state())
        assert n_acc >= 10


def test_hand_cpu_ram(oracle_lib):
    """k=4, 32 cores / 256 GB per server, empty.  A container asking for
    [4, 10] cores and [8, 20] GB gets its maxima.  One asking for [4, 40]
    and [8, 300] gets the whole server (32 and 256: U(i) = (0.8 + 256/300)
    / 2), and the server then has nothing left, so a container needing 30
    cores goes elsewhere."""
    inst = make_instance(4, 32, 256, 1000, 1000, 1000)
    o = O.Oracle(inst)
    r1 = _req([4], [8], [], cpu_max=[10], ram_max=[20])
    x = o.run_request(r1)
    assert x["status"] == 1 and x["cpu_a"].tolist() == [10] and x["ram_a"].tolist() == [20]
    u1 = int(x["hosts"][0])
    r2 = _req([4], [8], [], cpu_max=[40], ram_max=[300])
    x = o.run_request(r2, follow=np.array([u1 ^ 1], np.int32))
    assert x["status"] == 1 and x["cpu_a"].tolist() == [32] and x["ram_a"].tolist() == [256]
    ui, _ = utilities(r2, x)
    assert ui[0] == pytest.approx((32 / 40 + 256 / 300) / 2, abs=1e-15)
    st = o.state()
    assert st[0][u1 ^ 1] == 0 and st[1][u1 ^ 1] == 0
    assert st[0][u1] == 22 and st[1][u1] == 236
    x = o.run_request(_req([30], [1], []))
    assert x["status"] == 1 and int(x["hosts"][0]) not in (u1, u1 ^ 1)


def test_hand_bandwidth(oracle_lib):
    """Two containers that cannot share a server (32 cores each) joined by
    [300, 5000] Mbps on 1,000 Mbps links: the path is given its bottleneck,
    1,000 (U(ij) = 0.2), and every link on it is left at 0; routed at the
    end of the request the same.  A pair asking [300, 600] gets 600."""
    inst = make_instance(4, 32, 256, 1000, 1000, 1000)
    ends, _ = _ft_links(4)
    for route_end in (False, True):
        o = O.Oracle(inst, O.method(route_end=route_end))
        r = _req([32, 32], [1, 1], [[0, 1, 300]], bw_max=[5000])
        x = o.run_request(r, follow=np.array([0, 15], np.int32))
        assert x["status"] == 1 and x["bw_a"].tolist() == [1000]
        _, uij = utilities(r, x)
        assert uij[0] == 0.2
        links, bws = o.paths(x["rec_id"])
        assert bws.tolist() == [1000] and (links[0] >= 0).sum() == 6
        st = o.state()[3:].reshape(-1)
        assert all(st[l] == 0 for l in links[0] if l >= 0)
        x = o.run_request(_req([32, 32], [1, 1], [[0, 1, 300]], bw_max=[600]), follow=np.array([1, 14], np.int32))
        assert x["status"] == 1 and x["bw_a"].tolist() == [600]


def test_hand_route_end_minima_then_top_ups(oracle_lib):
    """k=4: containers 1 and 2 on server 4 each ask [600, 1400] Mbps to
    container 0 on server 0; core (0, 0)'s aggregation-core links hold 1500,
    the other cores' 1000.  Routed at each placement, the first pair takes
    its 600 over core (0, 0) and tops up to 1400; the second then finds core
    (0, 1) widest (1000), takes 600 and tops up by the 400 left: 1000.
    Routed at the end, both pairs pick core (0, 0) on the residuals the
    placement left; the two minima (1200) fit its 1500, and the top-ups in
    order give the first pair the 300 left: 900 and 600.  With minima of
    800 each (1600 > 1500) the request is rejected with failed_at = n and
    nothing taken."""
    inst = make_instance(4, 32, 256, 40000, 10000, 1000)
    r = _req([1, 1, 1], [1, 1, 1], [[0, 1, 600], [0, 2, 600]], bw_max=[1400, 1400])
    for route_end in (False, True):
        o = O.Oracle(inst, O.method(route_end=route_end))
        o.set_link(2 * 16 + 0, 1500)
        o.set_link(2 * 16 + 4, 1500)
        s0 = o.state().copy()
        x = o.run_request(r, follow=np.array([0, 4, 4], np.int32))
        assert x["status"] == 1
        links, bws = o.paths(x["rec_id"])
        got = [sorted(int(l) for l in p if l >= 0) for p in links]
        if not route_end:
            assert x["bw_a"].tolist() == [1400, 1000] and bws.tolist() == [1400, 1000]
            assert got == [[0, 4, 16, 20, 32, 36], [0, 4, 16, 20, 33, 37]]
        else:
            assert x["bw_a"].tolist() == [900, 600] and bws.tolist() == [900, 600]
            assert got == [[0, 4, 16, 20, 32, 36], [0, 4, 16, 20, 32, 36]]
            assert o.state()[5][0] == 0 and o.state()[5][4] == 0
        o2 = O.Oracle(inst, O.method(route_end=route_end))
        o2.set_link(2 * 16 + 0, 1500)
        o2.set_link(2 * 16 + 4, 1500)
        x = o2.run_request(_req([1, 1, 1], [1, 1, 1], [[0, 1, 800], [0, 2, 800]], bw_max=[1400, 1400]),
                           follow=np.array([0, 4, 4], np.int32))
        if route_end:
            assert x["status"] == 0 and x["failed_at"] == 3
            np.testing.assert_array_equal(o2.state(), s0)
        else:
            assert x["status"] == 1 and x["bw_a"].tolist() == [1400, 1000]


def test_pod_split_in_container_order(oracle_lib):
    """A pod of three containers [2, 10], [3, 5], [4, 20] cores is one unit
    asking [9, 35]; on a server with 12 cores left it gets 12, handed back
    in container order: 2 + 3 + 4 minima, then 3 more to the first."""
    inst = make_instance(4, 32, 256, 1000, 1000, 1000)
    o = O.Oracle(inst)
    o.run_request(_req([20], [1], []), follow=np.array([5], np.int32))
    x = o.run_request(_req([2, 3, 4], [1, 1, 1], [[0, 1, 10], [1, 2, 10]], cpu_max=[10, 5, 20], ram_max=[1, 1, 1],
                           bw_max=[50, 70], pod=[0, 0, 0]), follow=np.array([5], np.int32))
    assert x["status"] == 1 and x["hosts"].tolist() == [5, 5, 5]
    assert x["cpu_a"].tolist() == [5, 3, 4]
    assert x["bw_a"].tolist() == [50, 70]          # inside the pod: no link, maxima
    assert o.state()[0][5] == 0


@pytest.mark.parametrize("kind,route_end", [(O.TOPSIS, False), (O.AHP, False), (O.TOPSIS, True)])
def test_ranges_sound(oracle_lib, kind, route_end):
    """Loaded k=4, requests with intervals and pods.  Accepted: every
    allocation lies in [min, max]; a pod sits on one server; what each
    server and link loses is exactly what the request was given; CPU or
    RAM below the maximum leaves that server at 0 of it, a pod pair below
    its summed maximum leaves a link of its path at 0; within a pod, after
    the first container short of its maximum every later one has its
    minimum.  A one-container request is given min(max, residual) of the
    server it lands on.  Rejected: nothing changes.  Releasing everything
    restores the initial state."""
    rng = np.random.default_rng(71 + kind + 2 * route_end)
    inst = make_instance(4, 32, 256, 4000, 4000, 4000, background=0.7, rng=rng)
    o = O.Oracle(inst, O.method(kind, route_end=route_end))
    ends, _ = _ft_links(4)
    s0 = o.state().copy()
    n_acc = n_rej = n_short_c = n_short_b = 0
    live = []
    for t in range(90):
        n = int(rng.integers(1, 6))
        req = make_requests(1, rng, n, n, cpu_lo=1, cpu_hi=8, ram_lo=1, ram_hi=50, bw_lo=100, bw_hi=1500,
                            pod_frac=0.5, ranges="widen")[0]
        unit, groups = _pods_of(n, req.pod)
        before = o.state().astype(np.int64)
        res = o.run_request(req)
        after = o.state().astype(np.int64)
        assert np.all(after >= 0)
        if res["status"] != 1:
            n_rej += 1
            np.testing.assert_array_equal(after, before)
            continue
        n_acc += 1
        live.append(res["rec_id"])
        hosts, ca, ra, ba = res["hosts"], res["cpu_a"], res["ram_a"], res["bw_a"]
        assert np.all((req.cpu <= ca) & (ca <= req.cpu_max)) and np.all((req.ram <= ra) & (ra <= req.ram_max))
        assert np.all((req.edges[:, 2] <= ba) & (ba <= req.bw_max))
        for g in groups:
            assert len(set(hosts[g].tolist())) == 1
            for a_, mn, mx in ((ca, req.cpu, req.cpu_max), (ra, req.ram, req.ram_max)):
                short = [i for i in g if a_[i] < mx[i]]
                if short:
                    assert all(a_[i] == mn[i] for i in g if i > short[0])
        use_cpu = np.bincount(hosts, weights=ca, minlength=16).astype(np.int64)
        use_ram = np.bincount(hosts, weights=ra, minlength=16).astype(np.int64)
        np.testing.assert_array_equal(after[0], before[0] - use_cpu)
        np.testing.assert_array_equal(after[1], before[1] - use_ram)
        for i in range(n):
            if ca[i] < req.cpu_max[i] or ra[i] < req.ram_max[i]:
                n_short_c += 1
            if ca[i] < req.cpu_max[i]:
                assert after[0][hosts[i]] == 0
            if ra[i] < req.ram_max[i]:
                assert after[1][hosts[i]] == 0
        if len(groups) == 1:
            assert ca.sum() == min(req.cpu_max.sum(), before[0][hosts[0]])
            assert ra.sum() == min(req.ram_max.sum(), before[1][hosts[0]])
        # pod pairs: summed allocation on a path joining the two servers
        dem, mx = {}, {}
        for e, (a, b, _) in enumerate(req.edges):
            ua, ub = unit[a], unit[b]
            if ua == ub or hosts[a] == hosts[b]:
                assert ba[e] == req.bw_max[e]
                continue
            key = (max(ua, ub), min(ua, ub))
            dem[key] = dem.get(key, 0) + int(ba[e])
            mx[key] = mx.get(key, 0) + int(req.bw_max[e])
        links, bws = o.paths(res["rec_id"])
        link_use = np.zeros(48, np.int64)
        routed = [(p, int(b)) for p, b in zip(links, bws) if (p >= 0).any()]
        assert sorted(b for _, b in routed) == sorted(dem.values())
        for path, bw in routed:
            for l in path[path >= 0]:
                link_use[l] += bw
        for key, got in dem.items():
            if got < mx[key]:
                n_short_b += 1
                path = next(p for p, b in routed if b == got)
                assert any(after[3:].reshape(-1)[l] == 0 for l in path[path >= 0])
        np.testing.assert_array_equal(after[3:].reshape(-1), before[3:].reshape(-1) - link_use)
        if rng.random() < 0.3 and live:
            rid = live.pop(int(rng.integers(len(live))))
            assert o.release(rid) == 0
    assert n_acc >= 15 and n_rej >= 3 and n_short_c >= 3 and n_short_b >= 1
    for rid in live:
        assert o.release(rid) == 0
    np.testing.assert_array_equal(o.state(), s0)
