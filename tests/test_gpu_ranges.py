"""GPU parity for demand intervals (section II-A, utilities of Eqs. (1)-(2)):
what every container and container pair is given, against the FP64 oracle,
in every form, through the C ABI."""
import numpy as np
import pytest

import oracle as O
from parity import lockstep, trace_by_request
from workloads import make_config, make_instance, Request

pytestmark = pytest.mark.gpu

dc = pytest.importorskip("paper_1909_07673_amd")


def _run(insts, reqs, **kw):
    s = dc.Scheduler(insts, **kw)
    ids = [[s.submit(r, instance=i) for r in rl] for i, rl in enumerate(reqs)]
    res = {r.req_id: r for r in s.schedule()}
    return s, ids, res


def _short(req, res, sched, rid):
    """Containers and edges of an accepted request given less than their
    maximum."""
    ca, ra, ba = sched.alloc(rid, req.n, req.m)
    return int((ca < req.cpu_max).sum() + (ra < req.ram_max).sum()), int((ba < req.bw_max).sum())


@pytest.mark.parametrize("method,routing", [(dc.DC_TOPSIS, 0), (dc.DC_AHP, 0), (dc.DC_TOPSIS, 1), (dc.DC_AHP, 1)])
def test_ranges_tiny_lockstep(method, routing):
    """k=4, 5 Gbps links, intervals up to twice the minimum, with and
    without pods: every step, score vector, path and allocation against the
    oracle, the state after every request."""
    tot = dict(accepted=0, steps=0)
    short_c = short_b = 0
    for seed in range(10):
        for preset in ("tiny_ranges", "tiny_ranges_pods"):
            insts, reqs = make_config(preset, seed=seed)
            s = dc.Scheduler(insts, method=method, routing=routing, trace_stride=1, trace_cap=4096)
            o = O.Oracle(insts[0], O.method(kind=method, route_end=bool(routing)))
            for req in reqs[0]:
                rid = s.submit(req)
                res = {r.req_id: r for r in s.schedule()}
                st = lockstep(o, s, [rid], [req], res, trace=trace_by_request(s), check_paths=True,
                              check_alloc=True, state_every=True)
                assert st["scored_steps"] == st["steps"]
                for k in tot:
                    tot[k] += st[k]
                if res[rid].status == 1:
                    c, b = _short(req, res[rid], s, rid)
                    short_c += c
                    short_b += b
            s.close()
    assert tot["accepted"] > 100 and short_c > 20 and short_b >= 3


@pytest.mark.parametrize("routing", [0, 1])
def test_ranges_k16_forms_agree(routing):
    """k=16, 0-70 % background, pods and intervals: plain in lockstep with
    the oracle (allocations, paths, final state); batched, serving and the
    cooperative step bit-identical to plain, allocations included."""
    insts, reqs = make_config("ranges", seed=4, n_req=250)
    p, pids, pres = _run(insts, reqs, routing=routing, trace_stride=7, trace_cap=4096)
    o = O.Oracle(insts[0], O.method(kind=O.TOPSIS, route_end=bool(routing)))
    st = lockstep(o, p, pids[0], reqs[0], pres, trace=trace_by_request(p), check_paths=True, check_alloc=True)
    assert st["accepted"] > 20 and st["rejected"] > 0 and st["scored_steps"] > 10
    assert sum(_short(r, pres[x], p, x)[0] for x, r in zip(pids[0], reqs[0]) if pres[x].status == 1) > 0
    others = [_run(insts, reqs, mode=dc.DC_MODE_BATCHED, routing=routing), _run(insts, reqs, routing=routing, grid=2)]
    sv = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING, routing=routing)
    sids = [sv.submit(r) for r in reqs[0]]
    others.append((sv, [sids], {r.req_id: r for r in sv.drain()}))
    for sched, ids, res in others:
        for x, y, req in zip(pids[0], ids[0], reqs[0]):
            assert res[y].status == pres[x].status and res[y].failed_at == pres[x].failed_at
            np.testing.assert_array_equal(res[y].hosts, pres[x].hosts)
            np.testing.assert_array_equal(res[y].scores.view(np.uint32), pres[x].scores.view(np.uint32))
            if pres[x].status == 1:
                np.testing.assert_array_equal(sched.paths(y), p.paths(x))
                for a, b in zip(sched.alloc(y, req.n, req.m), p.alloc(x, req.n, req.m)):
                    np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(sched.state(0), p.state(0))
        sched.close()
    p.close()


@pytest.mark.parametrize("mode", [dc.DC_MODE_PLAIN, dc.DC_MODE_BATCHED, dc.DC_MODE_SERVING])
def test_ranges_release_restores_state(mode):
    """Releasing every accepted request with intervals gives back exactly
    what each was given: the state returns to the initial one."""
    insts, reqs = make_config("ranges", seed=9, n_req=200)
    s = dc.Scheduler(insts, mode=mode)
    s0 = s.state(0).copy()
    ids = [s.submit(r) for r in reqs[0]]
    res = {r.req_id: r for r in (s.drain() if mode == dc.DC_MODE_SERVING else s.schedule())}
    acc = [x for x in ids if res[x].status == 1]
    assert len(acc) > 20 and not np.array_equal(s.state(0), s0)
    for x in acc:
        assert s.release(x) == 0
    if mode == dc.DC_MODE_SERVING:
        s.drain()
    np.testing.assert_array_equal(s.state(0), s0)
    s.close()


def test_equal_bounds_equal_fixed_demands():
    """Intervals with max = min schedule bit-identically to fixed demands."""
    insts, reqs = make_config("pods", seed=6, n_req=150)
    a, aids, ares = _run(insts, reqs)
    same = [Request(r.cpu, r.ram, r.edges, r.pod, r.cpu.copy(), r.ram.copy(), r.edges[:, 2].copy()) for r in reqs[0]]
    b, bids, bres = _run(insts, [same])
    for x, y, r in zip(aids[0], bids[0], reqs[0]):
        assert ares[x].status == bres[y].status
        np.testing.assert_array_equal(ares[x].hosts, bres[y].hosts)
        np.testing.assert_array_equal(ares[x].scores.view(np.uint32), bres[y].scores.view(np.uint32))
        if ares[x].status == 1:
            ca, ra, ba = b.alloc(y, r.n, r.m)
            np.testing.assert_array_equal(ca, r.cpu)
            np.testing.assert_array_equal(ra, r.ram)
            np.testing.assert_array_equal(ba, r.edges[:, 2])
    np.testing.assert_array_equal(a.state(0), b.state(0))
    a.close()
    b.close()


def test_ranges_invalid():
    insts, _ = make_config("tiny", seed=0)
    s = dc.Scheduler(insts)
    one = lambda **kw: Request(np.array([4, 4], np.int32), np.array([8, 8], np.int32),
                               np.array([[0, 1, 100]], np.int32), **kw)
    for bad in (one(cpu_max=np.array([3, 4], np.int32)), one(ram_max=np.array([8, 7], np.int32)),
                one(bw_max=np.array([99], np.int32)),
                one(cpu_max=np.array([1 << 21, (1 << 21) + 1], np.int32), pod=np.zeros(2, np.int32))):
        with pytest.raises(dc.DcError):
            s.submit(bad)
    rid = s.submit(one(cpu_max=np.array([6, 4], np.int32)))
    res = s.schedule()
    assert res[0].status == 1
    ca, ra, ba = s.alloc(rid, 2, 1)
    assert ca.tolist() == [6, 4] and ra.tolist() == [8, 8] and ba.tolist() == [100]
    with pytest.raises(dc.DcError):
        s.alloc(rid + 1, 2, 1)
    s.close()


def test_ranges_k48_cooperative_serving_and_plain():
    """k=48 (27,648 servers), pods and intervals: the cooperative serving
    kernel and the single-workgroup plain form give the same servers,
    scores, allocations and state; plain in lockstep with the oracle."""
    insts, reqs = make_config("ranges", seed=2, n_req=12, k=48)
    p, pids, pres = _run(insts, reqs, trace_stride=9, trace_cap=64)
    o = O.Oracle(insts[0], O.method(kind=O.TOPSIS))
    st = lockstep(o, p, pids[0], reqs[0], pres, trace=trace_by_request(p), check_paths=True, check_alloc=True)
    assert st["accepted"] >= 2 and st["scored_steps"] >= 1
    sv = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING)
    sids = [sv.submit(r) for r in reqs[0]]
    sres = {r.req_id: r for r in sv.drain()}
    for x, y, req in zip(pids[0], sids, reqs[0]):
        assert sres[y].status == pres[x].status and sres[y].failed_at == pres[x].failed_at
        np.testing.assert_array_equal(sres[y].hosts, pres[x].hosts)
        np.testing.assert_array_equal(sres[y].scores.view(np.uint32), pres[x].scores.view(np.uint32))
        if pres[x].status == 1:
            np.testing.assert_array_equal(sv.paths(y), p.paths(x))
            for a, b in zip(sv.alloc(y, req.n, req.m), p.alloc(x, req.n, req.m)):
                np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(sv.state(0), p.state(0))
    sv.close()
    p.close()
