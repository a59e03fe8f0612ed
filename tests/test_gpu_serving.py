"""Serving form on the GPU: continuous batching over a device-resident data
center.  Each request's result is the same alone and in the mix; lockstep
parity with the oracle over interleaved requests and departures; memory
admission; release."""
import numpy as np
import pytest

import oracle as O
from parity import lockstep, TOL
from workloads import make_config, make_requests, make_trace

pytestmark = pytest.mark.gpu

dc = pytest.importorskip("paper_1909_07673_amd")


def _commands(reqs, lag=15):
    """Command sequence: submit request t, then depart request t - lag
    (if it was accepted)."""
    cmds = []
    for t in range(len(reqs)):
        cmds.append(("submit", t))
        if t >= lag and t % 2 == 0:
            cmds.append(("release", t - lag))
    return cmds


def _replay(s, reqs, cmds, alone):
    """Runs the command sequence; alone=True waits for every command to
    complete before the next, otherwise submissions stay in flight."""
    ids, res = {}, {}

    def absorb(rs):
        for r in rs:
            res[r.req_id] = r

    for kind, t in cmds:
        if kind == "submit":
            while True:
                rid = s.try_submit(reqs[t])
                if rid is not None:
                    break
                absorb(s.schedule())
            ids[t] = rid
        else:
            rid = ids[t]
            while rid not in res:            # the departure needs the decision
                absorb(s.schedule())
            if res[rid].status == 1:
                assert s.release(rid) == dc.DC_OK
        if alone:
            absorb(s.drain())
    absorb(s.drain())
    return ids, res


def _k16(preset="plain"):
    insts, reqs = make_config(preset, seed=21, n_req=160)
    return insts, reqs[0]


@pytest.mark.parametrize("grid,preset,routing", [(1, "plain", 0), (2, "plain", 0), (1, "pods", 1), (2, "pods", 0)])
def test_serving_alone_equals_mix_and_oracle(grid, preset, routing):
    """Each request's result is the same alone and in the mix (single
    workgroup against the cooperative kernel), and in lockstep with the
    oracle over interleaved requests and departures; also with pods and with
    links routed at the end of each request."""
    insts, reqs = _k16(preset)
    cmds = _commands(reqs)
    mix = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING, grid=grid, routing=routing)
    ids_m, res_m = _replay(mix, reqs, cmds, alone=False)
    alone = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING, grid=3 - grid, routing=routing)
    ids_a, res_a = _replay(alone, reqs, cmds, alone=True)
    for t in range(len(reqs)):
        a, b = res_m[ids_m[t]], res_a[ids_a[t]]
        assert (a.status, a.failed_at) == (b.status, b.failed_at), t
        np.testing.assert_array_equal(a.hosts, b.hosts)
        np.testing.assert_array_equal(a.scores.view(np.uint32), b.scores.view(np.uint32))
    np.testing.assert_array_equal(mix.state(0), alone.state(0))
    # the oracle replays the same commands in the same order
    o = O.Oracle(insts[0], O.method(kind=O.TOPSIS, route_end=bool(routing)))
    rec = {}
    for kind, t in cmds:
        if kind == "submit":
            st = lockstep(o, mix, [ids_m[t]], [reqs[t]], res_m, check_paths=False, final_state=False)
            rec[t] = st["rec_ids"][0]
        elif res_m[ids_m[t]].status == 1:
            assert o.release(rec[t]) == 0
    np.testing.assert_array_equal(mix.state(0), o.state())
    acc = sum(r.status for r in res_m.values())
    assert 0 < acc < len(reqs)
    mix.close()
    alone.close()


def test_serving_admission_by_memory():
    insts, reqs = _k16()
    s = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING, mem_budget=48 * 1024)
    refused = 0
    live = []
    done = {}
    for req in reqs[:80]:
        while True:
            rid = s.try_submit(req)
            if rid is not None:
                live.append(rid)
                break
            refused += 1
            for r in s.schedule():
                done[r.req_id] = r
                if r.status == 1:          # depart at once: frees its slot
                    assert s.release(r.req_id) == dc.DC_OK
    for r in s.drain():
        done[r.req_id] = r
        if r.status == 1:
            assert s.release(r.req_id) == dc.DC_OK
    s.drain()
    assert refused > 0 and len(done) == 80
    np.testing.assert_array_equal(s.state(0), dc.Scheduler(insts).state(0))


def test_serving_release_rules():
    insts, reqs = _k16()
    s = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING)
    rid = s.submit(reqs[0])
    res = {r.req_id: r for r in s.drain()}
    if res[rid].status == 1:
        assert s.release(rid) == dc.DC_OK
        assert s.release(rid) == dc.DC_ENOENT
    else:
        assert s.release(rid) == dc.DC_ENOENT
    assert s.release(12345) == dc.DC_ENOENT
    s.drain()


def test_serving_k48_sampled():
    """The serving workload's data center: k=48 (27,648 hosts), 0-70 %
    background; a few requests in lockstep with the oracle."""
    insts, _ = make_config("serving", seed=3, n_req=1)
    rng = np.random.default_rng(5)
    reqs = make_requests(4, rng, 2, 10)
    s = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING)
    ids = [s.submit(r) for r in reqs]
    res = {r.req_id: r for r in s.drain()}
    o = O.Oracle(insts[0], O.method(kind=O.TOPSIS))
    lockstep(o, s, ids, reqs, res, check_paths=True)


def test_serving_k48_trace_prefix_alone_equals_mix_and_oracle():
    """The serving workload's shape at full size: k=48 (27,648 servers,
    0-70 % background), the first 120 requests of the Poisson trace (2-64
    containers), every second one after the 15th followed by the departure
    of the request 15 before it (a departure of a rejected request is
    skipped).  The cooperative serving kernel (one
    workgroup per pod, the default at this size) with commands in flight
    against the single-workgroup kernel one command at a time: identical
    results and state; and the oracle, replaying the same commands, in
    lockstep with every request and the state at the end."""
    insts, _ = make_config("serving", seed=0, n_req=1)
    reqs, _, _ = make_trace(seed=0, duration_s=0.05)
    reqs = reqs[:120]
    cmds = _commands(reqs)
    assert sum(1 for c in cmds if c[0] == "release") >= 50
    mix = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING)
    ids_m, res_m = _replay(mix, reqs, cmds, alone=False)
    alone = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING, grid=1)
    ids_a, res_a = _replay(alone, reqs, cmds, alone=True)
    for t in range(len(reqs)):
        a, b = res_m[ids_m[t]], res_a[ids_a[t]]
        assert (a.status, a.failed_at) == (b.status, b.failed_at), t
        np.testing.assert_array_equal(a.hosts, b.hosts)
        np.testing.assert_array_equal(a.scores.view(np.uint32), b.scores.view(np.uint32))
    np.testing.assert_array_equal(mix.state(0), alone.state(0))
    alone.close()
    o = O.Oracle(insts[0], O.method(kind=O.TOPSIS))
    departed = {t for kind, t in cmds if kind == "release"}
    rec, steps = {}, 0
    for kind, t in cmds:
        if kind == "submit":
            # a departed request holds no links any more: its paths are checked
            # only while it is live, i.e. for the requests that never depart
            st = lockstep(o, mix, [ids_m[t]], [reqs[t]], res_m, check_paths=t not in departed,
                          final_state=False)
            rec[t] = st["rec_ids"][0]
            steps += st["steps"]
        elif res_m[ids_m[t]].status == 1:
            assert o.release(rec[t]) == 0
    np.testing.assert_array_equal(mix.state(0), o.state())
    # large requests on 0-70 % loaded 40 Gbps uplinks: most are rejected,
    # many of them once a later container's peers share a server whose
    # uplink cannot carry their summed demand
    accepted = sum(r.status for r in res_m.values())
    released = sum(1 for kind, t in cmds if kind == "release" and res_m[ids_m[t]].status == 1)
    assert steps > 1000 and accepted >= 15 and released >= 5, (steps, accepted, released)
    mix.close()
