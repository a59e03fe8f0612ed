"""GPU parity: the HIP path through the C ABI against the FP64 oracle, in
lockstep, on seeded synthetic fat-trees of the paper's shape."""
import numpy as np
import pytest

import oracle as O
from parity import lockstep, trace_by_request, TOL
from workloads import make_config, make_instance, make_requests, Request

pytestmark = pytest.mark.gpu

dc = pytest.importorskip("paper_1909_07673_amd")

C5 = (dc.DC_CRIT_CPU, dc.DC_CRIT_RAM, dc.DC_CRIT_UPLINK, dc.DC_CRIT_PATHBW, dc.DC_CRIT_HOPS)
C5_COST = (0, 0, 0, 0, 1)


def _omethod(method, crit=None, cost=None, scale=O.SAATY9):
    if crit is None:
        return O.method(kind=method, scale=scale)
    return O.method(kind=method, crit=crit, cost=list(cost), scale=scale)


def _run(insts, reqs, method=dc.DC_TOPSIS, mode=dc.DC_MODE_PLAIN, trace_stride=0, trace_cap=0, **kw):
    s = dc.Scheduler(insts, method=method, mode=mode, trace_stride=trace_stride, trace_cap=trace_cap, **kw)
    ids = [[s.submit(r, instance=i) for r in rl] for i, rl in enumerate(reqs)]
    res = {r.req_id: r for r in s.schedule()}
    return s, ids, res


@pytest.mark.parametrize("method", [dc.DC_TOPSIS, dc.DC_AHP])
def test_tiny_lockstep_many_seeds(method):
    """k=4, 16 hosts, no background, 20 requests of 2-6 containers: every
    step's score vector and every placement against the oracle."""
    tot = dict(steps=0, near_tie=0, rejected=0)
    for seed in range(40):
        insts, reqs = make_config("tiny", seed=seed)
        s = dc.Scheduler(insts, method=method, trace_stride=1, trace_cap=4096)
        o = O.Oracle(insts[0], _omethod(method))
        # one schedule call per request: the state is compared after each
        for req in reqs[0]:
            rid = s.submit(req)
            res = {r.req_id: r for r in s.schedule()}
            st = lockstep(o, s, [rid], [req], res, trace=trace_by_request(s), check_paths=True)
            assert st["scored_steps"] == st["steps"]
            for k in tot:
                tot[k] += st[k]
        s.close()
    assert tot["steps"] > 1000
    # exact ties (identical servers) must resolve to the lowest index on both
    # sides; near-ties in general are rare
    assert tot["near_tie"] <= tot["steps"] // 100


def test_plain_k16_prefix_every_step():
    """k=16 (1024 hosts), 0-70 % background: first 250 requests, every
    step's score vector compared."""
    insts, reqs = make_config("plain", seed=3, n_req=250)
    s, ids, res = _run(insts, reqs, trace_stride=1, trace_cap=8192)
    o = O.Oracle(insts[0], _omethod(O.TOPSIS))
    st = lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] == st["steps"] and st["steps"] > 2000
    assert st["accepted"] > 50 and st["rejected"] > 50


def test_plain_k16_full_size_sampled():
    """The full 2,000-request k=16 workload in the launch configuration the
    benchmark times: placements and state in lockstep for every request,
    score vectors on every 37th step."""
    insts, reqs = make_config("plain", seed=0)
    s, ids, res = _run(insts, reqs, trace_stride=37, trace_cap=4096)
    o = O.Oracle(insts[0], _omethod(O.TOPSIS))
    st = lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s))
    assert st["requests"] == 2000 and st["scored_steps"] > 300
    assert st["rejected"] > 0 and st["accepted"] > 0


def test_ahp_k16_every_step():
    insts, reqs = make_config("plain", seed=5, n_req=12)
    s, ids, res = _run(insts, reqs, method=dc.DC_AHP, trace_stride=1, trace_cap=1024)
    o = O.Oracle(insts[0], _omethod(O.AHP))
    st = lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] == st["steps"] > 20


def test_ahp_k32_five_criteria_sampled():
    """The large AHP shape: k=32 (8192 hosts), criteria CPU, RAM, uplink,
    path bandwidth, hops (cost), Saaty 1-9 scale; one request, every step."""
    insts, reqs = make_config("ahp", seed=0, n_req=1)
    req = reqs[0][0]
    req = Request(req.cpu[:6].copy(), req.ram[:6].copy(),
                  np.array([e for e in req.edges if e[0] < 6 and e[1] < 6], np.int32).reshape(-1, 3))
    s, ids, res = _run(insts, [[req]], method=dc.DC_AHP, crit=C5, cost=C5_COST, trace_stride=1, trace_cap=64)
    o = O.Oracle(insts[0], _omethod(O.AHP, crit=C5, cost=C5_COST))
    st = lockstep(o, s, ids[0], [req], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] == st["steps"] >= 1


def test_ahp_k32_full_requests_every_step():
    """The large AHP workload at its full size and in the benchmark's launch
    configuration: k=32 (8,192 servers, criteria over four workgroups), C=5
    with hops as a cost.  First the workload's first two requests whole (52
    and 61 containers; like most large requests of this workload they are
    rejected after 17-18 containers, once the uplinks of the servers
    holding the first ones cannot carry the traffic to the next), then a
    dense request of 28 light containers (every pair linked, 10-100 Mbps,
    1-2 cores), accepted, whose containers 17-27 have more placed peers than
    one peer chunk (16 at this size): the path tables are built in two
    chunks and the partial criteria carried between them.  Every step's
    score vector, placement, path and the state after each request against
    the oracle (threaded over the comparison matrices)."""
    insts, reqs = make_config("ahp", seed=0, n_req=2)
    rng = np.random.default_rng(32)
    dense = make_requests(1, rng, 28, 28, cpu_hi=2, ram_hi=4, bw_lo=10, bw_hi=100, density=1.0)[0]
    O.set_threads(0)
    s = dc.Scheduler(insts, method=dc.DC_AHP, crit=C5, cost=C5_COST, trace_stride=1, trace_cap=128)
    o = O.Oracle(insts[0], _omethod(O.AHP, crit=C5, cost=C5_COST))
    big = 0
    for req in reqs[0] + [dense]:
        rid = s.submit(req)
        res = {r.req_id: r for r in s.schedule()}
        st = lockstep(o, s, [rid], [req], res, trace=trace_by_request(s), check_paths=True)
        assert st["scored_steps"] == st["steps"] > 0
        peers = [sum(1 for e in req.edges if max(e[0], e[1]) == i) for i in range(req.n)]
        big += sum(p > 16 for p in peers[: st["steps"]])
    assert res[rid].status == 1 and big >= 11
    s.close()


@pytest.mark.parametrize("k", [20, 24, 34])
def test_ahp_saaty_sorted_and_pairwise_sizes(k):
    """The 1-9 scale through both forms of the column and row sums: k=20
    (2,000 hosts, not a multiple of the 256-thread block) and k=24 (3,456
    hosts) take the sorted passes, whose sorting network then holds 2 and 4
    slots per thread (k=16 and below: 1, k=32: 8); k=34 (9,826 hosts) is
    beyond their LDS limit of 8,192 hosts and takes the pairwise passes.
    One request of three containers (two at k=34, where the oracle takes
    about 5 s per step), every step and score vector against the oracle."""
    insts, reqs = make_config("ahp", seed=3, n_req=1, k=k)
    req, n = reqs[0][0], 2 if k == 34 else 3
    req = Request(req.cpu[:n].copy(), req.ram[:n].copy(),
                  np.array([e for e in req.edges if e[0] < n and e[1] < n], np.int32).reshape(-1, 3))
    s, ids, res = _run(insts, [[req]], method=dc.DC_AHP, crit=C5, cost=C5_COST, trace_stride=1, trace_cap=8)
    o = O.Oracle(insts[0], _omethod(O.AHP, crit=C5, cost=C5_COST))
    st = lockstep(o, s, ids[0], [req], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] == st["steps"] >= 1


def test_ahp_ratio_scale_priorities():
    """Ratio-scale AHP (consistent matrices): PG equals sum_c w_c v_c / sum(v_c)."""
    insts, reqs = make_config("tiny", seed=9)
    reqs = [reqs[0][:4]]          # few requests: every value stays positive
    s, ids, res = _run(insts, reqs, method=dc.DC_AHP, ahp_scale=dc.DC_AHP_RATIO,
                       crit=(dc.DC_CRIT_CPU, dc.DC_CRIT_RAM), trace_stride=1, trace_cap=512)
    o = O.Oracle(insts[0], O.method(kind=O.AHP, crit=(O.CRIT_CPU, O.CRIT_RAM), scale=O.RATIO))
    lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s))


def test_ahp_difference_scale_tiny_lockstep():
    """AHP on the difference scale of section V-B's rule: k=4, with and
    without pods, every step and score vector against the oracle."""
    tot = dict(steps=0, accepted=0)
    for seed in range(12):
        for preset in ("tiny", "tiny_pods"):
            insts, reqs = make_config(preset, seed=seed)
            s = dc.Scheduler(insts, method=dc.DC_AHP, ahp_scale=dc.DC_AHP_DIFF, trace_stride=1, trace_cap=4096)
            o = O.Oracle(insts[0], O.method(kind=O.AHP, scale=O.DIFF))
            for req in reqs[0]:
                rid = s.submit(req)
                res = {r.req_id: r for r in s.schedule()}
                st = lockstep(o, s, [rid], [req], res, trace=trace_by_request(s), check_paths=True)
                assert st["scored_steps"] == st["steps"]
                for k in tot:
                    tot[k] += st[k]
            s.close()
    assert tot["steps"] > 500 and tot["accepted"] > 100


def test_ahp_difference_scale_k16_and_k32():
    """Difference scale at k=16 (every step of a prefix, 0-70 % background)
    and at the k=32 five-criteria shape with hops as a cost (one request)."""
    insts, reqs = make_config("plain", seed=8, n_req=10)
    s, ids, res = _run(insts, reqs, method=dc.DC_AHP, ahp_scale=dc.DC_AHP_DIFF, trace_stride=1, trace_cap=1024)
    o = O.Oracle(insts[0], O.method(kind=O.AHP, scale=O.DIFF))
    st = lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] == st["steps"] > 20
    s.close()
    insts, reqs = make_config("ahp", seed=1, n_req=1)
    req = reqs[0][0]
    req = Request(req.cpu[:5].copy(), req.ram[:5].copy(),
                  np.array([e for e in req.edges if e[0] < 5 and e[1] < 5], np.int32).reshape(-1, 3))
    s, ids, res = _run(insts, [[req]], method=dc.DC_AHP, ahp_scale=dc.DC_AHP_DIFF, crit=C5, cost=C5_COST,
                       trace_stride=1, trace_cap=64)
    o = O.Oracle(insts[0], O.method(kind=O.AHP, crit=C5, cost=list(C5_COST), scale=O.DIFF))
    st = lockstep(o, s, ids[0], [req], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] == st["steps"] >= 1
    s.close()


def test_topsis_five_criteria_with_cost():
    insts, reqs = make_config("plain", seed=4, n_req=80)
    s, ids, res = _run(insts, reqs, crit=C5, cost=C5_COST, trace_stride=3, trace_cap=4096)
    o = O.Oracle(insts[0], _omethod(O.TOPSIS, crit=C5, cost=C5_COST))
    lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s), check_paths=True)


@pytest.mark.parametrize("method", [dc.DC_TOPSIS, dc.DC_AHP])
@pytest.mark.parametrize("w", [(0.17, 0.17, 0.5, 0.16), (0.17, 0.17, 0.16, 0.5)], ids=["clustering", "network"])
def test_table4_weight_scenarios(method, w):
    """Table IV 'Clustering' and 'Network' weights (CPU, RAM, fragmentation,
    bandwidth) with TOPSIS (k=16) and AHP (k=4, every step)."""
    if method == dc.DC_TOPSIS:
        insts, reqs = make_config("plain", seed=6, n_req=80)
        stride = 5
    else:
        insts, reqs = make_config("tiny", seed=6)
        stride = 1
    s, ids, res = _run(insts, reqs, method=method, weight=w, trace_stride=stride, trace_cap=4096)
    o = O.Oracle(insts[0], O.method(kind=method, weight=list(w)))
    st = lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] > 0


def test_batched_matches_oracle_and_plain():
    """Batched form (one persistent launch, state in LDS) against the oracle
    per instance, and bit-identical to the plain form on each instance."""
    insts, reqs = make_config("batched", seed=2, instances=6, n_req=40)
    s, ids, res = _run(insts, reqs, mode=dc.DC_MODE_BATCHED)
    for i in range(len(insts)):
        o = O.Oracle(insts[i], _omethod(O.TOPSIS))
        lockstep(o, s, ids[i], reqs[i], res, instance=i, check_paths=True)
        p, pids, pres = _run([insts[i]], [reqs[i]])
        for a, b in zip(ids[i], pids[0]):
            assert res[a].status == pres[b].status
            np.testing.assert_array_equal(res[a].hosts, pres[b].hosts)
            np.testing.assert_array_equal(res[a].scores, pres[b].scores)
        np.testing.assert_array_equal(s.state(i), p.state(0))
        p.close()


def test_batched_256_instances_sampled():
    """256 instances of k=16 with uneven request counts in one launch;
    sampled instances replayed by the oracle."""
    insts, reqs = make_config("batched", seed=4)
    reqs = [rl[: 8 + (i % 5) * 6] for i, rl in enumerate(reqs)]
    s, ids, res = _run(insts, reqs, mode=dc.DC_MODE_BATCHED)
    for i in (0, 77, 128, 255):
        o = O.Oracle(insts[i], _omethod(O.TOPSIS))
        lockstep(o, s, ids[i], reqs[i], res, instance=i)
    for i in range(len(insts)):
        assert s.state(i).min() >= 0


def test_batched_full_workload_instances():
    """The batched workload at its full size, in the benchmark's launch
    configuration (256 instances, every request, autotuned workgroup, HIP
    graph): the instance with the most container steps, the one with the
    fewest and two more replayed whole by the oracle in lockstep, with the
    state after the last request."""
    insts, reqs = make_config("batched", seed=0)
    s = dc.Scheduler(insts, mode=dc.DC_MODE_BATCHED)
    ids = [[s.submit(r, instance=i) for r in rl] for i, rl in enumerate(reqs)]
    s.autotune()
    res = {r.req_id: r for r in s.schedule()}
    steps = np.array([sum(res[q].n if res[q].status == 1 else res[q].failed_at + 1 for q in ids[i])
                      for i in range(len(insts))])
    pick = [int(steps.argmax()), int(steps.argmin()), 1, 200]
    assert steps.max() > 5000
    for i in pick:
        o = O.Oracle(insts[i], _omethod(O.TOPSIS))
        st = lockstep(o, s, ids[i], reqs[i], res, instance=i, check_paths=(i == pick[0]))
        assert st["steps"] == steps[i] and st["requests"] == len(reqs[i])
        o.close()
    s.close()


def test_autotune_keeps_results():
    insts, reqs = make_config("batched", seed=8, instances=4, n_req=20)
    s = dc.Scheduler(insts, mode=dc.DC_MODE_BATCHED)
    ids = [[s.submit(r, instance=i) for r in rl] for i, rl in enumerate(reqs)]
    bs = s.autotune()
    assert bs in (256, 512, 1024)
    res = {r.req_id: r for r in s.schedule()}
    s.rewind()
    res2 = {r.req_id: r for r in s.schedule()}
    for k in res:
        np.testing.assert_array_equal(res[k].hosts, res2[k].hosts)
    for i in range(len(insts)):
        o = O.Oracle(insts[i], _omethod(O.TOPSIS))
        lockstep(o, s, ids[i], reqs[i], res2, instance=i)


def test_release_restores_state_and_paths():
    insts, reqs = make_config("plain", seed=7, n_req=150)
    s, ids, res = _run(insts, reqs)
    s0 = dc.Scheduler(insts).state(0)
    o = O.Oracle(insts[0], _omethod(O.TOPSIS))
    lockstep(o, s, ids[0], reqs[0], res, check_paths=True)
    acc = [rid for rid in ids[0] if res[rid].status == 1]
    rej = [rid for rid in ids[0] if res[rid].status == 0]
    rng = np.random.default_rng(0)
    for rid in rng.permutation(acc):
        assert s.release(int(rid)) == dc.DC_OK
    np.testing.assert_array_equal(s.state(0), s0)
    assert s.release(int(acc[0])) == dc.DC_ENOENT
    if rej:
        assert s.release(int(rej[0])) == dc.DC_ENOENT
    assert s.release(10 ** 9) == dc.DC_ENOENT


def test_rewind_is_deterministic():
    insts, reqs = make_config("plain", seed=11, n_req=300)
    s, ids, res = _run(insts, reqs)
    st1 = s.state(0)
    s.rewind()
    res2 = {r.req_id: r for r in s.schedule()}
    np.testing.assert_array_equal(s.state(0), st1)
    for k in res:
        assert res[k].status == res2[k].status
        np.testing.assert_array_equal(res[k].hosts, res2[k].hosts)
        np.testing.assert_array_equal(res[k].scores.view(np.uint32), res2[k].scores.view(np.uint32))


def test_edge_cases():
    rng = np.random.default_rng(3)
    inst = make_instance(4, 32, 256, 10000, 10000, 10000)
    one = Request(np.array([4], np.int32), np.array([8], np.int32), np.zeros((0, 3), np.int32))
    noedge = Request(np.array([1, 2, 3], np.int32), np.array([1, 1, 1], np.int32), np.zeros((0, 3), np.int32))
    huge = Request(np.array([33], np.int32), np.array([1], np.int32), np.zeros((0, 3), np.int32))
    fat = Request(np.array([1, 1], np.int32), np.array([1, 1], np.int32), np.array([[0, 1, 10001]], np.int32))
    zero = Request(np.array([0, 0], np.int32), np.array([0, 0], np.int32), np.array([[0, 1, 5]], np.int32))
    reqs = [one, noedge, huge, fat, zero] + make_requests(60, rng, 2, 6, cpu_hi=16)   # saturates k=4
    s, ids, res = _run([inst], [reqs])
    assert res[ids[0][2]].status == 0 and res[ids[0][2]].failed_at == 0
    o = O.Oracle(inst, _omethod(O.TOPSIS))
    st = lockstep(o, s, ids[0], reqs, res, check_paths=True)
    assert st["rejected"] >= 5
    # 64 containers on k=16
    insts, _ = make_config("plain", seed=1, n_req=1)
    big = make_requests(1, rng, 64, 64)[0]
    s2, ids2, res2 = _run(insts, [[big]])
    o2 = O.Oracle(insts[0], _omethod(O.TOPSIS))
    lockstep(o2, s2, ids2[0], [big], res2, check_paths=True)


def test_invalid_arguments():
    inst = make_instance(4, 32, 256, 10000, 10000, 10000)
    with pytest.raises(dc.DcError) as e:
        dc.Scheduler([inst], weight=(0.5, 0.5, 0.5, 0.5))
    assert e.value.code == dc.DC_EINVAL
    with pytest.raises(dc.DcError):
        dc.Scheduler([inst], method=dc.DC_AHP, mode=dc.DC_MODE_BATCHED)
    s = dc.Scheduler([inst])
    bad = [Request(np.ones(2, np.int32), np.ones(2, np.int32), np.array([[0, 0, 5]], np.int32)),
           Request(np.ones(2, np.int32), np.ones(2, np.int32), np.array([[0, 1, 0]], np.int32)),
           Request(np.ones(2, np.int32), np.ones(2, np.int32), np.array([[0, 1, 5], [1, 0, 5]], np.int32)),
           Request(np.ones(65, np.int32), np.ones(65, np.int32), np.zeros((0, 3), np.int32))]
    for r in bad:
        with pytest.raises(dc.DcError) as e:
            s.submit(r)
        assert e.value.code == dc.DC_EINVAL
    with pytest.raises(dc.DcError):
        s.submit(bad[0], instance=3)


# ---------------------------------------------------------------- cooperative step
@pytest.mark.parametrize("seed", range(12))
def test_grid_tiny_lockstep(seed):
    """One cooperative workgroup per pod (k=4: four workgroups), forced on
    the small case: every step's score vector against the oracle."""
    insts, reqs = make_config("tiny", seed=seed)
    s = dc.Scheduler(insts, grid=2, trace_stride=1, trace_cap=4096)
    o = O.Oracle(insts[0], _omethod(O.TOPSIS))
    for req in reqs[0]:
        rid = s.submit(req)
        res = {r.req_id: r for r in s.schedule()}
        st = lockstep(o, s, [rid], [req], res, trace=trace_by_request(s), check_paths=True)
        assert st["scored_steps"] == st["steps"]
    s.close()


def test_grid_k16_matches_single_workgroup():
    """k=16 with one workgroup per pod: bit-identical to the single-workgroup
    step, and in lockstep with the oracle on every step's scores."""
    insts, reqs = make_config("plain", seed=3, n_req=200)
    g, gids, gres = _run(insts, reqs, grid=2, trace_stride=1, trace_cap=8192)
    p, pids, pres = _run(insts, reqs, grid=1)
    for a, b in zip(gids[0], pids[0]):
        assert gres[a].status == pres[b].status
        np.testing.assert_array_equal(gres[a].hosts, pres[b].hosts)
        np.testing.assert_array_equal(gres[a].scores.view(np.uint32), pres[b].scores.view(np.uint32))
    np.testing.assert_array_equal(g.state(0), p.state(0))
    o = O.Oracle(insts[0], _omethod(O.TOPSIS))
    st = lockstep(o, g, gids[0], reqs[0], gres, trace=trace_by_request(g), check_paths=True)
    assert st["scored_steps"] == st["steps"]


def test_grid_k48_sampled():
    """k=48 (27,648 hosts) on the cooperative step (grid = 2: 48
    workgroups, one per pod): a prefix in lockstep, score vectors on sampled
    steps."""
    insts, reqs = make_config("serving", seed=1, n_req=6)
    s, ids, res = _run(insts, reqs, grid=2, trace_stride=7, trace_cap=64)
    o = O.Oracle(insts[0], _omethod(O.TOPSIS))
    st = lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] >= 1


def test_schedule_array_matches_schedule():
    """The bulk result path returns the same records as the per-result one."""
    insts, reqs = make_config("batched", seed=2, instances=4)
    a, _, res = _run(insts, reqs, mode=dc.DC_MODE_BATCHED)
    b = dc.Scheduler(insts, mode=dc.DC_MODE_BATCHED)
    for i, rl in enumerate(reqs):
        for r in rl:
            b.submit(r, instance=i)
    arr = b.schedule_array()
    assert len(arr) == len(res)
    for row in arr:
        r = res[int(row["req_id"])]
        assert (row["instance"], row["status"], row["n"], row["failed_at"]) == (r.instance, r.status, r.n, r.failed_at)
        np.testing.assert_array_equal(row["host"][: r.n], r.hosts)
        np.testing.assert_array_equal(row["score"][: r.n].view(np.uint32), r.scores.view(np.uint32))
    a.close()
    b.close()


def test_batched_graph_replays_match_direct_launches():
    """Batched form: the launch captured in a HIP graph, replayed after each
    rewind (with the rewind's eager copies and fills in between), gives the
    same results and state as direct launches, on every replay."""
    insts, reqs = make_config("batched", seed=5, instances=6)

    def runs(graph):
        s = dc.Scheduler(insts, mode=dc.DC_MODE_BATCHED, graph=graph)
        for i, rl in enumerate(reqs):
            for r in rl:
                s.submit(r, instance=i)
        out = []
        for rep in range(4):
            if rep:
                s.rewind()
            arr = s.schedule_array()
            out.append((arr.copy(), np.stack([s.state(i) for i in range(len(insts))])))
        s.close()
        return out

    direct, graphed = runs(1), runs(2)
    for (a, sa), (b, sb) in zip(direct, graphed):
        assert a.tobytes() == b.tobytes()
        np.testing.assert_array_equal(sa, sb)
    for a, sa in direct[1:]:
        assert a.tobytes() == direct[0][0].tobytes()


@pytest.mark.parametrize("mode", [dc.DC_MODE_PLAIN, dc.DC_MODE_BATCHED, dc.DC_MODE_SERVING])
def test_rejected_results_place_nothing(mode):
    """A rejected request's result holds -1 for every container and names
    the first container with no server; its attempt stays readable; an
    accepted one holds a server for every container."""
    insts, reqs = make_config("plain", seed=8, n_req=300)
    s = dc.Scheduler(insts, mode=mode)
    ids = [s.submit(r) for r in reqs[0]]
    res = {r.req_id: r for r in (s.drain() if mode == dc.DC_MODE_SERVING else s.schedule())}
    assert len(res) == len(ids)
    rejected = 0
    for rid in ids:
        r = res[rid]
        if r.status:
            assert r.failed_at == -1 and np.all(r.hosts >= 0)
        else:
            rejected += 1
            assert 0 <= r.failed_at < r.n and np.all(r.hosts == -1)
            att = s.attempt(rid)
            assert np.all(att[: r.failed_at] >= 0) and np.all(att[r.failed_at:] == -1)
    assert rejected > 0
    s.close()


@pytest.mark.parametrize("mode", [dc.DC_MODE_PLAIN, dc.DC_MODE_SERVING])
def test_grid_barrier_timeout_is_reported(mode):
    """The cooperative step's barrier waits are bounded: with the limit forced
    down to 1 us from the host, the barriers give up, every workgroup leaves
    normally, and the context reports DC_EDEVICE from then on.  A fresh
    context on the same device then schedules the same requests correctly."""
    insts, reqs = make_config("serving", seed=4, n_req=8)
    s = dc.Scheduler(insts, mode=mode, grid=2, grid_timeout_us=1)
    with pytest.raises(dc.DcError) as e:
        if mode == dc.DC_MODE_SERVING:
            for r in reqs[0]:
                s.submit(r)
            s.drain(timeout_s=30.0)
        else:
            for r in reqs[0]:
                s.submit(r)
            s.schedule()
    assert e.value.code == dc.DC_EDEVICE
    with pytest.raises(dc.DcError):
        s.submit(reqs[0][0])
    s.close()
    a, ids, res = _run(insts, reqs, grid=2)
    b, ids2, res2 = _run(insts, reqs, grid=1)
    for x, y in zip(ids[0], ids2[0]):
        assert res[x].status == res2[y].status
        np.testing.assert_array_equal(res[x].hosts, res2[y].hosts)
    a.close()
    b.close()


# ---------------------------------------------------------------- pods
@pytest.mark.parametrize("method", [dc.DC_TOPSIS, dc.DC_AHP])
def test_pods_tiny_lockstep(method):
    """k=4 requests with pods (up to half the containers in pods of 2-4):
    every step (one per pod) against the oracle, score vectors included."""
    tot = dict(steps=0, accepted=0, rejected=0)
    for seed in range(20):
        insts, reqs = make_config("tiny_pods", seed=seed)
        s = dc.Scheduler(insts, method=method, trace_stride=1, trace_cap=4096)
        o = O.Oracle(insts[0], _omethod(method))
        for req in reqs[0]:
            rid = s.submit(req)
            res = {r.req_id: r for r in s.schedule()}
            st = lockstep(o, s, [rid], [req], res, trace=trace_by_request(s), check_paths=True)
            assert st["scored_steps"] == st["steps"]
            for k in tot:
                tot[k] += st[k]
        s.close()
    assert tot["accepted"] > 50 and tot["steps"] > 100


def test_pods_k16_plain_batched_serving():
    """k=16 with pods: plain in lockstep with the oracle (paths and final
    state), batched and serving bit-identical to plain."""
    insts, reqs = make_config("pods", seed=2, n_req=250)
    assert sum(r.pod is not None and (r.pod >= 0).any() for r in reqs[0]) > 50
    p, pids, pres = _run(insts, reqs, trace_stride=5, trace_cap=4096)
    o = O.Oracle(insts[0], _omethod(dc.DC_TOPSIS))
    st = lockstep(o, p, pids[0], reqs[0], pres, trace=trace_by_request(p), check_paths=True)
    assert st["accepted"] > 20 and st["rejected"] > 0 and st["scored_steps"] > 10
    b, bids, bres = _run(insts, reqs, mode=dc.DC_MODE_BATCHED)
    sv = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING)
    sids = [sv.submit(r) for r in reqs[0]]
    sres = {r.req_id: r for r in sv.drain()}
    for x, y, z in zip(pids[0], bids[0], sids):
        for other in (bres[y], sres[z]):
            assert other.status == pres[x].status and other.failed_at == pres[x].failed_at
            np.testing.assert_array_equal(other.hosts, pres[x].hosts)
            np.testing.assert_array_equal(other.scores.view(np.uint32), pres[x].scores.view(np.uint32))
    np.testing.assert_array_equal(b.state(0), p.state(0))
    np.testing.assert_array_equal(sv.state(0), p.state(0))
    for x, z in zip(pids[0], sids):
        if pres[x].status == 1:
            np.testing.assert_array_equal(sv.paths(z), p.paths(x))
    for sched in (p, b, sv):
        sched.close()


def test_pods_invalid():
    insts, _ = make_config("tiny", seed=0)
    s = dc.Scheduler(insts)
    big = Request(np.full(4, 1 << 21, np.int32), np.ones(4, np.int32), np.zeros((0, 3), np.int32),
                  np.zeros(4, np.int32))
    with pytest.raises(dc.DcError):
        s.submit(big)          # summed CPU of the pod beyond 2^22
    s.close()


def _ft_link_hops(paths):
    return int((paths >= 0).sum())


@pytest.mark.parametrize("wl", ["ahp", "plain", "pods", "pods_route_end", "ranges"])
def test_full_size_accounting(wl):
    """The measured configurations at full size (AHP k=32 with 500 requests,
    TOPSIS k=16 with 2,000 requests, with and without pods, with pods and
    links routed at each request's end, and with pods and demand
    intervals), checked by properties that hold at any size: the state
    change equals the accepted placements (CPU, RAM, placed counts per
    server) and their routes (link usage = summed demand x hops; with
    intervals, what was given, each within [min, max], and short of the
    maximum only where the server's resource ran out), nothing goes
    negative, and releasing every accepted request restores the initial
    state bit-exactly."""
    kw = {}
    if wl == "pods_route_end":
        wl = "pods"
        kw = dict(routing=dc.DC_ROUTE_END)
    insts, reqs = make_config(wl, seed=0)
    if wl == "ahp":
        kw = dict(method=dc.DC_AHP, crit=C5, cost=C5_COST)
    s = dc.Scheduler(insts, **kw)
    s0 = s.state(0).astype(np.int64)
    ids = [s.submit(r) for r in reqs[0]]
    res = {r.req_id: r for r in s.schedule()}
    s1 = s.state(0).astype(np.int64)
    assert np.all(s1 >= 0)
    N = insts[0].n_hosts
    cpu = np.zeros(N, np.int64)
    ram = np.zeros(N, np.int64)
    npl = np.zeros(N, np.int64)
    hops_bw = 0
    acc, short_c, short_r = [], [], []
    for rid, req in zip(ids, reqs[0]):
        r = res[rid]
        if r.status != 1:
            assert np.all(r.hosts == -1)
            continue
        acc.append(rid)
        ca, ra, ba = req.cpu, req.ram, req.edges[:, 2]
        if req.cpu_max is not None:
            ca, ra, ba = s.alloc(rid, req.n, req.m)
            assert np.all((req.cpu <= ca) & (ca <= req.cpu_max)) and np.all((req.ram <= ra) & (ra <= req.ram_max))
            assert np.all((req.edges[:, 2] <= ba) & (ba <= req.bw_max))
            short_c.extend(r.hosts[ca < req.cpu_max].tolist())
            short_r.extend(r.hosts[ra < req.ram_max].tolist())
        np.add.at(cpu, r.hosts, ca)
        np.add.at(ram, r.hosts, ra)
        if getattr(req, "pod", None) is None:
            np.add.at(npl, r.hosts, 1)
        else:
            unit, first = O.units(req.n, req.pod)
            np.add.at(npl, r.hosts[first], 1)
            for g in range(len(first)):
                assert np.all(r.hosts[unit == g] == r.hosts[first[g]])
        # demand per routed pair, in the paths' order
        unit, first = O.units(req.n, getattr(req, "pod", None))
        dem = {}
        for (a, b, _), bw in zip(req.edges, ba):
            ua, ub = unit[a], unit[b]
            if ua != ub:
                key = (max(ua, ub), min(ua, ub))
                dem[key] = dem.get(key, 0) + int(bw)
        paths = s.paths(rid)
        assert len(paths) == len(dem)
        for key, p in zip(sorted(dem), paths):
            hops_bw += dem[key] * _ft_link_hops(p)
    assert len(acc) > 10
    np.testing.assert_array_equal(s0[0] - s1[0], cpu)
    np.testing.assert_array_equal(s0[1] - s1[1], ram)
    np.testing.assert_array_equal(s1[2] - s0[2], npl)
    assert int((s0[3:] - s1[3:]).sum()) == hops_bw
    assert np.all(s1[0][short_c] == 0) and np.all(s1[1][short_r] == 0)
    if wl == "ranges":
        assert len(short_c) + len(short_r) > 0
    for rid in acc:
        assert s.release(rid) == dc.DC_OK
    np.testing.assert_array_equal(s.state(0), s0)
    s.close()


# ---------------------------------------------------------------- routing at the end of a request
@pytest.mark.parametrize("method", [dc.DC_TOPSIS, dc.DC_AHP])
def test_route_end_tiny_lockstep(method):
    """Links routed after the last container (section V-D): k=4, every step
    and every routed path against the oracle, with and without pods."""
    tot = dict(accepted=0, rejected=0, steps=0)
    for seed in range(16):
        for preset in ("tiny", "tiny_pods"):
            insts, reqs = make_config(preset, seed=seed)
            s = dc.Scheduler(insts, method=method, routing=dc.DC_ROUTE_END, trace_stride=1, trace_cap=4096)
            o = O.Oracle(insts[0], O.method(kind=method, route_end=True))
            for req in reqs[0]:
                rid = s.submit(req)
                res = {r.req_id: r for r in s.schedule()}
                st = lockstep(o, s, [rid], [req], res, trace=trace_by_request(s), check_paths=True)
                for k in tot:
                    tot[k] += st[k]
            s.close()
    assert tot["accepted"] > 100 and tot["steps"] > 300


def test_route_end_k16_forms_agree():
    """k=16, routing at the end: plain in lockstep with the oracle (some
    requests rejected because their links do not fit); batched, serving and
    the cooperative step bit-identical to plain."""
    insts, reqs = make_config("plain", seed=12, n_req=250)
    p, pids, pres = _run(insts, reqs, routing=dc.DC_ROUTE_END, trace_stride=7, trace_cap=4096)
    o = O.Oracle(insts[0], O.method(kind=O.TOPSIS, route_end=True))
    st = lockstep(o, p, pids[0], reqs[0], pres, trace=trace_by_request(p), check_paths=True)
    assert st["accepted"] > 20 and st["scored_steps"] > 10
    n = {x: r.n for x, r in zip(pids[0], reqs[0])}
    assert any(pres[x].status == 0 and pres[x].failed_at == n[x] for x in pids[0])
    others = [_run(insts, reqs, mode=dc.DC_MODE_BATCHED, routing=dc.DC_ROUTE_END),
              _run(insts, reqs, routing=dc.DC_ROUTE_END, grid=2)]
    sv = dc.Scheduler(insts, mode=dc.DC_MODE_SERVING, routing=dc.DC_ROUTE_END)
    sids = [sv.submit(r) for r in reqs[0]]
    others.append((sv, [sids], {r.req_id: r for r in sv.drain()}))
    for sched, ids, res in others:
        for x, y in zip(pids[0], ids[0]):
            assert res[y].status == pres[x].status and res[y].failed_at == pres[x].failed_at
            np.testing.assert_array_equal(res[y].hosts, pres[x].hosts)
            np.testing.assert_array_equal(res[y].scores.view(np.uint32), pres[x].scores.view(np.uint32))
            if pres[x].status == 1:
                np.testing.assert_array_equal(sched.paths(y), p.paths(x))
        np.testing.assert_array_equal(sched.state(0), p.state(0))
        sched.close()
    p.close()


def test_route_end_k48_cooperative_sampled():
    """k=48 on the cooperative step (grid = 2; workgroup 0 routes the
    request's links): lockstep on a prefix, score vectors sampled."""
    insts, reqs = make_config("serving", seed=3, n_req=6)
    s, ids, res = _run(insts, reqs, grid=2, routing=dc.DC_ROUTE_END, trace_stride=5, trace_cap=64)
    o = O.Oracle(insts[0], O.method(kind=O.TOPSIS, route_end=True))
    st = lockstep(o, s, ids[0], reqs[0], res, trace=trace_by_request(s), check_paths=True)
    assert st["scored_steps"] >= 1
    s.close()
