"""GPU selection on a hand-made k = 4 data center where the best-scored
server for a container passes every check made before scoring but fails
its joint commit (two paths through one edge switch uplink that carries
either alone), so the selection must mask it and take the next server
(section V-C, Eqs. (4)-(5)).  Every form runs the case, in lockstep with
the oracle, with every step's score vector compared; a control data center
with the same per-peer checks, where both paths fit, keeps the container
on the best server."""
import numpy as np
import pytest

import oracle as O
from parity import lockstep, trace_by_request
from select_cases import REQ, REQ_CUT, empty, loaded, peer_cut, split_fits
from workloads import Request

pytestmark = pytest.mark.gpu

dc = pytest.importorskip("paper_1909_07673_amd")

CPU_ONLY = dict(crit=(dc.DC_CRIT_CPU,), weight=(1.0,))

# (name, method, mode, grid): single workgroup, cooperative (one workgroup
# per pod), batched, serving with one workgroup and cooperative, AHP
FORMS = [("plain", dc.DC_TOPSIS, dc.DC_MODE_PLAIN, 1),
         ("plain_grid", dc.DC_TOPSIS, dc.DC_MODE_PLAIN, 2),
         ("batched", dc.DC_TOPSIS, dc.DC_MODE_BATCHED, 0),
         ("serving", dc.DC_TOPSIS, dc.DC_MODE_SERVING, 1),
         ("serving_grid", dc.DC_TOPSIS, dc.DC_MODE_SERVING, 2),
         ("ahp", dc.DC_AHP, dc.DC_MODE_PLAIN, 0)]


def _schedule(s, reqs, mode):
    ids = [s.submit(r) for r in reqs]
    res = s.drain() if mode == dc.DC_MODE_SERVING else s.schedule()
    return ids, {r.req_id: r for r in res}


@pytest.mark.parametrize("name,method,mode,grid", FORMS, ids=[f[0] for f in FORMS])
@pytest.mark.parametrize("case,want", [(loaded, [0, 4, 12]), (split_fits, [0, 4, 8])],
                         ids=["commit_fails", "control"])
def test_failed_commit_takes_next_server(name, method, mode, grid, case, want):
    inst = case()
    trace = mode != dc.DC_MODE_SERVING
    s = dc.Scheduler([inst], method=method, mode=mode, grid=grid, trace_stride=1 if trace else 0,
                     trace_cap=16 if trace else 0, **CPU_ONLY)
    ids, res = _schedule(s, [REQ], mode)
    r = res[ids[0]]
    assert r.status == 1 and r.hosts.tolist() == want, (name, r.status, r.hosts)
    kind = O.AHP if method == dc.DC_AHP else O.TOPSIS
    o = O.Oracle(inst, O.method(kind=kind, crit=(O.CRIT_CPU,), weight=[1.0]))
    st = lockstep(o, s, ids, [REQ], res, trace=trace_by_request(s) if trace else None, check_paths=True)
    if trace:
        assert st["scored_steps"] == 3
    assert st["near_tie"] == 0
    s.close()


@pytest.mark.parametrize("name,method,mode,grid", FORMS, ids=[f[0] for f in FORMS])
def test_identical_servers_take_lowest_index(name, method, mode, grid):
    """An empty data center scored on CPU alone: every server ties, so the
    first one-container request goes to server 0.  TOPSIS then ranks server
    0 (28 cores) last and the other fifteen tie again: server 1, then 2.
    On the Saaty scale 32 against 28 compares as 1, so all sixteen still
    tie under AHP: server 0 each time.  In lockstep with the oracle, whose
    exact-tie check flags any higher index."""
    inst = empty()
    reqs = [Request(np.array([4], np.int32), np.array([8], np.int32), np.zeros((0, 3), np.int32))
            for _ in range(3)]
    s = dc.Scheduler([inst], method=method, mode=mode, grid=grid, **CPU_ONLY)
    ids, res = _schedule(s, reqs, mode)
    want = [0, 1, 2] if method == dc.DC_TOPSIS else [0, 0, 0]
    assert [int(res[i].hosts[0]) for i in ids] == want
    kind = O.AHP if method == dc.DC_AHP else O.TOPSIS
    o = O.Oracle(inst, O.method(kind=kind, crit=(O.CRIT_CPU,), weight=[1.0]))
    st = lockstep(o, s, ids, reqs, res, check_paths=True)
    assert st["near_tie"] == 0
    s.close()


@pytest.mark.parametrize("name,method,mode,grid", FORMS[:5], ids=[f[0] for f in FORMS[:5]])
@pytest.mark.parametrize("uplink0,want", [(500, [0, 0, 0]), (600, [0, 0, 1])], ids=["cut_short", "cut_exact"])
def test_peer_uplink_cut(name, method, mode, grid, uplink0, want):
    """Both peers of the last container sit on server 0, whose uplink has
    500 Mbps left for their 2 x 300: no other server can route both paths,
    so the container goes to server 0 itself, the lowest-scored server
    (with 600 left both paths fit and the best server, 1, takes it).  In
    lockstep with the oracle, paths included."""
    inst = peer_cut(uplink0)
    s = dc.Scheduler([inst], method=method, mode=mode, grid=grid, **CPU_ONLY)
    ids, res = _schedule(s, [REQ_CUT], mode)
    r = res[ids[0]]
    assert r.status == 1 and r.hosts.tolist() == want, (name, r.status, r.hosts)
    o = O.Oracle(inst, O.method(kind=O.TOPSIS, crit=(O.CRIT_CPU,), weight=[1.0]))
    st = lockstep(o, s, ids, [REQ_CUT], res, check_paths=True)
    assert st["near_tie"] == 0
    s.close()
