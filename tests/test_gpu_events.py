"""The event replay of section VI-A on the library against an independent
replay on the oracle: per event the same waiting queue (FCFS, retried at
every event), the same placements and rejections (all or nothing), the same
allocations, the same fragmentation shares F(N^s), F(E^s) (section II-B),
and in the end the same number of events, delays and utilities U(i),
U(ij) (Eqs. (1)-(2)).  A k = 8 data center with heavier requests than the
paper's, so that requests wait."""
import numpy as np
import pytest

import oracle as O
from parity import lockstep
from workloads import make_event_workload

pytestmark = pytest.mark.gpu

dc = pytest.importorskip("paper_1909_07673_amd")
from paper_1909_07673_amd import events  # noqa: E402


class _Res:
    """A RESULT_DTYPE record with the attributes lockstep reads."""

    def __init__(self, r):
        self.req_id, self.status, self.failed_at = int(r["req_id"]), int(r["status"]), int(r["failed_at"])
        self.n = int(r["n"])
        self.hosts = r["host"][: self.n].copy()
        self.scores = r["score"][: self.n].copy()


@pytest.mark.parametrize("method", [dc.DC_TOPSIS, dc.DC_AHP])
def test_event_replay_matches_oracle_replay(method):
    inst, reqs, arrive, dur = make_event_workload(seed=1, k=8, n_req=400, total_events=80, span=40, cpu_hi=8,
                                                  bw_hi=200)
    caps = (inst.bw_host_edge, inst.bw_edge_agg, inst.bw_agg_core)
    s = dc.Scheduler([inst], method=method)
    log = []          # (event, submitted request indices, their results)
    rep = events.replay(s, reqs, arrive, dur, caps,
                        on_event=lambda ev, sub, res: log.append((ev, sub, [_Res(r) for r in res])))
    assert rep["events"] > 40 and (rep["delay"] > 0).sum() > 50 and rep["submissions"] > len(reqs) + 100

    # the oracle's own replay: its own queue, departures and fragmentation
    o = O.Oracle(inst, O.method(kind=O.AHP if method == dc.DC_AHP else O.TOPSIS))
    by_event = {ev: (sub, res) for ev, sub, res in log}
    placed = np.full(len(reqs), -1)
    rec, ends, queue = {}, {}, []
    nxt = ev = 0
    cap = np.array(caps, np.int64)[:, None]
    while nxt < len(reqs) or queue:
        for q in ends.pop(ev, []):
            assert o.release(rec[q]) == 0
        while nxt < len(reqs) and arrive[nxt] <= ev:
            queue.append(nxt)
            nxt += 1
        if queue:
            sub, res = by_event[ev]
            assert sub == queue, f"event {ev}: waiting queue differs"
            still = []
            for q, r in zip(queue, res):
                st = lockstep(o, s, [r.req_id], [reqs[q]], {r.req_id: r}, check_paths=True, check_alloc=True,
                              final_state=False)
                if r.status == 1:
                    placed[q] = ev
                    rec[q] = st["rec_ids"][0]
                    ends.setdefault(ev + int(dur[q]), []).append(q)
                else:
                    still.append(q)
            queue = still
        else:
            assert ev not in by_event
        state = o.state().astype(np.int64)
        assert float((state[2] > 0).mean()) == rep["frag_s"][ev], f"event {ev}: F(N^s)"
        assert float((state[3:] < cap).mean()) == rep["frag_l"][ev], f"event {ev}: F(E^s)"
        ev += 1
    np.testing.assert_array_equal(placed, rep["placed"])
    assert ev == len(rep["frag_s"]) and int(placed.max()) + 1 == rep["events"]
    np.testing.assert_array_equal(placed - arrive, rep["delay"])
    # utilities of what each request was given (allocations already equal
    # bit for bit in the lockstep above)
    ui, uij = [], []
    for q, req in enumerate(reqs):
        a, b = events.utilities(req, *s.alloc(int(rep["rid"][q]), req.n, req.m))
        assert np.all(a > 0) and np.all(a <= 1) and np.all(b > 0) and np.all(b <= 1)
        ui.append(a)
        uij.append(b)
    assert 0.5 < np.mean(np.concatenate(ui)) <= 1.0
    s.close()
    o.close()
