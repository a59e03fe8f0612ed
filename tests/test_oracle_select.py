"""Pins for the oracle's selection step (section V-C: servers are taken in
decreasing score, the first on which the container and its paths fit wins;
Eqs. (4)-(5) decide whether they fit).

Hand cases on a k = 4 fat-tree whose placements, scores and top-two gaps
are worked out below from the closed form of TOPSIS with one criterion,
closeness = (x - min) / (max - min), and from the Saaty comparisons of the
CPU values.  Each case is also run on copies of the oracle with a planted
mistake in the selection (ascending order, ties to the highest index, no
next candidate after a failed commit); every copy must fail a case.
Everything here runs on the CPU."""
import os

import numpy as np
import pytest

import oracle as O
from workloads import Request

from select_cases import N4, REQ, empty as _empty, loaded as _loaded, split_fits as _split_fits

CPU_ONLY = dict(crit=(O.CRIT_CPU,), weight=[1.0])


def check_identical_servers():
    """An empty data center: every server has the same criteria, so every
    score is equal (TOPSIS: 0, both distances being 0; AHP: 1/N) and the
    lowest index wins; the runner-up has the same score."""
    for kind in (O.TOPSIS, O.AHP):
        o = O.Oracle(_empty(), O.method(kind=kind))
        r = o.run_request(Request(np.array([4], np.int32), np.array([8], np.int32), np.zeros((0, 3), np.int32)),
                          detail=True)
        assert r["status"] == 1 and r["hosts"].tolist() == [0], (kind, r["hosts"])
        assert r["ref_gap"][0] == 0.0
        want = 0.0 if kind == O.TOPSIS else 1.0 / N4
        assert r["ref_top"][0] == pytest.approx(want, abs=1e-15)
        o.close()


def check_topsis_hand_case():
    """TOPSIS on CPU alone, closeness (x - min) / (max - min) over all 16
    servers.
    Container 0 (20 cores): min 10, max 32; servers 0 and 4 score 1, 8
      20/22, 12 19/22; only these four have 20 cores.  Exact tie: server 0,
      gap 0 (server 4 also scores 1).
    Container 1 (20 cores, no link to container 0): server 0 now has 12;
      server 4 scores 1, server 8 10/11: server 4, gap 1/11.
    Container 2 (1 core, 300 Mbps to servers 0 and 4): min 10, max 30;
      server 8 scores 1, 12 19/20, 0 and 4 1/10.  Server 8 passes the
      per-peer check (its widest path to each peer is 500 Mbps wide) and its
      uplink carries 600, but its commit fails: the path to server 0 takes
      300 of the 500 on edge switch 4's first uplink, leaving 200 and 100
      for the path to server 4.  The next server, 12, commits: score 19/20;
      the runner-up is server 0 (1/10): gap 17/20."""
    o = O.Oracle(_loaded(), O.method(kind=O.TOPSIS, **CPU_ONLY))
    before = o.state()
    r = o.run_request(REQ, detail=True)
    assert r["status"] == 1, r
    assert r["hosts"].tolist() == [0, 4, 12], r["hosts"]
    np.testing.assert_allclose(r["ref_top"], [1.0, 1.0, 19 / 20], rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["ref_gap"], [0.0, 1 / 11, 17 / 20], rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["scores"], [1.0, 1.0, 19 / 20], rtol=0, atol=1e-15)
    # state: CPU and placed counts; both paths from server 12 leave through
    # edge switch 6's first uplink and core 0 (every candidate is 700 wide
    # for the second, so the lowest aggregation and core win); the failed
    # attempt on server 8 left nothing behind
    want = before.copy()
    want[0, [0, 4, 12]] -= [20, 20, 1]
    want[1, [0, 4, 12]] -= 1
    want[2, [0, 4, 12]] += 1
    want[3, 12] -= 600
    want[3, [0, 4]] -= 300
    want[4, 6 * 2 + 0] -= 600          # edge switch 6, aggregation 0
    want[4, 0 * 2 + 0] -= 300          # edge switch 0, aggregation 0
    want[4, 2 * 2 + 0] -= 300          # edge switch 2, aggregation 0
    want[5, (3 * 2 + 0) * 2 + 0] -= 600   # pod 3, aggregation 0, core 0
    want[5, (0 * 2 + 0) * 2 + 0] -= 300   # pod 0
    want[5, (1 * 2 + 0) * 2 + 0] -= 300   # pod 1
    np.testing.assert_array_equal(o.state(), want)
    o.close()


def check_ahp_hand_case():
    """AHP on CPU alone (Saaty 1-9 scale).  Values within 32/29 of each
    other compare as 1, and 29..32 against 10 as 3, so servers 0, 4, 8 and
    12 tie exactly for container 0: server 0.  For container 1 server 0
    has 12: 32 and 30 against 12 give 3 (2.5 rounds up), 29 gives 2, so 4
    and 8 tie above 12: server 4.  For container 2 servers 0 and 4 have
    12: server 8 comes first, fails its commit as in the TOPSIS case, and
    server 12 takes the container."""
    o = O.Oracle(_loaded(), O.method(kind=O.AHP, **CPU_ONLY))
    r = o.run_request(REQ, detail=True)
    assert r["status"] == 1 and r["hosts"].tolist() == [0, 4, 12], r["hosts"]
    assert r["ref_gap"][0] == 0.0 and r["ref_gap"][1] == 0.0 and r["ref_gap"][2] > 0.0
    o.close()


def check_split_fits():
    """Control for the failed commit: with 600 and 0 Mbps left on edge
    switch 4's uplinks the per-peer checks are the same (each path 600
    wide, 600 in total), but both paths fit through the first uplink, so
    container 2 stays on server 8."""
    o = O.Oracle(_split_fits(), O.method(kind=O.TOPSIS, **CPU_ONLY))
    r = o.run_request(REQ, detail=True)
    assert r["status"] == 1 and r["hosts"].tolist() == [0, 4, 8], r["hosts"]
    assert r["ref_top"][2] == 1.0
    o.close()


def check_tie_low():
    """Lockstep on an empty data center: following server 5 for a container
    all servers score equally on is flagged (server 0 has the same
    criteria, is feasible and commits); following server 0 is not."""
    one = Request(np.array([4], np.int32), np.array([8], np.int32), np.zeros((0, 3), np.int32))
    o = O.Oracle(_empty(), O.method())
    assert o.run_request(one, follow=np.array([5], np.int32), detail=True)["tie_low"].tolist() == [0]
    assert o.run_request(one, follow=np.array([0], np.int32), detail=True)["tie_low"].tolist() == [-1]
    # servers 5 and 0 now hold a container and differ from the others:
    # following server 7 is flagged against server 1
    assert o.run_request(one, follow=np.array([7], np.int32), detail=True)["tie_low"].tolist() == [1]
    o.close()


CHECKS = (check_identical_servers, check_topsis_hand_case, check_ahp_hand_case, check_split_fits, check_tie_low)


@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_selection(oracle_lib, check):
    check()


# Planted mistakes in the selection step: (text in dc_oracle.c, replacement).
MUTANTS = {
    "ascending_order": ("if (a->s != b->s) return a->s > b->s ? -1 : 1;",
                        "if (a->s != b->s) return a->s < b->s ? -1 : 1;"),
    "ties_to_highest_index": ("return a->u < b->u ? -1 : (a->u > b->u);",
                              "return a->u > b->u ? -1 : (a->u < b->u);"),
    "no_next_candidate": ("            if (!feas[u]) continue;\n",
                          "            if (!feas[u]) continue;\n"
                          "            if (top1 < 0) {\n"
                          "                int c_b, r_b;\n"
                          "                if (!try_commit(d, u, cpu[i], cx, ram[i], rx, Pc, ph, pbw, pbx, tmp, &c_b, &r_b))"
                          " break;\n"
                          "                undo_commit(d, u, c_b, r_b, Pc, tmp);\n"
                          "            }\n"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_selection_mistakes_fail_a_pin(oracle_lib, tmp_path, monkeypatch, name):
    with open(O._SRC) as f:
        src = f.read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site of {name} not found once in the oracle source"
    path = O.build_variant(src.replace(old, new), os.path.join(str(tmp_path), f"liboracle_{name}.so"))
    monkeypatch.setattr(O, "_lib", O.load(path))
    caught = []
    for check in CHECKS:
        try:
            check()
        except AssertionError:
            caught.append(check.__name__)
    assert caught, f"planted mistake {name} passes every selection pin"
