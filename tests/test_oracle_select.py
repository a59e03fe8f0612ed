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

from select_cases import N4, REQ, REQ_CUT, empty as _empty, loaded as _loaded, peer_cut as _peer_cut, \
    split_fits as _split_fits

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


def check_peer_cut():
    """Both peers of container 2 sit on server 0, whose uplink has 500 Mbps
    left for their 2 x 300.  CPU closeness over min 8 (server 0) and max 14
    (server 1): server 1 scores 1, servers 2..15 1/3, server 0 0.  Every
    server but 0 passes the per-peer checks (each path 500 wide) and its own
    uplink carries 600, but routing the second path finds 200 left on
    server 0's uplink: all fifteen commits fail, and only server 0, which
    holds both peers and needs no link, takes the container (score 0, no
    runner-up).  With 600 left (the control) both paths fit exactly and
    server 1 takes it."""
    o = O.Oracle(_peer_cut(500), O.method(kind=O.TOPSIS, **CPU_ONLY))
    before = o.state()
    r = o.run_request(REQ_CUT, detail=True)
    assert r["status"] == 1 and r["hosts"].tolist() == [0, 0, 0], r["hosts"]
    np.testing.assert_allclose(r["scores"], [1.0, 1.0, 0.0], rtol=0, atol=1e-15)
    assert r["ref_gap"][2] == np.inf
    want = before.copy()
    want[0, 0] -= 25
    want[1, 0] -= 3
    want[2, 0] += 3
    np.testing.assert_array_equal(o.state(), want)     # no link used
    o.close()
    o = O.Oracle(_peer_cut(600), O.method(kind=O.TOPSIS, **CPU_ONLY))
    before = o.state()
    r = o.run_request(REQ_CUT, detail=True)
    assert r["status"] == 1 and r["hosts"].tolist() == [0, 0, 1], r["hosts"]
    assert r["scores"][2] == 1.0 and r["ref_gap"][2] == pytest.approx(2 / 3, abs=1e-15)
    want = before.copy()
    want[0, [0, 1]] -= [24, 1]
    want[1, [0, 1]] -= [2, 1]
    want[2, [0, 1]] += [2, 1]
    want[3, [0, 1]] -= 600                              # both paths: up[1], up[0]
    np.testing.assert_array_equal(o.state(), want)
    o.close()


CHECKS = (check_identical_servers, check_topsis_hand_case, check_ahp_hand_case, check_split_fits, check_tie_low,
          check_peer_cut)


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


def _tight_workload(seed):
    """k = 4 with 1,000 Mbps links, 0-70 % background and requests of 2-8
    containers at 100-900 Mbps per pair: many placements leave several peers
    on one server, so later commits often fail on a peer's uplink."""
    from workloads import make_instance, make_requests
    rng = np.random.default_rng(seed)
    inst = make_instance(4, 32, 256, 1000, 1000, 1000, background=0.7, rng=rng)
    return inst, make_requests(12, rng, 2, 8, bw_hi=900)


def _replay_all(seeds, kind):
    out = []
    for seed in seeds:
        inst, reqs = _tight_workload(seed)
        o = O.Oracle(inst, O.method(kind=kind))
        for req in reqs:
            r = o.run_request(req, detail=True)
            out.append((r["status"], r["failed_at"], r["hosts"].tolist(), r["ref_host"].tolist()))
        out.append(o.state().tolist())
        o.close()
    return out


# The cut pre-check of the commit only answers early what the routing would
# answer: a copy without it must agree everywhere.  Planted mistakes in it
# must fail a hand case or that agreement.
CUT_SITE = "        if (v == u) continue;\n        int64_t need = 0, cap = 0;\n"
CUT_MUTANTS = {
    "no_cut": ("    if (peer_cut_short(d, u, P, ph, pbw)) return 0;\n", ""),
    "cut_counts_own_server": (CUT_SITE, "        int64_t need = 0, cap = 0;\n"),
    "cut_strict_boundary": ("        if (cap < need) return 1;", "        if (cap <= need) return 1;"),
    "cut_sums_all_peers": ("for (int q = 0; q < P; ++q) if (ph[q] == v) need += pbw[q];",
                           "for (int q = 0; q < P; ++q) need += pbw[q];"),
}


def _variant(tmp_path, name):
    with open(O._SRC) as f:
        src = f.read()
    old, new = CUT_MUTANTS[name]
    assert src.count(old) == 1, f"mutation site of {name} not found once in the oracle source"
    return O.load(O.build_variant(src.replace(old, new), os.path.join(str(tmp_path), f"liboracle_{name}.so")))


def test_peer_cut_changes_no_result(oracle_lib, tmp_path, monkeypatch):
    seeds = range(40)
    base = {kind: _replay_all(seeds, kind) for kind in (O.TOPSIS, O.AHP)}
    rejected = sum(1 for rec in base[O.TOPSIS] if isinstance(rec, tuple) and rec[0] == 0)
    assert rejected >= 20, rejected
    monkeypatch.setattr(O, "_lib", _variant(tmp_path, "no_cut"))
    for kind in (O.TOPSIS, O.AHP):
        assert _replay_all(seeds, kind) == base[kind], kind
    check_peer_cut()


@pytest.mark.parametrize("name", sorted(set(CUT_MUTANTS) - {"no_cut"}))
def test_planted_cut_mistakes_fail_a_pin(oracle_lib, tmp_path, monkeypatch, name):
    seeds = range(40)
    base = _replay_all(seeds, O.TOPSIS)
    monkeypatch.setattr(O, "_lib", _variant(tmp_path, name))
    caught = []
    try:
        check_peer_cut()
    except AssertionError:
        caught.append("hand case")
    if _replay_all(seeds, O.TOPSIS) != base:
        caught.append("agreement")
    assert caught, f"planted mistake {name} passes the cut pins"
