"""Lockstep parity between the GPU library and the FP64 oracle.

The oracle replays every request and, at each container step, follows the
server the GPU chose.  It checks that choice against its own ranking:
equal to the oracle's best commit-successful server whenever the oracle's
top-two score gap exceeds the tolerance, otherwise scored within the
tolerance of the best, and never above a feasible, commit-successful server
of lower index with identical criteria (exact ties go to the lowest index).  The integer state (CPU, RAM, placed counts, link
residuals) must then be identical after every request.  Recorded GPU
score vectors are compared element by element with the oracle's.
"""
import numpy as np

import oracle as O

TOL = 1e-5   # relative score tolerance for FP32 scores against FP64


def gpu_follow(sched, rid, res, req=None):
    """Server the GPU gave each step (a pod, or a container without pods);
    -1 from the failing step on."""
    att = sched.attempt(rid)
    unit, first = O.units(len(att), getattr(req, "pod", None))
    follow = att[first].copy()
    if res.status == 0 and res.failed_at < res.n:      # failed_at == n: placed, links did not fit
        follow[unit[res.failed_at]:] = -1
    return follow


def check_scores(gpu, ref, tol=TOL, where=""):
    """|s_gpu - s_ref| <= tol * max|s_ref| everywhere, and relative error
    <= tol where s_ref >= 1e-3 * max."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    top = float(np.max(np.abs(ref))) if ref.size else 0.0
    scale = max(top, 1e-30)
    err = np.abs(gpu - ref)
    assert np.all(err <= tol * scale), f"{where}: max abs err {err.max():.3e} vs {tol * scale:.3e}"
    big = (np.abs(ref) >= 1e-3 * top) & (ref != 0)
    if big.any():
        rel = err[big] / np.abs(ref[big])
        assert np.all(rel <= tol), f"{where}: max rel err {rel.max():.3e}"


def lockstep(o, sched, ids, reqs, results, tol=TOL, trace=None, check_paths=False, state_every=False,
             instance=0, final_state=True, check_alloc=False):
    """Replays `reqs` (submitted to `sched` with ids `ids`, results keyed by
    id) on oracle `o` in lockstep, one step per pod (per container without
    pods).  trace: optional dict (request id -> list of (step, gpu score
    vector)).  state_every: compare the
    integer state after each request (only meaningful when the GPU has
    scheduled exactly these requests so far, one schedule call each).
    check_alloc: what each accepted request's containers and edges were
    given must equal the oracle's allocations bit for bit.
    Returns statistics."""
    st = dict(requests=0, accepted=0, rejected=0, steps=0, near_tie=0, scored_steps=0, rec_ids=[])
    for pos, (rid, req) in enumerate(zip(ids, reqs)):
        g = results[rid]
        follow = gpu_follow(sched, rid, g, req)
        unit, first = O.units(req.n, getattr(req, "pod", None))
        want_dump = trace is not None and rid in trace
        ref = o.run_request(req, follow=follow, detail=True, dump=want_dump)
        assert ref["status"] == g.status, f"request {pos}: oracle status {ref['status']} vs gpu {g.status}"
        assert ref["failed_at"] == g.failed_at
        steps = len(first) if g.status == 1 or g.failed_at == req.n else unit[g.failed_at] + 1
        for i in range(steps):
            if follow[i] < 0:
                assert ref["ref_host"][i] < 0, f"request {pos} step {i}: oracle found a server"
                continue
            top = ref["ref_top"][i]
            # exact ties (identical criteria) resolve to the lowest index
            assert ref["tie_low"][i] < 0, (
                f"request {pos} step {i}: gpu took server {follow[i]}, but server {ref['tie_low'][i]} has "
                f"identical criteria, is feasible and commits")
            if follow[i] != ref["ref_host"][i]:
                st["near_tie"] += 1
                assert ref["ref_gap"][i] <= tol * max(abs(top), 1e-30), (
                    f"request {pos} step {i}: gpu {follow[i]} vs oracle {ref['ref_host'][i]}, "
                    f"gap {ref['ref_gap'][i]:.3e} top {top:.6f}")
                assert ref["step_scores"][i] >= top - tol * max(abs(top), 1e-30)
            if g.status == 1:
                gs = float(g.scores[first[i]])
                assert abs(gs - ref["step_scores"][i]) <= tol * max(abs(top), 1e-30), (
                    f"request {pos} step {i}: score {gs} vs {ref['step_scores'][i]}")
        if want_dump:
            for i, vec in trace[rid]:
                check_scores(vec, ref["dump"][i], tol, where=f"request {pos} step {i}")
                st["scored_steps"] += 1
        if check_paths and g.status == 1:
            got = sched.paths(rid)
            want, _ = o.paths(ref["rec_id"])
            assert got.shape == want.shape
            for a, b in zip(got, want):
                assert sorted(a.tolist()) == sorted(b.tolist())
        if check_alloc and g.status == 1:
            ca, ra, ba = sched.alloc(rid, req.n, req.m)
            np.testing.assert_array_equal(ca, ref["cpu_a"], err_msg=f"request {pos}: cpu allocation")
            np.testing.assert_array_equal(ra, ref["ram_a"], err_msg=f"request {pos}: ram allocation")
            np.testing.assert_array_equal(ba, ref["bw_a"], err_msg=f"request {pos}: bandwidth allocation")
        if state_every:
            np.testing.assert_array_equal(sched.state(instance), o.state(), err_msg=f"after request {pos}")
        st["rec_ids"].append(ref["rec_id"])
        st["requests"] += 1
        st["accepted"] += g.status == 1
        st["rejected"] += g.status == 0
        st["steps"] += steps
    if final_state:
        np.testing.assert_array_equal(sched.state(instance), o.state())
    return st


def trace_by_request(sched, ids=None):
    """GPU trace grouped by request id: {id: [(container, scores)]}."""
    meta, scores = sched.trace()
    out = {}
    for (inst, rid, i, s), vec in zip(meta, scores):
        out.setdefault(int(rid), []).append((int(i), vec))
    return out
