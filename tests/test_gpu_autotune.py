"""The autotuner of the batched form: every launch shape it may pick gives
bit-identical results; the chosen shape is cached per (architecture, form,
method, servers, criteria) and read back; tuning leaves the trace as it
was."""
import numpy as np
import pytest

import oracle as O
from parity import lockstep
from workloads import make_config

pytestmark = pytest.mark.gpu

dc = pytest.importorskip("paper_1909_07673_amd")

SHAPES = [(256, 1), (256, 2), (256, 4), (512, 1), (512, 2), (512, 4), (1024, 1), (1024, 2)]


def _batched(insts, reqs, **kw):
    s = dc.Scheduler(insts, mode=dc.DC_MODE_BATCHED, **kw)
    ids = [[s.submit(r, instance=i) for r in rl] for i, rl in enumerate(reqs)]
    return s, ids


def _same(res_a, res_b):
    assert len(res_a) == len(res_b)
    for a, b in zip(res_a, res_b):
        assert (a.status, a.failed_at) == (b.status, b.failed_at)
        np.testing.assert_array_equal(a.hosts, b.hosts)
        np.testing.assert_array_equal(a.scores.view(np.uint32), b.scores.view(np.uint32))


def test_every_shape_is_bit_identical():
    """Eight instances of the batched workload's shape (up to 48 containers,
    so some containers have more peers than a small peer chunk): every built
    (block, servers per thread) pair with the largest peer chunk, 16 and 5
    gives the same servers, score bits and state as the default shape; the
    last shape's run of one instance in lockstep with the oracle."""
    insts, reqs = make_config("batched", seed=12, instances=8, n_req=60)
    s, ids = _batched(insts, reqs)
    base = s.shape()
    ref = s.schedule()
    ref_state = [s.state(i) for i in range(len(insts))]
    pcs = sorted({base["peer_chunk"], 16, 5})
    for bs, g in SHAPES:
        for pc in pcs:
            s.set_shape(bs, g, pc)
            assert s.shape() == {"block": bs, "host_group": g, "peer_chunk": pc}
            s.rewind()
            last = s.schedule()
            _same(ref, last)
            for i in range(len(insts)):
                np.testing.assert_array_equal(s.state(i), ref_state[i], err_msg=f"shape {bs},{g},{pc}")
    # the last shape run (1024 threads, 2 servers per thread, the largest
    # chunk) against the oracle on instance 3
    res = {r.req_id: r for r in last}
    o = O.Oracle(insts[3], O.method())
    lockstep(o, s, ids[3], reqs[3], res, instance=3, check_paths=True)
    with pytest.raises(dc.DcError):
        s.set_shape(1024, 4, 8)          # not built
    with pytest.raises(dc.DcError):
        s.set_shape(256, 1, base["peer_chunk"] + 1)
    s.close()


def test_autotune_cache_round_trip(tmp_path):
    """A tuned shape is written under its key and read back by a new
    context with the same data-center shape, without timing; the results
    after tuning equal the untuned ones."""
    path = str(tmp_path / "tune.jsonl")
    insts, reqs = make_config("batched", seed=13, instances=6, n_req=30)
    s, _ = _batched(insts, reqs)
    ref = s.schedule()
    s.rewind()
    t = s.autotune_cached(path)
    assert t["from_cache"] == 0 and t["candidates"] >= len(SHAPES) and t["ms"] > 0
    assert (t["block"], t["host_group"]) in SHAPES
    _same(ref, s.schedule())
    s.close()
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and '"key": "' in lines[0] and "|batched|topsis|N=1024|C=4" in lines[0]
    s2, _ = _batched(insts, reqs)
    t2 = s2.autotune_cached(path)
    assert t2["from_cache"] == 1 and t2["candidates"] == 0
    assert (t2["block"], t2["host_group"], t2["peer_chunk"]) == (t["block"], t["host_group"], t["peer_chunk"])
    assert s2.shape() == {"block": t["block"], "host_group": t["host_group"], "peer_chunk": t["peer_chunk"]}
    _same(ref, s2.schedule())
    s2.close()
    # another data-center size is another key: a second line
    insts4, reqs4 = make_config("tiny", seed=1)
    s3, _ = _batched(insts4, reqs4)
    assert s3.autotune_cached(path)["from_cache"] == 0
    assert len(open(path).read().splitlines()) == 2
    s3.close()


def test_autotune_leaves_trace_unchanged():
    """Tuning with a trace configured records nothing: the trace after the
    next schedule equals the trace of a context that never tuned."""
    insts, reqs = make_config("batched", seed=14, instances=1, n_req=20)
    a, _ = _batched(insts, reqs, trace_stride=1, trace_cap=1024)
    a.autotune()
    ra = a.schedule()
    b, _ = _batched(insts, reqs, trace_stride=1, trace_cap=1024)
    rb = b.schedule()
    _same(ra, rb)
    ma, sa = a.trace()
    mb, sb = b.trace()
    assert len(ma) > 0
    np.testing.assert_array_equal(ma, mb)
    np.testing.assert_array_equal(sa.view(np.uint32), sb.view(np.uint32))
    a.close()
    b.close()
