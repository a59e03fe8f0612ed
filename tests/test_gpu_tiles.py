"""dc_topsis_tiles (TOPSIS scoring and selection over materialised decision
matrices, section V-C) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle as O
from workloads import make_tiles

torch = pytest.importorskip("torch")
dc = pytest.importorskip("paper_1909_07673_amd")

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check_tile(x, feas, w, cost, sc, best, bscore):
    """Scores within TOL of the oracle (relative to the tile's maximum, and
    elementwise where not tiny); the chosen server is the oracle's best
    feasible one whenever the top-two gap exceeds TOL, otherwise within TOL
    of it; identical criteria vectors resolve to the lowest index."""
    ref = O.topsis(x.astype(np.float64), w, cost)
    top = max(ref.max(), 1e-300)
    if sc is not None:
        assert np.all(np.abs(sc - ref) <= TOL * top + 1e-7)
        big = ref >= 1e-3 * top
        assert np.all(np.abs(sc[big] - ref[big]) <= TOL * ref[big])
    ok = np.ones(x.shape[1], bool) if feas is None else feas.astype(bool)
    if not ok.any():
        assert best == -1 and bscore == 0.0
        return
    cand = np.flatnonzero(ok)
    order = cand[np.lexsort((cand, -ref[cand]))]
    t1 = order[0]
    gap = ref[t1] - (ref[order[1]] if len(order) > 1 else -np.inf)
    assert ok[best]
    if gap > TOL * ref[t1]:
        assert best == t1
    else:
        assert ref[best] >= ref[t1] - TOL * max(ref[t1], 1e-300)
    same = np.flatnonzero(ok & np.all(x == x[:, best:best + 1], axis=0))
    assert best == same.min()
    if sc is not None:
        assert np.float32(bscore).view(np.uint32) == np.float32(sc[best]).view(np.uint32)


def _run(x, feas, w, cost, scores=True):
    xd = _dev(x)
    fd = _dev(feas) if feas is not None else None
    b, bs, sc = dc.topsis_tiles(xd, w, cost, fd, scores=scores)
    torch.cuda.synchronize()
    return b.cpu().numpy(), bs.cpu().numpy(), (sc.cpu().numpy() if sc is not None else None)


SHAPES = [
    # T, C, N, feasible_p, cost     (paths: one wavefront per tile with the
    # tile in registers; slices of 2,048 servers over several workgroups with
    # partials in scratch, for up to 1,024 tiles of at least 4,096 servers;
    # otherwise one workgroup per tile with two passes)
    (9, 4, 1024, None, None),          # wavefront, four groups per lane
    (13, 2, 2048, 0.5, [1, 0]),        # wavefront, eight groups per lane
    (5, 1, 2048, 0.9, None),           # wavefront, eight groups per lane, one criterion
    (4, 1, 4096, 0.9, None),           # split, two slices
    (7, 3, 1000, 0.5, [0, 1, 0]),      # wavefront, ragged last group
    (6, 5, 512, 0.6, [0, 0, 0, 0, 1]), # wavefront, five criteria
    (5, 5, 2048, 0.6, [0, 0, 0, 0, 1]),  # two passes
    (3, 4, 4096, 0.3, None),           # split
    (4, 8, 3000, 0.5, [0, 1, 0, 0, 1, 0, 0, 0]),   # two passes, ragged last group
    (3, 3, 54, 0.7, None),             # k=6: N % 4 != 0, two passes
    (2, 4, 27648, 0.8, None),          # k=48: split, 14 slices, the last one half full
    (1, 5, 8193, 0.5, [0, 0, 0, 0, 1]),  # split, a last slice of one server
    (1, 4, 1 << 20, 0.9, None),        # the largest N: split, 512 slices
    (3, 1, 16, None, None),            # k=4, one criterion
    (2, 2, 1, 1.0, [1, 0]),
]


@pytest.mark.parametrize("T,C,N,p,cost", SHAPES)
def test_tiles_match_oracle(T, C, N, p, cost):
    x, feas = make_tiles(seed=T * 1000 + C * 10 + N, T=T, N=N, C=C, feasible_p=p)
    w = np.full(C, 1.0 / C)
    if cost is None:
        cost = [0] * C
    best, bscore, sc = _run(x, feas, w, cost)
    for t in range(T):
        _check_tile(x[t], None if feas is None else feas[t], w, cost, sc[t], best[t], bscore[t])


def test_tiles_edge_cases():
    """Constant and all-zero columns, an all-zero tile (every distance 0:
    score 0, lowest feasible index), no feasible server, exact duplicates of
    the best server at a lower index, unequal weights."""
    T, C, N = 6, 4, 1024
    x, feas = make_tiles(seed=77, T=T, N=N, C=C, feasible_p=0.5)
    x[0, 1, :] = 17                      # constant column
    x[1, :, :] = 0                       # all-zero tile
    feas[2, :] = 0                       # nothing feasible
    x[3, :, 5] = x[3, :, 900] = [32, 256, 0, 40000]   # identical ideal servers (column 2 is a cost)
    feas[3, 5] = feas[3, 900] = 1
    x[4, 2, :] = 0                       # all-zero column
    w = np.array([0.4, 0.3, 0.2, 0.1])
    cost = [0, 0, 1, 0]
    best, bscore, sc = _run(x, feas, w, cost)
    for t in range(T):
        _check_tile(x[t], feas[t], w, cost, sc[t], best[t], bscore[t])
    assert best[1] == np.flatnonzero(feas[1])[0] and sc[1].max() == 0.0
    assert best[2] == -1
    assert best[3] == 5


def test_tiles_paths_identical():
    """The wavefront path and the two-pass path (forced by a misaligned view
    of the same data) give bit-identical results; scores are optional."""
    T, C, N = 7, 4, 1024
    x, feas = make_tiles(seed=5, T=T, N=N, C=C, feasible_p=0.4)
    w = [0.25] * 4
    b1, s1, sc1 = _run(x, feas, w, None)
    big = torch.zeros(T * C * N + 1, dtype=torch.int32, device="cuda")
    big[1:] = _dev(x).reshape(-1)
    xv = big[1:].view(T, C, N)          # 4-byte aligned only
    b2, s2, sc2 = dc.topsis_tiles(xv, w, None, _dev(feas), scores=True)
    b3, s3, _ = dc.topsis_tiles(_dev(x), w, None, _dev(feas), scores=False)
    torch.cuda.synchronize()
    assert np.array_equal(b1, b2.cpu().numpy()) and np.array_equal(b1, b3.cpu().numpy())
    assert s1.tobytes() == s2.cpu().numpy().tobytes() == s3.cpu().numpy().tobytes()
    assert sc1.tobytes() == sc2.cpu().numpy().tobytes()


def test_tiles_split_equals_two_pass():
    """1,024 tiles of 4,096 servers take the split path, 1,025 the
    one-workgroup path: the first 1,024 tiles' results are bit-identical."""
    T, C, N = 1025, 4, 4096
    x, feas = make_tiles(seed=9, T=T, N=N, C=C, feasible_p=0.7)
    w = [0.4, 0.3, 0.2, 0.1]
    b1, s1, sc1 = _run(x[:1024], feas[:1024], w, [0, 1, 0, 0])
    b2, s2, sc2 = _run(x, feas, w, [0, 1, 0, 0])
    assert np.array_equal(b1, b2[:1024])
    assert s1.tobytes() == s2[:1024].tobytes() and sc1.tobytes() == sc2[:1024].tobytes()
    for t in (0, 511, 1023):
        _check_tile(x[t], feas[t], w, [0, 1, 0, 0], sc1[t], b1[t], s1[t])


def test_tiles_invalid_arguments():
    x = torch.zeros((2, 3, 8), dtype=torch.int32, device="cuda")
    with pytest.raises(dc.DcError):
        dc.topsis_tiles(x, [0.5, 0.5, 0.0])           # weight not positive
    with pytest.raises(ValueError):
        dc.topsis_tiles(x.float(), [1 / 3] * 3)
    b, s, _ = dc.topsis_tiles(torch.zeros((0, 3, 8), dtype=torch.int32, device="cuda"), [1 / 3] * 3)
    assert b.numel() == 0


def test_tiles_full_size_sampled():
    """The measured configuration (32,768 tiles of 4 x 1024, 512 MiB, best
    and best score only): sampled tiles against the oracle."""
    T, C, N = 32768, 4, 1024
    x, _ = make_tiles(seed=2024, T=T, N=N, C=C)
    w = [0.25] * 4
    best, bscore, _ = _run(x, None, w, None, scores=False)
    rng = np.random.default_rng(0)
    for t in sorted(set(rng.integers(0, T, 48).tolist()) | {0, T - 1}):
        _check_tile(x[t], None, w, [0] * 4, None, best[t], bscore[t])
        ref = O.topsis(x[t].astype(np.float64), w, [0] * 4)
        assert abs(bscore[t] - ref[best[t]]) <= TOL * ref.max()
