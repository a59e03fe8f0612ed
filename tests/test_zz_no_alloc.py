"""dc_topsis_tiles_noalloc: the tile scoring entry point that allocates no
device memory (its large-tile partials live in a static device array)
against dc_topsis_tiles, bit for bit, through the C ABI: two calls in a row
on the large-tile path, the second smaller than the first, then a call
beyond the static buffer, which is refused."""
import numpy as np
import pytest

import oracle as O
from workloads import make_tiles

torch = pytest.importorskip("torch")
dc = pytest.importorskip("paper_1909_07673_amd")

pytestmark = pytest.mark.gpu


def _split_bytes(T, N, C):
    """Scratch bytes of the large-tile path: per tile and slice of 2,048
    servers, C sums of squares (8 B), maxima and minima (4 B each) and one
    best key (8 B), each region rounded up to 256 B."""
    S = -(-N // 2048)
    al = lambda b: (b + 255) & ~255
    return al(T * S * C * 8) + 2 * al(T * S * C * 4) + al(T * S * 8)


def _device_tiles(seed, T, C, N, feasible_p):
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randint(0, 1 << 22, (T, C, N), generator=g, device="cuda", dtype=torch.int32)
    feas = (torch.rand((T, N), generator=g, device="cuda") < feasible_p).to(torch.uint8)
    return x, feas


def _both(x, feas, w, cost):
    T, _, N = x.shape
    b0, s0, sc0 = dc.topsis_tiles(x, w, cost, feas, scores=True)
    best = torch.full((T,), -7, dtype=torch.int32, device="cuda")
    bsc = torch.full((T,), -7.0, dtype=torch.float32, device="cuda")
    sc = torch.full((T, N), -7.0, dtype=torch.float32, device="cuda")
    dc.topsis_tiles_noalloc(x, w, best, bsc, cost, feas, sc)
    torch.cuda.synchronize()
    return (b0.cpu().numpy(), s0.cpu().numpy(), sc0.cpu().numpy()), (best.cpu().numpy(), bsc.cpu().numpy(),
                                                                     sc.cpu().numpy())


def _same(ref, got):
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1].view(np.uint32), ref[1].view(np.uint32))
    np.testing.assert_array_equal(got[2].view(np.uint32), ref[2].view(np.uint32))


def test_noalloc_matches_allocating_entry_point():
    torch.cuda.set_device(0)
    empty = torch.empty((0, 4, 4096), dtype=torch.int32, device="cuda")
    best0 = torch.empty((0,), dtype=torch.int32, device="cuda")
    dc.topsis_tiles_noalloc(empty, [0.25] * 4, best0)         # resolves the buffer's address
    # 1: close to the buffer's limit (960 tiles x 32 slices x 8 criteria)
    T, C, N = 960, 8, 65536
    assert _split_bytes(T, N, C) <= dc.DC_STATIC_SCRATCH_BYTES < _split_bytes(T + 64, N, C)
    x, feas = _device_tiles(11, T, C, N, 0.5)
    w, cost = [1.0 / C] * C, [0, 1, 0, 0, 1, 0, 0, 0]
    ref, got = _both(x, feas, w, cost)
    _same(ref, got)
    assert (got[0] >= 0).all()
    del x, feas, ref, got
    # 2: smaller, on the buffer the first call left behind; also against the
    # FP64 oracle
    xs, fs = make_tiles(5, 3, 8193, 4, 0.5)
    xd, fd = torch.from_numpy(xs).cuda(), torch.from_numpy(fs).cuda()
    ref, got = _both(xd, fd, [0.25] * 4, None)
    _same(ref, got)
    for t in range(3):
        r = O.topsis(xs[t].astype(np.float64), [0.25] * 4)
        top = r.max()
        assert np.all(np.abs(got[2][t] - r) <= 1e-5 * top + 1e-7)
        ok = np.flatnonzero(fs[t])
        order = ok[np.lexsort((ok, -r[ok]))]
        if r[order[0]] - r[order[1]] > 1e-5 * r[order[0]]:
            assert got[0][t] == order[0]
    # 3: a shape that needs no scratch (one wavefront per tile)
    xs, fs = make_tiles(6, 9, 1024, 4, 0.7)
    ref, got = _both(torch.from_numpy(xs).cuda(), torch.from_numpy(fs).cuda(), [0.25] * 4, None)
    _same(ref, got)


def test_noalloc_refuses_beyond_static_buffer():
    T, C, N = 1024, 8, 65536
    assert _split_bytes(T, N, C) > dc.DC_STATIC_SCRATCH_BYTES
    x = torch.empty((T, C, N), dtype=torch.int32, device="cuda")   # never read: refused before launch
    best = torch.empty((T,), dtype=torch.int32, device="cuda")
    with pytest.raises(dc.DcError) as e:
        dc.topsis_tiles_noalloc(x, [1.0 / C] * C, best)
    assert e.value.code == dc.DC_ETOOBIG
    # arguments are still checked first
    with pytest.raises(dc.DcError) as e:
        dc.topsis_tiles_noalloc(x[:1], [0.0] * C, best[:1])
    assert e.value.code == dc.DC_EINVAL
