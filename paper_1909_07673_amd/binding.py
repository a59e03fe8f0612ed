"""ctypes binding of libdcsched (include/dcsched.h): same names, argument
marshalling only.  Every step of the scheduling path runs in the library's
HIP kernels; there is no CPU fallback, and loading fails loudly when the
library has not been built."""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Iterable, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdcsched.so")

DC_OK, DC_EINVAL, DC_ENOMEM, DC_EAGAIN, DC_ENOENT, DC_EDEVICE, DC_ESTATE, DC_ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7
DC_STATIC_SCRATCH_BYTES = 4 << 20
DC_TOPSIS, DC_AHP = 0, 1
DC_AHP_SAATY9, DC_AHP_RATIO, DC_AHP_DIFF = 0, 1, 2
DC_MODE_PLAIN, DC_MODE_BATCHED, DC_MODE_SERVING = 0, 1, 2
DC_ROUTE_EACH, DC_ROUTE_END = 0, 1
DC_CRIT_CPU, DC_CRIT_RAM, DC_CRIT_ACTIVE, DC_CRIT_PATHBW, DC_CRIT_UPLINK, DC_CRIT_HOPS = range(6)
DC_MAX_CONTAINERS, DC_MAX_CRIT = 64, 8

DEFAULT_CRIT = (DC_CRIT_CPU, DC_CRIT_RAM, DC_CRIT_ACTIVE, DC_CRIT_PATHBW)


class dc_config(C.Structure):
    _fields_ = [("k", C.c_int32), ("n_instances", C.c_int32), ("mode", C.c_int32),
                ("method", C.c_int32), ("ahp_scale", C.c_int32),
                ("host_cpu", C.c_int32), ("host_ram", C.c_int32),
                ("bw_host_edge", C.c_int32), ("bw_edge_agg", C.c_int32), ("bw_agg_core", C.c_int32),
                ("ncrit", C.c_int32), ("crit", C.c_int32 * 8), ("crit_cost", C.c_int32 * 8),
                ("weight", C.c_float * 8),
                ("host_used", C.c_void_p), ("link_used", C.c_void_p), ("stream", C.c_void_p),
                ("mem_budget", C.c_size_t), ("block", C.c_int32), ("trace_stride", C.c_int32),
                ("trace_cap", C.c_int32), ("grid", C.c_int32), ("graph", C.c_int32),
                ("grid_timeout_us", C.c_int32), ("routing", C.c_int32),
                ("reserved", C.c_int32 * 1)]


class dc_result(C.Structure):
    _fields_ = [("req_id", C.c_int64), ("instance", C.c_int32), ("status", C.c_int32),
                ("n", C.c_int32), ("failed_at", C.c_int32),
                ("host", C.c_int32 * DC_MAX_CONTAINERS), ("score", C.c_float * DC_MAX_CONTAINERS)]


class dc_tune(C.Structure):
    _fields_ = [("block", C.c_int32), ("host_group", C.c_int32), ("peer_chunk", C.c_int32),
                ("from_cache", C.c_int32), ("ms", C.c_float), ("candidates", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# dc_result as a NumPy record (same layout), for bulk result transfer.
RESULT_DTYPE = np.dtype([("req_id", np.int64), ("instance", np.int32), ("status", np.int32),
                         ("n", np.int32), ("failed_at", np.int32),
                         ("host", np.int32, DC_MAX_CONTAINERS), ("score", np.float32, DC_MAX_CONTAINERS)], align=True)
assert RESULT_DTYPE.itemsize == C.sizeof(dc_result)


class DcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


_lib = None


def lib():
    """Load libdcsched.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libdcsched.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i32p = C.POINTER(C.c_int32)
        L.dc_create.argtypes = [C.POINTER(dc_config), C.POINTER(P)]
        L.dc_submit_request.argtypes = [P, C.c_int32, C.c_int32, i32p, i32p, C.c_int32, i32p, i32p,
                                        C.POINTER(C.c_int64)]
        L.dc_submit_request_ranged.argtypes = [P, C.c_int32, C.c_int32, i32p, i32p, i32p, i32p, C.c_int32, i32p,
                                               i32p, i32p, C.POINTER(C.c_int64)]
        L.dc_get_alloc.argtypes = [P, C.c_int64, i32p, i32p, i32p]
        L.dc_schedule.argtypes = [P, C.c_int32, C.POINTER(dc_result), C.POINTER(C.c_int32)]
        L.dc_release.argtypes = [P, C.c_int64]
        L.dc_get_paths.argtypes = [P, C.c_int64, C.c_int32, i32p, C.POINTER(C.c_int32)]
        L.dc_get_attempt.argtypes = [P, C.c_int64, C.c_int32, i32p, C.POINTER(C.c_int32)]
        L.dc_get_state.argtypes = [P, C.c_int32, i32p]
        L.dc_get_latency.argtypes = [P, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_int32)]
        L.dc_rewind.argtypes = [P]
        L.dc_get_trace.argtypes = [P, C.c_int32, i32p, C.POINTER(C.c_float), C.POINTER(C.c_int32)]
        L.dc_autotune.argtypes = [P, C.POINTER(C.c_int32)]
        L.dc_autotune_cached.argtypes = [P, C.c_char_p, C.POINTER(dc_tune)]
        L.dc_set_shape.argtypes = [P, C.POINTER(dc_tune)]
        L.dc_get_shape.argtypes = [P, C.POINTER(dc_tune)]
        L.dc_last_timing.argtypes = [P, C.POINTER(C.c_float), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.dc_pending.argtypes = [P, C.POINTER(C.c_int64)]
        L.dc_topsis_tiles.argtypes = [C.c_int64, C.c_int32, C.c_int32, P, P, i32p, C.POINTER(C.c_float), P, P, P, P]
        L.dc_topsis_tiles_noalloc.argtypes = L.dc_topsis_tiles.argtypes
        L.dc_destroy.argtypes = [P]
        L.dc_destroy.restype = None
        L.dc_strerror.argtypes = [C.c_int]
        L.dc_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().dc_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != DC_OK:
        raise DcError(rc, what)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p32(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _stream_handle(stream) -> Optional[int]:
    """Accepts None, an int handle, or a torch.cuda.Stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Result:
    __slots__ = ("req_id", "instance", "status", "n", "failed_at", "hosts", "scores")

    def __init__(self, r: dc_result):
        self.req_id, self.instance, self.status = r.req_id, r.instance, r.status
        self.n, self.failed_at = r.n, r.failed_at
        self.hosts = np.frombuffer(r.host, dtype=np.int32, count=r.n).copy()
        self.scores = np.frombuffer(r.score, dtype=np.float32, count=r.n).copy()


# Contexts still open when the interpreter exits are destroyed by an exit
# hook, while the HIP runtime is whole, rather than by garbage collection
# during the interpreter's own teardown.
_live = weakref.WeakSet()


@atexit.register
def _close_live():
    for s in list(_live):
        s.close()


class Scheduler:
    """One libdcsched context (dc_create ... dc_destroy)."""

    def __init__(self, instances: List, method: int = DC_TOPSIS, mode: int = DC_MODE_PLAIN,
                 crit: Iterable[int] = DEFAULT_CRIT, cost: Optional[Iterable[int]] = None,
                 weight: Optional[Iterable[float]] = None, ahp_scale: int = DC_AHP_SAATY9,
                 stream=None, block: int = 0, trace_stride: int = 0, trace_cap: int = 0,
                 mem_budget: int = 0, grid: int = 0, graph: int = 0, grid_timeout_us: int = 0,
                 routing: int = 0):
        inst0 = instances[0]
        crit = list(crit)
        cost = list(cost) if cost is not None else [0] * len(crit)
        weight = list(weight) if weight is not None else [1.0 / len(crit)] * len(crit)
        cfg = dc_config()
        cfg.k, cfg.n_instances, cfg.mode, cfg.method, cfg.ahp_scale = inst0.k, len(instances), mode, method, ahp_scale
        cfg.host_cpu, cfg.host_ram = inst0.host_cpu, inst0.host_ram
        cfg.bw_host_edge, cfg.bw_edge_agg, cfg.bw_agg_core = inst0.bw_host_edge, inst0.bw_edge_agg, inst0.bw_agg_core
        cfg.ncrit = len(crit)
        for c in range(len(crit)):
            cfg.crit[c], cfg.crit_cost[c], cfg.weight[c] = crit[c], cost[c], weight[c]
        N = inst0.k ** 3 // 4
        self._hu = self._lu = None
        if any(i.host_used is not None for i in instances):
            self._hu = np.concatenate([(i.host_used if i.host_used is not None else np.zeros((2, N), np.int32))
                                       .reshape(-1) for i in instances]).astype(np.int32)
            cfg.host_used = self._hu.ctypes.data
        if any(i.link_used is not None for i in instances):
            self._lu = np.concatenate([(i.link_used if i.link_used is not None else np.zeros((3, N), np.int32))
                                       .reshape(-1) for i in instances]).astype(np.int32)
            cfg.link_used = self._lu.ctypes.data
        h = _stream_handle(stream)
        cfg.stream = h if h else None
        cfg.block, cfg.trace_stride, cfg.trace_cap, cfg.mem_budget = block, trace_stride, trace_cap, mem_budget
        cfg.grid = grid
        cfg.graph = graph
        cfg.grid_timeout_us = grid_timeout_us
        cfg.routing = routing
        self.N, self.I, self.k = N, len(instances), inst0.k
        self.cfg = cfg
        self._ctx = C.c_void_p()
        _check(lib().dc_create(C.byref(cfg), C.byref(self._ctx)), "dc_create")
        _live.add(self)

    def close(self):
        if self._ctx:
            lib().dc_destroy(self._ctx)
            self._ctx = C.c_void_p()
        _live.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, req, instance: int = 0) -> int:
        """Queue a request; with any of req.cpu_max, req.ram_max, req.bw_max
        set its demands are intervals (dc_submit_request_ranged)."""
        cpu, ram = _i32(req.cpu), _i32(req.ram)
        edges = _i32(req.edges).reshape(-1)
        pod = getattr(req, "pod", None)
        pod = _i32(pod) if pod is not None else None
        rid = C.c_int64()
        mx = [getattr(req, k, None) for k in ("cpu_max", "ram_max", "bw_max")]
        if all(x is None for x in mx):
            _check(lib().dc_submit_request(self._ctx, instance, len(cpu), _p32(cpu), _p32(ram), len(edges) // 3,
                                           _p32(edges) if len(edges) else None,
                                           _p32(pod) if pod is not None else None, C.byref(rid)),
                   "dc_submit_request")
            return rid.value
        cx, rx, bx = (None if x is None else _i32(x) for x in mx)
        opt = lambda a: _p32(a) if a is not None and len(a) else None
        _check(lib().dc_submit_request_ranged(self._ctx, instance, len(cpu), _p32(cpu), opt(cx), _p32(ram), opt(rx),
                                              len(edges) // 3, opt(edges), opt(bx), opt(pod), C.byref(rid)),
               "dc_submit_request_ranged")
        return rid.value

    def alloc(self, req_id: int, n: int, m: int):
        """What accepted request req_id (n containers, m edges) was given:
        (cpu[n], ram[n], bw[m])."""
        cpu, ram, bw = np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(max(m, 1), np.int32)
        _check(lib().dc_get_alloc(self._ctx, req_id, _p32(cpu), _p32(ram), _p32(bw)), "dc_get_alloc")
        return cpu, ram, bw[:m]

    def schedule(self, max_results: int = 1 << 20) -> List[Result]:
        out = []
        buf = (dc_result * 4096)()
        n = C.c_int32()
        remaining = max_results
        while True:
            _check(lib().dc_schedule(self._ctx, min(4096, remaining), buf, C.byref(n)), "dc_schedule")
            out.extend(Result(buf[i]) for i in range(n.value))
            remaining -= n.value
            if n.value < 4096 or remaining <= 0:
                return out

    def schedule_array(self, out: Optional[np.ndarray] = None) -> np.ndarray:
        """dc_schedule into a record array of RESULT_DTYPE (no per-result
        Python objects): returns the filled prefix of `out`, which is
        allocated for every queued request when not given."""
        if out is None:
            out = np.zeros(max(self.pending(), 1), RESULT_DTYPE)
        n = C.c_int32()
        _check(lib().dc_schedule(self._ctx, len(out), out.ctypes.data_as(C.POINTER(dc_result)), C.byref(n)),
               "dc_schedule")
        return out[: n.value]

    def release(self, req_id: int) -> int:
        return lib().dc_release(self._ctx, req_id)

    def paths(self, req_id: int) -> np.ndarray:
        n = C.c_int32()
        cap = DC_MAX_CONTAINERS * DC_MAX_CONTAINERS
        buf = np.zeros(6 * cap, np.int32)
        _check(lib().dc_get_paths(self._ctx, req_id, cap, _p32(buf), C.byref(n)), "dc_get_paths")
        return buf[: 6 * n.value].reshape(n.value, 6)

    def attempt(self, req_id: int) -> np.ndarray:
        n = C.c_int32()
        buf = np.zeros(DC_MAX_CONTAINERS, np.int32)
        _check(lib().dc_get_attempt(self._ctx, req_id, DC_MAX_CONTAINERS, _p32(buf), C.byref(n)), "dc_get_attempt")
        return buf[: n.value].copy()

    def latency_us(self) -> np.ndarray:
        """Service latency (us) of every scheduled request, id order."""
        n = C.c_int32()
        _check(lib().dc_get_latency(self._ctx, 0, None, C.byref(n)), "dc_get_latency")
        out = np.zeros(max(n.value, 1), np.float32)
        _check(lib().dc_get_latency(self._ctx, n.value, out.ctypes.data_as(C.POINTER(C.c_float)), C.byref(n)),
               "dc_get_latency")
        return out[: n.value]

    def state(self, instance: int = 0) -> np.ndarray:
        out = np.zeros(6 * self.N, np.int32)
        _check(lib().dc_get_state(self._ctx, instance, _p32(out)), "dc_get_state")
        return out.reshape(6, self.N)

    def rewind(self):
        _check(lib().dc_rewind(self._ctx), "dc_rewind")

    def trace(self):
        cap = self.cfg.trace_cap
        meta = np.zeros(4 * max(cap, 1), np.int32)
        scores = np.zeros(max(cap, 1) * self.N, np.float32)
        n = C.c_int32()
        _check(lib().dc_get_trace(self._ctx, cap, _p32(meta), scores.ctypes.data_as(C.POINTER(C.c_float)),
                                  C.byref(n)), "dc_get_trace")
        return meta[: 4 * n.value].reshape(-1, 4), scores[: n.value * self.N].reshape(-1, self.N)

    def autotune(self) -> int:
        b = C.c_int32()
        _check(lib().dc_autotune(self._ctx, C.byref(b)), "dc_autotune")
        return b.value

    def autotune_cached(self, cache_path: Optional[str] = None) -> dict:
        """dc_autotune_cached: the chosen shape (block, host_group,
        peer_chunk), whether it came from the cache, its time and the number
        of shapes timed."""
        t = dc_tune()
        path = cache_path.encode() if cache_path else None
        _check(lib().dc_autotune_cached(self._ctx, path, C.byref(t)), "dc_autotune_cached")
        return t.as_dict()

    def set_shape(self, block: int, host_group: int, peer_chunk: int):
        t = dc_tune(block, host_group, peer_chunk, 0, 0.0, 0)
        _check(lib().dc_set_shape(self._ctx, C.byref(t)), "dc_set_shape")

    def shape(self) -> dict:
        t = dc_tune()
        _check(lib().dc_get_shape(self._ctx, C.byref(t)), "dc_get_shape")
        return {"block": t.block, "host_group": t.host_group, "peer_chunk": t.peer_chunk}

    def pending(self) -> int:
        n = C.c_int64()
        _check(lib().dc_pending(self._ctx, C.byref(n)), "dc_pending")
        return n.value

    def try_submit(self, req, instance: int = 0):
        """Serving form: returns the request id, or None when admission is
        refused for now (DC_EAGAIN)."""
        try:
            return self.submit(req, instance)
        except DcError as e:
            if e.code == DC_EAGAIN:
                return None
            raise

    def drain(self, timeout_s: float = 120.0) -> List[Result]:
        """Serving form: polls until every published command completed."""
        import time
        out = []
        t0 = time.monotonic()
        while True:
            out.extend(self.schedule())
            if self.pending() == 0:
                out.extend(self.schedule())
                return out
            if time.monotonic() - t0 > timeout_s:
                raise TimeoutError("serving commands did not complete")
            time.sleep(1e-4)

    def last_timing(self):
        ms, la, st = C.c_float(), C.c_int64(), C.c_int64()
        _check(lib().dc_last_timing(self._ctx, C.byref(ms), C.byref(la), C.byref(st)), "dc_last_timing")
        return ms.value, la.value, st.value


def topsis_tiles(x, weight, cost=None, feasible=None, scores: bool = False, stream=None):
    """dc_topsis_tiles on device tensors: x int32 [T][C][N] (contiguous, on
    the GPU), feasible uint8 [T][N] or None.  Returns (best int32 [T],
    best_score float32 [T], scores float32 [T][N] or None), launched on
    `stream` (default: torch's current stream of x's device)."""
    import torch
    if x.dtype != torch.int32 or x.dim() != 3 or not x.is_cuda:
        raise ValueError("x must be an int32 [T][C][N] device tensor")
    x = x.contiguous()
    T, Cn, N = x.shape
    dev = x.device
    best = torch.empty(T, dtype=torch.int32, device=dev)
    bscore = torch.empty(T, dtype=torch.float32, device=dev)
    sc = torch.empty((T, N), dtype=torch.float32, device=dev) if scores else None
    fp = None
    if feasible is not None:
        if feasible.dtype != torch.uint8 or tuple(feasible.shape) != (T, N) or feasible.device != dev:
            raise ValueError("feasible must be a uint8 [T][N] tensor on x's device")
        feasible = feasible.contiguous()
        fp = feasible.data_ptr()
    w = (C.c_float * Cn)(*[float(v) for v in weight])
    cv = (C.c_int32 * Cn)(*[int(v) for v in (cost if cost is not None else [0] * Cn)])
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    _check(lib().dc_topsis_tiles(T, Cn, N, x.data_ptr(), fp, cv, w, sc.data_ptr() if sc is not None else None,
                                 best.data_ptr(), bscore.data_ptr(), _stream_handle(stream)),
           "dc_topsis_tiles")
    return best, bscore, sc


def topsis_tiles_noalloc(x, weight, best, best_score=None, cost=None, feasible=None, scores=None, stream=None):
    """dc_topsis_tiles_noalloc on caller-owned device tensors: x int32
    [T][C][N], feasible uint8 [T][N] or None, outputs best int32 [T],
    best_score float32 [T] or None, scores float32 [T][N] or None, all
    contiguous on one device.  Allocates nothing on the device; launched on
    `stream` (default: torch's current stream of x's device)."""
    import torch
    if x.dtype != torch.int32 or x.dim() != 3 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous int32 [T][C][N] device tensor")
    T, Cn, N = x.shape
    dev = x.device

    def out(t, dtype, shape, name):
        if t is None:
            return None
        if t.dtype != dtype or tuple(t.shape) != shape or t.device != dev or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} {list(shape)} tensor on x's device")
        return t.data_ptr()

    bp = out(best, torch.int32, (T,), "best")
    if bp is None:
        raise ValueError("best is required")
    sp = out(best_score, torch.float32, (T,), "best_score")
    scp = out(scores, torch.float32, (T, N), "scores")
    fp = out(feasible, torch.uint8, (T, N), "feasible")
    w = (C.c_float * Cn)(*[float(v) for v in weight])
    cv = (C.c_int32 * Cn)(*[int(v) for v in (cost if cost is not None else [0] * Cn)])
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    _check(lib().dc_topsis_tiles_noalloc(T, Cn, N, x.data_ptr(), fp, cv, w, scp, bp, sp, _stream_handle(stream)),
           "dc_topsis_tiles_noalloc")
