"""FP64 CPU oracle for the network-aware container scheduler (arXiv 1909.07673).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It wraps the plain C
implementation in ``dc_oracle.c`` (explicit fat-tree graph, literal TOPSIS
and AHP steps, FCFS commit / rollback / release) and shares no code with the
GPU library.  Every function is pinned by the CPU tests; none is
"parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CRIT_CPU, CRIT_RAM, CRIT_ACTIVE, CRIT_PATHBW, CRIT_UPLINK, CRIT_HOPS = range(6)
TOPSIS, AHP = 0, 1
SAATY9, RATIO, DIFF = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Method(C.Structure):
    _fields_ = [("method", C.c_int32), ("ahp_scale", C.c_int32), ("ncrit", C.c_int32),
                ("route_end", C.c_int32), ("crit", C.c_int32 * 8), ("cost", C.c_int32 * 8),
                ("weight", C.c_double * 8)]


def method(kind=TOPSIS, crit=(CRIT_CPU, CRIT_RAM, CRIT_ACTIVE, CRIT_PATHBW), cost=None,
           weight=None, scale=SAATY9, route_end=False) -> Method:
    """route_end: route a request's links after its last pod is placed
    (section V-D) instead of at each placement."""
    m = Method()
    m.method, m.ahp_scale, m.ncrit, m.route_end = kind, scale, len(crit), int(route_end)
    cost = cost or [0] * len(crit)
    weight = weight or [1.0 / len(crit)] * len(crit)
    for c in range(len(crit)):
        m.crit[c], m.cost[c], m.weight[c] = crit[c], cost[c], weight[c]
    return m


def build_variant(src_text: str, out_path: str) -> str:
    """Compile oracle C source text (a variant of dc_oracle.c with a planted
    mistake, written by a test) into out_path."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", out_path, src, "-lm"])
    return out_path


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = load(_LIB)
    return _lib


def load(path: str):
    """Load an oracle library and declare its entry points."""
    L = C.CDLL(path)
    P = C.c_void_p
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
    L.or_create.restype = P
    L.or_create.argtypes = [C.c_int] * 6 + [P, P]
    L.or_destroy.argtypes = [P]
    L.or_num_hosts.argtypes = [P]
    L.or_get_state.argtypes = [P, i32p]
    L.or_set_link.argtypes = [P, C.c_int, C.c_int64]
    L.or_widest_from.argtypes = [P, C.c_int, i64p, i32p]
    L.or_widest_enum.argtypes = [P, C.c_int, C.c_int, C.POINTER(C.c_int64), i32p, C.POINTER(C.c_int32)]
    L.or_topsis.argtypes = [C.c_int, C.c_int, f64p, f64p, i32p, f64p]
    L.or_ahp.argtypes = [C.c_int, C.c_int, f64p, f64p, i32p, C.c_int, f64p, P, P]
    L.or_saaty.restype = C.c_double
    L.or_saaty.argtypes = [C.c_double, C.c_double]
    L.or_diff.restype = C.c_double
    L.or_diff.argtypes = [C.c_double, C.c_double]
    L.or_step_scores.argtypes = [P, C.POINTER(Method), C.c_int, C.c_int, C.c_int, i32p, i32p,
                                 f64p, i32p, f64p]
    L.or_run_request.argtypes = [P, C.POINTER(Method), C.c_int, i32p, i32p, C.c_int, P, P, P, P, P,
                                 P, P, P, P, P, P, P, P, P, P, P, P]
    L.or_run_request_pods.argtypes = [P, C.POINTER(Method), C.c_int, i32p, i32p, C.c_int, P, P, P, P, P,
                                      P, P, P, P, P, P, P, P, P, P, P, P, P]
    L.or_units.argtypes = [C.c_int, P, i32p, i32p]
    L.or_release.argtypes = [P, C.c_int64]
    L.or_get_paths.argtypes = [P, C.c_int64, C.c_int, i32p, i64p]
    L.or_get_hosts.argtypes = [P, C.c_int64, i32p]
    L.or_set_threads.argtypes = [C.c_int]
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def topsis(X, w, cost=None):
    """TOPSIS closeness of every alternative; X is criterion-major [C][N]."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Cn, N = X.shape
    out = np.zeros(N)
    c = np.ascontiguousarray(cost if cost is not None else [0] * Cn, dtype=np.int32)
    lib().or_topsis(N, Cn, X, np.ascontiguousarray(w, dtype=np.float64), c, out)
    return out


def ahp(X, w, cost=None, scale=SAATY9, return_levels=False):
    """AHP global priority PG of every alternative; X is criterion-major [C][N]."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Cn, N = X.shape
    out = np.zeros(N)
    p1 = np.zeros(Cn)
    p2 = np.zeros((Cn, N))
    c = np.ascontiguousarray(cost if cost is not None else [0] * Cn, dtype=np.int32)
    lib().or_ahp(N, Cn, X, np.ascontiguousarray(w, dtype=np.float64), c, scale, out,
                 _ptr(p1), _ptr(p2))
    return (out, p1, p2) if return_levels else out


def units(n, pod=None):
    """Pods of a request as the oracle numbers them: (unit[i] = pod of
    container i, first[g] = smallest container of pod g); without pods every
    container is its own pod."""
    unit = np.zeros(n, dtype=np.int32)
    first = np.zeros(n, dtype=np.int32)
    p = None if pod is None else np.ascontiguousarray(pod, dtype=np.int32)
    nu = lib().or_units(n, _ptr(p), unit, first)
    return unit, first[:nu].copy()


def set_threads(n: int = 0) -> int:
    """Threads the AHP comparison matrices are shared out over (0: keep the
    current count, from OMP_NUM_THREADS or the CPU count); the results do not
    depend on it.  Returns the count in effect."""
    return lib().or_set_threads(n)


def saaty(p, q) -> float:
    return lib().or_saaty(float(p), float(q))


def diff(p, q) -> float:
    return lib().or_diff(float(p), float(q))


class Oracle:
    """One data center held by the oracle."""

    def __init__(self, inst, meth: Method = None):
        self.k = inst.k
        self.N = inst.k ** 3 // 4
        hu = None if inst.host_used is None else np.ascontiguousarray(inst.host_used, dtype=np.int32)
        lu = None if inst.link_used is None else np.ascontiguousarray(inst.link_used, dtype=np.int32)
        self._keep = (hu, lu)
        self.h = lib().or_create(inst.k, inst.host_cpu, inst.host_ram, inst.bw_host_edge,
                                 inst.bw_edge_agg, inst.bw_agg_core, _ptr(hu), _ptr(lu))
        if not self.h:
            raise ValueError("bad fat-tree parameters")
        self.m = meth if meth is not None else method()

    def close(self):
        if self.h:
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self) -> np.ndarray:
        out = np.zeros(6 * self.N, dtype=np.int32)
        lib().or_get_state(self.h, out)
        return out.reshape(6, self.N)

    def set_link(self, link: int, res: int):
        lib().or_set_link(self.h, link, res)

    def widest_from(self, src: int):
        W = np.zeros(self.N, dtype=np.int64)
        hops = np.zeros(self.N, dtype=np.int32)
        lib().or_widest_from(self.h, src, W, hops)
        return W, hops

    def widest_enum(self, u: int, v: int):
        b = C.c_int64()
        hops = C.c_int32()
        links = np.zeros(6, dtype=np.int32)
        cnt = lib().or_widest_enum(self.h, u, v, C.byref(b), links, C.byref(hops))
        return cnt, b.value, hops.value, links[: hops.value].copy()

    def step_scores(self, cpu, ram, peer_hosts, peer_bw):
        ph = np.ascontiguousarray(peer_hosts, dtype=np.int32)
        pb = np.ascontiguousarray(peer_bw, dtype=np.int32)
        X = np.zeros((8, self.N))
        feas = np.zeros(self.N, dtype=np.int32)
        score = np.zeros(self.N)
        lib().or_step_scores(self.h, C.byref(self.m), cpu, ram, len(ph), ph, pb, X, feas, score)
        return X[: self.m.ncrit].copy(), feas.astype(bool), score

    def run_request(self, req, follow=None, detail=False, dump=False):
        """Schedule one request.  Returns a dict with status (1 accepted,
        0 rejected, <0 error), hosts, scores (per container), failed_at,
        rec_id, the allocations cpu_a, ram_a (per container) and bw_a (per
        edge) of an accepted request and, with detail=True, the per-step own
        choice / top score / top-two gap / chosen score (ref_host, ref_top,
        ref_gap, step_scores) and, when following, tie_low: per step the
        lowest-index server below the followed one with identical criteria
        that is feasible and commits (-1 when none; anything else breaks
        the lowest-index rule on exact ties).  A step places one pod (one container without
        pods); follow and the per-step outputs are indexed by step.  The
        request's cpu, ram and edge demands are minima; optional cpu_max,
        ram_max and bw_max give the interval maxima (section II-A)."""
        n = req.n
        cpu = np.ascontiguousarray(req.cpu, dtype=np.int32)
        ram = np.ascontiguousarray(req.ram, dtype=np.int32)
        edges = np.ascontiguousarray(req.edges, dtype=np.int32).reshape(-1)

        def opt(name):
            v = getattr(req, name, None)
            return None if v is None else np.ascontiguousarray(v, dtype=np.int32)
        cx, rx, bx = opt("cpu_max"), opt("ram_max"), opt("bw_max")
        cpu_a = np.full(n, -1, dtype=np.int32)
        ram_a = np.full(n, -1, dtype=np.int32)
        bw_a = np.full(max(req.m, 1), -1, dtype=np.int32)
        pod = getattr(req, "pod", None)
        pod = None if pod is None else np.ascontiguousarray(pod, dtype=np.int32)
        nu = len(units(n, pod)[1])
        fol = None if follow is None else np.ascontiguousarray(follow, dtype=np.int32)
        host = np.full(n, -1, dtype=np.int32)
        score = np.zeros(n)
        rh = np.full(nu, -1, dtype=np.int32) if detail else None
        rt = np.zeros(nu) if detail else None
        rg = np.zeros(nu) if detail else None
        tl = np.full(nu, -1, dtype=np.int32) if detail else None
        dmp = np.zeros((nu, self.N)) if dump else None
        fa = np.zeros(1, dtype=np.int32)
        rid = np.zeros(1, dtype=np.int64)
        if pod is None:
            st = lib().or_run_request(self.h, C.byref(self.m), n, cpu, ram, req.m, _ptr(edges), _ptr(cx),
                                      _ptr(rx), _ptr(bx), _ptr(fol), _ptr(host), _ptr(score), _ptr(rh),
                                      _ptr(rt), _ptr(rg), _ptr(dmp), _ptr(fa), _ptr(rid), _ptr(cpu_a),
                                      _ptr(ram_a), _ptr(bw_a), _ptr(tl))
        else:
            st = lib().or_run_request_pods(self.h, C.byref(self.m), n, cpu, ram, req.m, _ptr(edges), _ptr(cx),
                                           _ptr(rx), _ptr(bx), _ptr(pod), _ptr(fol), _ptr(host), _ptr(score),
                                           _ptr(rh), _ptr(rt), _ptr(rg), _ptr(dmp), _ptr(fa), _ptr(rid),
                                           _ptr(cpu_a), _ptr(ram_a), _ptr(bw_a), _ptr(tl))
        out = dict(status=st, hosts=host, scores=score, failed_at=int(fa[0]), rec_id=int(rid[0]),
                   cpu_a=cpu_a, ram_a=ram_a, bw_a=bw_a[: req.m])
        if detail:
            unit, first = units(n, pod)
            out.update(ref_host=rh, ref_top=rt, ref_gap=rg, step_scores=score[first], tie_low=tl)
        if dump:
            out["dump"] = dmp
        return out

    def release(self, rec_id: int) -> int:
        return lib().or_release(self.h, rec_id)

    def paths(self, rec_id: int):
        cap = 64 * 64
        links = np.zeros(6 * cap, dtype=np.int32)
        bw = np.zeros(cap, dtype=np.int64)
        n = lib().or_get_paths(self.h, rec_id, cap, links, bw)
        return links[: 6 * n].reshape(n, 6), bw[:n]
