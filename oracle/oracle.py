"""ctypes binding of the C oracle (jet_oracle.c). TEST INFRASTRUCTURE ONLY.

Builds ``oracle/_build/libjetoracle.so`` with gcc on first use (or via
``build()``), then exposes numpy-level calls:

  refine(g, part0, k, ...)      -> RefineResult  (Algorithm 3 loop)
  jetlp(g, part, locked, k, ...) -> dict          (one Jetlp step, Algorithm 4)
  rebalance(g, part, kind, t, ...) -> dict        (one Jetrw / Jetrs step)
  partition(g, k, ...)           -> (part, traces, level_sizes)  (Algorithm 1)
  hem_map(g, level, seed)        -> (nc, map)
  contract(g, map, nc)           -> Graph
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jet_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "libjetoracle.so")

LP, RW, RS = 1, 2, 3


class OgGraph(C.Structure):
    _fields_ = [("n", C.c_int32), ("xadj", C.c_void_p), ("adjncy", C.c_void_p),
                ("vwgt", C.c_void_p), ("adjwgt", C.c_void_p)]


class OgParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("lambda_ppm", C.c_int32), ("c_num", C.c_int32),
                ("c_den", C.c_int32), ("phi_num", C.c_int32), ("phi_den", C.c_int32),
                ("stall_limit", C.c_int32), ("bmax", C.c_int32), ("deadzone_div", C.c_int32),
                ("level", C.c_int32), ("max_iters", C.c_int32), ("flags", C.c_int32),
                ("seed", C.c_uint64)]


class OgTrace(C.Structure):
    _fields_ = [("level", C.c_int32), ("t", C.c_int32), ("kind", C.c_int32), ("nX", C.c_int32),
                ("nM", C.c_int32), ("stall", C.c_int32), ("wcount", C.c_int32),
                ("balanced", C.c_int32), ("moved_w", C.c_int64), ("cut", C.c_int64),
                ("maxw", C.c_int64), ("best_cut", C.c_int64), ("digest", C.c_uint64)]


TRACE_FIELDS = [f[0] for f in OgTrace._fields_]


def build(force: bool = False) -> str:
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _configure(C.CDLL(build()))
    return _lib


def _configure(l):
    l.og_jetlp.restype = C.c_int32
    l.og_rebalance.restype = C.c_int32
    l.og_refine.restype = C.c_int32
    l.og_partition.restype = C.c_int32
    l.og_hem_map.restype = C.c_int32
    l.og_slot.restype = C.c_int32
    l.og_slot.argtypes = [C.c_int64]
    l.og_digest.restype = C.c_uint64
    return l


class use_library:
    """Context manager: route every call through another build of the oracle
    (used by the mutation test, which plants mistakes in a copy)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _configure(C.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data) if a is not None else None


class _G:
    """Keeps contiguous copies alive while the C struct points at them."""

    def __init__(self, g):
        self.xadj = np.ascontiguousarray(g.xadj, dtype=np.int64)
        self.adjncy = np.ascontiguousarray(g.adjncy, dtype=np.int32)
        self.vwgt = np.ascontiguousarray(g.vwgt, dtype=np.int32)
        self.adjwgt = np.ascontiguousarray(g.adjwgt, dtype=np.int32)
        self.s = OgGraph(int(self.xadj.shape[0] - 1), self.xadj.ctypes.data, self.adjncy.ctypes.data,
                         self.vwgt.ctypes.data, self.adjwgt.ctypes.data)


# Jetlp ablation flags (same bit values as the library's public interface)
F_NO_LOCKS = 0x8
F_NO_AFTERBURNER = 0x10
F_TWO_HOP = 0x20
F_BFS_START = 0x40


def make_params(k, lambda_ppm=30000, c=None, phi=(999, 1000), stall_limit=12, bmax=2,
                deadzone_div=10, level=0, max_iters=0, seed=0, flags=0) -> OgParams:
    cn, cd = (0, 0) if c is None else c
    return OgParams(k, lambda_ppm, cn, cd, phi[0], phi[1], stall_limit, bmax, deadzone_div, level,
                    max_iters, flags, seed & ((1 << 64) - 1))


def trace_to_dicts(arr, n):
    out = []
    for i in range(n):
        r = arr[i]
        out.append({f: getattr(r, f) for f in TRACE_FIELDS})
    return out


def slot(x: int) -> int:
    return lib().og_slot(int(x))


def digest(part: np.ndarray) -> int:
    p = np.ascontiguousarray(part, dtype=np.int32)
    return int(lib().og_digest(C.c_int32(p.shape[0]), _ptr(p)))


def jetlp(g, part, locked, k, **kw):
    G = _G(g)
    n = G.s.n
    prm = make_params(k, **kw)
    P = np.ascontiguousarray(part, dtype=np.int32)
    L = np.ascontiguousarray(locked, dtype=np.uint8)
    pd = np.zeros(n, np.int32); F = np.zeros(n, np.int64); cs = np.zeros(n, np.int64)
    inX = np.zeros(n, np.uint8); F2 = np.zeros(n, np.int64); mv = np.zeros(n, np.uint8)
    nX = C.c_int32(0)
    nM = lib().og_jetlp(C.byref(G.s), C.byref(prm), _ptr(P), _ptr(L), _ptr(pd), _ptr(F), _ptr(cs),
                        _ptr(inX), _ptr(F2), _ptr(mv), C.byref(nX))
    return dict(pd=pd, F=F, conn_s=cs, inX=inX.astype(bool), F2=F2, move=mv.astype(bool),
                nX=nX.value, nM=nM)


def rebalance(g, part, kind, t, k, **kw):
    G = _G(g)
    n = G.s.n
    prm = make_params(k, **kw)
    P = np.ascontiguousarray(part, dtype=np.int32)
    dest = np.zeros(n, np.int32); loss = np.zeros(n, np.int64); sl = np.zeros(n, np.int32)
    cd = np.zeros(n, np.int32)
    nc = C.c_int32(0)
    nM = lib().og_rebalance(C.byref(G.s), C.byref(prm), _ptr(P), C.c_int32(kind), C.c_int32(t),
                            _ptr(dest), _ptr(loss), _ptr(sl), _ptr(cd), C.byref(nc))
    return dict(dest=dest, loss=loss, slot=sl, cand_dest=cd, ncand=nc.value, nM=nM)


@dataclass
class RefineResult:
    part: np.ndarray        # P_best
    iter_part: np.ndarray   # P_iter at exit
    iters: int
    trace: list
    cut: int
    maxw: int
    balanced: bool
    o: int


def refine(g, part0, k, trace_cap=100000, **kw) -> RefineResult:
    G = _G(g)
    n = G.s.n
    prm = make_params(k, **kw)
    P = np.ascontiguousarray(part0, dtype=np.int32).copy()
    it = np.zeros(n, np.int32)
    tr = (OgTrace * max(trace_cap, 1))()
    st = np.zeros(4, np.int64)
    iters = lib().og_refine(C.byref(G.s), C.byref(prm), _ptr(P), tr, C.c_int32(trace_cap), _ptr(it),
                            _ptr(st))
    return RefineResult(P, it, iters, trace_to_dicts(tr, min(iters, trace_cap)), int(st[0]),
                        int(st[1]), bool(st[2]), int(st[3]))


def partition(g, k, trace_cap=200000, **kw):
    G = _G(g)
    n = G.s.n
    prm = make_params(k, **kw)
    P = np.zeros(n, np.int32)
    tr = (OgTrace * max(trace_cap, 1))()
    ntr = C.c_int32(0)
    sizes = np.zeros(64, np.int32)
    st = np.zeros(4, np.int64)
    nl = lib().og_partition(C.byref(G.s), C.byref(prm), _ptr(P), tr, C.c_int32(trace_cap), C.byref(ntr),
                            _ptr(sizes), _ptr(st))
    return dict(part=P, trace=trace_to_dicts(tr, ntr.value), level_sizes=sizes[:nl].copy(),
                cut=int(st[0]), maxw=int(st[1]), balanced=bool(st[2]), o=int(st[3]))


def bfs_part(g, k):
    """Graph-growing start of a coarsest graph (og_bfs_part): components
    searched breadth-first from their smallest id, vertices ordered by (that
    id, distance, id), the order cut into k runs of equal vertex weight."""
    G = _G(g)
    P = np.zeros(max(G.s.n, 1), np.int32)
    lib().og_bfs_part(C.byref(G.s), C.c_int32(k), _ptr(P))
    return P[:G.s.n]


def hem_map(g, level, seed, two_hop=False):
    G = _G(g)
    m = np.zeros(max(G.s.n, 1), np.int32)
    nc = lib().og_hem_map(C.byref(G.s), C.c_int32(level), C.c_uint64(seed & ((1 << 64) - 1)),
                          C.c_int32(1 if two_hop else 0), _ptr(m))
    return nc, m[:G.s.n]


def contract(g, cmap, nc):
    from paper_2304_13194_amd.inputs import Graph
    G = _G(g)
    M = np.ascontiguousarray(cmap, dtype=np.int32)
    cx = C.c_void_p(); ca = C.c_void_p(); cv = C.c_void_p(); cw = C.c_void_p()
    lib().og_contract(C.byref(G.s), _ptr(M), C.c_int32(nc), C.byref(cx), C.byref(ca), C.byref(cv),
                      C.byref(cw))
    xadj = np.ctypeslib.as_array(C.cast(cx, C.POINTER(C.c_int64)), shape=(nc + 1,)).copy()
    nnz = int(xadj[-1])
    adj = (np.ctypeslib.as_array(C.cast(ca, C.POINTER(C.c_int32)), shape=(max(nnz, 1),))[:nnz].copy())
    vw = np.ctypeslib.as_array(C.cast(cv, C.POINTER(C.c_int32)), shape=(max(nc, 1),))[:nc].copy()
    ew = (np.ctypeslib.as_array(C.cast(cw, C.POINTER(C.c_int32)), shape=(max(nnz, 1),))[:nnz].copy())
    for p in (cx, ca, cv, cw):
        lib().og_free(p)
    return Graph(xadj, adj, vw, ew, name="coarse")
