"""Python binding of libjet.so: argument marshalling only.

Every computation runs in the library's HIP kernels; this module converts
torch CUDA tensors into the C ABI's device pointers and structs and passes
torch's current HIP stream. It raises if libjet.so is missing or if a
tensor is not on the GPU; there is no fallback path.

Names follow the C ABI (include/jet.h): ``refine``, ``refine_batch``,
``lp_step``, ``rebalance_step``, ``coarsen``, ``partition`` and ``Server``
(``jet_server_*``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libjet.so")

JET_OK, JET_EINVAL, JET_EGRAPH, JET_EPART, JET_EOVERFLOW, JET_ENOMEM, JET_EHIP, JET_EAGAIN, JET_ELIMIT = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
JET_F_VALIDATE = 0x1
JET_F_RETURN_ITER = 0x2
JET_F_PROFILE = 0x4
JET_F_LP_NO_LOCKS = 0x8
JET_F_LP_NO_AFTERBURNER = 0x10
JET_F_TWO_HOP = 0x20
JET_F_BFS_START = 0x40
JET_F_ASYNC = 0x80
JET_F_CONN_TABLE = 0x100
KIND_LP, KIND_RW, KIND_RS = 1, 2, 3

# Every function declared in include/jet.h.
EXPORTS = [
    "jet_context_create", "jet_context_destroy", "jet_strerror", "jet_last_hip_error",
    "jet_refine", "jet_refine_noalloc", "jet_refine_batch", "jet_lp_step", "jet_rebalance_step", "jet_coarsen",
    "jet_hierarchy_levels", "jet_hierarchy_level", "jet_hierarchy_free", "jet_partition",
    "jet_bfs_start", "jet_gather_ceiling", "jet_server_create", "jet_server_submit", "jet_server_poll", "jet_server_wait",
    "jet_server_info_get", "jet_server_destroy",
]


class JetError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("reserved", C.c_int32), ("nnz", C.c_int64),
                ("xadj", C.c_void_p), ("adjncy", C.c_void_p), ("vwgt", C.c_void_p),
                ("adjwgt", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("lambda_ppm", C.c_int32), ("c_num", C.c_int32),
                ("c_den", C.c_int32), ("phi_num", C.c_int32), ("phi_den", C.c_int32),
                ("stall_limit", C.c_int32), ("weak_rebalance_iters", C.c_int32),
                ("deadzone_div", C.c_int32), ("level", C.c_int32), ("max_iters", C.c_int32),
                ("flags", C.c_uint32), ("seed", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [("cut", C.c_int64), ("max_part_weight", C.c_int64), ("o", C.c_int64),
                ("sigma", C.c_int64), ("total_weight", C.c_int64), ("balanced", C.c_int32),
                ("iters", C.c_int32), ("lp_iters", C.c_int32), ("rw_iters", C.c_int32),
                ("rs_iters", C.c_int32), ("levels", C.c_int32), ("ms_total", C.c_float),
                ("ms_refine", C.c_float), ("ms_coarsen", C.c_float), ("ms_init", C.c_float),
                ("ms_gain", C.c_float), ("gain_passes", C.c_int32), ("gain_entries", C.c_int64),
                ("gain_rows", C.c_int64), ("gain_vertices", C.c_int64), ("batch_tile", C.c_int32),
                ("batch_group", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TraceRec(C.Structure):
    _fields_ = [("level", C.c_int32), ("t", C.c_int32), ("kind", C.c_int32), ("nX", C.c_int32),
                ("nM", C.c_int32), ("stall", C.c_int32), ("wcount", C.c_int32),
                ("balanced", C.c_int32), ("moved_w", C.c_int64), ("cut", C.c_int64),
                ("maxw", C.c_int64), ("best_cut", C.c_int64), ("digest", C.c_uint64)]


class Trace(C.Structure):
    _fields_ = [("recs", C.c_void_p), ("cap", C.c_int32), ("count", C.c_int32),
                ("total", C.c_int32), ("reserved", C.c_int32)]


class Job(C.Structure):
    _fields_ = [("graph", Csr), ("params", Params), ("part_out", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("levels", C.c_int32), ("iters", C.c_int32),
                ("balanced", C.c_int32), ("cut", C.c_int64), ("max_part_weight", C.c_int64),
                ("t_submit_ms", C.c_double), ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double),
                ("steps", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("steps", C.c_int64),
                ("step_jobs", C.c_int64), ("active", C.c_int32), ("queued", C.c_int32),
                ("hbm_in_use", C.c_int64), ("busy_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


TRACE_FIELDS = [f for f, _ in TraceRec._fields_]

_lib = None
_hiplib = None


def _hip():
    """The HIP runtime, for copying library-owned hierarchy levels to the host."""
    global _hiplib
    if _hiplib is None:
        _hiplib = C.CDLL("libamdhip64.so")
    return _hiplib


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libjet.so not built ({LIB_PATH}); run python -m paper_2304_13194_amd.build")
        L = C.CDLL(LIB_PATH)
        L.jet_strerror.restype = C.c_char_p
        L.jet_hierarchy_level.argtypes = [C.c_void_p, C.c_int, C.POINTER(Csr), C.POINTER(C.c_void_p)]
        L.jet_hierarchy_levels.argtypes = [C.c_void_p]
        L.jet_hierarchy_free.argtypes = [C.c_void_p]
        L.jet_context_destroy.argtypes = [C.c_void_p]
        L.jet_last_hip_error.argtypes = [C.c_void_p]
        L.jet_server_create.argtypes = [C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t, C.c_int32]
        L.jet_server_submit.argtypes = [C.c_void_p, C.POINTER(Job), C.POINTER(C.c_uint64)]
        L.jet_server_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Result)]
        L.jet_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(Result)]
        L.jet_server_info_get.argtypes = [C.c_void_p, C.POINTER(ServerInfo)]
        L.jet_server_destroy.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _check(st, what):
    if st != JET_OK:
        raise JetError(st, f"{what}: {lib().jet_strerror(st).decode()}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class DeviceGraph:
    """Device CSR; vwgt / adjwgt may be None (unit weights)."""
    xadj: torch.Tensor
    adjncy: torch.Tensor
    vwgt: torch.Tensor | None
    adjwgt: torch.Tensor | None

    @property
    def n(self):
        return int(self.xadj.shape[0] - 1)

    @property
    def nnz(self):
        return int(self.adjncy.shape[0])

    def csr(self) -> Csr:
        return Csr(self.n, 0, self.nnz, _ptr(self.xadj), _ptr(self.adjncy), _ptr(self.vwgt),
                   _ptr(self.adjwgt))


def to_device(g, unit_vwgt=False, unit_adjwgt=False, device="cuda") -> DeviceGraph:
    """Copy a host graph (``inputs.Graph``) to the GPU."""
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
    return DeviceGraph(t(g.xadj, np.int64), t(g.adjncy, np.int32),
                       None if unit_vwgt else t(g.vwgt, np.int32),
                       None if unit_adjwgt else t(g.adjwgt, np.int32))


def make_params(k, lambda_ppm=30000, c=None, phi=None, stall_limit=0, weak_rebalance_iters=0,
                deadzone_div=0, level=0, max_iters=0, flags=0, seed=0) -> Params:
    cn, cd = (0, 0) if c is None else c
    pn, pd = (0, 0) if phi is None else phi
    return Params(k, lambda_ppm, cn, cd, pn, pd, stall_limit, weak_rebalance_iters, deadzone_div,
                  level, max_iters, flags, seed & ((1 << 64) - 1))


class Context:
    def __init__(self, device=None):
        dev = torch.cuda.current_device() if device is None else device
        self.h = C.c_void_p()
        _check(lib().jet_context_create(C.byref(self.h), C.c_int(dev)), "jet_context_create")

    def close(self):
        if self.h:
            lib().jet_context_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def _trace_buf(cap):
    if cap <= 0:
        return None, None
    arr = (TraceRec * cap)()
    return arr, Trace(C.cast(arr, C.c_void_p), cap, 0, 0, 0)


def _trace_list(arr, tr):
    if tr is None:
        return None
    return [{f: getattr(arr[i], f) for f in TRACE_FIELDS} for i in range(tr.count)]


def refine(g: DeviceGraph, part: torch.Tensor, k: int, trace_cap=0, ctx=None, part_weights=False,
           **kw):
    """jet_refine: refines ``part`` (int32 device tensor) in place to P_best.

    Returns (stats dict, trace list or None, part weights tensor or None)."""
    ctx = ctx or default_context()
    prm = make_params(k, **kw)
    st = Stats()
    arr, tr = _trace_buf(trace_cap)
    pw = torch.empty(k, dtype=torch.int64, device=part.device) if part_weights else None
    csr = g.csr()
    s = lib().jet_refine(ctx.h, C.byref(csr), C.byref(prm), _ptr(part), _ptr(pw), C.byref(st),
                         C.byref(tr) if tr is not None else None, _stream())
    _check(s, "jet_refine")
    out = st.as_dict()
    if tr is not None:
        out["trace_total"] = tr.total
    return out, _trace_list(arr, tr), pw


class AsyncRefine:
    """Handle of a jet_refine call made with JET_F_ASYNC: keeps the host
    buffers the library completes from the stream alive until ``wait``."""

    def __init__(self, st, arr, tr, pw, stream):
        self._st, self._arr, self._tr, self._pw, self._stream = st, arr, tr, pw, stream

    def wait(self):
        """Synchronises the call's stream; returns (stats, trace, part weights)."""
        self._stream.synchronize()
        out = self._st.as_dict()
        if self._tr is not None:
            out["trace_total"] = self._tr.total
        return out, _trace_list(self._arr, self._tr), self._pw


def refine_async(g: DeviceGraph, part: torch.Tensor, k: int, max_iters: int, trace_cap=0, ctx=None,
                 part_weights=False, flags=0, **kw) -> AsyncRefine:
    """jet_refine with JET_F_ASYNC: returns once the iterations are enqueued
    on torch's current stream."""
    ctx = ctx or default_context()
    prm = make_params(k, max_iters=max_iters, flags=flags | JET_F_ASYNC, **kw)
    st = Stats()
    arr, tr = _trace_buf(trace_cap)
    pw = torch.empty(k, dtype=torch.int64, device=part.device) if part_weights else None
    csr = g.csr()
    stream = torch.cuda.current_stream()
    s = lib().jet_refine(ctx.h, C.byref(csr), C.byref(prm), _ptr(part), _ptr(pw), C.byref(st),
                         C.byref(tr) if tr is not None else None, C.c_void_p(stream.cuda_stream))
    _check(s, "jet_refine (asynchronous)")
    return AsyncRefine(st, arr, tr, pw, stream)


# Size of the static workspace array of jet_refine_noalloc (bytes per GPU).
NOALLOC_SCRATCH_BYTES = 128 << 20


def refine_noalloc(g: DeviceGraph, part: torch.Tensor, k: int, trace_cap=0, ctx=None, part_weights=False,
                   **kw):
    """jet_refine_noalloc: as ``refine``, with the library's workspace taken
    from its static per-GPU scratch array (the call allocates nothing).
    ``part_weights`` must then be a preallocated int64 device tensor of k
    entries (or False); the trace buffer is host memory."""
    ctx = ctx or default_context()
    prm = make_params(k, **kw)
    st = Stats()
    arr, tr = _trace_buf(trace_cap)
    pw = part_weights if isinstance(part_weights, torch.Tensor) else None
    csr = g.csr()
    s = lib().jet_refine_noalloc(ctx.h, C.byref(csr), C.byref(prm), _ptr(part), _ptr(pw), C.byref(st),
                                 C.byref(tr) if tr is not None else None, _stream())
    _check(s, "jet_refine_noalloc")
    out = st.as_dict()
    if tr is not None:
        out["trace_total"] = tr.total
    return out, _trace_list(arr, tr), pw


def refine_batch(graphs, parts, params, trace_cap=0, ctx=None):
    """jet_refine_batch: refines ``parts[i]`` of ``graphs[i]`` in place, all in
    one launch sequence. ``params`` is a list of keyword dicts for
    ``make_params`` (``k`` included). Returns (list of stats dicts, list of
    traces or None)."""
    ctx = ctx or default_context()
    m = len(graphs)
    if len(parts) != m or len(params) != m:
        raise ValueError("graphs, parts and params must have the same length")
    csrs = (Csr * max(m, 1))(*[g.csr() for g in graphs])
    prms = (Params * max(m, 1))(*[make_params(**p) for p in params])
    ptrs = (C.c_void_p * max(m, 1))(*[_ptr(p) for p in parts])
    stats = (Stats * max(m, 1))()
    bufs, trs = [], None
    if trace_cap > 0:
        trs = (Trace * max(m, 1))()
        for i in range(m):
            arr, tr = _trace_buf(trace_cap)
            bufs.append(arr)
            trs[i] = tr
    s = lib().jet_refine_batch(ctx.h, C.c_int32(m), csrs, prms, ptrs, stats,
                               trs if trs is not None else None, _stream())
    _check(s, "jet_refine_batch")
    out = [stats[i].as_dict() for i in range(m)]
    traces = None
    if trs is not None:
        traces = []
        for i in range(m):
            out[i]["trace_total"] = trs[i].total
            traces.append(_trace_list(bufs[i], trs[i]))
    return out, traces


def lp_step(g: DeviceGraph, part: torch.Tensor, locked: torch.Tensor, k: int, ctx=None, **kw):
    """jet_lp_step: one Jetlp step. Returns dict of device tensors."""
    ctx = ctx or default_context()
    prm = make_params(k, **kw)
    n = g.n
    dev = part.device
    out = dict(pd=torch.empty(n, dtype=torch.int32, device=dev),
               F=torch.empty(n, dtype=torch.int64, device=dev),
               conn_s=torch.empty(n, dtype=torch.int64, device=dev),
               inX=torch.empty(n, dtype=torch.uint8, device=dev),
               F2=torch.empty(n, dtype=torch.int64, device=dev),
               move=torch.empty(n, dtype=torch.uint8, device=dev))
    csr = g.csr()
    s = lib().jet_lp_step(ctx.h, C.byref(csr), C.byref(prm), _ptr(part), _ptr(locked), _ptr(out["pd"]),
                          _ptr(out["F"]), _ptr(out["conn_s"]), _ptr(out["inX"]), _ptr(out["F2"]),
                          _ptr(out["move"]), _stream())
    _check(s, "jet_lp_step")
    return out


def rebalance_step(g: DeviceGraph, part: torch.Tensor, kind: int, t: int, k: int, ctx=None, **kw):
    """jet_rebalance_step: one Jetrw (kind 2) / Jetrs (kind 3) step."""
    ctx = ctx or default_context()
    prm = make_params(k, **kw)
    n = g.n
    dev = part.device
    out = dict(dest=torch.empty(n, dtype=torch.int32, device=dev),
               loss=torch.empty(n, dtype=torch.int64, device=dev),
               slot=torch.empty(n, dtype=torch.int32, device=dev))
    csr = g.csr()
    s = lib().jet_rebalance_step(ctx.h, C.byref(csr), C.byref(prm), _ptr(part), C.c_int32(kind),
                                 C.c_int32(t), _ptr(out["dest"]), _ptr(out["loss"]), _ptr(out["slot"]),
                                 _stream())
    _check(s, "jet_rebalance_step")
    return out


def partition(g: DeviceGraph, k: int, trace_cap=0, ctx=None, **kw):
    """jet_partition: full multilevel partition. Returns (part tensor, stats, trace)."""
    ctx = ctx or default_context()
    prm = make_params(k, **kw)
    st = Stats()
    arr, tr = _trace_buf(trace_cap)
    part = torch.empty(g.n, dtype=torch.int32, device=g.xadj.device)
    csr = g.csr()
    s = lib().jet_partition(ctx.h, C.byref(csr), C.byref(prm), _ptr(part), C.byref(st),
                            C.byref(tr) if tr is not None else None, _stream())
    _check(s, "jet_partition")
    out = st.as_dict()
    if tr is not None:
        out["trace_total"] = tr.total
    return part, out, _trace_list(arr, tr)


def bfs_start(g: DeviceGraph, k: int, ctx=None):
    """jet_bfs_start: graph-growing partition (components grown breadth-first
    from their smallest id, cut into k runs of equal vertex weight)."""
    ctx = ctx or default_context()
    part = torch.empty(g.n, dtype=torch.int32, device=g.xadj.device)
    csr = g.csr()
    s = lib().jet_bfs_start(ctx.h, C.byref(csr), C.c_int32(k), _ptr(part), _stream())
    _check(s, "jet_bfs_start")
    return part


def gather_ceiling(g: DeviceGraph, part: torch.Tensor, k: int, reps=10, ctx=None) -> float:
    """jet_gather_ceiling: milliseconds of one pass that only streams the CSR
    entries of g and gathers their neighbours' parts (held as refinement holds
    them for k parts)."""
    ctx = ctx or default_context()
    ms = C.c_float()
    csr = g.csr()
    _check(lib().jet_gather_ceiling(ctx.h, C.byref(csr), _ptr(part), C.c_int32(k), C.c_int32(reps), C.byref(ms),
                                    _stream()),
           "jet_gather_ceiling")
    return ms.value


class Hierarchy:
    """jet_coarsen result; levels are views into library-owned device memory."""

    def __init__(self, h):
        self.h = h

    @property
    def levels(self):
        return lib().jet_hierarchy_levels(self.h)

    def level(self, i):
        """(n, xadj, adjncy, vwgt, adjwgt, map) of level i as host numpy arrays."""
        view = Csr()
        mp = C.c_void_p()
        _check(lib().jet_hierarchy_level(self.h, i, C.byref(view), C.byref(mp)), "jet_hierarchy_level")
        n, nnz = view.n, view.nnz

        def fetch(ptr, count, dt):
            if not ptr:
                return None
            out = np.empty(count, dt)
            if count:
                torch.cuda.synchronize()
                st = _hip().hipMemcpy(C.c_void_p(out.ctypes.data), C.c_void_p(ptr), C.c_size_t(out.nbytes),
                                      C.c_int(2))  # hipMemcpyDeviceToHost
                if st != 0:
                    raise RuntimeError(f"hipMemcpy failed ({st})")
            return out

        return dict(n=n, xadj=fetch(view.xadj, n + 1, np.int64), adjncy=fetch(view.adjncy, nnz, np.int32),
                    vwgt=fetch(view.vwgt, n, np.int32), adjwgt=fetch(view.adjwgt, nnz, np.int32),
                    map=fetch(mp.value, n, np.int32))

    def close(self):
        if self.h:
            lib().jet_hierarchy_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def coarsen(g: DeviceGraph, k: int, ctx=None, **kw) -> Hierarchy:
    ctx = ctx or default_context()
    prm = make_params(k, **kw)
    h = C.c_void_p()
    csr = g.csr()
    _check(lib().jet_coarsen(ctx.h, C.byref(csr), C.byref(prm), C.byref(h), _stream()), "jet_coarsen")
    return Hierarchy(h)


class Server:
    """jet_server_*: continuous-batching partition server on its own context.

    Graphs and output tensors passed to ``submit`` must stay alive (and the
    graph unchanged) until the job is done; ``submit`` keeps references to
    them until its result is taken."""

    def __init__(self, hbm_budget_bytes=0, max_slots=64, device=None):
        self.ctx = Context(device)
        self.h = C.c_void_p()
        _check(lib().jet_server_create(C.byref(self.h), self.ctx.h, C.c_size_t(hbm_budget_bytes),
                                       C.c_int32(max_slots)), "jet_server_create")
        self._keep = {}

    def submit(self, g: DeviceGraph, part_out: torch.Tensor, k: int, **kw) -> int:
        job = Job(g.csr(), make_params(k, **kw), _ptr(part_out))
        t = C.c_uint64()
        _check(lib().jet_server_submit(self.h, C.byref(job), C.byref(t)), "jet_server_submit")
        self._keep[t.value] = (g, part_out)
        return t.value

    def _take(self, st, ticket, r):
        if st == JET_EAGAIN:
            return None
        _check(st, "jet_server result")
        self._keep.pop(ticket, None)
        return r.as_dict()

    def poll(self, ticket: int):
        """Result dict once the job is done, else None."""
        r = Result()
        return self._take(lib().jet_server_poll(self.h, C.c_uint64(ticket), C.byref(r)), ticket, r)

    def wait(self, ticket: int, timeout_ms: int = -1):
        r = Result()
        return self._take(lib().jet_server_wait(self.h, C.c_uint64(ticket), C.c_int32(timeout_ms), C.byref(r)),
                          ticket, r)

    def info(self):
        i = ServerInfo()
        _check(lib().jet_server_info_get(self.h, C.byref(i)), "jet_server_info_get")
        return i.as_dict()

    def close(self):
        if self.h:
            lib().jet_server_destroy(self.h)
            self.h = C.c_void_p()
            self._keep.clear()
        self.ctx.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
