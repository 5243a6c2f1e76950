"""Python binding of libsimrank.so (the C ABI in include/simrank.h).

Argument marshalling only: every step of a query runs in the library's HIP
kernels.  There is no CPU fallback: if the library cannot be loaded, every
call raises.  Function names are those of the C ABI.  Device buffers for the
asynchronous call are any objects with a device address (torch tensors are
accepted directly); PyTorch is used only for that memory and for streams.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SIMRANK_LIB may name another build of the same sources (e.g. one compiled
# with different -D options); the default is the package's own library.
LIB_PATH = os.environ.get("SIMRANK_LIB") or os.path.join(HERE, "libsimrank.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HEADER = os.path.join(INCLUDE, "simrank.h")

SIMRANK_OK, SIMRANK_EINVAL, SIMRANK_ENOMEM, SIMRANK_EDEVICE, SIMRANK_ESTATE, SIMRANK_EIO = 0, 1, 2, 3, 4, 5
MODE_PLAIN, MODE_STITCHED, MODE_STRATIFIED = 0, 1, 2
PLAN_GROUPS = 1                   # simrank_batch_plan_create_ex flag
_ERRNAMES = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EIO"}


class SimRankError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"simrank error {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class simrank_query(C.Structure):
    _fields_ = [("graph", C.c_int32), ("s", C.c_int32), ("c", C.c_double), ("eps", C.c_double),
                ("delta", C.c_double), ("seed", C.c_uint64), ("walk_cap", C.c_int32),
                ("R_override", C.c_int32), ("mode", C.c_int32), ("union_bound", C.c_int32)]


class simrank_params(C.Structure):
    _fields_ = [("R", C.c_int32), ("L", C.c_int32), ("T", C.c_uint32), ("reserved", C.c_int32)]


class simrank_stats(C.Structure):
    _fields_ = [("pairs", C.c_uint64), ("pairs_walked", C.c_uint64), ("moves", C.c_uint64),
                ("draws", C.c_uint64), ("meets", C.c_uint64), ("tail_steps", C.c_uint64),
                ("source_moves", C.c_uint64), ("ms", C.c_double), ("meet_ms", C.c_double),
                ("R", C.c_int32),
                ("L", C.c_int32), ("T", C.c_uint32), ("reserved", C.c_int32)]

    def asdict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class simrank_strat_params(C.Structure):
    _fields_ = [("z", C.c_double), ("N", C.c_int32), ("phi", C.c_int32),
                ("shuffle_b", C.c_int32), ("shuffle_A", C.c_int32)]


class simrank_index_params(C.Structure):
    _fields_ = [("seg_log2", C.c_int32), ("reserved", C.c_int32), ("kappa", C.c_double),
                ("c", C.c_double), ("seed", C.c_uint64)]


class simrank_server_params(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("max_R", C.c_int32), ("max_L", C.c_int32),
                ("group_max", C.c_int32), ("hbm_budget", C.c_int64)]


class simrank_tuning(C.Structure):
    _fields_ = [("unit_nodes", C.c_int32), ("tile_walks", C.c_int32), ("seg_log2", C.c_int32),
                ("reserved", C.c_int32), ("meet_ms", C.c_double), ("build_ms", C.c_double)]

    def asdict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class simrank_request_info(C.Structure):
    _fields_ = [("queue_s", C.c_double), ("latency_s", C.c_double), ("stats", simrank_stats)]


class simrank_rate(C.Structure):
    _fields_ = [("per_s", C.c_double), ("ms", C.c_double), ("count", C.c_double)]

    def asdict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class simrank_index_summary(C.Structure):
    _fields_ = [("segments", C.c_int64), ("bytes", C.c_int64), ("seg_log2", C.c_int32),
                ("levels", C.c_int32), ("build_ms", C.c_double), ("build_moves", C.c_uint64),
                ("segments_ms", C.c_double), ("doubling_ms", C.c_double)]

    def asdict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it is missing (build it with build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2304_04015_amd/build.py "
                          "(or __graft_entry__.build()) first; there is no fallback")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7.  When
    # torch is loaded first, the loader satisfies this library's dependency on
    # that soname with torch's copy, so device pointers and stream handles are
    # shared; loading this library first would bring a second runtime that
    # torch then fails to initialise next to.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
    P = C.POINTER
    sig = {
        "simrank_load_graph": [i32, i64, vp, vp, P(vp)],
        "simrank_free_graph": [vp],
        "simrank_graph_info": [vp, P(i32), P(i64), P(i32), P(i64)],
        "simrank_derive_params": [P(simrank_query), i32, P(simrank_params)],
        "simrank_single_source": [vp, i32, dbl, dbl, dbl, vp],
        "simrank_single_source_ex": [vp, P(simrank_query), vp, vp, P(simrank_stats)],
        "simrank_workspace_create": [vp, i32, i32, P(vp)],
        "simrank_workspace_free": [vp],
        "simrank_single_source_async": [vp, P(simrank_query), vp, vp, vp, vp],
        "simrank_workspace_stats": [vp, P(simrank_stats)],
        "simrank_single_source_noalloc": [vp, P(simrank_query), vp, vp, vp],
        "simrank_walks": [vp, P(simrank_query), vp, vp, i64, vp, vp],
        "simrank_derive_stratified": [P(simrank_query), i32, P(simrank_strat_params)],
        "simrank_single_source_stratified": [vp, P(simrank_query), vp, vp, vp, P(simrank_stats)],
        "simrank_stratified_async": [vp, P(simrank_query), vp, vp, vp, vp, vp],
        "simrank_stratified_walks": [vp, P(simrank_query), vp, vp, i64, vp, vp, vp, vp],
        "simrank_tuple_meets": [vp, P(simrank_query), i32, vp, P(simrank_stats)],
        "simrank_build_index": [vp, P(simrank_index_params)],
        "simrank_index_info": [vp, P(simrank_index_summary)],
        "simrank_index_read": [vp, vp, i64, vp, vp, vp, vp],
        "simrank_index_save": [vp, C.c_char_p],
        "simrank_index_load": [vp, C.c_char_p],
        "simrank_batch": [P(vp), i32, P(simrank_query), i32, P(vp), P(vp), P(simrank_stats)],
        "simrank_batch_plan_create": [P(vp), i32, P(simrank_query), i32, P(vp)],
        "simrank_tune_ex": [vp, P(simrank_query), P(simrank_tuning)],
        "simrank_set_tuning": [vp, i32, i32],
        "simrank_tune_index": [vp, P(simrank_query), P(simrank_index_params), P(i32), i32,
                               P(simrank_tuning), P(dbl)],
        "simrank_batch_plan_create_ex": [P(vp), i32, P(simrank_query), i32, u32, P(vp), P(i32)],
        "simrank_batch_plan_run": [vp, vp],
        "simrank_batch_plan_wait": [vp, P(simrank_stats)],
        "simrank_batch_plan_read": [vp, i32, vp, vp],
        "simrank_batch_plan_read_stratified": [vp, i32, vp, vp, vp],
        "simrank_batch_plan_free": [vp],
        "simrank_tune": [vp, P(simrank_query), P(i32)],
        "simrank_server_create": [vp, P(simrank_server_params), P(vp)],
        "simrank_server_info": [vp, P(i32), P(i64)],
        "simrank_server_counts": [vp, P(C.c_uint64), P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)],
        "simrank_server_submit": [vp, P(simrank_query), P(C.c_uint64)],
        "simrank_server_wait": [vp, C.c_uint64, dbl, vp, vp, P(simrank_request_info)],
        "simrank_server_destroy": [vp],
        "simrank_server_poll": [vp, C.c_uint64, P(i32)],
        "simrank_server_load": [vp, P(i32), P(i64), P(i64), P(C.c_uint64)],
        "simrank_server_wait_stratified": [vp, C.c_uint64, dbl, vp, vp, vp,
                                           P(simrank_request_info)],
        "simrank_roofline_gather": [i64, i32, i32, P(simrank_rate)],
        "simrank_roofline_gather_grid": [i64, i32, i32, i32, P(simrank_rate)],
        "simrank_roofline_philox": [P(simrank_rate)],
        "simrank_roofline_copy": [i64, P(simrank_rate)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.simrank_last_error.argtypes = []
    L.simrank_last_error.restype = C.c_char_p
    L.simrank_version.argtypes = []
    L.simrank_version.restype = C.c_char_p
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions the headers under include/ declare."""
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(simrank_\w+)\s*\(", text, re.M))
    return sorted(names)


def _check(rc: int) -> None:
    if rc != SIMRANK_OK:
        raise SimRankError(rc, lib().simrank_last_error().decode())


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _dev_ptr(t, n: int, itemsize: int, name: str) -> int | None:
    """Device address of buffer t for n elements of itemsize bytes.  A tensor
    must live on a GPU, be contiguous, have that element size and hold at
    least n elements (the kernels write n); a raw integer address is passed
    through as the caller's promise."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        dev = getattr(t, "device", None)
        if dev is not None and getattr(dev, "type", "cuda") != "cuda":
            raise SimRankError(SIMRANK_EINVAL, f"{name}: not a device tensor ({dev})")
        if hasattr(t, "is_contiguous") and not t.is_contiguous():
            raise SimRankError(SIMRANK_EINVAL, f"{name}: not contiguous")
        if t.element_size() != itemsize:
            raise SimRankError(SIMRANK_EINVAL, f"{name}: element size {t.element_size()}, "
                                               f"expected {itemsize}")
        if t.numel() < n:
            raise SimRankError(SIMRANK_EINVAL, f"{name}: {t.numel()} elements, needs {n}")
        return int(t.data_ptr())
    return int(t)


def make_query(s: int, c: float = 0.6, eps: float = 0.02, delta: float = 1e-3, seed: int = 0,
               walk_cap: int = 64, R: int = 0, mode: int = MODE_PLAIN, union_bound: bool = False,
               graph: int = 0) -> simrank_query:
    return simrank_query(s=s, graph=graph, c=c, eps=eps, delta=delta, seed=seed,
                         walk_cap=walk_cap, R_override=R, mode=mode,
                         union_bound=1 if union_bound else 0)


class Graph:
    """A device-resident graph handle (simrank_load_graph / simrank_free_graph)."""

    def __init__(self, handle: int, n: int, m: int):
        self.handle = C.c_void_p(handle)
        self.n = n
        self.m = m

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self) -> None:
        if self.handle and self.handle.value:
            _check(lib().simrank_free_graph(self.handle))
            self.handle = C.c_void_p(None)

    def info(self) -> dict:
        n, na = C.c_int32(), C.c_int32()
        m, b = C.c_int64(), C.c_int64()
        _check(lib().simrank_graph_info(self.handle, C.byref(n), C.byref(m), C.byref(na),
                                        C.byref(b)))
        return dict(n=n.value, m=m.value, n_active=na.value, device_bytes=b.value)


def simrank_load_graph(n: int, in_off, in_src) -> Graph:
    in_off = np.ascontiguousarray(in_off, np.int32)
    in_src = np.ascontiguousarray(in_src, np.int32)
    if in_off.shape != (n + 1,):
        raise ValueError("in_off must have n + 1 entries")
    h = C.c_void_p()
    _check(lib().simrank_load_graph(n, in_src.size, _ptr(in_off), _ptr(in_src) if in_src.size else None,
                                    C.byref(h)))
    return Graph(h.value, n, int(in_src.size))


def load_csr(g) -> Graph:
    """Loads an object with fields n, in_off, in_src (e.g. inputs.CSR)."""
    return simrank_load_graph(g.n, g.in_off, g.in_src)


def simrank_derive_params(q: simrank_query, n: int) -> simrank_params:
    p = simrank_params()
    _check(lib().simrank_derive_params(C.byref(q), n, C.byref(p)))
    return p


def simrank_single_source(g: Graph, s: int, c: float, eps: float, delta: float) -> np.ndarray:
    out = np.empty(g.n, np.float64)
    _check(lib().simrank_single_source(g.handle, s, c, eps, delta, _ptr(out)))
    return out


def simrank_single_source_ex(g: Graph, q: simrank_query, want_out: bool = True,
                             want_counts: bool = True):
    out = np.empty(g.n, np.float64) if want_out else None
    cnt = np.empty(g.n, np.uint32) if want_counts else None
    st = simrank_stats()
    _check(lib().simrank_single_source_ex(g.handle, C.byref(q),
                                          _ptr(out) if out is not None else None,
                                          _ptr(cnt) if cnt is not None else None, C.byref(st)))
    return out, cnt, st


class Workspace:
    def __init__(self, g: Graph, max_R: int, max_L: int):
        h = C.c_void_p()
        _check(lib().simrank_workspace_create(g.handle, max_R, max_L, C.byref(h)))
        self.handle = h
        self.graph = g

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self) -> None:
        if self.handle and self.handle.value:
            _check(lib().simrank_workspace_free(self.handle))
            self.handle = C.c_void_p(None)


def simrank_workspace_create(g: Graph, max_R: int, max_L: int) -> Workspace:
    return Workspace(g, max_R, max_L)


def simrank_single_source_async(g: Graph, q: simrank_query, ws: Workspace, out_dev, counts_dev,
                                stream=None) -> None:
    """out_dev: float64 device buffer of n (or None); counts_dev: uint32/int32 device
    buffer of n; stream: a torch.cuda.Stream, a raw hipStream_t int, or None."""
    sp = None
    if stream is not None:
        sp = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)
    _check(lib().simrank_single_source_async(g.handle, C.byref(q), ws.handle,
                                             _dev_ptr(out_dev, g.n, 8, "out_dev"),
                                             _dev_ptr(counts_dev, g.n, 4, "counts_dev"), sp))


def simrank_single_source_noalloc(g: Graph, q: simrank_query, out_dev, counts_dev,
                                  stream=None) -> None:
    """The allocation-free query: as simrank_single_source_async, without a
    workspace (the library's fixed per-GPU scratch)."""
    sp = None
    if stream is not None:
        sp = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)
    _check(lib().simrank_single_source_noalloc(g.handle, C.byref(q),
                                               _dev_ptr(out_dev, g.n, 8, "out_dev"),
                                               _dev_ptr(counts_dev, g.n, 4, "counts_dev"), sp))


def simrank_workspace_stats(ws: Workspace) -> simrank_stats:
    st = simrank_stats()
    _check(lib().simrank_workspace_stats(ws.handle, C.byref(st)))
    return st


def simrank_walks(g: Graph, q: simrank_query, vs, js):
    vs = np.ascontiguousarray(vs, np.int32)
    js = np.ascontiguousarray(js, np.uint32)
    p = simrank_derive_params(q, g.n)
    paths = np.empty((vs.size, p.L + 1), np.int32)
    lens = np.empty(vs.size, np.int32)
    _check(lib().simrank_walks(g.handle, C.byref(q), _ptr(vs), _ptr(js), vs.size, _ptr(paths),
                               _ptr(lens)))
    return paths, lens


def make_stratified_query(s: int, c: float = 0.6, eps: float = 0.02, seed: int = 0, phi: int = 0,
                          z: int = 0, delta: float = 1e-3, graph: int = 0) -> simrank_query:
    """A query for the length-stratified estimator; phi = 0 and z = 0 select
    Algorithm 1's cap and Algorithm 2's z (z, when given, is an integer)."""
    return simrank_query(s=s, graph=graph, c=c, eps=eps, delta=delta, seed=seed, walk_cap=phi,
                         R_override=z, mode=MODE_STRATIFIED, union_bound=0)


def simrank_derive_stratified(q: simrank_query, n: int) -> simrank_strat_params:
    p = simrank_strat_params()
    _check(lib().simrank_derive_stratified(C.byref(q), n, C.byref(p)))
    return p


def simrank_single_source_stratified(g: Graph, q: simrank_query, want_out: bool = True):
    """(Algorithm 2's estimate, the N-normalised estimate, weighted sums, stats)."""
    out = np.empty(g.n, np.float64) if want_out else None
    out_n = np.empty(g.n, np.float64) if want_out else None
    wsum = np.empty(g.n, np.uint64)
    st = simrank_stats()
    _check(lib().simrank_single_source_stratified(
        g.handle, C.byref(q), _ptr(out) if want_out else None, _ptr(out_n) if want_out else None,
        _ptr(wsum), C.byref(st)))
    return out, out_n, wsum, st


def simrank_stratified_async(g: Graph, q: simrank_query, ws: Workspace, out_dev, out_n_dev,
                             wsum_dev, stream=None) -> None:
    """Device buffers (torch tensors or raw pointers): out_dev, out_n_dev float64[n]
    or None, wsum_dev uint64/int64[n]."""
    sp = None
    if stream is not None:
        sp = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)
    _check(lib().simrank_stratified_async(g.handle, C.byref(q), ws.handle,
                                          _dev_ptr(out_dev, g.n, 8, "out_dev"),
                                          _dev_ptr(out_n_dev, g.n, 8, "out_n_dev"),
                                          _dev_ptr(wsum_dev, g.n, 8, "wsum_dev"), sp))


def simrank_stratified_walks(g: Graph, q: simrank_query, vs, js, with_paths: bool = True):
    """(slots, classes, paths [count][phi+1] or None, lens or None)."""
    vs = np.ascontiguousarray(vs, np.int32)
    js = np.ascontiguousarray(js, np.uint32)
    p = simrank_derive_stratified(q, g.n)
    slots = np.empty(vs.size, np.uint32)
    cls = np.empty(vs.size, np.int32)
    paths = np.empty((vs.size, p.phi + 1), np.int32) if with_paths else None
    lens = np.empty(vs.size, np.int32) if with_paths else None
    _check(lib().simrank_stratified_walks(g.handle, C.byref(q), _ptr(vs), _ptr(js), vs.size,
                                          _ptr(slots), _ptr(cls),
                                          _ptr(paths) if with_paths else None,
                                          _ptr(lens) if with_paths else None))
    return slots, cls, paths, lens


def simrank_tuple_meets(g: Graph, queries: list):
    """Algorithm 2's tuple form for up to 32 queries sharing everything but the
    source: (sums uint64[k][n], stats)."""
    k = len(queries)
    arr = (simrank_query * k)(*queries)
    sums = np.empty((k, g.n), np.uint64)
    st = simrank_stats()
    _check(lib().simrank_tuple_meets(g.handle, arr, k, _ptr(sums), C.byref(st)))
    return sums, st


def simrank_build_index(g: Graph, seg_log2: int = 3, kappa: float = 1.0, c: float = 0.6,
                        seed: int = 0) -> dict:
    p = simrank_index_params(seg_log2=seg_log2, reserved=0, kappa=kappa, c=c, seed=seed)
    _check(lib().simrank_build_index(g.handle, C.byref(p)))
    return simrank_index_info(g)


def simrank_index_info(g: Graph) -> dict:
    s = simrank_index_summary()
    _check(lib().simrank_index_info(g.handle, C.byref(s)))
    return s.asdict()


def simrank_index_save(g: Graph, path: str) -> None:
    """Writes the graph's stitched index to `path`."""
    _check(lib().simrank_index_save(g.handle, os.fsencode(path)))


def simrank_index_load(g: Graph, path: str) -> None:
    """Makes the index saved at `path` the graph's index (refused, leaving the
    current index, if the file does not belong to this graph or is damaged)."""
    _check(lib().simrank_index_load(g.handle, os.fsencode(path)))


def simrank_index_read(g: Graph, sigma, with_chain: bool = True):
    sigma = np.ascontiguousarray(sigma, np.int64)
    info = simrank_index_info(g)
    seg_len = 1 << info["seg_log2"]
    width = 64 // seg_len
    nodes = np.empty((sigma.size, seg_len), np.int32)
    lens = np.empty(sigma.size, np.int32)
    succ = np.empty(sigma.size, np.int64)
    chain = np.empty((sigma.size, width), np.int64) if with_chain else None
    _check(lib().simrank_index_read(g.handle, _ptr(sigma), sigma.size, _ptr(nodes), _ptr(lens),
                                    _ptr(succ), _ptr(chain) if with_chain else None))
    return nodes, lens, succ, chain


def simrank_batch(graphs: list[Graph], queries: list[simrank_query], want_counts: bool = True):
    """(outs, counts, stats); a stratified query's counts entry is left unwritten."""
    ng = len(graphs)
    nq = len(queries)
    garr = (C.c_void_p * ng)(*[g.handle.value for g in graphs])
    qarr = (simrank_query * nq)(*queries)
    # an invalid graph index is the library's to reject (EINVAL); size its buffers at 1
    sizes = [graphs[q.graph].n if 0 <= q.graph < ng else 1 for q in queries]
    outs = [np.empty(n, np.float64) for n in sizes]
    cnts = [np.empty(n, np.uint32) for n in sizes] if want_counts else None
    oarr = (C.c_void_p * nq)(*[o.ctypes.data for o in outs])
    carr = (C.c_void_p * nq)(*[c.ctypes.data for c in cnts]) if want_counts else None
    st = simrank_stats()
    _check(lib().simrank_batch(garr, ng, qarr, nq, oarr, carr, C.byref(st)))
    if cnts is not None:
        cnts = [None if q.mode == MODE_STRATIFIED else c for q, c in zip(queries, cnts)]
    return outs, cnts, st


def simrank_roofline_gather(footprint_bytes: int, entry_bytes: int = 8,
                            dependent: bool = False) -> dict:
    r = simrank_rate()
    _check(lib().simrank_roofline_gather(int(footprint_bytes), entry_bytes, 1 if dependent else 0,
                                         C.byref(r)))
    return r.asdict()


def simrank_roofline_gather_grid(footprint_bytes: int, entry_bytes: int, blocks: int,
                                 block_threads: int) -> dict:
    r = simrank_rate()
    _check(lib().simrank_roofline_gather_grid(int(footprint_bytes), entry_bytes, blocks,
                                              block_threads, C.byref(r)))
    return r.asdict()


def simrank_roofline_philox() -> dict:
    r = simrank_rate()
    _check(lib().simrank_roofline_philox(C.byref(r)))
    return r.asdict()


def simrank_roofline_copy(nbytes: int) -> dict:
    r = simrank_rate()
    _check(lib().simrank_roofline_copy(int(nbytes), C.byref(r)))
    return r.asdict()


class BatchPlan:
    """simrank_batch_plan_*: device buffers and a captured launch of a query set."""

    def __init__(self, graphs: list, queries: list, groups: bool = True):
        """groups: let plain queries with equal (graph, seed, c, cap) share
        their walks from every node (SIMRANK_PLAN_GROUPS); n_groups says how
        many groups were formed."""
        ng, nq = len(graphs), len(queries)
        garr = (C.c_void_p * ng)(*[g.handle.value for g in graphs])
        qarr = (simrank_query * nq)(*queries)
        h = C.c_void_p()
        ngr = C.c_int32(0)
        _check(lib().simrank_batch_plan_create_ex(garr, ng, qarr, nq,
                                                  PLAN_GROUPS if groups else 0,
                                                  C.byref(h), C.byref(ngr)))
        self.n_groups = int(ngr.value)
        self.handle = h
        self.graphs = graphs
        self.queries = list(queries)

    def run(self, stream=None) -> None:
        sp = None
        if stream is not None:
            sp = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().simrank_batch_plan_run(self.handle, sp))

    def wait(self) -> simrank_stats:
        st = simrank_stats()
        _check(lib().simrank_batch_plan_wait(self.handle, C.byref(st)))
        return st

    def read(self, i: int, want_out: bool = True, want_counts: bool = True):
        n = self.graphs[self.queries[i].graph].n
        out = np.empty(n, np.float64) if want_out else None
        cnt = np.empty(n, np.uint32) if want_counts else None
        _check(lib().simrank_batch_plan_read(self.handle, i,
                                             _ptr(out) if out is not None else None,
                                             _ptr(cnt) if cnt is not None else None))
        return out, cnt

    def read_stratified(self, i: int):
        """(out, out_n, wsum) of stratified query i after the last run."""
        n = self.graphs[self.queries[i].graph].n
        out, out_n, wsum = np.empty(n), np.empty(n), np.empty(n, np.uint64)
        _check(lib().simrank_batch_plan_read_stratified(self.handle, i, _ptr(out), _ptr(out_n),
                                                        _ptr(wsum)))
        return out, out_n, wsum

    def free(self) -> None:
        if self.handle and self.handle.value:
            _check(lib().simrank_batch_plan_free(self.handle))
            self.handle = C.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """simrank_server_*: continuous batching of single-source requests."""

    def __init__(self, g: Graph, max_slots: int = 4, max_R: int = 9502, max_L: int = 64,
                 hbm_budget: int = 0, group_max: int = 0):
        """group_max >= 2: waiting requests with equal walks (mode, seed, c, cap)
        are admitted together as one query group."""
        p = simrank_server_params(max_slots=max_slots, max_R=max_R, max_L=max_L,
                                  group_max=group_max, hbm_budget=hbm_budget)
        h = C.c_void_p()
        _check(lib().simrank_server_create(g.handle, C.byref(p), C.byref(h)))
        self.handle = h
        self.graph = g

    def info(self) -> dict:
        s, b = C.c_int32(), C.c_int64()
        _check(lib().simrank_server_info(self.handle, C.byref(s), C.byref(b)))
        return dict(slots=s.value, slot_bytes=b.value)

    def counts(self) -> dict:
        """Requests done and failed, query groups launched and the requests they held."""
        v = [C.c_uint64() for _ in range(4)]
        _check(lib().simrank_server_counts(self.handle, *[C.byref(x) for x in v]))
        return dict(zip(("done", "failed", "groups", "grouped"), (x.value for x in v)))

    def submit(self, q: simrank_query) -> int:
        t = C.c_uint64()
        _check(lib().simrank_server_submit(self.handle, C.byref(q), C.byref(t)))
        return t.value

    def load(self) -> dict:
        """Most requests in flight at once, the device pool's size and peak use,
        persistent meet kernels and group launches made."""
        a, b, c, d = C.c_int32(), C.c_int64(), C.c_int64(), C.c_uint64()
        _check(lib().simrank_server_load(self.handle, C.byref(a), C.byref(b), C.byref(c),
                                         C.byref(d)))
        return dict(inflight_peak=a.value, pool_bytes=b.value, pool_peak=c.value,
                    launches=d.value)

    def poll(self, ticket: int) -> int:
        """0 queued, 1 running, 2 finished (its wait returns at once)."""
        st = C.c_int32()
        _check(lib().simrank_server_poll(self.handle, ticket, C.byref(st)))
        return st.value

    def wait(self, ticket: int, timeout_s: float = -1.0, want_out: bool = True,
             want_counts: bool = True):
        n = self.graph.n
        out = np.empty(n, np.float64) if want_out else None
        cnt = np.empty(n, np.uint32) if want_counts else None
        info = simrank_request_info()
        _check(lib().simrank_server_wait(self.handle, ticket, float(timeout_s),
                                         _ptr(out) if out is not None else None,
                                         _ptr(cnt) if cnt is not None else None, C.byref(info)))
        return out, cnt, info

    def wait_stratified(self, ticket: int, timeout_s: float = -1.0):
        """A stratified request's (out, out_n, wsum, info)."""
        n = self.graph.n
        out = np.empty(n, np.float64)
        out_n = np.empty(n, np.float64)
        wsum = np.empty(n, np.uint64)
        info = simrank_request_info()
        _check(lib().simrank_server_wait_stratified(self.handle, ticket, float(timeout_s),
                                                    _ptr(out), _ptr(out_n), _ptr(wsum),
                                                    C.byref(info)))
        return out, out_n, wsum, info

    def destroy(self) -> None:
        if self.handle and self.handle.value:
            _check(lib().simrank_server_destroy(self.handle))
            self.handle = C.c_void_p(None)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def simrank_tune(g: Graph, q: simrank_query) -> int:
    vb = C.c_int32()
    _check(lib().simrank_tune(g.handle, C.byref(q), C.byref(vb)))
    return vb.value


def simrank_tune_ex(g: Graph, q: simrank_query) -> dict:
    """Nodes per unit and walks per tile chosen for g (kept for later queries)."""
    t = simrank_tuning()
    _check(lib().simrank_tune_ex(g.handle, C.byref(q), C.byref(t)))
    return t.asdict()


def simrank_set_tuning(g: Graph, unit_nodes: int = 0, tile_walks: int = 0) -> None:
    _check(lib().simrank_set_tuning(g.handle, int(unit_nodes), int(tile_walks)))


def simrank_tune_index(g: Graph, q: simrank_query, seg_log2=(2, 3, 4), kappa: float = 1.0,
                       c: float = 0.6, seed: int = 0) -> tuple[dict, list]:
    """Builds the stitched index with each segment length 2^k, times stitched
    query q on each and leaves the fastest built: (choice, ms per k)."""
    ks = (C.c_int32 * len(seg_log2))(*seg_log2)
    ms = (C.c_double * len(seg_log2))()
    p = simrank_index_params(seg_log2=int(seg_log2[0]), reserved=0, kappa=kappa, c=c, seed=seed)
    t = simrank_tuning()
    _check(lib().simrank_tune_index(g.handle, C.byref(q), C.byref(p), ks, len(seg_log2),
                                    C.byref(t), ms))
    return t.asdict(), list(ms)


def simrank_version() -> str:
    return lib().simrank_version().decode()


@dataclass
class Params:
    R: int
    L: int
    T: int
