"""The CPU oracle: a plain, slow, obviously correct statement of what the GPU
path computes.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library and never imports it.

* `exact`   : exact SimRank by FP64 power iteration (Eq. 1) and the parameter
              formulas (Hoeffding sample size, truncation bias).
* this file : ctypes bindings of the single-threaded C oracle in
              `simrank_oracle.c` (Philox4x32-10, plain and stitched sqrt(c)-walks,
              meet counts, walk tables; the length-stratified estimator of
              Algorithms 1 and 2: class sizes, shuffle, fixed-length walks,
              weighted meet sums).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import exact  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "simrank_oracle.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no contraction of a*b+c)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(LIB_PATH)
                or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)):
            build()
        L = C.CDLL(LIB_PATH)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_continue_threshold.argtypes = [C.c_double]
        L.oracle_continue_threshold.restype = C.c_uint32
        L.oracle_walk_plain.argtypes = [i32p, i32p, C.c_uint64, C.c_uint32, C.c_int32,
                                        C.c_int32, C.c_uint32, i32p]
        L.oracle_walk_plain.restype = C.c_int32
        L.oracle_meet_counts_plain.argtypes = [i32p, i32p, C.c_uint64, C.c_uint32, C.c_int32,
                                               C.c_int32, C.c_int32, i32p, C.c_int64, u32p,
                                               C.c_void_p]
        L.oracle_meet_counts_plain.restype = None
        L.oracle_walk_table_plain.argtypes = [i32p, i32p, C.c_uint64, C.c_uint32, C.c_int32,
                                              i32p, u32p, C.c_int64, i32p, i32p]
        L.oracle_walk_table_plain.restype = None
        L.oracle_pool_sizes.argtypes = [C.c_int32, C.c_int64, i32p, C.c_double, i64p]
        L.oracle_pool_sizes.restype = None
        L.oracle_segment.argtypes = [i32p, i32p, C.c_uint64, C.c_uint32, C.c_int32, C.c_int32,
                                     C.c_uint32, i32p]
        L.oracle_segment.restype = C.c_int32
        L.oracle_walk_stitched.argtypes = [i32p, i32p, C.c_uint64, C.c_uint64, C.c_uint32,
                                           C.c_int32, C.c_int32, i64p, C.c_int32, C.c_uint32, i32p]
        L.oracle_walk_stitched.restype = C.c_int32
        L.oracle_walk_table_stitched.argtypes = [i32p, i32p, C.c_uint64, C.c_uint64, C.c_uint32,
                                                 C.c_int32, C.c_int32, i64p, i32p, u32p, C.c_int64,
                                                 i32p, i32p]
        L.oracle_walk_table_stitched.restype = None
        L.oracle_meet_counts_stitched.argtypes = [i32p, i32p, C.c_uint64, C.c_uint64, C.c_uint32,
                                                  C.c_int32, C.c_int32, i64p, C.c_int32, C.c_int32,
                                                  i32p, C.c_int64, u32p]
        L.oracle_meet_counts_stitched.restype = None
        L.oracle_draw_block.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_int64, u32p]
        L.oracle_draw_block.restype = None
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.oracle_strat_params.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double,
                                          C.c_int32, C.POINTER(C.c_double),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int64), f64p, i64p]
        L.oracle_strat_params.restype = C.c_int
        L.oracle_shuffle_slot.argtypes = [C.c_uint64, C.c_int32, C.c_uint32, C.c_int64]
        L.oracle_shuffle_slot.restype = C.c_uint32
        L.oracle_walk_strat.argtypes = [i32p, i32p, C.c_uint64, C.c_int32, C.c_int32, C.c_uint32,
                                        i32p]
        L.oracle_walk_strat.restype = C.c_int32
        L.oracle_walk_table_strat.argtypes = [i32p, i32p, C.c_uint64, i64p, C.c_int32, C.c_int64,
                                              i32p, u32p, C.c_int64, i32p, i32p, u32p, i32p]
        L.oracle_walk_table_strat.restype = None
        L.oracle_strat_weight.argtypes = [f64p, i64p, C.c_int32, C.c_int32]
        L.oracle_strat_weight.restype = C.c_uint64
        L.oracle_strat_sums.argtypes = [i32p, i32p, C.c_uint64, f64p, i64p, C.c_int32, C.c_int64,
                                        C.c_int32, i32p, C.c_int64, u64p, C.c_void_p, C.c_void_p]
        L.oracle_strat_sums.restype = None
        L.oracle_strat_estimates.argtypes = [u64p, i32p, C.c_int64, C.c_int32, C.c_double,
                                             C.c_int64, f64p, f64p]
        L.oracle_strat_estimates.restype = None
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(np.ascontiguousarray(ctr, np.uint32),
                               np.ascontiguousarray(key, np.uint32), out)
    return out


def draw_block(seed: int, c0: int, c1: int, c2_first: int, c3: int, count: int) -> np.ndarray:
    out = np.zeros((count, 4), np.uint32)
    lib().oracle_draw_block(seed, c0, c1, c2_first, c3, count, out)
    return out


def continue_threshold(c: float) -> int:
    return int(lib().oracle_continue_threshold(float(c)))


def walk_plain(g, seed: int, c: float, L: int, v: int, j: int) -> np.ndarray:
    path = np.full(L + 1, -1, np.int32)
    n = lib().oracle_walk_plain(_i32(g.in_off), _i32(g.in_src), seed, continue_threshold(c),
                                L, v, j, path)
    return path[: n + 1].copy()


def meet_counts_plain(g, s: int, seed: int, c: float, L: int, R: int, vs=None, with_work=False):
    vs = np.arange(g.n, dtype=np.int32) if vs is None else _i32(vs)
    cnt = np.zeros(vs.size, np.uint32)
    work = np.zeros(vs.size, np.uint64) if with_work else None
    lib().oracle_meet_counts_plain(_i32(g.in_off), _i32(g.in_src), seed, continue_threshold(c),
                                   L, R, s, vs, vs.size, cnt,
                                   work.ctypes.data if with_work else None)
    return (cnt, work) if with_work else cnt


def walk_table_plain(g, seed: int, c: float, L: int, vs, js):
    vs = _i32(vs)
    js = np.ascontiguousarray(js, np.uint32)
    paths = np.empty((vs.size, L + 1), np.int32)
    lens = np.empty(vs.size, np.int32)
    lib().oracle_walk_table_plain(_i32(g.in_off), _i32(g.in_src), seed, continue_threshold(c), L,
                                  vs, js, vs.size, paths, lens)
    return paths, lens


def pool_sizes(g, kappa: float) -> np.ndarray:
    P = np.zeros(g.n, np.int64)
    lib().oracle_pool_sizes(g.n, g.m, _i32(g.in_src), float(kappa), P)
    return P


def segment(g, index_seed: int, c: float, seglen: int, y: int, i: int) -> np.ndarray:
    nodes = np.full(seglen, -1, np.int32)
    k = lib().oracle_segment(_i32(g.in_off), _i32(g.in_src), index_seed, continue_threshold(c),
                             seglen, y, i, nodes)
    return nodes[:k].copy()


def walk_stitched(g, seed, index_seed, c, L, seglen, P, v, j) -> np.ndarray:
    path = np.full(L + 1, -1, np.int32)
    n = lib().oracle_walk_stitched(_i32(g.in_off), _i32(g.in_src), seed, index_seed,
                                   continue_threshold(c), L, seglen,
                                   np.ascontiguousarray(P, np.int64), v, j, path)
    return path[: n + 1].copy()


def walk_table_stitched(g, seed, index_seed, c, L, seglen, P, vs, js):
    vs = _i32(vs)
    js = np.ascontiguousarray(js, np.uint32)
    paths = np.empty((vs.size, L + 1), np.int32)
    lens = np.empty(vs.size, np.int32)
    lib().oracle_walk_table_stitched(_i32(g.in_off), _i32(g.in_src), seed, index_seed,
                                     continue_threshold(c), L, seglen,
                                     np.ascontiguousarray(P, np.int64), vs, js, vs.size,
                                     paths, lens)
    return paths, lens


def meet_counts_stitched(g, s, seed, index_seed, c, L, seglen, P, R, vs=None):
    vs = np.arange(g.n, dtype=np.int32) if vs is None else _i32(vs)
    cnt = np.zeros(vs.size, np.uint32)
    lib().oracle_meet_counts_stitched(_i32(g.in_off), _i32(g.in_src), seed, index_seed,
                                      continue_threshold(c), L, seglen,
                                      np.ascontiguousarray(P, np.int64), R, s, vs, vs.size, cnt)
    return cnt


# --------------------------------------------------------------------------
# Length-stratified estimator (Algorithms 1 and 2)
# --------------------------------------------------------------------------

class StratParams:
    """z, walk cap phi, class sizes Z_l (expected) and Zhat_l = ceil(Z_l)
    (generated), N = sum Zhat_l walks per node."""

    def __init__(self, z, phi, N, Z, Zhat):
        self.z, self.phi, self.N = z, phi, N
        self.Z, self.Zhat = Z, Zhat

    def __repr__(self):
        return f"StratParams(z={self.z!r}, phi={self.phi}, N={self.N})"


def strat_params(n: int, c: float, eps: float, z: float = 0.0, phi: int = 0) -> StratParams:
    Z = np.zeros(256, np.float64)
    Zhat = np.zeros(256, np.int64)
    zo, po, No = C.c_double(), C.c_int32(), C.c_int64()
    rc = lib().oracle_strat_params(n, float(c), float(eps), float(z), int(phi), C.byref(zo),
                                   C.byref(po), C.byref(No), Z, Zhat)
    if rc != 0:
        raise ValueError("invalid stratified-estimator parameters")
    k = po.value + 1
    return StratParams(zo.value, po.value, No.value, Z[:k].copy(), Zhat[:k].copy())


def _padded(P: StratParams):
    Z = np.zeros(256, np.float64)
    Zhat = np.zeros(256, np.int64)
    Z[: P.phi + 1] = P.Z
    Zhat[: P.phi + 1] = P.Zhat
    return Z, Zhat


def shuffle_slot(seed: int, v: int, j: int, N: int) -> int:
    return int(lib().oracle_shuffle_slot(seed, v, j, N))


def walk_strat(g, seed: int, length: int, v: int, r: int) -> np.ndarray:
    path = np.full(length + 1, -1, np.int32)
    k = lib().oracle_walk_strat(_i32(g.in_off), _i32(g.in_src), seed, length, v, r, path)
    return path[: k + 1].copy()


def walk_table_strat(g, seed: int, P: StratParams, vs, js):
    """Walk j of node v after the shuffle, for the listed (v, j): paths
    [count][phi+1] (-1 padded), lengths, generated slots and classes."""
    vs = _i32(vs)
    js = np.ascontiguousarray(js, np.uint32)
    _, Zhat = _padded(P)
    paths = np.empty((vs.size, P.phi + 1), np.int32)
    lens = np.empty(vs.size, np.int32)
    slots = np.empty(vs.size, np.uint32)
    cls = np.empty(vs.size, np.int32)
    lib().oracle_walk_table_strat(_i32(g.in_off), _i32(g.in_src), seed, Zhat, P.phi, P.N, vs, js,
                                  vs.size, paths, lens, slots, cls)
    return paths, lens, slots, cls


def strat_weight(P: StratParams, l1: int, l2: int) -> int:
    Z, Zhat = _padded(P)
    return int(lib().oracle_strat_weight(Z, Zhat, l1, l2))


def strat_sums(g, s: int, seed: int, P: StratParams, vs=None, with_stats=False):
    """Weighted meet sums (fixed point, 2^40 = weight 1) of walk pairs (s, u)."""
    vs = np.arange(g.n, dtype=np.int32) if vs is None else _i32(vs)
    Z, Zhat = _padded(P)
    wsum = np.zeros(vs.size, np.uint64)
    meets = np.zeros(vs.size, np.uint32)
    work = np.zeros(vs.size, np.uint64)
    lib().oracle_strat_sums(_i32(g.in_off), _i32(g.in_src), seed, Z, Zhat, P.phi, P.N, s, vs,
                            vs.size, wsum, meets.ctypes.data, work.ctypes.data)
    return (wsum, meets, work) if with_stats else wsum


def strat_estimates(wsum, s: int, P: StratParams, vs=None):
    """(Algorithm 2's estimate, the estimate normalised by the N pairs)."""
    wsum = np.ascontiguousarray(wsum, np.uint64)
    vs = np.arange(wsum.size, dtype=np.int32) if vs is None else _i32(vs)
    out = np.empty(vs.size, np.float64)
    out_n = np.empty(vs.size, np.float64)
    lib().oracle_strat_estimates(wsum, vs, vs.size, s, P.z, P.N, out, out_n)
    return out, out_n
