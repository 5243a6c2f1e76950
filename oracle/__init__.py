"""The CPU oracle: a plain, slow, obviously correct statement of what the GPU
path computes.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library and never imports it.

* `exact`   : exact SimRank by FP64 power iteration (Eq. 1) and the parameter
              formulas (Hoeffding sample size, truncation bias).
* this file : ctypes bindings of the single-threaded C oracle in
              `simrank_oracle.c` (Philox4x32-10, plain and stitched sqrt(c)-walks,
              meet counts, walk tables).
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
