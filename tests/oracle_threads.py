"""Host-thread fan-out of the CPU oracle for parity checks at full size.

The oracle's per-node calls (meet counts, stitched meet counts, weighted sums)
are single-threaded C functions that keep no shared state; ctypes releases
the GIL while they run.  Splitting the listed nodes into chunks and running
one unchanged call per chunk on a host thread gives the same result as one
call over all nodes (each node's result depends only on the graph, the source
and the keys), which lets the GPU tests compare thousands of nodes of the
full-size workloads against the oracle in seconds.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O


def host_threads(cap: int = 16) -> int:
    """Threads to use: the CPUs this process may run on, at most `cap` (the
    host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def _fan_out(fn, vs, threads: int | None = None):
    vs = np.ascontiguousarray(vs, dtype=np.int32)
    nt = min(threads or host_threads(), max(1, vs.size))
    parts = [p for p in np.array_split(vs, nt) if p.size]
    if len(parts) <= 1:
        return fn(vs)
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        outs = list(ex.map(fn, parts))
    return np.concatenate(outs)


def meet_counts_plain(g, s, seed, c, L, R, vs, threads=None):
    return _fan_out(lambda p: O.meet_counts_plain(g, s, seed, c, L, R, vs=p), vs, threads)


def meet_counts_stitched(g, s, seed, index_seed, c, L, seglen, P, R, vs, threads=None):
    return _fan_out(lambda p: O.meet_counts_stitched(g, s, seed, index_seed, c, L, seglen, P, R,
                                                     vs=p), vs, threads)


def strat_sums(g, s, seed, P, vs, threads=None):
    return _fan_out(lambda p: O.strat_sums(g, s, seed, P, vs=p), vs, threads)


def sample_nodes(g, n_random: int, n_top: int, n_isolated: int, seed: int, extra=()) -> np.ndarray:
    """Sorted node sample: the n_top highest in-degree nodes, n_random random
    nodes with in-edges, n_isolated nodes without in-edges, plus `extra`."""
    deg = g.in_degree()
    rng = np.random.default_rng(seed)
    act = np.nonzero(deg > 0)[0]
    none = np.nonzero(deg == 0)[0]
    parts = [np.argsort(deg, kind="stable")[-n_top:] if n_top else np.zeros(0, np.int64),
             rng.choice(act, min(n_random, act.size), replace=False),
             rng.choice(none, min(n_isolated, none.size), replace=False) if none.size else
             np.zeros(0, np.int64),
             np.asarray(list(extra), dtype=np.int64)]
    return np.unique(np.concatenate(parts)).astype(np.int32)
