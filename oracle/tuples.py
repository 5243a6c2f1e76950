"""Algorithm 2's tuple form of meet detection, written from its description.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3.2 ("Decomposing Random Walks") and Algorithm 2: every walk
{v_0, v_1, ..., v_len} is decomposed into one tuple per step after the start,
(j, i, v_i, len, v_0) for i = 1..len (j = the walk's index after the shuffle);
all tuples are sorted on (j, i, node) with the source's tuples first among
equal keys (Section 4.4: "the node ID of source node s smaller than other
nodes"); each tuple not from s is linked to the closest tuple from s before it
(PREDECESSOR); a link with equal (j, i, node) is a meet of walk j of s and
walk j of the tuple's start node; each such pair counts once; a meet adds
weight 1 (plain walks, s_hat = count / R) or Lemma 5's weight (stratified).

This is an independent statement of the same counts as the direct pairwise
comparison in simrank_oracle.c: the walks come from the oracle's walk tables,
the detection is a library sort, a running maximum and set operations here.
"""
from __future__ import annotations

import math

import numpy as np

from . import StratParams, walk_table_plain, walk_table_strat


def decompose(paths: np.ndarray, lens: np.ndarray, starts: np.ndarray, js: np.ndarray):
    """Tuples (j, i, node, start) of the walks given as padded path rows."""
    L1 = paths.shape[1]
    i = np.arange(L1)[None, :]
    keep = (i >= 1) & (i <= lens[:, None])
    rows, steps = np.nonzero(keep)
    return js[rows].astype(np.int64), steps.astype(np.int64), \
        paths[rows, steps].astype(np.int64), starts[rows].astype(np.int64)


def link_meets(j, i, node, start, s: int):
    """Sort, label, PREDECESSOR-link; returns the set of (start, j) pairs whose
    walk j meets walk j of s (start != s)."""
    label = (start != s).astype(np.int64)                 # 0: tuple of s, sorts first
    order = np.lexsort((label, node, i, j))
    j, i, node, start, label = j[order], i[order], node[order], start[order], label[order]
    pos = np.arange(j.size)
    last_src = np.maximum.accumulate(np.where(label == 0, pos, -1)) if j.size else pos
    cand = (label == 1) & (last_src >= 0)
    p = pos[cand]
    q = last_src[cand]
    same = (j[p] == j[q]) & (i[p] == i[q]) & (node[p] == node[q])
    met = np.unique(np.stack([start[p[same]], j[p[same]]], axis=1), axis=0) \
        if same.any() else np.zeros((0, 2), np.int64)
    return met


def counts_plain(g, s: int, seed: int, c: float, L: int, R: int) -> np.ndarray:
    """Meet counts of the plain sqrt(c)-walk estimator by the tuple form; the
    count of s itself is R (every pair meets at step 0)."""
    vs = np.repeat(np.arange(g.n, dtype=np.int32), R)
    js = np.tile(np.arange(R, dtype=np.uint32), g.n)
    paths, lens = walk_table_plain(g, seed, c, L, vs, js)
    met = link_meets(*decompose(paths, lens, vs, js), s)
    cnt = np.bincount(met[:, 0], minlength=g.n).astype(np.uint32) if met.size else \
        np.zeros(g.n, np.uint32)
    cnt[s] = R
    return cnt


def sums_stratified(g, s: int, seed: int, P: StratParams) -> np.ndarray:
    """Weighted meet sums (2^40 = weight 1) of the length-stratified estimator
    by the tuple form; each meeting pair adds Lemma 5's weight of its two
    walks' classes, truncated to fixed point."""
    vs = np.repeat(np.arange(g.n, dtype=np.int32), P.N)
    js = np.tile(np.arange(P.N, dtype=np.uint32), g.n)
    paths, lens, _, cls = walk_table_strat(g, seed, P, vs, js)
    met = link_meets(*decompose(paths, lens, vs, js), s)
    a = P.Z / P.Zhat
    cls = cls.reshape(g.n, P.N)
    out = np.zeros(g.n, np.uint64)
    for u, j in met:
        out[u] += np.uint64(int(math.ldexp(a[cls[s, j]] * a[cls[u, j]], 40)))
    return out
