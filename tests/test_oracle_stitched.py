"""Checks of the stitched-walk oracle (per-node segment pools joined end to start).

What pins it: pool sizes by an independent count; a segment length of at least
the walk cap reduces a stitched walk to the plain walk bit for bit; the private
head equals the plain walk's prefix; every move follows an in-edge; segment
chains re-derived here from single draws.  The effect of shared tails is
pinned exactly on a tiny graph in test_oracle_stitched_exact.py; below it is
also bounded empirically against exact SimRank.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import exact
from paper_2304_04015_amd import inputs

C = 0.6
SEED = 0x2304040150000003
ISEED = 0x2304040150000013


def _is_walk(g, p):
    for t in range(1, p.size):
        row = g.in_src[g.in_off[p[t - 1]]:g.in_off[p[t - 1] + 1]]
        if p[t] not in row:
            return False
    return True


@pytest.fixture(scope="module")
def g():
    return inputs.rmat_in(10, 8 << 10, seed=9)


@pytest.mark.parametrize("kappa", [1.0, 0.5, 2.5])
def test_pool_sizes(g, kappa):
    P = O.pool_sizes(g, kappa)
    dbar = np.bincount(g.in_src, minlength=g.n)
    assert np.array_equal(P, np.ceil(kappa * dbar.astype(np.float64)).astype(np.int64))


def test_reduces_to_plain_when_segment_covers_cap(g):
    P = O.pool_sizes(g, 1.0)
    vs = np.repeat(np.arange(0, g.n, 37, dtype=np.int32), 5)
    js = np.tile(np.arange(5, dtype=np.uint32), vs.size // 5)
    for L, seglen in ((8, 8), (8, 16), (5, 8)):
        a, la = O.walk_table_plain(g, SEED, C, L, vs, js)
        b, lb = O.walk_table_stitched(g, SEED, ISEED, C, L, seglen, P, vs, js)
        assert np.array_equal(a, b) and np.array_equal(la, lb)


def test_head_is_plain_prefix_and_moves_follow_in_edges(g):
    P = O.pool_sizes(g, 1.0)
    L, seglen = 64, 8
    deg = g.in_degree()
    vs = np.nonzero(deg > 0)[0][:200].astype(np.int32)
    long_tails = 0
    for v in vs:
        for j in range(20):
            w = O.walk_stitched(g, SEED, ISEED, C, L, seglen, P, int(v), j)
            p = O.walk_plain(g, SEED, C, L, int(v), j)
            h = min(seglen, p.size - 1, w.size - 1)
            assert np.array_equal(w[: h + 1], p[: h + 1])
            assert _is_walk(g, w)
            long_tails += w.size - 1 > seglen
    assert long_tails > 0


def _slot(seed, node, walk, domain, k):
    x = O.philox([node, walk, 0, domain], [seed & 0xffffffff, seed >> 32])
    return (int(x[0]) * int(k)) >> 32


def test_tail_is_chain_of_pool_segments(g):
    """After a full head the walk enters slot pick(draw(v,j,0,2).x0, P(y)) of its
    end node's pool and follows successor picks draw(y,i,0,3); re-derived here
    from single draws and single segments."""
    P = O.pool_sizes(g, 1.0)
    L, seglen = 64, 4
    checked = 0
    for v in range(g.n):
        for j in range(8):
            w = O.walk_stitched(g, SEED, ISEED, C, L, seglen, P, v, j)
            if w.size - 1 <= seglen:
                continue
            y = int(w[seglen])
            i = _slot(SEED, v, j, 2, P[y])
            path = list(w[: seglen + 1])
            while True:
                seg = O.segment(g, ISEED, C, seglen, y, i)
                path += [int(x) for x in seg][: L - (len(path) - 1)]
                if seg.size < seglen or len(path) - 1 >= L:
                    break
                z = int(seg[-1])
                i = _slot(ISEED, y, i, 3, P[z])
                y = z
            assert np.array_equal(np.array(path, np.int32), w)
            checked += 1
        if checked > 200:
            break
    assert checked > 50


def test_segments_are_sqrt_c_walks(g):
    """Segment lengths follow the truncated geometric law of a sqrt(c)-walk on a
    graph region without dead ends (the 6-cycle)."""
    cyc = inputs.tiny_graphs()["cycle6"]
    q = O.continue_threshold(C) / 2 ** 32
    seglen = 8
    lens = np.array([O.segment(cyc, ISEED, C, seglen, 0, i).size for i in range(20000)])
    h = np.bincount(lens, minlength=seglen + 1)
    pl = np.array([q ** l * (1 - q) for l in range(seglen)] + [q ** seglen])
    exp = pl * lens.size
    assert float(((h - exp) ** 2 / exp).sum()) < seglen + 6 * math.sqrt(2 * seglen)


def test_stitched_estimator_close_to_exact():
    """Empirical bound only (shared tails: no closed form).  On C1 with 8-step
    segments the tail is used by a pair only if both walks survive 9 steps
    (probability c^9 ~ 0.01), so the stitched estimate stays within the plain
    Hoeffding radius of exact SimRank."""
    cfg = inputs.C1
    gg = inputs.workload_graph(cfg)
    S = exact.exact_simrank(gg.n, gg.in_off, gg.in_src, C)
    P = O.pool_sizes(gg, 1.0)
    R = 2000
    cnt = O.meet_counts_stitched(gg, 0, cfg["walk_seed"], ISEED, C, cfg["L"], 8, P, R)
    err = np.abs(cnt / R - S[0])
    assert err.max() <= math.sqrt(math.log(2 * gg.n / 1e-3) / (2 * R)) + C ** (cfg["L"] + 1)
    assert cnt[0] == R
