"""Pins for the exact-SimRank oracle (FP64 power iteration of Eq. 1).

The values come from hand derivations (tests/golden/simrank_closed_forms.txt),
from invariants that Eq. 1 forces, and from an independent brute-force
enumeration of pairs of sqrt(c)-walks (Lemma 2) on tiny graphs.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import exact
from paper_2304_04015_amd import inputs

C = 0.6
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "simrank_closed_forms.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            name, u, v, val = line.split()
            rows.append((name, int(u), int(v), float(val)))
    return rows


@pytest.fixture(scope="module")
def exact_tiny():
    out = {}
    for name, g in inputs.tiny_graphs().items():
        out[name] = exact.exact_simrank(g.n, g.in_off, g.in_src, C)
    return out


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"{r[0]}-{r[1]}-{r[2]}")
def test_closed_forms(exact_tiny, row):
    name, u, v, val = row
    S = exact_tiny[name]
    assert S[u, v] == pytest.approx(val, abs=1e-12)
    assert S[v, u] == pytest.approx(val, abs=1e-12)


def test_invariants_on_er():
    g = inputs.erdos_renyi_in(120, 3.0, seed=7)
    S = exact.exact_simrank(g.n, g.in_off, g.in_src, C)
    assert np.allclose(S, S.T, atol=1e-14)                   # symmetry
    assert np.all(np.diag(S) == 1.0)                          # s(u,u) = 1
    off = S[~np.eye(g.n, dtype=bool)]
    assert off.min() >= 0.0 and off.max() <= C + 1e-15       # 0 <= s <= c off the diagonal
    empty = np.nonzero(g.in_degree() == 0)[0]
    assert empty.size > 0
    for u in empty:                                           # I(u) empty => s(u, v) = 0
        row = S[u].copy()
        row[u] = 0.0
        assert np.all(row == 0.0)
    # Eq. 1 holds at the fixed point, entry by entry (written with explicit sums)
    rng = np.random.default_rng(0)
    for _ in range(200):
        u, v = rng.integers(0, g.n, 2)
        if u == v:
            continue
        Iu = g.in_src[g.in_off[u]:g.in_off[u + 1]]
        Iv = g.in_src[g.in_off[v]:g.in_off[v + 1]]
        if Iu.size == 0 or Iv.size == 0:
            assert S[u, v] == 0.0
            continue
        rhs = C / (Iu.size * Iv.size) * sum(S[a, b] for a in Iu for b in Iv)
        assert S[u, v] == pytest.approx(rhs, abs=1e-13)


def test_truncation_monotone_and_bounded():
    g = inputs.erdos_renyi_in(80, 4.0, seed=3)
    S = exact.exact_simrank(g.n, g.in_off, g.in_src, C)
    prev = None
    for k in range(0, 12):
        Sk = exact.simrank_iterates(g.n, g.in_off, g.in_src, C, k)
        gap = S - Sk
        assert gap.min() >= -1e-15
        assert gap.max() <= C ** (k + 1) + 1e-15
        if prev is not None:
            assert np.all(Sk >= prev - 1e-15)
        prev = Sk


def _walk_distribution(g, u, q, k):
    """All walks from u truncated at k steps, with their exact probabilities
    (continue with probability q, then a uniform in-neighbour; a node without
    in-neighbours ends the walk)."""
    out = []

    def rec(path, p):
        cur = path[-1]
        nb = g.in_src[g.in_off[cur]:g.in_off[cur + 1]]
        if len(path) - 1 == k:
            out.append((tuple(path), p))
            return
        if nb.size == 0:
            out.append((tuple(path), p))
            return
        out.append((tuple(path), p * (1.0 - q)))
        for w in nb:
            rec(path + [int(w)], p * q / nb.size)

    rec([u], 1.0)
    return out


def _meet_probability_brute(g, u, v, c, k):
    q = math.sqrt(c)
    A = _walk_distribution(g, u, q, k)
    B = _walk_distribution(g, v, q, k)
    tot = 0.0
    for (a, pa), (b, pb) in itertools.product(A, B):
        lim = min(len(a), len(b))
        if any(a[i] == b[i] for i in range(lim)):
            tot += pa * pb
    return tot


@pytest.mark.parametrize("name,k", [("path5", 5), ("K_2_2", 5), ("bip_dir_3_4", 3),
                                    ("star_out5", 3), ("cycle6", 6)])
def test_lemma2_brute_force_enumeration(name, k):
    """S_k(u,v) equals Pr[two walks meet within k steps], by enumerating walk pairs."""
    g = inputs.tiny_graphs()[name]
    Sk = exact.simrank_iterates(g.n, g.in_off, g.in_src, C, k)
    for u in range(g.n):
        for v in range(u, g.n):
            p = _meet_probability_brute(g, u, v, C, k)
            assert Sk[u, v] == pytest.approx(p, abs=1e-13), (u, v)


def test_lemma2_brute_force_random_graph():
    g = inputs.from_edges(6, [0, 1, 2, 3, 4, 5, 0, 2, 4, 1], [1, 2, 3, 4, 5, 0, 3, 5, 1, 4])
    k = 4
    Sk = exact.simrank_iterates(g.n, g.in_off, g.in_src, C, k)
    for u, v in itertools.combinations(range(g.n), 2):
        assert Sk[u, v] == pytest.approx(_meet_probability_brute(g, u, v, C, k), abs=1e-13)


def test_hoeffding_R():
    # ln(2/delta) / (2 (eps - c^(L+1))^2) at eps = .02, .05, .01, delta = 1e-3, L = 64
    assert exact.hoeffding_R(0.02, 1e-3, C, 64) == 9502
    assert exact.hoeffding_R(0.05, 1e-3, C, 64) == 1521
    assert exact.hoeffding_R(0.01, 1e-3, C, 64) == 38005
    # union bound over n nodes: ln(2n/delta)
    n = 1 << 20
    assert exact.hoeffding_R(0.02, 1e-3, C, 64, n=n) == math.ceil(math.log(2 * n / 1e-3) / (2 * 0.02 ** 2))
    with pytest.raises(ValueError):
        exact.hoeffding_R(1e-16, 1e-3, C, 64)
