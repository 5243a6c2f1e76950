"""The stitched-walk oracle against the exact law of stitched walks on a tiny
graph (Theorem 2 and Section 4.1: long walks assembled from per-node pools of
short segments joined end to start).

Two stitched walks that enter the same pool slot share its segment and its
successor, so their meeting probability is not the plain walks' S_L of
Lemma 2.  Here it is computed exactly: every outcome of both walks' private
heads, their entry picks and, lazily, the contents of each pool slot they
reach (the segment's steps and its successor pick) is enumerated with its
probability, the slots revealed so far being shared by both walks.  The
oracle's meet counts, averaged over many (walk seed, index seed) pairs, must
agree with it to within sampling error; and the sampling error is small
enough that plain S_L (what walks with fresh segments, i.e. without the
sharing, would give) is rejected.
"""
import numpy as np
import pytest

import oracle as O
from paper_2304_04015_amd import inputs

C = 0.6
TWO32 = 1 << 32
# six nodes with in-degrees 2..3 and rows that list each node 1..3 times
EDGES = [(1, 0), (2, 0), (0, 1), (3, 1), (4, 1), (0, 2), (5, 2), (1, 3), (2, 3), (2, 4),
         (3, 4), (0, 5), (4, 5)]


def _cdiv(a, b):
    return -(-a // b)


def _uniform_pick(d):
    """Probabilities of floor(x * d / 2^32) = k for x uniform on [0, 2^32)."""
    return [(_cdiv((k + 1) * TWO32, d) - _cdiv(k * TWO32, d)) / TWO32 for k in range(d)]


class StitchedLaw:
    def __init__(self, g, P):
        self.off = np.asarray(g.in_off)
        self.src = np.asarray(g.in_src)
        self.go = O.continue_threshold(C) / TWO32      # a step continues with T / 2^32
        self.P = [int(p) for p in P]
        self.memo = {}

    def walks(self, x, cap):
        """Every walk of at most cap moves from x, as (probability, positions after x)."""
        if (x, cap) in self.memo:
            return self.memo[(x, cap)]
        d = int(self.off[x + 1] - self.off[x])
        if cap == 0 or d == 0:
            out = [(1.0, ())]
        else:
            out = [(1.0 - self.go, ())]
            for k, pk in enumerate(_uniform_pick(d)):
                u = int(self.src[self.off[x] + k])
                out += [(self.go * pk * q, (u,) + rest) for q, rest in self.walks(u, cap - 1)]
        self.memo[(x, cap)] = out
        return out

    def slot(self, y, seglen):
        """Every content of a pool slot of y: its segment and, if the segment
        made all seglen moves, its successor slot in the pool of its end node."""
        out = []
        for q, seg in self.walks(y, seglen):
            if len(seg) == seglen:
                out += [(q * pi, seg, (seg[-1], i)) for i, pi in enumerate(_uniform_pick(self.P[seg[-1]]))]
            else:
                out.append((q, seg, None))
        return out

    def later(self, t, a, b, known, L, seglen):
        """P(meet after time t | walks at slots a and b at time t, slot contents known)."""
        total = 0.0
        for qa, sa, na in ([(1.0, *known[a])] if a in known else self.slot(a[0], seglen)):
            ka = known if a in known else {**known, a: (sa, na)}
            for qb, sb, nb in ([(1.0, *ka[b])] if b in ka else self.slot(b[0], seglen)):
                if any(sa[k] == sb[k] for k in range(min(len(sa), len(sb), L - t))):
                    total += qa * qb
                elif na is not None and nb is not None and t + seglen < L:
                    kb = ka if b in ka else {**ka, b: (sb, nb)}
                    total += qa * qb * self.later(t + seglen, na, nb, kb, L, seglen)
        return total

    def meet(self, s, v, L, seglen):
        total = 0.0
        for ps, hs in self.walks(s, min(seglen, L)):
            for pv, hv in self.walks(v, min(seglen, L)):
                a, b = (s,) + hs, (v,) + hv
                if any(a[k] == b[k] for k in range(min(len(a), len(b)))):
                    total += ps * pv
                elif len(hs) == len(hv) == seglen < L:
                    for i, qi in enumerate(_uniform_pick(self.P[hs[-1]])):
                        for k, qk in enumerate(_uniform_pick(self.P[hv[-1]])):
                            total += ps * pv * qi * qk * self.later(
                                seglen, (hs[-1], i), (hv[-1], k), {}, L, seglen)
        return total

    def plain(self, s, v, L):
        total = 0.0
        for ps, a in self.walks(s, L):
            for pv, b in self.walks(v, L):
                if any(x == y for x, y in zip((s,) + a, (v,) + b)):
                    total += ps * pv
        return total


@pytest.fixture(scope="module")
def g():
    return inputs.from_edges(6, [a for a, _ in EDGES], [b for _, b in EDGES], "six")


def _sampled(g, P, L, seglen, s, pairs, R):
    """Mean of cnt/R over independent (walk seed, index seed) pairs, and its
    standard error from the spread of the per-pair means."""
    est = np.array([O.meet_counts_stitched(g, s, 0x5EED0000 + k, 0x1D0E0000 + 7 * k, C, L, seglen,
                                           P, R) / R for k in range(pairs)])
    return est.mean(0), est.std(0, ddof=1) / np.sqrt(pairs)


def test_uniform_pick_probabilities():
    for d in (1, 2, 3, 5, 7, 1000):
        p = _uniform_pick(d)
        assert abs(sum(p) - 1.0) < 1e-15 and max(p) - min(p) <= 1.0 / TWO32 + 1e-18


def test_one_round_of_tails_is_plain(g):
    """With a single segment after the heads, the two walks sit at distinct
    nodes when they enter their pools, so no slot is shared: exactly S_L."""
    law = StitchedLaw(g, O.pool_sizes(g, 1.0))
    for v in range(1, g.n):
        assert law.meet(0, v, 4, 2) == pytest.approx(law.plain(0, v, 4), abs=1e-12)


@pytest.mark.parametrize("kappa,L,seglen", [(0.5, 4, 1), (0.5, 5, 1), (1.0, 4, 1)])
def test_oracle_meets_at_the_exact_stitched_rate(g, kappa, L, seglen):
    P = O.pool_sizes(g, kappa)
    law = StitchedLaw(g, P)
    s = 0
    want = np.array([law.meet(s, v, L, seglen) for v in range(g.n)])
    plain = np.array([law.plain(s, v, L) for v in range(g.n)])
    got, se = _sampled(g, P, L, seglen, s, 1600, 2000)
    for v in range(1, g.n):
        assert abs(got[v] - want[v]) <= 4.5 * se[v], (v, got[v], want[v], se[v])
    # the sampling error resolves the effect of shared slots: walks with fresh
    # segments (meeting at the plain rate) would be off by more than six
    # standard errors over the five nodes together (chi-square, 5 degrees of
    # freedom: P(> 36) ~ 1e-6)
    sharing = (plain[1:] - want[1:]) / se[1:]
    assert np.sqrt(np.sum(sharing ** 2)) > 6.0, sharing
