"""Pins of the oracle's length-stratified estimator (Algorithm 1: N_l walks of
exact length l per node, then a shuffle; Algorithm 2 with Lemma 5: weighted
meets / z) against what the paper and the mathematics fix: the class sizes'
closed forms, the shuffle being a permutation with the class histogram Zhat,
uniform steps, first-meeting probabilities that rebuild the SimRank iterates
of Eq. 1, and the estimator's mean."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import exact as X
from paper_2304_04015_amd import inputs

SEED = 0x2304040150000021


def _no_dead_ends(n, mean_in, seed):
    """Random graph in which every node has at least one in-neighbour."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for v in range(n):
        k = 1 + rng.poisson(mean_in - 1)
        us = rng.choice(n, size=min(k, n), replace=False)
        src += list(us)
        dst += [v] * len(us)
    g = inputs.from_edges(n, src, dst, dedupe=True, drop_self_loops=False)
    assert (g.in_degree() > 0).all()
    return g


def _star(n):
    """Every node's only in-neighbour is node 0, which has a self-loop."""
    return inputs.from_edges(n, [0] * n, list(range(n)), dedupe=True, drop_self_loops=False)


@pytest.mark.parametrize("n,c,eps", [(500, 0.6, 0.05), (1 << 20, 0.6, 0.02), (1 << 24, 0.6, 0.02),
                                     (1000, 0.8, 0.03), (50, 0.3, 0.2)])
def test_class_sizes_closed_forms(n, c, eps):
    P = O.strat_params(n, c, eps)
    r = math.sqrt(c)
    # z from Algorithm 2's formula; the classes are a truncated geometric series
    assert P.z == pytest.approx(math.log(2 * n) / (2 * (eps - 3 / n) ** 2), rel=1e-14)
    assert P.Z.sum() == pytest.approx(P.z * (1 - r ** (P.phi + 1)), rel=1e-12)
    assert np.all(P.Zhat >= P.Z) and np.all(P.Zhat < P.Z + 1)
    assert 0 <= P.N - P.Z.sum() < P.phi + 1
    assert P.N == int(P.Zhat.sum())
    # phi = floor(log_{1/sqrt c} n): sqrt(c)^phi >= 1/n > sqrt(c)^(phi+1)
    assert r ** P.phi >= 1.0 / n * (1 - 1e-12)
    assert r ** (P.phi + 1) < 1.0 / n
    with pytest.raises(ValueError):
        O.strat_params(n, c, 3.0 / n)            # eps must exceed 3/n


def test_medium_workload_sizes():
    """At n = 2^20, c = 0.6, eps = 0.02: phi = 54 and z / N = 0.998 (the
    estimator forms slightly more pairs than z)."""
    P = O.strat_params(1 << 20, 0.6, 0.02)
    assert P.phi == 54
    assert P.N == 18234
    assert abs(P.z / P.N - 0.9982) < 1e-4


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 8, 9, 100, 1000, 4096, 4097, 18234])
def test_shuffle_is_a_permutation(N):
    for v in (0, 1, 12345, 2 ** 31 - 1):
        slots = np.array([O.shuffle_slot(SEED, v, j, N) for j in range(N)])
        assert np.array_equal(np.sort(slots), np.arange(N)), (N, v)


def test_shuffled_classes_have_histogram_zhat():
    g = _no_dead_ends(30, 3.0, 1)
    P = O.strat_params(g.n, 0.6, 0.0, z=700.0, phi=9)
    for v in (0, 7, 29):
        js = np.arange(P.N, dtype=np.uint32)
        _, lens, slots, cls = O.walk_table_strat(g, SEED, P, np.full(P.N, v), js)
        assert np.array_equal(np.bincount(cls, minlength=P.phi + 1), P.Zhat)
        assert np.array_equal(lens, cls)          # no dead ends: every walk has its class length
        start = np.concatenate([[0], np.cumsum(P.Zhat)])
        assert np.all((start[cls] <= slots) & (slots < start[cls + 1]))


def test_shuffle_is_uniform():
    """Walk j's slot over many nodes is uniform on [0, N), and two walks of a
    node are in distinct slots with the without-replacement joint law."""
    N, nv = 40, 40000
    s0 = np.array([O.shuffle_slot(SEED, v, 0, N) for v in range(nv)])
    s1 = np.array([O.shuffle_slot(SEED, v, 1, N) for v in range(nv)])
    exp = nv / N
    chi0 = ((np.bincount(s0, minlength=N) - exp) ** 2 / exp).sum()
    chi1 = ((np.bincount(s1, minlength=N) - exp) ** 2 / exp).sum()
    # chi-square with 39 degrees of freedom: the 1e-6 upper quantile is about 95
    assert chi0 < 95 and chi1 < 95
    assert np.all(s0 != s1)
    # joint: both in the lower half with probability (20/40)(19/39)
    both = np.mean((s0 < N // 2) & (s1 < N // 2))
    assert abs(both - (20 / 40) * (19 / 39)) < 5 * math.sqrt(0.25 * 0.75 / nv)


def test_fixed_length_walks_take_uniform_steps():
    g = _star(6)
    g2 = _no_dead_ends(12, 4.0, 5)
    off, src = g2.in_off, g2.in_src
    v = int(np.argmax(g2.in_degree()))
    nbrs = src[off[v]:off[v + 1]]
    first = np.array([O.walk_strat(g2, SEED, 3, v, r)[1] for r in range(30000)])
    for w in O.walk_strat(g2, SEED, 3, v, 5), O.walk_strat(g2, SEED, 3, v, 6):
        assert w.size == 4
        for a, b in zip(w[:-1], w[1:]):
            assert b in src[off[a]:off[a + 1]]
    cnt = np.array([np.sum(first == u) for u in nbrs])
    exp = first.size / nbrs.size
    assert cnt.sum() == first.size
    assert ((cnt - exp) ** 2 / exp).sum() < 40
    # a walk on the star is at node 0 from step 1 on
    assert np.array_equal(O.walk_strat(g, SEED, 4, 3, 11), [3, 0, 0, 0, 0])


def test_walk_ends_at_a_dead_end():
    g = inputs.from_edges(4, [1, 2], [0, 1])       # 0 <- 1 <- 2, node 2 has no in-neighbour
    assert np.array_equal(O.walk_strat(g, SEED, 5, 0, 0), [0, 1, 2])
    assert np.array_equal(O.walk_strat(g, SEED, 0, 0, 0), [0])


@pytest.mark.parametrize("seed", [2, 3])
def test_first_meeting_rebuilds_simrank_iterates(seed):
    """Without dead ends, S_k(s, u) = sum_{t <= k} c^t F_t(s, u) (each step of
    both sqrt(c)-walks survives with probability c; Lemma 2)."""
    g = _no_dead_ends(14, 2.5, seed)
    c = 0.6
    for s in (0, 5):
        F = X.first_meet_probs(g.n, g.in_off, g.in_src, s, 8)
        for k in (1, 2, 5, 8):
            S = X.simrank_iterates(g.n, g.in_off, g.in_src, c, k)
            rebuilt = sum(c ** t * F[t] for t in range(1, k + 1))
            u = np.arange(g.n) != s
            assert np.allclose(rebuilt[u], S[s, u], atol=1e-13, rtol=0), (s, k)


def test_star_graph_meets_at_step_one():
    g = _star(8)
    F = X.first_meet_probs(g.n, g.in_off, g.in_src, 3, 5)
    u = np.arange(8) != 3
    assert np.allclose(F[1, u], 1.0) and np.allclose(F[2:, u], 0.0)
    c, phi = 0.6, 7
    E = X.stratified_expectation(g.n, g.in_off, g.in_src, c, 3, phi)
    r = math.sqrt(c)
    assert np.allclose(E[u], (r - r ** (phi + 1)) ** 2, rtol=1e-14)


def test_star_graph_sums_are_the_class_pairing():
    """On the star every pair of walks with both lengths >= 1 meets at step 1,
    so the weighted sum is fixed by the shuffles alone."""
    g = _star(10)
    P = O.strat_params(g.n, 0.6, 0.0, z=200.0, phi=6)
    s = 4
    wsum, meets, work = O.strat_sums(g, s, SEED, P, with_stats=True)
    cls_s = O.walk_table_strat(g, SEED, P, np.full(P.N, s), np.arange(P.N))[3]
    a = P.Z / P.Zhat
    for u in range(g.n):
        if u == s:
            assert wsum[u] == 0 and meets[u] == 0
            continue
        cls_u = O.walk_table_strat(g, SEED, P, np.full(P.N, u), np.arange(P.N))[3]
        both = (cls_s >= 1) & (cls_u >= 1)
        want = sum(int(math.ldexp(a[x] * a[y], 40)) for x, y in zip(cls_s[both], cls_u[both]))
        assert int(wsum[u]) == want
        assert meets[u] == both.sum() and work[u] == both.sum()


def test_sums_equal_brute_force_pairing():
    g = _no_dead_ends(16, 2.0, 9)
    P = O.strat_params(g.n, 0.7, 0.0, z=300.0, phi=8)
    s = 2
    vs = np.array([0, 1, 2, 7, 15], np.int32)
    wsum, meets, work = O.strat_sums(g, s, SEED, P, vs=vs, with_stats=True)
    js = np.arange(P.N, dtype=np.uint32)
    ps, ls, _, cs = O.walk_table_strat(g, SEED, P, np.full(P.N, s), js)
    a = P.Z / P.Zhat
    for i, u in enumerate(vs):
        if u == s:
            assert wsum[i] == 0
            continue
        pu, lu, _, cu = O.walk_table_strat(g, SEED, P, np.full(P.N, u), js)
        acc = m = w = 0
        for j in range(P.N):
            lim = min(ls[j], lu[j])
            hit = [t for t in range(1, lim + 1) if ps[j, t] == pu[j, t]]
            if hit:
                acc += int(math.ldexp(a[cs[j]] * a[cu[j]], 40))
                m += 1
                w += hit[0]
            else:
                w += lim
        assert (int(wsum[i]), int(meets[i]), int(work[i])) == (acc, m, w), u


def test_weights_are_lemma_5_ratios():
    P = O.strat_params(2000, 0.6, 0.04)
    a = P.Z / P.Zhat
    for l1, l2 in [(0, 0), (0, 5), (5, 0), (3, P.phi), (P.phi, P.phi)]:
        w = O.strat_weight(P, l1, l2)
        assert w == O.strat_weight(P, l2, l1)
        assert w <= 1 << 40
        assert abs(w / 2.0 ** 40 - (P.Z[l1] * P.Z[l2]) / (P.Zhat[l1] * P.Zhat[l2])) < 2.0 ** -39


def test_estimator_mean_over_seeds():
    """With few walks (z = 30, so the rounding Zhat_l = ceil(Z_l) distorts the
    length law strongly) the average over many seeds of the N-normalised
    estimate matches its exact mean, and Algorithm 2's estimate is z/N times
    it.  A weight that ignored Lemma 5's correction would be off by far more
    than the tolerance here."""
    g = _no_dead_ends(12, 2.0, 4)
    c, s = 0.6, 0
    P = O.strat_params(g.n, c, 0.0, z=30.0, phi=6)
    E = X.stratified_expectation(g.n, g.in_off, g.in_src, c, s, P.phi)
    runs = []
    for k in range(600):
        w = O.strat_sums(g, s, SEED + 7919 * k, P)
        out, out_n = O.strat_estimates(w, s, P)
        assert out[s] == out_n[s] == 1.0
        assert np.allclose(np.delete(out, s) * P.N / P.z, np.delete(out_n, s), rtol=1e-15)
        runs.append(out_n)
    runs = np.array(runs)
    mean, se = runs.mean(axis=0), runs.std(axis=0) / math.sqrt(len(runs))
    u = np.arange(g.n) != s
    assert np.all(np.abs(mean[u] - E[u]) < 5 * se[u] + 1e-3), (mean - E, se)
    # the uncorrected mean (every meet weighted 1, i.e. lengths drawn with the
    # sampling law Zhat_l / N instead of the geometric law) is far off
    F = X.first_meet_probs(g.n, g.in_off, g.in_src, s, P.phi)
    tail = np.array([P.Zhat[t:].sum() / P.N for t in range(P.phi + 1)])
    E_unweighted = (tail[1:, None] ** 2 * F[1:]).sum(axis=0)
    assert np.max(np.abs(E_unweighted[u] - E[u])) > 20 * np.max(se[u])


def test_estimate_within_eps_at_paper_z():
    """One estimate at Algorithm 2's z for eps = 0.05 on a graph without dead
    ends lies within eps of the exact SimRank for every node (Theorem 5)."""
    g = _no_dead_ends(40, 3.0, 6)
    c, s, eps = 0.6, 1, 0.1
    P = O.strat_params(g.n, c, eps)
    S = X.exact_simrank(g.n, g.in_off, g.in_src, c)
    w = O.strat_sums(g, s, SEED, P)
    out, out_n = O.strat_estimates(w, s, P)
    assert np.max(np.abs(out - S[s])) < eps
    assert np.max(np.abs(out_n - S[s])) < eps


# ---------------------------------------------------------------- tuple form

def test_tuple_form_equals_pairwise_plain():
    """Algorithm 2's sort + PREDECESSOR detection and the direct pairwise
    comparison are two statements of the same counts."""
    from oracle import tuples as TU
    for seed, gg in [(1, _no_dead_ends(40, 3.0, 11)), (2, inputs.rmat_in(7, 5 << 7, seed=12)),
                     (3, _star(9))]:
        for s in (0, 3):
            want = O.meet_counts_plain(gg, s, SEED + seed, 0.6, 16, 300)
            got = TU.counts_plain(gg, s, SEED + seed, 0.6, 16, 300)
            assert np.array_equal(got, want), (seed, s)


def test_tuple_form_equals_pairwise_stratified():
    from oracle import tuples as TU
    for seed, gg in [(4, _no_dead_ends(30, 2.5, 13)), (5, inputs.rmat_in(7, 4 << 7, seed=14))]:
        P = O.strat_params(gg.n, 0.6, 0.0, z=250.0, phi=9)
        for s in (1, 6):
            want = O.strat_sums(gg, s, SEED + seed, P)
            got = TU.sums_stratified(gg, s, SEED + seed, P)
            assert np.array_equal(got, want), (seed, s)


def test_tuple_form_counts_a_pair_once():
    """On the star every pair of walks of length >= 2 coincides at steps 1 and
    2 (both at node 0): two linked tuples, one meet."""
    from oracle import tuples as TU
    g = _star(5)
    js = np.arange(4, dtype=np.uint32)
    paths = np.array([[1, 0, 0, -1], [1, 0, -1, -1], [2, 0, 0, 0], [2, -1, -1, -1]], np.int32)
    lens = np.array([2, 1, 3, 0])
    starts = np.array([1, 1, 2, 2])
    jj = np.array([0, 1, 0, 1], np.uint32)
    met = TU.link_meets(*TU.decompose(paths, lens, starts, jj), 1)
    assert met.tolist() == [[2, 0]]
    assert js.size == 4 and g.n == 5
