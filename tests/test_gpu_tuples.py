"""Algorithm 2's tuple form on the GPU (decompose, radix sort, PREDECESSOR,
count once) against the fused meet kernel and against the oracle's tuple
form: counts and weighted sums must agree bit for bit."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import tuples as TU
from paper_2304_04015_amd import inputs
from paper_2304_04015_amd import simrank as S

pytestmark = pytest.mark.gpu

SEED = 0x2304040150000041


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small():
    g = inputs.rmat_in(10, 8 << 10, seed=81)
    return g, S.load_csr(g)


def _sources(g, k, seed):
    return [int(x) for x in inputs.sources_with_in_edges(g, k, seed)]


def test_plain_counts_equal_fused_and_oracle(small):
    g, G = small
    srcs = _sources(g, 5, 1) + [int(np.argmax(g.in_degree() == 0))]   # one source without in-edges
    qs = [S.make_query(s, c=0.6, seed=SEED, walk_cap=20, R=700) for s in srcs]
    sums, st = S.simrank_tuple_meets(G, qs)
    _say(f"tuple form: {st.moves} tuples, {st.meets} meets, {st.ms:.1f} ms")
    for q, s in enumerate(srcs):
        fused = S.simrank_single_source_ex(G, qs[q])[1]
        assert np.array_equal(sums[q], fused.astype(np.uint64)), q
    want = TU.counts_plain(g, srcs[0], SEED, 0.6, 20, 700)
    assert np.array_equal(sums[0], want.astype(np.uint64))
    assert st.meets == int(sum(sums[q].sum() - 700 for q in range(len(srcs))))


def test_stratified_sums_equal_fused_and_oracle(small):
    g, G = small
    srcs = _sources(g, 3, 2)
    qs = [S.make_stratified_query(s, c=0.6, eps=0.1, seed=SEED, z=600, phi=12) for s in srcs]
    sums, st = S.simrank_tuple_meets(G, qs)
    for q in range(len(srcs)):
        assert np.array_equal(sums[q], S.simrank_single_source_stratified(G, qs[q])[2]), q
    P = O.strat_params(g.n, 0.6, 0.1, z=600.0, phi=12)
    assert np.array_equal(sums[1], TU.sums_stratified(g, srcs[1], SEED, P))


def test_many_chunks_and_sources():
    """2^17 nodes x 3,000 walks: more tuples than one chunk holds, so nodes are
    processed in several chunks; 32 sources at once."""
    g = inputs.rmat_in(17, 12 << 17, seed=82)
    G = S.load_csr(g)
    srcs = _sources(g, 32, 3)
    qs = [S.make_query(s, c=0.6, seed=SEED, walk_cap=64, R=3000) for s in srcs]
    sums, st = S.simrank_tuple_meets(G, qs)
    _say(f"tuple form 2^17: {st.moves} tuples, {st.meets} meets, {st.ms:.1f} ms, "
         f"sort {st.meet_ms:.1f} ms / {st.draws} bytes")
    assert st.moves > (1 << 28)          # more tuples than one chunk holds
    # the sort's time and bytes: every tuple (sources' copies included) passes
    # through at least one histogram and one scatter pass
    assert 0 < st.meet_ms < st.ms and st.draws >= 32 * st.moves
    for q in (0, 13, 31):
        fused = S.simrank_single_source_ex(G, qs[q])[1]
        assert np.array_equal(sums[q], fused.astype(np.uint64)), q


def test_rejects(small):
    g, G = small
    q = S.make_query(1, seed=SEED, R=100)
    with pytest.raises(S.SimRankError):
        S.simrank_tuple_meets(G, [])
    with pytest.raises(S.SimRankError):
        S.simrank_tuple_meets(G, [q] * 33)
    with pytest.raises(S.SimRankError):
        S.simrank_tuple_meets(G, [q, S.make_query(2, seed=SEED + 1, R=100)])
    with pytest.raises(S.SimRankError):
        S.simrank_tuple_meets(G, [q, S.make_query(2, seed=SEED, R=101)])
    with pytest.raises(S.SimRankError):
        S.simrank_tuple_meets(G, [S.make_query(1, seed=SEED, R=100, mode=S.MODE_STITCHED)])
    with pytest.raises(S.SimRankError):
        S.simrank_tuple_meets(G, [S.make_query(g.n, seed=SEED, R=100)])
