"""The host-thread fan-out used by the full-size parity tests returns exactly
what one oracle call over all listed nodes returns (plain counts, stitched
counts, stratified weighted sums), for any number of threads, including
chunks smaller than the thread count and a single node."""
import numpy as np

import oracle as O
import oracle_threads as OT
from paper_2304_04015_amd import inputs


def test_fan_out_equals_one_call():
    g = inputs.rmat_in(9, 8 << 9, seed=5)
    s = int(np.argmax(g.in_degree()))
    vs = OT.sample_nodes(g, 60, 8, 4, seed=3, extra=[s])
    assert np.all(np.diff(vs) > 0) and s in vs
    want = O.meet_counts_plain(g, s, 77, 0.6, 32, 300, vs=vs)
    P = O.pool_sizes(g, 1.0)
    want_st = O.meet_counts_stitched(g, s, 78, 79, 0.7, 32, 4, P, 200, vs=vs)
    SP = O.strat_params(g.n, 0.6, 0.1, z=400.0, phi=8)
    want_w = O.strat_sums(g, s, 80, SP, vs=vs)
    for nt in (1, 3, 7, 200):
        assert np.array_equal(OT.meet_counts_plain(g, s, 77, 0.6, 32, 300, vs, threads=nt), want)
        assert np.array_equal(OT.meet_counts_stitched(g, s, 78, 79, 0.7, 32, 4, P, 200, vs,
                                                      threads=nt), want_st)
        assert np.array_equal(OT.strat_sums(g, s, 80, SP, vs, threads=nt), want_w)
    one = vs[:1]
    assert np.array_equal(OT.meet_counts_plain(g, s, 77, 0.6, 32, 300, one, threads=4), want[:1])
    assert want.sum() > 300 and want_w.sum() > 0
