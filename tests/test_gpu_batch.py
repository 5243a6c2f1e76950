"""Batched queries (one captured launch sequence over many queries and graphs)
and the work-unit tuner: every result must equal the lone query's, bit for
bit, and the lone query's equals the oracle's (test_gpu_parity)."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle_threads as OT
from paper_2304_04015_amd import inputs
from paper_2304_04015_amd import simrank as S

pytestmark = pytest.mark.gpu

ISEED = 0x2304040150000013


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def graphs():
    gs = [inputs.erdos_renyi_in(700, 4.0, seed=31), inputs.rmat_in(12, 12 << 12, seed=32),
          inputs.rmat_in(14, 20 << 14, seed=33), inputs.from_edges(6, [0] * 5, [1, 2, 3, 4, 5])]
    Gs = [S.load_csr(g) for g in gs]
    S.simrank_build_index(Gs[1], seg_log2=3, kappa=1.0, c=0.6, seed=ISEED)
    return gs, Gs


def _mix(gs, nq, seed):
    rng = np.random.default_rng(seed)
    qs = []
    for i in range(nq):
        gi = int(rng.integers(0, len(gs)))
        act = np.nonzero(gs[gi].in_degree() > 0)[0]
        s = int(rng.choice(act)) if act.size and rng.random() < 0.9 else int(rng.integers(0, gs[gi].n))
        eps = float(rng.choice([0.05, 0.03, 0.02]))
        mode = S.MODE_STITCHED if (gi == 1 and rng.random() < 0.5) else S.MODE_PLAIN
        qs.append(S.make_query(s, c=0.6, eps=eps, delta=1e-3, seed=1000 + i, walk_cap=64,
                               mode=mode, graph=gi))
    return qs


def test_batch_equals_lone_queries(graphs):
    gs, Gs = graphs
    qs = _mix(gs, 40, 1)
    outs, cnts, st = S.simrank_batch(Gs, qs)
    for i, q in enumerate(qs):
        o1, c1, _ = S.simrank_single_source_ex(Gs[q.graph], q)
        assert np.array_equal(cnts[i], c1), i
        assert np.array_equal(outs[i], o1), i
    assert st.moves > 0
    # one plain and one stitched query also against the oracle
    P = O.pool_sizes(gs[1], 1.0)
    for i, q in enumerate(qs[:12]):
        g = gs[q.graph]
        if q.mode == S.MODE_STITCHED:
            want = O.meet_counts_stitched(g, q.s, q.seed, ISEED, 0.6, 64, 8, P,
                                          S.simrank_derive_params(q, g.n).R)
        else:
            want = O.meet_counts_plain(g, q.s, q.seed, 0.6, 64, S.simrank_derive_params(q, g.n).R)
        assert np.array_equal(cnts[i], want), i


def test_plan_replays_match(graphs):
    """The captured graph is replayed several times, with the program's own
    eager work and synchronisations between replays; every replay must equal
    the eager results."""
    import torch
    gs, Gs = graphs
    qs = _mix(gs, 24, 2)
    lone = [S.simrank_single_source_ex(Gs[q.graph], q)[1] for q in qs]
    plan = S.BatchPlan(Gs, qs)
    stream = torch.cuda.Stream()
    for rep in range(3):
        plan.run(stream)
        st = plan.wait()
        for i in range(len(qs)):
            _, c = plan.read(i, want_out=False)
            assert np.array_equal(c, lone[i]), (rep, i)
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        y = (x * 2).sum()
        torch.cuda.synchronize()
        o, c, _ = S.simrank_single_source_ex(Gs[qs[0].graph], qs[0])
        assert np.array_equal(c, lone[0]) and float(y) == float(y)
    assert st.pairs > 0
    plan.free()


def test_tuner_keeps_results(graphs):
    gs, Gs = graphs
    g, G = gs[2], Gs[2]
    q = S.make_query(int(np.argmax(g.in_degree())), c=0.6, eps=0.03, seed=77)
    before = S.simrank_single_source_ex(G, q)[1]
    vb = S.simrank_tune(G, q)
    assert vb in (32, 64, 128, 256)
    after = S.simrank_single_source_ex(G, q)[1]
    assert np.array_equal(before, after)


def test_batch_rejects_bad_queries(graphs):
    gs, Gs = graphs
    q = S.make_query(0, graph=7)
    with pytest.raises(S.SimRankError):
        S.simrank_batch(Gs, [q])
    q = S.make_query(10 ** 6, graph=0)
    with pytest.raises(S.SimRankError):
        S.simrank_batch(Gs, [q])
    q = S.make_query(1, graph=2, mode=S.MODE_STITCHED)       # graph 2 has no index
    with pytest.raises(S.SimRankError):
        S.simrank_batch(Gs, [q])


def test_batch_with_stratified_queries(graphs):
    """Stratified queries mixed into a batch (and a captured plan) give what
    the lone stratified call gives, bit for bit."""
    gs, Gs = graphs
    mix = _mix(gs, 12, 5)
    strat = [S.make_stratified_query(q.s, c=0.6, eps=0.2, seed=2000 + i, z=700 + 50 * i, phi=12,
                                     graph=q.graph) for i, q in enumerate(mix[:6])]
    qs = [x for pair in zip(mix[6:], strat) for x in pair]
    outs, cnts, st = S.simrank_batch(Gs, qs)
    plan = S.BatchPlan(Gs, qs)
    plan.run()
    plan.wait()
    for i, q in enumerate(qs):
        if q.mode == S.MODE_STRATIFIED:
            o1, on1, w1, _ = S.simrank_single_source_stratified(Gs[q.graph], q)
            assert np.array_equal(outs[i], o1), i
            o, on, w = plan.read_stratified(i)
            assert np.array_equal(w, w1) and np.array_equal(on, on1) and np.array_equal(o, o1), i
            with pytest.raises(S.SimRankError):
                plan.read(i, want_out=False, want_counts=True)
        else:
            o1, c1, _ = S.simrank_single_source_ex(Gs[q.graph], q)
            assert np.array_equal(cnts[i], c1) and np.array_equal(outs[i], o1), i
            assert np.array_equal(plan.read(i)[1], c1), i
    plan.free()


def test_shared_seed_groups_equal_lone_queries(graphs):
    """Plain queries with equal (graph, seed, c, cap) run in groups that share
    the walks from every node: 11 on one graph (a group of more than 8 members
    with different R, spanning several group tiles with a ragged last one, a
    repeated source, a source without in-edges), 3 on another, 2 with another
    cap, 2 on the star graph, 40 on the small graph with another seed (two
    groups of 20); stitched and stratified queries with the same seed and lone
    plain queries stay out of the groups; stitched queries form groups of their
    own (3 and 12 members).  Every result equals the lone query's and the
    ungrouped plan's, bit for bit."""
    gs, Gs = graphs
    g2 = gs[2]
    act = np.nonzero(g2.in_degree() > 0)[0]
    rng = np.random.default_rng(9)
    S1, S2 = 0x2304040150000051, 0x2304040150000052
    srcs = [int(x) for x in rng.choice(act, 9, replace=False)]
    srcs += [srcs[0], int(np.argmax(g2.in_degree() == 0))]
    Rs = [3000, 4100, 2500, 1, 3000, 700, 5200, 3000, 3333, 4100, 2000]
    qs = [S.make_query(s, c=0.6, seed=S1, walk_cap=64, R=R, graph=2) for s, R in zip(srcs, Rs)]
    qs += [S.make_query(int(s), c=0.6, seed=S1, walk_cap=64, R=1500, graph=0)
           for s in rng.choice(np.nonzero(gs[0].in_degree() > 0)[0], 3, replace=False)]
    qs += [S.make_query(srcs[k], c=0.6, seed=S2, walk_cap=20, R=2048, graph=2) for k in (1, 2)]
    qs += [S.make_query(s, c=0.6, seed=S1, walk_cap=64, R=900, graph=3) for s in (1, 0)]
    act0 = np.nonzero(gs[0].in_degree() > 0)[0]
    qs += [S.make_query(int(s), c=0.6, seed=S2, walk_cap=64, R=int(R), graph=0)
           for s, R in zip(rng.choice(act0, 40), rng.integers(200, 3000, 40))]
    qs += [S.make_query(srcs[3], c=0.5, seed=S1, walk_cap=64, R=3000, graph=2)]   # lone: other c
    act1 = np.nonzero(gs[1].in_degree() > 0)[0]
    qs += [S.make_query(int(act1[3]), c=0.6, seed=S1, walk_cap=64, R=3000, graph=1,
                        mode=S.MODE_STITCHED)]                                 # lone stitched
    qs += [S.make_query(int(s), c=0.6, seed=S2, walk_cap=64, R=int(R), graph=1,
                        mode=S.MODE_STITCHED)                                  # stitched, 3 and 12
           for s, R in zip(rng.choice(act1, 3), (1800, 2500, 900))]
    qs += [S.make_query(int(s), c=0.6, seed=S1 + 7, walk_cap=64, R=int(R), graph=1,
                        mode=S.MODE_STITCHED)
           for s, R in zip(rng.choice(act1, 12), rng.integers(300, 3000, 12))]
    qs += [S.make_query(int(act1[5]), c=0.6, seed=S2, walk_cap=64, R=1000, graph=1)]   # plain
    qs += [S.make_stratified_query(srcs[4], c=0.6, eps=0.2, seed=S1, z=700, phi=12, graph=2)]
    order = rng.permutation(len(qs))
    qs = [qs[i] for i in order]
    _say(f"shared-seed batch: {len(qs)} queries")
    plan = S.BatchPlan(Gs, qs)
    assert plan.n_groups == 8
    plan.run()
    st_g = plan.wait()
    flat = S.BatchPlan(Gs, qs, groups=False)
    assert flat.n_groups == 0
    flat.run()
    st_f = flat.wait()
    for i, q in enumerate(qs):
        if q.mode == S.MODE_STRATIFIED:
            assert np.array_equal(plan.read_stratified(i)[2], flat.read_stratified(i)[2]), i
            continue
        o1, c1, _ = S.simrank_single_source_ex(Gs[q.graph], q)
        o, c = plan.read(i)
        of, cf = flat.read(i)
        assert np.array_equal(c, c1) and np.array_equal(o, o1), i
        assert np.array_equal(cf, c1), i
    assert st_g.meets == st_f.meets
    assert st_g.moves < st_f.moves            # the shared walks are taken once
    # a member on the small graph against the oracle
    for seed in (S1, S2):
        i = next(k for k, q in enumerate(qs) if q.graph == 0 and q.seed == seed)
        want = O.meet_counts_plain(gs[0], qs[i].s, seed, 0.6, 64, qs[i].R_override)
        assert np.array_equal(plan.read(i)[1], want), seed
    P = O.pool_sizes(gs[1], 1.0)
    i = next(k for k, q in enumerate(qs) if q.mode == S.MODE_STITCHED and q.seed == S1 + 7)
    want = O.meet_counts_stitched(gs[1], qs[i].s, S1 + 7, ISEED, 0.6, 64, 8, P, qs[i].R_override)
    assert np.array_equal(plan.read(i)[1], want)
    plan.free()
    flat.free()


@pytest.mark.parametrize("nq,mode", [(8, S.MODE_PLAIN), (21, S.MODE_PLAIN),
                                     (6, S.MODE_STITCHED), (21, S.MODE_STITCHED)])
def test_shared_seed_group_full_size(nq, mode):
    """Queries with the medium workload's shape (2^16-node R-MAT graph, eps
    0.02, R = 9,502, cap 64) and one seed, plain and stitched (index with
    k = 3, kappa = 1), as one group of up to 8 and one of 21: the group's
    counts equal the lone queries', bit for bit."""
    g = inputs.rmat_in(16, 16 << 16, seed=72)
    G = S.load_csr(g)
    if mode == S.MODE_STITCHED:
        S.simrank_build_index(G, seg_log2=3, kappa=1.0, c=0.6, seed=ISEED)
    srcs = [int(x) for x in inputs.sources_with_in_edges(g, nq, 74)]
    qs = [S.make_query(s, c=0.6, eps=0.02, delta=1e-3, seed=0x2304040150000053, walk_cap=64,
                       mode=mode) for s in srcs]
    assert S.simrank_derive_params(qs[0], g.n).R == 9502
    plan = S.BatchPlan([G], qs)
    assert plan.n_groups == 1
    plan.run()
    st = plan.wait()
    _say(f"group of {nq} at full size: {st.ms:.1f} ms, {st.moves} moves")
    for i, q in enumerate(qs):
        assert np.array_equal(plan.read(i, want_out=False)[1], S.simrank_single_source_ex(G, q)[1]), i
    plan.free()


def test_group_of_32_medium_workload_vs_oracle():
    """32 queries of the medium workload's shape on its own graph (R-MAT
    n = 2^20, eps 0.02, R = 9,502, cap 64) with one seed form one query group;
    every member's counts on 512 random nodes with in-edges and the 32 highest
    in-degree nodes equal the oracle's for its source (run over host
    threads), and its estimate is count / R."""
    cfg = inputs.C2
    g = inputs.workload_graph(cfg)
    G = S.load_csr(g)
    srcs = [int(x) for x in inputs.sources_with_in_edges(g, 32, 76)]
    qs = [S.make_query(s, c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"], seed=cfg["walk_seed"],
                       walk_cap=cfg["L"]) for s in srcs]
    plan = S.BatchPlan([G], qs)
    assert plan.n_groups == 1
    plan.run()
    st = plan.wait()
    _say(f"group of 32 on the medium graph: {st.ms:.1f} ms, {st.moves} moves")
    smp0 = OT.sample_nodes(g, 512, 32, 0, seed=77)
    for i, s in enumerate(srcs):
        out, cnt = plan.read(i)
        smp = np.union1d(smp0, [s]).astype(np.int32)
        want = OT.meet_counts_plain(g, s, cfg["walk_seed"], cfg["c"], cfg["L"], 9502, smp)
        assert np.array_equal(cnt[smp], want), i
        assert np.array_equal(out[smp], np.where(smp == s, 1.0, want / 9502.0)), i
    plan.free()
    G.free()


def test_batching_workload_graphs_vs_oracle():
    """Four graphs of the batching workload (R-MAT, n from 6,544 to 573,161,
    average in-degree 13 to 27) with a query at each of its eps levels (0.05,
    0.02, 0.01: R = 1,521, 9,502, 38,005; a seed per query) in one captured
    plan: every query's counts on 256 random nodes with in-edges, the 16
    highest in-degree nodes, 4 nodes without in-edges and its source equal the
    oracle's, and its estimate is count / R."""
    specs = inputs.batch_graph_specs()
    cfg = inputs.C4
    picks = (1, 9, 0, 2)
    gs = [inputs.batch_graph(specs[i]) for i in picks]
    Gs = [S.load_csr(g) for g in gs]
    rng = np.random.default_rng(88)
    qs = []
    for gi, g in enumerate(gs):
        act = np.nonzero(g.in_degree() > 0)[0]
        for k, eps in enumerate(cfg["eps_choices"]):
            qs.append(S.make_query(int(rng.choice(act)), c=cfg["c"], eps=eps, delta=cfg["delta"],
                                   seed=0x6B00 + 3 * gi + k, walk_cap=cfg["L"], graph=gi))
    plan = S.BatchPlan(Gs, qs)
    plan.run()
    st = plan.wait()
    _say(f"batching-workload graphs, 12 queries: {st.ms:.1f} ms, {st.moves} moves")
    for i, q in enumerate(qs):
        g = gs[q.graph]
        R = S.simrank_derive_params(q, g.n).R
        out, cnt = plan.read(i)
        smp = np.union1d(OT.sample_nodes(g, 256, 16, 4, seed=89 + i), [q.s]).astype(np.int32)
        want = OT.meet_counts_plain(g, q.s, q.seed, cfg["c"], cfg["L"], R, smp)
        assert np.array_equal(cnt[smp], want), i
        assert np.array_equal(out[smp], np.where(smp == q.s, 1.0, want / float(R))), i
    assert sorted({S.simrank_derive_params(q, 10).R for q in qs}) == [1521, 9502, 38005]
    plan.free()
    for G in Gs:
        G.free()


def test_tile_and_unit_settings_keep_results(graphs):
    """Walks per tile and nodes per unit, set by hand or by the tuner, change
    the work's partition only: plain, stitched and stratified counts, alone and
    in a batch, stay equal to the default tuning's, bit for bit."""
    gs, Gs = graphs
    g, G = gs[1], Gs[1]                  # has an index
    s = int(np.argmax(g.in_degree()))
    qp = S.make_query(s, c=0.6, seed=91, walk_cap=64, R=9000)
    qs_ = S.make_query(s, c=0.6, seed=92, walk_cap=64, R=5000, mode=S.MODE_STITCHED)
    qr = S.make_stratified_query(s, c=0.6, eps=0.1, seed=93, z=3000, phi=12)
    S.simrank_set_tuning(G, 0, 0)
    want_p = S.simrank_single_source_ex(G, qp)[1]
    want_s = S.simrank_single_source_ex(G, qs_)[1]
    want_r = S.simrank_single_source_stratified(G, qr)[2]
    for vb, tj in ((32, 2048), (256, 4096), (64, 8192), (128, 6000)):
        S.simrank_set_tuning(G, vb, tj)
        assert np.array_equal(S.simrank_single_source_ex(G, qp)[1], want_p), (vb, tj)
        assert np.array_equal(S.simrank_single_source_ex(G, qs_)[1], want_s), (vb, tj)
        assert np.array_equal(S.simrank_single_source_stratified(G, qr)[2], want_r), (vb, tj)
        plan = S.BatchPlan([G], [S.make_query(s, c=0.6, seed=91, walk_cap=64, R=9000, graph=0)])
        plan.run()
        plan.wait()
        assert np.array_equal(plan.read(0, want_out=False)[1], want_p), (vb, tj)
        plan.free()
    t = S.simrank_tune_ex(G, qp)
    _say(f"tuner: {t}")
    assert t["unit_nodes"] in (32, 64, 128, 256) and t["tile_walks"] in (2048, 4096, 8192)
    assert np.array_equal(S.simrank_single_source_ex(G, qp)[1], want_p)
    for bad in ((-1, 0), (257, 0), (0, 1024), (0, 16384)):
        with pytest.raises(S.SimRankError):
            S.simrank_set_tuning(G, *bad)
    S.simrank_set_tuning(G, 0, 0)


def test_stratified_groups_equal_lone(graphs):
    """Stratified queries with one seed, z and phi form groups that walk each
    (v, j) once (walk j of v: slot pi_v(j), its class, its steps); every
    member's weighted sums, and both estimates, equal its lone run's, bit for
    bit; queries with another z or seed stay in groups of their own."""
    gs, Gs = graphs
    g, G = gs[2], Gs[2]
    rng = np.random.default_rng(17)
    act = np.nonzero(g.in_degree() > 0)[0]
    S1, S2 = 0x2304040150000061, 0x2304040150000062
    srcs = [int(x) for x in rng.choice(act, 14, replace=False)]
    qs = [S.make_stratified_query(s, c=0.6, eps=0.1, seed=S1, z=2500, phi=12, graph=2)
          for s in srcs[:11]]
    qs += [S.make_stratified_query(s, c=0.6, eps=0.1, seed=S1, z=900, phi=12, graph=2)
           for s in srcs[11:14]]
    qs += [S.make_stratified_query(s, c=0.6, eps=0.1, seed=S2, z=2500, phi=12, graph=2)
           for s in srcs[:2]]
    qs += [S.make_query(srcs[0], c=0.6, seed=S1, walk_cap=12, R=1000, graph=2)]   # plain, alone
    plan = S.BatchPlan(Gs, qs)
    assert plan.n_groups == 3          # 11, 3, 2
    plan.run()
    st = plan.wait()
    flat = S.BatchPlan(Gs, qs, groups=False)
    flat.run()
    fst = flat.wait()
    _say(f"stratified groups: {st.moves} moves vs {fst.moves} ungrouped")
    for i, q in enumerate(qs):
        if q.mode != S.MODE_STRATIFIED:
            continue
        o1, on1, w1, _ = S.simrank_single_source_stratified(G, q)
        o, on, w = plan.read_stratified(i)
        assert np.array_equal(w, w1) and np.array_equal(o, o1) and np.array_equal(on, on1), i
        assert np.array_equal(flat.read_stratified(i)[2], w1), i
        with pytest.raises(S.SimRankError):
            plan.read(i, want_out=False, want_counts=True)
    assert st.meets == fst.meets and st.moves < fst.moves
    P = O.strat_params(g.n, 0.6, 0.1, z=900.0, phi=12)
    assert np.array_equal(plan.read_stratified(11)[2], O.strat_sums(g, srcs[11], S1, P))
    plan.free()
    flat.free()


@pytest.mark.parametrize("nq", [8, 13])
def test_stratified_group_full_size(nq):
    """Stratified queries with Algorithm 2's z and Algorithm 1's cap on a
    2^16-node R-MAT graph (N = 14,825, phi = 43) and one seed: one group of 8
    and one of 13 (the instance for more than 8 members, its 64-bit sums in LDS
    for 256 nodes per unit), each member's weighted sums equal to its lone
    run's."""
    g = inputs.rmat_in(16, 16 << 16, seed=72)
    G = S.load_csr(g)
    srcs = [int(x) for x in inputs.sources_with_in_edges(g, nq, 75)]
    qs = [S.make_stratified_query(s, c=0.6, eps=0.02, seed=0x2304040150000063) for s in srcs]
    plan = S.BatchPlan([G], qs)
    assert plan.n_groups == 1
    plan.run()
    st = plan.wait()
    _say(f"stratified group of {nq} at full size: {st.ms:.1f} ms, {st.moves} moves")
    for i, q in enumerate(qs):
        assert np.array_equal(plan.read_stratified(i)[2],
                              S.simrank_single_source_stratified(G, q)[2]), i
    plan.free()


def test_group_edge_cases():
    """Groups at the edges: walk cap 1, R = 1, every member with the same
    source, a member whose source has no in-edges (no entries of its own),
    a star graph, and stitched groups on indexes with 1-step and 64-step
    segments; every count equals the lone query's."""
    g = inputs.from_edges(6, [0, 0, 0, 0, 1, 2, 3], [1, 2, 3, 4, 0, 0, 5])
    G = S.load_csr(g)
    no_in = int(np.argmax(g.in_degree() == 0))
    cases = [
        [S.make_query(s, c=0.6, seed=0xE1, walk_cap=1, R=R) for s, R in ((0, 1), (1, 2), (5, 5))],
        [S.make_query(1, c=0.6, seed=0xE2, walk_cap=8, R=R) for R in (40, 41, 7)],   # one source
        [S.make_query(s, c=0.6, seed=0xE3, walk_cap=64, R=300) for s in (no_in, 0, 1)],
    ]
    for qs in cases:
        plan = S.BatchPlan([G], qs)
        assert plan.n_groups == 1
        plan.run()
        plan.wait()
        for i, q in enumerate(qs):
            assert np.array_equal(plan.read(i)[1], S.simrank_single_source_ex(G, q)[1]), (i, q.s)
        plan.free()
    g2 = inputs.rmat_in(10, 8 << 10, seed=83)
    G2 = S.load_csr(g2)
    srcs = [int(x) for x in inputs.sources_with_in_edges(g2, 5, 84)]
    for k in (0, 6):
        S.simrank_build_index(G2, seg_log2=k, kappa=1.0, c=0.6, seed=ISEED)
        qs = [S.make_query(s, c=0.6, seed=0xE4, walk_cap=64, R=700, mode=S.MODE_STITCHED)
              for s in srcs]
        plan = S.BatchPlan([G2], qs)
        assert plan.n_groups == 1
        plan.run()
        plan.wait()
        for i, q in enumerate(qs):
            assert np.array_equal(plan.read(i)[1], S.simrank_single_source_ex(G2, q)[1]), (k, i)
        plan.free()


def test_plan_refuses_units_beyond_32_bits():
    """A kind's work units are numbered in 32 bits across all queries of a
    plan: 18 queries with R = 2^24 on a 2^20-node ring (each alone below 2^31
    units, together about 4.5e9) are refused with EINVAL before anything is
    allocated or launched."""
    n = 1 << 20
    src = np.arange(n, dtype=np.int64)
    g = inputs.from_edges(n, src, (src + 1) % n)
    G = S.load_csr(g)
    qs = [S.make_query(i, c=0.6, seed=0xF00 + i, walk_cap=64, R=1 << 24) for i in range(18)]
    with pytest.raises(S.SimRankError) as e:
        S.BatchPlan([G], qs, groups=False)
    assert e.value.code == S.SIMRANK_EINVAL and "2^32" in str(e.value)
    G.free()
