"""The serving loop: requests admitted into slots as they free up, running
concurrently; each result must equal the lone query's bit for bit."""
import time

import numpy as np
import pytest

import oracle as O
import oracle_threads as OT
from paper_2304_04015_amd import inputs
from paper_2304_04015_amd import simrank as S

pytestmark = pytest.mark.gpu

ISEED = 0x2304040150000013


@pytest.fixture(scope="module")
def served():
    g = inputs.rmat_in(14, 16 << 14, seed=41)
    G = S.load_csr(g)
    S.simrank_build_index(G, seg_log2=3, kappa=1.0, c=0.6, seed=ISEED)
    return g, G


def _requests(g, k, seed):
    rng = np.random.default_rng(seed)
    deg = g.in_degree().astype(np.float64)
    qs = []
    for i in range(k):
        s = int(rng.choice(g.n, p=deg / deg.sum()))
        eps = float(rng.choice([0.05, 0.02]))
        mode = S.MODE_STITCHED if i % 7 == 3 else S.MODE_PLAIN
        qs.append(S.make_query(s, c=0.6, eps=eps, delta=1e-3, seed=0x5E12 + i, mode=mode))
    return qs


def test_results_in_the_mix_equal_lone(served):
    g, G = served
    qs = _requests(g, 30, 1)
    lone = [S.simrank_single_source_ex(G, q) for q in qs]
    srv = S.Server(G, max_slots=4, max_R=9502, max_L=64)
    assert srv.info()["slots"] == 4
    tickets = []
    for i, q in enumerate(qs):
        tickets.append(srv.submit(q))
        if i % 5 == 4:
            time.sleep(0.002)          # arrivals while earlier requests run
    for t, (o1, c1, _) in zip(tickets, lone):
        o, c, info = srv.wait(t)
        assert np.array_equal(c, c1)
        assert np.array_equal(o, o1)
        assert info.latency_s >= info.queue_s >= 0.0
        assert info.stats.moves > 0 or c1.sum() == info.stats.R
    srv.destroy()


@pytest.mark.parametrize("group_max", [0, 8])
def test_served_results_equal_oracle(served, group_max):
    """Plain and stitched requests served alone (a seed per request) and in
    query groups (requests sharing a seed): every served count vector equals
    the oracle's for all 16,384 nodes (the Monte Carlo estimator of Section
    2.2 with the pairing of Section 3.2; stitched walks by serial traversal of
    the segment chain), and each estimate is count / R."""
    g, G = served
    rng = np.random.default_rng(40 + group_max)
    act = np.nonzero(g.in_degree() > 0)[0]
    srcs = [int(x) for x in rng.choice(act, 6, replace=False)]
    shared = group_max > 0
    qs = []
    for i, s in enumerate(srcs):
        mode = S.MODE_STITCHED if i >= 4 else S.MODE_PLAIN
        seed = (0x5EB0 + (i >= 4)) if shared else 0x5EC0 + i
        qs.append(S.make_query(s, c=0.6, eps=0.05, delta=1e-3, seed=seed, mode=mode))
    srv = S.Server(G, max_slots=6, max_R=9502, max_L=64, group_max=group_max)
    tickets = [srv.submit(q) for q in qs]
    P = O.pool_sizes(g, 1.0)
    allv = np.arange(g.n, dtype=np.int32)
    for t, q in zip(tickets, qs):
        o, c, info = srv.wait(t)
        R = info.stats.R
        assert R == 1521
        if q.mode == S.MODE_STITCHED:
            want = OT.meet_counts_stitched(g, q.s, q.seed, ISEED, 0.6, 64, 8, P, R, allv)
        else:
            want = OT.meet_counts_plain(g, q.s, q.seed, 0.6, 64, R, allv)
        assert np.array_equal(c, want), (q.s, q.mode)
        assert np.array_equal(o, np.where(allv == q.s, 1.0, want / float(R)))
    k = srv.counts()
    assert k["done"] == len(qs) and k["failed"] == 0
    if shared:
        assert k["grouped"] >= 2
    srv.destroy()


def test_budget_limits_slots(served):
    g, G = served
    probe = S.Server(G, max_slots=1, max_R=1521, max_L=64)
    per = probe.info()["slot_bytes"]
    probe.destroy()
    srv = S.Server(G, max_slots=8, max_R=1521, max_L=64, hbm_budget=int(2.5 * per))
    assert srv.info()["slots"] == 2
    qs = [S.make_query(q.s, c=0.6, eps=0.05, seed=q.seed, mode=q.mode) for q in _requests(g, 6, 2)]
    ts = [srv.submit(q) for q in qs]
    for t, q in zip(ts, qs):
        _, c, _ = srv.wait(t)
        assert np.array_equal(c, S.simrank_single_source_ex(G, q)[1])
    srv.destroy()
    with pytest.raises(S.SimRankError) as e:
        S.Server(G, max_slots=2, max_R=1521, max_L=64, hbm_budget=per // 2)
    assert e.value.code == S.SIMRANK_ENOMEM


def test_rejects(served):
    g, G = served
    srv = S.Server(G, max_slots=1, max_R=1521, max_L=64)
    with pytest.raises(S.SimRankError):
        srv.submit(S.make_query(0, eps=0.02))            # R = 9502 > the slots' 1521
    with pytest.raises(S.SimRankError):
        srv.submit(S.make_query(g.n, eps=0.05))          # source out of range
    with pytest.raises(S.SimRankError):
        srv.wait(123456)
    srv.destroy()


def test_grouped_admission_equals_lone(served):
    """group_max = 8 with 8 slots: requests with one seed (plain, and stitched)
    that wait together are admitted as query groups; requests with other seeds
    and a lone stitched request run alone between them.  Every result equals
    the lone query's, bit for bit."""
    g, G = served
    rng = np.random.default_rng(3)
    deg = g.in_degree().astype(np.float64)
    qs = []
    for i in range(40):
        s = int(rng.choice(g.n, p=deg / deg.sum()))
        eps = float(rng.choice([0.05, 0.02]))
        if i % 10 == 9:
            q = S.make_query(s, c=0.6, eps=eps, delta=1e-3, seed=0x5E99 + i)          # own seed
        elif i % 4 == 1:
            q = S.make_query(s, c=0.6, eps=eps, delta=1e-3, seed=0x5E77, mode=S.MODE_STITCHED)
        else:
            q = S.make_query(s, c=0.6, eps=eps, delta=1e-3, seed=0x5E77)
        qs.append(q)
    lone = [S.simrank_single_source_ex(G, q) for q in qs]
    srv = S.Server(G, max_slots=8, max_R=9502, max_L=64, group_max=8)
    tickets = [srv.submit(q) for q in qs]          # all arrive while the first ones run
    for i, (t, (o1, c1, _)) in enumerate(zip(tickets, lone)):
        o, c, info = srv.wait(t)
        assert np.array_equal(c, c1), i
        assert np.array_equal(o, o1), i
        assert info.latency_s >= info.queue_s >= 0.0
    k = srv.counts()
    assert k["done"] == len(qs) and k["failed"] == 0
    assert k["groups"] >= 2 and k["grouped"] >= 2 * k["groups"]
    srv.destroy()
    with pytest.raises(S.SimRankError):
        S.Server(G, max_slots=2, group_max=33)


def test_arrivals_during_a_run_gather_into_a_group(served):
    """A grouping server: one request starts alone; eight more with the same
    walks arrive while it runs, wait for it, and start together as one group.
    Every result equals the lone query's."""
    g, G = served
    rng = np.random.default_rng(29)
    act = np.nonzero(g.in_degree() > 0)[0]
    qs = [S.make_query(int(rng.choice(act)), c=0.6, eps=0.02 if i == 0 else 0.05, delta=1e-3,
                       seed=0x5EC0) for i in range(9)]
    lone = [S.simrank_single_source_ex(G, q)[1] for q in qs]
    srv = S.Server(G, max_slots=8, max_R=9502, max_L=64, group_max=8)
    tickets = [srv.submit(q) for q in qs]
    for t, c1 in zip(tickets, lone):
        _, c, _ = srv.wait(t, timeout_s=120.0, want_out=False)
        assert np.array_equal(c, c1)
    k = srv.counts()
    assert k["done"] == 9 and k["failed"] == 0
    assert k["groups"] >= 1 and k["grouped"] >= 8, k
    srv.destroy()


def test_concurrent_submitters_with_groups(served):
    """Four client threads submit and wait at once (plain and stitched requests,
    two seeds) into a grouping server: every result equals the lone query's."""
    import threading
    g, G = served
    rng = np.random.default_rng(23)
    deg = g.in_degree().astype(np.float64)
    per_thread = []
    for t in range(4):
        qs = []
        for i in range(8):
            s = int(rng.choice(g.n, p=deg / deg.sum()))
            mode = S.MODE_STITCHED if (t + i) % 3 == 0 else S.MODE_PLAIN
            qs.append(S.make_query(s, c=0.6, eps=0.05, delta=1e-3, seed=0x5EA0 + (i % 2), mode=mode))
        per_thread.append(qs)
    lone = [[S.simrank_single_source_ex(G, q)[1] for q in qs] for qs in per_thread]
    srv = S.Server(G, max_slots=8, max_R=9502, max_L=64, group_max=8)
    errors = []

    def client(t):
        try:
            tickets = [srv.submit(q) for q in per_thread[t]]
            for k, tk in enumerate(tickets):
                _, c, _ = srv.wait(tk, want_out=False)
                if not np.array_equal(c, lone[t][k]):
                    errors.append((t, k))
        except Exception as e:   # reported below
            errors.append((t, repr(e)))

    threads = [threading.Thread(target=client, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads)
    assert not errors, errors
    k = srv.counts()
    assert k["done"] == 32 and k["failed"] == 0
    srv.destroy()


def test_destroy_finishes_requests_in_flight(served):
    """Destroying a server with requests still queued and running drains them
    and returns; the graph then answers queries as before."""
    g, G = served
    qs = _requests(g, 6, 77)
    srv = S.Server(G, max_slots=2, max_R=9502, max_L=64)
    for q in qs:
        srv.submit(q)
    srv.destroy()
    q = qs[0]
    a = S.simrank_single_source_ex(G, q)[1]
    b = S.simrank_single_source_ex(G, q)[1]
    assert np.array_equal(a, b)


def test_serving_workload_size_vs_oracle():
    """The serving workload's graph (R-MAT n = 2^22, average in-degree 16)
    with its stitched index (2^4-step segments, kappa = 1): a plain request at
    eps 0.02 (R = 9,502) and a stitched request at eps 0.05 (R = 1,521) served
    together; their counts on 512 random nodes with in-edges, the 32 highest
    in-degree nodes, 8 nodes without in-edges and the sources equal the
    oracle's (plain walks, and stitched walks traversed serially over segments
    regenerated from the CSR), and each estimate is count / R."""
    cfg = inputs.C5
    g = inputs.workload_graph(cfg)
    G = S.load_csr(g)
    iseed = 0x2304040150000023
    S.simrank_build_index(G, seg_log2=4, kappa=1.0, c=cfg["c"], seed=iseed)
    srcs = [int(x) for x in inputs.sources_by_degree(g, 2, 81)]
    qp = S.make_query(srcs[0], c=cfg["c"], eps=0.02, delta=cfg["delta"], seed=0x5F10,
                      walk_cap=cfg["L"])
    qs = S.make_query(srcs[1], c=cfg["c"], eps=0.05, delta=cfg["delta"], seed=0x5F11,
                      walk_cap=cfg["L"], mode=S.MODE_STITCHED)
    srv = S.Server(G, max_slots=4, max_R=9502, max_L=64)
    tp, ts = srv.submit(qp), srv.submit(qs)
    op, cp, _ = srv.wait(tp, timeout_s=120.0)
    os_, cs, _ = srv.wait(ts, timeout_s=120.0)
    srv.destroy()
    smp0 = OT.sample_nodes(g, 512, 32, 8, seed=82)
    P = O.pool_sizes(g, 1.0)
    Rp, Rs = S.simrank_derive_params(qp, g.n).R, S.simrank_derive_params(qs, g.n).R
    assert (Rp, Rs) == (9502, 1521)
    for q, o, c, R in ((qp, op, cp, Rp), (qs, os_, cs, Rs)):
        smp = np.union1d(smp0, [q.s]).astype(np.int32)
        if q.mode == S.MODE_STITCHED:
            want = OT.meet_counts_stitched(g, q.s, q.seed, iseed, cfg["c"], cfg["L"], 16, P, R, smp)
        else:
            want = OT.meet_counts_plain(g, q.s, q.seed, cfg["c"], cfg["L"], R, smp)
        assert np.array_equal(c[smp], want), q.mode
        assert np.array_equal(o[smp], np.where(smp == q.s, 1.0, want / float(R))), q.mode
    G.free()


def test_two_waits_on_one_ticket(served):
    """Two threads wait on the same ticket: one receives the result (equal to
    the lone query's), the other an EINVAL for the retired ticket."""
    import threading
    g, G = served
    q = _requests(g, 1, 5)[0]
    lone = S.simrank_single_source_ex(G, q)[1]
    srv = S.Server(G, max_slots=2, max_R=9502, max_L=64)
    tk = srv.submit(q)
    got, errs = [], []

    def waiter():
        try:
            got.append(srv.wait(tk, want_out=False)[1])
        except S.SimRankError as e:
            errs.append(e.code)

    threads = [threading.Thread(target=waiter) for _ in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not any(th.is_alive() for th in threads)
    assert len(got) == 1 and len(errs) == 1
    assert np.array_equal(got[0], lone)
    assert errs[0] == S.SIMRANK_EINVAL
    srv.destroy()


def test_stratified_and_mixed_requests(served):
    """Plain, stitched and stratified requests (Algorithms 1-2 at a small z)
    in one stream of arrivals: each served result equals the lone call's bit
    for bit, the stratified ones also the oracle's weighted sums; a
    stratified ticket is refused by the counts wait and a plain one by the
    stratified wait, without retiring either."""
    g, G = served
    rng = np.random.default_rng(51)
    act = np.nonzero(g.in_degree() > 0)[0]
    qs = []
    for i in range(12):
        s = int(rng.choice(act))
        if i % 3 == 0:
            qs.append(S.make_stratified_query(s, c=0.6, eps=0.05, seed=0x5F00 + i, z=1200, phi=12))
        else:
            mode = S.MODE_STITCHED if i % 3 == 1 else S.MODE_PLAIN
            qs.append(S.make_query(s, c=0.6, eps=0.05, delta=1e-3, seed=0x5F00 + i, mode=mode))
    srv = S.Server(G, max_slots=6, max_R=9502, max_L=64)
    tickets = []
    for i, q in enumerate(qs):
        tickets.append(srv.submit(q))
        if i % 4 == 3:
            time.sleep(0.003)
    for t, q in zip(tickets, qs):
        if q.mode == S.MODE_STRATIFIED:
            with pytest.raises(S.SimRankError):
                srv.wait(t)
            o, on, w, info = srv.wait_stratified(t)
            o1, on1, w1, _ = S.simrank_single_source_stratified(G, q)
            assert np.array_equal(w, w1) and np.array_equal(o, o1) and np.array_equal(on, on1)
            P = O.strat_params(g.n, 0.6, 0.05, z=1200.0, phi=12)
            assert np.array_equal(w, OT.strat_sums(g, q.s, q.seed, P, np.arange(g.n)))
        else:
            with pytest.raises(S.SimRankError):
                srv.wait_stratified(t)
            o, c, info = srv.wait(t)
            o1, c1, _ = S.simrank_single_source_ex(G, q)
            assert np.array_equal(c, c1) and np.array_equal(o, o1)
        assert info.latency_s >= info.queue_s >= 0.0
    k = srv.counts()
    assert k["done"] == len(qs) and k["failed"] == 0
    srv.destroy()


def test_stratified_requests_in_groups(served):
    """group_max = 16: stratified requests that share the seed, z and phi are
    admitted as query groups, which take walk j of v (its slot and class,
    Algorithms 1-2) once for all members; a group of more than 8 runs on the
    instance that keeps its 64-bit sums in LDS.  One request with another z
    and one with another seed run alone beside them.  Every member's weighted sums and both estimates
    equal its lone call's bit for bit, and one member's sums equal the
    oracle's."""
    g, G = served
    rng = np.random.default_rng(53)
    act = np.nonzero(g.in_degree() > 0)[0]
    srcs = [int(x) for x in rng.choice(act, 15, replace=False)]
    qs = [S.make_stratified_query(s, c=0.6, eps=0.05, seed=0x5F80, z=1200, phi=12) for s in srcs[:13]]
    qs.append(S.make_stratified_query(srcs[13], c=0.6, eps=0.05, seed=0x5F80, z=900, phi=12))
    qs.append(S.make_stratified_query(srcs[14], c=0.6, eps=0.05, seed=0x5F81, z=1200, phi=12))
    srv = S.Server(G, max_slots=16, max_R=9502, max_L=64, group_max=16)
    tickets = [srv.submit(q) for q in qs]
    ws = []
    for i, (t, q) in enumerate(zip(tickets, qs)):
        o, on, w, info = srv.wait_stratified(t, timeout_s=120.0)
        o1, on1, w1, _ = S.simrank_single_source_stratified(G, q)
        assert np.array_equal(w, w1) and np.array_equal(o, o1) and np.array_equal(on, on1), i
        ws.append(w)
    P = O.strat_params(g.n, 0.6, 0.05, z=1200.0, phi=12)
    assert np.array_equal(ws[3], OT.strat_sums(g, qs[3].s, qs[3].seed, P, np.arange(g.n)))
    k = srv.counts()
    assert k["done"] == len(qs) and k["failed"] == 0
    assert k["groups"] >= 1 and k["grouped"] >= 2 * k["groups"], k
    srv.destroy()


def test_arrivals_join_running_work(served):
    """Continuous batching: requests that arrive while others run are admitted
    at once (ring entries and memory are free) rather than after the running
    ones finish, several are in flight together, and each result equals the
    lone call's.  poll() reports a finished request as 2."""
    g, G = served
    rng = np.random.default_rng(61)
    act = np.nonzero(g.in_degree() > 0)[0]
    qs = [S.make_query(int(rng.choice(act)), c=0.6, eps=0.02, delta=1e-3, seed=0x6000 + i)
          for i in range(10)]
    lone = [S.simrank_single_source_ex(G, q)[1] for q in qs]
    srv = S.Server(G, max_slots=8, max_R=9502, max_L=64)
    tickets = [srv.submit(qs[0])]
    time.sleep(0.002)
    tickets += [srv.submit(q) for q in qs[1:]]
    infos = []
    for t, c1 in zip(tickets, lone):
        _, c, info = srv.wait(t, want_out=False)
        assert np.array_equal(c, c1)
        infos.append(info)
    ld = srv.load()
    assert ld["inflight_peak"] >= 2 and ld["launches"] >= 1
    assert ld["pool_peak"] <= ld["pool_bytes"]
    # the later arrivals were admitted while the first one still ran
    first_done = infos[0].latency_s
    assert min(i.queue_s for i in infos[1:]) < first_done
    t = srv.submit(qs[0])
    _, c, _ = srv.wait(t, want_out=False)
    with pytest.raises(S.SimRankError):
        srv.poll(t)                      # retired
    t2 = srv.submit(qs[1])
    while srv.poll(t2) != 2:
        time.sleep(0.001)
    assert np.array_equal(srv.wait(t2, want_out=False)[1], lone[1])
    srv.destroy()


def test_memory_admission_per_request(served):
    """Admission by each request's own memory: a pool that holds one request
    of the server's largest R holds several small ones, which then run
    together; a request larger than the whole pool is refused at submit."""
    g, G = served
    probe = S.Server(G, max_slots=1, max_R=9502, max_L=64)
    big = probe.info()["slot_bytes"]
    probe.destroy()
    srv = S.Server(G, max_slots=8, max_R=9502, max_L=64, hbm_budget=int(1.2 * big))
    rng = np.random.default_rng(71)
    act = np.nonzero(g.in_degree() > 0)[0]
    small = [S.make_query(int(rng.choice(act)), c=0.6, eps=0.2, delta=1e-3, seed=0x6100 + i)
             for i in range(8)]             # R = 95
    tickets = [srv.submit(q) for q in small]
    for t, q in zip(tickets, small):
        assert np.array_equal(srv.wait(t, want_out=False)[1], S.simrank_single_source_ex(G, q)[1])
    assert srv.load()["inflight_peak"] >= 2
    tb = srv.submit(S.make_query(int(act[0]), c=0.6, eps=0.02, seed=0x6200))   # fits alone
    assert srv.wait(tb, want_out=False)[1][int(act[0])] == 9502
    srv.destroy()
    # a stratified request of nearly the largest N and cap 64 needs more than
    # a plain request of the largest R: beyond a pool of exactly that size
    srv = S.Server(G, max_slots=2, max_R=9502, max_L=64, hbm_budget=big)
    qz = S.make_stratified_query(int(act[0]), c=0.6, eps=0.05, seed=0x6300, z=9400, phi=64)
    assert S.simrank_derive_stratified(qz, g.n).N <= 9502
    with pytest.raises(S.SimRankError) as e:
        srv.submit(qz)
    assert e.value.code == S.SIMRANK_ENOMEM
    srv.destroy()


def test_groups_in_a_pool_for_one_request(served):
    """Group admission with a pool that holds one request of the largest R:
    same-walk requests cannot start together, so they run one after another
    instead of waiting for a group (each wait has a time limit), and each
    equals its lone call."""
    g, G = served
    probe = S.Server(G, max_slots=1, max_R=9502, max_L=64)
    big = probe.info()["slot_bytes"]
    probe.destroy()
    srv = S.Server(G, max_slots=4, max_R=9502, max_L=64, hbm_budget=big, group_max=8)
    act = np.nonzero(g.in_degree() > 0)[0]
    qs = [S.make_query(int(act[i]), c=0.6, eps=0.02, seed=0x6400) for i in range(3)]
    tickets = [srv.submit(q) for q in qs]
    for t, q in zip(tickets, qs):
        assert np.array_equal(srv.wait(t, timeout_s=120.0, want_out=False)[1],
                              S.simrank_single_source_ex(G, q)[1])
    assert srv.counts()["groups"] == 0 and srv.load()["inflight_peak"] == 1
    srv.destroy()


def test_entry_reuse_with_other_sizes(served):
    """Ring entries reused many times by requests of other sizes and kinds
    (plain and stitched with R = 1521 or 9502, stratified with N = 1,150;
    two entries): every request completes (waits with a time limit) and
    equals the lone call.  A block that took units of a reused entry under
    the previous request's tag, or with the previous request's kind, would
    leave the new request's completion count off by its units (never
    finishing) or add counts walked with the wrong kernel."""
    g, G = served
    rng = np.random.default_rng(81)
    act = np.nonzero(g.in_degree() > 0)[0]
    qs = []
    for i in range(36):
        s = int(rng.choice(act))
        if i % 4 == 3:
            qs.append(S.make_stratified_query(s, c=0.6, eps=0.05, seed=0x6400 + i, z=1200, phi=12))
        else:
            qs.append(S.make_query(s, c=0.6, eps=(0.05, 0.02)[i % 2], delta=1e-3, seed=0x6400 + i,
                                   mode=S.MODE_STITCHED if i % 3 == 2 else S.MODE_PLAIN))
    lone = [S.simrank_single_source_stratified(G, q)[2] if q.mode == S.MODE_STRATIFIED
            else S.simrank_single_source_ex(G, q)[1] for q in qs]
    srv = S.Server(G, max_slots=2, max_R=9502, max_L=64)
    for burst in range(3):
        chunk = list(range(burst * 12, burst * 12 + 12))
        tickets = [srv.submit(qs[i]) for i in chunk]
        for t, i in zip(tickets, chunk):
            if qs[i].mode == S.MODE_STRATIFIED:
                got = srv.wait_stratified(t, timeout_s=120.0)[2]
            else:
                got = srv.wait(t, timeout_s=120.0, want_out=False)[1]
            assert np.array_equal(got, lone[i]), i
    srv.destroy()
