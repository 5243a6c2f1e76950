"""GPU parity of the stitched-walk index and stitched queries against the
CPU oracle's serial traversal (segments regenerated from the CSR under the
same Philox keys)."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle_threads as OT
from paper_2304_04015_amd import inputs
from paper_2304_04015_amd import simrank as S

pytestmark = pytest.mark.gpu

SEED = 0x2304040150000003
ISEED = 0x2304040150000013


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small():
    g = inputs.rmat_in(11, 12 << 11, seed=7)
    return g


@pytest.mark.parametrize("k,kappa", [(3, 1.0), (2, 0.5), (4, 2.5), (1, 1.0)])
def test_index_entries_match_oracle(small, k, kappa):
    g = small
    G = S.load_csr(g)
    info = S.simrank_build_index(G, seg_log2=k, kappa=kappa, c=0.6, seed=ISEED)
    P = O.pool_sizes(g, kappa)
    assert info["segments"] == int(P.sum())
    assert info["levels"] == int(np.log2(64 >> k))
    pool_off = np.concatenate([[0], np.cumsum(P)])
    owner = np.repeat(np.arange(g.n), P)
    rng = np.random.default_rng(k)
    sig = np.unique(np.concatenate([np.arange(min(600, P.sum())),
                                    rng.integers(0, P.sum(), 2000)])).astype(np.int64)
    nodes, lens, succ, chain = S.simrank_index_read(G, sig)
    seglen = 1 << k
    T = O.continue_threshold(0.6)
    for r, s in enumerate(sig):
        y = int(owner[s])
        i = int(s - pool_off[y])
        want = O.segment(g, ISEED, 0.6, seglen, y, i)
        assert lens[r] == want.size
        assert np.array_equal(nodes[r, : want.size], want)
        assert np.all(nodes[r, want.size:] == -1)
        if want.size == seglen:
            x = O.philox([y, i, 0, 3], [ISEED & 0xffffffff, ISEED >> 32])
            z = int(want[-1])
            assert succ[r] == pool_off[z] + ((int(x[0]) * int(P[z])) >> 32)
        else:
            assert succ[r] == -1
    # chain[s] = (s, succ(s), succ^2(s), ...) from the doubling rounds
    all_sig = np.arange(P.sum(), dtype=np.int64)
    _, _, succ_all, _ = S.simrank_index_read(G, all_sig, with_chain=False)
    for r, s in enumerate(sig[:500]):
        cur = int(s)
        for m in range(chain.shape[1]):
            assert chain[r, m] == cur
            cur = int(succ_all[cur]) if cur >= 0 else -1
    assert T > 0


@pytest.mark.parametrize("k", [3, 2])
def test_stitched_walks_bit_exact(small, k):
    g = small
    G = S.load_csr(g)
    S.simrank_build_index(G, seg_log2=k, kappa=1.0, c=0.6, seed=ISEED)
    P = O.pool_sizes(g, 1.0)
    rng = np.random.default_rng(3)
    vs = rng.integers(0, g.n, 20000).astype(np.int32)
    js = rng.integers(0, 50000, 20000).astype(np.uint32)
    q = S.make_query(0, c=0.6, seed=SEED, walk_cap=64, mode=S.MODE_STITCHED)
    paths, lens = S.simrank_walks(G, q, vs, js)
    opaths, olens = O.walk_table_stitched(g, SEED, ISEED, 0.6, 64, 1 << k, P, vs, js)
    assert np.array_equal(lens, olens)
    assert np.array_equal(paths, opaths)
    assert (lens > (1 << k)).sum() > 100          # the tails were exercised
    # heads equal the plain walks' prefixes
    qp = S.make_query(0, c=0.6, seed=SEED, walk_cap=64)
    ppaths, plens = S.simrank_walks(G, qp, vs, js)
    h = 1 << k
    head = np.minimum(plens, h)
    for r in range(0, vs.size, 97):
        assert np.array_equal(paths[r, : head[r] + 1], ppaths[r, : head[r] + 1])


def test_stitched_counts_bit_exact(small):
    g = small
    G = S.load_csr(g)
    S.simrank_build_index(G, seg_log2=3, kappa=1.0, c=0.6, seed=ISEED)
    P = O.pool_sizes(g, 1.0)
    deg = g.in_degree()
    s = int(np.argsort(deg)[-3])
    for c_, L in ((0.6, 64), ):
        q = S.make_query(s, c=c_, seed=SEED, walk_cap=L, R=3000, mode=S.MODE_STITCHED)
        out, cnt, st = S.simrank_single_source_ex(G, q)
        want = O.meet_counts_stitched(g, s, SEED, ISEED, c_, L, 8, P, 3000)
        assert np.array_equal(cnt, want)
        _say(f"stitched: tail_steps={st.tail_steps} moves={st.moves}")


def test_stitched_long_walks_bit_exact():
    """c = 0.95 keeps most walks alive past the head, so tails carry the meets."""
    g = inputs.erdos_renyi_in(400, 4.0, seed=19)
    G = S.load_csr(g)
    S.simrank_build_index(G, seg_log2=3, kappa=1.0, c=0.95, seed=ISEED)
    P = O.pool_sizes(g, 1.0)
    q = S.make_query(5, c=0.95, seed=SEED, walk_cap=64, R=1500, mode=S.MODE_STITCHED)
    out, cnt, st = S.simrank_single_source_ex(G, q)
    want = O.meet_counts_stitched(g, 5, SEED, ISEED, 0.95, 64, 8, P, 1500)
    assert np.array_equal(cnt, want)
    assert st.tail_steps > 10000


def test_full_segment_reduces_to_plain(small):
    g = small
    G = S.load_csr(g)
    S.simrank_build_index(G, seg_log2=6, kappa=1.0, c=0.6, seed=ISEED)
    s = 11
    a = S.simrank_single_source_ex(G, S.make_query(s, seed=SEED, R=2000, mode=S.MODE_STITCHED))[1]
    b = S.simrank_single_source_ex(G, S.make_query(s, seed=SEED, R=2000))[1]
    assert np.array_equal(a, b)


def test_plan_refuses_a_rebuilt_index(small):
    """A plan's stitched queries hold the addresses of the index they were
    planned with: after a rebuild the plan refuses to run (ESTATE), a plan
    without stitched queries still runs, and a new plan gives the new index's
    counts."""
    g = small
    G = S.load_csr(g)
    S.simrank_build_index(G, seg_log2=3, kappa=1.0, c=0.6, seed=ISEED)
    qs = [S.make_query(s, seed=SEED, R=500, mode=S.MODE_STITCHED) for s in (3, 11)]
    plain = S.BatchPlan([G], [S.make_query(3, seed=SEED, R=500)])
    plan = S.BatchPlan([G], qs)
    plan.run()
    plan.wait()
    S.simrank_build_index(G, seg_log2=2, kappa=1.0, c=0.6, seed=ISEED)
    with pytest.raises(S.SimRankError) as e:
        plan.run()
    assert e.value.code == S.SIMRANK_ESTATE
    plain.run()
    plain.wait()
    fresh = S.BatchPlan([G], qs)
    fresh.run()
    fresh.wait()
    want = S.simrank_single_source_ex(G, qs[1])[1]
    assert np.array_equal(fresh.read(1, want_out=False)[1], want)


def test_stitched_requires_matching_index(small):
    G = S.load_csr(small)
    with pytest.raises(S.SimRankError) as e:
        S.simrank_single_source_ex(G, S.make_query(1, mode=S.MODE_STITCHED, R=10))
    assert e.value.code == S.SIMRANK_ESTATE
    S.simrank_build_index(G, seg_log2=3, c=0.5)
    with pytest.raises(S.SimRankError) as e:
        S.simrank_single_source_ex(G, S.make_query(1, c=0.6, mode=S.MODE_STITCHED, R=10))
    assert e.value.code == S.SIMRANK_EINVAL


def test_index_checkpoint_and_resume(small, tmp_path):
    """An index saved to a file and loaded into a fresh copy of the graph gives
    the same entries and the same stitched counts (equal to the oracle's);
    files for another graph, damaged, truncated or too long are refused with
    the graph's current index kept."""
    g = small
    G = S.load_csr(g)
    info = S.simrank_build_index(G, seg_log2=3, kappa=1.0, c=0.6, seed=ISEED)
    s = int(np.argsort(g.in_degree())[-5])
    q = S.make_query(s, seed=SEED, R=3000, mode=S.MODE_STITCHED)
    want = S.simrank_single_source_ex(G, q)[1]
    assert np.array_equal(want, O.meet_counts_stitched(g, s, SEED, ISEED, 0.6, 64, 8,
                                                       O.pool_sizes(g, 1.0), 3000))
    sig = np.arange(0, info["segments"], 37, dtype=np.int64)
    before = S.simrank_index_read(G, sig)
    path = tmp_path / "index.bin"
    S.simrank_index_save(G, str(path))
    G2 = S.load_csr(g)
    with pytest.raises(S.SimRankError) as e:
        S.simrank_index_save(G2, str(tmp_path / "none.bin"))
    assert e.value.code == S.SIMRANK_ESTATE
    S.simrank_index_load(G2, str(path))
    after = S.simrank_index_read(G2, sig)
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    info2 = S.simrank_index_info(G2)
    for key in ("segments", "levels", "bytes"):
        assert info2[key] == info[key], key
    assert np.array_equal(S.simrank_single_source_ex(G2, q)[1], want)

    data = path.read_bytes()
    damaged = bytearray(data)
    damaged[128 + (len(data) - 128) // 2] ^= 0x5A
    cases = {"damaged": bytes(damaged), "truncated": data[:-3], "too_long": data + b"\0"}
    for name, blob in cases.items():
        p = tmp_path / f"{name}.bin"
        p.write_bytes(blob)
        with pytest.raises(S.SimRankError) as e:
            S.simrank_index_load(G2, str(p))
        assert e.value.code == S.SIMRANK_EINVAL, name
    # the refused loads left the loaded index in place
    assert np.array_equal(S.simrank_single_source_ex(G2, q)[1], want)
    # same n and m, one edge moved: another graph
    src = g.in_src.copy()
    a = int(np.nonzero(np.diff(g.in_off) > 1)[0][0])
    row = src[g.in_off[a]:g.in_off[a + 1]]
    spare = int(next(u for u in range(g.n) if u not in set(row.tolist())))
    src[g.in_off[a]] = spare
    other = inputs.CSR(g.n, g.in_off.copy(), src, "one edge moved")
    G3 = S.load_csr(other)
    with pytest.raises(S.SimRankError) as e:
        S.simrank_index_load(G3, str(path))
    assert e.value.code == S.SIMRANK_EINVAL
    with pytest.raises(S.SimRankError) as e:
        S.simrank_index_load(G3, str(tmp_path / "missing.bin"))
    assert e.value.code == S.SIMRANK_EIO
    G3.free()
    G2.free()
    G.free()


@pytest.mark.slow
def test_c3_stitching_at_scale():
    """Stitching workload at full size: R-MAT n=2^24, avg degree 16 (~2.6e8
    edges), segment pools sized by in-degree (kappa=1, 2^3-step segments,
    3 doubling rounds), eps=0.02 -> R=9502, L=64.  Bit-exact against the
    oracle's direct generation (each segment regenerated from the CSR under the
    same Philox keys): the index size, 4096 sampled slots (segment, successor),
    all R source walks, 2^20 sampled stitched walks (v, j), and the stitched
    query's meet counts and estimates on 2,048 random nodes with in-edges, the
    64 highest in-degree nodes and 8 without in-edges (the oracle run over
    host threads)."""
    cfg = inputs.C3
    _say("generating the R-MAT scale-24 graph")
    g = inputs.workload_graph(cfg)
    _say(f"n={g.n} m={g.m}; loading")
    G = S.load_csr(g)
    k = cfg["seg_log2"]
    info = S.simrank_build_index(G, seg_log2=k, kappa=cfg["kappa"], c=cfg["c"],
                                 seed=cfg["index_seed"])
    _say(f"index: {info}")
    P = O.pool_sizes(g, cfg["kappa"])
    assert info["segments"] == int(P.sum()) and info["levels"] == 3
    pool_off = np.concatenate([[0], np.cumsum(P)])
    rng = np.random.default_rng(24)
    # sampled slots: segment nodes and successor slot
    sig = np.sort(rng.integers(0, int(P.sum()), 4096)).astype(np.int64)
    nodes, lens, succ, chain = S.simrank_index_read(G, sig)
    owner = np.searchsorted(pool_off, sig, side="right") - 1
    for r, s_ in enumerate(sig):
        y = int(owner[r])
        i = int(s_ - pool_off[y])
        want = O.segment(g, cfg["index_seed"], cfg["c"], 1 << k, y, i)
        assert lens[r] == want.size and np.array_equal(nodes[r, : want.size], want)
        if want.size == (1 << k):
            x = O.philox([y, i, 0, 3], [cfg["index_seed"] & 0xffffffff, cfg["index_seed"] >> 32])
            z = int(want[-1])
            assert succ[r] == pool_off[z] + ((int(x[0]) * int(P[z])) >> 32)
        else:
            assert succ[r] == -1
    s = int(inputs.sources_with_in_edges(g, 1, cfg["source_seed"])[0])
    q = S.make_query(s, c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"], seed=cfg["walk_seed"],
                     walk_cap=cfg["L"], mode=S.MODE_STITCHED)
    R = S.simrank_derive_params(q, g.n).R
    assert R == 9502
    act = np.nonzero(g.in_degree() > 0)[0]
    vs = np.concatenate([np.full(R, s), rng.choice(act, 1 << 20)]).astype(np.int32)
    js = np.concatenate([np.arange(R), rng.integers(0, R, 1 << 20)]).astype(np.uint32)
    _say("stitched walks on the GPU")
    paths, plens = S.simrank_walks(G, q, vs, js)
    _say("stitched walks in the oracle")
    opaths, olens = O.walk_table_stitched(g, cfg["walk_seed"], cfg["index_seed"], cfg["c"],
                                          cfg["L"], 1 << k, P, vs, js)
    assert np.array_equal(plens, olens)
    assert np.array_equal(paths, opaths)
    assert (plens > (1 << k)).sum() > 10000
    _say("stitched query")
    out, cnt, st = S.simrank_single_source_ex(G, q)
    smp = OT.sample_nodes(g, 2048, 64, 8, seed=25, extra=[s])
    _say(f"stitched counts in the oracle: {smp.size} nodes, {OT.host_threads()} threads")
    want = OT.meet_counts_stitched(g, s, cfg["walk_seed"], cfg["index_seed"], cfg["c"], cfg["L"],
                                   1 << k, P, R, smp)
    assert np.array_equal(cnt[smp], want)
    assert np.array_equal(out[smp], np.where(smp == s, 1.0, want / float(R)))
    _say(f"query: moves={st.moves} tail_steps={st.tail_steps} meet_ms={st.meet_ms:.1f}")


def test_index_tuner_picks_a_segment_length(small):
    """The segment-length tuner builds the index for k = 2, 3, 4, times a
    stitched query on each and leaves the fastest built; the query's counts on
    that index equal the oracle's for the chosen k."""
    g = small
    G = S.load_csr(g)
    s = int(np.argsort(g.in_degree())[-2])
    q = S.make_query(s, c=0.6, seed=SEED, walk_cap=64, R=2000, mode=S.MODE_STITCHED)
    choice, ms = S.simrank_tune_index(G, q, seg_log2=(2, 3, 4), kappa=1.0, c=0.6, seed=ISEED)
    _say(f"index tuner: {choice}, meet ms per k {ms}")
    k = choice["seg_log2"]
    assert k in (2, 3, 4) and len(ms) == 3 and all(x > 0 for x in ms)
    assert ms[(2, 3, 4).index(k)] == min(ms)
    assert S.simrank_index_info(G)["seg_log2"] == k
    cnt = S.simrank_single_source_ex(G, q)[1]
    want = O.meet_counts_stitched(g, s, SEED, ISEED, 0.6, 64, 1 << k, O.pool_sizes(g, 1.0), 2000)
    assert np.array_equal(cnt, want)
    with pytest.raises(S.SimRankError):   # plain query
        S.simrank_tune_index(G, S.make_query(s, seed=SEED, R=100), seg_log2=(3,), seed=ISEED)
    with pytest.raises(S.SimRankError):   # c differs from the index's
        S.simrank_tune_index(G, q, seg_log2=(3,), c=0.5, seed=ISEED)
    with pytest.raises(S.SimRankError):
        S.simrank_tune_index(G, q, seg_log2=(7,), seed=ISEED)
