"""GPU parity of the plain single-source path against the CPU oracle.

Meet counts and walk tables are integer results: they must equal the oracle's
bit for bit.  Estimates are counts / R in FP64 on both sides, so they are
equal too; the accuracy checks against exact SimRank use the Hoeffding radius.
Every call goes through the C ABI (ctypes binding).
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import oracle_threads as OT
from oracle import exact
from paper_2304_04015_amd import inputs
from paper_2304_04015_amd import simrank as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _counts(G, q):
    out, cnt, st = S.simrank_single_source_ex(G, q)
    return out, cnt, st


@pytest.fixture(scope="module")
def c1():
    cfg = inputs.C1
    g = inputs.workload_graph(cfg)
    return cfg, g, S.load_csr(g)


def test_c1_walk_tables_bit_exact(c1):
    cfg, g, G = c1
    _say("C1 walk tables: 500 nodes x 2000 walks x 33")
    vs = np.repeat(np.arange(g.n, dtype=np.int32), cfg["R"])
    js = np.tile(np.arange(cfg["R"], dtype=np.uint32), g.n)
    q = S.make_query(cfg["s"], c=cfg["c"], seed=cfg["walk_seed"], walk_cap=cfg["L"], R=cfg["R"])
    paths, lens = S.simrank_walks(G, q, vs, js)
    opaths, olens = O.walk_table_plain(g, cfg["walk_seed"], cfg["c"], cfg["L"], vs, js)
    assert np.array_equal(lens, olens)
    assert np.array_equal(paths, opaths)


def test_c1_counts_bit_exact_and_accurate(c1):
    cfg, g, G = c1
    _say("C1 counts")
    q = S.make_query(cfg["s"], c=cfg["c"], seed=cfg["walk_seed"], walk_cap=cfg["L"], R=cfg["R"])
    out, cnt, st = _counts(G, q)
    want, work = O.meet_counts_plain(g, cfg["s"], cfg["walk_seed"], cfg["c"], cfg["L"], cfg["R"],
                                     with_work=True)
    assert np.array_equal(cnt, want)
    assert np.array_equal(out, want / float(cfg["R"]))
    assert out[cfg["s"]] == 1.0
    assert st.moves == int(work.sum())          # the kernel walks exactly as far as needed
    assert st.meets == int(want.sum()) - cfg["R"]
    S_exact = exact.exact_simrank(g.n, g.in_off, g.in_src, cfg["c"])[cfg["s"]]
    bound = math.sqrt(math.log(2 * g.n / 1e-3) / (2 * cfg["R"])) + cfg["c"] ** (cfg["L"] + 1)
    assert np.max(np.abs(out - S_exact)) <= bound


@pytest.mark.parametrize("name", sorted(inputs.tiny_graphs()))
def test_tiny_graphs_bit_exact_and_closed_forms(name):
    g = inputs.tiny_graphs()[name]
    G = S.load_csr(g)
    S_exact = exact.exact_simrank(g.n, g.in_off, g.in_src, 0.6)
    for s in range(g.n):
        q = S.make_query(s, c=0.6, eps=0.02, delta=1e-3, seed=77 + s, walk_cap=16)
        out, cnt, st = _counts(G, q)
        want = O.meet_counts_plain(g, s, 77 + s, 0.6, 16, st.R)
        assert np.array_equal(cnt, want), (name, s)
        # eps = 0.02 with per-node delta = 1e-3: a miss is possible only with tiny probability
        assert np.max(np.abs(out - S_exact[s])) <= 0.02 + 0.6 ** 17


def test_many_tiles_ragged():
    """R and L large enough that the source walks span several LDS tiles (both
    the 1024-walk and the node-window limits) and the active nodes several
    256-node chunks with a ragged last one."""
    g = inputs.erdos_renyi_in(700, 3.0, seed=12)
    for s, R, L, c in ((3, 6000, 64, 0.6), (11, 2500, 255, 0.92)):
        _say(f"tiles: s={s} R={R} L={L} c={c}")
        q = S.make_query(s, c=c, seed=999 + s, walk_cap=L, R=R)
        out, cnt, st = _counts(G := S.load_csr(g), q)
        want = O.meet_counts_plain(g, s, 999 + s, c, L, R)
        assert np.array_equal(cnt, want)
        G.free()


@pytest.mark.parametrize("case", ["no_in_edges_source", "edgeless", "single_node", "R1_L1",
                                  "union_bound", "self_loops", "last_node"])
def test_edge_cases(case):
    if case == "edgeless":
        g = inputs.from_edges(10, [], [])
        s, R, L = 3, 100, 8
    elif case == "single_node":
        g = inputs.from_edges(1, [], [])
        s, R, L = 0, 50, 8
    elif case == "self_loops":
        g = inputs.from_edges(5, [0, 1, 1, 2, 3, 4, 2], [0, 1, 2, 2, 3, 0, 4])
        s, R, L = 2, 3000, 20
    else:
        g = inputs.erdos_renyi_in(150, 2.0, seed=4)
        deg = g.in_degree()
        if case == "no_in_edges_source":
            s = int(np.nonzero(deg == 0)[0][0])
            R, L = 700, 16
        elif case == "R1_L1":
            s, R, L = int(np.nonzero(deg > 0)[0][0]), 1, 1
        elif case == "last_node":
            s, R, L = g.n - 1, 900, 40
        else:
            s, R, L = 5, 0, 32
    G = S.load_csr(g)
    q = S.make_query(s, c=0.6, eps=0.05, delta=1e-3, seed=31337, walk_cap=L, R=R,
                     union_bound=(case == "union_bound"))
    out, cnt, st = _counts(G, q)
    want = O.meet_counts_plain(g, s, 31337, 0.6, L, st.R)
    assert np.array_equal(cnt, want)
    assert cnt[s] == st.R and out[s] == 1.0
    if case in ("no_in_edges_source", "edgeless", "single_node"):
        assert cnt.sum() == st.R


def test_hub_with_huge_in_degree():
    """A hub with 300,000 in-neighbours (every other node points to it and it
    points to every other node, plus one random edge per node): neighbour picks
    over a row far longer than any tile or wave, and many meets at the hub at
    step 1.  Counts equal the oracle's on a sample of nodes and the hub."""
    n = 300_001
    rng = np.random.default_rng(77)
    leaves = np.arange(1, n)
    extra = rng.integers(1, n, n - 1)
    src = np.concatenate([leaves, np.zeros(n - 1, np.int64), extra])
    dst = np.concatenate([np.zeros(n - 1, np.int64), leaves, leaves])
    g = inputs.from_edges(n, src, dst)
    assert g.in_degree()[0] == n - 1
    G = S.load_csr(g)
    q = S.make_query(1, c=0.6, seed=0xB0B, walk_cap=16, R=3000)
    out, cnt, st = _counts(G, q)
    vs = np.union1d(rng.choice(n, 3000, replace=False), [0, 1, n - 1]).astype(np.int32)
    want = O.meet_counts_plain(g, 1, 0xB0B, 0.6, 16, 3000, vs=vs)
    assert np.array_equal(cnt[vs], want)
    assert cnt[1] == 3000 and cnt[2:].max() > 0
    G.free()


def test_repeat_is_deterministic_and_async_matches():
    import torch
    g = inputs.erdos_renyi_in(2000, 5.0, seed=8)
    G = S.load_csr(g)
    q = S.make_query(17, c=0.6, eps=0.03, delta=1e-3, seed=4242)
    _, a, st = _counts(G, q)
    _, b, _ = _counts(G, q)
    assert np.array_equal(a, b)
    ws = S.simrank_workspace_create(G, st.R, 64)
    out_d = torch.empty(g.n, dtype=torch.float64, device="cuda")
    cnt_d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    for _ in range(3):
        S.simrank_single_source_async(G, q, ws, out_d, cnt_d, stream)
        st2 = S.simrank_workspace_stats(ws)
        assert np.array_equal(cnt_d.cpu().numpy().view(np.uint32), a)
        assert st2.moves == st.moves and st2.meets == st.meets
    vs = np.arange(0, g.n, 7, dtype=np.int32)
    want = O.meet_counts_plain(g, 17, 4242, 0.6, 64, st.R, vs=vs)
    assert np.array_equal(a[vs], want)


@pytest.fixture(scope="module")
def c2():
    cfg = inputs.C2
    _say("generating the R-MAT scale-20 graph")
    g = inputs.workload_graph(cfg)
    return cfg, g, S.load_csr(g)


def test_c2_full_size_sampled(c2):
    """Full-size medium workload (R-MAT n=2^20, R=9502, L=64) in the launch
    configuration the benchmark times, for all 8 of its sources: counts of
    4,096 random nodes with in-edges, the 256 highest in-degree nodes and 8
    nodes without in-edges against the oracle (run over host threads), and
    the estimate of every sampled node equal to count / R."""
    cfg, g, G = c2
    sources = inputs.sources_with_in_edges(g, cfg["n_sources"], cfg["source_seed"])
    assert len(sources) == 8
    deg = g.in_degree()
    sample = OT.sample_nodes(g, 4096, 256, 8, seed=5)
    for s in sources:
        _say(f"C2 source {s}: GPU")
        q = S.make_query(int(s), c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"],
                         seed=cfg["walk_seed"], walk_cap=cfg["L"])
        out, cnt, st = _counts(G, q)
        assert st.R == 9502
        smp = np.union1d(sample, [s]).astype(np.int32)
        _say(f"  oracle on {smp.size} nodes, {OT.host_threads()} threads")
        want = OT.meet_counts_plain(g, int(s), cfg["walk_seed"], cfg["c"], cfg["L"], st.R, smp)
        assert np.array_equal(cnt[smp], want)
        assert np.array_equal(out[smp], np.where(smp == s, 1.0, want / float(st.R)))
        assert cnt[s] == st.R
        assert np.all(cnt[deg == 0][np.nonzero(deg == 0)[0] != s] == 0)
        _say(f"  moves={st.moves} draws={st.draws} meet_ms={st.meet_ms:.2f} ms={st.ms:.2f}")


def test_roofline_probes_run():
    r = S.simrank_roofline_gather(1 << 24, 8, dependent=False)
    assert r["per_s"] > 1e9 and r["ms"] > 0
    r = S.simrank_roofline_gather(1 << 24, 4, dependent=True)
    assert r["per_s"] > 1e8
    assert S.simrank_roofline_philox()["per_s"] > 1e10
    assert S.simrank_roofline_copy(1 << 26)["per_s"] > 1e11
    with pytest.raises(S.SimRankError):
        S.simrank_roofline_gather(100, 8)
    r = S.simrank_roofline_gather_grid(1 << 24, 8, 16, 64)
    assert r["per_s"] > 1e8 and r["count"] >= 16 * 64 * 4 * 256
    for blocks, threads in ((0, 64), (16, 32), (16, 96), (16, 2048)):
        with pytest.raises(S.SimRankError):
            S.simrank_roofline_gather_grid(1 << 24, 8, blocks, threads)
