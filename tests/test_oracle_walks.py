"""Pins for the C walk oracle: Philox known answers, the stop and neighbour-pick
distributions, meet-count special cases with exact laws, and the estimator
against exact SimRank (Lemma 2, Hoeffding bound of Section 3)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from oracle import exact
from paper_2304_04015_amd import inputs

C = 0.6
SEED = 0x2304040150000001
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(row):
    ctr, key, want = row
    assert list(O.philox(ctr, key)) == want


ROCRAND_H = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.mark.skipif(not (os.path.exists(ROCRAND_H) and shutil.which("g++")),
                    reason="rocRAND headers or g++ not present")
def test_philox_equals_rocrand(tmp_path):
    """The oracle's Philox4x32-10 against rocRAND's (header-only, built for the
    host): 4,096 random (counter, key) pairs plus the counter forms the walks
    use (node, walk, step, domain) and all-zero / all-one words."""
    src = os.path.join(os.path.dirname(__file__), "philox_rocrand_probe.cpp")
    exe = str(tmp_path / "probe")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", src, "-o", exe],
                   check=True, capture_output=True, timeout=120)
    rng = np.random.default_rng(20230404)
    rows = [list(r) for r in rng.integers(0, 2 ** 32, size=(4096, 6), dtype=np.uint64)]
    k0, k1 = SEED & 0xFFFFFFFF, SEED >> 32
    rows += [[v, j, t, d, k0, k1] for v in (0, 1, 1048575) for j in (0, 9501)
             for t in (0, 1, 64) for d in range(6)]
    rows += [[0] * 6, [0xFFFFFFFF] * 6, [0xFFFFFFFF] * 4 + [0, 0], [0] * 4 + [0xFFFFFFFF] * 2]
    text = "".join(" ".join(f"{int(w):08x}" for w in r) + "\n" for r in rows)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True, timeout=120)
    got = [[int(w, 16) for w in line.split()] for line in out.stdout.splitlines()]
    assert len(got) == len(rows)
    for r, g in zip(rows, got):
        assert list(O.philox([int(w) for w in r[:4]], [int(w) for w in r[4:]])) == g, r


def test_philox_uniform_words():
    x = O.draw_block(SEED, 7, 11, 0, 0, 1 << 18)
    for k in range(4):
        h = np.bincount(x[:, k] >> 24, minlength=256)           # top byte histogram
        exp = x.shape[0] / 256
        chi2 = float(((h - exp) ** 2 / exp).sum())
        assert chi2 < 255 + 6 * math.sqrt(2 * 255)               # ~6 sigma above the mean
    # counters that differ in one word give unrelated words
    y = O.draw_block(SEED, 7, 12, 0, 0, 1 << 12)
    assert np.mean(x[: 1 << 12, 0] == y[:, 0]) < 0.01


def test_continue_threshold():
    T = O.continue_threshold(C)
    assert T == math.floor(math.sqrt(C) * 2 ** 32)
    assert O.continue_threshold(1.0) == 2 ** 32 - 1
    assert abs(T / 2 ** 32 - math.sqrt(C)) < 2 ** -32


def test_walk_follows_in_edges_and_stop_rate():
    # cycle 0->1->...->5->0: I(v) = {v-1}; a walk from v visits v, v-1, v-2, ...
    g = inputs.tiny_graphs()["cycle6"]
    L = 40
    T = O.continue_threshold(C)
    q = T / 2 ** 32
    lens = []
    for j in range(20000):
        p = O.walk_plain(g, SEED, C, L, 2, j)
        assert all(p[t] == (2 - t) % 6 for t in range(p.size))
        lens.append(p.size - 1)
    lens = np.array(lens)
    # length law: Pr[len = l] = q^l (1 - q) for l < L, Pr[len = L] = q^L
    h = np.bincount(np.minimum(lens, 12), minlength=13)
    pl = np.array([q ** l * (1 - q) for l in range(12)] + [q ** 12])
    exp = pl * lens.size
    chi2 = float(((h - exp) ** 2 / exp).sum())
    assert chi2 < 12 + 6 * math.sqrt(24)


def test_neighbour_pick_uniform():
    # node 3 of the undirected K_{3,4} has I = {0,1,2} (not a power of two)
    g = inputs.tiny_graphs()["K_3_4"]
    first = []
    for j in range(30000):
        p = O.walk_plain(g, SEED, C, 1, 3, j)
        if p.size > 1:
            first.append(p[1])
    h = np.bincount(first, minlength=3)[:3]
    exp = len(first) / 3
    assert float(((h - exp) ** 2 / exp).sum()) < 2 + 6 * 2
    assert len(first) / 30000 == pytest.approx(math.sqrt(C), abs=0.01)


def test_counts_special_cases():
    g = inputs.erdos_renyi_in(200, 3.0, seed=5)
    R, L = 300, 32
    deg = g.in_degree()
    s = int(np.nonzero(deg > 0)[0][0])
    cnt = O.meet_counts_plain(g, s, SEED, C, L, R)
    assert cnt[s] == R                                   # the pair (s, s) meets at index 0
    assert np.all(cnt[deg == 0][np.nonzero(deg == 0)[0] != s] == 0)   # I(v) empty
    s0 = int(np.nonzero(deg == 0)[0][0])                  # a source without in-neighbours
    cnt0 = O.meet_counts_plain(g, s0, SEED, C, L, R)
    assert cnt0[s0] == R and cnt0.sum() == R


@pytest.mark.parametrize("p", [1, 2, 4])
def test_counts_binomial_law(p):
    """Directed A -> B with |A| = p a power of two: two walks from b, b' meet iff
    both continue at step 1 and pick the same a (a has no in-neighbour, so the
    walks end there).  The pick floor(x*p/2^32) is exactly uniform for p | 2^32,
    so cnt ~ Binomial(R, (T/2^32)^2 / p) exactly."""
    q = 2
    g = inputs.from_edges(p + q, [a for a in range(p) for _ in range(q)],
                          [p + b for _ in range(p) for b in range(q)])
    R = 40000
    cnt = O.meet_counts_plain(g, p, SEED, C, 16, R, vs=[p + 1])[0]
    pr = (O.continue_threshold(C) / 2 ** 32) ** 2 / p
    mu, sd = R * pr, math.sqrt(R * pr * (1 - pr))
    assert abs(cnt - mu) < 5 * sd


def test_estimator_mean_matches_truncated_simrank():
    """E[cnt/R] = S_L with sqrt(c) replaced by T/2^32 (Lemma 2 and the key identity
    S_k = Pr[meet within k]).  z-test of the seed-averaged estimate, every node."""
    g = inputs.erdos_renyi_in(40, 2.5, seed=11)
    L, R, seeds = 12, 400, 24
    q = O.continue_threshold(C) / 2 ** 32
    S_L = exact.simrank_iterates(g.n, g.in_off, g.in_src, q * q, L)
    s = 3
    tot = np.zeros(g.n)
    for k in range(seeds):
        tot += O.meet_counts_plain(g, s, SEED + 1000 * k, C, L, R)
    mean = tot / (R * seeds)
    p = S_L[s]
    sd = np.sqrt(np.maximum(p * (1 - p), 1e-12) / (R * seeds))
    z = np.abs(mean - p) / sd
    assert z.max() < 5.0
    # and a node with I(v) empty or unreachable similarity is exactly zero
    assert np.all(mean[p == 0] == 0)


def test_c1_accuracy_vs_exact():
    """Workload C1 (ER n=500, R=2000, L=32): max_v |s_hat - s| stays within the
    union-bound Hoeffding radius sqrt(ln(2n/delta)/(2R)) + c^(L+1), delta=1e-3."""
    cfg = inputs.C1
    g = inputs.workload_graph(cfg)
    S = exact.exact_simrank(g.n, g.in_off, g.in_src, C)
    cnt = O.meet_counts_plain(g, cfg["s"], cfg["walk_seed"], C, cfg["L"], cfg["R"])
    est = cnt / cfg["R"]
    err = np.abs(est - S[cfg["s"]])
    bound = math.sqrt(math.log(2 * g.n / 1e-3) / (2 * cfg["R"])) + C ** (cfg["L"] + 1)
    assert err.max() <= bound
    assert est[cfg["s"]] == 1.0


def test_walk_table_matches_single_walks():
    g = inputs.erdos_renyi_in(50, 3.0, seed=2)
    vs = np.array([0, 5, 9, 9, 49], np.int32)
    js = np.array([0, 3, 3, 4, 1000], np.uint32)
    paths, lens = O.walk_table_plain(g, SEED, C, 16, vs, js)
    for i in range(vs.size):
        p = O.walk_plain(g, SEED, C, 16, int(vs[i]), int(js[i]))
        assert lens[i] == p.size - 1
        assert np.array_equal(paths[i, : p.size], p)
        assert np.all(paths[i, p.size:] == -1)


def test_work_counts_definition():
    """work = sum_j min(len_s, len_v, first meet index) for v != s, recomputed
    here from explicit walk tables."""
    g = inputs.erdos_renyi_in(60, 3.0, seed=4)
    s, R, L = 1, 50, 20
    vs = np.arange(g.n, dtype=np.int32)
    cnt, work = O.meet_counts_plain(g, s, SEED, C, L, R, vs=vs, with_work=True)
    for v in (0, 2, 17, 33):
        w = 0
        c = 0
        for j in range(R):
            a = O.walk_plain(g, SEED, C, L, s, j)
            b = O.walk_plain(g, SEED, C, L, v, j)
            lim = min(a.size, b.size) - 1
            hit = [t for t in range(lim + 1) if a[t] == b[t]]
            c += bool(hit)
            w += min(lim, hit[0]) if hit else lim
        assert cnt[v] == c and work[v] == w
    assert work[s] == 0
