"""Seeded synthetic inputs: graphs as int32 CSR of in-edges, sources and query mixes.

This module holds no part of the SimRank method.  It only draws graphs and query
parameters from fixed seeds, so the CPU oracle and the GPU library can be fed the
same bytes.  Every graph is returned as the in-edge CSR of the reversed graph
(Algorithm 1, "reverse the edges"): row v lists I(v), the in-neighbours of v,
sorted ascending, as `in_off` int32[n+1] and `in_src` int32[m].

Recipes (numpy PCG64 throughout):

* `erdos_renyi_in(n, mean_in, seed)`: every node v draws k ~ Poisson(mean_in)
  in-edges whose sources are uniform on [0, n); self-loops and repeated
  sources are dropped (I(v) is a set in Eq. 1); nodes left with no in-edge stay.
* `rmat_in(scale, n_edges, abcd, seed, n=None)`: R-MAT edge draws u->v with the
  recursive quadrant probabilities (a, b, c, d); duplicates removed, self-loops
  kept; a seeded random relabelling of the vertices so hub ids are not
  clustered near 0.  With `n` below 2**scale, draws with an endpoint >= n are
  rejected and drawing continues until `n_edges` draws are kept (the batching
  mix uses this for n that are not powers of two).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "erdos_renyi_in", "rmat_in", "from_edges", "sources_with_in_edges",
    "tiny_graphs", "C1", "C2", "C3", "C4", "C5", "workload_graph",
]


@dataclass
class CSR:
    """In-edge CSR: I(v) = in_src[in_off[v]:in_off[v+1]]."""
    n: int
    in_off: np.ndarray  # int32[n+1]
    in_src: np.ndarray  # int32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.in_src.shape[0])

    def in_degree(self) -> np.ndarray:
        return np.diff(self.in_off.astype(np.int64))

    def nbytes(self) -> int:
        return int(self.in_off.nbytes + self.in_src.nbytes)


def _csr_from_sorted_keys(n: int, dst: np.ndarray, src: np.ndarray, name: str) -> CSR:
    counts = np.bincount(dst, minlength=n).astype(np.int64)
    off = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    if off[-1] > np.iinfo(np.int32).max:
        raise ValueError("edge count exceeds int32 offsets")
    return CSR(n, off.astype(np.int32), src.astype(np.int32), name)


def from_edges(n: int, src, dst, name: str = "", dedupe: bool = True,
               drop_self_loops: bool = False) -> CSR:
    """Build the in-edge CSR of G from directed edges src[i] -> dst[i]."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    if src.size and (src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    if drop_self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    key = dst * n + src
    key = np.unique(key) if dedupe else np.sort(key, kind="stable")
    dst = key // n
    src = key - dst * n
    return _csr_from_sorted_keys(n, dst, src, name)


def erdos_renyi_in(n: int, mean_in: float = 5.0, seed: int = 1) -> CSR:
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.poisson(mean_in, size=n)
    dst = np.repeat(np.arange(n, dtype=np.int64), k)
    src = rng.integers(0, n, size=dst.size, dtype=np.int64)
    return from_edges(n, src, dst, name=f"er_n{n}_p{mean_in}_s{seed}",
                      dedupe=True, drop_self_loops=True)


def _rmat_chunk(seed_seq, scale: int, e: int, t_a, t_ab, t_abc, n: int, full: int):
    """e R-MAT draws from one independent stream; returns (u, v) kept draws."""
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    u = np.zeros(e, np.int64)
    v = np.zeros(e, np.int64)
    for bit in range(scale):
        r = rng.random(e, dtype=np.float32)
        ub = r >= t_ab                                  # quadrants c, d: lower half of rows
        vb = ((r >= t_a) & (r < t_ab)) | (r >= t_abc)   # quadrants b, d
        u |= ub.astype(np.int64) << bit
        v |= vb.astype(np.int64) << bit
    if n < full:
        keep = (u < n) & (v < n)
        u, v = u[keep], v[keep]
    return u, v


def _unique_keys_parallel(key: np.ndarray, n_buckets: int, threads: int) -> np.ndarray:
    """np.unique(key) for non-negative keys, computed bucket by bucket (buckets by
    the top bits of the key, split with one radix argsort) on a thread pool."""
    import concurrent.futures as cf
    if key.size == 0:
        return key
    kmax = int(key.max()) + 1
    shift = max(0, int(kmax - 1).bit_length() - int(n_buckets - 1).bit_length())
    b = (key >> shift).astype(np.uint8)
    order = np.argsort(b, kind="stable")       # radix sort of small integers
    key = key[order]
    del order
    bounds = np.concatenate([[0], np.cumsum(np.bincount(b, minlength=n_buckets))])
    del b
    parts = [key[bounds[i]:bounds[i + 1]] for i in range(n_buckets)]
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(np.unique, parts))
    return np.concatenate(parts)


def rmat_in(scale: int, n_edges: int, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 2,
            n: int | None = None, permute: bool = True, chunk: int = 1 << 22,
            threads: int | None = None) -> CSR:
    """R-MAT draws in chunks of `chunk`; chunk i is drawn from the child stream
    SeedSequence(seed, spawn_key=(i,)), so the graph does not depend on the
    thread count."""
    import concurrent.futures as cf
    a, b, c, d = abcd
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("R-MAT probabilities must sum to 1")
    full = 1 << scale
    n = full if n is None else int(n)
    if not (0 < n <= full):
        raise ValueError("n must lie in (0, 2**scale]")
    threads = threads or min(16, os.cpu_count() or 1)
    t_ab, t_abc = np.float32(a + b), np.float32(a + b + c)
    t_a = np.float32(a)
    us, vs = [], []
    kept = 0
    next_child = 0
    # draw rounds of `threads` chunks until n_edges draws are kept (rejection for n < 2^scale)
    while kept < n_edges:
        need = int(n_edges) - kept
        nch = max(1, min(threads, -(-need // chunk)))
        seqs = [np.random.SeedSequence(seed, spawn_key=(next_child + i,)) for i in range(nch)]
        next_child += nch
        sizes = [min(chunk, max(need - i * chunk, 1 << 16)) for i in range(nch)]
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            res = list(ex.map(lambda ar: _rmat_chunk(ar[0], scale, ar[1], t_a, t_ab, t_abc, n, full),
                              zip(seqs, sizes)))
        for u, v in res:
            take = min(u.size, int(n_edges) - kept)
            if take <= 0:
                break
            us.append(u[:take])
            vs.append(v[:take])
            kept += take
    u = np.concatenate(us)
    v = np.concatenate(vs)
    del us, vs
    if permute:
        perm = np.random.Generator(np.random.PCG64(seed ^ 0x5EED)).permutation(n).astype(np.int64)
        u = perm[u]
        v = perm[v]
    key = v * n + u
    del u, v
    key = _unique_keys_parallel(key, 64, threads)
    dst = key // n
    src = key - dst * n
    name = f"rmat_s{scale}_n{n}_e{n_edges}_seed{seed}"
    return _csr_from_sorted_keys(n, dst, src, name)


def sources_with_in_edges(g: CSR, count: int, seed: int) -> np.ndarray:
    """`count` distinct sources drawn uniformly among nodes with |I(v)| >= 1."""
    cand = np.nonzero(g.in_degree() > 0)[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(cand, size=min(count, cand.size), replace=False)).astype(np.int32)


def sources_by_degree(g: CSR, count: int, seed: int) -> np.ndarray:
    """Sources drawn with probability proportional to in-degree (with replacement)."""
    deg = g.in_degree().astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.choice(g.n, size=count, replace=True, p=deg / deg.sum()).astype(np.int32)


# ---------------------------------------------------------------------------
# Small hand-checkable graphs (edges u->v of G; the walks follow in-edges)
# ---------------------------------------------------------------------------

def tiny_graphs() -> dict[str, CSR]:
    g = {}
    k = 5
    g["star_out5"] = from_edges(k + 1, [0] * k, list(range(1, k + 1)), "star_out5")
    # directed complete bipartite A -> B, |A| = p
    for p, q in ((3, 4), (2, 3), (4, 2), (1, 3)):
        src = [a for a in range(p) for _ in range(q)]
        dst = [p + b for _ in range(p) for b in range(q)]
        g[f"bip_dir_{p}_{q}"] = from_edges(p + q, src, dst, f"bip_dir_{p}_{q}")
    # undirected complete bipartite K_{p,q} (both directions)
    for p, q in ((2, 2), (3, 4)):
        src, dst = [], []
        for a in range(p):
            for b in range(q):
                src += [a, p + b]
                dst += [p + b, a]
        g[f"K_{p}_{q}"] = from_edges(p + q, src, dst, f"K_{p}_{q}")
    # undirected paths
    for L in (3, 5):
        src = [i for i in range(L - 1)] + [i + 1 for i in range(L - 1)]
        dst = [i + 1 for i in range(L - 1)] + [i for i in range(L - 1)]
        g[f"path{L}"] = from_edges(L, src, dst, f"path{L}")
    g["cycle6"] = from_edges(6, list(range(6)), [(i + 1) % 6 for i in range(6)], "cycle6")
    return g


# ---------------------------------------------------------------------------
# The workloads
# ---------------------------------------------------------------------------

C1 = dict(kind="er", n=500, mean_in=5.0, seed=1, c=0.6, L=32, R=2000, s=0,
          walk_seed=0x2304040150000001)
C2 = dict(kind="rmat", scale=20, edge_factor=16, seed=2, c=0.6, eps=0.02, delta=1e-3,
          L=64, n_sources=8, source_seed=3, walk_seed=0x2304040150000002)
C3 = dict(kind="rmat", scale=24, edge_factor=16, seed=4, c=0.6, eps=0.02, delta=1e-3,
          L=64, seg_log2=3, kappa=1.0, source_seed=5, walk_seed=0x2304040150000003,
          index_seed=0x2304040150000013)
C4 = dict(n_graphs=16, n_queries=512, log2n=(12, 22), deg=(8, 32), graph_seed0=10,
          eps_choices=(0.05, 0.02, 0.01), delta=1e-3, c=0.6, L=64, mix_seed=26)
C5 = dict(kind="rmat", scale=22, edge_factor=16, seed=30, c=0.6, delta=1e-3, L=64,
          eps_choices=(0.05, 0.02))


def workload_graph(cfg: dict) -> CSR:
    if cfg.get("kind") == "er":
        return erdos_renyi_in(cfg["n"], cfg["mean_in"], cfg["seed"])
    scale = cfg["scale"]
    return rmat_in(scale, cfg["edge_factor"] << scale, seed=cfg["seed"])


def batch_graph_specs(cfg: dict = C4) -> list[dict]:
    """The 16 graphs of the batching mix: n = floor(2**U(lo, hi)), avg degree U{8..32}."""
    rng = np.random.Generator(np.random.PCG64(cfg["mix_seed"]))
    lo, hi = cfg["log2n"]
    specs = []
    for i in range(cfg["n_graphs"]):
        n = int(math.floor(2.0 ** rng.uniform(lo, hi)))
        deg = int(rng.integers(cfg["deg"][0], cfg["deg"][1] + 1))
        specs.append(dict(n=n, scale=max(1, math.ceil(math.log2(n))), deg=deg,
                          seed=cfg["graph_seed0"] + i))
    return specs


def batch_graph(spec: dict) -> CSR:
    n, scale = spec["n"], spec["scale"]
    return rmat_in(scale, n * spec["deg"], seed=spec["seed"], n=n)
