"""Benchmark: single-source sqrt(c)-walk SimRank on one MI355X.

Workload (the medium configuration): R-MAT graph, n = 2^20 nodes, 16 n edge
draws with (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), duplicates removed,
vertices relabelled by a seeded permutation; c = 0.6, eps = 0.02,
delta = 1e-3 (R = 9502 walks per node from Hoeffding), walk cap L = 64;
8 sources drawn uniformly among nodes with in-edges, each run as its own
single-source query.  One step = those 8 queries, each a full pass of the
query path (source walks, compaction, fused walk + meet + count, estimate),
with the graph already resident in HBM.

Prints one JSON line.  `value` is walk steps per second (moves along in-edges
made by the meet kernel, plus the source walks' steps); `queries_per_s` is
single-source queries per second with the estimates left in device memory,
`queries_per_s_with_d2h` the same with each estimate copied to pinned host
memory.  `batched` runs the same 8 queries as one captured batch plan (a seed
per query, and the line's shared seed as one query group) against the plain
one-at-a-time rate.  `roofline` reports the fused walk + meet kernel:
algorithmic bytes (12 per move: an 8-byte row read and a 4-byte edge read)
over its launch time measured with HIP events on the stream it runs on,
against the published HBM peak; the kernel's real limit, the rate of random
128-byte line requests the memory system serves, is stated beside it.
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walk-steps/s + single-source queries/s at eps=0.02; batched vs plain, % roofline"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per walk step: reading the current node's row (offset and
# degree, 8 bytes) and one edge of it (4 bytes).  The library's gather layout
# reads the two as one 8-byte slot per step; that figure is reported beside.
BYTES_PER_MOVE = 12
BYTES_PER_MOVE_GATHERED = 8
# Host threads for the threaded CPU baseline: the host share of one GPU.
CPU_THREADS_CAP = 16


def roofline(kernel: str, moves: float, seconds: float, traffic=None, traffic_source=None,
             bound: str = "random-gather") -> dict:
    """The roofline object of a walk kernel: algorithmic bytes (BYTES_PER_MOVE
    per move) per second against the published HBM peak."""
    achieved = BYTES_PER_MOVE * moves / seconds / 1e9 if seconds > 0 else 0.0
    r = {
        "bound": bound,
        "kernel": kernel,
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "bytes_per_move": BYTES_PER_MOVE,
        "achieved_8B_gather_layout": BYTES_PER_MOVE_GATHERED * moves / seconds / 1e9
        if seconds > 0 else 0.0,
    }
    if traffic_source:
        r["traffic_source"] = traffic_source
    return r


STITCH_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_stitching_rmat24.json")
SEG_SLOTS = 2   # segments in flight per lane of the index build's walk kernel


def strip_comments(src: str) -> str:
    """C++ source without its comments and blank-line and trailing-space
    differences: what the compiler sees of the code (string and character
    literals kept as they are)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":                       # a literal: copy it whole
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).split("\n"))
    return "\n".join(ln for ln in lines if ln)


def kernel_fingerprint() -> str:
    """sha256 (16 hex digits) of the code, comments left out, of the sources the
    walk kernels are built from (the meet kernels and the index build)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2304_04015_amd", "csrc")
    h = "\n".join(strip_comments(open(os.path.join(csrc, f)).read())
                  for f in ("query.hip", "group.hip", "index.hip", "device_common.hpp", "philox.hpp",
                            "common.hpp"))
    return hashlib.sha256(h.encode()).hexdigest()[:16]


def measured_traffic(path: str, kernel: str = None):
    """HBM bytes per launch from the profiler's byte counters (scaled by a copy
    kernel of known size), if they were taken on the current kernel sources;
    `kernel` picks one kernel of a record that holds several (mean over its
    launches)."""
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("source_sha256_16") != kernel_fingerprint():
        return None
    if kernel is None:
        return t.get("bytes_per_launch")
    b = t.get("kernels", {}).get(kernel, {}).get("bytes_per_launch")
    return float(sum(b) / len(b)) if b else None


def copy_probe(args) -> None:
    """Copies a buffer of --copy-probe-mib MiB once: a kernel of known traffic
    that calibrates the profiler's byte counters."""
    import torch
    if args.copy_probe_mib:
        a = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="medium",
                    choices=["medium", "stitching", "batching", "serving", "stratified", "tuples",
                             "grouped"],
                    help="medium: the default line; stitching: R-MAT n=2^24 index build "
                         "and stitched query; batching: 512 queries over 16 graphs, "
                         "one captured batch vs one query at a time; serving: Poisson "
                         "arrivals on R-MAT n=2^22 at fractions of the plain capacity; "
                         "stratified: the medium graph and sources with the paper's "
                         "length-stratified estimator (Algorithms 1-2); tuples: the medium "
                         "graph's 8 sources (and 32) through Algorithm 2's tuple form")
    ap.add_argument("--requests", type=int, default=32, help="serving: requests per load level")
    ap.add_argument("--queries", type=int, default=512, help="batching: number of queries")
    ap.add_argument("--tune-index", action="store_true",
                    help="stitching: also run the segment-length tuner (k = 2, 3, 4) and report it")
    ap.add_argument("--group-max", type=int, default=0,
                    help="serving: admit waiting requests with one walk seed as query groups of "
                         "up to this many (0: every request alone, with its own seed)")
    ap.add_argument("--group-queries", type=int, default=32,
                    help="grouped: number of same-seed queries on the medium graph")
    ap.add_argument("--group-kind", default="plain", choices=["plain", "stratified"],
                    help="grouped: plain queries (groups of up to 32) or stratified ones (up to 8)")
    ap.add_argument("--served-mode", default="stitched", choices=["stitched", "plain", "stratified"],
                    help="serving: walks of the requests (stitched through the resident index, "
                         "plain, or Algorithms 1-2's stratified estimator with its own z and cap)")
    ap.add_argument("--shared-seed", action="store_true",
                    help="batching: one walk seed per graph instead of one per query, so that "
                         "the queries of a graph share their walks from every node (query groups)")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-nodes", type=int, default=6144,
                    help="nodes in the CPU oracle's sample (x R pairs, one source)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the queries, copy a buffer of this many MiB once (a kernel "
                         "of known traffic that calibrates the profiler's byte counters)")
    ap.add_argument("--tune", action="store_true",
                    help="medium: run the work-unit tuner on the graph before timing")
    ap.add_argument("--no-roofs", action="store_true",
                    help="skip the measured gather / Philox / copy ceilings")
    ap.add_argument("--no-batched", action="store_true",
                    help="medium: skip the batched leg (so that every launch of the meet "
                         "kernel is one query, e.g. under the profiler's counters)")
    ap.add_argument("--scale", type=int, default=0,
                    help="R-MAT scale of the graph (0: the medium workload's 20)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_meet_medium.json"),
                    help="measured HBM traffic per meet launch (JSON), if present")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard over nodes v with no exchange: each GPU regenerates "
              "the source walks and counts its own slice of the nodes)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "stitching":
        return bench_stitching(args)
    if args.workload == "batching":
        return bench_batching(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "stratified":
        return bench_stratified(args)
    if args.workload == "tuples":
        return bench_tuples(args)
    if args.workload == "grouped":
        return bench_grouped(args)

    import numpy as np
    import torch

    from paper_2304_04015_amd import inputs
    from paper_2304_04015_amd import simrank as S

    cfg = dict(inputs.C2)
    if args.scale:
        cfg["scale"] = args.scale
    torch.cuda.set_device(0)
    copy_probe(args)
    t0 = time.time()
    g = inputs.workload_graph(cfg)
    sources = inputs.sources_with_in_edges(g, cfg["n_sources"], cfg["source_seed"])
    print(f"# graph n={g.n} m={g.m} generated in {time.time() - t0:.1f}s", file=sys.stderr)
    G = S.load_csr(g)
    queries = [S.make_query(int(s), c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"],
                            seed=cfg["walk_seed"], walk_cap=cfg["L"]) for s in sources]
    R = S.simrank_derive_params(queries[0], g.n).R
    tuned = S.simrank_tune(G, queries[0]) if args.tune else None
    stream = torch.cuda.Stream()
    wss = [S.simrank_workspace_create(G, R, cfg["L"]) for _ in queries]
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in queries]
    cnts = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in queries]
    hosts = [torch.empty(g.n, dtype=torch.float64, pin_memory=True) for _ in queries]

    def step(d2h: bool = False):
        for q, ws, o, c, h in zip(queries, wss, outs, cnts, hosts):
            S.simrank_single_source_async(G, q, ws, o, c, stream)
            if d2h:
                with torch.cuda.stream(stream):
                    h.copy_(o, non_blocking=True)
        sts = [S.simrank_workspace_stats(ws) for ws in wss]
        if d2h:
            stream.synchronize()
        return sts

    for _ in range(max(args.warmup, 1)):
        ref = step()
    work = [st.moves + st.tail_steps + st.source_moves for st in ref]
    steps_per_step = int(sum(work))

    torch.cuda.synchronize()
    meet_ms, query_ms = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        sts = step()
        for st, r in zip(sts, ref):
            assert st.moves == r.moves and st.meets == r.meets   # deterministic work
        meet_ms += [st.meet_ms for st in sts]
        query_ms += [st.ms for st in sts]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ref_counts = [c.cpu().numpy().view(np.uint32).copy() for c in cnts]

    # the same queries with each estimate copied to pinned host memory (the
    # synchronous call's PCIe leg); not part of `value`
    d2h_steps = max(2, args.steps // 4)
    step(d2h=True)
    torch.cuda.synchronize()
    t_d = time.perf_counter()
    for _ in range(d2h_steps):
        step(d2h=True)
    el_d2h = time.perf_counter() - t_d
    d2h_equal = all(np.array_equal(h.numpy(), o.cpu().numpy()) for h, o in zip(hosts, outs))

    nq = len(queries) * args.steps
    value = steps_per_step * args.steps / elapsed
    moves_per_launch = float(np.mean([st.moves for st in ref]))
    avg_meet_s = float(np.mean(meet_ms)) / 1e3
    traffic = measured_traffic(args.traffic)
    plain_qps = nq / elapsed

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"{'medium: ' if cfg['scale'] == 20 else ''}R-MAT n=2^{cfg['scale']}, "
                        "16n edge draws (.57,.19,.19,.05), dedup, "
                        "permuted; c=0.6 eps=0.02 delta=1e-3 R=9502 L=64; "
                        "8 single-source queries per step",
            "n": g.n, "m": g.m, "R": R, "L": cfg["L"], "queries_per_step": len(queries),
            "unit_nodes": tuned if tuned else "default",
        },
        "queries_per_s": plain_qps,
        "queries_per_s_with_d2h": len(queries) * d2h_steps / el_d2h,
        "d2h_estimates_equal_device": d2h_equal,
        "pairs_per_s": sum(st.pairs for st in ref) * args.steps / elapsed,
        "moves_per_query": moves_per_launch,
        "draws_per_query": float(np.mean([st.draws for st in ref])),
        "meet_kernel_ms": float(np.mean(meet_ms)),
        "query_ms": float(np.mean(query_ms)),
        "roofline": roofline(
            "k_meet<plain> (fused walk + meet + count)", moves_per_launch, avg_meet_s,
            traffic=traffic,
            traffic_source=("not measured in this run: bytes per launch from rocprofv3 "
                            "FETCH_SIZE and WRITE_SIZE of the same kernel source, "
                            "profiles/traffic_meet_medium.json") if traffic else None),
    }
    result["roofline"]["bound_detail"] = (
        "the graph's 133 MB gather array sits in the 256 MB Infinity Cache; the kernel is "
        "limited by the rate of random 128-byte line requests the memory system serves "
        "(measured_roofs.line_requests_vs_random_gather), not by HBM bytes")

    # The same 8 queries as one captured batch plan: (a) a walk seed per query
    # (no two queries share walks), (b) the line's own queries, whose shared
    # seed makes them one query group; against the one-at-a-time rate above.
    bsteps = 0 if args.no_batched else max(2, args.steps // 4)
    per_seed = [S.make_query(int(s), c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"],
                             seed=cfg["walk_seed"] + 1 + i, walk_cap=cfg["L"])
                for i, s in enumerate(sources)]
    batched = {}
    for name, qs_b in (() if args.no_batched else
                       (("seed_per_query", per_seed), ("shared_seed_groups", queries))):
        plan = S.BatchPlan([G], qs_b)
        plan.run(stream)
        plan.wait()
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        for _ in range(bsteps):
            plan.run(stream)
            bst = plan.wait()
        el_b = time.perf_counter() - t_b
        if name == "shared_seed_groups":
            equal = all(np.array_equal(plan.read(i, want_out=False)[1], ref_counts[i])
                        for i in range(len(queries)))
        else:   # each against the same query run alone
            equal = True
            for i, q in enumerate(qs_b):
                S.simrank_single_source_async(G, q, wss[i], outs[i], cnts[i], stream)
                S.simrank_workspace_stats(wss[i])
                equal &= bool(np.array_equal(plan.read(i, want_out=False)[1],
                                             cnts[i].cpu().numpy().view(np.uint32)))
        qps_b = len(qs_b) * bsteps / el_b
        batched[name] = {"queries_per_s": qps_b, "batched_vs_plain": qps_b / plain_qps,
                         "groups": plan.n_groups, "runs": bsteps,
                         "device_ms_per_run": bst.ms,
                         "walk_steps_per_s": (bst.moves + bst.tail_steps + bst.source_moves)
                         * bsteps / el_b,
                         "results_equal_lone": equal}
        plan.free()
    result["batched"] = batched

    if not args.no_roofs:
        info = G.info()
        slots_bytes = 8 * (info["m"] + info["n"] - info["n_active"])
        gi = S.simrank_roofline_gather(slots_bytes, 8, dependent=False)
        gd = S.simrank_roofline_gather(slots_bytes, 8, dependent=True)
        # the same gathers from half the CUs, and from one wave per CU: the rate
        # is the memory system's if these match the full grid's
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        gh = S.simrank_roofline_gather_grid(slots_bytes, 8, max(1, cus // 2), 1024)
        gw = S.simrank_roofline_gather_grid(slots_bytes, 8, cus, 64)
        ph = S.simrank_roofline_philox()
        cp = S.simrank_roofline_copy(1 << 30)
        moves_per_s = moves_per_launch / avg_meet_s
        draws_per_s = float(np.mean([st.draws for st in ref])) / avg_meet_s
        result["measured_roofs"] = {
            "footprint_bytes": slots_bytes,
            "random_gather_8B_per_s": gi["per_s"],
            "dependent_chain_gather_8B_per_s": gd["per_s"],
            "random_gather_8B_per_s_half_cus": gh["per_s"],
            "random_gather_8B_per_s_one_wave_per_cu": gw["per_s"],
            "philox_draws_per_s": ph["per_s"],
            "copy_bytes_per_s": cp["per_s"],
            "kernel_moves_per_s": moves_per_s,
            "kernel_draws_per_s": draws_per_s,
            "moves_vs_random_gather": moves_per_s / gi["per_s"],
            "draws_vs_philox": draws_per_s / ph["per_s"],
        }
        if traffic:
            # the kernel's 128-byte line requests per second (from the byte
            # counters) against the same machine's rate for random gathers
            # over the same footprint, each of which is one such request
            req_per_s = traffic / 128.0 / avg_meet_s
            result["measured_roofs"]["line_requests_per_s"] = req_per_s
            result["measured_roofs"]["line_requests_vs_random_gather"] = req_per_s / gi["per_s"]

    if not args.no_cpu:
        import oracle as O
        s0 = int(sources[0])
        rng = np.random.default_rng(11)
        act = np.nonzero(g.in_degree() > 0)[0]
        vs = np.sort(rng.choice(act, args.cpu_nodes, replace=False)).astype(np.int32)
        t1 = time.perf_counter()
        cnt, w = O.meet_counts_plain(g, s0, cfg["walk_seed"], cfg["c"], cfg["L"], R, vs=vs,
                                     with_work=True)
        dt = time.perf_counter() - t1
        same = bool(np.array_equal(ref_counts[0][vs], cnt))
        pairs = vs.size * R
        # the same oracle call on the same sample split over host threads (the
        # call holds no shared state and releases the GIL): as many threads as
        # this process may use, at most the host share of one GPU
        from concurrent.futures import ThreadPoolExecutor
        try:
            usable = len(os.sched_getaffinity(0))
        except AttributeError:
            usable = os.cpu_count() or 1
        nt = max(1, min(CPU_THREADS_CAP, usable))
        parts = np.array_split(vs, nt)
        t2 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=nt) as ex:
            outs_mt = list(ex.map(lambda p: O.meet_counts_plain(g, s0, cfg["walk_seed"], cfg["c"],
                                                                cfg["L"], R, vs=p, with_work=True),
                                  parts))
        dt_mt = time.perf_counter() - t2
        same_mt = bool(np.array_equal(np.concatenate([o[0] for o in outs_mt]), cnt))
        result["cpu_baseline"] = {
            "value": float(w.sum()) / dt,
            "unit": "walk-steps/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"source {s0}, {vs.size} random nodes with in-edges x R={R} pairs "
                      f"({pairs} pairs, {dt:.1f}s single-threaded); counts equal to the GPU's: {same}",
            "queries_per_s": pairs / dt / ((g.n - 1) * R),
            "host": {"nproc": os.cpu_count(), "usable_cpus": usable},
            "threads": {
                "value": float(w.sum()) / dt_mt,
                "cores": nt,
                "sample": f"the same sample in {nt} node chunks, one thread each ({dt_mt:.1f}s; "
                          f"{usable} CPUs usable by this process, at most {CPU_THREADS_CAP} "
                          f"used: the host share of one GPU); counts equal: {same_mt}",
                "queries_per_s": pairs / dt_mt / ((g.n - 1) * R),
            },
        }
    print(json.dumps(result))
    for ws in wss:
        ws.free()
    G.free()


def bench_stratified(args):
    """The medium graph and its 8 sources with the length-stratified estimator
    at Algorithm 2's own z for eps = 0.02 (N = 18,234 walks per node) and
    Algorithm 1's cap phi = 54, against the plain estimator on the same
    queries (R = 9,502, L = 64)."""
    import numpy as np
    import torch

    from paper_2304_04015_amd import inputs
    from paper_2304_04015_amd import simrank as S

    cfg = dict(inputs.C2)
    torch.cuda.set_device(0)
    copy_probe(args)
    t0 = time.time()
    g = inputs.workload_graph(cfg)
    sources = inputs.sources_with_in_edges(g, cfg["n_sources"], cfg["source_seed"])
    print(f"# graph n={g.n} m={g.m} generated in {time.time() - t0:.1f}s", file=sys.stderr)
    G = S.load_csr(g)
    sq = [S.make_stratified_query(int(s), c=cfg["c"], eps=cfg["eps"], seed=cfg["walk_seed"])
          for s in sources]
    pq = [S.make_query(int(s), c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"],
                       seed=cfg["walk_seed"], walk_cap=cfg["L"]) for s in sources]
    sp = S.simrank_derive_stratified(sq[0], g.n)
    R = S.simrank_derive_params(pq[0], g.n).R
    stream = torch.cuda.Stream()
    wss = [S.simrank_workspace_create(G, max(sp.N, R), max(sp.phi, cfg["L"])) for _ in sources]
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in sources]
    outn = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in sources]
    wsum = [torch.empty(g.n, dtype=torch.int64, device="cuda") for _ in sources]
    pout = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in sources]
    pcnt = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in sources]

    def run(stratified: bool):
        for i, ws in enumerate(wss):
            if stratified:
                S.simrank_stratified_async(G, sq[i], ws, outs[i], outn[i], wsum[i], stream)
            else:
                S.simrank_single_source_async(G, pq[i], ws, pout[i], pcnt[i], stream)
        return [S.simrank_workspace_stats(ws) for ws in wss]

    res = {}
    for kind in (True, False):
        ref = run(kind)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        meet_ms = []
        for _ in range(args.steps):
            sts = run(kind)
            for st, r in zip(sts, ref):
                assert st.moves == r.moves and st.meets == r.meets
            meet_ms += [st.meet_ms for st in sts]
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        steps = sum(st.moves + st.source_moves for st in ref) * args.steps
        res[kind] = dict(elapsed=el, steps=steps, q=len(sources) * args.steps,
                         meet_ms=float(np.mean(meet_ms)),
                         moves=float(np.mean([st.moves for st in ref])),
                         meets=float(np.mean([st.meets for st in ref])),
                         pairs_walked=float(np.mean([st.pairs_walked for st in ref])))
    st_, pl = res[True], res[False]
    diffs = [float((outn[i] - pout[i]).abs().max()) for i in range(len(sources))]
    value = st_["steps"] / st_["elapsed"]
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": 1e3 * st_["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "stratified: R-MAT n=2^20 (the medium graph), 8 sources; "
                        "length-stratified estimator at eps=0.02: z=ln(2n)/(2(eps-3/n)^2), "
                        f"N={sp.N} walks per node in classes l=0..{sp.phi}, shuffled; "
                        "Lemma 5 weights",
            "n": g.n, "m": g.m, "N": sp.N, "phi": sp.phi, "z": sp.z,
        },
        "queries_per_s": st_["q"] / st_["elapsed"],
        "plain_queries_per_s": pl["q"] / pl["elapsed"],
        "plain_walk_steps_per_s": pl["steps"] / pl["elapsed"],
        "moves_per_query": st_["moves"],
        "plain_moves_per_query": pl["moves"],
        "meet_kernel_ms": st_["meet_ms"],
        "plain_meet_kernel_ms": pl["meet_ms"],
        "max_abs_diff_vs_plain_estimate": max(diffs),
        "roofline": roofline(
            "k_meet<stratified> (fused walk + meet + weighted count)", st_["moves"],
            st_["meet_ms"] / 1e3,
            traffic=measured_traffic(os.path.join(ROOT, "profiles", "traffic_meet_stratified.json")),
            traffic_source="not measured in this run: profiles/traffic_meet_stratified.json"),
    }
    print(json.dumps(result))
    for ws in wss:
        ws.free()
    G.free()


def bench_tuples(args):
    """Algorithm 2's tuple form (decompose, sort, PREDECESSOR) on the medium
    graph: the workload's 8 sources in one call, and 32 sources (the 8 plus 24
    more, same seed and R), against the fused kernel on the same queries."""
    import numpy as np
    import torch

    from paper_2304_04015_amd import inputs
    from paper_2304_04015_amd import simrank as S

    cfg = dict(inputs.C2)
    torch.cuda.set_device(0)
    g = inputs.workload_graph(cfg)
    sources = [int(s) for s in inputs.sources_with_in_edges(g, 32, cfg["source_seed"])]
    G = S.load_csr(g)
    mk = lambda s: S.make_query(s, c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"],
                                seed=cfg["walk_seed"], walk_cap=cfg["L"])
    res = {}
    for k in (8, 32):
        qs = [mk(s) for s in sources[:k]]
        t0 = time.perf_counter()
        sums, st = S.simrank_tuple_meets(G, qs)
        el = time.perf_counter() - t0
        t1 = time.perf_counter()
        same = True
        for q in range(k):
            fused = S.simrank_single_source_ex(G, qs[q], want_out=False)[1]
            same &= bool(np.array_equal(sums[q], fused.astype(np.uint64)))
        fel = time.perf_counter() - t1
        res[k] = dict(seconds=el, device_ms=st.ms, tuples=st.moves, meets=st.meets,
                      queries_per_s=k / el, fused_queries_per_s=k / fel,
                      tuples_per_s=st.moves / (st.ms / 1e3), equal_to_fused=same,
                      sort_ms=st.meet_ms, sort_bytes=st.draws)
    r8 = res[8]
    # the radix sort dominates the call: its algorithmic bytes (8 per key a
    # histogram pass reads, 24 per tuple a scatter pass reads and writes) over
    # its passes' device time (HIP events on the call's stream)
    sort_gbs = r8["sort_bytes"] / (r8["sort_ms"] / 1e3) / 1e9
    result = {
        "metric": METRIC,
        "value": r8["tuples_per_s"],
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": 1e3 * r8["seconds"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "tuples: R-MAT n=2^20 (the medium graph); c=0.6 eps=0.02 R=9502 L=64; "
                        "Algorithm 2's tuple form for 8 and for 32 sources sharing the walks' key",
            "n": g.n, "m": g.m, "R": S.simrank_derive_params(mk(sources[0]), g.n).R,
        },
        "k8": res[8],
        "k32": res[32],
        "roofline": {
            "bound": "hbm",
            "kernel": "radix sort passes (k_rs_hist + k_rs_scatter), 8 sources",
            "achieved": sort_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": sort_gbs / HBM_PEAK_GBS,
            "traffic": None,
        },
    }
    print(json.dumps(result))
    G.free()


def bench_stitching(args):
    """Stitching workload: R-MAT n=2^24 (avg degree 16), segment pools sized by
    in-degree (kappa=1), 2^3-step segments, long walks of 64 steps by 3 pointer-
    doubling rounds; then one stitched single-source query at eps=0.02.  Prints
    one JSON line with the index build and the query."""
    import numpy as np
    import torch

    from paper_2304_04015_amd import inputs
    from paper_2304_04015_amd import simrank as S

    cfg = dict(inputs.C3)
    if args.scale:
        cfg["scale"] = args.scale
    torch.cuda.set_device(0)
    copy_probe(args)
    t0 = time.time()
    g = inputs.workload_graph(cfg)
    print(f"# graph n={g.n} m={g.m} generated in {time.time() - t0:.1f}s", file=sys.stderr)
    t_load = time.perf_counter()
    G = S.load_csr(g)
    load_s = time.perf_counter() - t_load
    builds = []
    for _ in range(max(1, args.steps)):
        builds.append(S.simrank_build_index(G, seg_log2=cfg["seg_log2"], kappa=cfg["kappa"],
                                            c=cfg["c"], seed=cfg["index_seed"]))
    info = builds[-1]
    s = int(inputs.sources_with_in_edges(g, 1, cfg["source_seed"])[0])
    q = S.make_query(s, c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"], seed=cfg["walk_seed"],
                     walk_cap=cfg["L"], mode=S.MODE_STITCHED)
    R = S.simrank_derive_params(q, g.n).R
    ws = S.simrank_workspace_create(G, R, cfg["L"])
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    cnt = torch.empty(g.n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    S.simrank_single_source_async(G, q, ws, out, cnt, stream)       # warm-up
    st0 = S.simrank_workspace_stats(ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.simrank_single_source_async(G, q, ws, out, cnt, stream)
    st = S.simrank_workspace_stats(ws)
    torch.cuda.synchronize()
    qs = time.perf_counter() - t1
    assert st.moves == st0.moves
    # the same source with plain walks (no index), and the machine's random
    # 8-byte gather rate over a buffer of the graph's size (HBM-bound here)
    qp = S.make_query(s, c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"], seed=cfg["walk_seed"],
                      walk_cap=cfg["L"])
    S.simrank_single_source_async(G, qp, ws, out, cnt, stream)
    stp = S.simrank_workspace_stats(ws)
    gi = G.info()
    footprint = 8 * (gi["m"] + gi["n"] - gi["n_active"])
    gather = S.simrank_roofline_gather(footprint, 8, dependent=False)
    build_ms = float(np.mean([b["build_ms"] for b in builds]))
    seg_ms = float(np.mean([b["segments_ms"] for b in builds]))
    dbl_ms = float(np.mean([b["doubling_ms"] for b in builds]))
    nseg = info["segments"]
    seg_len = 1 << cfg["seg_log2"]
    # algorithmic bytes: a segment walk's moves (12 B each) and its row, length
    # and successor (4 * 2^k + 1 + 4 B); a doubling round reads one random
    # 4-byte successor and copies 4 * 2^r bytes of chain per slot
    seg_bytes = BYTES_PER_MOVE * info["build_moves"] + nseg * (4 * seg_len + 5)
    dbl_bytes = sum(nseg * (4 + 4 + 4 * (1 << r) * 2) for r in range(info["levels"]))
    walk_steps = st.moves + st.tail_steps + st.source_moves
    steps_per_s = (st.moves + st.tail_steps) / (st.meet_ms / 1e3)
    result = {
        "metric": METRIC,
        "value": walk_steps / qs,
        "unit": "walk-steps/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": 1e3 * qs,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"stitching: R-MAT n=2^{cfg['scale']}, 16n edge draws, dedup, "
                               "permuted; kappa=1, 2^3-step segments, 3 doubling rounds; "
                               "c=0.6 eps=0.02 delta=1e-3 R=9502 L=64; one stitched query",
                   "n": g.n, "m": g.m, "R": R},
        "queries_per_s": 1.0 / qs,
        "index": {
            "segments": info["segments"], "bytes": info["bytes"], "levels": info["levels"],
            "build_ms": build_ms, "build_moves": info["build_moves"],
            "segments_per_s": info["segments"] / (build_ms * 1e-3),
            "build_moves_per_s": info["build_moves"] / (build_ms * 1e-3),
            "graph_load_s": load_s,
            "segments_kernel": {
                "ms": seg_ms,
                "traffic": measured_traffic(STITCH_TRAFFIC, f"k_segments<{SEG_SLOTS}, {seg_len}>")
                if cfg["seg_log2"] == 3 and args.scale == 0 else None,
                "moves_per_s": info["build_moves"] / (seg_ms * 1e-3),
                "moves_vs_random_gather": info["build_moves"] / (seg_ms * 1e-3) / gather["per_s"],
                "achieved_GBps": seg_bytes / (seg_ms * 1e-3) / 1e9,
                "frac": seg_bytes / (seg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            },
            "doubling_kernels": {
                "ms": dbl_ms,
                "traffic_per_round": measured_traffic(STITCH_TRAFFIC, "k_double")
                if args.scale == 0 else None,
                "rounds": info["levels"],
                "achieved_GBps": dbl_bytes / (dbl_ms * 1e-3) / 1e9 if dbl_ms > 0 else 0.0,
                "frac": dbl_bytes / (dbl_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if dbl_ms > 0 else 0.0,
            },
        },
        "query": {"moves": st.moves, "tail_steps": st.tail_steps, "draws": st.draws,
                  "meet_ms": st.meet_ms, "ms": st.ms, "pairs_walked": st.pairs_walked},
        "plain_query": {"moves": stp.moves, "meet_ms": stp.meet_ms, "ms": stp.ms},
        "roofline": roofline("k_meet<stitched> (fused walk + meet + count)",
                             st.moves + st.tail_steps, st.meet_ms / 1e3,
                             traffic=measured_traffic(STITCH_TRAFFIC, "k_meet<1, 2, false>"),
                             traffic_source="not measured in this run: bytes per launch from "
                                            "rocprofv3 FETCH_SIZE and WRITE_SIZE, "
                                            "profiles/traffic_stitching_rmat24.json",
                             bound="random-gather (HBM: the graph exceeds the Infinity Cache)"),
        "measured_roofs": {"footprint_bytes": footprint,
                           "random_gather_8B_per_s": gather["per_s"],
                           "kernel_steps_per_s": steps_per_s,
                           "steps_vs_random_gather": steps_per_s / gather["per_s"]},
    }
    if args.tune_index:
        # segment-length tuner: the index built with k = 2, 3, 4, the same
        # stitched query timed on each; the fastest index is left built
        choice, ms_k = S.simrank_tune_index(G, q, seg_log2=(2, 3, 4), kappa=cfg["kappa"],
                                            c=cfg["c"], seed=cfg["index_seed"])
        result["index_tuner"] = {"seg_log2": [2, 3, 4], "meet_ms": ms_k, "choice": choice}
    print(json.dumps(result))
    ws.free()
    G.free()


def bench_batching(args):
    """Batching workload: 16 R-MAT graphs with n = floor(2^U(12,22)) and average
    degree U{8..32}; queries with a uniform graph, a source drawn uniformly among
    its nodes with in-edges, eps from {0.05, 0.02, 0.01}, delta = 1e-3, L = 64 and
    a seed of their own (--shared-seed: one seed per graph).  The same queries
    run (a) one at a time through the asynchronous single-query call on one
    stream and (b) as one captured batch plan; both after the unit-size tuner
    has run once per graph.  With shared seeds the plan runs the queries of a
    graph as groups that walk each (v, j) once for all of them, and (c) the
    same plan without groups is timed as well."""
    import numpy as np
    import torch

    from paper_2304_04015_amd import inputs
    from paper_2304_04015_amd import simrank as S

    cfg = inputs.C4
    torch.cuda.set_device(0)
    t0 = time.time()
    specs = inputs.batch_graph_specs(cfg)
    gs = [inputs.batch_graph(sp) for sp in specs]
    print(f"# {len(gs)} graphs, {sum(g.m for g in gs)} edges, generated in "
          f"{time.time() - t0:.1f}s", file=sys.stderr)
    Gs = [S.load_csr(g) for g in gs]
    rng = np.random.default_rng(cfg["mix_seed"] + 1)
    queries = []
    for i in range(args.queries):
        gi = int(rng.integers(0, len(gs)))
        act = np.nonzero(gs[gi].in_degree() > 0)[0]
        eps = float(rng.choice(cfg["eps_choices"]))
        seed = 0x2304040150000400 + (0x1000 + gi if args.shared_seed else i)
        queries.append(S.make_query(int(rng.choice(act)), c=cfg["c"], eps=eps, delta=cfg["delta"],
                                    seed=seed, walk_cap=cfg["L"], graph=gi))
    tuned = []
    for gi, G in enumerate(Gs):
        act = np.nonzero(gs[gi].in_degree() > 0)[0]
        tq = S.make_query(int(act[0]), c=cfg["c"], eps=0.02, delta=cfg["delta"], walk_cap=cfg["L"])
        tuned.append(S.simrank_tune_ex(G, tq))
    # (a) one query at a time
    maxR = [1] * len(Gs)
    for q in queries:
        maxR[q.graph] = max(maxR[q.graph], S.simrank_derive_params(q, gs[q.graph].n).R)
    wss = [S.simrank_workspace_create(G, maxR[i], cfg["L"]) for i, G in enumerate(Gs)]
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g in gs]
    cnts = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in gs]
    stream = torch.cuda.Stream()
    check = {}
    walk_steps = 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i, q in enumerate(queries):
        S.simrank_single_source_async(Gs[q.graph], q, wss[q.graph], outs[q.graph], cnts[q.graph],
                                      stream)
        if i % 64 == 0:     # keep a few results to compare with the batch
            stream.synchronize()
            check[i] = cnts[q.graph].cpu().numpy().view(np.uint32).copy()
    stream.synchronize()
    t_plain = time.perf_counter() - t1
    # (b) the batch
    plan = S.BatchPlan(Gs, queries)
    plan.run(stream)
    plan.wait()                                             # warm-up run
    t2 = time.perf_counter()
    plan.run(stream)
    st = plan.wait()
    t_batch = time.perf_counter() - t2
    same = all(np.array_equal(plan.read(i, want_out=False)[1], c) for i, c in check.items())
    walk_steps = st.moves + st.tail_steps + st.source_moves
    nq = len(queries)
    flat = None
    if plan.n_groups:   # (c) the same plan without groups
        fplan = S.BatchPlan(Gs, queries, groups=False)
        fplan.run(stream)
        fplan.wait()
        t3 = time.perf_counter()
        fplan.run(stream)
        fst = fplan.wait()
        t_flat = time.perf_counter() - t3
        fsame = all(np.array_equal(fplan.read(i, want_out=False)[1], plan.read(i, want_out=False)[1])
                    for i in range(0, nq, 7))
        flat = {"queries_per_s": nq / t_flat, "ms": 1e3 * t_flat,
                "walk_steps": fst.moves + fst.tail_steps + fst.source_moves,
                "results_equal_grouped": fsame}
        fplan.free()
    # per graph: up to 4 of its queries alone (untimed above), the meet kernel's
    # moves per second and algorithmic bytes (8 B per move) against the HBM peak
    per_graph = []
    for gi, G in enumerate(Gs):
        mine = [q for q in queries if q.graph == gi][:4]
        moves = ms = 0.0
        for q in mine:
            S.simrank_single_source_async(G, q, wss[gi], outs[gi], cnts[gi], stream)
            qs_ = S.simrank_workspace_stats(wss[gi])
            moves += qs_.moves
            ms += qs_.meet_ms
        rate = moves / (ms / 1e3) if ms > 0 else 0.0
        per_graph.append({"n": gs[gi].n, "m": gs[gi].m, "queries": sum(q.graph == gi for q in queries),
                          "unit_nodes": tuned[gi]["unit_nodes"],
                          "tile_walks": tuned[gi]["tile_walks"], "moves_per_s": rate,
                          "achieved_GBps": BYTES_PER_MOVE * rate / 1e9,
                          "frac": BYTES_PER_MOVE * rate / 1e9 / HBM_PEAK_GBS})
    result = {
        "metric": METRIC,
        "value": walk_steps / t_batch,
        "unit": "walk-steps/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": 1e3 * t_batch,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"batching: {nq} single-source queries over 16 R-MAT graphs "
                               "(n = 2^U(12,22), avg degree U{8..32}), eps in {.05,.02,.01}, "
                               "delta=1e-3, L=64; one captured batch" +
                               ("; one walk seed per graph (query groups)" if args.shared_seed
                                else "; one walk seed per query"),
                   "graphs": [{"n": g.n, "m": g.m} for g in gs], "queries": nq},
        "queries_per_s": nq / t_batch,
        "plain_queries_per_s": nq / t_plain,
        "batched_vs_plain": t_plain / t_batch,
        "batch_results_equal_plain": same,
        "groups": plan.n_groups,
        "ungrouped_batch": flat,
        "tuned": [{"unit_nodes": t["unit_nodes"], "tile_walks": t["tile_walks"]} for t in tuned],
        "batch": {"moves": st.moves, "draws": st.draws, "device_ms": st.ms, "pairs": st.pairs},
        "per_graph": per_graph,
    }
    # the meet kernels dominate the plan: 8 algorithmic bytes per move (the
    # gathered slot) over the plan's device time (HIP events around the
    # captured graph on its stream)
    result["roofline"] = roofline(
        ("k_meet_group and k_meet over the plan's queries" if plan.n_groups
         else "k_meet over all the plan's queries, one launch") + " (whole plan's device time)",
        st.moves + st.tail_steps, st.ms / 1e3)
    print(json.dumps(result))
    plan.free()
    for ws in wss:
        ws.free()
    for G in Gs:
        G.free()


def bench_grouped(args):
    """Grouped workload: the medium graph (R-MAT n=2^20, 16n edge draws) and
    --group-queries single-source queries with eps = 0.02, delta = 1e-3
    (R = 9,502), L = 64 and the medium workload's walk seed, as one captured
    batch plan in which they form one query group: each walk (v, j) is taken
    once for all sources.  A step is one run of the plan.  The same plan
    without groups is run once for comparison; results must be equal."""
    import numpy as np
    import torch

    from paper_2304_04015_amd import inputs
    from paper_2304_04015_amd import simrank as S

    cfg = inputs.C2
    torch.cuda.set_device(0)
    copy_probe(args)
    g = inputs.workload_graph(cfg)
    G = S.load_csr(g)
    nq = args.group_queries
    strat = args.group_kind == "stratified"
    srcs = [int(x) for x in inputs.sources_with_in_edges(g, nq, cfg["source_seed"])]
    if strat:
        qs = [S.make_stratified_query(s, c=cfg["c"], eps=cfg["eps"], seed=cfg["walk_seed"])
              for s in srcs]
        R = S.simrank_derive_stratified(qs[0], g.n).N
    else:
        qs = [S.make_query(s, c=cfg["c"], eps=cfg["eps"], delta=cfg["delta"], seed=cfg["walk_seed"],
                           walk_cap=cfg["L"]) for s in srcs]
        R = S.simrank_derive_params(qs[0], g.n).R
    plan = S.BatchPlan([G], qs)
    stream = torch.cuda.Stream()
    for _ in range(args.warmup):
        plan.run(stream)
        plan.wait()
    torch.cuda.synchronize()
    steps, moves, dev_ms = args.steps, 0, 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(stream)
        st = plan.wait()
        moves += st.moves + st.source_moves
        dev_ms += st.ms
    dt = time.perf_counter() - t0
    def res(p, i):
        return p.read_stratified(i)[2] if strat else p.read(i, want_out=False)[1]
    grouped = [res(plan, i) for i in range(nq)]
    flat = S.BatchPlan([G], qs, groups=False)
    flat.run(stream)
    fst = flat.wait()
    same = all(np.array_equal(res(flat, i), grouped[i]) for i in range(nq))
    lone = np.array_equal(S.simrank_single_source_stratified(G, qs[0])[2] if strat else
                          S.simrank_single_source_ex(G, qs[0])[1], grouped[0])
    kernel_s = (dev_ms / steps) / 1e3
    result = {
        "metric": METRIC,
        "value": moves / dt,
        "unit": "walk-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"grouped: medium graph (R-MAT n=2^20, 16n edge draws), {nq} "
                               "single-source queries with one walk seed, eps=0.02 delta=1e-3 " +
                               (f"stratified (N={R}), one captured batch plan forming "
                                f"{plan.n_groups} query groups of up to 8" if strat else
                                f"R={R} L=64, one captured batch plan forming one query group"),
                   "n": g.n, "m": g.m, "R": R, "L": cfg["L"], "queries": nq,
                   "groups": plan.n_groups},
        "queries_per_s": nq * steps / dt,
        "ungrouped_queries_per_s": nq / (fst.ms / 1e3),
        "grouped_vs_ungrouped": (fst.ms / 1e3) / (dt / steps),
        "moves_per_query": st.moves / nq,
        "moves_per_query_ungrouped": fst.moves / nq,
        "results_equal_ungrouped": same,
        "first_equals_lone_query": lone,
        "roofline": roofline(
            ("k_meet_group<2, 2, 2>" if strat else "k_meet_group<2, 8, 0>") +
            " (whole plan's device time)", st.moves, kernel_s,
            traffic=None if strat else
            measured_traffic(os.path.join(ROOT, "profiles", "traffic_meet_grouped.json")),
            traffic_source=None if strat else
            "not measured in this run: profiles/traffic_meet_grouped.json"),
    }
    print(json.dumps(result))
    plan.free()
    flat.free()
    G.free()


def bench_serving(args):
    """Serving workload: R-MAT n=2^22, avg degree 16, graph and stitched segment
    index resident in HBM (segment length 2^k chosen among k = 2, 3, 4 by the
    segment-length tuner, then nodes per unit and walks per tile by the tuner).
    Requests: sources drawn proportionally to in-degree, eps uniform in
    {0.05, 0.02}, delta = 1e-3, L = 64, stitched walks, a walk seed per
    request.  First the plain capacity (requests back to back, one at a time,
    each estimate copied to the host); then Poisson arrivals at 0.5, 0.8, 1.0,
    1.2, 1.5 and 2 times that rate into the continuous-batching server (at most
    16 requests in flight): achieved queries/s and p50 / p99 latency per
    level.  --group-max G: the requests share one walk seed and the server
    admits those waiting together as query groups of up to G; offered loads
    0.5 to 4 times the plain capacity."""
    import numpy as np
    import torch

    from paper_2304_04015_amd import inputs
    from paper_2304_04015_amd import simrank as S

    cfg = dict(inputs.C5)
    if args.scale:
        cfg["scale"] = args.scale
    torch.cuda.set_device(0)
    t0 = time.time()
    g = inputs.workload_graph(cfg)
    print(f"# graph n={g.n} m={g.m} generated in {time.time() - t0:.1f}s", file=sys.stderr)
    G = S.load_csr(g)
    rng = np.random.default_rng(31)
    deg = g.in_degree().astype(np.float64)

    strat = args.served_mode == "stratified"

    def make(i):
        s = int(rng.choice(g.n, p=deg / deg.sum()))
        seed = 0x2304040150000500 + (0 if args.group_max >= 2 else i)
        eps = float(rng.choice(cfg["eps_choices"]))
        if strat:                       # Algorithm 2's z and Algorithm 1's cap
            return S.make_stratified_query(s, c=cfg["c"], eps=eps, seed=seed)
        return S.make_query(s, c=cfg["c"], eps=eps, delta=cfg["delta"], seed=seed,
                            walk_cap=cfg["L"],
                            mode=S.MODE_STITCHED if args.served_mode == "stitched"
                            else S.MODE_PLAIN)

    # the index's segment length and the work partition, chosen by the tuners
    # on one request of the workload (the index left built is the fastest one)
    s0 = int(rng.choice(g.n, p=deg / deg.sum()))
    _ = rng.choice(cfg["eps_choices"])        # the draws of one request, as make() takes them
    tq = S.make_query(s0, c=cfg["c"], eps=0.02, delta=cfg["delta"], seed=0x2304040150000500,
                      walk_cap=cfg["L"], mode=S.MODE_STITCHED)   # the larger R of the mix;
                                                                  # stitched for the index tuner
    index_choice, index_ms = S.simrank_tune_index(G, tq, seg_log2=(2, 3, 4), kappa=1.0,
                                                  c=cfg["c"], seed=0x2304040150000023)
    # the unit / tile tuner times plain or stitched queries (stratified
    # requests keep the graph's default partition)
    tq.mode = S.MODE_STITCHED if args.served_mode == "stitched" else S.MODE_PLAIN
    tuning = S.simrank_tune_ex(G, tq) if not strat else {}
    # the largest R (stratified: N) and cap of the mix size the workspace and the server
    if strat:
        sps = [S.simrank_derive_stratified(S.make_stratified_query(0, c=cfg["c"], eps=e), g.n)
               for e in cfg["eps_choices"]]
        max_R, max_L = max(p.N for p in sps), max(p.phi for p in sps)
    else:
        max_R, max_L = 9502, cfg["L"]
    # the requests: one list, replayed one at a time (the plain capacity) and
    # into the server at every load, so that every rate covers the same work
    warm = [make(i) for i in range(2)]
    cap_q = [make(1000 + i) for i in range(args.requests)]
    ws = S.simrank_workspace_create(G, max_R, max_L)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    cnt = torch.empty(g.n, dtype=torch.int32, device="cuda")
    out_n = torch.empty(g.n, dtype=torch.float64, device="cuda") if strat else None
    wsum = torch.empty(g.n, dtype=torch.int64, device="cuda") if strat else None
    stream = torch.cuda.Stream()

    def run_lone(q):
        if strat:
            S.simrank_stratified_async(G, q, ws, out, out_n, wsum, stream)
        else:
            S.simrank_single_source_async(G, q, ws, out, cnt, stream)
        return S.simrank_workspace_stats(ws)

    for q in warm:
        run_lone(q)
    t1 = time.perf_counter()
    steps = 0
    kmoves, kms = 0, 0.0
    lone_counts = []
    for i, q in enumerate(cap_q):
        st = run_lone(q)
        steps += st.moves + st.tail_steps + st.source_moves
        kmoves += st.moves + st.tail_steps
        kms += st.meet_ms
        _ = out.cpu()                       # results to host, as a served request has
        if strat:
            _ = out_n.cpu()
        if i < 4:
            lone_counts.append(wsum.cpu().numpy().view(np.uint64).copy() if strat
                               else cnt.cpu().numpy().view(np.uint32).copy())
    plain_s = time.perf_counter() - t1
    capacity = len(cap_q) / plain_s
    plain_steps_per_s = steps / plain_s
    ws.free()
    gi = G.info()
    footprint = 8 * (gi["m"] + gi["n"] - gi["n_active"])
    gather = S.simrank_roofline_gather(footprint, 8, dependent=False)
    kernel_rate = kmoves / (kms / 1e3)
    grouped = args.group_max >= 2
    srv = S.Server(G, max_slots=max(16, args.group_max), max_R=max_R, max_L=max_L,
                   group_max=args.group_max)
    levels = []
    served_equal = True
    for load in ((0.5, 1.0, 2.0, 3.0, 4.0, "burst") if grouped else
                 (0.5, 0.8, 1.0, 1.2, 1.5, 2.0, "burst")):
        # "burst": every request submitted at once (the server's saturated rate)
        qps = float("inf") if load == "burst" else load * capacity
        reqs = cap_q
        gaps = np.zeros(len(reqs)) if load == "burst" else rng.exponential(1.0 / qps, size=len(reqs))
        tickets = []
        t_start = time.perf_counter()
        t_next = t_start
        for q, gap in zip(reqs, gaps):
            t_next += gap
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(q))
        lat, qwait, wsteps = [], [], 0
        for i, t in enumerate(tickets):
            if strat:
                _, _, c, info = srv.wait_stratified(t, timeout_s=300.0)
                c = c if i < len(lone_counts) else None
            else:
                _, c, info = srv.wait(t, timeout_s=300.0, want_counts=i < len(lone_counts))
            if c is not None:
                served_equal &= bool(np.array_equal(c, lone_counts[i]))
            lat.append(info.latency_s)
            qwait.append(info.queue_s)
            wsteps += info.stats.moves + info.stats.tail_steps + info.stats.source_moves
        t_end = time.perf_counter()
        levels.append({"load": load, "offered_qps": qps if load != "burst" else None,
                       "arrivals_qps": (len(reqs) / float(np.sum(gaps))) if load != "burst"
                       else None,
                       "achieved_qps": len(reqs) / (t_end - t_start),
                       "served_vs_plain": len(reqs) / (t_end - t_start) / capacity,
                       "walk_steps_per_s": wsteps / (t_end - t_start),
                       "p50_latency_s": float(np.percentile(lat, 50)),
                       "p99_latency_s": float(np.percentile(lat, 99)),
                       "mean_queue_s": float(np.mean(qwait))})
        print(f"# load {load}: {levels[-1]}", file=sys.stderr)
    top = levels[-1]
    result = {
        "metric": METRIC,
        "value": top["walk_steps_per_s"],
        "unit": "walk-steps/s",
        "n_gpus": 1, "steps": len(levels), "warmup": len(warm),
        "ms_per_step": 1e3 * args.requests / top["achieved_qps"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"serving: R-MAT n=2^{cfg['scale']}, avg degree 16, index "
                               f"resident; sources by in-degree, eps in {{.05,.02}}, {args.served_mode}; " +
                               (f"one walk seed, query groups of up to {args.group_max}; Poisson "
                                "arrivals at 0.5-4x plain capacity; "
                                f"{max(16, args.group_max)} requests in flight at most" if grouped
                                else "a seed per request; Poisson arrivals at 0.5-2x plain "
                                "capacity; continuous batching, 16 requests in flight at most"),
                   "n": g.n, "m": g.m, "requests_per_level": args.requests,
                   "group_max": args.group_max},
        "queries_per_s": top["achieved_qps"],
        "plain_queries_per_s": capacity,
        "served_vs_plain": top["achieved_qps"] / capacity,
        "served_vs_plain_by_load": {str(lv["load"]): lv["served_vs_plain"] for lv in levels},
        "plain_walk_steps_per_s": plain_steps_per_s,
        "served_results_equal_lone": served_equal,
        "levels": levels,
        "server_counts": srv.counts(),
        "server_load": srv.load(),
        "index_tuner": {"seg_log2": [2, 3, 4], "meet_ms": index_ms, "choice": index_choice},
        "tuning": tuning,
        "roofline": roofline(f"k_meet<{args.served_mode}> (fused walk + meet + count), "
                             "requests one at a time",
                             kmoves, kms / 1e3),
        "measured_roofs": {"footprint_bytes": footprint,
                           "random_gather_8B_per_s": gather["per_s"],
                           "kernel_steps_per_s": kernel_rate,
                           "steps_vs_random_gather": kernel_rate / gather["per_s"]},
    }
    print(json.dumps(result))
    srv.destroy()
    G.free()


if __name__ == "__main__":
    main()
