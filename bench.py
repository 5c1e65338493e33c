"""Benchmark: single-source ProbeSim queries/s on one MI355X.

Workload: directed Chung-Lu power-law graph, 1M nodes, 10M edges, in/out
exponent 2.1 (synthetic stand-in for the paper's social/web graphs); 32 query
nodes drawn uniformly from the nodes with in-edges; c = 0.6, eps = 0.05,
delta = 0.01; walk seed 3 + query index.  One step = the 32 queries run one at
a time through ps_single_source (plain mode), every stage on the GPU, inputs
resident in HBM, estimates written to a device tensor.  The same 32 queries
are also timed as one ps_batch launch (batched mode).

Prints one JSON line.  The roofline entry covers the PROBE expansion kernel
(k_expand), timed with HIP events on the stream it runs on; its algorithmic
bytes per launch come from the kernel's own work counters (expand_bytes).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "cl_1m_10m"
C, EPS, DELTA = 0.6, 0.05, 0.01
NQ = 32
HYBRID_C0 = 0.003  # switch constant of Section 4.4 for the hybrid pass (the library's default)


def expand_bytes(st: dict) -> float:
    """Algorithmic bytes moved by k_expand for the given work counters:
    28 B per expanded entry (list entry 8, scaled score 4, row start/len 8,
    clearing its 8-byte grid sum),
    8 B per pushed out-edge (neighbour id 4, 1/|I(v)| 4; levels moved to the
    dense pass or switched are not pushed),
    16 B per inner-level contribution (64-bit grid sum read-modify-write),
    8 B per new next-level entry (list write),
    16 B per final contribution (FP64 estimate read-modify-write)."""
    F, E = st["entries_expanded"], st["pushed_edges"]
    N, Fin = st["next_entries"], st["pushed_final_adds"]
    inner = max(E - Fin, 0)
    return 28.0 * F + 8.0 * E + 16.0 * inner + 8.0 * N + 16.0 * Fin


def measured_traffic(avg_ms):
    """HBM bytes per k_expand dispatch from the committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE scaled by a copy-kernel calibration),
    used only while the kernel source is the one they were taken on; as GB/s
    over this run's average launch time.  None otherwise."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_expand_cl_1m_10m_traffic.json")
    if not os.path.exists(path) or avg_ms <= 0:
        return None, None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None, None
    b = rec["hbm_bytes_per_dispatch"]
    return b / (avg_ms * 1e-3) / 1e9, b


def cpu_baseline(n, s, d, q, seconds_target=15.0, threads=None):
    """The oracle (Alg. 1, FP64) on the host cores over a bounded sample: the
    first walks of the first query in chunks of 20, shared by `threads`
    worker threads (the oracle releases the GIL), for about seconds_target of
    wall time; scaled to queries/s by n_r (Alg. 1's cost is a sum of
    independent per-walk costs)."""
    import threading

    import oracle

    G = oracle.Graph(n, s, d)
    p = oracle.params(n, C, EPS, DELTA)
    u = int(q[0])
    threads = threads or max(1, min(16, os.cpu_count() or 1))
    chunk = 20
    lock = threading.Lock()
    state = {"next": 0, "walks": 0}
    t0 = time.perf_counter()

    def worker():
        while time.perf_counter() - t0 < seconds_target:
            with lock:
                k = state["next"]
                if k >= p.n_r:
                    return
                state["next"] = min(k + chunk, p.n_r)
            oracle.single_source(G, u, p, 3, k, min(k + chunk, p.n_r))
            with lock:
                state["walks"] += min(k + chunk, p.n_r) - k

    ts = [threading.Thread(target=worker) for _ in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    wall = time.perf_counter() - t0
    walks = state["walks"]
    return {"value": walks / wall / p.n_r, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"Alg. 1 oracle, query node {u}, {walks} of its n_r = {p.n_r} walks in chunks of {chunk} "
                      f"on {threads} threads, {wall:.1f} s, scaled by n_r / {walks}"}


def served(ps, G, q, n, seconds=8.0, rate_frac=0.5, seed=7, **defaults):
    """Continuous-batching server on the same graph and queries: closed-loop
    saturation throughput X_sat (all queries submitted at once), then
    open-loop Poisson arrivals at rate_frac * X_sat; latency is submit to
    result on the host.  defaults: options every served query runs with."""
    import threading

    import numpy as np

    srv = ps.Server(G, max_inflight=32, **defaults)
    try:
        t0 = time.perf_counter()
        ts = [srv.submit(int(u), C, EPS, DELTA, 1000 + i) for i, u in enumerate(q)]
        for t in ts:
            srv.wait(t)
        x_sat = len(q) / (time.perf_counter() - t0)
        rate = rate_frac * x_sat
        rng = np.random.default_rng(seed)
        count = max(16, int(rate * seconds))
        gaps = rng.exponential(1.0 / rate, size=count)
        lat = [None] * count
        lock = threading.Lock()
        pending = []

        def waiter(i, ticket, t_sub):
            srv.wait(ticket)
            with lock:
                lat[i] = time.perf_counter() - t_sub

        start = time.perf_counter()
        due = start
        for i in range(count):
            due += gaps[i]
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            u = int(q[i % len(q)])
            t_sub = time.perf_counter()
            tk = srv.submit(u, C, EPS, DELTA, 2000 + i)
            th = threading.Thread(target=waiter, args=(i, tk, t_sub))
            th.start()
            pending.append(th)
        for th in pending:
            th.join()
        wall = time.perf_counter() - start
        l = np.array(lat) * 1e3
        return {"x_sat_qps": x_sat, "offered_qps": rate, "served_qps": count / wall, "queries": count,
                "p50_ms": float(np.percentile(l, 50)), "p99_ms": float(np.percentile(l, 99))}
    finally:
        srv.stop()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the plain-versus-batched passes at eps = 0.1")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the passes with randomized PROBE and with the switch of Section 4.4")
    ap.add_argument("--hybrid-c0", type=float, default=HYBRID_C0)
    ap.add_argument("--probe-mode", choices=["deterministic", "randomized", "hybrid"], default="deterministic",
                    help="probe of the one-at-a-time and batched passes (the metric is quoted with deterministic PROBE)")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the passes with the error split tuned by measurement (Theorem 2)")
    ap.add_argument("--nq", type=int, default=NQ, help="query nodes per step (the workload uses 32)")
    ap.add_argument("--pull", type=int, default=0, help="pull threshold in out-edges (0 automatic, -1 never)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="also run a device-to-device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(queries would shard across GPUs by data parallelism over a replicated graph)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1709_06955_amd as ps
    from synth import graphs

    n, s, d = graphs.make_workload(WORKLOAD)
    q = graphs.query_nodes(n, d, NQ)[: args.nq]
    print(f"graph ready: n={n} m={s.size}", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    ctx = ps.Context(0, stream=stream)
    G = ps.Graph(ctx, n, s, d)
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    tune = None
    if not args.no_autotune and not args.slots and not args.pull:
        # launch settings only (results do not depend on them); outside the timed region
        t0 = time.perf_counter()
        tune = ps.ps_autotune(G, graphs.query_nodes(n, d, 2, seed=99), C, EPS, DELTA)
        tune["seconds"] = time.perf_counter() - t0
        print(f"autotune: {tune}", file=sys.stderr, flush=True)
    ctx.set_timing(True)

    mode_kw = {"deterministic": {}, "randomized": dict(probe_mode=ps.PROBE_RANDOMIZED),
               "hybrid": dict(probe_mode=ps.PROBE_HYBRID, hybrid_c0=args.hybrid_c0)}[args.probe_mode]

    def plain_step(acc, tag):
        for i, u in enumerate(q):
            ps.ps_single_source(G, int(u), C, EPS, DELTA, 3 + i, out=out, slots=args.slots, pull_edges=args.pull,
                                **mode_kw)
            st = ctx.stats()
            print(f"[{tag}] query {i} u={int(u)}: {st['total_ms']:.1f} ms, push {st['expand_ms']:.1f} ms + pull "
                  f"{st['pull_ms']:.1f} ms in {st['expand_launches']} steps, tree nodes {st['tree_nodes']}, "
                  f"edges {st['edges_scanned']}, entries {st['entries_expanded']}, next {st['next_entries']}, "
                  f"final {st['final_adds']}, pulled levels {st['pull_levels']} ({st['pull_edges']} in-edges)",
                  file=sys.stderr, flush=True)
            if i == 0 and tag != "warmup":
                tot = max(sum(st["level_hist_edges"]), 1)
                rows = [f"2^{b}:{c}/{100.0 * e / tot:.1f}%" for b, (c, e) in
                        enumerate(zip(st["level_hist_count"], st["level_hist_edges"])) if c]
                print("  level sizes (levels/edge share):", " ".join(rows), file=sys.stderr, flush=True)
            if acc is not None:
                for k in acc:
                    acc[k] += st[k]

    for _ in range(args.warmup):
        plain_step(None, "warmup")
    keys = ["expand_ms", "pull_ms", "pull_levels", "pull_edges", "expand_launches", "entries_expanded", "edges_scanned",
            "pushed_edges", "next_entries", "final_adds", "pushed_final_adds",
            "tree_nodes", "probe_levels", "steps", "walks", "entries_pruned"]
    acc = {k: 0 for k in keys}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step(acc, "timed")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    queries = len(q) * args.steps
    qps = queries / dt

    # Batched: the same 32 queries in one launch.
    outs = [(torch.empty(n, dtype=torch.float64, device="cuda:0"), None) for _ in range(len(q))]
    qlist = [dict(u=int(u), k=0, c=C, eps=EPS, delta=DELTA, seed=3 + i, **mode_kw) for i, u in enumerate(q)]
    ps.ps_batch(G, qlist, outs=outs, slots=args.slots, pull_edges=args.pull)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    ps.ps_batch(G, qlist, outs=outs, slots=args.slots, pull_edges=args.pull)
    torch.cuda.synchronize()
    batched_qps = len(q) / (time.perf_counter() - tb)
    print(f"batched: {batched_qps:.2f} queries/s", file=sys.stderr, flush=True)

    # Smaller queries (eps = 0.1, about a quarter of the walks): one query no
    # longer keeps every probe slot busy to its end, which batching recovers.
    small = None if args.no_small else {"eps": 0.1}
    qsmall = [dict(u=int(u), k=0, c=C, eps=0.1, delta=DELTA, seed=3 + i, **mode_kw) for i, u in enumerate(q)]
    for rep_ in range(0 if args.no_small else 2):  # the first pass is a warm-up
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for i, u in enumerate(q):
            ps.ps_single_source(G, int(u), C, 0.1, DELTA, 3 + i, out=outs[i][0], slots=args.slots, pull_edges=args.pull,
                                **mode_kw)
        torch.cuda.synchronize()
        small["plain_qps"] = len(q) / (time.perf_counter() - ts)
        ts = time.perf_counter()
        ps.ps_batch(G, qsmall, outs=outs, slots=args.slots, pull_edges=args.pull)
        torch.cuda.synchronize()
        small["batched_qps"] = len(q) / (time.perf_counter() - ts)
    if small is not None:
        small["batched_speedup"] = small["batched_qps"] / small["plain_qps"]
        print(f"eps 0.1: {small}", file=sys.stderr, flush=True)

    # The paper's other probes on the same queries, one pass each (reported
    # beside the metric, which is the deterministic path).
    variants = None
    if not args.no_variants:
        variants = {}
        for name, kw in (("randomized", dict(probe_mode=ps.PROBE_RANDOMIZED)),
                         ("hybrid", dict(probe_mode=ps.PROBE_HYBRID, hybrid_c0=args.hybrid_c0))):
            switched = probes = 0
            torch.cuda.synchronize()
            tv = time.perf_counter()
            for i, u in enumerate(q):
                ps.ps_single_source(G, int(u), C, EPS, DELTA, 3 + i, out=out, slots=args.slots, pull_edges=args.pull,
                                    **kw)
                st = ctx.stats()
                switched += st["switched_probes"]
                probes += st["tree_nodes"]
            torch.cuda.synchronize()
            v = {"qps": len(q) / (time.perf_counter() - tv)}
            if name == "hybrid":
                v.update(c0=args.hybrid_c0, switched_tree_nodes=switched / max(probes, 1))
            variants[name] = v
            print(f"{name}: {v}", file=sys.stderr, flush=True)

    # The error split of Theorem 2 tuned by measurement (another estimate with
    # the same guarantee; beside the metric, which uses the default split).
    split = None
    if not args.no_split:
        sample = graphs.query_nodes(n, d, 2, seed=99)
        t0 = time.perf_counter()
        tuned = ps.ps_tune_split(G, sample, C, EPS, DELTA)
        split = {"eps_s": tuned["eps_s"], "eps_t": tuned["eps_t"], "eps_p": tuned["eps_p"],
                 "n_r": ps.derive_params(n, C, EPS, DELTA, eps_s=tuned["eps_s"], eps_t=tuned["eps_t"],
                                         eps_p=tuned["eps_p"]).n_r,
                 "tune_seconds": time.perf_counter() - t0}
        kws = dict(eps_s=tuned["eps_s"], eps_t=tuned["eps_t"], eps_p=tuned["eps_p"], slots=args.slots,
                   pull_edges=args.pull)
        for name, kw in (("deterministic", {}),
                         ("hybrid", dict(probe_mode=ps.PROBE_HYBRID, hybrid_c0=args.hybrid_c0))):
            torch.cuda.synchronize()
            tv = time.perf_counter()
            for i, u in enumerate(q):
                ps.ps_single_source(G, int(u), C, EPS, DELTA, 3 + i, out=out, **kws, **kw)
            torch.cuda.synchronize()
            split[f"{name}_qps"] = len(q) / (time.perf_counter() - tv)
        print(f"tuned split: {split}", file=sys.stderr, flush=True)

    alg_bytes = expand_bytes(acc)
    launches = max(acc["expand_launches"], 1)
    avg_ms = acc["expand_ms"] / launches
    achieved = (alg_bytes / launches) / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic, traffic_bytes = measured_traffic(avg_ms)
    result = {
        "metric": "single-source queries/s at eps=0.05 (plain, one query at a time)" + (
            "" if args.probe_mode == "deterministic" else f", {args.probe_mode} PROBE"),
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 probes, f64 accumulation",
        "data": "synthetic (seeded Chung-Lu power-law graph; the paper's SNAP/LAW graphs are not available)",
        "config": {"workload": "Chung-Lu directed power-law graph, 1M nodes, 10M edges, exponent 2.1; "
                               "32 uniform query nodes with in-edges run one at a time; c=0.6, eps=0.05, "
                               "delta=0.01", "queries_per_step": len(q)},
        "autotune": tune,
        "batched_qps": batched_qps,
        "batched_speedup": batched_qps / qps,
        "small_queries": small,
        "probe_variants": variants,
        "tuned_split": split,
        "roofline": {"bound": "hbm", "kernel": "k_expand", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_ms": avg_ms, "alg_bytes_per_launch": alg_bytes / launches,
                     "hbm_bytes_per_launch": traffic_bytes},
        "work_per_query": {k: acc[k] / queries for k in keys if k not in ("expand_ms",)},
    }
    if args.calib_copy:
        a = torch.empty(args.calib_copy << 18, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"calibration copy: {args.calib_copy} MiB read + {args.calib_copy} MiB written", file=sys.stderr)
    if not args.no_served:
        result["served"] = served(ps, G, q, n)
        if split is not None:  # the same, every query with the tuned split and the switch of Section 4.4
            result["served_tuned"] = served(ps, G, q, n, eps_s=split["eps_s"], eps_t=split["eps_t"],
                                            eps_p=split["eps_p"], probe_mode=ps.PROBE_HYBRID,
                                            hybrid_c0=args.hybrid_c0)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(n, s, d, q)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
