"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module holds input generation only: graphs, query nodes and update
streams.  It contains none of ProbeSim's arithmetic (no walks, no probes, no
scores), so both sides can draw the same inputs without sharing method code.

The paper evaluates on public SNAP/LAW graphs (Section 6, Table 3: Wiki-Vote,
HepTh, AS, HepPh, LiveJournal, IT-2004, Twitter, Friendster).  None of them is
available here, so seeded synthetic graphs with the same character stand in:
a directed Erdos-Renyi graph for the small exact-ground-truth case and directed
Chung-Lu graphs with power-law in/out degrees for the large cases, with query
nodes drawn uniformly from the nodes of nonzero in-degree as in Section 6.1.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _rng(seed: int, stream: int) -> np.random.Generator:
    # numpy's Philox bit generator keyed by (seed, stream); only used to make
    # inputs, never by the method itself.
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def _unique_in_draw_order(keys: np.ndarray) -> np.ndarray:
    _, first = np.unique(keys, return_index=True)
    return keys[np.sort(first)]


def erdos_renyi(n: int, m: int, seed: int = 1):
    """Directed simple graph with m edges drawn uniformly (no self-loops,
    no multi-edges).  Returns (src, dst) int32 arrays sorted by (src, dst)."""
    if m > n * (n - 1):
        raise ValueError("too many edges for a simple digraph")
    rng = _rng(seed, 1)
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        draw = max(1024, int(need * 1.2) + 16)
        s = rng.integers(0, n, size=draw, dtype=np.int64)
        d = rng.integers(0, n, size=draw, dtype=np.int64)
        ok = s != d
        keys = _unique_in_draw_order(np.concatenate([keys, s[ok] * n + d[ok]]))
    keys = np.sort(keys[:m])
    return (keys // n).astype(np.int32), (keys % n).astype(np.int32)


def chung_lu_weights(n: int, m: int, gamma: float) -> np.ndarray:
    """Expected-degree weights w_i = (i+1)^(-1/(gamma-1)) scaled to sum m,
    clipped at d_max = min(n^(1/(gamma-1)), n/10) and renormalised twice."""
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    dmax = min(n ** (1.0 / (gamma - 1.0)), n / 10.0)
    w *= m / w.sum()
    for _ in range(2):
        np.minimum(w, dmax, out=w)
        w *= m / w.sum()
    return w


def chung_lu(n: int, m: int, gamma: float, seed: int = 1, progress=None):
    """Directed Chung-Lu graph: src ~ w_out, dst ~ w_in with independent
    seeded permutations of the same power-law weights; self-loops and
    duplicates rejected.  Draws about 10% more pairs than needed, keeps the
    distinct non-loop ones, tops up if short and drops a seeded uniform subset
    of the surplus to keep exactly m.  Returns (src, dst) int32 arrays sorted
    by (src, dst).

    Pairs are drawn in chunks of 2^22, each from its own Philox stream, so the
    chunks run on worker threads and the result does not depend on how many
    there are.  `progress` (optional) is called with a short message every
    64 chunks and after each merge, so that long generations report as they
    go."""
    rng = _rng(seed, 2)
    w = chung_lu_weights(n, m, gamma)
    w_out = np.empty(n)
    w_in = np.empty(n)
    w_out[rng.permutation(n)] = w
    w_in[rng.permutation(n)] = w
    cdf_out = np.cumsum(w_out)
    cdf_out /= cdf_out[-1]
    cdf_in = np.cumsum(w_in)
    cdf_in /= cdf_in[-1]
    del w_out, w_in
    step = 1 << 22

    def chunk(index, count):
        # Sorted uniforms make the inverse-CDF searches sequential; pairing the
        # sorted sources with a random permutation of the targets gives the
        # same distribution as independent pairs.
        r = _rng(seed, (1 << 20) + index)
        src = np.searchsorted(cdf_out, np.sort(r.random(count)), side="right")
        dst = np.searchsorted(cdf_in, np.sort(r.random(count)), side="right")[r.permutation(count)]
        np.minimum(src, n - 1, out=src)
        np.minimum(dst, n - 1, out=dst)
        k = src.astype(np.int64) * n + dst
        if progress is not None and index % 64 == 63:
            progress(f"chung_lu: chunk {index + 1} drawn")
        return k[src != dst]

    next_chunk = 0

    def draw(count):
        nonlocal next_chunk
        sizes = [min(step, count - a) for a in range(0, count, step)]
        ids = range(next_chunk, next_chunk + len(sizes))
        next_chunk += len(sizes)
        workers = max(1, min(16, os.cpu_count() or 1, len(sizes)))
        with ThreadPoolExecutor(workers) as ex:
            return np.concatenate(list(ex.map(chunk, ids, sizes)))

    keys = np.unique(draw(int(m * 1.1) + 1024))
    if progress is not None:
        progress(f"chung_lu: {keys.size} distinct pairs")
    while keys.size < m:
        keys = np.unique(np.concatenate([keys, draw(int((m - keys.size) * 2) + 1024)]))
    if keys.size > m:
        drop = np.ones(keys.size, dtype=bool)
        drop[rng.choice(keys.size, size=keys.size - m, replace=False)] = False
        keys = keys[drop]
    return (keys // n).astype(np.int32), (keys % n).astype(np.int32)


def in_degrees(n: int, dst: np.ndarray) -> np.ndarray:
    return np.bincount(dst, minlength=n).astype(np.int64)


def query_nodes(n: int, dst: np.ndarray, count: int, seed: int = 2) -> np.ndarray:
    """Query nodes drawn uniformly (without replacement) from the nodes of
    nonzero in-degree, as the paper's experiments do (Sections 6.1 and 6.2)."""
    rng = _rng(seed, 3)
    cand = np.nonzero(in_degrees(n, dst) > 0)[0]
    count = min(count, cand.size)
    return np.sort(rng.choice(cand, size=count, replace=False)).astype(np.int32)


def stratified_query_nodes(n: int, dst: np.ndarray, count: int, seed: int = 2) -> np.ndarray:
    """Query nodes stratified by floor(log2(in-degree)): equal share per
    bucket (remainder spread over the first buckets), uniform inside one."""
    rng = _rng(seed, 4)
    deg = in_degrees(n, dst)
    nz = np.nonzero(deg > 0)[0]
    bucket = np.floor(np.log2(deg[nz])).astype(np.int64)
    buckets = [nz[bucket == b] for b in np.unique(bucket)]
    share = [count // len(buckets)] * len(buckets)
    for i in range(count - sum(share)):
        share[i % len(buckets)] += 1
    out = []
    spill = 0
    for b, s in zip(buckets, share):
        take = min(b.size, s + spill)
        spill = s + spill - take
        out.append(rng.choice(b, size=take, replace=False))
    q = np.concatenate(out)
    if spill:
        rest = np.setdiff1d(nz, q)
        q = np.concatenate([q, rng.choice(rest, size=min(spill, rest.size), replace=False)])
    return rng.permutation(q).astype(np.int32)


def update_stream(n: int, src: np.ndarray, dst: np.ndarray, count: int, seed: int = 5):
    """Edge updates: half uniform inserts of absent non-self-loop edges, half
    deletes of live edges (uniform over the live set), interleaved in a
    seeded order.  Each update is valid against the edge set produced by the
    updates before it.  Membership in the base graph is a binary search of its
    sorted keys, so the cost does not grow with m beyond one sort.
    Returns (src, dst, op) with op 0 = insert, 1 = delete."""
    rng = _rng(seed, 5)
    base = np.sort(src.astype(np.int64) * n + dst.astype(np.int64))

    def in_base(key):
        i = int(np.searchsorted(base, key))
        return i < base.size and int(base[i]) == key

    deleted = set()  # base edges deleted so far
    added = []  # inserted edges, in insertion order
    added_live = {}  # live inserted edge -> its position in added
    ops = rng.permutation(np.repeat(np.array([0, 1], dtype=np.uint8), [count - count // 2, count // 2]))
    us = np.empty(count, np.int32)
    ud = np.empty(count, np.int32)
    for t, op in enumerate(ops):
        if op == 0:
            while True:
                a, b = (int(x) for x in rng.integers(0, n, size=2))
                key = a * n + b
                if a != b and key not in added_live and (key in deleted or not in_base(key)):
                    break
            deleted.discard(key)
            added_live[key] = len(added)
            added.append(key)
        else:
            while True:
                pos = int(rng.integers(0, base.size + len(added)))
                if pos < base.size:
                    key = int(base[pos])
                    if key not in deleted and key not in added_live:
                        deleted.add(key)
                        break
                else:
                    key = added[pos - base.size]
                    if added_live.get(key) == pos - base.size:
                        del added_live[key]
                        if in_base(key):
                            deleted.add(key)
                        break
        us[t] = key // n
        ud[t] = key % n
    return us, ud, ops


# Named workloads (sizes of the paper-scale stand-ins).
WORKLOADS = {
    "er_1k_10k": dict(kind="er", n=1_000, m=10_000, gamma=None),
    "cl_1m_10m": dict(kind="cl", n=1_000_000, m=10_000_000, gamma=2.1),
    "cl_5m_50m": dict(kind="cl", n=5_000_000, m=50_000_000, gamma=2.1),
    "cl_10m_200m": dict(kind="cl", n=10_000_000, m=200_000_000, gamma=2.1),
    "cl_40m_1400m": dict(kind="cl", n=40_000_000, m=1_400_000_000, gamma=2.0),
}


def make_workload(name: str, seed: int = 1, progress=None):
    spec = WORKLOADS[name]
    if spec["kind"] == "er":
        s, d = erdos_renyi(spec["n"], spec["m"], seed)
    else:
        s, d = chung_lu(spec["n"], spec["m"], spec["gamma"], seed, progress=progress)
    return spec["n"], s, d
