"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module holds input generation only: graphs, query nodes and update
streams.  It contains none of ProbeSim's arithmetic (no walks, no probes, no
scores), so both sides can draw the same inputs without sharing method code.

The paper evaluates on public SNAP/LAW graphs (Section 5, Table 3: Wiki-Vote,
HepTh, AS, HepPh, LiveJournal, IT-2004, Twitter, Friendster).  None of them is
available here, so seeded synthetic graphs with the same character stand in:
a directed Erdos-Renyi graph for the small exact-ground-truth case and directed
Chung-Lu graphs with power-law in/out degrees for the large cases, with query
nodes drawn uniformly from the nodes of nonzero in-degree as in Section 5.1.
"""

from __future__ import annotations

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


def chung_lu(n: int, m: int, gamma: float, seed: int = 1):
    """Directed Chung-Lu graph: src ~ w_out, dst ~ w_in with independent
    seeded permutations of the same power-law weights; self-loops and
    duplicates rejected.  Draws about 10% more pairs than needed, keeps the
    distinct non-loop ones, tops up if short and keeps a seeded uniform subset
    of exactly m.  Returns (src, dst) int32 arrays sorted by (src, dst)."""
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

    def draw(count):
        # Sorted uniforms make the inverse-CDF searches sequential; pairing the
        # sorted sources with a random permutation of the targets gives the
        # same distribution as independent pairs.
        keys = np.empty(count, dtype=np.int64)
        step = 1 << 24
        for a in range(0, count, step):
            b = min(count, a + step)
            src = np.searchsorted(cdf_out, np.sort(rng.random(b - a)), side="right")
            dst = np.searchsorted(cdf_in, np.sort(rng.random(b - a)), side="right")[rng.permutation(b - a)]
            np.minimum(src, n - 1, out=src)
            np.minimum(dst, n - 1, out=dst)
            k = src.astype(np.int64) * n + dst
            k[src == dst] = -1
            keys[a:b] = k
        return keys

    keys = np.unique(draw(int(m * 1.1) + 1024))
    keys = keys[keys >= 0]
    while keys.size < m:
        more = draw(int((m - keys.size) * 2) + 1024)
        keys = np.unique(np.concatenate([keys, more[more >= 0]]))
    if keys.size > m:
        keep = np.sort(rng.choice(keys.size, size=m, replace=False))
        keys = keys[keep]
    return (keys // n).astype(np.int32), (keys % n).astype(np.int32)


def in_degrees(n: int, dst: np.ndarray) -> np.ndarray:
    return np.bincount(dst, minlength=n).astype(np.int64)


def query_nodes(n: int, dst: np.ndarray, count: int, seed: int = 2) -> np.ndarray:
    """Query nodes drawn uniformly (without replacement) from the nodes of
    nonzero in-degree, as the paper's experiments do (Section 5.1)."""
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
    deletes of live edges, interleaved in a seeded order.  Each update is
    valid against the edge set produced by the updates before it.
    Returns (src, dst, op) with op 0 = insert, 1 = delete."""
    rng = _rng(seed, 5)
    live = set((src.astype(np.int64) * n + dst.astype(np.int64)).tolist())
    live_list = list(live)
    ops = rng.permutation(np.repeat(np.array([0, 1], dtype=np.uint8), [count - count // 2, count // 2]))
    us = np.empty(count, np.int32)
    ud = np.empty(count, np.int32)
    for t, op in enumerate(ops):
        if op == 0:
            while True:
                a, b = (int(x) for x in rng.integers(0, n, size=2))
                key = a * n + b
                if a != b and key not in live:
                    break
            live.add(key)
            live_list.append(key)
        else:
            while True:
                pos = int(rng.integers(0, len(live_list)))
                key = live_list[pos]
                live_list[pos] = live_list[-1]
                live_list.pop()
                if key in live:
                    break
            live.discard(key)
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


def make_workload(name: str, seed: int = 1):
    spec = WORKLOADS[name]
    if spec["kind"] == "er":
        s, d = erdos_renyi(spec["n"], spec["m"], seed)
    else:
        s, d = chung_lu(spec["n"], spec["m"], spec["gamma"], seed)
    return spec["n"], s, d
