"""ctypes binding of the ProbeSim CPU oracle.  TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never loads it and it never loads the GPU
library.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "probesim_oracle.cpp")

ORC_OK, ORC_EINVAL, ORC_ERANGE, ORC_ESELF, ORC_EDUP = range(5)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (host code only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["g++", "-O3", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC", "-Wall", "-Wextra", "-o", tmp,
             _SRC]
        )
        os.replace(tmp, _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [
        ("c", C.c_double), ("eps_a", C.c_double), ("delta", C.c_double),
        ("eps_s", C.c_double), ("eps_t", C.c_double), ("eps_p", C.c_double),
        ("n_r", C.c_int64), ("L", C.c_int32), ("t_stop", C.c_uint32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("walk_nodes", C.c_int64), ("probes", C.c_int64), ("entries_expanded", C.c_int64),
        ("entries_pruned", C.c_int64), ("edges_scanned", C.c_int64), ("next_entries", C.c_int64),
        ("final_entries", C.c_int64), ("near_threshold", C.c_int64), ("flip_allowance", C.c_double),
        ("tree_nodes", C.c_int64), ("switched", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = C.CDLL(_SO)
        P = C.POINTER
        L.orc_graph_build.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32), P(C.c_void_p)]
        L.orc_graph_free.argtypes = [C.c_void_p]
        L.orc_graph_free.restype = None
        L.orc_params_derive.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_int32, P(Params)]
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_philox4x32_10.restype = None
        L.orc_walk.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, P(Params), P(C.c_int32)]
        L.orc_walk.restype = C.c_int32
        L.orc_probe.argtypes = [C.c_void_p, P(C.c_int32), C.c_int32, C.c_double, C.c_double, C.c_int,
                                P(C.c_double)]
        L.orc_rprobe.argtypes = [C.c_void_p, P(C.c_int32), C.c_int32, C.c_double, C.c_uint64, C.c_int64,
                                 P(C.c_double)]
        for f in (L.orc_single_source, L.orc_batch):
            f.argtypes = [C.c_void_p, C.c_int32, P(Params), C.c_uint64, C.c_int64, C.c_int64, C.c_int, C.c_int,
                          P(C.c_double), P(Stats)]
        L.orc_batch_hybrid.argtypes = [C.c_void_p, C.c_int32, P(Params), C.c_uint64, C.c_int64, C.c_int64, C.c_int,
                                       C.c_int, C.c_double, P(C.c_double), P(Stats)]
        L.orc_merged.argtypes = [C.c_void_p, C.c_int32, P(Params), C.c_uint64, C.c_int64, C.c_int64, C.c_int,
                                 P(C.c_double), P(Stats)]
        L.orc_topk.argtypes = [P(C.c_double), C.c_int32, C.c_int32, C.c_int32, P(C.c_int32), P(C.c_double)]
        L.orc_pair_mc.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_uint64, C.c_int64, C.c_int64,
                                  P(C.c_int64)]
        _lib = L
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


class Graph:
    """Oracle copy of a directed simple graph given as edges src[i] -> dst[i]."""

    def __init__(self, n, src, dst):
        s, ps = _i32(src)
        d, pd = _i32(dst)
        h = C.c_void_p()
        rc = lib().orc_graph_build(int(n), int(s.size), ps, pd, C.byref(h))
        if rc != ORC_OK:
            raise ValueError(f"oracle graph build failed with code {rc}")
        self.n = int(n)
        self.m = int(s.size)
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_graph_free(self._h)
            self._h = None


def params(n, c, eps_a, delta, eps_s=-1.0, eps_t=-1.0, eps_p=-1.0, L=0) -> Params:
    p = Params()
    rc = lib().orc_params_derive(int(n), c, eps_a, delta, eps_s, eps_t, eps_p, int(L), C.byref(p))
    if rc != ORC_OK:
        raise ValueError(f"invalid parameters (code {rc})")
    return p


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def walk(g: Graph, u: int, k: int, seed: int, p: Params) -> np.ndarray:
    buf = np.zeros(p.L, dtype=np.int32)
    ln = lib().orc_walk(g._h, int(u), int(k), C.c_uint64(seed), C.byref(p),
                        buf.ctypes.data_as(C.POINTER(C.c_int32)))
    return buf[:ln].copy()


PRECISIONS = ("f64", "f32")


def _f32(precision: str) -> int:
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {PRECISIONS}")
    return int(precision == "f32")


def probe(g: Graph, path, c: float, eps_p: float = 0.0, precision: str = "f64") -> np.ndarray:
    """Alg. 2 scores of PROBE(path); precision "f64" evaluates the plain
    definition, "f32" the FP32 score model (Rule 2 decided in FP32)."""
    pa, pp = _i32(path)
    out = np.zeros(g.n, dtype=np.float64)
    rc = lib().orc_probe(g._h, pp, int(pa.size), c, eps_p, _f32(precision),
                         out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != ORC_OK:
        raise ValueError(f"probe failed with code {rc}")
    return out


PROBES = ("deterministic", "randomized", "hybrid")


def rprobe(g: Graph, path, c: float, seed: int, k: int) -> np.ndarray:
    """Alg. 4 (randomized PROBE) on `path` as the probe of that prefix of walk
    k: 1.0 for the nodes it returns, else 0."""
    pa, pp = _i32(path)
    out = np.zeros(g.n, dtype=np.float64)
    rc = lib().orc_rprobe(g._h, pp, int(pa.size), c, C.c_uint64(seed), int(k),
                          out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != ORC_OK:
        raise ValueError(f"rprobe failed with code {rc}")
    return out


def _run(fn, g, u, p, seed, k_begin, k_end, bias_shift, precision, probe="deterministic", c0=None):
    if probe not in PROBES:
        raise ValueError(f"probe must be one of {PROBES}")
    out = np.zeros(g.n, dtype=np.float64)
    st = Stats()
    kb = 0 if k_begin is None else int(k_begin)
    ke = int(p.n_r) if k_end is None else int(k_end)
    mode = _f32(precision) | (2 if probe == "randomized" else 0)
    args = [g._h, int(u), C.byref(p), C.c_uint64(seed), kb, ke, int(bias_shift), mode]
    if probe == "hybrid":
        if c0 is None:
            raise ValueError("the hybrid probe needs c0")
        fn = lib().orc_batch_hybrid
        args.append(float(c0))
    rc = fn(*args, out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st))
    if rc != ORC_OK:
        raise ValueError(f"query failed with code {rc}")
    return out, st.as_dict()


def single_source(g: Graph, u: int, p: Params, seed: int, k_begin=None, k_end=None, bias_shift=False,
                  precision: str = "f64", probe: str = "deterministic", c0=None):
    """Alg. 1 estimate s^(u, .) over walks [k_begin, k_end) (default all n_r),
    with deterministic (Alg. 2) or randomized (Alg. 4) probes; "hybrid" is
    the switch of Section 4.4 with constant c0, which works per tree node and
    so runs Alg. 3."""
    return _run(lib().orc_single_source, g, u, p, seed, k_begin, k_end, bias_shift, precision, probe, c0)


def batch(g: Graph, u: int, p: Params, seed: int, k_begin=None, k_end=None, bias_shift=False,
          precision: str = "f64", probe: str = "deterministic", c0=None):
    """Alg. 3 (reverse reachability tree) estimate; equal to Alg. 1 up to
    rounding.  probe="hybrid" adds the switch of Section 4.4 at constant c0."""
    return _run(lib().orc_batch, g, u, p, seed, k_begin, k_end, bias_shift, precision, probe, c0)


def merged(g: Graph, u: int, p: Params, seed: int, k_begin=None, k_end=None, bias_shift=False):
    """Alg. 3 with Rule 2 off (p.eps_p must be 0) and the probes of each
    subtree summed at its root before expansion; FP64.  Equal to batch() at
    eps_p = 0 up to rounding."""
    out = np.zeros(g.n, dtype=np.float64)
    st = Stats()
    kb = 0 if k_begin is None else int(k_begin)
    ke = int(p.n_r) if k_end is None else int(k_end)
    rc = lib().orc_merged(g._h, int(u), C.byref(p), C.c_uint64(seed), kb, ke, int(bias_shift),
                          out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st))
    if rc != ORC_OK:
        raise ValueError(f"merged query failed with code {rc}")
    return out, st.as_dict()


def topk(scores: np.ndarray, u: int, k: int):
    s = np.ascontiguousarray(scores, dtype=np.float64)
    nodes = np.zeros(k, dtype=np.int32)
    vals = np.zeros(k, dtype=np.float64)
    rc = lib().orc_topk(s.ctypes.data_as(C.POINTER(C.c_double)), int(s.size), int(u), int(k),
                        nodes.ctypes.data_as(C.POINTER(C.c_int32)), vals.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != ORC_OK:
        raise ValueError(f"topk failed with code {rc}")
    return nodes, vals


def pair_mc(g: Graph, u: int, vs, c: float, r: int, seed: int, threads: int = 0) -> np.ndarray:
    """Section 2.2's pairwise Monte Carlo: for each v in vs, the fraction of
    r sample pairs of sqrt(c)-walks from u and v that meet, an unbiased
    estimate of s(u, v) with standard deviation sqrt(s (1 - s) / r).  The
    samples of each pair are split into ranges run on `threads` threads (the
    C calls release the GIL); a sample's random numbers depend only on
    (seed, v, sample index), so the result does not depend on the threads."""
    from concurrent.futures import ThreadPoolExecutor

    vs = [int(v) for v in vs]
    threads = threads or min(16, os.cpu_count() or 1)
    parts = max(1, min(threads, int(r) // 4096))
    bounds = [int(r) * i // parts for i in range(parts + 1)]

    def run(task):
        v, i = task
        h = C.c_int64()
        rc = lib().orc_pair_mc(g._h, int(u), v, c, C.c_uint64(seed), bounds[i], bounds[i + 1], C.byref(h))
        if rc != ORC_OK:
            raise ValueError(f"pair Monte Carlo failed with code {rc}")
        return h.value

    tasks = [(v, i) for v in vs for i in range(parts)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        hits = list(ex.map(run, tasks))
    per = np.array(hits, dtype=np.int64).reshape(len(vs), parts).sum(axis=1)
    return per / float(r)
