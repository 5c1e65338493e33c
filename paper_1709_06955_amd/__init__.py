"""Python binding of the MI355X ProbeSim library (libprobesim.so).

Argument marshalling only: every step of a query runs in the library's HIP
kernels.  PyTorch supplies device memory (output tensors) and the stream.
The binding refuses to work without the built library; there is no fallback.
"""

from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprobesim.so")

PS_OK = 0
STATUS = {
    0: "PS_OK", 1: "PS_ERR_INVALID_ARG", 2: "PS_ERR_NODE_RANGE", 3: "PS_ERR_SELF_LOOP",
    4: "PS_ERR_DUP_EDGE", 5: "PS_ERR_NO_EDGE", 6: "PS_ERR_OOM", 7: "PS_ERR_BUSY",
    8: "PS_ERR_DEVICE", 9: "PS_ERR_TIMEOUT", 10: "PS_ERR_STATE",
}
PS_LOAD_DEDUP = 1
PS_LOAD_DROP_SELF_LOOPS = 2
PS_MAX_WALK_LEN = 64

# Every entry point declared in include/probesim.h.
PROBE_DETERMINISTIC, PROBE_RANDOMIZED, PROBE_HYBRID, PROBE_MERGED = 0, 1, 2, 3
RULE2_AS_STATED, RULE2_PROVEN = 0, 1

EXPORTS = [
    "ps_status_string", "ps_ctx_create", "ps_ctx_destroy", "ps_ctx_set_timing", "ps_graph_load",
    "ps_graph_free", "ps_graph_info", "ps_graph_update", "ps_graph_edges", "ps_options_default",
    "ps_derive_params", "ps_walks", "ps_single_source", "ps_single_source_sparse", "ps_topk",
    "ps_select_topk", "ps_select_topk_noalloc", "ps_batch",
    "ps_get_stats",
    "ps_server_start", "ps_server_get_stats", "ps_submit", "ps_wait", "ps_server_update", "ps_server_stop", "ps_autotune",
    "ps_tune_split",
]


class ProbeSimError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


class Options(C.Structure):
    _fields_ = [
        ("eps_s", C.c_double), ("eps_t", C.c_double), ("eps_p", C.c_double),
        ("max_len", C.c_int32), ("bias_shift", C.c_int32),
        ("walk_begin", C.c_int64), ("walk_end", C.c_int64),
        ("slots", C.c_int32), ("probe_mode", C.c_int32),
        ("pull_edges", C.c_int64), ("hybrid_c0", C.c_double),
        ("rule2_bound", C.c_int32), ("pad", C.c_int32),
    ]


class Params(C.Structure):
    _fields_ = [
        ("c", C.c_double), ("eps_a", C.c_double), ("delta", C.c_double),
        ("eps_s", C.c_double), ("eps_t", C.c_double), ("eps_p", C.c_double),
        ("n_r", C.c_int64), ("L", C.c_int32), ("t_stop", C.c_uint32),
    ]


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "queries", "walks", "walk_nodes", "tree_nodes", "probe_levels", "steps", "entries_expanded",
        "entries_pruned", "edges_scanned", "next_entries", "final_adds", "expand_launches", "pull_levels",
        "pull_edges", "near_threshold")] + [
        ("flip_allowance", C.c_double), ("expand_ms", C.c_double), ("pull_ms", C.c_double), ("total_ms", C.c_double),
        ("level_hist_count", C.c_int64 * 32), ("level_hist_edges", C.c_int64 * 32),
        ("switched_probes", C.c_int64), ("pushed_edges", C.c_int64), ("pushed_final_adds", C.c_int64),
        ("reduce_bins", C.c_int64), ("reduce_slices", C.c_int64), ("reduce_max_records", C.c_int64)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if k.startswith("level_hist") else v
        return d


class Query(C.Structure):
    _fields_ = [("u", C.c_int32), ("k", C.c_int32), ("c", C.c_double), ("eps", C.c_double),
                ("delta", C.c_double), ("seed", C.c_uint64), ("probe_mode", C.c_int32), ("pad", C.c_int32),
                ("hybrid_c0", C.c_double)]


class Result(C.Structure):
    _fields_ = [("scores", C.c_void_p), ("nodes", C.c_void_p), ("status", C.c_int32), ("count", C.c_int32),
                ("flip_allowance", C.c_double)]


class Tune(C.Structure):
    _fields_ = [("slots", C.c_int32), ("from_cache", C.c_int32), ("dense_edges", C.c_int64),
                ("ms_per_query", C.c_double)]


class Split(C.Structure):
    _fields_ = [("eps_s", C.c_double), ("eps_t", C.c_double), ("eps_p", C.c_double),
                ("ms_per_query", C.c_double), ("default_ms_per_query", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("queries_done", C.c_int64), ("update_batches", C.c_int64), ("updates", C.c_int64),
                ("update_latency_ms_mean", C.c_double), ("update_latency_ms_max", C.c_double),
                ("update_apply_ms_mean", C.c_double), ("update_apply_ms_max", C.c_double)]


class ServerCfg(C.Structure):
    _fields_ = [("ring", C.c_int32), ("max_inflight", C.c_int32), ("slots", C.c_int32),
                ("reserved", C.c_int32), ("frontier_bytes", C.c_int64), ("defaults", C.POINTER(Options))]


_lib = None
_live = []  # weak references to open servers, graphs and contexts, in creation order


def _track(obj):
    _live.append(weakref.ref(obj))


def _teardown():
    """Closes what is still open at interpreter exit, newest first (servers,
    then their graphs, then contexts).  Registered right after torch is
    imported, so it runs before torch's own exit handlers, while the HIP
    runtime is still up."""
    while _live:
        obj = _live.pop()()
        if obj is not None:
            try:
                obj.close()
            except Exception:
                pass


def load_library(path: str = LIB_PATH):
    """Loads libprobesim.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with python -m paper_1709_06955_amd.build")
    # torch bundles its own HIP runtime (same soname, libamdhip64.so.7).  Load
    # it first so that the library binds to that one: one HIP runtime per
    # process, shared streams and device pointers with torch.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    atexit.register(_teardown)  # after torch's handlers, so it runs before them
    L = C.CDLL(path)
    P, vp = C.POINTER, C.c_void_p
    sig = {
        "ps_status_string": ([C.c_int], C.c_char_p),
        "ps_ctx_create": ([C.c_int, vp, P(vp)], C.c_int),
        "ps_ctx_destroy": ([vp], None),
        "ps_ctx_set_timing": ([vp, C.c_int], C.c_int),
        "ps_graph_load": ([vp, C.c_int32, C.c_int64, vp, vp, C.c_uint32, P(vp)], C.c_int),
        "ps_graph_free": ([vp], None),
        "ps_graph_info": ([vp, P(C.c_int32), P(C.c_int64), P(C.c_uint64)], C.c_int),
        "ps_graph_update": ([vp, C.c_int64, vp, vp, vp, vp, P(C.c_uint64)], C.c_int),
        "ps_graph_edges": ([vp, C.c_int64, vp, vp, P(C.c_int64)], C.c_int),
        "ps_options_default": ([P(Options)], None),
        "ps_derive_params": ([C.c_int32, C.c_double, C.c_double, C.c_double, P(Options), P(Params)], C.c_int),
        "ps_walks": ([vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_uint64, P(Options), C.c_int64,
                      C.c_int64, vp, vp], C.c_int),
        "ps_single_source": ([vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_uint64, P(Options), vp],
                             C.c_int),
        "ps_single_source_sparse": ([vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_uint64, P(Options),
                                     C.c_int64, vp, vp, P(C.c_int64)], C.c_int),
        "ps_topk": ([vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_uint64, P(Options), vp,
                     vp], C.c_int),
        "ps_select_topk": ([vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp], C.c_int),
        "ps_select_topk_noalloc": ([vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp], C.c_int),
        "ps_batch": ([vp, C.c_int32, P(Query), P(Options), P(Result)], C.c_int),
        "ps_get_stats": ([vp, P(Stats)], C.c_int),
        "ps_server_start": ([vp, P(ServerCfg), P(vp)], C.c_int),
        "ps_server_get_stats": ([vp, P(ServerStats)], C.c_int),
        "ps_submit": ([vp, P(Query), P(Result), P(C.c_uint64)], C.c_int),
        "ps_wait": ([vp, C.c_uint64, C.c_int64], C.c_int),
        "ps_server_update": ([vp, C.c_int64, vp, vp, vp], C.c_int),
        "ps_server_stop": ([vp], C.c_int),
        "ps_autotune": ([vp, C.c_int32, vp, C.c_double, C.c_double, C.c_double, C.c_char_p, P(Tune)], C.c_int),
        "ps_tune_split": ([vp, C.c_int32, vp, C.c_double, C.c_double, C.c_double, P(Options), P(Split)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(code, what):
    if code != PS_OK:
        raise ProbeSimError(code, what)


def _ptr(a):
    """Data pointer of a numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def options(**kw) -> Options:
    o = Options()
    load_library().ps_options_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def derive_params(n, c, eps, delta, **opt) -> Params:
    p = Params()
    o = options(**opt)
    _check(load_library().ps_derive_params(int(n), c, eps, delta, C.byref(o), C.byref(p)), "ps_derive_params")
    return p


class Context:
    """A device context; pass a torch stream to launch on it."""

    def __init__(self, device: int = 0, stream=None):
        L = load_library()
        h = C.c_void_p()
        s = None
        if stream is not None:
            s = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        _check(L.ps_ctx_create(int(device), s, C.byref(h)), "ps_ctx_create")
        self._h = h
        self.device = device
        _track(self)

    def set_timing(self, on: bool):
        _check(load_library().ps_ctx_set_timing(self._h, int(on)), "ps_ctx_set_timing")

    def stats(self) -> dict:
        st = Stats()
        _check(load_library().ps_get_stats(self._h, C.byref(st)), "ps_get_stats")
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load_library().ps_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _edge_array(a):
    """(object kept alive, pointer, length) of an edge array."""
    if hasattr(a, "data_ptr") and getattr(a, "is_cuda", False):
        if str(a.dtype) != "torch.int32" or not a.is_contiguous():
            raise ValueError("device edge arrays must be contiguous int32 tensors")
        return a, a.data_ptr(), a.numel()
    h = np.ascontiguousarray(a, dtype=np.int32)
    return h, h.ctypes.data, h.size


class Graph:
    """A device-resident graph (edges src[i] -> dst[i])."""

    def __init__(self, ctx: Context, n: int, src, dst, flags: int = 0):
        """src, dst: int32 edge arrays (numpy/host, or contiguous int32 torch
        tensors on the context's GPU)."""
        s, sp, sm = _edge_array(src)
        d, dp, dm = _edge_array(dst)
        if sm != dm:
            raise ValueError("src and dst differ in length")
        h = C.c_void_p()
        _check(load_library().ps_graph_load(ctx._h, int(n), int(sm), sp, dp, int(flags), C.byref(h)),
               "ps_graph_load")
        self._h = h
        _track(self)
        self.ctx = ctx
        self.n = int(n)

    def info(self):
        n, m, v = C.c_int32(), C.c_int64(), C.c_uint64()
        _check(load_library().ps_graph_info(self._h, C.byref(n), C.byref(m), C.byref(v)), "ps_graph_info")
        return n.value, m.value, v.value

    def update(self, src, dst, op, per_edge: bool = True):
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        o = np.ascontiguousarray(op, dtype=np.uint8)
        pe = np.zeros(s.size, dtype=np.int32)
        ver = C.c_uint64()
        _check(load_library().ps_graph_update(self._h, int(s.size), s.ctypes.data, d.ctypes.data, o.ctypes.data,
                                              pe.ctypes.data if per_edge else None, C.byref(ver)),
               "ps_graph_update")
        return pe, ver.value

    def edges(self):
        _, m, _ = self.info()
        s = np.zeros(max(m, 1), np.int32)
        d = np.zeros(max(m, 1), np.int32)
        mm = C.c_int64()
        _check(load_library().ps_graph_edges(self._h, int(m), s.ctypes.data, d.ctypes.data, C.byref(mm)),
               "ps_graph_edges")
        return s[: mm.value], d[: mm.value]

    def close(self):
        if getattr(self, "_h", None):
            load_library().ps_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ps_walks(g: Graph, u, c, eps, delta, seed, k_begin, count, out_nodes=None, out_lens=None, **opt):
    """Walks k_begin .. k_begin+count-1 of the query (host arrays unless given)."""
    p = derive_params(g.n, c, eps, delta, **opt)
    nodes = out_nodes if out_nodes is not None else np.zeros((count, p.L), np.int32)
    lens = out_lens if out_lens is not None else np.zeros(count, np.int32)
    o = options(**opt)
    _check(load_library().ps_walks(g._h, int(u), c, eps, delta, C.c_uint64(seed), C.byref(o), int(k_begin),
                                   int(count), _ptr(nodes), _ptr(lens)), "ps_walks")
    return nodes, lens


def ps_single_source(g: Graph, u, c, eps, delta, seed, out=None, **opt):
    """Approximate single-source SimRank from u; `out` may be a device tensor."""
    if out is None:
        out = np.zeros(g.n, np.float64)
    o = options(**opt)
    _check(load_library().ps_single_source(g._h, int(u), c, eps, delta, C.c_uint64(seed), C.byref(o), _ptr(out)),
           "ps_single_source")
    return out


def ps_single_source_sparse(g: Graph, u, c, eps, delta, seed, cap=None, out_nodes=None, out_scores=None, **opt):
    """Nonzero estimates as (nodes ascending, scores); cap defaults to n.  A
    cap below the number of nonzero entries raises ProbeSimError with the
    needed count in its `count` attribute."""
    cap = g.n if cap is None else int(cap)
    nodes = out_nodes if out_nodes is not None else np.zeros(max(cap, 1), np.int32)
    scores = out_scores if out_scores is not None else np.zeros(max(cap, 1), np.float64)
    cnt = C.c_int64(0)
    o = options(**opt)
    code = load_library().ps_single_source_sparse(g._h, int(u), c, eps, delta, C.c_uint64(seed), C.byref(o), cap,
                                                  _ptr(nodes), _ptr(scores), C.byref(cnt))
    if code != PS_OK:
        err = ProbeSimError(code, "ps_single_source_sparse")
        err.count = cnt.value
        raise err
    return nodes[: cnt.value], scores[: cnt.value]


def ps_topk(g: Graph, u, k, c, eps, delta, seed, out_nodes=None, out_scores=None, **opt):
    nodes = out_nodes if out_nodes is not None else np.zeros(k, np.int32)
    scores = out_scores if out_scores is not None else np.zeros(k, np.float64)
    o = options(**opt)
    _check(load_library().ps_topk(g._h, int(u), int(k), c, eps, delta, C.c_uint64(seed), C.byref(o),
                                  _ptr(nodes), _ptr(scores)), "ps_topk")
    return nodes, scores


def ps_select_topk(ctx: Context, scores, u, k, out_nodes=None, out_scores=None):
    """Definition 2's selection over a given estimate vector (numpy array or
    device tensor of n doubles)."""
    if isinstance(scores, np.ndarray):
        scores = np.ascontiguousarray(scores, dtype=np.float64)
    n = int(scores.shape[0])
    nodes = out_nodes if out_nodes is not None else np.zeros(k, np.int32)
    vals = out_scores if out_scores is not None else np.zeros(k, np.float64)
    _check(load_library().ps_select_topk(ctx._h, _ptr(scores), n, int(u), int(k), _ptr(nodes), _ptr(vals)),
           "ps_select_topk")
    return nodes, vals


NOALLOC_MAX_K = 65536


def ps_select_topk_noalloc(ctx: Context, scores, u, k, out_nodes, out_scores):
    """ps_select_topk without any device allocation: scores, out_nodes and
    out_scores are device tensors; queued on the context's stream."""
    _check(load_library().ps_select_topk_noalloc(ctx._h, _ptr(scores), int(scores.shape[0]), int(u), int(k),
                                                 _ptr(out_nodes), _ptr(out_scores)), "ps_select_topk_noalloc")


def ps_autotune(g: Graph, nodes, c, eps, delta, cache_path=None) -> dict:
    """Times sample queries under candidate slot counts and dense thresholds
    and keeps the fastest as the graph's automatic setting."""
    nd = np.ascontiguousarray(nodes, dtype=np.int32)
    t = Tune()
    _check(load_library().ps_autotune(g._h, int(nd.size), nd.ctypes.data, c, eps, delta,
                                      cache_path.encode() if cache_path else None, C.byref(t)), "ps_autotune")
    return {k: getattr(t, k) for k, _ in t._fields_}


def ps_tune_split(g: Graph, nodes, c, eps, delta, **opt) -> dict:
    """Times the split candidates of Theorem 2 on the sample query nodes and
    returns the fastest split (eps_s, eps_t, eps_p) with the measured times;
    pass its eps_s/eps_t/eps_p to later queries to use it."""
    nd = np.ascontiguousarray(nodes, dtype=np.int32)
    o = options(**opt)
    t = Split()
    _check(load_library().ps_tune_split(g._h, int(nd.size), nd.ctypes.data, c, eps, delta, C.byref(o), C.byref(t)),
           "ps_tune_split")
    return {k: getattr(t, k) for k, _ in t._fields_}


class BatchResults(list):
    """Per-query results of ps_batch; `flip_allowance[i]` is query i's
    Rule-2 near-threshold allowance (ps_result.flip_allowance)."""

    flip_allowance: list


def ps_batch(g: Graph, queries, outs=None, **opt):
    """queries: list of dicts (u, k, c, eps, delta, seed; optional probe_mode,
    hybrid_c0).  Returns a list of
    score arrays (single-source) or (nodes, scores) pairs (top-k), with the
    per-query allowances in its `flip_allowance` attribute."""
    nq = len(queries)
    qa = (Query * max(nq, 1))()
    ra = (Result * max(nq, 1))()
    keep = []
    for i, q in enumerate(queries):
        qa[i] = Query(int(q["u"]), int(q.get("k", 0)), q["c"], q["eps"], q["delta"], int(q["seed"]),
                      int(q.get("probe_mode", 0)), 0, float(q.get("hybrid_c0", options().hybrid_c0)))
        if outs is not None:
            sc, nd = outs[i]
        elif q.get("k", 0) > 0:
            sc, nd = np.zeros(q["k"], np.float64), np.zeros(q["k"], np.int32)
        else:
            sc, nd = np.zeros(g.n, np.float64), None
        keep.append((sc, nd))
        ra[i].scores = _ptr(sc)
        ra[i].nodes = _ptr(nd) if nd is not None else None
    o = options(**opt)
    _check(load_library().ps_batch(g._h, nq, qa, C.byref(o), ra), "ps_batch")
    res = BatchResults()
    res.flip_allowance = []
    for i, (sc, nd) in enumerate(keep):
        _check(ra[i].status, f"query {i}")
        res.append(sc if nd is None else (nd, sc))
        res.flip_allowance.append(ra[i].flip_allowance)
    return res


class Server:
    """Continuous-batching query server on one graph."""

    def __init__(self, g: Graph, ring=1024, max_inflight=64, slots=0, frontier_bytes=0, **defaults):
        """defaults: ps_options fields every served query runs with (split,
        probe_mode, hybrid_c0, ...); a query's own probe_mode overrides."""
        cfg = ServerCfg(ring, max_inflight, slots, 0, frontier_bytes, None)
        if defaults:
            o = options(**defaults)
            cfg.defaults = C.pointer(o)
        h = C.c_void_p()
        _check(load_library().ps_server_start(g._h, C.byref(cfg), C.byref(h)), "ps_server_start")
        self._h = h
        _track(self)
        self.g = g
        self._pending = {}

    def submit(self, u, c, eps, delta, seed, k=0, probe_mode=0, hybrid_c0=None):
        c0 = options().hybrid_c0 if hybrid_c0 is None else float(hybrid_c0)
        q = Query(int(u), int(k), c, eps, delta, int(seed), int(probe_mode), 0, c0)
        if k > 0:
            sc, nd = np.zeros(k, np.float64), np.zeros(k, np.int32)
        else:
            sc, nd = np.zeros(self.g.n, np.float64), None
        r = Result(sc.ctypes.data, nd.ctypes.data if nd is not None else None, 0, 0, 0.0)
        t = C.c_uint64()
        code = load_library().ps_submit(self._h, C.byref(q), C.byref(r), C.byref(t))
        if code != PS_OK:
            raise ProbeSimError(code, "ps_submit")
        self._pending[t.value] = (q, r, sc, nd)
        return t.value

    def wait(self, ticket, timeout_us=-1, allowance=False):
        """The query's result; with allowance=True also its Rule-2
        near-threshold allowance (ps_result.flip_allowance)."""
        code = load_library().ps_wait(self._h, C.c_uint64(ticket), int(timeout_us))
        if code == 9:
            raise TimeoutError(ticket)
        q, r, sc, nd = self._pending.pop(ticket)
        _check(code, f"ticket {ticket}")
        out = sc if nd is None else (nd, sc)
        return (out, r.flip_allowance) if allowance else out

    def update(self, src, dst, op):
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        o = np.ascontiguousarray(op, dtype=np.uint8)
        _check(load_library().ps_server_update(self._h, int(s.size), s.ctypes.data, d.ctypes.data, o.ctypes.data),
               "ps_server_update")

    def stats(self) -> dict:
        st = ServerStats()
        _check(load_library().ps_server_get_stats(self._h, C.byref(st)), "ps_server_get_stats")
        return {k: getattr(st, k) for k, _ in st._fields_}

    def stop(self):
        if getattr(self, "_h", None):
            _check(load_library().ps_server_stop(self._h), "ps_server_stop")
            self._h = None

    def close(self):
        self.stop()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
