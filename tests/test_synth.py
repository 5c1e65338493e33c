"""Seeded input generators: shape, determinism and simple-graph invariants."""

import numpy as np

from synth import graphs


def _check_simple(n, s, d, m):
    assert s.size == m and d.size == m
    assert s.dtype == np.int32 and d.dtype == np.int32
    assert (s >= 0).all() and (s < n).all() and (d >= 0).all() and (d < n).all()
    assert not (s == d).any()
    keys = s.astype(np.int64) * n + d
    assert np.unique(keys).size == m


def test_erdos_renyi_is_simple_and_seeded():
    n, s, d = graphs.make_workload("er_1k_10k")
    _check_simple(n, s, d, 10_000)
    _, s2, d2 = graphs.make_workload("er_1k_10k")
    assert (s == s2).all() and (d == d2).all()


def test_chung_lu_power_law_shape():
    s, d = graphs.chung_lu(20_000, 200_000, 2.1, seed=3)
    _check_simple(20_000, s, d, 200_000)
    indeg = np.bincount(d, minlength=20_000)
    outdeg = np.bincount(s, minlength=20_000)
    # heavy tail: the largest degree is far above the mean of 10
    assert indeg.max() > 50 * indeg.mean() and outdeg.max() > 50 * outdeg.mean()
    w = graphs.chung_lu_weights(20_000, 200_000, 2.1)
    assert abs(w.sum() - 200_000) < 1e-6 * 200_000
    assert w.max() <= min(20_000 ** (1 / 1.1), 2000) * 1.05  # clipped, then renormalised


def test_query_nodes_have_in_edges():
    s, d = graphs.chung_lu(5_000, 40_000, 2.1, seed=1)
    q = graphs.query_nodes(5_000, d, 32)
    indeg = np.bincount(d, minlength=5_000)
    assert q.size == 32 and np.unique(q).size == 32 and (indeg[q] > 0).all()
    qs = graphs.stratified_query_nodes(5_000, d, 64)
    assert qs.size == 64 and (indeg[qs] > 0).all()


def test_update_stream_is_valid_in_order():
    s, d = graphs.erdos_renyi(200, 1500, seed=2)
    us, ud, op = graphs.update_stream(200, s, d, 400, seed=3)
    live = set((s.astype(np.int64) * 200 + d).tolist())
    for a, b, o in zip(us.tolist(), ud.tolist(), op.tolist()):
        k = a * 200 + b
        assert a != b
        if o == 0:
            assert k not in live
            live.add(k)
        else:
            assert k in live
            live.discard(k)
    assert (op == 0).sum() == 200
