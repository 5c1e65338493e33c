"""More pins of the CPU oracle: its Philox stream against an independent
implementation, and the eps_t/2 shift of Section 4.1 against what Rule 1 and
Theorem 2 fix."""

import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import refs

HERE = os.path.dirname(os.path.abspath(__file__))
ROCRAND = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    """Host build of tests/ref/philox_rocrand.cpp (rocRAND's header-only
    Philox4x32-10 engine, compiled for the host only)."""
    if not (os.path.exists(ROCRAND) and os.path.exists(HIPCC)):
        pytest.skip("rocRAND headers or hipcc not installed")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-nogpulib", "-O1", "-I/opt/rocm/include",
           os.path.join(HERE, "ref", "philox_rocrand.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_philox_matches_rocrand_bit_for_bit(orc, rocrand_philox):
    # Philox4x32-10 (Salmon et al., SC'11) drives every walk and every draw
    # of randomized PROBE.  10^4 random (counter, key) blocks, plus the
    # counters the walks use (k, t, u, 0) and the randomized probes use
    # (k, i << 16 | j, v, 1), against rocRAND's engine.
    rng = np.random.default_rng(2024)
    N = 10_000
    rec = rng.integers(0, 2**32, size=(N, 6), dtype=np.uint64).astype(np.uint32)
    rec[:100] = 0
    rec[:100, 0] = np.arange(100)                        # walk k
    rec[:100, 1] = np.arange(100) % 17                   # step t
    rec[:100, 2] = 11959                                 # query node u
    rec[:100, 4:] = [3, 0]                               # seed 3
    rec[100:200, 1] = (np.arange(100) % 17 << 16) | 5    # i << 16 | j
    rec[100:200, 3] = 1
    out = subprocess.run([rocrand_philox], input=rec.tobytes(), capture_output=True, check=True).stdout
    want = np.frombuffer(out, dtype=np.uint32).reshape(N, 4)
    for i in range(N):
        got = orc.philox(rec[i, :4], rec[i, 4:])
        assert np.array_equal(got, want[i]), (i, rec[i], got, want[i])


def test_bias_shift_adds_half_eps_t_off_the_diagonal(orc):
    # Section 4.1: after Rule 1 every estimate but u's own may be raised by
    # eps_t / 2.  Alg. 1 and Alg. 3, both precisions.
    from synth.graphs import erdos_renyi

    n = 300
    s_, d_ = erdos_renyi(n, 3000, seed=5)
    G = orc.Graph(n, s_, d_)
    p = orc.params(n, 0.6, 0.2, 0.05)
    for fn in (orc.single_source, orc.batch):
        for precision in ("f64", "f32"):
            a, _ = fn(G, 4, p, 1, precision=precision)
            b, _ = fn(G, 4, p, 1, precision=precision, bias_shift=True)
            d = b - a
            assert d[4] == 0.0 and b[4] == 1.0
            off = np.delete(d, 4)
            assert np.abs(off - p.eps_t / 2).max() <= 1e-15


def test_bias_shift_centres_the_truncation_error(orc):
    # Rule 1 makes the estimator one-sided: with walks cut at L nodes its
    # expectation E_L lies in [s - sqrt(c)^L, s] (the v-walk must survive L
    # steps to meet later).  The shift of Section 4.1 moves it by eps_t / 2,
    # so the seed mean of the shifted estimator sits within sqrt(c)^L - eps_t/2
    # of s when pruning is off.  E_L comes from the pair dynamic program and s
    # from the exact linear solve, neither from the oracle.
    rng = np.random.default_rng(9)
    n, c = 8, 0.9
    src, dst = refs.random_graph(n, 0.45, seed=11)
    s_exact = refs.exact_simrank(n, src, dst, c)
    G = orc.Graph(n, src, dst)
    eps_t = 0.5
    p = orc.params(n, c, 0.9, 0.5, eps_s=0.05, eps_t=eps_t, eps_p=0.0)
    L = p.L
    assert L == math.floor(math.log(eps_t) / math.log(math.sqrt(c)))
    u = 0
    EL = refs.expected_estimate(n, src, dst, u, c, L)
    bound = math.sqrt(c) ** L
    for v in range(n):
        if v != u:
            assert -1e-12 <= s_exact[u, v] - EL[v] <= bound + 1e-12
    R = 60
    seeds = rng.integers(0, 2**31, size=R)
    mean = np.zeros(n)
    for sd in seeds:
        est, _ = orc.single_source(G, u, p, int(sd), bias_shift=True)
        mean += est / R
    moved = False
    for v in range(n):
        if v == u:
            continue
        se = math.sqrt(max(EL[v], 1e-9) / (p.n_r * R))
        assert abs(mean[v] - (EL[v] + eps_t / 2)) <= 5 * se + 1e-12, v
        assert abs(mean[v] - s_exact[u, v]) <= max(eps_t / 2, bound - eps_t / 2) + 5 * se
        moved |= abs(mean[v] - EL[v]) > 5 * se
    assert moved


def test_guarantee_with_bias_shift_against_power_method(orc):
    # Theorem 2 with the shift on: eps_s + (1 + eps_s)/(1 - sqrt c) eps_p +
    # eps_t / 2 <= eps_a.  Take eps_t = eps_a / 2 (the truncation term is then
    # eps_a / 4, as in the default split without the shift): every estimate
    # stays within eps_a of SimRank (Power Method, 55 iterations).
    from synth.graphs import erdos_renyi

    n, c, eps = 1000, 0.6, 0.1
    s_, d_ = erdos_renyi(n, 10000, seed=1)
    S = refs.power_method(n, s_, d_, c, iters=55)
    G = orc.Graph(n, s_, d_)
    es, et = eps / 2, eps / 2
    ep = (eps / 4) * (1 - math.sqrt(c)) / (1 + es)
    assert es + (1 + es) / (1 - math.sqrt(c)) * ep + et / 2 <= eps * (1 + 1e-12)
    p = orc.params(n, c, eps, 0.01, eps_s=es, eps_t=et, eps_p=ep)
    for seed in range(2):
        for precision in ("f64", "f32"):
            est, _ = orc.batch(G, 0, p, seed, precision=precision, bias_shift=True)
            assert np.abs(est - S[0]).max() <= eps


def test_guarantee_under_proven_rule2_split(orc):
    # The split derived from the corrected Rule 2 bound ((i - 1) * eps_p per
    # probe): eps_s + (1 + eps_s) sqrt(c)/(1 - sqrt c)^2 eps_p + eps_t = eps_a.
    # Its estimates stay within eps_a of the Power Method, in both precisions.
    from synth.graphs import erdos_renyi

    n, c, eps = 1000, 0.6, 0.1
    sc = math.sqrt(c)
    s_, d_ = erdos_renyi(n, 10000, seed=1)
    S = refs.power_method(n, s_, d_, c, iters=55)
    G = orc.Graph(n, s_, d_)
    es, et = eps / 2, eps / 4
    ep = (eps / 4) * (1 - sc) ** 2 / ((1 + es) * sc)
    p = orc.params(n, c, eps, 0.01, eps_s=es, eps_t=et, eps_p=ep)
    for seed in range(2):
        for precision in ("f64", "f32"):
            est, _ = orc.batch(G, 0, p, seed, precision=precision)
            assert np.abs(est - S[0]).max() <= eps


def test_merged_probing_equals_tree_batch_without_pruning(orc):
    # Merged probing (every probe of a subtree summed at its root before the
    # shared level maps, Lemma 2 / Section 3.3 linearity) against Alg. 3 with
    # one probe per tree node, both with Rule 2 off (eps_p = 0): the same
    # estimate up to FP64 rounding, for whole queries, walk-range shards, the
    # walk cap and the bias shift.  The merged form never expands more
    # entries or edges than the per-probe form, whose level sets cover its
    # summed sets.
    from synth.graphs import chung_lu, erdos_renyi, query_nodes

    n = 1000
    s_, d_ = erdos_renyi(n, 10000, seed=1)
    G = orc.Graph(n, s_, d_)
    cases = [(G, n, 0, dict(), 1, None, None, False), (G, n, 3, dict(L=6), 2, None, None, False),
             (G, n, 0, dict(), 1, 100, 900, False), (G, n, 5, dict(), 4, None, None, True)]
    s2, d2 = chung_lu(5000, 40000, 2.1, seed=3)
    G2 = orc.Graph(5000, s2, d2)
    for u in query_nodes(5000, d2, 2, seed=9):
        cases.append((G2, 5000, int(u), dict(), 7, 0, 400, False))
    for g, nn, u, kw, seed, a, b, shift in cases:
        p = orc.params(nn, 0.6, 0.2, 0.01, eps_p=0.0, **kw)
        m, sm = orc.merged(g, u, p, seed, a, b, bias_shift=shift)
        t, stt = orc.batch(g, u, p, seed, a, b, bias_shift=shift)
        assert np.abs(m - t).max() <= 1e-12
        assert sm["tree_nodes"] == stt["tree_nodes"] and sm["walk_nodes"] == stt["walk_nodes"]
        assert sm["entries_expanded"] <= stt["entries_expanded"]
        assert sm["edges_scanned"] <= stt["edges_scanned"]
    with pytest.raises(ValueError):
        orc.merged(G, 0, orc.params(n, 0.6, 0.2, 0.01), 1)  # Rule 2 on: no merged form


def test_pair_monte_carlo_against_closed_forms_and_exact_simrank(orc):
    # Section 2.2: s(u, v) is the probability that sqrt(c)-walks from u and v
    # meet.  Closed forms: a and b whose only in-neighbour is x meet after one
    # step of each walk, s = c; one level further up (a <- x <- z, b <- y <- z)
    # s = c^2; nodes without in-neighbours never meet, s = 0; s(u, u) = 1.
    # Then every pair of a 40-node random graph against the exact solution of
    # the SimRank equations, within 5 standard deviations of the estimate.
    # The samples' random numbers depend only on (seed, v, sample), so the
    # estimate does not depend on the thread count.
    c, r = 0.6, 200_000
    g = orc.Graph(3, [0, 0], [1, 2])
    est = orc.pair_mc(g, 1, [2, 1, 0], c, r, 7)
    assert abs(est[0] - c) <= 5 * math.sqrt(c * (1 - c) / r)
    assert est[1] == 1.0 and est[2] == 0.0
    g2 = orc.Graph(5, [4, 4, 2, 3], [2, 3, 0, 1])  # z=4 -> x=2, y=3; x -> a=0, y -> b=1
    e2 = orc.pair_mc(g2, 0, [1], c, r, 9)[0]
    assert abs(e2 - c * c) <= 5 * math.sqrt(c * c * (1 - c * c) / r)
    s_, d_ = refs.random_graph(40, 0.1, 3)
    S = refs.exact_simrank(40, s_, d_, c)
    G = orc.Graph(40, s_, d_)
    for u in (0, 7):
        vs = list(range(40))
        est = orc.pair_mc(G, u, vs, c, r, 11 + u)
        sig = np.sqrt(np.maximum(S[u] * (1 - S[u]), 1.0 / r) / r)
        assert np.all(np.abs(est - S[u]) <= 5 * sig), np.abs(est - S[u]) / sig
    a = orc.pair_mc(G, 0, range(40), c, 20_000, 5, threads=1)
    b = orc.pair_mc(G, 0, range(40), c, 20_000, 5, threads=6)
    assert np.array_equal(a, b)
