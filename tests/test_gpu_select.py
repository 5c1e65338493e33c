"""GPU selection kernels against the plain definitions.

Top-k (Definition 2): the k nodes v != u with the largest value, ties to the
smaller id, in that order.  The expected list is a plain sort of (-s[v], v)
over v != u; node ids must match exactly and values bit for bit (they are the
input values).  The inputs stress what a radix select can get wrong: ties at
the k-th value across many workgroups, values that differ only in the last
mantissa bits, zeros and subnormals, signed zeros, k past the single-tile sort.

The nonzero list of ps_single_source_sparse is compared with the dense result
of the same query.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_1709_06955_amd as ps

    ps.load_library()
    return ps


@pytest.fixture(scope="module")
def ctx(ps):
    c = ps.Context(0)
    yield c
    c.close()


def expected_topk(s, u, k):
    ids = np.delete(np.arange(s.size), u)
    order = np.lexsort((ids, -s[ids]))
    top = ids[order[:k]]
    return top.astype(np.int32), s[top]


def check(ps, ctx, s, u, k, what):
    print(f"select case: {what} n={s.size} u={u} k={k}", flush=True)
    nodes, vals = ps.ps_select_topk(ctx, s, u, k)
    en, ev = expected_topk(s, u, k)
    assert np.array_equal(nodes, en), f"{what}: first mismatch at {np.argmax(nodes != en)}"
    assert np.array_equal(vals.view(np.uint64), ev.view(np.uint64)), what


def test_random_values_many_k(ps, ctx):
    rng = np.random.default_rng(1)
    s = rng.random(100_003)
    for k in (1, 2, 50, 63, 64, 65, 4095, 4096, 4097, 20_000, 100_002):
        check(ps, ctx, s, 17, k, "uniform")


def test_all_equal_and_zero(ps, ctx):
    for val in (0.0, 0.5, 5e-324):
        s = np.full(50_000, val)
        for k in (1, 100, 49_999):
            check(ps, ctx, s, 33, k, f"all {val}")


def test_ties_at_the_kth_value(ps, ctx):
    rng = np.random.default_rng(2)
    levels = np.array([0.0, 5e-324, 1e-300, 0.125, 0.25, 0.25 + 2**-54, 0.5, 1.0])
    s = levels[rng.integers(0, levels.size, 300_000)]
    counts = [(s == x).sum() for x in levels[::-1]]
    cum = np.cumsum(counts)
    # k landing inside each tie group, at its edges and one past
    ks = sorted({int(x) for c in cum[:-1] for x in (c - 1, c, c + 1)} | {1, 1000, 70_000})
    for k in ks:
        if 1 <= k <= s.size - 1:
            check(ps, ctx, s, 5, k, "tie groups")


def test_last_mantissa_bits(ps, ctx):
    # neighbouring doubles: the select must fix all 64 bits
    base = 0.3
    s = np.empty(20_000)
    x = base
    for i in range(s.size):
        s[i] = x
        x = np.nextafter(x, 1.0)
    rng = np.random.default_rng(3)
    rng.shuffle(s)
    s[::7] = s[1]  # plus exact duplicates of one value
    for k in (1, 10, 2857, 9999, 19_998):
        check(ps, ctx, s, 0, k, "adjacent doubles")


def test_signed_zero_and_negative(ps, ctx):
    s = np.array([0.0, -0.0, -1.0, 2.0, -0.0, 0.0, -3.5, 1e-310, -1e-310, 0.0])
    for u in (0, 3, 9):
        for k in range(1, s.size):
            check(ps, ctx, s, u, k, "signed zeros")


def test_tiny_and_large_n(ps, ctx):
    check(ps, ctx, np.array([0.2, 0.1]), 0, 1, "n=2")
    check(ps, ctx, np.array([0.2, 0.1, 0.2]), 1, 2, "n=3")
    rng = np.random.default_rng(4)
    n = 20_000_000
    s = np.zeros(n)
    nz = rng.choice(n, n // 100, replace=False)
    s[nz] = rng.random(nz.size) * 1e-3
    s[nz[:5000]] = 1e-3  # a tie group at the top
    for k in (50, 5001):
        check(ps, ctx, s, int(nz[0]), k, "sparse 20M")


def test_device_input_and_errors(ps, ctx):
    import torch

    rng = np.random.default_rng(5)
    s = rng.random(300_000)
    d = torch.from_numpy(s).to("cuda:0")
    on = torch.zeros(77, dtype=torch.int32, device="cuda:0")
    ov = torch.zeros(77, dtype=torch.float64, device="cuda:0")
    ps.ps_select_topk(ctx, d, 1, 77, out_nodes=on, out_scores=ov)
    en, ev = expected_topk(s, 1, 77)
    assert np.array_equal(on.cpu().numpy(), en) and np.array_equal(ov.cpu().numpy(), ev)
    with pytest.raises(ps.ProbeSimError):
        ps.ps_select_topk(ctx, s[:10], 10, 1)
    with pytest.raises(ps.ProbeSimError):
        ps.ps_select_topk(ctx, s[:10], 0, 10)
    with pytest.raises(ps.ProbeSimError):
        ps.ps_select_topk(ctx, s[:10], 0, 0)
