"""The allocation-free top-k entry point against the allocating one.

ps_select_topk_noalloc keeps its scratch in a fixed device array shared by
every call on the device; two calls in a row (the second on a smaller input,
so stale scratch from the first would show) must each equal ps_select_topk
on the same input exactly (node ids and values bit for bit).  Sizes past the
array's room and host pointers are rejected.  The check that no device
memory is allocated reads torch's allocator counters (the library does not
allocate through torch) and the device's free memory around the calls.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_matches_allocating_entry_point():
    import torch

    import paper_1709_06955_amd as ps

    ps.load_library()
    stream = torch.cuda.current_stream()
    ctx = ps.Context(0, stream=stream)
    try:
        rng = np.random.default_rng(11)
        cases = []
        big = rng.random(3_000_000)
        big[rng.choice(big.size, 1_000_000, replace=False)] = 0.25  # a large tie group
        cases.append((big, 123, 4097))
        small = np.repeat(rng.random(500), 7)[:3000]  # heavy ties, smaller n and k
        cases.append((small, 9, 50))
        # the device buffers the caller brings, allocated before the calls
        dev = [(torch.from_numpy(s).to("cuda:0"), torch.empty(k, dtype=torch.int32, device="cuda:0"),
                torch.empty(k, dtype=torch.float64, device="cuda:0")) for s, _, k in cases]
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        for (s, u, k), (ds, on, ov) in zip(cases, dev):
            print(f"noalloc case n={s.size} u={u} k={k}", flush=True)
            ps.ps_select_topk_noalloc(ctx, ds, u, k, on, ov)
            torch.cuda.synchronize()
            got_n, got_v = on.cpu().numpy(), ov.cpu().numpy()
            ref_n, ref_v = ps.ps_select_topk(ctx, s, u, k)
            assert np.array_equal(got_n, ref_n)
            assert np.array_equal(got_v.view(np.uint64), ref_v.view(np.uint64))
        # the reference calls above may allocate; the no-alloc calls alone must not
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        for (s, u, k), (ds, on, ov) in zip(cases, dev):
            ps.ps_select_topk_noalloc(ctx, ds, u, k, on, ov)
        torch.cuda.synchronize()
        free2, _ = torch.cuda.mem_get_info()
        assert free2 == free1, (free0, free1, free2)
        # limits
        ds, on, ov = dev[0]
        big_k = ps.NOALLOC_MAX_K + 1
        on2 = torch.empty(big_k, dtype=torch.int32, device="cuda:0")
        ov2 = torch.empty(big_k, dtype=torch.float64, device="cuda:0")
        with pytest.raises(ps.ProbeSimError):
            ps.ps_select_topk_noalloc(ctx, ds, 0, big_k, on2, ov2)
        with pytest.raises(ps.ProbeSimError):
            ps.ps_select_topk_noalloc(ctx, cases[1][0], 0, 5, on, ov)  # host input
        # the largest k the array holds
        k = ps.NOALLOC_MAX_K
        ps.ps_select_topk_noalloc(ctx, ds, 0, k, on2[:k], ov2[:k])
        torch.cuda.synchronize()
        ref_n, _ = ps.ps_select_topk(ctx, cases[0][0], 0, k)
        assert np.array_equal(on2[:k].cpu().numpy(), ref_n)
    finally:
        ctx.close()
