"""aw_histogram2d_noalloc under HIP graph capture, the use it is made for:
after one eager call on the device (which looks up the fixed array), the
call is captured into a graph through torch's capture stream and replayed
several times, with other GPU work and host synchronisation between the
replays and the inputs changed in place; every replay must give the result
of an eager aw_histogram2d call on the same inputs (counts and the dropped
count bit for bit, sums within 1e-12 relative)."""
import ctypes

import numpy as np
import pytest

from gpu_util import gpu, need_gpu, np_, print_case

pytestmark = gpu

W, H = 256, 128


def _call(torch, fn, a, b, v, counts, sums, dropped):
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    return fn(a.numel(), p(a), p(b), p(v), 0.0, 1.0, 0.0, 1.0, W, H, 0, p(counts), p(sums), p(dropped),
              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_histogram_replays_in_a_graph():
    need_gpu()
    import torch
    from paper_1107_4107_amd import _abi
    lib = _abi.load()
    print_case("noalloc histogram in a graph")
    N = 500_003
    g = torch.Generator(device="cpu").manual_seed(23)
    a = (torch.rand(N, generator=g, dtype=torch.float64) * 1.2 - 0.1).cuda()
    b = (torch.rand(N, generator=g, dtype=torch.float64) * 1.2 - 0.1).cuda()
    v = torch.rand(N, generator=g, dtype=torch.float64).cuda()
    counts = torch.zeros((H, W), dtype=torch.int32, device="cuda")
    sums = torch.zeros((H, W), dtype=torch.float64, device="cuda")
    dropped = torch.zeros((1,), dtype=torch.int64, device="cuda")
    _abi.check(_call(torch, lib.aw_histogram2d_noalloc, a, b, v, counts, sums, dropped))   # set-up call
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            st = _call(torch, lib.aw_histogram2d_noalloc, a, b, v, counts, sums, dropped)
    torch.cuda.current_stream().wait_stream(s)
    _abi.check(st)
    for rep in range(3):
        # new inputs in place, then a replay
        a.copy_((torch.rand(N, generator=g, dtype=torch.float64) * 1.2 - 0.1).cuda())
        v.copy_(torch.rand(N, generator=g, dtype=torch.float64).cuda())
        counts.fill_(-5)
        sums.fill_(-1.0)
        dropped.fill_(-3)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        rc = torch.empty_like(counts)
        rs = torch.empty_like(sums)
        rd = torch.empty_like(dropped)
        _abi.check(_call(torch, lib.aw_histogram2d, a, b, v, rc, rs, rd))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(np_(counts), np_(rc), err_msg=f"counts, replay {rep}")
        np.testing.assert_array_equal(np_(dropped), np_(rd), err_msg=f"dropped, replay {rep}")
        np.testing.assert_allclose(np_(sums), np_(rs), rtol=1e-12, atol=0, err_msg=f"sums, replay {rep}")
        assert int(np_(dropped)[0]) > 0
        x = torch.randn(1 << 16, device="cuda", dtype=torch.float64).sum()   # unrelated work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(x)
    del graph
