"""aw_histogram2d_noalloc -- the histogram entry point for callers that
cannot allocate device memory -- called through the C ABI and compared with
aw_histogram2d on the same inputs: two calls in a row, the second with fewer
items (so it runs over what the first left in the fixed scratch), with and
without values, and with items crowding into one tile (whose range the
accumulation splits into chunks with partial tiles in the fixed scratch).  Counts and the dropped count bit for bit; per-bin sums, whose
float order follows LDS atomics, within 1e-12 relative (values are >= 0).
After the first call on the device (which looks up the fixed array), the
device's free memory is the same before and after the calls, and a request
beyond the fixed scratch is refused with nothing enqueued."""
import ctypes

import numpy as np
import pytest

from gpu_util import gpu, need_gpu, np_, print_case

pytestmark = gpu

W, H = 512, 384
LO, HI = (0.0, -1.0), (2 * np.pi, 1.0)


def _inputs(torch, N, seed, crowded=False):
    g = torch.Generator(device="cpu").manual_seed(seed)
    # keys spill past both ends of the ranges so that some items are dropped
    a = (torch.rand(N, generator=g, dtype=torch.float64) * 1.1 - 0.05) * (2 * np.pi)
    b = torch.rand(N, generator=g, dtype=torch.float64) * 2.2 - 1.1
    v = torch.rand(N, generator=g, dtype=torch.float64) ** 2
    if crowded:   # 90% of the items in the 32 x 32 bins of one tile: its range splits into chunks
        m = torch.rand(N, generator=g) < 0.9
        k = int(m.sum())
        a[m] = (64 + 32 * torch.rand(k, generator=g, dtype=torch.float64)) * (2 * np.pi / W)
        b[m] = -1.0 + (96 + 32 * torch.rand(k, generator=g, dtype=torch.float64)) * (2.0 / H)
    return a.cuda(), b.cuda(), v.cuda()


def _outputs(torch, with_values):
    counts = torch.full((H, W), -7, dtype=torch.int32, device="cuda")
    sums = torch.full((H, W), -1.0, dtype=torch.float64, device="cuda") if with_values else None
    dropped = torch.full((1,), -3, dtype=torch.int64, device="cuda")
    return counts, sums, dropped


def _call(torch, fn, a, b, v, out=None, closed_upper=0):
    counts, sums, dropped = out if out is not None else _outputs(torch, v is not None)
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    st = fn(a.numel(), p(a), p(b), p(v), LO[0], HI[0], LO[1], HI[1], W, H, closed_upper, p(counts), p(sums),
            p(dropped), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, counts, sums, dropped


@pytest.mark.parametrize("with_values,crowded", [(True, False), (False, False), (True, True)])
def test_noalloc_histogram_matches_the_allocating_entry_point(with_values, crowded):
    need_gpu()
    import torch
    from paper_1107_4107_amd import _abi
    lib = _abi.load()
    print_case("noalloc histogram", "values" if with_values else "counts only", "crowded" if crowded else "")
    sizes = [2_000_003, 300_001]
    data = [_inputs(torch, N, 17 + k, crowded) for k, N in enumerate(sizes)]
    # reference calls first: they also load every histogram kernel
    refs = []
    for a, b, v in data:
        st, c, s, d = _call(torch, lib.aw_histogram2d, a, b, v if with_values else None)
        _abi.check(st)
        refs.append((c, s, d))
    # The first call on a device looks up the device address of the fixed
    # array; the runtime may place the array in device memory then.  Later
    # calls must leave the device's free memory as it is.
    a0, b0, v0 = _inputs(torch, 1000, 3)
    _abi.check(_call(torch, lib.aw_histogram2d_noalloc, a0, b0, v0 if with_values else None)[0])
    outs = [_outputs(torch, with_values) for _ in data]
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for (a, b, v), o in zip(data, outs):
        _abi.check(_call(torch, lib.aw_histogram2d_noalloc, a, b, v if with_values else None, out=o)[0])
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, f"device free memory moved by {free0 - free1} bytes across the no-allocation calls"
    for k, ((c, s, d), (rc, rs, rd)) in enumerate(zip(outs, refs)):
        np.testing.assert_array_equal(np_(c), np_(rc), err_msg=f"counts, call {k}")
        np.testing.assert_array_equal(np_(d), np_(rd), err_msg=f"dropped, call {k}")
        assert int(np_(d)[0]) > 0 and int(np_(c).astype(np.int64).sum()) + int(np_(d)[0]) == sizes[k]
        if with_values:
            np.testing.assert_allclose(np_(s), np_(rs), rtol=1e-12, atol=0, err_msg=f"sums, call {k}")
    print(f"calls of {sizes} items agree; dropped {[int(np_(o[2])[0]) for o in outs]}", flush=True)


def test_noalloc_histogram_refuses_more_than_its_scratch():
    need_gpu()
    import torch
    from paper_1107_4107_amd import _abi
    lib = _abi.load()
    print_case("noalloc histogram over the limit")
    N = 5_000_000   # about 15 bytes per item with values: beyond the 64 MiB array
    a, b, v = _inputs(torch, N, 5)
    st, c, s, d = _call(torch, lib.aw_histogram2d_noalloc, a, b, v)
    assert st == _abi.AW_EWORKSPACE
    assert b"fixed" in lib.aw_last_error()
    torch.cuda.synchronize()
    assert bool((c == -7).all()) and bool((s == -1.0).all()) and int(d[0]) == -3   # nothing enqueued
    # the same items without values fit (about 6.5 bytes per item) and match
    st, c, _, d = _call(torch, lib.aw_histogram2d_noalloc, a, b, None)
    _abi.check(st)
    st, rc, _, rd = _call(torch, lib.aw_histogram2d, a, b, None)
    _abi.check(st)
    np.testing.assert_array_equal(np_(c), np_(rc))
    np.testing.assert_array_equal(np_(d), np_(rd))
