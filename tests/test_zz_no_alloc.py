"""bt_prefix_scan_noalloc (for callers that cannot allocate): the prefix pass
with its scratch in the library's fixed device array gives exactly what
bt_prefix_scan gives.  Two calls in a row, the second on a smaller text, so
that the second runs on an array that still holds the first call's status
words; dense and sampled fingerprints; texts past the array's bound are
refused before any device work."""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_util import to_device, torch_cuda

pytestmark = pytest.mark.gpu

X = 0x1F2E3D4C5B6A7988 % ((1 << 61) - 1)
X32 = 0x2545F491


def _filled(torch, n, dtype, value):
    return torch.full((n,), value, dtype=dtype, device="cuda:0")


@pytest.mark.parametrize("sampled", [False, True])
def test_noalloc_equals_prefix_scan(sampled):
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    ctx = bt.Context(0)
    try:
        big = to_device(synth.cfg1_text(5_000_123))  # 153 tiles of 32 KiB
        small = to_device(synth.cfg1_text(70_001))   # 3 tiles
        want = [ctx.prefix_scan(t, X, X32, sampled) for t in (big, small)]
        outs = []
        for t in (big, small):
            n = t.numel()
            P = _filled(torch, n // 16 + 1 if sampled else n + 1, torch.uint64, 0xA5)
            H = _filled(torch, n + 1, torch.int32, -7)
            outs.append((P, H))
        # the two calls in a row: big, then small
        for t, (P, H) in zip((big, small), outs):
            ctx.prefix_scan_noalloc(t, X, X32, sampled, P=P, H=H)
        torch.cuda.synchronize()
        for (wp, wh), (P, H) in zip(want, outs):
            assert torch.equal(wp, P), "prefix fingerprints differ"
            assert torch.equal(wh, H), "32-bit prefix hashes differ"
    finally:
        ctx.close()


def test_noalloc_edges_and_bound():
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    ctx = bt.Context(0)
    try:
        for n in (0, 1, 63, 64, 32768, 32769):
            t = to_device(synth.random_text(n, 256, n + 1))
            wp, wh = ctx.prefix_scan(t, X, X32)
            P, H = ctx.prefix_scan_noalloc(t, X, X32)
            torch.cuda.synchronize()
            assert torch.equal(wp, P) and torch.equal(wh, H), n
        # past the fixed array's bound: refused on the host, nothing launched
        t = to_device(synth.random_text(64, 4, 1))
        P = _filled(torch, 65, torch.uint64, 0)
        H = _filled(torch, 65, torch.int32, 0)
        rc = bt.lib().bt_prefix_scan_noalloc(ctx.h, ctypes.c_void_p(t.data_ptr()), (1 << 33) + 1, X,
                                            X32, 0, ctypes.c_void_p(P.data_ptr()),
                                            ctypes.c_void_p(H.data_ptr()))
        assert rc == bt.BT_E_INVAL
        assert b"2^33" in bt.lib().bt_ctx_last_error(ctx.h)
        assert int(P.sum().item()) == 0 and int(H.sum().item()) == 0
    finally:
        ctx.close()
