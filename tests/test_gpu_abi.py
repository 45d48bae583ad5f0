"""Entry points of include/bt.h called through the C ABI itself: bt_build (the
spec call, with its rank/select support), contexts whose device memory
comes from the caller's allocator (torch's, and one that fails on purpose on
the host side), and the stream-ordered level copy."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import to_device, torch_cuda

pytestmark = pytest.mark.gpu


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def test_bt_build_against_oracle():
    """bt_build(ctx, text, n, sigma, tau, leaf_len) on its own: the canonical
    tree equals the oracle's, and rank/select (whose support bt_build always
    builds) equal counted prefixes."""
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    L = bt.lib()
    ctx = bt.Context(0)
    try:
        for T, sigma, tau, leaf in ((synth.cfg1_text(1 << 16), 4, 2, 16),
                                    (synth.markov_versions(50000, 2000, 30, 3e-3, 16, 7), 96, 4, 8),
                                    (synth.random_text(1001, 3, 5), 3, 3, 1)):
            d = to_device(T)
            h = ctypes.c_void_p()
            rc = L.bt_build(ctx.h, _vp(d), T.size, sigma, tau, leaf, ctypes.byref(h))
            assert rc == bt.BT_OK, L.bt_ctx_last_error(ctx.h)
            tree = bt.Tree(ctx, h)
            assert tree.serialize() == oracle.build_tree(T, tau, leaf).canonical
            rng = np.random.default_rng(T.size)
            alph = np.unique(T)
            m = 5000
            cs = alph[rng.integers(0, alph.size, m)].astype(np.uint8)
            pos = rng.integers(0, T.size + 1, m).astype(np.uint64)
            ks = rng.integers(1, T.size // max(alph.size, 1) + 2, m).astype(np.uint64)
            got_r = tree.rank(to_device(cs), torch.from_numpy(pos).to("cuda:0")).cpu().numpy()
            got_s = tree.select(to_device(cs), torch.from_numpy(ks).to("cuda:0")).cpu().numpy()
            assert np.array_equal(got_r, oracle.rank(T, cs, pos))
            assert np.array_equal(got_s, oracle.select(T, cs, ks))
            tree.free()
        # invalid arguments are refused with BT_E_INVAL
        h = ctypes.c_void_p()
        d = to_device(b"abcabc")
        assert L.bt_build(ctx.h, _vp(d), 6, 4, 1, 16, ctypes.byref(h)) == bt.BT_E_INVAL
        assert L.bt_build(ctx.h, _vp(d), 6, 2, 2, 16, ctypes.byref(h)) == bt.BT_E_INVAL  # sigma 2 < 3
    finally:
        ctx.close()


def test_torch_allocator_supplies_device_memory():
    """A context on torch's allocator: the pool's blocks are torch's allocated
    bytes, and trim gives them back."""
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    ctx = bt.Context(0, allocator="torch")
    T = synth.cfg1_text(1 << 18)
    d = to_device(T)
    base_d = torch.cuda.memory_allocated(0)
    tree = ctx.build(d, sigma=4, tau=2, leaf_len=16)
    assert tree.serialize() == oracle.build_tree(T, 2, 16).canonical
    m = ctx.memory()
    # torch rounds each block up to a multiple of 512 bytes (the pool's
    # smallest blocks are 256)
    delta = torch.cuda.memory_allocated(0) - base_d
    assert 0 < m["held"] <= delta <= m["held"] + (1 << 20)
    tree.free()
    ctx.trim()
    torch.cuda.synchronize()
    assert ctx.memory()["held"] == 0
    assert torch.cuda.memory_allocated(0) == base_d
    ctx.close()
    del d
    assert torch.cuda.memory_allocated(0) == base


@pytest.mark.parametrize("fail_after", [0, 3, 40])
def test_failing_allocator_gives_nomem(fail_after):
    """An allocator that refuses every block after the first `fail_after`: the
    build ends with BT_E_NOMEM, every block of the call is back in the pool,
    trim returns them all, and the same context then builds correctly once the
    allocator gives memory again."""
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    state = {"n": 0, "fail": True, "live": set()}

    def alloc(nbytes):
        state["n"] += 1
        if state["fail"] and state["n"] > fail_after:
            return None
        p = torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.current_stream(0))
        state["live"].add(p)
        return p

    def free(p):
        state["live"].discard(p)
        torch.cuda.caching_allocator_delete(p)

    al = bt.Allocator(alloc, free)
    T = synth.cfg1_text(1 << 17)
    d = to_device(T)
    torch.cuda.synchronize()
    ctx = bt.Context(0, allocator=al)
    try:
        with pytest.raises(bt.BtError) as ei:
            ctx.build(d, sigma=4, tau=2, leaf_len=16)
        assert ei.value.code == bt.BT_E_NOMEM
        torch.cuda.synchronize()
        m = ctx.memory()
        assert m["in_use"] == 0, m
        ctx.trim()
        assert ctx.memory()["held"] == 0 and not state["live"]
        state["fail"] = False
        tree = ctx.build(d, sigma=4, tau=2, leaf_len=16)
        assert tree.serialize() == oracle.build_tree(T, 2, 16).canonical
        tree.free()
    finally:
        ctx.close()
    assert not state["live"], "blocks left with the library after bt_ctx_destroy"


def test_level_copy_async():
    """bt_level_copy_async on a stream, into device and pinned host buffers,
    equals bt_level_copy."""
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    ctx = bt.Context(0)
    T = synth.cfg1_text(1 << 16)
    tree = ctx.build(to_device(T), sigma=4, tau=2, leaf_len=16)
    s = torch.cuda.Stream(0)
    for l in range(1, tree.height):
        b, marked, pb, po = tree.level(l)
        _, c, u = tree.level_info(l)
        nw = (c + 63) // 64
        dw = torch.empty(max(nw, 1), dtype=torch.int64, device="cuda:0")
        hp = torch.empty(max(u, 1), dtype=torch.int64).pin_memory()
        ho = torch.empty(max(u, 1), dtype=torch.int64).pin_memory()
        rc = bt.lib().bt_level_copy_async(tree.h, l, _vp(dw), ctypes.c_void_p(hp.data_ptr()),
                                          ctypes.c_void_p(ho.data_ptr()), ctypes.c_void_p(s.cuda_stream))
        assert rc == bt.BT_OK
        s.synchronize()
        bits = np.unpackbits(dw.cpu().numpy().view(np.uint8), bitorder="little")[:c]
        assert np.array_equal(bits, marked)
        assert np.array_equal(hp.numpy()[:u].view(np.uint64), pb)
        assert np.array_equal(ho.numpy()[:u].view(np.uint64), po)
    assert bt.lib().bt_level_copy_async(tree.h, tree.height, None, None, None, None) == bt.BT_E_INVAL
    tree.free()
    ctx.close()


def test_phase_counters():
    """Per-phase device counters of profiled builds: candidates never exceed
    windows, verified keys never exceed keys, keys never exceed blocks; no
    collisions with full fingerprints, some with 12-bit ones (every one then
    resolved exactly: the tree still equals the oracle's); the windows of the
    scanned phases equal the launch log's."""
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    T = synth.cfg1_text(1 << 18)
    want = oracle.build_tree(T, 2, 16).canonical
    d = to_device(T)
    ctx = bt.Context(0)
    try:
        for flags in (0, bt.BT_DBG_WEAK_HASH):
            ctx.reset_stats()
            ctx.profile(True)
            tree = ctx.build(d, sigma=4, tau=2, leaf_len=16, debug_flags=flags)
            ctx.profile(False)
            assert tree.serialize() == want
            ph = ctx.phases()
            assert len(ph) >= 2 * (tree.height - 2)
            for r in ph:
                assert r["candidates"] <= r["windows"]
                assert r["verified"] <= r["keys"] <= r["blocks"]
                assert r["collisions"] <= r["verified"]
            coll = sum(r["collisions"] for r in ph)
            if flags:
                assert coll > 0
            else:
                assert coll == 0
            scans = [r for r in ctx.launches() if r[0] in ("probe_scan", "byte_scan")]
            scanned = [r["windows"] for r in ph if r["keys"]]
            assert sorted(int(x[2]) for x in scans) == sorted(scanned)
            tree.free()
    finally:
        ctx.close()


def test_tuning_never_changes_a_tree():
    """Every setting of bt_tuning gives the same trees (single texts and a
    batch); values outside their ranges are refused."""
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    ctx = bt.Context(0)
    try:
        T = synth.markov_versions(300000, 20000, 15, 3e-3, 16, 11)
        d = to_device(T)
        # batch texts below 3 MiB (the expected trees come from the threaded
        # oracle construction, which tests/test_oracle_par.py pins)
        lens = synth.batch_lengths_of()
        texts = [synth.batch_text(i) for i in range(60) if lens[i] < (3 << 20)][:40]
        offs = np.zeros(len(texts) + 1, np.uint64)
        offs[1:] = np.cumsum([t.size for t in texts])
        db = to_device(np.concatenate(texts))
        want_single = oracle.build_tree(T, 4, 16).canonical
        want_batch = None
        for tune in ({}, {"table_load_log2": 3}, {"text_filter_bits_log2": 4},
                     {"text_filter_bits_log2": 7, "span_chunks": 16}, {"span_chunks": 1024},
                     {"filter2_max_log2": 16}, {"filter2_max_log2": 28, "table_load_log2": 2}):
            ctx.set_tuning(**dict(bt.DEFAULT_TUNING, **tune))
            assert ctx.build(d, sigma=96, tau=4, leaf_len=16, tuned=False).serialize() == want_single
            got = [tr.serialize() for tr in ctx.build_batch(db, offs, sigma=4, tau=4, leaf_len=16, tuned=False)]
            if want_batch is None:
                want_batch = [oracle.build_tree_par(t, 4, 16, levels=False).canonical for t in texts]
            assert got == want_batch, tune
        for bad in ({"table_load_log2": 0}, {"text_filter_bits_log2": 8}, {"span_chunks": 24},
                    {"filter2_max_log2": 29}):
            with pytest.raises(bt.BtError):
                ctx.set_tuning(**bad)
    finally:
        ctx.close()
