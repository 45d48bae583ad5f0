"""Batched builds: every text's tree from one bt_build_batch call equals the
oracle's tree of that text (and hence bt_build's), including empty texts,
texts shorter than a leaf, ragged lengths and texts of very different sizes
whose levels enter the shared level loop at different steps."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import to_device, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    import paper_2512_23314_amd as bt
    c = bt.Context(0)
    yield c
    c.close()


def _concat(texts, gap=0):
    parts, offs, o = [], [], 0
    for T in texts:
        offs.append(o)
        parts.append(np.asarray(T, np.uint8))
        o += len(T)
        if gap:
            parts.append(np.full(gap, 7, np.uint8))
            o += gap
    offs.append(o - gap if gap else o)
    # with gaps, text i is [offs[i], offs[i] + len_i); rebuild the offsets list
    return np.concatenate(parts) if parts else np.zeros(0, np.uint8), offs


def _texts(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        kind = k % 6
        n = int(rng.choice([0, 1, 5, 15, 16, 17, 100, 1000, 4096, 5000, 30000, 70000]))
        if kind == 0:
            out.append(synth.dna_copies(n, max(1, n // 8), 8, 0.01, 0.001, 4, int(rng.integers(1 << 30))))
        elif kind == 1:
            out.append(synth.random_text(n, 4, int(rng.integers(1 << 30))))
        elif kind == 2:
            out.append(synth.periodic_text(n, int(rng.integers(1, 40)), int(rng.integers(1 << 30))))
        elif kind == 3:
            out.append(np.full(n, 65, np.uint8))
        elif kind == 4:
            out.append(synth.markov_versions(n, max(1, n // 5), 5, 0.01, 8, int(rng.integers(1 << 30))))
        else:
            out.append(synth.cfg1_text(n) if n else np.zeros(0, np.uint8))
    return out


@pytest.mark.parametrize("tau,leaf,s_hint", [(2, 16, 1), (4, 16, 1), (3, 4, 1), (2, 8, 32)])
def test_batch_matches_oracle(ctx, tau, leaf, s_hint):
    texts = _texts(tau * 100 + leaf, 36)
    concat, offs = _concat(texts)
    trees = ctx.build_batch(to_device(concat), offs, tau=tau, leaf_len=leaf, s_hint=s_hint)
    assert len(trees) == len(texts)
    for T, tr in zip(texts, trees):
        want = oracle.build_tree(T, tau, leaf, s_hint=s_hint).canonical
        assert tr.serialize() == want, "text of length %d differs" % len(T)


def test_batch_with_offset_and_weak_hash(ctx):
    """Texts start at a non-zero offset; 12-bit fingerprints make fingerprints
    of different texts collide, which must never leak an occurrence from one
    text into another."""
    import paper_2512_23314_amd as bt
    base = synth.cfg1_text(1 << 12)
    texts = [base[:3000], base[:3000].copy(), base[500:3500], synth.random_text(2000, 4, 1), base[:1]]
    pad = np.full(13, 9, np.uint8)
    concat = np.concatenate([pad] + texts)
    offs = [13]
    for T in texts:
        offs.append(offs[-1] + len(T))
    for flags in (0, bt.BT_DBG_WEAK_HASH, bt.BT_DBG_NO_QUEUE, bt.BT_DBG_NO_QUEUE | bt.BT_DBG_WEAK_HASH,
                  bt.BT_DBG_NO_BYTE_SCAN):
        trees = ctx.build_batch(to_device(concat), offs, tau=2, leaf_len=4, debug_flags=flags)
        for T, tr in zip(texts, trees):
            assert tr.serialize() == oracle.build_tree(T, 2, 4).canonical


def test_batch_equals_single_builds(ctx):
    texts = [synth.markov_versions(n, 4096, 20, 2e-3, 16, n) for n in (65536, 100001, 250000, 9000)]
    concat, offs = _concat(texts)
    d = to_device(concat)
    trees = ctx.build_batch(d, offs, sigma=96, tau=4, leaf_len=16)
    for T, tr in zip(texts, trees):
        single = ctx.build(to_device(T), sigma=96, tau=4, leaf_len=16)
        assert tr.serialize() == single.serialize()


def test_batch_access(ctx):
    torch = torch_cuda()
    texts = _texts(5, 12)
    concat, offs = _concat(texts)
    trees = ctx.build_batch(to_device(concat), offs, tau=2, leaf_len=4)
    for T, tr in zip(texts, trees):
        if len(T) == 0:
            continue
        pos = torch.arange(len(T), device="cuda:0", dtype=torch.int64).to(torch.uint64)
        assert np.array_equal(tr.access(pos).cpu().numpy(), np.asarray(T, np.uint8))


def test_batch_on_reused_pool_memory(ctx):
    """Batched builds on a context whose cached device memory holds data from
    earlier builds (nonzero), so a kernel that read an entry it never wrote
    would see garbage rather than zeros."""
    torch_cuda()
    big = synth.markov_versions(400000, 8192, 40, 2e-3, 32, 5)
    ctx.build(to_device(big), sigma=256, tau=4, leaf_len=16).free()
    for seed in range(3):
        texts = _texts(900 + seed, 24)
        concat, offs = _concat(texts)
        trees = ctx.build_batch(to_device(concat), offs, tau=4, leaf_len=16)
        for T, tr in zip(texts, trees):
            assert tr.serialize() == oracle.build_tree(T, 4, 16).canonical
            tr.free()


def test_free_trees_returns_the_storage(ctx):
    """free_trees (bt_trees_free) on a batch's trees: every tree is freed in one
    call, and the pool holds no more in-use bytes than before the build."""
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    texts = _texts(31, 40)
    concat, offs = _concat(texts)
    d = to_device(concat)
    torch.cuda.synchronize()
    base = ctx.memory()["in_use"]
    trees = ctx.build_batch(d, offs, tau=4, leaf_len=16)
    assert ctx.memory()["in_use"] > base
    want = [oracle.build_tree(T, 4, 16).canonical for T in texts[:3]]
    assert [tr.serialize() for tr in trees[:3]] == want
    h0 = trees[0].height  # read before the batch free: stays readable
    bt.free_trees(trees)
    assert all(tr.h is None for tr in trees)
    assert trees[0].height == h0
    with pytest.raises(bt.BtError):
        trees[1].height  # never read before the free
    torch.cuda.synchronize()
    assert ctx.memory()["in_use"] == base
    # a single tree's size stays readable after tree.free()
    one = ctx.build(to_device(texts[0]), tau=4, leaf_len=16)
    n, h, b1 = one.n, one.height, one.b1
    one2 = ctx.build(to_device(texts[0]), tau=4, leaf_len=16)
    one2.free()
    assert (one2.n, one2.height, one2.b1) == (n, h, b1)
    one.free()


def test_batch_unqueued_scan(ctx):
    """The unqueued 61-bit scan on a batch with short final keys and salts."""
    import paper_2512_23314_amd as bt
    texts = _texts(77, 30)
    concat, offs = _concat(texts)
    trees = ctx.build_batch(to_device(concat), offs, tau=3, leaf_len=4,
                            debug_flags=bt.BT_DBG_NO_QUEUE)
    for T, tr in zip(texts, trees):
        assert tr.serialize() == oracle.build_tree(T, 3, 4).canonical


@pytest.mark.parametrize("count", [2048, 2500])
def test_batch_many_small_texts(ctx, count):
    """Per-text bookkeeping at the size where one workgroup scans the texts'
    counts (2048) and past it (the multi-launch path)."""
    rng = np.random.default_rng(count)
    texts = [synth.random_text(int(rng.integers(0, 60)), int(rng.integers(1, 4)), int(rng.integers(1 << 30)))
             for _ in range(count)]
    concat, offs = _concat(texts)
    trees = ctx.build_batch(to_device(concat), offs, tau=2, leaf_len=2)
    for k, (T, tr) in enumerate(zip(texts, trees)):
        assert tr.serialize() == oracle.build_tree(T, 2, 2).canonical, "text %d" % k


def test_batch_text_local_filters(ctx):
    """Per-text key filters: texts small enough that a workgroup loads their
    filter into LDS, texts whose filter stays in global memory (over 8192
    blocks on a level), and runs of tiny texts whose windows share a span.
    With dense and sampled prefix fingerprints and 12-bit fingerprints, every
    tree equals the oracle's and the shared-filter build's."""
    import paper_2512_23314_amd as bt
    rng = np.random.default_rng(41)
    texts = [synth.cfg1_text(1 << 20), synth.markov_versions(600000, 20000, 30, 3e-3, 16, 3)]
    texts += [synth.dna_copies(int(n), max(1, int(n) // 16), 16, 2e-3, 2e-4, 8, int(rng.integers(1 << 30)))
              for n in rng.integers(0, 3000, 300)]
    texts += [synth.cfg1_text(1 << 17), synth.random_text(40000, 4, 8)]
    concat, offs = _concat(texts)
    d = to_device(concat)
    want = [oracle.build_tree(T, 2, 16).canonical for T in texts]
    for kw in ({}, {"lean": True}, {"debug_flags": bt.BT_DBG_WEAK_HASH}):
        trees = ctx.build_batch(d, offs, tau=2, leaf_len=16, **kw)
        shared = ctx.build_batch(d, offs, tau=2, leaf_len=16,
                                 debug_flags=kw.get("debug_flags", 0) | bt.BT_DBG_SHARED_FILTERS,
                                 lean=kw.get("lean", False))
        for k, (w, tr, sh) in enumerate(zip(want, trees, shared)):
            got = tr.serialize()
            assert got == w, "text %d (length %d), %s" % (k, len(texts[k]), kw)
            assert sh.serialize() == w
            tr.free()
            sh.free()
