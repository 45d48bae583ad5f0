"""Memory-lean builds (BT_LEAN): prefix fingerprints kept one in 16 and formed
on demand from their sample and the text.  The tree must be bit-identical to
the oracle's, whatever path a fingerprint takes (keys, queued candidates, the
byte scan, short final keys, collision retries); and the build must use less
device memory than the dense one by the 11.25 bytes per text byte that P and
H cost beyond their samples.  The scans then roll the 32-bit window hashes
along consecutive windows; the tests cover the rolled path, the restart at
segment and text boundaries, and the short final keys rolled beside them."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_same_tree, to_device, torch_cuda
from tests.test_gpu_batch import _concat, _texts
from tests.test_gpu_build import CASES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    import paper_2512_23314_amd as bt
    c = bt.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name,gen,params", CASES, ids=[c[0] for c in CASES])
def test_lean_build_matches_oracle(ctx, name, gen, params):
    T = gen()
    for tau, leaf, s in params:
        tree = ctx.build(to_device(T), tau=tau, leaf_len=leaf, s_hint=s, lean=True)
        assert_same_tree(tree, oracle.build_tree(T, tau, leaf, s_hint=s))


@pytest.mark.parametrize("n", [1, 15, 16, 17, 31, 32, 33, 4095, 4096, 4097, 16384, 16400, 65536 * 3 + 7])
def test_lean_sizes_around_samples(ctx, n):
    """Text lengths around the 16-byte sample grid and the 16 KiB prefix tile
    (the last sample is P[n] itself when n is a multiple of 16)."""
    T = synth.random_text(n, 3, n + 11)
    for tau, leaf in ((2, 1), (3, 5)):
        tree = ctx.build(to_device(T), tau=tau, leaf_len=leaf, lean=True)
        assert tree.serialize() == oracle.build_tree(T, tau, leaf).canonical


def test_lean_retries_and_seeds(ctx):
    """12-bit fingerprints force collisions, so the retry walk forms a sampled
    fingerprint at every position it visits."""
    import paper_2512_23314_amd as bt
    for T in (synth.cfg1_text(1 << 13), synth.markov_versions(20000, 2000, 10, 5e-3, 16, 5),
              synth.random_text(9000, 2, 4)):
        ref = oracle.build_tree(T, 2, 4).canonical
        for kw in (dict(hash_seed=1), dict(hash_seed=0xDEADBEEF), dict(debug_flags=bt.BT_DBG_WEAK_HASH),
                   dict(debug_flags=bt.BT_DBG_NO_BYTE_SCAN)):
            assert ctx.build(to_device(T), tau=2, leaf_len=4, lean=True, **kw).serialize() == ref
        assert ctx.build(to_device(T), tau=2, leaf_len=16, lean=True,
                         debug_flags=bt.BT_DBG_WEAK_HASH).serialize() == oracle.build_tree(T, 2, 16).canonical


@pytest.mark.parametrize("tau,leaf", [(2, 16), (4, 16), (3, 4)])
def test_lean_batch(ctx, tau, leaf):
    """Salted texts with short tails, entering at different steps."""
    import paper_2512_23314_amd as bt
    texts = _texts(tau * 1000 + leaf, 30)
    concat, offs = _concat(texts)
    d = to_device(concat)
    for flags in (0, bt.BT_DBG_WEAK_HASH):
        trees = ctx.build_batch(d, offs, tau=tau, leaf_len=leaf, lean=True, debug_flags=flags)
        for T, tr in zip(texts, trees):
            assert tr.serialize() == oracle.build_tree(T, tau, leaf).canonical, "length %d" % len(T)


def test_lean_unaligned_views_and_pruning(ctx):
    T = synth.markov_versions(150001, 8192, 20, 2e-3, 32, 29)
    d = to_device(T)
    for off in (1, 3, 16, 21):
        tree = ctx.build(d[off:], tau=4, leaf_len=16, lean=True)
        assert tree.serialize() == oracle.build_tree(T[off:], 4, 16).canonical
    tree = ctx.build(d, tau=2, leaf_len=8, lean=True, prune=True)
    assert tree.serialize() == oracle.build_tree(T, 2, 8, prune=True).canonical


def test_lean_needs_less_memory(ctx):
    """Peak pool bytes of one build, lean against dense, on 32 MiB: the prefix
    fingerprints shrink from 2 (a single text's dense build keeps every 4th)
    to 0.5 bytes per text byte and the 32-bit prefix hashes from 4 to 0.25."""
    torch = torch_cuda()
    T = synth.markov_versions(32 << 20, 1 << 18, 1 << 10, 5e-4, 64, 3)
    d = to_device(T)
    peaks = {}
    for lean in (False, True):
        ctx.build(d, tau=4, leaf_len=16, lean=lean).free()  # warm the pool
        torch.cuda.synchronize()
        base = ctx.memory()["in_use"]
        ctx.reset_peak()
        tree = ctx.build(d, tau=4, leaf_len=16, lean=lean)
        peaks[lean] = ctx.memory()["peak"] - base
        tree.free()
    assert peaks[False] - peaks[True] >= 5 * len(T), peaks
    assert peaks[True] <= 3 * len(T), peaks
