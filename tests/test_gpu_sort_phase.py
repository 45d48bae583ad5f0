"""Sort-based phases (Section 5.1, BT_DBG_SORT_PHASES): leftmost occurrences
found by sorting the fingerprints of every scanned window and every key in
place of the hash-table scan.  The tree must be bit-identical to the oracle's,
also with 12-bit fingerprints (large groups of colliding keys), in batches,
with sampled prefix fingerprints and with pruning."""
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


def _flags():
    import paper_2512_23314_amd as bt
    return bt.BT_DBG_SORT_PHASES


@pytest.mark.parametrize("name,gen,params", CASES, ids=[c[0] for c in CASES])
def test_sort_phases_match_oracle(ctx, name, gen, params):
    T = gen()
    for tau, leaf, s in params:
        tree = ctx.build(to_device(T), tau=tau, leaf_len=leaf, s_hint=s, debug_flags=_flags())
        assert_same_tree(tree, oracle.build_tree(T, tau, leaf, s_hint=s))


def test_sort_phases_weak_hash_batch_lean_prune(ctx):
    import paper_2512_23314_amd as bt
    for T in (synth.cfg1_text(1 << 13), synth.markov_versions(20000, 2000, 10, 5e-3, 16, 5),
              synth.random_text(9000, 2, 4)):
        ref = oracle.build_tree(T, 2, 4).canonical
        d = to_device(T)
        assert ctx.build(d, tau=2, leaf_len=4, debug_flags=_flags() | bt.BT_DBG_WEAK_HASH).serialize() == ref
        assert ctx.build(d, tau=2, leaf_len=4, debug_flags=_flags(), lean=True).serialize() == ref
        assert ctx.build(d, tau=2, leaf_len=4, debug_flags=_flags(), prune=True).serialize() == \
            oracle.build_tree(T, 2, 4, prune=True).canonical
    texts = _texts(4242, 30)
    concat, offs = _concat(texts)
    trees = ctx.build_batch(to_device(concat), offs, tau=3, leaf_len=4, debug_flags=_flags())
    for T, tr in zip(texts, trees):
        assert tr.serialize() == oracle.build_tree(T, 3, 4).canonical


def test_sort_phases_unaligned_view(ctx):
    T = synth.markov_versions(120001, 8192, 20, 2e-3, 32, 31)
    d = to_device(T)
    tree = ctx.build(d[3:], tau=4, leaf_len=16, debug_flags=_flags())
    assert tree.serialize() == oracle.build_tree(T[3:], 4, 16).canonical
