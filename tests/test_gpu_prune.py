"""GPU parity of the optional pruning phase (Section 4.1): builds with BT_PRUNE
through the C ABI against the oracle's pruned trees, element by element, on
seeded texts that span several levels and end in ragged tails; batches whose
texts enter the level loop at different steps; every scan mode; queries on
pruned trees; the closed form of a unary text."""
import numpy as np
import pytest

import oracle
import synth
from tests import treecheck
from tests.gpu_util import assert_same_tree, shape_of, to_device, torch_cuda
from tests.test_gpu_batch import _concat, _texts
from tests.test_gpu_queries import _check_queries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    import paper_2512_23314_amd as bt
    c = bt.Context(0)
    yield c
    c.close()


CASES = [
    ("cfg1_16k", lambda: synth.cfg1_text(1 << 14), [(2, 16, 1), (2, 4, 1), (4, 4, 1)]),
    ("random2_ragged", lambda: synth.random_text(30011, 2, 7), [(2, 1, 1), (3, 2, 1), (4, 1, 1)]),
    ("markov_versions", lambda: synth.markov_versions(120007, 8192, 20, 2e-3, 32, 17),
     [(4, 16, 1), (2, 8, 1), (4, 16, 64)]),
    ("periodic", lambda: synth.periodic_text(40001, 89, 3), [(2, 16, 1), (3, 2, 1)]),
    ("unary", lambda: np.full(50000, 65, np.uint8), [(2, 16, 1), (4, 3, 1)]),
    ("dna_copies_tiny", lambda: synth.dna_copies(5000, 300, 20, 0.01, 0.002, 4, 9), [(2, 1, 1), (3, 2, 1)]),
]


@pytest.mark.parametrize("name,gen,params", CASES, ids=[c[0] for c in CASES])
def test_pruned_build_matches_oracle(ctx, name, gen, params):
    T = gen()
    for tau, leaf, s in params:
        ora = oracle.build_tree(T, tau, leaf, s_hint=s, prune=True)
        tree = ctx.build(to_device(T), tau=tau, leaf_len=leaf, s_hint=s, prune=True)
        assert_same_tree(tree, ora)
        if len(T) <= 16384:
            treecheck.check_pruned(shape_of(tree, tau, leaf), bytes(T))


def test_pruned_random_small_texts(ctx):
    """Many short random texts, where chains of candidates (one candidate's
    pointer spilling into two others) and kept parents of targeted children
    occur; one batch per parameter set."""
    rng = np.random.default_rng(4)
    texts = [synth.random_text(int(rng.integers(8, 400)), int(rng.integers(2, 4)), int(rng.integers(1 << 30)))
             for _ in range(200)]
    concat, offs = _concat(texts)
    d = to_device(concat)
    for tau, leaf in ((2, 1), (3, 1), (2, 2)):
        trees = ctx.build_batch(d, offs, tau=tau, leaf_len=leaf, prune=True)
        for T, tr in zip(texts, trees):
            assert tr.serialize() == oracle.build_tree(T, tau, leaf, prune=True).canonical, \
                "text %r (tau %d, leaf %d)" % (bytes(T), tau, leaf)


@pytest.mark.parametrize("tau,leaf,s_hint", [(2, 16, 1), (4, 16, 1), (3, 4, 1)])
def test_pruned_batch_matches_oracle(ctx, tau, leaf, s_hint):
    texts = _texts(tau * 100 + leaf + 7, 30)
    concat, offs = _concat(texts)
    trees = ctx.build_batch(to_device(concat), offs, tau=tau, leaf_len=leaf, s_hint=s_hint, prune=True)
    for T, tr in zip(texts, trees):
        want = oracle.build_tree(T, tau, leaf, s_hint=s_hint, prune=True).canonical
        assert tr.serialize() == want, "text of length %d differs" % len(T)


def test_pruned_scan_modes_and_hashes(ctx):
    """Seeds, 12-bit fingerprints and the unqueued scan give the same pruned tree."""
    import paper_2512_23314_amd as bt
    for T in (synth.cfg1_text(1 << 13), synth.markov_versions(20000, 2000, 10, 5e-3, 16, 5),
              synth.random_text(9000, 2, 4)):
        ref = oracle.build_tree(T, 2, 4, prune=True).canonical
        for seed in (1, 0xDEADBEEF):
            assert ctx.build(to_device(T), tau=2, leaf_len=4, hash_seed=seed, prune=True).serialize() == ref
        for flags in (bt.BT_DBG_WEAK_HASH, bt.BT_DBG_NO_QUEUE, bt.BT_DBG_NO_QUEUE | bt.BT_DBG_WEAK_HASH):
            assert ctx.build(to_device(T), tau=2, leaf_len=4, debug_flags=flags,
                             prune=True).serialize() == ref


@pytest.mark.parametrize("n,tau,leaf", [(1, 2, 16), (15, 2, 16), (16, 2, 16), (17, 2, 16),
                                        (33, 2, 16), (2, 2, 1), (100, 3, 7), (257, 2, 1)])
def test_pruned_edge_sizes(ctx, n, tau, leaf):
    T = synth.random_text(n, 3, n + 5)
    ora = oracle.build_tree(T, tau, leaf, prune=True)
    assert_same_tree(ctx.build(to_device(T), tau=tau, leaf_len=leaf, prune=True), ora)


def test_pruned_empty_text(ctx):
    torch = torch_cuda()
    d = torch.zeros(1, dtype=torch.uint8, device="cuda:0")[:0]
    tree = ctx.build(d, tau=2, leaf_len=16, prune=True)
    assert_same_tree(tree, oracle.build_tree(np.zeros(0, np.uint8), 2, 16, prune=True))


def test_pruned_unary_closed_form(ctx):
    """a^n: one marked block per internal level, tau blocks below level 1, and
    tau*leaf leaf bytes."""
    for tau, leaf, n in ((2, 1, 4000), (4, 4, 100000), (3, 2, 59049)):
        T = np.full(n, 97, np.uint8)
        tree = ctx.build(to_device(T), tau=tau, leaf_len=leaf, prune=True)
        for l in range(1, tree.height):
            b, marked, pb, po = tree.level(l)
            assert marked.tolist() == [1] + [0] * (marked.size - 1)
            assert not pb.any() and not po.any()
            if l > 1:
                assert marked.size == tau
        assert tree.leaves().tobytes() == b"a" * (tau * leaf)


PRUNED_QUERY_TEXTS = [
    ("cfg1_64k", lambda: synth.cfg1_text(1 << 16), 2, 16),
    ("markov", lambda: synth.markov_versions(200003, 8192, 25, 2e-3, 32, 3), 4, 16),
    ("random2", lambda: synth.random_text(50001, 2, 9), 3, 4),
    ("unary", lambda: np.full(30000, 66, np.uint8), 2, 16),
]


@pytest.mark.parametrize("name,gen,tau,leaf", PRUNED_QUERY_TEXTS, ids=[t[0] for t in PRUNED_QUERY_TEXTS])
def test_pruned_queries(ctx, name, gen, tau, leaf):
    """access/rank/select on pruned trees against counted prefixes."""
    T = gen()
    tree = ctx.build(to_device(T), tau=tau, leaf_len=leaf, rank_select=True, prune=True)
    _check_queries(tree, T, len(T) + 1)


def test_pruned_queries_batch(ctx):
    texts = [synth.cfg1_text(n, seed=n) if n else np.zeros(0, np.uint8) for n in (0, 1, 100, 4096, 30000)]
    texts.append(synth.random_text(5000, 3, 1))
    concat, offs = _concat(texts)
    trees = ctx.build_batch(to_device(concat), offs, tau=4, leaf_len=8, rank_select=True, prune=True)
    for k, (T, tr) in enumerate(zip(texts, trees)):
        _check_queries(tr, T, 300 + k, m=3000)
